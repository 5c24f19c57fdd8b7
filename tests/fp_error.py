"""Rounding-error floor of the engine's amplitudes, derived from the plan.

Test infrastructure: the parity tests judge each amplitude against the
oracle with this floor beside the plain relative tolerance.

Why a floor.  Every amplitude is a sum over exponentially many paths; the
engine stores every tensor in complex64 and accumulates every product in
FP32, so each rounding perturbs an intermediate entry C_e by a relative
delta_e (|delta_e| <= u = 2^-24 with round to nearest; modelled as
independent, zero-mean, uniform, rms u/sqrt(3)).  To first order the
amplitude moves by sum_e delta_e g_e C_e, where g = da/dC is the rest of
the network contracted against C (the environment of the step).  The
variance of that sum is (u^2/3) sum_e |g_e C_e|^2.  For a cut through a
unitary circuit the squared path weights sum, over all output bitstrings,
to the norm of the state: sum_x sum_e |g_e(x) C_e|^2 = sum_x |a(x)|^2 = 1,
so one rounding of one tensor contributes on average (u^2/3) 2^-n to
|a_hat - a|^2 -- the typical squared magnitude 2^-n, not |a(x)|^2.  That is
why single precision has an absolute error floor at the typical magnitude
and the plain relative error of an amplitude far below 2^(-n/2) is not
bounded by the arithmetic.

Counting the roundings of one amplitude (units of (u^2/3) 2^-n):
  * each leaf: 1 (complex128 -> complex64 at load);
  * each step: 1 (its output stored in complex64);
  * a step summing K terms per output element in FP32 in one running
    accumulator rounds K times; with a random-walk partial sum of size
    sqrt(k) at term k the accumulated variance is sum_k k / K = K/2 units
    (relative to the result).  The kernel sums K/s consecutive terms per
    range and adds the s ranges in float64 (tn_kernel_cgemm_shape gives the
    class and s), so the count is K/(2s); the K-parallel dot kernel sums in
    float64 and counts 0;
  * 3M forms Re C = P1 - P2 and Im C = P3 - P1 - P2 from three real
    products, P3 = (Ar + Ai)(Br + Bi) with |P3| about twice |P1|, so the
    accumulation count doubles, and the two operand sums add 2;
  * a hi/lo split (bf16, or scaled fp16) represents each operand entry to
    within 2^-16 of itself (hi rounds to 8 significant bits, lo rounds the
    remainder to 8 more), rms 2^-16/3, and drops the lo*lo product of the
    same size: 3 such events per step, (2^-16/3)^2 / (2^-48/3) = 2^16/3
    units each; plain bf16 rounding (one product) has 2 events of rms
    2^-8/sqrt(3), 2^32 units each.

sigma = sqrt(count * u^2/3) * 2^(-n/2) is the predicted rms error (u^2/3
is the largest mean square relative error of one rounding, reached by
significands at the bottom of their binade).  For a complex error with
independent Gaussian parts, P(|err| > lam sigma) = exp(-lam^2); the floor
is lam = 4 (1.1e-7 per result).

The one assumption is the cut identity above (rho = 1: each rounded tensor
weighs like a state of the circuit).  An FP32 evaluation of the plan on the
CPU (evaluate_plan) measures rms / sigma of 0.65 to 1.05 for the lattice
and stack families.  IQP circuits do not satisfy it: between their two
Hadamard layers every intermediate is a partial sum of unit-modulus phases
over the same hyperedge variables its environment sums, and the measured
ratio grows slowly with size (1.3 at 12 qubits, 1.5 to 1.7 at 20 to 36,
1.9 at the 48-qubit 6 x 8 workload; 2.3 on the GPU there).  Their floors
carry rho = RHO_DIAGONAL, an empirical constant that the CPU tests pin
against the emulation up to 48 qubits.  The GPU tests compare the
prediction with the measured rms error where the oracle is exact.
"""
import math

import numpy as np

U_RMS2 = 2.0 ** -48 / 3.0            # (u/sqrt(3))^2, u = 2^-24
SPLIT_UNITS = 2.0 ** 16 / 3.0         # one hi/lo event, in units of U_RMS2
BF16_1TERM_UNITS = 2.0 ** 32          # one plain bf16 rounding, in units of U_RMS2
LAMBDA = 4.0
RHO_DIAGONAL = 2.5                    # IQP-type networks (diagonal gates between H layers)


def _steps(plan):
    """Per-slice, per-bitstring (M, N, K, nbatch) of every step, from the
    plan's network and step list (output and sliced labels fixed)."""
    net = plan.net
    sl = set(plan.sliced)
    fixed = {l for l, lab in net.labels.items() if lab.kind == "out"} | sl
    bits = {l: int(round(math.log2(lab.dim))) for l, lab in net.labels.items()}
    live = {i: set(l for l in f.labels if l not in fixed) for i, f in enumerate(net.factors)}
    cnt = {}
    for s in live.values():
        for l in s:
            cnt[l] = cnt.get(l, 0) + 1
    nid = len(net.factors)
    out = []
    for a, b in plan.steps:
        la, lb = live.pop(a), live.pop(b)
        u = la | lb
        lc = set(l for l in u if cnt[l] - (l in la) - (l in lb) > 0)
        for l in la:
            cnt[l] -= 1
        for l in lb:
            cnt[l] -= 1
        for l in lc:
            cnt[l] += 1
        e = lambda s: 1 << sum(bits[l] for l in s)
        out.append((e(la - lb), e(lb - la), e((la & lb) - lc), e(la & lb & lc)))
        live[nid] = lc
        nid += 1
    return out


def rounding_units(plan, precision, kernel_sums=True):
    """Rounding count of one amplitude, in units of (u^2/3) 2^-n.  With
    kernel_sums=False every step is taken to sum its K terms in one FP32
    running accumulator (the CPU emulation below)."""
    from paper_2208_01498_amd import binding as B
    units = float(len(plan.net.factors))
    for M, N, K, nbatch in _steps(plan):
        kind, s = B.tn_kernel_cgemm_shape(M, N, K, nbatch) if kernel_sums else (1, 1)
        units += 1.0
        if kind == 0:              # float64 dot product, any mode
            continue
        acc = K / (2.0 * s)
        if precision == B.TN_FP32_3M:
            units += 2.0 * acc + 2.0
        else:
            units += acc
        if precision in (B.TN_SPLIT_BF16, B.TN_SPLIT_FP16):
            units += 3.0 * SPLIT_UNITS
        elif precision == B.TN_BF16_1TERM:
            units += 2.0 * BF16_1TERM_UNITS
    return units


def predicted_rms(plan, precision, kernel_sums=True):
    """Predicted rms error in units of the typical magnitude."""
    return math.sqrt(rounding_units(plan, precision, kernel_sums) * U_RMS2)


def evaluate_plan(plan, word, dtype):
    """The plan's own network and pairwise order evaluated on the CPU with
    numpy in `dtype` (no slicing): every leaf rounded to dtype once, every
    step an einsum whose sums run in dtype, every result stored in dtype.
    With complex64 this is an FP32 rounding experiment on the plan (it
    checks the rounding model's assumptions, not the GPU kernels)."""
    net = plan.net
    assert not plan.sliced
    live = {}
    for i, f in enumerate(net.factors):
        arr = np.asarray(f.data, dtype=np.complex128)
        labels = list(f.labels)
        idx = []
        keep = []
        for ax, l in enumerate(labels):
            lab = net.labels[l]
            if lab.kind == "out":
                idx.append((int(word) >> lab.qubit) & 1)
            else:
                idx.append(slice(None))
                keep.append(l)
        live[i] = (arr[tuple(idx)].astype(dtype), keep)
    cnt = {}
    for _, ls in live.values():
        for l in ls:
            cnt[l] = cnt.get(l, 0) + 1
    nid = len(net.factors)
    letters = {}

    def sym(l):
        if l not in letters:
            letters[l] = chr(ord("a") + len(letters)) if len(letters) < 26 else chr(ord("A") + len(letters) - 26)
        return letters[l]

    for a, b in plan.steps:
        (A, la), (B_, lb) = live.pop(a), live.pop(b)
        for l in la:
            cnt[l] -= 1
        for l in lb:
            cnt[l] -= 1
        lc = [l for l in dict.fromkeys(la + lb) if cnt[l] > 0]
        letters.clear()
        spec = "".join(sym(l) for l in la) + "," + "".join(sym(l) for l in lb) + "->" + \
            "".join(sym(l) for l in lc)
        C = np.einsum(spec, A, B_, optimize=False).astype(dtype)
        for l in lc:
            cnt[l] += 1
        live[nid] = (C, lc)
        nid += 1
    (root, lr), = live.values()
    assert not lr
    return complex(root) * complex(net.scale)


def floor(plan, precision, typical, lam=LAMBDA, rho=None):
    """Absolute error floor: lam x rho x predicted rms x typical magnitude;
    rho defaults to RHO_DIAGONAL for a circuit whose every non-diagonal
    gate is a Hadamard (IQP type), else 1."""
    if rho is None:
        rho = RHO_DIAGONAL if is_diagonal_type(plan.circ) else 1.0
    return lam * rho * predicted_rms(plan, precision) * typical


def is_diagonal_type(circ):
    """Every gate diagonal or a Hadamard: the IQP form H^n D H^n."""
    h = np.array([[1, 1], [1, -1]]) / math.sqrt(2.0)
    for g in circ.gates:
        m = np.asarray(g.matrix)
        if np.count_nonzero(np.abs(m - np.diag(np.diag(m))) > 1e-12) == 0:
            continue
        if m.shape == (2, 2) and np.allclose(m, h):
            continue
        return False
    return True


def check(got, ref, typical, tol, floor_abs, label=""):
    """Per-result criterion.  An amplitude with |a_ref| >= 1e-2 typical
    passes when |a - a_ref| <= max(tol |a_ref|, floor): the plain relative
    tolerance wherever it lies above the derived floor.  The rare tail
    below 1e-2 typical is judged in units of the typical magnitude,
    |a - a_ref| <= max(tol typical, floor), and listed separately.  Prints
    every result's plain relative error; returns a summary."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    err = np.abs(got - ref)
    mag = np.abs(ref) / typical
    rel = err / np.maximum(np.abs(ref), 1e-300)
    main = mag >= 1e-2
    bound = np.where(main, np.maximum(tol * np.abs(ref), floor_abs),
                     np.maximum(tol * typical, floor_abs))
    ok = err <= bound
    print("%s: %d results (%d in the tail below 1e-2 typical); floor %.3e typical; "
          "plain relative <= %.0e for %d of %d; max plain relative %.3e; max |err|/typical %.3e"
          % (label, len(ref), int((~main).sum()), floor_abs / typical, tol,
             int((rel[main] <= tol).sum()), int(main.sum()),
             rel[main].max() if main.any() else 0.0, (err / typical).max()), flush=True)
    # every result of a small batch; of a large one, the 16 largest plain
    # relative errors, the tail and every failure
    show = np.arange(len(ref))
    if len(ref) > 64:
        worst = np.argsort(-np.where(main, rel, 0.0))[:16]
        show = np.unique(np.concatenate([worst, np.flatnonzero(~main), np.flatnonzero(~ok)]))
    for i in show:
        print("  %s[%d] |a_ref|/typical %.4f plain rel %.3e |err|/typical %.3e %s%s"
              % (label, i, mag[i], rel[i], err[i] / typical, "ok" if ok[i] else "FAIL",
                 "" if main[i] else " (tail)"), flush=True)
    assert ok.all(), "%s: %d results above max(tol |a_ref|, floor)" % (label, int((~ok).sum()))
    return dict(n=len(ref), tail=int((~main).sum()), plain_ok=int((rel[main] <= tol).sum()),
                max_rel=float(rel[main].max()) if main.any() else 0.0,
                max_err_typical=float((err / typical).max()),
                rms_err_typical=float(np.sqrt(np.mean((err / typical) ** 2))))
