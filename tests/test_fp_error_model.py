"""CPU pins of the rounding model behind the parity floor (fp_error)."""
import numpy as np
import pytest

import fp_error
from circuits import (lattice_circuit, iqp_lattice_circuit, stack3d_circuit, paper_iqp_circuit,
                      random_bitstrings)
from oracle import statevector_amplitudes

U = 2.0 ** -24


@pytest.mark.parametrize("K", [64, 512, 4096])
def test_running_fp32_sum_variance_is_at_most_K_over_2_units(K):
    """A running FP32 sum of K random complex terms: the relative mean
    square error lies below (u^2/3) K/2 (the model's accumulation count)
    and above a third of it (the count is not vacuous)."""
    rng = np.random.default_rng(K)
    R = 3000
    re = rng.standard_normal((R, K)).astype(np.float32)
    im = rng.standard_normal((R, K)).astype(np.float32)
    s = (np.cumsum(re, axis=1, dtype=np.float32)[:, -1].astype(np.float64)
         + 1j * np.cumsum(im, axis=1, dtype=np.float32)[:, -1].astype(np.float64))
    exact = re.astype(np.float64).sum(1) + 1j * im.astype(np.float64).sum(1)
    ratio = np.mean(np.abs(s - exact) ** 2) / np.mean(np.abs(exact) ** 2) / (U * U / 3 * K / 2)
    print("K", K, "measured / modelled variance", ratio)
    assert 0.33 <= ratio <= 1.0


def _bf16(x):
    """Round float32 to bfloat16 (round to nearest even), as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def test_bf16_split_event_sizes():
    """x = hi + lo + r with hi = bf16(x), lo = bf16(x - hi): |r| <= 2^-16 |x|
    and rms(r/x) below the model's 2^-16/3; the dropped lo_a lo_b term
    likewise; one plain bf16 rounding below 2^-8/sqrt(3)."""
    rng = np.random.default_rng(7)
    x = rng.standard_normal(200000).astype(np.float32)
    y = rng.standard_normal(200000).astype(np.float32)
    hx, hy = _bf16(x), _bf16(y)
    lx, ly = _bf16(x - hx), _bf16(y - hy)
    r = (x.astype(np.float64) - hx - lx) / x
    assert np.abs(r).max() <= 2.0 ** -16
    assert np.sqrt(np.mean(r ** 2)) <= 2.0 ** -16 / 3
    d = lx.astype(np.float64) * ly / (x.astype(np.float64) * y)
    assert np.sqrt(np.mean(d ** 2)) <= 2.0 ** -16 / 3
    e1 = (x.astype(np.float64) - hx) / x
    assert np.sqrt(np.mean(e1 ** 2)) <= 2.0 ** -8 / np.sqrt(3)


def test_model_counts_on_a_plan():
    """Counts grow with the arithmetic: 3M above 4M, the split modes far
    above FP32, every leaf and step at least once."""
    from paper_2208_01498_amd import binding as B
    from paper_2208_01498_amd.planner.plan import make_plan
    plan = make_plan(lattice_circuit(4, 4, 10, 203, "haar", "cz"), n_slices=0, B=8, trials=1)
    u4 = fp_error.rounding_units(plan, B.TN_FP32_4M)
    u3 = fp_error.rounding_units(plan, B.TN_FP32_3M)
    ub = fp_error.rounding_units(plan, B.TN_SPLIT_BF16)
    assert u4 >= len(plan.net.factors) + len(plan.steps)
    assert u3 > u4
    assert ub > 100 * u4
    assert fp_error.rounding_units(plan, B.TN_FP32_4M, kernel_sums=False) >= u4


EMUL = [
    ("haar_cz_4x4_d10", lambda: lattice_circuit(4, 4, 10, 203, "haar", "cz"), 1.0),
    ("sqrt_cz_3x4_d6", lambda: lattice_circuit(3, 4, 6, 201, "sqrt", "cz"), 1.0),
    ("sqrt_fsim_4x4_d8", lambda: lattice_circuit(4, 4, 8, 212, "sqrt", "fsim"), 1.0),
    ("stack_2x3x3", lambda: stack3d_circuit(2, 3, 3, 10, 213), 1.0),
    ("iqp_3x4", lambda: iqp_lattice_circuit(3, 4, 205), fp_error.RHO_DIAGONAL),
    ("iqp_4x5", lambda: iqp_lattice_circuit(4, 5, 206), fp_error.RHO_DIAGONAL),
    ("paper_iqp_4x4_T16", lambda: paper_iqp_circuit(4, 16, 207), fp_error.RHO_DIAGONAL),
]


@pytest.mark.parametrize("name,mk,rho", EMUL, ids=[e[0] for e in EMUL])
def test_model_bounds_an_fp32_evaluation_of_the_plan(name, mk, rho):
    """The plan evaluated with every leaf, sum and intermediate in complex64
    (numpy, CPU), 96 bitstrings against the state vector: the rms error in
    units of 2^(-n/2) is at most rho times the model's prediction (with
    running sums everywhere) and at least a third of it."""
    from paper_2208_01498_amd.planner.plan import make_plan
    circ = mk()
    plan = make_plan(circ, n_slices=0, B=96, trials=1)
    words = random_bitstrings(circ.n, 96, 11)
    ref = statevector_amplitudes(circ, words)
    got = np.array([fp_error.evaluate_plan(plan, w, np.complex64) for w in words])
    typ = 2.0 ** (-circ.n / 2)
    rms = np.sqrt(np.mean(np.abs(got - ref) ** 2)) / typ
    pred = fp_error.predicted_rms(plan, 0, kernel_sums=False)
    print(name, "rms %.3e predicted %.3e ratio %.2f rho %.2f" % (rms, pred, rms / pred, rho))
    assert rho == (fp_error.RHO_DIAGONAL if fp_error.is_diagonal_type(circ) else 1.0)
    assert pred / 3 <= rms <= 1.25 * rho * pred


def test_iqp_workload_rounding_ratio_stays_below_rho():
    """The 48-qubit IQP workload's plan evaluated in complex64 against the
    same evaluation in complex128 (no state vector at this size): the rms
    difference stays within rho = RHO_DIAGONAL of the prediction."""
    from circuits import make_config
    from paper_2208_01498_amd.planner.plan import make_plan
    circ, words, _ = make_config("cfg4")
    plan = make_plan(circ, n_slices=0, B=64, trials=1)
    w = words[:64]
    a64 = np.array([fp_error.evaluate_plan(plan, x, np.complex64) for x in w])
    a128 = np.array([fp_error.evaluate_plan(plan, x, np.complex128) for x in w])
    typ = 2.0 ** (-circ.n / 2)
    rms = np.sqrt(np.mean(np.abs(a64 - a128) ** 2)) / typ
    pred = fp_error.predicted_rms(plan, 0, kernel_sums=False)
    print("iqp 6x8 rms %.3e predicted %.3e ratio %.2f" % (rms, pred, rms / pred))
    assert pred <= rms <= fp_error.RHO_DIAGONAL * pred
