"""GPU parity: the HIP path through the C ABI against the CPU oracle."""
import numpy as np
import pytest

from circuits import (make_config, lattice_circuit, stack3d_circuit, iqp_lattice_circuit,
                      random_bitstrings, mirror, product_circuit, paper_iqp_circuit,
                      sycamore_type_circuit, cavity_circuit)
from oracle import statevector_amplitudes, pairwise_amplitudes

import fp_error

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-5, 2: 1e-3, 3: 1e-3, 4: 2e-2}   # 4: plain bf16 rounding, kernel check only


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available()
    from paper_2208_01498_amd import binding as B
    e = B.Engine(0, arena_bytes=256 << 20)
    yield e
    e.close()


def _plan(circ, ns=0, B=8, **kw):
    from paper_2208_01498_amd.planner.plan import make_plan
    kw.setdefault("trials", 1)      # one hierarchy seed: parity does not depend on the cost
    return make_plan(circ, n_slices=ns, B=B, **kw)


def _judge(got, ref, n, plan, prec, label, typical=None):
    """Per-result parity against the oracle: plain relative error within
    TOL[prec] wherever that lies above the rounding floor the plan's
    arithmetic implies (fp_error), the floor below it, the tail under
    1e-2 typical in units of the typical magnitude 2^(-n/2)."""
    typical = 2.0 ** (-n / 2) if typical is None else typical
    return fp_error.check(got, ref, typical, TOL[prec], fp_error.floor(plan, prec, typical), label)


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("ns", [0, 3])
def test_cfg1_all_bitstrings(eng, prec, ns):
    circ, words, _ = make_config("cfg1")
    print("case cfg1 prec", prec, "slices", ns, flush=True)
    plan = _plan(circ, ns, B=len(words))
    p = eng.load(plan.to_blob())
    got = eng.amplitudes(p, words, prec)
    ref = statevector_amplitudes(circ, words)
    _judge(got, ref, circ.n, plan, prec, "cfg1 prec %d slices %d" % (prec, ns))


FAMILIES = [
    ("sqrt_cz_3x4_d6", lambda: lattice_circuit(3, 4, 6, 201, "sqrt", "cz")),
    ("sqrt_fsim_3x3_d5", lambda: lattice_circuit(3, 3, 5, 202, "sqrt", "fsim")),
    ("haar_cz_4x4_d10", lambda: lattice_circuit(4, 4, 10, 203, "haar", "cz")),
    ("stack_2x2x3", lambda: stack3d_circuit(2, 2, 3, 6, 204)),
    ("iqp_3x4", lambda: iqp_lattice_circuit(3, 4, 205)),
    ("product_8", lambda: product_circuit(8, 3, 206)),
    ("paper_iqp_4x4_T16", lambda: paper_iqp_circuit(4, 16, 207)),
    ("sycamore_type_4x4_p05", lambda: sycamore_type_circuit(4, 5, 0.5, 208)),
    ("cavity_4x4_T10_S2", lambda: cavity_circuit(4, 209, T=10, S=2, lam=3.0)),
]


@pytest.mark.parametrize("name,mk", FAMILIES, ids=[f[0] for f in FAMILIES])
@pytest.mark.parametrize("ns", [0, 2])
@pytest.mark.parametrize("prec", [0, 1, 3])
def test_families_vs_statevector(eng, name, mk, ns, prec):
    circ = mk()
    words = random_bitstrings(circ.n, 37, 300)       # odd batch
    print("case", name, "slices", ns, "prec", prec, flush=True)
    plan = _plan(circ, ns, B=len(words))
    p = eng.load(plan.to_blob())
    got = eng.amplitudes(p, words, prec)
    ref = statevector_amplitudes(circ, words)
    _judge(got, ref, circ.n, plan, prec, "%s slices %d prec %d" % (name, ns, prec))


@pytest.mark.parametrize("prec", [0, 3])
def test_chunking_is_bitwise_invariant(prec):
    """A small arena forces chunks of a few bitstrings; results must be
    bitwise identical to a single-chunk run (in the split fp16 mode too: its
    scales depend on one bitstring's rows only)."""
    from paper_2208_01498_amd import binding as B
    circ = lattice_circuit(5, 5, 10, 211, "haar", "cz")
    words = random_bitstrings(25, 64, 212)
    plan = _plan(circ, 2, B=64)
    blob = plan.to_blob()
    info = B.tn_plan_validate(blob)
    small_bytes = max(1 << 20, info["peak_bytes_fixed"] + 12 * info["peak_bytes_per_b"])
    print("arena for ~12 bitstrings", small_bytes, flush=True)
    big = B.Engine(0, arena_bytes=256 << 20)
    small = B.Engine(0, arena_bytes=int(small_bytes))
    try:
        a = big.amplitudes(big.load(blob), words, prec)
        st_big = B.tn_last_exec_stats(big.ctx)
        b = small.amplitudes(small.load(blob), words, prec)
        st_small = B.tn_last_exec_stats(small.ctx)
        print("chunks", st_big["n_chunks"], st_small["n_chunks"], flush=True)
        assert st_small["n_chunks"] > st_big["n_chunks"]
        assert np.array_equal(a, b)
    finally:
        big.close()
        small.close()


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


GEMM_SHAPES = [(1, 1, 1), (4, 2, 1), (2, 2, 1 << 16), (1, 1, 1 << 14), (32, 16, 8), (64, 64, 8),
               (128, 128, 8), (256, 128, 64), (128, 256, 16), (64, 32, 2), (512, 64, 128),
               (1024, 1024, 32), (1024, 4, 4096), (4, 512, 2048), (16, 8, 256), (256, 256, 4096),
               (128, 2, 1)]


@pytest.mark.parametrize("M,N,K", GEMM_SHAPES)
@pytest.mark.parametrize("tA,tB", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4])
def test_kernel_cgemm(M, N, K, tA, tB, prec):
    import torch
    from paper_2208_01498_amd import binding as B
    rng = np.random.Generator(np.random.PCG64(M * 7 + N * 3 + K + tA * 2 + tB))
    nbatch, nb = 3, 2
    A = (rng.standard_normal((nb, nbatch, M, K)) + 1j * rng.standard_normal((nb, nbatch, M, K))).astype(np.complex64)
    Bm = (rng.standard_normal((nbatch, K, N)) + 1j * rng.standard_normal((nbatch, K, N))).astype(np.complex64)
    As = np.swapaxes(A, -1, -2).copy() if tA else A
    Bs = np.swapaxes(Bm, -1, -2).copy() if tB else Bm
    dA, dB = _dev(As.view(np.float32)), _dev(Bs.view(np.float32))
    dC = torch.zeros(nb * nbatch * M * N * 2, dtype=torch.float32, device="cuda")
    sb = B.tn_kernel_cgemm_scratch_bytes(M, N, K, nbatch, nb)
    scratch = torch.empty(max(sb, 8), dtype=torch.uint8, device="cuda")
    print("case gemm", M, N, K, tA, tB, prec, "scratch", sb, flush=True)
    B.tn_kernel_cgemm(dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), M, N, K, tA, tB, nbatch, nb,
                      sAb=nbatch * M * K, sBb=0, sCb=nbatch * M * N, sAi=M * K, sBi=K * N,
                      sCi=M * N, precision=prec, scratch=scratch.data_ptr(), scratch_bytes=sb)
    torch.cuda.synchronize()
    C = dC.cpu().numpy().view(np.complex64).reshape(nb, nbatch, M, N)
    ref = np.matmul(A.astype(np.complex128), Bm.astype(np.complex128)[None])
    scale = np.sqrt(K) * 2
    err = np.max(np.abs(C - ref)) / scale
    assert err <= TOL[prec], err


@pytest.mark.parametrize("M,N,K", [(128, 128, 64), (256, 64, 512), (64, 256, 8), (128, 2, 32),
                                   (2, 128, 4096)])
@pytest.mark.parametrize("tA,tB", [(0, 0), (1, 1), (1, 0)])
@pytest.mark.parametrize("prec", [0, 2, 3])
def test_kernel_cgemm_row_scales(M, N, K, tA, tB, prec):
    """Rows of A and columns of B whose magnitudes span 2^-100 .. 1 (far
    outside the fp16 range, and far apart within one operand), one all-zero
    row and column: every output element is judged against its own row and
    column scale, so a shared per-tensor scale or an fp16 underflow fails."""
    import torch
    from paper_2208_01498_amd import binding as B
    rng = np.random.Generator(np.random.PCG64(M * 13 + N * 5 + K + 7 * tA + tB))
    nbatch, nb = 2, 2
    ea = rng.integers(0, 101, size=(nb, nbatch, M))
    eb = rng.integers(0, 61, size=(nbatch, N))
    sa, sb_ = 2.0 ** (-ea.astype(float)), 2.0 ** (-eb.astype(float))
    A = (rng.standard_normal((nb, nbatch, M, K)) + 1j * rng.standard_normal((nb, nbatch, M, K)))
    Bm = (rng.standard_normal((nbatch, K, N)) + 1j * rng.standard_normal((nbatch, K, N)))
    A = (A * sa[..., None]).astype(np.complex64)
    Bm = (Bm * sb_[:, None, :]).astype(np.complex64)
    A[0, 0, M // 2, :] = 0
    Bm[0, :, N // 2] = 0
    As = np.swapaxes(A, -1, -2).copy() if tA else A
    Bs = np.swapaxes(Bm, -1, -2).copy() if tB else Bm
    dA, dB = _dev(As.view(np.float32)), _dev(Bs.view(np.float32))
    dC = torch.zeros(nb * nbatch * M * N * 2, dtype=torch.float32, device="cuda")
    sbytes = B.tn_kernel_cgemm_scratch_bytes(M, N, K, nbatch, nb)
    scratch = torch.empty(max(sbytes, 8), dtype=torch.uint8, device="cuda")
    print("case gemm row scales", M, N, K, tA, tB, prec, flush=True)
    B.tn_kernel_cgemm(dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), M, N, K, tA, tB, nbatch, nb,
                      sAb=nbatch * M * K, sBb=0, sCb=nbatch * M * N, sAi=M * K, sBi=K * N,
                      sCi=M * N, precision=prec, scratch=scratch.data_ptr(), scratch_bytes=sbytes)
    torch.cuda.synchronize()
    C = dC.cpu().numpy().view(np.complex64).reshape(nb, nbatch, M, N).astype(np.complex128)
    ref = np.matmul(A.astype(np.complex128), Bm.astype(np.complex128)[None])
    unit = np.sqrt(K) * 2 * sa[..., :, None] * sb_[None, :, None, :]
    # outputs below the FP32 normal range are not representable in any mode
    ok = unit > 2.0 ** -100
    err = (np.abs(C - ref) / unit)[ok].max()
    print("max error in row-column units", err, flush=True)
    assert err <= TOL[prec], err
    assert np.all(C[0, 0, M // 2, :] == 0) and np.all(C[:, 0, :, N // 2] == 0)


@pytest.mark.parametrize("rank,nb", [(1, 1), (3, 5), (8, 2), (12, 3), (17, 1), (20, 2)])
def test_kernel_permute(rank, nb):
    import torch
    from paper_2208_01498_amd import binding as B
    rng = np.random.Generator(np.random.PCG64(rank * 31 + nb))
    perm = [int(x) for x in rng.permutation(rank)]
    x = (rng.standard_normal((nb, 1 << rank)) + 1j * rng.standard_normal((nb, 1 << rank))).astype(np.complex64)
    dx = _dev(x.view(np.float32))
    dy = torch.zeros_like(dx)
    print("case permute", rank, nb, perm, flush=True)
    B.tn_kernel_permute(dx.data_ptr(), dy.data_ptr(), rank, perm, nb)
    torch.cuda.synchronize()
    y = dy.cpu().numpy().view(np.complex64).reshape(nb, 1 << rank)
    # destination bit p takes source bit perm[p]: as C-order axes (axis 0 is
    # the most significant bit), destination axis rank-1-p is source axis
    # rank-1-perm[p]
    src = x.reshape((nb,) + (2,) * rank)
    axes = [0] + [1 + (rank - 1 - perm[rank - 1 - a]) for a in range(rank)]
    want = np.transpose(src, axes).reshape(nb, 1 << rank)
    assert np.array_equal(y, want)


def test_slice_block_is_bitwise_invariant():
    """Slices computed one per pass or in blocks of 2^r (folded into the
    GEMMs) give bitwise identical amplitudes."""
    from paper_2208_01498_amd import binding as B
    circ = lattice_circuit(4, 4, 10, 221, "haar", "cz")
    words = random_bitstrings(16, 24, 222)
    plan = _plan(circ, 5, B=24)
    blob = plan.to_blob()
    eng = B.Engine(0, arena_bytes=128 << 20)
    try:
        p = eng.load(blob)
        res = {}
        for r in (0, 1, 3, 5, -1):
            B.tn_ctx_set_slice_block(eng.ctx, r)
            res[r] = eng.amplitudes(p, words, 0)
            st = B.tn_last_exec_stats(eng.ctx)
            print("slice block", r, "->", st["slice_block"], "chunk", st["chunk"], flush=True)
        for r in res:
            assert np.array_equal(res[r], res[0]), r
        ref = statevector_amplitudes(circ, words)
        _judge(res[0], ref, circ.n, plan, 0, "4x4 d10 2^5 slices prec 0")
        # the 3M and split paths too
        for prec in (1, 2, 3):
            B.tn_ctx_set_slice_block(eng.ctx, 0)
            a = eng.amplitudes(p, words, prec)
            B.tn_ctx_set_slice_block(eng.ctx, 5)
            b = eng.amplitudes(p, words, prec)
            assert np.array_equal(a, b), prec
            _judge(a, ref, circ.n, plan, prec, "4x4 d10 2^5 slices prec %d" % prec)
    finally:
        eng.close()


def _projectors(n, word, traced):
    P = []
    for q in range(n):
        if q in traced:
            P.append(np.eye(2))
        else:
            e = np.zeros((2, 2))
            e[(int(word) >> q) & 1, (int(word) >> q) & 1] = 1.0
            P.append(e)
    return P


@pytest.mark.parametrize("traced", [(), (0, 5, 11), tuple(range(2, 12))])
@pytest.mark.parametrize("prec", [0, 1])
def test_projector_mode_vs_doubled_oracle(eng, traced, prec):
    """The paper's quantity <0|C^dag (x)_q P_q C|0> (P_q = |x_q><x_q| on
    projected qubits, 1 on traced ones) through the same executor, against
    the oracle's doubled expectation; tracing all but two qubits, the four
    marginal probabilities sum to 1."""
    from oracle import doubled_expectation
    circ = lattice_circuit(3, 4, 6, 460, "haar", "cz")
    mask = sum(1 << q for q in traced)
    if len(traced) == circ.n - 2:
        free = [q for q in range(circ.n) if q not in traced]
        words = np.array([(a << free[0]) | (b << free[1]) for a in (0, 1) for b in (0, 1)], dtype=np.uint64)
    else:
        words = np.array([int(w) & ~mask for w in random_bitstrings(circ.n, 9, 461)], dtype=np.uint64)
    print("case projector traced", traced, "prec", prec, flush=True)
    plan = _plan(circ, 2, B=len(words), projector=traced)
    got = eng.amplitudes(eng.load(plan.to_blob()), words, prec)
    ref = np.array([doubled_expectation(circ, _projectors(circ.n, w, traced), method="statevector")
                    for w in words])
    # c is a probability of n - |traced| projected bits: typical size 2^-(n - |traced|)
    _judge(got, ref, circ.n, plan, prec, "projector traced %d prec %d" % (len(traced), prec),
           typical=2.0 ** (-(circ.n - len(traced))))
    if len(traced) == circ.n - 2:
        assert abs(got.sum() - 1) <= 1e-5
