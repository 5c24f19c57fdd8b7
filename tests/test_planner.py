"""Planner tests (CPU): the plan's order, evaluated by the oracle, equals the
state vector; step costs match a brute-force multiplication count; the
separators satisfy the sphere separator conditions; the SSA geometry."""
import itertools
import math

import numpy as np
import pytest

from circuits import (make_config, lattice_circuit, stack3d_circuit, iqp_lattice_circuit,
                      random_bitstrings, product_circuit)
from oracle import statevector_amplitudes, pairwise_amplitudes
from paper_2208_01498_amd.planner.plan import make_plan
from paper_2208_01498_amd.planner.network import build_network
from paper_2208_01498_amd.planner.hierarchy import TreeBuilder, tree_steps
from paper_2208_01498_amd.planner.cost import plan_stats
from paper_2208_01498_amd.planner import ssa


CIRCS = [
    ("cfg1", lambda: make_config("cfg1")[0]),
    ("fsim_3x3_d6", lambda: lattice_circuit(3, 3, 6, 401, "sqrt", "fsim")),
    ("haar_cz_4x3_d8", lambda: lattice_circuit(4, 3, 8, 402, "haar", "cz")),
    ("stack_2x2x3", lambda: stack3d_circuit(2, 2, 3, 8, 403)),
    ("iqp_3x4", lambda: iqp_lattice_circuit(3, 4, 404)),
    ("product_6", lambda: product_circuit(6, 2, 405)),
]


@pytest.mark.parametrize("name,mk", CIRCS, ids=[c[0] for c in CIRCS])
@pytest.mark.parametrize("ns", [0, 3])
def test_plan_order_evaluated_by_oracle(name, mk, ns):
    circ = mk()
    words = random_bitstrings(circ.n, 4, 410)
    plan = make_plan(circ, n_slices=ns, B=4)
    spec = plan.order_spec()
    got = pairwise_amplitudes(circ, words, order=spec, sliced=spec["sliced"])
    ref = statevector_amplitudes(circ, words)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1e-300, np.max(np.abs(ref)))


def test_every_gate_in_exactly_one_leaf():
    circ = make_config("cfg1")[0]
    plan = make_plan(circ, n_slices=2, B=8)
    gates = [g for leaf in plan.order_spec()["leaves"] for g in leaf]
    assert sorted(gates) == list(range(len(circ.gates)))


def _brute_force_step(A, la, B, lb, keep):
    """Explicit loops over every assignment of the union of indices; returns
    the result and the number of scalar multiplications."""
    u = list(dict.fromkeys(list(la) + list(lb)))
    out = [l for l in u if l in keep]
    C = np.zeros((2,) * len(out), dtype=np.complex128)
    mults = 0
    for vals in itertools.product((0, 1), repeat=len(u)):
        v = dict(zip(u, vals))
        C[tuple(v[l] for l in out)] += A[tuple(v[l] for l in la)] * B[tuple(v[l] for l in lb)]
        mults += 1
    return C, out, mults


def test_step_cost_equals_brute_force_count():
    """Eq. (3): a step over index union U takes prod dim multiplications; the
    planner's flop count is 8 per complex multiply-add."""
    circ = lattice_circuit(2, 3, 3, 420, "haar", "cz")
    net = build_network(circ)
    tb = TreeBuilder(net, np.random.Generator(np.random.PCG64(0)), bottom=4)
    steps = tree_steps(tb.build(), len(net.factors))
    stats = plan_stats(net, steps)
    is_out = {l: L.kind == "out" for l, L in net.labels.items()}
    live = {i: (f.data, [l for l in f.labels]) for i, f in enumerate(net.factors)}
    # fix outputs to zero so every tensor is over wire labels only
    for i, (d, ls) in list(live.items()):
        idx = tuple(0 if is_out[l] else slice(None) for l in ls)
        live[i] = (d[idx], [l for l in ls if not is_out[l]])
    nid = len(net.factors)
    for (a, b), rec in zip(steps, stats["steps"]):
        A, la = live.pop(a)
        B, lb = live.pop(b)
        others = set(l for _, ls in live.values() for l in ls)
        keep = set(l for l in set(la) | set(lb) if l in others)
        C, lc, mults = _brute_force_step(A, la, B, lb, keep)
        assert rec[8] == 8.0 * mults
        live[nid] = (C, lc)
        nid += 1


def test_separators_satisfy_balance():
    circ = make_config("cfg3")[0]
    net = build_network(circ)
    tb = TreeBuilder(net, np.random.Generator(np.random.PCG64(1)), bottom=40)
    seen = []
    orig = ssa.eq_checks

    def rec(side, d, k):
        r = orig(side, d, k)
        seen.append(r)
        return r
    ssa.eq_checks = rec
    import paper_2208_01498_amd.planner.hierarchy as H
    H.eq_checks = rec
    try:
        tb.build()
    finally:
        ssa.eq_checks = orig
        H.eq_checks = orig
    assert seen
    # the hierarchy only accepts candidates passing Eq. (2); many SSA circles
    # pass both equations
    assert sum(1 for a, b in seen if a and b) > 0


def test_stereographic_projection_and_rotation():
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.standard_normal((50, 2)) * 3
    y = ssa.stereo(x)
    assert np.allclose(np.linalg.norm(y, axis=1), 1.0)
    assert np.allclose(ssa.stereo_inv(y), x)
    c = rng.standard_normal(3)
    c /= 2 * np.linalg.norm(c)
    R = ssa._householder_to_pole(c)
    assert np.allclose(R @ R.T, np.eye(3))
    assert np.allclose(R @ c, [0, 0, np.linalg.norm(c)])


def test_centerpoint_depth():
    """Every hyperplane through a centerpoint of m points in R^D leaves at
    least m/(D+1) points on each side (checked with a margin on random
    directions)."""
    rng = np.random.Generator(np.random.PCG64(4))
    P = ssa.stereo(rng.standard_normal((400, 2)))
    c = ssa.centerpoint(P, rng)
    worst = 1.0
    for _ in range(200):
        u = rng.standard_normal(3)
        side = (P - c) @ u
        worst = min(worst, np.mean(side > 0), np.mean(side < 0))
    assert worst >= 0.5 / 3


def test_plan_blob_accepted_by_library_validator():
    from paper_2208_01498_amd import binding as B
    B.load_library()
    for name, mk in CIRCS:
        plan = make_plan(mk(), n_slices=2, B=4)
        info = B.tn_plan_validate(plan.to_blob())
        assert info["n_steps"] == info["n_leaves"] - 1
        assert info["n_sliced"] == len(plan.sliced)


def _contract_plan_network(plan, word):
    """Dense FP64 contraction of the planner's own factors in the plan's
    order (test helper): output labels fixed to the bitstring, sliced labels
    summed by the contraction itself."""
    from oracle.pairwise import contract_pair
    net = plan.net
    live = {}
    for i, f in enumerate(net.factors):
        d, ls = f.data, list(f.labels)
        idx = tuple(((int(word) >> net.labels[l].qubit) & 1) if net.labels[l].kind == "out"
                    else slice(None) for l in ls)
        live[i] = (d[idx], [l for l in ls if net.labels[l].kind != "out"])
    nid = len(net.factors)
    for a, b in plan.steps:
        A, la = live.pop(a)
        B, lb = live.pop(b)
        others = set(l for _, ls in live.values() for l in ls)
        keep = set(l for l in set(la) | set(lb) if l in others)
        live[nid] = contract_pair(A, la, B, lb, keep)
        nid += 1
    (arr, ls), = live.values()
    return complex(np.asarray(arr).sum()) * net.scale


@pytest.mark.parametrize("name,mk", CIRCS, ids=[c[0] for c in CIRCS])
def test_plan_network_matches_statevector(name, mk):
    """The planner's network itself (diagonal hyperedges, wire exchanges,
    absorbed gates, structural zeros) contracted on the host equals the
    state vector."""
    circ = mk()
    words = random_bitstrings(circ.n, 3, 430)
    plan = make_plan(circ, n_slices=0, B=3)
    got = np.array([_contract_plan_network(plan, w) for w in words])
    ref = statevector_amplitudes(circ, words)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_swap_form_network_matches_statevector():
    from paper_2208_01498_amd.planner.network import build_network
    from paper_2208_01498_amd.planner.plan import Plan
    circ = lattice_circuit(3, 3, 5, 440, "sqrt", "fsim")
    words = random_bitstrings(circ.n, 3, 441)
    net = build_network(circ, swap_relabel=True)
    tb = TreeBuilder(net, np.random.Generator(np.random.PCG64(0)), bottom=8)
    steps = tree_steps(tb.build(), len(net.factors))
    plan = Plan(circ, net, steps, [], None, None, None, None)
    got = np.array([_contract_plan_network(plan, w) for w in words])
    ref = statevector_amplitudes(circ, words)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def _contract_net_host(net, steps, word):
    """Dense FP64 contraction of a planner network in a plan's order, output
    labels fixed to the bits of `word` (test helper)."""
    from oracle.pairwise import contract_pair
    live = {}
    for i, f in enumerate(net.factors):
        d, ls = f.data, list(f.labels)
        idx = tuple(((int(word) >> net.labels[l].qubit) & 1) if net.labels[l].kind == "out"
                    else slice(None) for l in ls)
        live[i] = (d[idx], [l for l in ls if net.labels[l].kind != "out"])
    nid = len(net.factors)
    for a, b in steps:
        A, la = live.pop(a)
        B, lb = live.pop(b)
        others = set(l for _, ls in live.values() for l in ls)
        keep = set(l for l in set(la) | set(lb) if l in others)
        live[nid] = contract_pair(A, la, B, lb, keep)
        nid += 1
    (arr, ls), = live.values()
    return complex(np.asarray(arr).sum()) * net.scale


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


@pytest.mark.parametrize("traced", [(), (0, 5), (1, 2, 3, 7, 9)])
@pytest.mark.parametrize("twoq", ["cz", "fsim"])
def test_projector_network_matches_doubled_oracle(traced, twoq):
    """The planner's network of C and its conjugate (the paper's
    <0|C^dag (x) P_q C|0>) contracted in the plan's order equals the oracle's
    doubled expectation, for projected and traced qubits (fSim(pi/2, pi/6)
    also in its SWAP-times-diagonal form)."""
    from oracle import doubled_expectation
    circ = lattice_circuit(3, 4, 5, 450, "haar" if twoq == "cz" else "sqrt", twoq)
    plan = make_plan(circ, n_slices=0, B=2, projector=traced)
    for w in random_bitstrings(circ.n, 3, 451):
        w = int(w) & ~sum(1 << q for q in traced)
        got = _contract_net_host(plan.net, plan.steps, w)
        ref = doubled_expectation(circ, _projectors(circ.n, w, traced), method="statevector")
        assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-300)


def test_projector_marginals_sum_to_one():
    """Tracing all but two qubits gives a distribution over their four
    values: the four planner-network values sum to 1."""
    circ = lattice_circuit(2, 3, 4, 452, "haar", "cz")
    traced = (1, 2, 3, 4)
    plan = make_plan(circ, n_slices=0, B=4, projector=traced)
    tot = sum(_contract_net_host(plan.net, plan.steps, w) for w in (0b000000, 0b000001, 0b100000, 0b100001))
    assert abs(tot - 1) <= 1e-12


def test_projector_blob_accepted_and_amplitude_blob_rules_kept():
    from paper_2208_01498_amd import binding as B
    B.load_library()
    circ = lattice_circuit(3, 3, 4, 453, "haar", "cz")
    info = B.tn_plan_validate(make_plan(circ, B=2, projector=(0, 4)).to_blob())
    assert info["n_steps"] == info["n_leaves"] - 1
    # the same two-outputs-per-qubit network without the projector flag is
    # rejected
    blob = bytearray(make_plan(circ, B=2, projector=()).to_blob())
    flags_off = 4 + 6 * 4
    assert blob[flags_off] == 1
    blob[flags_off] = 0
    with pytest.raises(B.TnError):
        B.tn_plan_validate(bytes(blob))


@pytest.mark.parametrize("name,mk", CIRCS[:4], ids=[c[0] for c in CIRCS[:4]])
def test_exact_top_order_never_costs_more(name, mk):
    """The exact order of the top frontier is chosen among all pairwise
    orders of the frontier, which include the hierarchy's own order: the
    refined tree never costs more (Eq. (3) count), and the refined plan is
    still the same contraction (oracle-evaluated order equals the state
    vector)."""
    circ = mk()
    # B = 1: the exact order minimises the same count that plan_stats reports
    base = make_plan(circ, B=1, top_exact=0)
    ref = make_plan(circ, B=1, top_exact=10)
    fb = plan_stats(base.net, base.steps, B=1)["flops"]
    fr = plan_stats(ref.net, ref.steps, B=1)["flops"]
    assert fr <= fb * (1 + 1e-12)
    words = random_bitstrings(circ.n, 3, 470)
    spec = ref.order_spec()
    got = pairwise_amplitudes(circ, words, order=spec, sliced=spec["sliced"])
    assert np.max(np.abs(got - statevector_amplitudes(circ, words))) <= 1e-12


def test_seed_trials_keep_the_cheapest_sliced_plan():
    """make_plan builds one hierarchy per seed (Algorithm 1 is randomised),
    refines and slices each, and keeps the least total cost over all
    slices: never more than any single seed's plan."""
    circ = lattice_circuit(4, 5, 10, 480, "haar", "cz")
    kw = dict(n_slices=3, B=4)
    kept = make_plan(circ, trials=3, **kw).stats["total_flops_per_b"]
    singles = [make_plan(circ, seed=s, trials=1, **kw).stats["total_flops_per_b"] for s in range(3)]
    assert kept <= min(singles) * (1 + 1e-12)
    assert kept in singles


@pytest.mark.parametrize("traced", [(), (2, 6)])
def test_doubled_network_swap_form_matches_oracle(traced):
    """The doubled network built with fSim(pi/2, pi/6) as a wire exchange
    times a diagonal factor (both layers) gives the oracle's doubled
    expectation, contracted in a hierarchy order."""
    import numpy as np
    from oracle import doubled_expectation
    from paper_2208_01498_amd.planner.network import build_doubled_network
    from paper_2208_01498_amd.planner.hierarchy import TreeBuilder, tree_steps
    circ = lattice_circuit(3, 3, 4, 455, "sqrt", "fsim")
    net = build_doubled_network(circ, traced=traced, swap_relabel=True)
    root = TreeBuilder(net, np.random.Generator(np.random.PCG64(1)), bottom=8).build()
    steps = tree_steps(root, len(net.factors))
    for w in random_bitstrings(circ.n, 2, 456):
        w = int(w) & ~sum(1 << q for q in traced)
        got = _contract_net_host(net, steps, w)
        ref = doubled_expectation(circ, _projectors(circ.n, w, traced), method="statevector")
        assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-300)


@pytest.mark.parametrize("D", [2, 3, 4])
def test_lp_centerpoint_has_centerpoint_depth(D):
    """Algorithm 1's LP route: the point it returns for 16 points in R^D
    lies in no open halfspace missing more than D/(D+1) of them, i.e. every
    closed halfspace through it holds at least ceil(16/(D+1)) points
    (checked over 20000 random directions)."""
    import math
    import numpy as np
    from paper_2208_01498_amd.planner.ssa import centerpoint_lp
    for seed in range(4):
        rng = np.random.Generator(np.random.PCG64(900 + seed))
        S = rng.standard_normal((16, D)) * np.array([1.0, 3.0, 0.2, 1.0][:D])
        c = centerpoint_lp(S, rng, sample=16)
        U = rng.standard_normal((20000, D))
        U /= np.linalg.norm(U, axis=1, keepdims=True)
        depth = int(((S - c) @ U.T >= -1e-12).sum(axis=0).min())
        assert depth >= math.ceil(16 / (D + 1))


def test_lp_centerpoint_plans_are_exact():
    """A plan built with the LP centerpoint is the same contraction."""
    circ = lattice_circuit(3, 4, 6, 910, "haar", "cz")
    plan = make_plan(circ, n_slices=2, B=3, centerpoint="lp", bottom=8)
    words = random_bitstrings(circ.n, 3, 911)
    spec = plan.order_spec()
    got = pairwise_amplitudes(circ, words, order=spec, sliced=spec["sliced"])
    assert np.max(np.abs(got - statevector_amplitudes(circ, words))) <= 1e-12




def test_ssa_candidates_with_centerpoint_on_a_shared_point():
    """Coincident factor positions (here 40 of 64 points at the mean, the
    rest in symmetric pairs) put the LP centerpoint on the shared point,
    which the rotation sends to the pole where the dilation is undefined:
    the candidates still come out finite, with no division warning."""
    import warnings
    g = np.random.Generator(np.random.PCG64(5))
    half = g.standard_normal((12, 2)) * 2.0
    pts = np.vstack([np.zeros((40, 2)), half, -half])
    radii = np.full(len(pts), 0.26)
    # the case is reached: the centerpoint of the projected points is the
    # image of the shared point, the south pole of S^2
    mu = pts.mean(axis=0)
    y = ssa.stereo((pts - mu) / np.max(np.linalg.norm(pts - mu, axis=1)))
    c = ssa.centerpoint_lp(y, np.random.Generator(np.random.PCG64(900)))
    assert np.linalg.norm(c - np.array([0.0, 0.0, -1.0])) < 1e-9
    with warnings.catch_warnings():
        warnings.simplefilter("error", RuntimeWarning)
        seps = ssa.ssa_candidates(pts, radii, np.random.Generator(np.random.PCG64(900)),
                                  n_circles=24, method="lp")
    assert seps
    for kind, a, b in seps:
        assert np.all(np.isfinite(a)) and np.isfinite(b)


@pytest.mark.parametrize("name,mk", CIRCS[:5], ids=[c[0] for c in CIRCS[:5]])
def test_planar_separator_plans_are_exact(name, mk):
    """Plans whose hierarchy comes from planar level separators (qubit-graph
    BFS levels) are the same contraction, evaluated by the oracle in their
    order, with slices."""
    circ = mk()
    words = random_bitstrings(circ.n, 3, 930)
    plan = make_plan(circ, n_slices=2, B=3, separators="planar", bottom=8)
    spec = plan.order_spec()
    got = pairwise_amplitudes(circ, words, order=spec, sliced=spec["sliced"])
    ref = statevector_amplitudes(circ, words)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_planar_levels_are_balanced_and_thin_on_a_lattice():
    """On an 8x8 lattice network the first planar level split leaves at most
    2n/3 leaves on either side and its separator is one BFS front of the
    qubit lattice: at most 8 qubits (sqrt(N) for N = 64); nearly every later
    split is balanced too."""
    from paper_2208_01498_amd.planner.planar import PlanarTreeBuilder
    circ = lattice_circuit(8, 8, 8, 931, "haar", "cz")
    net = build_network(circ)
    tb = PlanarTreeBuilder(net, np.random.Generator(np.random.PCG64(0)), bottom=8)
    idx = list(range(len(net.factors)))
    A, B, balanced = tb.level_split(idx)
    assert balanced
    n = len(idx)
    assert max(len(A), len(B)) <= 2 * n / 3 + 1e-9 and len(A) + len(B) == n
    qa = set().union(*(tb._qubits(i) for i in A))
    qb = set().union(*(tb._qubits(i) for i in B))
    assert len(qa & qb) <= 8
    # deeper down, a few small clusters have no level that balances them
    # (the cycle phase of the Lipton-Tarjan construction is not built)
    tb.build(idx)
    assert tb.split_sources["planar"] >= 10 * tb.split_sources["planar_unbalanced"]


def test_split_sources_are_counted():
    """The kept hierarchy reports where its splits came from; without the
    median planes none comes from them."""
    circ = make_config("cfg1")[0]
    a = make_plan(circ, n_slices=0, B=8)
    b = make_plan(circ, n_slices=0, B=8, separators="ssa")
    assert sum(a.stats["split_sources"][k] for k in ("ssa", "plane", "time")) >= 1
    assert a.stats["split_sources"]["ssa_eq1"] <= a.stats["split_sources"]["ssa"]
    assert b.stats["split_sources"]["plane"] == 0
