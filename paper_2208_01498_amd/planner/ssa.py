"""Sphere Separator Algorithm (Algorithm 1 of the supplemental material) and
the separator checks of the Sphere Separator Theorem, Eqs. (1)-(2).

Steps, in the paper's order:
  1. stereographic projection Pi of the sphere centres onto S^d in R^{d+1};
  2. an approximate centerpoint c of the projected points: the paper's
     route, a linear program over a random subset (`centerpoint_lp`), or
     iterated Radon points of random subsets (`centerpoint`, a standard
     randomized approximation);
  3. an orthogonal R with R c = (0, ..., 0, |c|);
  4. the dilation D_alpha = Pi o (alpha 1) o Pi^{-1},
     alpha = sqrt((1 - |c|)/(1 + |c|));
  5. a random great circle C of S^d;
  6. S = Pi^{-1} o R^T o D_alpha^{-1}(C), a sphere (or hyperplane) of R^d;
  7. accept S if |Gamma_O| <= c_d k^{1/d} n^{1-1/d} and
     |Gamma_E|, |Gamma_I| <= (d+1)/(d+2) n, counting a sphere of radius r_i
     as cut when its centre lies within r_i of S; otherwise retry with a new
     great circle.
"""
import numpy as np

C_D = {1: 1.0, 2: 2.0, 3: 2.135, 4: 2.280, 5: 2.421}


def stereo(x):
    """Pi: R^d -> S^d,  x -> (2x, |x|^2 - 1) / (|x|^2 + 1)."""
    s = np.sum(x * x, axis=-1, keepdims=True)
    return np.concatenate([2 * x, s - 1], axis=-1) / (s + 1)


def stereo_inv(y):
    """Pi^{-1}: S^d minus the pole (0,...,0,1) -> R^d."""
    return y[..., :-1] / (1 - y[..., -1:])


def radon_point(P):
    """Radon point of d+2 points in R^d (rows of P)."""
    m, d = P.shape
    A = np.vstack([P.T, np.ones((1, m))])
    _, _, vt = np.linalg.svd(A)
    lam = vt[-1]
    pos = lam > 0
    if not np.any(pos) or np.all(pos):
        return P.mean(axis=0)
    return (lam[pos] @ P[pos]) / lam[pos].sum()


def centerpoint(P, rng, rounds=None):
    """Iterated Radon points: repeatedly replace random groups of d+2 points
    by their Radon point until one point remains."""
    m, d = P.shape
    g = d + 2
    pts = P[rng.permutation(m)]
    size = g ** max(1, int(np.ceil(np.log(max(m, g)) / np.log(g))))
    if len(pts) < size:
        extra = pts[rng.integers(0, len(pts), size - len(pts))]
        pts = np.vstack([pts, extra])
    else:
        pts = pts[:size]
    while len(pts) > 1:
        pts = np.array([radon_point(pts[i:i + g]) for i in range(0, len(pts), g)])
    return pts[0]


def centerpoint_lp(P, rng, sample=16):
    """Centerpoint of a random subset of the points by linear programming.
    A point of R^D is a centerpoint of a set of a points when every closed
    halfspace containing it holds at least a/(D+1) of them; equivalently it
    lies in every closed halfspace holding more than a D/(D+1) of them.  The
    halfspaces used are those bounded by hyperplanes through D of the
    subset's points (both sides); the LP finds a point in their
    intersection, which Helly's theorem makes non-empty.  Falls back to
    iterated Radon points if the solver finds none (degenerate subsets)."""
    from itertools import combinations
    from scipy.optimize import linprog
    m, D = P.shape
    S = P[rng.choice(m, size=min(sample, m), replace=False)]
    a = len(S)
    if a <= D:
        return S.mean(axis=0)
    thr = a * D / (D + 1)
    rows, rhs = [], []
    scale = max(1.0, float(np.max(np.abs(S))))
    for comb in combinations(range(a), D):
        Q = S[list(comb)]
        M = Q[1:] - Q[0]
        _, sv, vt = np.linalg.svd(M, full_matrices=True)
        if len(sv) and sv.min() < 1e-9 * scale:
            continue                       # the D points span less than a hyperplane
        nrm = vt[-1]
        off = float(nrm @ Q[0])
        s = S @ nrm - off
        tol = 1e-12 * scale
        for sign in (1.0, -1.0):
            if np.count_nonzero(sign * s >= -tol) > thr:
                # sign * (nrm . c - off) >= 0
                rows.append(-sign * nrm)
                rhs.append(-sign * off)
    if not rows:
        return centerpoint(P, rng)
    res = linprog(np.zeros(D), A_ub=np.array(rows), b_ub=np.array(rhs),
                  bounds=[(None, None)] * D, method="highs")
    if res.status != 0:
        return centerpoint(P, rng)
    return res.x


def _householder_to_pole(c):
    """Orthogonal R with R c = (0, ..., 0, |c|)."""
    D = len(c)
    nc = np.linalg.norm(c)
    if nc < 1e-15:
        return np.eye(D)
    u = c / nc
    e = np.zeros(D)
    e[-1] = 1.0
    v = u - e
    if np.linalg.norm(v) < 1e-15:
        return np.eye(D)
    v /= np.linalg.norm(v)
    return np.eye(D) - 2 * np.outer(v, v)


def _dilate(y, alpha):
    """D_alpha on points of S^d."""
    return stereo(alpha * stereo_inv(y))


def _fit_sphere(Q):
    """Sphere (centre, radius) through d+1 points of R^d, or a hyperplane
    (normal, offset) when they are (nearly) affinely dependent on a plane."""
    m, d = Q.shape
    A = np.hstack([2 * Q, np.ones((m, 1))])
    b = np.sum(Q * Q, axis=1)
    try:
        sol, res, rank, sv = np.linalg.lstsq(A, b, rcond=None)
    except np.linalg.LinAlgError:
        sol, rank, sv = None, 0, [0]
    if sol is None or rank < d + 1 or sv[-1] / sv[0] < 1e-9:
        X = Q - Q.mean(axis=0)
        _, _, vt = np.linalg.svd(X)
        nrm = vt[-1]
        return ("plane", nrm, float(nrm @ Q.mean(axis=0)))
    ctr = sol[:d]
    r2 = sol[d] + ctr @ ctr
    if r2 <= 0 or np.sqrt(r2) > 1e6:
        X = Q - Q.mean(axis=0)
        _, _, vt = np.linalg.svd(X)
        nrm = vt[-1]
        return ("plane", nrm, float(nrm @ Q.mean(axis=0)))
    return ("sphere", ctr, float(np.sqrt(r2)))


def classify(sep, pts, radii):
    """-1 inside (Gamma_I), +1 outside (Gamma_E), 0 cut (Gamma_O)."""
    kind, a, b = sep
    if kind == "sphere":
        dist = np.linalg.norm(pts - a, axis=1) - b
    else:
        dist = pts @ a - b
    out = np.where(dist > 0, 1, -1)
    out[np.abs(dist) < radii] = 0
    return out


def max_overlap(pts, radii):
    """k: the largest number of spheres containing any sphere centre (an
    estimate of the ply of the sphere set)."""
    if len(pts) == 0:
        return 1
    d2 = np.sum((pts[:, None, :] - pts[None, :, :]) ** 2, axis=-1)
    return int(np.max(np.sum(d2 <= (radii[None, :] ** 2), axis=1)))


def eq_checks(side, d, k):
    n = len(side)
    nO = int(np.sum(side == 0))
    nE = int(np.sum(side == 1))
    nI = int(np.sum(side == -1))
    ok1 = nO <= C_D.get(d, 2.5) * k ** (1.0 / d) * n ** (1.0 - 1.0 / d)
    ok2 = max(nE, nI) <= (d + 1) / (d + 2) * n
    return ok1, ok2


def ssa_candidates(pts, radii, rng, n_circles=24, method="radon"):
    """Separator candidates from Algorithm 1 (one centerpoint, several random
    great circles).  Returns a list of separators (see classify).
    `method`: centerpoint by iterated Radon points ("radon") or by the LP
    over a random subset ("lp")."""
    m, d = pts.shape
    mu = pts.mean(axis=0)
    sc = np.max(np.linalg.norm(pts - mu, axis=1))
    sc = sc if sc > 0 else 1.0
    x = (pts - mu) / sc
    y = stereo(x)                                            # step 1
    c = centerpoint_lp(y, rng) if method == "lp" else centerpoint(y, rng)   # step 2
    R = _householder_to_pole(c)                              # step 3
    nc = min(np.linalg.norm(c), 1 - 1e-9)
    alpha = np.sqrt((1 - nc) / (1 + nc))                     # step 4
    yr = y @ R.T
    # choose the dilation direction that centres the points (the map moves
    # the point (0,..,0,|c|) to the origin for one of alpha, 1/alpha).  A
    # centerpoint on a data point that several factors share (coincident
    # positions) puts those points on the pole, where the map is undefined:
    # they are left out of the score
    best = None
    for a in (alpha, 1.0 / alpha):
        with np.errstate(divide="ignore", invalid="ignore"):
            z = _dilate(yr, a)
        z = z[np.all(np.isfinite(z), axis=1)]
        score = np.linalg.norm(z.mean(axis=0)) if len(z) else np.inf
        if best is None or score < best[0]:
            best = (score, a)
    a = best[1]
    seps = []
    D = d + 1
    for _ in range(n_circles):
        u = rng.standard_normal(D)                           # step 5
        u /= np.linalg.norm(u)
        # d+1 points on the great circle {y : u.y = 0}
        basis = np.linalg.svd(u[None, :])[2][1:]             # orthonormal complement
        coef = rng.standard_normal((d + 1, d))
        coef /= np.linalg.norm(coef, axis=1, keepdims=True)
        on = coef @ basis                                    # points of S^d with u.y = 0
        with np.errstate(divide="ignore", invalid="ignore"):
            back = _dilate(on, 1.0 / a) @ R                   # step 6: D^{-1}, then R^T
            back = np.clip(back, -1, 1 - 1e-12)
            Q = stereo_inv(back) * sc + mu
        if not np.all(np.isfinite(Q)):
            continue                                         # circle through the pole
        seps.append(_fit_sphere(Q))
    return seps


def plane_candidates(pts):
    """Median coordinate hyperplanes (spheres of infinite radius)."""
    m, d = pts.shape
    seps = []
    for ax in range(d):
        v = np.sort(pts[:, ax])
        for q in (0.5, 0.45, 0.55):
            t = v[min(len(v) - 1, int(q * len(v)))]
            nrm = np.zeros(d)
            nrm[ax] = 1.0
            # put the cut between distinct coordinate values
            lo = v[v <= t].max() if np.any(v <= t) else t
            hi = v[v > t].min() if np.any(v > t) else t
            seps.append(("plane", nrm, 0.5 * (lo + hi)))
    return seps
