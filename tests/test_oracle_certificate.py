"""Pins of the oracle's certificate pieces (oracle/cert.c), against what the paper and the
mathematics fix:

* the valid lower bound (refined certificate of suboptimality, Sec. "Algorithmic Backbone"):
  lb(y) <= <C, X(z)> = f(z) for ANY y and any feasible z, once R_beta bounds the traces of the
  rank-one lifting's blocks (here R_beta = those traces, and twice them);
* at y = 0 the bound is sum_beta R_beta min(0, lambda_min(C_beta)), checked against numpy's
  eigvalsh (a library routine, independent of the oracle's Jacobi);
* extraction (Sec. "Sparse Moment Relaxation"): the moment blocks of the lifting X(z) are rank
  one, and the top eigenvector scaled to first entry 1 carries z's clique variables as its
  degree-one entries (the basis is graded, degree one in variable order).
"""
import numpy as np
import pytest

CASES = [("PENDULUM", 4, [0.5, 0.0]), ("CARTPOLE", 3, [0.1, 0.2, 0.5, 0.3]),
         ("CAR", 3, [1, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1]), ("PAPER_CARTPOLE", 3, [0.1, 0.2, 0.3, 0.5])]


def _block_traces(sdp, X):
    tr, off = [], 0
    for n in sdp.bsize:
        n = int(n)
        tr.append(sum(X[off + j * (j + 1) // 2 + j] for j in range(n)))
        off += n * (n + 1) // 2
    return np.array(tr)


def _feasible(orc, f, N, prm, seed):
    sdp = orc.relax(f, N, prm)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.5, 0.5, N * sdp.du)
    z, obj = orc.rollout(f, N, prm, u, sdp.dx, sdp.du)
    X, _ = orc.lift(f, N, prm, z)
    return sdp, z, X, obj


@pytest.mark.parametrize("fam,N,prm", CASES)
def test_dual_bound_below_feasible_objective(orc, fam, N, prm):
    f = getattr(orc, fam)
    sdp, z, X, obj = _feasible(orc, f, N, prm, 3)
    tr = _block_traces(sdp, X)
    assert np.all(tr >= -1e-12)
    rng = np.random.default_rng(11)
    for scale in [0.1, 1.0, 10.0]:
        y = scale * rng.standard_normal(sdp.m)
        for R in (tr, 2.0 * tr):
            lb, lam = orc.dual_bound(sdp, y, R)
            assert lb <= obj + 1e-9 * (1 + abs(obj)), (scale, lb, obj)
        # the bound decomposes as <b,y> + sum R min(0, lam)
        assert abs(lb - (sdp.b @ y + np.sum(2.0 * tr * np.minimum(0.0, lam)))) <= 1e-9 * (1 + abs(lb))


def test_dual_bound_at_zero_is_the_spectrum_of_C(orc):
    sdp = orc.relax(orc.PENDULUM, 3, [0.5, 0.0])
    R = np.linspace(1.0, 2.0, sdp.nblocks)
    lb, lam = orc.dual_bound(sdp, np.zeros(sdp.m), R)
    off, ref = 0, []
    for n in sdp.bsize:
        n = int(n)
        a = np.zeros((n, n))
        for j in range(n):
            for i in range(j + 1):
                v = sdp.C[off + j * (j + 1) // 2 + i] * (1.0 if i == j else np.sqrt(0.5))
                a[i, j] = a[j, i] = v
        ref.append(np.linalg.eigvalsh(a)[0])
        off += n * (n + 1) // 2
    ref = np.array(ref)
    assert np.allclose(lam, ref, atol=1e-12 * max(1.0, np.abs(sdp.C).max()))
    assert abs(lb - np.sum(R * np.minimum(0.0, ref))) <= 1e-12 * (1 + abs(lb))


@pytest.mark.parametrize("fam,N,prm", CASES)
def test_extract_recovers_the_lifted_point(orc, fam, N, prm):
    f = getattr(orc, fam)
    sdp, z, X, _ = _feasible(orc, f, N, prm, 5)
    moment = [k for k in range(sdp.nblocks) if sdp.bkind[k] == 0]
    assert len(moment) == N
    lam, vt = orc.extract(sdp, X, moment)
    d = sdp.nclique_vars
    for t, k in enumerate(moment):
        assert lam[t, 1] <= 1e-12 * lam[t, 0]  # rank one
        zk = orc.clique_vars(sdp, z, int(sdp.bclique[k]))
        assert len(zk) == d
        assert abs(vt[t][0] - 1.0) <= 1e-14
        assert np.allclose(vt[t][1:1 + d], zk, atol=1e-10 * max(1.0, np.abs(zk).max()))


def test_warm_start_shifted_horizon_reaches_the_cold_optimum(orc):
    """Receding horizon: the problem one step later (initial state from the extracted z of
    clique 0), started from the previous X and S shifted by one clique and the previous final
    sigma, converges to the optimum of the cold start (Algorithm 1 takes any X0, S0 and sigma0)."""
    import math
    import workloads as W
    N = 6
    sdp0 = orc.relax(W.PENDULUM, N, [2.0, 0.0])
    r0 = orc.admm_solve(sdp0, tol=1e-7, maxiter=50000)
    assert r0["converged"]
    _, vt = orc.extract(sdp0, r0["X"], [0])
    sdp1 = orc.relax(W.PENDULUM, N, [math.atan2(vt[0][6], vt[0][5]), 8.0 * vt[0][7]])
    bs = [int(n) for n in sdp1.bsize]
    cold = orc.admm_solve(sdp1, tol=1e-7, maxiter=50000)
    warm = orc.admm_solve(sdp1, X0=W.shift_one_clique(bs, r0["X"]), S0=W.shift_one_clique(bs, r0["S"]),
                          sigma0=r0["sigma"], tol=1e-7, maxiter=50000)
    assert cold["converged"] and warm["converged"]
    assert abs(warm["pobj"] - cold["pobj"]) <= 1e-5 * (1.0 + abs(cold["pobj"]))


@pytest.mark.parametrize("fam,N,prm", [("CARTPOLE", 4, [0.1, 0.2, 0.5, 0.3]), ("CARTPOLE", 3, [-0.4, 0.5, 2.9, -1.0]),
                                       ("CAR", 3, [0, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1]),
                                       ("CAR", 3, [1, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1]),
                                       ("PAPER_PENDULUM", 3, [0.3, 0.5]), ("TOY1D", 4, [2.0, 0.1, 1.0]),
                                       ("PAPER_CARTPOLE", 3, [0.1, 0.2, 0.3, 0.5]),
                                       ("PAPER_CARTPOLE", 2, [-0.4, 0.5, -0.3, 0.9])])
def test_trace_bounds_hold_for_feasible_points(orc, fam, N, prm):
    """App. "Existence of R_beta" (with the proof's dropped square restored): every block of the
    rank-one lifting of a feasible trajectory has trace <= R_beta.  Feasible points: rollouts of
    random controls inside the control box, kept when every inequality holds (their lifted
    localizing blocks are then PSD with nonnegative diagonals)."""
    f = getattr(orc, fam)
    R = orc.trace_bounds(f, N, prm)
    sdp = orc.relax(f, N, prm)
    assert R is not None and len(R) == sdp.nblocks and np.all(R > 0)
    rng = np.random.default_rng(7)
    kept = 0
    for trial in range(200):
        u = rng.uniform(-1.0, 1.0, N * sdp.du) * rng.uniform(0.0, 1.0)
        z, _ = orc.rollout(f, N, prm, u, sdp.dx, sdp.du)
        if not np.all(np.isfinite(z)):
            continue
        X, _ = orc.lift(f, N, prm, z)
        tr = _block_traces(sdp, X)
        if np.any(tr[sdp.bkind == 1] < 0):  # an inequality fails: not a feasible point
            continue
        kept += 1
        assert np.all(tr <= R * (1 + 1e-12)), (trial, np.max(tr / R))
    assert kept >= 20


def test_trace_bounds_hold_on_the_variable_box(orc):
    """The car back-in, whose separation inequalities are products of two variables (their
    localizing bounds take |c| R^2 for each product term): the traces of the lifting stay below
    R_beta at points anywhere in the box of the variable bounds, feasible or not (the bound needs
    only |z_v| <= R_k), including its corners, where the products reach their largest values."""
    prm = [3.0, 4.0, 0.1]
    N = 2
    R = orc.trace_bounds(orc.BACKIN, N, prm)
    sdp = orc.relax(orc.BACKIN, N, prm)
    assert R is not None and len(R) == sdp.nblocks
    dx, du = sdp.dx, sdp.du
    bx = np.array([(abs(prm[0]) + 2) / 10, max(8.0, abs(prm[1])) / 10, 1.0, 1.0])
    bu = np.ones(du)
    box = np.concatenate([np.concatenate([bx, bu]) for _ in range(N)] + [bx])
    rng = np.random.default_rng(5)
    worst = 0.0
    for trial in range(300):
        if trial < 100:  # corners
            z = box * rng.choice([-1.0, 1.0], size=box.size)
        else:
            z = box * rng.uniform(-1.0, 1.0, size=box.size)
        X, _ = orc.lift(orc.BACKIN, N, prm, z)
        tr = _block_traces(sdp, X)
        worst = max(worst, float(np.max(tr / R)))
        assert np.all(tr <= R * (1 + 1e-12)), (trial, np.max(tr / R))
    assert worst > 0.1  # the corners come within an order of magnitude of the bound


def test_trace_bounds_need_bounded_variables(orc):
    assert orc.trace_bounds(orc.PENDULUM, 3, [0.5, 0.0]) is None  # the angular rate has no bound
