"""Pins of the oracle's sGS-ADMM loop (Algorithm 1) and of the whole relaxation (CPU only).

* textbook SDPs with closed-form optima: min <C,X> s.t. tr X = 1 has optimum lambda_min(C);
  a linear program written with 1x1 blocks, checked by enumerating its vertices;
* invariants of Algorithm 1: with tau = 1 every iterate satisfies A(X) = b (step 4 with the
  exact y-solve of step 3), S stays PSD;
* tiny trajectory problems (the paper's toy system, the pendulum) against a brute-force
  grid search over the controls: the relaxation value is a lower bound
  (convergence theorem (ii)) and, when every moment matrix is rank one, equals the global
  optimum (theorem (iii)) and its degree-one moments are the optimal trajectory.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.optimize as so


def _svec(a):
    n = a.shape[0]
    return np.array([a[i, j] * (1 if i == j else math.sqrt(2)) for j in range(n) for i in range(j + 1)])


def _smat(v, n):
    a = np.zeros((n, n))
    k = 0
    for j in range(n):
        for i in range(j + 1):
            a[i, j] = a[j, i] = v[k] * (1 if i == j else 1 / math.sqrt(2))
            k += 1
    return a


def _sdp(orc, sizes, A_dense, b, C):
    import scipy.sparse as sp
    A = sp.csr_matrix(A_dense)
    return orc.SDP(nblocks=len(sizes), bsize=np.array(sizes, dtype=np.int32), m=A.shape[0],
                   nsvec=A.shape[1], rowptr=A.indptr.astype(np.int64), col=A.indices.astype(np.int32),
                   val=A.data.astype(np.float64), b=np.asarray(b, float), C=np.asarray(C, float))


def test_trace_sdp_min_eigenvalue(orc):
    rng = np.random.default_rng(11)
    for n in [3, 6, 9]:
        Cm = rng.standard_normal((n, n)); Cm = Cm + Cm.T
        s = _sdp(orc, [n], _svec(np.eye(n))[None, :], [1.0], _svec(Cm))
        r = orc.admm_solve(s, tol=1e-10, maxiter=20000)
        lmin = np.linalg.eigvalsh(Cm)[0]
        assert r["converged"]
        assert abs(r["pobj"] - lmin) <= 1e-8 * (1 + abs(lmin))
        assert abs(r["dobj"] - lmin) <= 1e-8 * (1 + abs(lmin))


def test_two_block_trace_sdp(orc):
    rng = np.random.default_rng(12)
    C1 = rng.standard_normal((4, 4)); C1 += C1.T
    C2 = rng.standard_normal((7, 7)); C2 += C2.T
    row = np.concatenate([_svec(np.eye(4)), _svec(np.eye(7))])
    s = _sdp(orc, [4, 7], row[None, :], [1.0], np.concatenate([_svec(C1), _svec(C2)]))
    r = orc.admm_solve(s, tol=1e-10, maxiter=50000)
    want = min(np.linalg.eigvalsh(C1)[0], np.linalg.eigvalsh(C2)[0])
    assert abs(r["pobj"] - want) <= 1e-7 * (1 + abs(want))


def test_lp_with_scalar_blocks_vertex_enumeration(orc):
    rng = np.random.default_rng(13)
    m, n = 3, 7
    A = rng.standard_normal((m, n))
    b = A @ rng.uniform(0.5, 1.5, n)
    c = rng.uniform(0.2, 2.0, n) + A.T @ rng.standard_normal(m) * 0.3
    best = np.inf
    for basis in itertools.combinations(range(n), m):
        B = A[:, basis]
        if abs(np.linalg.det(B)) < 1e-12:
            continue
        xb = np.linalg.solve(B, b)
        if (xb >= -1e-12).all():
            best = min(best, c[list(basis)] @ xb)
    s = _sdp(orc, [1] * n, A, b, c)
    r = orc.admm_solve(s, tol=1e-10, maxiter=100000)
    assert r["converged"]
    assert abs(r["pobj"] - best) <= 1e-7 * (1 + abs(best))
    assert (r["X"] >= -1e-9).all()


def test_tau_one_keeps_primal_feasible(orc):
    sdp = orc.relax(orc.PENDULUM, 3, [0.7, 0.0])
    for k in [1, 2, 5]:
        r = orc.admm_solve(sdp, tau=1.0, maxiter=k, sigma_every=0, tol=0.0)
        assert np.linalg.norm(sdp.A @ r["X"] - sdp.b) <= 1e-9
        off = 0
        for n in sdp.bsize:
            t = n * (n + 1) // 2
            assert np.linalg.eigvalsh(_smat(r["S"][off:off + t], n)).min() >= -1e-10
            off += t


# ----------------------------------------------------------------- brute force on tiny POPs

def _toy_cost(u, x0=2.0, dt=0.1, Pf=1.0):
    u = np.atleast_2d(u)
    x = np.full(u.shape[0], x0)
    J = np.zeros(u.shape[0])
    for k in range(u.shape[1]):
        J += u[:, k] ** 2 + x ** 2
        x = x - dt * (1 + u[:, k]) * x
    return J + Pf * x ** 2


def _pend_cost(u, th0):
    """Pendulum from upright angle th0 at rest: omega' = omega + dt(g/l sin th - b omega/(ml^2)
    + u/(ml^2)); the heading turns by 2 atan(dt omega / 2) (Cayley step); cost
    (1-cos th)^2 + 0.1 omega^2 + 0.01 u^2 per step plus the terminal (1-cos th)^2 + 0.1 omega^2."""
    m = l = 1.0; b = 0.1; g = 9.8; dt = 0.1
    u = np.atleast_2d(u)
    th = np.full(u.shape[0], th0); w = np.zeros(u.shape[0]); J = np.zeros(u.shape[0])
    for k in range(u.shape[1]):
        J += (1 - np.cos(th)) ** 2 + 0.1 * w ** 2 + 0.01 * u[:, k] ** 2
        w_new = w + dt * (g / l * np.sin(th) - b / (m * l * l) * w + u[:, k] / (m * l * l))
        th = th + 2 * np.arctan(dt * w / 2)
        w = w_new
    return J + (1 - np.cos(th)) ** 2 + 0.1 * w ** 2


def _brute(cost, N, umax, pts=201):
    grid = np.linspace(-umax, umax, pts)
    U = np.array(list(itertools.product(grid, repeat=N)))
    J = cost(U)
    best = (np.inf, None)
    for i in np.argsort(J)[:8]:
        res = so.minimize(lambda v: cost(v[None, :])[0], U[i], bounds=[(-umax, umax)] * N,
                          method="L-BFGS-B", options={"ftol": 1e-15, "gtol": 1e-12})
        if res.fun < best[0]:
            best = (res.fun, res.x)
    return best


def _moment_blocks(sdp, X):
    out = []
    for bk in range(sdp.nblocks):
        if sdp.bkind[bk] == 0:
            n = int(sdp.bsize[bk]); off = int(sdp.boff[bk])
            out.append(_smat(X[off:off + n * (n + 1) // 2], n))
    return out


@pytest.mark.parametrize("N", [1, 2, 3])
def test_toy_relaxation_vs_brute_force(orc, N):
    """The worked-example system: lower bound, and here also equal to the global optimum
    (the optimal face contains higher-rank points, so rank one is not asserted)."""
    sdp = orc.relax(orc.TOY1D, N, [2.0, 0.1, 1.0])
    pstar, _ = _brute(_toy_cost, N, 1.0, 201 if N < 3 else 61)
    r = orc.admm_solve(sdp, tol=1e-9, maxiter=100000)
    assert r["converged"]
    assert r["pobj"] <= pstar + 1e-7 * (1 + abs(pstar))
    assert abs(r["pobj"] - pstar) <= 1e-6 * (1 + abs(pstar))


@pytest.mark.parametrize("th0,N", [(2.5, 1), (2.5, 2), (0.5, 2), (3.0, 2)])
def test_pendulum_relaxation_vs_brute_force(orc, th0, N):
    sdp = orc.relax(orc.PENDULUM, N, [th0, 0.0])
    pstar, uopt = _brute(lambda U: _pend_cost(U, th0), N, 2.0)
    r = orc.admm_solve(sdp, tol=1e-9, maxiter=100000)
    assert r["converged"]
    pk = r["pobj"]
    assert pk <= pstar + 1e-7 * (1 + abs(pstar))            # lower bound
    Ms = _moment_blocks(sdp, r["X"])
    ratios = [np.linalg.eigvalsh(M)[-2] / np.linalg.eigvalsh(M)[-1] for M in Ms]
    assert max(ratios) <= 1e-4                               # rank one ...
    assert abs(pk - pstar) <= 1e-6 * (1 + abs(pstar))         # ... hence tight
    # degree-one moments of clique k = (x_k, u_k, x_{k+1}): u_k/2 sits at index dx + 1
    ubar = np.array([M[0, 1 + sdp.dx] for M in Ms]) * 2.0
    assert np.allclose(ubar, uopt, atol=2e-3)
