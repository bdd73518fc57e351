"""Pins of the oracle's KKT residuals (the termination rule after Algorithm 1, Sec. "Algorithmic
Backbone"): the checker every converged GPU test relies on.

* a hand-computed case: one 2x2 block and two rows with chosen A, b, C, X, y, S, whose residuals
  were worked out on the dense matrices (not on svec vectors), so a wrong normalization, a dropped
  S, a missing sqrt(2) on an off-diagonal or a squared norm changes the result;
* an exact KKT point in closed form (min <C,X> s.t. tr X = 1: X = v v^T for the eigenvector of
  lambda_min(C), y = lambda_min, S = C - y I) has zero residuals;
* orc_kkt on the final (X, y, S) of a solve equals the residuals the solve reports itself.
"""
import math

import numpy as np


def _svec(a):
    n = a.shape[0]
    return np.array([a[i, j] * (1 if i == j else math.sqrt(2)) for j in range(n) for i in range(j + 1)])


def _sdp(orc, sizes, A_rows, b, C):
    import scipy.sparse as sp
    A = sp.csr_matrix(np.asarray(A_rows, dtype=float))
    return orc.SDP(nblocks=len(sizes), bsize=np.array(sizes, dtype=np.int32), m=A.shape[0],
                   nsvec=A.shape[1], rowptr=A.indptr.astype(np.int64), col=A.indices.astype(np.int32),
                   val=A.data.astype(np.float64), b=np.asarray(b, float), C=np.asarray(C, float))


def test_kkt_hand_computed_case(orc):
    # Dense data:  A_1 = I, A_2 = [[0,1],[1,0]], b = (2, 0.4), C = [[1,0.3],[0.3,0]],
    #              X = [[1,0.5],[0.5,2]], y = (0.25, 0.1), S = [[0.5,0.1],[0.1,0]].
    # By hand:  A(X) = (tr X, 2 X_12) = (3, 1), so A(X) - b = (1, 0.6): ||.||^2 = 1.36, ||b||^2 = 4.16.
    #           A^*y + S - C = [[0.25+0.5-1, 0.1+0.1-0.3], [., 0.25]] = [[-0.25,-0.1],[-0.1,0.25]]:
    #           squared Frobenius norm 0.145;  ||C||_F^2 = 1 + 2 * 0.09 = 1.18.
    #           <C,X> = 1 + 2 * 0.3 * 0.5 = 1.3;  <b,y> = 0.5 + 0.04 = 0.54.
    A_rows = [_svec(np.eye(2)), _svec(np.array([[0.0, 1.0], [1.0, 0.0]]))]
    C = _svec(np.array([[1.0, 0.3], [0.3, 0.0]]))
    sdp = _sdp(orc, [2], A_rows, [2.0, 0.4], C)
    X = _svec(np.array([[1.0, 0.5], [0.5, 2.0]]))
    S = _svec(np.array([[0.5, 0.1], [0.1, 0.0]]))
    k = orc.kkt(sdp, X, np.array([0.25, 0.1]), S)
    assert abs(k["eta_p"] - math.sqrt(1.36) / (1 + math.sqrt(4.16))) <= 1e-15
    assert abs(k["eta_d"] - math.sqrt(0.145) / (1 + math.sqrt(1.18))) <= 1e-15
    assert abs(k["eta_g"] - 0.76 / 2.84) <= 1e-15
    assert abs(k["pobj"] - 1.3) <= 1e-15 and abs(k["dobj"] - 0.54) <= 1e-15
    assert k["eta"] == max(k["eta_p"], k["eta_d"], k["eta_g"])


def test_kkt_zero_at_closed_form_optimum(orc):
    rng = np.random.default_rng(21)
    for n in [2, 5, 9]:
        Cm = rng.standard_normal((n, n)); Cm = Cm + Cm.T
        w, V = np.linalg.eigh(Cm)
        v = V[:, 0]
        sdp = _sdp(orc, [n], [_svec(np.eye(n))], [1.0], _svec(Cm))
        k = orc.kkt(sdp, _svec(np.outer(v, v)), np.array([w[0]]), _svec(Cm - w[0] * np.eye(n)))
        assert max(k["eta_p"], k["eta_d"], k["eta_g"]) <= 1e-14, k
        assert abs(k["pobj"] - w[0]) <= 1e-13 * (1 + abs(w[0]))
        # moving y off the optimum by d shows up in eta_d (||d I||_F = d sqrt(n)) and in the gap
        d = 1e-3
        k2 = orc.kkt(sdp, _svec(np.outer(v, v)), np.array([w[0] + d]), _svec(Cm - w[0] * np.eye(n)))
        assert abs(k2["eta_d"] - d * math.sqrt(n) / (1 + np.linalg.norm(Cm))) <= 1e-13
        assert abs(k2["eta_g"] - d / (1 + abs(w[0]) + abs(w[0] + d))) <= 1e-13


def test_kkt_agrees_with_the_solver_report(orc):
    sdp = orc.relax(orc.PENDULUM, 3, [0.7, 0.0])
    for iters in [1, 7, 40]:
        r = orc.admm_solve(sdp, maxiter=iters, tol=0.0)
        k = orc.kkt(sdp, r["X"], r["y"], r["S"])
        for f in ("eta_p", "eta_d", "eta_g", "pobj", "dobj"):
            assert abs(k[f] - r[f]) <= 1e-12 * max(1.0, abs(r[f])), (iters, f, k[f], r[f])
