"""Pins of the oracle's Jacobi projection and sparse LDL^T (CPU only).

Projection (parallel PSD cone projection of Sec. "GPU Speedup": eig, clamp, rebuild):
closed forms (diagonal, 2x2, PSD -> identity, NSD -> 0, +-rank one), idempotence,
Moreau decomposition X = Pi(X) - Pi(-X) with orthogonal parts, and a cross-check against
numpy.linalg.eigh used as an independent library reference.
LDL^T (hybrid solver equation, eps I + A A^* = P L D L^T P^T): residual of the solve and a
dense solve on small instances.
"""
import numpy as np
import pytest


def _sym(rng, n, spectrum=None):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    if spectrum is None:
        spectrum = rng.standard_normal(n)
    return (Q * spectrum) @ Q.T


def _proj_ref(a):
    w, V = np.linalg.eigh(a)
    return (V * np.maximum(w, 0)) @ V.T


def test_jacobi_eigenpairs(orc):
    rng = np.random.default_rng(1)
    for n in [1, 2, 3, 8, 13, 36, 55, 78]:
        a = _sym(rng, n)
        w, V, sweeps = orc.jacobi_eig(a)
        assert sweeps < 30
        assert np.allclose(np.sort(w), np.linalg.eigvalsh(a), atol=1e-13 * max(1, np.abs(a).max()))
        assert np.abs(V.T @ V - np.eye(n)).max() < 1e-13
        assert np.abs(a @ V - V * w).max() < 1e-12 * max(1, np.abs(a).max())


def test_projection_closed_forms(orc):
    d = np.array([3.0, -1.0, 0.0, 2.5, -7.0])
    assert np.array_equal(orc.project_psd(np.diag(d)), np.diag(np.maximum(d, 0)))
    # 2x2: eigenvalues (a+c)/2 +- sqrt(((a-c)/2)^2 + b^2)
    a, b, c = 1.0, 2.0, -0.5
    lam = (a + c) / 2 + np.sqrt(((a - c) / 2) ** 2 + b * b)
    v = np.array([b, lam - a]); v /= np.linalg.norm(v)
    assert np.allclose(orc.project_psd(np.array([[a, b], [b, c]])), lam * np.outer(v, v), atol=1e-15)
    rng = np.random.default_rng(2)
    P = _sym(rng, 20, rng.uniform(0.1, 2.0, 20))
    assert np.allclose(orc.project_psd(P), P, atol=1e-13)
    assert np.allclose(orc.project_psd(-P), 0, atol=1e-13)
    x = rng.standard_normal(30)
    assert np.allclose(orc.project_psd(np.outer(x, x)), np.outer(x, x), atol=1e-13)
    assert np.allclose(orc.project_psd(-np.outer(x, x)), 0, atol=1e-13)
    assert np.array_equal(orc.project_psd(np.zeros((6, 6))), np.zeros((6, 6)))


@pytest.mark.parametrize("n", [4, 8, 12, 36, 78, 105])
def test_projection_properties(orc, n):
    rng = np.random.default_rng(n)
    for kind in ["random", "clustered", "near_zero"]:
        if kind == "random":
            a = _sym(rng, n)
        elif kind == "clustered":
            a = _sym(rng, n, np.repeat([-1.0, 1e-3, 2.0], (n + 2) // 3)[:n] + 1e-12 * rng.standard_normal(n))
        else:
            a = _sym(rng, n, 1e-9 * rng.standard_normal(n))
        p = orc.project_psd(a)
        scale = max(1.0, np.linalg.norm(a))
        assert np.array_equal(p, p.T)
        assert np.linalg.eigvalsh(p).min() >= -1e-12 * scale
        assert np.linalg.norm(orc.project_psd(p) - p) <= 1e-12 * scale          # idempotent
        m = orc.project_psd(-a)
        assert np.linalg.norm(p - m - a) <= 1e-12 * scale                        # Moreau
        assert abs(np.sum(p * m)) <= 1e-12 * scale ** 2                           # orthogonal
        assert np.linalg.norm(p - _proj_ref(a)) <= 1e-12 * scale                  # vs eigh


def test_projection_nonexpansive(orc):
    rng = np.random.default_rng(3)
    for _ in range(5):
        a, b = _sym(rng, 15), _sym(rng, 15)
        assert np.linalg.norm(orc.project_psd(a) - orc.project_psd(b)) <= np.linalg.norm(a - b) * (1 + 1e-12)


def test_project_svec_blocks(orc):
    rng = np.random.default_rng(4)
    sizes = [3, 10, 1, 7]
    mats = [_sym(rng, n) for n in sizes]
    def svec(a):
        n = a.shape[0]
        return np.array([a[i, j] * (1 if i == j else np.sqrt(2)) for j in range(n) for i in range(j + 1)])
    x = np.concatenate([svec(a) for a in mats])
    y = orc.project_svec(sizes, x)
    assert np.allclose(y, np.concatenate([svec(_proj_ref(a)) for a in mats]), atol=1e-13)


@pytest.mark.parametrize("fam,N,prm", [("TOY1D", 3, [2.0, 0.1, 1.0]), ("PENDULUM", 3, [0.5, 0.0]),
                                       ("CARTPOLE", 2, [0.1, 0.2, 0.5, 0.3])])
def test_ldl_solve(orc, fam, N, prm):
    sdp = orc.relax(getattr(orc, fam), N, prm)
    F = orc.LDL(sdp)
    A = sdp.A
    K = (A @ A.T).toarray()
    assert abs(F.eps - 1e-12 * np.diag(K).max()) <= 1e-25
    K += F.eps * np.eye(sdp.m)
    rng = np.random.default_rng(5)
    # right-hand sides in the range of A (as in Algorithm 1) and arbitrary ones
    kf = np.linalg.norm(K)
    for r in [A @ rng.standard_normal(sdp.nsvec), rng.standard_normal(sdp.m)]:
        y = F.solve(r)
        # backward-stable solve: small residual relative to ||K|| ||y||
        assert np.linalg.norm(K @ y - r) <= 1e-13 * kf * np.linalg.norm(y)
    r = A @ rng.standard_normal(sdp.nsvec)
    y = F.solve(r)
    yd = np.linalg.solve(K, r)
    # y is fixed only up to the (numerical) null space of A^*: compare A^* y
    assert np.linalg.norm(A.T @ (y - yd)) <= 1e-8 * np.linalg.norm(A.T @ yd)


def test_ldl_factor_dense_reference(orc):
    """A generic full-row-rank A: LDL^T solve equals the dense solve to rounding."""
    import scipy.sparse as sp
    rng = np.random.default_rng(6)
    m, n = 40, 120
    A = sp.random(m, n, density=0.08, random_state=7, format="csr") + sp.eye(m, n, format="csr")
    A = A.tocsr()
    s = orc.SDP(m=m, nsvec=n, rowptr=A.indptr.astype(np.int64), col=A.indices.astype(np.int32),
                val=A.data.astype(np.float64))
    F = orc.LDL(s)
    K = (A @ A.T).toarray() + F.eps * np.eye(m)
    r = rng.standard_normal(m)
    assert np.allclose(F.solve(r), np.linalg.solve(K, r), rtol=1e-10, atol=1e-12)
