"""Blocks beyond one workgroup's LDS (n > 113 in FP64): the multi-workgroup block Jacobi, through
the C ABI, against the FP64 oracle.  Needs an MI355X.

The sizes are those of the paper's larger moment blocks (Table 1: 190 for the car back-in and
the vehicle landing, 231 for the flying robot) and a few around them (115 just past the
one-workgroup limit, 256 a whole number of tiles, 300 more than four tiles).  Tolerances as in
test_gpu_parity: projection ||Pi_gpu - Pi_oracle||_F / max(1, ||X||_F) <= 1e-10; ADMM iterates
blockwise <= 1e-9.
"""
import numpy as np
import pytest
from parity_util import blockwise_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    import paper_2406_05846_amd as S
    return S


@pytest.fixture(scope="module")
def ctx(S):
    c = S.Context(0)
    yield c
    c.close()


def _rand_sym(rng, n, kind="random"):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    if kind == "random":
        w = rng.standard_normal(n)
    elif kind == "clustered":
        w = np.repeat([-1.0, 1e-3, 2.0], (n + 2) // 3)[:n] + 1e-12 * rng.standard_normal(n)
    elif kind == "psd":
        w = rng.uniform(0.1, 2.0, n)
    else:  # nsd
        w = -rng.uniform(0.1, 2.0, n)
    a = (Q * w) @ Q.T
    return (a + a.T) / 2


def _dense_call(S, ctx, mats, fn):
    import torch
    sizes = [m.shape[0] for m in mats]
    offs = np.concatenate([[0], np.cumsum([n * n for n in sizes])[:-1]]).astype(np.int64)
    flat = np.concatenate([m.reshape(-1, order="F") for m in mats])
    x = torch.tensor(flat, dtype=torch.float64, device="cuda")
    nd = torch.tensor(sizes, dtype=torch.int32, device="cuda")
    od = torch.tensor(offs, dtype=torch.int64, device="cuda")
    return fn(x, nd, od, sizes, offs)


@pytest.mark.parametrize("kind", ["random", "clustered", "psd", "nsd"])
def test_big_projection_vs_oracle(S, ctx, orc, kind):
    import torch
    rng = np.random.default_rng(200)
    sizes = [190, 231, 115, 12]  # a small block rides along, padded to the launch's size
    mats = [_rand_sym(rng, n, kind) for n in sizes]

    def run(x, nd, od, sizes, offs):
        out = torch.empty_like(x)
        ctx.project_psd_batched(nd, od, x, out, max(sizes))
        torch.cuda.synchronize()
        res = out.cpu().numpy()
        return [res[o:o + n * n].reshape((n, n), order="F") for o, n in zip(offs, sizes)]

    got = _dense_call(S, ctx, mats, run)
    for a, p in zip(mats, got):
        ref = orc.project_psd(a)
        err = np.linalg.norm(p - ref) / max(1.0, np.linalg.norm(a))
        assert err <= 1e-10, (a.shape[0], kind, err)
        assert np.array_equal(p, p.T)
        if kind == "psd":
            assert np.linalg.norm(p - a) <= 1e-10 * max(1.0, np.linalg.norm(a))
        if kind == "nsd":
            assert np.abs(p).max() <= 1e-10 * max(1.0, np.linalg.norm(a))


@pytest.mark.parametrize("n", [256, 300, 512])
def test_big_projection_sizes(S, ctx, orc, n):
    """Whole tiles (256), a ragged fifth tile (300), the largest supported size (512), in place."""
    import torch
    rng = np.random.default_rng(201 + n)
    a = _rand_sym(rng, n)
    x = torch.tensor(a.reshape(-1, order="F"), dtype=torch.float64, device="cuda")
    nd = torch.tensor([n], dtype=torch.int32, device="cuda")
    od = torch.tensor([0], dtype=torch.int64, device="cuda")
    ctx.project_psd_batched(nd, od, x, x, n)  # in == out
    p = x.cpu().numpy().reshape((n, n), order="F")
    err = np.linalg.norm(p - orc.project_psd(a)) / np.linalg.norm(a)
    assert err <= 1e-10, (n, err)


def test_big_eig_vs_oracle(S, ctx, orc):
    """Eigenvalues ascending against the oracle's Jacobi; eigenvectors through their residual and
    orthogonality (the eigenvector of a simple eigenvalue is unique up to sign)."""
    import torch
    rng = np.random.default_rng(202)
    sizes = [231, 140]
    mats = [_rand_sym(rng, n) for n in sizes]

    def run(x, nd, od, sizes, offs):
        woff = torch.tensor(np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64), device="cuda")
        w = torch.empty(sum(sizes), dtype=torch.float64, device="cuda")
        v = torch.empty_like(x)
        ctx.eig_batched(nd, od, x, woff, w, v, max(sizes))
        torch.cuda.synchronize()
        return w.cpu().numpy(), v.cpu().numpy(), woff.cpu().numpy()

    w, v, woff = _dense_call(S, ctx, mats, run)
    o = 0
    for a, n, wo in zip(mats, sizes, woff):
        lam = w[wo:wo + n]
        ref, _, _ = orc.jacobi_eig(a)
        assert np.all(np.diff(lam) >= 0)
        assert np.abs(lam - np.sort(ref)).max() <= 1e-10 * np.linalg.norm(a)
        V = v[o:o + n * n].reshape((n, n), order="F")
        assert np.linalg.norm(a @ V - V * lam) <= 1e-10 * np.linalg.norm(a)
        assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-12 * n
        o += n * n


def _synthetic_sdp(orc, S, sizes, m, seed):
    """A feasible, bounded instance with the given blocks (workloads.synthetic), for both sides."""
    from workloads.synthetic import large_block_sdp
    d = large_block_sdp(sizes, m, seed)
    osdp = orc.SDP(nblocks=len(d["block_sizes"]), bsize=d["block_sizes"], boff=d["boff"], nsvec=d["nsvec"], m=m,
                   nnz=len(d["val"]), rowptr=d["rowptr"], col=d["col"], val=d["val"], b=d["b"], C=d["C"])
    prob = S.Problem(d["block_sizes"], d["rowptr"], d["col"], d["val"], d["b"], d["C"])
    return osdp, prob


def test_big_admm_iterates_fixed_sigma(S, ctx, orc):
    """Iterates of Algorithm 1 on an instance with two large blocks (200, 130) and a small one:
    after 1 iteration (cold projection) and 12 (warm-started projections), fixed sigma."""
    osdp, prob = _synthetic_sdp(orc, S, [200, 130, 12], 300, 7)
    inst = S.Instance(ctx, prob, S.default_opts(sigma_every=0, kkt_every=1, tol=0.0))
    for k in [1, 12]:
        inst.set_iterate(np.zeros(prob.nsvec), np.zeros(prob.m), np.zeros(prob.nsvec))
        inst.step(k)
        Xg, yg, Sg = inst.get_iterate()
        r = orc.admm_solve(osdp, maxiter=k, tol=0.0, sigma_every=0)
        assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9, k
        assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9, k
        kk = inst.kkt()
        for f in ("eta_p", "eta_d", "eta_g"):
            assert abs(kk[f] - r[f]) <= 1e-9 * max(1.0, r[f]) + 1e-12, (f, kk[f], r[f])
    inst.close()


def test_big_admm_sigma_rule(S, ctx, orc):
    """100 iterations with the sigma rule (its cone projection of X runs through the same path)
    and the rounds replayed from HIP graphs: same iterates and sigma as the oracle."""
    osdp, prob = _synthetic_sdp(orc, S, [160, 12, 12], 200, 8)
    inst = S.Instance(ctx, prob, S.default_opts(tol=0.0, kkt_every=10, sigma_every=50))
    info = inst.step(100)
    Xg, yg, Sg = inst.get_iterate()
    r = orc.admm_solve(osdp, maxiter=100, tol=0.0, sigma_every=50)
    assert abs(info["sigma"] - r["sigma"]) <= 1e-12 * r["sigma"], (info["sigma"], r["sigma"])
    assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9
    assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9
    inst.close()


def test_big_batch_rejected(S, ctx, orc):
    osdp, prob = _synthetic_sdp(orc, S, [130, 12], 50, 9)
    inst = S.Instance(ctx, prob)
    with pytest.raises(S.StromError):
        S.Batch(ctx, [inst])
    inst.close()


def test_big_only_instance_and_serving_refusal(S, ctx, orc):
    """An instance whose every block takes the block Jacobi (no one-workgroup launch at all):
    fixed-sigma iterates against the oracle; the request loop refuses such a problem at submit."""
    osdp, prob = _synthetic_sdp(orc, S, [150, 120], 80, 12)
    inst = S.Instance(ctx, prob, S.default_opts(sigma_every=0, kkt_every=1, tol=0.0))
    inst.step(4)
    Xg, yg, Sg = inst.get_iterate()
    r = orc.admm_solve(osdp, maxiter=4, tol=0.0, sigma_every=0)
    assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9
    assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9
    inst.close()
    with pytest.raises(S.StromError):
        ctx.submit(prob)


def test_big_certificate_vs_oracle(S, ctx, orc):
    """The dual bound's smallest eigenvalues of C - A^* y on the large blocks (eigenvalues-only
    path of the multi-workgroup solver) against the oracle's."""
    osdp, prob = _synthetic_sdp(orc, S, [150, 12], 120, 10)
    inst = S.Instance(ctx, prob, S.default_opts(tol=0.0, sigma_every=0, kkt_every=1))
    inst.step(5)
    X, y, Sv = inst.get_iterate()
    R = np.full(osdp.nblocks, 3.0)
    lb, lam = inst.dual_bound(R)
    ref_lb, ref_lam = orc.dual_bound(osdp, y, R)
    assert abs(lb - ref_lb) <= 1e-9 * max(1.0, abs(ref_lb))
    assert np.abs(lam - ref_lam).max() <= 1e-9 * max(1.0, np.abs(ref_lam).max())
    inst.close()


def test_big_boundary_sizes(S, ctx, orc):
    """n = 113 is the last FP64 size of the one-workgroup kernel and 114 the first of the block
    Jacobi (both against the oracle); FP32 data beyond 122 is refused (the block Jacobi is FP64)."""
    import torch
    rng = np.random.default_rng(203)
    for n in (113, 114):
        a = _rand_sym(rng, n)
        x = torch.tensor(a.reshape(-1, order="F"), dtype=torch.float64, device="cuda")
        nd = torch.tensor([n], dtype=torch.int32, device="cuda")
        od = torch.tensor([0], dtype=torch.int64, device="cuda")
        ctx.project_psd_batched(nd, od, x, x, n)
        p = x.cpu().numpy().reshape((n, n), order="F")
        assert np.linalg.norm(p - orc.project_psd(a)) / np.linalg.norm(a) <= 1e-10, n
    x32 = torch.zeros(123 * 123, dtype=torch.float32, device="cuda")
    nd = torch.tensor([123], dtype=torch.int32, device="cuda")
    od = torch.tensor([0], dtype=torch.int64, device="cuda")
    with pytest.raises(S.StromError):
        ctx.project_psd_batched(nd, od, x32, x32, 123)


@pytest.mark.parametrize("fam_name", ["FLYING", "LANDING", "BACKIN"])
def test_paper_family_iterates(S, ctx, orc, fam_name):
    """The paper's flying robot (231 x 231 moment blocks), vehicle landing and car back-in (190 x 190)
    relaxations,
    whose moment blocks take the block Jacobi, N = 2: iterates after 1 and 6 iterations with a fixed
    sigma against the oracle (its own generator, LDL^T and Jacobi)."""
    import workloads as W
    fam = getattr(W, fam_name)
    prm = W.instance_params(fam, 0)
    osdp = orc.relax(fam, 2, prm)
    prob = S.generate(fam, 2, prm)
    inst = S.Instance(ctx, prob, S.default_opts(sigma_every=0, kkt_every=1, tol=0.0))
    for k in [1, 6]:
        inst.set_iterate(np.zeros(prob.nsvec), np.zeros(prob.m), np.zeros(prob.nsvec))
        inst.step(k)
        Xg, yg, Sg = inst.get_iterate()
        r = orc.admm_solve(osdp, maxiter=k, tol=0.0, sigma_every=0)
        assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9, k
        assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9, k
    inst.close()
