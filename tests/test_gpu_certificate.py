"""GPU parity of the certificate entry points (strom_eig_batched, strom_dual_bound,
strom_extract) with the oracle, through the C ABI."""
import time

import numpy as np
import pytest

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


def _eig_dense(S, ctx, mats, dtype, want_v):
    import torch
    sizes = [m.shape[0] for m in mats]
    offs = np.concatenate([[0], np.cumsum([n * n for n in sizes])[:-1]]).astype(np.int64)
    woff = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    td = torch.float64 if dtype == "f64" else torch.float32
    x = torch.tensor(np.concatenate([m.reshape(-1, order="F") for m in mats]), dtype=td, device="cuda")
    w = torch.zeros(sum(sizes), dtype=td, device="cuda")
    v = torch.zeros_like(x) if want_v else None
    ctx.eig_batched(torch.tensor(sizes, dtype=torch.int32, device="cuda"), torch.tensor(offs, device="cuda"), x,
                    torch.tensor(woff, device="cuda"), w, v, max(sizes))
    torch.cuda.synchronize()
    wh = w.double().cpu().numpy()
    ws = [wh[o:o + n] for o, n in zip(woff, sizes)]
    vs = None
    if want_v:
        vh = v.double().cpu().numpy()
        vs = [vh[o:o + n * n].reshape((n, n), order="F") for o, n in zip(offs, sizes)]
    return ws, vs


SIZES = [1, 2, 3, 7, 8, 12, 13, 36, 55, 78, 91, 105]


def test_eig_batched_f64(S, ctx):
    rng = np.random.default_rng(41)
    mats = []
    for n in SIZES:
        b = rng.standard_normal((n, n))
        mats.append((b + b.T) / 2)
    ws, vs = _eig_dense(S, ctx, mats, "f64", True)
    w_only, _ = _eig_dense(S, ctx, mats, "f64", False)
    for a, w, v, wo in zip(mats, ws, vs, w_only):
        n = a.shape[0]
        na = max(1.0, np.linalg.norm(a))
        assert np.all(np.diff(w) >= 0)
        assert np.abs(w - np.linalg.eigvalsh(a)).max() <= 1e-12 * na, n
        assert np.linalg.norm(a @ v - v * w) <= 1e-12 * na, n
        assert np.linalg.norm(v.T @ v - np.eye(n)) <= 1e-12 * n, n
        assert np.array_equal(w, wo)  # the eigenvalues-only mode runs the same rotations


def test_eig_batched_f32(S, ctx):
    rng = np.random.default_rng(42)
    mats = []
    for n in SIZES + [120]:
        b = rng.standard_normal((n, n))
        mats.append((b + b.T) / 2)
    ws, _ = _eig_dense(S, ctx, mats, "f32", False)
    for a, w in zip(mats, ws):
        a32 = a.astype(np.float32).astype(np.float64)
        assert np.abs(w - np.linalg.eigvalsh(a32)).max() <= 2e-5 * max(1.0, np.linalg.norm(a32)), a.shape[0]


@pytest.mark.parametrize("fam,N,prm", [(1, 10, [0.5, 0.0]), (2, 4, [0.1, 0.2, 0.5, 0.3])])
def test_dual_bound_vs_oracle(S, ctx, orc, fam, N, prm):
    osdp = orc.relax(fam, N, prm)
    inst = S.Instance(ctx, S.generate(fam, N, prm), S.default_opts(sigma_every=0, tol=0.0))
    inst.step(30)
    _, y, _ = inst.get_iterate()
    R = np.linspace(1.0, 3.0, osdp.nblocks)
    lb, lam = inst.dual_bound(R)
    lb_o, lam_o = orc.dual_bound(osdp, y, R)
    scale = 1.0 + np.abs(lam_o).max()
    assert np.abs(lam - lam_o).max() <= 1e-10 * scale
    assert abs(lb - lb_o) <= 1e-10 * (1.0 + abs(lb_o))
    inst.close()


@pytest.mark.parametrize("fam,N,prm,rank_tol", [
    (1, 6, [0.5, 0.0], 1e-11),
    (4, 3, [1, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1], 1e-11),
    # the paper's car back-in and flying robot: 190 x 190 and 231 x 231 moment blocks, whose
    # eigenvectors come from the block Jacobi (stopped at off(W) <= 1e-11 ||W||_F, so the null
    # space's eigenvalues are resolved to about that)
    (7, 2, [3.0, 4.0, 0.1], 1e-10),
    (5, 2, [3.0, -2.0, 0.5, 0.5, -0.5, 0.2], 1e-10),
    # the paper's cart-pole: cliques with lookahead variables (a_{k+2}, rs_{k+2})
    (8, 3, [0.1, 0.2, 0.3, 0.5], 1e-11),
])
def test_extract_vs_oracle_on_a_lifting(S, ctx, orc, fam, N, prm, rank_tol):
    osdp = orc.relax(fam, N, prm)
    rng = np.random.default_rng(9)
    z, _ = orc.rollout(fam, N, prm, rng.uniform(-0.5, 0.5, N * osdp.du), osdp.dx, osdp.du)
    X, _ = orc.lift(fam, N, prm, z)
    inst = S.Instance(ctx, S.generate(fam, N, prm))
    inst.set_iterate(X=X)
    blocks = [k for k in range(osdp.nblocks) if osdp.bkind[k] == 0] + [1]  # moment blocks and one localizing
    lam, vt = inst.extract(blocks, [int(osdp.bsize[k]) for k in blocks])
    lam_o, vt_o = orc.extract(osdp, X, blocks)
    assert np.abs(lam - lam_o).max() <= 1e-11 * (1.0 + np.abs(lam_o).max())
    d = osdp.nclique_vars
    for t, k in enumerate(blocks):
        if osdp.bkind[k] != 0:
            continue
        assert lam[t, 1] <= rank_tol * lam[t, 0]
        assert np.allclose(vt[t], vt_o[t], atol=1e-9)
        assert np.allclose(vt[t][1:1 + d], orc.clique_vars(osdp, z, int(osdp.bclique[k])), atol=1e-9)
    inst.close()


def test_warm_started_resolve_reaches_the_cold_optimum(S, ctx):
    """Receding-horizon step: the problem one step later, solved from the previous solution
    shifted by one clique and the previous final sigma, converges to the optimum of the cold
    solve."""
    import math
    import workloads as W
    ins0 = S.Instance(ctx, S.generate(W.PENDULUM, 8, [0.8, 0.0]))
    r0 = ins0.step(50000)
    assert r0["state"] == S.CONVERGED
    X, _, Sv = ins0.get_iterate()
    _, vt = ins0.extract([0], [36])
    ins0.close()
    prob1 = S.generate(W.PENDULUM, 8, [math.atan2(vt[0][6], vt[0][5]), 8.0 * vt[0][7]])
    bs = [int(n) for n in prob1.block_sizes]
    res = {}
    for label, X0, S0 in (("cold", None, None), ("warm", W.shift_one_clique(bs, X), W.shift_one_clique(bs, Sv))):
        ins = S.Instance(ctx, prob1, None if X0 is None else S.default_opts(sigma0=r0["sigma"]))
        if X0 is not None:
            ins.set_iterate(X=X0, S=S0)
        res[label] = ins.step(50000)
        ins.close()
    assert res["cold"]["state"] == S.CONVERGED and res["warm"]["state"] == S.CONVERGED
    pc, pw = res["cold"]["pobj"], res["warm"]["pobj"]
    assert abs(pw - pc) <= 1e-4 * (1.0 + abs(pc))
    # the same warm start through the request loop: X0 and S0 in the problem, sigma0 in opts
    warm_prob = S.Problem(prob1.block_sizes, prob1.rowptr, prob1.col, prob1.val, prob1.b, prob1.C,
                          X0=W.shift_one_clique(bs, X), S0=W.shift_one_clique(bs, Sv))
    t = ctx.submit(warm_prob, S.default_opts(sigma0=r0["sigma"]))
    t0 = time.time()
    while (r := ctx.poll(t)) is None:
        assert time.time() - t0 < 60, "request loop did not finish"
        time.sleep(0.01)
    assert r[0]["state"] == S.CONVERGED
    assert r[0]["iters"] == res["warm"]["iters"]
    assert abs(r[0]["pobj"] - pw) <= 1e-9 * (1.0 + abs(pw))


def test_car_full_size_certificate(S, ctx, orc):
    """Car N = 50, bicycle-13 (seed 1: 50 moment blocks 105 x 105, 400 localizing), solved to
    eta <= 1e-6: the valid lower bound with the family's trace bounds R_beta (App. "Existence of
    R_beta"; the same values from both generators) through strom_dual_bound, against the
    oracle's bound at the device's y, block by block; the bound sits below <b, y>; the rank test
    and extraction of the moment blocks against the oracle's."""
    import workloads as W
    prm = W.instance_params(W.CAR, 1)
    prob = S.generate(W.CAR, 50, prm)
    R = prob.trace_bounds
    assert R is not None and np.array_equal(R, orc.trace_bounds(W.CAR, 50, prm))
    inst = S.Instance(ctx, prob, S.default_opts(maxiter=30000))
    info = inst.step(30000)
    assert info["state"] == S.CONVERGED, info
    lb, lam = inst.dual_bound(R)
    X, y, _ = inst.get_iterate()
    osdp = orc.relax(W.CAR, 50, prm)
    ref_lb, ref_lam = orc.dual_bound(osdp, y, R)
    assert np.abs(lam - ref_lam).max() <= 1e-9 * max(1.0, np.abs(ref_lam).max())
    assert abs(lb - ref_lb) <= 1e-9 * (1.0 + abs(ref_lb))
    assert lb <= info["dobj"]
    gap = (info["pobj"] - lb) / (1.0 + abs(info["pobj"]) + abs(lb))
    assert 0.0 <= gap <= 5e-2, (info["pobj"], lb)
    moments = [k for k in range(osdp.nblocks) if osdp.bkind[k] == 0]
    lt, vt = inst.extract(moments, [int(osdp.bsize[k]) for k in moments])
    lt_o, vt_o = orc.extract(osdp, X, moments)
    assert np.abs(lt - lt_o).max() <= 1e-9 * (1.0 + np.abs(lt_o).max())
    inst.close()


@pytest.mark.parametrize("fam,N,seed", [(8, 3, 0), (7, 2, 0)])
def test_paper_problem_certificates(S, ctx, orc, fam, N, seed):
    """The paper's cart-pole (its last clique's lookahead a_{N+1} bounded through the dynamics) and
    car back-in (separation inequalities with products of two variables): the trace bounds R_beta
    agree between the generators, and after a solve (to 1e-8; the back-in 1,000 iterations) the
    device's valid lower bound equals the oracle's at the device's y, block by block, and lies
    below <b, y> and the objective."""
    import workloads as W
    prm = W.instance_params(fam, seed)
    prob = S.generate(fam, N, prm)
    R = prob.trace_bounds
    assert R is not None and np.array_equal(R, orc.trace_bounds(fam, N, prm))
    cap = 20000 if fam == 8 else 1000  # the bound is valid at any y: the back-in stops at a short cap
    inst = S.Instance(ctx, prob, S.default_opts(maxiter=cap, tol=1e-8))
    info = inst.step(cap)
    if fam == 8:
        assert info["state"] == S.CONVERGED, info
    lb, lam = inst.dual_bound(R)
    _, y, _ = inst.get_iterate()
    osdp = orc.relax(fam, N, prm)
    ref_lb, ref_lam = orc.dual_bound(osdp, y, R)
    assert np.abs(lam - ref_lam).max() <= 1e-9 * max(1.0, np.abs(ref_lam).max())
    assert abs(lb - ref_lb) <= 1e-9 * (1.0 + abs(ref_lb))
    assert lb <= info["dobj"] + 1e-12 * (1.0 + abs(info["dobj"]))
    assert lb <= info["pobj"] + 1e-9 * (1.0 + abs(info["pobj"]))
    inst.close()
