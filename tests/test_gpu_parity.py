"""Parity of the HIP path (through the C ABI) with the FP64 oracle.  Needs an MI355X.

Tolerances (stated per quantity):
* PSD projection, per block: ||Pi_gpu - Pi_oracle||_F / max(1, ||X||_F) <= 1e-10 in FP64 and
  <= 1e-5 in FP32 (the FP32 path projects the FP32-rounded input; the oracle projects the
  same rounded values in FP64);
* ADMM iterates with a fixed sigma, after k iterations: ||X_gpu - X_orc|| / max(1, ||X_orc||)
  <= 1e-9, the same for S and for A^* y (y itself is fixed only up to the null space of A^*);
* converged solves: the oracle's own KKT evaluation of the GPU iterate gives eta <= 1e-6
  (x 1.05 for the rounding of the two evaluations), and the objective gap
  |pobj_gpu - pobj_orc| / (1 + |pobj_gpu| + |pobj_orc|) <= 1e-6 against the oracle's optimum
  at 1e-8 (the normalization of eta_g); at tol = 1e-7 also |p_gpu - p_orc| / (1 + |p_orc|).
"""
import json
import math
import os

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
    return (Q * w) @ Q.T


def _run_dense(S, ctx, mats, dtype):
    import torch
    sizes = [m.shape[0] for m in mats]
    offs = np.concatenate([[0], np.cumsum([n * n for n in sizes])[:-1]]).astype(np.int64)
    flat = np.concatenate([m.reshape(-1, order="F") for m in mats])
    td = torch.float64 if dtype == "f64" else torch.float32
    x = torch.tensor(flat, dtype=td, device="cuda")
    out = torch.empty_like(x)
    nd = torch.tensor(sizes, dtype=torch.int32, device="cuda")
    od = torch.tensor(offs, dtype=torch.int64, device="cuda")
    ctx.project_psd_batched(nd, od, x, out, max(sizes))
    torch.cuda.synchronize()
    res = out.double().cpu().numpy()
    return [res[o:o + n * n].reshape((n, n), order="F") for o, n in zip(offs, sizes)], x


SIZES = [1, 2, 3, 8, 12, 13, 14, 36, 55, 78, 91, 105]


@pytest.mark.parametrize("kind", ["random", "clustered", "psd", "nsd"])
def test_projection_f64_vs_oracle(S, ctx, orc, kind):
    rng = np.random.default_rng(100)
    mats = [_rand_sym(rng, n, kind) for n in SIZES]
    got, _ = _run_dense(S, ctx, mats, "f64")
    for a, p in zip(mats, got):
        ref = orc.project_psd(a)
        err = np.linalg.norm(p - ref) / max(1.0, np.linalg.norm(a))
        assert err <= 1e-10, (a.shape[0], err)
        assert np.array_equal(p, p.T)
        if kind == "psd":
            assert np.linalg.norm(p - a) <= 1e-10 * max(1.0, np.linalg.norm(a))
        if kind == "nsd":
            assert np.abs(p).max() <= 1e-10 * max(1.0, np.linalg.norm(a))


def test_projection_f32_vs_oracle(S, ctx, orc):
    rng = np.random.default_rng(101)
    mats = [_rand_sym(rng, n) for n in SIZES + [120]]
    got, x = _run_dense(S, ctx, mats, "f32")
    for a, p in zip(mats, got):
        a32 = a.astype(np.float32).astype(np.float64)
        ref = orc.project_psd(a32)
        err = np.linalg.norm(p - ref) / max(1.0, np.linalg.norm(a32))
        assert err <= 1e-5, (a.shape[0], err)


def test_projection_in_place_and_errors(S, ctx, orc):
    import torch
    rng = np.random.default_rng(102)
    a = _rand_sym(rng, 20)
    x = torch.tensor(a.reshape(-1, order="F"), dtype=torch.float64, device="cuda")
    nd = torch.tensor([20], dtype=torch.int32, device="cuda")
    od = torch.tensor([0], dtype=torch.int64, device="cuda")
    ctx.project_psd_batched(nd, od, x, x, 20)  # in == out
    p = x.cpu().numpy().reshape((20, 20), order="F")
    assert np.linalg.norm(p - orc.project_psd(a)) <= 1e-10 * np.linalg.norm(a)
    with pytest.raises(S.StromError):  # block larger than max_n
        ctx.project_psd_batched(nd, od, x, x, 10)
    with pytest.raises(S.StromError):  # over the largest block size (512)
        ctx.project_psd_batched(nd, od, x, x, 600)
    empty_n = torch.zeros(0, dtype=torch.int32, device="cuda")
    empty_o = torch.zeros(0, dtype=torch.int64, device="cuda")
    ctx.project_psd_batched(empty_n, empty_o, x, x, 20)  # nothing to do


# ----------------------------------------------------------------- ADMM iterates

def _opts(S, **kw):
    return S.default_opts(**kw)


@pytest.mark.parametrize("fam,N,prm,iters", [
    (0, 3, [2.0, 0.1, 1.0], 20),
    (1, 10, [0.5, 0.0], 20),
    (1, 4, [2.9, 0.0], 7),
])
def test_iterates_fixed_sigma_vs_oracle(S, ctx, orc, fam, N, prm, iters):
    """k iterations of Algorithm 1 with a fixed sigma, same starting point."""
    osdp = orc.relax(fam, N, prm)
    prob = S.generate(fam, N, prm)
    A = osdp.A
    inst = S.Instance(ctx, prob, _opts(S, sigma_every=0, kkt_every=1, tol=0.0))
    for k in [1, iters]:
        inst.set_iterate(np.zeros(prob.nsvec), np.zeros(prob.m), np.zeros(prob.nsvec))
        inst.step(k)
        Xg, yg, Sg = inst.get_iterate()
        r = orc.admm_solve(osdp, maxiter=k, tol=0.0, sigma_every=0)
        assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9, k
        assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9, k
        aty, atyo = A.T @ yg, A.T @ r["y"]
        assert np.linalg.norm(aty - atyo) / max(1.0, np.linalg.norm(atyo)) <= 1e-9, k
        kk = inst.kkt()
        for f in ("eta_p", "eta_d", "eta_g"):
            assert abs(kk[f] - r[f]) <= 1e-9 * max(1.0, r[f]) + 1e-12, (f, kk[f], r[f])
    inst.close()


def test_cartpole_full_size_iterates(S, ctx, orc):
    """Cart-pole, N = 30 (n_svec 97,110, m 78,267): three iterations with a fixed sigma."""
    import workloads as W
    prm = W.instance_params(W.CARTPOLE, 0)
    osdp = orc.relax(W.CARTPOLE, 30, prm)
    prob = S.generate(W.CARTPOLE, 30, prm)
    inst = S.Instance(ctx, prob, _opts(S, sigma_every=0, kkt_every=1, tol=0.0))
    inst.step(3)
    Xg, yg, Sg = inst.get_iterate()
    r = orc.admm_solve(osdp, maxiter=3, tol=0.0, sigma_every=0)
    assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9
    assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9
    inst.close()


@pytest.mark.parametrize("env", [
    {"STROM_STAGE_ROWS": "0"},  # every task solved in place in global memory
    {"STROM_TASK_SPLIT": "0", "STROM_STAGE_ROWS": "600", "STROM_BLOCK_ROWS": "32"},  # mixed, more phases
])
def test_solve_schedule_variants_iterates(S, ctx, orc, monkeypatch, env):
    """Cart-pole N = 10 under other solve schedules (the analysis reads these variables):
    five iterations with a fixed sigma against the oracle."""
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    prm = [0.1, 0.2, 0.5, 0.3]
    osdp = orc.relax(2, 10, prm)
    prob = S.generate(2, 10, prm)
    inst = S.Instance(ctx, prob, _opts(S, sigma_every=0, kkt_every=1, tol=0.0))
    inst.step(5)
    Xg, yg, Sg = inst.get_iterate()
    r = orc.admm_solve(osdp, maxiter=5, tol=0.0, sigma_every=0)
    assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9
    assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9
    aty, atyo = osdp.A.T @ yg, osdp.A.T @ r["y"]
    assert np.linalg.norm(aty - atyo) / max(1.0, np.linalg.norm(atyo)) <= 1e-9
    inst.close()


def _converged_ref(seed):
    """Oracle optimum of the pendulum workload (N = 10) at eta <= 1e-8, written by
    tests/golden/make_converged_refs.py."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "converged_refs.json")) as f:
        refs = json.load(f)
    return next(c for c in refs["cases"] if c["seed"] == seed)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pendulum_converged_vs_oracle(S, ctx, orc, seed):
    """Pendulum, N = 10: solve to eta <= 1e-6 on the device, check the result with the oracle's
    KKT residuals and against the oracle's optimal value (solved to 1e-8)."""
    import workloads as W
    prm = W.instance_params(W.PENDULUM, seed)
    ref = _converged_ref(seed)
    assert np.allclose(ref["params"], prm, rtol=0, atol=0)
    prob = S.generate(W.PENDULUM, 10, prm)
    osdp = orc.relax(W.PENDULUM, 10, prm)
    inst = S.Instance(ctx, prob)
    info = inst.step(20000)
    assert info["state"] == S.CONVERGED, info
    X, y, Sv = inst.get_iterate()
    k = orc.kkt(osdp, X, y, Sv)
    assert max(k["eta_p"], k["eta_d"], k["eta_g"]) <= 1e-6 * 1.05, k
    # relative gap in the normalization of the paper's eta_g (both objectives in the denominator)
    gap = abs(info["pobj"] - ref["pobj"]) / (1 + abs(info["pobj"]) + abs(ref["pobj"]))
    assert gap <= 1e-6, (info["pobj"], ref["pobj"])
    inst.close()


def test_pendulum_tight_tolerance_objective(S, ctx):
    """At tol = 1e-7 the device objective is within 1e-6 of the oracle's optimum also in the
    stricter normalization |p - p_ref| / (1 + |p_ref|)."""
    import workloads as W
    prm = W.instance_params(W.PENDULUM, 0)
    ref = _converged_ref(0)
    inst = S.Instance(ctx, S.generate(W.PENDULUM, 10, prm), S.default_opts(tol=1e-7))
    info = inst.step(40000)
    assert info["state"] == S.CONVERGED, info
    assert abs(info["pobj"] - ref["pobj"]) / (1 + abs(ref["pobj"])) <= 1e-6
    inst.close()


def test_setup_rejects_bad_problems(S, ctx):
    prob = S.generate(1, 2, [0.5, 0.0])
    bad = S.Problem(prob.block_sizes, prob.rowptr, prob.col.copy(), prob.val, prob.b, prob.C)
    bad.col[3] = prob.nsvec + 5
    with pytest.raises(S.StromError) as e:
        S.Instance(ctx, bad)
    assert e.value.code == -1
    with pytest.raises(S.StromError):  # the binding checks the sizes first ...
        S.Problem(np.array([0] + list(prob.block_sizes[1:]), np.int32), prob.rowptr, prob.col, prob.val,
                  prob.b, prob.C)
    bad2 = S.Problem(prob.block_sizes.copy(), prob.rowptr, prob.col, prob.val, prob.b, prob.C)
    bad2.block_sizes[0] = 0  # ... and the library rejects them too
    with pytest.raises(S.StromError) as e:
        S.Instance(ctx, bad2)
    assert e.value.code == -1
    with pytest.raises(S.StromError):
        S.Instance(ctx, prob, S.default_opts(tau=2.5))


def test_hbm_budget(S):
    small = S.Context(0, hbm_budget=1 << 16)
    prob = S.generate(1, 3, [0.5, 0.0])
    with pytest.raises(S.StromError) as e:
        S.Instance(small, prob)
    assert e.value.code == -2
    small.close()


# ----------------------------------------------------------------- reduced-precision form

@pytest.mark.parametrize("seed", [0, 1])
def test_pendulum_f32_polish_converges(S, ctx, orc, seed):
    """FP32 projection with the FP64 polish switch reaches the same optimum as the oracle:
    eta <= 1e-6 by the oracle's own KKT evaluation and the objective gap of the FP64 form."""
    import workloads as W
    prm = W.instance_params(W.PENDULUM, seed)
    ref = _converged_ref(seed)
    prob = S.generate(W.PENDULUM, 10, prm)
    inst = S.Instance(ctx, prob, S.default_opts(proj_dtype=S.F32))
    info = inst.step(50000)
    assert info["state"] == S.CONVERGED, info
    X, y, Sv = inst.get_iterate()
    k = orc.kkt(orc.relax(W.PENDULUM, 10, prm), X, y, Sv)
    assert max(k["eta_p"], k["eta_d"], k["eta_g"]) <= 1e-6 * 1.05, k
    gap = abs(info["pobj"] - ref["pobj"]) / (1 + abs(info["pobj"]) + abs(ref["pobj"]))
    assert gap <= 1e-6, (info["pobj"], ref["pobj"])
    inst.close()


# ----------------------------------------------------------------- serving

def test_serving_same_result_alone_and_in_the_mix(S, ctx):
    """Requests solved through strom_submit / strom_poll while others share the device give the
    same iterates and iteration counts as the same instances solved alone."""
    import time
    import workloads as W
    cases = [(W.PENDULUM, 10, W.instance_params(W.PENDULUM, s)) for s in range(5)]
    cases += [(W.TOY1D, 4, [1.5, 0.1, 1.0]), (W.PENDULUM, 6, W.instance_params(W.PENDULUM, 7))]
    probs = [S.generate(f, N, p) for f, N, p in cases]
    alone = []
    for pr in probs:
        inst = S.Instance(ctx, pr)
        info = inst.step(50000)
        alone.append((info, inst.get_iterate()))
        inst.close()
    tickets = [ctx.submit(pr) for pr in probs]
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        assert time.time() - t0 < 120, "serving loop did not finish"
        for t, pr in zip(tickets, probs):
            if t in done:
                continue
            r = ctx.poll(t, pr.nsvec, pr.m)
            if r is not None:
                done[t] = r
        time.sleep(0.01)
    for (ia, (Xa, ya, Sa)), t in zip(alone, tickets):
        info, X, y, Sv = done[t]
        assert info["state"] == ia["state"] == S.CONVERGED
        assert info["iters"] == ia["iters"]
        assert np.linalg.norm(X - Xa) <= 1e-9 * max(1.0, np.linalg.norm(Xa))
        assert np.linalg.norm(Sv - Sa) <= 1e-9 * max(1.0, np.linalg.norm(Sa))
        assert abs(info["pobj"] - ia["pobj"]) <= 1e-9 * (1 + abs(ia["pobj"]))


# ----------------------------------------------------------------- car family (both variants)

@pytest.mark.parametrize("seed", [0, 1])
def test_car_iterates_vs_oracle(S, ctx, orc, seed):
    """Planar car, unicycle-12 (seed 0) and bicycle-13 (seed 1): N = 3 for 15 iterations and the
    full N = 50 (blocks 91x91 / 105x105, n_svec 236,600 / 309,750) for 3 iterations, fixed
    sigma, same start: X, S and A^* y within 1e-9 of the oracle."""
    import workloads as W
    prm = W.instance_params(W.CAR, seed)
    for N, k in [(3, 15), (50, 3)]:
        osdp = orc.relax(W.CAR, N, prm)
        prob = S.generate(W.CAR, N, prm)
        assert prob.nsvec == osdp.nsvec and prob.m == osdp.m
        inst = S.Instance(ctx, prob, _opts(S, sigma_every=0, kkt_every=1, tol=0.0))
        inst.step(k)
        Xg, yg, Sg = inst.get_iterate()
        r = orc.admm_solve(osdp, maxiter=k, tol=0.0, sigma_every=0)
        assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9, (N, k)
        assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9, (N, k)
        A = osdp.A
        aty, atyo = A.T @ yg, A.T @ r["y"]
        assert np.linalg.norm(aty - atyo) / max(1.0, np.linalg.norm(atyo)) <= 1e-9, (N, k)
        inst.close()


# ----------------------------------------------------------------- batch of mixed instances

def test_mixed_batch_through_request_loop(S, ctx, orc):
    """Mixed families and horizons submitted together (the batched form at test size): every
    converged result satisfies the oracle's KKT check at 1e-6, and instances that reach the
    iteration cap report it."""
    import time
    import workloads as W
    rng = W.SplitMix64(4242)
    cases = []
    for k in range(10):
        fam = [W.PENDULUM, W.PENDULUM, W.TOY1D, W.CARTPOLE, W.CAR][k % 5]
        N = {W.PENDULUM: rng.randint(4, 10), W.TOY1D: rng.randint(2, 6), W.CARTPOLE: 2, W.CAR: 2}[fam]
        cases.append((fam, N, W.instance_params(fam, 100 + k)))
    opts = S.default_opts(maxiter=30000)
    probs = [S.generate(f, N, p) for f, N, p in cases]
    tickets = [ctx.submit(pr, opts) for pr in probs]
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        assert time.time() - t0 < 240, "request loop did not finish"
        for t, pr in zip(tickets, probs):
            if t not in done:
                r = ctx.poll(t, pr.nsvec, pr.m)
                if r is not None:
                    done[t] = r
        time.sleep(0.01)
    nconv = 0
    for (fam, N, prm), t in zip(cases, tickets):
        info, X, y, Sv = done[t]
        assert info["state"] in (S.CONVERGED, S.MAXITER), info
        k = orc.kkt(orc.relax(fam, N, prm), X, y, Sv)
        eta = max(k["eta_p"], k["eta_d"], k["eta_g"])
        if info["state"] == S.CONVERGED:
            nconv += 1
            assert eta <= 1e-6 * 1.05, (fam, N, k)
        else:
            assert info["iters"] == 30000
            assert abs(eta - max(info["eta_p"], info["eta_d"], info["eta_g"])) <= 1e-6 + 1e-3 * eta
    assert nconv >= 6


def test_batched_instances_on_streams_match_alone(S):
    """The batched form: instances advanced together, each on a context with its own stream,
    give exactly the iterates each one gives alone (the kernels have no order-dependent
    reductions)."""
    import torch
    probs = [S.generate(1, 10, [0.5 + 0.3 * k, 0.0]) for k in range(3)]
    opts = S.default_opts(tol=0.0, maxiter=10**6)
    alone = []
    c0 = S.Context(0)
    for p in probs:
        ins = S.Instance(c0, p, opts)
        ins.enqueue(40)
        torch.cuda.synchronize()
        alone.append(ins.get_iterate())
        ins.close()
    c0.close()
    ctxs = [S.Context(0, stream=torch.cuda.Stream()) for _ in probs]
    insts = [S.Instance(c, p, opts) for c, p in zip(ctxs, probs)]
    for ins in insts:
        ins.enqueue(40)
    torch.cuda.synchronize()
    for ins, ref in zip(insts, alone):
        got = ins.get_iterate()
        for g, r in zip(got, ref):
            assert np.array_equal(g, r)
        ins.close()
    for c in ctxs:
        c.close()


def test_paper_pendulum_full_size_iterates(S, ctx, orc):
    """The paper's own pendulum shape (variational-integrator dynamics; n_svec 49,500, m 47,351,
    30 moment blocks 55x55 + 60 localizing 10x10): three iterations with a fixed sigma."""
    import workloads as W
    prm = W.instance_params(W.PAPER_PENDULUM, 0)
    osdp = orc.relax(W.PAPER_PENDULUM, 30, prm)
    prob = S.generate(W.PAPER_PENDULUM, 30, prm)
    assert (prob.nsvec, prob.m) == (49500, 47351)
    inst = S.Instance(ctx, prob, _opts(S, sigma_every=0, kkt_every=1, tol=0.0))
    inst.step(3)
    Xg, yg, Sg = inst.get_iterate()
    r = orc.admm_solve(osdp, maxiter=3, tol=0.0, sigma_every=0)
    assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9
    assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9
    aty, atyo = osdp.A.T @ yg, osdp.A.T @ r["y"]
    assert np.linalg.norm(aty - atyo) / max(1.0, np.linalg.norm(atyo)) <= 1e-9
    inst.close()


def test_paper_cart_pole_full_size_iterates(S, ctx, orc):
    """The paper's cart-pole (variational integrator with second differences; 30 moment blocks of
    105 over 13-variable cliques that share 7 variables with the next, 90 localizing blocks of 14;
    n_svec 176,400, m 159,721): three iterations with a fixed sigma against the oracle."""
    import workloads as W
    prm = W.instance_params(W.PAPER_CARTPOLE, 0)
    osdp = orc.relax(W.PAPER_CARTPOLE, 30, prm)
    prob = S.generate(W.PAPER_CARTPOLE, 30, prm)
    assert (prob.nsvec, prob.m) == (176400, 159721)
    inst = S.Instance(ctx, prob, _opts(S, sigma_every=0, kkt_every=1, tol=0.0))
    inst.step(3)
    Xg, yg, Sg = inst.get_iterate()
    r = orc.admm_solve(osdp, maxiter=3, tol=0.0, sigma_every=0)
    assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9
    assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9
    aty, atyo = osdp.A.T @ yg, osdp.A.T @ r["y"]
    assert np.linalg.norm(aty - atyo) / max(1.0, np.linalg.norm(atyo)) <= 1e-9
    inst.close()


@pytest.mark.parametrize("split,rows", [(0, 0), (1, 64), (2, 32)])
def test_task_split_option_iterates(S, ctx, orc, split, rows):
    """The solve schedule chosen per instance (strom_opts.task_split, strom_opts.block_rows):
    cart-pole N = 10, five fixed-sigma iterations against the oracle; out-of-range values are
    rejected."""
    prm = [0.1, 0.2, 0.5, 0.3]
    osdp = orc.relax(2, 10, prm)
    prob = S.generate(2, 10, prm)
    inst = S.Instance(ctx, prob, _opts(S, sigma_every=0, kkt_every=1, tol=0.0, task_split=split, block_rows=rows))
    inst.step(5)
    Xg, yg, Sg = inst.get_iterate()
    r = orc.admm_solve(osdp, maxiter=5, tol=0.0, sigma_every=0)
    assert blockwise_rel(Xg, r["X"], osdp.bsize) <= 1e-9
    assert blockwise_rel(Sg, r["S"], osdp.bsize) <= 1e-9
    inst.close()
    for bad in (dict(task_split=3), dict(block_rows=300)):
        with pytest.raises(S.StromError) as e:
            S.Instance(ctx, prob, _opts(S, **bad))
        assert e.value.code == -1


def test_serving_under_a_tight_budget_with_mixed_round_structures(S, ctx):
    """The request loop under an HBM budget that holds about two instances at a time (setup
    workers wait for retirements), with requests of two round structures (kkt_every 10 and 5,
    which go to separate batches): every request ends as it does alone."""
    import time
    import workloads as W
    probs = [S.generate(W.PENDULUM, 5 + k % 3, W.instance_params(W.PENDULUM, 40 + k)) for k in range(6)]
    optsets = [S.default_opts(), S.default_opts(kkt_every=5, sigma_every=50)]
    alone = []
    for k, pr in enumerate(probs):
        ins = S.Instance(ctx, pr, optsets[k % 2])
        alone.append(ins.step(50000))
        ins.close()
    budget = 1 << 16  # smallest power of two that holds the largest request, found by doubling
    while True:
        c = S.Context(0, hbm_budget=budget)
        try:
            S.Instance(c, probs[2]).close()
            c.close()
            break
        except S.StromError:
            c.close()
            budget *= 2
    small = S.Context(0, hbm_budget=2 * budget)
    tickets = [small.submit(pr, optsets[k % 2]) for k, pr in enumerate(probs)]
    done, t0 = {}, time.time()
    while len(done) < len(tickets):
        assert time.time() - t0 < 240, "request loop did not finish"
        for t in tickets:
            if t not in done:
                r = small.poll(t)
                if r is not None:
                    done[t] = r[0]
        time.sleep(0.01)
    small.close()
    for a, t in zip(alone, tickets):
        b = done[t]
        assert a["state"] == b["state"] == S.CONVERGED
        assert b["iters"] == a["iters"]
        assert abs(b["pobj"] - a["pobj"]) <= 1e-9 * (1.0 + abs(a["pobj"]))


@pytest.mark.parametrize("fam,N,prm", [(2, 4, [0.1, 0.2, 0.5, 0.3]), (4, 2, [1, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1]),
                                       (8, 2, [0.1, 0.2, 0.3, 0.5])])
def test_fp32_admm_projection_per_block(S, ctx, orc, fam, N, prm):
    """The FP32 projection inside an iteration (warm-started from the eigenvectors the previous
    iterations kept): the device's Pi(X_b) = X_b + sigma S, block by block, against the oracle's
    FP64 projection of the same X_b, within 1e-5 of max(1, ||X_b||) per block.  X_b is formed on
    the host from the device iterate (y-solve through the oracle's factor), which agrees with the
    device's own X_b to rounding (~1e-12), far below the bound."""
    from parity_util import block_slices
    osdp = orc.relax(fam, N, prm)
    prob = S.generate(fam, N, prm)
    inst = S.Instance(ctx, prob, _opts(S, sigma_every=0, kkt_every=1, tol=0.0, proj_dtype=S.F32))
    inst.step(12)  # the eigenvectors of the 12th projection are kept for the next one
    X, _, Sv = inst.get_iterate()
    sigma = 1.0
    A = osdp.A
    ldl = orc.LDL(osdp)
    yh = ldl.solve(osdp.b / sigma - A @ (X / sigma + Sv - osdp.C))
    Xb = X + sigma * (A.T @ yh - osdp.C)
    inst.step(1)
    _, _, S2 = inst.get_iterate()
    got = Xb + sigma * S2
    ref = orc.project_svec(osdp.bsize, Xb)
    for n, s in zip(osdp.bsize, block_slices(osdp.bsize)):
        err = np.linalg.norm(got[s] - ref[s]) / max(1.0, np.linalg.norm(Xb[s]))
        assert err <= 1e-5, (int(n), err)
    inst.close()


def _family_refs():
    with open(os.path.join(os.path.dirname(__file__), "golden", "converged_refs_families.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", range(4))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_family_converged_vs_oracle(S, ctx, orc, case, dtype):
    """Cart-pole N = 6, the bicycle car N = 4 and the paper's cart-pole N = 3, solved on the device (FP64, or the FP32 projection
    with the FP64 polish) to tol 1e-8, the oracle's own accuracy: the oracle's KKT evaluation of
    the device iterate is <= 1e-6 and the objective is within 1e-6 of the oracle's optimum.  (At
    tol 1e-6 the objective of cart-pole N = 6 seed 0 is 3.4e-6 away in this normalization, and
    1.5e-6 away at 1e-7 after the FP32 phase: the termination rule's residuals leave out the cone
    part of primal feasibility, X's negative eigenvalues, which moves <C, X> too.)"""
    import workloads as W
    ref = _family_refs()[case]
    fam = {"cartpole": W.CARTPOLE, "car": W.CAR, "paper_cartpole": W.PAPER_CARTPOLE}[ref["family"]]
    prm = W.instance_params(fam, ref["seed"])
    assert np.allclose(ref["params"], prm, rtol=0, atol=0)
    prob = S.generate(fam, ref["N"], prm)
    inst = S.Instance(ctx, prob, S.default_opts(proj_dtype=dtype, maxiter=50000, tol=1e-8))
    info = inst.step(50000)
    assert info["state"] == S.CONVERGED, info
    X, y, Sv = inst.get_iterate()
    k = orc.kkt(orc.relax(fam, ref["N"], prm), X, y, Sv)
    assert max(k["eta_p"], k["eta_d"], k["eta_g"]) <= 1e-6 * 1.05, k
    gap = abs(info["pobj"] - ref["pobj"]) / (1 + abs(info["pobj"]) + abs(ref["pobj"]))
    assert gap <= 1e-6, (info["pobj"], ref["pobj"])
    inst.close()


def test_cartpole_full_size_converged_kkt(S, ctx, orc):
    """Cart-pole N = 30 (n_svec 101,790), seed 7, which reaches 1e-6 in a few hundred iterations:
    the converged device iterate passes the oracle's KKT check at 1e-6."""
    import workloads as W
    prm = W.instance_params(W.CARTPOLE, 7)
    inst = S.Instance(ctx, S.generate(W.CARTPOLE, 30, prm), S.default_opts(maxiter=20000))
    info = inst.step(20000)
    assert info["state"] == S.CONVERGED, info
    X, y, Sv = inst.get_iterate()
    k = orc.kkt(orc.relax(W.CARTPOLE, 30, prm), X, y, Sv)
    assert max(k["eta_p"], k["eta_d"], k["eta_g"]) <= 1e-6 * 1.05, k
    assert abs(k["pobj"] - info["pobj"]) <= 1e-9 * (1 + abs(info["pobj"]))
    inst.close()
