"""GPU tests of the merged form (strom_batch_*): instances of different families and sizes
advanced together, one launch per step over all of them, through the C ABI.  Each instance
must follow the iterates it follows alone (same kernels, same thread counts per block), and
those of the oracle; retired instances must stay unchanged."""
import numpy as np
import pytest
from parity_util import blockwise_rel

pytestmark = pytest.mark.gpu

CAR_PRM = [1, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1]


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


def _cases():
    import workloads as W
    return [(W.PENDULUM, 5, [0.5, 0.0]), (W.CARTPOLE, 3, [0.1, 0.2, 0.5, 0.3]), (W.CAR, 3, CAR_PRM),
            (W.PENDULUM, 12, [-2.0, 0.4]), (W.PAPER_CARTPOLE, 2, [0.1, 0.2, 0.3, 0.5])]


def _rel(a, b):
    return np.linalg.norm(a - b) / max(1.0, np.linalg.norm(b))


def _brel(a, b, osdp):
    return blockwise_rel(a, b, osdp.bsize)


def test_batch_fixed_sigma_iterates_match_alone_and_oracle(S, ctx, orc):
    """25 iterations with a fixed sigma (a first round launched directly, one graph round, a
    partial round): every instance of the batch equals its own run alone and the oracle's."""
    cases = _cases()
    opts = S.default_opts(sigma_every=0, tol=0.0)
    alone = []
    for fam, N, prm in cases:
        ins = S.Instance(ctx, S.generate(fam, N, prm), opts)
        ins.step(25)
        alone.append(ins.get_iterate())
        ins.close()
    insts = [S.Instance(ctx, S.generate(fam, N, prm), opts) for fam, N, prm in cases]
    bat = S.Batch(ctx, insts)
    infos = bat.step(25)
    assert [i["iters"] for i in infos] == [25] * len(cases)
    bat.close()
    for (fam, N, prm), ins, (Xa, ya, Sa) in zip(cases, insts, alone):
        Xg, yg, Sg = ins.get_iterate()
        assert _rel(Xg, Xa) <= 1e-12 and _rel(Sg, Sa) <= 1e-12, (fam, N)
        osdp = orc.relax(fam, N, prm)
        r = orc.admm_solve(osdp, maxiter=25, tol=0.0, sigma_every=0)
        assert _brel(Xg, r["X"], osdp) <= 1e-9 and _brel(Sg, r["S"], osdp) <= 1e-9, (fam, N)
        assert _rel(osdp.A.T @ yg, osdp.A.T @ r["y"]) <= 1e-9, (fam, N)
        ins.close()


def test_batch_converged_solves_match_alone_and_retire(S, ctx):
    """Default rules (sigma balancing, tol 1e-6), one instance with the FP32 projection and the
    FP64 polish: every instance converges at the iteration it converges alone, to the same
    objective, and stays unchanged once retired."""
    import workloads as W
    cases = [(W.PENDULUM, 6, [2.0, 0.0], "f64"), (W.PENDULUM, 8, [0.8, 0.0], "f32"),
             (W.PENDULUM, 5, [-1.2, 0.5], "f64")]
    alone = []
    for fam, N, prm, dt in cases:
        ins = S.Instance(ctx, S.generate(fam, N, prm), S.default_opts(proj_dtype=dt))
        alone.append(ins.step(50000))
        ins.close()
    insts = [S.Instance(ctx, S.generate(fam, N, prm), S.default_opts(proj_dtype=dt)) for fam, N, prm, dt in cases]
    bat = S.Batch(ctx, insts)
    infos = bat.step(50000)
    frozen = [ins.get_iterate()[0] for ins in insts]
    again = bat.step(100)
    for a, b, c in zip(alone, infos, again):
        assert a["state"] == b["state"] == S.CONVERGED
        assert b["iters"] == a["iters"], (a["iters"], b["iters"])
        assert abs(b["pobj"] - a["pobj"]) <= 1e-9 * (1.0 + abs(a["pobj"]))
        assert c["iters"] == b["iters"] and c["pobj"] == b["pobj"]
    for ins, X0 in zip(insts, frozen):
        assert np.array_equal(ins.get_iterate()[0], X0)
    bat.close()
    for ins in insts:
        ins.close()


def test_batch_tune_keeps_the_iterates(S, ctx, orc):
    """The autotuner picks a thread count per block class among those the kernel accepts; the
    iterates after it stay those of the oracle."""
    cases = _cases()[:3]
    opts = S.default_opts(sigma_every=0, tol=0.0, proj_dtype="f64")
    insts = [S.Instance(ctx, S.generate(fam, N, prm), opts) for fam, N, prm in cases]
    bat = S.Batch(ctx, insts)
    bat.step(10)
    cls = bat.tune(reps=2)
    assert len(cls) >= 2
    for n, t64, t32 in cls:
        assert t64 in (64, 128, 256, 512, 1024) and t64 >= n
    bat.step(10)
    bat.close()
    for (fam, N, prm), ins in zip(cases, insts):
        Xg, yg, Sg = ins.get_iterate()
        osdp = orc.relax(fam, N, prm)
        r = orc.admm_solve(osdp, maxiter=20, tol=0.0, sigma_every=0)
        assert _brel(Xg, r["X"], osdp) <= 1e-9 and _brel(Sg, r["S"], osdp) <= 1e-9, (fam, N)
        ins.close()


def test_batch_membership_is_enforced(S, ctx):
    import workloads as W
    ins = S.Instance(ctx, S.generate(W.PENDULUM, 4, [0.5, 0.0]))
    bat = S.Batch(ctx, [ins])
    with pytest.raises(S.StromError) as e:
        ins.step(1)
    assert e.value.code == -7
    with pytest.raises(S.StromError):
        S.Batch(ctx, [ins])  # already in a batch
    bat.step(1)
    bat.close()
    assert ins.step(1)["iters"] == 2
    ins.close()


def test_batch_members_at_different_iteration_counts(S, ctx):
    """An instance that has run a round joins a fresh one (their counts agree modulo kkt_every):
    each keeps its own sigma schedule, so after 50 batched iterations each equals its own run
    alone (60 and 50 iterations, default sigma rule)."""
    import workloads as W
    pa, pb = S.generate(W.PENDULUM, 5, [0.7, 0.0]), S.generate(W.PENDULUM, 6, [-1.9, 0.3])
    opts = S.default_opts(tol=0.0)
    ref = []
    for pr, n in ((pa, 60), (pb, 50)):
        ins = S.Instance(ctx, pr, opts)
        info = ins.step(n)
        ref.append((info, ins.get_iterate()))
        ins.close()
    a, b = S.Instance(ctx, pa, opts), S.Instance(ctx, pb, opts)
    a.step(10)
    bat = S.Batch(ctx, [a, b])
    infos = bat.step(50)
    assert bat.step(0) == infos  # no iteration: the same state again
    bat.close()
    for ins, inf, (ri, (Xr, yr, Sr)) in zip((a, b), infos, ref):
        assert inf["iters"] == ri["iters"] and inf["sigma"] == ri["sigma"]
        X, y, Sv = ins.get_iterate()
        assert _rel(X, Xr) <= 1e-12 and _rel(Sv, Sr) <= 1e-12
        ins.close()


def test_batch_rejects_mismatched_rounds(S, ctx):
    import workloads as W
    pr = S.generate(W.PENDULUM, 4, [0.5, 0.0])
    a, b = S.Instance(ctx, pr), S.Instance(ctx, pr, S.default_opts(kkt_every=5, sigma_every=50))
    with pytest.raises(S.StromError) as e:
        S.Batch(ctx, [a, b])
    assert e.value.code == -1
    c = S.Instance(ctx, pr)
    c.step(5)  # mid-round: its count differs from a's modulo kkt_every
    with pytest.raises(S.StromError) as e:
        S.Batch(ctx, [a, c])
    assert e.value.code == -1
    for ins in (a, b, c):
        ins.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-9), ("f32", 1e-4)])
def test_full_batch_sampled_against_the_oracle(S, ctx, orc, dtype, tol):
    """The whole 256-instance mixed batch (families uniform, N ~ U{10..60}) in the benchmark's
    launch configuration (task split 1, 64-row components, merged launches), with a fixed sigma
    for three iterations, in FP64 and with the FP32 projection (the FP32 form's iterates differ
    from the FP64 oracle's by the float rounding of the projection, ~1e-6 per block and
    iteration: bound 1e-4); the smallest instance of each family is checked against the oracle,
    which can afford those one at a time."""
    from concurrent.futures import ThreadPoolExecutor
    import workloads as W
    cases = W.mixed_batch(0, count=256, nmin=10, nmax=60)
    opts = S.default_opts(sigma_every=0, tol=0.0, task_split=1, block_rows=64, proj_dtype=dtype)
    probs = [S.generate(f, N, p) for f, N, p in cases]
    with ThreadPoolExecutor(max_workers=16) as ex:
        insts = list(ex.map(lambda pr: S.Instance(ctx, pr, opts), probs))
    bat = S.Batch(ctx, insts)
    infos = bat.step(3)
    bat.close()
    assert all(i["iters"] == 3 for i in infos)
    picks = {}
    for k, (f, N, _) in enumerate(cases):
        if f not in picks or N < cases[picks[f]][1]:
            picks[f] = k
    assert len(picks) == 3
    for k in picks.values():
        f, N, prm = cases[k]
        Xg, yg, Sg = insts[k].get_iterate()
        osdp = orc.relax(f, N, prm)
        r = orc.admm_solve(osdp, maxiter=3, tol=0.0, sigma_every=0)
        assert _brel(Xg, r["X"], osdp) <= tol and _brel(Sg, r["S"], osdp) <= tol, (f, N)
        assert _rel(osdp.A.T @ yg, osdp.A.T @ r["y"]) <= tol, (f, N)
    for ins in insts:
        ins.close()
