"""Failure handling through the C ABI (GPU): an instance whose iterate turns NaN retires as
DIVERGED at its next residual check while the others of its batch, or of the request loop,
finish exactly as they do alone; an iteration cap ends a solve as MAXITER; a factorization
that overflows is refused with E_FACTOR.  NaN arithmetic only: every kernel's loops are
bounded by counts, so nothing here can fault or hang the device."""
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


def _probs(S):
    import workloads as W
    return [S.generate(W.PENDULUM, 5 + k, W.instance_params(W.PENDULUM, 60 + k)) for k in range(3)]


def _alone(S, ctx, probs):
    out = []
    for pr in probs:
        ins = S.Instance(ctx, pr)
        out.append(ins.step(50000))
        ins.close()
    return out


def test_nan_instance_retires_diverged_in_a_batch(S, ctx):
    probs = _probs(S)
    alone = _alone(S, ctx, probs)
    insts = [S.Instance(ctx, pr) for pr in probs]
    bad = np.zeros(probs[1].nsvec)
    bad[5] = np.nan
    insts[1].set_iterate(X=bad)
    bat = S.Batch(ctx, insts)
    infos = bat.step(50000)
    bat.close()
    assert infos[1]["state"] == S.DIVERGED and infos[1]["iters"] <= 10
    for k in (0, 2):
        assert infos[k]["state"] == S.CONVERGED
        assert infos[k]["iters"] == alone[k]["iters"]
        assert infos[k]["pobj"] == alone[k]["pobj"]
    for ins in insts:
        ins.close()


def test_nan_request_retires_diverged_in_the_request_loop(S, ctx):
    probs = _probs(S)
    alone = _alone(S, ctx, probs)
    bad = probs[1]
    x0 = np.zeros(bad.nsvec)
    x0[3] = np.nan
    reqs = [probs[0], S.Problem(bad.block_sizes, bad.rowptr, bad.col, bad.val, bad.b, bad.C, X0=x0), probs[2]]
    tickets = [ctx.submit(pr) for pr in reqs]
    done, t0 = {}, time.time()
    while len(done) < len(tickets):
        assert time.time() - t0 < 120, "request loop did not finish"
        for t in tickets:
            if t not in done:
                r = ctx.poll(t)
                if r is not None:
                    done[t] = r[0]
        time.sleep(0.01)
    infos = [done[t] for t in tickets]
    assert infos[1]["state"] == S.DIVERGED
    for k in (0, 2):
        assert infos[k]["state"] == S.CONVERGED and infos[k]["iters"] == alone[k]["iters"]
        assert abs(infos[k]["pobj"] - alone[k]["pobj"]) <= 1e-12 * (1 + abs(alone[k]["pobj"]))


def test_iteration_cap_ends_as_maxiter(S, ctx):
    import workloads as W
    pr = S.generate(W.CARTPOLE, 4, W.instance_params(W.CARTPOLE, 0))
    for cap in (1, 25):
        ins = S.Instance(ctx, pr, S.default_opts(maxiter=cap))
        info = ins.step(1000)
        assert info["state"] == S.MAXITER and info["iters"] == cap, info
        again = ins.step(10)  # a retired instance does not move
        assert again["iters"] == cap
        ins.close()


def test_overflowing_factorization_is_refused(S, ctx):
    import workloads as W
    pr = S.generate(W.PENDULUM, 3, W.instance_params(W.PENDULUM, 0))
    val = pr.val.copy()
    val[pr.rowptr[7]:pr.rowptr[8]] = 1e160  # (A A^*)_77 overflows the double range
    bad = S.Problem(pr.block_sizes, pr.rowptr, pr.col, val, pr.b, pr.C)
    with pytest.raises(S.StromError) as e:
        S.Instance(ctx, bad)
    assert e.value.code == -4, e.value
