"""The Python binding rejects malformed arguments before anything reaches the library (CPU only):
a bad problem, iterates of the wrong length, poll buffers of the wrong size, and dense block
arguments with wrong index types, devices, float types or extents."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def S():
    import paper_2406_05846_amd as S
    return S


def _tiny(S, **over):
    # one 2x2 block (svec length 3), one row: trace = 1
    kw = dict(block_sizes=[2], rowptr=[0, 2], col=[0, 2], val=[1.0, 1.0], b=[1.0], C_svec=[1.0, 0.0, 2.0])
    kw.update(over)
    return S.Problem(**kw)


def test_problem_lengths(S):
    _tiny(S)
    _tiny(S, X0=np.zeros(3), S0=np.zeros(3))
    bad = [dict(C_svec=[1.0, 0.0]), dict(X0=np.zeros(4)), dict(S0=np.zeros(2)), dict(block_sizes=[0]),
           dict(rowptr=[0, 2, 2]), dict(val=[1.0]), dict(rowptr=[0, 3]), dict(block_sizes=[])]
    for kw in bad:
        with pytest.raises(S.StromError) as e:
            _tiny(S, **kw)
        assert e.value.code == -1, kw


def test_set_iterate_lengths(S):
    inst = S.Instance.__new__(S.Instance)
    inst.nsvec, inst.m, inst._h = 10, 4, None
    for kw in (dict(X=np.zeros(9)), dict(y=np.zeros(5)), dict(S=np.zeros(11))):
        with pytest.raises(S.StromError):
            inst.set_iterate(**kw)


def test_poll_buffers_follow_the_request(S):
    ctx = S.Context.__new__(S.Context)
    ctx._sizes, ctx._h = {7: (10, 4)}, None
    with pytest.raises(S.StromError):
        ctx.poll(7, 9, 4)  # short X / S buffers
    with pytest.raises(S.StromError):
        ctx.poll(7, 10, 3)
    with pytest.raises(S.StromError):
        ctx.poll(8, 10, 4)  # unknown ticket with sizes asked for


def test_dense_block_arguments(S):
    import torch
    from paper_2406_05846_amd import _check_dense_blocks as chk
    cpu = torch.device("cpu")
    n = torch.tensor([3, 2], dtype=torch.int32)
    o = torch.tensor([0, 9], dtype=torch.int64)
    x = torch.zeros(13, dtype=torch.float64)
    chk(n, o, x, x.clone(), 3, cpu)  # fits exactly
    bad = [
        (n.to(torch.int64), o, x, x, 3),             # sizes not int32
        (n, o.to(torch.int32), x, x, 3),             # offsets not int64
        (n, o, x, x.float(), 3),                     # out dtype differs
        (n, o, x.to(torch.int32), x, 3),             # not a float type
        (n, o, x[:12], x, 3),                        # second block past the end of in
        (n, o, x, x[:12], 3),                        # ... of out
        (n, o, x, x, 2),                             # a block above max_n
        (n, torch.tensor([0, -1]), x, x, 3),         # negative offset
        (n, o[:1], x, x, 3),                         # lengths differ
        (n, o, torch.zeros(26, dtype=torch.float64)[::2], x, 3),  # not contiguous
    ]
    for args in bad:
        with pytest.raises(S.StromError):
            chk(*args, cpu)
    with pytest.raises(S.StromError):  # wrong device
        chk(n, o, x, x, 3, torch.device("meta"))
