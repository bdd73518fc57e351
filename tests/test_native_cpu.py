"""Host-side checks of the native library (CPU only, no compute on the device).

* libstrom.so loads and exports every function declared in include/*.h;
* the product's own relaxation generator (strom_gen_*) reproduces the oracle's relaxation row
  by row -- two independent implementations of the same conventions;
* argument validation of the generator.
"""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(strom_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    import ctypes
    import paper_2406_05846_amd as S
    lib = ctypes.CDLL(S.LIB_PATH)
    declared = _declared_functions()
    assert len(declared) >= 20
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(S.EXPORTS) <= declared


def test_default_opts():
    import paper_2406_05846_amd as S
    o = S.default_opts()
    assert o.sigma0 == 1.0 and o.tau == 1.6 and o.tol == 1e-6 and o.kkt_every == 10 and o.sigma_every == 50
    assert o.task_split == -1 and o.block_rows == 0


CASES = [
    (0, 3, [2.0, 0.1, 1.0]),
    (1, 10, [0.5, 0.0]),
    (2, 6, [0.1, 0.2, 0.5, 0.3]),
    (3, 4, [0.3, 0.5]),
    (4, 3, [0, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1]),
    (4, 3, [1, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1]),
    (5, 2, [3.0, -2.0, 0.5, 0.5, -0.5, 0.2]),
    (6, 2, [5.0, 80.0, 0.1, 0.5, -1.0, 0.05]),
    (7, 2, [3.0, 4.0, 0.1]),
    (8, 3, [0.1, 0.2, 0.3, 0.5]),
    (8, 1, [-0.2, 0.4, -0.3, -0.8]),
]


@pytest.mark.parametrize("fam,N,prm", CASES)
def test_generators_agree(orc, fam, N, prm):
    import paper_2406_05846_amd as S
    p = S.generate(fam, N, prm)
    o = orc.relax(fam, N, prm)
    assert p.m == o.m and p.nsvec == o.nsvec
    assert np.array_equal(p.block_sizes, o.bsize)
    assert np.array_equal(p.rowptr, o.rowptr)
    assert np.array_equal(p.col, o.col)
    assert np.array_equal(p.row_kind, o.rowkind)
    assert np.abs(p.val - o.val).max() <= 4e-16
    assert np.abs(p.b - o.b).max() == 0.0
    assert np.abs(p.C - o.C).max() <= 1e-14 * max(1.0, np.abs(o.C).max())


def test_generator_rejects_bad_arguments():
    import paper_2406_05846_amd as S
    with pytest.raises(S.StromError):
        S.generate(9, 3, [0.0])
    with pytest.raises(S.StromError):
        S.generate(1, 0, [0.5, 0.0])
    with pytest.raises(S.StromError):
        S.generate(2, 3, [0.1])


def test_workloads_are_seeded():
    import workloads as W
    a = W.instance_params(W.CARTPOLE, 3)
    assert a == W.instance_params(W.CARTPOLE, 3)
    assert a != W.instance_params(W.CARTPOLE, 4)
    b = W.mixed_batch(0, 16)
    assert b == W.mixed_batch(0, 16)
    assert all(10 <= N <= 60 for _, N, _ in b)
    car = W.instance_params(W.CAR, 5)
    assert car[0] == 1.0  # odd seed -> bicycle-13
    r = W.poisson_arrivals(0, 100.0, 1.0)
    ts = [t for t, *_ in r]
    assert ts == sorted(ts) and 50 < len(ts) < 150


def test_shift_one_clique_moves_whole_cliques():
    """The receding-horizon warm start moves clique k+1's blocks to clique k and repeats the
    last clique (blocks in clique order, the moment block of each clique first)."""
    import workloads as W
    sizes = [5, 2, 2, 5, 2, 2, 5, 2, 2]  # three cliques: one moment block and two localizing each
    lens = [n * (n + 1) // 2 for n in sizes]
    x = np.arange(float(sum(lens)))
    per = sum(lens[:3])
    out = W.shift_one_clique(sizes, x)
    assert out.shape == x.shape
    assert np.array_equal(out[:per], x[per:2 * per])
    assert np.array_equal(out[per:2 * per], x[2 * per:])
    assert np.array_equal(out[2 * per:], x[2 * per:])


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it says so and exits before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_trace_bounds_agree_with_the_oracle(orc):
    import paper_2406_05846_amd as S
    import workloads as W
    for fam, N, seed in [(W.CARTPOLE, 5, 0), (W.CAR, 4, 0), (W.CAR, 4, 1), (W.PAPER_PENDULUM, 3, 0), (W.FLYING, 2, 0),
                         (W.LANDING, 2, 0), (W.BACKIN, 2, 0), (W.BACKIN, 30, 1), (W.PAPER_CARTPOLE, 3, 0),
                         (W.PAPER_CARTPOLE, 3, 1)]:
        prm = W.instance_params(fam, seed)
        ref = orc.trace_bounds(fam, N, prm)
        got = S.generate(fam, N, prm).trace_bounds
        assert got is not None and np.array_equal(got, ref), (fam, N)
    assert S.generate(W.PENDULUM, 3, W.instance_params(W.PENDULUM, 0)).trace_bounds is None
