"""The device solve schedule, executed on the CPU (no GPU needed).

tests/native/solve_schedule_sim.cpp runs the library's host analysis (row order, FP64 LDL^T,
task split, phases, component inverses, push segments, task-local staging, phase streams,
launch groups, the top levels of the coupling sets' dissection tree merged into the root task)
and then walks the schedule exactly as the solve kernels read it.  Its
y = (eps I + A A^*)^{-1} r must match the oracle's own sparse factorization: a schedule that
drops, doubles or misindexes a stream entry, or runs a task before one it depends on, fails
here.  Every case runs with the task split of every group task, of the overweight ones only
and none, with every task staged in LDS, some staged, and none (the in-place kernel
path), and with the groups' interior rows in their own order and in minimum-degree order (by
default the analysis keeps the one whose schedule has fewer stream entries on the longest
path, the largest task of every launch group; with the throughput schedule of merged batches,
task split 1, the one with fewer entries in all).
"""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = [  # (family, N, parameters): pendulum, cart-pole, car, the paper's cart-pole (the split applies to the first two)
    (1, 10, [0.5, 0.0]),
    (2, 10, [0.1, 0.2, 0.5, 0.3]),
    (4, 4, [1, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1]),
    (8, 4, [0.1, 0.2, 0.3, 0.5]),  # the paper's cart-pole: 330-row coupling sets (7 shared variables)
]
VARIANTS = [  # environment of the analysis
    {},
    {"STROM_TASK_SPLIT": "0"},
    {"STROM_TASK_SPLIT": "1"},
    {"STROM_STAGE_ROWS": "0"},
    {"STROM_STAGE_ROWS": "600", "STROM_BLOCK_ROWS": "32"},
    {"STROM_TOP_LEVELS": "1"},  # only the root coupling set in the root task
    {"STROM_TOP_LEVELS": "4"},  # the top four levels of the dissection tree in one task
    {"STROM_ROW_ORDER": "0"},  # the interior rows of every group in their own order
    {"STROM_ROW_ORDER": "1"},  # ... in minimum-degree order
    {"STROM_TASK_SPLIT": "1", "STROM_ROW_ORDER": "0"},  # the throughput schedule in both orders
    {"STROM_TASK_SPLIT": "1", "STROM_ROW_ORDER": "1"},
]


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sim") / "solve_schedule_sim")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe,
                    os.path.join(ROOT, "tests", "native", "solve_schedule_sim.cpp"),
                    os.path.join(ROOT, "paper_2406_05846_amd", "csrc", "setup.cpp")], check=True)
    return exe


@pytest.mark.parametrize("fam,N,prm", CASES)
def test_schedule_solves_the_system(sim, orc, tmp_path, fam, N, prm):
    p = orc.relax(fam, N, prm)
    A = p.A.tocsr()
    rng = np.random.default_rng(fam * 100 + N)
    r = A @ rng.standard_normal(p.nsvec)
    F = orc.LDL(p)
    yo = F.solve(r)
    for name, arr in [("bs", np.asarray(p.bsize, dtype=np.int32)), ("rp", A.indptr.astype(np.int64)),
                      ("ci", A.indices.astype(np.int32)), ("av", A.data.astype(np.float64)), ("r", r)]:
        arr.tofile(str(tmp_path / name))
    tasks = {}
    for env in VARIANTS:
        out = subprocess.run([sim, str(tmp_path)], env={**os.environ, **env}, capture_output=True, text=True)
        assert out.returncode == 0, (env, out.stdout, out.stderr)
        fields = out.stdout.split()
        tasks[tuple(sorted(env.items()))] = dict(zip(fields[0::2], map(int, fields[1::2])))
        y = np.fromfile(str(tmp_path / "y"))
        resid = A @ (A.T @ y) + F.eps * y - r
        assert np.linalg.norm(resid) <= 1e-12 * np.linalg.norm(r), env
        # same system, two factorizations in different orders: agree to rounding
        assert np.linalg.norm(A.T @ (y - yo)) <= 1e-10 * np.linalg.norm(A.T @ yo), env
    base = tasks[()]
    assert base["staged"] == base["tasks"]
    assert tasks[(("STROM_STAGE_ROWS", "0"),)]["staged"] == 0
    assert base["fwd_groups"] == tasks[(("STROM_TASK_SPLIT", "0"),)]["fwd_groups"]  # no added depth
    if fam in (1, 2):  # the first clique carries the initial-state rows: its task is split
        assert base["tasks"] > tasks[(("STROM_TASK_SPLIT", "0"),)]["tasks"]
        assert base["fwd_groups"] == tasks[(("STROM_TASK_SPLIT", "0"),)]["fwd_groups"]
    nat, md = tasks[(("STROM_ROW_ORDER", "0"),)], tasks[(("STROM_ROW_ORDER", "1"),)]
    assert md["nnzL"] < nat["nnzL"]  # minimum degree: less fill
    pick = md if md["solve_entries"] < nat["solve_entries"] else nat
    assert (base["nnzL"], base["solve_entries"]) == (pick["nnzL"], pick["solve_entries"])
    # the throughput schedule (task split 1, merged batches) keeps the order with fewer entries in all
    s1 = tasks[(("STROM_TASK_SPLIT", "1"),)]
    nat1 = tasks[(("STROM_ROW_ORDER", "0"), ("STROM_TASK_SPLIT", "1"))]
    md1 = tasks[(("STROM_ROW_ORDER", "1"), ("STROM_TASK_SPLIT", "1"))]
    pick1 = md1 if md1["total_entries"] < nat1["total_entries"] else nat1
    assert (s1["nnzL"], s1["total_entries"]) == (pick1["nnzL"], pick1["total_entries"])
