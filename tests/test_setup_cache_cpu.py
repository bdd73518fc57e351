"""The host analysis's pattern cache (no GPU needed): an instance whose sparsity pattern was
analysed before (same family, variant and horizon; another initial state or obstacle) reuses
the symbolic part and recomputes only the numbers.  tests/native/setup_cache_check.cpp checks
that this gives, field by field and bit for bit, the analysis from scratch, and that the
parallel factorization (tasks of one dependency level in threads) gives the one-thread bits."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("cache") / "setup_cache_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", out,
                    os.path.join(ROOT, "tests", "native", "setup_cache_check.cpp"),
                    os.path.join(ROOT, "paper_2406_05846_amd", "csrc", "setup.cpp")], check=True)
    return out


@pytest.mark.parametrize("fam,N,seeds", [(1, 8, (0, 1)), (2, 8, (0, 3)), (4, 5, (0, 2)), (4, 5, (1, 3))])
def test_cached_analysis_equals_fresh(exe, tmp_path, fam, N, seeds):
    import paper_2406_05846_amd as S
    import workloads as W
    pa, pb = (S.generate(fam, N, W.instance_params(fam, s)) for s in seeds)
    assert np.array_equal(pa.rowptr, pb.rowptr) and np.array_equal(pa.col, pb.col)
    assert not np.array_equal(pa.val, pb.val)
    d = str(tmp_path)
    pa.block_sizes.tofile(d + "/bs")
    pa.rowptr.tofile(d + "/rp")
    pa.col.tofile(d + "/ci")
    pa.val.tofile(d + "/av_a")
    pb.val.tofile(d + "/av_b")
    r = subprocess.run([exe, d], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "identical" in r.stdout
