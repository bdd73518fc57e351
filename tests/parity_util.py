"""Comparison helpers shared by the GPU parity tests (no method arithmetic)."""
import numpy as np


def block_slices(block_sizes):
    off = 0
    for n in block_sizes:
        t = int(n) * (int(n) + 1) // 2
        yield slice(off, off + t)
        off += t


def blockwise_rel(got, ref, block_sizes):
    """max over PSD blocks of ||got_b - ref_b|| / max(1, ||ref_b||) on svec vectors, so a small
    block's error cannot hide under the norm of the large ones."""
    worst = 0.0
    for s in block_slices(block_sizes):
        d = np.linalg.norm(got[s] - ref[s]) / max(1.0, np.linalg.norm(ref[s]))
        worst = max(worst, d)
    return worst
