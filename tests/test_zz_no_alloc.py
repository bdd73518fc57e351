"""strom_dual_bound_noalloc (static per-device work buffer, no device allocation) against
strom_dual_bound (per-call allocation) through the C ABI: two calls in a row on different
instances, the second smaller, each equal to the allocating entry point's result bit for bit
(the same kernels on the same inputs), and the eigenvalues checked against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_dual_bound_noalloc_matches_allocating_entry_point(orc):
    import torch
    assert torch.cuda.is_available()
    import paper_2406_05846_amd as S
    import workloads as W
    ctx = S.Context(0)
    assert S.lib().strom_scratch_bytes() == 32 << 20
    cases = [(W.CARTPOLE, 8, W.instance_params(W.CARTPOLE, 3)), (W.PENDULUM, 3, W.instance_params(W.PENDULUM, 1))]
    for fam, N, prm in cases:  # the second instance is smaller than the first
        prob = S.generate(fam, N, prm)
        inst = S.Instance(ctx, prob, S.default_opts(sigma_every=0, tol=0.0))
        inst.step(30)
        R = np.linspace(1.0, 3.0, len(prob.block_sizes))
        lb_a, lam_a = inst.dual_bound(R)
        lb_n, lam_n = inst.dual_bound(R, noalloc=True)
        assert lb_n == lb_a and np.array_equal(lam_n, lam_a), (fam, N)
        # and both agree with the oracle's bound at the device's y
        _, y, _ = inst.get_iterate()
        ref_lb, ref_lam = orc.dual_bound(orc.relax(fam, N, prm), y, R)
        assert np.max(np.abs(lam_n - ref_lam)) <= 1e-9 * max(1.0, np.max(np.abs(ref_lam)))
        assert abs(lb_n - ref_lb) <= 1e-9 * max(1.0, abs(ref_lb))
        inst.close()
    ctx.close()
