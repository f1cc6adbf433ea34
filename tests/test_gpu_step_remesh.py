"""lbm_step_remesh (a coarse step, the particle advance and the grid update, the
particle work on a second stream overlapping the step) against the three calls in
order, through the C ABI: two and three levels, particles moving fast enough that the
block set changes at every other update; particles, block keys and every moment equal
bit for bit (the same kernels run on the same data in the same order)."""
import numpy as np
import pytest
import torch

from paper_2603_14982_amd import workloads as W

pytestmark = pytest.mark.gpu

P = W.PERIODIC


@pytest.mark.parametrize("levels", [2, 3])
def test_step_remesh_equals_the_three_calls(levels):
    from paper_2603_14982_amd import lbm
    n = (128, 128, 128)
    host = W.slab_particles(3000, 6, (24.0, 24.0, 40.0), (104.0, 104.0, 56.0))
    u0 = W.smooth_random_velocity(n, 9, kmax=4.0, rms=0.02)
    sims, parts = [], []
    for _ in range(2):
        p = torch.as_tensor(host).cuda()
        sim = lbm.Sim(levels, n, (P,) * 6, 0.6, particles=p)
        for l in range(levels):
            keys = sim.block_keys(l).cpu().numpy()
            sim.set_block_moments(l, keys, W.velocity_moments(l, keys, u0).astype(np.float32))
        sims.append(sim)
        parts.append(p)
    d = (2.5, -1.0, 3.0)
    changes = 0
    for it in range(6):
        before = sims[0].block_keys(0).cpu().numpy()
        sims[0].step(1)
        sims[0].advance_particles(parts[0], d)
        sims[0].remesh(parts[0])
        after = sims[0].block_keys(0).cpu().numpy()
        changes += int(not np.array_equal(before, after))
    sims[1].step_remesh(2, parts[1], d)
    sims[1].step_remesh(4, parts[1], d)
    torch.cuda.synchronize()
    print(f"{levels} levels: level-0 block set changed at {changes} of 6 updates", flush=True)
    assert changes >= 2
    assert torch.equal(parts[0], parts[1])
    for l in range(levels):
        k0, v0 = sims[0].get_moments(l)
        k1, v1 = sims[1].get_moments(l)
        assert torch.equal(k0, k1), l
        assert torch.equal(v0, v1), l
