"""lbm_reduce_f64_noalloc (the FP64 sums with their partials in the library's static
device array, for callers that cannot allocate) against lbm_reduce_f64 (partials in
the meta buffer) through the C ABI: the same kernels in the same order, so the sums
agree bit for bit; two calls in a row, the second over fewer blocks than the first,
so a stale partial of the first call would show."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2603_14982_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_reduction_matches_the_workspace_reduction():
    from paper_2603_14982_amd import lbm
    L = lbm.lib()
    n = (64, 64, 64)
    particles = W.slab_particles(200, 7, (18.0, 18.0, 30.0), (46.0, 46.0, 38.0))
    sim = lbm.Sim(2, n, (W.PERIODIC,) * 6, 0.6, particles=particles)
    for l in range(2):
        keys = sim.block_keys(l).cpu().numpy()
        sim.set_block_moments(l, keys, W.tgv3d_field(l, keys, n, 0.05, pressure=True).astype(np.float32))
    sim.step(2)
    nb = [sim.num_blocks(l) for l in range(2)]
    print("blocks per level", nb, flush=True)
    big = int(np.argmax(nb))
    calls = [(big, (0, 0, 0), n), (1 - big, (8, 16, 0), (56, 48, 40))]
    assert nb[calls[1][0]] < nb[calls[0][0]]
    out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    for level, lo, hi in calls:
        lo_ = (ctypes.c_int32 * 3)(*lo)
        hi_ = (ctypes.c_int32 * 3)(*hi)
        st = L.lbm_reduce_f64_noalloc(sim.h, level, lo_, hi_, ctypes.c_void_p(out.data_ptr()))
        assert st == 0, L.lbm_last_error(sim.h)
        got = out.cpu().numpy()
        ref = (ctypes.c_double * 5)()
        assert L.lbm_reduce_f64(sim.h, level, lo_, hi_, ref) == 0
        ref = np.array(list(ref))
        print(f"level {level} box {lo}..{hi}: {got}", flush=True)
        assert np.array_equal(got, ref), (level, got, ref)
        assert got[0] > 0
