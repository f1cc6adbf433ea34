"""Coarse steps replayed as HIP graphs (LBM_OPT_GRAPHS) against the same steps with
every kernel launched by itself: bit-identical moments after every replay, with the
program's own work and synchronisations between replays (moments read back, particle
advance and grid update through the C-ABI, block-set changes that force new
captures), for lbm_step, lbm_step(n) and lbm_step_remesh, 2 and 3 levels."""
import numpy as np
import pytest
import torch

from paper_2603_14982_amd import workloads as W

pytestmark = pytest.mark.gpu

P = W.PERIODIC


def _sim(levels, graphs, storage="f32"):
    lbm = pytest.importorskip("paper_2603_14982_amd.lbm")
    n = (128, 128, 128)
    p = W.slab_particles(4000, 3, (24.0, 24.0, 72.0), (104.0, 104.0, 88.0))
    scale = [64.0, 8.0, 8.0, 8.0, 64.0, 64.0, 64.0, 64.0, 64.0, 64.0] if storage != "f32" else None
    sim = lbm.Sim(levels, n, (P,) * 6, 0.6, particles=p, storage=storage, scale=scale)
    for l in range(levels):
        keys = sim.block_keys(l).cpu().numpy()
        sim.set_block_moments(l, keys, W.tgv3d_field(l, keys, n, 0.05, pressure=True).astype(np.float32))
    sim.set_option("tile_min_blocks", 0)
    sim.set_option("graphs", 1 if graphs else 0)
    return sim, torch.as_tensor(p).cuda()


def _state(sim):
    out = []
    for l in range(sim.levels):
        k, v = sim.get_moments(l)
        out.append((k.cpu().numpy(), v.cpu().numpy()))
    return out


def _same(a, b, label):
    for l, ((ka, va), (kb, vb)) in enumerate(zip(a, b)):
        assert np.array_equal(ka, kb), f"{label} level {l}: block keys differ"
        assert np.array_equal(va, vb), f"{label} level {l}: moments differ"


@pytest.mark.parametrize("levels", [2, 3])
def test_graph_replays_match_eager_launches(levels):
    g, pg = _sim(levels, True)
    e, pe = _sim(levels, False)
    d = np.array([0.0, 0.0, -1.25], dtype=np.float32)
    changes = 0
    for it in range(8):
        # one coarse step at a time, then the caller's own work between replays
        g.step(1)
        e.step(1)
        torch.cuda.synchronize()
        _same(_state(g), _state(e), f"L={levels} step {it}")
        before = [g.num_blocks(l) for l in range(levels)]
        g.advance_particles(pg, d)
        g.remesh(pg)
        e.advance_particles(pe, d)
        e.remesh(pe)
        changes += before != [g.num_blocks(l) for l in range(levels)]
    # several steps per call
    g.step(3)
    e.step(3)
    _same(_state(g), _state(e), f"L={levels} after step(3)")
    assert changes >= 1  # at least one replay after a new capture on a changed hierarchy


def test_graph_step_remesh_and_profiling_match_eager():
    g, pg = _sim(3, True, storage="bf16")
    e, pe = _sim(3, False, storage="bf16")
    d = (0.0, 0.0, -1.25)
    for it in range(5):
        g.step_remesh(1, pg, d)
        e.step_remesh(1, pe, d)
        _same(_state(g), _state(e), f"step_remesh {it}")
    # with profiling on, the steps run eagerly and are timed
    g.set_profiling(True)
    g.step(2)
    prof = g.profile()
    g.set_profiling(False)
    e.step(2)
    assert prof["sc_pair"][1] == 4 and prof["sc1"][1] == 4 and prof["sc2"][1] == 2, prof
    _same(_state(g), _state(e), "profiled steps")
    g.step(2)
    e.step(2)
    _same(_state(g), _state(e), "graph replays after profiling")
