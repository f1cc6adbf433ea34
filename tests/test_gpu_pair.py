"""The finest level's two substeps of a parent step in one tiled sweep, against the
same steps taken as two sweeps and against the FP64 oracle. The tile threshold is
set to zero so that levels of a few hundred blocks run on tiles (partial tiles,
ghost shells and periodic wrap inside a tile's two-node halo all occur); the
grid is updated after every coarse step."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W
from tests.test_gpu_parity import compare, setup_pair
from tests.util import group_errors

pytestmark = pytest.mark.gpu

P = W.PERIODIC


def _moments(sim):
    out = []
    for l in range(sim.levels):
        k, v = sim.get_moments(l)
        out.append((k.cpu().numpy(), v.cpu().numpy().astype(np.float64), sim.roles(l).cpu().numpy()))
    return out


def _agree(a, b, tol, label):
    """Two GPU runs: identical block sets and roles, moments of the owned (non-ghost)
    nodes within tol (relative L2 per group; 0: bit-identical). Ghost values are excluded: at the end of
    a coarse step two sweeps leave the first substep's ghosts in the current time level
    and one sweep the second's; both are overwritten before they are read."""
    for l, ((ka, _, ra), (kb, _, rb)) in enumerate(zip(a, b)):
        assert np.array_equal(ka, kb), f"{label} level {l}: block keys differ"
        assert np.array_equal(ra, rb), f"{label} level {l}: roles differ"
    own = np.concatenate([(r & 7) != 1 for _, _, r in a])
    errs = group_errors(np.concatenate([v for _, v, _ in a]), np.concatenate([v for _, v, _ in b]), mask=own)
    print(label, errs, flush=True)
    for g, e in errs.items():
        assert e <= tol, f"{label}: {g} differs by {e:.3e}"


def _slab_run(levels, storage="f32", fuse=True, steps=6, oracle=False, pair_run=None, switch=None, zr=(72.0, 88.0)):
    """pair_run: tiles per z run of the one-sweep form (None: the default); switch: the
    value it takes from the middle coarse step on; zr: the slab's z extent"""
    lbm = pytest.importorskip("paper_2603_14982_amd.lbm")
    n = (128, 128, 128)
    p = W.slab_particles(4000, 3, (24.0, 24.0, zr[0]), (104.0, 104.0, zr[1]))
    init = lambda l, k: W.tgv3d_field(l, k, n, 0.05, pressure=True)
    scale = [64.0, 8.0, 8.0, 8.0, 64.0, 64.0, 64.0, 64.0, 64.0, 64.0] if storage != "f32" else None
    if oracle:
        gpu, ora = setup_pair(levels, n, (P,) * 6, 0.6, init, particles=p, storage=storage, scale=scale)
    else:
        gpu = lbm.Sim(levels, n, (P,) * 6, 0.6, particles=p, storage=storage, scale=scale)
        for l in range(levels):
            keys = gpu.block_keys(l).cpu().numpy()
            gpu.set_block_moments(l, keys, init(l, keys).astype(np.float32))
        ora = None
    gpu.set_option("tile_min_blocks", 0)
    if fuse is not None:  # None: the default (one sweep with every storage format)
        gpu.set_option("fuse_substeps", 2 if fuse else 0)
    if pair_run is not None:
        gpu.set_option("pair_run", pair_run)
    gpu.set_profiling(True)
    pg = torch.as_tensor(p).cuda()
    po = p.copy()
    d = np.array([0.0, 0.0, -1.25], dtype=np.float32)
    for it in range(steps):
        if switch is not None and it == steps // 2:
            gpu.set_option("pair_run", switch)  # regroups the current hierarchy's tiles
        gpu.step(1)
        gpu.advance_particles(pg, d)
        gpu.remesh(pg)
        if ora is not None:
            ora.step(1)
            O.advance_particles(po, d)
            ora.remesh(po)
    prof = gpu.profile()
    return gpu, ora, prof


@pytest.mark.parametrize("levels", [2, 3])
def test_pair_against_oracle_and_two_sweeps(levels):
    gpu, ora, prof = _slab_run(levels, oracle=True)
    # every parent step of level 1 ran the finest level's substeps as one sweep
    assert prof["sc_pair"][1] == 6 * 2 ** (levels - 2) and prof["sc0"][1] == 0, prof
    compare(gpu, ora, label=f"pair L={levels}")
    two, _, prof2 = _slab_run(levels, fuse=False)
    assert prof2["sc_pair"][1] == 0 and prof2["sc0"][1] == 6 * 2 ** (levels - 1)
    # the reconstruction fixes its own roundings (no contraction left to the compiler),
    # so both paths evaluate the same operations in the same order: bit-identical
    _agree(_moments(gpu), _moments(two), 0.0, f"pair vs two sweeps L={levels}")


@pytest.mark.parametrize("run,switch", [(1, None), (2, None), (3, 6), (5, None), (6, 1)])
def test_pair_z_runs_bit_identical(run, switch):
    # a slab 80 nodes deep: columns of up to 6 tiles along z, cut into runs of up to
    # `run` tiles (and regrouped halfway through); every grouping computes the same
    # operations as two sweeps
    zr = (24.0, 104.0)
    a, _, pa = _slab_run(3, pair_run=run, switch=switch, zr=zr, steps=4)
    b, _, pb = _slab_run(3, fuse=False, zr=zr, steps=4)
    assert pa["sc_pair"][1] == 8 and pb["sc_pair"][1] == 0, (pa, pb)
    _agree(_moments(a), _moments(b), 0.0, f"runs of {run} (then {switch})")


@pytest.mark.parametrize("storage,run", [("bf16", None), ("f16", None), ("bf16", 4), ("f16", 1)])
def test_pair_half_precision_matches_two_sweeps(storage, run):
    # the intermediate moments go through the storage format as if stored and read back;
    # any run length (None: the default with 16-bit storage) gives the same result
    zr = (24.0, 104.0) if run else (72.0, 88.0)
    a, _, pa = _slab_run(2, storage=storage, fuse=True, steps=4, pair_run=run, zr=zr)
    b, _, pb = _slab_run(2, storage=storage, fuse=False, steps=4, zr=zr)
    assert pa["sc_pair"][1] == 4 and pb["sc_pair"][1] == 0
    _agree(_moments(a), _moments(b), 0.0, f"pair {storage} runs of {run}")


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_default_fuses_substeps_with_every_storage(storage):
    _, _, prof = _slab_run(2, storage=storage, fuse=None, steps=2)
    assert prof["sc_pair"][1] == 2 and prof["sc0"][1] == 0, prof


def test_fuse_option_one_fuses_with_f32_storage_only():
    lbm = pytest.importorskip("paper_2603_14982_amd.lbm")
    sim = lbm.Sim(2, (64, 64, 64), (P,) * 6, 0.6, particles=W.slab_particles(300, 5, (8.0, 8.0, 8.0), (56.0, 56.0, 24.0)),
                  storage="bf16", scale=[64.0, 8.0, 8.0, 8.0, 64.0, 64.0, 64.0, 64.0, 64.0, 64.0])
    sim.set_option("tile_min_blocks", 0)
    sim.set_option("fuse_substeps", 1)
    sim.set_profiling(True)
    sim.step(1)
    prof = sim.profile()
    assert prof["sc_pair"][1] == 0 and prof["sc0"][1] == 2, prof


def test_pair_not_used_with_bounce_back_or_outflow():
    # no-slip walls at the z faces, with the finest level next to the lower one: its
    # bounce-back nodes keep it on two sweeps per parent step (on the oracle)
    lbm = pytest.importorskip("paper_2603_14982_amd.lbm")
    n = (64, 64, 64)
    bc = (P, P, P, P, W.WALL, W.WALL)
    p = W.slab_particles(300, 5, (8.0, 8.0, 1.0), (56.0, 56.0, 6.0))
    u0 = W.smooth_random_velocity(n, 21, kmax=3.0, rms=0.03)
    gpu, ora = setup_pair(2, n, bc, 0.6, lambda l, k: W.velocity_moments(l, k, u0), particles=p)
    # computed finest-level nodes on the first plane (next to the wall): bounce-back nodes
    pos = W.node_positions(0, ora.block_keys(0))
    assert ((pos[..., 2] == 0) & (ora.roles(0) == O.R_INTERIOR)).any()
    gpu.set_option("tile_min_blocks", 0)
    gpu.set_profiling(True)
    gpu.step(3)
    ora.step(3)
    prof = gpu.profile()
    assert prof["sc_pair"][1] == 0 and prof["sc0"][1] == 6, prof
    compare(gpu, ora, label="walls, tiled, two sweeps")


def test_options_rejected_values():
    lbm = pytest.importorskip("paper_2603_14982_amd.lbm")
    sim = lbm.Sim(1, (16, 16, 16), (P,) * 6, 0.6)
    with pytest.raises(lbm.LBMError):
        sim.set_option("tile_min_blocks", -1)
    with pytest.raises(lbm.LBMError):
        sim.set_option("fuse_substeps", 3)
    with pytest.raises(lbm.LBMError):
        sim.set_option("graphs", 2)
    for v in (0, 7):
        with pytest.raises(lbm.LBMError):
            sim.set_option("pair_run", v)
    assert lbm.lib().lbm_set_option(sim.h, 7, 0) == -1  # unknown option


def test_profiling_phase_mask():
    # timing only the fused finest-level launches leaves every other phase untimed
    lbm = pytest.importorskip("paper_2603_14982_amd.lbm")
    p = W.slab_particles(300, 5, (8.0, 8.0, 8.0), (56.0, 56.0, 24.0))
    sim = lbm.Sim(2, (64, 64, 64), (P,) * 6, 0.6, particles=p)
    sim.set_option("tile_min_blocks", 0)
    sim.set_profiling(True, phases=["sc_pair"])
    sim.step(2)
    prof = sim.profile()
    assert prof["sc_pair"][1] == 2, prof
    assert all(n == 0 for k, (_, n) in prof.items() if k != "sc_pair"), prof
    sim.set_profiling(True)
    sim.step(1)
    prof = sim.profile()
    assert prof["sc_pair"][1] == 1 and prof["sc1"][1] == 1, prof
    assert lbm.lib().lbm_set_profiling_phases(sim.h, 1 << len(lbm.PROFILE_PHASES)) == -1
