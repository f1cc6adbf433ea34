"""Full-size GPU checks in the launch configuration the benchmark times.

- The two-level sphere case (128^3, 500 coarse steps; also with BF16 and FP16
  storage, against the FP64 sample and the FP32-storage run) and the three-level slab
  case (512^3, 2M particles, 20 coarse steps with grid updates) against stored
  samples of the FP64 oracle's state (tests/golden/, written by
  tests/golden/make_golden.py from the oracle alone).
- The three-level slab case over its full 200 coarse steps: the block sets after
  every grid update equal the canonical hierarchy of the particle positions,
  computed by a set brute force; moments stay finite; the kinetic energy of the
  coarse bottom half decays at the viscous rate.
"""
import os

import numpy as np
import pytest
import torch

from paper_2603_14982_amd import workloads as W
from tests.util import canonical_sets

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lbm():
    from paper_2603_14982_amd import lbm
    return lbm


def _compare_sample(sim, path, tol):
    g = np.load(path, allow_pickle=False)
    assert [sim.num_blocks(l) for l in range(sim.levels)] == list(g["blocks_per_level"])
    got = np.empty_like(g["values"])
    for l in range(sim.levels):
        sel = g["level"] == l
        if not sel.any():
            continue
        keys, vals = sim.get_moments(l)
        keys = keys.cpu().numpy()
        vals = vals.cpu().numpy()
        idx = np.searchsorted(keys, g["key"][sel])
        assert np.array_equal(keys[idx], g["key"][sel])
        got[sel] = vals[idx, :, g["node"][sel]]
    ref = g["values"]
    errs = {}
    for name, sl in {"rho-1": slice(0, 1), "u": slice(1, 4), "S": slice(4, 10)}.items():
        errs[name] = float(np.linalg.norm(got[:, sl] - ref[:, sl]) / np.linalg.norm(ref[:, sl]))
    print(f"{os.path.basename(path)} rel L2 over {len(ref)} sampled nodes: {errs}", flush=True)
    for k, v in errs.items():
        assert v <= (tol[k] if isinstance(tol, dict) else tol), (k, v)


def _slab_sim(wl):
    lbm = _lbm()
    p = torch.as_tensor(W.slab_particles(wl["particles"], wl["seed"], wl["lo"], wl["hi"])).cuda()
    sim = lbm.Sim(wl["levels"], wl["n"], wl["bc"], wl["tau0"], particles=p, max_blocks=48000)
    for l in range(3):
        keys = sim.block_keys(l).cpu().numpy()
        for s in range(0, len(keys), 4096):
            k = keys[s:s + 4096]
            sim.set_block_moments(l, k, W.tgv3d_field(l, k, wl["n"], wl["amp"]).astype(np.float32))
    sub = 1 << (wl["levels"] - 1)
    d = tuple(v * sub for v in wl["v_fine"])
    return sim, p, d


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "sphere128_oracle_sample.npz")),
                    reason="stored oracle sample not generated")
def test_sphere128_full_run_against_oracle_sample():
    lbm = _lbm()
    wl = W.workload("sphere128")
    c, r = wl["sphere"]
    print("sphere128: 500 coarse steps", flush=True)
    sim = lbm.Sim(2, wl["n"], wl["bc"], wl["tau0"], uin=wl["uin"], solid=W.sphere_solid(wl["n"], c, r))
    for l in range(2):
        keys = sim.block_keys(l).cpu().numpy()
        sim.set_block_moments(l, keys, W.uniform_field(l, keys).astype(np.float32))
    sim.step(wl["steps"])
    torch.cuda.synchronize()
    assert sim.check_finite()
    _compare_sample(sim, os.path.join(GOLDEN, "sphere128_oracle_sample.npz"), 1e-5)


SCALES = [64.0, 8.0, 8.0, 8.0, 64.0, 64.0, 64.0, 64.0, 64.0, 64.0]


def _sphere_run(storage):
    lbm = _lbm()
    wl = W.workload("sphere128")
    c, r = wl["sphere"]
    sim = lbm.Sim(2, wl["n"], wl["bc"], wl["tau0"], uin=wl["uin"], solid=W.sphere_solid(wl["n"], c, r),
                  storage=storage, scale=None if storage == "f32" else SCALES)
    for l in range(2):
        keys = sim.block_keys(l).cpu().numpy()
        sim.set_block_moments(l, keys, W.uniform_field(l, keys).astype(np.float32))
    sim.step(wl["steps"])
    torch.cuda.synchronize()
    assert sim.check_finite()
    return sim


HALF_BOUNDS = {  # relative L2 per group after 500 coarse steps (measured 2.1/4.2/9.0% and 0.13/0.29/0.85%)
    "bf16": {"rho-1": 0.03, "u": 0.06, "S": 0.12},
    "f16": {"rho-1": 0.002, "u": 0.004, "S": 0.012},
}


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "sphere128_oracle_sample.npz")),
                    reason="stored oracle sample not generated")
@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_sphere128_half_precision_full_run(storage):
    tol_oracle = tol_f32 = HALF_BOUNDS[storage]
    # the sphere case's 500 coarse steps with 16-bit moment storage (FP32 arithmetic):
    # error against the stored FP64 oracle sample and against the FP32-storage run
    print(f"sphere128 {storage}: 500 coarse steps", flush=True)
    half = _sphere_run(storage)
    _compare_sample(half, os.path.join(GOLDEN, "sphere128_oracle_sample.npz"), tol_oracle)
    ref = _sphere_run("f32")
    from tests.util import group_errors
    A, B = [], []
    for l in range(2):
        A.append(half.get_moments(l)[1].cpu().numpy().astype(np.float64))
        B.append(ref.get_moments(l)[1].cpu().numpy().astype(np.float64))
    own = np.concatenate([(half.roles(l).cpu().numpy() != 1) for l in range(2)])
    errs = group_errors(np.concatenate(A), np.concatenate(B), mask=own)
    print(f"sphere128 {storage} vs the FP32-storage run, rel L2 over owned nodes: {errs}", flush=True)
    for k, v in errs.items():
        assert v <= tol_f32[k], (k, v)


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "slab512_oracle_sample.npz")),
                    reason="stored oracle sample not generated")
def test_slab512_full_size_against_oracle_sample():
    wl = W.workload("slab512")
    g = np.load(os.path.join(GOLDEN, "slab512_oracle_sample.npz"), allow_pickle=False)
    steps = int(g["steps"])
    print(f"slab512: {steps} coarse steps with grid updates", flush=True)
    sim, p, d = _slab_sim(wl)
    for _ in range(steps):
        sim.step(1)
        sim.advance_particles(p, d)
        sim.remesh(p)
    torch.cuda.synchronize()
    _compare_sample(sim, os.path.join(GOLDEN, "slab512_oracle_sample.npz"), 1e-5)


def test_slab512_full_run_hierarchy_and_invariants():
    wl = W.workload("slab512")
    print("slab512: 200 coarse steps", flush=True)
    sim, p, d = _slab_sim(wl)
    host = W.slab_particles(wl["particles"], wl["seed"], wl["lo"], wl["hi"])
    dd = np.array(d, dtype=np.float32)
    ke0 = sim.reduce(2, (0, 0, 0), (512, 512, 256))[4]
    changes = 0
    prev = None
    for step in range(wl["steps"]):
        sim.step(1)
        sim.advance_particles(p, d)
        sim.remesh(p)
        host = host + dd  # float32 add, the same rounding as the device
        counts = tuple(sim.num_blocks(l) for l in range(3))
        if counts != prev:
            changes += 1
            prev = counts
            assert np.array_equal(p.cpu().numpy(), host)
            t0 = {tuple(b) for b in np.unique(np.floor(host * np.float32(0.125)).astype(np.int64) % 64, axis=0)}
            active, _ = canonical_sets(3, (64, 64, 64), (True, True, True), t0)
            for l in range(3):
                bx, by, bz = W.morton_decode(sim.block_keys(l).cpu().numpy())
                assert set(zip(bx.tolist(), by.tolist(), bz.tolist())) == active[l], (step, l)
            print(f"step {step + 1}: hierarchy {counts} matches the canonical sets", flush=True)
    torch.cuda.synchronize()
    assert changes >= 2
    assert sim.check_finite()
    # viscous decay of the vortex in the bottom half, which stays on the coarsest
    # level: linear Taylor-Green decay exp(-6 nu k^2 t) with nu = (tau0 - 1/2)/3 in
    # fine units over 4 fine steps per coarse step (0.976), nonlinear transfer and
    # the start from S = u u allowed for by the band
    ke1 = sim.reduce(2, (0, 0, 0), (512, 512, 256))[4]
    ratio = ke1 / ke0
    print(f"kinetic energy ratio (z < 256) after {wl['steps']} coarse steps: {ratio:.5f}", flush=True)
    assert 0.95 < ratio < 0.995, ratio
