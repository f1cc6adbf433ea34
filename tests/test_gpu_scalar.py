"""The finest level's powder-snow volume fraction on the GPU against the FP64 oracle
(semi-Lagrangian RK3 advection through the LBM velocity, forward-Euler diffusion, a
source; phi on the owned nodes of the finest level), through the C ABI: a two-level slab with grid updates between the steps
(blocks that stay keep phi, new ones start at 0), and the sphere case (solid nodes,
inflow and outflow faces). Relative L2 of phi <= 1e-5 (FP32 against FP64, including
the small differences of the velocity fields the two sides advect with)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W
from tests.test_gpu_parity import compare

pytestmark = pytest.mark.gpu

P = W.PERIODIC


def _lbm():
    from paper_2603_14982_amd import lbm
    return lbm


def _phi(keys, seed):
    pos = W.node_positions(0, keys).astype(np.float64)
    rng = np.random.default_rng(seed)
    ph = [rng.uniform(0, 6) for _ in range(3)]
    return 0.5 + 0.4 * np.sin(2 * np.pi * pos[..., 0] / 24 + ph[0]) * np.cos(2 * np.pi * pos[..., 1] / 20 + ph[1]) \
        * np.sin(2 * np.pi * pos[..., 2] / 16 + ph[2])


def _compare_phi(gpu, ora, label):
    kg, pg = gpu.scalar_get()
    kg = kg.cpu().numpy()
    po = ora.scalar_get()
    assert np.array_equal(kg, ora.block_keys(0)), label
    pg = pg.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(pg - po) / np.linalg.norm(po)
    print(label, "phi rel L2", err, flush=True)
    assert err <= 1e-5, (label, err)


def test_scalar_on_a_moving_slab_against_oracle():
    lbm = _lbm()
    n = (128, 128, 128)
    p = W.slab_particles(4000, 3, (24.0, 24.0, 64.0), (104.0, 104.0, 80.0))
    u0 = W.smooth_random_velocity(n, 9, kmax=3.0, rms=0.04)
    ora = O.OracleSim(2, n, (P,) * 6, 0.6, particles=p)
    gpu = lbm.Sim(2, n, (P,) * 6, 0.6, particles=p, scalar=True)
    for l in range(2):
        keys = ora.block_keys(l)
        vals = W.velocity_moments(l, keys, u0)
        ora.set_block_moments(l, keys, vals)
        gpu.set_block_moments(l, keys, vals.astype(np.float32))
    k0 = ora.block_keys(0)
    phi = _phi(k0, 1)
    ora.scalar_set(k0, phi)
    gpu.scalar_set(k0, phi.astype(np.float32))
    pg = torch.as_tensor(p).cuda()
    po = p.copy()
    d = np.array([0.0, 2.0, -1.0], dtype=np.float32)
    rng = np.random.default_rng(4)
    for it in range(4):
        gpu.step(1)
        ora.step(1)
        q = 1e-3 * rng.uniform(0, 1, size=(ora.num_blocks(0), 512))
        ora.scalar_advance(2.0, 0.03, q)
        gpu.scalar_advance(2.0, 0.03, q.astype(np.float32))
        _compare_phi(gpu, ora, f"slab it={it}")
        gpu.advance_particles(pg, d)
        O.advance_particles(po, d)
        gpu.remesh(pg)
        ora.remesh(po)
    compare(gpu, ora, label="slab with scalar")


def test_scalar_around_a_sphere_against_oracle():
    lbm = _lbm()
    wl = W.workload("sphere128")
    c, r = wl["sphere"]
    solid = W.sphere_solid(wl["n"], c, r)
    ora = O.OracleSim(2, wl["n"], wl["bc"], wl["tau0"], uin=wl["uin"], solid=solid)
    gpu = lbm.Sim(2, wl["n"], wl["bc"], wl["tau0"], uin=wl["uin"], solid=solid, scalar=True)
    u0 = W.smooth_random_velocity(wl["n"], 12, kmax=3.0, rms=0.03)
    for l in range(2):
        keys = ora.block_keys(l)
        vals = W.velocity_moments(l, keys, u0)
        ora.set_block_moments(l, keys, vals)
        gpu.set_block_moments(l, keys, vals.astype(np.float32))
    k0 = ora.block_keys(0)
    phi = _phi(k0, 2)
    ora.scalar_set(k0, phi)
    gpu.scalar_set(k0, phi.astype(np.float32))
    for it in range(5):
        gpu.step(1)
        ora.step(1)
        ora.scalar_advance(2.0, 0.05)
        gpu.scalar_advance(2.0, 0.05)
    _, pg = gpu.scalar_get()
    assert np.all(pg.cpu().numpy()[np.isin(ora.roles(0), (O.R_SOLID, O.R_GHOST))] == 0.0)
    _compare_phi(gpu, ora, "sphere")


def test_scalar_departure_range_against_oracle():
    """Velocities above one node per step with dt up to 7: sample points of the backtrace
    that would leave the 7-node range are held at it, on both sides (two levels, so
    the range also meets ghost nodes and missing blocks)."""
    lbm = _lbm()
    n = (64, 64, 64)
    particles = W.slab_particles(40, 9, (20.0, 20.0, 20.0), (44.0, 44.0, 44.0))
    ora = O.OracleSim(2, n, (P,) * 6, 0.6, particles=particles)
    gpu = lbm.Sim(2, n, (P,) * 6, 0.6, particles=particles, scalar=True)
    u0 = W.smooth_random_velocity(n, 21, kmax=3.0, rms=1.2)
    for l in range(2):
        keys = ora.block_keys(l)
        vals = W.velocity_moments(l, keys, u0)
        ora.set_block_moments(l, keys, vals)
        gpu.set_block_moments(l, keys, vals.astype(np.float32))
    k0 = ora.block_keys(0)
    ua = np.abs(ora.get_block_moments(0)[1][:, 1:4])
    assert (ua * 6.5 > 7).any(), "the field must reach beyond the range"
    phi = _phi(k0, 5)
    for dt in (6.5, 7.0, 3.0):
        ora.scalar_set(k0, phi)
        gpu.scalar_set(k0, phi.astype(np.float32))
        ora.scalar_advance(dt, 0.02)
        gpu.scalar_advance(dt, 0.02)
        _compare_phi(gpu, ora, f"fast field dt={dt}")


def test_scalar_arguments_rejected():
    lbm = _lbm()
    sim = lbm.Sim(1, (32, 32, 32), (P,) * 6, 0.6, scalar=True)
    with pytest.raises(lbm.LBMError):
        sim.scalar_advance(2.0, 0.1)  # D dt > 1/6
    with pytest.raises(lbm.LBMError):
        sim.scalar_advance(0.0, 0.01)
    with pytest.raises(lbm.LBMError):
        sim.scalar_advance(7.5, 0.0)  # beyond the 7-node departure range
    bad = np.array([W.morton_encode(np.array([9]), np.array([0]), np.array([0]))[0]], dtype=np.int64)
    with pytest.raises(lbm.LBMError):
        sim.scalar_set(bad, np.zeros((1, 512), dtype=np.float32))
    plain = lbm.Sim(1, (32, 32, 32), (P,) * 6, 0.6)
    with pytest.raises(lbm.LBMError):
        plain.scalar_advance(1.0, 0.01)
