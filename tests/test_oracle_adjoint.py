"""Pins of the complex-step derivative of the oracle, the reference of every
gradient check: the complex instance runs the same templated FP64 code on
std::complex<double>, so its imaginary part along a direction must equal the
central finite difference of the real oracle, and its real part the real run.

Configurations (two coarse steps each):
- two levels, 80^3 periodic, level 0 over [16, 64)^3 fixed by marker particles
  (stream-collide on both levels, downward and upward transfers);
- the same block set from a solid sphere (r = 3 at the centre) with an inflow
  face at x- and an outflow face at x+ (bounce-back, inflow, outflow copy);
- the sphere with a logarithmic inflow profile along z, a convective outflow face
  and no-slip z faces (the outflow step and its velocity-dependent rate).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W

P, INF, OUT, CONV, WALL = W.PERIODIC, W.INFLOW, W.OUTFLOW, W.OUTFLOW_CONV, W.WALL
N = (80, 80, 80)
BOX = ((16, 16, 16), (64, 64, 64))


def _config(kind):
    if kind == "periodic":
        return dict(bc=(P,) * 6, particles=W.block_centre_markers((4, 5)), solid=None, uin=(0.0, 0.0, 0.0))
    solid = W.sphere_solid(N, (40.0, 40.0, 40.0), 3.0)
    if kind == "open":
        return dict(bc=(INF, CONV, P, P, WALL, WALL), particles=None, solid=solid, uin=(0.03, 0.0, 0.0),
                    log_inflow=(2, 0.08, 0.0))
    return dict(bc=(INF, OUT, P, P, P, P), particles=None, solid=solid, uin=(0.03, 0.0, 0.0))


def _fields(sim, seed):
    """Initial moments (smooth velocity with a density and stress perturbation) and a
    random direction over every moment of every node, per level."""
    u0 = W.smooth_random_velocity(N, seed, kmax=4.0, rms=0.03)
    rng = np.random.default_rng(seed + 1)
    x, v = [], []
    for l in range(2):
        keys = sim.block_keys(l)
        q = W.velocity_moments(l, keys, u0)
        q[:, 0] += 1e-3 * rng.standard_normal(q[:, 0].shape)
        q[:, 4:] += 1e-4 * rng.standard_normal(q[:, 4:].shape)
        x.append(q)
        v.append(rng.standard_normal(q.shape))
    return x, v


def _real_loss(kind, x, steps):
    c = _config(kind)
    sim = O.OracleSim(2, N, c["bc"], 0.6, uin=c["uin"], solid=c["solid"], particles=c["particles"],
                      log_inflow=c.get("log_inflow"))
    for l in range(2):
        sim.set_block_moments(l, sim.block_keys(l), x[l])
    sim.step(steps)
    return sim.kinetic_energy(0, *BOX) + sim.kinetic_energy(1, *BOX)


def _complex_loss(kind, x, v, h, steps):
    c = _config(kind)
    sim = O.OracleSimComplex(2, N, c["bc"], 0.6, uin=c["uin"], solid=c["solid"], particles=c["particles"],
                             log_inflow=c.get("log_inflow"))
    for l in range(2):
        sim.set_block_moments(l, sim.block_keys(l), x[l], h * v[l])
    sim.step(steps)
    return sim.kinetic_energy(0, *BOX) + sim.kinetic_energy(1, *BOX)


@pytest.mark.parametrize("kind", ["periodic", "sphere", "open"])
def test_complex_step_matches_central_difference(kind):
    c = _config(kind)
    probe = O.OracleSim(2, N, c["bc"], 0.6, uin=c["uin"], solid=c["solid"], particles=c["particles"],
                        log_inflow=c.get("log_inflow"))
    assert probe.num_blocks(0) == 216 and probe.num_blocks(1) == 124
    roles0 = probe.roles(0)
    assert (roles0 == O.R_GHOST).any()
    if kind != "periodic":
        assert (roles0 == O.R_SOLID).any()
        assert (probe.roles(1) == O.R_OUTFLOW).any() and (probe.roles(1) == O.R_INFLOW).any()
    x, v = _fields(probe, 11)
    steps = 2
    base = _real_loss(kind, x, steps)
    cs = _complex_loss(kind, x, v, 1e-30, steps)
    # the real part of the complex run is the real run
    assert abs(cs.real - base) <= 1e-13 * abs(base)
    d_cs = cs.imag / 1e-30
    # central differences: truncation O(eps^2), rounding O(1e-16 L / eps)
    fd = []
    for eps in (1e-5, 1e-6):
        xp = [a + eps * b for a, b in zip(x, v)]
        xm = [a - eps * b for a, b in zip(x, v)]
        fd.append((_real_loss(kind, xp, steps) - _real_loss(kind, xm, steps)) / (2 * eps))
    print(f"{kind}: loss {base:.6e}, complex step {d_cs:.10e}, central differences {fd}")
    assert abs(fd[0] - fd[1]) <= 1e-6 * abs(d_cs)
    assert abs(d_cs - fd[1]) <= 1e-6 * abs(d_cs)


def _remesh_loss(x, v, h, moves):
    """Loss after coarse steps with a grid update after each that moves the refined
    region (new fine blocks on one side, coarsened ones on the other), and a last
    coarse step; with h > 0 in the complex instance along direction v."""
    c = _config("periodic")
    p = c["particles"].copy()
    if h:
        sim = O.OracleSimComplex(2, N, c["bc"], 0.6, particles=p)
        for l in range(2):
            sim.set_block_moments(l, sim.block_keys(l), x[l], h * v[l])
    else:
        sim = O.OracleSim(2, N, c["bc"], 0.6, particles=p)
        for l in range(2):
            sim.set_block_moments(l, sim.block_keys(l), x[l])
    for d in moves:
        sim.step(1)
        O.advance_particles(p, np.array(d, dtype=np.float32))
        sim.remesh(p)
    sim.step(1)
    return sim.kinetic_energy(0, *BOX) + sim.kinetic_energy(1, *BOX)


def test_complex_step_through_grid_updates_matches_central_difference():
    # the refined region moves by two level-0 blocks along x, then by two along y and
    # back along z: every update creates and deletes blocks on both levels (72 and 1,
    # then 120 and 1 each way), so new nodes are sampled downward (refinement) and
    # upward (coarsening)
    c = _config("periodic")
    probe = O.OracleSim(2, N, c["bc"], 0.6, particles=c["particles"])
    x, v = _fields(probe, 13)
    moves = [(16.0, 0.0, 0.0), (0.0, 16.0, -16.0)]
    base = _remesh_loss(x, None, 0.0, moves)
    cs = _remesh_loss(x, v, 1e-30, moves)
    assert abs(cs.real - base) <= 1e-13 * abs(base)
    d_cs = cs.imag / 1e-30
    fd = []
    for eps in (1e-5, 1e-6):
        xp = [a + eps * b for a, b in zip(x, v)]
        xm = [a - eps * b for a, b in zip(x, v)]
        fd.append((_remesh_loss(xp, None, 0.0, moves) - _remesh_loss(xm, None, 0.0, moves)) / (2 * eps))
    print(f"through grid updates: loss {base:.6e}, complex step {d_cs:.10e}, central differences {fd}")
    assert abs(fd[0] - fd[1]) <= 1e-6 * abs(d_cs)
    assert abs(d_cs - fd[1]) <= 1e-6 * abs(d_cs)
