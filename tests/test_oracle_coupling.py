"""Pins of the oracle's finest-level coupling fields (Sec. 4: the relaxation time
scaled by the fluid fraction, tau -> eps tau; the external force density F through
the half-force velocity of Eq. rho_u_stress and the Guo source in the second
moments):

- eps = 1, F = 0 everywhere gives the uncoupled run bit for bit (two levels, grid
  updates included);
- a uniform F field gives the uniform body force (the Poiseuille-pinned path);
- a uniform eps gives the run with tau0 replaced by eps tau0;
- with smooth random eps and F fields on a periodic level the total momentum grows
  by exactly sum(F) per step (Guo forcing adds F to the momentum of every node).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W

P = O.PERIODIC


def _state(sim, level=0):
    _, v = sim.get_block_moments(level)
    return v


def _init(sim, n, seed=7):
    u0 = W.smooth_random_velocity(n, seed, kmax=3.0, rms=0.03)
    for l in range(sim.levels):
        k = sim.block_keys(l)
        sim.set_block_moments(l, k, W.velocity_moments(l, k, u0))


def _fields(keys, seed, eps=None, force=None):
    rng = np.random.default_rng(seed)
    f = np.zeros((len(keys), 4, 512))
    pos = W.node_positions(0, keys).astype(np.float64)
    f[:, 0] = 1.0 if eps is None else eps
    if eps is None:
        f[:, 0] = 0.85 + 0.1 * np.sin(2 * np.pi * pos[..., 0] / 32 + rng.uniform(0, 6))
    if force is None:
        for a in range(3):
            f[:, 1 + a] = 2e-5 * np.cos(2 * np.pi * pos[..., (a + 1) % 3] / 32 + rng.uniform(0, 6)) + 1e-5 * (a - 1)
    else:
        f[:, 1:4] = np.asarray(force)[None, :, None]
    return f


def test_unit_fields_give_the_uncoupled_run_exactly():
    n = (64, 64, 64)
    p = W.slab_particles(300, 4, (20.0, 20.0, 30.0), (44.0, 44.0, 40.0))
    a = O.OracleSim(2, n, (P,) * 6, 0.6, particles=p)
    b = O.OracleSim(2, n, (P,) * 6, 0.6, particles=p)
    _init(a, n)
    _init(b, n)
    k0 = b.block_keys(0)
    b.set_coupling(k0, _fields(k0, 1, eps=1.0, force=(0.0, 0.0, 0.0)))
    d = np.array([0.0, 0.0, -2.0], dtype=np.float32)
    for _ in range(3):
        a.step(1)
        b.step(1)
        O.advance_particles(p, d)
        a.remesh(p)
        b.remesh(p)
    for l in range(2):
        assert np.array_equal(_state(a, l), _state(b, l))


def test_uniform_force_field_equals_body_force():
    n = (32, 32, 32)
    F = (3e-5, -1e-5, 2e-5)
    a = O.OracleSim(1, n, (P, P, P, P, O.WALL, O.WALL), 0.7, force=F)
    b = O.OracleSim(1, n, (P, P, P, P, O.WALL, O.WALL), 0.7)
    _init(a, n)
    _init(b, n)
    k = b.block_keys(0)
    b.set_coupling(k, _fields(k, 2, eps=1.0, force=F))
    a.step(4)
    b.step(4)
    assert np.array_equal(_state(a), _state(b))


def test_uniform_fluid_fraction_scales_tau():
    n = (32, 32, 32)
    eps, tau0 = 0.8, 0.75
    a = O.OracleSim(1, n, (P,) * 6, eps * tau0)
    b = O.OracleSim(1, n, (P,) * 6, tau0)
    _init(a, n)
    _init(b, n)
    k = b.block_keys(0)
    b.set_coupling(k, _fields(k, 3, eps=eps, force=(0.0, 0.0, 0.0)))
    a.step(4)
    b.step(4)
    assert np.abs(_state(a) - _state(b)).max() < 1e-15


def test_momentum_grows_by_the_total_force():
    n = (32, 32, 32)
    sim = O.OracleSim(1, n, (P,) * 6, 0.8)  # eps in [0.75, 0.95]: eps tau0 >= 0.6
    _init(sim, n)
    k = sim.block_keys(0)
    f = _fields(k, 4)
    sim.set_coupling(k, f)
    total = f[:, 1:4].sum(axis=(0, 2))
    assert np.abs(total).max() > 0.1

    def momentum():
        v = _state(sim)
        return ((1.0 + v[:, 0:1]) * v[:, 1:4]).sum(axis=(0, 2))

    m0 = momentum()
    for s in range(3):
        sim.step(1)
        m1 = momentum()
        assert np.abs((m1 - m0) - total).max() < 1e-13 * max(1.0, np.abs(m1).max()), (s, m1 - m0, total)
        m0 = m1


def test_invalid_fluid_fraction_rejected():
    sim = O.OracleSim(1, (16, 16, 16), (P,) * 6, 0.6)
    k = sim.block_keys(0)
    f = _fields(k, 5, eps=0.8, force=(0.0, 0.0, 0.0))  # eps tau0 = 0.48 < 1/2
    with pytest.raises(ValueError):
        sim.set_coupling(k, f)
