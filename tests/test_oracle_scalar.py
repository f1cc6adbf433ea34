"""Pins of the oracle's powder-snow volume fraction (Sec. 7, powder snow: transport by
the fluid velocity, diffusion and a source; semi-Lagrangian RK3 advection and a
forward-Euler diffusion step) on the finest level.

- Uniform velocities that move the field by whole or half nodes per step give the
  shifted field exactly (trilinear weights 1 or 1/2, 1/4 ...), checked against numpy
  rolls of the periodic grid.
- Diffusion of a single spike: the closed values of one forward-Euler step of the
  7-point Laplacian; the source adds dt q.
- A solid-body rotation u = w x (x - c) of a linear field: the RK3 departure points
  are third-order accurate (error of order (w dt)^4 r), so the advected field equals
  the exactly rotated one to 1e-6 of its variation, while a first-order backtrace would
  miss by (w dt)^2 r.
"""
import numpy as np

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W

P, WALL = O.PERIODIC, O.WALL


def _grid(sim):
    keys = sim.block_keys(0)
    return keys, W.node_positions(0, keys)


def _set_velocity(sim, u_of_pos):
    keys, pos = _grid(sim)
    q = np.zeros((len(keys), 10, 512))
    u = u_of_pos(pos.astype(np.float64))
    q[:, 1:4] = u.transpose(0, 2, 1)
    sim.set_block_moments(0, keys, q)


def _dense(sim, vals, n):
    _, pos = _grid(sim)
    out = np.zeros(n)
    out[pos[..., 0], pos[..., 1], pos[..., 2]] = vals
    return out


def _random_phi(sim, seed):
    keys, pos = _grid(sim)
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 1.0, size=(len(keys), 512))
    sim.scalar_set(keys, phi)
    return phi


def test_uniform_velocity_shifts_exactly():
    n = (16, 16, 16)
    for U, expect in [((1.0, 0.0, 0.0), lambda f: np.roll(f, 1, axis=0)),
                      ((0.0, -1.0, 0.0), lambda f: np.roll(f, -1, axis=1)),
                      ((0.5, 0.25, 0.0), lambda f: 0.5 * 0.75 * f + 0.5 * 0.75 * np.roll(f, 1, 0)
                       + 0.5 * 0.25 * np.roll(f, 1, 1) + 0.5 * 0.25 * np.roll(np.roll(f, 1, 0), 1, 1))]:
        sim = O.OracleSim(1, n, (P,) * 6, 0.6)
        _set_velocity(sim, lambda p: np.broadcast_to(np.array(U), p.shape).copy())
        phi = _random_phi(sim, 1)
        before = _dense(sim, phi, n)
        sim.scalar_advance(1.0, 0.0)
        after = _dense(sim, sim.scalar_get(), n)
        assert np.abs(after - expect(before)).max() < 1e-14, U


def test_diffusion_of_a_spike_and_the_source():
    n = (16, 16, 16)
    sim = O.OracleSim(1, n, (P,) * 6, 0.6)
    keys, pos = _grid(sim)
    phi = np.zeros((len(keys), 512))
    spike = (pos[..., 0] == 5) & (pos[..., 1] == 6) & (pos[..., 2] == 7)
    phi[spike] = 1.0
    sim.scalar_set(keys, phi)
    q = np.full((len(keys), 512), 0.01)
    D, dt = 0.05, 2.0
    sim.scalar_advance(dt, D, q)
    got = _dense(sim, sim.scalar_get(), n)
    exp = np.full(n, dt * 0.01)
    exp[5, 6, 7] += 1.0 - 6 * D * dt
    for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        exp[5 + d[0], 6 + d[1], 7 + d[2]] += D * dt
    assert np.abs(got - exp).max() < 1e-15


def test_solid_body_rotation_third_order_backtrace():
    n = (48, 48, 48)
    c = np.array([23.5, 24.25, 24.0])
    w = np.array([0.004, -0.006, 0.01])  # rad per step
    sim = O.OracleSim(1, n, (WALL,) * 6, 0.6)
    _set_velocity(sim, lambda p: np.cross(w, p - c))
    keys, pos = _grid(sim)
    a = np.array([0.3, -0.2, 0.45])
    phi = (pos.astype(np.float64) - c) @ a + 2.0
    sim.scalar_set(keys, phi)
    dt = 1.5
    sim.scalar_advance(dt, 0.0)
    got = sim.scalar_get()
    # exact: phi(R(-w dt)(x - c) + c), R(th) the rotation by |th| about th
    th = -w * dt
    ang = np.linalg.norm(th)
    k = th / ang
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    R = np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K
    x = pos.astype(np.float64) - c
    exact = (x @ R.T) @ a + 2.0
    r = np.linalg.norm(x, axis=-1)
    inner = r < 16  # departure points stay well inside the walls
    err = np.abs(got - exact)[inner].max()
    first_order = np.abs(((x - dt * np.cross(w, x)) @ a + 2.0) - exact)[inner].max()
    print("RK3 error", err, "first-order backtrace error", first_order)
    assert err < 1e-6 * np.abs(a).sum() * 16
    assert first_order > 100 * err


def test_departure_points_stay_within_seven_nodes():
    """A uniform velocity of more than one node per step carries the departure point
    beyond the 7-node search range per axis: every sample point is held at 7 nodes, so
    the field moves by exactly 7 nodes (not u dt) along the axes where u dt exceeds 7,
    and by u dt where it does not."""
    n = (32, 32, 32)
    for U, dt, shift in [((1.5, 0.0, 0.0), 6.0, (7, 0, 0)),      # 9 nodes asked, 7 taken
                         ((-2.0, 0.5, 0.0), 5.0, (-7, 2.5, 0)),  # -10 -> -7; y within range
                         ((0.0, 0.0, 1.0), 7.0, (0, 0, 7))]:     # exactly at the limit
        sim = O.OracleSim(1, n, (P,) * 6, 0.6)
        _set_velocity(sim, lambda p: np.broadcast_to(np.array(U), p.shape).copy())
        phi = _random_phi(sim, 3)
        before = _dense(sim, phi, n)
        sim.scalar_advance(dt, 0.0)
        after = _dense(sim, sim.scalar_get(), n)
        exp = before
        for a, s in enumerate(shift):
            whole = int(np.floor(s))
            frac = s - whole
            exp = (1.0 - frac) * np.roll(exp, whole, axis=a) + frac * np.roll(exp, whole + 1, axis=a)
        assert np.abs(after - exp).max() < 1e-14, (U, dt)
