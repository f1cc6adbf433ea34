"""Pins of the oracle's open boundaries (Sec. 7): the convective outflow condition
and the logarithmic inflow profile.

- Against the population-form brute force of tests/brute.py on a 16 x 8 x 8 channel
  (inflow plane at x-, outflow plane at x+, y and z periodic), several steps from a
  random smooth state whose outward velocity changes sign over the outlet, for both
  outflow kinds.
- Special cases: flow that enters through a convective outlet leaves the outlet
  nodes unchanged (no transport into the domain); a uniform flow through inflow and
  convective outflow faces is a fixed point.
- The log profile at the heights where it has closed values (zero at and below h0,
  exactly u0 where 1 + beta (h - h0) = e), in fine units on every level, with
  S = u u at every inflow node.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W
from tests import brute as B

P, INF, ZG, CONV = O.PERIODIC, O.INFLOW, O.OUTFLOW, O.OUTFLOW_CONV
N = (16, 8, 8)


def _dense(sim, level=0):
    keys = sim.block_keys(level)
    _, v = sim.get_block_moments(level)
    g = W.node_positions(level, keys) >> level
    shape = tuple(n >> level for n in sim.n)
    out = np.zeros((10,) + shape)
    out[:, g[..., 0], g[..., 1], g[..., 2]] = v.transpose(1, 0, 2)
    return out


def _set_dense(sim, q):
    keys = sim.block_keys(0)
    g = W.node_positions(0, keys)
    sim.set_block_moments(0, keys, q[:, g[..., 0], g[..., 1], g[..., 2]].transpose(1, 0, 2).copy())


def _smooth_state(seed):
    rng = np.random.default_rng(seed)
    x, y, z = np.meshgrid(*[np.arange(n) for n in N], indexing="ij")
    q = np.zeros((10,) + N)
    q[0] = 2e-3 * np.sin(2 * np.pi * y / 8 + rng.uniform(0, 6)) * np.cos(2 * np.pi * z / 8)
    # outward velocity of both signs across the outlet plane
    q[1] = 0.03 * np.sin(2 * np.pi * (y + 0.3) / 8) + 0.01 * np.cos(2 * np.pi * x / 16)
    q[2] = 0.02 * np.cos(2 * np.pi * z / 8 + rng.uniform(0, 6))
    q[3] = 0.02 * np.sin(2 * np.pi * (x + y) / 16 + rng.uniform(0, 6))
    for k, (a, b) in enumerate(((1, 1), (2, 2), (3, 3), (1, 2), (1, 3), (2, 3))):
        q[4 + k] = q[a] * q[b] + 1e-4 * rng.standard_normal(N)
    return q


@pytest.mark.parametrize("outflow", ["zero_gradient", "convective"])
def test_channel_against_population_brute_force(outflow):
    tau = 0.6
    uin = (0.02, 0.0, 0.0)
    sim = O.OracleSim(1, N, (INF, ZG if outflow == "zero_gradient" else CONV, P, P, P, P), tau, uin=uin)
    roles = sim.roles(0)
    assert (roles == O.R_INFLOW).sum() == 64 and (roles == O.R_OUTFLOW).sum() == 64
    q = _smooth_state(3)
    _set_dense(sim, q)
    q0 = _dense(sim)  # inflow nodes now hold (1, uin, uin uin)
    assert np.allclose(q0[1, 0], 0.02) and np.allclose(q0[4, 0], 0.02 ** 2)
    assert (q0[1, -2] > 0).any() and (q0[1, -2] < 0).any()
    f = B.from_moments(q0)
    for _ in range(6):
        sim.step(1)
        f = B.step_channel(f, 1.0 / tau, outflow)
    got = _dense(sim)
    ref = B.to_moments(f)
    err = np.abs(got - ref).max()
    print(outflow, "max abs difference", err)
    assert err < 1e-13
    if outflow == "convective":
        # the condition differs from the copy where the flow leaves the domain
        zg = O.OracleSim(1, N, (INF, ZG, P, P, P, P), tau, uin=uin)
        _set_dense(zg, q)
        zg.step(6)
        assert np.abs(_dense(zg)[:, -1] - got[:, -1]).max() > 1e-6


def test_flow_entering_through_a_convective_outlet_leaves_it_unchanged():
    # u_x < 0 everywhere: u_n <= 0 on the x+ outlet, so its nodes keep their values
    q = _smooth_state(4)
    q[1] = -0.03 + 0.005 * np.sin(2 * np.pi * np.arange(8)[None, :, None] / 8)
    sim = O.OracleSim(1, N, (ZG, CONV, P, P, P, P), 0.6)
    _set_dense(sim, q)
    before = _dense(sim)[:, -1]
    sim.step(3)
    after = _dense(sim)
    assert np.array_equal(after[:, -1], before)
    assert np.abs(after[:, -2] - _dense(sim)[:, -2]).max() == 0.0
    assert np.abs(after[:, 1:-1] - q[:, 1:-1]).max() > 1e-6  # the interior did move


def test_uniform_flow_is_a_fixed_point():
    u = (0.04, 0.01, -0.02)
    sim = O.OracleSim(1, N, (INF, CONV, P, P, P, P), 0.6, uin=u)
    q = np.zeros((10,) + N)
    q[1:4] = np.array(u)[:, None, None, None]
    for k, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        q[4 + k] = u[a] * u[b]
    _set_dense(sim, q)
    sim.step(5)
    assert np.abs(_dense(sim) - q).max() < 1e-15


def test_log_inflow_profile_closed_values():
    # height along z; h0 = 4, and beta such that 1 + beta (12 - 4) = e: u(12) = u0
    h0, beta, u0 = 4.0, (math.e - 1.0) / 8.0, 0.05
    n = (32, 32, 32)
    p = W.slab_particles(200, 2, (2.0, 2.0, 2.0), (12.0, 12.0, 12.0))  # level 0 in one corner of the inflow face
    sim = O.OracleSim(2, n, (INF, ZG, P, P, P, P), 0.6, uin=(u0, 0.0, 0.0), particles=p,
                      log_inflow=(2, beta, h0))
    seen = set()
    for l in range(2):
        keys = sim.block_keys(l)
        _, v = sim.get_block_moments(l)
        pos = W.node_positions(l, keys)  # fine units
        inflow = sim.roles(l) == O.R_INFLOW
        assert inflow.any()
        h = pos[..., 2][inflow].astype(np.float64)
        ux = v[:, 1][inflow]
        assert np.all(ux[h <= h0] == 0.0)
        exact = np.isclose(h, 12.0)
        assert exact.any()
        assert np.allclose(ux[exact], u0, rtol=0, atol=1e-16)
        # monotone in height, positive above h0, equal at equal heights
        order = np.argsort(h, kind="stable")
        assert np.all(np.diff(ux[order]) >= 0) and np.all(ux[h > h0] > 0)
        assert np.allclose(v[:, 2][inflow], 0) and np.allclose(v[:, 3][inflow], 0)
        assert np.allclose(v[:, 4][inflow], ux * ux, rtol=0, atol=1e-18)
        assert np.all(v[:, 0][inflow] == 0.0)
        seen.add(l)
    assert seen == {0, 1}
