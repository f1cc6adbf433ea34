"""Single-level pins of the oracle: brute-force population LBM, exact
conservation, symmetry, Taylor-Green decay and Poiseuille flow (closed forms)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W
from tests import brute
from tests.util import blocks_to_dense, dense_to_blocks, rel_l2

P = O.PERIODIC


def _smooth_moments(n, seed, amp=0.04):
    """Smooth random stored-order moments on an n^3 periodic grid [10, X, Y, Z]."""
    rng = np.random.default_rng(seed)
    x = np.arange(n) * 2 * np.pi / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    q = np.zeros((10, n, n, n))
    for m in range(10):
        a = rng.standard_normal(6)
        q[m] = a[0] * np.sin(X + a[1]) * np.cos(Y + a[2]) + a[3] * np.sin(2 * Z + a[4]) * np.cos(X - a[5])
    q[0] *= 0.01
    q[1:4] *= amp
    q[4:10] *= 0.003
    uu = [q[1] * q[1], q[2] * q[2], q[3] * q[3], q[1] * q[2], q[1] * q[3], q[2] * q[3]]
    for k in range(6):
        q[4 + k] += uu[k]
    return q


def _oracle_from_dense(q, tau, bc=(P,) * 6, solid=None, force=(0.0, 0.0, 0.0)):
    n = q.shape[1:]
    sim = O.OracleSim(1, n, bc, tau, solid=solid, force=force)
    keys = sim.block_keys(0)
    sim.set_block_moments(0, keys, dense_to_blocks(0, keys, q))
    return sim


def _dense(sim):
    keys, v = sim.get_block_moments(0)
    return blocks_to_dense(0, keys, v, sim.n)


def test_matches_bruteforce_population_lbm_periodic():
    n, tau, steps = 16, 0.62, 10
    q0 = _smooth_moments(n, 11)
    sim = _oracle_from_dense(q0, tau)
    sim.step(steps)
    f = brute.from_moments(q0)
    for _ in range(steps):
        f = brute.step(f, 1.0 / tau)
    ref = brute.to_moments(f)
    got = _dense(sim)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_matches_bruteforce_population_lbm_bounce_back():
    n, tau, steps = 16, 0.7, 8
    q0 = _smooth_moments(n, 12)
    x = np.arange(n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    solid_xyz = ((X - 7.3) ** 2 + (Y - 8.1) ** 2 + (Z - 6.6) ** 2) <= 3.2 ** 2
    solid_zyx = np.ascontiguousarray(solid_xyz.transpose(2, 1, 0)).astype(np.uint8)
    sim = _oracle_from_dense(q0, tau, solid=solid_zyx)
    sim.step(steps)
    q0s = q0.copy()
    q0s[:, solid_xyz] = 0.0  # rest state (rho-1 = 0, u = 0, S = 0) on solid nodes
    f = brute.from_moments(q0s)
    for _ in range(steps):
        f = brute.step(f, 1.0 / tau, solid=solid_xyz)
    ref = brute.to_moments(f)
    got = _dense(sim)
    fluid = ~solid_xyz
    assert np.max(np.abs(got[:, fluid] - ref[:, fluid])) < 1e-13
    assert np.max(np.abs(got[:, solid_xyz])) == 0.0


def test_exact_mass_and_momentum_conservation_periodic():
    q0 = _smooth_moments(16, 13)
    sim = _oracle_from_dense(q0, 0.55)
    r0 = sim.reduce(0)
    sim.step(20)
    r1 = sim.reduce(0)
    assert abs(r1[0] - r0[0]) / r0[0] < 1e-13
    assert np.all(np.abs(r1[1:4] - r0[1:4]) < 1e-13 * r0[0])


def _rot_z(q):
    """Rotate a stored-order moment field [10, X, Y, Z] by +90 deg about z:
    new(x', y') = R old, with (x', y') = (-y, x) on the periodic grid."""
    out = np.empty_like(q)
    # position map: new[i, j] = old[j, -i]
    def pos(a):
        return np.rot90(a, k=1, axes=(0, 1))
    rho, ux, uy, uz = q[0], q[1], q[2], q[3]
    sxx, syy, szz, sxy, sxz, syz = q[4:10]
    out[0] = pos(rho)
    out[1] = pos(-uy)
    out[2] = pos(ux)
    out[3] = pos(uz)
    out[4] = pos(syy)
    out[5] = pos(sxx)
    out[6] = pos(szz)
    out[7] = pos(-sxy)
    out[8] = pos(-syz)
    out[9] = pos(sxz)
    return out


def test_rotation_equivariance():
    # the D3Q27 step commutes with a 90-degree rotation of the whole field
    q0 = _smooth_moments(16, 14)
    a = _oracle_from_dense(q0, 0.6)
    a.step(5)
    b = _oracle_from_dense(_rot_z(q0), 0.6)
    b.step(5)
    assert np.max(np.abs(_rot_z(_dense(a)) - _dense(b))) < 1e-15


def test_translation_equivariance():
    q0 = _smooth_moments(16, 15)
    a = _oracle_from_dense(q0, 0.6)
    a.step(4)
    sh = (8, 0, 8)
    b = _oracle_from_dense(np.roll(q0, sh, axis=(1, 2, 3)), 0.6)
    b.step(4)
    assert np.max(np.abs(np.roll(_dense(a), sh, axis=(1, 2, 3)) - _dense(b))) < 1e-16


def test_taylor_green_2d_decay_rate():
    # 2D TGV (exact incompressible NS solution) embedded in 3D:
    # amplitude decays as exp(-2 nu k^2 t), nu = (tau - 1/2)/3
    nx, tau, U, steps = 64, 0.6, 0.05, 50
    k = 2 * np.pi / nx
    nu = (tau - 0.5) / 3.0
    x = np.arange(nx)
    X, Y, Z = np.meshgrid(x, x, np.arange(8), indexing="ij")
    ux = U * np.sin(k * X) * np.cos(k * Y)
    uy = -U * np.cos(k * X) * np.sin(k * Y)
    q = np.zeros((10, nx, nx, 8))
    q[1], q[2] = ux, uy
    # S = u u - 2 cs^2 tau sym(grad u)  (Chapman-Enskog pre-collision state)
    dxux = U * k * np.cos(k * X) * np.cos(k * Y)
    dyuy = -dxux
    dyux = -U * k * np.sin(k * X) * np.sin(k * Y)
    dxuy = U * k * np.sin(k * X) * np.sin(k * Y)
    q[4] = ux * ux - 2 * tau / 3 * dxux
    q[5] = uy * uy - 2 * tau / 3 * dyuy
    q[7] = ux * uy - tau / 3 * (dyux + dxuy)
    sim = _oracle_from_dense(q, tau)
    basis = np.sin(k * X) * np.cos(k * Y)
    a0 = (ux * basis).sum() / (basis * basis).sum()
    sim.step(steps)
    got = _dense(sim)
    a1 = (got[1] * basis).sum() / (basis * basis).sum()
    nu_eff = -np.log(a1 / a0) / (2 * k * k * steps)
    assert abs(nu_eff / nu - 1.0) < 0.02, nu_eff / nu


def _poiseuille_error(H, tau, umax, steps):
    nu = (tau - 0.5) / 3.0
    g = 8 * nu * umax / H ** 2
    y = np.arange(H)
    # walls half a node outside the first and last fluid nodes
    exact = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    q = np.zeros((10, 8, H, 8))
    q[1] = exact[None, :, None]
    q[4] = q[1] ** 2
    sim = _oracle_from_dense(q, tau, bc=(P, P, O.WALL, O.WALL, P, P), force=(g, 0.0, 0.0))
    sim.step(steps)
    got = _dense(sim)
    prof = got[1].mean(axis=(0, 2))
    assert np.allclose(got[1], prof[None, :, None], atol=1e-14)
    assert np.allclose(got[2:4], 0.0, atol=1e-14)
    return rel_l2(prof, exact)


def test_poiseuille_profile_and_convergence():
    # body-driven channel with halfway bounce-back walls: parabolic steady state
    tau, umax = 0.8, 0.02
    nu = (tau - 0.5) / 3.0
    e8 = _poiseuille_error(8, tau, umax, int(3 * 8 ** 2 / nu))
    e16 = _poiseuille_error(16, tau, umax, int(3 * 16 ** 2 / nu))
    assert e16 < 2e-3
    assert e8 / e16 > 3.5, (e8, e16)  # second order: 4.0
