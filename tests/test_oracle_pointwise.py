"""Pins of the oracle's single-node arithmetic (lattice, reconstruction, collision)
against closed forms of Sec. 3.1 and textbook Hermite identities."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O

CS2 = 1.0 / 3.0


def test_lattice_identities():
    # D3Q27 (reading of Sec. 3.1: the xyz third-order component needs corner velocities)
    c, w = O.lattice()
    assert c.shape == (27, 3)
    assert {tuple(v) for v in c} == set(itertools.product((-1, 0, 1), repeat=3))
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * np.eye(3), atol=1e-16)
    d = np.eye(3)
    iso4 = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-16)
    assert abs(w[13] - 8.0 / 27.0) < 1e-16  # rest particle


def _random_q(rng, amp=0.05):
    q = np.empty(10)
    q[0] = 1.0 + 0.02 * rng.standard_normal()
    q[1:4] = amp * rng.standard_normal(3)
    q[4:10] = 0.01 * rng.standard_normal(6)
    return q


def _S(q):
    S = np.empty((3, 3))
    for (a, b), k in {(0, 0): 4, (1, 1): 5, (2, 2): 6, (0, 1): 7, (0, 2): 8, (1, 2): 9}.items():
        S[a, b] = S[b, a] = q[k]
    return S


def test_reconstruction_reproduces_stored_moments():
    # Eq. rho_u_stress applied to Eq. three_order_f returns (rho, u, S) exactly
    rng = np.random.default_rng(1)
    c, w = O.lattice()
    for _ in range(20):
        q = _random_q(rng)
        f = O.reconstruct(q)
        rho = f.sum()
        u = (c * f[:, None]).sum(0) / rho
        S = np.einsum("ia,ib,i->ab", c, c, f) / rho - CS2 * np.eye(3)
        assert abs(rho - q[0]) < 1e-14
        assert np.allclose(u, q[1:4], atol=1e-15)
        assert np.allclose(S, _S(q), atol=1e-15)


def test_third_order_projection_equals_rho_gamma():
    # sum_i H3_abc(c_i) f_i = rho Gamma_abc for every D3Q27-supported component
    # (fails by a factor 1/2 on xyz if 1/(2cs^6) were used for xyz as printed)
    rng = np.random.default_rng(2)
    c, w = O.lattice()
    d = np.eye(3)
    H3 = (np.einsum("ia,ib,ic->iabc", c, c, c)
          - CS2 * (np.einsum("ia,bc->iabc", c, d) + np.einsum("ib,ac->iabc", c, d) + np.einsum("ic,ab->iabc", c, d)))
    for _ in range(10):
        q = _random_q(rng)
        S = _S(q)
        u = q[1:4]
        gam = (np.einsum("ab,c->abc", S, u) + np.einsum("ac,b->abc", S, u) + np.einsum("bc,a->abc", S, u)
               - 2 * np.einsum("a,b,c->abc", u, u, u))
        f = O.reconstruct(q)
        proj = np.einsum("iabc,i->abc", H3, f)
        for (a, b, cc) in [(0, 0, 1), (0, 1, 1), (0, 0, 2), (0, 2, 2), (1, 2, 2), (1, 1, 2), (0, 1, 2)]:
            assert abs(proj[a, b, cc] - q[0] * gam[a, b, cc]) < 1e-15, (a, b, cc)


def test_collision_at_tau_one_gives_third_order_equilibrium():
    # omega = 1: S -> u u, so f is the textbook third-order Hermite equilibrium
    # f_eq = w rho [1 + c.u/cs2 + (c.u)^2/(2cs4) - u^2/(2cs2) + H3:uuu/(6cs6)]
    rng = np.random.default_rng(3)
    c, w = O.lattice()
    d = np.eye(3)
    H3 = (np.einsum("ia,ib,ic->iabc", c, c, c)
          - CS2 * (np.einsum("ia,bc->iabc", c, d) + np.einsum("ib,ac->iabc", c, d) + np.einsum("ic,ab->iabc", c, d)))
    for _ in range(10):
        q = _random_q(rng)
        u = q[1:4]
        p = O.collide(q, 1.0)
        f = O.reconstruct(p)
        cu = c @ u
        feq = w * q[0] * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - u @ u / (2 * CS2)
                          + np.einsum("iabc,a,b,c->i", H3, u, u, u) / (6 * CS2 ** 3))
        assert np.allclose(f, feq, atol=1e-16, rtol=1e-14)


def test_collision_relaxes_only_second_moments():
    rng = np.random.default_rng(4)
    for omega in (0.5, 1.0, 1.7):
        q = _random_q(rng)
        p = O.collide(q, omega)
        assert np.array_equal(p[:4], q[:4])
        uu = np.outer(q[1:4], q[1:4])
        S = _S(q)
        assert np.allclose(_S(p), S + omega * (uu - S), atol=1e-17)


def test_forced_collision_moments():
    # Guo forcing in moment form: carried first moment u + F/(2 rho); S gains (1-omega/2)(uF+Fu)/rho
    q = np.array([1.01, 0.02, -0.01, 0.03, 0.001, 0.002, 0.0005, 0.0001, -0.0002, 0.0003])
    F = np.array([1e-4, -2e-4, 3e-4])
    om = 1.4
    p = O.collide(q, om, F)
    assert np.allclose(p[1:4], q[1:4] + F / (2 * q[0]), atol=1e-18)
    u = q[1:4]
    expect = _S(q) + om * (np.outer(u, u) - _S(q)) + (1 - om / 2) * (np.outer(u, F) + np.outer(F, u)) / q[0]
    assert np.allclose(_S(p), expect, atol=1e-18)


def test_storage_rounding_matches_ieee_half_and_bfloat16():
    # the oracle's 16-bit storage emulation against numpy's float16 and torch's
    # bfloat16 conversions (both round to nearest even), after the f32 rounding
    import torch
    rng = np.random.default_rng(7)
    vals = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-9, 2, 2000),
                           [0.0, 1e-8, -3e-6, 2.0 ** -24, 2.0 ** -15, 0.5, 65000.0]])
    for scale in (1.0, 64.0, 8.0):
        for v in vals:
            f = np.float32(v * scale)
            e16 = float(np.float16(f)) / scale
            eb = float(torch.tensor(float(f), dtype=torch.float32).to(torch.bfloat16).float()) / scale
            assert O.store_round(v, "f16", scale) == e16, (v, scale)
            assert O.store_round(v, "bf16", scale) == eb, (v, scale)
