"""Multi-level pins of the oracle: canonical hierarchy against a set-based brute
force, uniform-state invariance through transfers and grid updates, exactness of
the downward interpolation on linear fields, translation equivariance, and the
cross-interface shear wave that decides the S^neq rescaling factors."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W
from tests.util import canonical_sets, blocks_to_dense, level_index

P = O.PERIODIC


def _keys_to_set(keys):
    bx, by, bz = W.morton_decode(keys)
    return set(zip(bx.tolist(), by.tolist(), bz.tolist()))


def _t0_from_particles(p, n, periodic):
    t0 = set()
    for q in p:
        b = []
        ok = True
        for a in range(3):
            v = np.floor(np.float32(q[a]) * np.float32(0.125))
            nb = n[a] // 8
            if not periodic[a] and not (0 <= q[a] < n[a]):
                ok = False
            b.append(int(v) % nb if periodic[a] else int(v))
        if ok:
            t0.add(tuple(b))
    return t0


def _brute_roles(levels, n, bc, active, deleted, level, keys):
    """Role of every node of the listed blocks from the block sets (no solid)."""
    nl = [v >> level for v in n]
    nb = [v // 8 for v in nl]
    per = [bc[2 * a] == P for a in range(3)]
    g = level_index(level, keys)
    roles = np.zeros(g.shape[:2], dtype=np.uint8)
    act, dele = active[level], deleted[level]
    for bi in range(g.shape[0]):
        for ni in range(512):
            x = g[bi, ni]
            face = None
            for a in range(3):
                if per[a]:
                    continue
                if x[a] == 0 and bc[2 * a] in (O.INFLOW, O.OUTFLOW):
                    face = bc[2 * a]
                    break
                if x[a] == nl[a] - 1 and bc[2 * a + 1] in (O.INFLOW, O.OUTFLOW):
                    face = bc[2 * a + 1]
                    break
            if face is not None:
                roles[bi, ni] = O.R_INFLOW if face == O.INFLOW else O.R_OUTFLOW
                continue
            ghost = iu = False
            for d in np.ndindex(3, 3, 3):
                if d == (1, 1, 1):
                    continue
                h = [x[a] + d[a] - 1 for a in range(3)]
                out = False
                for a in range(3):
                    if not (0 <= h[a] < nl[a]):
                        if per[a]:
                            h[a] %= nl[a]
                        else:
                            out = True
                if out:
                    continue
                hb = tuple(h[a] // 8 for a in range(3))
                if hb in dele:
                    iu = True
                elif hb not in act:
                    ghost = True
            roles[bi, ni] = O.R_GHOST if ghost else (O.R_IU if iu else O.R_INTERIOR)
    return roles


@pytest.mark.parametrize("levels,n,bc,seed,count,box", [
    (2, (64, 64, 64), (P,) * 6, 1, 40, ((10, 10, 10), (30, 50, 20))),
    (3, (64, 64, 64), (P,) * 6, 2, 25, ((0, 0, 0), (20, 20, 64))),
    (3, (128, 64, 64), (O.INFLOW, O.OUTFLOW, P, P, O.WALL, O.WALL), 3, 30, ((40, 10, 0), (80, 40, 20))),
    (2, (32, 32, 32), (O.WALL,) * 6, 4, 10, ((0, 0, 0), (32, 32, 32))),
])
def test_hierarchy_matches_set_brute_force(levels, n, bc, seed, count, box):
    p = W.slab_particles(count, seed, box[0], box[1])
    sim = O.OracleSim(levels, n, bc, 0.6, particles=p)
    per = [bc[2 * a] == P for a in range(3)]
    t0 = _t0_from_particles(p, n, per)
    active, deleted = canonical_sets(levels, [v // 8 for v in n], per, t0)
    for l in range(levels):
        keys = sim.block_keys(l)
        assert np.all(np.diff(keys) > 0)  # Morton-sorted
        assert _keys_to_set(keys) == active[l], l
    # every particle sits in an active level-0 block; nesting of regions
    assert t0 <= active[0]
    for l in range(1, levels):
        for b in deleted[l]:
            for c in np.ndindex(2, 2, 2):
                ch = tuple(2 * b[a] + c[a] for a in range(3))
                assert ch in active[l - 1] or ch in deleted[l - 1]
    # roles of the finest and a coarse level against a node-level brute force
    for l in sorted({0, levels - 1}):
        keys = sim.block_keys(l)
        sel = np.linspace(0, len(keys) - 1, min(len(keys), 24)).astype(int)
        got = sim.roles(l)[sel]
        exp = _brute_roles(levels, n, bc, active, deleted, l, keys[sel])
        assert np.array_equal(got, exp), l


def test_ghost_and_upward_shells_are_separated():
    # downward targets (ghosts of level l) and upward sources (nodes 2q of I^u_{l+1})
    # are at least 14 fine nodes apart, so the transfers never read each other's output
    from scipy.spatial import cKDTree
    n = 256
    p = W.slab_particles(50, 7, (80, 80, 80), (150, 130, 110))
    sim = O.OracleSim(3, (n, n, n), (P,) * 6, 0.6, particles=p)
    for l in range(2):
        kf, kc = sim.block_keys(l), sim.block_keys(l + 1)
        gpos = W.node_positions(l, kf)[sim.roles(l) == O.R_GHOST]
        upos = W.node_positions(l + 1, kc)[sim.roles(l + 1) == O.R_IU]
        assert len(gpos) and len(upos), l
        d, _ = cKDTree(upos, boxsize=n).query(gpos, p=np.inf)
        assert d.min() >= 14, (l, d.min())


def _uniform_all(sim, u):
    for l in range(sim.levels):
        keys = sim.block_keys(l)
        sim.set_block_moments(l, keys, W.uniform_field(l, keys, 1.0, u))


def test_uniform_state_invariant_through_transfers_and_grid_updates():
    u = (0.05, 0.02, -0.01)
    p = W.slab_particles(60, 8, (20, 20, 20), (50, 40, 30))
    sim = O.OracleSim(3, (64, 64, 64), (P,) * 6, 0.6, particles=p)
    _uniform_all(sim, u)
    exp = W.uniform_field(0, np.zeros(1, dtype=np.int64), 1.0, u)[0]
    d = np.array([0.0, 0.0, -1.5], dtype=np.float32)
    for it in range(4):
        sim.step(1)
        O.advance_particles(p, d * 4)
        sim.remesh(p)
        for l in range(3):
            _, v = sim.get_block_moments(l)
            r = sim.roles(l)
            own = (r != O.R_GHOST)
            if not own.any():
                continue
            err = np.abs(v.transpose(0, 2, 1)[own] - exp.T[0][None, :]).max()
            assert err < 1e-14, (it, l, err)


def test_downward_interpolation_exact_on_linear_fields():
    # new fine blocks are sampled from the coarse level: rho and u linear fields are
    # reproduced exactly and S^neq is the linear field times the downward factor
    n = (128, 128, 128)
    sim = O.OracleSim(2, n, (O.WALL,) * 6, 0.6)
    keys = sim.block_keys(1)
    x = W.node_positions(1, keys).astype(np.float64)
    a = np.array([1e-4, -2e-4, 3e-4])

    def lin(pos):
        r = pos @ a
        u = [0.01 + pos @ (a * (k + 1)) for k in range(3)]
        sneq = [pos @ (a * (k - 2)) for k in range(6)]
        S = [u[0] * u[0], u[1] * u[1], u[2] * u[2], u[0] * u[1], u[0] * u[2], u[1] * u[2]]
        return r, u, sneq, S

    r, u, sneq, S = lin(x)
    sim.set_block_moments(1, keys, W.moments_from_fields(r, u, [S[k] + sneq[k] for k in range(6)]))
    tau, a_up, a_down = sim.level_params()
    sim.remesh(W.slab_particles(20, 9, (56, 56, 56), (72, 72, 72)))
    k0, v0 = sim.get_block_moments(0)
    assert len(k0) > 0
    r, u, sneq, S = lin(W.node_positions(0, k0).astype(np.float64))
    assert np.abs(v0[:, 0] - r).max() < 1e-15
    for k in range(3):
        assert np.abs(v0[:, 1 + k] - u[k]).max() < 1e-15
    for k in range(6):
        assert np.abs(v0[:, 4 + k] - (S[k] + a_down[0] * sneq[k])).max() < 1e-15
    # and the coarse nodes that stay active are untouched
    k1, v1 = sim.get_block_moments(1)
    r, u, sneq, S = lin(W.node_positions(1, k1).astype(np.float64))
    assert np.abs(v1[:, 0] - r).max() < 1e-15


def test_level_parameters():
    sim = O.OracleSim(3, (64, 64, 64), (P,) * 6, 0.6)
    tau, a_up, a_down = sim.level_params()
    assert np.allclose(tau, [0.6, 0.55, 0.525], atol=1e-15)  # tau_{l+1} = tau_l/2 + 1/4
    nu = (tau - 0.5) / 3
    assert np.allclose(nu[1:] * 2, nu[:-1])                   # nu_{l+1} = nu_l / 2
    assert np.allclose(a_up[:2] * a_down[:2], 1.0)            # mutually inverse
    assert abs(a_up[0] - 2 * 0.55 / 0.6) < 1e-15
    sim2 = O.OracleSim(3, (64, 64, 64), (P,) * 6, 0.6, rescale="printed")
    _, pu, pd = sim2.level_params()
    assert abs(pu[0] - 0.55 / 1.2) < 1e-15 and abs(pd[0] - 1.1 / 0.6) < 1e-15


def _smooth_level_field(level, keys, n, amp):
    p = W.node_positions(level, keys).astype(np.float64)
    k = 2 * np.pi / np.array(n, dtype=np.float64)
    x, y, z = p[..., 0] * k[0], p[..., 1] * k[1], p[..., 2] * k[2]
    ux = amp * np.sin(y + 0.3) * np.cos(z)
    uy = amp * np.sin(z + 1.1) * np.cos(x)
    uz = amp * np.sin(x - 0.7) * np.cos(y)
    return W.moments_from_fields(0.001 * np.cos(x + y), [ux, uy, uz])


def test_translation_equivariance_multilevel():
    # shifting the field and the particles by one coarsest block shifts the result
    n = (64, 64, 64)
    p = W.slab_particles(30, 10, (12, 20, 16), (30, 36, 30))
    shift = np.array([32, 0, 32])
    outs = []
    for s in (np.zeros(3, int), shift):
        ps = (p + s.astype(np.float32)) % np.float32(64)
        sim = O.OracleSim(3, n, (P,) * 6, 0.6, particles=ps)
        for l in range(3):
            keys = sim.block_keys(l)
            nl = [v >> l for v in n]
            # field defined on the unshifted frame
            pos = (W.node_positions(l, keys) - s[None, None, :]) % 64
            kk = W.morton_encode(pos[:, 0, 0] // (8 << l), pos[:, 0, 1] // (8 << l), pos[:, 0, 2] // (8 << l))
            sim.set_block_moments(l, keys, _smooth_level_field(l, kk, n, 0.03))
        sim.step(2)
        sim.remesh(ps)
        sim.step(1)
        dense = []
        for l in range(3):
            k, v = sim.get_block_moments(l)
            r = sim.roles(l)
            v = np.where((r == O.R_GHOST)[:, None, :], np.nan, v)
            dense.append(blocks_to_dense(l, k, v, [x >> l for x in n]))
        outs.append(dense)
    for l in range(3):
        sl = shift >> l
        a = np.roll(outs[0][l], tuple(sl), axis=(1, 2, 3))
        b = outs[1][l]
        assert np.array_equal(np.isnan(a), np.isnan(b))
        m = ~np.isnan(a)
        if m.any():
            assert np.abs(a[m] - b[m]).max() < 1e-15, l


def _shear_run(levels, rescale, n, steps, amp, tau0):
    p = W.slab_particles(400, 11, (0, 0, 48), (n[0], n[1], 80)) if levels > 1 else None
    sim = O.OracleSim(levels, n, (P,) * 6, tau0, particles=p, rescale=rescale)
    tau, _, _ = sim.level_params()
    k = 2 * np.pi / n[2]
    for l in range(levels):
        keys = sim.block_keys(l)
        z = W.node_positions(l, keys)[..., 2].astype(np.float64)
        ux = amp * np.sin(k * z)
        zero = np.zeros_like(ux)
        # Chapman-Enskog pre-collision stress in level-l lattice units
        sxz = -tau[l] / 3.0 * amp * k * np.cos(k * z) * 2.0 ** l
        S = [ux * ux, zero, zero, zero, sxz, zero]
        sim.set_block_moments(l, keys, W.moments_from_fields(zero, [ux, zero, zero], S))
    sim.step(steps)
    prof = {}
    for l in range(levels):
        keys, v = sim.get_block_moments(l)
        r = sim.roles(l)
        z = W.node_positions(l, keys)[..., 2]
        own = (r == O.R_INTERIOR)
        prof[l] = (z[own], v[:, 1][own], v[:, 8][own] / (2.0 ** l * tau[l]))
    return prof


def test_shear_wave_across_interface_selects_rescaling():
    # Sec. 5.2 rescaling of S^neq, checked on a decaying shear wave crossing a
    # two-level interface. Reference: the same wave on the uniform fine grid.
    n, amp, tau0 = (16, 16, 128), 0.02, 0.6
    ref = _shear_run(1, "ce", n, 200, amp, tau0)
    zr, ur, sr = ref[0]
    order = np.argsort(zr)
    zr, ur, sr = zr[order], ur[order], sr[order]
    errs = {}
    for mode in ("ce", "printed"):
        prof = _shear_run(2, mode, n, 100, amp, tau0)
        eu = es = 0.0
        for l in (0, 1):
            z, u, s = prof[l]
            uref = np.interp(z, zr, ur)
            sref = np.interp(z, zr, sr)
            eu = max(eu, np.abs(u - uref).max() / amp)
            es = max(es, np.abs(s - sref).max() / np.abs(sr).max())
        errs[mode] = (eu, es)
    # Chapman-Enskog factors keep both velocity and viscous stress continuous
    assert errs["ce"][0] < 2e-3 and errs["ce"][1] < 2e-2, errs
    # the factors as printed leave a visible stress jump at the interface
    assert errs["printed"][1] > 5 * errs["ce"][1], errs
