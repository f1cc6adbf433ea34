"""Test-side helpers: dense <-> block-keyed moment arrays, hierarchy brute force."""
import numpy as np

from paper_2603_14982_amd import workloads as W


def level_index(level, keys):
    """Level-l node coordinates of every node of the blocks: int64 [nb, 512, 3]."""
    return W.node_positions(level, keys) >> level


def dense_to_blocks(level, keys, dense):
    """dense [c, X, Y, Z] on the level-l node grid -> [nb, c, 512]"""
    g = level_index(level, keys)
    return dense[:, g[..., 0], g[..., 1], g[..., 2]].transpose(1, 0, 2).copy()


def blocks_to_dense(level, keys, vals, shape):
    """[nb, c, 512] -> dense [c, X, Y, Z] (unset nodes NaN)"""
    g = level_index(level, keys)
    out = np.full((vals.shape[1],) + tuple(shape), np.nan)
    out[:, g[..., 0], g[..., 1], g[..., 2]] = vals.transpose(1, 0, 2)
    return out


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


GROUPS = {"rho-1": slice(0, 1), "u": slice(1, 4), "S": slice(4, 10)}


def group_errors(a, b, mask=None):
    """Relative L2 per moment group over [nb, 10, 512] arrays (mask: [nb, 512] bool)."""
    out = {}
    for name, sl in GROUPS.items():
        x = a[:, sl]
        y = b[:, sl]
        if mask is not None:
            x = x.transpose(1, 0, 2)[:, mask]
            y = y.transpose(1, 0, 2)[:, mask]
        out[name] = rel_l2(x, y)
    return out


# ---- hierarchy brute force (sets of block coordinates) ----------------------
def canonical_sets(levels, nblk0, periodic, t0):
    """Sets of active / deleted block coordinates per level for the canonical
    hierarchy built from the level-0 target blocks t0 (set of tuples).
    nblk0: block counts per axis at level 0; periodic: per-axis bool."""
    def nb(l):
        return tuple(v >> l for v in nblk0)

    def neighbours(b, l):
        out = []
        for d in np.ndindex(3, 3, 3):
            c = [b[a] + d[a] - 1 for a in range(3)]
            ok = True
            for a in range(3):
                if not (0 <= c[a] < nb(l)[a]):
                    if periodic[a]:
                        c[a] %= nb(l)[a]
                    else:
                        ok = False
            if ok:
                out.append(tuple(c))
        return out

    D = [set() for _ in range(levels)]
    B = [set() for _ in range(levels)]
    if levels > 1:
        D[1] = {tuple(v // 2 for v in b) for b in t0}
        for l in range(1, levels):
            B[l] = {c for b in D[l] for c in neighbours(b, l)} - D[l]
            if l + 1 < levels:
                D[l + 1] = {tuple(v // 2 for v in b) for b in D[l] | B[l]}
    active = []
    for l in range(levels):
        if l == levels - 1:
            allb = set(np.ndindex(*nb(l)))
            active.append(allb - D[l])
        else:
            ch = {(2 * b[0] + i, 2 * b[1] + j, 2 * b[2] + k) for b in D[l + 1] | B[l + 1]
                  for i in (0, 1) for j in (0, 1) for k in (0, 1)}
            active.append(ch - D[l])
    return active, D


# ---- composite conservation sums over a multi-level state --------------------
def composite_weights(levels, keys, roles):
    """Per level [nb, 512] weights of the composite grid: every owned node (not ghost,
    not solid) of level l weighs 8^l fine-node volumes, and a node of level l+1 counts
    only if level l does not own the node at the same position (coarse node q sits on
    fine node 2q), so the overlap of two levels is counted once, on the finer one.
    keys[l]: sorted block keys; roles[l]: [nb, 512]."""
    out = []
    node = np.arange(512)
    nx, ny, nz = node & 7, (node >> 3) & 7, node >> 6
    for l in range(levels):
        own = (roles[l] != 1) & (roles[l] != 3)
        if l > 0 and len(keys[l]):
            # the coincident node 2q of level l-1: block 2b + n // 4, node 2n % 8
            bx, by, bz = W.morton_decode(np.asarray(keys[l]))
            fb = [2 * bx[:, None] + (nx >> 2)[None], 2 * by[:, None] + (ny >> 2)[None],
                  2 * bz[:, None] + (nz >> 2)[None]]
            fk = W.morton_encode(fb[0].ravel(), fb[1].ravel(), fb[2].ravel()).reshape(fb[0].shape)
            fn = ((2 * nx) & 7) + 8 * ((2 * ny) & 7) + 64 * ((2 * nz) & 7)
            fine_keys = np.asarray(keys[l - 1])
            covered = np.zeros_like(own)
            if len(fine_keys):
                idx = np.clip(np.searchsorted(fine_keys, fk), 0, len(fine_keys) - 1)
                hit = fine_keys[idx] == fk
                fr = roles[l - 1][idx, np.broadcast_to(fn[None], fk.shape)]
                covered = hit & (fr != 1) & (fr != 3)
            own = own & ~covered
        out.append(own)
    return out


def composite_sums(levels, keys, vals, roles, counted=None):
    """FP64 sums over the composite grid (composite_weights): {"volume", "mass_excess"
    (sum w (rho - 1)), "momentum" (sum w rho u, 3)}. vals[l]: [nb, 10, 512] moments with
    rho - 1 in slot 0; counted: composite_weights of the same hierarchy, if at hand."""
    out = {"volume": 0.0, "mass_excess": 0.0, "momentum": np.zeros(3)}
    counted = composite_weights(levels, keys, roles) if counted is None else counted
    for l in range(levels):
        own = counted[l]
        w = float(8 ** l)
        v = np.asarray(vals[l], dtype=np.float64)
        r = v[:, 0][own]
        rho = 1.0 + r
        out["volume"] += w * own.sum()
        out["mass_excess"] += w * r.sum()
        for a in range(3):
            out["momentum"][a] += w * (rho * v[:, 1 + a][own]).sum()
    return out
