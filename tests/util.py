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
