"""Brute-force population-form LBM on small periodic grids (numpy, FP64).

An independent check of the oracle written in a different representation:
27 population arrays, np.roll streaming, and the third-order Hermite
reconstruction written as full tensor contractions over all (a, b, c)
index triples (Sec. 3.1, Eq. three_order_f in its general Hermite form:
f_i = w_i rho [1 + H1.u/cs^2 + H2:S/(2 cs^4) + H3:Gamma/(6 cs^6)]).
Regularised collision: moments of the streamed populations, S relaxed to u u
at rate omega, populations rebuilt from the relaxed moments.
"""
import itertools

import numpy as np

CS2 = 1.0 / 3.0
C = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.float64)  # own ordering
W1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}
W = np.array([W1[int(a)] * W1[int(b)] * W1[int(c)] for a, b, c in C])
OPP = np.array([int(np.where((C == -C[i]).all(1))[0][0]) for i in range(27)])
I3 = np.eye(3)
H1 = C
H2 = np.einsum("ia,ib->iab", C, C) - CS2 * I3[None]
H3 = (np.einsum("ia,ib,ic->iabc", C, C, C)
      - CS2 * (np.einsum("ia,bc->iabc", C, I3) + np.einsum("ib,ac->iabc", C, I3) + np.einsum("ic,ab->iabc", C, I3)))


def moments(f):
    """f: [27, ...] -> rho, u [3, ...], S [3, 3, ...]"""
    rho = f.sum(0)
    j = np.einsum("ia,i...->a...", C, f)
    pi = np.einsum("ia,ib,i...->ab...", C, C, f)
    u = j / rho
    S = pi / rho - CS2 * I3.reshape(3, 3, *([1] * rho.ndim))
    return rho, u, S


def hermite(rho, u, S):
    gam = (np.einsum("ab...,c...->abc...", S, u) + np.einsum("ac...,b...->abc...", S, u)
           + np.einsum("bc...,a...->abc...", S, u) - 2.0 * np.einsum("a...,b...,c...->abc...", u, u, u))
    t1 = np.einsum("ia,a...->i...", H1, u) / CS2
    t2 = np.einsum("iab,ab...->i...", H2, S) / (2.0 * CS2 ** 2)
    t3 = np.einsum("iabc,abc...->i...", H3, gam) / (6.0 * CS2 ** 3)
    shp = (27,) + (1,) * rho.ndim
    return W.reshape(shp) * rho[None] * (1.0 + t1 + t2 + t3)


def collide(rho, u, S, omega):
    uu = np.einsum("a...,b...->ab...", u, u)
    return rho, u, S + omega * (uu - S)


def step(f, omega, solid=None):
    """One stream-collide step on a periodic grid; f is [27, X, Y, Z] (axis order x, y, z).
    solid: bool [X, Y, Z] or None (halfway bounce-back in pull form)."""
    rho, u, S = moments(f)
    fp = hermite(*collide(rho, u, S, omega))
    out = np.empty_like(fp)
    for i in range(27):
        out[i] = np.roll(fp[i], shift=tuple(int(v) for v in C[i]), axis=(0, 1, 2))
        if solid is not None:
            src_solid = np.roll(solid, shift=tuple(int(v) for v in C[i]), axis=(0, 1, 2))
            out[i] = np.where(src_solid, fp[OPP[i]], out[i])
    if solid is not None:
        out[:, solid] = f[:, solid]
    return out


def from_moments(q):
    """q: [10, X, Y, Z] stored-order moments (rho-1 first) -> populations [27, X, Y, Z]."""
    rho = 1.0 + q[0]
    u = q[1:4]
    S = np.empty((3, 3) + q.shape[1:])
    for (a, b), k in {(0, 0): 4, (1, 1): 5, (2, 2): 6, (0, 1): 7, (0, 2): 8, (1, 2): 9}.items():
        S[a, b] = q[k]
        S[b, a] = q[k]
    return hermite(rho, u, S)


def to_moments(f):
    rho, u, S = moments(f)
    return np.stack([rho - 1.0, u[0], u[1], u[2], S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2]])


def step_channel(f, omega, outflow="zero_gradient"):
    """One step with a held inflow plane at x = 0 and an outflow plane at x = X - 1
    (y, z periodic); f is [27, X, Y, Z]. Interior planes pull from their neighbours;
    the inflow plane keeps its populations; the outflow plane takes, per node, the
    new moments of its inner neighbour (zero gradient) or one implicit upwind step of
    dM/dt + u_n dM/dn = 0 with u_n = max(u_x of that neighbour, 0) (convective)."""
    rho, u, S = moments(f)
    fp = hermite(*collide(rho, u, S, omega))
    out = np.empty_like(fp)
    for i in range(27):
        out[i] = np.roll(fp[i], shift=tuple(int(v) for v in C[i]), axis=(0, 1, 2))
    out[:, 0] = f[:, 0]
    q_old = to_moments(f[:, -1:])[:, 0]
    q_in = to_moments(out[:, -2:-1])[:, 0]
    if outflow == "zero_gradient":
        q_new = q_in
    else:
        lam = np.maximum(q_in[1], 0.0)
        q_new = (q_old + lam[None] * q_in) / (1.0 + lam[None])
    out[:, -1] = from_moments(q_new[:, None])[:, 0]
    return out
