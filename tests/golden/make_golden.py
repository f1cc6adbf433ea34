"""Writes the stored expected values of the full-size parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generators; no value
here comes from the GPU path. Each output holds a seeded sample of owned nodes
(level, block key, node index, 10 moments) of the oracle's state; the slab file
holds samples by node class after 20 and 200 coarse steps and the composite
conservation sums every 10 steps.

  python tests/golden/make_golden.py sphere128   # 500 coarse steps
  python tests/golden/make_golden.py slab512     # 200 coarse steps with grid updates
  python tests/golden/make_golden.py adjoint128  # loss and 16 directional derivatives

The adjoint file holds the kinetic-energy loss after 200 coarse steps of the
two-level 128^3 case and its derivatives along 16 unit directions of the initial
velocity, by the complex step (step 1e-30) in the complex instance of the oracle.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2603_14982_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_state(sim, per_level, seed):
    rng = np.random.default_rng(seed)
    out = {"level": [], "key": [], "node": [], "values": []}
    counts = []
    for l in range(sim.levels):
        keys, vals = sim.get_block_moments(l)
        roles = sim.roles(l)
        counts.append(len(keys))
        own = np.argwhere(roles != O.R_GHOST)
        if len(own) == 0:
            continue
        pick = own[rng.choice(len(own), size=min(per_level, len(own)), replace=False)]
        out["level"].append(np.full(len(pick), l, dtype=np.int32))
        out["key"].append(keys[pick[:, 0]])
        out["node"].append(pick[:, 1].astype(np.int32))
        out["values"].append(vals[pick[:, 0], :, pick[:, 1]])
    res = {k: np.concatenate(v) for k, v in out.items()}
    res["blocks_per_level"] = np.array(counts, dtype=np.int64)
    return res


def sphere128(steps=500):
    wl = W.workload("sphere128")
    c, r = wl["sphere"]
    solid = W.sphere_solid(wl["n"], c, r)
    sim = O.OracleSim(2, wl["n"], wl["bc"], wl["tau0"], uin=wl["uin"], solid=solid)
    for l in range(2):
        keys = sim.block_keys(l)
        sim.set_block_moments(l, keys, W.uniform_field(l, keys))
    t = time.time()
    for i in range(steps):
        sim.step(1)
        if i % 50 == 49:
            print(f"sphere128 step {i + 1} ({time.time() - t:.0f} s)", flush=True)
    res = sample_state(sim, 4096, seed=128)
    res["steps"] = np.array(steps)
    np.savez_compressed(os.path.join(HERE, "sphere128_oracle_sample.npz"), **res)


SAMPLE_CLASSES = ("bulk", "iu", "edge")


def sample_classes(sim, seed, per_class=(8192, 4096, 4096)):
    """Seeded samples of one state in three classes per level: "bulk" (computed nodes),
    "iu" (upward-interface nodes, written by the upward transfer) and "edge" (computed
    nodes of blocks that hold ghost nodes: the ones whose neighbours the downward
    transfer writes)."""
    rng = np.random.default_rng(seed)
    out = {"level": [], "cls": [], "key": [], "node": [], "values": []}
    counts = []
    for l in range(sim.levels):
        keys, vals = sim.get_block_moments(l)
        roles = sim.roles(l)
        counts.append(len(keys))
        has_ghost = (roles == O.R_GHOST).any(axis=1)
        masks = (roles == O.R_INTERIOR, roles == O.R_IU, (roles == O.R_INTERIOR) & has_ghost[:, None])
        for c, (m, k) in enumerate(zip(masks, per_class)):
            cand = np.argwhere(m)
            if len(cand) == 0:
                continue
            pick = cand[np.sort(rng.choice(len(cand), size=min(k, len(cand)), replace=False))]
            out["level"].append(np.full(len(pick), l, dtype=np.int32))
            out["cls"].append(np.full(len(pick), c, dtype=np.int32))
            out["key"].append(keys[pick[:, 0]])
            out["node"].append(pick[:, 1].astype(np.int32))
            out["values"].append(vals[pick[:, 0], :, pick[:, 1]])
    res = {k: np.concatenate(v) for k, v in out.items()}
    res["blocks_per_level"] = np.array(counts, dtype=np.int64)
    return res


def conservation(sim):
    """Composite sums of one oracle state: volume, mass excess, momentum (tests/util.py)."""
    from tests.util import composite_sums
    keys, vals, roles = [], [], []
    for l in range(sim.levels):
        k, v = sim.get_block_moments(l)
        keys.append(k)
        vals.append(v)
        roles.append(sim.roles(l))
    c = composite_sums(sim.levels, keys, vals, roles)
    return np.array([c["volume"], c["mass_excess"], *c["momentum"]])


def slab512(coarse_steps=None, sample_at=(20,), sums_every=10):
    """The three-level slab case over its coarse steps with grid updates: samples of
    every class after `sample_at` steps and at the end, composite conservation sums
    every `sums_every` steps (and at step 0)."""
    wl = W.workload("slab512")
    coarse_steps = wl["steps"] if coarse_steps is None else coarse_steps
    p = W.slab_particles(wl["particles"], wl["seed"], wl["lo"], wl["hi"])
    t = time.time()
    sim = O.OracleSim(3, wl["n"], wl["bc"], wl["tau0"], particles=p)
    print(f"slab512 hierarchy built ({time.time() - t:.0f} s)", flush=True)
    for l in range(3):
        keys = sim.block_keys(l)
        for s in range(0, len(keys), 2048):
            k = keys[s:s + 2048]
            sim.set_block_moments(l, k, W.tgv3d_field(l, k, wl["n"], wl["amp"]))
    sub = 1 << (wl["levels"] - 1)
    d = np.array([v * sub for v in wl["v_fine"]], dtype=np.float32)
    res = {"steps": np.array(coarse_steps), "sums_steps": [0], "sums": [conservation(sim)]}
    for i in range(coarse_steps):
        sim.step(1)
        O.advance_particles(p, d)
        sim.remesh(p)
        done = i + 1
        if done in sample_at or done == coarse_steps:
            s = sample_classes(sim, seed=512 + done)
            for k, v in s.items():
                res[f"s{done}_{k}"] = v
        if done % sums_every == 0 or done == coarse_steps:
            res["sums_steps"].append(done)
            res["sums"].append(conservation(sim))
            print(f"slab512 step {done}: sums {res['sums'][-1]}", flush=True)
        print(f"slab512 coarse step {done} ({time.time() - t:.0f} s)", flush=True)
    res["sums_steps"] = np.array(res["sums_steps"])
    res["sums"] = np.array(res["sums"])
    res["sample_steps"] = np.array(sorted(set(sample_at) | {coarse_steps}))
    np.savez_compressed(os.path.join(HERE, "slab512_oracle_run.npz"), **res)


def adjoint_setup(wl):
    """The oracle's initial moments of the two-level adjoint case: real part from the
    velocity u0, imaginary part (per direction) the moments' derivative along d."""
    u0 = W.smooth_random_velocity(wl["n"], wl["seed"], wl["kmax"], wl["rms"])
    return u0, W.unit_directions(wl["n"], wl["direction_seeds"], wl["kmax"])


def moment_tangent(level, keys, u0, d):
    """d/dh of the moments (rho = 1, u = u0 + h d, S = u u) at h = 0: (0, d, u0 d + d u0)."""
    a = W.sample_dense(level, keys, u0)
    b = W.sample_dense(level, keys, d)
    nb = a.shape[0]
    out = np.zeros((nb, 10, 512))
    out[:, 1:4] = b
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for k, (i, j) in enumerate(pairs):
        out[:, 4 + k] = a[:, i] * b[:, j] + b[:, i] * a[:, j]
    return out


def adjoint128(steps=None):
    wl = W.workload("adjoint128")
    steps = wl["steps"] if steps is None else steps
    u0, dirs = adjoint_setup(wl)
    lo, hi = wl["box"]
    h = 1e-30
    t = time.time()
    real = O.OracleSim(2, wl["n"], wl["bc"], wl["tau0"], particles=wl["markers"])
    for l in range(2):
        keys = real.block_keys(l)
        real.set_block_moments(l, keys, W.velocity_moments(l, keys, u0))
    real.step(steps)
    loss = real.kinetic_energy(0, lo, hi)
    print(f"adjoint128 loss {loss!r} ({time.time() - t:.0f} s)", flush=True)
    deriv = []
    for k, d in enumerate(dirs):
        sim = O.OracleSimComplex(2, wl["n"], wl["bc"], wl["tau0"], particles=wl["markers"])
        for l in range(2):
            keys = sim.block_keys(l)
            sim.set_block_moments(l, keys, W.velocity_moments(l, keys, u0), h * moment_tangent(l, keys, u0, d))
        sim.step(steps)
        v = sim.kinetic_energy(0, lo, hi)
        deriv.append(v.imag / h)
        print(f"direction {k}: loss {v.real!r} derivative {deriv[-1]!r} ({time.time() - t:.0f} s)", flush=True)
        del sim
    np.savez(os.path.join(HERE, "adjoint128_oracle_derivatives.npz"), loss=np.array(loss),
             derivatives=np.array(deriv), steps=np.array(steps), h=np.array(h),
             seeds=np.array(wl["direction_seeds"]))


if __name__ == "__main__":
    for name in sys.argv[1:]:
        {"sphere128": sphere128, "slab512": slab512, "adjoint128": adjoint128}[name]()
