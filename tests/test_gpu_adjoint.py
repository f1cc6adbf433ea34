"""The adjoint on the GPU (C ABI through the Python binding) against the
complex-step derivative of the FP64 oracle, plus the state save/load it rests on.

- Directional derivatives of a kinetic-energy loss after a few coarse steps with
  respect to every initial moment, along random directions, on one level (periodic at
  three sizes; walls for bounce-back), two levels (periodic; sphere with inflow and outflow
  faces; the same with a logarithmic inflow profile, convective outflow and walls)
  and three levels: relative error <= 1e-4 (FP32 adjoint vs FP64 complex
  step). With BF16 storage the gradient stays within 3% of the FP32 one.
- Entries of the gradient at nodes that carry no state (ghost, solid, inflow) are 0.
- The checkpointed autograd rollout equals the chain of single adjoint steps and
  leaves the simulation at its final state, also when the simulation stepped on
  before the backward pass; the rollout that keeps its whole undo log (no
  checkpoints) gives the same gradient; a recording is dropped by a step.
- Full size: the two-level 128^3 case, 200 coarse steps with checkpoints every 20,
  gradient with respect to the initial velocity field, against the 16 stored
  complex-step derivatives (tests/golden/, written from the oracle alone).
"""
import os
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W

pytestmark = pytest.mark.gpu

P, INF, OUT, WALL, CONV = W.PERIODIC, W.INFLOW, W.OUTFLOW, W.WALL, W.OUTFLOW_CONV
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

CASES = {
    # levels, extent, bc, uin, solid, particles, loss boxes per level
    "single": (1, (32, 32, 32), (P,) * 6, (0.0, 0.0, 0.0), None, None, {0: ((8, 8, 8), (24, 24, 24))}),
    "walls": (1, (32, 32, 32), (P, P, P, P, WALL, WALL), (0.0, 0.0, 0.0), None, None,
              {0: ((0, 0, 0), (32, 32, 32))}),
    # levels of 1728 and 4096 blocks: the transpose takes a block's output planes in
    # 2 workgroups and in 1 (levels under 1024 blocks, as in every other case, in 4)
    "single96": (1, (96, 96, 96), (P,) * 6, (0.0, 0.0, 0.0), None, None, {0: ((24, 24, 24), (72, 72, 72))}),
    "single128": (1, (128, 128, 128), (P,) * 6, (0.0, 0.0, 0.0), None, None, {0: ((32, 32, 32), (96, 96, 96))}),
    "two_level": (2, (80, 80, 80), (P,) * 6, (0.0, 0.0, 0.0), None, W.block_centre_markers((4, 5)),
                  {0: ((16, 16, 16), (64, 64, 64)), 1: ((0, 0, 0), (80, 80, 80))}),
    "sphere": (2, (80, 80, 80), (INF, OUT, P, P, P, P), (0.03, 0.0, 0.0),
               W.sphere_solid((80, 80, 80), (40.0, 40.0, 40.0), 3.0), None,
               {0: ((16, 16, 16), (64, 64, 64)), 1: ((0, 0, 0), (80, 80, 80))}),
    # log inflow along z (zero at the lower wall), convective outflow, no-slip z faces
    "open": (2, (80, 80, 80), (INF, CONV, P, P, WALL, WALL), (0.03, 0.0, 0.0),
             W.sphere_solid((80, 80, 80), (40.0, 40.0, 40.0), 3.0), None,
             {0: ((16, 16, 16), (64, 64, 64)), 1: ((0, 0, 0), (80, 80, 80))}),
    # three levels: 512 + 504 + 56 blocks, two interfaces
    "three_level": (3, (128, 128, 128), (P,) * 6, (0.0, 0.0, 0.0), None, W.block_centre_markers((7, 8)),
                    {0: ((32, 32, 32), (96, 96, 96)), 1: ((0, 0, 0), (128, 128, 128)),
                     2: ((0, 0, 0), (128, 128, 128))}),
}


def _lbm():
    from paper_2603_14982_amd import lbm
    return lbm


LOG_INFLOW = {"open": (2, 0.08, 0.0)}  # axis, beta, h0


def _gpu(case):
    L, n, bc, uin, solid, parts, _ = CASES[case]
    return _lbm().Sim(L, n, bc, 0.6, uin=uin, solid=solid, particles=parts, log_inflow=LOG_INFLOW.get(case))


def _oracle(case, complex_=False):
    L, n, bc, uin, solid, parts, _ = CASES[case]
    cls = O.OracleSimComplex if complex_ else O.OracleSim
    return cls(L, n, bc, 0.6, uin=uin, solid=solid, particles=parts, log_inflow=LOG_INFLOW.get(case))


def _fields(case, keys, seed):
    """FP64 initial moments per level and three random directions per level."""
    L, n = CASES[case][0], CASES[case][1]
    u0 = W.smooth_random_velocity(n, seed, kmax=4.0, rms=0.03)
    rng = np.random.default_rng(seed + 1)
    x, v = [], []
    for l in range(L):
        q = W.velocity_moments(l, keys[l], u0)
        q[:, 0] += 1e-3 * rng.standard_normal(q[:, 0].shape)
        q[:, 4:] += 1e-4 * rng.standard_normal(q[:, 4:].shape)
        x.append(q)
        v.append(rng.standard_normal((3,) + q.shape))
    return x, v


def _oracle_derivative(case, x, v, steps):
    sim = _oracle(case, complex_=True)
    for l in range(len(x)):
        sim.set_block_moments(l, sim.block_keys(l), x[l], 1e-30 * v[l])
    sim.step(steps)
    boxes = CASES[case][6]
    return sum(sim.kinetic_energy(l, *b) for l, b in boxes.items()).imag / 1e-30


def _gpu_gradient(sim, x, steps, boxes):
    """dLoss/d(initial moments), all-level layout, by saved states + adjoint steps."""
    L = sim.levels
    for l in range(L):
        sim.set_block_moments(l, sim.block_keys(l).cpu().numpy(), x[l].astype(np.float32))
    states = []
    for _ in range(steps):
        states.append(sim.save())
        sim.step(1)
    lam = sum(sim.loss_ke_grad(l, *b) for l, b in boxes.items())
    work = sim.adjoint_work()
    for st in reversed(states):
        sim.adjoint_step(st, lam, lam, work)
    torch.cuda.synchronize()
    return lam


@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_directional_derivatives_against_complex_step(case):
    print(f"adjoint case {case}", flush=True)
    sim = _gpu(case)
    keys = [sim.block_keys(l).cpu().numpy() for l in range(sim.levels)]
    ref = _oracle(case)
    for l in range(sim.levels):
        assert np.array_equal(ref.block_keys(l), keys[l])
    x, v = _fields(case, keys, 21)
    steps = 3
    lam = _gpu_gradient(sim, x, steps, CASES[case][6]).cpu().numpy().astype(np.float64)
    roles = np.concatenate([sim.roles(l).cpu().numpy() for l in range(sim.levels)])
    # no gradient at nodes without state
    dead = np.isin(roles, (O.R_GHOST, O.R_SOLID, O.R_INFLOW))
    assert np.all(lam.transpose(0, 2, 1)[dead] == 0.0)
    got, want = [], []
    for k in range(3):
        vk = [vl[k] for vl in v]
        got.append(float(np.sum(lam * np.concatenate(vk))))
        want.append(_oracle_derivative(case, x, vk, steps))
    got, want = np.array(got), np.array(want)
    err = np.abs(got - want) / np.linalg.norm(want)
    print(f"{case}: adjoint {got}, complex step {want}, rel err {err}", flush=True)
    assert np.all(err <= 1e-4), err


def test_state_save_load_roundtrip_and_replay():
    sim = _gpu("sphere")
    keys = [sim.block_keys(l).cpu().numpy() for l in range(2)]
    x, _ = _fields("sphere", keys, 3)
    for l in range(2):
        sim.set_block_moments(l, keys[l], x[l].astype(np.float32))
    sim.step(2)
    st = sim.save()
    assert st.numel() == sim.state_bytes() == 256 + sim.total_blocks() * 5120 * 4
    a = sim.get_all_moments().clone()
    sim.step(3)
    b = sim.get_all_moments().clone()
    sim.load(st)
    assert torch.equal(sim.get_all_moments(), a)
    sim.step(3)
    assert torch.equal(sim.get_all_moments(), b)
    # an adjoint step leaves the simulation at the state it was given
    lam = sim.loss_ke_grad(0, (16, 16, 16), (64, 64, 64))
    sim.adjoint_step(st, lam)
    assert torch.equal(sim.get_all_moments(), a)
    with pytest.raises(_lbm().LBMError):
        sim.load(st[:100])


def test_state_rejected_after_hierarchy_change():
    lbm = _lbm()
    p = torch.as_tensor(W.block_centre_markers((4, 5))).cuda()
    sim = lbm.Sim(2, (80, 80, 80), (P,) * 6, 0.6, particles=p)
    st = sim.save()
    sim.remesh(p)  # same particles: no change, the state stays valid
    sim.load(st)
    q = p + torch.tensor([16.0, 0.0, 0.0], device="cuda")
    sim.remesh(q)
    with pytest.raises(lbm.LBMError) as e:
        sim.load(st)
    assert e.value.status == -6


def _torch_init(sim, u0):
    """All-level moments from a dense velocity [3, Z, Y, X] (differentiable): rho = 1,
    u sampled at each node's fine position, S = u u."""
    parts = []
    for l in range(sim.levels):
        pos = torch.as_tensor(W.node_positions(l, sim.block_keys(l).cpu().numpy()), device=u0.device)
        u = u0[:, pos[..., 2], pos[..., 1], pos[..., 0]]  # [3, nb, 512]
        S = [u[0] * u[0], u[1] * u[1], u[2] * u[2], u[0] * u[1], u[0] * u[2], u[1] * u[2]]
        parts.append(torch.stack([torch.zeros_like(u[0]), u[0], u[1], u[2]] + S, dim=1))
    return torch.cat(parts)


def _torch_loss(sim, xt, level, box):
    lo, hi = box
    off = sum(sim.num_blocks(l) for l in range(level))
    nb = sim.num_blocks(level)
    q = xt[off:off + nb]
    pos = torch.as_tensor(W.node_positions(level, sim.block_keys(level).cpu().numpy()), device=xt.device)
    inside = torch.ones(pos.shape[:2], dtype=torch.bool, device=xt.device)
    for a in range(3):
        inside &= (pos[..., a] >= lo[a]) & (pos[..., a] < hi[a])
    r = sim.roles(level)
    owned = (r == 0) | (r == 2) | (r == 4) | (r == 5)
    m = (inside & owned).to(q.dtype)
    ke = 0.5 * (1.0 + q[:, 0]) * (q[:, 1] ** 2 + q[:, 2] ** 2 + q[:, 3] ** 2)
    return (ke * m).sum()


def test_rollout_autograd_equals_adjoint_chain():
    lbm = _lbm()
    sim = _gpu("two_level")
    u0 = torch.as_tensor(W.smooth_random_velocity((80, 80, 80), 4, kmax=4.0, rms=0.03), dtype=torch.float32,
                         device="cuda").requires_grad_(True)
    x0 = _torch_init(sim, u0)
    xt = lbm.rollout(sim, x0, 5, checkpoint_every=2)
    final = sim.get_all_moments().clone()
    loss = _torch_loss(sim, xt, 0, ((16, 16, 16), (64, 64, 64)))
    g_x0 = torch.autograd.grad(loss, x0, retain_graph=True)[0]
    assert torch.equal(sim.get_all_moments(), final)  # backward restores the final state
    # the same gradient from single adjoint steps over saved states
    keys = [sim.block_keys(l).cpu().numpy() for l in range(2)]
    sizes = [len(k) for k in keys]
    xs = x0.detach().cpu().numpy().astype(np.float64)
    x = [xs[:sizes[0]], xs[sizes[0]:]]
    lam = _gpu_gradient(sim, x, 5, {0: ((16, 16, 16), (64, 64, 64))})
    assert torch.allclose(g_x0, lam, rtol=0, atol=1e-6 * lam.abs().max().item())


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "adjoint128_oracle_derivatives.npz")),
                    reason="stored oracle derivatives not generated")
def test_adjoint128_gradient_against_oracle_derivatives():
    lbm = _lbm()
    wl = W.workload("adjoint128")
    g = np.load(os.path.join(GOLDEN, "adjoint128_oracle_derivatives.npz"), allow_pickle=False)
    steps = int(g["steps"])
    print(f"adjoint128: {steps} coarse steps, checkpoints every {wl['checkpoint_every']}", flush=True)
    sim = lbm.Sim(2, wl["n"], wl["bc"], wl["tau0"], particles=wl["markers"])
    assert (sim.num_blocks(0), sim.num_blocks(1)) == (512, 504)
    u0 = torch.as_tensor(W.smooth_random_velocity(wl["n"], wl["seed"], wl["kmax"], wl["rms"]),
                         dtype=torch.float32, device="cuda").requires_grad_(True)
    x0 = _torch_init(sim, u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xt = lbm.rollout(sim, x0, steps, checkpoint_every=wl["checkpoint_every"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = _torch_loss(sim, xt, 0, wl["box"])
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"loss {loss.item():.8e} (oracle {float(g['loss']):.8e}); forward {t1 - t0:.3f} s, "
          f"backward {t2 - t1:.3f} s", flush=True)
    assert abs(loss.item() - float(g["loss"])) <= 1e-5 * abs(float(g["loss"]))
    dirs = W.unit_directions(wl["n"], tuple(int(s) for s in g["seeds"]), wl["kmax"])
    G = u0.grad.detach().cpu().numpy().astype(np.float64)
    got = np.einsum("kcxyz,cxyz->k", dirs, G)
    want = g["derivatives"]
    err = np.abs(got - want) / np.linalg.norm(want)
    print(f"directional derivatives: max rel err {err.max():.3e}; "
          f"vector rel err {np.linalg.norm(got - want) / np.linalg.norm(want):.3e}", flush=True)
    assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want)
    assert np.all(err <= 1e-4)


def test_taped_rollout_equals_checkpointed_rollout():
    lbm = _lbm()
    sim = _gpu("sphere")
    u0 = torch.as_tensor(W.smooth_random_velocity((80, 80, 80), 6, kmax=4.0, rms=0.03), dtype=torch.float32,
                         device="cuda")
    box = ((16, 16, 16), (64, 64, 64))
    grads = []
    for every in (2, 0):
        x0 = _torch_init(sim, u0).detach().requires_grad_(True)
        xt = lbm.rollout(sim, x0, 5, checkpoint_every=every)
        final = sim.get_all_moments().clone()
        loss = _torch_loss(sim, xt, 0, box)
        (g,) = torch.autograd.grad(loss, x0)
        assert torch.equal(sim.get_all_moments(), final)
        grads.append(g)
    assert torch.allclose(grads[0], grads[1], rtol=0, atol=1e-6 * grads[0].abs().max().item())


def test_checkpointed_rollout_when_the_simulation_moved_on():
    # the forward pass records its last segment; if the simulation steps before the
    # backward pass, that recording is refused and the segment is replayed instead
    lbm = _lbm()
    sim = _gpu("two_level")
    u0 = torch.as_tensor(W.smooth_random_velocity((80, 80, 80), 8, kmax=4.0, rms=0.03), dtype=torch.float32,
                         device="cuda")
    box = ((16, 16, 16), (64, 64, 64))
    grads = []
    for moved in (False, True):
        x0 = _torch_init(sim, u0).detach().requires_grad_(True)
        xt = lbm.rollout(sim, x0, 5, checkpoint_every=2)
        final = sim.get_all_moments().clone()
        loss = _torch_loss(sim, xt, 0, box)
        if moved:
            sim.step(2)
        (g,) = torch.autograd.grad(loss, x0)
        assert torch.equal(sim.get_all_moments(), final)
        grads.append(g)
    assert torch.allclose(grads[0], grads[1], rtol=0, atol=1e-6 * grads[0].abs().max().item())


def test_recording_dropped_by_a_step():
    lbm = _lbm()
    sim = _gpu("two_level")
    work = sim.adjoint_work(2)
    sim.step_record(2, work)
    lam = sim.loss_ke_grad(0, (16, 16, 16), (64, 64, 64))
    sim.step(1)
    with pytest.raises(lbm.LBMError) as e:
        sim.adjoint_reverse(lam, work=work)
    assert e.value.status == -6


def test_bf16_storage_gradient_close_to_f32():
    # the adjoint passes the 16-bit rounding of stored values through unchanged: the
    # gradient of a BF16 run differs from the FP32 one by about the storage precision
    lbm = _lbm()
    L, n, bc, uin, solid, parts, boxes = CASES["two_level"]
    scale = [64.0, 8.0, 8.0, 8.0, 64.0, 64.0, 64.0, 64.0, 64.0, 64.0]
    grads = []
    for storage in ("f32", "bf16"):
        sim = lbm.Sim(L, n, bc, 0.6, uin=uin, solid=solid, particles=parts, storage=storage,
                      scale=scale if storage != "f32" else None)
        keys = [sim.block_keys(l).cpu().numpy() for l in range(L)]
        x, _ = _fields("two_level", keys, 31)
        grads.append(_gpu_gradient(sim, x, 3, boxes).double())
    err = (torch.linalg.norm(grads[1] - grads[0]) / torch.linalg.norm(grads[0])).item()
    print(f"bf16 vs f32 gradient: rel L2 {err:.3e}", flush=True)
    assert torch.isfinite(grads[1]).all() and err < 3e-2, err
