"""The adjoint through grid updates (Sec. 6.3: new nodes interpolated from the parent
level or transferred up from the children) on the GPU, through the C ABI, against the
complex-step derivative of the FP64 oracle over the same adaptive run.

A recording (lbm_record_begin / lbm_record_end) holds coarse steps and grid updates
that move the refined region (two level-0 blocks at a time on two levels, one
level-2 block on three), so that every update creates and deletes blocks on every
level: new fine nodes are sampled downward from the parent level and new coarse
nodes take the values of the children they replace.
The reverse sweep takes the adjoint of the final state (final hierarchy) back to the
initial state (initial hierarchy). Two and three levels; directional derivatives of a
kinetic-energy loss along random directions over every initial moment, relative
error <= 1e-4 (FP32 adjoint against the FP64 complex step). The simulation returns
to its initial hierarchy and state.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2603_14982_amd import workloads as W

pytestmark = pytest.mark.gpu

P = W.PERIODIC

CASES = {
    # levels, extent, marker blocks, moves of the particles (fine units), loss boxes per level
    "two_level": (2, (80, 80, 80), (4, 5), [(16.0, 0.0, 0.0), (0.0, 16.0, -16.0)],
                  {0: ((0, 0, 0), (80, 80, 80)), 1: ((0, 0, 0), (80, 80, 80))}),
    "three_level": (3, (128, 128, 128), (7, 8), [(32.0, 0.0, 0.0), (0.0, -32.0, 16.0)],
                    {0: ((0, 0, 0), (128, 128, 128)), 1: ((0, 0, 0), (128, 128, 128)),
                     2: ((0, 0, 0), (128, 128, 128))}),
}


def _lbm():
    from paper_2603_14982_amd import lbm
    return lbm


def _fields(levels, n, keys, seed):
    u0 = W.smooth_random_velocity(n, seed, kmax=4.0, rms=0.03)
    rng = np.random.default_rng(seed + 1)
    x, v = [], []
    for l in range(levels):
        q = W.velocity_moments(l, keys[l], u0)
        q[:, 0] += 1e-3 * rng.standard_normal(q[:, 0].shape)
        q[:, 4:] += 1e-4 * rng.standard_normal(q[:, 4:].shape)
        x.append(q)
        v.append(rng.standard_normal((3,) + q.shape))
    return x, v


def _oracle_derivative(case, x, vk):
    L, n, marks, moves, boxes = CASES[case]
    p = W.block_centre_markers(marks).copy()
    sim = O.OracleSimComplex(L, n, (P,) * 6, 0.6, particles=p)
    for l in range(L):
        sim.set_block_moments(l, sim.block_keys(l), x[l], 1e-30 * vk[l])
    for d in moves:
        sim.step(1)
        O.advance_particles(p, np.array(d, dtype=np.float32))
        sim.remesh(p)
    sim.step(1)
    return sum(sim.kinetic_energy(l, *b) for l, b in boxes.items()).imag / 1e-30


@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_through_grid_updates_against_complex_step(case):
    lbm = _lbm()
    L, n, marks, moves, boxes = CASES[case]
    print(f"adjoint through grid updates: {case}", flush=True)
    p = torch.as_tensor(W.block_centre_markers(marks)).cuda()
    sim = lbm.Sim(L, n, (P,) * 6, 0.6, particles=p)
    keys0 = [sim.block_keys(l).cpu().numpy() for l in range(L)]
    x, v = _fields(L, n, keys0, 31)
    for l in range(L):
        sim.set_block_moments(l, keys0[l], x[l].astype(np.float32))
    x0 = sim.get_all_moments().clone()
    work = sim.record_work(len(moves) + 1, len(moves))
    sim.record_begin(work)
    changed = []
    for d in moves:
        sim.step(1)
        before = [sim.block_keys(l).cpu().numpy() for l in range(L)]
        sim.advance_particles(p, d)
        sim.remesh(p)
        after = [sim.block_keys(l).cpu().numpy() for l in range(L)]
        changed.append([int(len(np.setdiff1d(a, b)) + len(np.setdiff1d(b, a))) for a, b in zip(after, before)])
    sim.step(1)
    sim.record_end()
    print(f"{case}: blocks created + deleted per level and update: {changed}", flush=True)
    assert all(c > 0 for ch in changed for c in ch)
    assert sim.total_blocks() > 0
    lam = sum(sim.loss_ke_grad(l, *b) for l, b in boxes.items())
    lam0 = sim.adjoint_reverse(lam, work=work)
    torch.cuda.synchronize()
    # back at the initial hierarchy and state
    for l in range(L):
        assert np.array_equal(sim.block_keys(l).cpu().numpy(), keys0[l])
    assert torch.equal(sim.get_all_moments(), x0)
    g = lam0.cpu().numpy().astype(np.float64)
    roles = np.concatenate([sim.roles(l).cpu().numpy() for l in range(L)])
    assert np.all(g.transpose(0, 2, 1)[np.isin(roles, (O.R_GHOST, O.R_SOLID, O.R_INFLOW))] == 0.0)
    got, want = [], []
    for k in range(3):
        vk = [vl[k] for vl in v]
        got.append(float(np.sum(g * np.concatenate(vk))))
        want.append(_oracle_derivative(case, x, vk))
    got, want = np.array(got), np.array(want)
    err = np.abs(got - want) / np.linalg.norm(want)
    print(f"{case}: adjoint {got}, complex step {want}, rel err {err}", flush=True)
    assert np.all(err <= 1e-4), err


def test_recording_guards():
    lbm = _lbm()
    p = torch.as_tensor(W.block_centre_markers((4, 5))).cuda()
    sim = lbm.Sim(2, (80, 80, 80), (P,) * 6, 0.6, particles=p)
    work = sim.record_work(1, 1)
    sim.record_begin(work)
    with pytest.raises(lbm.LBMError):
        sim.record_begin(work)
    with pytest.raises(lbm.LBMError):
        sim.adjoint_reverse(sim.loss_ke_grad(0, (0, 0, 0), (80, 80, 80)), work=work)
    keys = sim.block_keys(0).cpu().numpy()[:1]
    with pytest.raises(lbm.LBMError):
        sim.set_block_moments(0, keys, np.zeros((1, 10, 512), dtype=np.float32))
    with pytest.raises(lbm.LBMError):  # the run lists belong to the recorded hierarchy
        sim.set_option("pair_run", 2)
    sim.step(1)
    sim.remesh(p)  # same particles: nothing changes, nothing is logged
    sim.record_end()
    with pytest.raises(lbm.LBMError):
        sim.record_end()
