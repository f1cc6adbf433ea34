#!/usr/bin/env python3
"""Throughput of the block-adaptive D3Q27 moment LBM step on one MI355X.

Workload (the three-level adaptive configuration): 512^3 fine-equivalent
periodic box, 3 levels of 8^3-node blocks, 2,000,000 seeded particles in the
slab x, y in [64, 448), z in [352, 384) falling at 0.02 fine nodes per finest
step, 3D Taylor-Green initial field (U = 0.05, wavelength 512, rho = 1,
S = u u), tau_0 = 0.6, FP32 moments. One step = one coarse step of Alg. 1
(4 finest substeps, 2 on level 1, 1 on level 2, downward/upward transfers),
the particle advance and one grid update.

Prints one JSON line. `value` is MLUPS (computed-node updates per second over
the whole step, grid update included). The roofline object is the dominant
kernel, level 0's stream-collide on 2 x 2 x 2 block tiles: both substeps of a
level-1 step in one launch (2 launches per coarse step; with --no-fuse one substep
per launch, 4 per coarse step). `achieved` is its algorithmic bytes (80 B per
computed-node update with FP32 moments: 10 moments read and written, counted per
update, so a launch of two updates counts 160 B per node) over its average launch
duration, timed with HIP events around those launches in the timed region (no other
launch is bracketed there: each timed launch costs two event records); `hbm_achieved`
is the HBM traffic the counters measured for that launch (`traffic`, when the
stored counter run matches the kernel source) over the same duration. Every phase is
timed over --breakdown-steps further steps (`phase_ms_per_step`, and the figures over
every stream-collide launch of all levels given beside the roofline).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + achieved HBM GB/s per LBM step; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 80.0, "bf16": 40.0, "f16": 40.0}  # 10 moments read + 10 written
# per-moment power-of-two scales of the 16-bit formats: rho - 1, u (3), S (6)
HALF_SCALES = [64.0, 8.0, 8.0, 8.0, 64.0, 64.0, 64.0, 64.0, 64.0, 64.0]
STORE_NAME = {"f32": "StoreF32", "bf16": "StoreBF16", "f16": "StoreF16"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stream_collide_slab512_traffic.json")
VALU_CUS, VALU_CLOCK_HZ = 256, 2.4e9  # MI355X compute units and peak engine clock


def sc_source_hash():
    """Hash of the stream-collide source the stored counter figures belong to."""
    with open(os.path.join(ROOT, "paper_2603_14982_amd", "csrc", "stream_collide.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def init_fields(sim, wl, W):
    import numpy as np
    for l in range(sim.levels):
        keys = sim.block_keys(l).cpu().numpy()
        for s in range(0, len(keys), 4096):
            k = keys[s:s + 4096]
            sim.set_block_moments(l, k, W.tgv3d_field(l, k, wl["n"], wl["amp"]).astype(np.float32))


def computed_nodes(sim):
    return [int((sim.roles(l) == 0).sum().item()) for l in range(sim.levels)]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W):
    """The oracle on the benchmark's own inputs: the 512^3 three-level slab hierarchy of
    2M particles with the Taylor-Green field, one coarse step (4 finest substeps, every
    transfer) plus the particle advance and the grid update, timed once after the
    hierarchy is built (building it is not timed); its node updates per second. The
    same single step on one core would take minutes, so the one-core figure is taken on
    the workload scaled to 128^3 (31,250 particles in the scaled slab)."""
    import numpy as np
    from oracle import oracle as O
    wl = W.workload("slab512")
    p = W.slab_particles(wl["particles"], wl["seed"], wl["lo"], wl["hi"])
    sim = O.OracleSim(3, wl["n"], wl["bc"], wl["tau0"], particles=p)
    for l in range(3):
        keys = sim.block_keys(l)
        for s in range(0, len(keys), 2048):
            k = keys[s:s + 2048]
            sim.set_block_moments(l, k, W.tgv3d_field(l, k, wl["n"], wl["amp"]))
    roles = [sim.roles(l) for l in range(3)]
    updates = sum((roles[l] == 0).sum() * (1 << (2 - l)) for l in range(3))
    d = np.array([v * 4 for v in wl["v_fine"]], dtype=np.float32)
    cores = O.num_threads()
    t0 = time.perf_counter()
    sim.step(1)
    O.advance_particles(p, d)
    sim.remesh(p)
    dt = time.perf_counter() - t0
    del sim
    # one core, on the slab scaled to 128^3
    n = (128, 128, 128)
    ps = W.slab_particles(2_000_000 // 64, 3, (16.0, 16.0, 88.0), (112.0, 112.0, 96.0))
    small = O.OracleSim(3, n, (W.PERIODIC,) * 6, 0.6, particles=ps)
    for l in range(3):
        keys = small.block_keys(l)
        small.set_block_moments(l, keys, W.tgv3d_field(l, keys, n, 0.05))
    r = [small.roles(l) for l in range(3)]
    small_updates = sum((r[l] == 0).sum() * (1 << (2 - l)) for l in range(3))
    O.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        small.step(1)
        O.advance_particles(ps, d)
        small.remesh(ps)
        dt1 = time.perf_counter() - t0
    finally:
        O.set_num_threads(cores)
    return {"value": round(float(updates) / dt / 1e6, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "single_core": round(float(small_updates) / dt1 / 1e6, 3),
            "sample": "FP64 oracle on the benchmark's inputs (512^3, 3 levels, 2M particles, Taylor-Green): one "
                      f"coarse step with particle advance and grid update, {int(updates)} node updates, "
                      f"{dt:.1f} s on {cores} threads; single_core: the same step on the slab scaled to 128^3 "
                      f"({int(small_updates)} node updates) on one thread"}


def remesh_change(sim, particles, torch, ms_per_step, reps=4):
    """Grid updates that change the block set: the particles move by one level-0 block
    (8 fine nodes) along x and back, so every update creates and deletes blocks on every
    level and initialises the new ones; each update timed alone (host wall clock around
    lbm_remesh, with the device synchronised before and after)."""
    times = []
    before = sim.block_keys(0).cpu()
    for k in range(reps):
        sim.advance_particles(particles, (8.0 if k % 2 == 0 else -8.0, 0.0, 0.0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.remesh(particles)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        keys = sim.block_keys(0).cpu()
        assert keys.shape != before.shape or not torch.equal(keys, before), "the block set did not change"
        before = keys
    ms = sum(times) / len(times) * 1e3
    return {"ms": round(ms, 4), "frac_of_step": round(ms / ms_per_step, 4), "updates": reps,
            "note": "particles moved by one level-0 block (8 fine nodes) along x and back; every update "
                    "changes the block set of every level"}


def adjoint_ratio(lbm, W, torch):
    """Two-level 128^3 adjoint case: time of the plain forward of its 200 coarse steps
    vs the backward pass of the checkpointed rollout (checkpoints every 20 steps; per
    segment one replay that keeps the undo log, then the reverse sweep); medians of
    three runs."""
    wl = W.workload("adjoint128")
    sim = lbm.Sim(2, wl["n"], wl["bc"], wl["tau0"], particles=wl["markers"])
    u0 = W.smooth_random_velocity(wl["n"], wl["seed"], wl["kmax"], wl["rms"])
    for l in range(2):
        keys = sim.block_keys(l).cpu().numpy()
        sim.set_block_moments(l, keys, W.velocity_moments(l, keys, u0).astype("float32"))
    x0 = sim.get_all_moments().clone()
    steps = wl["steps"]
    # warm-up: one short differentiated rollout (fills torch's allocator cache with the
    # checkpoint and work buffers of the timed run)
    x = x0.clone().requires_grad_(True)
    lbm.rollout(sim, x, wl["checkpoint_every"], checkpoint_every=wl["checkpoint_every"]).backward(
        sim.loss_ke_grad(0, *wl["box"]))
    # each figure is the median of three runs (single runs of these ~15-45 ms measurements
    # vary by a few percent)
    fwds, ckpts, bwds = [], [], []
    for _ in range(3):
        sim.set_all_moments(x0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        fwds.append(time.perf_counter() - t0)
        x = x0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xt = lbm.rollout(sim, x, steps, checkpoint_every=wl["checkpoint_every"])
        torch.cuda.synchronize()
        ckpts.append(time.perf_counter() - t0)
        seed = sim.loss_ke_grad(0, *wl["box"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xt.backward(seed)
        torch.cuda.synchronize()
        bwds.append(time.perf_counter() - t0)
    fwd, fwd_ckpt, bwd = (sorted(v)[1] for v in (fwds, ckpts, bwds))
    # the same gradient with the whole undo log of the forward pass kept in HBM (no replay)
    x = x0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xt = lbm.rollout(sim, x, steps, checkpoint_every=0)
    torch.cuda.synchronize()
    fwd_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    xt.backward(seed)
    torch.cuda.synchronize()
    bwd_tape = time.perf_counter() - t0
    return {"value": round(bwd / fwd, 3), "forward_s": round(fwd, 4), "backward_s": round(bwd, 4),
            "rollout_forward_s": round(fwd_ckpt, 4),
            "note": "checkpoints every 20 steps; the rollout's forward pass records the last segment's undo log, "
                    "so the backward pass replays the other segments only",
            "workload": "adjoint128: 128^3, 2 levels (512 + 504 blocks), 200 coarse steps, checkpoints every 20",
            "full_tape": {"value": round(bwd_tape / fwd, 3), "forward_recording_s": round(fwd_rec, 4),
                          "backward_s": round(bwd_tape, 4),
                          "note": "no checkpoints: the forward pass keeps its undo log in HBM"}}


def adjoint_slab(lbm, W, torch, steps=10, every=5):
    """Adjoint/forward time ratio on the benchmark's hierarchy held fixed (512^3, 3 levels,
    39,060 blocks, states far beyond the caches): `steps` coarse steps, checkpoints every
    `every`; and the transposed stream-collide's achieved bandwidth against its
    algorithmic bytes (160 B per node: state and mu read, the adjoint read and written;
    280 B when the launch also takes the next stream-collide's first pass: its tape read,
    the state restored, its mu written)."""
    wl = W.workload("slab512")
    p = torch.as_tensor(W.slab_particles(wl["particles"], wl["seed"], wl["lo"], wl["hi"])).cuda()
    sim = lbm.Sim(wl["levels"], wl["n"], wl["bc"], wl["tau0"], particles=p, max_blocks=48000)
    init_fields(sim, wl, W)
    nodes = computed_nodes(sim)
    box = ((0, 0, 0), (512, 512, 512))
    x0 = sim.get_all_moments().clone()
    x = x0.clone().requires_grad_(True)
    lbm.rollout(sim, x, every, checkpoint_every=every).backward(sim.loss_ke_grad(0, *box))  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    x = x0.clone().requires_grad_(True)
    xt = lbm.rollout(sim, x, steps, checkpoint_every=every)
    seed = sim.loss_ke_grad(0, *box)
    torch.cuda.synchronize()
    sim.profile()
    sim.set_profiling(True)
    t0 = time.perf_counter()
    xt.backward(seed)
    torch.cuda.synchronize()
    bwd = time.perf_counter() - t0
    sim.set_profiling(False)
    prof = sim.profile()
    # per coarse step the reverse sweep transposes 4 level-0, 2 level-1 and 1 level-2
    # stream-collides; two level-0 launches also take the next one's first pass
    ms_u, n_u = prof["adj_sc"]
    ms_f, n_f = prof["adj_sc_fused"]
    bytes_u = 160.0 * steps * (2 * nodes[0] + 2 * nodes[1] + nodes[2])
    bytes_f = 280.0 * steps * 2 * nodes[0]
    out = {"value": round(bwd / fwd, 3), "forward_ms_per_step": round(fwd / steps * 1e3, 4),
           "backward_ms_per_step": round(bwd / steps * 1e3, 4),
           "workload": f"slab512 hierarchy held fixed (no grid updates), {steps} coarse steps, checkpoints every "
                       f"{every}, loss = kinetic energy of level 0",
           "transpose": None}
    if n_u == steps * 5 and n_f == steps * 2:
        achieved = (bytes_u + bytes_f) / ((ms_u + ms_f) / 1e3) / 1e9
        out["transpose"] = {"kernel": "k_sc_transpose<StoreF32> (all levels)", "achieved": round(achieved, 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                            "launches": n_u + n_f,
                            "avg_launch_ms": round((ms_u + ms_f) / (n_u + n_f), 5),
                            "ms_per_step": round((ms_u + ms_f) / steps, 4),
                            "other_adjoint_ms_per_step": round(prof["adj"][0] / steps, 4)}
    del sim
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward time ratio")
    ap.add_argument("--no-fuse", action="store_true",
                    help="run the finest level's two substeps of a parent step as two sweeps (comparison)")
    ap.add_argument("--fuse", type=int, choices=[0, 1, 2], default=None,
                    help="the library's substep-fusion option (0 never, 1 with FP32 storage, 2 always)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="print only the adjoint/forward measurement (for profiling the adjoint kernels)")
    ap.add_argument("--storage", choices=["f32", "bf16", "f16"], default="f32",
                    help="moment storage format (FP32 arithmetic in every case)")
    ap.add_argument("--separate-calls", action="store_true",
                    help="step, particle advance and grid update as three calls (each update then waits for "
                         "the step before it)")
    ap.add_argument("--no-adjoint-slab", action="store_true",
                    help="skip the adjoint/forward ratio on the benchmark's (fixed) hierarchy")
    ap.add_argument("--breakdown-steps", type=int, default=10,
                    help="coarse steps after the timed ones with every phase timed (phase_ms_per_step)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the block hierarchy is not sharded across GPUs "
              "(see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2603_14982_amd import lbm, workloads as W

    if args.adjoint_only:
        print(json.dumps({"adjoint_forward_ratio": adjoint_ratio(lbm, W, torch)}), flush=True)
        return
    wl = W.workload("slab512")
    print(f"[bench] workload slab512 n={wl['n']} levels={wl['levels']} particles={wl['particles']}",
          file=sys.stderr, flush=True)
    p_host = W.slab_particles(wl["particles"], wl["seed"], wl["lo"], wl["hi"])
    particles = torch.as_tensor(p_host).cuda()
    half = args.storage != "f32"
    sim = lbm.Sim(wl["levels"], wl["n"], wl["bc"], wl["tau0"], particles=particles, max_blocks=48000,
                  storage=args.storage, scale=HALF_SCALES if half else None)
    if args.no_fuse:
        sim.set_option("fuse_substeps", 0)
    elif args.fuse is not None:
        sim.set_option("fuse_substeps", args.fuse)
    init_fields(sim, wl, W)
    torch.cuda.synchronize()
    sub = 1 << (wl["levels"] - 1)
    d = (wl["v_fine"][0] * sub, wl["v_fine"][1] * sub, wl["v_fine"][2] * sub)

    def coarse_step():
        if args.separate_calls:
            sim.step(1)
            sim.advance_particles(particles, d)
            sim.remesh(particles)
        else:
            # the same three operations, the particle work overlapping the step
            sim.step_remesh(1, particles, d)

    for _ in range(args.warmup):
        coarse_step()
    torch.cuda.synchronize()
    nodes_before = computed_nodes(sim)
    blocks_before = [sim.num_blocks(l) for l in range(sim.levels)]
    print(f"[bench] warm-up done; blocks {blocks_before}, computed nodes {nodes_before}", file=sys.stderr, flush=True)

    # the timed region brackets only the finest level's stream-collide launches with
    # events (each timed launch costs two event records between dependent launches);
    # every phase is timed over a few further steps afterwards
    sim.profile()
    sim.set_profiling(True, phases=["sc_pair", "sc0"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        coarse_step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sim.set_profiling(False)
    prof = sim.profile()
    sim.set_profiling(True)
    for i in range(args.breakdown_steps):
        coarse_step()
    sim.set_profiling(False)
    prof_all = sim.profile()
    nodes_after = computed_nodes(sim)
    blocks_after = [sim.num_blocks(l) for l in range(sim.levels)]
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s; blocks {blocks_after}", file=sys.stderr, flush=True)
    assert sim.check_finite(), "non-finite moments"

    per_level = [(a + b) / 2.0 for a, b in zip(nodes_before, nodes_after)]
    updates = sum(per_level[l] * (1 << (sim.levels - 1 - l)) for l in range(sim.levels))
    fine_equiv = float(np.prod(wl["n"])) * sub
    ms_per_step = elapsed / args.steps * 1e3
    mlups = updates * args.steps / elapsed / 1e6

    # the dominant kernel: level 0's stream-collide on 2 x 2 x 2 block tiles, either both
    # substeps of a parent step in one launch (two updates of every node, 2 launches per
    # coarse step) or one substep per launch (4 launches per coarse step)
    if prof["sc_pair"][1]:
        sc_ms, sc_n = prof["sc_pair"]
        launch_updates = 2 * per_level[0]
        kernel = f"k_stream_collide_pair<{STORE_NAME[args.storage]}> (level 0, two substeps per launch)"
    else:
        sc_ms, sc_n = prof["sc0"]
        launch_updates = per_level[0]
        kernel = f"k_stream_collide_tile<{STORE_NAME[args.storage]}> (level 0)"
    sc_avg_s = sc_ms / sc_n / 1e3
    alg_bytes = BYTES_PER_UPDATE[args.storage] * launch_updates
    achieved = alg_bytes / sc_avg_s / 1e9
    traffic = None
    valu = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_src_sha") == sc_source_hash() and tr.get("kernel") == kernel:
            traffic = tr.get("hbm_bytes_per_launch")
            insts = tr.get("valu_wave_instructions_per_launch")
            if insts:
                # issue rate: one wave64 FP32 instruction per cycle per CU (4 SIMDs of 16 lanes)
                valu = {"wave_instructions_per_launch": insts,
                        "lane_instructions_per_update": round(insts * 64 / launch_updates, 1),
                        "issue_frac": round(insts / (VALU_CUS * VALU_CLOCK_HZ * sc_avg_s), 4)}
    # all stream-collide launches of all levels, over the breakdown steps
    all_ms = sum(prof_all[f"sc{l}"][0] for l in range(sim.levels)) + prof_all["sc_pair"][0]
    all_n = sum(prof_all[f"sc{l}"][1] for l in range(sim.levels)) + prof_all["sc_pair"][1]
    sc_updates = sum(per_level[l] * (1 << (sim.levels - 1 - l)) for l in range(sim.levels)) * args.breakdown_steps
    all_bytes = BYTES_PER_UPDATE[args.storage] * sc_updates / all_n
    all_avg_s = all_ms / all_n / 1e3
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "slab512: 512^3 fine-equivalent periodic, 3 levels of 8^3 blocks, 2M seeded particles "
                        "falling at 0.02/finest step drive the grid update every coarse step, 3D Taylor-Green "
                        f"U=0.05, tau0=0.6, {args.storage} moments",
            "storage": args.storage,
            "levels": sim.levels,
            "fine_extent": list(wl["n"]),
            "blocks_per_level": blocks_after,
            "computed_nodes_per_level": [int(v) for v in per_level],
            "node_updates_per_step": int(updates),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "hbm_achieved": round(traffic / sc_avg_s / 1e9, 1) if traffic else None,
            "hbm_frac": round(traffic / sc_avg_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
            "valu": valu,
            "kernel": kernel,
            "algorithmic_bytes_per_launch": int(alg_bytes),
            "avg_launch_ms": round(sc_avg_s * 1e3, 5),
            "launches": sc_n,
            "all_levels": {"achieved": round(all_bytes / all_avg_s / 1e9, 1), "avg_launch_ms": round(all_avg_s * 1e3, 5),
                           "launches": all_n, "algorithmic_bytes_per_launch": int(all_bytes)},
        },
        "effective_mlups": round(fine_equiv * args.steps / elapsed / 1e6, 1),
        "stream_collide_mlups": round(sc_updates / (all_ms / 1e3) / 1e6, 1),
        "adjoint_forward_ratio": None,  # filled below
        "phase_ms_per_step": {k: round(v[0] / args.breakdown_steps, 4) for k, v in prof_all.items() if v[1]},
    }
    out["remesh_block_change"] = remesh_change(sim, particles, torch, ms_per_step)
    if args.calibrate_copy_mib > 0:
        # one elementwise kernel that reads and writes the buffer once (torch's neg)
        src = torch.ones(args.calibrate_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = args.calibrate_copy_mib << 20
    if not args.no_adjoint:
        print("[bench] adjoint/forward ratio (adjoint128)", file=sys.stderr, flush=True)
        out["adjoint_forward_ratio"] = adjoint_ratio(lbm, W, torch)
    if not args.no_adjoint and not args.no_adjoint_slab:
        del sim
        torch.cuda.empty_cache()
        print("[bench] adjoint/forward ratio (slab512 hierarchy, fixed)", file=sys.stderr, flush=True)
        out["adjoint_forward_ratio"]["slab512"] = adjoint_slab(lbm, W, torch)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
