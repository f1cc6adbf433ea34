/*
 * lbm.h - C ABI of the block-adaptive, moment-encoded D3Q27 lattice Boltzmann
 * step for MI355X (gfx950), after arXiv 2603.14982 ("Adaptive GPU Kinetic
 * Solver for Fluid-Granular Flows").
 *
 * The problem (Sec. 5.1-5.4 of the paper): a domain split into levels with
 * spacing dx_l = 2^l dx_0 (level 0 finest), finest relaxation time tau_0 which
 * fixes tau_l = tau_0/2^l + (2^l-1)/2^(l+1) (Sec. 5.2), a level-selection
 * function Phi driven by particles or geometry (Sec. 5.4), initial moments
 * {rho, u, S} per node (Sec. 3.1, Eq. rho_u_stress); the outputs are the
 * moments per level after stepping.
 *
 * Conventions
 *  - Every function returns an lbm_status; nothing throws across the ABI.
 *  - All pointers marked "device" are HIP device pointers owned by the caller;
 *    the context borrows them and never frees them. Host pointers are read
 *    (or written) only during the call.
 *  - Calls run asynchronously on cfg.stream unless marked "synchronises".
 *  - Block keys are Morton codes of block coordinates (bx, by, bz), x in the
 *    lowest bit of each 3-bit group; a level-l block covers level-l nodes
 *    8*b .. 8*b+7 per axis, i.e. fine positions 2^l * (8*b + k).
 *  - Moment arrays use [block][moment][node], node = x + 8y + 64z, moment order
 *    (rho - 1, ux, uy, uz, Sxx, Syy, Szz, Sxy, Sxz, Syz), f32.
 *  - Per-level block lists are in increasing key order.
 *  - Arguments are validated on the host before any launch; on error the
 *    context is unchanged and lbm_last_error() says why.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument or configuration */
  LBM_ENOMEM = -2,     /* caller buffers smaller than lbm_pool_bytes / lbm_meta_bytes */
  LBM_ECAPACITY = -3,  /* the block pool cannot hold the requested hierarchy */
  LBM_EDEVICE = -4,    /* a HIP call failed */
  LBM_ENAN = -5,       /* non-finite moments found */
  LBM_ESTATE = -6      /* call not valid in the current state */
} lbm_status;

typedef enum { LBM_F32 = 0, LBM_BF16 = 1, LBM_F16 = 2 } lbm_storage;

/* Per-face boundary kind. INFLOW holds nodes on the face at the equilibrium
 * moments (1, u, u u) of the inflow velocity u (inflow_u, times the log profile
 * below if selected); OUTFLOW copies the inward neighbour after each step (zero
 * gradient); OUTFLOW_CONV is the convective outflow condition of Sec. 7 (dune
 * migration): after each step every moment M of a face node takes one implicit
 * upwind step of dM/dt + u_n dM/dn = 0, M <- (M + lam M_in) / (1 + lam), with M_in
 * the new moments of the inward neighbour and lam = max(u_n, 0) its outward
 * velocity; WALL is halfway bounce-back half a node outside the face. Faces of one
 * axis are either both PERIODIC or neither. */
typedef enum { LBM_PERIODIC = 0, LBM_INFLOW = 1, LBM_OUTFLOW = 2, LBM_WALL = 3, LBM_OUTFLOW_CONV = 4 } lbm_bc;

/* Inflow velocity profile (Sec. 7, sand ripples): UNIFORM holds inflow_u on every
 * inflow node; LOG holds inflow_u * ln(1 + inflow_beta (h - inflow_h0)) at height h
 * (the node's coordinate along inflow_axis, in fine-level node units), zero where
 * h <= inflow_h0. */
typedef enum { LBM_INFLOW_UNIFORM = 0, LBM_INFLOW_LOG = 1 } lbm_inflow_profile;

typedef struct {
  int32_t levels;          /* L in 1..5; level 0 is the finest */
  int32_t fine_extent[3];  /* fine-equivalent nodes per axis; each a multiple of 8*2^(L-1) */
  int32_t bc[6];           /* lbm_bc for faces x-, x+, y-, y+, z-, z+ */
  float inflow_u[3];       /* velocity held on INFLOW faces */
  double tau0;             /* finest-level relaxation time, > 1/2 */
  int32_t storage;         /* lbm_storage of the stored moments */
  int32_t rescale;         /* 0: Chapman-Enskog S^neq factors (default); 1: factors as printed in Sec. 5.2-5.3 */
  float scale[10];         /* per-moment power-of-two storage scales for BF16/F16 (ignored for F32) */
  int64_t max_blocks;      /* block-pool capacity over all levels */
  void* pool;              /* device, >= lbm_pool_bytes(cfg): moment storage, two time levels */
  void* meta;              /* device, >= lbm_meta_bytes(cfg): hierarchy tables and scratch */
  void* stream;            /* hipStream_t the context launches on (NULL = default stream) */
  int32_t inflow_profile;  /* lbm_inflow_profile */
  int32_t inflow_axis;     /* LOG: axis of the height (0, 1, 2) */
  float inflow_beta;       /* LOG: shear coefficient, >= 0, per fine node */
  float inflow_h0;         /* LOG: height of the profile's zero, fine nodes */
  int32_t coupling;        /* 1: the finest level carries coupling fields (lbm_set_coupling); 0: none */
  int32_t scalar;          /* 1: the finest level carries the powder-snow volume fraction (lbm_scalar_*) */
} lbm_config;

typedef struct lbm_ctx lbm_ctx;

/* Sizes of the caller-owned device buffers for a configuration (0 if invalid). */
size_t lbm_pool_bytes(const lbm_config* cfg);
size_t lbm_meta_bytes(const lbm_config* cfg);

/* Builds the hierarchy H(Phi) (Sec. 5.4 Phi, Sec. 6.3): level-0 blocks hold every
 * particle and every solid node; coarser levels follow with one block of overlap.
 * solid_fine: device uint8 [Z][Y][X] over the fine extent (nonzero = solid), or
 *   NULL; it must stay valid for the life of the context.
 * particles: device float [n][3] in fine units, or NULL with n = 0.
 * All nodes start at rest (rho = 1, u = 0, S = 0), INFLOW nodes at their state.
 * Synchronises. */
lbm_status lbm_create(const lbm_config* cfg, const uint8_t* solid_fine, const float* particles,
                      int64_t n, lbm_ctx** out);
lbm_status lbm_destroy(lbm_ctx* ctx);

/* Number of active blocks on a level. Host-side, no synchronisation. */
lbm_status lbm_num_blocks(lbm_ctx* ctx, int32_t level, int64_t* out);

/* Keys of the active blocks of a level into keys_out (device int64 [nb]). */
lbm_status lbm_block_keys(lbm_ctx* ctx, int32_t level, int64_t* keys_out);

/* Writes moments (layout above, device f32 [nb][10][512]) into both time levels of
 * the listed blocks (keys: device int64 [nb], each an active block of the level;
 * LBM_EINVAL otherwise). SOLID nodes keep the rest state and INFLOW nodes their
 * face state. Synchronises (to report unknown keys). */
lbm_status lbm_set_block_moments(lbm_ctx* ctx, int32_t level, const int64_t* keys, const float* in,
                                 int64_t nb);

/* Advances n coarse steps: each is one call of AdvanceLBM(L-1, 1) of Alg. 1
 * (Sec. 5.3): stream-collide per level with two fine substeps per coarser step,
 * downward transfer (Eq. downward_rescale, with temporal interpolation) before
 * each fine stream-collide, upward transfer (Eq. upload_S) after the second. */
lbm_status lbm_step(lbm_ctx* ctx, int32_t n);

/* Advances n finest-level steps: Alg. 1 with a stop after every finest-level
 * stream-collide, the exchange point of the coupling loop (Sec. 5.4 and Fig. pipeline:
 * fluid step, granular step, exchange; Sec. 7 runs one granular step per finest LBM
 * step). A coarse step is 2^(L-1) finest steps. After each one the finest level's
 * stored moments (the state before collision, where an external solver reads u and
 * supplies the next F through lbm_set_coupling) are one finest step on; coarser levels
 * are where Alg. 1 has taken them (ahead of the finest level inside a coarse step).
 * The finest level runs one stream-collide per substep (never the two-substep sweep),
 * so a whole coarse step taken this way computes what lbm_step computes. While a
 * coarse step is under way (lbm_finest_phase != 0), lbm_step, lbm_remesh,
 * lbm_set_block_moments, lbm_save, lbm_load and the adjoint calls return LBM_ESTATE.
 * Async.
 * lbm_finest_phase: finest steps taken since the last coarse-step boundary (0 at a
 * boundary). Host-side. */
lbm_status lbm_step_finest(lbm_ctx* ctx, int32_t n);
lbm_status lbm_finest_phase(lbm_ctx* ctx, int32_t* out);

/* Coupling fields of the finest level, the hook for an external granular solver
 * (Sec. 4): per node the fluid fraction eps, which scales the relaxation time to
 * eps tau0, and a force density F (lattice units, the external part of the paper's
 * force, e.g. drag and gravity over the conversion factor). The collision of a node
 * then uses rate 1 / (eps tau0) and Guo's force terms in moment form (S gains
 * (1 - om/2)(u F + F u)/rho, the carried velocity is u + F/(2 rho)), and its stored
 * velocity after streaming is (sum c f + F/2) / rho (Eq. rho_u_stress). The stored
 * moments between steps are the state before collision, where the external solver
 * reads the velocity and supplies the next F.
 * keys: device int64 [nb], keys of active finest-level blocks (lbm_block_keys);
 * fields: device f32 [nb][4][512] = (eps, Fx, Fy, Fz) per node (may be called between
 * the finest steps of lbm_step_finest). Blocks keep their
 * fields until set again; blocks created by a grid update start at eps = 1, F = 0;
 * solid nodes keep eps = 1, F = 0. Requires cfg.coupling = 1 (LBM_EINVAL otherwise).
 * LBM_EINVAL, with no field changed, if a key is not an active finest-level block or
 * a value is not finite or has eps tau0 <= 1/2. Synchronises. With coupling fields
 * the finest level always runs one stream-collide per substep, and the adjoint entry
 * points return LBM_EINVAL. */
lbm_status lbm_set_coupling(lbm_ctx* ctx, const int64_t* keys, const float* fields, int64_t nb);

/* Powder-snow volume fraction phi on the finest level (Sec. 7, powder snow), with
 * cfg.scalar = 1 (LBM_EINVAL otherwise): dphi/dt + u . grad phi = q + D lap phi.
 * lbm_scalar_advance takes one step of dt finest-level time steps: semi-Lagrangian
 * advection through the finest level's current velocity (departure point by Ralston's
 * third-order Runge-Kutta, trilinear interpolation of u and phi), then one forward-
 * Euler step of the 7-point Laplacian, then dt q. phi lives on the finest level's
 * owned nodes: nodes outside its blocks, its ghost nodes, nodes beyond walls and
 * solid nodes count as phi = 0, u = 0 (and stay at phi = 0). Every sample point of
 * the backtrace is kept within 7 nodes of its node per axis: with dt <= 7 this only
 * acts where a velocity component exceeds one node per step, beyond the lattice's
 * range (a run with |u| that large has lost accuracy anyway).
 * source: device f32 [nb][512] in the key order of the finest level's blocks (as
 * lbm_scalar_get returns them), or NULL. LBM_EINVAL unless 0 < dt <= 7, D >= 0 and
 * D dt <= 1/6. Async.
 * lbm_scalar_set: phi of the listed finest-level blocks (device keys [nb], values
 * [nb][512]); solid and ghost nodes are set to 0. LBM_EINVAL for a key that is not an active
 * finest-level block (blocks listed before it may have been written). Synchronises.
 * lbm_scalar_get: keys and phi of every finest-level block, key order (keys_out
 * [nb], phi_out [nb][512], nb = lbm_num_blocks(ctx, 0)). Async.
 * Blocks keep phi through grid updates; blocks created by one start at 0; phi of a
 * block that leaves the finest level is dropped. */
lbm_status lbm_scalar_set(lbm_ctx* ctx, const int64_t* keys, const float* phi, int64_t nb);
lbm_status lbm_scalar_get(lbm_ctx* ctx, int64_t* keys_out, float* phi_out);
lbm_status lbm_scalar_advance(lbm_ctx* ctx, float dt, float D, const float* source);

/* Moves particles by d (fine units) in f32: p[i] = p[i] + d, as a prescribed
 * stand-in for the granular solver. particles: device float [n][3]. */
lbm_status lbm_advance_particles(lbm_ctx* ctx, float* particles, int64_t n, const float d[3]);

/* Grid update (Sec. 6.3) at a coarse-step boundary: rebuilds H(Phi) for the given
 * particles; new nodes take the value of the old hierarchy (own level, else the
 * finest coincident node transferred upward, else interpolated downward).
 * Transactional: on LBM_ECAPACITY the context is unchanged. Synchronises once
 * (block counts), twice when the block set changes. */
lbm_status lbm_remesh(lbm_ctx* ctx, const float* particles, int64_t n);

/* n coarse steps of a run whose grid follows prescribed particle motion, each one
 * lbm_step(1), lbm_advance_particles(particles, d) and lbm_remesh(particles) in that
 * order, with the same results. The particle advance and the check whether the
 * level-0 target set changed (the grid update's first stage, Sec. 6.3) run on a
 * second stream of the context, concurrently with the step, after everything issued
 * on cfg.stream before the call; the host waits for that check only, not for the
 * step, and runs the rest of the grid update on cfg.stream when the targets changed.
 * particles: device float [np][3]; d: host float[3]. Synchronises with the check
 * (once per step) and as lbm_remesh when the block set changes. Inside a recording
 * (lbm_record_begin) the three calls run in order on cfg.stream. */
lbm_status lbm_step_remesh(lbm_ctx* ctx, int32_t n, float* particles, int64_t np, const float d[3]);

/* Current moments of a level (decoded to f32): keys_out device int64 [nb] (may be
 * NULL), out device f32 [nb][10][512], blocks in key order. */
lbm_status lbm_get_moments(lbm_ctx* ctx, int32_t level, int64_t* keys_out, float* out);

/* Node roles of a level, device uint8 [nb][512]: 0 computed, 1 ghost (filled by
 * the downward transfer), 2 upward-interface node, 3 solid, 4 inflow, 5 outflow. */
lbm_status lbm_get_roles(lbm_ctx* ctx, int32_t level, uint8_t* out);

/* FP64 sums over the owned (non-ghost, non-solid) nodes of one level whose fine
 * position lies in [lo, hi): out = {sum rho, sum rho ux, sum rho uy, sum rho uz,
 * 1/2 sum rho |u|^2} (host double[5]). Synchronises. */
lbm_status lbm_reduce_f64(lbm_ctx* ctx, int32_t level, const int32_t lo[3], const int32_t hi[3],
                          double out[5]);

/* The sums of lbm_reduce_f64 for callers that cannot allocate device memory or
 * wait on the stream (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): out is device double[5], written on cfg.stream without
 * synchronising. The per-block partials live in a static device array of the
 * library instead of the meta buffer: one per GPU, 2^18 blocks x 5 doubles
 * (10 MiB), held until the process ends. LBM_EINVAL if the level has more than
 * 2^18 blocks. Every call on a GPU shares that array: calls that overlap in time on
 * one GPU (other streams, other contexts) race; calls on one stream are ordered.
 * Allocates nothing. */
lbm_status lbm_reduce_f64_noalloc(lbm_ctx* ctx, int32_t level, const int32_t lo[3], const int32_t hi[3],
                                  double* out);

/* LBM_ENAN if any stored moment of an active block is not finite. Synchronises. */
lbm_status lbm_check_finite(lbm_ctx* ctx);

/* Phase timers. With profiling on, every launch of the listed phases is bracketed
 * by HIP events on cfg.stream; lbm_get_profile synchronises, returns the summed
 * milliseconds and launch counts per phase since the last call, and resets them.
 * Phases: stream-collide of levels 0..4 (one substep per launch), downward
 * transfers, upward transfers, outflow copies, whole grid updates (lbm_remesh, host
 * time between its events included), the finest level's two substeps of a
 * parent step in one launch (see LBM_OPT_FUSE_SUBSTEPS), and in the adjoint's reverse
 * sweep: the transposed stream-collide (k_sc_transpose), the same launch when it also
 * takes the first pass of the next stream-collide in the sweep, and every other
 * adjoint launch (first passes, transfers, outflow). */
enum {
  LBM_PROF_SC0 = 0,            /* + level */
  LBM_PROF_DOWN = 5,
  LBM_PROF_UP = 6,
  LBM_PROF_OUTFLOW = 7,
  LBM_PROF_REMESH = 8,
  LBM_PROF_SC_PAIR = 9,
  LBM_PROF_ADJ_SC = 10,
  LBM_PROF_ADJ_SC_FUSED = 11,
  LBM_PROF_ADJ = 12,
  LBM_PROFILE_PHASES = 13
};
lbm_status lbm_set_profiling(lbm_ctx* ctx, int32_t on);
/* Phase timers for a subset of the phases: bit p of mask times phase p; 0 turns
 * profiling off, and lbm_set_profiling(ctx, 1) is the mask of all phases. Every timed
 * launch costs two event records on the stream (a few microseconds each between
 * dependent launches), so timing only the phase of interest keeps that cost off the
 * others. LBM_EINVAL for a bit at or above LBM_PROFILE_PHASES. */
lbm_status lbm_set_profiling_phases(lbm_ctx* ctx, uint32_t mask);
lbm_status lbm_get_profile(lbm_ctx* ctx, double ms[LBM_PROFILE_PHASES], int64_t count[LBM_PROFILE_PHASES]);

/* Execution options (they change how a step is scheduled on the GPU, not what it
 * computes; results agree to rounding).
 * LBM_OPT_TILE_MIN_BLOCKS: a level with at least this many blocks (counted as
 *   8 per 2 x 2 x 2 tile) runs its stream-collide on tiles of 2 x 2 x 2 blocks,
 *   smaller levels one block per 64-lane workgroup. Default 16384; >= 0.
 * LBM_OPT_FUSE_SUBSTEPS: 2 runs the two substeps of every parent step of the
 *   finest level (Alg. 1, levels >= 2) in one tiled sweep when that level is
 *   tiled and has no outflow or bounce-back nodes, and the step is not being
 *   recorded for the adjoint (default: one sweep is faster with every storage
 *   format); 1 does so with LBM_F32 storage only; 0 always runs them as two sweeps.
 * LBM_OPT_GRAPHS: 1 replays each coarse step of lbm_step and lbm_step_remesh as a
 *   HIP graph, captured once per launch state (buffer parities, hierarchy, options)
 *   on a stream of the context's own and launched on cfg.stream; not while
 *   profiling or recording. 0 (default) launches every kernel itself: the replay
 *   was no faster (the steps are bound by the kernels and the gaps between them on
 *   the device, not by host launches).
 * LBM_OPT_PAIR_RUN: 1 .. 6 (default 4 with LBM_F32 storage, 2 with 16-bit storage,
 *   each the fastest measured on the three-level slab): the one-sweep form of the finest level's
 *   two substeps gives each workgroup a run of up to this many 2 x 2 x 2-block
 *   tiles stacked along z (runs break below a missing tile and at tile positions
 *   z = 0 mod the value), longest runs launched first; the planes at the shared
 *   faces of a run's tiles are read and recomputed once. The results do not depend
 *   on it (bit for bit). LBM_ESTATE inside a recording.
 * LBM_EINVAL for an unknown option or a value out of range. */
enum { LBM_OPT_TILE_MIN_BLOCKS = 0, LBM_OPT_FUSE_SUBSTEPS = 1, LBM_OPT_GRAPHS = 2, LBM_OPT_PAIR_RUN = 3 };
lbm_status lbm_set_option(lbm_ctx* ctx, int32_t option, int64_t value);

/* ---- states and the adjoint (gradient of a loss of the final moments with
 * respect to the initial moments; Sec. 7 differentiates the solver) ----
 *
 * A state is the current time level of every block of every level, in level
 * order and key order, behind a 256-byte header that names the block hierarchy
 * it belongs to (the coupling fields and the powder-snow field are not part of
 * it). The hierarchy must not change between saving and loading.
 *
 * lbm_state_bytes: size of a state under the current hierarchy (0 for NULL).
 * lbm_save: writes the state to dst (device, >= lbm_state_bytes bytes); async.
 * lbm_load: makes a saved state current. Synchronises (reads the header).
 *   LBM_ESTATE if src holds no state of this context or was saved under another
 *   hierarchy (a grid update that changed blocks happened since). */
size_t lbm_state_bytes(const lbm_ctx* ctx);
lbm_status lbm_save(lbm_ctx* ctx, void* dst, size_t bytes);
lbm_status lbm_load(lbm_ctx* ctx, const void* src, size_t bytes);

/* One reverse-mode step (Sec. 7: the gradient is the transposed Jacobian of the
 * update applied to the adjoint, coarse step by coarse step, backwards).
 *   state      device, a state saved at the start of the coarse step (lbm_save);
 *   lam_next   device f32 [sum over levels of nb_l][10][512], levels in order and
 *              blocks in key order (the layout of lbm_get_moments, concatenated):
 *              dLoss/d(moments after the step). Only nodes that carry state
 *              (computed, upward-interface and outflow nodes) are read; ghost,
 *              solid and inflow entries are ignored.
 *   lam_out    device f32, same layout: dLoss/d(moments of `state`), i.e. with
 *              respect to the values lbm_set_block_moments would write (zero at
 *              ghost, solid and inflow nodes, which do not influence the step).
 *              May alias lam_next.
 *   work       device scratch of >= lbm_adjoint_work_bytes(ctx, 1) bytes (caller-owned):
 *              the adjoint of both time levels, two buffers of the adjoint of
 *              the per-node moment sums, one flag byte per block slot, and the
 *              undo log of the replayed step.
 * The call loads `state` (synchronises once), replays the coarse step while the
 * forward kernels keep the old value of every node they overwrite (the undo log),
 * then walks the log backwards: adjoint of each operation, whose kernels also put
 * back what the operation overwrote. On return the simulation is at `state`; after
 * a failed call its state is undefined (load a saved state).
 * The adjoint is that of the f32 arithmetic; with 16-bit storage the rounding
 * of stored values is passed through unchanged. Grid updates are not part of
 * the step and are not differentiated. */
size_t lbm_adjoint_work_bytes(const lbm_ctx* ctx, int32_t n_steps);
lbm_status lbm_adjoint_step(lbm_ctx* ctx, const void* state, size_t state_bytes, const float* lam_next,
                            float* lam_out, void* work, size_t work_bytes);

/* The same over n_steps coarse steps at once (a checkpoint segment): one load, one
 * replay of the n steps with the undo log, one reverse sweep. lam_next is the
 * adjoint of the state n_steps after `state`; work >= lbm_adjoint_work_bytes(ctx,
 * n_steps) (the undo log grows linearly with n_steps). lbm_adjoint_step is this
 * call with n_steps = 1. */
lbm_status lbm_adjoint_steps(lbm_ctx* ctx, const void* state, size_t state_bytes, int32_t n_steps,
                             const float* lam_next, float* lam_out, void* work, size_t work_bytes);

/* The two halves of lbm_adjoint_steps, for callers that keep the whole undo log of
 * a forward pass resident instead of recomputing it from checkpoints (one coarse
 * step of the two-level 128^3 case logs ~45 MB; 200 steps fit easily in HBM):
 * lbm_step_record runs n_steps coarse steps from the current state, logging into
 * work (>= lbm_adjoint_work_bytes(ctx, n_steps)); lbm_adjoint_reverse then turns the
 * adjoint of the final state (lam_next) into that of the state before the recorded
 * steps (lam_out) and puts the simulation back at that state. The reverse call takes
 * the same work buffer; LBM_ESTATE if nothing is recorded in it (lbm_step,
 * lbm_remesh, lbm_load and lbm_set_block_moments in between drop the recording).
 * lbm_adjoint_reverse also takes the recordings of lbm_record_begin / lbm_record_end
 * (below), grid updates included. */
lbm_status lbm_step_record(lbm_ctx* ctx, int32_t n_steps, void* work, size_t work_bytes);
lbm_status lbm_adjoint_reverse(lbm_ctx* ctx, const float* lam_next, float* lam_out, void* work, size_t work_bytes);

/* A recording that may include grid updates (Sec. 6.3), for the adjoint of adaptive
 * runs: between lbm_record_begin and lbm_record_end, lbm_step runs its coarse steps
 * with the undo log (one stream-collide per finest substep) and lbm_remesh logs every
 * grid update that changes the block set: the meta buffer and both time levels of
 * every block before it. lbm_adjoint_reverse then walks the whole log back: the
 * adjoint of a grid update sends the adjoint of every node the update wrote through
 * the transposed new-node sampler (own value, upward from the nearest finer level
 * with S^neq times a_up, trilinear downward with a_down) into the nodes of the old
 * hierarchy it was sampled from, and restores the old hierarchy. lam_next is then in
 * the layout of the hierarchy at lbm_record_end, lam_out in that of the hierarchy at
 * lbm_record_begin (its block count), and the simulation returns to the state and
 * hierarchy at lbm_record_begin.
 * While a recording is open, lbm_set_block_moments, lbm_load, lbm_step_finest,
 * lbm_step_record and lbm_adjoint_reverse return LBM_ESTATE; LBM_ECAPACITY when the log
 * is full (the step or update that did not fit is not applied, the recording stays
 * open; close it and start again with a larger buffer).
 * lbm_record_work_bytes: a work size for n_steps coarse steps and n_updates grid
 * updates on hierarchies the size of the current one (the adjoint buffers sized for
 * the pool capacity, so that any hierarchy fits them). Synchronises: no. */
size_t lbm_record_work_bytes(const lbm_ctx* ctx, int32_t n_steps, int32_t n_updates);
lbm_status lbm_record_begin(lbm_ctx* ctx, void* work, size_t work_bytes);
lbm_status lbm_record_end(lbm_ctx* ctx);

/* Adjoint seed of the kinetic energy 1/2 sum rho |u|^2 over the owned nodes of
 * `level` whose fine position lies in [lo, hi): writes lam (device f32, the
 * all-level layout of lbm_adjoint_step) with d(loss)/d(moments) of the current
 * state, zero outside the level's owned state nodes in the box. */
lbm_status lbm_loss_ke_grad(lbm_ctx* ctx, int32_t level, const int32_t lo[3], const int32_t hi[3], float* lam);

/* Message of the last failed call on this context (or of lbm_create, for NULL). */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
