// Host-side launchers of the HIP kernels (one translation unit per kernel family).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace lbmx {

// ---- stream-collide (one level, one step) ----
struct ScLaunch {
  const void* in;            // pool time level read (storage type)
  void* out;                 // pool time level written
  const int32_t* blocks;     // slots of the level, key order
  int32_t nblocks;
  const int32_t* nbr;        // [slot][27]
  const uint8_t* role;       // [slot][512]
  int32_t zero_slot;         // all-zero block read in place of missing neighbours
  float omega;
  Scales sc;
  int storage;
  // 2 x 2 x 2 tiles: first block of every tile (slots), the level's geometry and directory
  const int32_t* tiles;
  int32_t ntiles;
  const int32_t* dir;
  const int4* coord;
  LevelGeom lg;
  int periodic[3];
  const float* cpl;          // finest level with coupling fields: [slot][4][512] (eps, F); else null
  // two-substep sweep: runs of k + 1 tiles stacked along z, class k at runs + k * run_stride
  // (first tile's first block, key order), nrun[k] of them
  const int32_t* runs;
  int64_t run_stride;
  int32_t nrun[kRunMax];
};
hipError_t launch_stream_collide(const ScLaunch& a, hipStream_t s);
// both substeps of a parent step of the finest level, in -> out (tiles required; the
// level has no outflow or bounce-back nodes, and out holds the ghosts of the second)
hipError_t launch_stream_collide_pair(const ScLaunch& a, hipStream_t s);

// ---- interface transfers and outflow ----
struct TransferLaunch {
  Geom G;
  int level;                 // fine level l (down: l+1 -> l, up: l -> l+1)
  const int32_t* blocks;     // blocks holding target nodes (level l for down, l+1 for up)
  int32_t nblocks;
  const int32_t* dir;        // all-level cell -> slot
  const uint8_t* role;       // [slot][512]
  const int4* coord;         // [slot] block coordinates and level
  const void* src_a;         // source time level (down: coarse t; up: fine current)
  const void* src_b;         // down only: coarse t+2
  void* dst;                 // target time level (down: the first fine substep's ghosts)
  void* dst2;                // down only: the second fine substep's ghosts (midpoint of src_a and src_b)
  float factor;              // S^neq rescaling factor
  Scales sc;
  int storage;
  void* tape;                // adjoint replay: old values of the nodes written in dst, [list index][10][512]
  void* tape2;               // down, adjoint replay: the same for dst2
  const int32_t* gbox;       // down: per slot bounding box of the ghost nodes (from the grid update)
};
hipError_t launch_downward(const TransferLaunch& a, hipStream_t s);
hipError_t launch_upward(const TransferLaunch& a, hipStream_t s);
// outflow copy on the level's outflow blocks: dst = src_new (computed inward
// neighbour) or the node's own old value
struct OutflowLaunch {
  Geom G;
  int level;
  const int32_t* blocks;
  int32_t nblocks;
  const uint8_t* role;
  const int4* coord;
  const void* old_buf;
  void* new_buf;
  Scales sc;
  int storage;
  void* tape = nullptr;      // adjoint replay: old values of the written nodes, [list index][10][512]
};
hipError_t launch_outflow(const OutflowLaunch& a, hipStream_t s);

// ---- hierarchy (grid update) ----
struct HierLaunch {
  Geom G;
  uint8_t* t0;               // level-0 target cells
  const uint8_t* t0_static;  // level-0 cells holding solid nodes
  uint8_t* flags;            // all-level cells: bit0 D (covered by finer), bit1 B (ring)
  uint8_t* st_new;           // all-level cells: new state
  const uint8_t* st_old;
};
hipError_t launch_mark_static(const Geom& G, const uint8_t* solid, uint8_t* t0_static, hipStream_t s);
// level-0 targets: the static ones, then the particles' positions (flag, if given, is cleared)
hipError_t launch_targets(const HierLaunch& h, const float* particles, int64_t n, int32_t* flag, hipStream_t s);
// particles moved by d, the level-0 target set of their new positions, and flag = 1 if
// it differs from t0_prev (the flag cleared first), in three launches
hipError_t launch_advance_targets(const HierLaunch& h, float* particles, int64_t n, const float d[3],
                                  const uint8_t* t0_prev, int32_t* flag, hipStream_t s);
// the new block state of every cell of every level (one pass over all levels after
// the per-level flag passes); with `flag` non-null, any cell whose state differs from
// st_old sets *flag = tag (tag never 0 or 1: a stale value cannot read as a change)
hipError_t launch_states(const HierLaunch& h, int32_t* flag, int32_t tag, hipStream_t s);
// *flag = 1 if any of the n bytes of a and b differ (left alone otherwise: clear it first)
hipError_t launch_diff(const uint8_t* a, const uint8_t* b, int64_t n, int32_t* flag, hipStream_t s);

// Order-preserving compaction (ballot + device prefix scan) of several segments in
// three launches: per wave the count of every predicate, one single-workgroup scan over
// every segment's wave counts, then the scatter. Each segment's items start on a wave.
constexpr int kMaxSegs = 8;
// cells of levels in Morton order; predicates: active now, new (active now, not
// before), removed (active before, not now); outputs are the cells' level-linear indices
struct CellSegs {
  Geom G;
  const uint8_t* st_new;
  const uint8_t* st_old;
  int nseg;
  int level[kMaxLevels];
  int32_t* out[kMaxLevels][3];   // compacted cells per predicate (may be null)
  int32_t* count[kMaxLevels];    // device: the segment's three totals
};
// entries of int32 lists (block slots) with a predicate byte per slot (bits 0..5)
struct ByteSegs {
  int nseg;
  const int32_t* items[kMaxSegs];
  const uint8_t* bytes[kMaxSegs];
  int32_t n[kMaxSegs];
  int32_t* out[kMaxSegs][6];     // compacted slots per predicate (may be null)
  int32_t* count[kMaxSegs][2];   // device: totals of predicates 0..2, then 3..5
};
// wave_ints: capacity of the wave scratch (int32 entries); a segment set that needs
// more is refused (hipErrorInvalidValue)
hipError_t launch_compact_cells(const CellSegs& c, int32_t* wave_scratch, int64_t wave_ints, hipStream_t s);
hipError_t launch_compact_bytes(const ByteSegs& b, int32_t* wave_scratch, int64_t wave_ints, hipStream_t s);
// wave scratch entries the two need at most: all levels' cells, and block lists of
// `list_items` entries in total over at most kMaxSegs segments
int64_t compact_cells_ints(const Geom& G);
int64_t compact_bytes_ints(int64_t list_items);
// run class of every tile of a level for the two-substep sweep: the first tile of each
// run of up to `run_max` tiles stacked along z gets bit (h - 1) for the run's height h;
// runs break below a missing tile and at tile positions z = 0 (mod run_max)
hipError_t launch_tile_runs(const Geom& G, int level, const int32_t* blocks, int32_t n, const uint8_t* summary,
                            const uint8_t* st, const int4* coord, int run_max, uint8_t* run_class, hipStream_t s);

struct AllocLaunch {
  const int32_t* cells;      // new cells of one level
  int32_t n;
  int level;
  Geom G;
  const int32_t* free_stack;
  int32_t free_top;          // stack top before this level's allocation
  int32_t* dir_new;
  int4* coord;
};
hipError_t launch_alloc(const AllocLaunch& a, hipStream_t s);
hipError_t launch_release(const int32_t* cells, int32_t n, int64_t level_off, const int32_t* dir_old,
                          int32_t* free_stack, int32_t free_top, int32_t* dir_new, hipStream_t s);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* dst, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* dst, uint8_t v, int64_t n, hipStream_t s);

// every level in one launch: workgroups [wg0[l], wg0[l + 1]) take level l's cells, four
// per workgroup (the launcher fills wg0)
struct RoleLaunch {
  Geom G;
  const int32_t* cells[kMaxLevels];  // active cells of each level (new hierarchy), Morton order
  int32_t n[kMaxLevels];
  int32_t* blocks[kMaxLevels];       // out: each level's slots in key order
  int32_t wg0[kMaxLevels + 1];
  const int32_t* dir;        // new directory
  const uint8_t* st;         // new states
  const uint8_t* st_old;     // old states (a block whose 27 positions kept their states keeps its roles)
  const uint8_t* solid;      // fine solid field or null
  uint8_t* role;             // [slot][512] new roles
  uint8_t* summary;          // [slot]
  int32_t* gbox;             // [slot] bounding box of the ghost nodes (3 bits per bound: lo x, hi x, lo y, ...)
  int32_t* nbr;              // out: [slot][27]
  uint8_t* run_class;        // out: [slot] z-run class of the finest level's tile heads (0 elsewhere), or null
  int run_max;               // tiles per run at most
};
hipError_t launch_roles(const RoleLaunch& r, hipStream_t s);

struct InitLaunch {
  Geom G;
  int level;
  const int32_t* cells;      // active cells of the level (new hierarchy), or null: slots
  const int32_t* slots;      // with cells null: the level's blocks that may hold new nodes
  const int4* coord;         // block coordinates by slot (with slots)
  int32_t n;                 // list length, or with n_dev an upper bound of it
  const int32_t* n_dev;      // device: the list length (read by the kernel), or null
  const int32_t* dir_new;
  const uint8_t* st_old;
  const int32_t* dir_old;
  const uint8_t* role_old;
  const uint8_t* role_new;
  const void* cur[kMaxLevels];   // current time level of every level (old hierarchy)
  void* dst_cur;             // current time level of this level
  void* dst_other;           // other time level of this level
  float a_up[kMaxLevels];
  float a_down[kMaxLevels];
  int create;                // 1: no old hierarchy, start at rest
  Scales sc;
  int storage;
  float* cpl;                // finest level with coupling fields: reset for new blocks; else null
  float* phi;                // finest level with a powder-snow field: zero for new blocks; else null
};
// the levels' initialisations (a[0 .. nlev - 1], one storage format) in one launch
hipError_t launch_init(const InitLaunch* a, int nlev, hipStream_t s);
// adjoint of launch_init over the same cells: lam[p] is the adjoint of time level p
// (f32 slot layout), parity[k] the current time level of level k
struct InitAdjLaunch {
  InitLaunch f;
  float* lam[2];
  int parity[kMaxLevels];
};
hipError_t launch_init_adj(const InitAdjLaunch& x, hipStream_t s);

// ---- powder-snow volume fraction on the finest level ----
struct ScalarLaunch {
  const int32_t* blocks;     // the finest level's blocks (key order)
  int32_t nblocks;
  const int32_t* nbr;        // [slot][27] neighbour slots (< 0: none / wall)
  const uint8_t* role;       // [slot][512]
  const void* moments;       // the finest level's current time level (velocity)
  Scales sc;
  int storage;
  const float* phi_in;       // [slot][512]
  float* phi_out;            // [slot][512]
  const float* source;       // [list index][512] or null (diffusion step only)
  float dt, D;
};
hipError_t launch_scalar_advect(const ScalarLaunch& a, hipStream_t s);
hipError_t launch_scalar_diffuse(const ScalarLaunch& a, hipStream_t s);
hipError_t launch_scalar_set(const LevelGeom& g, const int64_t* keys, const float* in, int64_t nb, const int32_t* dir,
                             const uint8_t* role, float* phi, int32_t* err, hipStream_t s);
hipError_t launch_scalar_get(const int32_t* blocks, int32_t nblocks, const float* phi, float* out, hipStream_t s);

// ---- data movement and reductions ----
struct IoLaunch {
  Geom G;
  int level;
  const int32_t* blocks;
  int32_t nblocks;
  const int4* coord;
  const uint8_t* role;
  void* buf;                 // current time level
  void* other;               // other time level (set only)
  Scales sc;
  int storage;
};
hipError_t launch_get(const IoLaunch& a, int64_t* keys, float* out, hipStream_t s);
hipError_t launch_get_roles(const IoLaunch& a, uint8_t* out, hipStream_t s);
// finest-level coupling fields [slot][4][512] (eps, F)
hipError_t launch_cpl_default(float* cpl, int64_t nslots, hipStream_t s);
hipError_t launch_cpl_check(const LevelGeom& g, const int64_t* keys, const float* in, int64_t nb, const int32_t* dir,
                            float tau0, int32_t* err, hipStream_t s);
hipError_t launch_cpl_set(const LevelGeom& g, const int64_t* keys, const float* in, int64_t nb, const int32_t* dir,
                          const uint8_t* role, float* cpl, hipStream_t s);
hipError_t launch_set(const IoLaunch& a, const int64_t* keys, const float* in, int64_t nb,
                      const int32_t* dir, int32_t* err_flag, hipStream_t s);
hipError_t launch_keys(const IoLaunch& a, int64_t* keys, hipStream_t s);
hipError_t launch_reduce(const IoLaunch& a, const int32_t lo[3], const int32_t hi[3], double* partial,
                         double* out, hipStream_t s);
hipError_t launch_finite(const IoLaunch& a, int32_t* flag, hipStream_t s);
// partials of the reductions of callers that cannot allocate: a static device array of
// kNoAllocReduceBlocks x 5 doubles per GPU; noalloc_reduce_scratch returns its device
// address on the current device (looked up once per device)
constexpr int64_t kNoAllocReduceBlocks = int64_t(1) << 18;
hipError_t noalloc_reduce_scratch(double** out);
hipError_t launch_advance_particles(float* p, int64_t n, float dx, float dy, float dz, hipStream_t s);

// ---- adjoint (reverse mode) ----
// adjoint of one level's stream-collide, two passes:
//   launch_sc_mu: mu = (dY/dM)^T lambda_Y at computed nodes (zero elsewhere), lambda_Y
//     cleared and the outputs y restored from the tape at computed and solid nodes;
//   launch_sc_transpose: lam_x += (da/dX)^T L^T mu over the level's blocks.
struct AdjScLaunch {
  const void* x;             // forward input time level (storage type)
  void* y;                   // forward output time level (restored from the tape)
  const void* tape;          // old values of y, [list index][10][512]
  float* mu;                 // adjoint of the scaled moments M (f32 pool layout, zero at zero_slot)
  float* lam_x;              // adjoint of the input time level (f32 pool layout), accumulated
  float* lam_y;              // adjoint of the output time level
  const int32_t* blocks;
  int32_t nblocks;
  const int32_t* nbr;
  const uint8_t* role;
  int32_t zero_slot;
  float omega;
  Scales sc;
  int storage;
  // transpose only: if next_mu is set, the next operation of the reverse sweep is the
  // stream-collide of this level that wrote x; the transpose then also does that
  // operation's k_sc_mu pass (its mu into next_mu, x restored from next_tape, the
  // adjoint of x cleared at computed and solid nodes)
  void* next_x;
  const void* next_tape;
  float* next_mu;
};
hipError_t launch_sc_mu(const AdjScLaunch& a, hipStream_t s);
hipError_t launch_sc_transpose(const AdjScLaunch& a, hipStream_t s);

struct AdjTransferLaunch {
  Geom G;
  int level;                 // fine level l
  const int32_t* blocks;     // blocks visited (see each launcher)
  int32_t nblocks;
  const int32_t* dir;
  const uint8_t* role;
  const int4* coord;
  const void* src_a;         // forward sources (down: coarse t and t + 2; up: fine current)
  const void* src_b;
  float factor;
  Scales sc;
  int storage;
  float* lam_fine;           // adjoint of the level-l time level involved (down: the s = 1 ghosts')
  float* lam_fine2;          // down: adjoint of the time level holding the s = 2 ghosts
  float* lam_coarse_a;       // adjoint of the level-(l+1) time level src_a (up: the target)
  float* lam_coarse_b;       // adjoint of the level-(l+1) time level src_b
  float* scratch;            // down: per ghost block [list index][10][125] coarse-footprint partials for src_a
  float* scratch2;           // down: the same for src_b
  const int32_t* gidx;       // down: ghost-list index per slot (-1 if not a ghost block of level l)
  void* undo_dst;            // time level the forward operation wrote (restored from undo_tape)
  const void* undo_tape;     // its old values, [list index][10][512]
  void* undo_dst2;           // down: the time level of the s = 2 ghosts
  const void* undo_tape2;    // down: its old values
  uint8_t* flags;            // per slot: level-(l+1) block read by a level-l ghost
};
// downward transfer: (a) over the ghost blocks of level l, (b) over the blocks of level l+1
hipError_t launch_down_adj_lin(const AdjTransferLaunch& a, hipStream_t s);
hipError_t launch_down_adj_gather(const AdjTransferLaunch& a, hipStream_t s);
// sets flags[slot] = 1 for the level-(l+1) blocks the ghosts of the level-l ghost blocks read
hipError_t launch_mark_gather(const AdjTransferLaunch& a, hipStream_t s);
// gidx[blocks[i]] = i
hipError_t launch_ghost_index(const int32_t* blocks, int32_t n, int32_t* gidx, hipStream_t s);
// upward transfer over the interface blocks of level l+1
hipError_t launch_up_adj(const AdjTransferLaunch& a, hipStream_t s);
// outflow copy over the outflow blocks of a level: lam_coarse_a = adjoint of the new
// time level, lam_fine = adjoint of the old one
hipError_t launch_outflow_adj(const AdjTransferLaunch& a, hipStream_t s);
// d(1/2 sum rho |u|^2)/d(moments) over the owned nodes of the level inside a fine-unit
// box, written per block in key order (out[i] for blocks[i]) from the time level src_a
hipError_t launch_loss_ke_grad(const AdjTransferLaunch& a, float* out, const int32_t lo[3], const int32_t hi[3],
                               hipStream_t s);
// adjoint given per block in key order -> pool layout at the state nodes (computed,
// interface, outflow), zero elsewhere
hipError_t launch_lam_scatter(const float* in, float* lam, const int32_t* blocks, const uint8_t* role, int32_t n,
                              hipStream_t s);
hipError_t launch_zero_blocks(float* buf, const int32_t* blocks, int32_t n, hipStream_t s);
// dst[i] = src[blocks[i]] / dst[blocks[i]] = src[i], whole blocks of block_bytes (multiple of 16)
hipError_t launch_gather_blocks(const void* src, void* dst, const int32_t* blocks, int32_t n, size_t block_bytes,
                                hipStream_t s);
hipError_t launch_scatter_blocks(const void* src, void* dst, const int32_t* blocks, int32_t n, size_t block_bytes,
                                 hipStream_t s);
// dst[i] = src_a[blocks[i]] and dst[n + i] = src_b[blocks[i]] in one launch
hipError_t launch_gather_blocks2(const void* src_a, const void* src_b, void* dst, const int32_t* blocks, int32_t n,
                                 size_t block_bytes, hipStream_t s);
// eight 64-bit words written by a kernel (kernel arguments: no host buffer to keep alive)
struct Words8 { uint64_t v[8]; };
hipError_t launch_write_words(uint64_t* dst, Words8 w, hipStream_t s);

}  // namespace lbmx
