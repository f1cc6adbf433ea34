// Host runtime behind the C ABI of include/lbm.h: configuration checks, the
// layout of the caller-owned device buffers, the Alg. 1 driver (Sec. 5.3) and the
// grid-update pipeline (Sec. 6.3).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"
#include "lbm.h"

using namespace lbmx;

namespace {

thread_local std::string g_create_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  size_t t0, t0s, t0p, flags, st[2], dir[2], lists, wave, counts, coord, nbr, role[2], summary, gbox, free_stack, blocks,
      gblocks, iblocks, oblocks, tblocks, runs, run_class, red_partial, red_out, flag, cpl, phi;
  size_t total;
  int64_t level_list_off[kMaxLevels];  // offset (elements) of each level's segment in blocks / g/i/o lists
  int64_t level_list_cap[kMaxLevels];
  int64_t wave_ints;                   // int32 entries of the compactions' wave scratch
};

bool make_geom(const lbm_config* c, Geom& G, std::string& err) {
  if (!c) { err = "null configuration"; return false; }
  if (c->levels < 1 || c->levels > kMaxLevels) { err = "levels must be in 1..5"; return false; }
  std::memset(&G, 0, sizeof(G));
  G.L = c->levels;
  const int unit = kEdge << (c->levels - 1);
  for (int a = 0; a < 3; ++a) {
    if (c->fine_extent[a] <= 0 || c->fine_extent[a] % unit != 0) {
      err = "fine_extent must be a positive multiple of 8*2^(levels-1)";
      return false;
    }
    if (c->fine_extent[a] > (1 << 20)) { err = "fine_extent too large"; return false; }
    G.N[a] = c->fine_extent[a];
  }
  for (int f = 0; f < 6; ++f) {
    if (c->bc[f] < 0 || c->bc[f] > LBM_OUTFLOW_CONV) { err = "unknown boundary kind"; return false; }
    G.bc[f] = c->bc[f];
  }
  for (int a = 0; a < 3; ++a) {
    const bool p0 = c->bc[2 * a] == LBM_PERIODIC, p1 = c->bc[2 * a + 1] == LBM_PERIODIC;
    if (p0 != p1) { err = "periodic faces must come in pairs"; return false; }
    G.periodic[a] = p0 ? 1 : 0;
  }
  int64_t off = 0;
  for (int l = 0; l < G.L; ++l) {
    LevelGeom& g = G.lv[l];
    int mx = 0;
    for (int a = 0; a < 3; ++a) {
      g.nn[a] = G.N[a] >> l;
      g.nb[a] = g.nn[a] / kEdge;
      mx = g.nb[a] > mx ? g.nb[a] : mx;
    }
    g.mbits = 0;
    while ((1 << g.mbits) < mx) ++g.mbits;
    g.ncell = (int64_t)g.nb[0] * g.nb[1] * g.nb[2];
    g.off = off;
    off += g.ncell;
  }
  // block positions are indexed with int32 (cell lists, directory entries)
  if (off > INT32_MAX) { err = "domain too large: more than 2^31 block positions over all levels"; return false; }
  if (!(c->tau0 > 0.5) || !std::isfinite(c->tau0)) { err = "tau0 must be finite and exceed 1/2"; return false; }
  if (c->storage < LBM_F32 || c->storage > LBM_F16) { err = "unknown storage format"; return false; }
  if (c->rescale != 0 && c->rescale != 1) { err = "rescale must be 0 or 1"; return false; }
  if (c->coupling != 0 && c->coupling != 1) { err = "coupling must be 0 or 1"; return false; }
  if (c->scalar != 0 && c->scalar != 1) { err = "scalar must be 0 or 1"; return false; }
  if (c->max_blocks < 1 || c->max_blocks > (int64_t(1) << 26)) { err = "max_blocks must be in 1..2^26"; return false; }
  if (c->storage != LBM_F32)
    for (int m = 0; m < kMom; ++m)
      if (!(c->scale[m] > 0.0f) || !std::isfinite(c->scale[m])) { err = "storage scales must be positive"; return false; }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(c->inflow_u[a])) { err = "inflow_u must be finite"; return false; }
  if (c->inflow_profile != LBM_INFLOW_UNIFORM && c->inflow_profile != LBM_INFLOW_LOG) {
    err = "unknown inflow profile";
    return false;
  }
  if (c->inflow_profile == LBM_INFLOW_LOG &&
      (c->inflow_axis < 0 || c->inflow_axis > 2 || !(c->inflow_beta >= 0.0f) || !std::isfinite(c->inflow_beta) ||
       !std::isfinite(c->inflow_h0))) {
    err = "log inflow profile: axis 0..2, finite beta >= 0 and h0";
    return false;
  }
  for (int a = 0; a < 3; ++a) G.inflow[a] = c->inflow_u[a];
  G.inflow_profile = c->inflow_profile;
  G.inflow_axis = c->inflow_profile == LBM_INFLOW_LOG ? c->inflow_axis : 0;
  G.inflow_beta = c->inflow_beta;
  G.inflow_h0 = c->inflow_h0;
  return true;
}

Layout make_layout(const lbm_config* c, const Geom& G) {
  Layout L;
  std::memset(&L, 0, sizeof(L));
  const int64_t cap = c->max_blocks;
  int64_t ncell = 0, nlist = 0;
  for (int l = 0; l < G.L; ++l) {
    ncell += G.lv[l].ncell;
    L.level_list_off[l] = nlist;
    L.level_list_cap[l] = G.lv[l].ncell < cap ? G.lv[l].ncell : cap;
    nlist += L.level_list_cap[l];
  }
  // all levels' cells in one compaction; all block lists plus the level-0 runs in another
  const int64_t wc = compact_cells_ints(G), wb = compact_bytes_ints(nlist + L.level_list_cap[0]);
  L.wave_ints = wc > wb ? wc : wb;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, 256); return r; };
  L.t0 = take(G.lv[0].ncell);
  L.t0s = take(G.lv[0].ncell);
  L.t0p = take(G.lv[0].ncell);
  L.flags = take(ncell);
  L.st[0] = take(ncell);
  L.st[1] = take(ncell);
  L.dir[0] = take(ncell * 4);
  L.dir[1] = take(ncell * 4);
  L.lists = take(3 * ncell * 4);
  L.wave = take(L.wave_ints * 4);
  L.counts = take(64 * 4);
  L.coord = take(cap * 16);
  L.nbr = take(cap * 27 * 4);
  L.role[0] = take(cap * kNodes);
  L.role[1] = take(cap * kNodes);
  L.summary = take(cap);
  L.gbox = take(cap * 4);
  L.free_stack = take(cap * 4);
  L.blocks = take(nlist * 4);
  L.gblocks = take(nlist * 4);
  L.iblocks = take(nlist * 4);
  L.oblocks = take(nlist * 4);
  L.tblocks = take(nlist * 4);
  // z runs of level-0 tiles by height (class k: runs of k + 1 tiles), and every level-0
  // block's run class
  L.runs = take((size_t)kRunMax * L.level_list_cap[0] * 4);
  L.run_class = take(cap);
  L.red_partial = take(cap * 5 * 8);
  L.red_out = take(8 * 8);
  L.flag = take(64);
  // finest-level coupling fields (eps, F) per slot and for the all-zero slot
  L.cpl = c->coupling ? take((size_t)(cap + 1) * 4 * kNodes * sizeof(float)) : 0;
  // finest-level powder-snow volume fraction, current and intermediate field per slot
  L.phi = c->scalar ? take((size_t)2 * cap * kNodes * sizeof(float)) : 0;
  L.total = o;
  return L;
}

size_t elem_bytes(int storage) { return storage == LBM_F32 ? 4 : 2; }

}  // namespace

struct lbm_ctx {
  lbm_config cfg;
  Geom G;
  Layout lay;
  hipStream_t stream = nullptr;
  // lbm_step_remesh: the particle advance and the target-set check run on `side`
  // (default priority) while the step runs on `stream`
  hipStream_t side = nullptr;
  hipEvent_t ev_before = nullptr, ev_side = nullptr;
  int64_t cap = 0;
  double tau[kMaxLevels], a_up[kMaxLevels], a_down[kMaxLevels];
  int parity[kMaxLevels];
  Scales sc;
  size_t elem = 4;
  char* pool = nullptr;
  char* meta = nullptr;
  int hier = 0;   // which of st/dir is current
  int rcur = 0;   // which role array is current
  const uint8_t* solid = nullptr;
  int64_t nblk[kMaxLevels], ngb[kMaxLevels], nib[kMaxLevels], nob[kMaxLevels], ntile[kMaxLevels];
  int64_t nbb[kMaxLevels];          // blocks holding bounce-back nodes
  int64_t tile_min_blocks = 16384;  // LBM_OPT_TILE_MIN_BLOCKS
  int fuse_substeps = 2;            // LBM_OPT_FUSE_SUBSTEPS: 0 never, 1 with FP32 storage, 2 always
  int use_graphs = 0;               // LBM_OPT_GRAPHS
  int pair_run = 4;                 // LBM_OPT_PAIR_RUN: tiles per run of the two-substep sweep (4, 2 with 16-bit storage)
  int64_t nrun[kRunMax] = {0};      // level-0 runs of k + 1 tiles
  uint32_t state_tag = 0;           // grid updates that compared block states (tags their flag)
  // Coarse steps replayed as HIP graphs: the launch arguments of a coarse step follow
  // from the host state in LaunchKey alone (buffer parities, hierarchy and role-table
  // selectors, list lengths, options), so a graph captured for one key replays any
  // later step that starts from the same key.
  struct LaunchKey {
    int32_t hier, rcur, fuse, parity[kMaxLevels];
    int64_t tile_min, nblk[kMaxLevels], ngb[kMaxLevels], nib[kMaxLevels], nob[kMaxLevels], ntile[kMaxLevels],
        nbb[kMaxLevels], nrun[kRunMax];
  };
  struct StepGraph {
    LaunchKey key;
    int32_t parity_after[kMaxLevels];
    hipGraphExec_t exec;
  };
  std::vector<StepGraph> graphs;
  hipStream_t gstream = nullptr;    // capture stream (the caller's may be the null stream)
  int32_t free_top = 0;
  int32_t* host_counts = nullptr;  // pinned
  double* noalloc_partial = nullptr;  // this GPU's static reduction partials (lbm_reduce_f64_noalloc)
  // Alg. 1 of one coarse step as a flat list (lbm_step_finest stops after a finest-level
  // stream-collide); fine_cursor = operations of the current coarse step already run
  struct SchedOp { int kind, level, s; };
  std::vector<SchedOp> sched;
  size_t fine_cursor = 0;
  std::string err;
  // phase timers (HIP events around launches, enabled on request)
  bool profiling = false;
  uint32_t prof_mask = 0;  // phases timed while profiling
  struct Timed { int phase; hipEvent_t a, b; };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> spare;
  double prof_ms[LBM_PROFILE_PHASES] = {0};
  int64_t prof_n[LBM_PROFILE_PHASES] = {0};
  uint64_t generation = 0;  // bumped by every grid update that changes the hierarchy
  // undo log of one coarse step replayed for the adjoint: before every operation
  // the blocks it is about to overwrite are copied to the tape
  enum { OP_SC = 0, OP_DOWN = 1, OP_UP = 2, OP_REMESH = 3 };
  // OP_REMESH: off = the meta buffer before the update, off2 = both time levels of every
  // block before it (level order, key order), aux = index of the host-side counts in hier_saves
  struct TapeOp { int kind, level, s, pf, pc; size_t off, off2; int aux = -1; };
  struct HierSave {
    int64_t nblk[kMaxLevels], ngb[kMaxLevels], nib[kMaxLevels], nob[kMaxLevels], ntile[kMaxLevels],
        nbb[kMaxLevels], nrun[kRunMax];
    int hier, rcur;
    int32_t free_top;
    uint64_t generation;
    int parity[kMaxLevels];  // time-level parity of every level (a grid update leaves it)
  };
  std::vector<HierSave> hier_saves;
  bool rec_open = false;     // a recording opened by lbm_record_begin (steps and grid updates)
  size_t rec_aux = 0;        // bytes of the work buffer's aux region for the recording
  bool recording = false;
  char* tape = nullptr;
  size_t tape_cap = 0, tape_used = 0;
  std::vector<TapeOp> ops;
  size_t pending_sc_tape = SIZE_MAX;   // tape of the finest level's second substep, taken with the first's
  const void* rec_work = nullptr;      // work buffer holding the recorded steps (null: none)
  uint64_t rec_generation = 0;         // hierarchy they were recorded on
  int rec_parity[kMaxLevels] = {0};    // time-level parities before them

  template <class T> T* m(size_t off) const { return reinterpret_cast<T*>(meta + off); }
  uint8_t* st(int k) const { return m<uint8_t>(lay.st[k]); }
  int32_t* dir(int k) const { return m<int32_t>(lay.dir[k]); }
  uint8_t* role(int k) const { return m<uint8_t>(lay.role[k]); }
  int32_t* lists(int l, int k) const {
    int64_t off = 0;
    for (int j = 0; j < l; ++j) off += 3 * G.lv[j].ncell;
    return m<int32_t>(lay.lists) + off + k * G.lv[l].ncell;
  }
  int32_t* blocks(int l) const { return m<int32_t>(lay.blocks) + lay.level_list_off[l]; }
  int32_t* gblocks(int l) const { return m<int32_t>(lay.gblocks) + lay.level_list_off[l]; }
  int32_t* iblocks(int l) const { return m<int32_t>(lay.iblocks) + lay.level_list_off[l]; }
  int32_t* oblocks(int l) const { return m<int32_t>(lay.oblocks) + lay.level_list_off[l]; }
  // one block of every stream-collide tile (kTileX x 2 x 2 blocks) of the level
  int32_t* tblocks(int l) const { return m<int32_t>(lay.tblocks) + lay.level_list_off[l]; }
  // finest-level coupling fields [slot][4][512] (eps, F), null without coupling
  float* cpl() const { return cfg.coupling ? m<float>(lay.cpl) : nullptr; }
  // finest-level powder-snow volume fraction [k][slot][512], k = 0 current, 1 intermediate
  float* phi(int k) const { return cfg.scalar ? m<float>(lay.phi) + (size_t)k * cap * kNodes : nullptr; }
  // time level p of the pool: cap block slots plus one all-zero slot (index cap)
  void* buf(int l, int p) const { return pool + (size_t)p * (size_t)(cap + 1) * kBlockStride * elem; }
  void* cur(int l) const { return buf(l, parity[l]); }
  void* other(int l) const { return buf(l, 1 - parity[l]); }

  lbm_status fail(lbm_status s, const std::string& msg) { err = msg; return s; }
  hipEvent_t take_event() {
    if (!spare.empty()) { hipEvent_t e = spare.back(); spare.pop_back(); return e; }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
  }
  // open a timed region of a phase; returns its index or -1 (timing is best effort:
  // a region whose events cannot be created or recorded is left out)
  int tic(int phase) {
    if (!profiling || !((prof_mask >> phase) & 1u)) return -1;
    Timed t{phase, take_event(), take_event()};
    if (!t.a || !t.b || hipEventRecord(t.a, stream) != hipSuccess) {
      if (t.a) spare.push_back(t.a);
      if (t.b) spare.push_back(t.b);
      return -1;
    }
    timed.push_back(t);
    return (int)timed.size() - 1;
  }
  void toc(int k) {
    if (k >= 0 && hipEventRecord(timed[(size_t)k].b, stream) != hipSuccess) timed[(size_t)k].phase = -1;
  }
  void collect() {
    if (timed.empty()) return;
    const bool synced = hipStreamSynchronize(stream) == hipSuccess;
    for (auto& t : timed) {
      float ms = 0.0f;
      if (synced && t.phase >= 0 && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
        prof_ms[t.phase] += ms;
        prof_n[t.phase] += 1;
      }
      spare.push_back(t.a);
      spare.push_back(t.b);
    }
    timed.clear();
  }
  lbm_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return LBM_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EDEVICE;
  }
};

#define HIPCHK(ctx, expr)                                        \
  do {                                                           \
    lbm_status _s = (ctx)->hip_check((expr), #expr);             \
    if (_s != LBM_OK) return _s;                                 \
  } while (0)

namespace {

IoLaunch io_of(const lbm_ctx* c, int level) {
  IoLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.G = c->G;
  a.level = level;
  a.blocks = c->blocks(level);
  a.nblocks = (int32_t)c->nblk[level];
  a.coord = c->m<int4>(c->lay.coord);
  a.role = c->role(c->rcur);
  a.buf = c->cur(level);
  a.other = c->other(level);
  a.sc = c->sc;
  a.storage = c->cfg.storage;
  return a;
}

int32_t* counts_flag(lbm_ctx* c) { return c->m<int32_t>(c->lay.counts) + 63; }

// Level-0 tiles grouped into z runs of up to pair_run tiles (the two-substep sweep's
// work items): the run class of every level-0 block, then (as segment k of a byte
// compaction) the runs by height, counts in counts[48 .. 53].
lbm_status tile_runs(lbm_ctx* c, int64_t nb0) {
  HIPCHK(c, launch_tile_runs(c->G, 0, c->blocks(0), (int32_t)nb0, c->m<uint8_t>(c->lay.summary), c->st(c->hier),
                             c->m<int4>(c->lay.coord), c->pair_run, c->m<uint8_t>(c->lay.run_class), c->stream));
  return LBM_OK;
}
void runs_segment(lbm_ctx* c, int64_t nb0, ByteSegs& b, int k) {
  int32_t* counts = c->m<int32_t>(c->lay.counts);
  b.items[k] = c->blocks(0);
  b.bytes[k] = c->m<uint8_t>(c->lay.run_class);
  b.n[k] = (int32_t)nb0;
  for (int r = 0; r < kRunMax; ++r) b.out[k][r] = c->m<int32_t>(c->lay.runs) + (size_t)r * c->lay.level_list_cap[0];
  b.count[k][0] = counts + 48;
  b.count[k][1] = counts + 51;
}
lbm_status build_runs(lbm_ctx* c, int64_t nb0) {
  if (lbm_status st = tile_runs(c, nb0)) return st;
  ByteSegs b;
  std::memset(&b, 0, sizeof(b));
  b.nseg = 1;
  runs_segment(c, nb0, b, 0);
  HIPCHK(c, launch_compact_bytes(b, c->m<int32_t>(c->lay.wave), c->lay.wave_ints, c->stream));
  return LBM_OK;
}

// Grid update: H(Phi) for the particles (plus static solid blocks), new nodes
// initialised from the old hierarchy (or at rest when creating).
// targets_ready: the level-0 target set is already in place and known to differ from
// the one the hierarchy was built from (lbm_step_remesh checks it on its side stream).
lbm_status rebuild(lbm_ctx* c, const float* particles, int64_t n, bool create, bool targets_ready = false) {
  const Geom& G = c->G;
  hipStream_t s = c->stream;
  const int L = G.L;
  const int nh = 1 - c->hier;
  HierLaunch h;
  h.G = G;
  h.t0 = c->m<uint8_t>(c->lay.t0);
  h.t0_static = c->m<uint8_t>(c->lay.t0s);
  h.flags = c->m<uint8_t>(c->lay.flags);
  h.st_new = c->st(nh);
  h.st_old = c->st(c->hier);
  // (the target copy clears the change flag of the check below)
  if (!targets_ready) HIPCHK(c, launch_targets(h, particles, n, counts_flag(c), s));
  int32_t* counts = c->m<int32_t>(c->lay.counts);
  int32_t* wave = c->m<int32_t>(c->lay.wave);
  uint8_t* t0_prev = c->m<uint8_t>(c->lay.t0p);
  int64_t ncell = 0;
  for (int l = 0; l < L; ++l) ncell += G.lv[l].ncell;
  if (!create && !targets_ready) {
    // fast path: H(Phi) depends on the level-0 target set T0 alone. If T0 equals a
    // target set the current hierarchy is built from, nothing changes.
    HIPCHK(c, launch_diff(h.t0, t0_prev, G.lv[0].ncell, counts + 63, s));
    HIPCHK(c, hipMemcpyAsync(c->host_counts, counts + 63, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (c->host_counts[0] == 0) return LBM_OK;
  }
  // otherwise the new block states are compared with the current ones (a change writes
  // this update's tag into the flag); the flag comes back with the compaction counts
  // (one synchronisation for both)
  const int32_t tag = (int32_t)(0x40000000u | (++c->state_tag & 0x3fffffffu));
  HIPCHK(c, launch_states(h, create ? nullptr : counts + 63, tag, s));
  {
    CellSegs cs;
    std::memset(&cs, 0, sizeof(cs));
    cs.G = G;
    cs.st_new = h.st_new;
    cs.st_old = h.st_old;
    cs.nseg = L;
    for (int l = 0; l < L; ++l) {
      cs.level[l] = l;
      for (int k = 0; k < 3; ++k) cs.out[l][k] = c->lists(l, k);
      cs.count[l] = counts + 3 * l;
    }
    HIPCHK(c, launch_compact_cells(cs, wave, c->lay.wave_ints, s));
  }
  HIPCHK(c, hipMemcpyAsync(c->host_counts, counts, 64 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (!create && c->host_counts[63] != tag) {
    HIPCHK(c, hipMemcpyAsync(t0_prev, h.t0, (size_t)G.lv[0].ncell, hipMemcpyDeviceToDevice, s));
    return LBM_OK;
  }
  int64_t nact[kMaxLevels], nnew[kMaxLevels], nrem[kMaxLevels];
  int64_t tot_new = 0, tot_act = 0;
  for (int l = 0; l < L; ++l) {
    nact[l] = c->host_counts[3 * l];
    nnew[l] = c->host_counts[3 * l + 1];
    nrem[l] = c->host_counts[3 * l + 2];
    tot_new += nnew[l];
    tot_act += nact[l];
    if (nact[l] > c->lay.level_list_cap[l]) return c->fail(LBM_ECAPACITY, "level block count exceeds the pool capacity");
  }
  if (tot_new > c->free_top || tot_act > c->cap)
    return c->fail(LBM_ECAPACITY, "block pool too small for the new hierarchy (" + std::to_string(tot_act) +
                                      " blocks needed, max_blocks " + std::to_string(c->cap) + ")");
  // ---- from here on the update commits
  int32_t* dir_old = c->dir(c->hier);
  int32_t* dir_new = c->dir(nh);
  HIPCHK(c, launch_copy_i32(dir_old, dir_new, ncell, s));
  int32_t top = c->free_top;
  int4* coord = c->m<int4>(c->lay.coord);
  int32_t* fstack = c->m<int32_t>(c->lay.free_stack);
  for (int l = 0; l < L; ++l) {
    AllocLaunch a;
    a.cells = c->lists(l, 1);
    a.n = (int32_t)nnew[l];
    a.level = l;
    a.G = G;
    a.free_stack = fstack;
    a.free_top = top;
    a.dir_new = dir_new;
    a.coord = coord;
    HIPCHK(c, launch_alloc(a, s));
    top -= (int32_t)nnew[l];
  }
  for (int l = 0; l < L; ++l) {
    HIPCHK(c, launch_release(c->lists(l, 2), (int32_t)nrem[l], G.lv[l].off, dir_old, fstack, top, dir_new, s));
    top += (int32_t)nrem[l];
  }
  uint8_t* role_old = c->role(c->rcur);
  uint8_t* role_new = c->role(1 - c->rcur);
  uint8_t* summary = c->m<uint8_t>(c->lay.summary);
  {
    RoleLaunch r;
    std::memset(&r, 0, sizeof(r));
    r.G = G;
    for (int l = 0; l < L; ++l) {
      r.cells[l] = c->lists(l, 0);
      r.n[l] = (int32_t)nact[l];
      r.blocks[l] = c->blocks(l);
    }
    r.dir = dir_new;
    r.st = h.st_new;
    r.st_old = h.st_old;
    r.solid = c->solid;
    r.role = role_new;
    r.summary = summary;
    r.gbox = c->m<int32_t>(c->lay.gbox);
    r.nbr = c->m<int32_t>(c->lay.nbr);
    r.run_class = L >= 2 ? c->m<uint8_t>(c->lay.run_class) : nullptr;
    r.run_max = c->pair_run;
    HIPCHK(c, launch_roles(r, s));
  }
  c->hier = nh;
  c->rcur = 1 - c->rcur;
  c->free_top = top;
  c->generation++;
  HIPCHK(c, hipMemcpyAsync(t0_prev, h.t0, (size_t)G.lv[0].ncell, hipMemcpyDeviceToDevice, s));
  // one compaction of every level's blocks by summary bit and of the level-0 tiles' z runs
  // (their class bytes written by the role pass) by height
  {
    ByteSegs b;
    std::memset(&b, 0, sizeof(b));
    b.nseg = L;
    for (int l = 0; l < L; ++l) {
      b.items[l] = c->blocks(l);
      b.bytes[l] = summary;
      b.n[l] = (int32_t)nact[l];
      b.out[l][0] = c->gblocks(l);
      b.out[l][1] = c->iblocks(l);
      b.out[l][2] = c->oblocks(l);
      b.out[l][3] = c->tblocks(l);
      b.out[l][4] = nullptr;         // bounce-back blocks: counted only
      b.out[l][5] = c->lists(l, 1);  // blocks that may hold new nodes (SUM_FRESH)
      b.count[l][0] = counts + 3 * l;
      b.count[l][1] = counts + 32 + 3 * l;
    }
    if (L >= 2) runs_segment(c, nact[0], b, b.nseg++);
    HIPCHK(c, launch_compact_bytes(b, wave, c->lay.wave_ints, s));
  }
  // new nodes: on a first build every block starts at rest; after that only blocks whose
  // 27 surrounding block positions changed state can hold nodes the update makes owned
  // (their count stays on the device: the launch strides over it), all levels in one launch
  InitLaunch inits[kMaxLevels];
  for (int l = 0; l < L; ++l) {
    InitLaunch& a = inits[l];
    std::memset(&a, 0, sizeof(a));
    a.G = G;
    a.level = l;
    if (create) {
      a.cells = c->lists(l, 0);
      a.n = (int32_t)nact[l];
    } else {
      a.slots = c->lists(l, 1);
      a.coord = coord;
      a.n = (int32_t)nact[l];
      a.n_dev = counts + 34 + 3 * l;
    }
    a.dir_new = dir_new;
    a.st_old = h.st_old;
    a.dir_old = dir_old;
    a.role_old = role_old;
    a.role_new = role_new;
    for (int k = 0; k < L; ++k) a.cur[k] = c->cur(k);
    a.dst_cur = c->cur(l);
    a.dst_other = c->other(l);
    for (int k = 0; k < L; ++k) {
      a.a_up[k] = (float)c->a_up[k];
      a.a_down[k] = (float)c->a_down[k];
    }
    a.create = create ? 1 : 0;
    a.sc = c->sc;
    a.storage = c->cfg.storage;
    a.cpl = l == 0 ? c->cpl() : nullptr;
    a.phi = l == 0 ? c->phi(0) : nullptr;
  }
  HIPCHK(c, launch_init(inits, L, s));
  HIPCHK(c, hipMemcpyAsync(c->host_counts, counts, 54 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (int l = 0; l < L; ++l) {
    c->nblk[l] = nact[l];
    c->ngb[l] = c->host_counts[3 * l];
    c->nib[l] = c->host_counts[3 * l + 1];
    c->nob[l] = c->host_counts[3 * l + 2];
    c->ntile[l] = c->host_counts[32 + 3 * l];
    c->nbb[l] = c->host_counts[33 + 3 * l];
  }
  for (int k = 0; k < kRunMax; ++k) c->nrun[k] = L >= 2 ? c->host_counts[48 + k] : 0;
  return LBM_OK;
}

size_t block_bytes(const lbm_ctx* c) { return (size_t)kBlockStride * c->elem; }

// undo-log entry of the next operation: room for the old values of the n blocks it
// writes (and of the n2 outflow blocks of a stream-collide); filled by a bulk copy
// before a stream-collide, by the transfer and outflow kernels themselves otherwise
lbm_status record(lbm_ctx* c, int kind, int l, int s, int64_t n, int64_t n2, void** tape, void** tape2) {
  const size_t bytes = (size_t)(n + n2) * block_bytes(c);
  if (c->tape_used + bytes > c->tape_cap) return c->fail(LBM_ECAPACITY, "adjoint tape too small");
  lbm_ctx::TapeOp op;
  op.kind = kind;
  op.level = l;
  op.s = s;
  op.pf = c->parity[l];
  op.pc = l + 1 < c->G.L ? c->parity[l + 1] : 0;
  op.off = c->tape_used;
  op.off2 = c->tape_used + (size_t)n * block_bytes(c);
  *tape = c->tape + op.off;
  if (tape2) *tape2 = c->tape + op.off2;
  c->tape_used += bytes;
  c->ops.push_back(op);
  return LBM_OK;
}

// ---- Alg. 1 (Sec. 5.3) ----
bool tiled(const lbm_ctx* c, int l) { return c->ntile[l] > 0 && c->ntile[l] * 4 * kTileX >= c->tile_min_blocks; }

ScLaunch sc_base(lbm_ctx* c, int l) {
  ScLaunch a;
  a.in = c->cur(l);
  a.out = c->other(l);
  a.blocks = c->blocks(l);
  a.nblocks = (int32_t)c->nblk[l];
  a.nbr = c->m<int32_t>(c->lay.nbr);
  a.role = c->role(c->rcur);
  a.zero_slot = (int32_t)c->cap;
  a.omega = (float)(1.0 / c->tau[l]);
  a.sc = c->sc;
  a.storage = c->cfg.storage;
  // tiles once the level has enough blocks (16384 by default) to fill the chip
  // several times with them; single blocks below
  const bool t = tiled(c, l);
  a.tiles = t ? c->tblocks(l) : nullptr;
  a.ntiles = t ? (int32_t)c->ntile[l] : 0;
  a.dir = c->dir(c->hier);
  a.coord = c->m<int4>(c->lay.coord);
  a.lg = c->G.lv[l];
  for (int k = 0; k < 3; ++k) a.periodic[k] = c->G.periodic[k];
  a.cpl = l == 0 ? c->cpl() : nullptr;
  a.runs = c->m<int32_t>(c->lay.runs);
  a.run_stride = c->lay.level_list_cap[0];
  for (int k = 0; k < kRunMax; ++k) a.nrun[k] = l == 0 ? (int32_t)c->nrun[k] : 0;
  return a;
}

lbm_status sc_level(lbm_ctx* c, int l, int s) {
  ScLaunch a = sc_base(c, l);
  void* otape = nullptr;
  if (c->recording) {
    // the whole blocks of the written time level go to the tape (one bulk copy). On
    // the finest level (below a coarser one) nothing else runs between the two
    // substeps of a parent step, and the first does not write the time level the
    // second writes, whose computed and solid nodes (all its undo restores; the
    // downward transfer restores ghosts itself) are already final: both copies are
    // taken in one launch before the first substep.
    const int64_t nb = c->nblk[l];
    const bool pair = l == 0 && c->G.L >= 2;
    void* tape = nullptr;
    lbm_status st;
    if (pair && s == 2 && c->pending_sc_tape != SIZE_MAX) {
      st = record(c, lbm_ctx::OP_SC, l, 0, 0, c->nob[l], &tape, &otape);
      if (st != LBM_OK) return st;
      c->ops.back().off = c->pending_sc_tape;
      c->pending_sc_tape = SIZE_MAX;
    } else {
      st = record(c, lbm_ctx::OP_SC, l, 0, pair && s == 1 ? 2 * nb : nb, c->nob[l], &tape, &otape);
      if (st != LBM_OK) return st;
      if (pair && s == 1) {
        HIPCHK(c, launch_gather_blocks2(c->other(l), c->cur(l), tape, c->blocks(l), (int32_t)nb, block_bytes(c),
                                        c->stream));
        c->pending_sc_tape = c->ops.back().off + (size_t)nb * block_bytes(c);
      } else {
        HIPCHK(c, launch_gather_blocks(c->other(l), tape, c->blocks(l), (int32_t)nb, block_bytes(c), c->stream));
      }
    }
  }
  const int k = c->tic(LBM_PROF_SC0 + l);
  HIPCHK(c, launch_stream_collide(a, c->stream));
  c->toc(k);
  if (c->nob[l] > 0) {
    OutflowLaunch o;
    o.G = c->G;
    o.level = l;
    o.blocks = c->oblocks(l);
    o.nblocks = (int32_t)c->nob[l];
    o.role = c->role(c->rcur);
    o.coord = c->m<int4>(c->lay.coord);
    o.old_buf = c->cur(l);
    o.new_buf = c->other(l);
    o.sc = c->sc;
    o.storage = c->cfg.storage;
    o.tape = otape;
    const int ko = c->tic(LBM_PROF_OUTFLOW);
    HIPCHK(c, launch_outflow(o, c->stream));
    c->toc(ko);
  }
  c->parity[l] ^= 1;
  return LBM_OK;
}

TransferLaunch transfer_base(lbm_ctx* c, int l) {
  TransferLaunch t;
  std::memset(&t, 0, sizeof(t));
  t.G = c->G;
  t.level = l;
  t.dir = c->dir(c->hier);
  t.role = c->role(c->rcur);
  t.coord = c->m<int4>(c->lay.coord);
  t.sc = c->sc;
  t.storage = c->cfg.storage;
  return t;
}

// DownwardTransfer(l+1, s): ghosts of level l from level l+1 (old: t, current: t+2).
// Both fine substeps read the same two coarse time levels, so the s = 2 ghosts are
// written together with the s = 1 ghosts, into the time level the first fine
// stream-collide writes (it leaves ghost nodes alone); the s = 2 call then has
// nothing left to do. The adjoint replay keeps the old values of both ghost sets.
lbm_status down_level(lbm_ctx* c, int l, int s) {
  if (c->ngb[l] == 0 || s == 2) return LBM_OK;
  TransferLaunch t = transfer_base(c, l);
  t.blocks = c->gblocks(l);
  t.nblocks = (int32_t)c->ngb[l];
  t.src_a = c->other(l + 1);
  t.src_b = c->cur(l + 1);
  t.dst = c->cur(l);
  t.dst2 = c->other(l);
  t.factor = (float)c->a_down[l];
  t.gbox = c->m<int32_t>(c->lay.gbox);
  if (c->recording) {
    lbm_status st = record(c, lbm_ctx::OP_DOWN, l, s, c->ngb[l], c->ngb[l], &t.tape, &t.tape2);
    if (st != LBM_OK) return st;
  }
  const int k = c->tic(LBM_PROF_DOWN);
  HIPCHK(c, launch_downward(t, c->stream));
  c->toc(k);
  return LBM_OK;
}

// UpwardTransfer(l): interface nodes of level l+1 from level l
lbm_status up_level(lbm_ctx* c, int l) {
  if (c->nib[l + 1] == 0) return LBM_OK;
  TransferLaunch t = transfer_base(c, l);
  t.blocks = c->iblocks(l + 1);
  t.nblocks = (int32_t)c->nib[l + 1];
  t.src_a = c->cur(l);
  t.dst = c->cur(l + 1);
  t.factor = (float)c->a_up[l];
  if (c->recording) {
    lbm_status st = record(c, lbm_ctx::OP_UP, l, 0, c->nib[l + 1], 0, &t.tape, nullptr);
    if (st != LBM_OK) return st;
  }
  const int k = c->tic(LBM_PROF_UP);
  HIPCHK(c, launch_upward(t, c->stream));
  c->toc(k);
  return LBM_OK;
}

// Both substeps of a parent step of the finest level in one sweep: its ghosts for
// both are in place after the first downward transfer, and nothing else runs between
// the two substeps. The result goes to the other time level, so the level's parity
// flips once instead of twice; the intermediate time level is never stored (no finer
// level interpolates from it).
bool pair_ok(const lbm_ctx* c) {
  // with 16-bit storage the two sweeps are faster: they move half the bytes, while
  // the one-sweep kernel is bound by its arithmetic, to which the codec adds
  const bool want = c->fuse_substeps == 2 || (c->fuse_substeps == 1 && c->cfg.storage == LBM_F32);
  return want && !c->recording && c->G.L >= 2 && tiled(c, 0) && c->nob[0] == 0 && c->nbb[0] == 0 &&
         !c->cfg.coupling;
}

lbm_status sc_pair(lbm_ctx* c) {
  ScLaunch a = sc_base(c, 0);
  const int k = c->tic(LBM_PROF_SC_PAIR);
  HIPCHK(c, launch_stream_collide_pair(a, c->stream));
  c->toc(k);
  c->parity[0] ^= 1;
  return LBM_OK;
}

lbm_status advance(lbm_ctx* c, int l, int s) {
  const int L = c->G.L;
  lbm_status st;
  if (l < L - 1 && (st = down_level(c, l, s)) != LBM_OK) return st;
  if ((st = sc_level(c, l, s)) != LBM_OK) return st;
  if (l < L - 1 && s == 2 && (st = up_level(c, l)) != LBM_OK) return st;
  if (l == 1 && pair_ok(c)) {
    if ((st = down_level(c, 0, 1)) != LBM_OK) return st;
    if ((st = sc_pair(c)) != LBM_OK) return st;
    if ((st = up_level(c, 0)) != LBM_OK) return st;
  } else if (l > 0) {
    if ((st = advance(c, l - 1, 1)) != LBM_OK) return st;
    if ((st = advance(c, l - 1, 2)) != LBM_OK) return st;
  }
  return LBM_OK;
}

lbm_ctx::LaunchKey launch_key(const lbm_ctx* c) {
  lbm_ctx::LaunchKey k;
  std::memset(&k, 0, sizeof(k));
  k.hier = c->hier;
  k.rcur = c->rcur;
  k.fuse = c->fuse_substeps;
  k.tile_min = c->tile_min_blocks;
  for (int l = 0; l < c->G.L; ++l) {
    k.parity[l] = c->parity[l];
    k.nblk[l] = c->nblk[l];
    k.ngb[l] = c->ngb[l];
    k.nib[l] = c->nib[l];
    k.nob[l] = c->nob[l];
    k.ntile[l] = c->ntile[l];
    k.nbb[l] = c->nbb[l];
  }
  for (int r = 0; r < kRunMax; ++r) k.nrun[r] = c->nrun[r];
  return k;
}

// One coarse step (Alg. 1 from the coarsest level). Outside profiling and recording
// the step's launches are captured once per launch state into a HIP graph (on a
// stream of the context's own) and replayed on the context's stream; the host-side
// parities advance as the launches would have advanced them.
lbm_status coarse_step(lbm_ctx* c) {
  const int L = c->G.L;
  if (!c->use_graphs || c->profiling || c->recording) return advance(c, L - 1, 1);
  const lbm_ctx::LaunchKey key = launch_key(c);
  for (const auto& g : c->graphs)
    if (std::memcmp(&g.key, &key, sizeof(key)) == 0) {
      HIPCHK(c, hipGraphLaunch(g.exec, c->stream));
      for (int l = 0; l < L; ++l) c->parity[l] = g.parity_after[l];
      return LBM_OK;
    }
  if (!c->gstream) HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
  hipStream_t user = c->stream;
  HIPCHK(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
  c->stream = c->gstream;
  const lbm_status st = advance(c, L - 1, 1);
  c->stream = user;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c->gstream, &graph);
  if (st != LBM_OK) {
    if (e == hipSuccess && graph) (void)hipGraphDestroy(graph);
    return st;
  }
  HIPCHK(c, e);
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(c, ei);
  if (c->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  lbm_ctx::StepGraph g;
  g.key = key;
  for (int l = 0; l < kMaxLevels; ++l) g.parity_after[l] = l < L ? c->parity[l] : 0;
  g.exec = exec;
  c->graphs.push_back(g);
  HIPCHK(c, hipGraphLaunch(exec, c->stream));
  return LBM_OK;
}

// The operations of AdvanceLBM(l, s) in the order advance() runs them unfused.
void plan(int L, int l, int s, std::vector<lbm_ctx::SchedOp>& out) {
  if (l < L - 1) out.push_back({lbm_ctx::OP_DOWN, l, s});
  out.push_back({lbm_ctx::OP_SC, l, s});
  if (l < L - 1 && s == 2) out.push_back({lbm_ctx::OP_UP, l, s});
  if (l > 0) {
    plan(L, l - 1, 1, out);
    plan(L, l - 1, 2, out);
  }
}

// One finest-level step: the operations up to and including the next finest-level
// stream-collide, then the upward transfers that follow it.
lbm_status finest_step(lbm_ctx* c) {
  const auto& q = c->sched;
  bool done = false;
  while (c->fine_cursor < q.size()) {
    const lbm_ctx::SchedOp& op = q[c->fine_cursor];
    if (done && op.kind != lbm_ctx::OP_UP) break;
    lbm_status st = op.kind == lbm_ctx::OP_DOWN ? down_level(c, op.level, op.s)
                    : op.kind == lbm_ctx::OP_UP ? up_level(c, op.level)
                                                : sc_level(c, op.level, op.s);
    if (st != LBM_OK) return st;
    if (op.kind == lbm_ctx::OP_SC && op.level == 0) done = true;
    ++c->fine_cursor;
  }
  if (c->fine_cursor == q.size()) c->fine_cursor = 0;
  return LBM_OK;
}

bool level_ok(lbm_ctx* c, int level) { return c && level >= 0 && level < c->G.L; }

// calls that need every level at the same time (a coarse-step boundary)
lbm_status need_boundary(lbm_ctx* c) {
  if (c->fine_cursor != 0)
    return c->fail(LBM_ESTATE, "a coarse step is under way (lbm_step_finest): finish it with lbm_step_finest first");
  return LBM_OK;
}

// ---- adjoint of one coarse step: reverse sweep over the undo log ----
constexpr uint64_t kStateMagic = 0x4554415453424c4dull;  // "MLBSTATE"
constexpr size_t kStateHeader = 256;

struct AdjBufs {
  float* lam[2];   // adjoint of the pool's two time levels (f32, slot layout)
  float* mu[2];    // adjoint of the scaled moments M (f32, slot layout; two, see adjoint_op)
  float* part;     // downward transfer: coarse-footprint partials per ghost block, all levels
  int32_t* gidx;   // per slot: index in its level's ghost-block list, or -1
  uint8_t* flags;  // per slot: coarse block read by ghosts of the next finer level
};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }
size_t part_bytes(const lbm_ctx* c) {
  int64_t n = 0;
  for (int l = 0; l < c->G.L; ++l) n += c->ngb[l];
  return round256((size_t)n * 2 * kMom * 125 * sizeof(float));  // two per ghost block
}
size_t aux_bytes(const lbm_ctx* c) {
  return part_bytes(c) + round256((size_t)(c->cap + 1) * 4) + round256((size_t)(c->cap + 1));
}

// the aux region sized for any hierarchy the pool can hold (recordings with grid updates)
size_t aux_bytes_cap(const lbm_ctx* c) {
  return round256((size_t)c->cap * 2 * kMom * 125 * sizeof(float)) + round256((size_t)(c->cap + 1) * 4) +
         round256((size_t)(c->cap + 1));
}

lbm_ctx::HierSave save_hier(const lbm_ctx* c) {
  lbm_ctx::HierSave h;
  for (int l = 0; l < kMaxLevels; ++l) {
    h.nblk[l] = c->nblk[l]; h.ngb[l] = c->ngb[l]; h.nib[l] = c->nib[l];
    h.nob[l] = c->nob[l]; h.ntile[l] = c->ntile[l]; h.nbb[l] = c->nbb[l];
  }
  for (int k = 0; k < kRunMax; ++k) h.nrun[k] = c->nrun[k];
  h.hier = c->hier;
  h.rcur = c->rcur;
  h.free_top = c->free_top;
  h.generation = c->generation;
  for (int l = 0; l < kMaxLevels; ++l) h.parity[l] = c->parity[l];
  return h;
}
void load_hier(lbm_ctx* c, const lbm_ctx::HierSave& h) {
  for (int l = 0; l < kMaxLevels; ++l) {
    c->nblk[l] = h.nblk[l]; c->ngb[l] = h.ngb[l]; c->nib[l] = h.nib[l];
    c->nob[l] = h.nob[l]; c->ntile[l] = h.ntile[l]; c->nbb[l] = h.nbb[l];
  }
  for (int k = 0; k < kRunMax; ++k) c->nrun[k] = h.nrun[k];
  c->hier = h.hier;
  c->rcur = h.rcur;
  c->free_top = h.free_top;
  c->generation = h.generation;
}

size_t slot_floats(const lbm_ctx* c) { return (size_t)(c->cap + 1) * kBlockStride; }

// Grid update inside a recording: the meta buffer and both time levels of every block
// go to the undo log first; if the update changes nothing (or is refused), the log
// entry is dropped and the meta buffer, whose scratch parts the update used, is put
// back, so that the tables of earlier recorded updates stay intact.
lbm_status rebuild_recorded(lbm_ctx* c, const float* particles, int64_t n) {
  hipStream_t s = c->stream;
  const size_t bb = block_bytes(c);
  int64_t nb = 0;
  for (int l = 0; l < c->G.L; ++l) nb += c->nblk[l];
  const size_t meta_bytes = round256(c->lay.total);
  const size_t bytes = meta_bytes + (size_t)nb * 2 * bb;
  if (c->tape_used + bytes > c->tape_cap) return c->fail(LBM_ECAPACITY, "adjoint tape too small for a grid update");
  const size_t off = c->tape_used;
  HIPCHK(c, hipMemcpyAsync(c->tape + off, c->meta, c->lay.total, hipMemcpyDeviceToDevice, s));
  size_t o = off + meta_bytes;
  for (int l = 0; l < c->G.L; ++l) {
    HIPCHK(c, launch_gather_blocks2(c->cur(l), c->other(l), c->tape + o, c->blocks(l), (int32_t)c->nblk[l], bb, s));
    o += (size_t)c->nblk[l] * 2 * bb;
  }
  const lbm_ctx::HierSave before = save_hier(c);
  const uint64_t gen = c->generation;
  lbm_status st = rebuild(c, particles, n, false);
  if (st != LBM_OK || c->generation == gen) {
    // nothing changed (or refused): the scratch parts of meta back, the entry dropped
    HIPCHK(c, hipMemcpyAsync(c->meta, c->tape + off, c->lay.total, hipMemcpyDeviceToDevice, s));
    return st;
  }
  lbm_ctx::TapeOp op;
  op.kind = lbm_ctx::OP_REMESH;
  op.level = op.s = op.pf = op.pc = 0;
  op.off = off;
  op.off2 = off + meta_bytes;
  op.aux = (int)c->hier_saves.size();
  c->hier_saves.push_back(before);
  c->ops.push_back(op);
  c->tape_used += bytes;
  return LBM_OK;
}
constexpr size_t kAdjSlotBufs = 4;  // lam[2], mu[2]

size_t tape_bytes(const lbm_ctx* c) {
  const int L = c->G.L;
  int64_t nb = 0;
  for (int l = 0; l < L; ++l) {
    const int64_t calls = int64_t(1) << (L - 1 - l);  // advance(l, s) calls per coarse step
    nb += calls * (c->nblk[l] + c->nob[l]);
    if (l + 1 < L) nb += calls * c->ngb[l] + (calls / 2) * c->nib[l + 1];
  }
  return (size_t)nb * block_bytes(c);
}

int64_t total_blocks(const lbm_ctx* c) {
  int64_t nb = 0;
  for (int l = 0; l < c->G.L; ++l) nb += c->nblk[l];
  return nb;
}

AdjTransferLaunch adj_base(lbm_ctx* c, int l) {
  AdjTransferLaunch t;
  std::memset(&t, 0, sizeof(t));
  t.G = c->G;
  t.level = l;
  t.dir = c->dir(c->hier);
  t.role = c->role(c->rcur);
  t.coord = c->m<int4>(c->lay.coord);
  t.sc = c->sc;
  t.storage = c->cfg.storage;
  return t;
}

// state carried from one operation of the reverse sweep to the next
struct AdjSweep {
  int mu_cur = 0;         // mu buffer of the next stream-collide
  bool mu_ready = false;  // its first pass (k_sc_mu) already done by the previous transpose
};

// adjoint of one recorded operation in the state right after it, then its undo
// (folded into the adjoint kernels: each restores the nodes the operation wrote).
// next: the operation the sweep takes after this one (recorded just before it).
// per-slot tables of the downward transfer's adjoint for the current hierarchy
lbm_status adjoint_tables(lbm_ctx* c, const AdjBufs& b) {
  hipStream_t s = c->stream;
  HIPCHK(c, launch_fill_u8(b.flags, 0, c->cap + 1, s));
  HIPCHK(c, launch_fill_i32(b.gidx, -1, c->cap + 1, s));
  for (int l = 0; l + 1 < c->G.L; ++l) {
    AdjTransferLaunch t = adj_base(c, l);
    t.blocks = c->gblocks(l);
    t.nblocks = (int32_t)c->ngb[l];
    t.flags = b.flags;
    HIPCHK(c, launch_mark_gather(t, s));
    HIPCHK(c, launch_ghost_index(c->gblocks(l), (int32_t)c->ngb[l], b.gidx, s));
  }
  return LBM_OK;
}

// Reverse of a recorded grid update (Sec. 6.3 new-node initialisation), in the state
// right after it: the old state goes back into the old blocks' slots (it is what the
// sampler read), the adjoint of every node the update wrote flows through the
// transposed sampler into the old nodes, then the old tables and counts come back.
// The time levels are those current at the update (the reverse sweep keeps the
// context's parity at the end of the recording).
lbm_status reverse_remesh(lbm_ctx* c, const lbm_ctx::TapeOp& op, const AdjBufs& b) {
  hipStream_t s = c->stream;
  const int L = c->G.L;
  const lbm_ctx::HierSave& old = c->hier_saves[(size_t)op.aux];
  const char* msnap = c->tape + op.off;
  const size_t bb = block_bytes(c);
  size_t o = op.off2;
  for (int l = 0; l < L; ++l) {
    const int32_t n = (int32_t)old.nblk[l];
    const int32_t* blocks_old =
        reinterpret_cast<const int32_t*>(msnap + c->lay.blocks) + c->lay.level_list_off[l];
    HIPCHK(c, launch_scatter_blocks(c->tape + o, c->buf(l, old.parity[l]), blocks_old, n, bb, s));
    HIPCHK(c, launch_scatter_blocks(c->tape + o + (size_t)n * bb, c->buf(l, 1 - old.parity[l]), blocks_old, n, bb,
                                    s));
    o += (size_t)n * 2 * bb;
  }
  for (int l = 0; l < L; ++l) {
    InitAdjLaunch x;
    std::memset(&x, 0, sizeof(x));
    InitLaunch& a = x.f;
    a.G = c->G;
    a.level = l;
    a.cells = c->lists(l, 0);
    a.n = (int32_t)c->nblk[l];
    a.dir_new = c->dir(c->hier);
    a.dir_old = c->dir(1 - c->hier);
    a.st_old = c->st(1 - c->hier);
    a.role_new = c->role(c->rcur);
    a.role_old = c->role(1 - c->rcur);
    for (int k = 0; k < L; ++k) {
      a.cur[k] = c->buf(k, old.parity[k]);
      a.a_up[k] = (float)c->a_up[k];
      a.a_down[k] = (float)c->a_down[k];
      x.parity[k] = old.parity[k];
    }
    a.sc = c->sc;
    a.storage = c->cfg.storage;
    x.lam[0] = b.lam[0];
    x.lam[1] = b.lam[1];
    HIPCHK(c, launch_init_adj(x, s));
  }
  HIPCHK(c, hipMemcpyAsync(c->meta, msnap, c->lay.total, hipMemcpyDeviceToDevice, s));
  load_hier(c, old);
  return adjoint_tables(c, b);
}

lbm_status adjoint_op(lbm_ctx* c, const lbm_ctx::TapeOp& op, const lbm_ctx::TapeOp* next, const AdjBufs& b,
                      AdjSweep& sw) {
  const int l = op.level;
  hipStream_t s = c->stream;
  if (op.kind == lbm_ctx::OP_REMESH) return reverse_remesh(c, op, b);
  if (op.kind == lbm_ctx::OP_SC) {
    const int p = op.pf;  // input time level; the sweep wrote 1 - p
    if (c->nob[l] > 0) {
      AdjTransferLaunch t = adj_base(c, l);
      t.blocks = c->oblocks(l);
      t.nblocks = (int32_t)c->nob[l];
      t.lam_coarse_a = b.lam[1 - p];
      t.lam_fine = b.lam[p];
      t.undo_dst = c->buf(l, 1 - p);
      t.src_a = c->buf(l, p);  // the old time level (convective outflow)
      t.undo_tape = c->tape + op.off2;
      const int k = c->tic(LBM_PROF_ADJ);
      HIPCHK(c, launch_outflow_adj(t, s));
      c->toc(k);
    }
    AdjScLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.x = c->buf(l, p);
    a.y = c->buf(l, 1 - p);
    a.tape = c->tape + op.off;
    a.mu = b.mu[sw.mu_cur];
    a.lam_x = b.lam[p];
    a.lam_y = b.lam[1 - p];
    a.blocks = c->blocks(l);
    a.nblocks = (int32_t)c->nblk[l];
    a.nbr = c->m<int32_t>(c->lay.nbr);
    a.role = c->role(c->rcur);
    a.zero_slot = (int32_t)c->cap;
    a.omega = (float)(1.0 / c->tau[l]);
    a.sc = c->sc;
    a.storage = c->cfg.storage;
    if (!sw.mu_ready) {
      const int k = c->tic(LBM_PROF_ADJ);
      HIPCHK(c, launch_sc_mu(a, s));
      c->toc(k);
    }
    // the next operation is the stream-collide of this level that wrote this one's
    // input (consecutive substeps of the finest level, or consecutive steps of a
    // single level), with no outflow adjoint before its first pass: the transpose
    // does that pass per node, into the other mu buffer
    const bool fuse = next && next->kind == lbm_ctx::OP_SC && next->level == l && next->pf == 1 - p &&
                      c->nob[l] == 0;
    if (fuse) {
      a.next_x = c->buf(l, p);
      a.next_tape = c->tape + next->off;
      a.next_mu = b.mu[1 - sw.mu_cur];
    }
    const int k = c->tic(fuse ? LBM_PROF_ADJ_SC_FUSED : LBM_PROF_ADJ_SC);
    HIPCHK(c, launch_sc_transpose(a, s));
    c->toc(k);
    sw.mu_ready = fuse;
    if (fuse) sw.mu_cur = 1 - sw.mu_cur;
  } else if (op.kind == lbm_ctx::OP_DOWN) {
    // both substeps' ghosts: s = 1 in time level pf, s = 2 in 1 - pf
    AdjTransferLaunch t = adj_base(c, l);
    t.blocks = c->gblocks(l);
    t.nblocks = (int32_t)c->ngb[l];
    t.src_a = c->buf(l + 1, 1 - op.pc);
    t.src_b = c->buf(l + 1, op.pc);
    t.factor = (float)c->a_down[l];
    t.lam_fine = b.lam[op.pf];
    t.lam_fine2 = b.lam[1 - op.pf];
    t.lam_coarse_a = b.lam[1 - op.pc];
    t.lam_coarse_b = b.lam[op.pc];
    size_t poff = 0;
    for (int k = 0; k < l; ++k) poff += (size_t)c->ngb[k] * 2 * kMom * 125;
    t.scratch = b.part + poff;
    t.scratch2 = t.scratch + (size_t)c->ngb[l] * kMom * 125;
    t.gidx = b.gidx;
    t.flags = b.flags;
    t.undo_dst = c->buf(l, op.pf);
    t.undo_dst2 = c->buf(l, 1 - op.pf);
    t.undo_tape = c->tape + op.off;
    t.undo_tape2 = c->tape + op.off2;
    const int k = c->tic(LBM_PROF_ADJ);
    HIPCHK(c, launch_down_adj_lin(t, s));
    t.blocks = c->blocks(l + 1);
    t.nblocks = (int32_t)c->nblk[l + 1];
    HIPCHK(c, launch_down_adj_gather(t, s));
    c->toc(k);
  } else {
    AdjTransferLaunch t = adj_base(c, l);
    t.blocks = c->iblocks(l + 1);
    t.nblocks = (int32_t)c->nib[l + 1];
    t.src_a = c->buf(l, op.pf);
    t.factor = (float)c->a_up[l];
    t.lam_fine = b.lam[op.pf];
    t.lam_coarse_a = b.lam[op.pc];
    t.undo_dst = c->buf(l + 1, op.pc);
    t.undo_tape = c->tape + op.off;
    const int k = c->tic(LBM_PROF_ADJ);
    HIPCHK(c, launch_up_adj(t, s));
    c->toc(k);
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_pool_bytes(const lbm_config* cfg) {
  Geom G;
  std::string e;
  if (!make_geom(cfg, G, e)) return 0;
  return 2 * (size_t)(cfg->max_blocks + 1) * kBlockStride * elem_bytes(cfg->storage);
}

size_t lbm_meta_bytes(const lbm_config* cfg) {
  Geom G;
  std::string e;
  if (!make_geom(cfg, G, e)) return 0;
  return make_layout(cfg, G).total;
}

lbm_status lbm_create(const lbm_config* cfg, const uint8_t* solid_fine, const float* particles, int64_t n,
                      lbm_ctx** out) {
  if (!out) { g_create_error = "null output pointer"; return LBM_EINVAL; }
  *out = nullptr;
  Geom G;
  if (!make_geom(cfg, G, g_create_error)) return LBM_EINVAL;
  if (!cfg->pool || !cfg->meta) { g_create_error = "pool and meta buffers are required"; return LBM_EINVAL; }
  if (n < 0 || (n > 0 && !particles)) { g_create_error = "bad particle array"; return LBM_EINVAL; }
  lbm_ctx* c = new lbm_ctx();
  c->cfg = *cfg;
  c->G = G;
  c->lay = make_layout(cfg, G);
  c->stream = static_cast<hipStream_t>(cfg->stream);
  c->cap = cfg->max_blocks;
  c->elem = elem_bytes(cfg->storage);
  // tiles per z run of the two-substep sweep: measured fastest on the benchmark with each format
  c->pair_run = cfg->storage == LBM_F32 ? 4 : 2;
  c->pool = static_cast<char*>(cfg->pool);
  c->meta = static_cast<char*>(cfg->meta);
  c->solid = solid_fine;
  plan(G.L, G.L - 1, 1, c->sched);
  for (int l = 0; l < G.L; ++l) {
    const double k = std::ldexp(1.0, l);
    c->tau[l] = cfg->tau0 / k + (k - 1.0) / (2.0 * k);  // tau_{l} from tau_0 (Sec. 5.2)
    c->parity[l] = 0;
    c->nblk[l] = c->ngb[l] = c->nib[l] = c->nob[l] = c->ntile[l] = c->nbb[l] = 0;
  }
  for (int l = 0; l < G.L; ++l) {
    c->a_up[l] = c->a_down[l] = 1.0;
    if (l + 1 < G.L) {
      if (cfg->rescale == 0) {
        // Chapman-Enskog: S^neq ~ -cs^2 tau_l dx_l (grad u + grad u^T)
        c->a_up[l] = 2.0 * c->tau[l + 1] / c->tau[l];
        c->a_down[l] = c->tau[l] / (2.0 * c->tau[l + 1]);
      } else {
        c->a_up[l] = c->tau[l + 1] / (2.0 * c->tau[l]);
        c->a_down[l] = 2.0 * c->tau[l + 1] / c->tau[l];
      }
    }
  }
  for (int mm = 0; mm < kMom; ++mm) {
    const float s = cfg->storage == LBM_F32 ? 1.0f : cfg->scale[mm];
    c->sc.s[mm] = s;
    c->sc.inv[mm] = 1.0f / s;
  }
  if (hipHostMalloc((void**)&c->host_counts, 64 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    g_create_error = "pinned host allocation failed";
    delete c;
    return LBM_EDEVICE;
  }
  int64_t ncell = 0;
  for (int l = 0; l < G.L; ++l) ncell += G.lv[l].ncell;
  lbm_status st = LBM_OK;
  auto chk = [&](hipError_t e, const char* what) {
    if (st == LBM_OK && e != hipSuccess) {
      st = LBM_EDEVICE;
      g_create_error = std::string(what) + ": " + hipGetErrorString(e);
    }
  };
  chk(launch_fill_u8(c->st(0), ST_ABSENT, ncell, c->stream), "clear states");
  for (int p = 0; p < 2; ++p)  // the all-zero slot of each time level
    chk(launch_fill_u8(static_cast<uint8_t*>(c->buf(0, p)) + (size_t)c->cap * kBlockStride * c->elem, 0,
                       (int64_t)kBlockStride * (int64_t)c->elem, c->stream),
        "zero slot");
  chk(launch_fill_i32(c->dir(0), NBR_NONE, ncell, c->stream), "clear directory");
  if (c->cpl()) chk(launch_cpl_default(c->cpl(), c->cap + 1, c->stream), "coupling fields");
  if (c->phi(0)) chk(launch_fill_i32(reinterpret_cast<int32_t*>(c->phi(0)), 0, 2 * c->cap * kNodes, c->stream), "phi");
  std::vector<int32_t> fs((size_t)c->cap);
  for (int64_t i = 0; i < c->cap; ++i) fs[(size_t)i] = (int32_t)(c->cap - 1 - i);
  chk(hipMemcpyAsync(c->m<int32_t>(c->lay.free_stack), fs.data(), fs.size() * 4, hipMemcpyHostToDevice, c->stream),
      "free list");
  c->free_top = (int32_t)c->cap;
  chk(launch_mark_static(G, solid_fine, c->m<uint8_t>(c->lay.t0s), c->stream), "static targets");
  chk(noalloc_reduce_scratch(&c->noalloc_partial), "address of the static reduction partials");
  chk(hipStreamSynchronize(c->stream), "synchronise");
  if (st == LBM_OK) {
    st = rebuild(c, particles, n, true);
    if (st != LBM_OK) g_create_error = c->err;
  }
  if (st != LBM_OK) {
    (void)hipHostFree(c->host_counts);
    delete c;
    return st;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return LBM_EINVAL;
  // teardown: release what can be released; a device error here has no remedy
  bool synced = hipStreamSynchronize(ctx->stream) == hipSuccess;
  if (ctx->side) synced = hipStreamSynchronize(ctx->side) == hipSuccess && synced;
  ctx->collect();
  for (hipEvent_t e : ctx->spare) (void)hipEventDestroy(e);
  if (ctx->ev_before) (void)hipEventDestroy(ctx->ev_before);
  if (ctx->ev_side) (void)hipEventDestroy(ctx->ev_side);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
  (void)hipHostFree(ctx->host_counts);
  delete ctx;
  return synced ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_num_blocks(lbm_ctx* ctx, int32_t level, int64_t* out) {
  if (!level_ok(ctx, level) || !out) return ctx ? ctx->fail(LBM_EINVAL, "bad level or null output") : LBM_EINVAL;
  *out = ctx->nblk[level];
  return LBM_OK;
}

lbm_status lbm_block_keys(lbm_ctx* ctx, int32_t level, int64_t* keys) {
  if (!level_ok(ctx, level) || !keys) return ctx ? ctx->fail(LBM_EINVAL, "bad level or null output") : LBM_EINVAL;
  HIPCHK(ctx, launch_keys(io_of(ctx, level), keys, ctx->stream));
  return LBM_OK;
}

lbm_status lbm_set_block_moments(lbm_ctx* ctx, int32_t level, const int64_t* keys, const float* in, int64_t nb) {
  if (!level_ok(ctx, level)) return ctx ? ctx->fail(LBM_EINVAL, "bad level") : LBM_EINVAL;
  if (nb < 0 || (nb > 0 && (!keys || !in))) return ctx->fail(LBM_EINVAL, "bad block arrays");
  if (lbm_status st = need_boundary(ctx)) return st;
  if (ctx->rec_open) return ctx->fail(LBM_ESTATE, "a recording is open (lbm_record_end first)");
  if (nb == 0) return LBM_OK;
  ctx->rec_work = nullptr;
  int32_t* flag = ctx->m<int32_t>(ctx->lay.flag);
  HIPCHK(ctx, launch_fill_i32(flag, 0, 1, ctx->stream));
  HIPCHK(ctx, launch_set(io_of(ctx, level), keys, in, nb, ctx->dir(ctx->hier), flag, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(ctx->host_counts, flag, 4, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->host_counts[0]) return ctx->fail(LBM_EINVAL, "a key is not an active block of this level");
  return LBM_OK;
}

lbm_status lbm_set_coupling(lbm_ctx* ctx, const int64_t* keys, const float* fields, int64_t nb) {
  if (!ctx) return LBM_EINVAL;
  if (!ctx->cfg.coupling) return ctx->fail(LBM_EINVAL, "coupling fields not enabled in the configuration");
  if (nb < 0 || (nb > 0 && (!keys || !fields))) return ctx->fail(LBM_EINVAL, "bad block arrays");
  if (nb == 0) return LBM_OK;
  int32_t* flag = ctx->m<int32_t>(ctx->lay.flag);
  HIPCHK(ctx, launch_fill_i32(flag, 0, 1, ctx->stream));
  HIPCHK(ctx, launch_cpl_check(ctx->G.lv[0], keys, fields, nb, ctx->dir(ctx->hier), (float)ctx->tau[0], flag,
                               ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(ctx->host_counts, flag, 4, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->host_counts[0] == 1) return ctx->fail(LBM_EINVAL, "a key is not an active finest-level block");
  if (ctx->host_counts[0] == 2) return ctx->fail(LBM_EINVAL, "coupling fields must be finite with eps tau0 > 1/2");
  HIPCHK(ctx, launch_cpl_set(ctx->G.lv[0], keys, fields, nb, ctx->dir(ctx->hier), ctx->role(ctx->rcur), ctx->cpl(),
                             ctx->stream));
  return LBM_OK;
}

lbm_status lbm_scalar_set(lbm_ctx* ctx, const int64_t* keys, const float* phi, int64_t nb) {
  if (!ctx) return LBM_EINVAL;
  if (!ctx->cfg.scalar) return ctx->fail(LBM_EINVAL, "the powder-snow field is not enabled in the configuration");
  if (nb < 0 || (nb > 0 && (!keys || !phi))) return ctx->fail(LBM_EINVAL, "bad block arrays");
  if (nb == 0) return LBM_OK;
  int32_t* flag = ctx->m<int32_t>(ctx->lay.flag);
  HIPCHK(ctx, launch_fill_i32(flag, 0, 1, ctx->stream));
  HIPCHK(ctx, launch_scalar_set(ctx->G.lv[0], keys, phi, nb, ctx->dir(ctx->hier), ctx->role(ctx->rcur), ctx->phi(0), flag,
                                ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(ctx->host_counts, flag, 4, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->host_counts[0]) return ctx->fail(LBM_EINVAL, "a key is not an active finest-level block");
  return LBM_OK;
}

lbm_status lbm_scalar_get(lbm_ctx* ctx, int64_t* keys_out, float* phi_out) {
  if (!ctx) return LBM_EINVAL;
  if (!ctx->cfg.scalar) return ctx->fail(LBM_EINVAL, "the powder-snow field is not enabled in the configuration");
  if (ctx->nblk[0] > 0 && (!keys_out || !phi_out)) return ctx->fail(LBM_EINVAL, "null output");
  HIPCHK(ctx, launch_keys(io_of(ctx, 0), keys_out, ctx->stream));
  HIPCHK(ctx, launch_scalar_get(ctx->blocks(0), (int32_t)ctx->nblk[0], ctx->phi(0), phi_out, ctx->stream));
  return LBM_OK;
}

lbm_status lbm_scalar_advance(lbm_ctx* ctx, float dt, float D, const float* source) {
  if (!ctx) return LBM_EINVAL;
  if (!ctx->cfg.scalar) return ctx->fail(LBM_EINVAL, "the powder-snow field is not enabled in the configuration");
  if (!(dt > 0.0f) || !std::isfinite(dt) || !(D >= 0.0f) || !std::isfinite(D))
    return ctx->fail(LBM_EINVAL, "dt must be positive and D non-negative");
  if (D * dt > 1.0f / 6.0f) return ctx->fail(LBM_EINVAL, "forward-Euler diffusion needs D dt <= 1/6");
  if (dt > 7.0f)
    return ctx->fail(LBM_EINVAL, "dt must not exceed 7 finest-level steps (departure points are searched within "
                                 "7 nodes)");
  ScalarLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.blocks = ctx->blocks(0);
  a.nblocks = (int32_t)ctx->nblk[0];
  a.nbr = ctx->m<int32_t>(ctx->lay.nbr);
  a.role = ctx->role(ctx->rcur);
  a.moments = ctx->cur(0);
  a.sc = ctx->sc;
  a.storage = ctx->cfg.storage;
  a.dt = dt;
  a.D = D;
  a.phi_in = ctx->phi(0);
  a.phi_out = ctx->phi(1);
  HIPCHK(ctx, launch_scalar_advect(a, ctx->stream));
  a.phi_in = ctx->phi(1);
  a.phi_out = ctx->phi(0);
  a.source = source;
  HIPCHK(ctx, launch_scalar_diffuse(a, ctx->stream));
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* ctx, int32_t n) {
  if (!ctx) return LBM_EINVAL;
  if (n < 0) return ctx->fail(LBM_EINVAL, "negative step count");
  if (lbm_status st = need_boundary(ctx)) return st;
  if (!ctx->rec_open) ctx->rec_work = nullptr;  // a recorded undo log no longer matches the state
  for (int32_t i = 0; i < n; ++i) {
    lbm_status st = coarse_step(ctx);
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

lbm_status lbm_step_finest(lbm_ctx* ctx, int32_t n) {
  if (!ctx) return LBM_EINVAL;
  if (n < 0) return ctx->fail(LBM_EINVAL, "negative step count");
  if (ctx->rec_open) return ctx->fail(LBM_ESTATE, "a recording is open (lbm_record_end first)");
  ctx->rec_work = nullptr;
  for (int32_t i = 0; i < n; ++i) {
    lbm_status st = finest_step(ctx);
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

lbm_status lbm_finest_phase(lbm_ctx* ctx, int32_t* out) {
  if (!ctx || !out) return ctx ? ctx->fail(LBM_EINVAL, "null output") : LBM_EINVAL;
  int32_t k = 0;
  for (size_t i = 0; i < ctx->fine_cursor; ++i)
    if (ctx->sched[i].kind == lbm_ctx::OP_SC && ctx->sched[i].level == 0) ++k;
  *out = k;
  return LBM_OK;
}

lbm_status lbm_advance_particles(lbm_ctx* ctx, float* particles, int64_t n, const float d[3]) {
  if (!ctx) return LBM_EINVAL;
  if (n < 0 || (n > 0 && (!particles || !d))) return ctx->fail(LBM_EINVAL, "bad particle arguments");
  HIPCHK(ctx, launch_advance_particles(particles, n, d[0], d[1], d[2], ctx->stream));
  return LBM_OK;
}

lbm_status lbm_remesh(lbm_ctx* ctx, const float* particles, int64_t n) {
  if (!ctx) return LBM_EINVAL;
  if (n < 0 || (n > 0 && !particles)) return ctx->fail(LBM_EINVAL, "bad particle array");
  if (lbm_status st = need_boundary(ctx)) return st;
  const int k = ctx->tic(LBM_PROF_REMESH);
  lbm_status st;
  if (ctx->rec_open) {
    st = rebuild_recorded(ctx, particles, n);
  } else {
    ctx->rec_work = nullptr;
    st = rebuild(ctx, particles, n, false);
  }
  ctx->toc(k);
  return st;
}

lbm_status lbm_step_remesh(lbm_ctx* ctx, int32_t n, float* particles, int64_t np, const float d[3]) {
  if (!ctx) return LBM_EINVAL;
  if (n < 0) return ctx->fail(LBM_EINVAL, "negative step count");
  if (np < 0 || (np > 0 && (!particles || !d))) return ctx->fail(LBM_EINVAL, "bad particle arguments");
  if (lbm_status st = need_boundary(ctx)) return st;
  if (ctx->rec_open) {
    // a recording logs the three calls in their order
    for (int32_t i = 0; i < n; ++i) {
      lbm_status st;
      if ((st = lbm_step(ctx, 1)) != LBM_OK || (st = lbm_advance_particles(ctx, particles, np, d)) != LBM_OK ||
          (st = lbm_remesh(ctx, particles, np)) != LBM_OK)
        return st;
    }
    return LBM_OK;
  }
  if (!ctx->side) {
    HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_before, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_side, hipEventDisableTiming));
  }
  ctx->rec_work = nullptr;
  const Geom& G = ctx->G;
  int32_t* flag = ctx->m<int32_t>(ctx->lay.counts) + 63;
  for (int32_t i = 0; i < n; ++i) {
    // everything issued before this step (the caller's writes to the particles too)
    HIPCHK(ctx, hipEventRecord(ctx->ev_before, ctx->stream));
    lbm_status st = coarse_step(ctx);
    if (st != LBM_OK) return st;
    // meanwhile, on the side stream: particles forward, then the level-0 target set
    // compared with the one the hierarchy was built from (the step reads neither)
    HIPCHK(ctx, hipStreamWaitEvent(ctx->side, ctx->ev_before, 0));
    HierLaunch h;
    h.G = G;
    h.t0 = ctx->m<uint8_t>(ctx->lay.t0);
    h.t0_static = ctx->m<uint8_t>(ctx->lay.t0s);
    h.flags = ctx->m<uint8_t>(ctx->lay.flags);
    h.st_new = ctx->st(1 - ctx->hier);
    h.st_old = ctx->st(ctx->hier);
    HIPCHK(ctx, launch_advance_targets(h, particles, np, d, ctx->m<uint8_t>(ctx->lay.t0p), flag, ctx->side));
    HIPCHK(ctx, hipMemcpyAsync(ctx->host_counts, flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->side));
    HIPCHK(ctx, hipEventRecord(ctx->ev_side, ctx->side));
    // later work on the context's stream sees the new particle positions
    HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_side, 0));
    HIPCHK(ctx, hipEventSynchronize(ctx->ev_side));
    if (ctx->host_counts[0] != 0) {
      // the targets changed: the grid update proper, after the step, on the context's stream
      const int k = ctx->tic(LBM_PROF_REMESH);
      st = rebuild(ctx, particles, np, false, true);
      ctx->toc(k);
      if (st != LBM_OK) return st;
    }
  }
  return LBM_OK;
}

lbm_status lbm_set_profiling(lbm_ctx* ctx, int32_t on) {
  return lbm_set_profiling_phases(ctx, on ? (1u << LBM_PROFILE_PHASES) - 1u : 0u);
}

lbm_status lbm_set_profiling_phases(lbm_ctx* ctx, uint32_t mask) {
  if (!ctx) return LBM_EINVAL;
  if (mask >> LBM_PROFILE_PHASES) return ctx->fail(LBM_EINVAL, "profiling mask names an unknown phase");
  ctx->collect();
  ctx->profiling = mask != 0;
  ctx->prof_mask = mask;
  return LBM_OK;
}

lbm_status lbm_set_option(lbm_ctx* ctx, int32_t option, int64_t value) {
  if (!ctx) return LBM_EINVAL;
  switch (option) {
    case LBM_OPT_TILE_MIN_BLOCKS:
      if (value < 0) return ctx->fail(LBM_EINVAL, "tile threshold must be >= 0");
      ctx->tile_min_blocks = value;
      return LBM_OK;
    case LBM_OPT_FUSE_SUBSTEPS:
      if (value < 0 || value > 2) return ctx->fail(LBM_EINVAL, "LBM_OPT_FUSE_SUBSTEPS takes 0, 1 or 2");
      ctx->fuse_substeps = (int)value;
      return LBM_OK;
    case LBM_OPT_GRAPHS:
      if (value < 0 || value > 1) return ctx->fail(LBM_EINVAL, "LBM_OPT_GRAPHS takes 0 or 1");
      ctx->use_graphs = (int)value;
      return LBM_OK;
    case LBM_OPT_PAIR_RUN: {
      if (value < 1 || value > kRunMax) return ctx->fail(LBM_EINVAL, "LBM_OPT_PAIR_RUN takes 1 .. 6");
      if (ctx->rec_open) return ctx->fail(LBM_ESTATE, "LBM_OPT_PAIR_RUN cannot change inside a recording");
      ctx->pair_run = (int)value;
      if (ctx->G.L < 2 || ctx->nblk[0] == 0) return LBM_OK;
      // the run lists of the current hierarchy, regrouped
      if (lbm_status st = build_runs(ctx, ctx->nblk[0])) return st;
      HIPCHK(ctx, hipMemcpyAsync(ctx->host_counts, ctx->m<int32_t>(ctx->lay.counts) + 48, kRunMax * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      for (int k = 0; k < kRunMax; ++k) ctx->nrun[k] = ctx->host_counts[k];
      return LBM_OK;
    }
  }
  return ctx->fail(LBM_EINVAL, "unknown option");
}

lbm_status lbm_get_profile(lbm_ctx* ctx, double ms[LBM_PROFILE_PHASES], int64_t count[LBM_PROFILE_PHASES]) {
  if (!ctx || !ms || !count) return ctx ? ctx->fail(LBM_EINVAL, "null output") : LBM_EINVAL;
  ctx->collect();
  for (int k = 0; k < LBM_PROFILE_PHASES; ++k) {
    ms[k] = ctx->prof_ms[k];
    count[k] = ctx->prof_n[k];
    ctx->prof_ms[k] = 0.0;
    ctx->prof_n[k] = 0;
  }
  return LBM_OK;
}

lbm_status lbm_get_moments(lbm_ctx* ctx, int32_t level, int64_t* keys_out, float* out) {
  if (!level_ok(ctx, level) || !out) return ctx ? ctx->fail(LBM_EINVAL, "bad level or null output") : LBM_EINVAL;
  HIPCHK(ctx, launch_get(io_of(ctx, level), keys_out, out, ctx->stream));
  return LBM_OK;
}

lbm_status lbm_get_roles(lbm_ctx* ctx, int32_t level, uint8_t* out) {
  if (!level_ok(ctx, level) || !out) return ctx ? ctx->fail(LBM_EINVAL, "bad level or null output") : LBM_EINVAL;
  HIPCHK(ctx, launch_get_roles(io_of(ctx, level), out, ctx->stream));
  return LBM_OK;
}

lbm_status lbm_reduce_f64(lbm_ctx* ctx, int32_t level, const int32_t lo[3], const int32_t hi[3], double out[5]) {
  if (!level_ok(ctx, level) || !lo || !hi || !out) return ctx ? ctx->fail(LBM_EINVAL, "bad arguments") : LBM_EINVAL;
  double* dev = ctx->m<double>(ctx->lay.red_out);
  HIPCHK(ctx, launch_reduce(io_of(ctx, level), lo, hi, ctx->m<double>(ctx->lay.red_partial), dev, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(out, dev, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return LBM_OK;
}

lbm_status lbm_reduce_f64_noalloc(lbm_ctx* ctx, int32_t level, const int32_t lo[3], const int32_t hi[3],
                                  double* out) {
  if (!level_ok(ctx, level) || !lo || !hi || !out) return ctx ? ctx->fail(LBM_EINVAL, "bad arguments") : LBM_EINVAL;
  if (ctx->nblk[level] > kNoAllocReduceBlocks)
    return ctx->fail(LBM_EINVAL, "level has more blocks than the static reduction partials hold (2^18)");
  if (!ctx->noalloc_partial) return ctx->fail(LBM_EDEVICE, "static reduction partials not available");
  // every partial the final pass reads is written by this call's first pass
  HIPCHK(ctx, launch_reduce(io_of(ctx, level), lo, hi, ctx->noalloc_partial, out, ctx->stream));
  return LBM_OK;
}

lbm_status lbm_check_finite(lbm_ctx* ctx) {
  if (!ctx) return LBM_EINVAL;
  int32_t* flag = ctx->m<int32_t>(ctx->lay.flag);
  HIPCHK(ctx, launch_fill_i32(flag, 0, 1, ctx->stream));
  for (int l = 0; l < ctx->G.L; ++l) HIPCHK(ctx, launch_finite(io_of(ctx, l), flag, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(ctx->host_counts, flag, 4, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->host_counts[0]) return ctx->fail(LBM_ENAN, "non-finite moments");
  return LBM_OK;
}

size_t lbm_state_bytes(const lbm_ctx* ctx) {
  if (!ctx) return 0;
  return kStateHeader + (size_t)total_blocks(ctx) * block_bytes(ctx);
}

lbm_status lbm_save(lbm_ctx* ctx, void* dst, size_t bytes) {
  if (!ctx) return LBM_EINVAL;
  if (lbm_status st = need_boundary(ctx)) return st;
  if (!dst || bytes < lbm_state_bytes(ctx)) return ctx->fail(LBM_EINVAL, "state buffer missing or too small");
  Words8 w;
  std::memset(&w, 0, sizeof(w));
  w.v[0] = kStateMagic;
  w.v[1] = ctx->generation;
  w.v[2] = (uint64_t)ctx->G.L;
  w.v[3] = (uint64_t)total_blocks(ctx);
  w.v[4] = (uint64_t)ctx->elem;
  HIPCHK(ctx, launch_write_words(static_cast<uint64_t*>(dst), w, ctx->stream));
  char* p = static_cast<char*>(dst) + kStateHeader;
  for (int l = 0; l < ctx->G.L; ++l) {
    HIPCHK(ctx, launch_gather_blocks(ctx->cur(l), p, ctx->blocks(l), (int32_t)ctx->nblk[l], block_bytes(ctx),
                                     ctx->stream));
    p += (size_t)ctx->nblk[l] * block_bytes(ctx);
  }
  return LBM_OK;
}

lbm_status lbm_load(lbm_ctx* ctx, const void* src, size_t bytes) {
  if (!ctx) return LBM_EINVAL;
  if (lbm_status st = need_boundary(ctx)) return st;
  if (ctx->rec_open) return ctx->fail(LBM_ESTATE, "a recording is open (lbm_record_end first)");
  if (!src || bytes < lbm_state_bytes(ctx)) return ctx->fail(LBM_EINVAL, "state buffer missing or too small");
  HIPCHK(ctx, hipMemcpyAsync(ctx->host_counts, src, 64, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const uint64_t* w = reinterpret_cast<const uint64_t*>(ctx->host_counts);
  if (w[0] != kStateMagic || w[2] != (uint64_t)ctx->G.L || w[4] != (uint64_t)ctx->elem)
    return ctx->fail(LBM_ESTATE, "not a state of this simulation");
  if (w[1] != ctx->generation || w[3] != (uint64_t)total_blocks(ctx))
    return ctx->fail(LBM_ESTATE, "state was saved under another block hierarchy");
  ctx->rec_work = nullptr;
  const char* p = static_cast<const char*>(src) + kStateHeader;
  for (int l = 0; l < ctx->G.L; ++l) {
    HIPCHK(ctx, launch_scatter_blocks(p, ctx->cur(l), ctx->blocks(l), (int32_t)ctx->nblk[l], block_bytes(ctx),
                                      ctx->stream));
    p += (size_t)ctx->nblk[l] * block_bytes(ctx);
  }
  return LBM_OK;
}

size_t lbm_adjoint_work_bytes(const lbm_ctx* ctx, int32_t n_steps) {
  if (!ctx || n_steps < 1) return 0;
  return kAdjSlotBufs * slot_floats(ctx) * sizeof(float) + aux_bytes(ctx) + (size_t)n_steps * tape_bytes(ctx);
}

lbm_status lbm_adjoint_step(lbm_ctx* ctx, const void* state, size_t state_bytes, const float* lam_next, float* lam_out,
                            void* work, size_t work_bytes) {
  return lbm_adjoint_steps(ctx, state, state_bytes, 1, lam_next, lam_out, work, work_bytes);
}

lbm_status lbm_adjoint_steps(lbm_ctx* ctx, const void* state, size_t state_bytes, int32_t n_steps,
                             const float* lam_next, float* lam_out, void* work, size_t work_bytes) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->cfg.coupling) return ctx->fail(LBM_EINVAL, "the adjoint does not cover coupling fields");
  if (n_steps < 1) return ctx->fail(LBM_EINVAL, "step count must be positive");
  if (!lam_next || !lam_out || !work) return ctx->fail(LBM_EINVAL, "null adjoint buffer");
  if (work_bytes < lbm_adjoint_work_bytes(ctx, n_steps)) return ctx->fail(LBM_EINVAL, "adjoint work buffer too small");
  lbm_status st = lbm_load(ctx, state, state_bytes);
  if (st != LBM_OK) return st;
  if ((st = lbm_step_record(ctx, n_steps, work, work_bytes)) != LBM_OK) return st;
  return lbm_adjoint_reverse(ctx, lam_next, lam_out, work, work_bytes);
}

lbm_status lbm_step_record(lbm_ctx* ctx, int32_t n_steps, void* work, size_t work_bytes) {
  if (!ctx) return LBM_EINVAL;
  if (lbm_status st = need_boundary(ctx)) return st;
  if (ctx->cfg.coupling) return ctx->fail(LBM_EINVAL, "the adjoint does not cover coupling fields");
  if (n_steps < 1) return ctx->fail(LBM_EINVAL, "step count must be positive");
  if (!work) return ctx->fail(LBM_EINVAL, "null adjoint buffer");
  if (work_bytes < lbm_adjoint_work_bytes(ctx, n_steps)) return ctx->fail(LBM_EINVAL, "adjoint work buffer too small");
  if (ctx->rec_open) return ctx->fail(LBM_ESTATE, "a recording is open (lbm_record_end first)");
  const int L = ctx->G.L;
  const size_t sf = slot_floats(ctx);
  char* aux = reinterpret_cast<char*>(static_cast<float*>(work) + kAdjSlotBufs * sf);
  ctx->rec_aux = aux_bytes(ctx);
  ctx->tape = aux + ctx->rec_aux;
  ctx->tape_cap = work_bytes - kAdjSlotBufs * sf * sizeof(float) - ctx->rec_aux;
  ctx->tape_used = 0;
  ctx->ops.clear();
  ctx->hier_saves.clear();
  ctx->pending_sc_tape = SIZE_MAX;
  ctx->rec_work = work;
  ctx->rec_generation = ctx->generation;
  for (int l = 0; l < L; ++l) ctx->rec_parity[l] = ctx->parity[l];
  // the coarse steps, each forward kernel keeping the old value of what it overwrites
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  ctx->recording = true;
  lbm_status st = LBM_OK;
  for (int32_t i = 0; i < n_steps && st == LBM_OK; ++i) st = advance(ctx, L - 1, 1);
  ctx->recording = false;
  ctx->profiling = prof;
  if (st != LBM_OK) {
    ctx->ops.clear();
    ctx->rec_work = nullptr;
  }
  return st;
}

lbm_status lbm_adjoint_reverse(lbm_ctx* ctx, const float* lam_next, float* lam_out, void* work, size_t work_bytes) {
  if (!ctx) return LBM_EINVAL;
  if (lbm_status st = need_boundary(ctx)) return st;
  if (!lam_next || !lam_out || !work) return ctx->fail(LBM_EINVAL, "null adjoint buffer");
  if (ctx->rec_open) return ctx->fail(LBM_ESTATE, "a recording is open (lbm_record_end first)");
  if (ctx->rec_work == nullptr || ctx->ops.empty() || work != ctx->rec_work)
    return ctx->fail(LBM_ESTATE, "no recorded steps for this work buffer");
  if (ctx->rec_generation != ctx->generation)
    return ctx->fail(LBM_ESTATE, "the block hierarchy changed since the steps were recorded");
  if (work_bytes < kAdjSlotBufs * slot_floats(ctx) * sizeof(float) + ctx->rec_aux + ctx->tape_used)
    return ctx->fail(LBM_EINVAL, "adjoint work buffer too small");
  hipStream_t s = ctx->stream;
  const int L = ctx->G.L;
  const size_t sf = slot_floats(ctx);
  AdjBufs b;
  b.lam[0] = static_cast<float*>(work);
  b.lam[1] = b.lam[0] + sf;
  b.mu[0] = b.lam[1] + sf;
  b.mu[1] = b.mu[0] + sf;
  char* aux = reinterpret_cast<char*>(b.mu[1] + sf);
  // the partials take what the gidx and flag tables (sized by the capacity) leave
  const size_t tables = round256((size_t)(ctx->cap + 1) * 4) + round256((size_t)(ctx->cap + 1));
  b.part = reinterpret_cast<float*>(aux);
  b.gidx = reinterpret_cast<int32_t*>(aux + ctx->rec_aux - tables);
  b.flags = reinterpret_cast<uint8_t*>(aux + ctx->rec_aux - tables + round256((size_t)(ctx->cap + 1) * 4));
  ctx->tape = aux + ctx->rec_aux;
  lbm_status st = LBM_OK;
  {
    // adjoint of the state after the steps: lam_next at the state nodes of the current time level
    for (int k = 0; k < 2; ++k)
      HIPCHK(ctx, launch_fill_i32(reinterpret_cast<int32_t*>(b.mu[k] + (size_t)ctx->cap * kBlockStride), 0, kBlockStride, s));
    if ((st = adjoint_tables(ctx, b)) != LBM_OK) return st;
    // with grid updates in the log, blocks of earlier hierarchies receive adjoint too:
    // every slot starts at zero
    if (!ctx->hier_saves.empty())
      for (int k = 0; k < 2; ++k)
        HIPCHK(ctx, launch_fill_i32(reinterpret_cast<int32_t*>(b.lam[k]), 0, (int64_t)sf, s));
    size_t off = 0;
    for (int l = 0; l < L; ++l) {
      const int32_t n = (int32_t)ctx->nblk[l];
      HIPCHK(ctx, launch_zero_blocks(b.lam[1 - ctx->parity[l]], ctx->blocks(l), n, s));
      HIPCHK(ctx, launch_lam_scatter(lam_next + off, b.lam[ctx->parity[l]], ctx->blocks(l), ctx->role(ctx->rcur), n, s));
      off += (size_t)n * kBlockStride;
    }
  }
  // reverse sweep over every logged operation of every step (a failure leaves the
  // simulation state undefined: the undo is part of the adjoint kernels)
  AdjSweep sw;
  for (size_t i = ctx->ops.size(); st == LBM_OK && i-- > 0;)
    st = adjoint_op(ctx, ctx->ops[i], i > 0 ? &ctx->ops[i - 1] : nullptr, b, sw);
  for (int l = 0; l < L; ++l) ctx->parity[l] = ctx->rec_parity[l];
  ctx->ops.clear();
  ctx->hier_saves.clear();
  ctx->rec_work = nullptr;
  ctx->tape = nullptr;
  ctx->tape_cap = 0;
  if (st != LBM_OK) return st;
  size_t off = 0;
  for (int l = 0; l < L; ++l) {
    const int32_t n = (int32_t)ctx->nblk[l];
    HIPCHK(ctx, launch_gather_blocks(b.lam[ctx->parity[l]], lam_out + off, ctx->blocks(l), n,
                                     kBlockStride * sizeof(float), s));
    off += (size_t)n * kBlockStride;
  }
  return LBM_OK;
}

size_t lbm_record_work_bytes(const lbm_ctx* ctx, int32_t n_steps, int32_t n_updates) {
  if (!ctx || n_steps < 0 || n_updates < 0) return 0;
  const size_t state = (size_t)total_blocks(ctx) * 2 * block_bytes(ctx);
  return kAdjSlotBufs * slot_floats(ctx) * sizeof(float) + aux_bytes_cap(ctx) + (size_t)n_steps * tape_bytes(ctx) +
         (size_t)n_updates * (round256(ctx->lay.total) + state);
}

lbm_status lbm_record_begin(lbm_ctx* ctx, void* work, size_t work_bytes) {
  if (!ctx) return LBM_EINVAL;
  if (lbm_status st = need_boundary(ctx)) return st;
  if (ctx->cfg.coupling) return ctx->fail(LBM_EINVAL, "the adjoint does not cover coupling fields");
  if (ctx->rec_open) return ctx->fail(LBM_ESTATE, "a recording is already open");
  if (!work) return ctx->fail(LBM_EINVAL, "null adjoint buffer");
  const size_t fixed = kAdjSlotBufs * slot_floats(ctx) * sizeof(float) + aux_bytes_cap(ctx);
  if (work_bytes < fixed) return ctx->fail(LBM_EINVAL, "adjoint work buffer too small");
  char* aux = reinterpret_cast<char*>(static_cast<float*>(work) + kAdjSlotBufs * slot_floats(ctx));
  ctx->rec_aux = aux_bytes_cap(ctx);
  ctx->tape = aux + ctx->rec_aux;
  ctx->tape_cap = work_bytes - fixed;
  ctx->tape_used = 0;
  ctx->ops.clear();
  ctx->hier_saves.clear();
  ctx->pending_sc_tape = SIZE_MAX;
  ctx->rec_work = work;
  for (int l = 0; l < ctx->G.L; ++l) ctx->rec_parity[l] = ctx->parity[l];
  ctx->recording = true;
  ctx->rec_open = true;
  return LBM_OK;
}

lbm_status lbm_record_end(lbm_ctx* ctx) {
  if (!ctx) return LBM_EINVAL;
  if (!ctx->rec_open) return ctx->fail(LBM_ESTATE, "no recording is open");
  ctx->recording = false;
  ctx->rec_open = false;
  ctx->rec_generation = ctx->generation;
  if (ctx->ops.empty()) ctx->rec_work = nullptr;
  return LBM_OK;
}

lbm_status lbm_loss_ke_grad(lbm_ctx* ctx, int32_t level, const int32_t lo[3], const int32_t hi[3], float* lam) {
  if (!level_ok(ctx, level) || !lo || !hi || !lam) return ctx ? ctx->fail(LBM_EINVAL, "bad arguments") : LBM_EINVAL;
  HIPCHK(ctx, launch_fill_i32(reinterpret_cast<int32_t*>(lam), 0, total_blocks(ctx) * kBlockStride, ctx->stream));
  size_t off = 0;
  for (int l = 0; l < level; ++l) off += (size_t)ctx->nblk[l] * kBlockStride;
  AdjTransferLaunch t = adj_base(ctx, level);
  t.blocks = ctx->blocks(level);
  t.nblocks = (int32_t)ctx->nblk[level];
  t.src_a = ctx->cur(level);
  HIPCHK(ctx, launch_loss_ke_grad(t, lam + off, lo, hi, ctx->stream));
  return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
