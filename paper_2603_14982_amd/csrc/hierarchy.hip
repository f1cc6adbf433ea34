// Block hierarchy: level selection, refine/coarsen/delete flags, order-preserving
// compaction, slot allocation, node roles, neighbour table and the
// initialisation of new nodes (Sec. 5.4 Phi, Sec. 6.1-6.3).
//
// The target hierarchy H(Phi) is written as set algebra on dense per-level flag
// grids (one byte per block position):
//   T_0 = level-0 blocks holding a particle or a solid node       (Phi = 0 there)
//   D_1 = parent(T_0),  B_l = N26(D_l) \ D_l,  D_{l+1} = parent(D_l u B_l)
//   active_l = children(D_{l+1} u B_{l+1}) \ D_l   (top level: everything \ D_{L-1})
// D_l are the blocks deleted because the finer level covers them; B_l is the
// one-block overlap ring. The refine / coarsen / delete decisions of Sec. 6.3 are
// the differences between the new and the current states of each position.
// Lists are produced by wavefront ballots + a device prefix scan, visiting block
// positions in Morton order so every list comes out sorted by key.
#include "common.h"
#include "kernels.h"

namespace lbmx {
namespace {

constexpr uint8_t F_D = 1, F_B = 2;

__device__ inline bool in_level(const LevelGeom& g, int x, int y, int z) {
  return x >= 0 && y >= 0 && z >= 0 && x < g.nb[0] && y < g.nb[1] && z < g.nb[2];
}

// ---------------------------------------------------------------- level-0 targets
__global__ void k_mark_static(Geom G, const uint8_t* solid, uint8_t* t0s) {
  const LevelGeom& g = G.lv[0];
  const int64_t cell = blockIdx.x;
  const int bx = (int)(cell % g.nb[0]), by = (int)((cell / g.nb[0]) % g.nb[1]), bz = (int)(cell / ((int64_t)g.nb[0] * g.nb[1]));
  int any = 0;
  for (int n = threadIdx.x; n < kNodes; n += blockDim.x) {
    const int64_t x = bx * kEdge + (n & 7), y = by * kEdge + ((n >> 3) & 7), z = bz * kEdge + (n >> 6);
    any |= solid[x + (int64_t)G.N[0] * (y + (int64_t)G.N[1] * z)] != 0;
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) t0s[cell] = any ? 1 : 0;
}

// dst = src (or zero); with a flag, the flag is cleared too
__global__ void k_copy_or_clear(uint8_t* dst, const uint8_t* src, int64_t n, int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src ? src[i] : 0;
  if (flag && i == 0) *flag = 0;
}

// the level-0 block position of a particle into the target set (particles outside a
// non-periodic domain mark nothing)
__device__ __forceinline__ void mark_particle(const Geom& G, const float q[3], uint8_t* t0) {
  const LevelGeom& g = G.lv[0];
  int b[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!G.periodic[a] && !(q[a] >= 0.0f && q[a] < (float)G.N[a])) return;
    int v = (int)floorf(q[a] * 0.125f);
    if (G.periodic[a]) {
      v %= g.nb[a];
      if (v < 0) v += g.nb[a];
    }
    b[a] = v;
  }
  t0[cell_lin(g, b[0], b[1], b[2])] = 1;
}

__global__ void k_mark_particles(Geom G, const float* p, int64_t n, uint8_t* t0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float q[3] = {p[3 * i], p[3 * i + 1], p[3 * i + 2]};
  mark_particle(G, q, t0);
}

// the particles moved by d (rounded like the separate advance) and marked at their new
// positions, in one pass
__global__ void k_advance_mark(Geom G, float* p, int64_t n, float dx, float dy, float dz, uint8_t* t0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float q[3] = {__fadd_rn(p[3 * i], dx), __fadd_rn(p[3 * i + 1], dy), __fadd_rn(p[3 * i + 2], dz)};
  p[3 * i] = q[0];
  p[3 * i + 1] = q[1];
  p[3 * i + 2] = q[2];
  mark_particle(G, q, t0);
}

// D_l from the finer level: any child flagged (T_0 for l = 1, D|B for l > 1)
__global__ void k_deleted(Geom G, int l, const uint8_t* finer, uint8_t mask, uint8_t* flags_l) {
  const LevelGeom& g = G.lv[l];
  const LevelGeom& f = G.lv[l - 1];
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  const int bx = (int)(cell % g.nb[0]), by = (int)((cell / g.nb[0]) % g.nb[1]), bz = (int)(cell / ((int64_t)g.nb[0] * g.nb[1]));
  uint8_t any = 0;
  for (int c = 0; c < 8; ++c)
    any |= finer[cell_lin(f, 2 * bx + (c & 1), 2 * by + ((c >> 1) & 1), 2 * bz + (c >> 2))] & mask;
  flags_l[cell] = any ? F_D : 0;
}

// B_l = N26(D_l) \ D_l
__global__ void k_ring(Geom G, int l, uint8_t* flags_l) {
  const LevelGeom& g = G.lv[l];
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  const uint8_t own = flags_l[cell] & F_D;
  if (own) return;
  const int b[3] = {(int)(cell % g.nb[0]), (int)((cell / g.nb[0]) % g.nb[1]), (int)(cell / ((int64_t)g.nb[0] * g.nb[1]))};
  bool ring = false;
  for (int d = 0; d < 27 && !ring; ++d) {
    if (d == 13) continue;
    int h[3] = {b[0] + d % 3 - 1, b[1] + (d / 3) % 3 - 1, b[2] + d / 9 - 1};
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
      if (h[a] < 0 || h[a] >= g.nb[a]) {
        if (!G.periodic[a]) { ok = false; break; }
        h[a] = h[a] < 0 ? h[a] + g.nb[a] : h[a] - g.nb[a];
      }
    }
    if (ok && (flags_l[cell_lin(g, h[0], h[1], h[2])] & F_D)) ring = true;
  }
  if (ring) flags_l[cell] = F_B;
}

// every cell of every level (all-level index gi): deleted if covered by finer blocks,
// active on the coarsest level or where the parent position is covered or on a ring,
// absent otherwise; with a flag, a wave holding a cell whose state changes writes tag
__global__ void k_state(Geom G, const uint8_t* flags, uint8_t* st_new, const uint8_t* st_old, int64_t ntot,
                        int32_t* flag, int32_t tag) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool changed = false;
  if (gi < ntot) {
    int l = 0;
    while (l + 1 < G.L && gi >= G.lv[l + 1].off) ++l;
    const LevelGeom& g = G.lv[l];
    const int64_t cell = gi - g.off;
    uint8_t s;
    if (l >= 1 && (flags[gi] & F_D)) {
      s = ST_DELETED;
    } else if (l == G.L - 1) {
      s = ST_ACTIVE;
    } else {
      const LevelGeom& u = G.lv[l + 1];
      const int bx = (int)(cell % g.nb[0]), by = (int)((cell / g.nb[0]) % g.nb[1]),
                bz = (int)(cell / ((int64_t)g.nb[0] * g.nb[1]));
      s = (flags[u.off + cell_lin(u, bx >> 1, by >> 1, bz >> 1)] & (F_D | F_B)) ? ST_ACTIVE : ST_ABSENT;
    }
    st_new[gi] = s;
    changed = flag && s != st_old[gi];
  }
  if (flag && __ballot(changed) != 0ull && (threadIdx.x & 63) == 0) *flag = tag;
}

// any block position of any level whose state changes -> flag = 1
__global__ void k_diff(const uint8_t* st_new, const uint8_t* st_old, int64_t n, int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool d = i < n && st_new[i] != st_old[i];
  if (__ballot(d) != 0ull && (threadIdx.x & 63) == 0) *flag = 1;
}

// ---------------------------------------------------------------- compaction
// Each wave evaluates the predicates on 64 consecutive items of one segment, counts
// them with ballots, a single-workgroup scan turns every segment's wave counts into
// offsets, and the scatter pass writes every selected item at offset + rank-in-wave.
// Segment s takes waves [wave0[s], wave0[s + 1]); its counts sit at NP wave0[s] +
// k (wave0[s + 1] - wave0[s]) + wave for predicate k.
struct SegWaves {
  int nseg;
  int64_t wave0[kMaxSegs + 1];
  int64_t nitems[kMaxSegs];
};
struct SegCounts {
  int32_t* c[kMaxSegs][2];  // totals of predicates 0..2, then 3..5
};

__device__ __forceinline__ int seg_of(const SegWaves& q, int64_t wave) {
  int s = 0;
  while (s + 1 < q.nseg && wave >= q.wave0[s + 1]) ++s;
  return s;
}

__device__ inline void cell_preds(const Geom& G, int l, int64_t t, const uint8_t* st_new, const uint8_t* st_old,
                                  uint32_t& bits, int32_t& lin) {
  const LevelGeom& g = G.lv[l];
  int x, y, z;
  morton_decode3((uint64_t)t, x, y, z);
  bits = 0;
  lin = -1;
  if (!in_level(g, x, y, z)) return;
  lin = (int32_t)cell_lin(g, x, y, z);
  const bool a = st_new[g.off + lin] == ST_ACTIVE;
  const bool o = st_old[g.off + lin] == ST_ACTIVE;
  bits = (a ? 1u : 0u) | ((a && !o) ? 2u : 0u) | ((o && !a) ? 4u : 0u);
}

__global__ void k_cells_count(CellSegs c, SegWaves q, int32_t* wcount) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wave = t >> 6;
  const int sg = seg_of(q, wave);
  const int64_t i = t - 64 * q.wave0[sg];
  uint32_t bits = 0;
  int32_t lin;
  if (i < q.nitems[sg]) cell_preds(c.G, c.level[sg], i, c.st_new, c.st_old, bits, lin);
  const int64_t nw = q.wave0[sg + 1] - q.wave0[sg], w = wave - q.wave0[sg];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint64_t m = __ballot((bits >> k) & 1u);
    if ((threadIdx.x & 63) == 0 && w < nw) wcount[3 * q.wave0[sg] + k * nw + w] = __popcll(m);
  }
}

__global__ void k_cells_scatter(CellSegs c, SegWaves q, const int32_t* woff) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wave = t >> 6;
  const int sg = seg_of(q, wave);
  const int64_t i = t - 64 * q.wave0[sg];
  uint32_t bits = 0;
  int32_t lin = -1;
  if (i < q.nitems[sg]) cell_preds(c.G, c.level[sg], i, c.st_new, c.st_old, bits, lin);
  const int64_t nw = q.wave0[sg + 1] - q.wave0[sg], w = wave - q.wave0[sg];
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const bool p = (bits >> k) & 1u;
    const uint64_t m = __ballot(p);
    int32_t* out = c.out[sg][k];
    if (p && out) out[woff[3 * q.wave0[sg] + k * nw + w] + __popcll(m & below)] = lin;
  }
}

__global__ void k_bytes_count(ByteSegs b, SegWaves q, int32_t* wcount) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wave = t >> 6;
  const int sg = seg_of(q, wave);
  const int64_t i = t - 64 * q.wave0[sg];
  const uint32_t bits = i < q.nitems[sg] ? (uint32_t)b.bytes[sg][b.items[sg][i]] : 0u;
  const int64_t nw = q.wave0[sg + 1] - q.wave0[sg], w = wave - q.wave0[sg];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const uint64_t m = __ballot((bits >> k) & 1u);
    if ((threadIdx.x & 63) == 0 && w < nw) wcount[6 * q.wave0[sg] + k * nw + w] = __popcll(m);
  }
}

__global__ void k_bytes_scatter(ByteSegs b, SegWaves q, const int32_t* woff) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wave = t >> 6;
  const int sg = seg_of(q, wave);
  const int64_t i = t - 64 * q.wave0[sg];
  const int32_t slot = i < q.nitems[sg] ? b.items[sg][i] : -1;
  const uint32_t bits = i < q.nitems[sg] ? (uint32_t)b.bytes[sg][slot] : 0u;
  const int64_t nw = q.wave0[sg + 1] - q.wave0[sg], w = wave - q.wave0[sg];
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const bool p = (bits >> k) & 1u;
    const uint64_t m = __ballot(p);
    int32_t* out = b.out[sg][k];
    if (p && out) out[woff[6 * q.wave0[sg] + k * nw + w] + __popcll(m & below)] = slot;
  }
}

// Exclusive scan (in place) of the NP arrays of wave counts of every segment; the totals
// go to c[s][0][0..2], then c[s][1][0..2]. Each (segment, predicate) array is scanned by
// one wave of the workgroup on its own, in chunks of 64 x 16 counts: each lane sums its
// 16 consecutive counts, the lane sums are scanned by cross-lane shifts, and a carry
// runs from chunk to chunk (no workgroup barrier: the waves share nothing).
__device__ __forceinline__ int32_t wave_inclusive_scan(int32_t v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}
template <int NP>
__global__ __launch_bounds__(1024) void k_scan(int32_t* w, SegWaves q, SegCounts tot) {
  constexpr int E = 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int job = wave; job < q.nseg * NP; job += 16) {
    const int sg = job / NP, k = job % NP;
    const int64_t nw = q.wave0[sg + 1] - q.wave0[sg];
    int32_t* a = w + NP * q.wave0[sg] + k * nw;
    int32_t carry = 0;
    for (int64_t base = 0; base < nw; base += 64 * E) {
      const int64_t i0 = base + (int64_t)lane * E;
      int32_t v[E];
      int32_t sum = 0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        v[e] = i0 + e < nw ? a[i0 + e] : 0;
        sum += v[e];
      }
      const int32_t inc = wave_inclusive_scan(sum, lane);
      int32_t run = carry + inc - sum;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (i0 + e < nw) a[i0 + e] = run;
        run += v[e];
      }
      carry += __shfl(inc, 63, 64);  // the chunk's total
    }
    int32_t* c = tot.c[sg][k / 3];
    if (lane == 0 && c) c[k % 3] = carry;
  }
}

// ---------------------------------------------------------------- slots
__global__ void k_alloc(AllocLaunch a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const LevelGeom& g = a.G.lv[a.level];
  const int32_t cell = a.cells[i];
  const int32_t slot = a.free_stack[a.free_top - 1 - i];
  a.dir_new[g.off + cell] = slot;
  const int bx = cell % g.nb[0], by = (cell / g.nb[0]) % g.nb[1], bz = cell / (g.nb[0] * g.nb[1]);
  a.coord[slot] = make_int4(bx, by, bz, a.level);
}

__global__ void k_release(const int32_t* cells, int32_t n, int64_t off, const int32_t* dir_old, int32_t* free_stack,
                          int32_t free_top, int32_t* dir_new) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t cell = cells[i];
  free_stack[free_top + i] = dir_old[off + cell];
  dir_new[off + cell] = NBR_NONE;
}

__global__ void k_copy_i32(const int32_t* src, int32_t* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
__global__ void k_fill_i32(int32_t* dst, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}
__global__ void k_fill_u8(uint8_t* dst, uint8_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

// ---------------------------------------------------------------- roles + neighbours
__device__ inline bool solid_at(const Geom& G, const uint8_t* solid, int l, int gx, int gy, int gz) {
  if (!solid) return false;
  const int64_t x = (int64_t)gx << l, y = (int64_t)gy << l, z = (int64_t)gz << l;
  return solid[x + (int64_t)G.N[0] * (y + (int64_t)G.N[1] * z)] != 0;
}

// The 27 block positions around a block, d = (ox + 1) + 3 (oy + 1) + 9 (oz + 1), as bits
// of a mask. The 26 neighbours of a node fall in the positions ox in {-1, 0} if its local
// x is 0, {0} if it is 1..6, {0, 1} if it is 7 (likewise y, z): reach_mask gives them.
__device__ __forceinline__ uint32_t reach_axis(int c) { return c == 0 ? 3u : (c == kEdge - 1 ? 6u : 2u); }
__device__ __forceinline__ uint32_t reach_mask(int lx, int ly, int lz) {
  const uint32_t ax = reach_axis(lx), ay = reach_axis(ly), az = reach_axis(lz);
  const uint32_t xm = ((ax & 1u) ? 0x1249249u : 0u) | ((ax & 2u) ? 0x2492492u : 0u) | ((ax & 4u) ? 0x4924924u : 0u);
  const uint32_t row = 0x7u | (0x7u << 9) | (0x7u << 18);  // positions with oy = -1
  const uint32_t ym = ((ay & 1u) ? row : 0u) | ((ay & 2u) ? row << 3 : 0u) | ((ay & 4u) ? row << 6 : 0u);
  const uint32_t zm = ((az & 1u) ? 0x1ffu : 0u) | ((az & 2u) ? 0x1ffu << 9 : 0u) | ((az & 4u) ? 0x1ffu << 18 : 0u);
  return xm & ym & zm & ~(1u << 13);
}

// Role of a node from its own position on a domain face (inflow, outflow) and from the
// block positions its 26 neighbours fall in (without a solid field): a neighbour in an
// absent block makes it a ghost node, one in a deleted block an interface node, one
// outside the domain across a wall a bounce-back node.
__device__ inline uint8_t mask_role(const Geom& G, const LevelGeom& g, const int b[3], int lx, int ly, int lz,
                                    uint32_t absent, uint32_t deleted, uint32_t wall) {
  const int lc[3] = {lx, ly, lz};
  for (int a = 0; a < 3; ++a) {
    if (G.periodic[a]) continue;
    const int gc = b[a] * kEdge + lc[a];
    int kind = -1;
    if (gc == 0) kind = G.bc[2 * a];
    else if (gc == g.nn[a] - 1) kind = G.bc[2 * a + 1];
    if (kind == BC_INFLOW) return ROLE_INFLOW;
    if (is_outflow_bc(kind)) return ROLE_OUTFLOW;
  }
  const uint32_t m = reach_mask(lx, ly, lz);
  if (absent & m) return ROLE_GHOST;
  if (deleted & m) return ROLE_IU;
  return (uint8_t)(ROLE_COMPUTED | ((wall & m) ? ROLE_BB : 0));
}

__device__ bool tile_exists(const LevelGeom& g, const uint8_t* st, int tx, int ty, int tz) {
  if (tz < 0 || 2 * tz >= g.nb[2]) return false;
  for (int m = 0; m < 4 * kTileX; ++m) {
    const int x = tx * kTileX + m % kTileX, y = 2 * ty + (m / kTileX) % 2, z = 2 * tz + m / (2 * kTileX);
    if (x < g.nb[0] && y < g.nb[1] && z < g.nb[2] && st[g.off + cell_lin(g, x, y, z)] == ST_ACTIVE) return true;
  }
  return false;
}

// run class of the tile at tile position (tx, ty, tz) if it starts a run: bit h - 1 for a
// run of h tiles, 0 if the tile continues the run of the tile below
__device__ uint8_t run_class_of(const LevelGeom& g, const uint8_t* st, int tx, int ty, int tz, int run_max) {
  if (tz % run_max != 0 && tile_exists(g, st, tx, ty, tz - 1)) return 0;
  int h = 1;
  while (h < run_max && (tz + h) % run_max != 0 && tile_exists(g, st, tx, ty, tz + h)) ++h;
  return (uint8_t)(1u << (h - 1));
}

// Role of a node by testing each of its 26 neighbours (with a solid field)
__device__ inline uint8_t test_role(const RoleLaunch& r, int l, const LevelGeom& g, const int b[3], int node,
                                    const uint8_t* s_st, const uint8_t* s_wall) {
  const Geom& G = r.G;
  const int lc[3] = {node & 7, (node >> 3) & 7, node >> 6};
  const int gc[3] = {b[0] * kEdge + lc[0], b[1] * kEdge + lc[1], b[2] * kEdge + lc[2]};
  if (solid_at(G, r.solid, l, gc[0], gc[1], gc[2])) return ROLE_SOLID;
  for (int a = 0; a < 3; ++a) {
    if (G.periodic[a]) continue;
    int kind = -1;
    if (gc[a] == 0) kind = G.bc[2 * a];
    else if (gc[a] == g.nn[a] - 1) kind = G.bc[2 * a + 1];
    if (kind == BC_INFLOW) return ROLE_INFLOW;
    if (is_outflow_bc(kind)) return ROLE_OUTFLOW;
  }
  bool ghost = false, iu = false, bb = false;
  for (int d = 0; d < 27; ++d) {
    if (d == 13) continue;
    const int dd[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
    int h[3], o[3];
    bool outside = false;
    for (int a = 0; a < 3; ++a) {
      const int v = lc[a] + dd[a];
      o[a] = v < 0 ? 0 : (v > 7 ? 2 : 1);
      h[a] = gc[a] + dd[a];
      if (h[a] < 0 || h[a] >= g.nn[a]) {
        if (G.periodic[a]) h[a] = h[a] < 0 ? h[a] + g.nn[a] : h[a] - g.nn[a];
        else outside = true;
      }
    }
    const int nd = o[0] + 3 * o[1] + 9 * o[2];
    if (outside) {
      if (s_wall[nd]) bb = true;
      continue;
    }
    const uint8_t stv = s_st[nd];
    if (stv == ST_ABSENT) ghost = true;
    else if (stv == ST_DELETED) iu = true;
    if (solid_at(G, r.solid, l, h[0], h[1], h[2])) bb = true;
  }
  return ghost ? ROLE_GHOST : (iu ? ROLE_IU : (uint8_t)(ROLE_COMPUTED | (bb ? ROLE_BB : 0)));
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// One 64-lane wave per block, four blocks per workgroup. Lanes 0..26 look up the 27
// surrounding block positions (neighbour table, states); ballots turn their states into
// masks. Lane i owns the 8 nodes of row (y, z) = (i & 7, i >> 3) and writes them as one
// 8-byte word.
__global__ __launch_bounds__(256) void k_roles(RoleLaunch r) {
  __shared__ uint8_t s_st_w[4][32];    // per wave: state of the 27 positions (255 = outside)
  __shared__ uint8_t s_wall_w[4][32];  // per wave: outside the domain across wall faces only
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const Geom& G = r.G;
  int l = 0;
  while (l + 1 < G.L && (int32_t)blockIdx.x >= r.wg0[l + 1]) ++l;
  const LevelGeom& g = G.lv[l];
  const int64_t bi = (int64_t)(blockIdx.x - r.wg0[l]) * 4 + wv;
  uint8_t* s_st = s_st_w[wv];
  uint8_t* s_wall = s_wall_w[wv];
  const int32_t n = r.n[l];
  const int32_t cell = bi < n ? r.cells[l][bi] : 0;
  const int32_t slot = bi < n ? r.dir[g.off + cell] : -1;
  const bool valid = slot >= 0;  // every active cell holds a slot; never write out of bounds
  const int b[3] = {cell % g.nb[0], (cell / g.nb[0]) % g.nb[1], cell / (g.nb[0] * g.nb[1])};
  uint8_t stv = 255;
  bool wallpos = false, changed = false;
  if (valid && lane < 27) {
    const int d = lane;
    int h[3] = {b[0] + d % 3 - 1, b[1] + (d / 3) % 3 - 1, b[2] + d / 9 - 1};
    bool inside = true, wall = true;
    for (int a = 0; a < 3; ++a) {
      if (h[a] < 0 || h[a] >= g.nb[a]) {
        if (G.periodic[a]) {
          h[a] = h[a] < 0 ? h[a] + g.nb[a] : h[a] - g.nb[a];
        } else {
          inside = false;
          if (G.bc[2 * a + (h[a] < 0 ? 0 : 1)] != BC_WALL) wall = false;
        }
      }
    }
    int32_t ns = NBR_NONE;
    if (inside) {
      const int64_t hc = g.off + cell_lin(g, h[0], h[1], h[2]);
      stv = r.st[hc];
      if (stv == ST_ACTIVE) ns = r.dir[hc];
      changed = r.st_old[hc] != stv;
    } else if (wall) {
      ns = NBR_WALL;
    }
    wallpos = !inside && wall;
    s_st[d] = stv;
    s_wall[d] = wallpos ? 1 : 0;
    r.nbr[(size_t)slot * 27 + d] = ns;
  }
  __syncthreads();  // the per-wave position tables (read by the per-neighbour test)
  if (!valid) return;
  if (lane == 0) r.blocks[l][bi] = slot;
  const uint32_t active = (uint32_t)__ballot(lane < 27 && stv == ST_ACTIVE);
  const uint32_t absent = (uint32_t)__ballot(lane < 27 && stv == ST_ABSENT);
  const uint32_t deleted = (uint32_t)__ballot(lane < 27 && stv == ST_DELETED);
  const uint32_t wall = (uint32_t)__ballot(lane < 27 && wallpos);
  const bool any_changed = __ballot(lane < 27 && changed) != 0ull;

  const int ly = lane & 7, lz = lane >> 3;
  uint8_t rl[8];
  if (r.solid == nullptr) {
    // a block whose 26 neighbour positions all hold active blocks has only computed
    // nodes; otherwise nodes 1..6 of the row share one role
    if (active == 0x7ffffffu) {
#pragma unroll
      for (int i = 0; i < 8; ++i) rl[i] = ROLE_COMPUTED;
    } else {
      const uint8_t r0 = mask_role(G, g, b, 0, ly, lz, absent, deleted, wall);
      const uint8_t r1 = mask_role(G, g, b, 1, ly, lz, absent, deleted, wall);
      const uint8_t r7 = mask_role(G, g, b, 7, ly, lz, absent, deleted, wall);
      rl[0] = r0;
#pragma unroll
      for (int i = 1; i < 7; ++i) rl[i] = r1;
      rl[7] = r7;
    }
  } else {
#pragma unroll 1
    for (int i = 0; i < 8; ++i) rl[i] = test_role(r, l, g, b, 8 * lane + i, s_st, s_wall);
  }
  uint64_t word = 0;
  uint8_t sum = 0;
  int lo[3] = {kEdge, kEdge, kEdge}, hi[3] = {-1, -1, -1};
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    word |= (uint64_t)rl[i] << (8 * i);
    const uint8_t rk = rl[i] & ROLE_MASK;
    if (rk == ROLE_GHOST) {
      const int lc[3] = {i, ly, lz};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = min(lo[a], lc[a]);
        hi[a] = max(hi[a], lc[a]);
      }
    }
    sum |= rk == ROLE_GHOST ? SUM_GHOST : (rk == ROLE_IU ? SUM_IU : (rk == ROLE_OUTFLOW ? SUM_OUTFLOW : 0));
    if (rl[i] & ROLE_BB) sum |= SUM_BB;
  }
  *reinterpret_cast<uint64_t*>(r.role + (size_t)slot * kNodes + 8 * lane) = word;
  const bool any_g = __ballot(sum & SUM_GHOST) != 0ull;
  const bool any_i = __ballot(sum & SUM_IU) != 0ull;
  const bool any_o = __ballot(sum & SUM_OUTFLOW) != 0ull;
  const bool any_b = __ballot(sum & SUM_BB) != 0ull;
  // ghost-node bounding box (all-ghost-free blocks keep lo 7, hi 0)
  int box[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    box[a] = min(wave_min(lo[a]), 7);
    box[3 + a] = max(wave_max(hi[a]), 0);
  }
  if (lane == 0) {
    // one representative per stream-collide tile of kTileX x 2 x 2 blocks: the
    // active member with the lowest index (x fastest); members are never wrapped
    const int c = (b[0] & (kTileX - 1)) + kTileX * ((b[1] & 1) + 2 * (b[2] & 1));
    bool start = true;
    for (int m = 0; m < c; ++m) {
      const int mx = (b[0] & ~(kTileX - 1)) + m % kTileX, my = (b[1] & ~1) + (m / kTileX) % 2,
                mz = (b[2] & ~1) + m / (2 * kTileX);
      if (mx < g.nb[0] && my < g.nb[1] && mz < g.nb[2] && r.st[g.off + cell_lin(g, mx, my, mz)] == ST_ACTIVE)
        start = false;
    }
    r.summary[slot] = (any_g ? SUM_GHOST : 0) | (any_i ? SUM_IU : 0) | (any_o ? SUM_OUTFLOW : 0) |
                      (start ? SUM_TILE : 0) | (any_b ? SUM_BB : 0) | (any_changed ? SUM_FRESH : 0);
    // the finest level's tiles: the z-run class of a tile head (two-substep sweep)
    if (l == 0 && r.run_class)
      r.run_class[slot] = start ? run_class_of(g, r.st, b[0] / kTileX, b[1] >> 1, b[2] >> 1, r.run_max) : 0;
    r.gbox[slot] = box[0] | box[3] << 3 | box[1] << 6 | box[4] << 9 | box[2] << 12 | box[5] << 15;
  }
}

// ---------------------------------------------------------------- z runs of tiles
// The two-substep sweep of the finest level (Alg. 1, both fine substeps of a parent
// step in one pass) reads every plane of a tile with a two-node halo and recomputes a
// one-node ring of the first substep; a workgroup that sweeps several tiles stacked
// along z reads and recomputes the planes at their shared faces once. Runs break below
// a missing tile and at tile positions z = 0 (mod run_max), so that a run is found from
// its first tile alone.
__global__ void k_tile_runs(Geom G, int level, const int32_t* blocks, int32_t n, const uint8_t* summary,
                            const uint8_t* st, const int4* coord, int run_max, uint8_t* run_class) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int32_t slot = blocks[t];
  uint8_t cls = 0;
  if (summary[slot] & SUM_TILE) {
    const int4 c = coord[slot];
    cls = run_class_of(G.lv[level], st, c.x / kTileX, c.y >> 1, c.z >> 1, run_max);
  }
  run_class[slot] = cls;
}

// ---------------------------------------------------------------- new-node initialisation
// Value of level-l node g in the old hierarchy, as a linear combination in
// (rho-1, u, S^neq) of old owned nodes with weight w and S^neq factor sf: the node's
// own value if owned; else the nearest finer level owning the coincident node
// (upward, S^neq times a_up per level); else trilinear from level l+1 (downward,
// times a_down). visit() hands every source node with its weight and factor to fn.
template <class S> struct Sampler {
  const InitLaunch& a;
  __device__ explicit Sampler(const InitLaunch& x) : a(x) {}

  // slot and node of level-k node (gx, gy, gz) if the old hierarchy owns it
  __device__ bool source(int k, int gx, int gy, int gz, int32_t& slot, int& node) const {
    const LevelGeom& g = a.G.lv[k];
    const int64_t c = g.off + cell_lin(g, gx >> 3, gy >> 3, gz >> 3);
    if (a.st_old[c] != ST_ACTIVE) return false;
    slot = a.dir_old[c];
    if (slot < 0) return false;
    node = (gx & 7) + 8 * (gy & 7) + 64 * (gz & 7);
    const uint8_t r = a.role_old[(size_t)slot * kNodes + node] & ROLE_MASK;
    return r == ROLE_COMPUTED || r == ROLE_IU || r == ROLE_INFLOW || r == ROLE_OUTFLOW;
  }
  __device__ void load(int k, int32_t slot, int node, float q[kMom]) const {
    const typename S::type* p = static_cast<const typename S::type*>(a.cur[k]) + (size_t)slot * kBlockStride + node;
#pragma unroll
    for (int m = 0; m < kMom; ++m) q[m] = Codec<S>::load(p[m * kNodes], a.sc.inv[m]);
  }

  template <class F> __device__ bool upchain(int l, const int g[3], float w, float sf, F& fn) const {
    float f = sf;
    for (int k = l; k >= 0; --k) {
      const int sh = l - k;
      int32_t slot;
      int node;
      if (source(k, g[0] << sh, g[1] << sh, g[2] << sh, slot, node)) {
        fn(k, slot, node, w, f);
        return true;
      }
      if (k > 0) f *= a.a_up[k - 1];
    }
    return false;
  }

  template <int D, class F>
  __device__ bool visit(int l, const int g[3], float w, float sf, F& fn) const {
    if (upchain(l, g, w, sf, fn)) return true;
    if constexpr (D == 0) {
      return false;
    } else {
      if (l + 1 >= a.G.L) return false;
      const LevelGeom& cg = a.G.lv[l + 1];
      int cand[3][2], cnt[3];
      float wv[3][2];
      for (int ax = 0; ax < 3; ++ax) {
        const int nc = cg.nn[ax];
        if ((g[ax] & 1) == 0) { cand[ax][0] = g[ax] >> 1; wv[ax][0] = 1.0f; cnt[ax] = 1; }
        else { cand[ax][0] = (g[ax] - 1) >> 1; cand[ax][1] = (g[ax] + 1) >> 1; wv[ax][0] = wv[ax][1] = 0.5f; cnt[ax] = 2; }
        for (int k = 0; k < cnt[ax]; ++k) {
          int v = cand[ax][k];
          if (a.G.periodic[ax]) v = v < 0 ? v + nc : (v >= nc ? v - nc : v);
          else v = v < 0 ? 0 : (v >= nc ? nc - 1 : v);
          cand[ax][k] = v;
        }
      }
      bool ok = true;
      for (int kz = 0; kz < cnt[2]; ++kz)
        for (int ky = 0; ky < cnt[1]; ++ky)
          for (int kx = 0; kx < cnt[0]; ++kx) {
            const int j[3] = {cand[0][kx], cand[1][ky], cand[2][kz]};
            ok = visit<D - 1>(l + 1, j, w * wv[0][kx] * wv[1][ky] * wv[2][kz], sf * a.a_down[l], fn) && ok;
          }
      return ok;
    }
  }

  // accumulated (rho-1, u, S^neq) of V_old(l, g)
  __device__ void sample(int l, const int g[3], float acc[kMom]) const {
#pragma unroll
    for (int m = 0; m < kMom; ++m) acc[m] = 0.0f;
    auto add = [&](int k, int32_t slot, int node, float w, float f) {
      float q[kMom];
      load(k, slot, node, q);
      acc[0] += w * q[0];
      acc[1] += w * q[1]; acc[2] += w * q[2]; acc[3] += w * q[3];
      const float ws = w * f;
      acc[4] += ws * (q[4] - q[1] * q[1]); acc[5] += ws * (q[5] - q[2] * q[2]); acc[6] += ws * (q[6] - q[3] * q[3]);
      acc[7] += ws * (q[7] - q[1] * q[2]); acc[8] += ws * (q[8] - q[1] * q[3]); acc[9] += ws * (q[9] - q[2] * q[3]);
    };
    visit<kMaxLevels - 1>(l, g, 1.0f, 1.0f, add);
  }
};

// the nodes a grid update writes in a block of the new hierarchy: every node of a new
// block, and the nodes of a surviving block that become owned
__device__ inline bool fresh_node(const InitLaunch& a, bool new_block, int32_t slot, int node, uint8_t rn) {
  if (new_block) return true;
  const uint8_t ro = a.role_old[(size_t)slot * kNodes + node] & ROLE_MASK;
  const bool own_old = ro == ROLE_COMPUTED || ro == ROLE_IU || ro == ROLE_INFLOW || ro == ROLE_OUTFLOW;
  const bool own_new = rn == ROLE_COMPUTED || rn == ROLE_IU || rn == ROLE_INFLOW || rn == ROLE_OUTFLOW;
  return !own_old && own_new;
}

template <class S>
__device__ void init_block(const InitLaunch& a, int32_t item) {
  const LevelGeom& g = a.G.lv[a.level];
  int32_t cell;
  if (a.cells) {
    cell = a.cells[item];
  } else {
    const int4 q = a.coord[a.slots[item]];
    cell = (int32_t)cell_lin(g, q.x, q.y, q.z);
  }
  const int32_t slot = a.dir_new[g.off + cell];
  if (slot < 0) return;  // every active cell holds a slot; never write out of bounds
  const bool new_block = a.create || a.st_old[g.off + cell] != ST_ACTIVE;
  const int b[3] = {cell % g.nb[0], (cell / g.nb[0]) % g.nb[1], cell / (g.nb[0] * g.nb[1])};
  typedef typename S::type T;
  T* cur = static_cast<T*>(a.dst_cur) + (size_t)slot * kBlockStride;
  T* oth = static_cast<T*>(a.dst_other) + (size_t)slot * kBlockStride;
  Sampler<S> smp(a);
  if (a.cpl && new_block) {
    // a new finest-level block starts with eps = 1, F = 0
    float* c = a.cpl + (size_t)slot * 4 * kNodes;
    for (int i = threadIdx.x; i < 4 * kNodes; i += 256) c[i] = i < kNodes ? 1.0f : 0.0f;
  }
  if (a.phi && new_block) {
    // and with no powder snow
    for (int i = threadIdx.x; i < kNodes; i += 256) a.phi[(size_t)slot * kNodes + i] = 0.0f;
  }
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    const uint8_t rn = a.role_new[(size_t)slot * kNodes + node] & ROLE_MASK;
    if (!fresh_node(a, new_block, slot, node, rn)) continue;
    float q[kMom];
#pragma unroll
    for (int m = 0; m < kMom; ++m) q[m] = 0.0f;
    if (rn == ROLE_INFLOW) {
      const int gn[3] = {b[0] * kEdge + (node & 7), b[1] * kEdge + ((node >> 3) & 7), b[2] * kEdge + (node >> 6)};
      inflow_velocity(a.G, a.level, gn, q + 1);
      q[4] = q[1] * q[1]; q[5] = q[2] * q[2]; q[6] = q[3] * q[3];
      q[7] = q[1] * q[2]; q[8] = q[1] * q[3]; q[9] = q[2] * q[3];
    } else if (rn != ROLE_SOLID && !a.create) {
      const int gn[3] = {b[0] * kEdge + (node & 7), b[1] * kEdge + ((node >> 3) & 7), b[2] * kEdge + (node >> 6)};
      float acc[kMom];
      smp.sample(a.level, gn, acc);
      q[0] = acc[0];
      q[1] = acc[1]; q[2] = acc[2]; q[3] = acc[3];
      q[4] = acc[4] + acc[1] * acc[1]; q[5] = acc[5] + acc[2] * acc[2]; q[6] = acc[6] + acc[3] * acc[3];
      q[7] = acc[7] + acc[1] * acc[2]; q[8] = acc[8] + acc[1] * acc[3]; q[9] = acc[9] + acc[2] * acc[3];
    }
#pragma unroll
    for (int m = 0; m < kMom; ++m) {
      const T v = Codec<S>::store(q[m], a.sc.s[m]);
      cur[m * kNodes + node] = v;
      oth[m * kNodes + node] = v;
    }
  }
}

// the blocks of every level's list, the grid striding over each (a list's length read
// from the device where a.n_dev is set)
struct InitLevels {
  InitLaunch a[kMaxLevels];
  int nlev;
};
template <class S>
__global__ __launch_bounds__(256) void k_init(InitLevels x) {
  for (int l = 0; l < x.nlev; ++l) {
    const InitLaunch& a = x.a[l];
    const int32_t n = a.n_dev ? *a.n_dev : a.n;
    for (int32_t i = blockIdx.x; i < n; i += gridDim.x) init_block<S>(a, i);
  }
}

// Adjoint of k_init (reverse sweep of a recorded grid update): the pool holds the old
// state again and the tables of both hierarchies are in place. For every node the
// update wrote, its adjoint (both time levels: the update wrote the same value into
// each) goes through the transposed sampler into the adjoint of the old nodes it was
// sampled from, and is then cleared. Sources are nodes the old hierarchy owns, written
// nodes are not, so the atomic adds never touch a node read in the same launch.
template <class S>
__global__ __launch_bounds__(256) void k_init_adj(InitAdjLaunch x) {
  const InitLaunch& a = x.f;
  const LevelGeom& g = a.G.lv[a.level];
  const int32_t cell = a.cells[blockIdx.x];
  const int32_t slot = a.dir_new[g.off + cell];
  if (slot < 0) return;
  const bool new_block = a.st_old[g.off + cell] != ST_ACTIVE;
  const int b[3] = {cell % g.nb[0], (cell / g.nb[0]) % g.nb[1], cell / (g.nb[0] * g.nb[1])};
  Sampler<S> smp(a);
  float* lc = x.lam[x.parity[a.level]] + (size_t)slot * kBlockStride;
  float* lo = x.lam[1 - x.parity[a.level]] + (size_t)slot * kBlockStride;
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    const uint8_t rn = a.role_new[(size_t)slot * kNodes + node] & ROLE_MASK;
    if (!fresh_node(a, new_block, slot, node, rn)) continue;
    if (rn != ROLE_INFLOW && rn != ROLE_SOLID) {
      const int gn[3] = {b[0] * kEdge + (node & 7), b[1] * kEdge + ((node >> 3) & 7), b[2] * kEdge + (node >> 6)};
      float acc[kMom], lq[kMom], la[kMom];
      smp.sample(a.level, gn, acc);
#pragma unroll
      for (int m = 0; m < kMom; ++m) lq[m] = lc[m * kNodes + node] + lo[m * kNodes + node];
      // q = (acc0, acc_u, acc_N + acc_u acc_u)
      la[0] = lq[0];
#pragma unroll
      for (int m = 4; m < kMom; ++m) la[m] = lq[m];
      la[1] = lq[1] + 2.0f * acc[1] * lq[4] + acc[2] * lq[7] + acc[3] * lq[8];
      la[2] = lq[2] + 2.0f * acc[2] * lq[5] + acc[1] * lq[7] + acc[3] * lq[9];
      la[3] = lq[3] + 2.0f * acc[3] * lq[6] + acc[1] * lq[8] + acc[2] * lq[9];
      // each source: (rho-1, u, f (S - u u)) with weight w
      auto scatter = [&](int k, int32_t s, int nd, float w, float f) {
        float q[kMom];
        smp.load(k, s, nd, q);
        float* t = x.lam[x.parity[k]] + (size_t)s * kBlockStride + nd;
        const float ws = w * f;
        float ln[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) ln[j] = ws * la[4 + j];
        atomicAdd(t, w * la[0]);
        atomicAdd(t + 1 * kNodes, w * la[1] - (2.0f * q[1] * ln[0] + q[2] * ln[3] + q[3] * ln[4]));
        atomicAdd(t + 2 * kNodes, w * la[2] - (2.0f * q[2] * ln[1] + q[1] * ln[3] + q[3] * ln[5]));
        atomicAdd(t + 3 * kNodes, w * la[3] - (2.0f * q[3] * ln[2] + q[1] * ln[4] + q[2] * ln[5]));
#pragma unroll
        for (int j = 0; j < 6; ++j) atomicAdd(t + (4 + j) * kNodes, ln[j]);
      };
      smp.template visit<kMaxLevels - 1>(a.level, gn, 1.0f, 1.0f, scatter);
    }
#pragma unroll
    for (int m = 0; m < kMom; ++m) {
      lc[m * kNodes + node] = 0.0f;
      lo[m * kNodes + node] = 0.0f;
    }
  }
}

inline unsigned grid1(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_mark_static(const Geom& G, const uint8_t* solid, uint8_t* t0s, hipStream_t s) {
  if (!solid) {
    hipLaunchKernelGGL(k_copy_or_clear, dim3(grid1(G.lv[0].ncell, 256)), dim3(256), 0, s, t0s, (const uint8_t*)nullptr,
                       G.lv[0].ncell, (int32_t*)nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_mark_static, dim3((unsigned)G.lv[0].ncell), dim3(256), 0, s, G, solid, t0s);
  return hipGetLastError();
}

hipError_t launch_targets(const HierLaunch& h, const float* p, int64_t n, int32_t* flag, hipStream_t s) {
  const int64_t n0 = h.G.lv[0].ncell;
  hipLaunchKernelGGL(k_copy_or_clear, dim3(grid1(n0, 256)), dim3(256), 0, s, h.t0, h.t0_static, n0, flag);
  if (p && n > 0) hipLaunchKernelGGL(k_mark_particles, dim3(grid1(n, 256)), dim3(256), 0, s, h.G, p, n, h.t0);
  return hipGetLastError();
}

hipError_t launch_advance_targets(const HierLaunch& h, float* p, int64_t n, const float d[3], const uint8_t* t0_prev,
                                  int32_t* flag, hipStream_t s) {
  const int64_t n0 = h.G.lv[0].ncell;
  hipLaunchKernelGGL(k_copy_or_clear, dim3(grid1(n0, 256)), dim3(256), 0, s, h.t0, h.t0_static, n0, flag);
  if (p && n > 0)
    hipLaunchKernelGGL(k_advance_mark, dim3(grid1(n, 256)), dim3(256), 0, s, h.G, p, n, d[0], d[1], d[2], h.t0);
  hipLaunchKernelGGL(k_diff, dim3(grid1(n0, 256)), dim3(256), 0, s, (const uint8_t*)h.t0, t0_prev, n0, flag);
  return hipGetLastError();
}

hipError_t launch_states(const HierLaunch& h, int32_t* flag, int32_t tag, hipStream_t s) {
  const Geom& G = h.G;
  for (int l = 1; l < G.L; ++l) {
    const LevelGeom& g = G.lv[l];
    const uint8_t* finer = (l == 1) ? h.t0 : h.flags + G.lv[l - 1].off;
    const uint8_t mask = (l == 1) ? 1 : (F_D | F_B);
    hipLaunchKernelGGL(k_deleted, dim3(grid1(g.ncell, 256)), dim3(256), 0, s, G, l, finer, mask, h.flags + g.off);
    hipLaunchKernelGGL(k_ring, dim3(grid1(g.ncell, 256)), dim3(256), 0, s, G, l, h.flags + g.off);
  }
  int64_t ntot = 0;
  for (int l = 0; l < G.L; ++l) ntot += G.lv[l].ncell;
  hipLaunchKernelGGL(k_state, dim3(grid1(ntot, 256)), dim3(256), 0, s, G, (const uint8_t*)h.flags, h.st_new,
                     h.st_old, ntot, flag, tag);
  return hipGetLastError();
}

hipError_t launch_diff(const uint8_t* a, const uint8_t* b, int64_t n, int32_t* flag, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_diff, dim3(grid1(n, 256)), dim3(256), 0, s, a, b, n, flag);
  return hipGetLastError();
}

// the segments' wave ranges; false if they need more than `wave_ints` counts
static bool seg_waves(int nseg, const int64_t* nitems, int np, int64_t wave_ints, SegWaves& q) {
  if (nseg < 1 || nseg > kMaxSegs) return false;
  q.nseg = nseg;
  int64_t w = 0;
  for (int k = 0; k < nseg; ++k) {
    if (nitems[k] < 0) return false;
    q.wave0[k] = w;
    q.nitems[k] = nitems[k];
    w += (nitems[k] + 63) >> 6;
  }
  for (int k = nseg; k <= kMaxSegs; ++k) q.wave0[k] = w;
  return w * np <= wave_ints;
}

static int64_t morton_items(const LevelGeom& g) { return (int64_t)1 << (3 * g.mbits); }

int64_t compact_cells_ints(const Geom& G) {
  int64_t w = 0;
  for (int l = 0; l < G.L; ++l) w += (morton_items(G.lv[l]) + 63) >> 6;
  return 3 * w;
}
int64_t compact_bytes_ints(int64_t list_items) { return 6 * ((list_items + 63) / 64 + kMaxSegs); }

hipError_t launch_compact_cells(const CellSegs& c, int32_t* wave_scratch, int64_t wave_ints, hipStream_t s) {
  if (c.nseg > kMaxLevels) return hipErrorInvalidValue;
  int64_t nitems[kMaxSegs];
  SegCounts tot;
  for (int k = 0; k < c.nseg; ++k) {
    nitems[k] = morton_items(c.G.lv[c.level[k]]);
    tot.c[k][0] = c.count[k];
    tot.c[k][1] = nullptr;
  }
  SegWaves q;
  if (!seg_waves(c.nseg, nitems, 3, wave_ints, q)) return hipErrorInvalidValue;
  const int64_t threads = 64 * q.wave0[c.nseg];
  if (threads > 0)
    hipLaunchKernelGGL(k_cells_count, dim3(grid1(threads, 256)), dim3(256), 0, s, c, q, wave_scratch);
  hipLaunchKernelGGL(k_scan<3>, dim3(1), dim3(1024), 0, s, wave_scratch, q, tot);
  if (threads > 0)
    hipLaunchKernelGGL(k_cells_scatter, dim3(grid1(threads, 256)), dim3(256), 0, s, c, q,
                       (const int32_t*)wave_scratch);
  return hipGetLastError();
}

hipError_t launch_compact_bytes(const ByteSegs& b, int32_t* wave_scratch, int64_t wave_ints, hipStream_t s) {
  int64_t nitems[kMaxSegs];
  SegCounts tot;
  for (int k = 0; k < b.nseg && k < kMaxSegs; ++k) {
    nitems[k] = b.n[k];
    tot.c[k][0] = b.count[k][0];
    tot.c[k][1] = b.count[k][1];
  }
  SegWaves q;
  if (!seg_waves(b.nseg, nitems, 6, wave_ints, q)) return hipErrorInvalidValue;
  const int64_t threads = 64 * q.wave0[b.nseg];
  if (threads > 0)
    hipLaunchKernelGGL(k_bytes_count, dim3(grid1(threads, 256)), dim3(256), 0, s, b, q, wave_scratch);
  hipLaunchKernelGGL(k_scan<6>, dim3(1), dim3(1024), 0, s, wave_scratch, q, tot);
  if (threads > 0)
    hipLaunchKernelGGL(k_bytes_scatter, dim3(grid1(threads, 256)), dim3(256), 0, s, b, q,
                       (const int32_t*)wave_scratch);
  return hipGetLastError();
}

hipError_t launch_tile_runs(const Geom& G, int level, const int32_t* blocks, int32_t n, const uint8_t* summary,
                            const uint8_t* st, const int4* coord, int run_max, uint8_t* run_class, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (run_max < 1 || run_max > kRunMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tile_runs, dim3(grid1(n, 256)), dim3(256), 0, s, G, level, blocks, n, summary, st, coord,
                     run_max, run_class);
  return hipGetLastError();
}

hipError_t launch_alloc(const AllocLaunch& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_alloc, dim3(grid1(a.n, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_release(const int32_t* cells, int32_t n, int64_t off, const int32_t* dir_old, int32_t* free_stack,
                          int32_t free_top, int32_t* dir_new, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_release, dim3(grid1(n, 256)), dim3(256), 0, s, cells, n, off, dir_old, free_stack, free_top, dir_new);
  return hipGetLastError();
}
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_i32, dim3(grid1(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* dst, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid1(n, 256)), dim3(256), 0, s, dst, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_u8(uint8_t* dst, uint8_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(grid1(n, 256)), dim3(256), 0, s, dst, v, n);
  return hipGetLastError();
}
hipError_t launch_roles(const RoleLaunch& r0, hipStream_t s) {
  RoleLaunch r = r0;
  int32_t wg = 0;
  for (int l = 0; l < r.G.L; ++l) {
    if (r.n[l] < 0) return hipErrorInvalidValue;
    r.wg0[l] = wg;
    wg += (r.n[l] + 3) / 4;
  }
  for (int l = r.G.L; l <= kMaxLevels; ++l) r.wg0[l] = wg;
  if (wg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_roles, dim3(wg), dim3(256), 0, s, r);
  return hipGetLastError();
}
hipError_t launch_init(const InitLaunch* a, int nlev, hipStream_t s) {
  if (nlev < 1 || nlev > kMaxLevels) return hipErrorInvalidValue;
  InitLevels x;
  x.nlev = nlev;
  int32_t grid = 0;
  for (int l = 0; l < nlev; ++l) {
    if (a[l].storage != a[0].storage) return hipErrorInvalidValue;
    x.a[l] = a[l];
    grid = a[l].n > grid ? a[l].n : grid;  // n: the list length, or its bound
  }
  if (grid <= 0) return hipSuccess;
  grid = grid < 2048 ? grid : 2048;
  switch (a[0].storage) {
    case 0: hipLaunchKernelGGL(k_init<StoreF32>, dim3(grid), dim3(256), 0, s, x); break;
    case 1: hipLaunchKernelGGL(k_init<StoreBF16>, dim3(grid), dim3(256), 0, s, x); break;
    case 2: hipLaunchKernelGGL(k_init<StoreF16>, dim3(grid), dim3(256), 0, s, x); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_init_adj(const InitAdjLaunch& x, hipStream_t s) {
  if (x.f.n <= 0) return hipSuccess;
  switch (x.f.storage) {
    case 0: hipLaunchKernelGGL(k_init_adj<StoreF32>, dim3(x.f.n), dim3(256), 0, s, x); break;
    case 1: hipLaunchKernelGGL(k_init_adj<StoreBF16>, dim3(x.f.n), dim3(256), 0, s, x); break;
    case 2: hipLaunchKernelGGL(k_init_adj<StoreF16>, dim3(x.f.n), dim3(256), 0, s, x); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lbmx
