// Shared device-side definitions of the MI355X block-adaptive D3Q27 moment LBM.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmx {

constexpr int kEdge = 8;       // nodes per block edge
constexpr int kNodes = 512;    // nodes per block
constexpr int kMom = 10;       // stored moments per node
constexpr int kMaxLevels = 5;
constexpr int kBlockStride = kMom * kNodes;  // elements per block per time level

// node roles (low 3 bits of the role byte); bit 7 marks computed nodes with a
// solid neighbour or a wall (they need the bounce-back correction)
enum : uint8_t { ROLE_COMPUTED = 0, ROLE_GHOST = 1, ROLE_IU = 2, ROLE_SOLID = 3, ROLE_INFLOW = 4, ROLE_OUTFLOW = 5 };
constexpr uint8_t ROLE_MASK = 7;
constexpr uint8_t ROLE_BB = 0x80;
// block state per level
enum : uint8_t { ST_ABSENT = 0, ST_ACTIVE = 1, ST_DELETED = 2 };
// boundary kinds
enum : int { BC_PERIODIC = 0, BC_INFLOW = 1, BC_OUTFLOW = 2, BC_WALL = 3, BC_OUTFLOW_CONV = 4 };
__host__ __device__ inline bool is_outflow_bc(int kind) { return kind == BC_OUTFLOW || kind == BC_OUTFLOW_CONV; }
// neighbour-table sentinels
constexpr int32_t NBR_NONE = -1;
constexpr int32_t NBR_WALL = -2;
// per-block summary bits
constexpr uint8_t SUM_GHOST = 1, SUM_IU = 2, SUM_OUTFLOW = 4, SUM_TILE = 8, SUM_BB = 16, SUM_FRESH = 32;
// stream-collide tiles of large levels: kTileX x 2 x 2 blocks (kTileX a power of two)
constexpr int kTileX = 2;
// the two-substep sweep of the finest level takes runs of up to kRunMax tiles stacked
// along z (class k of the run lists: runs of k + 1 tiles)
constexpr int kRunMax = 6;

struct LevelGeom {
  int nb[3];       // blocks per axis
  int nn[3];       // nodes per axis
  int mbits;       // Morton bits per axis covering nb
  int pad;
  int64_t ncell;   // nb[0]*nb[1]*nb[2]
  int64_t off;     // offset of this level in the all-level dense cell arrays
};

struct Geom {
  int L;
  int bc[6];
  int periodic[3];
  int N[3];
  LevelGeom lv[kMaxLevels];
  float inflow[3];       // inflow velocity (times the profile factor)
  int inflow_profile;    // 0 uniform, 1 logarithmic in the height along inflow_axis
  int inflow_axis;
  float inflow_beta, inflow_h0;
};

// inflow velocity of level-l node g: inflow (times ln(1 + beta (h - h0)) for the
// logarithmic profile, h the node's height in fine-level nodes; zero at or below h0)
__device__ inline void inflow_velocity(const Geom& G, int l, const int g[3], float u[3]) {
  float f = 1.0f;
  if (G.inflow_profile == 1) {
    const float h = (float)(g[G.inflow_axis] << l);
    f = h > G.inflow_h0 ? logf(1.0f + G.inflow_beta * (h - G.inflow_h0)) : 0.0f;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = G.inflow[a] * f;
}

__host__ __device__ inline int64_t cell_lin(const LevelGeom& g, int bx, int by, int bz) {
  return bx + (int64_t)g.nb[0] * (by + (int64_t)g.nb[1] * bz);
}

__host__ __device__ inline uint64_t morton_encode3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t k = 0;
  for (int bit = 0; bit < 21; ++bit) {
    k |= (uint64_t)((x >> bit) & 1u) << (3 * bit);
    k |= (uint64_t)((y >> bit) & 1u) << (3 * bit + 1);
    k |= (uint64_t)((z >> bit) & 1u) << (3 * bit + 2);
  }
  return k;
}
__host__ __device__ inline void morton_decode3(uint64_t k, int& x, int& y, int& z) {
  x = y = z = 0;
  for (int bit = 0; bit < 21; ++bit) {
    x |= (int)((k >> (3 * bit)) & 1u) << bit;
    y |= (int)((k >> (3 * bit + 1)) & 1u) << bit;
    z |= (int)((k >> (3 * bit + 2)) & 1u) << bit;
  }
}

// wrap a level-l node coordinate; false if it leaves a non-periodic axis
__device__ inline bool wrap_node(const Geom& G, int l, int g[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int n = G.lv[l].nn[a];
    if (g[a] < 0 || g[a] >= n) {
      if (!G.periodic[a]) return false;
      g[a] = g[a] < 0 ? g[a] + n : g[a] - n;
    }
  }
  return true;
}

// ---- storage codec: f32, bf16 (RNE) or f16 (RNE), per-moment power-of-two scales
struct StoreF32 { typedef float type; };
struct StoreBF16 { typedef uint16_t type; };
struct StoreF16 { typedef uint16_t type; };

template <class S> struct Codec;
template <> struct Codec<StoreF32> {
  __device__ static inline float load(float q, float) { return q; }
  __device__ static inline float store(float v, float) { return v; }
};
template <> struct Codec<StoreBF16> {
  __device__ static inline float load(uint16_t q, float inv) { return __uint_as_float((uint32_t)q << 16) * inv; }
  __device__ static inline uint16_t store(float v, float s) {
    uint32_t b = __float_as_uint(v * s);
    b += 0x7fffu + ((b >> 16) & 1u);  // round to nearest even
    return (uint16_t)(b >> 16);
  }
};
template <> struct Codec<StoreF16> {
  __device__ static inline float load(uint16_t q, float inv) {
    _Float16 h;
    __builtin_memcpy(&h, &q, 2);
    return (float)h * inv;
  }
  __device__ static inline uint16_t store(float v, float s) {
    _Float16 h = (_Float16)(v * s);
    uint16_t q;
    __builtin_memcpy(&q, &h, 2);
    return q;
  }
};

struct Scales {
  float s[kMom];
  float inv[kMom];
};

}  // namespace lbmx
