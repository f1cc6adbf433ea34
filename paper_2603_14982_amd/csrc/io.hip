// Moment upload / download, node roles, FP64 reductions, finiteness check and the
// prescribed particle motion.
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace lbmx {
namespace {

template <class S>
__global__ __launch_bounds__(256) void k_get(IoLaunch a, int64_t* keys, float* out) {
  const int32_t slot = a.blocks[blockIdx.x];
  const typename S::type* src = static_cast<const typename S::type*>(a.buf) + (size_t)slot * kBlockStride;
  float* dst = out + (size_t)blockIdx.x * kBlockStride;
  for (int i = threadIdx.x; i < kBlockStride; i += 256) dst[i] = Codec<S>::load(src[i], a.sc.inv[i / kNodes]);
  if (keys && threadIdx.x == 0) {
    const int4 c = a.coord[slot];
    keys[blockIdx.x] = (int64_t)morton_encode3(c.x, c.y, c.z);
  }
}

__global__ void k_keys(IoLaunch a, int64_t* keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nblocks) return;
  const int4 c = a.coord[a.blocks[i]];
  keys[i] = (int64_t)morton_encode3(c.x, c.y, c.z);
}

__global__ __launch_bounds__(256) void k_get_roles(IoLaunch a, uint8_t* out) {
  const int32_t slot = a.blocks[blockIdx.x];
  for (int i = threadIdx.x; i < kNodes; i += 256)
    out[(size_t)blockIdx.x * kNodes + i] = a.role[(size_t)slot * kNodes + i] & ROLE_MASK;
}

template <class S>
__global__ __launch_bounds__(256) void k_set(IoLaunch a, const int64_t* keys, const float* in, const int32_t* dir,
                                             int32_t* err) {
  const LevelGeom& g = a.G.lv[a.level];
  int bx, by, bz;
  morton_decode3((uint64_t)keys[blockIdx.x], bx, by, bz);
  int32_t slot = -1;
  if (bx < g.nb[0] && by < g.nb[1] && bz < g.nb[2]) slot = dir[g.off + cell_lin(g, bx, by, bz)];
  if (slot < 0) {
    if (threadIdx.x == 0) *err = 1;
    return;
  }
  typedef typename S::type T;
  T* cur = static_cast<T*>(a.buf) + (size_t)slot * kBlockStride;
  T* oth = static_cast<T*>(a.other) + (size_t)slot * kBlockStride;
  const float* src = in + (size_t)blockIdx.x * kBlockStride;
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    const uint8_t r = a.role[(size_t)slot * kNodes + node] & ROLE_MASK;
    float q[kMom];
#pragma unroll
    for (int m = 0; m < kMom; ++m) q[m] = src[m * kNodes + node];
    if (r == ROLE_SOLID) {
#pragma unroll
      for (int m = 0; m < kMom; ++m) q[m] = 0.0f;
    } else if (r == ROLE_INFLOW) {
      const int gn[3] = {bx * kEdge + (node & 7), by * kEdge + ((node >> 3) & 7), bz * kEdge + (node >> 6)};
      q[0] = 0.0f;
      inflow_velocity(a.G, a.level, gn, q + 1);
      q[4] = q[1] * q[1]; q[5] = q[2] * q[2]; q[6] = q[3] * q[3];
      q[7] = q[1] * q[2]; q[8] = q[1] * q[3]; q[9] = q[2] * q[3];
    }
#pragma unroll
    for (int m = 0; m < kMom; ++m) {
      const T v = Codec<S>::store(q[m], a.sc.s[m]);
      cur[m * kNodes + node] = v;
      oth[m * kNodes + node] = v;
    }
  }
}

// per-block FP64 partial sums; the final sum runs in fixed block order
template <class S>
__global__ __launch_bounds__(256) void k_reduce_blocks(IoLaunch a, int lx, int ly, int lz, int hx, int hy, int hz,
                                                       double* partial) {
  __shared__ double sh[5][256];
  const int32_t slot = a.blocks[blockIdx.x];
  const int4 c = a.coord[slot];
  const typename S::type* src = static_cast<const typename S::type*>(a.buf) + (size_t)slot * kBlockStride;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    const uint8_t r = a.role[(size_t)slot * kNodes + node] & ROLE_MASK;
    if (!(r == ROLE_COMPUTED || r == ROLE_IU || r == ROLE_INFLOW || r == ROLE_OUTFLOW)) continue;
    const int64_t fx = (int64_t)(c.x * kEdge + (node & 7)) << a.level;
    const int64_t fy = (int64_t)(c.y * kEdge + ((node >> 3) & 7)) << a.level;
    const int64_t fz = (int64_t)(c.z * kEdge + (node >> 6)) << a.level;
    if (fx < lx || fx >= hx || fy < ly || fy >= hy || fz < lz || fz >= hz) continue;
    const double rho = 1.0 + (double)Codec<S>::load(src[node], a.sc.inv[0]);
    const double ux = Codec<S>::load(src[kNodes + node], a.sc.inv[1]);
    const double uy = Codec<S>::load(src[2 * kNodes + node], a.sc.inv[2]);
    const double uz = Codec<S>::load(src[3 * kNodes + node], a.sc.inv[3]);
    acc[0] += rho;
    acc[1] += rho * ux; acc[2] += rho * uy; acc[3] += rho * uz;
    acc[4] += 0.5 * rho * (ux * ux + uy * uy + uz * uz);
  }
  for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 5) partial[(size_t)blockIdx.x * 5 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_reduce_final(const double* partial, int32_t n, double* out) {
  __shared__ double sh[5][256];
  double acc[5] = {0, 0, 0, 0, 0};
  for (int32_t i = threadIdx.x; i < n; i += 256)
    for (int k = 0; k < 5; ++k) acc[k] += partial[(size_t)i * 5 + k];
  for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 5) out[threadIdx.x] = sh[threadIdx.x][0];
}

template <class S>
__global__ __launch_bounds__(256) void k_finite(IoLaunch a, int32_t* flag) {
  const int32_t slot = a.blocks[blockIdx.x];
  const typename S::type* src = static_cast<const typename S::type*>(a.buf) + (size_t)slot * kBlockStride;
  int bad = 0;
  for (int i = threadIdx.x; i < kBlockStride; i += 256) {
    const uint8_t r = a.role[(size_t)slot * kNodes + (i % kNodes)] & ROLE_MASK;
    if (r == ROLE_GHOST) continue;
    const float v = Codec<S>::load(src[i], a.sc.inv[i / kNodes]);
    if (!__builtin_isfinite(v)) bad = 1;
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) *flag = 1;
}

__global__ void k_advance(float* p, int64_t n, float dx, float dy, float dz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[3 * i + 0] = __fadd_rn(p[3 * i + 0], dx);
  p[3 * i + 1] = __fadd_rn(p[3 * i + 1], dy);
  p[3 * i + 2] = __fadd_rn(p[3 * i + 2], dz);
}

// ---- finest-level coupling fields [slot][4][512]: eps, Fx, Fy, Fz ----
// every slot (the all-zero one included) starts at eps = 1, F = 0
__global__ void k_cpl_default(float* cpl, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cpl[i] = ((i / kNodes) & 3) == 0 ? 1.0f : 0.0f;
}
// check of the caller's fields of finest-level blocks: err 1 for a key that is no
// active block, 2 for a value that is not finite or an eps with eps tau0 <= 1/2
__global__ __launch_bounds__(256) void k_cpl_check(LevelGeom g, const int64_t* keys, const float* in,
                                                   const int32_t* dir, float tau0, int32_t* err) {
  int bx, by, bz;
  morton_decode3((uint64_t)keys[blockIdx.x], bx, by, bz);
  int32_t slot = -1;
  if (bx < g.nb[0] && by < g.nb[1] && bz < g.nb[2]) slot = dir[g.off + cell_lin(g, bx, by, bz)];
  if (slot < 0) {
    if (threadIdx.x == 0) atomicMax(err, 1);
    return;
  }
  const float* src = in + (size_t)blockIdx.x * 4 * kNodes;
  int bad = 0;
  for (int i = threadIdx.x; i < 4 * kNodes; i += 256) {
    const float v = src[i];
    if (!__builtin_isfinite(v) || (i < kNodes && !(v * tau0 > 0.5f))) bad = 1;
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicMax(err, 2);
}
// scatter into the slots; solid nodes keep eps = 1, F = 0 (they carry no moments, and
// a force there would give them nonzero populations)
__global__ __launch_bounds__(256) void k_cpl_set(LevelGeom g, const int64_t* keys, const float* in, const int32_t* dir,
                                                 const uint8_t* role, float* cpl) {
  int bx, by, bz;
  morton_decode3((uint64_t)keys[blockIdx.x], bx, by, bz);
  if (!(bx < g.nb[0] && by < g.nb[1] && bz < g.nb[2])) return;
  const int32_t slot = dir[g.off + cell_lin(g, bx, by, bz)];
  if (slot < 0) return;
  const float* src = in + (size_t)blockIdx.x * 4 * kNodes;
  float* dst = cpl + (size_t)slot * 4 * kNodes;
  for (int i = threadIdx.x; i < 4 * kNodes; i += 256) {
    const bool solid = (role[(size_t)slot * kNodes + (i % kNodes)] & ROLE_MASK) == ROLE_SOLID;
    dst[i] = solid ? (i < kNodes ? 1.0f : 0.0f) : src[i];
  }
}

template <template <class> class K, class... Args>
hipError_t dispatch(int storage, dim3 g, dim3 b, hipStream_t s, Args... args) {
  switch (storage) {
    case 0: hipLaunchKernelGGL(K<StoreF32>::fn, g, b, 0, s, args...); break;
    case 1: hipLaunchKernelGGL(K<StoreBF16>::fn, g, b, 0, s, args...); break;
    case 2: hipLaunchKernelGGL(K<StoreF16>::fn, g, b, 0, s, args...); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <class S> struct GetK { static constexpr auto fn = k_get<S>; };
template <class S> struct SetK { static constexpr auto fn = k_set<S>; };
template <class S> struct RedK { static constexpr auto fn = k_reduce_blocks<S>; };
template <class S> struct FinK { static constexpr auto fn = k_finite<S>; };

}  // namespace

hipError_t launch_get(const IoLaunch& a, int64_t* keys, float* out, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  return dispatch<GetK>(a.storage, dim3(a.nblocks), dim3(256), s, a, keys, out);
}
hipError_t launch_keys(const IoLaunch& a, int64_t* keys, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_keys, dim3((a.nblocks + 255) / 256), dim3(256), 0, s, a, keys);
  return hipGetLastError();
}
hipError_t launch_get_roles(const IoLaunch& a, uint8_t* out, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_get_roles, dim3(a.nblocks), dim3(256), 0, s, a, out);
  return hipGetLastError();
}
hipError_t launch_set(const IoLaunch& a, const int64_t* keys, const float* in, int64_t nb, const int32_t* dir,
                      int32_t* err, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  return dispatch<SetK>(a.storage, dim3((unsigned)nb), dim3(256), s, a, keys, in, dir, err);
}
hipError_t launch_reduce(const IoLaunch& a, const int32_t lo[3], const int32_t hi[3], double* partial, double* out,
                         hipStream_t s) {
  if (a.nblocks > 0) {
    hipError_t e = dispatch<RedK>(a.storage, dim3(a.nblocks), dim3(256), s, a, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2],
                                  partial);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (const double*)partial, a.nblocks, out);
  return hipGetLastError();
}
// One array per GPU, held until the process ends. In host code its name is a host-side
// stand-in, not a device address: kernels get the address hipGetSymbolAddress returns
// for the current device.
static __device__ __align__(256) double scratch[kNoAllocReduceBlocks * 5];

hipError_t noalloc_reduce_scratch(double** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_finite(const IoLaunch& a, int32_t* flag, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  return dispatch<FinK>(a.storage, dim3(a.nblocks), dim3(256), s, a, flag);
}
hipError_t launch_cpl_default(float* cpl, int64_t nslots, hipStream_t s) {
  const int64_t n = nslots * 4 * kNodes;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpl_default, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cpl, n);
  return hipGetLastError();
}
hipError_t launch_cpl_check(const LevelGeom& g, const int64_t* keys, const float* in, int64_t nb, const int32_t* dir,
                            float tau0, int32_t* err, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpl_check, dim3((unsigned)nb), dim3(256), 0, s, g, keys, in, dir, tau0, err);
  return hipGetLastError();
}
hipError_t launch_cpl_set(const LevelGeom& g, const int64_t* keys, const float* in, int64_t nb, const int32_t* dir,
                          const uint8_t* role, float* cpl, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpl_set, dim3((unsigned)nb), dim3(256), 0, s, g, keys, in, dir, role, cpl);
  return hipGetLastError();
}
hipError_t launch_advance_particles(float* p, int64_t n, float dx, float dy, float dz, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_advance, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, dx, dy, dz);
  return hipGetLastError();
}

}  // namespace lbmx
