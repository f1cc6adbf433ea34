// Powder-snow volume fraction phi on the finest level (Sec. 7, powder snow): phi is
// carried by the fluid velocity, diffuses and gains a source,
//   dphi/dt + u . grad phi = q + D lap phi,
// advanced by one semi-Lagrangian step (departure point by Ralston's third-order
// Runge-Kutta backwards in time through the trilinearly interpolated velocity,
// phi interpolated trilinearly there), then one forward-Euler step of the 7-point
// Laplacian, then the source.
//
// Layout: phi[2][slot][512] f32 (the current field and the intermediate one); the
// velocity is read from the finest level's stored moments. phi lives on the finest
// level's owned nodes: nodes outside its blocks, its ghost nodes (the coarser
// level's region), nodes beyond walls and solid nodes read phi = 0 and u = 0 and
// keep phi = 0; periodic axes wrap through the neighbour table. A departure point is kept within
// 7 nodes of its node per axis, so every interpolation corner lies in the block or
// one of its 26 neighbours.
#include "common.h"
#include "kernels.h"

namespace lbmx {
namespace {

__device__ __forceinline__ bool off_scalar(uint8_t r) {
  const uint8_t k = r & ROLE_MASK;
  return k == ROLE_SOLID || k == ROLE_GHOST;
}

// finest-level node at block-relative coordinates (l in [-8, 15]) -> slot and node,
// or slot -1 (no block there, or outside a wall)
__device__ __forceinline__ int rel_node(const int* s_nbr, int lx, int ly, int lz, int& node) {
  const int ox = (lx + 8) >> 3, oy = (ly + 8) >> 3, oz = (lz + 8) >> 3;  // 0, 1, 2
  node = (lx & 7) + 8 * (ly & 7) + 64 * (lz & 7);
  return s_nbr[ox + 3 * oy + 9 * oz];
}

template <class S>
__device__ __forceinline__ void u_at(const ScalarLaunch& a, const int* s_nbr, int lx, int ly, int lz, float u[3]) {
  int node;
  const int ns = rel_node(s_nbr, lx, ly, lz, node);
  u[0] = u[1] = u[2] = 0.0f;
  if (ns < 0 || off_scalar(a.role[(size_t)ns * kNodes + node])) return;
  const typename S::type* q = static_cast<const typename S::type*>(a.moments) + (size_t)ns * kBlockStride + node;
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = Codec<S>::load(q[(1 + k) * kNodes], a.sc.inv[1 + k]);
}

__device__ __forceinline__ float phi_at(const ScalarLaunch& a, const float* phi, const int* s_nbr, int lx, int ly,
                                        int lz) {
  int node;
  const int ns = rel_node(s_nbr, lx, ly, lz, node);
  if (ns < 0 || off_scalar(a.role[(size_t)ns * kNodes + node])) return 0.0f;
  return phi[(size_t)ns * kNodes + node];
}

// corner and weights of a block-relative point y, clamped to within 7 nodes of the
// node x (per axis)
__device__ __forceinline__ void cell_of(const float x[3], const float y[3], int i0[3], float w[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float v = fminf(fmaxf(y[k], x[k] - 7.0f), x[k] + 7.0f);
    const float f = floorf(v);
    i0[k] = (int)f;
    w[k] = v - f;
  }
}

template <class S>
__device__ void u_interp(const ScalarLaunch& a, const int* s_nbr, const float x[3], const float y[3], float u[3]) {
  int i0[3];
  float w[3];
  cell_of(x, y, i0, w);
  u[0] = u[1] = u[2] = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
    const float wt = (dx ? w[0] : 1.0f - w[0]) * (dy ? w[1] : 1.0f - w[1]) * (dz ? w[2] : 1.0f - w[2]);
    float v[3];
    u_at<S>(a, s_nbr, i0[0] + dx, i0[1] + dy, i0[2] + dz, v);
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] += wt * v[k];
  }
}

__device__ void load_nbr(const ScalarLaunch& a, int slot, int* s_nbr) {
  if (threadIdx.x < 27) {
    const int ns = a.nbr[(size_t)slot * 27 + threadIdx.x];
    s_nbr[threadIdx.x] = ns >= 0 ? ns : -1;
  }
  __syncthreads();
}

template <class S>
__global__ __launch_bounds__(256) void k_scalar_advect(ScalarLaunch a) {
  __shared__ int s_nbr[27];
  const int slot = a.blocks[blockIdx.x];
  load_nbr(a, slot, s_nbr);
  const float dt = a.dt;
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    float out = 0.0f;
    if (!off_scalar(a.role[(size_t)slot * kNodes + node])) {
      const float x[3] = {(float)(node & 7), (float)((node >> 3) & 7), (float)(node >> 6)};
      float k1[3], k2[3], k3[3], y[3];
      u_interp<S>(a, s_nbr, x, x, k1);
#pragma unroll
      for (int k = 0; k < 3; ++k) y[k] = x[k] - 0.5f * dt * k1[k];
      u_interp<S>(a, s_nbr, x, y, k2);
#pragma unroll
      for (int k = 0; k < 3; ++k) y[k] = x[k] - 0.75f * dt * k2[k];
      u_interp<S>(a, s_nbr, x, y, k3);
#pragma unroll
      for (int k = 0; k < 3; ++k) y[k] = x[k] - dt * (2.0f * k1[k] + 3.0f * k2[k] + 4.0f * k3[k]) / 9.0f;
      int i0[3];
      float w[3];
      cell_of(x, y, i0, w);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
        const float wt = (dx ? w[0] : 1.0f - w[0]) * (dy ? w[1] : 1.0f - w[1]) * (dz ? w[2] : 1.0f - w[2]);
        out += wt * phi_at(a, a.phi_in, s_nbr, i0[0] + dx, i0[1] + dy, i0[2] + dz);
      }
    }
    a.phi_out[(size_t)slot * kNodes + node] = out;
  }
}

__global__ __launch_bounds__(256) void k_scalar_diffuse(ScalarLaunch a) {
  __shared__ int s_nbr[27];
  const int slot = a.blocks[blockIdx.x];
  load_nbr(a, slot, s_nbr);
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    float out = 0.0f;
    if (!off_scalar(a.role[(size_t)slot * kNodes + node])) {
      const int lx = node & 7, ly = (node >> 3) & 7, lz = node >> 6;
      const float c = a.phi_in[(size_t)slot * kNodes + node];
      const float lap = (phi_at(a, a.phi_in, s_nbr, lx - 1, ly, lz) - c) + (phi_at(a, a.phi_in, s_nbr, lx + 1, ly, lz) - c) +
                        (phi_at(a, a.phi_in, s_nbr, lx, ly - 1, lz) - c) + (phi_at(a, a.phi_in, s_nbr, lx, ly + 1, lz) - c) +
                        (phi_at(a, a.phi_in, s_nbr, lx, ly, lz - 1) - c) + (phi_at(a, a.phi_in, s_nbr, lx, ly, lz + 1) - c);
      out = c + a.D * a.dt * lap;
      if (a.source) out += a.dt * a.source[(size_t)blockIdx.x * kNodes + node];
    }
    a.phi_out[(size_t)slot * kNodes + node] = out;
  }
}

// caller's phi of finest-level blocks (key order) into the slots; solid and ghost nodes 0
__global__ __launch_bounds__(256) void k_scalar_set(LevelGeom g, const int64_t* keys, const float* in,
                                                    const int32_t* dir, const uint8_t* role, float* phi, int32_t* err) {
  int bx, by, bz;
  morton_decode3((uint64_t)keys[blockIdx.x], bx, by, bz);
  int32_t slot = -1;
  if (bx < g.nb[0] && by < g.nb[1] && bz < g.nb[2]) slot = dir[g.off + cell_lin(g, bx, by, bz)];
  if (slot < 0) {
    if (threadIdx.x == 0) *err = 1;
    return;
  }
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    const bool off = off_scalar(role[(size_t)slot * kNodes + node]);
    phi[(size_t)slot * kNodes + node] = off ? 0.0f : in[(size_t)blockIdx.x * kNodes + node];
  }
}

__global__ __launch_bounds__(256) void k_scalar_get(const int32_t* blocks, const float* phi, float* out) {
  const int slot = blocks[blockIdx.x];
  for (int node = threadIdx.x; node < kNodes; node += 256)
    out[(size_t)blockIdx.x * kNodes + node] = phi[(size_t)slot * kNodes + node];
}

template <class S> hipError_t adv_t(const ScalarLaunch& a, hipStream_t s) {
  hipLaunchKernelGGL(k_scalar_advect<S>, dim3(a.nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_scalar_advect(const ScalarLaunch& a, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  switch (a.storage) {
    case 0: return adv_t<StoreF32>(a, s);
    case 1: return adv_t<StoreBF16>(a, s);
    case 2: return adv_t<StoreF16>(a, s);
  }
  return hipErrorInvalidValue;
}
hipError_t launch_scalar_diffuse(const ScalarLaunch& a, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scalar_diffuse, dim3(a.nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_scalar_set(const LevelGeom& g, const int64_t* keys, const float* in, int64_t nb, const int32_t* dir,
                             const uint8_t* role, float* phi, int32_t* err, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scalar_set, dim3((unsigned)nb), dim3(256), 0, s, g, keys, in, dir, role, phi, err);
  return hipGetLastError();
}
hipError_t launch_scalar_get(const int32_t* blocks, int32_t nblocks, const float* phi, float* out, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scalar_get, dim3(nblocks), dim3(256), 0, s, blocks, phi, out);
  return hipGetLastError();
}

}  // namespace lbmx
