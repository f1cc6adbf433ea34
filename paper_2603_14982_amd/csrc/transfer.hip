// Interface transfers between levels (Sec. 5.3, Alg. 1) and the zero-gradient
// outflow copy.
//
// DownwardTransfer(l+1, s): every ghost node of level l (the one-node outer shell
// of the level's region) takes rho and u interpolated from its nearest 2^3 coarse
// nodes (trilinear, node-centred: coarse node q sits on fine node 2q) and
// S = a_down * sum_j w_j S^neq_j + u u (Eq. downward_rescale). For the second fine
// substep (s = 2) the coarse rho, u and S^neq are first averaged between coarse
// times t and t + 2 dt_l (temporal interpolation to the midpoint).
//
// UpwardTransfer(l): every upward-interface node q of level l+1 copies rho and u
// of the coincident fine node 2q and rescales S^neq by a_up (Eq. upload_S).
//
// Threads: one 256-lane workgroup per interface block, two nodes per lane; only
// lanes whose node has the target role do work.
#include "common.h"
#include "kernels.h"

namespace lbmx {
namespace {

template <class S> struct Mom {
  __device__ static inline void load(const void* base, int slot, int node, const Scales& sc, float q[kMom]) {
    const typename S::type* p = static_cast<const typename S::type*>(base) + (size_t)slot * kBlockStride + node;
#pragma unroll
    for (int m = 0; m < kMom; ++m) q[m] = Codec<S>::load(p[m * kNodes], sc.inv[m]);
  }
  __device__ static inline void store(void* base, int slot, int node, const Scales& sc, const float q[kMom]) {
    typename S::type* p = static_cast<typename S::type*>(base) + (size_t)slot * kBlockStride + node;
#pragma unroll
    for (int m = 0; m < kMom; ++m) p[m * kNodes] = Codec<S>::store(q[m], sc.s[m]);
  }
};

// adjoint replay: copy the node's current value (about to be overwritten) to the
// tape entry of the block's list index
template <class S>
__device__ inline void keep_old(const void* buf, void* tape, int slot, int idx, int node) {
  const typename S::type* p = static_cast<const typename S::type*>(buf) + (size_t)slot * kBlockStride + node;
  typename S::type* t = static_cast<typename S::type*>(tape) + (size_t)idx * kBlockStride + node;
#pragma unroll
  for (int m = 0; m < kMom; ++m) t[m * kNodes] = p[m * kNodes];
}

// (rho-1, u, S) -> (rho-1, u, S^neq = S - u u), in place
__device__ inline void to_neq(float q[kMom]) {
  q[4] -= q[1] * q[1]; q[5] -= q[2] * q[2]; q[6] -= q[3] * q[3];
  q[7] -= q[1] * q[2]; q[8] -= q[1] * q[3]; q[9] -= q[2] * q[3];
}
__device__ inline void from_neq(float q[kMom]) {
  q[4] += q[1] * q[1]; q[5] += q[2] * q[2]; q[6] += q[3] * q[3];
  q[7] += q[1] * q[2]; q[8] += q[1] * q[3]; q[9] += q[2] * q[3];
}

// One workgroup per fine block holding ghost nodes. The coarse nodes under the
// bounding box of the block's ghost nodes (recorded by the grid update; within coarse
// indices 4b .. 4b+4 per axis) are staged once in LDS as (rho-1, u, S^neq), already
// averaged in time for the midpoint substep; each ghost node in the box then combines
// its 1, 2, 4 or 8 trilinear sources from LDS. Staged positions in blocks that hold
// no coarse data (covered by the fine level) read as zero; no ghost node of a valid
// hierarchy uses them.
// trilinear interpolation of the staged (rho-1, u, S^neq) at local fine node lc,
// S^neq rescaled by `factor`, back to (rho-1, u, S)
__device__ inline void interp_ghost(const float (*cq)[125], const int lc[3], float factor, float acc[kMom]) {
  int i0[3], i1[3];
  float w1[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    // fine node 8b + lc sits on coarse 4b + lc/2 (even) or between the two neighbours (odd)
    i0[ax] = lc[ax] >> 1;
    i1[ax] = (lc[ax] + 1) >> 1;
    w1[ax] = (lc[ax] & 1) ? 0.5f : 0.0f;
  }
#pragma unroll
  for (int m = 0; m < kMom; ++m) acc[m] = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int kx = c & 1, ky = (c >> 1) & 1, kz = c >> 2;
    const float w = (kx ? w1[0] : 1.0f - w1[0]) * (ky ? w1[1] : 1.0f - w1[1]) * (kz ? w1[2] : 1.0f - w1[2]);
    if (w == 0.0f) continue;
    const int t = (kx ? i1[0] : i0[0]) + 5 * (ky ? i1[1] : i0[1]) + 25 * (kz ? i1[2] : i0[2]);
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] += w * cq[m][t];
    const float ws = w * factor;
#pragma unroll
    for (int m = 4; m < kMom; ++m) acc[m] += ws * cq[m][t];
  }
  from_neq(acc);
}

constexpr int kDownThreads = 256;

// both substeps of the fine level at once: s = 1 (coarse t, src_a) into a.dst and
// s = 2 (the midpoint of src_a and src_b) into a.dst2, the time level the first
// fine stream-collide writes (it never writes ghost nodes)
template <class S>
__global__ __launch_bounds__(kDownThreads) void k_downward(TransferLaunch a) {
  __shared__ float cq[2][kMom][125];
  const int slot = a.blocks[blockIdx.x];
  const int4 bc = a.coord[slot];
  const int l = a.level;
  const LevelGeom& cg = a.G.lv[l + 1];
  const int base[3] = {4 * bc.x, 4 * bc.y, 4 * bc.z};
  // only the ghost nodes' bounding box and the coarse nodes under it
  const int box = a.gbox[slot];
  const int lo[3] = {box & 7, (box >> 6) & 7, (box >> 12) & 7};
  const int hi[3] = {(box >> 3) & 7, (box >> 9) & 7, (box >> 15) & 7};
  const int clo[3] = {lo[0] >> 1, lo[1] >> 1, lo[2] >> 1};
  const int cn[3] = {((hi[0] + 1) >> 1) - clo[0] + 1, ((hi[1] + 1) >> 1) - clo[1] + 1, ((hi[2] + 1) >> 1) - clo[2] + 1};
  for (int k = threadIdx.x; k < cn[0] * cn[1] * cn[2]; k += kDownThreads) {
    const int t = (clo[0] + k % cn[0]) + 5 * (clo[1] + (k / cn[0]) % cn[1]) + 25 * (clo[2] + k / (cn[0] * cn[1]));
    int j[3] = {base[0] + t % 5, base[1] + (t / 5) % 5, base[2] + t / 25};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int nc = cg.nn[ax];
      if (a.G.periodic[ax]) j[ax] = j[ax] >= nc ? j[ax] - nc : j[ax];
      else j[ax] = j[ax] >= nc ? nc - 1 : j[ax];
    }
    const int cs = a.dir[cg.off + cell_lin(cg, j[0] >> 3, j[1] >> 3, j[2] >> 3)];
    float q[kMom], h[kMom];
#pragma unroll
    for (int m = 0; m < kMom; ++m) q[m] = h[m] = 0.0f;
    if (cs >= 0) {
      const int cn = (j[0] & 7) + 8 * (j[1] & 7) + 64 * (j[2] & 7);
      float r[kMom];
      Mom<S>::load(a.src_a, cs, cn, a.sc, q);
      Mom<S>::load(a.src_b, cs, cn, a.sc, r);
      to_neq(q);
      to_neq(r);
#pragma unroll
      for (int m = 0; m < kMom; ++m) h[m] = 0.5f * (q[m] + r[m]);
    }
#pragma unroll
    for (int m = 0; m < kMom; ++m) {
      cq[0][m][t] = q[m];
      cq[1][m][t] = h[m];
    }
  }
  __syncthreads();
  const int nn[3] = {hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1};
  for (int k = threadIdx.x; k < nn[0] * nn[1] * nn[2]; k += kDownThreads) {
    const int lc[3] = {lo[0] + k % nn[0], lo[1] + (k / nn[0]) % nn[1], lo[2] + k / (nn[0] * nn[1])};
    const int node = lc[0] + 8 * lc[1] + 64 * lc[2];
    if ((a.role[(size_t)slot * kNodes + node] & ROLE_MASK) != ROLE_GHOST) continue;
    float acc[kMom];
    interp_ghost(cq[0], lc, a.factor, acc);
    if (a.tape) keep_old<S>(a.dst, a.tape, slot, blockIdx.x, node);
    Mom<S>::store(a.dst, slot, node, a.sc, acc);
    interp_ghost(cq[1], lc, a.factor, acc);
    if (a.tape2) keep_old<S>(a.dst2, a.tape2, slot, blockIdx.x, node);
    Mom<S>::store(a.dst2, slot, node, a.sc, acc);
  }
}

template <class S>
__global__ __launch_bounds__(256) void k_upward(TransferLaunch a) {
  const int slot = a.blocks[blockIdx.x];
  const int4 bc = a.coord[slot];
  const int l = a.level;
  const LevelGeom& fg = a.G.lv[l];
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    if ((a.role[(size_t)slot * kNodes + node] & ROLE_MASK) != ROLE_IU) continue;
    const int f[3] = {2 * (bc.x * kEdge + (node & 7)), 2 * (bc.y * kEdge + ((node >> 3) & 7)), 2 * (bc.z * kEdge + (node >> 6))};
    const int fs = a.dir[fg.off + cell_lin(fg, f[0] >> 3, f[1] >> 3, f[2] >> 3)];
    if (fs < 0) continue;  // cannot happen for a valid hierarchy; never read out of bounds
    const int fn = (f[0] & 7) + 8 * (f[1] & 7) + 64 * (f[2] & 7);
    float q[kMom];
    Mom<S>::load(a.src_a, fs, fn, a.sc, q);
    to_neq(q);
#pragma unroll
    for (int m = 4; m < kMom; ++m) q[m] *= a.factor;
    from_neq(q);
    if (a.tape) keep_old<S>(a.dst, a.tape, slot, blockIdx.x, node);
    Mom<S>::store(a.dst, slot, node, a.sc, q);
  }
}

template <class S>
__global__ __launch_bounds__(256) void k_outflow(OutflowLaunch a) {
  const int slot = a.blocks[blockIdx.x];
  const int4 bc = a.coord[slot];
  const LevelGeom& lg = a.G.lv[a.level];
  typedef typename S::type T;
  const T* oldb = static_cast<const T*>(a.old_buf) + (size_t)slot * kBlockStride;
  T* newb = static_cast<T*>(a.new_buf) + (size_t)slot * kBlockStride;
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    if ((a.role[(size_t)slot * kNodes + node] & ROLE_MASK) != ROLE_OUTFLOW) continue;
    const int lc[3] = {node & 7, (node >> 3) & 7, node >> 6};
    const int g[3] = {bc.x * kEdge + lc[0], bc.y * kEdge + lc[1], bc.z * kEdge + lc[2]};
    // the first outflow face of the node (axis order): inward step, kind, outward sign
    int step = 0, kind = BC_OUTFLOW, sgn = 0, axn = 0;
    for (int ax = 0; ax < 3 && step == 0; ++ax) {
      if (a.G.periodic[ax]) continue;
      const int stride = ax == 0 ? 1 : (ax == 1 ? 8 : 64);
      if (g[ax] == 0 && is_outflow_bc(a.G.bc[2 * ax])) {
        step = stride; kind = a.G.bc[2 * ax]; sgn = -1; axn = ax;  // inward is +axis
      } else if (g[ax] == lg.nn[ax] - 1 && is_outflow_bc(a.G.bc[2 * ax + 1])) {
        step = -stride; kind = a.G.bc[2 * ax + 1]; sgn = 1; axn = ax;
      }
    }
    const int src = node + step;
    const bool computed = step != 0 && (a.role[(size_t)slot * kNodes + src] & ROLE_MASK) == ROLE_COMPUTED;
    if (a.tape) keep_old<S>(a.new_buf, a.tape, slot, blockIdx.x, node);
    if (!computed || kind == BC_OUTFLOW) {
      // zero gradient: the inward neighbour's new value (or the node's own)
#pragma unroll
      for (int m = 0; m < kMom; ++m) newb[m * kNodes + node] = computed ? newb[m * kNodes + src] : oldb[m * kNodes + node];
    } else {
      // convective (Sec. 7): one implicit upwind step of dM/dt + u_n dM/dn = 0
      float qh[kMom], qb[kMom];
#pragma unroll
      for (int m = 0; m < kMom; ++m) {
        qh[m] = Codec<S>::load(newb[m * kNodes + src], a.sc.inv[m]);
        qb[m] = Codec<S>::load(oldb[m * kNodes + node], a.sc.inv[m]);
      }
      const float un = sgn * qh[1 + axn];
      const float lam = un > 0.0f ? un : 0.0f;
#pragma unroll
      for (int m = 0; m < kMom; ++m)
        newb[m * kNodes + node] = Codec<S>::store((qb[m] + lam * qh[m]) / (1.0f + lam), a.sc.s[m]);
    }
  }
}

template <class S> hipError_t down_t(const TransferLaunch& a, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_downward<S>, dim3(a.nblocks), dim3(kDownThreads), 0, s, a);
  return hipGetLastError();
}
template <class S> hipError_t up_t(const TransferLaunch& a, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_upward<S>, dim3(a.nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <class S> hipError_t out_t(const OutflowLaunch& a, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_outflow<S>, dim3(a.nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_downward(const TransferLaunch& a, hipStream_t s) {
  switch (a.storage) {
    case 0: return down_t<StoreF32>(a, s);
    case 1: return down_t<StoreBF16>(a, s);
    case 2: return down_t<StoreF16>(a, s);
  }
  return hipErrorInvalidValue;
}
hipError_t launch_upward(const TransferLaunch& a, hipStream_t s) {
  switch (a.storage) {
    case 0: return up_t<StoreF32>(a, s);
    case 1: return up_t<StoreBF16>(a, s);
    case 2: return up_t<StoreF16>(a, s);
  }
  return hipErrorInvalidValue;
}
hipError_t launch_outflow(const OutflowLaunch& a, hipStream_t s) {
  switch (a.storage) {
    case 0: return out_t<StoreF32>(a, s);
    case 1: return out_t<StoreBF16>(a, s);
    case 2: return out_t<StoreF16>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbmx
