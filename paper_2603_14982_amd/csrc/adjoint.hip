// Hand-written adjoint of one coarse step (reverse mode, transposed Jacobians).
//
// Stream-collide: Y = F(M), M = L a(X) with L the (linear, integer) stream +
// projection operator and a the per-node coefficient map (collision included).
// The adjoint is computed in two passes over a level:
//   1. k_sc_mu: mu = (dF/dM)^T lambda_Y per computed node. F only divides by
//      216 rho' = 216 (1 + Y0), so mu needs the outputs Y, not the stencil;
//   2. k_sc_transpose applies L^T to mu (the same three 1D passes, transposed:
//      back-maps and shifts swap roles, x and y through LDS on a halo plane, z
//      over a register window) and adds (da/dX)^T (L^T mu) to lambda_X.
// The undo of every forward operation (the old values it overwrote, kept on a
// tape during the replay) is folded into the first adjoint kernel that runs after
// the values were last needed.
// Bounce-back adds, at a flagged computed node, populations built from the node's
// own coefficients; its transpose is a per-node term of the same sweep. Solid and
// inflow nodes hold fixed values and collect no adjoint.
// Interface transfers: the downward transfer is transposed per ghost block (the
// block's contribution to each coarse node under it, summed in LDS) and then per
// coarse node (a fixed-order sum of the at most eight ghost blocks' contributions);
// the upward transfer is a one-to-one scatter; both use the forward values they
// depend on.
// Every kernel is deterministic: no atomics, each output written by one lane.
#include "common.h"
#include "kernels.h"

namespace lbmx {
namespace {

// transposes of the 1D maps of the forward sweep (times-6 populations, p2' basis)
// back3: (P+,P0,P-) -> (P+ + P0 + P-, P+ - P-, 2(P+ + P-) - P0)
__device__ __forceinline__ void back3_t(float m0, float m1, float m2, float& pp, float& p0, float& pm) {
  pp = m0 + m1 + 2.0f * m2;
  p0 = m0 - m2;
  pm = m0 - m1 + 2.0f * m2;
}
// fwd3: (a0,a1,a2) -> (a0 + a1 + 2a2, 4(a0 - a2), a0 - a1 + 2a2)
__device__ __forceinline__ void fwd3_t(float pp, float p0, float pm, float& a0, float& a1, float& a2) {
  a0 = pp + 4.0f * p0 + pm;
  a1 = pp - pm;
  a2 = 2.0f * (pp + pm) - 4.0f * p0;
}

// adjoint of the division by 216 rho' at one computed node: Y0 = M0 / 216, Y_m =
// M_m / (216 + M0) (u and off-diagonal S; a further / 3 on the diagonal S), so
// mu_m = lambda_m dY_m/dM_m and mu_0 = lambda_0 / 216 - sum_m lambda_m Y_m / (216 + M0)
__device__ __forceinline__ void mu_of(const float Y[kMom], const float L[kMom], float g[kMom]) {
  const float inv = 1.0f / (216.0f * (1.0f + Y[0]));
  float dot = 0.0f;
#pragma unroll
  for (int m = 1; m < kMom; ++m) {
    g[m] = L[m] * ((m >= 4 && m <= 6) ? inv * (1.0f / 3.0f) : inv);
    dot += L[m] * Y[m];
  }
  g[0] = L[0] * (1.0f / 216.0f) - dot * inv;
}

template <class S> struct TrArgs {
  const typename S::type* x;  // forward input time level
  const float* mu;            // adjoint of M (one f32 time level, all-zero slot at zero_slot)
  float* lam_x;               // adjoint of the input time level (accumulated)
  const int32_t* blocks;
  const int32_t* nbr;
  const uint8_t* role;
  int32_t nblocks;
  int32_t zero_slot;
  int32_t zsplit;             // workgroups per block, each over 8 / zsplit output planes
  float omega;
  Scales sc;
  // FUSE: the next operation of the reverse sweep is the stream-collide of the same
  // level that wrote x; its first pass (k_sc_mu) is done here per output node
  typename S::type* x_next;    // = x, written: restored from tape_next
  const typename S::type* tape_next;
  float* mu_next;              // its mu (the other mu buffer)
};

// lambda_X += (da/dX)^T nu for one source node; nu[m] indexed [mx][my][mz]
__device__ inline void coeff_jacobian_t(const float q[kMom], float omega, const float nu[3][3][3], float lam[kMom]) {
  const float drho = q[0];
  const float rho = 1.0f + drho;
  const float u[3] = {q[1], q[2], q[3]};
  const float w1 = 1.0f - omega;
  float sp[3][3];
  sp[0][0] = q[4] + omega * (u[0] * u[0] - q[4]);
  sp[1][1] = q[5] + omega * (u[1] * u[1] - q[5]);
  sp[2][2] = q[6] + omega * (u[2] * u[2] - q[6]);
  sp[0][1] = sp[1][0] = q[7] + omega * (u[0] * u[1] - q[7]);
  sp[0][2] = sp[2][0] = q[8] + omega * (u[0] * u[2] - q[8]);
  sp[1][2] = sp[2][1] = q[9] + omega * (u[1] * u[2] - q[9]);
  // unit vectors of the per-axis index for the coefficient (a, a, b) of Gamma_aab:
  // index 2 on axis a, 1 on axis b
  float ub[3], spb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  float drb = nu[0][0][0];
  // first-order coefficients 3 rho u_a
  const float n1[3] = {nu[1][0][0], nu[0][1][0], nu[0][0][1]};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ub[a] = 3.0f * rho * n1[a];
    drb += 3.0f * u[a] * n1[a];
  }
  // diagonal second-order 1.5 rho Sp_aa
  const float n2[3] = {nu[2][0][0], nu[0][2][0], nu[0][0][2]};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    spb[a][a] += 1.5f * rho * n2[a];
    drb += 1.5f * sp[a][a] * n2[a];
  }
  // off-diagonal second-order 9 rho Sp_ab
  const float n11[3] = {nu[1][1][0], nu[1][0][1], nu[0][1][1]};
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    spb[pa[k]][pb[k]] += 9.0f * rho * n11[k];
    drb += 9.0f * sp[pa[k]][pb[k]] * n11[k];
  }
  // third order 4.5 rho Gamma_aab, Gamma_aab = Sp_aa u_b + 2 Sp_ab u_a - 2 u_a^2 u_b
  const int ga[6] = {0, 1, 0, 2, 1, 2}, gb[6] = {1, 0, 2, 0, 2, 1};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int a = ga[k], b = gb[k];
    int idx[3] = {0, 0, 0};
    idx[a] = 2;
    idx[b] = 1;
    const float n3 = nu[idx[0]][idx[1]][idx[2]];
    const float gam = sp[a][a] * u[b] + 2.0f * sp[a][b] * u[a] - 2.0f * u[a] * u[a] * u[b];
    drb += 4.5f * gam * n3;
    const float gbar = 4.5f * rho * n3;
    spb[a][a] += gbar * u[b];
    ub[b] += gbar * (sp[a][a] - 2.0f * u[a] * u[a]);
    spb[a < b ? a : b][a < b ? b : a] += 2.0f * gbar * u[a];
    ub[a] += gbar * (2.0f * sp[a][b] - 4.0f * u[a] * u[b]);
  }
  // 27 rho Gamma_xyz, Gamma_xyz = Sp_xy u_z + Sp_xz u_y + Sp_yz u_x - 2 u_x u_y u_z
  {
    const float n3 = nu[1][1][1];
    const float gam = sp[0][1] * u[2] + sp[0][2] * u[1] + sp[1][2] * u[0] - 2.0f * u[0] * u[1] * u[2];
    drb += 27.0f * gam * n3;
    const float gbar = 27.0f * rho * n3;
    spb[0][1] += gbar * u[2];
    spb[0][2] += gbar * u[1];
    spb[1][2] += gbar * u[0];
    ub[2] += gbar * (sp[0][1] - 2.0f * u[0] * u[1]);
    ub[1] += gbar * (sp[0][2] - 2.0f * u[0] * u[2]);
    ub[0] += gbar * (sp[1][2] - 2.0f * u[1] * u[2]);
  }
  // collision Sp = (1 - omega) S + omega u u
#pragma unroll
  for (int a = 0; a < 3; ++a) ub[a] += 2.0f * omega * u[a] * spb[a][a];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float g = spb[pa[k]][pb[k]];
    ub[pa[k]] += omega * u[pb[k]] * g;
    ub[pb[k]] += omega * u[pa[k]] * g;
  }
  lam[0] += drb;
  lam[1] += ub[0]; lam[2] += ub[1]; lam[3] += ub[2];
  lam[4] += w1 * spb[0][0]; lam[5] += w1 * spb[1][1]; lam[6] += w1 * spb[2][2];
  lam[7] += w1 * spb[0][1]; lam[8] += w1 * spb[0][2]; lam[9] += w1 * spb[1][2];
}

// transpose of the bounce-back correction of one computed node: the node's own
// coefficients receive, for every direction c whose source x - c is solid (or
// behind a wall), w_c (mu . e(c)) times the basis values at the outgoing -c
template <class S>
__device__ void bounce_back_t(const TrArgs<S>& a, int slot, int lx, int ly, int lz, float nu[3][3][3]) {
  const int32_t* nbr = a.nbr + (size_t)slot * 27;
  const int node = lx + 8 * ly + 64 * lz;
  const float* mp = a.mu + (size_t)slot * kBlockStride + node;
  float g[kMom];
#pragma unroll
  for (int m = 0; m < kMom; ++m) g[m] = mp[m * kNodes];
#pragma unroll 1
  for (int i = 0; i < 27; ++i) {
    if (i == 13) continue;
    const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
    const int hx = lx - cx, hy = ly - cy, hz = lz - cz;
    const int ox = hx < 0 ? -1 : (hx > 7 ? 1 : 0);
    const int oy = hy < 0 ? -1 : (hy > 7 ? 1 : 0);
    const int oz = hz < 0 ? -1 : (hz > 7 ? 1 : 0);
    const int ns = nbr[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)];
    bool solid = (ns == NBR_WALL);
    if (ns >= 0) solid = (a.role[(size_t)ns * kNodes + (hx & 7) + 8 * (hy & 7) + 64 * (hz & 7)] & ROLE_MASK) == ROLE_SOLID;
    if (!solid) continue;
    const float fx = (float)cx, fy = (float)cy, fz = (float)cz;
    const float pe = g[0] + g[1] * fx + g[2] * fy + g[3] * fz + g[4] * (3.0f * fx * fx - 1.0f)
                     + g[5] * (3.0f * fy * fy - 1.0f) + g[6] * (3.0f * fz * fz - 1.0f) + g[7] * fx * fy
                     + g[8] * fx * fz + g[9] * fy * fz;
    const float w = (cx ? 1.0f : 4.0f) * (cy ? 1.0f : 4.0f) * (cz ? 1.0f : 4.0f);
    const float fb = w * pe;
    const float px[3] = {1.0f, -fx, 3.0f * fx * fx - 1.0f};
    const float py[3] = {1.0f, -fy, 3.0f * fy * fy - 1.0f};
    const float pz[3] = {1.0f, -fz, 3.0f * fz * fz - 1.0f};
#pragma unroll
    for (int mx = 0; mx < 3; ++mx)
#pragma unroll
      for (int my = 0; my < 3; ++my)
#pragma unroll
        for (int mz = 0; mz < 3; ++mz) nu[mx][my][mz] += fb * px[mx] * py[my] * pz[mz];
  }
}

// LDS plane rows as in the forward sweep: row r = plane row y + 1
//   x-pass input: [kind][col 0..9][group 0..5]   (180 floats)
//   y-pass input: [kind][col 0..7][triple 0..8, pad 10] (240 floats)
constexpr int kRowT = 240;
__device__ __forceinline__ int ta_off(int row, int kind, int col) { return row * kRowT + kind * 60 + col * 6; }
__device__ __forceinline__ int tb_off(int row, int kind, int col) { return row * kRowT + kind * 80 + col * 10; }

__device__ __forceinline__ bool plane_point_t(int lane, int r, int& px, int& py) {
  if (r == 0) { px = lane & 7; py = lane >> 3; return true; }
  if (lane < 10) { px = lane - 1; py = -1; return true; }
  if (lane < 20) { px = lane - 11; py = 8; return true; }
  if (lane < 28) { px = -1; py = lane - 20; return true; }
  if (lane < 36) { px = 8; py = lane - 28; return true; }
  return false;
}

__device__ __forceinline__ void x_pass_t(const float* lds, int row, int x, float yb[27]) {
  float E[3][6];
#pragma unroll
  for (int g = 0; g < 6; ++g) {
    const float pp = lds[ta_off(row, 0, x + 2) + g];  // P+ of column x+1
    const float pz = lds[ta_off(row, 1, x + 1) + g];  // P0 of column x
    const float pm = lds[ta_off(row, 2, x) + g];      // P- of column x-1
    fwd3_t(pp, pz, pm, E[0][g], E[1][g], E[2][g]);
  }
  // (qy, qz) groups: 0 (0,0), 1 (1,0), 2 (0,1), 3 (2,0), 4 (0,2), 5 (1,1)
#pragma unroll
  for (int mx = 0; mx < 3; ++mx) {
    float pp, pz, pm;
    back3_t(E[mx][0], E[mx][1], E[mx][3], pp, pz, pm);  // qz = 0, qy = 0,1,2
    yb[3 * mx + 0] = pp; yb[9 + 3 * mx + 0] = pz; yb[18 + 3 * mx + 0] = pm;
    back3_t(E[mx][2], E[mx][5], 0.0f, pp, pz, pm);      // qz = 1, qy = 0,1
    yb[3 * mx + 1] = pp; yb[9 + 3 * mx + 1] = pz; yb[18 + 3 * mx + 1] = pm;
    back3_t(E[mx][4], 0.0f, 0.0f, pp, pz, pm);          // qz = 2, qy = 0
    yb[3 * mx + 2] = pp; yb[9 + 3 * mx + 2] = pz; yb[18 + 3 * mx + 2] = pm;
  }
}

__device__ __forceinline__ int xcd_remap_t(int bid, int n) {
  const int per = n >> 3, rem = n & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

// One workgroup per block and z range: output planes zlo .. zlo + zn - 1 take the
// planes zlo - 1 .. zlo + zn (the window of the z pass); every output node has one
// writer. The parts of a block go to neighbouring workgroup indices after the remap,
// which places them on one XCD (one L2) except at the ends of an XCD's range.
// FUSE: each output node, once its adjoint is final, also gets the next operation's
// first pass (the same node's mu, adjoint cleared, value restored), as k_sc_mu would
// do right after this kernel; mu itself is read from the other buffer, so no
// workgroup's halo reads see the new values.
template <class S, bool FUSE>
__global__ __launch_bounds__(64) void k_sc_transpose(TrArgs<S> a) {
  __shared__ __align__(16) float lds[10 * kRowT];
  __shared__ int s_src[27];
  const int lane = threadIdx.x;
  const int item = xcd_remap_t(blockIdx.x, a.nblocks * a.zsplit);
  const int slot = a.blocks[item / a.zsplit];
  const int zn = 8 / a.zsplit;
  const int zlo = (item % a.zsplit) * zn;
  if (lane < 27) {
    const int ns = a.nbr[(size_t)slot * 27 + lane];
    s_src[lane] = ns >= 0 ? ns : a.zero_slot;
  }
  __syncthreads();
  int px[2], py[2];
  bool has[2];
  has[0] = plane_point_t(lane, 0, px[0], py[0]);
  has[1] = plane_point_t(lane, 1, px[1], py[1]);
  const int ox = lane & 7, oy = lane >> 3;

  // z window over the 8 (mx, my) pairs: P0 of plane z-1, P- of planes z-1 and z-2
  float w0[8], wm1[8], wm2[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) w0[k] = wm1[k] = wm2[k] = 0.0f;
  const int pmx[8] = {0, 1, 2, 0, 1, 2, 0, 1};
  const int pmy[8] = {0, 0, 0, 1, 1, 1, 2, 2};

  // mu of a plane point, one plane ahead of its use
  auto load_mu = [&](int r, int z, float m[kMom]) {
    const int ox_ = px[r] < 0 ? -1 : (px[r] > 7 ? 1 : 0);
    const int oy_ = py[r] < 0 ? -1 : (py[r] > 7 ? 1 : 0);
    const int oz_ = z < 0 ? -1 : (z > 7 ? 1 : 0);
    const int ns = s_src[(ox_ + 1) + 3 * (oy_ + 1) + 9 * (oz_ + 1)];
    const float* src = a.mu + (size_t)ns * kBlockStride + (px[r] & 7) + 8 * (py[r] & 7) + 64 * (z & 7);
#pragma unroll
    for (int k = 0; k < kMom; ++k) m[k] = src[k * kNodes];
  };
  float mnxt[2][kMom];
#pragma unroll
  for (int r = 0; r < 2; ++r)
    if (has[r]) load_mu(r, zlo - 1, mnxt[r]);

  for (int z = zlo - 1; z <= zlo + zn; ++z) {
    // ---- the output node of this plane (zo = z - 1): role, state and adjoint, loaded
    // before the passes so that the loads overlap them
    const int zo = z - 1;
    const int onode = ox + 8 * oy + 64 * (zo < zlo ? zlo : zo);
    const uint8_t orole = zo >= zlo ? a.role[(size_t)slot * kNodes + onode] : (uint8_t)ROLE_SOLID;
    const uint8_t orm = orole & ROLE_MASK;
    const bool oact = zo >= zlo && orm != ROLE_SOLID && orm != ROLE_INFLOW;
    typename S::type xq[kMom];
    float L[kMom];
    if (oact) {
      const typename S::type* xs = a.x + (size_t)slot * kBlockStride + onode;
      const float* lam = a.lam_x + (size_t)slot * kBlockStride + onode;
#pragma unroll
      for (int m = 0; m < kMom; ++m) {
        xq[m] = xs[m * kNodes];
        L[m] = lam[m * kNodes];
      }
    }
    // FUSE: the next operation's old values of this node (its undo), loaded with the rest
    typename S::type tn[kMom];
    if (FUSE && zo >= zlo && (orm == ROLE_COMPUTED || orm == ROLE_SOLID)) {
      const typename S::type* tp = a.tape_next + (size_t)(item / a.zsplit) * kBlockStride + onode;
#pragma unroll
      for (int m = 0; m < kMom; ++m) tn[m] = tp[m * kNodes];
    }
    // ---- mu of plane z (+ halo) -> transposed x back-map per (qy, qz) group
    float mcur[2][kMom];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < kMom; ++k) mcur[r][k] = mnxt[r][k];
    if (z < zlo + zn) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (has[r]) load_mu(r, z + 1, mnxt[r]);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (!has[r]) continue;
      const float* m = mcur[r];
      float P[3][6];
      back3_t(m[0], m[1], m[4], P[0][0], P[1][0], P[2][0]);  // (qy,qz) = (0,0): mu000, mu100, mu200
      back3_t(m[2], m[7], 0.0f, P[0][1], P[1][1], P[2][1]);  // (1,0): mu010, mu110
      back3_t(m[3], m[8], 0.0f, P[0][2], P[1][2], P[2][2]);  // (0,1): mu001, mu101
      back3_t(m[5], 0.0f, 0.0f, P[0][3], P[1][3], P[2][3]);  // (2,0): mu020
      back3_t(m[6], 0.0f, 0.0f, P[0][4], P[1][4], P[2][4]);  // (0,2): mu002
      back3_t(m[9], 0.0f, 0.0f, P[0][5], P[1][5], P[2][5]);  // (1,1): mu011
      const int row = py[r] + 1, col = px[r] + 1;
#pragma unroll
      for (int kind = 0; kind < 3; ++kind)
#pragma unroll
        for (int g = 0; g < 6; ++g) lds[ta_off(row, kind, col) + g] = P[kind][g];
    }
    __syncthreads();
    // ---- x pass (rows 0..7, then 8..9), each row overwritten by its own y-pass input
    {
      float yb[27];
      x_pass_t(lds, oy, ox, yb);
      __syncthreads();
#pragma unroll
      for (int kind = 0; kind < 3; ++kind)
#pragma unroll
        for (int t = 0; t < 9; ++t) lds[tb_off(oy, kind, ox) + t] = yb[9 * kind + t];
    }
    {
      float yb[27];
      const int row = 8 + (oy & 1);
      x_pass_t(lds, row, ox, yb);
      __syncthreads();
      if (lane < 16) {
#pragma unroll
        for (int kind = 0; kind < 3; ++kind)
#pragma unroll
          for (int t = 0; t < 9; ++t) lds[tb_off(row, kind, ox) + t] = yb[9 * kind + t];
      }
    }
    __syncthreads();
    // ---- y pass for the owned column, then transposed z back-map per (mx, my)
    float cp[8], cz[8], cm[8];
    {
      float F[3][3][3];  // [mx][my][qz]
#pragma unroll
      for (int mx = 0; mx < 3; ++mx)
#pragma unroll
        for (int qz = 0; qz < 3; ++qz) {
          const int t = 3 * mx + qz;
          const float pp = lds[tb_off(oy + 2, 0, ox) + t];  // P+ of row y+1
          const float pz = lds[tb_off(oy + 1, 1, ox) + t];  // P0 of row y
          const float pm = lds[tb_off(oy, 2, ox) + t];      // P- of row y-1
          fwd3_t(pp, pz, pm, F[mx][0][qz], F[mx][1][qz], F[mx][2][qz]);
        }
#pragma unroll
      for (int k = 0; k < 8; ++k) back3_t(F[pmx[k]][pmy[k]][0], F[pmx[k]][pmy[k]][1], F[pmx[k]][pmy[k]][2], cp[k], cz[k], cm[k]);
    }
    __syncthreads();
    // ---- z pass: source plane zo = z - 1 takes P+ of plane z, P0 of z-1, P- of z-2
    if (oact) {
      float nu[3][3][3];
#pragma unroll
      for (int k = 0; k < 8; ++k) fwd3_t(cp[k], w0[k], wm2[k], nu[pmx[k]][pmy[k]][0], nu[pmx[k]][pmy[k]][1], nu[pmx[k]][pmy[k]][2]);
      nu[2][2][0] = nu[2][2][1] = nu[2][2][2] = 0.0f;
      if (orm == ROLE_COMPUTED && (orole & ROLE_BB)) bounce_back_t<S>(a, slot, ox, oy, zo, nu);
      float q[kMom];
#pragma unroll
      for (int m = 0; m < kMom; ++m) q[m] = Codec<S>::load(xq[m], a.sc.inv[m]);
      coeff_jacobian_t(q, a.omega, nu, L);
      float* lam = a.lam_x + (size_t)slot * kBlockStride + onode;
      if (FUSE && orm == ROLE_COMPUTED) {
        float g[kMom];
        mu_of(q, L, g);
        typename S::type* xw = a.x_next + (size_t)slot * kBlockStride + onode;
        float* mn = a.mu_next + (size_t)slot * kBlockStride + onode;
#pragma unroll
        for (int m = 0; m < kMom; ++m) {
          lam[m * kNodes] = 0.0f;
          xw[m * kNodes] = tn[m];
          mn[m * kNodes] = g[m];
        }
      } else {
#pragma unroll
        for (int m = 0; m < kMom; ++m) lam[m * kNodes] = L[m];
        if (FUSE) {
          float* mn = a.mu_next + (size_t)slot * kBlockStride + onode;
#pragma unroll
          for (int m = 0; m < kMom; ++m) mn[m * kNodes] = 0.0f;
        }
      }
    } else if (FUSE && zo >= zlo) {
      // solid or inflow node: no adjoint of its own; a solid node is restored
      float* mn = a.mu_next + (size_t)slot * kBlockStride + onode;
      if (orm == ROLE_SOLID) {
        float* lam = a.lam_x + (size_t)slot * kBlockStride + onode;
        typename S::type* xw = a.x_next + (size_t)slot * kBlockStride + onode;
#pragma unroll
        for (int m = 0; m < kMom; ++m) {
          lam[m * kNodes] = 0.0f;
          xw[m * kNodes] = tn[m];
        }
      }
#pragma unroll
      for (int m = 0; m < kMom; ++m) mn[m * kNodes] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      wm2[k] = wm1[k];
      wm1[k] = cm[k];
      w0[k] = cz[k];
    }
  }
}

// ---- adjoint of the division by 216 rho' (per computed node, mu_of); the outputs
// are then restored from the tape and their adjoint cleared
template <class S>
__global__ __launch_bounds__(kNodes) void k_sc_mu(AdjScLaunch a) {
  typedef typename S::type T;
  const int slot = a.blocks[blockIdx.x];
  T* y = static_cast<T*>(a.y) + (size_t)slot * kBlockStride;
  const T* tp = static_cast<const T*>(a.tape) + (size_t)blockIdx.x * kBlockStride;
  float* lam = a.lam_y + (size_t)slot * kBlockStride;
  float* mu = a.mu + (size_t)slot * kBlockStride;
  for (int node = threadIdx.x; node < kNodes; node += kNodes) {
    const uint8_t r = a.role[(size_t)slot * kNodes + node] & ROLE_MASK;
    float g[kMom];
#pragma unroll
    for (int m = 0; m < kMom; ++m) g[m] = 0.0f;
    if (r == ROLE_COMPUTED) {
      float Y[kMom], L[kMom];
#pragma unroll
      for (int m = 0; m < kMom; ++m) {
        Y[m] = Codec<S>::load(y[m * kNodes + node], a.sc.inv[m]);
        L[m] = lam[m * kNodes + node];
      }
      mu_of(Y, L, g);
    }
    if (r == ROLE_COMPUTED || r == ROLE_SOLID) {
#pragma unroll
      for (int m = 0; m < kMom; ++m) {
        lam[m * kNodes + node] = 0.0f;
        y[m * kNodes + node] = tp[m * kNodes + node];
      }
    }
#pragma unroll
    for (int m = 0; m < kMom; ++m) mu[m * kNodes + node] = g[m];
  }
}

// restore the node's pre-operation value from the tape entry of list index idx
template <class S>
__device__ inline void undo_node(void* buf, const void* tape, int slot, int idx, int node) {
  typename S::type* p = static_cast<typename S::type*>(buf) + (size_t)slot * kBlockStride + node;
  const typename S::type* t = static_cast<const typename S::type*>(tape) + (size_t)idx * kBlockStride + node;
#pragma unroll
  for (int m = 0; m < kMom; ++m) p[m * kNodes] = t[m * kNodes];
}

// ---- downward transfer, transposed --------------------------------------------
// One forward launch wrote the ghosts of both fine substeps: s = 1 from coarse t
// (src_a) into undo_dst, s = 2 from the midpoint of t and t + 2 into undo_dst2.
// (a) one workgroup per ghost block of level l: adjoint of every ghost's moments ->
//     adjoint of its interpolated (rho-1, u, S^neq) (the u u term needs the
//     interpolated u of its substep); ghost adjoints cleared and ghost values
//     restored; the s = 2 part splits evenly over the two coarse time levels, so
//     per ghost node ga = g1 + g2 / 2 goes to t and gb = g2 / 2 to t + 2 (in LDS);
//     then the block's contribution to each of the 5^3 coarse nodes under it (the
//     transposed trilinear weights, a fixed-order sum over <= 27 ghosts), written
//     to the partials [list index][10][125] of t (scratch) and of t + 2 (scratch2).
template <class S>
__global__ __launch_bounds__(kNodes) void k_down_adj_lin(AdjTransferLaunch a) {
  __shared__ float cu[2][3][125];
  __shared__ float gl[2][kMom][kNodes];
  const int slot = a.blocks[blockIdx.x];
  const int4 bc = a.coord[slot];
  const int l = a.level;
  const LevelGeom& cg = a.G.lv[l + 1];
  const int base[3] = {4 * bc.x, 4 * bc.y, 4 * bc.z};
  typedef typename S::type T;
  for (int t = threadIdx.x; t < 125; t += kNodes) {
    int j[3] = {base[0] + t % 5, base[1] + (t / 5) % 5, base[2] + t / 25};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int nc = cg.nn[ax];
      if (a.G.periodic[ax]) j[ax] = j[ax] >= nc ? j[ax] - nc : j[ax];
      else j[ax] = j[ax] >= nc ? nc - 1 : j[ax];
    }
    const int cs = a.dir[cg.off + cell_lin(cg, j[0] >> 3, j[1] >> 3, j[2] >> 3)];
    float u[3] = {0.0f, 0.0f, 0.0f}, h[3] = {0.0f, 0.0f, 0.0f};
    if (cs >= 0) {
      const int cn = (j[0] & 7) + 8 * (j[1] & 7) + 64 * (j[2] & 7);
      const T* pa = static_cast<const T*>(a.src_a) + (size_t)cs * kBlockStride + cn;
      const T* pb = static_cast<const T*>(a.src_b) + (size_t)cs * kBlockStride + cn;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        u[k] = Codec<S>::load(pa[(1 + k) * kNodes], a.sc.inv[1 + k]);
        h[k] = 0.5f * (u[k] + Codec<S>::load(pb[(1 + k) * kNodes], a.sc.inv[1 + k]));
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cu[0][k][t] = u[k];
      cu[1][k][t] = h[k];
    }
  }
  __syncthreads();
  const size_t boff = (size_t)slot * kBlockStride;
  const size_t toff = (size_t)blockIdx.x * kBlockStride;
  for (int node = threadIdx.x; node < kNodes; node += kNodes) {
    float ga[kMom], gb[kMom];
#pragma unroll
    for (int m = 0; m < kMom; ++m) ga[m] = gb[m] = 0.0f;
    if ((a.role[(size_t)slot * kNodes + node] & ROLE_MASK) == ROLE_GHOST) {
      const int lc[3] = {node & 7, (node >> 3) & 7, node >> 6};
#pragma unroll
      for (int sub = 0; sub < 2; ++sub) {
        float* lamb = (sub ? a.lam_fine2 : a.lam_fine) + boff;
        T* dstb = static_cast<T*>(sub ? a.undo_dst2 : a.undo_dst) + boff;
        const T* tapeb = static_cast<const T*>(sub ? a.undo_tape2 : a.undo_tape) + toff;
        float L[kMom];
        T old[kMom];
#pragma unroll
        for (int m = 0; m < kMom; ++m) {
          L[m] = lamb[m * kNodes + node];
          old[m] = tapeb[m * kNodes + node];
        }
        float ug[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int kx = c & 1, ky = (c >> 1) & 1, kz = c >> 2;
          const float wx = (lc[0] & 1) ? 0.5f : (kx ? 0.0f : 1.0f);
          const float wy = (lc[1] & 1) ? 0.5f : (ky ? 0.0f : 1.0f);
          const float wz = (lc[2] & 1) ? 0.5f : (kz ? 0.0f : 1.0f);
          const float w = wx * wy * wz;
          if (w == 0.0f) continue;
          const int t = ((lc[0] + kx) >> 1) + 5 * ((lc[1] + ky) >> 1) + 25 * ((lc[2] + kz) >> 1);
#pragma unroll
          for (int k = 0; k < 3; ++k) ug[k] += w * cu[sub][k][t];
        }
        float g[kMom];
        g[0] = L[0];
        g[1] = L[1] + 2.0f * L[4] * ug[0] + L[7] * ug[1] + L[8] * ug[2];
        g[2] = L[2] + 2.0f * L[5] * ug[1] + L[7] * ug[0] + L[9] * ug[2];
        g[3] = L[3] + 2.0f * L[6] * ug[2] + L[8] * ug[0] + L[9] * ug[1];
#pragma unroll
        for (int m = 4; m < kMom; ++m) g[m] = a.factor * L[m];
        if (sub == 0) {
#pragma unroll
          for (int m = 0; m < kMom; ++m) ga[m] = g[m];
        } else {
#pragma unroll
          for (int m = 0; m < kMom; ++m) {
            ga[m] += 0.5f * g[m];
            gb[m] = 0.5f * g[m];
          }
        }
#pragma unroll
        for (int m = 0; m < kMom; ++m) {
          lamb[m * kNodes + node] = 0.0f;
          dstb[m * kNodes + node] = old[m];
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kMom; ++m) {
      gl[0][m][node] = ga[m];
      gl[1][m][node] = gb[m];
    }
  }
  __syncthreads();
  // footprint node t (coarse 4b + t per axis) collects fine local 2t-1, 2t, 2t+1
  // (weights 1/2, 1, 1/2) that lie inside the block; threads 0..124 take the
  // partial of t, threads 128..252 that of t + 2
  if (threadIdx.x >= 256) return;
  const int tl = threadIdx.x >> 7;
  const int t = threadIdx.x & 127;
  if (t >= 125) return;
  const int tt[3] = {t % 5, (t / 5) % 5, t / 25};
  float acc[kMom];
#pragma unroll
  for (int m = 0; m < kMom; ++m) acc[m] = 0.0f;
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = 2 * tt[2] + dz;
    if (z < 0 || z > 7) continue;
    const float wz = dz ? 0.5f : 1.0f;
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = 2 * tt[1] + dy;
      if (y < 0 || y > 7) continue;
      const float wy = dy ? 0.5f : 1.0f;
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = 2 * tt[0] + dx;
        if (x < 0 || x > 7) continue;
        const float w = wz * wy * (dx ? 0.5f : 1.0f);
        const int n = x + 8 * y + 64 * z;
#pragma unroll
        for (int m = 0; m < kMom; ++m) acc[m] += w * gl[tl][m][n];
      }
    }
  }
  float* part = (tl ? a.scratch2 : a.scratch) + (size_t)blockIdx.x * (kMom * 125);
#pragma unroll
  for (int m = 0; m < kMom; ++m) part[m * 125 + t] = acc[m];
}

// (b) per coarse node of a flagged level-(l+1) block: for each coarse time level,
//     the sum of its partials from the <= 2 x 2 x 2 ghost blocks whose footprint
//     holds the node (fixed order), then the Jacobian of lin = (rho-1, u, S - u u)
//     at that time level
template <class S>
__global__ __launch_bounds__(kNodes) void k_down_adj_gather(AdjTransferLaunch a) {
  const int cslot = a.blocks[blockIdx.x];
  if (!a.flags[cslot]) return;  // no ghost of level l interpolates from this block
  const int4 bc = a.coord[cslot];
  const int l = a.level;
  const LevelGeom& fg = a.G.lv[l];
  const LevelGeom& cg = a.G.lv[l + 1];
  typedef typename S::type T;
  for (int node = threadIdx.x; node < kNodes; node += kNodes) {
    const int j[3] = {bc.x * kEdge + (node & 7), bc.y * kEdge + ((node >> 3) & 7), bc.z * kEdge + (node >> 6)};
    // per axis: (fine block, footprint index) pairs whose staged coarse index is j
    int nb[3], fb[3][2], ft[3][2];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int nbf = fg.nb[ax], nc = cg.nn[ax];
      int k = 0;
      fb[ax][k] = j[ax] >> 2; ft[ax][k] = j[ax] & 3; ++k;
      if ((j[ax] & 3) == 0) {
        const int b = (j[ax] >> 2) - 1;
        if (b >= 0) { fb[ax][k] = b; ft[ax][k] = 4; ++k; }
        else if (a.G.periodic[ax]) { fb[ax][k] = nbf - 1; ft[ax][k] = 4; ++k; }
      }
      if (!a.G.periodic[ax] && j[ax] == nc - 1) { fb[ax][k] = nbf - 1; ft[ax][k] = 4; ++k; }
      nb[ax] = k;
    }
    float acc[2][kMom];
#pragma unroll
    for (int m = 0; m < kMom; ++m) acc[0][m] = acc[1][m] = 0.0f;
    bool any = false;
    for (int iz = 0; iz < nb[2]; ++iz)
      for (int iy = 0; iy < nb[1]; ++iy)
        for (int ix = 0; ix < nb[0]; ++ix) {
          const int fs = a.dir[fg.off + cell_lin(fg, fb[0][ix], fb[1][iy], fb[2][iz])];
          if (fs < 0) continue;
          const int gi = a.gidx[fs];
          if (gi < 0) continue;
          const size_t po = (size_t)gi * (kMom * 125) + ft[0][ix] + 5 * ft[1][iy] + 25 * ft[2][iz];
#pragma unroll
          for (int m = 0; m < kMom; ++m) {
            acc[0][m] += a.scratch[po + m * 125];
            acc[1][m] += a.scratch2[po + m * 125];
          }
          any = true;
        }
    if (!any) continue;
#pragma unroll
    for (int tl = 0; tl < 2; ++tl) {
      const T* qs = static_cast<const T*>(tl == 0 ? a.src_a : a.src_b) + (size_t)cslot * kBlockStride + node;
      float* lam = (tl == 0 ? a.lam_coarse_a : a.lam_coarse_b) + (size_t)cslot * kBlockStride + node;
      const float* g = acc[tl];
      float u[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) u[k] = Codec<S>::load(qs[(1 + k) * kNodes], a.sc.inv[1 + k]);
      const float gu0 = g[1] - (2.0f * g[4] * u[0] + g[7] * u[1] + g[8] * u[2]);
      const float gu1 = g[2] - (2.0f * g[5] * u[1] + g[7] * u[0] + g[9] * u[2]);
      const float gu2 = g[3] - (2.0f * g[6] * u[2] + g[8] * u[0] + g[9] * u[1]);
      lam[0] += g[0];
      lam[kNodes] += gu0;
      lam[2 * kNodes] += gu1;
      lam[3 * kNodes] += gu2;
#pragma unroll
      for (int m = 4; m < kMom; ++m) lam[m * kNodes] += g[m];
    }
  }
}

// ghost-list index of every ghost block of a level (gidx[slot]; -1 elsewhere)
__global__ void k_ghost_index(const int32_t* blocks, int32_t n, int32_t* gidx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) gidx[blocks[i]] = i;
}

// flags the level-(l+1) blocks under the 5^3 coarse-node footprint of every ghost
// block of level l (the nodes its ghosts interpolate from); every writer stores 1
__global__ void k_mark_gather(AdjTransferLaunch a) {
  const int slot = a.blocks[blockIdx.x];
  const int4 bc = a.coord[slot];
  const LevelGeom& cg = a.G.lv[a.level + 1];
  const int t = threadIdx.x;
  if (t >= 8) return;
  int j[3] = {4 * bc.x + 4 * (t & 1), 4 * bc.y + 4 * ((t >> 1) & 1), 4 * bc.z + 4 * (t >> 2)};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int nc = cg.nn[ax];
    if (a.G.periodic[ax]) j[ax] = j[ax] >= nc ? j[ax] - nc : j[ax];
    else j[ax] = j[ax] >= nc ? nc - 1 : j[ax];
  }
  const int cs = a.dir[cg.off + cell_lin(cg, j[0] >> 3, j[1] >> 3, j[2] >> 3)];
  if (cs >= 0) a.flags[cs] = 1;
}

// ---- upward transfer, transposed ------------------------------------------------
template <class S>
__global__ __launch_bounds__(kNodes) void k_up_adj(AdjTransferLaunch a) {
  const int slot = a.blocks[blockIdx.x];
  const int4 bc = a.coord[slot];
  const LevelGeom& fg = a.G.lv[a.level];
  typedef typename S::type T;
  const float f = a.factor;
  for (int node = threadIdx.x; node < kNodes; node += kNodes) {
    if ((a.role[(size_t)slot * kNodes + node] & ROLE_MASK) != ROLE_IU) continue;
    const int p[3] = {2 * (bc.x * kEdge + (node & 7)), 2 * (bc.y * kEdge + ((node >> 3) & 7)), 2 * (bc.z * kEdge + (node >> 6))};
    const int fs = a.dir[fg.off + cell_lin(fg, p[0] >> 3, p[1] >> 3, p[2] >> 3)];
    if (fs < 0) continue;
    const int fn = (p[0] & 7) + 8 * (p[1] & 7) + 64 * (p[2] & 7);
    float* lq = a.lam_coarse_a + (size_t)slot * kBlockStride + node;
    float L[kMom];
#pragma unroll
    for (int m = 0; m < kMom; ++m) { L[m] = lq[m * kNodes]; lq[m * kNodes] = 0.0f; }
    undo_node<S>(a.undo_dst, a.undo_tape, slot, blockIdx.x, node);
    const T* qs = static_cast<const T*>(a.src_a) + (size_t)fs * kBlockStride + fn;
    float u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = Codec<S>::load(qs[(1 + k) * kNodes], a.sc.inv[1 + k]);
    // S_q = f S_f + (1 - f) u_f u_f
    const float h = 1.0f - f;
    float* lf = a.lam_fine + (size_t)fs * kBlockStride + fn;
    lf[0] += L[0];
    lf[kNodes] += L[1] + h * (2.0f * L[4] * u[0] + L[7] * u[1] + L[8] * u[2]);
    lf[2 * kNodes] += L[2] + h * (2.0f * L[5] * u[1] + L[7] * u[0] + L[9] * u[2]);
    lf[3 * kNodes] += L[3] + h * (2.0f * L[6] * u[2] + L[8] * u[0] + L[9] * u[1]);
#pragma unroll
    for (int m = 4; m < kMom; ++m) lf[m * kNodes] += f * L[m];
  }
}

// ---- outflow conditions, transposed ----------------------------------------------
// Phase 1: every outflow node hands its adjoint to its inward computed neighbour
// (through LDS) and to its own old value: all of it to one of them for the zero-
// gradient copy; for the convective step y = (x + lam h) / (1 + lam), lam =
// max(s h_n, 0) (x the node's old value, h the neighbour's new value, s the outward
// sign), 1 / (1 + lam) of it to x and lam / (1 + lam) to h, plus the derivative
// through lam, sum_m ybar_m (h_m - x_m) / (1 + lam)^2 times s, to h_n where lam > 0.
// Phase 2: every computed node collects from the outflow nodes that read it (at most
// one per face).
__device__ inline int outflow_src(const Geom& G, const LevelGeom& lg, const int4 bc, const uint8_t* role, int node,
                                  int& kind, int& sgn, int& axn) {
  const int g[3] = {bc.x * kEdge + (node & 7), bc.y * kEdge + ((node >> 3) & 7), bc.z * kEdge + (node >> 6)};
  int step = 0;
  kind = BC_OUTFLOW;
  sgn = 0;
  axn = 0;
  for (int ax = 0; ax < 3 && step == 0; ++ax) {
    if (G.periodic[ax]) continue;
    const int stride = ax == 0 ? 1 : (ax == 1 ? 8 : 64);
    if (g[ax] == 0 && is_outflow_bc(G.bc[2 * ax])) {
      step = stride; kind = G.bc[2 * ax]; sgn = -1; axn = ax;
    } else if (g[ax] == lg.nn[ax] - 1 && is_outflow_bc(G.bc[2 * ax + 1])) {
      step = -stride; kind = G.bc[2 * ax + 1]; sgn = 1; axn = ax;
    }
  }
  if (step == 0) return -1;
  const int src = node + step;
  return (role[src] & ROLE_MASK) == ROLE_COMPUTED ? src : -1;
}

template <class S>
__global__ __launch_bounds__(256) void k_outflow_adj(AdjTransferLaunch a) {
  __shared__ float sv[kMom][kNodes];
  __shared__ int16_t sdst[kNodes];
  const int slot = a.blocks[blockIdx.x];
  const int4 bc = a.coord[slot];
  const LevelGeom& lg = a.G.lv[a.level];
  const uint8_t* role = a.role + (size_t)slot * kNodes;
  float* ly = a.lam_coarse_a + (size_t)slot * kBlockStride;  // adjoint of the new time level
  float* lx = a.lam_fine + (size_t)slot * kBlockStride;      // adjoint of the old time level
  typedef typename S::type T;
  const T* newb = static_cast<const T*>(a.undo_dst) + (size_t)slot * kBlockStride;  // state after the step
  const T* oldb = static_cast<const T*>(a.src_a) + (size_t)slot * kBlockStride;
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    int dst = -1;
    if ((role[node] & ROLE_MASK) == ROLE_OUTFLOW) {
      int kind, sgn, axn;
      dst = outflow_src(a.G, lg, bc, role, node, kind, sgn, axn);
      float v[kMom];
#pragma unroll
      for (int m = 0; m < kMom; ++m) {
        v[m] = ly[m * kNodes + node];
        ly[m * kNodes + node] = 0.0f;
      }
      if (dst < 0) {
#pragma unroll
        for (int m = 0; m < kMom; ++m) lx[m * kNodes + node] += v[m];
      } else if (kind == BC_OUTFLOW) {
#pragma unroll
        for (int m = 0; m < kMom; ++m) sv[m][node] = v[m];
      } else {
        float qh[kMom], qb[kMom];
#pragma unroll
        for (int m = 0; m < kMom; ++m) {
          qh[m] = Codec<S>::load(newb[m * kNodes + dst], a.sc.inv[m]);
          qb[m] = Codec<S>::load(oldb[m * kNodes + node], a.sc.inv[m]);
        }
        const float un = sgn * qh[1 + axn];
        const float lam = un > 0.0f ? un : 0.0f;
        const float w = 1.0f / (1.0f + lam);
        float dl = 0.0f;
#pragma unroll
        for (int m = 0; m < kMom; ++m) {
          lx[m * kNodes + node] += w * v[m];
          sv[m][node] = lam * w * v[m];
          dl += v[m] * (qh[m] - qb[m]);
        }
        if (un > 0.0f) sv[1 + axn][node] += sgn * dl * w * w;
      }
      undo_node<S>(a.undo_dst, a.undo_tape, slot, blockIdx.x, node);
    }
    sdst[node] = (int16_t)dst;
  }
  __syncthreads();
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    if ((role[node] & ROLE_MASK) != ROLE_COMPUTED) continue;
    const int lc[3] = {node & 7, (node >> 3) & 7, node >> 6};
    float acc[kMom];
    bool any = false;
#pragma unroll
    for (int m = 0; m < kMom; ++m) acc[m] = 0.0f;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int ax = f >> 1, sgn = (f & 1) ? 1 : -1;
      const int c = lc[ax] + sgn;
      if (c < 0 || c > 7) continue;
      const int nb = node + sgn * (ax == 0 ? 1 : (ax == 1 ? 8 : 64));
      if (sdst[nb] != node) continue;
      any = true;
#pragma unroll
      for (int m = 0; m < kMom; ++m) acc[m] += sv[m][nb];
    }
    if (any) {
#pragma unroll
      for (int m = 0; m < kMom; ++m) ly[m * kNodes + node] += acc[m];
    }
  }
}

// ---- loss L = 1/2 sum rho |u|^2 over owned nodes in a fine-unit box: dL/dQ ------
// Inflow nodes count in the loss but hold fixed values: their entry stays zero.
template <class S>
__global__ __launch_bounds__(256) void k_loss_ke_grad(AdjTransferLaunch a, float* out, int lx, int ly, int lz, int hx,
                                                      int hy, int hz) {
  const int slot = a.blocks[blockIdx.x];
  const int4 c = a.coord[slot];
  typedef typename S::type T;
  const T* q = static_cast<const T*>(a.src_a) + (size_t)slot * kBlockStride;
  float* lam = out + (size_t)blockIdx.x * kBlockStride;
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    const uint8_t r = a.role[(size_t)slot * kNodes + node] & ROLE_MASK;
    const int64_t fx = (int64_t)(c.x * kEdge + (node & 7)) << a.level;
    const int64_t fy = (int64_t)(c.y * kEdge + ((node >> 3) & 7)) << a.level;
    const int64_t fz = (int64_t)(c.z * kEdge + (node >> 6)) << a.level;
    const bool in = fx >= lx && fx < hx && fy >= ly && fy < hy && fz >= lz && fz < hz;
    const bool st = r == ROLE_COMPUTED || r == ROLE_IU || r == ROLE_OUTFLOW;
    float g[kMom];
#pragma unroll
    for (int m = 0; m < kMom; ++m) g[m] = 0.0f;
    if (in && st) {
      const float rho = 1.0f + Codec<S>::load(q[node], a.sc.inv[0]);
      float u[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) u[k] = Codec<S>::load(q[(1 + k) * kNodes + node], a.sc.inv[1 + k]);
      g[0] = 0.5f * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
#pragma unroll
      for (int k = 0; k < 3; ++k) g[1 + k] = rho * u[k];
    }
#pragma unroll
    for (int m = 0; m < kMom; ++m) lam[m * kNodes + node] = g[m];
  }
}

__global__ __launch_bounds__(256) void k_lam_scatter(const float* in, float* lam, const int32_t* blocks,
                                                     const uint8_t* role) {
  const int32_t slot = blocks[blockIdx.x];
  const float* src = in + (size_t)blockIdx.x * kBlockStride;
  float* dst = lam + (size_t)slot * kBlockStride;
  for (int node = threadIdx.x; node < kNodes; node += 256) {
    const uint8_t r = role[(size_t)slot * kNodes + node] & ROLE_MASK;
    const bool st = r == ROLE_COMPUTED || r == ROLE_IU || r == ROLE_OUTFLOW;
#pragma unroll
    for (int m = 0; m < kMom; ++m) dst[m * kNodes + node] = st ? src[m * kNodes + node] : 0.0f;
  }
}

__global__ void k_zero_blocks(float* buf, const int32_t* blocks, int32_t n) {
  const int32_t slot = blocks[blockIdx.x];
  float* p = buf + (size_t)slot * kBlockStride;
  for (int i = threadIdx.x; i < kBlockStride; i += blockDim.x) p[i] = 0.0f;
}

// block copies between the pool and a packed list (source and target never overlap,
// so the loads of several iterations can be in flight together)
__global__ __launch_bounds__(256) void k_gather_blocks(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                       const int32_t* blocks, int32_t per_block) {
  const uint4* s = src + (size_t)blocks[blockIdx.x] * per_block;
  uint4* d = dst + (size_t)blockIdx.x * per_block;
#pragma unroll 5
  for (int i = threadIdx.x; i < per_block; i += 256) d[i] = s[i];
}
__global__ __launch_bounds__(256) void k_gather_blocks2(const uint4* __restrict__ src_a,
                                                        const uint4* __restrict__ src_b, uint4* __restrict__ dst,
                                                        const int32_t* blocks, int32_t n, int32_t per_block) {
  const int i = blockIdx.x < n ? blockIdx.x : blockIdx.x - n;
  const uint4* s = (blockIdx.x < n ? src_a : src_b) + (size_t)blocks[i] * per_block;
  uint4* d = dst + (size_t)blockIdx.x * per_block;
#pragma unroll 5
  for (int k = threadIdx.x; k < per_block; k += 256) d[k] = s[k];
}
__global__ __launch_bounds__(256) void k_scatter_blocks(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                        const int32_t* blocks, int32_t per_block) {
  const uint4* s = src + (size_t)blockIdx.x * per_block;
  uint4* d = dst + (size_t)blocks[blockIdx.x] * per_block;
#pragma unroll 5
  for (int i = threadIdx.x; i < per_block; i += 256) d[i] = s[i];
}
__global__ void k_write_words(uint64_t* dst, Words8 w) {
  if (threadIdx.x < 8) dst[threadIdx.x] = w.v[threadIdx.x];
}

constexpr int64_t kTransposeWaves = 2048;
template <class S> hipError_t tr_t(const AdjScLaunch& l, hipStream_t s) {
  if (l.nblocks <= 0) return hipSuccess;
  TrArgs<S> a;
  a.x = static_cast<const typename S::type*>(l.x);
  a.mu = l.mu;
  a.lam_x = l.lam_x;
  a.blocks = l.blocks;
  a.nbr = l.nbr;
  a.role = l.role;
  a.nblocks = l.nblocks;
  a.zero_slot = l.zero_slot;
  a.omega = l.omega;
  a.sc = l.sc;
  a.x_next = static_cast<typename S::type*>(l.next_x);
  a.tape_next = static_cast<const typename S::type*>(l.next_tape);
  a.mu_next = l.next_mu;
  // split the blocks' z ranges over 2 or 4 workgroups while the level has too few
  // blocks to give every SIMD of the chip a wave (4 per CU, 256 CUs)
  a.zsplit = 1;
  while (a.zsplit < 4 && (int64_t)l.nblocks * a.zsplit < kTransposeWaves) a.zsplit *= 2;
  if (l.next_mu)
    hipLaunchKernelGGL((k_sc_transpose<S, true>), dim3(l.nblocks * a.zsplit), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((k_sc_transpose<S, false>), dim3(l.nblocks * a.zsplit), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <template <class> class K, int NT>
hipError_t dispatch_adj(const AdjTransferLaunch& a, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  switch (a.storage) {
    case 0: hipLaunchKernelGGL(K<StoreF32>::fn, dim3(a.nblocks), dim3(NT), 0, s, a); break;
    case 1: hipLaunchKernelGGL(K<StoreBF16>::fn, dim3(a.nblocks), dim3(NT), 0, s, a); break;
    case 2: hipLaunchKernelGGL(K<StoreF16>::fn, dim3(a.nblocks), dim3(NT), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <class S> struct DownLinK { static constexpr auto fn = k_down_adj_lin<S>; };
template <class S> struct DownGatherK { static constexpr auto fn = k_down_adj_gather<S>; };
template <class S> struct UpAdjK { static constexpr auto fn = k_up_adj<S>; };
template <class S> struct OutflowAdjK { static constexpr auto fn = k_outflow_adj<S>; };

}  // namespace

hipError_t launch_sc_transpose(const AdjScLaunch& l, hipStream_t s) {
  switch (l.storage) {
    case 0: return tr_t<StoreF32>(l, s);
    case 1: return tr_t<StoreBF16>(l, s);
    case 2: return tr_t<StoreF16>(l, s);
  }
  return hipErrorInvalidValue;
}
// one lane per node where the kernel allows it (more loads in flight on small levels)
hipError_t launch_down_adj_lin(const AdjTransferLaunch& a, hipStream_t s) { return dispatch_adj<DownLinK, kNodes>(a, s); }
hipError_t launch_down_adj_gather(const AdjTransferLaunch& a, hipStream_t s) { return dispatch_adj<DownGatherK, kNodes>(a, s); }
hipError_t launch_up_adj(const AdjTransferLaunch& a, hipStream_t s) { return dispatch_adj<UpAdjK, kNodes>(a, s); }
hipError_t launch_outflow_adj(const AdjTransferLaunch& a, hipStream_t s) { return dispatch_adj<OutflowAdjK, 256>(a, s); }
hipError_t launch_ghost_index(const int32_t* blocks, int32_t n, int32_t* gidx, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ghost_index, dim3((n + 255) / 256), dim3(256), 0, s, blocks, n, gidx);
  return hipGetLastError();
}
hipError_t launch_mark_gather(const AdjTransferLaunch& a, hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_gather, dim3(a.nblocks), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_sc_mu(const AdjScLaunch& l, hipStream_t s) {
  if (l.nblocks <= 0) return hipSuccess;
  switch (l.storage) {
    case 0: hipLaunchKernelGGL(k_sc_mu<StoreF32>, dim3(l.nblocks), dim3(kNodes), 0, s, l); break;
    case 1: hipLaunchKernelGGL(k_sc_mu<StoreBF16>, dim3(l.nblocks), dim3(kNodes), 0, s, l); break;
    case 2: hipLaunchKernelGGL(k_sc_mu<StoreF16>, dim3(l.nblocks), dim3(kNodes), 0, s, l); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_loss_ke_grad(const AdjTransferLaunch& a, float* out, const int32_t lo[3], const int32_t hi[3],
                               hipStream_t s) {
  if (a.nblocks <= 0) return hipSuccess;
  switch (a.storage) {
    case 0: hipLaunchKernelGGL(k_loss_ke_grad<StoreF32>, dim3(a.nblocks), dim3(256), 0, s, a, out, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]); break;
    case 1: hipLaunchKernelGGL(k_loss_ke_grad<StoreBF16>, dim3(a.nblocks), dim3(256), 0, s, a, out, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]); break;
    case 2: hipLaunchKernelGGL(k_loss_ke_grad<StoreF16>, dim3(a.nblocks), dim3(256), 0, s, a, out, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_lam_scatter(const float* in, float* lam, const int32_t* blocks, const uint8_t* role, int32_t n,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lam_scatter, dim3(n), dim3(256), 0, s, in, lam, blocks, role);
  return hipGetLastError();
}
hipError_t launch_zero_blocks(float* buf, const int32_t* blocks, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_blocks, dim3(n), dim3(256), 0, s, buf, blocks, n);
  return hipGetLastError();
}
hipError_t launch_gather_blocks(const void* src, void* dst, const int32_t* blocks, int32_t n, size_t block_bytes,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (block_bytes % 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_blocks, dim3(n), dim3(256), 0, s, static_cast<const uint4*>(src),
                     static_cast<uint4*>(dst), blocks, (int32_t)(block_bytes / 16));
  return hipGetLastError();
}
hipError_t launch_gather_blocks2(const void* src_a, const void* src_b, void* dst, const int32_t* blocks, int32_t n,
                                 size_t block_bytes, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (block_bytes % 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_blocks2, dim3(2 * n), dim3(256), 0, s, static_cast<const uint4*>(src_a),
                     static_cast<const uint4*>(src_b), static_cast<uint4*>(dst), blocks, n,
                     (int32_t)(block_bytes / 16));
  return hipGetLastError();
}
hipError_t launch_scatter_blocks(const void* src, void* dst, const int32_t* blocks, int32_t n, size_t block_bytes,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (block_bytes % 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scatter_blocks, dim3(n), dim3(256), 0, s, static_cast<const uint4*>(src),
                     static_cast<uint4*>(dst), blocks, (int32_t)(block_bytes / 16));
  return hipGetLastError();
}
hipError_t launch_write_words(uint64_t* dst, Words8 w, hipStream_t s) {
  hipLaunchKernelGGL(k_write_words, dim3(1), dim3(64), 0, s, dst, w);
  return hipGetLastError();
}

}  // namespace lbmx
