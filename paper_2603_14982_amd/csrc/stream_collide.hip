// Stream-collide of one level (Sec. 3.1 "Collision and Streaming", Eq. three_order_f).
//
// For every computed node x the step pulls the 27 populations reconstructed
// (third-order Hermite, Eq. three_order_f) from the collided moments of the
// neighbours x - c_i and takes their moments (Eq. rho_u_stress). Moments are
// stored before collision; collision (S <- S + omega (u u - S)) is applied when
// a node is read.
//
// Design for gfx950: the population field is never formed. Per source node the
// reconstruction is written in a per-axis tensor basis (p0 = 1, p1 = c and a
// quadratic p2; 17 nonzero coefficients); the stream + moment projection factorises
// into three 1D passes (x, y, z), each: moment->population along the axis, shift
// by one node, population->moment. The sweep runs plane by plane in z: the x and
// y passes exchange through LDS on a halo plane, the z pass runs in registers over
// a sliding window of three planes, and every lane owns one (x, y) column.
// Two kernels: k_stream_collide, one 64-lane wave per 8^3 block on a 10 x 10 halo
// plane; k_stream_collide_tile, four waves per tile of 2 x 2 x 2 blocks on an
// 18 x 18 plane (fewer halo reads and idle lanes; used on levels large enough to
// fill the chip with tiles). Bounce-back at solid neighbours is a per-node
// correction on the few flagged nodes.
//
// Only the deviation rho - 1 enters the coefficients: the rest state maps to
// itself exactly, so rho - 1 is produced without cancellation against 1.
//
// Exact arithmetic of the weights: the per-axis basis is p0 = 1, p1 = c,
// p2' = 3c^2 - 1, and every 1D pass works on six times the populations, so the
// lattice weights become the integers (1, 4, 1) and all basis constants are small
// integers. Only additions round (to nearest, unbiased); the factor 6^3 = 216 is
// removed per output without multiplying by a rounded constant reciprocal (an
// FMA-corrected quotient for rho - 1, a reciprocal with one Newton step for the
// others). Inexact weights such as fl(1/6) would bias every step the same way and
// the error would grow linearly.
#include "common.h"
#include "kernels.h"

namespace lbmx {
namespace {

template <class S> struct ScArgs {
  const float* cpl;  // coupling fields of the finest level, [slot][4][512] (eps, F), or null
  const typename S::type* in;
  typename S::type* out;
  const int32_t* blocks;
  const int32_t* nbr;
  const uint8_t* role;
  int32_t nblocks;
  int32_t zero_slot;
  float omega;
  Scales sc;
  const int32_t* tiles;
  int32_t ntiles;
  const int32_t* dir;
  const int4* coord;
  LevelGeom lg;
  int periodic[3];
  // two-substep sweep: workgroups [run_off[c], run_off[c + 1]) take the runs of
  // kRunMax - c tiles (list runs + (kRunMax - c - 1) * run_stride, run_n[c] of them; the
  // range is padded to a multiple of 8 workgroups)
  const int32_t* runs;
  int64_t run_stride;
  int32_t run_off[kRunMax + 1];
  int32_t run_n[kRunMax];
};

// x-direction populations (times 6) of the 8 (my, mz) coefficient groups of a
// source node, three per group (P(+1), P(0), P(-1)):
//   P(+-1) = a0 +- a1 + 2 a2,  P(0) = 4 (a0 - a2)
// for the group's coefficients (a0, a1, a2) of p0, p1, p2' along x.
// With coupling fields c4 = (eps, F) (CPL) the node relaxes at omega / eps (tau
// scaled by the fluid fraction) and the force enters in Guo's moment form: S gains
// (1 - om/2)(u F + F u)/rho, and the carried velocity is u + F/(2 rho).
//
// Every product that meets an addition is fused or not as written here (contraction
// by the compiler is off in this function): the kernels that reconstruct a node in
// different code (one substep per sweep, two substeps per sweep) round it the same
// way, so they agree bit for bit.
template <bool CPL>
__device__ __forceinline__ void source_pops(const float q[kMom], float omega, const float c4[4], float p[24]) {
#pragma clang fp contract(off)
  const float drho = q[0];
  const float rho = 1.0f + drho;
  float ux = q[1], uy = q[2], uz = q[3];
  const float om = CPL ? omega / c4[0] : omega;
  // collision: S relaxes to u u
  float sxx = __builtin_fmaf(om, __builtin_fmaf(ux, ux, -q[4]), q[4]);
  float syy = __builtin_fmaf(om, __builtin_fmaf(uy, uy, -q[5]), q[5]);
  float szz = __builtin_fmaf(om, __builtin_fmaf(uz, uz, -q[6]), q[6]);
  float sxy = __builtin_fmaf(om, __builtin_fmaf(ux, uy, -q[7]), q[7]);
  float sxz = __builtin_fmaf(om, __builtin_fmaf(ux, uz, -q[8]), q[8]);
  float syz = __builtin_fmaf(om, __builtin_fmaf(uy, uz, -q[9]), q[9]);
  if (CPL) {
    const float g = (1.0f - 0.5f * om) / rho;
    const float fx = c4[1], fy = c4[2], fz = c4[3];
    sxx = __builtin_fmaf(g, 2.0f * (ux * fx), sxx);
    syy = __builtin_fmaf(g, 2.0f * (uy * fy), syy);
    szz = __builtin_fmaf(g, 2.0f * (uz * fz), szz);
    sxy = __builtin_fmaf(g, __builtin_fmaf(ux, fy, fx * uy), sxy);
    sxz = __builtin_fmaf(g, __builtin_fmaf(ux, fz, fx * uz), sxz);
    syz = __builtin_fmaf(g, __builtin_fmaf(uy, fz, fy * uz), syz);
    const float h = 0.5f / rho;
    ux = __builtin_fmaf(h, fx, ux);
    uy = __builtin_fmaf(h, fy, uy);
    uz = __builtin_fmaf(h, fz, uz);
  }
  // third-order terms Gamma_aab = S_aa u_b + 2 S_ab u_a - 2 u_a^2 u_b
  //                             = u_b (S_aa - 2 u_a^2) + 2 S_ab u_a
  const float tx = __builtin_fmaf(-2.0f * ux, ux, sxx);
  const float ty = __builtin_fmaf(-2.0f * uy, uy, syy);
  const float tz = __builtin_fmaf(-2.0f * uz, uz, szz);
  const float s2xy = 2.0f * sxy, s2xz = 2.0f * sxz, s2yz = 2.0f * syz;
  const float gxxy = __builtin_fmaf(uy, tx, s2xy * ux);
  const float gyyx = __builtin_fmaf(ux, ty, s2xy * uy);
  const float gxxz = __builtin_fmaf(uz, tx, s2xz * ux);
  const float gzzx = __builtin_fmaf(ux, tz, s2xz * uz);
  const float gyyz = __builtin_fmaf(uz, ty, s2yz * uy);
  const float gzzy = __builtin_fmaf(uy, tz, s2yz * uz);
  const float gxyz = __builtin_fmaf(sxy, uz, __builtin_fmaf(sxz, uy, __builtin_fmaf(syz, ux, (-2.0f * (ux * uy)) * uz)));
  // tensor-basis coefficients (Eq. three_order_f in the p0/p1/p2' basis); per
  // (my, mz) group with coefficients (a0, a1, a2) along x:
  //   P(+-1) = (a0 + 2 a2) +- a1,  P(0) = 4 (a0 - a2)
  // a1 enters fused; a0 and a2 are rounded once (each is used twice)
  const float r3 = 3.0f * rho, r15 = 1.5f * rho, r9 = 9.0f * rho, r45 = 4.5f * rho, r27 = 27.0f * rho;
  const float a010 = r3 * uy, a001 = r3 * uz;
  const float a200 = r15 * sxx, a020 = r15 * syy, a002 = r15 * szz;
  const float a011 = r9 * syz;
  const float a210 = r45 * gxxy, a201 = r45 * gxxz;
  const float a021 = r45 * gyyz, a012 = r45 * gzzy;
  float e;
  // (my,mz) = (0,0): (a000, a100, a200)
  e = __builtin_fmaf(2.0f, a200, drho);
  p[0] = __builtin_fmaf(r3, ux, e);  p[1] = 4.0f * (drho - a200);  p[2] = __builtin_fmaf(-r3, ux, e);
  // (1,0): (a010, a110, a210)
  e = __builtin_fmaf(2.0f, a210, a010);
  p[3] = __builtin_fmaf(r9, sxy, e);  p[4] = 4.0f * (a010 - a210);  p[5] = __builtin_fmaf(-r9, sxy, e);
  // (0,1): (a001, a101, a201)
  e = __builtin_fmaf(2.0f, a201, a001);
  p[6] = __builtin_fmaf(r9, sxz, e);  p[7] = 4.0f * (a001 - a201);  p[8] = __builtin_fmaf(-r9, sxz, e);
  // (2,0): (a020, a120, 0)
  p[9] = __builtin_fmaf(r45, gyyx, a020);  p[10] = 4.0f * a020;  p[11] = __builtin_fmaf(-r45, gyyx, a020);
  // (0,2): (a002, a102, 0)
  p[12] = __builtin_fmaf(r45, gzzx, a002);  p[13] = 4.0f * a002;  p[14] = __builtin_fmaf(-r45, gzzx, a002);
  // (1,1): (a011, a111, 0)
  p[15] = __builtin_fmaf(r27, gxyz, a011);  p[16] = 4.0f * a011;  p[17] = __builtin_fmaf(-r27, gxyz, a011);
  // (2,1): (a021, 0, 0)
  p[18] = a021;  p[19] = 4.0f * a021;  p[20] = a021;
  // (1,2): (a012, 0, 0)
  p[21] = a012;  p[22] = 4.0f * a012;  p[23] = a012;
}
__device__ __forceinline__ void source_pops(const float q[kMom], float omega, float p[24]) {
  source_pops<false>(q, omega, nullptr, p);
}

// The 17 tensor-basis coefficients of a node (bounce-back path only), p2' basis.
template <bool CPL>
__device__ void node_coeffs(const float q[kMom], float omega, const float c4[4], float a[17]) {
  const float drho = q[0];
  const float rho = 1.0f + drho;
  float ux = q[1], uy = q[2], uz = q[3];
  const float om = CPL ? omega / c4[0] : omega;
  float sxx = q[4] + om * (ux * ux - q[4]);
  float syy = q[5] + om * (uy * uy - q[5]);
  float szz = q[6] + om * (uz * uz - q[6]);
  float sxy = q[7] + om * (ux * uy - q[7]);
  float sxz = q[8] + om * (ux * uz - q[8]);
  float syz = q[9] + om * (uy * uz - q[9]);
  if (CPL) {
    const float g = (1.0f - 0.5f * om) / rho;
    const float fx = c4[1], fy = c4[2], fz = c4[3];
    sxx += g * (ux * fx + fx * ux);
    syy += g * (uy * fy + fy * uy);
    szz += g * (uz * fz + fz * uz);
    sxy += g * (ux * fy + fx * uy);
    sxz += g * (ux * fz + fx * uz);
    syz += g * (uy * fz + fy * uz);
    const float h = 0.5f / rho;
    ux += h * fx;
    uy += h * fy;
    uz += h * fz;
  }
  a[0] = drho;                      // 000
  a[1] = 3.0f * (rho * ux);         // 100
  a[2] = 3.0f * (rho * uy);         // 010
  a[3] = 3.0f * (rho * uz);         // 001
  a[4] = 1.5f * (rho * sxx);        // 200
  a[5] = 1.5f * (rho * syy);        // 020
  a[6] = 1.5f * (rho * szz);        // 002
  a[7] = 9.0f * (rho * sxy);        // 110
  a[8] = 9.0f * (rho * sxz);        // 101
  a[9] = 9.0f * (rho * syz);        // 011
  a[10] = 4.5f * (rho * (sxx * uy + 2.0f * sxy * ux - 2.0f * ux * ux * uy));  // 210
  a[11] = 4.5f * (rho * (syy * ux + 2.0f * sxy * uy - 2.0f * uy * uy * ux));  // 120
  a[12] = 4.5f * (rho * (sxx * uz + 2.0f * sxz * ux - 2.0f * ux * ux * uz));  // 201
  a[13] = 4.5f * (rho * (szz * ux + 2.0f * sxz * uz - 2.0f * uz * uz * ux));  // 102
  a[14] = 4.5f * (rho * (syy * uz + 2.0f * syz * uy - 2.0f * uy * uy * uz));  // 021
  a[15] = 4.5f * (rho * (szz * uy + 2.0f * syz * uz - 2.0f * uz * uz * uy));  // 012
  a[16] = 27.0f * (rho * (sxy * uz + sxz * uy + syz * ux - 2.0f * ux * uy * uz));  // 111
}

// 1D population->moment map after the shift (times 6 populations):
// (P+, P0, P-) -> (m0, m1, m2') = (P+ + P0 + P-, P+ - P-, 2 (P+ + P-) - P0)
__device__ __forceinline__ void back3(float pp, float p0, float pm, float& m0, float& m1, float& m2) {
  const float s = pp + pm;
  m0 = s + p0;
  m1 = pp - pm;
  m2 = 2.0f * s - p0;
}
// 1D moment->population map (times 6): (a0, a1, a2') -> (P+, P0, P-)
__device__ __forceinline__ void fwd3(float a0, float a1, float a2, float& pp, float& p0, float& pm) {
  const float e = a0 + 2.0f * a2;
  pp = e + a1;
  pm = e - a1;
  p0 = 4.0f * (a0 - a2);
}

// halo-plane point (px, py) in [-1, 8]^2 of round r for a lane
__device__ __forceinline__ bool plane_point(int lane, int r, int& px, int& py) {
  if (r == 0) { px = lane & 7; py = lane >> 3; return true; }
  if (lane < 10) { px = lane - 1; py = -1; return true; }
  if (lane < 20) { px = lane - 11; py = 8; return true; }
  if (lane < 28) { px = -1; py = lane - 20; return true; }
  if (lane < 36) { px = 8; py = lane - 28; return true; }
  return false;
}

// Missing neighbours (no block, wall) read the pool's all-zero slot: zero
// moments give zero coefficients, the same as a solid node.
template <class S>
__device__ __forceinline__ void fetch_point(const ScArgs<S>& a, const int* s_src, int px, int py, int pz,
                                            typename S::type raw[kMom]) {
  const int ox = px < 0 ? -1 : (px > 7 ? 1 : 0);
  const int oy = py < 0 ? -1 : (py > 7 ? 1 : 0);
  const int oz = pz < 0 ? -1 : (pz > 7 ? 1 : 0);
  const int ns = s_src[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)];
  const int node = (px & 7) + 8 * (py & 7) + 64 * (pz & 7);
  const typename S::type* src = a.in + (size_t)ns * kBlockStride + node;
#pragma unroll
  for (int m = 0; m < kMom; ++m) raw[m] = src[m * kNodes];
}

// coupling fields (eps, F) of a plane point of the single-block kernel / of a node
__device__ __forceinline__ void load_cpl(const float* cpl, int slot, int node, float c4[4]) {
  const float* src = cpl + (size_t)slot * 4 * kNodes + node;
#pragma unroll
  for (int m = 0; m < 4; ++m) c4[m] = src[m * kNodes];
}
__device__ __forceinline__ void fetch_cpl_point(const float* cpl, const int* s_src, int px, int py, int pz,
                                                float c4[4]) {
  const int ox = px < 0 ? -1 : (px > 7 ? 1 : 0);
  const int oy = py < 0 ? -1 : (py > 7 ? 1 : 0);
  const int oz = pz < 0 ? -1 : (pz > 7 ? 1 : 0);
  load_cpl(cpl, s_src[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)], (px & 7) + 8 * (py & 7) + 64 * (pz & 7), c4);
}

// bounce-back correction of one computed node: every direction c_i whose source
// x - c_i is solid (or behind a wall) receives f_{-c_i}(x) instead.
template <class S, bool CPL>
__device__ void bounce_back(const ScArgs<S>& a, int slot, int lx, int ly, int lz, const float c4[4], float M[10]) {
  const int32_t* nbr = a.nbr + (size_t)slot * 27;
  float q[kMom];
  const int node = lx + 8 * ly + 64 * lz;
  const typename S::type* src = a.in + (size_t)slot * kBlockStride + node;
  for (int m = 0; m < kMom; ++m) q[m] = Codec<S>::load(src[m * kNodes], a.sc.inv[m]);
  float c[17];
  node_coeffs<CPL>(q, a.omega, c4, c);
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
    // outgoing direction d = -c: basis values p1(d) = d, p2'(d) = 3 d^2 - 1
    const float dx = -cx, dy = -cy, dz = -cz;
    const float ex = 3.0f * dx * dx - 1.0f, ey = 3.0f * dy * dy - 1.0f, ez = 3.0f * dz * dz - 1.0f;
    const float sum = c[0] + c[1] * dx + c[2] * dy + c[3] * dz + c[4] * ex + c[5] * ey + c[6] * ez
                      + c[7] * dx * dy + c[8] * dx * dz + c[9] * dy * dz + c[10] * ex * dy + c[11] * dx * ey
                      + c[12] * ex * dz + c[13] * dx * ez + c[14] * ey * dz + c[15] * dy * ez
                      + c[16] * dx * dy * dz;
    // 216 w_c = product of the integer per-axis weights (4 at rest, 1 moving)
    const float w = (cx ? 1.0f : 4.0f) * (cy ? 1.0f : 4.0f) * (cz ? 1.0f : 4.0f);
    const float f = w * sum;
    const float fx = f * cx, fy = f * cy, fz = f * cz;
    M[0] += f;
    M[1] += fx; M[2] += fy; M[3] += fz;
    M[4] += f * (3.0f * cx * cx - 1.0f); M[5] += f * (3.0f * cy * cy - 1.0f); M[6] += f * (3.0f * cz * cz - 1.0f);
    M[7] += fx * cy; M[8] += fx * cz; M[9] += fy * cz;
  }
}

// workgroup -> block with consecutive blocks on the same XCD (workgroups are
// dealt to the 8 XCDs round-robin; neighbours in key order then share an L2)
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int per = n >> 3, rem = n & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

// LDS plane buffer, row-major so that the x pass of a row only overwrites its
// own row: row r (plane row y = r - 1) holds
//   x-pass input:  [kind (P+, P0, P-)][half][col 0..9][4]                (240 floats)
//   y-pass input:  [kind (P+, P0, P-)][col 0..7][triple 0..8, pad 10]   (240 floats)
// The 8 group values of a point are split in two 4-float halves, so that the
// 128-bit accesses of neighbouring lanes are 16 bytes apart (no bank conflicts);
// the y-pass input moves with 64-bit accesses. Rows are 16 banks apart.
constexpr int kRow = 240;
constexpr int kHalf = 40;
__device__ __forceinline__ int a_off(int row, int kind, int col) { return row * kRow + kind * 80 + col * 4; }
__device__ __forceinline__ int b_off(int row, int kind, int col) { return row * kRow + kind * 80 + col * 10; }

__device__ __forceinline__ void st8(float* lds, int row, int kind, int col, const float v[8]) {
  const int off = a_off(row, kind, col);
  *reinterpret_cast<float4*>(lds + off) = make_float4(v[0], v[1], v[2], v[3]);
  *reinterpret_cast<float4*>(lds + off + kHalf) = make_float4(v[4], v[5], v[6], v[7]);
}
__device__ __forceinline__ void ld8(const float* lds, int row, int kind, int col, float v[8]) {
  const int off = a_off(row, kind, col);
  const float4 a = *reinterpret_cast<const float4*>(lds + off);
  const float4 b = *reinterpret_cast<const float4*>(lds + off + kHalf);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
__device__ __forceinline__ void st9(float* lds, int off, const float v[9]) {
  float2* p = reinterpret_cast<float2*>(lds + off);
  p[0] = make_float2(v[0], v[1]);
  p[1] = make_float2(v[2], v[3]);
  p[2] = make_float2(v[4], v[5]);
  p[3] = make_float2(v[6], v[7]);
  lds[off + 8] = v[8];
}
__device__ __forceinline__ void ld9(const float* lds, int off, float v[9]) {
  const float2* p = reinterpret_cast<const float2*>(lds + off);
  const float2 a = p[0], b = p[1], c = p[2], d = p[3];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x; v[5] = c.y; v[6] = d.x; v[7] = d.y;
  v[8] = lds[off + 8];
}

// reciprocal to within about half an ulp: hardware estimate plus one Newton step
__device__ __forceinline__ float recip(float r) {
  float y = __builtin_amdgcn_rcpf(r);
  const float e = __builtin_fmaf(-r, y, 1.0f);
  return __builtin_fmaf(y, e, y);
}

// x pass for one row of the owned 8 columns: back-map the 8 groups after the
// shift, then forward-map along y for the 9 (qx, mz) triples
__device__ __forceinline__ void x_pass(const float* lds, int row, int x, float yb[27]) {
  float pp[8], pz[8], pm[8];
  ld8(lds, row, 0, x, pp);       // P+ of column x-1
  ld8(lds, row, 1, x + 1, pz);   // P0 of column x
  ld8(lds, row, 2, x + 2, pm);   // P- of column x+1
  float B[3][3][3];  // [qx][my][mz]
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    float m0, m1, m2;
    back3(pp[g], pz[g], pm[g], m0, m1, m2);
    const int my = (g == 1 || g == 5 || g == 7) ? 1 : ((g == 3 || g == 6) ? 2 : 0);
    const int mz = (g == 2 || g == 5 || g == 6) ? 1 : ((g == 4 || g == 7) ? 2 : 0);
    B[0][my][mz] = m0; B[1][my][mz] = m1; B[2][my][mz] = m2;
  }
#pragma unroll
  for (int qx = 0; qx < 3; ++qx)
#pragma unroll
    for (int mz = 0; mz < 3; ++mz) {
      const float b2 = (mz == 2) ? 0.0f : B[qx][2][mz];  // no (my, mz) = (2, 2) coefficient
      const int t = 3 * qx + mz;
      fwd3(B[qx][0][mz], B[qx][1][mz], b2, yb[t], yb[9 + t], yb[18 + t]);
    }
}

template <class S, bool CPL>
__global__ __launch_bounds__(64) void k_stream_collide(ScArgs<S> a) {
  __shared__ __align__(16) float lds[10 * kRow];
  __shared__ int s_src[27];
  const int lane = threadIdx.x;
  const int slot = a.blocks[xcd_remap(blockIdx.x, a.nblocks)];
  if (lane < 27) {
    const int ns = a.nbr[(size_t)slot * 27 + lane];
    s_src[lane] = ns >= 0 ? ns : a.zero_slot;
  }
  __syncthreads();

  int px[2], py[2];
  bool has[2];
  has[0] = plane_point(lane, 0, px[0], py[0]);
  has[1] = plane_point(lane, 1, px[1], py[1]);
  const int ox = lane & 7, oy = lane >> 3;   // owned column
  const float c216 = 1.0f / 216.0f;

  // roles of the owned column, loaded before the sweep so that no wait inside
  // the plane loop has to drain the prefetch of the next plane
  uint64_t col_roles = 0;
  {
    const uint8_t* rp = a.role + (size_t)slot * kNodes + ox + 8 * oy;
#pragma unroll
    for (int zz = 0; zz < 8; ++zz) col_roles |= (uint64_t)rp[64 * zz] << (8 * zz);
  }

  typedef typename S::type T;
  T nxt[2][kMom];
  float ncp[2][4];  // coupling fields of the prefetched points
#pragma unroll
  for (int r = 0; r < 2; ++r)
    if (has[r]) {
      fetch_point<S>(a, s_src, px[r], py[r], -1, nxt[r]);
      if (CPL) fetch_cpl_point(a.cpl, s_src, px[r], py[r], -1, ncp[r]);
    }

  float zp1[6], zp2[6], z0[6];  // z-window: pop+ of planes z-1, z-2; pop0 of plane z-1
#pragma unroll
  for (int k = 0; k < 6; ++k) zp1[k] = zp2[k] = z0[k] = 0.0f;

  for (int z = -1; z <= 8; ++z) {
    // ---- pass 0: moments of plane z (+ halo) -> x-populations, into LDS
    T cur[2][kMom];
    float ccp[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int m = 0; m < kMom; ++m) cur[r][m] = nxt[r][m];
#pragma unroll
      for (int m = 0; m < 4; ++m) ccp[r][m] = CPL ? ncp[r][m] : 0.0f;
    }
    if (z < 8) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (has[r]) {
          fetch_point<S>(a, s_src, px[r], py[r], z + 1, nxt[r]);
          if (CPL) fetch_cpl_point(a.cpl, s_src, px[r], py[r], z + 1, ncp[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (!has[r]) continue;
      float q[kMom];
#pragma unroll
      for (int m = 0; m < kMom; ++m) q[m] = Codec<S>::load(cur[r][m], a.sc.inv[m]);
      float p[24];
      source_pops<CPL>(q, a.omega, ccp[r], p);
      float v[8];
      const int row = py[r] + 1, col = px[r] + 1;
#pragma unroll
      for (int kind = 0; kind < 3; ++kind) {
#pragma unroll
        for (int g = 0; g < 8; ++g) v[g] = p[3 * g + kind];
        st8(lds, row, kind, col, v);
      }
    }
    __syncthreads();

    // ---- pass x on rows 0..7 (plane rows -1..6), then rows 8..9 (plane rows 7..8);
    // each row is overwritten by its own y-pass input once all its reads are done
    {
      float yb[27];
      x_pass(lds, oy, ox, yb);
      __syncthreads();
      st9(lds, b_off(oy, 0, ox), yb);
      st9(lds, b_off(oy, 1, ox), yb + 9);
      st9(lds, b_off(oy, 2, ox), yb + 18);
    }
    {
      float yb[27];
      const int row = 8 + (oy & 1);  // lanes 16..63 repeat rows 8..9 and do not store
      x_pass(lds, row, ox, yb);
      __syncthreads();
      if (lane < 16) {
        st9(lds, b_off(row, 0, ox), yb);
        st9(lds, b_off(row, 1, ox), yb + 9);
        st9(lds, b_off(row, 2, ox), yb + 18);
      }
    }
    __syncthreads();

    // ---- pass y: shift + back along y for the owned column, then z-forward
    float zpp[6], zpz[6], zpm[6];
    {
      float bp[9], bz[9], bm[9];
      ld9(lds, b_off(oy, 0, ox), bp);       // P+ of row y-1
      ld9(lds, b_off(oy + 1, 1, ox), bz);   // P0 of row y
      ld9(lds, b_off(oy + 2, 2, ox), bm);   // P- of row y+1
      float C[3][3][3];                     // [qx][qy][mz]
#pragma unroll
      for (int qx = 0; qx < 3; ++qx)
#pragma unroll
        for (int mz = 0; mz < 3; ++mz) {
          const int t = 3 * qx + mz;
          float m0, m1, m2;
          back3(bp[t], bz[t], bm[t], m0, m1, m2);
          C[qx][0][mz] = m0; C[qx][1][mz] = m1; C[qx][2][mz] = m2;
        }
      // (qx, qy) pairs needed by the ten output moments:
      // (0,0) (1,0) (0,1) (2,0) (0,2) (1,1)
      fwd3(C[0][0][0], C[0][0][1], C[0][0][2], zpp[0], zpz[0], zpm[0]);
      fwd3(C[1][0][0], C[1][0][1], C[1][0][2], zpp[1], zpz[1], zpm[1]);
      fwd3(C[0][1][0], C[0][1][1], C[0][1][2], zpp[2], zpz[2], zpm[2]);
      fwd3(C[2][0][0], C[2][0][1], C[2][0][2], zpp[3], zpz[3], zpm[3]);
      fwd3(C[0][2][0], C[0][2][1], C[0][2][2], zpp[4], zpz[4], zpm[4]);
      fwd3(C[1][1][0], C[1][1][1], C[1][1][2], zpp[5], zpz[5], zpm[5]);
    }
    __syncthreads();

    // ---- pass z: output plane zo = z - 1 from planes z-2 (pop+), z-1 (pop0), z (pop-)
    const int zo = z - 1;
    if (zo >= 0) {
      float M[10];
      float m0, m1, m2;
      back3(zp2[0], z0[0], zpm[0], m0, m1, m2);  // (0,0): M000, M001, M002
      M[0] = m0; M[3] = m1; M[6] = m2;
      back3(zp2[1], z0[1], zpm[1], m0, m1, m2);  // (1,0): M100, M101
      M[1] = m0; M[8] = m1;
      back3(zp2[2], z0[2], zpm[2], m0, m1, m2);  // (0,1): M010, M011
      M[2] = m0; M[9] = m1;
      back3(zp2[3], z0[3], zpm[3], m0, m1, m2);  // (2,0): M200
      M[4] = m0;
      back3(zp2[4], z0[4], zpm[4], m0, m1, m2);  // (0,2): M020
      M[5] = m0;
      back3(zp2[5], z0[5], zpm[5], m0, m1, m2);  // (1,1): M110
      M[7] = m0;
      const int node = ox + 8 * oy + 64 * zo;
      const uint8_t role = (uint8_t)(col_roles >> (8 * zo));
      typename S::type* dst = a.out + (size_t)slot * kBlockStride + node;
      if ((role & ROLE_MASK) == ROLE_COMPUTED) {
        float c4[4] = {1.0f, 0.0f, 0.0f, 0.0f};
        if (CPL) load_cpl(a.cpl, slot, node, c4);
        if (role & ROLE_BB) bounce_back<S, CPL>(a, slot, ox, oy, zo, c4, M);
        // half the node's force in its velocity (Eq. rho_u_stress); 108 = 216 / 2
        if (CPL) {
          M[1] += 108.0f * c4[1];
          M[2] += 108.0f * c4[2];
          M[3] += 108.0f * c4[3];
        }
        // remove the 6^3 scale of the three passes; no constant reciprocal of
        // 216 or 3 multiplies a result (it would bias every step the same way)
        const float q0 = M[0] * c216;
        const float drho = __builtin_fmaf(__builtin_fmaf(-q0, 216.0f, M[0]), c216, q0);  // M0 / 216
        const float r216 = 216.0f + M[0];          // 216 rho'
        const float inv = recip(r216);
        const float inv3 = recip(3.0f * r216);     // p2' = 3 p2 on the diagonal stresses
        float v[kMom];
        v[0] = drho;
        v[1] = M[1] * inv; v[2] = M[2] * inv; v[3] = M[3] * inv;
        v[4] = M[4] * inv3; v[5] = M[5] * inv3; v[6] = M[6] * inv3;
        v[7] = M[7] * inv; v[8] = M[8] * inv; v[9] = M[9] * inv;
#pragma unroll
        for (int m = 0; m < kMom; ++m) dst[m * kNodes] = Codec<S>::store(v[m], a.sc.s[m]);
      } else if ((role & ROLE_MASK) == ROLE_SOLID) {
#pragma unroll
        for (int m = 0; m < kMom; ++m) dst[m * kNodes] = Codec<S>::store(0.0f, a.sc.s[m]);
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      zp2[k] = zp1[k];
      zp1[k] = zpp[k];
      z0[k] = zpz[k];
    }
  }
}

// y pass of one column of a plane buffer whose y-pass input is [kind][col][10]
// (kinds KINDB apart, rows ROW apart): rows r0, r0 + 1, r0 + 2 hold the rows y - 1,
// y, y + 1 of the column's row y. Back-map after the shift along y, then forward-map
// along z the six (qx, qy) groups the ten output moments need:
// (0,0) (1,0) (0,1) (2,0) (0,2) (1,1).
template <int ROW, int KINDB>
__device__ __forceinline__ void y_pass_col(const float* lds, int r0, int col, float zpp[6], float zpz[6],
                                           float zpm[6]) {
  float bp[9], bz[9], bm[9];
  ld9(lds, r0 * ROW + 0 * KINDB + col * 10, bp);        // P+ of row y-1
  ld9(lds, (r0 + 1) * ROW + 1 * KINDB + col * 10, bz);  // P0 of row y
  ld9(lds, (r0 + 2) * ROW + 2 * KINDB + col * 10, bm);  // P- of row y+1
  float C[3][3][3];  // [qx][qy][mz]
#pragma unroll
  for (int qx = 0; qx < 3; ++qx)
#pragma unroll
    for (int mz = 0; mz < 3; ++mz) {
      const int t = 3 * qx + mz;
      float m0, m1, m2;
      back3(bp[t], bz[t], bm[t], m0, m1, m2);
      C[qx][0][mz] = m0; C[qx][1][mz] = m1; C[qx][2][mz] = m2;
    }
  fwd3(C[0][0][0], C[0][0][1], C[0][0][2], zpp[0], zpz[0], zpm[0]);
  fwd3(C[1][0][0], C[1][0][1], C[1][0][2], zpp[1], zpz[1], zpm[1]);
  fwd3(C[0][1][0], C[0][1][1], C[0][1][2], zpp[2], zpz[2], zpm[2]);
  fwd3(C[2][0][0], C[2][0][1], C[2][0][2], zpp[3], zpz[3], zpm[3]);
  fwd3(C[0][2][0], C[0][2][1], C[0][2][2], zpp[4], zpz[4], zpm[4]);
  fwd3(C[1][1][0], C[1][1][1], C[1][1][2], zpp[5], zpz[5], zpm[5]);
}

// z pass of one node: its ten moment sums (times 216) from pop+ of the plane below,
// pop0 of its own plane and pop- of the plane above
__device__ __forceinline__ void z_back(const float zp[6], const float z0[6], const float zm[6], float M[10]) {
  float m0, m1, m2;
  back3(zp[0], z0[0], zm[0], m0, m1, m2);  // (0,0): M000, M001, M002
  M[0] = m0; M[3] = m1; M[6] = m2;
  back3(zp[1], z0[1], zm[1], m0, m1, m2);  // (1,0): M100, M101
  M[1] = m0; M[8] = m1;
  back3(zp[2], z0[2], zm[2], m0, m1, m2);  // (0,1): M010, M011
  M[2] = m0; M[9] = m1;
  back3(zp[3], z0[3], zm[3], m0, m1, m2);  // (2,0): M200
  M[4] = m0;
  back3(zp[4], z0[4], zm[4], m0, m1, m2);  // (0,2): M020
  M[5] = m0;
  back3(zp[5], z0[5], zm[5], m0, m1, m2);  // (1,1): M110
  M[7] = m0;
}

// stored moments from the moment sums: remove the 6^3 scale of the three passes; no
// constant reciprocal of 216 or 3 multiplies a result (it would bias every step the
// same way)
__device__ __forceinline__ void finish_moments(const float M[10], float v[kMom]) {
  const float c216 = 1.0f / 216.0f;
  const float q0 = M[0] * c216;
  v[0] = __builtin_fmaf(__builtin_fmaf(-q0, 216.0f, M[0]), c216, q0);  // M0 / 216
  const float r216 = 216.0f + M[0];          // 216 rho'
  const float inv = recip(r216);
  const float inv3 = recip(3.0f * r216);     // p2' = 3 p2 on the diagonal stresses
  v[1] = M[1] * inv; v[2] = M[2] * inv; v[3] = M[3] * inv;
  v[4] = M[4] * inv3; v[5] = M[5] * inv3; v[6] = M[6] * inv3;
  v[7] = M[7] * inv; v[8] = M[8] * inv; v[9] = M[9] * inv;
}

// ---- 2 x 2 x 2 block tiles ------------------------------------------------------
// One workgroup of four waves sweeps a tile of 2 x 2 x 2 blocks (16 x 16 columns,
// 16 planes) in z. The halo plane is 18 x 18 points instead of four separate 10 x 10
// planes and the sweep crosses the two blocks in z without re-reading halo planes:
// the faces shared inside the tile are read once, the points are spread over all
// 256 lanes (source and x passes), and each wave keeps one column of blocks for the
// y and z passes and the stores. Missing blocks of a tile read as the all-zero slot
// and are not written.
// Tile geometry for TX blocks along x (2 or 4) by 2 along y and z.
template <int TX> struct Tile {
  static constexpr int NX = 8 * TX;              // tile columns along x
  static constexpr int CX = NX + 2;              // halo plane points along x
  static constexpr int CY = 18;                  // halo plane points along y
  static constexpr int PTS = CX * CY;
  static constexpr int WAVES = 2 * TX;           // one per block column
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int NXB = TX + 2;             // neighbourhood blocks along x
  // LDS row (plane row y = row - 1): x-pass input [kind][half][col 0..CX-1][4] (the 8
  // group values of a point split in two halves, so that neighbouring lanes' 128-bit
  // accesses are 16 bytes apart), later overwritten by the y-pass input
  // [kind][col 0..NX-1][10]. The row stride is 16 banks off a multiple of 32 so that
  // the two rows read by one 16-lane group of the y pass fall on different banks.
  static constexpr int ROW = 3 * NX * 10 + 16;
  static constexpr int HALF = CX * 4;
  static constexpr int KINDA = 2 * HALF;
  static constexpr int KINDB = NX * 10;
  static_assert(3 * KINDA <= ROW, "x-pass input must fit in a row");
};

template <int HALF>
__device__ __forceinline__ void st8_h(float* lds, int off, const float v[8]) {
  *reinterpret_cast<float4*>(lds + off) = make_float4(v[0], v[1], v[2], v[3]);
  *reinterpret_cast<float4*>(lds + off + HALF) = make_float4(v[4], v[5], v[6], v[7]);
}
template <int HALF>
__device__ __forceinline__ void ld8_h(const float* lds, int off, float v[8]) {
  const float4 a = *reinterpret_cast<const float4*>(lds + off);
  const float4 b = *reinterpret_cast<const float4*>(lds + off + HALF);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
template <int TX>
__device__ __forceinline__ void st8_at(float* lds, int off, const float v[8]) {
  st8_h<Tile<TX>::HALF>(lds, off, v);
}

// x pass of one output column from the eight P+ of column x - 1, the eight P0 of
// column x and the eight P- of column x + 1: back-map the 8 groups after the shift,
// then forward-map along y for the 9 (qx, mz) triples
__device__ __forceinline__ void x_pass_vals(const float pp[8], const float pz[8], const float pm[8], float yb[27]) {
  float B[3][3][3];  // [qx][my][mz]
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    float m0, m1, m2;
    back3(pp[g], pz[g], pm[g], m0, m1, m2);
    const int my = (g == 1 || g == 5 || g == 7) ? 1 : ((g == 3 || g == 6) ? 2 : 0);
    const int mz = (g == 2 || g == 5 || g == 6) ? 1 : ((g == 4 || g == 7) ? 2 : 0);
    B[0][my][mz] = m0; B[1][my][mz] = m1; B[2][my][mz] = m2;
  }
#pragma unroll
  for (int qx = 0; qx < 3; ++qx)
#pragma unroll
    for (int mz = 0; mz < 3; ++mz) {
      const float b2 = (mz == 2) ? 0.0f : B[qx][2][mz];
      const int t = 3 * qx + mz;
      fwd3(B[qx][0][mz], B[qx][1][mz], b2, yb[t], yb[9 + t], yb[18 + t]);
    }
}

// x pass for one row of a plane buffer (x-pass input at `base`, kinds KINDA apart,
// 4 floats per column, halves HALF apart), output column x (input columns x, x+1, x+2)
template <int HALF, int KINDA>
__device__ __forceinline__ void x_pass_row(const float* lds, int base, int x, float yb[27]) {
  float pp[8], pz[8], pm[8];
  ld8_h<HALF>(lds, base + 0 * KINDA + x * 4, pp);        // P+ of column x-1
  ld8_h<HALF>(lds, base + 1 * KINDA + (x + 1) * 4, pz);  // P0 of column x
  ld8_h<HALF>(lds, base + 2 * KINDA + (x + 2) * 4, pm);  // P- of column x+1
  x_pass_vals(pp, pz, pm, yb);
}

// Cross-lane moves of a wave (data-parallel primitives): lane i receives the value
// of lane i - 1 (lane_prev) or lane i + 1 (lane_next); the lanes at the ends of the
// wave receive zero. All 64 lanes must be active.
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// x pass of the lane's column when the lanes before and after it hold the columns
// x - 1 and x + 1 of the same row (p: the lane's own x-populations)
__device__ __forceinline__ void x_pass_lanes(const float p[24], float yb[27]) {
  float pp[8], pz[8], pm[8];
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    pp[g] = lane_prev(p[3 * g]);
    pz[g] = p[3 * g + 1];
    pm[g] = lane_next(p[3 * g + 2]);
  }
  x_pass_vals(pp, pz, pm, yb);
}

// x pass for tile row `row` (plane row row - 1), tile column x
template <int TX>
__device__ __forceinline__ void x_pass_tile(const float* lds, int row, int x, float yb[27]) {
  typedef Tile<TX> G;
  x_pass_row<G::HALF, G::KINDA>(lds, row * G::ROW, x, yb);
}

template <class S, int TX>
__device__ __forceinline__ void fetch_tile(const ScArgs<S>& a, const int* s_src, int px, int py, int pz,
                                           typename S::type raw[kMom]) {
  // node coordinates from the tile origin (at least -8) -> neighbourhood block per axis
  constexpr int NXB = Tile<TX>::NXB;
  const int ns = s_src[((px + 8) >> 3) + NXB * ((py + 8) >> 3) + 4 * NXB * ((pz + 8) >> 3)];
  const int node = (px & 7) + 8 * (py & 7) + 64 * (pz & 7);
  const typename S::type* src = a.in + (size_t)ns * kBlockStride + node;
#pragma unroll
  for (int m = 0; m < kMom; ++m) raw[m] = src[m * kNodes];
}

template <int TX>
__device__ __forceinline__ void fetch_cpl_tile(const float* cpl, const int* s_src, int px, int py, int pz,
                                               float c4[4]) {
  constexpr int NXB = Tile<TX>::NXB;
  const int ns = s_src[((px + 8) >> 3) + NXB * ((py + 8) >> 3) + 4 * NXB * ((pz + 8) >> 3)];
  load_cpl(cpl, ns, (px & 7) + 8 * (py & 7) + 64 * (pz & 7), c4);
}

template <class S, int TX, bool CPL>
__global__ __launch_bounds__(64 * 2 * TX) void k_stream_collide_tile(ScArgs<S> a) {
  typedef Tile<TX> G;
  __shared__ __align__(16) float lds[G::CY * G::ROW];
  __shared__ int s_src[G::NXB * 16];  // blocks (qx - 1 .. qx + TX) x (qy - 1 .. qy + 2) x (qz - 1 .. qz + 2)
  __shared__ int s_mem[4 * TX];       // the tile's blocks (or -1), x fastest
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int4 c0 = a.coord[a.tiles[xcd_remap(blockIdx.x, a.ntiles)]];
  const int qx = c0.x & ~(TX - 1), qy = c0.y & ~1, qz = c0.z & ~1;
  if (tid < G::NXB * 16) {
    const int ix = tid % G::NXB, iy = (tid / G::NXB) & 3, iz = tid / (4 * G::NXB);
    int h[3] = {qx + ix - 1, qy + iy - 1, qz + iz - 1};
    bool inside = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int nb = a.lg.nb[ax];
      if (h[ax] < 0 || h[ax] >= nb) {
        if (a.periodic[ax]) h[ax] = h[ax] < 0 ? h[ax] + nb : h[ax] - nb;
        else inside = false;
      }
    }
    const int ns = inside ? a.dir[a.lg.off + cell_lin(a.lg, h[0], h[1], h[2])] : -1;
    s_src[tid] = ns >= 0 ? ns : a.zero_slot;
    if (ix >= 1 && ix <= TX && iy >= 1 && iy <= 2 && iz >= 1 && iz <= 2) {
      const bool own = qx + ix - 1 < a.lg.nb[0] && qy + iy - 1 < a.lg.nb[1] && qz + iz - 1 < a.lg.nb[2];  // not wrapped
      s_mem[(ix - 1) + TX * (iy - 1) + 2 * TX * (iz - 1)] = own ? ns : -1;
    }
  }
  __syncthreads();

  // source points: THREADS in the first round, the rest on the last two waves (wave 0
  // takes the two extra rows of the x pass), which evens out the work per wave
  constexpr int base1 = G::THREADS - 128;
  int px[2], py[2];
  bool has[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int p = r == 0 ? tid : G::THREADS + (tid - base1);
    has[r] = r == 0 || (tid >= base1 && p < G::PTS);
    px[r] = p % G::CX - 1;
    py[r] = p / G::CX - 1;
  }
  const int slots[2] = {s_mem[wave], s_mem[wave + 2 * TX]};  // this wave's blocks, lower and upper
  const int ox = lane & 7, oy = lane >> 3;
  const int tx = (wave % TX) * 8 + ox, ty = (wave / TX) * 8 + oy;  // tile column of this lane
  uint64_t col_roles[2] = {0, 0};
#pragma unroll
  for (int zb = 0; zb < 2; ++zb) {
    if (slots[zb] < 0) continue;
    const uint8_t* rp = a.role + (size_t)slots[zb] * kNodes + ox + 8 * oy;
#pragma unroll
    for (int zz = 0; zz < 8; ++zz) col_roles[zb] |= (uint64_t)rp[64 * zz] << (8 * zz);
  }

  typedef typename S::type T;
  T nxt[2][kMom];
  float ncp[2][4];  // coupling fields of the prefetched points
#pragma unroll
  for (int r = 0; r < 2; ++r)
    if (has[r]) {
      fetch_tile<S, TX>(a, s_src, px[r], py[r], -1, nxt[r]);
      if (CPL) fetch_cpl_tile<TX>(a.cpl, s_src, px[r], py[r], -1, ncp[r]);
    }

  float zp1[6], zp2[6], z0[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) zp1[k] = zp2[k] = z0[k] = 0.0f;

  for (int z = -1; z <= 16; ++z) {
    // ---- source: moments of plane z (+ halo) -> x-populations, into LDS
    T cur[2][kMom];
    float ccp[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int m = 0; m < kMom; ++m) cur[r][m] = nxt[r][m];
#pragma unroll
      for (int m = 0; m < 4; ++m) ccp[r][m] = CPL ? ncp[r][m] : 0.0f;
    }
    if (z < 16) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (has[r]) {
          fetch_tile<S, TX>(a, s_src, px[r], py[r], z + 1, nxt[r]);
          if (CPL) fetch_cpl_tile<TX>(a.cpl, s_src, px[r], py[r], z + 1, ncp[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (!has[r]) continue;
      float q[kMom];
#pragma unroll
      for (int m = 0; m < kMom; ++m) q[m] = Codec<S>::load(cur[r][m], a.sc.inv[m]);
      float p[24];
      source_pops<CPL>(q, a.omega, ccp[r], p);
      float v[8];
      const int row = py[r] + 1, col = px[r] + 1;
#pragma unroll
      for (int kind = 0; kind < 3; ++kind) {
#pragma unroll
        for (int g = 0; g < 8; ++g) v[g] = p[3 * g + kind];
        st8_at<TX>(lds, row * G::ROW + kind * G::KINDA + col * 4, v);
      }
    }
    __syncthreads();

    // ---- x pass: CY rows x NX columns in two rounds (rows 0..15, then 16..17); each
    // row is overwritten by its y-pass input once its reads are done
    {
      float yb[27];
      const int row = tid / G::NX, x = tid % G::NX;
      x_pass_tile<TX>(lds, row, x, yb);
      __syncthreads();
      st9(lds, row * G::ROW + 0 * G::KINDB + x * 10, yb);
      st9(lds, row * G::ROW + 1 * G::KINDB + x * 10, yb + 9);
      st9(lds, row * G::ROW + 2 * G::KINDB + x * 10, yb + 18);
    }
    if (tid < 2 * G::NX) {
      float yb[27];
      const int row = 16 + tid / G::NX, x = tid % G::NX;
      x_pass_tile<TX>(lds, row, x, yb);
      st9(lds, row * G::ROW + 0 * G::KINDB + x * 10, yb);
      st9(lds, row * G::ROW + 1 * G::KINDB + x * 10, yb + 9);
      st9(lds, row * G::ROW + 2 * G::KINDB + x * 10, yb + 18);
    }
    __syncthreads();

    // ---- y pass for the lane's column, then z-forward
    float zpp[6], zpz[6], zpm[6];
    y_pass_col<G::ROW, G::KINDB>(lds, ty, tx, zpp, zpz, zpm);
    __syncthreads();

    // ---- z pass: output plane zo = z - 1 (block zo / 8 of the wave's column)
    const int zo = z - 1;
    const int slot = zo >= 8 ? slots[1] : slots[0];
    if (zo >= 0 && slot >= 0) {
      float M[10];
      z_back(zp2, z0, zpm, M);
      const int lz = zo & 7;
      const int node = ox + 8 * oy + 64 * lz;
      const uint8_t role = (uint8_t)((zo >= 8 ? col_roles[1] : col_roles[0]) >> (8 * lz));
      typename S::type* dst = a.out + (size_t)slot * kBlockStride + node;
      if ((role & ROLE_MASK) == ROLE_COMPUTED) {
        float c4[4] = {1.0f, 0.0f, 0.0f, 0.0f};
        if (CPL) load_cpl(a.cpl, slot, node, c4);
        if (role & ROLE_BB) bounce_back<S, CPL>(a, slot, ox, oy, lz, c4, M);
        // half the node's force in its velocity (Eq. rho_u_stress); 108 = 216 / 2
        if (CPL) {
          M[1] += 108.0f * c4[1];
          M[2] += 108.0f * c4[2];
          M[3] += 108.0f * c4[3];
        }
        float v[kMom];
        finish_moments(M, v);
#pragma unroll
        for (int m = 0; m < kMom; ++m) dst[m * kNodes] = Codec<S>::store(v[m], a.sc.s[m]);
      } else if ((role & ROLE_MASK) == ROLE_SOLID) {
#pragma unroll
        for (int m = 0; m < kMom; ++m) dst[m * kNodes] = Codec<S>::store(0.0f, a.sc.s[m]);
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      zp2[k] = zp1[k];
      zp1[k] = zpp[k];
      z0[k] = zpz[k];
    }
  }
}


// The next plane's source moments of a point, held while the current plane is
// processed: one register per moment in FP32, two 16-bit moments per register with
// 16-bit storage (the prefetch then holds 5 registers instead of 10).
template <class S> struct Prefetch {
  typename S::type v[kMom];
  __device__ void zero() {
#pragma unroll
    for (int m = 0; m < kMom; ++m) v[m] = typename S::type(0);
  }
  __device__ void fetch(const ScArgs<S>& a, const int* s_src, int px, int py, int pz) {
    fetch_tile<S, 2>(a, s_src, px, py, pz, v);
  }
  __device__ void load(const typename S::type* src) {  // the ten moments of one node
#pragma unroll
    for (int m = 0; m < kMom; ++m) v[m] = src[m * kNodes];
  }
  __device__ float get(int m, float inv) const { return Codec<S>::load(v[m], inv); }
};
template <class S> struct Prefetch16 {
  uint32_t w[kMom / 2];
  __device__ void zero() {
#pragma unroll
    for (int k = 0; k < kMom / 2; ++k) w[k] = 0u;
  }
  __device__ void fetch(const ScArgs<S>& a, const int* s_src, int px, int py, int pz) {
    uint16_t raw[kMom];
    fetch_tile<S, 2>(a, s_src, px, py, pz, raw);
    pack(raw);
  }
  __device__ void load(const uint16_t* src) {
    uint16_t raw[kMom];
#pragma unroll
    for (int m = 0; m < kMom; ++m) raw[m] = src[m * kNodes];
    pack(raw);
  }
  __device__ void pack(const uint16_t raw[kMom]) {
#pragma unroll
    for (int k = 0; k < kMom / 2; ++k) w[k] = (uint32_t)raw[2 * k] | ((uint32_t)raw[2 * k + 1] << 16);
  }
  __device__ float get(int m, float inv) const {
    const uint16_t b = (uint16_t)((m & 1) ? (w[m >> 1] >> 16) : (w[m >> 1] & 0xffffu));
    return Codec<S>::load(b, inv);
  }
};
// the ring values (loaded for a few lanes only, read in the same plane) are held packed
template <class S> struct Packed : Prefetch<S> {};
template <> struct Packed<StoreBF16> : Prefetch16<StoreBF16> {};
template <> struct Packed<StoreF16> : Prefetch16<StoreF16> {};

// ---- two substeps of the finest level in one sweep ----------------------------------
// The finest level takes its two substeps of a parent step back to back (Alg. 1):
// between them only its ghost nodes change, and their values for the second substep
// are written before the first. One workgroup takes a run of h 2 x 2 x 2 block tiles
// stacked along z (16 x 16 columns, Z = 16 h planes) through both. Substep A runs on
// the run plus a one-node ring (18 x 18 columns, planes -1 to Z) from the input with a
// two-node halo (20 x 20 points, planes -2 to Z + 1); substep B runs on the run from
// A's results, one plane behind. The halo and ring planes cost the same for any h, so
// taller runs spend less of the sweep on them (the first substep's ring and the halo:
// Z + 5 plane iterations for Z output planes). A's result never leaves the
// chip: the lane that finishes A's column p is the lane that feeds point p into B's
// source stage. The input is read once (with a two-node halo) and the output written
// once for two updates of every node.
// Each wave holds whole rows of a plane in consecutive lanes (three rows of 20 source
// points, three rows of 18 A columns, four rows of 16 B columns), so both x passes
// take their neighbours' populations by cross-lane moves; only the y passes go
// through LDS, with separate buffers for A and B. Per plane: phase 1 (A source and x
// pass of plane z; B y and z pass of the plane B got in the previous iteration),
// barrier, phase 2 (A y and z pass, B source and x pass), barrier.
// Nodes of A's ring that A does not compute take what the second substep reads
// otherwise: zero for solid nodes and missing blocks, the value already in the output
// time level for ghost and inflow nodes (never written by either substep). Outflow
// nodes (copied after every substep) and bounce-back nodes (whose correction needs the
// node's own intermediate moments) are not handled: levels that have them run the two
// substeps as two sweeps.
struct Pair {
  static constexpr int THREADS = 512;
  static constexpr int CXA = 20;               // A source plane: 20 x 20 points
  static constexpr int CA = 18;                // A columns (= B source points): 18 x 18
  static constexpr int KA = CA * 10;           // A y-pass input [row 0..19][kind][col 0..17][10]
  static constexpr int ROWA = 3 * KA + 24;     // 564 floats: 20 banks past a multiple of 32
  static constexpr int KB = 16 * 10;           // B y-pass input [row 0..17][kind][col 0..15][10]
  static constexpr int ROWB = 3 * KB;          // 480 floats: a multiple of 32 banks
  // Work of each wave, 4 bits per wave (wave w at bits 4w, 0xf: none), spread so that
  // the two waves of each SIMD (w, w + 4) carry similar loads in each phase (measured
  // 4% faster than the first seven, six and last four waves):
  static constexpr uint32_t SRC = 0x65f43210u;  // source rows 3s .. 3s + 2 (s = 0..6): waves 0-4, 6, 7
  static constexpr uint32_t COL = 0xff543210u;  // A column rows 3c .. 3c + 2 (c = 0..5): waves 0-5
  static constexpr uint32_t BCO = 0xff3f210fu;  // B column rows 4b .. 4b + 3 (b = 0..3): waves 1-3, 5
};

// role code of an A node: the role byte, or kPairZero for the all-zero slot
constexpr uint32_t kPairZero = 0xffu;

template <class S>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_stream_collide_pair(ScArgs<S> a) {
  typedef Pair P;
  typedef typename S::type T;
  __shared__ __align__(16) float lda[P::CXA * P::ROWA];
  __shared__ __align__(16) float ldb[P::CA * P::ROWB];
  __shared__ int s_src[16 * (2 * kRunMax + 2)];  // blocks (qx - 1 .. qx + 2) x (qy - 1 .. qy + 2) x (qz - 1 .. qz + 2h)
  __shared__ int s_mem[8 * kRunMax];             // the run's blocks (or -1), x fastest
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the workgroup's run: height class, then the run within the class (consecutive runs
  // on one XCD)
  const int bid = blockIdx.x;
  int cls = 0;
  while (cls < kRunMax - 1 && bid >= a.run_off[cls + 1]) ++cls;
  const int idx = xcd_remap(bid - a.run_off[cls], a.run_off[cls + 1] - a.run_off[cls]);
  if (idx >= a.run_n[cls]) return;  // padding of the class's range
  const int nt = kRunMax - cls;      // tiles in the run
  const int Z = 16 * nt;             // output planes
  const int4 c0 = a.coord[a.runs[(size_t)(nt - 1) * a.run_stride + idx]];
  const int qx = c0.x & ~1, qy = c0.y & ~1, qz = c0.z & ~1;
  if (tid < 16 * (2 * nt + 2)) {
    const int ix = tid & 3, iy = (tid >> 2) & 3, iz = tid >> 4;
    int h[3] = {qx + ix - 1, qy + iy - 1, qz + iz - 1};
    bool inside = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int nb = a.lg.nb[ax];
      if (h[ax] < 0 || h[ax] >= nb) {
        if (a.periodic[ax]) h[ax] = h[ax] < 0 ? h[ax] + nb : h[ax] - nb;
        else inside = false;
      }
    }
    const int ns = inside ? a.dir[a.lg.off + cell_lin(a.lg, h[0], h[1], h[2])] : -1;
    s_src[tid] = ns >= 0 ? ns : a.zero_slot;
    if (ix >= 1 && ix <= 2 && iy >= 1 && iy <= 2 && iz >= 1 && iz <= 2 * nt) {
      const bool own = qx + ix - 1 < a.lg.nb[0] && qy + iy - 1 < a.lg.nb[1] && qz + iz - 1 < a.lg.nb[2];
      s_mem[(ix - 1) + 2 * (iy - 1) + 4 * (iz - 1)] = own ? ns : -1;
    }
  }
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ss = (P::SRC >> (4 * wave)) & 0xf;
  const int cs = (P::COL >> (4 * wave)) & 0xf;
  const int bs = (P::BCO >> (4 * wave)) & 0xf;
  // A source point (20 x 20 plane, two-node halo); the lanes at row positions 1..18
  // write A's x-pass output of column position - 1
  const bool swave = ss != 0xf;
  const int sr = swave ? 3 * ss + lane / P::CXA : 0, sx = lane % P::CXA;
  const bool shas = swave && lane < 3 * P::CXA && sr < P::CXA;
  const bool swr = shas && sx >= 1 && sx <= P::CA;
  const int spx = sx - 2, spy = sr - 2;
  // A column (18 x 18: tile columns -1 .. 16), also B's source point; the lanes at
  // row positions 1..16 write B's x-pass output of column position - 1
  const bool cwave = cs != 0xf;
  const bool chas = cwave && lane < 3 * P::CA;
  const int cr = chas ? 3 * cs + lane / P::CA : 0, cxl = chas ? lane % P::CA : 0;
  const bool cwr = chas && cxl >= 1 && cxl <= 16;
  const int cx = cxl - 1, cy = cr - 1;
  const int cnode = (cx & 7) + 8 * (cy & 7);
  const int cblk = ((cx + 8) >> 3) + 4 * ((cy + 8) >> 3);
  // B output column (16 x 16)
  const bool bwave = bs != 0xf;
  const int tx = lane & 15, ty = 4 * (bwave ? bs : 0) + (lane >> 4);
  const int bq = (tx >> 3) + 2 * (ty >> 3);
  const int bnode = (tx & 7) + 8 * (ty & 7);

  Prefetch<S> nxt;
  nxt.zero();
  if (shas) nxt.fetch(a, s_src, spx, spy, -2);

  float azp1[6], azp2[6], az0[6];  // A's z window (the lane's A column)
  float bzp1[6], bzp2[6], bz0[6];  // B's z window (the lane's B column)
#pragma unroll
  for (int k = 0; k < 6; ++k) azp1[k] = azp2[k] = az0[k] = bzp1[k] = bzp2[k] = bz0[k] = 0.0f;
  uint32_t arole = kPairZero;  // role code of the A column's node at A's output plane
  int bslot = -1;              // block and role of the B column's node at B's next output plane
  uint32_t brole = ROLE_GHOST;

  for (int z = -2; z <= Z + 2; ++z) {
    const int zi = z - 1;  // A's output plane (B's source plane) of this iteration
    // ---- phase 1: A source and x pass of input plane z
    if (swave && z <= Z + 1) {
      const Prefetch<S> cur = nxt;
      if (shas && z < Z + 1) nxt.fetch(a, s_src, spx, spy, z + 1);
      float q[kMom];
#pragma unroll
      for (int m = 0; m < kMom; ++m) q[m] = cur.get(m, a.sc.inv[m]);
      float p[24];
      source_pops(q, a.omega, p);
      float yb[27];
      x_pass_lanes(p, yb);
      if (swr) {
        const int off = sr * P::ROWA + (sx - 1) * 10;
        st9(lda, off + 0 * P::KA, yb);
        st9(lda, off + 1 * P::KA, yb + 9);
        st9(lda, off + 2 * P::KA, yb + 18);
      }
    }
    // ---- phase 1: B y and z pass of B's source plane z - 2 (output plane z - 3)
    if (bwave) {
      if (z >= 1) {
        float zpp[6], zpz[6], zpm[6];
        y_pass_col<P::ROWB, P::KB>(ldb, ty, tx, zpp, zpz, zpm);
        if (bslot >= 0) {
          float M[10];
          z_back(bzp2, bz0, zpm, M);
          T* dst = a.out + (size_t)bslot * kBlockStride + bnode + 64 * ((z - 3) & 7);
          if ((brole & ROLE_MASK) == ROLE_COMPUTED) {
            float v[kMom];
            finish_moments(M, v);
#pragma unroll
            for (int m = 0; m < kMom; ++m) dst[m * kNodes] = Codec<S>::store(v[m], a.sc.s[m]);
          } else if ((brole & ROLE_MASK) == ROLE_SOLID) {
#pragma unroll
            for (int m = 0; m < kMom; ++m) dst[m * kNodes] = Codec<S>::store(0.0f, a.sc.s[m]);
          }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          bzp2[k] = bzp1[k];
          bzp1[k] = zpp[k];
          bz0[k] = zpz[k];
        }
      }
      // block and role of the next output plane z - 2
      const int zo = z - 2;
      bslot = zo >= 0 && zo < Z ? s_mem[bq + 4 * (zo >> 3)] : -1;
      brole = bslot >= 0 ? a.role[(size_t)bslot * kNodes + bnode + 64 * (zo & 7)] : ROLE_GHOST;
    }
    // value of A's output node (plane zi) where A does not compute it (ghost, inflow),
    // and the role code of the next output plane (plane z)
    Packed<S> pv;
    const uint32_t rk = arole & ROLE_MASK;
    const bool pass = chas && zi >= -1 && zi <= Z && arole != kPairZero && rk != ROLE_COMPUTED &&
                      rk != ROLE_SOLID;
    if (pass) {
      const int ns = s_src[cblk + 16 * ((zi + 8) >> 3)];
      pv.load(a.out + (size_t)ns * kBlockStride + cnode + 64 * (zi & 7));
    }
    uint32_t nrole = kPairZero;
    if (chas && z >= -1 && z <= Z) {
      const int ns = s_src[cblk + 16 * ((z + 8) >> 3)];
      if (ns != a.zero_slot) nrole = a.role[(size_t)ns * kNodes + cnode + 64 * (z & 7)];
    }
    __syncthreads();

    // ---- phase 2: A y and z pass (output plane zi), B source and x pass of plane zi
    if (cwave && z <= Z + 1) {
      float zpp[6], zpz[6], zpm[6];
      y_pass_col<P::ROWA, P::KA>(lda, cr, cxl, zpp, zpz, zpm);
      if (zi >= -1) {
        float qa[kMom];
        if (chas && arole != kPairZero && rk == ROLE_COMPUTED) {
          float M[10];
          z_back(azp2, az0, zpm, M);
          float v[kMom];
          finish_moments(M, v);
          // what the second substep would read back from memory
#pragma unroll
          for (int m = 0; m < kMom; ++m) qa[m] = Codec<S>::load(Codec<S>::store(v[m], a.sc.s[m]), a.sc.inv[m]);
        } else if (pass) {
#pragma unroll
          for (int m = 0; m < kMom; ++m) qa[m] = pv.get(m, a.sc.inv[m]);
        } else {
#pragma unroll
          for (int m = 0; m < kMom; ++m) qa[m] = 0.0f;
        }
        float p[24];
        source_pops(qa, a.omega, p);
        float yb[27];
        x_pass_lanes(p, yb);
        if (cwr) {
          const int off = cr * P::ROWB + cx * 10;
          st9(ldb, off + 0 * P::KB, yb);
          st9(ldb, off + 1 * P::KB, yb + 9);
          st9(ldb, off + 2 * P::KB, yb + 18);
        }
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        azp2[k] = azp1[k];
        azp1[k] = zpp[k];
        az0[k] = zpz[k];
      }
    }
    arole = nrole;
    __syncthreads();
  }
}

template <class S> hipError_t launch_sc_t(const ScLaunch& l, hipStream_t s) {
  if (l.nblocks <= 0) return hipSuccess;
  ScArgs<S> a;
  a.in = static_cast<const typename S::type*>(l.in);
  a.out = static_cast<typename S::type*>(l.out);
  a.blocks = l.blocks;
  a.nbr = l.nbr;
  a.role = l.role;
  a.nblocks = l.nblocks;
  a.zero_slot = l.zero_slot;
  a.omega = l.omega;
  a.sc = l.sc;
  a.tiles = l.tiles;
  a.ntiles = l.ntiles;
  a.dir = l.dir;
  a.coord = l.coord;
  a.lg = l.lg;
  for (int k = 0; k < 3; ++k) a.periodic[k] = l.periodic[k];
  a.cpl = l.cpl;
  const dim3 tg(Tile<kTileX>::THREADS);
  if (l.tiles) {
    if (l.ntiles <= 0) return hipSuccess;
    if (l.cpl) hipLaunchKernelGGL((k_stream_collide_tile<S, kTileX, true>), dim3(l.ntiles), tg, 0, s, a);
    else hipLaunchKernelGGL((k_stream_collide_tile<S, kTileX, false>), dim3(l.ntiles), tg, 0, s, a);
  } else {
    if (l.cpl) hipLaunchKernelGGL((k_stream_collide<S, true>), dim3(l.nblocks), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((k_stream_collide<S, false>), dim3(l.nblocks), dim3(64), 0, s, a);
  }
  return hipGetLastError();
}

template <class S> hipError_t launch_pair_t(const ScLaunch& l, hipStream_t s) {
  if (!l.tiles || l.ntiles <= 0) return l.tiles ? hipSuccess : hipErrorInvalidValue;
  if (!l.runs) return hipErrorInvalidValue;
  ScArgs<S> a;
  a.in = static_cast<const typename S::type*>(l.in);
  a.out = static_cast<typename S::type*>(l.out);
  a.blocks = l.blocks;
  a.nbr = l.nbr;
  a.role = l.role;
  a.nblocks = l.nblocks;
  a.zero_slot = l.zero_slot;
  a.omega = l.omega;
  a.sc = l.sc;
  a.tiles = l.tiles;
  a.ntiles = l.ntiles;
  a.dir = l.dir;
  a.coord = l.coord;
  a.lg = l.lg;
  for (int k = 0; k < 3; ++k) a.periodic[k] = l.periodic[k];
  a.cpl = nullptr;  // levels with coupling fields run two sweeps
  if (l.cpl) return hipErrorInvalidValue;
  // tallest runs first (the short ones fill in at the end of the launch); each class's
  // range of workgroups padded to a multiple of the 8 XCDs
  a.runs = l.runs;
  a.run_stride = l.run_stride;
  int64_t total = 0, tiles = 0;
  for (int c = 0; c < kRunMax; ++c) {
    const int h = kRunMax - c;
    const int32_t n = l.nrun[h - 1];
    if (n < 0 || n > l.run_stride) return hipErrorInvalidValue;
    a.run_off[c] = (int32_t)total;
    a.run_n[c] = n;
    total += (n + 7) / 8 * 8;
    tiles += (int64_t)h * n;
  }
  a.run_off[kRunMax] = (int32_t)total;
  if (tiles != l.ntiles) return hipErrorInvalidValue;  // the runs must cover the tiles
  hipLaunchKernelGGL(k_stream_collide_pair<S>, dim3((unsigned)total), dim3(Pair::THREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stream_collide_pair(const ScLaunch& a, hipStream_t s) {
  switch (a.storage) {
    case 0: return launch_pair_t<StoreF32>(a, s);
    case 1: return launch_pair_t<StoreBF16>(a, s);
    case 2: return launch_pair_t<StoreF16>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stream_collide(const ScLaunch& a, hipStream_t s) {
  switch (a.storage) {
    case 0: return launch_sc_t<StoreF32>(a, s);
    case 1: return launch_sc_t<StoreBF16>(a, s);
    case 2: return launch_sc_t<StoreF16>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbmx
