// Oracle: plain, slow, FP64 CPU reference of the block-adaptive, moment-encoded
// D3Q27 lattice Boltzmann step (arXiv 2603.14982, "Adaptive GPU Kinetic Solver
// for Fluid-Granular Flows").
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the package's smoke check and
// the CPU-baseline leg of the benchmark may load this library. It shares no
// code, header, table or constant with the GPU library: everything here is
// written out again from the paper's definitions.
//
// What it follows, section by section:
//   * Sec. 3.1, Eq. (rho_u_stress): the stored moments {rho, u, S} of a node.
//   * Sec. 3.1, Eq. (three_order_f): third-order Hermite reconstruction of the
//     populations from {rho, u, S}; full Hermite projection weights (1/(2cs^6)
//     for the six aab-type components, 1/cs^6 for xyz).
//   * Sec. 3.1, "Collision and Streaming": reconstruct, stream, take moments,
//     relax in moment space. Moments are stored before collision and relaxed
//     when read (BGK projected on S: S <- S + (uu - S)/tau).
//   * Sec. 5.1: levels with dx_l = 2^l dx_0, node-centred alignment (coarse node
//     q coincides with fine node 2q), 8^3-node blocks.
//   * Sec. 5.2: tau_l rescaling; S^neq rescaling across levels (Chapman-Enskog
//     factors by default, the printed factors selectable for comparison).
//   * Sec. 5.3, Alg. 1 (AdvanceLBM), Eq. (downward_rescale) with temporal
//     interpolation, and the upward transfer of Eq. (upload_S).
//   * Sec. 5.4: level selection Phi from particles (plus static solid nodes).
//   * Sec. 6.3: the block set after a grid update, written as the canonical
//     hierarchy H(Phi); new nodes initialised by downward interpolation from
//     coarser or upward transfer from finer nodes of the old hierarchy.
//   * Sec. 7 (dune migration, sand ripples): the convective outflow condition
//     (the moments of a boundary node obey dM/dt + u_n dM/dn = 0, u_n from the
//     nearest inner node along the face normal), taken as the implicit upwind
//     step M_b(t+1) = (M_b(t) + lam M_h(t+1)) / (1 + lam), lam = max(u_n, 0); and
//     the logarithmic inflow profile u(h) = u0 ln(1 + beta (h - h0)) over the
//     height h above h0 (zero at or below h0).
//   * Sec. 7 (powder snow): the volume fraction phi carried by the fluid velocity,
//     diffused and fed by a source (semi-Lagrangian RK3 advection, forward-Euler
//     diffusion), on the finest level.
//   * Sec. 4: the fluid fraction eps scaling tau and an external force density on
//     the finest level (Guo's forcing in moment form), the coupling hook.
// Bounce-back, periodic wrap, uniform inflow and zero-gradient outflow are not in
// the paper; they are the halfway bounce-back and equilibrium/copy conditions of
// the standard LBM literature.
//
// Everything is templated on the scalar type so that std::complex<double> can
// run the same arithmetic for complex-step derivatives.

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <functional>
#include <cstdint>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int kBlock = 8;            // nodes per block edge
constexpr int kNodes = 512;          // nodes per block
constexpr int kMom = 10;             // rho, u(3), S(6)

// node roles
enum : uint8_t { R_INTERIOR = 0, R_GHOST = 1, R_IU = 2, R_SOLID = 3, R_INFLOW = 4, R_OUTFLOW = 5 };
// boundary kinds per domain face
enum : int { BC_PERIODIC = 0, BC_INFLOW = 1, BC_OUTFLOW = 2, BC_WALL = 3, BC_OUTFLOW_CONV = 4 };
// block state per level
enum : uint8_t { ST_ABSENT = 0, ST_ACTIVE = 1, ST_DELETED = 2 };

// ---------------------------------------------------------------------------
// D3Q27 lattice: c_i in {-1,0,1}^3, i = (cx+1) + 3(cy+1) + 9(cz+1);
// w_i = w1(cx) w1(cy) w1(cz) with w1(0) = 2/3, w1(+-1) = 1/6; cs^2 = 1/3.
struct Lattice {
  int c[27][3];
  double w[27];
  int opp[27];
  Lattice() {
    for (int i = 0; i < 27; ++i) {
      c[i][0] = i % 3 - 1;
      c[i][1] = (i / 3) % 3 - 1;
      c[i][2] = i / 9 - 1;
      double wi = 1.0;
      for (int a = 0; a < 3; ++a) wi *= (c[i][a] == 0) ? 2.0 / 3.0 : 1.0 / 6.0;
      w[i] = wi;
    }
    for (int i = 0; i < 27; ++i)
      for (int j = 0; j < 27; ++j)
        if (c[j][0] == -c[i][0] && c[j][1] == -c[i][1] && c[j][2] == -c[i][2]) opp[i] = j;
  }
};
const Lattice LAT;
const double CS2 = 1.0 / 3.0;

// symmetric-tensor component index in the stored order xx,yy,zz,xy,xz,yz
inline int sidx(int a, int b) {
  if (a == b) return a;
  int lo = std::min(a, b), hi = std::max(a, b);
  if (lo == 0 && hi == 1) return 3;
  if (lo == 0 && hi == 2) return 4;
  return 5;
}

// Node moments in the oracle's own layout: q[0]=rho, q[1..3]=u, q[4..9]=S.
template <class T> struct Mom {
  T v[kMom];
  T rho() const { return v[0]; }
  T u(int a) const { return v[1 + a]; }
  T S(int a, int b) const { return v[4 + sidx(a, b)]; }
  T& S(int a, int b) { return v[4 + sidx(a, b)]; }
};

// Collision in moment space (BGK projected on the second moments): rho and u
// are kept, S relaxes to its equilibrium S^eq = u u (Eq. Seq with the
// second-order f^eq of Eq. lbe_feq) at rate omega = 1/tau.  With a body force
// F (Guo form in moments) the carried first moment becomes u + F/(2 rho) and S
// gains (1 - omega/2)(uF + Fu)/rho.
template <class T> Mom<T> collide(const Mom<T>& q, double omega, const double F[3]) {
  Mom<T> p = q;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      T seq = q.u(a) * q.u(b);
      T s = q.S(a, b) + omega * (seq - q.S(a, b));
      s = s + (1.0 - 0.5 * omega) * (q.u(a) * F[b] + F[a] * q.u(b)) / q.rho();
      p.S(a, b) = s;
    }
  for (int a = 0; a < 3; ++a) p.v[1 + a] = q.u(a) + 0.5 * F[a] / q.rho();
  return p;
}

// Eq. (three_order_f): f_i = rho w_i [1 + c.u/cs^2 + H2(c):S/(2cs^4)
//   + sum over the seven D3Q27-supported third-order components of
//     H3_abg(c) Gamma_abg / (2 cs^6) (xyz counted with its full Hermite
//     multiplicity, i.e. 1/cs^6) ],
//   Gamma_abg = S_ab u_g + S_ag u_b + S_bg u_a - 2 u_a u_b u_g.
template <class T> T reconstruct(const Mom<T>& p, int i) {
  const int* c = LAT.c[i];
  T cu = T(0);
  for (int a = 0; a < 3; ++a) cu = cu + double(c[a]) * p.u(a);
  T h2 = T(0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) h2 = h2 + (double(c[a] * c[b]) - (a == b ? CS2 : 0.0)) * p.S(a, b);
  auto Gam = [&](int a, int b, int g) {
    return p.S(a, b) * p.u(g) + p.S(a, g) * p.u(b) + p.S(b, g) * p.u(a) - 2.0 * p.u(a) * p.u(b) * p.u(g);
  };
  // H3_aab(c) = (c_a^2 - cs^2) c_b for a != b; H3_xyz(c) = c_x c_y c_z
  T h3 = T(0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      if (a == b) continue;
      double H = (double(c[a] * c[a]) - CS2) * double(c[b]);
      h3 = h3 + H * Gam(a, a, b) / (2.0 * CS2 * CS2 * CS2);
    }
  h3 = h3 + double(c[0] * c[1] * c[2]) * Gam(0, 1, 2) / (CS2 * CS2 * CS2);
  return p.rho() * LAT.w[i] * (1.0 + cu / CS2 + h2 / (2.0 * CS2 * CS2) + h3);
}

// Storage rounding of one stored value v (already shifted: rho-1 for the first
// moment) with scale s: v*s rounded to f32 (nearest even), then to bf16 or f16
// (nearest even), divided by s again.
inline double round_bf16(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  b += 0x7fffu + ((b >> 16) & 1u);
  b &= 0xffff0000u;
  float r;
  std::memcpy(&r, &b, 4);
  return double(r);
}
inline double round_f16(float f) {
  // nearest-even rounding to IEEE binary16 (normal and subnormal ranges, overflow to infinity)
  double a = std::fabs(double(f));
  if (a == 0.0) return double(f);
  int e;
  std::frexp(a, &e);                 // a = m 2^e, m in [0.5, 1)
  int ulp_exp = std::max(e - 11, -24);  // 11 significant bits; subnormal spacing 2^-24
  double q = std::ldexp(std::nearbyint(std::ldexp(a, -ulp_exp)), ulp_exp);
  if (q >= 65536.0) q = HUGE_VAL;  // beyond the largest finite binary16 (65504)
  return f < 0 ? -q : q;
}
inline double store_round(double v, int storage, double scale) {
  if (storage == 0) return v;
  float f = float(v * scale);
  double r = storage == 1 ? round_bf16(f) : round_f16(f);
  return r / scale;
}

inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t k = 0;
  for (int bit = 0; bit < 21; ++bit) {
    k |= uint64_t((x >> bit) & 1u) << (3 * bit);
    k |= uint64_t((y >> bit) & 1u) << (3 * bit + 1);
    k |= uint64_t((z >> bit) & 1u) << (3 * bit + 2);
  }
  return k;
}
inline void demorton3(uint64_t k, int b[3]) {
  b[0] = b[1] = b[2] = 0;
  for (int bit = 0; bit < 21; ++bit)
    for (int a = 0; a < 3; ++a) b[a] |= int((k >> (3 * bit + a)) & 1u) << bit;
}

}  // namespace

extern "C" {
// Mirrors the GPU library's configuration in meaning only (no shared header).
struct oc_config {
  int32_t levels;
  int32_t n[3];        // fine-equivalent nodes per axis
  int32_t bc[6];       // x-, x+, y-, y+, z-, z+
  double uin[3];       // inflow velocity
  double tau0;         // finest-level relaxation time
  double force[3];     // body force on level 0 (oracle-only physics checks)
  int32_t rescale;     // 0: Chapman-Enskog S^neq factors; 1: factors as printed
  int32_t storage;     // 0: exact; 1: bf16, 2: f16 storage emulation (rho-1 shift, scales)
  double scale[10];    // per-moment power-of-two storage scales
  int32_t inflow_profile;  // 0: uniform uin; 1: uin * ln(1 + beta (h - h0)) over the height h
  int32_t inflow_axis;     // axis of the height h (fine units)
  double inflow_beta;
  double inflow_h0;
};
}

namespace {

// real part (branch decisions of the complex-step instance follow the real run)
inline double re(double v) { return v; }
inline double re(const std::complex<double>& v) { return v.real(); }

template <class T> Mom<T> quantize(const Mom<T>& q, const oc_config&) { return q; }
template <> Mom<double> quantize(const Mom<double>& q, const oc_config& c) {
  if (c.storage == 0) return q;
  Mom<double> r = q;
  r.v[0] = 1.0 + store_round(q.v[0] - 1.0, c.storage, c.scale[0]);
  for (int m = 1; m < kMom; ++m) r.v[m] = store_round(q.v[m], c.storage, c.scale[m]);
  return r;
}

template <class T> struct Blk {
  int lvl = 0;
  int b[3] = {0, 0, 0};
  uint64_t key = 0;
  std::vector<Mom<T>> cur, prev;      // state at t and before the last SC
  uint8_t role[kNodes];
  Blk* nb[27];                        // same-level neighbour blocks (periodic wrap), or null
  long idx = 0;                       // position in the per-step block list
  // finest level only: coupling fields [4][512] (fluid fraction eps, force density
  // F), empty for eps = 1, F = 0
  std::vector<double> cpl;
  // finest level only: the powder-snow volume fraction phi [512], empty for 0
  std::vector<double> phi;
};

template <class T> struct Sim {
  oc_config cfg;
  int L = 1;
  int N[3];
  std::vector<double> tau, omega, a_up, a_down;
  std::vector<uint8_t> solid;                            // fine field, empty if none
  std::vector<std::map<uint64_t, Blk<T>>> lv;            // active blocks per level
  std::vector<std::map<uint64_t, uint8_t>> st;           // ACTIVE / DELETED per level
  std::string err;

  int nl(int l, int a) const { return N[a] >> l; }
  int nbk(int l, int a) const { return (N[a] >> l) / kBlock; }
  bool periodic(int a) const { return cfg.bc[2 * a] == BC_PERIODIC; }

  // --- per-level physical parameters (Sec. 5.2) ---
  void setup_levels() {
    tau.resize(L); omega.resize(L); a_up.assign(L, 1.0); a_down.assign(L, 1.0);
    for (int l = 0; l < L; ++l) {
      double k = std::ldexp(1.0, l);
      tau[l] = cfg.tau0 / k + (k - 1.0) / (2.0 * k);
      omega[l] = 1.0 / tau[l];
    }
    for (int l = 0; l + 1 < L; ++l) {
      if (cfg.rescale == 0) {
        // Chapman-Enskog: S^neq ~ -cs^2 tau_l dx_l (grad u + grad u^T)
        a_up[l] = 2.0 * tau[l + 1] / tau[l];      // fine l -> coarse l+1
        a_down[l] = tau[l] / (2.0 * tau[l + 1]);  // coarse l+1 -> fine l
      } else {
        a_up[l] = tau[l + 1] / (2.0 * tau[l]);    // Eq. upload_S as printed
        a_down[l] = 2.0 * tau[l + 1] / tau[l];    // Eq. downward_rescale as printed
      }
    }
  }
  void force_at(int l, double F[3]) const {
    for (int a = 0; a < 3; ++a) F[a] = cfg.force[a] * std::ldexp(1.0, l);
  }
  // relaxation rate and force of node n of a block on level l: the level's, with the
  // finest level's coupling fields (Sec. 4: tau scaled by the fluid fraction eps,
  // the external force density F added to the body force)
  void node_params(int l, const Blk<T>& B, int n, double& om, double F[3]) const {
    force_at(l, F);
    om = omega[l];
    if (l != 0 || B.cpl.empty()) return;
    om = 1.0 / (B.cpl[n] * tau[0]);
    for (int a = 0; a < 3; ++a) F[a] += B.cpl[(1 + a) * kNodes + n];
  }

  // --- domain helpers ---
  // wrap node coordinate g on level l; returns false if outside a non-periodic axis
  bool wrap_node(int l, int g[3]) const {
    for (int a = 0; a < 3; ++a) {
      int n = nl(l, a);
      if (g[a] < 0 || g[a] >= n) {
        if (!periodic(a)) return false;
        g[a] = ((g[a] % n) + n) % n;
      }
    }
    return true;
  }
  bool wrap_block(int l, int b[3]) const {
    for (int a = 0; a < 3; ++a) {
      int n = nbk(l, a);
      if (b[a] < 0 || b[a] >= n) {
        if (!periodic(a)) return false;
        b[a] = ((b[a] % n) + n) % n;
      }
    }
    return true;
  }
  bool solid_node(int l, const int g[3]) const {
    if (solid.empty()) return false;
    int64_t x = int64_t(g[0]) << l, y = int64_t(g[1]) << l, z = int64_t(g[2]) << l;
    return solid[size_t(x + int64_t(N[0]) * (y + int64_t(N[1]) * z))] != 0;
  }
  // wall neighbour: outside the domain across a WALL face
  bool wall_outside(int l, const int g[3]) const {
    for (int a = 0; a < 3; ++a) {
      if (g[a] < 0 && cfg.bc[2 * a] == BC_WALL) return true;
      if (g[a] >= nl(l, a) && cfg.bc[2 * a + 1] == BC_WALL) return true;
    }
    return false;
  }
  uint8_t state_of(int l, const int b[3]) const {
    auto it = st[l].find(morton3(b[0], b[1], b[2]));
    return it == st[l].end() ? uint8_t(ST_ABSENT) : it->second;
  }
  Blk<T>* find_block(int l, const int b[3]) {
    auto it = lv[l].find(morton3(b[0], b[1], b[2]));
    return it == lv[l].end() ? nullptr : &it->second;
  }
  // locate a level-l node (already wrapped) in the active blocks
  Blk<T>* locate(int l, const int g[3], int& node) {
    int b[3] = {g[0] / kBlock, g[1] / kBlock, g[2] / kBlock};
    node = (g[0] % kBlock) + kBlock * ((g[1] % kBlock) + kBlock * (g[2] % kBlock));
    return find_block(l, b);
  }

  // --- roles (inflow/outflow on domain faces; ghost = outer shell of a level's
  //     region; IU = nodes next to blocks covered by the finer level) ---
  static bool is_outflow(int kind) { return kind == BC_OUTFLOW || kind == BC_OUTFLOW_CONV; }
  // outward normal of the first outflow face (in axis order) the node lies on;
  // returns that face's kind, or 0 if none
  int face_normal_outflow(int l, const int g[3], int normal[3]) const {
    for (int a = 0; a < 3; ++a) {
      if (periodic(a)) continue;
      if (g[a] == 0 && is_outflow(cfg.bc[2 * a])) {
        normal[0] = normal[1] = normal[2] = 0; normal[a] = -1; return cfg.bc[2 * a];
      }
      if (g[a] == nl(l, a) - 1 && is_outflow(cfg.bc[2 * a + 1])) {
        normal[0] = normal[1] = normal[2] = 0; normal[a] = 1; return cfg.bc[2 * a + 1];
      }
    }
    return 0;
  }
  uint8_t face_role(int l, const int g[3]) const {
    for (int a = 0; a < 3; ++a) {
      if (periodic(a)) continue;
      int kind = -1;
      if (g[a] == 0) kind = cfg.bc[2 * a];
      else if (g[a] == nl(l, a) - 1) kind = cfg.bc[2 * a + 1];
      if (kind == BC_INFLOW) return R_INFLOW;
      if (is_outflow(kind)) return R_OUTFLOW;
    }
    return 255;
  }
  uint8_t node_role(int l, const int g[3]) const {
    if (solid_node(l, g)) return R_SOLID;
    uint8_t fr = face_role(l, g);
    if (fr != 255) return fr;
    bool ghost = false, iu = false;
    for (int i = 0; i < 27; ++i) {
      if (i == 13) continue;
      int h[3] = {g[0] + LAT.c[i][0], g[1] + LAT.c[i][1], g[2] + LAT.c[i][2]};
      if (!wrap_node(l, h)) continue;  // outside a non-periodic face: wall or boundary
      int hb[3] = {h[0] / kBlock, h[1] / kBlock, h[2] / kBlock};
      uint8_t s = state_of(l, hb);
      if (s == ST_ABSENT) ghost = true;
      if (s == ST_DELETED) iu = true;
    }
    if (ghost) return R_GHOST;
    if (iu) return R_IU;
    return R_INTERIOR;
  }
  static bool owned(uint8_t r) { return r == R_INTERIOR || r == R_IU || r == R_INFLOW || r == R_OUTFLOW; }

  // storage emulation of the GPU's 16-bit formats (identity for exact storage)
  Mom<T> stored(const Mom<T>& q) const { return quantize(q, cfg); }

  void link_level(int l) {
    for (auto& kv : lv[l]) {
      Blk<T>& B = kv.second;
      for (int i = 0; i < 27; ++i) {
        int b[3] = {B.b[0] + LAT.c[i][0], B.b[1] + LAT.c[i][1], B.b[2] + LAT.c[i][2]};
        B.nb[i] = wrap_block(l, b) ? find_block(l, b) : nullptr;
      }
    }
  }
  void assign_roles(Blk<T>& B) {
    for (int n = 0; n < kNodes; ++n) {
      int g[3] = {B.b[0] * kBlock + n % kBlock, B.b[1] * kBlock + (n / kBlock) % kBlock, B.b[2] * kBlock + n / (kBlock * kBlock)};
      B.role[n] = node_role(B.lvl, g);
    }
  }

  // --- canonical hierarchy H(Phi) (Sec. 5.4 Phi, Sec. 6.3 refinement) ---
  // T0: level-0 blocks holding a particle or a solid node.
  // D_1 = parent(T0); B_l = N26(D_l) \ D_l; D_{l+1} = parent(D_l u B_l);
  // A_0 = children(D_1 u B_1); A_l = children(D_{l+1} u B_{l+1}) \ D_l; A_{L-1} = all \ D_{L-1}.
  typedef std::map<uint64_t, std::array<int, 3>> BSet;
  void insert(BSet& s, const int b[3]) { s[morton3(b[0], b[1], b[2])] = {b[0], b[1], b[2]}; }

  std::vector<std::map<uint64_t, uint8_t>> hierarchy_states(const BSet& T0) {
    std::vector<BSet> D(L), Bring(L);
    if (L > 1) {
      for (auto& kv : T0) { int p[3] = {kv.second[0] / 2, kv.second[1] / 2, kv.second[2] / 2}; insert(D[1], p); }
      for (int l = 1; l < L; ++l) {
        for (auto& kv : D[l])
          for (int i = 0; i < 27; ++i) {
            int b[3] = {kv.second[0] + LAT.c[i][0], kv.second[1] + LAT.c[i][1], kv.second[2] + LAT.c[i][2]};
            if (!wrap_block(l, b)) continue;
            if (!D[l].count(morton3(b[0], b[1], b[2]))) insert(Bring[l], b);
          }
        if (l + 1 < L) {
          for (auto* S : {&D[l], &Bring[l]})
            for (auto& kv : *S) { int p[3] = {kv.second[0] / 2, kv.second[1] / 2, kv.second[2] / 2}; insert(D[l + 1], p); }
        }
      }
    }
    std::vector<std::map<uint64_t, uint8_t>> out(L);
    for (int l = 0; l < L; ++l) {
      for (auto& kv : D[l]) out[l][kv.first] = ST_DELETED;
      if (l == L - 1) {
        for (int z = 0; z < nbk(l, 2); ++z)
          for (int y = 0; y < nbk(l, 1); ++y)
            for (int x = 0; x < nbk(l, 0); ++x) {
              uint64_t k = morton3(x, y, z);
              if (!D[l].count(k)) out[l][k] = ST_ACTIVE;
            }
      } else {
        for (auto* S : {&D[l + 1], &Bring[l + 1]})
          for (auto& kv : *S)
            for (int ci = 0; ci < 8; ++ci) {
              int b[3] = {2 * kv.second[0] + (ci & 1), 2 * kv.second[1] + ((ci >> 1) & 1), 2 * kv.second[2] + ((ci >> 2) & 1)};
              uint64_t k = morton3(b[0], b[1], b[2]);
              if (!D[l].count(k)) out[l][k] = ST_ACTIVE;
            }
      }
    }
    return out;
  }

  BSet mark_T0(const float* p, int64_t np) {
    BSet T0;
    for (int64_t i = 0; i < np; ++i) {
      int b[3];
      bool inside = true;
      for (int a = 0; a < 3; ++a) {
        float q = p[3 * i + a];
        if (!periodic(a) && (q < 0.0f || q >= float(N[a]))) inside = false;
        float s = std::floor(q * 0.125f);
        long v = long(s);
        b[a] = int(v);
      }
      if (!inside) continue;
      if (!wrap_block(0, b)) continue;
      insert(T0, b);
    }
    if (!solid.empty()) {
      for (int z = 0; z < N[2]; ++z)
        for (int y = 0; y < N[1]; ++y)
          for (int x = 0; x < N[0]; ++x)
            if (solid[size_t(x + int64_t(N[0]) * (y + int64_t(N[1]) * z))]) {
              int b[3] = {x / kBlock, y / kBlock, z / kBlock};
              insert(T0, b);
            }
    }
    return T0;
  }

  Mom<T> rest_state() const {
    Mom<T> q;
    for (int m = 0; m < kMom; ++m) q.v[m] = T(0);
    q.v[0] = T(1);
    return q;
  }
  // inflow node g of level l: rho = 1, u = uin (times the log profile at the node's
  // height), S = u u
  Mom<T> inflow_state(int l, const int g[3]) const {
    double f = 1.0;
    if (cfg.inflow_profile == 1) {
      const double h = double(g[cfg.inflow_axis]) * double(1 << l);  // fine units
      f = h > cfg.inflow_h0 ? std::log(1.0 + cfg.inflow_beta * (h - cfg.inflow_h0)) : 0.0;
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = cfg.uin[a] * f;
    Mom<T> q = rest_state();
    for (int a = 0; a < 3; ++a) q.v[1 + a] = T(u[a]);
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) q.S(a, b) = T(u[a] * u[b]);
    return q;
  }
  static void node_coords(const int b[3], int n, int g[3]) {
    g[0] = b[0] * kBlock + n % kBlock;
    g[1] = b[1] * kBlock + (n / kBlock) % kBlock;
    g[2] = b[2] * kBlock + n / (kBlock * kBlock);
  }

  void build(const std::vector<std::map<uint64_t, uint8_t>>& states) {
    st = states;
    lv.assign(L, {});
    for (int l = 0; l < L; ++l)
      for (auto& kv : st[l]) {
        if (kv.second != ST_ACTIVE) continue;
        Blk<T>& B = lv[l][kv.first];
        B.lvl = l; B.key = kv.first;
        demorton3(kv.first, B.b);
        B.cur.assign(kNodes, rest_state());
        B.prev = B.cur;
      }
    for (int l = 0; l < L; ++l) {
      link_level(l);
      for (auto& kv : lv[l]) assign_roles(kv.second);
    }
  }

  // --- Eq. (downward_rescale) + temporal interpolation, written for a single
  //     target node: rho, u and S^neq = S - uu are interpolated linearly ---
  struct Lin { T rho; T u[3]; T sn[6]; };
  Lin lin_of(const Mom<T>& q) const {
    Lin r; r.rho = q.rho();
    for (int a = 0; a < 3; ++a) r.u[a] = q.u(a);
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) r.sn[sidx(a, b)] = q.S(a, b) - q.u(a) * q.u(b);
    return r;
  }
  Mom<T> mom_of(const Lin& r) const {
    Mom<T> q; q.v[0] = r.rho;
    for (int a = 0; a < 3; ++a) q.v[1 + a] = r.u[a];
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) q.S(a, b) = r.sn[sidx(a, b)] + r.u[a] * r.u[b];
    return q;
  }
  static void lin_axpy(Lin& acc, double w, const Lin& x, double sfac) {
    acc.rho = acc.rho + w * x.rho;
    for (int a = 0; a < 3; ++a) acc.u[a] = acc.u[a] + w * x.u[a];
    for (int k = 0; k < 6; ++k) acc.sn[k] = acc.sn[k] + (w * sfac) * x.sn[k];
  }
  static Lin lin_zero() { Lin r; r.rho = T(0); for (auto& x : r.u) x = T(0); for (auto& x : r.sn) x = T(0); return r; }

  // nearest 2^D coarse nodes of fine node g (level l) on level l+1 with weights
  int coarse_stencil(int l, const int g[3], int js[8][3], double ws[8]) const {
    int cand[3][2], cw[3][2], cnt[3];
    double wv[3][2];
    for (int a = 0; a < 3; ++a) {
      int nc = nl(l + 1, a);
      if (g[a] % 2 == 0) { cand[a][0] = g[a] / 2; wv[a][0] = 1.0; cnt[a] = 1; }
      else { cand[a][0] = (g[a] - 1) / 2; cand[a][1] = (g[a] + 1) / 2; wv[a][0] = wv[a][1] = 0.5; cnt[a] = 2; }
      for (int k = 0; k < cnt[a]; ++k) {
        int v = cand[a][k];
        if (periodic(a)) v = ((v % nc) + nc) % nc;
        else v = std::min(std::max(v, 0), nc - 1);
        cand[a][k] = v;
      }
      (void)cw;
    }
    int n = 0;
    for (int kz = 0; kz < cnt[2]; ++kz)
      for (int ky = 0; ky < cnt[1]; ++ky)
        for (int kx = 0; kx < cnt[0]; ++kx) {
          js[n][0] = cand[0][kx]; js[n][1] = cand[1][ky]; js[n][2] = cand[2][kz];
          ws[n] = wv[0][kx] * wv[1][ky] * wv[2][kz];
          ++n;
        }
    return n;
  }

  // DownwardTransfer(l+1, s): fill the ghost nodes of level l from level l+1.
  void downward(int l, int s) {
    std::vector<std::pair<Blk<T>*, int>> todo;
    for (auto& kv : lv[l])
      for (int n = 0; n < kNodes; ++n)
        if (kv.second.role[n] == R_GHOST) todo.push_back({&kv.second, n});
    const double ad = a_down[l];
    std::string local_err;
#pragma omp parallel for schedule(static)
    for (long t = 0; t < long(todo.size()); ++t) {
      Blk<T>* B = todo[t].first; int n = todo[t].second;
      int g[3] = {B->b[0] * kBlock + n % kBlock, B->b[1] * kBlock + (n / kBlock) % kBlock, B->b[2] * kBlock + n / (kBlock * kBlock)};
      int js[8][3]; double ws[8];
      int cnt = coarse_stencil(l, g, js, ws);
      Lin acc = lin_zero();
      for (int k = 0; k < cnt; ++k) {
        int node;
        Blk<T>* C = locate(l + 1, js[k], node);
        if (!C || C->role[node] == R_GHOST || C->role[node] == R_IU || C->role[node] == R_SOLID) {
#pragma omp critical
          local_err = "downward transfer: coarse source node is not computed";
          continue;
        }
        Lin src;
        if (s == 1) src = lin_of(C->prev[node]);
        else {
          // temporal interpolation to the midpoint of the coarse step
          Lin a0 = lin_of(C->prev[node]), a1 = lin_of(C->cur[node]);
          src = lin_zero(); lin_axpy(src, 0.5, a0, 1.0); lin_axpy(src, 0.5, a1, 1.0);
        }
        lin_axpy(acc, ws[k], src, ad);
      }
      B->cur[n] = stored(mom_of(acc));
    }
    if (!local_err.empty()) throw std::runtime_error(local_err);
  }

  // UpwardTransfer(l): fill the IU nodes of level l+1 from the coincident
  // level-l nodes with S^neq rescaled (Eq. upload_S).
  void upward(int l) {
    std::vector<std::pair<Blk<T>*, int>> todo;
    for (auto& kv : lv[l + 1])
      for (int n = 0; n < kNodes; ++n)
        if (kv.second.role[n] == R_IU) todo.push_back({&kv.second, n});
    const double au = a_up[l];
    std::string local_err;
#pragma omp parallel for schedule(static)
    for (long t = 0; t < long(todo.size()); ++t) {
      Blk<T>* B = todo[t].first; int n = todo[t].second;
      int q[3] = {B->b[0] * kBlock + n % kBlock, B->b[1] * kBlock + (n / kBlock) % kBlock, B->b[2] * kBlock + n / (kBlock * kBlock)};
      int f[3] = {2 * q[0], 2 * q[1], 2 * q[2]};
      int node;
      Blk<T>* F = locate(l, f, node);
      if (!F || F->role[node] != R_INTERIOR) {
#pragma omp critical
        local_err = "upward transfer: fine source node is not computed";
        continue;
      }
      Lin acc = lin_zero();
      lin_axpy(acc, 1.0, lin_of(F->cur[node]), au);
      B->cur[n] = stored(mom_of(acc));
    }
    if (!local_err.empty()) throw std::runtime_error(local_err);
  }

  // StreamingCollision(l): for every computed node, pull the 27 populations
  // reconstructed from the (collided) neighbours, with halfway bounce-back at
  // solid nodes and walls, then take moments.
  void stream_collide(int l) {
    std::vector<Blk<T>*> blocks;
    for (auto& kv : lv[l]) blocks.push_back(&kv.second);
    // collision applied at every node (moments stored before collision)
    std::vector<std::vector<Mom<T>>> post(blocks.size());
    for (size_t k = 0; k < blocks.size(); ++k) blocks[k]->idx = long(k);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < long(blocks.size()); ++k) {
      post[k].resize(kNodes);
      for (int n = 0; n < kNodes; ++n) {
        double om, F[3];
        node_params(l, *blocks[k], n, om, F);
        post[k][n] = collide(blocks[k]->cur[n], om, F);
      }
    }
    std::vector<std::vector<Mom<T>>> next(blocks.size());
    std::string local_err;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < long(blocks.size()); ++k) {
      Blk<T>* B = blocks[k];
      next[k] = B->cur;
      for (int n = 0; n < kNodes; ++n) {
        if (B->role[n] != R_INTERIOR) continue;
        int lx = n % kBlock, ly = (n / kBlock) % kBlock, lz = n / (kBlock * kBlock);
        int g[3] = {B->b[0] * kBlock + lx, B->b[1] * kBlock + ly, B->b[2] * kBlock + lz};
        T rho = T(0), j[3] = {T(0), T(0), T(0)}, pi[3][3];
        for (auto& r : pi) for (auto& x : r) x = T(0);
        for (int i = 0; i < 27; ++i) {
          int h[3] = {g[0] - LAT.c[i][0], g[1] - LAT.c[i][1], g[2] - LAT.c[i][2]};
          T f;
          bool bounce = false;
          const Mom<T>* src = nullptr;
          if (!wrap_node(l, h)) {
            if (!wall_outside(l, h)) {
#pragma omp critical
              local_err = "stream: computed node pulls from outside the domain";
            }
            bounce = true;
          } else {
            // neighbour block through the block's own link table
            int ox = (lx - LAT.c[i][0] < 0) ? -1 : (lx - LAT.c[i][0] >= kBlock ? 1 : 0);
            int oy = (ly - LAT.c[i][1] < 0) ? -1 : (ly - LAT.c[i][1] >= kBlock ? 1 : 0);
            int oz = (lz - LAT.c[i][2] < 0) ? -1 : (lz - LAT.c[i][2] >= kBlock ? 1 : 0);
            Blk<T>* NB = B->nb[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)];
            int node = (h[0] % kBlock) + kBlock * ((h[1] % kBlock) + kBlock * (h[2] % kBlock));
            if (!NB) {
#pragma omp critical
              local_err = "stream: computed node pulls from a missing block";
              bounce = true;
            } else if (NB->role[node] == R_SOLID) {
              bounce = true;
            } else {
              src = &post[NB->idx][node];
            }
          }
          if (bounce) f = reconstruct(post[k][n], LAT.opp[i]);
          else f = reconstruct(*src, i);
          rho = rho + f;
          for (int a = 0; a < 3; ++a) j[a] = j[a] + double(LAT.c[i][a]) * f;
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) pi[a][b] = pi[a][b] + double(LAT.c[i][a] * LAT.c[i][b]) * f;
        }
        double om_n, F[3];
        node_params(l, *B, n, om_n, F);
        Mom<T> q;
        q.v[0] = rho;
        for (int a = 0; a < 3; ++a) q.v[1 + a] = (j[a] + 0.5 * F[a]) / rho;
        for (int a = 0; a < 3; ++a)
          for (int b = a; b < 3; ++b) q.S(a, b) = pi[a][b] / rho - (a == b ? CS2 : 0.0);
        next[k][n] = stored(q);
      }
    }
    if (!local_err.empty()) throw std::runtime_error(local_err);
    // outflow nodes, from the new value of the inward neighbour when that
    // neighbour is a computed node (otherwise the node keeps its value):
    // zero gradient copies it; the convective condition takes one implicit upwind
    // step of dM/dt + u_n dM/dn = 0 with u_n the neighbour's new outward velocity
    // (clamped at zero: no transport into the domain through an outlet).
    for (size_t k = 0; k < blocks.size(); ++k) {
      Blk<T>* B = blocks[k];
      for (int n = 0; n < kNodes; ++n) {
        if (B->role[n] != R_OUTFLOW) continue;
        int g[3];
        node_coords(B->b, n, g);
        int nrm[3];
        const int kind = face_normal_outflow(l, g, nrm);
        int h[3] = {g[0] - nrm[0], g[1] - nrm[1], g[2] - nrm[2]};
        int node;
        Blk<T>* S = locate(l, h, node);
        if (!(S && S->role[node] == R_INTERIOR)) continue;
        const Mom<T>& qh = next[S->idx][node];
        if (kind == BC_OUTFLOW) {
          next[k][n] = qh;
          continue;
        }
        T un = T(0.0);
        for (int a = 0; a < 3; ++a) un = un + double(nrm[a]) * qh.v[1 + a];
        const T lam = re(un) > 0.0 ? un : T(0.0);
        const Mom<T>& qb = B->cur[n];
        Mom<T> q;
        for (int m = 0; m < kMom; ++m) q.v[m] = (qb.v[m] + lam * qh.v[m]) / (1.0 + lam);
        next[k][n] = stored(q);
      }
    }
    for (size_t k = 0; k < blocks.size(); ++k) {
      blocks[k]->prev.swap(blocks[k]->cur);
      blocks[k]->cur.swap(next[k]);
    }
  }

  // --- powder-snow volume fraction phi on the finest level (Sec. 7, powder snow):
  //     dphi/dt + u . grad phi = q + D lap phi, advected semi-Lagrangian with an RK3
  //     backtrace, then diffused with one forward-Euler step, then the source added.
  //     phi lives on the finest level's owned nodes: values outside its blocks, at its
  //     ghost nodes (the coarser level's region), beyond walls and at solid nodes are
  //     0, velocities there 0; periodic axes wrap.
  static bool off_scalar(uint8_t r) { return r == R_SOLID || r == R_GHOST; }
  static constexpr double kReach = 7.0;  // departure search range, nodes per axis
  double phi_node(const int g0[3]) {
    int g[3] = {g0[0], g0[1], g0[2]};
    if (!wrap_node(0, g)) return 0.0;
    int node;
    Blk<T>* B = locate(0, g, node);
    if (!B || B->phi.empty() || off_scalar(B->role[node])) return 0.0;
    return B->phi[node];
  }
  void u_node(const int g0[3], double u[3]) {
    int g[3] = {g0[0], g0[1], g0[2]};
    u[0] = u[1] = u[2] = 0.0;
    if (!wrap_node(0, g)) return;
    int node;
    Blk<T>* B = locate(0, g, node);
    if (!B || off_scalar(B->role[node])) return;
    for (int a = 0; a < 3; ++a) u[a] = re(B->cur[node].v[1 + a]);
  }
  // trilinear interpolation at a point x (finest-level node units)
  template <class F> void trilinear(const double x[3], int ncomp, F value, double* out) {
    int i0[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
      const double f = std::floor(x[a]);
      i0[a] = int(f);
      w[a] = x[a] - f;
    }
    for (int c = 0; c < ncomp; ++c) out[c] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
          const int g[3] = {i0[0] + dx, i0[1] + dy, i0[2] + dz};
          double v[3];
          value(g, v);
          for (int c = 0; c < ncomp; ++c) out[c] += wt * v[c];
        }
  }
  void scalar_advance(double dt, double D, const double* source /* [nb][512] key order or null */) {
    std::vector<Blk<T>*> blocks;
    for (auto& kv : lv[0]) blocks.push_back(&kv.second);
    auto uval = [&](const int g[3], double* v) { u_node(g, v); };
    auto pval = [&](const int g[3], double* v) { v[0] = phi_node(g); };
    // semi-Lagrangian advection: departure point by Ralston's RK3 backwards in time
    std::vector<std::vector<double>> adv(blocks.size(), std::vector<double>(kNodes, 0.0));
#pragma omp parallel for schedule(static)
    for (long k = 0; k < long(blocks.size()); ++k) {
      Blk<T>* B = blocks[k];
      for (int n = 0; n < kNodes; ++n) {
        if (off_scalar(B->role[n])) continue;
        int g[3];
        node_coords(B->b, n, g);
        const double x[3] = {double(g[0]), double(g[1]), double(g[2])};
        // every sample point is kept within kReach nodes of x per axis (the reading
        // of the search range: the paper bounds no departure distance)
        auto reach = [&](double* y) {
          for (int a = 0; a < 3; ++a) y[a] = std::min(std::max(y[a], x[a] - kReach), x[a] + kReach);
        };
        double k1[3], k2[3], k3[3], y[3];
        trilinear(x, 3, uval, k1);
        for (int a = 0; a < 3; ++a) y[a] = x[a] - 0.5 * dt * k1[a];
        reach(y);
        trilinear(y, 3, uval, k2);
        for (int a = 0; a < 3; ++a) y[a] = x[a] - 0.75 * dt * k2[a];
        reach(y);
        trilinear(y, 3, uval, k3);
        for (int a = 0; a < 3; ++a) y[a] = x[a] - dt * (2.0 * k1[a] + 3.0 * k2[a] + 4.0 * k3[a]) / 9.0;
        reach(y);
        trilinear(y, 1, pval, &adv[k][n]);
      }
    }
    for (size_t k = 0; k < blocks.size(); ++k) blocks[k]->phi = adv[k];
    // forward-Euler diffusion (7-point Laplacian) and the source
    std::vector<std::vector<double>> out(blocks.size(), std::vector<double>(kNodes, 0.0));
#pragma omp parallel for schedule(static)
    for (long k = 0; k < long(blocks.size()); ++k) {
      Blk<T>* B = blocks[k];
      for (int n = 0; n < kNodes; ++n) {
        if (off_scalar(B->role[n])) continue;
        int g[3];
        node_coords(B->b, n, g);
        const double c = B->phi[n];
        double lap = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int sgn = -1; sgn <= 1; sgn += 2) {
            int h[3] = {g[0], g[1], g[2]};
            h[a] += sgn;
            lap += phi_node(h) - c;
          }
        out[k][n] = c + D * dt * lap + (source ? dt * source[k * kNodes + n] : 0.0);
      }
    }
    for (size_t k = 0; k < blocks.size(); ++k) blocks[k]->phi = out[k];
  }

  // Alg. 1
  void advance(int l, int s) {
    if (ops_taken != 0) throw std::runtime_error("a coarse step is under way (finest steps)");
    if (l < L - 1) downward(l, s);
    stream_collide(l);
    if (l < L - 1 && s == 2) upward(l);
    if (l > 0) { advance(l - 1, 1); advance(l - 1, 2); }
  }

  // --- finest-level steps: the coupling loop exchanges with the granular solver
  //     after every finest-level step (Sec. 5.4, Fig. pipeline; Sec. 7). The walk is
  //     the recursion of Alg. 1 for the current coarse step; an operation runs only if
  //     it is the next one not yet taken and finest steps remain to be taken. A finest
  //     step ends with the finest level's stream-collide (and, on its second substep,
  //     the upward transfer that follows it).
  long ops_taken = 0;  // operations of the current coarse step taken so far
  long ops_seen = 0;   // operations met by the current walk
  int fine_left = 0;   // finest steps this call still has to take
  bool due() {
    const bool run = fine_left > 0 && ops_seen == ops_taken;
    ++ops_seen;
    if (run) ++ops_taken;
    return run;
  }
  void walk(int l, int s) {
    if (l < L - 1 && due()) downward(l, s);
    const bool sc = due();
    if (sc) stream_collide(l);
    if (l < L - 1 && s == 2 && due()) upward(l);
    if (l == 0 && sc) --fine_left;
    if (l > 0) { walk(l - 1, 1); walk(l - 1, 2); }
  }
  void step_finest(int n) {
    fine_left = n;
    while (fine_left > 0) {
      ops_seen = 0;
      walk(L - 1, 1);
      if (ops_taken == ops_seen) ops_taken = 0;  // the coarse step is complete
    }
  }
  int finest_phase() const {
    // finest steps whose stream-collide is among the operations taken: count them by
    // walking the operation numbers of Alg. 1's recursion
    long seen = 0;
    int k = 0;
    std::function<void(int, int)> count = [&](int l, int s) {
      if (l < L - 1) ++seen;
      if (seen++ < ops_taken && l == 0) ++k;
      if (l < L - 1 && s == 2) ++seen;
      if (l > 0) { count(l - 1, 1); count(l - 1, 2); }
    };
    count(L - 1, 1);
    return k;
  }
  void need_boundary(const char* what) const {
    if (ops_taken != 0) throw std::runtime_error(std::string(what) + ": a coarse step is under way (finest steps)");
  }

  // --- grid update (Sec. 6.3) ---
  // V_old(l, g): value of level-l node g from the current (old) hierarchy: its
  // own value if owned; else the nearest finer level owning the coincident node,
  // transferred upward; else interpolated downward from level l+1.
  bool upchain(int l, const int g[3], Lin& out) {
    double sfac = 1.0;
    for (int k = l; k >= 0; --k) {
      int m[3] = {g[0] << (l - k), g[1] << (l - k), g[2] << (l - k)};
      int node;
      Blk<T>* B = locate(k, m, node);
      if (B && owned(B->role[node])) {
        out = lin_zero();
        lin_axpy(out, 1.0, lin_of(B->cur[node]), sfac);
        return true;
      }
      if (k > 0) sfac *= a_up[k - 1];
    }
    return false;
  }
  Lin sample_old(int l, const int g[3]) {
    Lin r;
    if (upchain(l, g, r)) return r;
    if (l == L - 1) throw std::runtime_error("sampler: position not covered by any level");
    int js[8][3]; double ws[8];
    int cnt = coarse_stencil(l, g, js, ws);
    Lin acc = lin_zero();
    for (int k = 0; k < cnt; ++k) lin_axpy(acc, ws[k], sample_old(l + 1, js[k]), a_down[l]);
    return acc;
  }

  // 1/2 sum rho |u|^2 over the owned nodes of one level inside the fine box [lo, hi)
  // (no conjugation: the analytic continuation used by complex-step derivatives)
  T kinetic_energy(int level, const int32_t lo[3], const int32_t hi[3]) const {
    T sum = T(0);
    for (auto& kv : lv[level])
      for (int n = 0; n < kNodes; ++n) {
        if (!owned(kv.second.role[n])) continue;
        const int g[3] = {kv.second.b[0] * kBlock + n % kBlock, kv.second.b[1] * kBlock + (n / kBlock) % kBlock,
                          kv.second.b[2] * kBlock + n / (kBlock * kBlock)};
        bool in = true;
        for (int a = 0; a < 3; ++a) {
          const int64_t f = int64_t(g[a]) << level;
          if (f < lo[a] || f >= hi[a]) in = false;
        }
        if (!in) continue;
        const Mom<T>& q = kv.second.cur[n];
        sum = sum + 0.5 * q.rho() * (q.u(0) * q.u(0) + q.u(1) * q.u(1) + q.u(2) * q.u(2));
      }
    return sum;
  }

  int remesh(const float* p, int64_t np) {
    BSet T0 = mark_T0(p, np);
    auto states = hierarchy_states(T0);
    // new blocks and their roles
    std::vector<std::map<uint64_t, Blk<T>>> nlv(L);
    auto old_st = st;
    st = states;  // roles of the new hierarchy are computed against the new states
    for (int l = 0; l < L; ++l)
      for (auto& kv : states[l]) {
        if (kv.second != ST_ACTIVE) continue;
        Blk<T>& B = nlv[l][kv.first];
        B.lvl = l; B.key = kv.first; demorton3(kv.first, B.b);
        assign_roles(B);
      }
    std::vector<std::map<uint64_t, uint8_t>> new_st = states;
    st = old_st;  // the sampler reads the old hierarchy
    std::vector<std::vector<Blk<T>*>> work(L);
    for (int l = 0; l < L; ++l)
      for (auto& kv : nlv[l]) work[l].push_back(&kv.second);
    std::string local_err;
    for (int l = 0; l < L; ++l) {
#pragma omp parallel for schedule(static)
      for (long k = 0; k < long(work[l].size()); ++k) {
        Blk<T>* B = work[l][k];
        Blk<T>* O = find_block(l, B->b);
        B->cur.assign(kNodes, rest_state());
        // coupling fields and phi stay with blocks that remain; new blocks start at
        // eps = 1, F = 0, phi = 0
        if (O) {
          B->cpl = O->cpl;
          B->phi = O->phi;
        }
        for (int n = 0; n < kNodes; ++n) {
          uint8_t r = B->role[n];
          bool fresh = (O == nullptr) || (!owned(O->role[n]) && owned(r));
          if (!fresh) { B->cur[n] = O->cur[n]; continue; }
          if (r == R_SOLID) { B->cur[n] = rest_state(); continue; }
          int g[3];
          node_coords(B->b, n, g);
          if (r == R_INFLOW) { B->cur[n] = stored(inflow_state(l, g)); continue; }
          try {
            B->cur[n] = stored(mom_of(sample_old(l, g)));
          } catch (const std::exception& e) {
#pragma omp critical
            local_err = e.what();
          }
        }
        B->prev = B->cur;
      }
    }
    if (!local_err.empty()) throw std::runtime_error(local_err);
    lv.swap(nlv);
    st = new_st;
    for (int l = 0; l < L; ++l) link_level(l);
    return 0;
  }
};

void validate(const oc_config& c) {
  if (c.levels < 1 || c.levels > 5) throw std::runtime_error("levels must be in 1..5");
  for (int a = 0; a < 3; ++a) {
    int unit = kBlock << (c.levels - 1);
    if (c.n[a] <= 0 || c.n[a] % unit != 0) throw std::runtime_error("extent must be a positive multiple of 8*2^(L-1)");
    bool p0 = c.bc[2 * a] == BC_PERIODIC, p1 = c.bc[2 * a + 1] == BC_PERIODIC;
    if (p0 != p1) throw std::runtime_error("periodic faces must come in pairs");
  }
  for (int f = 0; f < 6; ++f)
    if (c.bc[f] < 0 || c.bc[f] > 4) throw std::runtime_error("bad boundary kind");
  if (c.inflow_profile < 0 || c.inflow_profile > 1) throw std::runtime_error("bad inflow profile");
  if (c.inflow_profile == 1 && (c.inflow_axis < 0 || c.inflow_axis > 2 || !(c.inflow_beta >= 0.0)))
    throw std::runtime_error("bad log inflow profile");
  if (!(c.tau0 > 0.5)) throw std::runtime_error("tau0 must exceed 1/2");
  if (c.storage < 0 || c.storage > 2) throw std::runtime_error("bad storage emulation");
  if (c.storage != 0)
    for (int m = 0; m < kMom; ++m)
      if (!(c.scale[m] > 0.0)) throw std::runtime_error("storage scales must be positive");
}

template <class T> Sim<T>* create(const oc_config* cfg, const uint8_t* solid, const float* p, int64_t np) {
  validate(*cfg);
  auto* s = new Sim<T>();
  s->cfg = *cfg;
  s->L = cfg->levels;
  for (int a = 0; a < 3; ++a) s->N[a] = cfg->n[a];
  s->setup_levels();
  if (solid) s->solid.assign(solid, solid + size_t(cfg->n[0]) * cfg->n[1] * cfg->n[2]);
  auto T0 = s->mark_T0(p, p ? np : 0);
  s->build(s->hierarchy_states(T0));
  // static nodes start at their fixed states
  for (int l = 0; l < s->L; ++l)
    for (auto& kv : s->lv[l])
      for (int n = 0; n < kNodes; ++n) {
        if (kv.second.role[n] == R_INFLOW) {
          int g[3];
          s->node_coords(kv.second.b, n, g);
          kv.second.cur[n] = s->stored(s->inflow_state(l, g));
        }
        kv.second.prev[n] = kv.second.cur[n];
      }
  return s;
}

thread_local std::string g_err;

}  // namespace

// ---------------------------------------------------------------------------
// C interface (ctypes). Moment arrays use the layout [block][moment][node] with
// moments (rho-1, ux, uy, uz, Sxx, Syy, Szz, Sxy, Sxz, Syz) and node index
// x + 8y + 64z; blocks are listed in increasing Morton order of their block
// coordinates (x in the lowest bit).
extern "C" {

typedef Sim<double> OSim;

const char* oc_last_error() { return g_err.c_str(); }

void* oc_create(const oc_config* cfg, const uint8_t* solid, const float* particles, int64_t np) {
  try { return create<double>(cfg, solid, particles, np); }
  catch (const std::exception& e) { g_err = e.what(); return nullptr; }
}
void oc_destroy(void* h) { delete static_cast<OSim*>(h); }

int64_t oc_num_blocks(void* h, int level) {
  auto* s = static_cast<OSim*>(h);
  if (level < 0 || level >= s->L) return -1;
  return int64_t(s->lv[level].size());
}
void oc_block_keys(void* h, int level, int64_t* keys) {
  auto* s = static_cast<OSim*>(h);
  int64_t k = 0;
  for (auto& kv : s->lv[level]) keys[k++] = int64_t(kv.first);
}
int oc_set_block_moments(void* h, int level, const int64_t* keys, const double* in, int64_t nb) {
  auto* s = static_cast<OSim*>(h);
  for (int64_t k = 0; k < nb; ++k) {
    auto it = s->lv[level].find(uint64_t(keys[k]));
    if (it == s->lv[level].end()) { g_err = "set_block_moments: unknown block"; return -1; }
    auto& B = it->second;
    for (int n = 0; n < kNodes; ++n) {
      Mom<double> q;
      for (int m = 0; m < kMom; ++m) q.v[m] = in[(k * kMom + m) * kNodes + n];
      q.v[0] += 1.0;
      if (B.role[n] == R_SOLID) q = s->rest_state();
      if (B.role[n] == R_INFLOW) {
        int g[3];
        s->node_coords(B.b, n, g);
        q = s->inflow_state(level, g);
      }
      q = s->stored(q);
      B.cur[n] = q;
      B.prev[n] = q;
    }
  }
  return 0;
}
// powder-snow volume fraction of the finest level: set per block, get all (key order),
// advance by dt finest-level steps with diffusivity D and a source [nb][512] (or null)
int oc_scalar_set(void* h, const int64_t* keys, const double* in, int64_t nb) {
  auto* s = static_cast<OSim*>(h);
  for (int64_t k = 0; k < nb; ++k) {
    auto it = s->lv[0].find(uint64_t(keys[k]));
    if (it == s->lv[0].end()) { g_err = "scalar_set: unknown finest-level block"; return -1; }
    it->second.phi.assign(in + size_t(k) * kNodes, in + size_t(k + 1) * kNodes);
    for (int n = 0; n < kNodes; ++n)
      if (it->second.role[n] == R_SOLID || it->second.role[n] == R_GHOST) it->second.phi[n] = 0.0;
  }
  return 0;
}
void oc_scalar_get(void* h, double* out) {
  auto* s = static_cast<OSim*>(h);
  size_t k = 0;
  for (auto& kv : s->lv[0]) {
    for (int n = 0; n < kNodes; ++n) out[k * kNodes + n] = kv.second.phi.empty() ? 0.0 : kv.second.phi[n];
    ++k;
  }
}
void oc_scalar_advance(void* h, double dt, double D, const double* source) {
  static_cast<OSim*>(h)->scalar_advance(dt, D, source);
}
// finest-level coupling fields of the given blocks: in [nb][4][512] (eps, Fx, Fy, Fz)
int oc_set_coupling(void* h, const int64_t* keys, const double* in, int64_t nb) {
  auto* s = static_cast<OSim*>(h);
  for (int64_t k = 0; k < nb; ++k) {
    auto it = s->lv[0].find(uint64_t(keys[k]));
    if (it == s->lv[0].end()) { g_err = "set_coupling: unknown finest-level block"; return -1; }
    const double* src = in + size_t(k) * 4 * kNodes;
    for (int n = 0; n < kNodes; ++n)
      if (!(src[n] * s->tau[0] > 0.5) || !std::isfinite(src[n])) { g_err = "set_coupling: eps tau0 must exceed 1/2"; return -1; }
    it->second.cpl.assign(src, src + 4 * kNodes);
  }
  return 0;
}
void oc_get_block_moments(void* h, int level, int64_t* keys, double* out) {
  auto* s = static_cast<OSim*>(h);
  int64_t k = 0;
  for (auto& kv : s->lv[level]) {
    if (keys) keys[k] = int64_t(kv.first);
    for (int n = 0; n < kNodes; ++n)
      for (int m = 0; m < kMom; ++m) {
        double v = kv.second.cur[n].v[m];
        if (m == 0) v -= 1.0;
        out[(k * kMom + m) * kNodes + n] = v;
      }
    ++k;
  }
}
void oc_get_roles(void* h, int level, uint8_t* out) {
  auto* s = static_cast<OSim*>(h);
  int64_t k = 0;
  for (auto& kv : s->lv[level]) {
    std::memcpy(out + k * kNodes, kv.second.role, kNodes);
    ++k;
  }
}
int oc_step(void* h, int n) {
  auto* s = static_cast<OSim*>(h);
  try {
    for (int i = 0; i < n; ++i) s->advance(s->L - 1, 1);
  } catch (const std::exception& e) { g_err = e.what(); return -1; }
  return 0;
}
int oc_step_finest(void* h, int n) {
  auto* s = static_cast<OSim*>(h);
  try { s->step_finest(n); }
  catch (const std::exception& e) { g_err = e.what(); return -1; }
  return 0;
}
int oc_finest_phase(void* h) { return static_cast<OSim*>(h)->finest_phase(); }
int oc_remesh(void* h, const float* particles, int64_t np) {
  auto* s = static_cast<OSim*>(h);
  try {
    s->need_boundary("remesh");
    return s->remesh(particles, np);
  }
  catch (const std::exception& e) { g_err = e.what(); return -1; }
}
double oc_loss_ke(void* h, int level, const int32_t lo[3], const int32_t hi[3]) {
  return static_cast<OSim*>(h)->kinetic_energy(level, lo, hi);
}

// ---- complex-step instance: the same templated code on std::complex<double> ----
typedef Sim<std::complex<double>> CSim;
void* occ_create(const oc_config* cfg, const uint8_t* solid, const float* particles, int64_t np) {
  try {
    if (cfg->storage != 0) throw std::runtime_error("complex-step runs need exact storage");
    return create<std::complex<double>>(cfg, solid, particles, np);
  } catch (const std::exception& e) { g_err = e.what(); return nullptr; }
}
void occ_destroy(void* h) { delete static_cast<CSim*>(h); }
int occ_set_block_moments(void* h, int level, const int64_t* keys, const double* re, const double* im, int64_t nb) {
  auto* s = static_cast<CSim*>(h);
  for (int64_t k = 0; k < nb; ++k) {
    auto it = s->lv[level].find(uint64_t(keys[k]));
    if (it == s->lv[level].end()) { g_err = "set_block_moments: unknown block"; return -1; }
    auto& B = it->second;
    for (int n = 0; n < kNodes; ++n) {
      Mom<std::complex<double>> q;
      for (int m = 0; m < kMom; ++m) {
        const size_t i = size_t((k * kMom + m) * kNodes + n);
        q.v[m] = std::complex<double>(re[i], im ? im[i] : 0.0);
      }
      q.v[0] += 1.0;
      if (B.role[n] == R_SOLID) q = s->rest_state();
      if (B.role[n] == R_INFLOW) {
        int g[3];
        s->node_coords(B.b, n, g);
        q = s->inflow_state(level, g);
      }
      B.cur[n] = q;
      B.prev[n] = q;
    }
  }
  return 0;
}
int occ_step(void* h, int n) {
  auto* s = static_cast<CSim*>(h);
  try {
    for (int i = 0; i < n; ++i) s->advance(s->L - 1, 1);
  } catch (const std::exception& e) { g_err = e.what(); return -1; }
  return 0;
}
int occ_remesh(void* h, const float* particles, int64_t np) {
  auto* s = static_cast<CSim*>(h);
  try { return s->remesh(particles, np); }
  catch (const std::exception& e) { g_err = e.what(); return -1; }
}
void occ_loss_ke(void* h, int level, const int32_t lo[3], const int32_t hi[3], double out[2]) {
  const std::complex<double> v = static_cast<CSim*>(h)->kinetic_energy(level, lo, hi);
  out[0] = v.real();
  out[1] = v.imag();
}

// FP32 particle advance p += d (no contraction), as the GPU path does it.
void oc_advance_particles(float* p, int64_t np, const float d[3]) {
  for (int64_t i = 0; i < np; ++i)
    for (int a = 0; a < 3; ++a) {
      volatile float s = p[3 * i + a] + d[a];
      p[3 * i + a] = s;
    }
}
// Sums over owned nodes of one level inside the fine-unit box [lo, hi):
// out = {sum rho, sum rho ux, sum rho uy, sum rho uz, 1/2 sum rho |u|^2}.
void oc_reduce(void* h, int level, const int32_t lo[3], const int32_t hi[3], double out[5]) {
  auto* s = static_cast<OSim*>(h);
  for (int k = 0; k < 5; ++k) out[k] = 0.0;
  for (auto& kv : s->lv[level])
    for (int n = 0; n < kNodes; ++n) {
      uint8_t r = kv.second.role[n];
      if (!OSim::owned(r)) continue;
      int g[3] = {kv.second.b[0] * kBlock + n % kBlock, kv.second.b[1] * kBlock + (n / kBlock) % kBlock, kv.second.b[2] * kBlock + n / (kBlock * kBlock)};
      bool in = true;
      for (int a = 0; a < 3; ++a) {
        int64_t f = int64_t(g[a]) << level;
        if (f < lo[a] || f >= hi[a]) in = false;
      }
      if (!in) continue;
      const auto& q = kv.second.cur[n];
      double rho = q.v[0];
      out[0] += rho;
      double ke = 0.0;
      for (int a = 0; a < 3; ++a) { out[1 + a] += rho * q.v[1 + a]; ke += q.v[1 + a] * q.v[1 + a]; }
      out[4] += 0.5 * rho * ke;
    }
}
void oc_level_params(void* h, double* tau, double* a_up, double* a_down) {
  auto* s = static_cast<OSim*>(h);
  for (int l = 0; l < s->L; ++l) { tau[l] = s->tau[l]; a_up[l] = s->a_up[l]; a_down[l] = s->a_down[l]; }
}

double oc_store_round(double v, int storage, double scale) { return store_round(v, storage, scale); }

int oc_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void oc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// Single-node pieces, exposed for the pinning tests.
void oc_lattice(int32_t* c, double* w) {
  for (int i = 0; i < 27; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = LAT.c[i][a];
    w[i] = LAT.w[i];
  }
}
// moments (rho, u, S) in stored order -> 27 populations
void oc_reconstruct(const double* q, double* f) {
  Mom<double> p;
  for (int m = 0; m < kMom; ++m) p.v[m] = q[m];
  for (int i = 0; i < 27; ++i) f[i] = reconstruct(p, i);
}
void oc_collide(const double* q, double omega, const double F[3], double* out) {
  Mom<double> p;
  for (int m = 0; m < kMom; ++m) p.v[m] = q[m];
  Mom<double> r = collide(p, omega, F);
  for (int m = 0; m < kMom; ++m) out[m] = r.v[m];
}
}
