// lbm_d2q9.hip -- gfx950 kernels of the D2Q9 phase-field lattice Boltzmann
// step (Li, Luo & Gao, arXiv:1110.5004).
//
// One fused kernel performs a whole time step for a tile of TX x TY nodes:
//   A  pull f from the stored (post-collision) populations and sum phi over
//      the tile plus a halo of R = 3 (corrected model) or 2 nodes; phi -> LDS
//   B  isotropic Laplacian -> mu = theta'(phi) - kappa lap phi (Eq. 1a and
//      the definition of mu) over the tile plus R - 1; mu -> LDS
//   C  over the tile plus 1: grad phi, lap mu (corrected model), pull gbar,
//      recover u and p with F_s = mu grad phi, G and -F_a (Eq. 5, Eq. 12 and
//      the paragraph after it); u, p -> LDS
//   D  over the tile: grad p -> grad psi, BGK collision of f (order
//      parameter) and of gbar with the forcing of Eq. 8, store.
// With the correction from data (RF = 2) phase C first forms the uncorrected
// rho u over the tile plus 2, then the rate (rho^n - rho^(n-1)) + div(rho u)
// over the tile plus 1 as the coefficient of -F_a; phi^(n-1) comes from a
// plane that every state copy carries.
// Stencil positions beyond a wall hold the values of their mirror node
// (halfway bounce-back walls, neutral wetting); positions beyond a periodic
// seam hold the wrapped node.  Every per-node quantity is a function of the
// state only, so a halo position computes exactly what its owner tile does.
//
// Populations are stored post-collision in SoA planes and pulled (x - e_i)
// when read, so a tile reads populations of its own nodes and of a halo and
// writes only its own nodes (no write conflicts between workgroups).
#include "lbm_dev.h"
#include "lbm_kernels.h"
#include "lbm_lattice.h"

namespace lbm {
namespace d2q9 {


// Differences of a float-float LDS field (hi, lo arrays, row pitch P):
// hi differences of close values are exact, so the stencils below see phi to
// the precision of the stored state.
template <int P>
struct FF {
  const float* h;
  const float* l;
  __device__ __forceinline__ float d(int a, int b) const { return (h[a] - h[b]) + (l[a] - l[b]); }
};

// Isotropic central gradient (3 sum w_i e_i phi_i) of a float-float field.
template <int P>
__device__ __forceinline__ void grad_ff(const FF<P>& f, int c, float& gx, float& gy) {
  gx = (1.0f / 3.0f) * f.d(c + 1, c - 1) +
       (1.0f / 12.0f) * (f.d(c + P + 1, c + P - 1) + f.d(c - P + 1, c - P - 1));
  gy = (1.0f / 3.0f) * f.d(c + P, c - P) +
       (1.0f / 12.0f) * (f.d(c + P + 1, c - P + 1) + f.d(c + P - 1, c - P - 1));
}

// Isotropic Laplacian 6 sum_i w_i (phi_i - phi) of a float-float field.
template <int P>
__device__ __forceinline__ float lap_ff(const FF<P>& f, int c) {
  return (2.0f / 3.0f) * ((f.d(c + 1, c) + f.d(c + P, c)) + (f.d(c - 1, c) + f.d(c - P, c))) +
         (1.0f / 6.0f) * ((f.d(c + P + 1, c) + f.d(c + P - 1, c)) +
                          (f.d(c - P - 1, c) + f.d(c - P + 1, c)));
}

// The same stencils on a plain float LDS array (mu and p).
template <int P>
__device__ __forceinline__ float lap_only(const float* s, int cx, int cy) {
  const float* r0 = s + cy * P + cx;
  const float c = r0[0];
  return (2.0f / 3.0f) * (((r0[1] - c) + (r0[P] - c)) + ((r0[-1] - c) + (r0[-P] - c))) +
         (1.0f / 6.0f) * (((r0[P + 1] - c) + (r0[P - 1] - c)) + ((r0[-P - 1] - c) + (r0[-P + 1] - c)));
}

template <int P>
__device__ __forceinline__ void grad_only(const float* s, int cx, int cy, float& gx, float& gy) {
  const float* r0 = s + cy * P + cx;
  const float e = r0[1], w = r0[-1], n = r0[P], so = r0[-P];
  const float ne = r0[P + 1], nw = r0[P - 1], sw = r0[-P - 1], se = r0[-P + 1];
  gx = (1.0f / 3.0f) * (e - w) + (1.0f / 12.0f) * ((ne - nw) + (se - sw));
  gy = (1.0f / 3.0f) * (n - so) + (1.0f / 12.0f) * ((ne - se) + (nw - sw));
}

// Velocity, total force and pressure from the moments of gbar:
//   (rho - c/2) u = 3 sum e gbar + (F_s + G)/2,   F = F_s + G + c u,
//   p = sum gbar + (1/6) drho u . grad phi        (u . grad p dropped),
// with cc the coefficient of the cancelled -F_a = c u: drho theta_M lap mu
// (Eq. 5), the rate D taken from the data, or 0 (original model).
__device__ __forceinline__ void recover(const CaseDev& c, float phi, float gx, float gy, float mu,
                                        float cc, float m0, float m1x, float m1y, float& ux,
                                        float& uy, float& p) {
  const float rho = c.rho0 + phi * c.drho;
  const float fsx = mu * gx;
  const float fsy = mu * gy - (rho - c.rho_ref) * c.gravity;
  const float iden = __builtin_amdgcn_rcpf(rho - 0.5f * cc);
  ux = (3.0f * m1x + 0.5f * fsx) * iden;
  uy = (3.0f * m1y + 0.5f * fsy) * iden;
  p = m0 + (1.0f / 6.0f) * c.drho * (ux * gx + uy * gy);
}

// Stored word of f_i (i > 0) and of g_i: a float, or 16 bits.
template <int S>
using Raw = typename std::conditional<S == ST_FP32, float, uint16_t>::type;

// Interior tiles: per-direction uniform base pointers already shifted by
// -e_i, so that every pulled population of node idx is base_i[idx] and all
// loads of a node share one per-lane offset.
template <int S>
struct InnerPtrs {
  const char* f[Q];  // f_i pulled (f_0: own node)
  const char* g[Q];
  const char* f0lo;
  __device__ __forceinline__ InnerPtrs(const CaseDev& c, const char* src) {
    using P = Pops<S, Q>;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int sh = EX(i) + c.nx * EY(i);
      const int fw = (S == ST_FP32 || i == 0) ? 4 : 2;
      const int gw = S == ST_FP32 ? 4 : 2;
      f[i] = src + P::fofs(c, i, 0) - (long)sh * fw;
      g[i] = src + P::gofs(c, i, 0) - (long)sh * gw;
    }
    f0lo = src + (size_t)(2 * Q) * 4 * c.stride;
  }
};

// A load coordinate g of a tile or its halo mapped into the grid: the
// periodic image or the wall mirror, then clamped.  Every position a real
// node reads lies at most R + 1 <= 4 <= n outside the grid, where one fold is
// exact; positions farther out occur only in the unused part of a ragged
// tile, where the clamp keeps the load in bounds.
__device__ __forceinline__ int fold_axis(int g, int n, int wall) {
  if (g < 0) g = wall ? -g - 1 : g + n;
  else if (g >= n) g = wall ? 2 * n - 1 - g : g - n;
  return min(max(g, 0), n - 1);
}

// Near the boundary: byte offset of f_i (G = false) or g_i pulled by the
// in-grid node idx, whose position is flagged at the grid's edges (x0: x = 0,
// x1: x = nx - 1, y0, y1 likewise).  The source is the neighbour x - e_i,
// wrapped across a periodic seam, or (across a wall) the node itself in the
// opposite direction.  e_i is a compile-time constant, so each axis takes one
// flag and the offset is formed without branches.
template <int S, bool G>
__device__ __forceinline__ unsigned edge_ofs(const CaseDev& c, unsigned idx, bool x0, bool x1,
                                             bool y0, bool y1, int i) {
  using P = Pops<S, Q>;
  if (i == 0) return G ? P::gofs(c, 0, idx) : P::fofs(c, 0, idx);
  const int ex = EX(i), ey = EY(i);
  const bool hx = ex > 0 ? x0 : (ex < 0 ? x1 : false);  // x - e_x leaves the grid
  const bool hy = ey > 0 ? y0 : (ey < 0 ? y1 : false);
  const bool bb = (hx && c.wall_x) || (hy && c.wall_y);
  const int nxy = c.nx * c.ny;
  int j = (int)idx - ex - c.nx * ey;
  j += (hx && !c.wall_x) ? (ex > 0 ? c.nx : -c.nx) : 0;
  j += (hy && !c.wall_y) ? (ey > 0 ? nxy : -nxy) : 0;
  const unsigned own = G ? P::gofs(c, OPP(i), idx) : P::fofs(c, OPP(i), idx);
  const unsigned pulled = G ? P::gofs(c, i, (unsigned)j) : P::fofs(c, i, (unsigned)j);
  return bb ? own : pulled;
}

// Raw loads of the populations a node pulls.  FV: f_0, its low part and
// f_1..f_8; GV: gbar_0..gbar_8.
template <int S, bool INNER>
struct Puller {
  const CaseDev& c;
  const char* src;
  InnerPtrs<S> ip;
  __device__ __forceinline__ Puller(const CaseDev& cc, const char* s) : c(cc), src(s), ip(cc, s) {}
  // node index of an in-grid position (sides < 2^24, checked at set-up)
  __device__ __forceinline__ unsigned node(int x, int y) const {
    return (unsigned)x + __umul24((unsigned)c.nx, (unsigned)y);
  }
  __device__ __forceinline__ void fpop(int x, int y, float& f0, uint16_t& lo, Raw<S>* fr) const {
    using P = Pops<S, Q>;
    const unsigned idx = node(x, y);
    constexpr unsigned W = sizeof(Raw<S>);
    const bool x0 = x == 0, x1 = x == c.nx - 1, y0 = y == 0, y1 = y == c.ny - 1;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if constexpr (INNER) fr[i] = gload<Raw<S>>(ip.f[i], W * idx);
      else fr[i] = gload<Raw<S>>(src, edge_ofs<S, false>(c, idx, x0, x1, y0, y1, i));
    }
    f0 = INNER ? gload<float>(ip.f[0], 4u * idx) : gload<float>(src, P::fofs(c, 0, idx));
    if constexpr (S == ST_FP32) lo = gload<uint16_t>(ip.f0lo, 2u * idx);
    else lo = 0;
  }
  __device__ __forceinline__ void gpop(int x, int y, Raw<S>* gr) const {
    const unsigned idx = node(x, y);
    constexpr unsigned W = sizeof(Raw<S>);
    const bool x0 = x == 0, x1 = x == c.nx - 1, y0 = y == 0, y1 = y == c.ny - 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if constexpr (INNER) gr[i] = gload<Raw<S>>(ip.g[i], W * idx);
      else gr[i] = gload<Raw<S>>(src, edge_ofs<S, true>(c, idx, x0, x1, y0, y1, i));
    }
  }
};

// phi = f_0 + sum_{i>0} f_i as hi + lo, from raw pulled words.
template <int S>
__device__ __forceinline__ void phi_sum(const CaseDev& c, float f0, uint16_t lo,
                                        const Raw<S>* fr, float* fv, float& hi, float& plo) {
  using P = Pops<S, Q>;
  float sm = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    fv[i] = P::dec_f(c, fr[i]);
    sm += fv[i];
  }
  two_sum(f0, P::dec_lo(lo) + sm, hi, plo);
}

// Zeroth and first moments of gbar from raw pulled words.
template <int S>
__device__ __forceinline__ void g_sum(const CaseDev& c, const Raw<S>* gr, float* gv, float& m0,
                                      float& m1x, float& m1y) {
  using P = Pops<S, Q>;
  m0 = m1x = m1y = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float v = P::dec_g(c, gr[i], WT(i));
    gv[i] = v;
    m0 += v;
    if (EX(i)) m1x += EX(i) > 0 ? v : -v;
    if (EY(i)) m1y += EY(i) > 0 ? v : -v;
  }
}

// The own nodes' pulled populations between the loads and the collision.
// FP32 storage: decoded floats.  16-bit storage: the stored words, two per
// register, decoded where the collision reads them (the same decode, hence the
// same values); this halves the registers they occupy through phases B and C.
template <int S, int NPT, bool WIDE = (S == ST_FP32)>
struct OwnPops;

template <int S, int NPT>
struct OwnPops<S, NPT, true> {
  float fv[NPT][Q], gv[NPT][Q];
  __device__ __forceinline__ void set(int j, const float* f, const float* g, const Raw<S>*,
                                      const Raw<S>*) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      fv[j][i] = f[i];
      gv[j][i] = g[i];
    }
  }
  __device__ __forceinline__ float f(const CaseDev&, int j, int i) const { return fv[j][i]; }
  __device__ __forceinline__ float g(const CaseDev&, int j, int i, float) const {
    return gv[j][i];
  }
};

template <int S, int NPT>
struct OwnPops<S, NPT, false> {
  uint32_t fp[NPT][(Q - 1 + 1) / 2];  // f_1 | f_2 << 16, f_3 | f_4 << 16, ...
  uint32_t gp[NPT][(Q + 1) / 2];      // g_0 | g_1 << 16, ..., g_8
  __device__ __forceinline__ void set(int j, const float*, const float*, const Raw<S>* fr,
                                      const Raw<S>* gr) {
#pragma unroll
    for (int m = 0; m < (Q - 1 + 1) / 2; ++m) {
      const int a = 2 * m + 1, b = 2 * m + 2;
      fp[j][m] = (uint32_t)fr[a] | (b < Q ? (uint32_t)fr[b] << 16 : 0u);
    }
#pragma unroll
    for (int m = 0; m < (Q + 1) / 2; ++m) {
      const int a = 2 * m, b = 2 * m + 1;
      gp[j][m] = (uint32_t)gr[a] | (b < Q ? (uint32_t)gr[b] << 16 : 0u);
    }
  }
  __device__ __forceinline__ float f(const CaseDev& c, int j, int i) const {
    const uint32_t w = fp[j][(i - 1) >> 1];
    return Pops<S, Q>::dec_f(c, (uint16_t)((i - 1) & 1 ? w >> 16 : w & 0xffffu));
  }
  __device__ __forceinline__ float g(const CaseDev& c, int j, int i, float wi) const {
    const uint32_t w = gp[j][i >> 1];
    return Pops<S, Q>::dec_g(c, (uint16_t)(i & 1 ? w >> 16 : w & 0xffffu), wi);
  }
};

struct FieldOut {
  float* phi;
  float* ux;
  float* uy;
  float* uz;
  float* p;
  float* mu;
  float* fax;
  float* fay;
  float* faz;
};

// LDS of one tile.  RF = 0: original model; 1: lap mu formed (Eq. 5
// correction, or the F_a dump); 2: correction from data.
template <int TX, int TY, int RF>
struct TileLds {
  static constexpr int R = RF ? 3 : 2;   // phi radius
  static constexpr int RM = R - 1;       // mu radius
  static constexpr int MR = 1;           // radius of the gbar moments
  static constexpr int PW = TX + 2 * R, PH = TY + 2 * R;
  static constexpr int MW = TX + 2 * RM, MH = TY + 2 * RM;
  static constexpr int UW = TX + 2, UH = TY + 2;
  static constexpr int VW = UW, VH = UH;  // moment region
  float ph[PW * PH];  // phi = ph + pl
  float pl[PW * PH];
  float mu[MW * MH];
  float ux[UW * UH];  // first moments of gbar, then u
  float uy[UW * UH];
  float p[UW * UH];   // zeroth moment of gbar, then p
  float gx[TX * TY];  // grad phi and lap mu of the tile nodes, kept from C for D
  float gy[TX * TY];
  float lm[TX * TY];
  __device__ __forceinline__ float* m0() { return p; }
  __device__ __forceinline__ float* m1x() { return ux; }
  __device__ __forceinline__ float* m1y() { return uy; }
};

// RF = 2: the rate D = (rho^n - rho^(n-1)) + div(rho u_o) is needed at the
// tile + 1, so u_o (the uncorrected velocity) at the tile + 2 and the gbar
// moments there; phi^(n-1) at the tile + 1.
template <int TX, int TY>
struct TileLds<TX, TY, 2> {
  static constexpr int R = 3, RM = 2, MR = 2;
  static constexpr int PW = TX + 2 * R, PH = TY + 2 * R;
  static constexpr int MW = TX + 2 * RM, MH = TY + 2 * RM;
  static constexpr int UW = TX + 2, UH = TY + 2;
  static constexpr int VW = TX + 2 * MR, VH = TY + 2 * MR;
  float ph[PW * PH];
  float pl[PW * PH];
  float mu[MW * MH];
  float g0[VW * VH];  // moments of gbar over the tile + 2
  float g1x[VW * VH];
  float g1y[VW * VH];
  float qx[VW * VH];  // rho u_o over the tile + 2
  float qy[VW * VH];
  float pv[UW * UH];  // phi^(n-1) over the tile + 1
  float ux[UW * UH];  // u, p over the tile + 1
  float uy[UW * UH];
  float p[UW * UH];
  float gx[TX * TY];  // grad phi and D of the tile nodes, kept from C for D
  float gy[TX * TY];
  float lm[TX * TY];
  __device__ __forceinline__ float* m0() { return g0; }
  __device__ __forceinline__ float* m1x() { return g1x; }
  __device__ __forceinline__ float* m1y() { return g1y; }
};

// Position k of the ring of width r around a TX x TY tile inside a region
// of width W = TX + 2r: first the r rows above, then the r rows below, then
// the r columns on each side of the tile rows.
template <int TX, int TY, int r>
__device__ __forceinline__ void ring_pos(int k, int& lx, int& ly) {
  constexpr int W = TX + 2 * r;
  if (k < 2 * r * W) {
    const int row = k / W;
    lx = k - row * W;
    ly = row < r ? row : TY + row;
  } else {
    const int s = k - 2 * r * W;
    const int row = s / (2 * r);
    const int col = s - row * 2 * r;
    ly = r + row;
    lx = col < r ? col : TX + col;
  }
}

// threadIdx.x behind an empty asm: values derived from it are recomputed per
// tile instead of being hoisted out of a workgroup's tile loop, where dozens
// of per-thread LDS offsets would stay live (and spill) across all phases.
__device__ __forceinline__ int tile_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Everything one tile loads from global memory, held in registers as stored
// words between issue (loads in flight) and consume (sums into LDS).  One
// tile has NT = TX * TY / NPT threads; node j of a thread is tile position
// tid + j NT.  Rings around the tile: phi at radius R (f pulled) and the
// gbar moments at radius 1.
template <int TX, int TY, int NPT, int RF, int S>
struct TileLoads {
  using T = TileLds<TX, TY, RF>;
  static constexpr int NT = TX * TY / NPT;
  static constexpr int R = T::R;
  static constexpr int MR = T::MR;
  static constexpr int NRA = T::PW * T::PH - TX * TY;  // phi ring
  static constexpr int NRC = T::VW * T::VH - TX * TY;  // moment ring
  static constexpr int NPV = RF == 2 ? T::UW * T::UH : 0;  // phi^(n-1), tile + 1
  static constexpr int IA = (NRA + NT - 1) / NT;
  static constexpr int IC = (NRC + NT - 1) / NT;
  static constexpr int IP = (NPV + NT - 1) / NT;
  float f0[NPT];
  uint16_t lo[NPT];
  Raw<S> fr[NPT][Q];
  Raw<S> gr[NPT][Q];
  float af0[IA];
  uint16_t alo[IA];
  Raw<S> afr[IA][Q];
  Raw<S> cgr[IC][Q];
  float pvr[IP > 0 ? IP : 1];
  int tid = tile_tid();

  // Loads of one element: own node j, phi-ring slot it, moment-ring slot it.
  template <bool INNER>
  __device__ __forceinline__ void issue_own(const Puller<S, INNER>& pu, int x0, int y0, int j) {
    const int kk = tid + j * NT;
    int mx = x0 + kk % TX, my = y0 + kk / TX;
    if constexpr (!INNER) {
      mx = fold_axis(mx, pu.c.nx, pu.c.wall_x);
      my = fold_axis(my, pu.c.ny, pu.c.wall_y);
    }
    pu.fpop(mx, my, f0[j], lo[j], fr[j]);
    pu.gpop(mx, my, gr[j]);
  }
  template <bool INNER>
  __device__ __forceinline__ void issue_phi(const Puller<S, INNER>& pu, int x0, int y0, int it) {
    const int k = tid + it * NT;
    if (k < NRA) {
      int lx, ly;
      ring_pos<TX, TY, R>(k, lx, ly);
      int gx = x0 - R + lx, gy = y0 - R + ly;
      if constexpr (!INNER) {
        gx = fold_axis(gx, pu.c.nx, pu.c.wall_x);
        gy = fold_axis(gy, pu.c.ny, pu.c.wall_y);
      }
      pu.fpop(gx, gy, af0[it], alo[it], afr[it]);
    }
  }
  template <bool INNER>
  __device__ __forceinline__ void issue_mom(const Puller<S, INNER>& pu, int x0, int y0, int it) {
    const int k = tid + it * NT;
    if (k < NRC) {
      int lx, ly;
      ring_pos<TX, TY, MR>(k, lx, ly);
      int gx = x0 - MR + lx, gy = y0 - MR + ly;
      if constexpr (!INNER) {
        gx = fold_axis(gx, pu.c.nx, pu.c.wall_x);
        gy = fold_axis(gy, pu.c.ny, pu.c.wall_y);
      }
      pu.gpop(gx, gy, cgr[it]);
    }
  }
  // phi^(n-1) at position k of the tile + 1 (the mirror node beyond a wall)
  template <bool INNER>
  __device__ __forceinline__ void issue_pv(const Puller<S, INNER>& pu, int x0, int y0, int it) {
    const int k = tid + it * NT;
    if (k < NPV) {
      int gx = x0 - 1 + k % T::UW, gy = y0 - 1 + k / T::UW;
      if constexpr (!INNER) {
        gx = fold_axis(gx, pu.c.nx, pu.c.wall_x);
        gy = fold_axis(gy, pu.c.ny, pu.c.wall_y);
      }
      pvr[it] = gload<float>(pu.src, pu.c.phiv + 4u * pu.node(gx, gy));
    }
  }

  // Sums of one element into LDS; own nodes also keep their decoded
  // populations in fv, gv.
  __device__ __forceinline__ void consume_own(const CaseDev& c, T& L, int j,
                                              OwnPops<S, NPT>& own) const {
    const int kk = tid + j * NT;
    const int lx0 = kk % TX, ly0 = kk / TX;
    float fv[Q], gv[Q];
    float hi, plo;
    phi_sum<S>(c, f0[j], lo[j], fr[j], fv, hi, plo);
    const int pk = (ly0 + R) * T::PW + (lx0 + R);
    L.ph[pk] = hi;
    L.pl[pk] = plo;
    float m0, m1x, m1y;
    g_sum<S>(c, gr[j], gv, m0, m1x, m1y);
    const int uk = (ly0 + MR) * T::VW + (lx0 + MR);
    L.m0()[uk] = m0;
    L.m1x()[uk] = m1x;
    L.m1y()[uk] = m1y;
    own.set(j, fv, gv, fr[j], gr[j]);
  }
  __device__ __forceinline__ void consume_phi(const CaseDev& c, T& L, int it) const {
    const int k = tid + it * NT;
    if (k < NRA) {
      int lx, ly;
      ring_pos<TX, TY, R>(k, lx, ly);
      float tmp[Q], hi, plo;
      phi_sum<S>(c, af0[it], alo[it], afr[it], tmp, hi, plo);
      L.ph[ly * T::PW + lx] = hi;
      L.pl[ly * T::PW + lx] = plo;
    }
  }
  __device__ __forceinline__ void consume_mom(const CaseDev& c, T& L, int it) const {
    const int k = tid + it * NT;
    if (k < NRC) {
      int lx, ly;
      ring_pos<TX, TY, MR>(k, lx, ly);
      float tmp[Q], m0, m1x, m1y;
      g_sum<S>(c, cgr[it], tmp, m0, m1x, m1y);
      L.m0()[ly * T::VW + lx] = m0;
      L.m1x()[ly * T::VW + lx] = m1x;
      L.m1y()[ly * T::VW + lx] = m1y;
    }
  }
  __device__ __forceinline__ void consume_pv(T& L, int it) const {
    if constexpr (RF == 2) {
      const int k = tid + it * NT;
      if (k < NPV) L.pv[k] = pvr[it];
    }
  }

  // Each element loaded and summed in turn (the compiler hoists loads as
  // far as registers allow).
  template <bool INNER>
  __device__ __forceinline__ void load_all(const CaseDev& c, const char* src, int x0, int y0,
                                           T& L, OwnPops<S, NPT>& own) {
    const Puller<S, INNER> pu(c, src);
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      issue_own<INNER>(pu, x0, y0, j);
      consume_own(c, L, j, own);
    }
#pragma unroll
    for (int it = 0; it < IA; ++it) {
      issue_phi<INNER>(pu, x0, y0, it);
      consume_phi(c, L, it);
    }
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      issue_mom<INNER>(pu, x0, y0, it);
      consume_mom(c, L, it);
    }
#pragma unroll
    for (int it = 0; it < IP; ++it) {
      issue_pv<INNER>(pu, x0, y0, it);
      consume_pv(L, it);
    }
  }
};

// Phases B, C and D of one tile whose phi and gbar moments are in LDS (and
// a barrier has passed since they were written); fv, gv hold the own nodes'
// pulled populations.  Ends with a barrier, after which LDS is free.
// INNER: every pulled population of the phi region lies inside the grid (no
// wrap, no wall), so no position needs mirroring.
template <int TX, int TY, int NPT, int RF, int S, bool FIELDS, bool INNER>
__device__ __forceinline__ void tile_bcd(TileLds<TX, TY, RF>& L, const CaseDev& c, int x0, int y0,
                                         char* dst, const FieldOut& fo,
                                         const OwnPops<S, NPT>& own, uint32_t skey) {
  using T = TileLds<TX, TY, RF>;
  constexpr int NT = TX * TY / NPT;
  constexpr int R = T::R, RM = T::RM;
  constexpr int PW = T::PW, MW = T::MW, MH = T::MH, UW = T::UW, UH = T::UH;
  constexpr int IB = (MW * MH + NT - 1) / NT;
  constexpr int ICC = (UW * UH + NT - 1) / NT;
  const FF<PW> phi{L.ph, L.pl};
  const int tid = tile_tid();
  const int nx = c.nx, ny = c.ny;
  const OutPtrs<S, Q> op(c, dst);

  // ---- B: mu over the tile + RM
#pragma unroll
  for (int it = 0; it < IB; ++it) {
    const int k = tid + it * NT;
    if (k < MW * MH) {
      int lx = k % MW, ly = k / MW;
      if constexpr (!INNER) {
        lx = mirror_local(lx, x0 - RM, nx, c.wall_x, MW);
        ly = mirror_local(ly, y0 - RM, ny, c.wall_y, MH);
      }
      const int pc = (ly + 1) * PW + (lx + 1);  // phi-region index
      L.mu[k] = dtheta(c, L.ph[pc], L.pl[pc]) - c.kappa * lap_ff<PW>(phi, pc);
    }
  }
  __syncthreads();

  if constexpr (RF == 2) {
    // ---- C1: rho u_o over the tile + 2, u_o the velocity of the uncorrected
    // recovery (the correction from data must not depend on the u it
    // corrects).  Positions beyond a wall stand for their mirror node, as in C.
    constexpr int VW = T::VW, VH = T::VH;
    constexpr int IC1 = (VW * VH + NT - 1) / NT;
#pragma unroll
    for (int it = 0; it < IC1; ++it) {
      const int k = tid + it * NT;
      if (k < VW * VH) {
        int lx = k % VW, ly = k / VW;
        if constexpr (!INNER) {
          lx = mirror_local(lx, x0 - 2, nx, c.wall_x, VW);
          ly = mirror_local(ly, y0 - 2, ny, c.wall_y, VH);
        }
        const int pc = (ly + R - 2) * PW + (lx + R - 2);
        float gx, gy;
        grad_ff<PW>(phi, pc, gx, gy);
        const float ph = L.ph[pc] + L.pl[pc];
        const float mu = L.mu[ly * MW + lx];  // the mu region is the tile + 2
        float ux, uy, p;
        recover(c, ph, gx, gy, mu, 0.0f, L.g0[k], L.g1x[k], L.g1y[k], ux, uy, p);
        const float rho = c.rho0 + ph * c.drho;
        L.qx[k] = rho * ux;
        L.qy[k] = rho * uy;
      }
    }
    __syncthreads();
    // ---- C2: over the tile + 1, the rate D = drho (phi - phi^(n-1)) +
    // div(rho u_o), then u and p with -F_a = D u.
#pragma unroll
    for (int it = 0; it < ICC; ++it) {
      const int k = tid + it * NT;
      if (k < UW * UH) {
        const int kx = k % UW, ky = k / UW;
        int lx = kx, ly = ky;
        if constexpr (!INNER) {
          lx = mirror_local(lx, x0 - 1, nx, c.wall_x, UW);
          ly = mirror_local(ly, y0 - 1, ny, c.wall_y, UH);
        }
        const int pc = (ly + R - 1) * PW + (lx + R - 1);
        const int mx = lx + (RM - 1), my = ly + (RM - 1);
        float gx, gy;
        grad_ff<PW>(phi, pc, gx, gy);
        const float ph = L.ph[pc] + L.pl[pc];
        const float mu = L.mu[my * MW + mx];
        float qxx, qxy, qyx, qyy;
        grad_only<VW>(L.qx, lx + 1, ly + 1, qxx, qxy);
        grad_only<VW>(L.qy, lx + 1, ly + 1, qyx, qyy);
        const float dd = (ph - L.pv[k]) * c.drho + (qxx + qyy);
        const int vk = (ky + 1) * VW + (kx + 1);  // the position's own moments
        float ux, uy, p;
        recover(c, ph, gx, gy, mu, dd, L.g0[vk], L.g1x[vk], L.g1y[vk], ux, uy, p);
        L.ux[k] = ux;
        L.uy[k] = uy;
        L.p[k] = p;
        const int tx = kx - 1, ty = ky - 1;
        if (tx >= 0 && tx < TX && ty >= 0 && ty < TY) {
          L.gx[ty * TX + tx] = gx;
          L.gy[ty * TX + tx] = gy;
          L.lm[ty * TX + tx] = dd;
        }
      }
    }
    __syncthreads();
  } else {
  // ---- C: u, p over the tile + 1, in place of the moments.  A position
  // beyond a wall stands for its mirror node: its moments were pulled from
  // that node in A, and its stencils are read around the mirror position, so
  // it gets the mirror node's u and p.  Each thread reads and writes only its
  // own position k.
#pragma unroll
  for (int it = 0; it < ICC; ++it) {
    const int k = tid + it * NT;
    if (k < UW * UH) {
      const int kx = k % UW, ky = k / UW;
      int lx = kx, ly = ky;
      if constexpr (!INNER) {
        lx = mirror_local(lx, x0 - 1, nx, c.wall_x, UW);
        ly = mirror_local(ly, y0 - 1, ny, c.wall_y, UH);
      }
      const int pc = (ly + R - 1) * PW + (lx + R - 1);
      const int mx = lx + (RM - 1), my = ly + (RM - 1);
      float gx, gy;
      grad_ff<PW>(phi, pc, gx, gy);
      const float ph = L.ph[pc] + L.pl[pc];
      const float mu = L.mu[my * MW + mx];
      const float lmu = RF ? lap_only<MW>(L.mu, mx, my) : 0.0f;
      const float cc = c.corr * lmu;
      float ux, uy, p;
      recover(c, ph, gx, gy, mu, cc, L.p[k], L.ux[k], L.uy[k], ux, uy, p);
      L.ux[k] = ux;
      L.uy[k] = uy;
      L.p[k] = p;
      // tile nodes keep grad phi and lap mu for D (no mirroring applies to
      // a node inside the grid, and ragged positions outside it are unused)
      const int tx = kx - 1, ty = ky - 1;
      if (tx >= 0 && tx < TX && ty >= 0 && ty < TY) {
        L.gx[ty * TX + tx] = gx;
        L.gy[ty * TX + tx] = gy;
        L.lm[ty * TX + tx] = lmu;
      }
    }
  }
  __syncthreads();
  }

  // ---- D: collide (or dump fields) the own nodes
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int kk = tid + j * NT;
    const int lx0 = kk % TX, ly0 = kk / TX;
    const int gx0 = x0 + lx0, gy0 = y0 + ly0;
    if (!(INNER || (gx0 < nx && gy0 < ny))) continue;
    const unsigned idx = gx0 + nx * gy0;
    const int pc = (ly0 + R) * PW + (lx0 + R);
    const int mx = lx0 + RM, my = ly0 + RM;
    const int uc = (ly0 + 1) * UW + (lx0 + 1);
    const float phh = L.ph[pc], phl = L.pl[pc];
    const float ph = phh + phl;
    const float gx = L.gx[kk], gy = L.gy[kk];
    const float mu = L.mu[my * MW + mx];
    const float lmu = L.lm[kk];  // lap mu, or D for RF = 2
    const float ux = L.ux[uc];
    const float uy = L.uy[uc];
    const float p = L.p[uc];

    if constexpr (FIELDS) {
      fo.phi[idx] = ph;
      fo.ux[idx] = ux;
      fo.uy[idx] = uy;
      fo.p[idx] = p;
      fo.mu[idx] = mu;
      // F_a by Eq. 5, whichever correction runs
      const float lap_mu = RF == 2 ? lap_only<MW>(L.mu, mx, my) : lmu;
      fo.fax[idx] = -ux * c.fa_coef * lap_mu;
      fo.fay[idx] = -uy * c.fa_coef * lap_mu;
    } else {
      const float rho = c.rho0 + ph * c.drho;
      const float cc = RF == 2 ? lmu : c.corr * lmu;
      const float fx = mu * gx + cc * ux;
      const float fy = mu * gy - (rho - c.rho_ref) * c.gravity + cc * uy;
      float gpx, gpy;
      grad_only<UW>(L.p, lx0 + 1, ly0 + 1, gpx, gpy);
      const float gpsx = gpx - (1.0f / 3.0f) * c.drho * gx;
      const float gpsy = gpy - (1.0f / 3.0f) * c.drho * gy;
      // tau = 1/2 + 3 nu, nu = mu_dyn(phi) / rho
      const float mud = c.mu0 + ph * c.dmu;
      const float om = rho * __builtin_amdgcn_rcpf(0.5f * rho + 3.0f * mud);  // 1 / tau
      const float half = 1.0f - 0.5f * om;
      const float uu = ux * ux + uy * uy;
      // BGK with the Eq. 8 forcing, regrouped per direction as
      //   g* = (1 - om) g + w [A + B_i + t_i (C + D_i)]
      // with t_i = omega_i / w_i - 1, g^eq = w p + (rho/3) w t_i,
      // S_i = w [(e.F - u.F)(1 + t_i) - t_i (e.grad psi - u.grad psi)]:
      //   A = om p - half u.F,  C = om rho/3 - half u.F + half u.grad psi,
      //   B_i = half e.F,  D_i = half e.(F - grad psi);
      // and f* = (1 - om_f) f + w (om_f 3 Gamma mu + om_f phi t_i).
      const float uf = ux * fx + uy * fy;
      const float ug = ux * gpsx + uy * gpsy;
      const float A = om * p - half * uf;
      const float Cc = om * (1.0f / 3.0f) * rho - half * uf + half * ug;
      const float hfx = half * fx, hfy = half * fy;
      const float hdx = half * (fx - gpsx), hdy = half * (fy - gpsy);
      const float m15 = -1.5f * uu;
      const float omg = 1.0f - om;
      const float omf = 1.0f - c.omega_f;
      const float fP = c.omega_f * c.gamma3 * mu;
      const float fQ = c.omega_f * ph;
      const uint32_t nkey = S == ST_FP32 ? 0u : sr_node_key(skey, idx);
      float fsum = 0.0f;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        // e_i . v for e_i with components in {-1, 0, 1}
        const float eu = (EX(i) ? (EX(i) > 0 ? ux : -ux) : 0.0f) +
                         (EY(i) ? (EY(i) > 0 ? uy : -uy) : 0.0f);
        const float bi = (EX(i) ? (EX(i) > 0 ? hfx : -hfx) : 0.0f) +
                         (EY(i) ? (EY(i) > 0 ? hfy : -hfy) : 0.0f);
        const float di = (EX(i) ? (EX(i) > 0 ? hdx : -hdx) : 0.0f) +
                         (EY(i) ? (EY(i) > 0 ? hdy : -hdy) : 0.0f);
        const float ti = eu * (3.0f + 4.5f * eu) + m15;  // omega_i / w_i - 1
        if (i > 0) {
          const float fn = omf * own.f(c, j, i) + WT(i) * (fP + fQ * ti);
          fsum += op.put_f(c, i, idx, fn);
        }
        const float gn = omg * own.g(c, j, i, WT(i)) + WT(i) * ((A + bi) + ti * (Cc + di));
        op.put_g(c, i, idx, gn, WT(i), sr_bits(nkey, i));
      }
      float h0, e0;
      two_sum(phh, -fsum, h0, e0);
      op.put_f0(idx, h0, e0 + phl);
      // the copy carries this step's phi, the next step's phi^(n-1)
      if constexpr (RF == 2) gstore_nt<float>(dst, c.phiv + 4u * idx, ph);
    }
  }
  __syncthreads();
}

// RF = 1: lap mu is formed (corrected model, or the F_a dump); phi halo 3.
// RF = 2: the correction from data (phases C1, C2); phi halo 3.
// WPE > 0 asks the compiler for at least that many waves per SIMD (fewer
// registers, more tiles in flight per CU).
//
// Tile order: workgroup b runs on XCD b % 8.  Each XCD walks its own
// contiguous chunk of the tile list (which the host orders in narrow
// vertical strips), so the tiles in flight on one XCD are neighbours and
// share their halos through that XCD's L2.
struct TileWalk {
  int t, t_end, step;
  __device__ __forceinline__ explicit TileWalk(int ntiles) {
    step = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7;
    const int chunk = (ntiles + 7) >> 3;
    t_end = min(ntiles, (xcd + 1) * chunk);
    t = xcd * chunk + (blockIdx.x >> 3);
  }
};

template <int TX, int TY, int RF>
__device__ __forceinline__ bool tile_inner(const CaseDev& c, const TileDev& tl) {
  constexpr int R = TileLds<TX, TY, RF>::R;
  return (tl.x0 - R - 1 >= 0) && (tl.x0 + TX + R + 1 <= c.nx) && (tl.y0 - R - 1 >= 0) &&
         (tl.y0 + TY + R + 1 <= c.ny);
}

// One tile per iteration: all loads of a tile are issued in one batch,
// summed into LDS, then B, C, D.
template <int TX, int TY, int NPT, int RF, int S, bool FIELDS, int WPE>
__global__ void __launch_bounds__(TX * TY / NPT)
__attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
k_tile(const CaseDev* __restrict__ cases, const TileDev* __restrict__ tiles, int ntiles,
       int parity, FieldOut fo) {
  static_assert(sizeof(TileLds<TX, TY, RF>) <= 160 * 1024, "tile exceeds the LDS of a CU");
  __shared__ TileLds<TX, TY, RF> lds;
  uint32_t skey = 0;  // stochastic rounding of the 16-bit g stores
  if constexpr (S != ST_FP32 && !FIELDS) skey = sr_step_key(sr_clock(cases[0], parity));
  for (TileWalk w(ntiles); w.t < w.t_end; w.t += w.step) {
    const TileDev tl = tiles[w.t];
    const CaseDev c = cases[tl.icase];
    const char* src = parity ? c.state[1] : c.state[0];
    char* dst = parity ? c.state[0] : c.state[1];
    TileLoads<TX, TY, NPT, RF, S> ld;
    OwnPops<S, NPT> own;
    if (tile_inner<TX, TY, RF>(c, tl)) {
      ld.template load_all<true>(c, src, tl.x0, tl.y0, lds, own);
      __syncthreads();
      tile_bcd<TX, TY, NPT, RF, S, FIELDS, true>(lds, c, tl.x0, tl.y0, dst, fo, own, skey);
    } else {
      ld.template load_all<false>(c, src, tl.x0, tl.y0, lds, own);
      __syncthreads();
      tile_bcd<TX, TY, NPT, RF, S, FIELDS, false>(lds, c, tl.x0, tl.y0, dst, fo, own, skey);
    }
  }
}

// Initial populations: equilibria of phi0, mu(phi0), u0, p0 written where
// the pull of the first step will find them (the inverse of streaming).  The
// FP64 phi0 is split into hi + lo floats, the representation of f_0.
template <int S>
__global__ void __launch_bounds__(256)
k_init(CaseDev c, int parity, const double* __restrict__ phi0, const double* __restrict__ u0,
       const double* __restrict__ p0) {
  using P = Pops<S, Q>;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c.n) return;
  const int x = idx % c.nx, y = idx / c.nx;
  float nh[Q], nl[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int sx = map_axis(x + EX(i), c.nx, c.wall_x);
    const int sy = map_axis(y + EY(i), c.ny, c.wall_y);
    const double v = phi0[sx + c.nx * sy];
    nh[i] = (float)v;
    nl[i] = (float)(v - (double)nh[i]);
  }
  auto d = [&](int a) { return (nh[a] - nh[0]) + (nl[a] - nl[0]); };
  const float lap = (2.0f / 3.0f) * ((d(1) + d(2)) + (d(3) + d(4))) +
                    (1.0f / 6.0f) * ((d(5) + d(6)) + (d(7) + d(8)));
  const float mu = dtheta(c, nh[0], nl[0]) - c.kappa * lap;
  const float ph = nh[0] + nl[0];
  const float ux = (float)u0[idx], uy = (float)u0[c.n + idx];
  const float p = (float)p0[idx];
  const float rho = c.rho0 + ph * c.drho;
  const float uu = ux * ux + uy * uy;
  char* dst = parity ? c.state[1] : c.state[0];
  float fsum = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float eu = EX(i) * ux + EY(i) * uy;
    const float ti = 3.0f * eu + 4.5f * eu * eu - 1.5f * uu;
    const float wt = WT(i) * ti;
    const float geq = WT(i) * p + (1.0f / 3.0f) * rho * wt;
    // population i of node x is pulled from x - e_i, or from x itself in the
    // opposite direction across a wall
    int dir = i;
    unsigned j = idx;
    if (i > 0) {
      bool bb;
      const unsigned s = pull_src(c, x, y, 0, EX(i), EY(i), 0, &bb);
      if (!bb) j = s;
      else dir = OPP(i);
      const float feq = WT(i) * (c.gamma3 * mu + ph * ti);
      fsum += P::put_f(c, dst, dir, j, feq);
    }
    P::put_g(c, dst, dir, j, geq, WT(i));
  }
  float h0, e0;
  two_sum(nh[0], -fsum, h0, e0);
  P::put_f0(c, dst, idx, h0, e0 + nl[0]);
  // correction from data: phi^(n-1) of the first step is phi0
  if (c.phiv) gstore_nt<float>(dst, c.phiv + 4u * idx, ph);
}

}  // namespace d2q9

// ------------------------------------------------------------ launchers
namespace {
using d2q9::FieldOut;

template <int TX, int TY, int NPT, int RF, int S, int WPE>
hipError_t launch_step_t(const LaunchArgs& a) {
  FieldOut fo{};
  hipLaunchKernelGGL((d2q9::k_tile<TX, TY, NPT, RF, S, false, WPE>), dim3(a.grid),
                     dim3(TX * TY / NPT), 0, a.stream, a.cases, a.tiles, a.ntiles, a.parity, fo);
  return hipGetLastError();
}

template <int TX, int TY, int NPT, int WPE, int S>
hipError_t launch_fields_t(const LaunchArgs& a, const FieldPtrs& f) {
  FieldOut fo{f.phi, f.u[0], f.u[1], f.u[2], f.p, f.mu, f.fa[0], f.fa[1], f.fa[2]};
  if (a.rf == 2)
    hipLaunchKernelGGL((d2q9::k_tile<TX, TY, NPT, 2, S, true, WPE>), dim3(a.grid),
                       dim3(TX * TY / NPT), 0, a.stream, a.cases, a.tiles, a.ntiles, a.parity,
                       fo);
  else
    hipLaunchKernelGGL((d2q9::k_tile<TX, TY, NPT, 1, S, true, WPE>), dim3(a.grid),
                       dim3(TX * TY / NPT), 0, a.stream, a.cases, a.tiles, a.ntiles, a.parity,
                       fo);
  return hipGetLastError();
}

template <int TX, int TY, int NPT = 1, int WPE = 0>
hipError_t launch_step_v(const LaunchArgs& a) {
  if (a.rf == 2) {
    switch (a.storage) {
      case ST_FP32: return launch_step_t<TX, TY, NPT, 2, ST_FP32, WPE>(a);
      case ST_FP16: return launch_step_t<TX, TY, NPT, 2, ST_FP16, WPE>(a);
      default: return launch_step_t<TX, TY, NPT, 2, ST_BF16, WPE>(a);
    }
  }
  if (a.rf) {
    switch (a.storage) {
      case ST_FP32: return launch_step_t<TX, TY, NPT, 1, ST_FP32, WPE>(a);
      case ST_FP16: return launch_step_t<TX, TY, NPT, 1, ST_FP16, WPE>(a);
      default: return launch_step_t<TX, TY, NPT, 1, ST_BF16, WPE>(a);
    }
  }
  switch (a.storage) {
    case ST_FP32: return launch_step_t<TX, TY, NPT, 0, ST_FP32, WPE>(a);
    case ST_FP16: return launch_step_t<TX, TY, NPT, 0, ST_FP16, WPE>(a);
    default: return launch_step_t<TX, TY, NPT, 0, ST_BF16, WPE>(a);
  }
}
}  // namespace

// Compiled tile shapes of the D2Q9 step (index = launch variant): tile width,
// height, depth, threads per workgroup (one, two or four nodes per thread) and
// the strip width of the tile order (0: default).  The last three reuse
// kernels of earlier entries with 1024-node strips (measured faster on
// 4096^2 grids; narrower strips were slower).  Variants 8 and 9 also ask for
// 6 waves per SIMD, which their 512-thread tiles' LDS allows: the 16-bit
// kernels then fit 80 VGPRs instead of 82-93 (5 waves).
const TileShape kD2Q9Tiles[] = {
    {32, 16, 1, 512, 0},  {64, 8, 1, 512, 0},    {64, 16, 1, 512, 0},  {128, 8, 1, 512, 0},
    {128, 16, 1, 1024, 0}, {64, 32, 1, 1024, 0}, {64, 8, 1, 256, 0},   {64, 16, 1, 256, 0},
    {64, 16, 1, 512, 1024}, {128, 8, 1, 512, 1024}, {64, 8, 1, 256, 1024}};
const int kD2Q9TileCount = sizeof(kD2Q9Tiles) / sizeof(kD2Q9Tiles[0]);

hipError_t d2q9_step(int variant, const LaunchArgs& a) {
  switch (variant) {
    case 0: return launch_step_v<32, 16>(a);
    case 1: return launch_step_v<64, 8>(a);
    case 2: return launch_step_v<64, 16, 2, 4>(a);
    case 3: return launch_step_v<128, 8, 2, 4>(a);
    case 4: return launch_step_v<128, 16, 2, 4>(a);
    case 5: return launch_step_v<64, 32, 2, 4>(a);
    case 6: return launch_step_v<64, 8, 2, 4>(a);
    case 7: return launch_step_v<64, 16, 4, 4>(a);
    case 8: return launch_step_v<64, 16, 2, 6>(a);
    case 9: return launch_step_v<128, 8, 2, 6>(a);
    case 10: return launch_step_v<64, 8, 2, 4>(a);
    default: return hipErrorInvalidValue;
  }
}

// The field dump: 64 x 16 tiles, two nodes per thread (the shape of the
// step's variant 2).
const TileShape kD2Q9FieldShape = {64, 16, 1, 512, 0};

hipError_t d2q9_fields(const LaunchArgs& a, const FieldPtrs& f) {
  switch (a.storage) {
    case ST_FP32: return launch_fields_t<64, 16, 2, 4, ST_FP32>(a, f);
    case ST_FP16: return launch_fields_t<64, 16, 2, 4, ST_FP16>(a, f);
    default: return launch_fields_t<64, 16, 2, 4, ST_BF16>(a, f);
  }
}

hipError_t d2q9_init(const CaseDev& c, int storage, int parity, const double* phi0,
                     const double* u0, const double* p0, hipStream_t stream) {
  const int grid = (c.n + 255) / 256;
  switch (storage) {
    case ST_FP32:
      hipLaunchKernelGGL(d2q9::k_init<ST_FP32>, dim3(grid), dim3(256), 0, stream, c, parity,
                         phi0, u0, p0);
      break;
    case ST_FP16:
      hipLaunchKernelGGL(d2q9::k_init<ST_FP16>, dim3(grid), dim3(256), 0, stream, c, parity,
                         phi0, u0, p0);
      break;
    default:
      hipLaunchKernelGGL(d2q9::k_init<ST_BF16>, dim3(grid), dim3(256), 0, stream, c, parity,
                         phi0, u0, p0);
  }
  return hipGetLastError();
}

}  // namespace lbm
