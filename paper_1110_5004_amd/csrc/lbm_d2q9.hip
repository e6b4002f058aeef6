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

// theta'(phi) for theta = beta phi^2 (phi - 1)^2, with phi = hi + lo carried
// as two floats: phi - 1 and 2 phi - 1 are formed before rounding to one
// float, so they keep their absolute precision near phi = 1 and phi = 1/2.
__device__ __forceinline__ float dtheta(const CaseDev& c, float hi, float lo) {
  const float a = hi + lo;
  const float b = (hi - 1.0f) + lo;
  const float d = (2.0f * hi - 1.0f) + 2.0f * lo;
  return c.beta2 * a * b * d;
}

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
// with c = remove_fa drho theta_M lap mu, the cancelled -F_a = c u.
__device__ __forceinline__ void recover(const CaseDev& c, float phi, float gx, float gy, float mu,
                                        float lmu, float m0, float m1x, float m1y, float& ux,
                                        float& uy, float& p) {
  const float rho = c.rho_g + phi * c.drho;
  const float fsx = mu * gx;
  const float fsy = mu * gy - (rho - c.rho_ref) * c.gravity;
  const float cc = c.corr * lmu;
  const float den = rho - 0.5f * cc;
  ux = (3.0f * m1x + 0.5f * fsx) / den;
  uy = (3.0f * m1y + 0.5f * fsy) / den;
  p = m0 + (1.0f / 6.0f) * c.drho * (ux * gx + uy * gy);
}

// phi = f_0 + sum_{i>0} f_i as hi + lo (pulled populations).
template <int S>
__device__ __forceinline__ void phi_pull(const CaseDev& c, const char* src, int x, int y,
                                         bool inner, float& hi, float& lo) {
  using P = Pops<S, Q>;
  const int idx = x + c.nx * y;
  float sm = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    int dir = i, j;
    if (inner) j = idx - EX(i) - c.nx * EY(i);
    else j = pull_src(c, x, y, 0, EX(i), EY(i), 0, i, OPP(i), &dir);
    sm += P::f(c, src, dir, j);
  }
  two_sum(P::f(c, src, 0, idx), P::f0lo(c, src, idx) + sm, hi, lo);
}

template <int S>
__device__ __forceinline__ void g_moments(const CaseDev& c, const char* src, int x, int y,
                                          bool inner, float& m0, float& m1x, float& m1y) {
  using P = Pops<S, Q>;
  const int idx = x + c.nx * y;
  m0 = m1x = m1y = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int dir = i, j = idx;
    if (i > 0) {
      if (inner) j = idx - EX(i) - c.nx * EY(i);
      else j = pull_src(c, x, y, 0, EX(i), EY(i), 0, i, OPP(i), &dir);
    }
    const float v = P::g(c, src, dir, j, WT(i));
    m0 += v;
    if (EX(i)) m1x += EX(i) > 0 ? v : -v;
    if (EY(i)) m1y += EY(i) > 0 ? v : -v;
  }
}

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

// RF = 1: lap mu is formed (corrected model, or the F_a dump); phi halo 3.
// NT threads per tile; every phase loop has a compile-time trip count and is
// unrolled, so a thread issues the loads of all its positions at once.
template <int TX, int TY, int NT, int RF, int S, bool FIELDS>
__global__ void __launch_bounds__(NT)
k_tile(const CaseDev* __restrict__ cases, const TileDev* __restrict__ tiles, int ntiles,
       int parity, FieldOut fo) {
  constexpr int R = RF ? 3 : 2;   // phi radius
  constexpr int RM = R - 1;       // mu radius
  constexpr int PW = TX + 2 * R, PH = TY + 2 * R;
  constexpr int MW = TX + 2 * RM, MH = TY + 2 * RM;
  constexpr int UW = TX + 2, UH = TY + 2;
  constexpr int IA = (PW * PH + NT - 1) / NT;
  constexpr int IB = (MW * MH + NT - 1) / NT;
  constexpr int IC = (UW * UH + NT - 1) / NT;
  constexpr int ID = (TX * TY + NT - 1) / NT;
  __shared__ float s_ph[PW * PH];  // phi = s_ph + s_pl
  __shared__ float s_pl[PW * PH];
  __shared__ float s_mu[MW * MH];
  __shared__ float s_ux[UW * UH];
  __shared__ float s_uy[UW * UH];
  __shared__ float s_p[UW * UH];
  using P = Pops<S, Q>;
  const FF<PW> phi{s_ph, s_pl};

  // XCD-aware order: workgroup b runs on XCD b % 8; give each XCD a
  // contiguous run of tiles so that halos are shared through its L2.
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int v0 = (b & 7) * (G >> 3) + (b >> 3);
  const int tid = threadIdx.x;

  for (int t = v0; t < ntiles; t += G) {
    const TileDev tl = tiles[t];
    const CaseDev c = cases[tl.icase];
    const int nx = c.nx, ny = c.ny;
    const int x0 = tl.x0, y0 = tl.y0;
    const char* src = parity ? c.state[1] : c.state[0];
    char* dst = parity ? c.state[0] : c.state[1];
    // inner: every pulled population of the phi region lies inside the grid
    const bool inner = (x0 - R - 1 >= 0) && (x0 + TX + R + 1 <= nx) && (y0 - R - 1 >= 0) &&
                       (y0 + TY + R + 1 <= ny);

    // ---- A: phi over the tile + R
#pragma unroll
    for (int it = 0; it < IA; ++it) {
      const int k = tid + it * NT;
      if (k < PW * PH) {
        const int lx = k % PW, ly = k / PW;
        int gx = x0 - R + lx, gy = y0 - R + ly;
        if (!inner) {
          gx = map_axis(gx, nx, c.wall_x);
          gy = map_axis(gy, ny, c.wall_y);
        }
        float hi, lo;
        phi_pull<S>(c, src, gx, gy, inner, hi, lo);
        s_ph[k] = hi;
        s_pl[k] = lo;
      }
    }
    __syncthreads();

    // ---- B: mu over the tile + RM
#pragma unroll
    for (int it = 0; it < IB; ++it) {
      const int k = tid + it * NT;
      if (k < MW * MH) {
        int lx = k % MW, ly = k / MW;
        if (!inner) {
          lx = mirror_local(lx, x0 - RM, nx, c.wall_x, MW);
          ly = mirror_local(ly, y0 - RM, ny, c.wall_y, MH);
        }
        const int pc = (ly + 1) * PW + (lx + 1);  // phi-region index
        s_mu[k] = dtheta(c, s_ph[pc], s_pl[pc]) - c.kappa * lap_ff<PW>(phi, pc);
      }
    }
    __syncthreads();

    // ---- C: u, p over the tile + 1
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      const int k = tid + it * NT;
      if (k < UW * UH) {
        int lx = k % UW, ly = k / UW;
        if (!inner) {
          lx = mirror_local(lx, x0 - 1, nx, c.wall_x, UW);
          ly = mirror_local(ly, y0 - 1, ny, c.wall_y, UH);
        }
        int nxg = x0 - 1 + lx, nyg = y0 - 1 + ly;
        if (!inner) {
          nxg = map_axis(nxg, nx, c.wall_x);
          nyg = map_axis(nyg, ny, c.wall_y);
        }
        float m0, m1x, m1y;
        g_moments<S>(c, src, nxg, nyg, inner, m0, m1x, m1y);
        const int pc = (ly + R - 1) * PW + (lx + R - 1);
        const int mx = lx + (RM - 1), my = ly + (RM - 1);
        float gx, gy;
        grad_ff<PW>(phi, pc, gx, gy);
        const float ph = s_ph[pc] + s_pl[pc];
        const float mu = s_mu[my * MW + mx];
        const float lmu = RF ? lap_only<MW>(s_mu, mx, my) : 0.0f;
        float ux, uy, p;
        recover(c, ph, gx, gy, mu, lmu, m0, m1x, m1y, ux, uy, p);
        s_ux[k] = ux;
        s_uy[k] = uy;
        s_p[k] = p;
      }
    }
    __syncthreads();

    // ---- D: collide (or dump fields) over the tile
#pragma unroll
    for (int it = 0; it < ID; ++it) {
      const int k = tid + it * NT;
      const int lx = k % TX, ly = k / TX;
      const int gxn = x0 + lx, gyn = y0 + ly;
      if (k < TX * TY && gxn < nx && gyn < ny) {
        const int idx = gxn + nx * gyn;
        const int pc = (ly + R) * PW + (lx + R);
        const int mx = lx + RM, my = ly + RM;
        const int uc = (ly + 1) * UW + (lx + 1);
        const float phh = s_ph[pc], phl = s_pl[pc];
        const float ph = phh + phl;
        float gx, gy;
        grad_ff<PW>(phi, pc, gx, gy);
        const float mu = s_mu[my * MW + mx];
        const float lmu = RF ? lap_only<MW>(s_mu, mx, my) : 0.0f;
        const float ux = s_ux[uc];
        const float uy = s_uy[uc];
        const float p = s_p[uc];

        if constexpr (FIELDS) {
          fo.phi[idx] = ph;
          fo.ux[idx] = ux;
          fo.uy[idx] = uy;
          fo.p[idx] = p;
          fo.mu[idx] = mu;
          fo.fax[idx] = -ux * c.fa_coef * lmu;
          fo.fay[idx] = -uy * c.fa_coef * lmu;
        } else {
          // pull every population first (f_0 is not needed: the post-collision
          // f_0 closes sum_i f_i* = phi), then collide, then store
          float fv[Q], gv[Q];
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            int dir = i, j = idx;
            if (i > 0) {
              if (inner) j = idx - EX(i) - nx * EY(i);
              else j = pull_src(c, gxn, gyn, 0, EX(i), EY(i), 0, i, OPP(i), &dir);
              fv[i] = P::f(c, src, dir, j);
            }
            gv[i] = P::g(c, src, dir, j, WT(i));
          }
          const float rho = c.rho_g + ph * c.drho;
          const float cc = c.corr * lmu;
          const float fx = mu * gx + cc * ux;
          const float fy = mu * gy - (rho - c.rho_ref) * c.gravity + cc * uy;
          float gpx, gpy;
          grad_only<UW>(s_p, lx + 1, ly + 1, gpx, gpy);
          const float gpsx = gpx - (1.0f / 3.0f) * c.drho * gx;
          const float gpsy = gpy - (1.0f / 3.0f) * c.drho * gy;
          const float nu = (c.mu_g + ph * c.dmu) / rho;
          const float tau = 0.5f + 3.0f * nu;
          const float itau = 1.0f / tau;
          const float half = 1.0f - 0.5f * itau;
          const float uu = ux * ux + uy * uy;
          const float gm3 = c.gamma3 * mu;
          float fsum = 0.0f;
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const float eu = EX(i) * ux + EY(i) * uy;
            const float ti = 3.0f * eu + 4.5f * eu * eu - 1.5f * uu;  // omega_i / w_i - 1
            const float wt = WT(i) * ti;                               // omega_i - w_i
            if (i > 0) {
              const float feq = WT(i) * (gm3 + ph * ti);
              const float fn = fv[i] - c.omega_f * (fv[i] - feq);
              fsum += P::put_f(c, dst, i, idx, fn);
            }
            // g^eq = w p + rho cs^2 (omega - w);  S = (e - u).[F omega - (omega - w) grad psi]
            const float geq = WT(i) * p + (1.0f / 3.0f) * rho * wt;
            const float dx = EX(i) - ux, dy = EY(i) - uy;
            const float src_i =
                (dx * fx + dy * fy) * (WT(i) + wt) - wt * (dx * gpsx + dy * gpsy);
            const float gn = gv[i] - itau * (gv[i] - geq) + half * src_i;
            P::put_g(c, dst, i, idx, gn, WT(i));
          }
          float h0, e0;
          two_sum(phh, -fsum, h0, e0);
          P::put_f0(c, dst, idx, h0, e0 + phl);
        }
      }
    }
    __syncthreads();
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
  const float rho = c.rho_g + ph * c.drho;
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
    int dir = i, j = idx;
    if (i > 0) {
      int sdir;
      const int s = pull_src(c, x, y, 0, EX(i), EY(i), 0, i, OPP(i), &sdir);
      if (sdir == i) j = s;
      else dir = OPP(i);
      const float feq = WT(i) * (c.gamma3 * mu + ph * ti);
      fsum += P::put_f(c, dst, dir, j, feq);
    }
    P::put_g(c, dst, dir, j, geq, WT(i));
  }
  float h0, e0;
  two_sum(nh[0], -fsum, h0, e0);
  P::put_f0(c, dst, idx, h0, e0 + nl[0]);
}

}  // namespace d2q9

// ------------------------------------------------------------ launchers
namespace {
using d2q9::FieldOut;

template <int TX, int TY, int NT, int RF, int S>
hipError_t launch_step_t(const LaunchArgs& a) {
  FieldOut fo{};
  hipLaunchKernelGGL((d2q9::k_tile<TX, TY, NT, RF, S, false>), dim3(a.grid), dim3(NT), 0,
                     a.stream, a.cases, a.tiles, a.ntiles, a.parity, fo);
  return hipGetLastError();
}

template <int TX, int TY, int NT, int S>
hipError_t launch_fields_t(const LaunchArgs& a, const FieldPtrs& f) {
  FieldOut fo{f.phi, f.u[0], f.u[1], f.u[2], f.p, f.mu, f.fa[0], f.fa[1], f.fa[2]};
  hipLaunchKernelGGL((d2q9::k_tile<TX, TY, NT, 1, S, true>), dim3(a.grid), dim3(NT), 0,
                     a.stream, a.cases, a.tiles, a.ntiles, a.parity, fo);
  return hipGetLastError();
}

template <int TX, int TY, int NT>
hipError_t launch_step_v(const LaunchArgs& a) {
  if (a.rf) {
    switch (a.storage) {
      case ST_FP32: return launch_step_t<TX, TY, NT, 1, ST_FP32>(a);
      case ST_FP16: return launch_step_t<TX, TY, NT, 1, ST_FP16>(a);
      default: return launch_step_t<TX, TY, NT, 1, ST_BF16>(a);
    }
  }
  switch (a.storage) {
    case ST_FP32: return launch_step_t<TX, TY, NT, 0, ST_FP32>(a);
    case ST_FP16: return launch_step_t<TX, TY, NT, 0, ST_FP16>(a);
    default: return launch_step_t<TX, TY, NT, 0, ST_BF16>(a);
  }
}
}  // namespace

// Compiled tile shapes of the D2Q9 step (index = launch variant).
const TileShape kD2Q9Tiles[] = {{64, 16, 1, 1024}, {64, 8, 1, 512}, {32, 16, 1, 512},
                                {64, 32, 1, 1024}, {128, 8, 1, 1024}, {32, 8, 1, 256}};
const int kD2Q9TileCount = sizeof(kD2Q9Tiles) / sizeof(kD2Q9Tiles[0]);

hipError_t d2q9_step(int variant, const LaunchArgs& a) {
  switch (variant) {
    case 0: return launch_step_v<64, 16, 1024>(a);
    case 1: return launch_step_v<64, 8, 512>(a);
    case 2: return launch_step_v<32, 16, 512>(a);
    case 3: return launch_step_v<64, 32, 1024>(a);
    case 4: return launch_step_v<128, 8, 1024>(a);
    case 5: return launch_step_v<32, 8, 256>(a);
    default: return hipErrorInvalidValue;
  }
}

// The field dump uses the shape of variant 0.
hipError_t d2q9_fields(const LaunchArgs& a, const FieldPtrs& f) {
  switch (a.storage) {
    case ST_FP32: return launch_fields_t<64, 16, 1024, ST_FP32>(a, f);
    case ST_FP16: return launch_fields_t<64, 16, 1024, ST_FP16>(a, f);
    default: return launch_fields_t<64, 16, 1024, ST_BF16>(a, f);
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
