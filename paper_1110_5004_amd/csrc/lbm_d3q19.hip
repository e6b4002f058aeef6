// lbm_d3q19.hip -- gfx950 kernels of the D3Q19 form of the phase-field step.
//
// The same model as the D2Q9 step (Eq. 1a, Eq. 4a, Eq. 8, the -F_a switch of
// the paragraph after Eq. 12, isotropic central stencils), on 19 velocities.
// A step is either the fused kernel
//   k3_slab      one x-y tile marching up a z chunk, phi / mu / p rings in
//                LDS, the whole step per plane (see its comment); k3_slab2
//                the same one plane shorter when the Eq. 5 term is zero
// or three kernels that pass fields through HBM:
//   k3_pull      pull f and gbar; phi (float-float) and the gbar moments
//   k3_fields_t  on LDS tiles: mu = theta'(phi) - kappa lap phi, then grad
//                phi, lap mu, u and p (with -F_a in the corrected model)
//   k3_collide   grad phi and mu again from the phi planes, grad p ->
//                grad psi, BGK collision of f and gbar, store
// or, with 16-bit storage, two: k3_pull, then k3_fcm, which marches x-y
// tiles up z chunks doing the work of k3_fields_t and k3_collide with the
// fields in LDS rings.  All forms compute every node to the same bits.  Stencil neighbours go through
// the periodic / mirror mapping, so positions beyond a wall read their mirror
// node.
#include "lbm_d3q19_addr.h"
#include "lbm_d3q19_lean.h"
#include "lbm_dev.h"
#include "lbm_kernels.h"
#include "lbm_lattice.h"

namespace lbm {
namespace d3q19 {

// Launch shape of the node-parallel kernels (see Node3).
struct RowGrid {
  dim3 grid, block;
};
inline RowGrid row_grid(const CaseDev& c) {
  const int bx = c.nx >= 256 ? 256 : ((c.nx + 63) / 64) * 64;
  return {dim3(c.ny * c.nz, (c.nx + bx - 1) / bx), dim3(bx)};
}

struct Fields3 {
  float *phh, *phl, *m0, *m1x, *m1y, *m1z;  // pull
  float* mu;                                // mu
  float *ux, *uy, *uz, *p, *lmu;                 // fields
  float* dd;  // correction from data: the rate D of -F_a = D u
};

// Store of a field plane value that the next kernel of the step reads.
__device__ __forceinline__ void plane_put(float* a, unsigned idx, float v) {
  gstore_nt<float>(reinterpret_cast<char*>(a), 4u * idx, v);
}

// phi = sum_i f_i of the pulled populations (Eq. 4a's zeroth moment), as a
// float-float pair: f_0 (high and low part) plus the sum of the others.
template <int S, class N>
__device__ __forceinline__ void pull_phi(const CaseDev& c, const char* src, const N& nd,
                                         float& hi, float& lo) {
  using P = Pops<S, Q>;
  float sm = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) sm += P::f(c, src, i, pull3<S, false, N>(c, nd, i));
  two_sum(P::f(c, src, 0, P::fofs(c, 0, nd.idx)), P::f0lo(c, src, nd.idx) + sm, hi, lo);
}

// Zeroth and first moments of the pulled gbar (the inputs of the recovery of
// p and u).
template <int S, class N>
__device__ __forceinline__ void pull_moments(const CaseDev& c, const char* src, const N& nd,
                                             float& m0, float& mx, float& my, float& mz) {
  using P = Pops<S, Q>;
  m0 = mx = my = mz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float v = P::g(c, src, pull3<S, true, N>(c, nd, i), WT(i));
    m0 += v;
    if (EX(i)) mx += EX(i) > 0 ? v : -v;
    if (EY(i)) my += EY(i) > 0 ? v : -v;
    if (EZ(i)) mz += EZ(i) > 0 ? v : -v;
  }
}

// ---- 1: pull, phi, moments
// One grid row (y, z) per blockIdx.x.  zc = 0: rows in storage order.  zc > 0
// (ahead of k3_fcm on chunks of zc planes): the planes go offset-major
// through the chunks, from the last plane of every chunk down to the first,
// so that the first planes of each chunk -- the ones k3_fcm pulls first --
// are read last and are still in the Infinity Cache when k3_fcm starts;
// blockIdx.x then spans ny x zc x (number of chunks) rows, and the rows of
// planes beyond the grid exit.
template <int S>
__global__ void __launch_bounds__(256) k3_pull(CaseDev c, int parity, Fields3 fl, int zc) {
  const int x = blockIdx.y * blockDim.x + threadIdx.x;
  if (x >= c.nx) return;
  int z = blockIdx.x / c.ny;
  if (zc > 0) {
    const int nch = (c.nz + zc - 1) / zc;
    z = (z % nch) * zc + (zc - 1 - z / nch);
    if (z >= c.nz) return;
  }
  const Node3 nd(c, x, blockIdx.x % c.ny, z);
  const unsigned idx = nd.idx;
  const char* src = parity ? c.state[1] : c.state[0];
  float hi, lo, m0, mx, my, mz;
  if constexpr (S != ST_FP32) {
    // 16-bit storage: one-float phi and the moments from the stored words,
    // packed in pairs as the fused step holds them
    uint16_t fh[Q], gh[Q + 1];
#pragma unroll
    for (int i = 1; i < Q; ++i) fh[i] = gload<uint16_t>(src, pull3<S, false>(c, nd, i));
#pragma unroll
    for (int i = 0; i < Q; ++i) gh[i] = gload<uint16_t>(src, pull3<S, true>(c, nd, i));
    gh[Q] = 0;
    uint32_t Fr[10], Gr[10];
    Fr[0] = 0u;
#pragma unroll
    for (int j = 1; j <= 9; ++j) Fr[j] = pack16(fh[PI(j)], fh[PI(j) + 1]);
#pragma unroll
    for (int k = 0; k < 10; ++k) Gr[k] = pack16(gh[2 * k], gh[2 * k + 1]);
    hi = lean_phi_packed<S>(c, gload<float>(src, 4u * idx), Fr);
    lo = 0.0f;
    lean_moments_packed<S>(c, Gr, m0, mx, my, mz);
  } else {
    pull_phi<S>(c, src, nd, hi, lo);
    pull_moments<S>(c, src, nd, m0, mx, my, mz);
  }
  plane_put(fl.phh, idx, hi);
  if constexpr (S == ST_FP32) plane_put(fl.phl, idx, lo);  // 16-bit: phi is one float
  plane_put(fl.m0, idx, m0);
  plane_put(fl.m1x, idx, mx);
  plane_put(fl.m1y, idx, my);
  plane_put(fl.m1z, idx, mz);
}

// Isotropic gradient 3 sum_i w_i e_i f_i of a node field, from differences
// to the centre (the stencil of the step's grad p).
__device__ __forceinline__ void grad_f(const CaseDev& c, const float* f, const Node3& nd,
                                       float* g) {
  const float f0 = f[nd.idx];
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const float d = f[nbr3(c, nd, i)] - f0;
    const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);
    if (EX(i)) ax += EX(i) > 0 ? w * d : -w * d;
    if (EY(i)) ay += EY(i) > 0 ? w * d : -w * d;
    if (EZ(i)) az += EZ(i) > 0 ? w * d : -w * d;
  }
  g[0] = ax;
  g[1] = ay;
  g[2] = az;
}

// ---- 2+3: mu, grad phi, lap mu, u, p on a TX x TY x TZ tile through LDS.
// phi (float-float) is staged over the tile + 2, mu is formed over the tile
// + 1, then each node of the tile forms its gradient, lap mu, u and p.  A
// staged position holds the value of the node it maps to (periodic wrap or
// mirror ghost); a mu position beyond a wall is computed around its mirror
// position, so that it equals the mirror node's mu as the step defines it.
// Stencil sums run over i = 1..18 in lattice order, as in the node-parallel
// definition, so the result does not depend on the tile shape.
template <int TX, int TY, int TZ, bool RF2, bool LEAN>
struct FieldTile {
  static constexpr int NT = TX * TY * TZ;
  static constexpr int PX = TX + 4, PY = TY + 4, PZ = TZ + 4;  // phi region
  static constexpr int MX = TX + 2, MY = TY + 2, MZ = TZ + 2;  // mu region
  static constexpr int NP = PX * PY * PZ, NM = MX * MY * MZ;
  static constexpr int NQ = RF2 ? NM : 1;
  float ph[NP];
  float pl[LEAN ? 1 : NP];  // low part of phi (FP32 storage)
  float mu[NM];
  float qx[NQ], qy[NQ], qz[NQ];  // RF2: rho u_o over the mu region
};

// Offset of neighbour e_i in a region of row pitch X and plane pitch X * Y.
template <int X, int Y>
__device__ __forceinline__ constexpr int nofs(int i) {
  return EX(i) + X * (EY(i) + Y * EZ(i));
}

// The 18 neighbour values v[1..18] of position pc of an LDS region.
template <int X, int Y>
__device__ __forceinline__ void gather18(const float* f, int pc, float* v) {
#pragma unroll
  for (int i = 1; i < Q; ++i) v[i] = f[pc + nofs<X, Y>(i)];
}

// div q = sum_i 3 w_i e_i . q(x + e_i) of a vector field from its neighbour
// values (lean form: per opposite pair the difference e_{2j-1} . (q_{2j-1} -
// q_{2j}), axis pairs weighted 1/6, edge pairs 1/12).
__device__ __forceinline__ float lean_div(const float* qx, const float* qy, const float* qz) {
  float d[10];
#pragma unroll
  for (int j = 1; j <= 9; ++j) {
    const int i = PI(j);
    d[j] = edot(i, qx[i] - qx[i + 1], qy[i] - qy[i + 1], qz[i] - qz[i + 1]);
  }
  const float a = (d[1] + d[2]) + d[3];
  const float e = ((((d[4] + d[5]) + d[6]) + d[7]) + d[8]) + d[9];
  return __builtin_fmaf(1.0f / 6.0f, a, (1.0f / 12.0f) * e);
}

// rho u_o: rho times the velocity the uncorrected recovery gives (lean form).
__device__ __forceinline__ void lean_rho_uo(const CaseDev& c, float ph, float mu, float gx,
                                            float gy, float gz, float mx, float my, float mz,
                                            float& qx, float& qy, float& qz) {
  const LeanUP r = lean_recover(c, ph, mu, gx, gy, gz, 0.0f, 0.0f, mx, my, mz);
  const float rho = __builtin_fmaf(ph, c.drho, c.rho0);
  qx = rho * r.ux;
  qy = rho * r.uy;
  qz = rho * r.uz;
}

// RF2 (correction from data): also rho u_o over the tile + 1, u_o the
// uncorrected recovery from the moment planes, then at each node the rate
// D = drho (phi - phi^(n-1)) + div(rho u_o), with phi^(n-1) from the plane of
// the current state copy, in place of the Eq. 5 coefficient.  LEAN: the
// evaluation order of 16-bit storage (lbm_d3q19_lean.h), one-float phi.
template <int TX, int TY, int TZ, bool RF2, bool LEAN>
__global__ void __launch_bounds__(TX * TY * TZ)
k3_fields_t(CaseDev c, Fields3 fl, int dump, int parity) {
  using T = FieldTile<TX, TY, TZ, RF2, LEAN>;
  constexpr int PX = T::PX, PY = T::PY, MX = T::MX, MY = T::MY;
  __shared__ T L;
  // XCD-aware tile order: workgroup b runs on XCD b % 8 and takes the b / 8-th
  // tile of that XCD's contiguous chunk (neighbouring tiles share L2).
  const int ntx = (c.nx + TX - 1) / TX, nty = (c.ny + TY - 1) / TY, ntz = (c.nz + TZ - 1) / TZ;
  const int ntiles = ntx * nty * ntz;
  const int chunk = (ntiles + 7) >> 3;
  const int t = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
  if (blockIdx.x >= (unsigned)(8 * chunk) || t >= ntiles) return;
  const int x0 = (t % ntx) * TX, y0 = ((t / ntx) % nty) * TY, z0 = (t / (ntx * nty)) * TZ;
  const int tid = threadIdx.x;
  const bool inner = x0 >= 2 && x0 + TX + 2 <= c.nx && y0 >= 2 && y0 + TY + 2 <= c.ny &&
                     z0 >= 2 && z0 + TZ + 2 <= c.nz;
  // own node (ragged tiles: positions beyond the grid load node 0, unused)
  const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
  const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
  const bool own = gx < c.nx && gy < c.ny && gz < c.nz;
  const unsigned idx = own ? gx + c.nx * (gy + c.ny * gz) : 0u;
  const float m0 = fl.m0[idx], m1x = fl.m1x[idx], m1y = fl.m1y[idx], m1z = fl.m1z[idx];

  // phi over the tile + 2: every load issued before the first LDS store
  constexpr int IP = (T::NP + T::NT - 1) / T::NT;
  float hv[IP], lv[IP];
#pragma unroll
  for (int it = 0; it < IP; ++it) {
    const int k = tid + it * T::NT;
    if (k < T::NP) {
      const int px = k % PX, py = (k / PX) % PY, pz = k / (PX * PY);
      int qx = x0 - 2 + px, qy = y0 - 2 + py, qz = z0 - 2 + pz;
      if (!inner) {
        qx = fold3(qx, c.nx, c.wall_x);
        qy = fold3(qy, c.ny, c.wall_y);
        qz = fold3(qz, c.nz, c.wall_z);
      }
      const unsigned q = qx + c.nx * (qy + c.ny * qz);
      hv[it] = fl.phh[q];
      if constexpr (!LEAN) lv[it] = fl.phl[q];
    }
  }
#pragma unroll
  for (int it = 0; it < IP; ++it) {
    const int k = tid + it * T::NT;
    if (k < T::NP) {
      L.ph[k] = hv[it];
      if constexpr (!LEAN) L.pl[k] = lv[it];
    }
  }
  __syncthreads();

  // mu over the tile + 1
  for (int k = tid; k < T::NM; k += T::NT) {
    int mx = k % MX, my = (k / MX) % MY, mz = k / (MX * MY);
    if (!inner) {
      mx = mirror_local(mx, x0 - 1, c.nx, c.wall_x, MX);
      my = mirror_local(my, y0 - 1, c.ny, c.wall_y, MY);
      mz = mirror_local(mz, z0 - 1, c.nz, c.wall_z, T::MZ);
    }
    const int pc = (mx + 1) + PX * ((my + 1) + PY * (mz + 1));
    if constexpr (LEAN) {
      float v[Q];
      gather18<PX, PY>(L.ph, pc, v);
      const float h0 = L.ph[pc];
      L.mu[k] = lean_mu(c, h0, lean_lap(v, h0));
    } else {
      const float h0 = L.ph[pc], l0 = L.pl[pc];
      float la = 0.0f, le = 0.0f;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int j = pc + nofs<PX, PY>(i);
        const float d = (L.ph[j] - h0) + (L.pl[j] - l0);
        if (i <= 6) la += d;
        else le += d;
      }
      const float lap = (1.0f / 3.0f) * la + (1.0f / 6.0f) * le;
      L.mu[k] = dtheta(c, h0, l0) - c.kappa * lap;
    }
  }
  __syncthreads();

  if constexpr (RF2) {
    // rho u_o over the tile + 1; a position beyond a wall stands for its
    // mirror node (its stencils around the mirror position, as for mu, and
    // the mirror node's moments)
    for (int k = tid; k < T::NM; k += T::NT) {
      const int ax = k % MX, ay = (k / MX) % MY, az = k / (MX * MY);
      int mx = ax, my = ay, mz = az;
      int qx = x0 - 1 + ax, qy = y0 - 1 + ay, qz = z0 - 1 + az;
      if (!inner) {
        mx = mirror_local(mx, x0 - 1, c.nx, c.wall_x, MX);
        my = mirror_local(my, y0 - 1, c.ny, c.wall_y, MY);
        mz = mirror_local(mz, z0 - 1, c.nz, c.wall_z, T::MZ);
        qx = fold3(qx, c.nx, c.wall_x);
        qy = fold3(qy, c.ny, c.wall_y);
        qz = fold3(qz, c.nz, c.wall_z);
      }
      const unsigned q = qx + c.nx * (qy + c.ny * qz);
      const int pc = (mx + 1) + PX * ((my + 1) + PY * (mz + 1));
      const float mu = L.mu[k];
      if constexpr (LEAN) {
        float v[Q], g[3];
        gather18<PX, PY>(L.ph, pc, v);
        lean_grad(v, g[0], g[1], g[2]);
        lean_rho_uo(c, L.ph[pc], mu, g[0], g[1], g[2], fl.m1x[q], fl.m1y[q], fl.m1z[q],
                    L.qx[k], L.qy[k], L.qz[k]);
      } else {
        const float h0 = L.ph[pc], l0 = L.pl[pc];
        float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const int j = pc + nofs<PX, PY>(i);
          const float d = (L.ph[j] - h0) + (L.pl[j] - l0);
          const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);
          if (EX(i)) g[0] += EX(i) > 0 ? w * d : -w * d;
          if (EY(i)) g[1] += EY(i) > 0 ? w * d : -w * d;
          if (EZ(i)) g[2] += EZ(i) > 0 ? w * d : -w * d;
        }
        const float rho = c.rho0 + (h0 + l0) * c.drho;
        const float iden = __builtin_amdgcn_rcpf(rho);
        const float fsz = mu * g[2] - (rho - c.rho_ref) * c.gravity;
        L.qx[k] = rho * ((3.0f * fl.m1x[q] + 0.5f * (mu * g[0])) * iden);
        L.qy[k] = rho * ((3.0f * fl.m1y[q] + 0.5f * (mu * g[1])) * iden);
        L.qz[k] = rho * ((3.0f * fl.m1z[q] + 0.5f * fsz) * iden);
      }
    }
    __syncthreads();
  }

  // the tile's own nodes
  if (!own) return;
  const int pc = (lx + 2) + PX * ((ly + 2) + PY * (lz + 2));
  const int mc = (lx + 1) + MX * ((ly + 1) + MY * (lz + 1));
  const float mu = L.mu[mc];
  if constexpr (LEAN) {
    float v[Q], g[3];
    gather18<PX, PY>(L.ph, pc, v);
    lean_grad(v, g[0], g[1], g[2]);
    const float ph = L.ph[pc];
    float lmu = 0.0f;
    if (dump || c.corr != 0.0f) {
      gather18<MX, MY>(L.mu, mc, v);
      lmu = lean_lap(v, mu);
    }
    float cc = c.corr * lmu;
    if constexpr (RF2) {
      const char* src = parity ? c.state[1] : c.state[0];
      float qx[Q], qy[Q], qz[Q];
      gather18<MX, MY>(L.qx, mc, qx);
      gather18<MX, MY>(L.qy, mc, qy);
      gather18<MX, MY>(L.qz, mc, qz);
      cc = __builtin_fmaf(ph - gload<float>(src, c.phiv + 4u * idx), c.drho,
                          lean_div(qx, qy, qz));
      plane_put(fl.dd, idx, cc);
    }
    const LeanUP r = lean_recover(c, ph, mu, g[0], g[1], g[2], cc, m0, m1x, m1y, m1z);
    if (dump) fl.mu[idx] = mu;
    plane_put(fl.ux, idx, r.ux);
    plane_put(fl.uy, idx, r.uy);
    plane_put(fl.uz, idx, r.uz);
    plane_put(fl.p, idx, r.p);
    plane_put(fl.lmu, idx, lmu);
    return;
  } else {
    const float h0 = L.ph[pc], l0 = L.pl[pc];
    float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int j = pc + nofs<PX, PY>(i);
      const float d = (L.ph[j] - h0) + (L.pl[j] - l0);
      const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);  // 3 w_i
      if (EX(i)) g[0] += EX(i) > 0 ? w * d : -w * d;
      if (EY(i)) g[1] += EY(i) > 0 ? w * d : -w * d;
      if (EZ(i)) g[2] += EZ(i) > 0 ? w * d : -w * d;
    }
    float lmu = 0.0f;
    if (dump || c.corr != 0.0f) {
      float la = 0.0f, le = 0.0f;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const float d = L.mu[mc + nofs<MX, MY>(i)] - mu;
        if (i <= 6) la += d;
        else le += d;
      }
      lmu = (1.0f / 3.0f) * la + (1.0f / 6.0f) * le;
    }
    const float ph = h0 + l0;
    const float rho = c.rho0 + ph * c.drho;
    // (rho - c/2) u = 3 sum e gbar + (F_s + G)/2, gravity along -z
    const float fsx = mu * g[0], fsy = mu * g[1];
    const float fsz = mu * g[2] - (rho - c.rho_ref) * c.gravity;
    float cc = c.corr * lmu;
    if constexpr (RF2) {
      const char* src = parity ? c.state[1] : c.state[0];
      float dv = 0.0f;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int j = mc + nofs<MX, MY>(i);
        const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);  // 3 w_i
        float e = 0.0f;
        if (EX(i)) e += EX(i) > 0 ? L.qx[j] : -L.qx[j];
        if (EY(i)) e += EY(i) > 0 ? L.qy[j] : -L.qy[j];
        if (EZ(i)) e += EZ(i) > 0 ? L.qz[j] : -L.qz[j];
        dv += w * e;
      }
      cc = (ph - gload<float>(src, c.phiv + 4u * idx)) * c.drho + dv;
      plane_put(fl.dd, idx, cc);
    }
    const float iden = __builtin_amdgcn_rcpf(rho - 0.5f * cc);
    const float ux = (3.0f * m1x + 0.5f * fsx) * iden;
    const float uy = (3.0f * m1y + 0.5f * fsy) * iden;
    const float uz = (3.0f * m1z + 0.5f * fsz) * iden;
    // mu for the field dump only: the collision forms mu and grad phi again from
    // the phi planes (phi_grad_mu), with these expressions in this order
    if (dump) fl.mu[idx] = mu;
    plane_put(fl.ux, idx, ux);
    plane_put(fl.uy, idx, uy);
    plane_put(fl.uz, idx, uz);
    plane_put(fl.p, idx, m0 + (1.0f / 6.0f) * c.drho * (ux * g[0] + uy * g[1] + uz * g[2]));
    plane_put(fl.lmu, idx, lmu);
  }
}

// ---- 4: collision and store
// Per-node inputs of the collision (all at the node itself, ∇p included).
struct NodeFields {
  float phh, phl, mu, cc, p, ux, uy, uz, gx, gy, gz, gpx, gpy, gpz;  // cc: -F_a = cc u
};

// grad psi, the regrouped BGK collision of f and gbar with the Eq. 8 forcing
// (see the D2Q9 step):
//   g* = (1 - om) g + w [A + B_i + t_i (C + D_i)],  f* = (1 - om_f) f + w (P + Q t_i)
// and the stores of node idx.  fv[1..18], gv[0..18]: its pulled populations.
// Destination of the stores by the copy's base address alone (each store forms
// its plane offset), for kernels short of scalar registers; the same stores as
// OutPtrs.
template <int S>
struct BaseOut {
  char* base;
  __device__ __forceinline__ float put_f(const CaseDev& c, int i, unsigned idx, float v) const {
    return Pops<S, Q>::put_f(c, base, i, idx, v);
  }
  __device__ __forceinline__ void put_g(const CaseDev& c, int i, unsigned idx, float v,
                                        float wi, uint32_t) const {
    static_assert(S == ST_FP32, "16-bit steps store through lean_collide");
    Pops<S, Q>::put_g(c, base, i, idx, v, wi);
  }
  __device__ __forceinline__ void put_f0(const CaseDev& c, unsigned idx, float hi,
                                         float lo) const {
    Pops<S, Q>::put_f0(c, base, idx, hi, lo);
  }
};

template <int S>
__device__ __forceinline__ void put_f0(const CaseDev&, const OutPtrs<S, Q>& op, unsigned idx,
                                       float hi, float lo) {
  op.put_f0(idx, hi, lo);
}
template <int S>
__device__ __forceinline__ void put_f0(const CaseDev& c, const BaseOut<S>& op, unsigned idx,
                                       float hi, float lo) {
  op.put_f0(c, idx, hi, lo);
}

template <int S, class Out>
__device__ __forceinline__ void collide_node(const CaseDev& c, const Out& op,
                                             unsigned idx, const float* fv, const float* gv,
                                             const NodeFields& n) {
  const float ph = n.phh + n.phl;
  const float ux = n.ux, uy = n.uy, uz = n.uz, p = n.p, mu = n.mu;
  const float rho = c.rho0 + ph * c.drho;
  const float cc = n.cc;
  const float fx = mu * n.gx + cc * ux;
  const float fy = mu * n.gy + cc * uy;
  const float fz = mu * n.gz - (rho - c.rho_ref) * c.gravity + cc * uz;
  const float gpsx = n.gpx - (1.0f / 3.0f) * c.drho * n.gx;
  const float gpsy = n.gpy - (1.0f / 3.0f) * c.drho * n.gy;
  const float gpsz = n.gpz - (1.0f / 3.0f) * c.drho * n.gz;
  const float mud = c.mu0 + ph * c.dmu;
  const float om = rho * __builtin_amdgcn_rcpf(0.5f * rho + 3.0f * mud);  // 1 / tau
  const float half = 1.0f - 0.5f * om;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float uf = ux * fx + uy * fy + uz * fz;
  const float ug = ux * gpsx + uy * gpsy + uz * gpsz;
  const float A = om * p - half * uf;
  const float Cc = om * (1.0f / 3.0f) * rho - half * uf + half * ug;
  const float hfx = half * fx, hfy = half * fy, hfz = half * fz;
  const float hdx = half * (fx - gpsx), hdy = half * (fy - gpsy), hdz = half * (fz - gpsz);
  const float m15 = -1.5f * uu;
  const float omg = 1.0f - om;
  const float omf = 1.0f - c.omega_f;
  const float fP = c.omega_f * c.gamma3 * mu;
  const float fQ = c.omega_f * ph;
  float fsum = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float eu = (EX(i) ? (EX(i) > 0 ? ux : -ux) : 0.0f) +
                     (EY(i) ? (EY(i) > 0 ? uy : -uy) : 0.0f) +
                     (EZ(i) ? (EZ(i) > 0 ? uz : -uz) : 0.0f);
    const float bi = (EX(i) ? (EX(i) > 0 ? hfx : -hfx) : 0.0f) +
                     (EY(i) ? (EY(i) > 0 ? hfy : -hfy) : 0.0f) +
                     (EZ(i) ? (EZ(i) > 0 ? hfz : -hfz) : 0.0f);
    const float di = (EX(i) ? (EX(i) > 0 ? hdx : -hdx) : 0.0f) +
                     (EY(i) ? (EY(i) > 0 ? hdy : -hdy) : 0.0f) +
                     (EZ(i) ? (EZ(i) > 0 ? hdz : -hdz) : 0.0f);
    const float ti = eu * (3.0f + 4.5f * eu) + m15;
    if (i > 0) {
      const float fn = omf * fv[i] + WT(i) * (fP + fQ * ti);
      fsum += op.put_f(c, i, idx, fn);
    }
    const float gn = omg * gv[i] + WT(i) * ((A + bi) + ti * (Cc + di));
    op.put_g(c, i, idx, gn, WT(i), 0u);  // FP32 storage only (16-bit: lean_collide)
  }
  float h0, e0;
  two_sum(n.phh, -fsum, h0, e0);
  put_f0<S>(c, op, idx, h0, e0 + n.phl);
}

template <int S>
__device__ __forceinline__ void pull_node(const CaseDev& c, const char* src, const Node3& nd,
                                          float* fv, float* gv) {
  using N = Node3;
  using P = Pops<S, Q>;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (i > 0) fv[i] = P::f(c, src, i, pull3<S, false, N>(c, nd, i));
    gv[i] = P::g(c, src, pull3<S, true, N>(c, nd, i), WT(i));
  }
}

// The pulled f_1..f_18 of a node, and its phi from them as pull_phi forms it.
template <int S, class N>
__device__ __forceinline__ void pull_f(const CaseDev& c, const char* src, const N& nd,
                                       float* fv) {
  using P = Pops<S, Q>;
#pragma unroll
  for (int i = 1; i < Q; ++i) fv[i] = P::f(c, src, i, pull3<S, false, N>(c, nd, i));
}
template <int S, class N>
__device__ __forceinline__ void phi_of(const CaseDev& c, const char* src, const N& nd,
                                       const float* fv, float& hi, float& lo) {
  using P = Pops<S, Q>;
  float sm = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) sm += fv[i];
  two_sum(P::f(c, src, 0, P::fofs(c, 0, nd.idx)), P::f0lo(c, src, nd.idx) + sm, hi, lo);
}
template <int S, class N>
__device__ __forceinline__ void pull_g(const CaseDev& c, const char* src, const N& nd,
                                       float* gv) {
  using P = Pops<S, Q>;
#pragma unroll
  for (int i = 0; i < Q; ++i) gv[i] = P::g(c, src, pull3<S, true, N>(c, nd, i), WT(i));
}

// phi (float-float), grad phi and mu = theta'(phi) - kappa lap phi of a node
// from the phi planes: the fields kernel's expressions, summed in its order
// over the same neighbour values (mirror node across a wall, image across a
// periodic seam), so the same bits as the values it formed in LDS.
__device__ __forceinline__ void phi_grad_mu(const CaseDev& c, const Fields3& fl, const Node3& nd,
                                            NodeFields& n) {
  const float h0 = fl.phh[nd.idx], l0 = fl.phl[nd.idx];
  float la = 0.0f, le = 0.0f;
  float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const unsigned j = nbr3(c, nd, i);
    const float d = (fl.phh[j] - h0) + (fl.phl[j] - l0);
    if (i <= 6) la += d;
    else le += d;
    const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);  // 3 w_i
    if (EX(i)) g[0] += EX(i) > 0 ? w * d : -w * d;
    if (EY(i)) g[1] += EY(i) > 0 ? w * d : -w * d;
    if (EZ(i)) g[2] += EZ(i) > 0 ? w * d : -w * d;
  }
  const float lap = (1.0f / 3.0f) * la + (1.0f / 6.0f) * le;
  n.phh = h0;
  n.phl = l0;
  n.mu = dtheta(c, h0, l0) - c.kappa * lap;
  n.gx = g[0];
  n.gy = g[1];
  n.gz = g[2];
}

// Stores of one node in the 16-bit layout from the packed results of
// lean_collide: f_0 as a float, f_{2j-1} / f_{2j} from the low / high half of
// of[j], g_{2k} / g_{2k+1} from og[k] (g_18 in the low half of og[9]).
template <int S>
__device__ __forceinline__ void store_lean(const CaseDev& c, char* dst, unsigned idx, float f0,
                                           const uint32_t* og, const uint32_t* of) {
  using P = Pops<S, Q>;
  gstore_nt<float>(dst, 4u * idx, f0);
#pragma unroll
  for (int j = 1; j <= 9; ++j) {
    gstore_nt<uint16_t>(dst, P::fofs(c, PI(j), idx), (uint16_t)(of[j] & 0xffffu));
    gstore_nt<uint16_t>(dst, P::fofs(c, PI(j) + 1, idx), (uint16_t)(of[j] >> 16));
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    gstore_nt<uint16_t>(dst, P::gofs(c, 2 * k, idx), (uint16_t)(og[k] & 0xffffu));
    if (2 * k + 1 < Q)
      gstore_nt<uint16_t>(dst, P::gofs(c, 2 * k + 1, idx), (uint16_t)(og[k] >> 16));
  }
}

template <int S>
__global__ void __launch_bounds__(256) k3_collide(CaseDev c, int parity, Fields3 fl) {
  const int x = blockIdx.y * blockDim.x + threadIdx.x;
  if (x >= c.nx) return;
  const Node3 nd(c, x, blockIdx.x);
  const unsigned idx = nd.idx;
  const char* src = parity ? c.state[1] : c.state[0];
  char* dst = parity ? c.state[0] : c.state[1];
  if constexpr (S != ST_FP32) {
    // 16-bit storage: the lean form (lbm_d3q19_lean.h)
    uint16_t fh[Q], gh[Q + 1];
    float v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (i > 0) fh[i] = gload<uint16_t>(src, pull3<S, false>(c, nd, i));
      gh[i] = gload<uint16_t>(src, pull3<S, true>(c, nd, i));
    }
    gh[Q] = 0;
    uint32_t Fr[10], Gr[10];
#pragma unroll
    for (int j = 1; j <= 9; ++j) Fr[j] = pack16(fh[PI(j)], fh[PI(j) + 1]);
#pragma unroll
    for (int k = 0; k < 10; ++k) Gr[k] = pack16(gh[2 * k], gh[2 * k + 1]);
    LeanNode n;
    n.ph = fl.phh[idx];
#pragma unroll
    for (int i = 1; i < Q; ++i) v[i] = fl.phh[nbr3(c, nd, i)];
    lean_grad(v, n.gx, n.gy, n.gz);
    n.mu = lean_mu(c, n.ph, lean_lap(v, n.ph));
#pragma unroll
    for (int i = 1; i < Q; ++i) v[i] = fl.p[nbr3(c, nd, i)];
    float gp[3];
    lean_grad(v, gp[0], gp[1], gp[2]);
    n.cc = c.phiv ? fl.dd[idx] : c.corr * fl.lmu[idx];
    n.p = fl.p[idx];
    n.ux = fl.ux[idx];
    n.uy = fl.uy[idx];
    n.uz = fl.uz[idx];
    uint32_t og[10], of[10];
    const uint32_t nkey = sr_node_key(sr_step_key(sr_clock(c, parity)), idx);
    const float f0 = lean_collide<S>(c, n, gp[0], gp[1], gp[2], Gr, Fr, og, of, nkey);
    store_lean<S>(c, dst, idx, f0, og, of);
    if (c.phiv) gstore_nt<float>(dst, c.phiv + 4u * idx, n.ph);
    return;
  }
  const OutPtrs<S, Q> op(c, dst);
  float fv[Q], gv[Q];
  pull_node<S>(c, src, nd, fv, gv);
  float gp[3];
  grad_f(c, fl.p, nd, gp);
  NodeFields n;
  phi_grad_mu(c, fl, nd, n);
  n.cc = c.phiv ? fl.dd[idx] : c.corr * fl.lmu[idx];
  n.p = fl.p[idx];
  n.ux = fl.ux[idx];
  n.uy = fl.uy[idx];
  n.uz = fl.uz[idx];
  n.gpx = gp[0];
  n.gpy = gp[1];
  n.gpz = gp[2];
  collide_node<S>(c, op, idx, fv, gv, n);
  // correction from data: the copy carries this step's phi
  if (c.phiv) gstore_nt<float>(dst, c.phiv + 4u * idx, n.phh + n.phl);
}

// ---- 2+3+4 as one march (16-bit storage): k3_fcm
//
// The step's second kernel after k3_pull.  A workgroup owns a TX x TY tile
// of the x-y plane and the planes [za, zb) of one z chunk, and keeps rings of
// planes in LDS:
//   phi over the tile + 3, 4 planes (read from the plane k3_pull wrote)
//   mu over the tile + 2, 3 planes
//   p over the tile + 1, 3 planes
// Iteration z stages phi(z + 3), forms mu(z + 2), forms grad phi, lap mu, u
// and p at z + 1 from the moment planes of k3_pull (the own node keeps its
// fields in registers for the next iteration), then collides plane z with
// the own node's pulled populations.  No field plane goes back to HBM and the
// stencils of the collision read LDS.  Every quantity is the same expression
// in the same order as in k3_fields_t and k3_collide, so the step gives the
// bits of the three-kernel step.
//
// Positions beyond a wall: phi is staged from the mirror node (periodic image
// on periodic axes); in the x-y plane mu, u and p at such a position are
// formed around the mirror position with the mirror node's moments, so they
// equal the mirror node's values; along z the planes beyond a wall are not
// formed and their reads go to the mirror plane.
//
// RF2 (correction from data): the mu stage also forms rho u_o, the
// uncorrected recovery, over the tile + 2 (a ring of 3 planes, from the
// gbar moment planes), and the u, p stage takes as the coefficient of -F_a
// the rate D = drho (phi - phi^(n-1)) + div(rho u_o), with phi^(n-1) from the
// phi plane of the source copy, as k3_fields_t does; the collision writes
// phi to the phi plane of the destination copy, as k3_collide does.
template <int TX, int TY, bool RF2>
struct FcmLds {
  static constexpr int PX = TX + 6, PY = TY + 6, NP = PX * PY;  // phi, tile + 3
  static constexpr int MX = TX + 4, MY = TY + 4, NM = MX * MY;  // mu, tile + 2
  static constexpr int UX = TX + 2, UY = TY + 2, NU = UX * UY;  // p, tile + 1
  static constexpr int NQ = RF2 ? NM : 1;
  float ph[4][NP];
  float mu[3][NM];
  float p[3][NU];
  float q[3][3][NQ];  // RF2: rho u_o, plane slot x component
};

// 64-wide tiles ask for 3 waves per SIMD (at most 168 VGPRs): BF16 decoding
// otherwise needs one register more and runs at 2
template <int S, int TX, int TY, bool RF2>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(TX == 64 ? 3 : 1)))
k3_fcm(CaseDev c, int parity, Fields3 fl, int zc) {
  static_assert(S != ST_FP32, "the lean arithmetic of 16-bit storage");
  using T = FcmLds<TX, TY, RF2>;
  constexpr int NT = TX * TY, PX = T::PX, MX = T::MX, MY = T::MY, UX = T::UX, UY = T::UY;
  constexpr int KP = (T::NP + NT - 1) / NT;      // phi positions per thread (at most)
  constexpr int NRING = T::NU - NT;              // u, p positions outside the tile
  constexpr int KU = 1 + (NRING + NT - 1) / NT;  // u, p positions per thread: own + ring
  __shared__ T L;
  // every workgroup reads the step counter; workgroup 0 advances it
  const uint32_t skey = sr_step_key(sr_clock(c, parity));
  // XCD-aware tile order: workgroup b runs on XCD b % 8 and takes the b / 8-th
  // tile of that XCD's contiguous chunk (x fastest, then y, then the z chunk)
  const int ntx = (c.nx + TX - 1) / TX, nty = (c.ny + TY - 1) / TY, ntz = (c.nz + zc - 1) / zc;
  const int ntiles = ntx * nty * ntz;
  const int chunk = (ntiles + 7) >> 3;
  const int t = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
  if (blockIdx.x >= (unsigned)(8 * chunk) || t >= ntiles) return;
  const int x0 = (t % ntx) * TX, y0 = ((t / ntx) % nty) * TY, za = (t / (ntx * nty)) * zc;
  const int zb = min(za + zc, c.nz);
  const int tid = threadIdx.x;
  // no x-y position of the phi region needs the periodic or mirror mapping
  const bool inner = x0 >= 3 && x0 + TX + 3 <= c.nx && y0 >= 3 && y0 + TY + 3 <= c.ny;
  const int lx = tid % TX, ly = tid / TX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool own = gx < c.nx && gy < c.ny;
  const unsigned pln = (unsigned)(c.nx * c.ny);
  const char* src = parity ? c.state[1] : c.state[0];
  char* dst = parity ? c.state[0] : c.state[1];
  auto s4 = [](int k) { return (k + 8) & 3; };  // ring slots (k >= -6)
  auto s3 = [](int k) { return (k + 6) % 3; };
  auto zr = [&](int k) { return c.wall_z ? min(max(k, 0), c.nz - 1) : k; };
  auto beyond = [&](int k) { return c.wall_z && (k < 0 || k >= c.nz); };

  // x-y source node of each phi position this thread stages
  unsigned psrc[KP];
#pragma unroll
  for (int it = 0; it < KP; ++it) {
    const int k = tid + it * NT;
    int qx = x0 - 3 + k % PX, qy = y0 - 3 + k / PX;
    if (!inner) {
      qx = fold3(qx, c.nx, c.wall_x);
      qy = fold3(qy, c.ny, c.wall_y);
    }
    psrc[it] = k < T::NP ? (unsigned)(qx + c.nx * qy) : 0u;
  }
  // u, p positions of this thread: its own node, then ring positions (top
  // row, bottom row, then the two side columns row by row).  upos: the
  // position; ust: the position whose stencils it takes (its mirror beyond
  // a wall); usrc: x-y offset of the node whose moments it takes.
  int upos[KU], ust[KU];
  unsigned usrc[KU];
  bool uon[KU];
#pragma unroll
  for (int q = 0; q < KU; ++q) {
    const int r = tid + (q - 1) * NT;
    int ux = 0, uy = 0;
    uon[q] = q == 0 || r < NRING;
    if (q == 0) {
      ux = lx + 1;
      uy = ly + 1;
    } else if (r < UX) {
      ux = r;
    } else if (r < 2 * UX) {
      ux = r - UX;
      uy = UY - 1;
    } else if (r < NRING) {
      const int w = r - 2 * UX;
      ux = (w & 1) ? UX - 1 : 0;
      uy = 1 + (w >> 1);
    }
    upos[q] = ux + UX * uy;
    int sx = ux, sy = uy, qx = x0 - 1 + ux, qy = y0 - 1 + uy;
    if (!inner) {
      sx = mirror_local(sx, x0 - 1, c.nx, c.wall_x, UX);
      sy = mirror_local(sy, y0 - 1, c.ny, c.wall_y, UY);
      qx = fold3(qx, c.nx, c.wall_x);
      qy = fold3(qy, c.ny, c.wall_y);
    }
    ust[q] = sx + UX * sy;
    usrc[q] = (unsigned)(qx + c.nx * qy);
  }

  float hv[KP];  // phi plane in flight
  auto load_phi = [&](int k) {
    const unsigned zo = pln * (unsigned)fold3(k, c.nz, c.wall_z);
#pragma unroll
    for (int it = 0; it < KP; ++it)
      if (tid + it * NT < T::NP) hv[it] = fl.phh[zo + psrc[it]];
  };
  auto store_phi = [&](int k) {
    float* d = L.ph[s4(k)];
#pragma unroll
    for (int it = 0; it < KP; ++it)
      if (tid + it * NT < T::NP) d[tid + it * NT] = hv[it];
  };
  float mv[KU][4];  // gbar moments of the u, p positions, one plane ahead
  float pv[KU];     // RF2: phi^(n-1) of the u, p positions, one plane ahead
  auto load_m = [&](int k) {
    if (beyond(k)) return;
    const unsigned zo = pln * (unsigned)fold3(k, c.nz, c.wall_z);
#pragma unroll
    for (int q = 0; q < KU; ++q) {
      if (!uon[q]) continue;
      const unsigned j = zo + usrc[q];
      mv[q][0] = fl.m0[j];
      mv[q][1] = fl.m1x[j];
      mv[q][2] = fl.m1y[j];
      mv[q][3] = fl.m1z[j];
      if constexpr (RF2) pv[q] = gload<float>(src, c.phiv + 4u * j);
    }
  };
  // mu at plane k over the tile + 2 (k3_fields_t's mu stage)
  auto mu_plane = [&](int k) {
    if (beyond(k)) return;
    const float* pm = L.ph[s4(k - 1)];
    const float* p0 = L.ph[s4(k)];
    const float* pp = L.ph[s4(k + 1)];
    float* d = L.mu[s3(k)];
    const unsigned zo = RF2 ? pln * (unsigned)fold3(k, c.nz, c.wall_z) : 0u;
    for (int pos = tid; pos < T::NM; pos += NT) {
      int mx = pos % MX, my = pos / MX;
      // RF2: the node whose moments the position takes (mirror beyond a wall)
      int qx = x0 - 2 + mx, qy = y0 - 2 + my;
      if (!inner) {
        mx = mirror_local(mx, x0 - 2, c.nx, c.wall_x, MX);
        my = mirror_local(my, y0 - 2, c.ny, c.wall_y, MY);
      }
      const int pc = (mx + 1) + PX * (my + 1);
      float v[Q];
#pragma unroll
      for (int i = 1; i < Q; ++i)
        v[i] = (EZ(i) < 0 ? pm : (EZ(i) > 0 ? pp : p0))[pc + EX(i) + PX * EY(i)];
      const float h0 = p0[pc];
      const float mu = lean_mu(c, h0, lean_lap(v, h0));
      d[pos] = mu;
      if constexpr (RF2) {
        // rho u_o at the position (k3_fields_t's RF2 stage)
        if (!inner) {
          qx = fold3(qx, c.nx, c.wall_x);
          qy = fold3(qy, c.ny, c.wall_y);
        }
        const unsigned j = zo + (unsigned)(qx + c.nx * qy);
        float g[3];
        lean_grad(v, g[0], g[1], g[2]);
        lean_rho_uo(c, h0, mu, g[0], g[1], g[2], fl.m1x[j], fl.m1y[j], fl.m1z[j],
                    L.q[s3(k)][0][pos], L.q[s3(k)][1][pos], L.q[s3(k)][2][pos]);
      }
    }
  };
  // grad phi, lap mu, u and p at plane k over the tile + 1 (k3_fields_t's
  // own-node stage); the own node's values go to nxt
  LeanNode nxt{};
  auto up_plane = [&](int k) {
    if (beyond(k)) return;
    float* dp = L.p[s3(k)];
#pragma unroll
    for (int q = 0; q < KU; ++q) {
      if (!uon[q]) continue;
      const int sx = ust[q] % UX, sy = ust[q] / UX;
      const int pc = (sx + 2) + PX * (sy + 2), mc = (sx + 1) + MX * (sy + 1);
      float v[Q], g[3];
#pragma unroll
      for (int i = 1; i < Q; ++i) v[i] = L.ph[s4(k + EZ(i))][pc + EX(i) + PX * EY(i)];
      lean_grad(v, g[0], g[1], g[2]);
      const float ph = L.ph[s4(k)][pc];
      const float mu = L.mu[s3(k)][mc];
      float cc;
      if constexpr (RF2) {
        // D = drho (phi - phi^(n-1)) + div(rho u_o) (k3_fields_t's RF2 rate)
        float qx[Q], qy[Q], qz[Q];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const int sl = s3(zr(k + EZ(i))), o = mc + EX(i) + MX * EY(i);
          qx[i] = L.q[sl][0][o];
          qy[i] = L.q[sl][1][o];
          qz[i] = L.q[sl][2][o];
        }
        cc = __builtin_fmaf(ph - pv[q], c.drho, lean_div(qx, qy, qz));
      } else {
        float lmu = 0.0f;
        if (c.corr != 0.0f) {
#pragma unroll
          for (int i = 1; i < Q; ++i) v[i] = L.mu[s3(zr(k + EZ(i)))][mc + EX(i) + MX * EY(i)];
          lmu = lean_lap(v, mu);
        }
        cc = c.corr * lmu;
      }
      const LeanUP r =
          lean_recover(c, ph, mu, g[0], g[1], g[2], cc, mv[q][0], mv[q][1], mv[q][2], mv[q][3]);
      dp[upos[q]] = r.p;
      if (q == 0) {
        nxt.ph = ph;
        nxt.mu = mu;
        nxt.cc = cc;
        nxt.p = r.p;
        nxt.ux = r.ux;
        nxt.uy = r.uy;
        nxt.uz = r.uz;
        nxt.gx = g[0];
        nxt.gy = g[1];
        nxt.gz = g[2];
      }
    }
  };

  // prologue: phi(za - 3) and phi(za - 2) staged, phi(za - 1) in flight; the
  // first four iterations only fill the rings
  load_phi(za - 3);
  store_phi(za - 3);
  load_phi(za - 2);
  store_phi(za - 2);
  load_phi(za - 1);
  const int uc = (lx + 1) + UX * (ly + 1);
  for (int z = za - 4; z < zb; ++z) {
    // the own node's pulled populations for the collision of plane z, issued
    // first so that they arrive while the stages run
    const bool coll = own && z >= za;
    const unsigned idx = (unsigned)(gx + c.nx * (gy + c.ny * z));
    uint16_t fh[Q], gh[Q + 1];
    if (coll) {
      const Node3 nd(c, gx, gy, z);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (i > 0) fh[i] = gload<uint16_t>(src, pull3<S, false>(c, nd, i));
        gh[i] = gload<uint16_t>(src, pull3<S, true>(c, nd, i));
      }
    }
    store_phi(z + 3);
    if (z + 4 <= zb + 2) load_phi(z + 4);
    __syncthreads();
    if (z + 2 >= za - 2) mu_plane(z + 2);
    __syncthreads();
    const LeanNode cur = nxt;  // the own node's fields at plane z
    if (z + 1 >= za - 1) up_plane(z + 1);
    if (z + 2 >= za - 1 && z + 2 <= zb) load_m(z + 2);
    __syncthreads();
    if (coll) {
      gh[Q] = 0;
      uint32_t Fr[10], Gr[10];
      Fr[0] = 0u;
#pragma unroll
      for (int j = 1; j <= 9; ++j) Fr[j] = pack16(fh[PI(j)], fh[PI(j) + 1]);
#pragma unroll
      for (int k = 0; k < 10; ++k) Gr[k] = pack16(gh[2 * k], gh[2 * k + 1]);
      float v[Q], gp[3];
#pragma unroll
      for (int i = 1; i < Q; ++i) v[i] = L.p[s3(zr(z + EZ(i)))][uc + EX(i) + UX * EY(i)];
      lean_grad(v, gp[0], gp[1], gp[2]);
      uint32_t og[10], of[10];
      const float f0 = lean_collide<S>(c, cur, gp[0], gp[1], gp[2], Gr, Fr, og, of,
                                       sr_node_key(skey, idx));
      store_lean<S>(c, dst, idx, f0, og, of);
      // correction from data: the copy carries this step's phi
      if constexpr (RF2) gstore_nt<float>(dst, c.phiv + 4u * idx, cur.ph);
    }
  }
}

// ---- fused step: one x-y tile of the grid marching up a chunk of z planes
//
// A workgroup owns a TX x TY tile of the x-y plane and the planes [za, zb) of
// one z chunk.  It keeps rings of planes in LDS:
//   phi (float-float) over the tile + 3, 4 planes  (summed from pulled f)
//   mu over the tile + 2, 3 planes
//   p over the tile + 1, 3 planes
// and iteration z stages phi(z + 3), forms mu(z + 2), pulls the gbar moments
// and forms u and p at z + 1 (the tile's own nodes keep u, grad phi, mu and the
// correction coefficient in registers), then collides plane z.  No field plane
// goes through HBM, and each population is fetched from it about once: a
// thread keeps its own node's pulled f_1..f_18 in registers from the phi stage
// to the collision three planes later, reads that node's gbar again at the top
// of the next iteration while it is still in L2, and the halo positions mostly
// hit L2.
//
// Positions beyond a wall: phi is staged from the mirror node (periodic image
// on periodic axes); in the x-y plane mu, u and p at such a position are
// formed around the mirror position, so they equal the mirror node's values;
// along z the planes beyond a wall are not formed and their reads go to the
// mirror plane (a halfway wall mirrors the plane next to it).  Every quantity
// is the same expression, in the same order, as in the three-kernel step, so
// the two give the same bits.
//
// RF2 (correction from data): the mu stage also pulls the gbar moments and
// forms rho u_o, the uncorrected recovery, over the tile + 2 (a ring of 3
// planes; the moments go to a ring of 2, which the u and p stage of the next
// plane reads instead of pulling again), and the u and p stage takes as the
// coefficient of -F_a the rate
// D = drho (phi - phi^(n-1)) + div(rho u_o) in place of the Eq. 5 one, with
// phi^(n-1) from the plane of the source copy; the collision writes phi to the
// plane of the destination copy.  The divergence replaces lap mu, so the
// pipeline keeps its depth.
template <int TX, int TY, bool RF2>
struct SlabLds {
  static constexpr int PX = TX + 6, PY = TY + 6, NP = PX * PY;  // phi plane
  static constexpr int MX = TX + 4, MY = TY + 4, NM = MX * MY;  // mu plane
  static constexpr int UX = TX + 2, UY = TY + 2, NU = UX * UY;  // p plane
  static constexpr int NQ = RF2 ? NM : 1;
  float ph[4][NP];
  float pl[4][NP];
  float mu[3][NM];
  float p[3][NU];
  float q[3][3][NQ];  // RF2: rho u_o, plane slot x component
  float m[2][4][NQ];  // RF2: the gbar moments m0, m1 behind it, for the u, p stage
};

// Ring slot of plane k (k >= -6).
__device__ __forceinline__ int slot4(int k) { return (k + 8) & 3; }
__device__ __forceinline__ int slot3(int k) { return (k + 6) % 3; }

// The plane whose mu / p a read of plane k takes: k itself, or across a wall
// along z the mirror plane.
__device__ __forceinline__ int zread(const CaseDev& c, int k) {
  return c.wall_z ? min(max(k, 0), c.nz - 1) : k;
}

// mu = theta'(phi) - kappa lap phi at position pc of a phi plane of row pitch
// PX; bm, b0, bp: offsets of the planes below, at and above.
template <int PX>
__device__ __forceinline__ float slab_mu(const CaseDev& c, const float* ph, const float* pl,
                                         int bm, int b0, int bp, int pc) {
  const float h0 = ph[b0 + pc], l0 = pl[b0 + pc];
  float la = 0.0f, le = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int j = (EZ(i) < 0 ? bm : (EZ(i) > 0 ? bp : b0)) + pc + EX(i) + PX * EY(i);
    const float d = (ph[j] - h0) + (pl[j] - l0);
    if (i <= 6) la += d;
    else le += d;
  }
  const float lap = (1.0f / 3.0f) * la + (1.0f / 6.0f) * le;
  return dtheta(c, h0, l0) - c.kappa * lap;
}

template <int S, int TX, int TY, bool RF2>
__global__ void __launch_bounds__(TX * TY) k3_slab(CaseDev c, int parity, int zs) {
  using T = SlabLds<TX, TY, RF2>;
  constexpr int NT = TX * TY, PX = T::PX, PY = T::PY, MX = T::MX, UX = T::UX, UY = T::UY;
  constexpr int NPRING = T::NP - NT;  // positions of the tile + 3 outside the tile
  constexpr int NRING = T::NU - NT;   // positions of the tile + 1 outside the tile
  __shared__ T L;
  // XCD-aware tile order as in the fields kernel; x fastest, then y, then the
  // z chunk, so an XCD's consecutive tiles share their x-y halos
  const int ntx = (c.nx + TX - 1) / TX, nty = (c.ny + TY - 1) / TY;
  const int ntiles = ntx * nty * ((c.nz + zs - 1) / zs);
  const int chunk = (ntiles + 7) >> 3;
  const int t = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
  if (blockIdx.x >= (unsigned)(8 * chunk) || t >= ntiles) return;
  const int x0 = (t % ntx) * TX, y0 = ((t / ntx) % nty) * TY;
  const int za = (t / (ntx * nty)) * zs, zb = min(za + zs, c.nz);
  const int tid = threadIdx.x;
  const bool inner = x0 >= 3 && x0 + TX + 3 <= c.nx && y0 >= 3 && y0 + TY + 3 <= c.ny;
  const int lx = tid % TX, ly = tid / TX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool own = gx < c.nx && gy < c.ny;
  const char* src = parity ? c.state[1] : c.state[0];
  const BaseOut<S> op{parity ? c.state[0] : c.state[1]};
  float* const php = &L.ph[0][0];
  float* const plp = &L.pl[0][0];
  float* const mup = &L.mu[0][0];
  float* const pp = &L.p[0][0];

  NodeFields cur{}, nxt{};  // own node: plane z (collided now), plane z + 1
  // own node's pulled f_1..f_18 at planes z, z + 1, z + 2 and z + 3 (fn)
  float fa[Q], fb[Q], fc[Q], fn[Q];
  for (int z = za - 6; z < zb; ++z) {
    // the own node's gbar for the collision at the end of the iteration: issued
    // first, so the loads complete while phi, mu, u and p are formed
    float gv[Q];
    if (z >= za && own) pull_g<S>(c, src, Node3(c, gx, gy, z), gv);
    // P: phi at plane z + 3 over the tile + 3: first each thread's own node,
    // whose pulled f_1..f_18 it keeps for the collision of that plane three
    // iterations later, then the 3-wide ring around the tile
    {
      const int k = z + 3;
      const int qz = fold3(k, c.nz, c.wall_z);
      const int b = slot4(k) * T::NP;
      for (int r = tid - NT; r < NPRING; r += NT) {
        int px, py;
        if (r < 0) {
          px = lx + 3;
          py = ly + 3;
        } else if (r < 3 * PX) {
          px = r % PX;
          py = r / PX;
        } else if (r < 6 * PX) {
          px = (r - 3 * PX) % PX;
          py = PY - 3 + (r - 3 * PX) / PX;
        } else {
          const int q = r - 6 * PX, col = q % 6;
          px = col < 3 ? col : PX - 6 + col;
          py = 3 + q / 6;
        }
        int qx = x0 - 3 + px, qy = y0 - 3 + py;
        if (!inner) {
          qx = fold3(qx, c.nx, c.wall_x);
          qy = fold3(qy, c.ny, c.wall_y);
        }
        const Node3 nd(c, qx, qy, qz);
        float hv, lv;
        if (r < 0) {
          pull_f<S>(c, src, nd, fn);
          phi_of<S>(c, src, nd, fn, hv, lv);
        } else {
          pull_phi<S>(c, src, nd, hv, lv);
        }
        php[b + px + PX * py] = hv;
        plp[b + px + PX * py] = lv;
      }
    }
    __syncthreads();

    // M: mu at plane z + 2 over the tile + 2
    {
      const int k = z + 2;
      if (k >= za - 2 && !(c.wall_z && (k < 0 || k >= c.nz))) {
        const int bm = slot4(k - 1) * T::NP, b0 = slot4(k) * T::NP, bp = slot4(k + 1) * T::NP;
        const int b = slot3(k) * T::NM;
        const int qz = fold3(k, c.nz, c.wall_z);
        for (int pos = tid; pos < T::NM; pos += NT) {
          int mx = pos % MX, my = pos / MX;
          if (!inner) {
            mx = mirror_local(mx, x0 - 2, c.nx, c.wall_x, MX);
            my = mirror_local(my, y0 - 2, c.ny, c.wall_y, T::MY);
          }
          const int pc = (mx + 1) + PX * (my + 1);
          const float mu = slab_mu<PX>(c, php, plp, bm, b0, bp, pc);
          mup[b + pos] = mu;
          if constexpr (RF2) {
            // rho u_o at the same position: the mirror node's moments and the
            // stencil around the mirror position
            int qx = x0 - 2 + pos % MX, qy = y0 - 2 + pos / MX;
            if (!inner) {
              qx = fold3(qx, c.nx, c.wall_x);
              qy = fold3(qy, c.ny, c.wall_y);
            }
            float m0, m1x, m1y, m1z;
            pull_moments<S>(c, src, Node3(c, qx, qy, qz), m0, m1x, m1y, m1z);
            const float h0 = php[b0 + pc], l0 = plp[b0 + pc];
            float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 1; i < Q; ++i) {
              const int j = (EZ(i) < 0 ? bm : (EZ(i) > 0 ? bp : b0)) + pc + EX(i) + PX * EY(i);
              const float d = (php[j] - h0) + (plp[j] - l0);
              const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);  // 3 w_i
              if (EX(i)) g[0] += EX(i) > 0 ? w * d : -w * d;
              if (EY(i)) g[1] += EY(i) > 0 ? w * d : -w * d;
              if (EZ(i)) g[2] += EZ(i) > 0 ? w * d : -w * d;
            }
            const float rho = c.rho0 + (h0 + l0) * c.drho;
            const float iden = __builtin_amdgcn_rcpf(rho);
            const float fsz = mu * g[2] - (rho - c.rho_ref) * c.gravity;
            const int sq = slot3(k), sm = (k + 8) & 1;
            L.m[sm][0][pos] = m0;
            L.m[sm][1][pos] = m1x;
            L.m[sm][2][pos] = m1y;
            L.m[sm][3][pos] = m1z;
            L.q[sq][0][pos] = rho * ((3.0f * m1x + 0.5f * (mu * g[0])) * iden);
            L.q[sq][1][pos] = rho * ((3.0f * m1y + 0.5f * (mu * g[1])) * iden);
            L.q[sq][2][pos] = rho * ((3.0f * m1z + 0.5f * fsz) * iden);
          }
        }
      }
    }
    __syncthreads();

    // U: gbar moments, grad phi, lap mu, u and p at plane z + 1 over the
    // tile + 1; first each thread's own node, then the ring around the tile
    {
      const int k = z + 1;
      if (k >= za - 1 && !(c.wall_z && (k < 0 || k >= c.nz))) {
        const int qz = fold3(k, c.nz, c.wall_z);
        const int bm = slot4(k - 1) * T::NP, b0 = slot4(k) * T::NP, bp = slot4(k + 1) * T::NP;
        const int um = slot3(zread(c, k - 1)) * T::NM, u0 = slot3(k) * T::NM,
                  up = slot3(zread(c, k + 1)) * T::NM;
        const int pb = slot3(k) * T::NU;
        for (int r = tid - NT; r < NRING; r += NT) {
          // r < 0: the own node; else the r-th ring position
          int ux, uy;
          if (r < 0) {
            ux = lx + 1;
            uy = ly + 1;
          } else if (r < UX) {
            ux = r;
            uy = 0;
          } else if (r < 2 * UX) {
            ux = r - UX;
            uy = UY - 1;
          } else {
            ux = ((r - 2 * UX) & 1) ? UX - 1 : 0;
            uy = 1 + ((r - 2 * UX) >> 1);
          }
          int qx = x0 - 1 + ux, qy = y0 - 1 + uy, mx = ux, my = uy;
          if (!inner) {
            mx = mirror_local(ux, x0 - 1, c.nx, c.wall_x, UX);
            my = mirror_local(uy, y0 - 1, c.ny, c.wall_y, UY);
            qx = fold3(qx, c.nx, c.wall_x);
            qy = fold3(qy, c.ny, c.wall_y);
          }
          float m0, m1x, m1y, m1z;
          const Node3 nq(c, qx, qy, qz);
          if constexpr (RF2) {
            // the mu stage of the previous iteration pulled them at this node
            const int sm = (k + 8) & 1, jm = (ux + 1) + MX * (uy + 1);
            m0 = L.m[sm][0][jm];
            m1x = L.m[sm][1][jm];
            m1y = L.m[sm][2][jm];
            m1z = L.m[sm][3][jm];
          } else {
            pull_moments<S>(c, src, nq, m0, m1x, m1y, m1z);
          }
          const int pc = (mx + 2) + PX * (my + 2);
          const int mc = (mx + 1) + MX * (my + 1);
          const float h0 = php[b0 + pc], l0 = plp[b0 + pc];
          float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int i = 1; i < Q; ++i) {
            const int j = (EZ(i) < 0 ? bm : (EZ(i) > 0 ? bp : b0)) + pc + EX(i) + PX * EY(i);
            const float d = (php[j] - h0) + (plp[j] - l0);
            const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);  // 3 w_i
            if (EX(i)) g[0] += EX(i) > 0 ? w * d : -w * d;
            if (EY(i)) g[1] += EY(i) > 0 ? w * d : -w * d;
            if (EZ(i)) g[2] += EZ(i) > 0 ? w * d : -w * d;
          }
          const float mu = mup[u0 + mc];
          float lmu = 0.0f;
          if (c.corr != 0.0f) {
            float la = 0.0f, le = 0.0f;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
              const int j = (EZ(i) < 0 ? um : (EZ(i) > 0 ? up : u0)) + mc + EX(i) + MX * EY(i);
              const float d = mup[j] - mu;
              if (i <= 6) la += d;
              else le += d;
            }
            lmu = (1.0f / 3.0f) * la + (1.0f / 6.0f) * le;
          }
          const float ph = h0 + l0;
          const float rho = c.rho0 + ph * c.drho;
          const float fsx = mu * g[0], fsy = mu * g[1];
          const float fsz = mu * g[2] - (rho - c.rho_ref) * c.gravity;
          float cc = c.corr * lmu;
          if constexpr (RF2) {
            const int qm = slot3(zread(c, k - 1)), q0 = slot3(k), qp = slot3(zread(c, k + 1));
            float dv = 0.0f;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
              const int sl = EZ(i) < 0 ? qm : (EZ(i) > 0 ? qp : q0);
              const int j = mc + EX(i) + MX * EY(i);
              const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);  // 3 w_i
              float e = 0.0f;
              if (EX(i)) e += EX(i) > 0 ? L.q[sl][0][j] : -L.q[sl][0][j];
              if (EY(i)) e += EY(i) > 0 ? L.q[sl][1][j] : -L.q[sl][1][j];
              if (EZ(i)) e += EZ(i) > 0 ? L.q[sl][2][j] : -L.q[sl][2][j];
              dv += w * e;
            }
            cc = (ph - gload<float>(src, c.phiv + 4u * nq.idx)) * c.drho + dv;
          }
          const float iden = __builtin_amdgcn_rcpf(rho - 0.5f * cc);
          const float vx = (3.0f * m1x + 0.5f * fsx) * iden;
          const float vy = (3.0f * m1y + 0.5f * fsy) * iden;
          const float vz = (3.0f * m1z + 0.5f * fsz) * iden;
          const float p = m0 + (1.0f / 6.0f) * c.drho * (vx * g[0] + vy * g[1] + vz * g[2]);
          pp[pb + ux + UX * uy] = p;
          if (r < 0) {
            nxt.phh = h0;
            nxt.phl = l0;
            nxt.mu = mu;
            nxt.cc = cc;
            nxt.p = p;
            nxt.ux = vx;
            nxt.uy = vy;
            nxt.uz = vz;
            nxt.gx = g[0];
            nxt.gy = g[1];
            nxt.gz = g[2];
          }
        }
      }
    }
    __syncthreads();

    // C: grad p and the collision of the tile's nodes at plane z
    if (z >= za && own) {
      const Node3 nd(c, gx, gy, z);
      const int uc = (lx + 1) + UX * (ly + 1);
      const int pm = slot3(zread(c, z - 1)) * T::NU, p0 = slot3(z) * T::NU,
                pq = slot3(zread(c, z + 1)) * T::NU;
      const float f0 = pp[p0 + uc];
      float ax = 0.0f, ay = 0.0f, az = 0.0f;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const float d = pp[(EZ(i) < 0 ? pm : (EZ(i) > 0 ? pq : p0)) + uc + EX(i) + UX * EY(i)] - f0;
        const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);
        if (EX(i)) ax += EX(i) > 0 ? w * d : -w * d;
        if (EY(i)) ay += EY(i) > 0 ? w * d : -w * d;
        if (EZ(i)) az += EZ(i) > 0 ? w * d : -w * d;
      }
      cur.gpx = ax;
      cur.gpy = ay;
      cur.gpz = az;
      collide_node<S>(c, op, nd.idx, fa, gv, cur);
      // correction from data: the copy carries this step's phi
      if constexpr (RF2) gstore_nt<float>(op.base, c.phiv + 4u * nd.idx, cur.phh + cur.phl);
    }
    cur = nxt;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      fa[i] = fb[i];
      fb[i] = fc[i];
      fc[i] = fn[i];
    }
  }
}

// ---- fused step without the Eq. 5 term (its coefficient is zero: the
// original model, or theta_M = 0, or equal densities).  lap mu is not needed,
// so u and p at a position need mu only there, and the pipeline is one plane
// shorter than k3_slab's: iteration z stages phi(z + 2) over the tile + 2
// (ring of 3 planes), forms mu, grad phi, u and p at z + 1 over the tile + 1
// (mu from the phi stencil at the position itself), then collides plane z.
// The own node's pulled f is carried for two planes.  Walls, periodic seams
// and the expressions as in k3_slab, so the same bits.
template <int TX, int TY>
struct Slab2Lds {
  static constexpr int PX = TX + 4, PY = TY + 4, NP = PX * PY;  // phi plane
  static constexpr int UX = TX + 2, UY = TY + 2, NU = UX * UY;  // p plane
  float ph[3][NP];
  float pl[3][NP];
  float p[3][NU];
};

template <int S, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) k3_slab2(CaseDev c, int parity, int zs) {
  using T = Slab2Lds<TX, TY>;
  constexpr int NT = TX * TY, PX = T::PX, PY = T::PY, UX = T::UX, UY = T::UY;
  constexpr int NPRING = T::NP - NT;  // positions of the tile + 2 outside the tile
  constexpr int NRING = T::NU - NT;   // positions of the tile + 1 outside the tile
  __shared__ T L;
  const int ntx = (c.nx + TX - 1) / TX, nty = (c.ny + TY - 1) / TY;
  const int ntiles = ntx * nty * ((c.nz + zs - 1) / zs);
  const int chunk = (ntiles + 7) >> 3;
  const int t = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
  if (blockIdx.x >= (unsigned)(8 * chunk) || t >= ntiles) return;
  const int x0 = (t % ntx) * TX, y0 = ((t / ntx) % nty) * TY;
  const int za = (t / (ntx * nty)) * zs, zb = min(za + zs, c.nz);
  const int tid = threadIdx.x;
  const bool inner = x0 >= 2 && x0 + TX + 2 <= c.nx && y0 >= 2 && y0 + TY + 2 <= c.ny;
  const int lx = tid % TX, ly = tid / TX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool own = gx < c.nx && gy < c.ny;
  const char* src = parity ? c.state[1] : c.state[0];
  const BaseOut<S> op{parity ? c.state[0] : c.state[1]};
  float* const php = &L.ph[0][0];
  float* const plp = &L.pl[0][0];
  float* const pp = &L.p[0][0];

  NodeFields cur{}, nxt{};  // own node: plane z (collided now), plane z + 1
  // own node's pulled f_1..f_18 at planes z, z + 1 and z + 2 (fn)
  float fa[Q], fb[Q], fn[Q];
  for (int z = za - 4; z < zb; ++z) {
    // the own node's gbar for the collision at the end of the iteration
    float gv[Q];
    if (z >= za && own) pull_g<S>(c, src, Node3(c, gx, gy, z), gv);
    // phi at plane z + 2 over the tile + 2: the own node first (its f kept),
    // then the 2-wide ring around the tile
    {
      const int k = z + 2;
      const int qz = fold3(k, c.nz, c.wall_z);
      const int b = slot3(k) * T::NP;
      for (int r = tid - NT; r < NPRING; r += NT) {
        int px, py;
        if (r < 0) {
          px = lx + 2;
          py = ly + 2;
        } else if (r < 2 * PX) {
          px = r % PX;
          py = r / PX;
        } else if (r < 4 * PX) {
          px = (r - 2 * PX) % PX;
          py = PY - 2 + (r - 2 * PX) / PX;
        } else {
          const int q = r - 4 * PX, col = q % 4;
          px = col < 2 ? col : PX - 4 + col;
          py = 2 + q / 4;
        }
        int qx = x0 - 2 + px, qy = y0 - 2 + py;
        if (!inner) {
          qx = fold3(qx, c.nx, c.wall_x);
          qy = fold3(qy, c.ny, c.wall_y);
        }
        const Node3 nd(c, qx, qy, qz);
        float hv, lv;
        if (r < 0) {
          pull_f<S>(c, src, nd, fn);
          phi_of<S>(c, src, nd, fn, hv, lv);
        } else {
          pull_phi<S>(c, src, nd, hv, lv);
        }
        php[b + px + PX * py] = hv;
        plp[b + px + PX * py] = lv;
      }
    }
    __syncthreads();

    // mu, gbar moments, grad phi, u and p at plane z + 1 over the tile + 1
    {
      const int k = z + 1;
      if (k >= za - 1 && !(c.wall_z && (k < 0 || k >= c.nz))) {
        const int qz = fold3(k, c.nz, c.wall_z);
        const int bm = slot3(k - 1) * T::NP, b0 = slot3(k) * T::NP, bp = slot3(k + 1) * T::NP;
        const int pb = slot3(k) * T::NU;
        for (int r = tid - NT; r < NRING; r += NT) {
          int ux, uy;
          if (r < 0) {
            ux = lx + 1;
            uy = ly + 1;
          } else if (r < UX) {
            ux = r;
            uy = 0;
          } else if (r < 2 * UX) {
            ux = r - UX;
            uy = UY - 1;
          } else {
            ux = ((r - 2 * UX) & 1) ? UX - 1 : 0;
            uy = 1 + ((r - 2 * UX) >> 1);
          }
          int qx = x0 - 1 + ux, qy = y0 - 1 + uy, mx = ux, my = uy;
          if (!inner) {
            mx = mirror_local(ux, x0 - 1, c.nx, c.wall_x, UX);
            my = mirror_local(uy, y0 - 1, c.ny, c.wall_y, UY);
            qx = fold3(qx, c.nx, c.wall_x);
            qy = fold3(qy, c.ny, c.wall_y);
          }
          float m0, m1x, m1y, m1z;
          pull_moments<S>(c, src, Node3(c, qx, qy, qz), m0, m1x, m1y, m1z);
          const int pc = (mx + 1) + PX * (my + 1);
          const float mu = slab_mu<PX>(c, php, plp, bm, b0, bp, pc);
          const float h0 = php[b0 + pc], l0 = plp[b0 + pc];
          float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int i = 1; i < Q; ++i) {
            const int j = (EZ(i) < 0 ? bm : (EZ(i) > 0 ? bp : b0)) + pc + EX(i) + PX * EY(i);
            const float d = (php[j] - h0) + (plp[j] - l0);
            const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);  // 3 w_i
            if (EX(i)) g[0] += EX(i) > 0 ? w * d : -w * d;
            if (EY(i)) g[1] += EY(i) > 0 ? w * d : -w * d;
            if (EZ(i)) g[2] += EZ(i) > 0 ? w * d : -w * d;
          }
          const float ph = h0 + l0;
          const float rho = c.rho0 + ph * c.drho;
          const float fsx = mu * g[0], fsy = mu * g[1];
          const float fsz = mu * g[2] - (rho - c.rho_ref) * c.gravity;
          const float cc = c.corr * 0.0f;  // lap mu is not formed: the coefficient is zero
          const float iden = __builtin_amdgcn_rcpf(rho - 0.5f * cc);
          const float vx = (3.0f * m1x + 0.5f * fsx) * iden;
          const float vy = (3.0f * m1y + 0.5f * fsy) * iden;
          const float vz = (3.0f * m1z + 0.5f * fsz) * iden;
          const float p = m0 + (1.0f / 6.0f) * c.drho * (vx * g[0] + vy * g[1] + vz * g[2]);
          pp[pb + ux + UX * uy] = p;
          if (r < 0) {
            nxt.phh = h0;
            nxt.phl = l0;
            nxt.mu = mu;
            nxt.cc = cc;
            nxt.p = p;
            nxt.ux = vx;
            nxt.uy = vy;
            nxt.uz = vz;
            nxt.gx = g[0];
            nxt.gy = g[1];
            nxt.gz = g[2];
          }
        }
      }
    }
    __syncthreads();

    // grad p and the collision of the tile's nodes at plane z
    if (z >= za && own) {
      const Node3 nd(c, gx, gy, z);
      const int uc = (lx + 1) + UX * (ly + 1);
      const int pm = slot3(zread(c, z - 1)) * T::NU, p0 = slot3(z) * T::NU,
                pq = slot3(zread(c, z + 1)) * T::NU;
      const float f0 = pp[p0 + uc];
      float ax = 0.0f, ay = 0.0f, az = 0.0f;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const float d = pp[(EZ(i) < 0 ? pm : (EZ(i) > 0 ? pq : p0)) + uc + EX(i) + UX * EY(i)] - f0;
        const float w = i <= 6 ? (1.0f / 6.0f) : (1.0f / 12.0f);
        if (EX(i)) ax += EX(i) > 0 ? w * d : -w * d;
        if (EY(i)) ay += EY(i) > 0 ? w * d : -w * d;
        if (EZ(i)) az += EZ(i) > 0 ? w * d : -w * d;
      }
      cur.gpx = ax;
      cur.gpy = ay;
      cur.gpz = az;
      collide_node<S>(c, op, nd.idx, fa, gv, cur);
    }
    cur = nxt;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      fa[i] = fb[i];
      fb[i] = fn[i];
    }
  }
}

// ---- field dump for lbm_moments / diagnostics
// (one_float: 16-bit storage, whose phi is the one float of the phh plane;
// its pull leaves the phl plane unwritten)
__global__ void __launch_bounds__(256) k3_dump(CaseDev c, Fields3 fl, FieldPtrs out,
                                               int one_float) {
  const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (unsigned)c.n) return;
  const float ux = fl.ux[idx], uy = fl.uy[idx], uz = fl.uz[idx], lmu = fl.lmu[idx];
  out.phi[idx] = one_float ? fl.phh[idx] : fl.phh[idx] + fl.phl[idx];
  out.u[0][idx] = ux;
  out.u[1][idx] = uy;
  out.u[2][idx] = uz;
  out.p[idx] = fl.p[idx];
  out.mu[idx] = fl.mu[idx];
  out.fa[0][idx] = -ux * c.fa_coef * lmu;
  out.fa[1][idx] = -uy * c.fa_coef * lmu;
  out.fa[2][idx] = -uz * c.fa_coef * lmu;
}

// ---- initial populations (inverse of the first pull)
template <int S>
__global__ void __launch_bounds__(256)
k3_init(CaseDev c, int parity, const double* __restrict__ phi0, const double* __restrict__ u0,
        const double* __restrict__ p0) {
  using P = Pops<S, Q>;
  const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (unsigned)c.n) return;
  int x, y, z;
  coords(c, idx, x, y, z);
  const double v0 = phi0[idx];
  const float h0 = (float)v0, l0 = (float)(v0 - (double)h0);
  float la = 0.0f, le = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const double v = phi0[nbr(c, x, y, z, i, false, idx)];
    const float h = (float)v, l = (float)(v - (double)h);
    const float d = (h - h0) + (l - l0);
    if (i <= 6) la += d;
    else le += d;
  }
  const float lap = (1.0f / 3.0f) * la + (1.0f / 6.0f) * le;
  const float mu = dtheta(c, h0, l0) - c.kappa * lap;
  const float ph = h0 + l0;
  const unsigned n = c.n;
  const float ux = (float)u0[idx], uy = (float)u0[n + idx], uz = (float)u0[2 * n + idx];
  const float p = (float)p0[idx];
  const float rho = c.rho0 + ph * c.drho;
  const float uu = ux * ux + uy * uy + uz * uz;
  char* dst = parity ? c.state[1] : c.state[0];
  float fsum = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float eu = EX(i) * ux + EY(i) * uy + EZ(i) * uz;
    const float ti = 3.0f * eu + 4.5f * eu * eu - 1.5f * uu;
    const float geq = WT(i) * p + (1.0f / 3.0f) * rho * WT(i) * ti;
    int dir = i;
    unsigned j = idx;
    if (i > 0) {
      bool bb;
      const unsigned s = pull_src(c, x, y, z, EX(i), EY(i), EZ(i), &bb);
      if (!bb) j = s;
      else dir = OPP(i);
      const float feq = WT(i) * (c.gamma3 * mu + ph * ti);
      fsum += P::put_f(c, dst, dir, j, feq);
    }
    P::put_g(c, dst, dir, j, geq, WT(i));
  }
  float hh, ee;
  two_sum(h0, -fsum, hh, ee);
  P::put_f0(c, dst, idx, hh, ee + l0);
  // correction from data: phi^(n-1) of the first step is phi0
  if (c.phiv) gstore_nt<float>(dst, c.phiv + 4u * idx, ph);
}

}  // namespace d3q19

// ------------------------------------------------------------ launchers
// Variants 0-4: the three-kernel step, by the tile of its fields kernel (the
// pull and collision kernels are node-parallel, 256 threads).  Variants 5-12:
// the fused step, by its x-y tile and z chunk (tz planes); the 64-wide tiles
// give the 16-bit step one 128-byte line per row and plane.  All give the same
// bits, in every model and storage layout.
const TileShape kD3Q19Tiles[] = {
    {16, 8, 4, 512, 0, FORM_THREE},  {32, 4, 4, 512, 0, FORM_THREE},
    {32, 8, 2, 512, 0, FORM_THREE},  {16, 16, 2, 512, 0, FORM_THREE},
    {8, 8, 8, 512, 0, FORM_THREE},   {32, 8, 16, 256, 0, FORM_FUSED},
    {32, 8, 32, 256, 0, FORM_FUSED}, {32, 16, 16, 512, 0, FORM_FUSED},
    {32, 16, 32, 512, 0, FORM_FUSED}, {32, 8, 64, 256, 0, FORM_FUSED},
    {32, 16, 64, 512, 0, FORM_FUSED}, {64, 8, 32, 512, 0, FORM_FUSED},
    {64, 8, 64, 512, 0, FORM_FUSED}, {64, 4, 16, 256, 0, FORM_TWO},
    {64, 4, 22, 256, 0, FORM_TWO},   {64, 4, 43, 256, 0, FORM_TWO},
    {128, 2, 16, 256, 0, FORM_TWO}};
const int kD3Q19TileCount = sizeof(kD3Q19Tiles) / sizeof(kD3Q19Tiles[0]);

namespace {
d3q19::Fields3 fields3(const Field3Ptrs& f) {
  d3q19::Fields3 fl;
  fl.phh = f.plane[0];
  fl.phl = f.plane[1];
  fl.m0 = f.plane[2];
  fl.m1x = f.plane[3];
  fl.m1y = f.plane[4];
  fl.m1z = f.plane[5];
  fl.mu = f.plane[6];
  fl.ux = f.plane[7];
  fl.uy = f.plane[8];
  fl.uz = f.plane[9];
  fl.p = f.plane[10];
  fl.lmu = f.plane[11];
  fl.dd = f.plane[12];
  return fl;
}

template <int FX, int FY, int FZ, bool LEAN>
void launch_fields_t(const CaseDev& c, const d3q19::Fields3& fl, int dump, int parity,
                     hipStream_t s) {
  const int ft = ((c.nx + FX - 1) / FX) * ((c.ny + FY - 1) / FY) * ((c.nz + FZ - 1) / FZ);
  if (c.phiv)
    hipLaunchKernelGGL((d3q19::k3_fields_t<FX, FY, FZ, true, LEAN>), dim3(8 * ((ft + 7) / 8)),
                       dim3(FX * FY * FZ), 0, s, c, fl, dump, parity);
  else
    hipLaunchKernelGGL((d3q19::k3_fields_t<FX, FY, FZ, false, LEAN>), dim3(8 * ((ft + 7) / 8)),
                       dim3(FX * FY * FZ), 0, s, c, fl, dump, parity);
}

template <int S, int TX, int TY>
void launch_slab(const CaseDev& c, int parity, int zs, hipStream_t s) {
  static_assert(S == ST_FP32, "16-bit storage runs the fused step k3_march");
  const int ft = ((c.nx + TX - 1) / TX) * ((c.ny + TY - 1) / TY) * ((c.nz + zs - 1) / zs);
  if (!c.phiv && c.corr == 0.0f)  // no Eq. 5 term: the shorter pipeline
    hipLaunchKernelGGL((d3q19::k3_slab2<S, TX, TY>), dim3(8 * ((ft + 7) / 8)), dim3(TX * TY),
                       0, s, c, parity, zs);
  else if (c.phiv)
    hipLaunchKernelGGL((d3q19::k3_slab<S, TX, TY, true>), dim3(8 * ((ft + 7) / 8)),
                       dim3(TX * TY), 0, s, c, parity, zs);
  else
    hipLaunchKernelGGL((d3q19::k3_slab<S, TX, TY, false>), dim3(8 * ((ft + 7) / 8)),
                       dim3(TX * TY), 0, s, c, parity, zs);
}

// The second kernel of the two-kernel step (16-bit storage).
template <int S, int TX, int TY>
void launch_fcm(const CaseDev& c, int parity, const d3q19::Fields3& fl, int zc, hipStream_t s) {
  const int ft = ((c.nx + TX - 1) / TX) * ((c.ny + TY - 1) / TY) * ((c.nz + zc - 1) / zc);
  if (c.phiv)
    hipLaunchKernelGGL((d3q19::k3_fcm<S, TX, TY, true>), dim3(8 * ((ft + 7) / 8)),
                       dim3(TX * TY), 0, s, c, parity, fl, zc);
  else
    hipLaunchKernelGGL((d3q19::k3_fcm<S, TX, TY, false>), dim3(8 * ((ft + 7) / 8)),
                       dim3(TX * TY), 0, s, c, parity, fl, zc);
}

template <int S>
hipError_t pipeline(int variant, const CaseDev& c, int parity, const d3q19::Fields3& fl,
                    int dump, bool collide, hipStream_t s) {
  const int form = variant >= 0 && variant < kD3Q19TileCount ? kD3Q19Tiles[variant].form : -1;
  if (form == FORM_TWO) {
    // 16-bit storage; FP32 storage (and a field dump) runs the three-kernel
    // step
    if constexpr (S != ST_FP32) {
      if (collide && !dump) {
        const TileShape& t = kD3Q19Tiles[variant];
        d3q19::RowGrid rg = d3q19::row_grid(c);
        if (rg.grid.y > 65535u) return hipErrorInvalidConfiguration;
        rg.grid.x = (unsigned)(c.ny * t.tz * ((c.nz + t.tz - 1) / t.tz));
        hipLaunchKernelGGL(d3q19::k3_pull<S>, rg.grid, rg.block, 0, s, c, parity, fl, t.tz);
        if (t.tx == 64) launch_fcm<S, 64, 4>(c, parity, fl, t.tz, s);
        else launch_fcm<S, 128, 2>(c, parity, fl, t.tz, s);
        return hipGetLastError();
      }
    }
    variant = 1;
  }
  if (form == FORM_FUSED) {
    // 16-bit storage with the correction from data, or on a grid of odd
    // width (the fused 16-bit step pairs x-adjacent nodes), runs the
    // three-kernel step
    if (collide && (S == ST_FP32 || (!c.phiv && !(c.nx & 1)))) {
      const TileShape& t = kD3Q19Tiles[variant];
      if constexpr (S != ST_FP32) {
        return d3q19_march(c, S, t.tx, t.ty, t.tz, parity, s);
      } else {
        if (t.tx == 32 && t.ty == 8) launch_slab<S, 32, 8>(c, parity, t.tz, s);
        else if (t.tx == 64) launch_slab<S, 64, 8>(c, parity, t.tz, s);
        else launch_slab<S, 32, 16>(c, parity, t.tz, s);
        return hipGetLastError();
      }
    }
    variant = 1;
  }
  const d3q19::RowGrid rg = d3q19::row_grid(c);
  if (rg.grid.y > 65535u) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(d3q19::k3_pull<S>, rg.grid, rg.block, 0, s, c, parity, fl, 0);
  switch (variant) {
    case 0: launch_fields_t<16, 8, 4, (S != ST_FP32)>(c, fl, dump, parity, s); break;
    case 1: launch_fields_t<32, 4, 4, (S != ST_FP32)>(c, fl, dump, parity, s); break;
    case 2: launch_fields_t<32, 8, 2, (S != ST_FP32)>(c, fl, dump, parity, s); break;
    case 3: launch_fields_t<16, 16, 2, (S != ST_FP32)>(c, fl, dump, parity, s); break;
    case 4: launch_fields_t<8, 8, 8, (S != ST_FP32)>(c, fl, dump, parity, s); break;
    default: return hipErrorInvalidValue;
  }
  if (collide) hipLaunchKernelGGL(d3q19::k3_collide<S>, rg.grid, rg.block, 0, s, c, parity, fl);
  return hipGetLastError();
}
}  // namespace

hipError_t d3q19_step_case(int variant, const CaseDev& c, int storage, int parity,
                           const Field3Ptrs& f, hipStream_t stream) {
  const d3q19::Fields3 fl = fields3(f);
  switch (storage) {
    case ST_FP32: return pipeline<ST_FP32>(variant, c, parity, fl, 0, true, stream);
    case ST_FP16: return pipeline<ST_FP16>(variant, c, parity, fl, 0, true, stream);
    default: return pipeline<ST_BF16>(variant, c, parity, fl, 0, true, stream);
  }
}

hipError_t d3q19_fields_case(const CaseDev& c, int storage, int parity, const Field3Ptrs& f,
                             const FieldPtrs& out, hipStream_t stream) {
  const d3q19::Fields3 fl = fields3(f);
  hipError_t e;
  switch (storage) {
    case ST_FP32: e = pipeline<ST_FP32>(0, c, parity, fl, 1, false, stream); break;
    case ST_FP16: e = pipeline<ST_FP16>(0, c, parity, fl, 1, false, stream); break;
    default: e = pipeline<ST_BF16>(0, c, parity, fl, 1, false, stream);
  }
  if (e != hipSuccess) return e;
  const int grid = (c.n + 255) / 256;
  hipLaunchKernelGGL(d3q19::k3_dump, dim3(grid), dim3(256), 0, stream, c, fl, out,
                     storage != ST_FP32 ? 1 : 0);
  return hipGetLastError();
}

hipError_t d3q19_init(const CaseDev& c, int storage, int parity, const double* phi0,
                      const double* u0, const double* p0, hipStream_t stream) {
  const int grid = (c.n + 255) / 256;
  switch (storage) {
    case ST_FP32:
      hipLaunchKernelGGL(d3q19::k3_init<ST_FP32>, dim3(grid), dim3(256), 0, stream, c, parity,
                         phi0, u0, p0);
      break;
    case ST_FP16:
      hipLaunchKernelGGL(d3q19::k3_init<ST_FP16>, dim3(grid), dim3(256), 0, stream, c, parity,
                         phi0, u0, p0);
      break;
    default:
      hipLaunchKernelGGL(d3q19::k3_init<ST_BF16>, dim3(grid), dim3(256), 0, stream, c, parity,
                         phi0, u0, p0);
  }
  return hipGetLastError();
}

}  // namespace lbm
