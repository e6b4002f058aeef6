// lbm_d3q19_lean.h -- per-node arithmetic of the D3Q19 step with 16-bit
// population storage, shared by every D3Q19 kernel that runs it (the fused
// step k3_march and the pull / fields / collision kernels of the three-kernel
// step), so that all of them compute each node to the same bits.
//
// The model is the one of the FP32 path (Eq. 1a / 1b, Eq. 4a / 4b, Eq. 8 and
// the -F_a switch of the paragraph after Eq. 12, isotropic central stencils);
// only the evaluation order differs, chosen for the instruction count of a
// bandwidth-bound kernel:
//   - phi is one float: the 16-bit populations resolve it to ~1e-6, far
//     coarser than a float's 6e-8, so the float-float phi of the FP32 path
//     buys nothing here;
//   - lattice sums run over the nine opposite pairs (2j-1, 2j), j = 1..9,
//     of the D3Q19 order (e_{2j-1} = -e_{2j}): gradients from pair
//     differences, moments from pair sums and differences;
//   - the Laplacian keeps the differences to the centre, so a uniform field
//     has a Laplacian of exactly zero;
//   - the collision pairs direction i with its opposite, whose equilibrium
//     and forcing terms differ only in the sign of the odd part, and works on
//     the stored (scaled, rest-relative) values directly: with w_i s and the
//     rest pressure p0 folded into its coefficients, a stored word is decoded
//     once (v_fma_mix / shift) and encoded once (v_cvt_pk_*).
// Every multiply-add is an explicit fmaf, so the result does not depend on
// the contraction choices of the compiler.
#pragma once

#include "lbm_dev.h"
#include "lbm_lattice.h"

namespace lbm {
namespace d3q19 {

// the member 2j - 1 of pair j carries the sign of the odd terms
__host__ __device__ constexpr int PI(int j) { return 2 * j - 1; }

// e_i . (x, y, z), summed x, y, z without adding zero terms (x + 0 is not
// an identity under IEEE signed zeros, so a literal zero would cost an add).
__device__ __forceinline__ float edot(int i, float x, float y, float z) {
  float s = 0.0f;
  bool first = true;
  if (EX(i)) {
    s = EX(i) > 0 ? x : -x;
    first = false;
  }
  if (EY(i)) {
    s = first ? (EY(i) > 0 ? y : -y) : (EY(i) > 0 ? s + y : s - y);
    first = false;
  }
  if (EZ(i)) s = first ? (EZ(i) > 0 ? z : -z) : (EZ(i) > 0 ? s + z : s - z);
  return s;
}

// Scaled value of a stored 16-bit word (the float the word encodes; the
// population is that times the inverse scale, plus w_i p0 for g).
template <int S>
__device__ __forceinline__ float raw16(uint16_t h) {
  return dec16<S>(h);
}

// Encode two floats into the packed 16-bit words of a pair (low half first),
// round to nearest even.  The floats pass through an empty asm first: left
// visible, a multiply-add feeding the conversion may be fused into one
// v_fma_mix with a half result, which rounds once where the definition rounds
// to float and then to half, and differs on near-ties.
template <int S>
__device__ __forceinline__ uint32_t enc_pair(float a, float b) {
  if constexpr (S == ST_BF16) {
    return (uint32_t)enc_bf16(a) | ((uint32_t)enc_bf16(b) << 16);
  } else {
    asm volatile("" : "+v"(a), "+v"(b));
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = {a, b};
    const h2 h = __builtin_convertvector(v, h2);
    return __builtin_bit_cast(uint32_t, h);
  }
}
// The same pair rounded stochastically with the random bits ra, rb (see
// sr_word); no fusion hazard here, the integer steps keep the conversion apart.
template <int S>
__device__ __forceinline__ uint32_t enc_pair_sr(float a, float b, uint32_t ra, uint32_t rb) {
  const uint32_t ua = sr_word<S>(a, ra), ub = sr_word<S>(b, rb);
  if constexpr (S == ST_BF16) {
    return (ua >> 16) | (ub & 0xffff0000u);
  } else {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = {__uint_as_float(ua), __uint_as_float(ub)};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, h2));
  }
}
template <int S>
__device__ __forceinline__ float lo16(uint32_t w) {
  return dec16<S>((uint16_t)(w & 0xffffu));
}
template <int S>
__device__ __forceinline__ float hi16(uint32_t w) {
  return dec16<S>((uint16_t)(w >> 16));
}

// phi = f_0 + (1/s_f) sum_{i>0} f_i^stored, the f_i summed as nine pair sums
// in pair order.  d[1..18]: the scaled values of the pulled f_i.
__device__ __forceinline__ float lean_phi(const CaseDev& c, float f0, const float* d) {
  float s = d[1] + d[2];
#pragma unroll
  for (int j = 2; j <= 9; ++j) s += d[PI(j)] + d[PI(j) + 1];
  return __builtin_fmaf(c.inv_scale_f, s, f0);
}

// Zeroth and first moments of the pulled gbar from the scaled values
// G[0..18] (g_i = G_i / s_g + w_i p0): m0 = sum g, m1 = sum e g.  The w_i p0
// parts sum to p0 (zeroth) and to zero (first moments).
__device__ __forceinline__ void lean_moments(const CaseDev& c, const float* G, float& m0,
                                             float& mx, float& my, float& mz) {
  float a = G[0];
  float b[10];
#pragma unroll
  for (int j = 1; j <= 9; ++j) {
    a += G[PI(j)] + G[PI(j) + 1];
    b[j] = G[PI(j)] - G[PI(j) + 1];
  }
  float sx = b[1], sy = b[2], sz = b[3];
#pragma unroll
  for (int j = 4; j <= 9; ++j) {
    const int i = PI(j);
    if (EX(i)) sx = EX(i) > 0 ? sx + b[j] : sx - b[j];
    if (EY(i)) sy = EY(i) > 0 ? sy + b[j] : sy - b[j];
    if (EZ(i)) sz = EZ(i) > 0 ? sz + b[j] : sz - b[j];
  }
  m0 = __builtin_fmaf(c.inv_scale_g, a, c.p0);
  mx = c.inv_scale_g * sx;
  my = c.inv_scale_g * sy;
  mz = c.inv_scale_g * sz;
}

// Isotropic gradient 3 sum_i w_i e_i v_i from the 18 neighbour values
// v[1..18] (lattice order), as pair differences: the axis pair weighted 1/6,
// the four edge pairs of the axis 1/12.
__device__ __forceinline__ void lean_grad(const float* v, float& gx, float& gy, float& gz) {
  float d[10];
#pragma unroll
  for (int j = 1; j <= 9; ++j) d[j] = v[PI(j)] - v[PI(j) + 1];
  // edge pairs of each axis in pair order (the first one starts the sum)
  float ex = 0.0f, ey = 0.0f, ez = 0.0f;
  bool fx = true, fy = true, fz = true;
#pragma unroll
  for (int j = 4; j <= 9; ++j) {
    const int i = PI(j);
    if (EX(i)) {
      ex = fx ? (EX(i) > 0 ? d[j] : -d[j]) : (EX(i) > 0 ? ex + d[j] : ex - d[j]);
      fx = false;
    }
    if (EY(i)) {
      ey = fy ? (EY(i) > 0 ? d[j] : -d[j]) : (EY(i) > 0 ? ey + d[j] : ey - d[j]);
      fy = false;
    }
    if (EZ(i)) {
      ez = fz ? (EZ(i) > 0 ? d[j] : -d[j]) : (EZ(i) > 0 ? ez + d[j] : ez - d[j]);
      fz = false;
    }
  }
  gx = __builtin_fmaf(1.0f / 6.0f, d[1], (1.0f / 12.0f) * ex);
  gy = __builtin_fmaf(1.0f / 6.0f, d[2], (1.0f / 12.0f) * ey);
  gz = __builtin_fmaf(1.0f / 6.0f, d[3], (1.0f / 12.0f) * ez);
}

// Isotropic Laplacian 6 sum_{i>0} w_i (v_i - v_0): differences to the centre,
// summed per pair, axis pairs weighted 1/3 and edge pairs 1/6.
__device__ __forceinline__ float lean_lap(const float* v, float v0) {
  float p[10];
#pragma unroll
  for (int j = 1; j <= 9; ++j) p[j] = (v[PI(j)] - v0) + (v[PI(j) + 1] - v0);
  const float la = (p[1] + p[2]) + p[3];
  const float le = ((((p[4] + p[5]) + p[6]) + p[7]) + p[8]) + p[9];
  return __builtin_fmaf(1.0f / 3.0f, la, (1.0f / 6.0f) * le);
}

// theta'(phi) of the double well with a one-float phi.
__device__ __forceinline__ float lean_dtheta(const CaseDev& c, float ph) {
  return c.th_k * ph * (ph - c.th_r1) * (ph - c.th_r2);
}

// mu = theta'(phi) - kappa lap phi.
__device__ __forceinline__ float lean_mu(const CaseDev& c, float ph, float lap) {
  return __builtin_fmaf(-c.kappa, lap, lean_dtheta(c, ph));
}

// Recovery of u and p at a node (reading Z8 with -F_a = cc u):
//   (rho - cc/2) u = 3 m1 + (F_s + G)/2,   p = m0 + (drho / 6) u . grad phi,
// F_s = mu grad phi, G = -(rho - rho_ref) g along -z.
struct LeanUP {
  float ux, uy, uz, p;
};
__device__ __forceinline__ LeanUP lean_recover(const CaseDev& c, float ph, float mu, float gx,
                                               float gy, float gz, float cc, float m0, float mx,
                                               float my, float mz) {
  const float rho = __builtin_fmaf(ph, c.drho, c.rho0);
  const float fsx = mu * gx, fsy = mu * gy;
  const float fsz = __builtin_fmaf(mu, gz, -(rho - c.rho_ref) * c.gravity);
  const float iden = __builtin_amdgcn_rcpf(__builtin_fmaf(-0.5f, cc, rho));
  LeanUP r;
  r.ux = __builtin_fmaf(3.0f, mx, 0.5f * fsx) * iden;
  r.uy = __builtin_fmaf(3.0f, my, 0.5f * fsy) * iden;
  r.uz = __builtin_fmaf(3.0f, mz, 0.5f * fsz) * iden;
  const float ug = __builtin_fmaf(r.ux, gx, __builtin_fmaf(r.uy, gy, r.uz * gz));
  r.p = __builtin_fmaf((1.0f / 6.0f) * c.drho, ug, m0);
  return r;
}

// Packed stored words of one node: Fr[j] (j = 1..9) holds f_{2j-1} in its
// low and f_{2j} in its high half; Gr[k] (k = 0..9) holds gbar_{2k} low and
// gbar_{2k+1} high (gbar_18 in the low half of Gr[9]).
template <int S>
__device__ __forceinline__ float f_of(const uint32_t* Fr, int i) {
  return (i & 1) ? lo16<S>(Fr[(i + 1) >> 1]) : hi16<S>(Fr[i >> 1]);
}
template <int S>
__device__ __forceinline__ float g_of(const uint32_t* Gr, int i) {
  return (i & 1) ? hi16<S>(Gr[i >> 1]) : lo16<S>(Gr[i >> 1]);
}
__device__ __forceinline__ uint32_t pack16(uint16_t lo, uint16_t hi) {
  return (uint32_t)lo | ((uint32_t)hi << 16);
}

// phi and the moments from packed words.  FP16: each word's two halves
// enter a running FP32 sum through one v_dot2_f32_f16 with weights (1, 1),
// or (e_a, e_b) for a first moment; that adds both products and the sum with
// one rounding (products of a half and +-1 are exact; subnormal halves
// included).  BF16: decoded, then lean_phi / lean_moments.
typedef _Float16 lean_h2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float dot2_acc(uint32_t w, float a, float b, float acc) {
  const lean_h2 wt = {(_Float16)a, (_Float16)b};
  return __builtin_amdgcn_fdot2(__builtin_bit_cast(lean_h2, w), wt, acc, false);
}
template <int S>
__device__ __forceinline__ float lean_phi_packed(const CaseDev& c, float f0, const uint32_t* Fr) {
  if constexpr (S == ST_FP16) {
    // Fr[j] holds the opposite pair (2j - 1, 2j); summed in pair order
    float s = dot2_acc(Fr[1], 1.0f, 1.0f, 0.0f);
#pragma unroll
    for (int j = 2; j <= 9; ++j) s = dot2_acc(Fr[j], 1.0f, 1.0f, s);
    return __builtin_fmaf(c.inv_scale_f, s, f0);
  } else {
    float d[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) d[i] = f_of<S>(Fr, i);
    return lean_phi(c, f0, d);
  }
}
template <int S>
__device__ __forceinline__ void lean_moments_packed(const CaseDev& c, const uint32_t* Gr,
                                                    float& m0, float& mx, float& my,
                                                    float& mz) {
  if constexpr (S == ST_FP16) {
    // Gr[k] holds directions 2k and 2k + 1 (Gr[9]: direction 18 and a zero
    // half); each sum runs over the words in order, skipping words whose
    // weights are both zero
    float a = 0.0f, sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      const int i0 = 2 * k, i1 = 2 * k + 1 < Q ? 2 * k + 1 : 0;
      const float b1 = 2 * k + 1 < Q ? 1.0f : 0.0f;
      a = dot2_acc(Gr[k], 1.0f, b1, a);
      if (EX(i0) || (i1 && EX(i1))) sx = dot2_acc(Gr[k], EX(i0), i1 ? EX(i1) : 0, sx);
      if (EY(i0) || (i1 && EY(i1))) sy = dot2_acc(Gr[k], EY(i0), i1 ? EY(i1) : 0, sy);
      if (EZ(i0) || (i1 && EZ(i1))) sz = dot2_acc(Gr[k], EZ(i0), i1 ? EZ(i1) : 0, sz);
    }
    m0 = __builtin_fmaf(c.inv_scale_g, a, c.p0);
    mx = c.inv_scale_g * sx;
    my = c.inv_scale_g * sy;
    mz = c.inv_scale_g * sz;
  } else {
    float G[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) G[i] = g_of<S>(Gr, i);
    lean_moments(c, G, m0, mx, my, mz);
  }
}

// Inputs of the collision at a node.
struct LeanNode {
  float ph, mu, cc, p, ux, uy, uz, gx, gy, gz;  // cc: -F_a = cc u
};

// BGK collision of f and gbar with the Eq. 8 forcing on the stored values:
//   gbar* = gbar - (gbar - g^eq)/tau + (1 - 1/2tau)(e - u).K,
//   f*    = f - (f - f^eq)/tau_f,
// written per opposite pair (i, i') = (2j-1, 2j) with t_i = 3 e.u + 4.5 (e.u)^2
// - 1.5 u^2 = q +- r (q = 4.5 (e.u)^2 - 1.5 u^2, r = 3 e.u):
//   gbar*_i - w_i p0 = (1 - om)(gbar_i - w_i p0) + w_i (S +- D),
//   S = A' + q C + r d,  D = b + q d + r C,
// A' = om (p - p0) - h u.F, C = om rho/3 - h u.F + h u.grad psi, b = h e.F,
// d = h e.(F - grad psi), h = 1 - om/2, om = 1/tau(x); and
//   f*_i = (1 - om_f) f_i + w_i (P +- R),  P = om_f (3 Gamma mu + phi q),
// R = om_f phi r.  In stored units (times s_g, s_f) w_i becomes w_i s.
// F = F_s + G + cc u, grad psi = grad p - drho/3 grad phi.
//   Gr, Fr: the node's packed stored words (see f_of / g_of);
//   outg, outf: the packed encoded results in the same layout (f rounded to
//   nearest, g stochastically with the bits sr_bits(nkey, plane));
//   returns f_0* = phi - sum_{i>0} f*_i of the stored values.
template <int S>
__device__ __forceinline__ float lean_collide(const CaseDev& c, const LeanNode& n, float gpx,
                                              float gpy, float gpz, const uint32_t* Gr,
                                              const uint32_t* Fr, uint32_t* outg,
                                              uint32_t* outf, uint32_t nkey) {
  const float ph = n.ph, ux = n.ux, uy = n.uy, uz = n.uz;
  const float rho = __builtin_fmaf(ph, c.drho, c.rho0);
  const float fx = __builtin_fmaf(n.cc, ux, n.mu * n.gx);
  const float fy = __builtin_fmaf(n.cc, uy, n.mu * n.gy);
  const float fz = __builtin_fmaf(n.cc, uz, __builtin_fmaf(n.mu, n.gz,
                                                           -(rho - c.rho_ref) * c.gravity));
  const float k3 = (1.0f / 3.0f) * c.drho;
  const float psx = __builtin_fmaf(-k3, n.gx, gpx);
  const float psy = __builtin_fmaf(-k3, n.gy, gpy);
  const float psz = __builtin_fmaf(-k3, n.gz, gpz);
  const float mud = __builtin_fmaf(ph, c.dmu, c.mu0);
  const float om = rho * __builtin_amdgcn_rcpf(__builtin_fmaf(0.5f, rho, 3.0f * mud));
  const float h = __builtin_fmaf(-0.5f, om, 1.0f);
  const float omg = 1.0f - om;
  const float uu = __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
  const float uf = __builtin_fmaf(ux, fx, __builtin_fmaf(uy, fy, uz * fz));
  const float ug = __builtin_fmaf(ux, psx, __builtin_fmaf(uy, psy, uz * psz));
  const float hu = h * uf;
  const float A = __builtin_fmaf(om, n.p - c.p0, -hu);
  const float C = __builtin_fmaf(h, ug, __builtin_fmaf(om * (1.0f / 3.0f), rho, -hu));
  const float hfx = h * fx, hfy = h * fy, hfz = h * fz;
  const float hdx = h * (fx - psx), hdy = h * (fy - psy), hdz = h * (fz - psz);
  const float m15 = -1.5f * uu;
  const float omf = 1.0f - c.omega_f;
  const float fP = c.omega_f * (c.gamma3 * n.mu);  // om_f 3 Gamma mu
  const float fQ = c.omega_f * ph;
  const float sg = c.scale_g, sf = c.scale_f;
  // rest direction: t_0 = m15, S = A + m15 C
  const float x0 = __builtin_fmaf(m15, C, A);
  float gprev = __builtin_fmaf(omg, g_of<S>(Gr, 0), ((1.0f / 3.0f) * sg) * x0);
  float fsum = 0.0f;
#pragma unroll
  for (int j = 1; j <= 9; ++j) {
    const int i = PI(j);
    const float eu = edot(i, ux, uy, uz);
    const float b = edot(i, hfx, hfy, hfz);
    const float d = edot(i, hdx, hdy, hdz);
    const float r = 3.0f * eu;
    const float q = __builtin_fmaf(4.5f * eu, eu, m15);
    const float Sv = __builtin_fmaf(r, d, __builtin_fmaf(q, C, A));
    const float Dv = __builtin_fmaf(r, C, __builtin_fmaf(q, d, b));
    const float ws = WT(i) * sg;
    const float gp = __builtin_fmaf(omg, g_of<S>(Gr, i), ws * (Sv + Dv));
    const float gm = __builtin_fmaf(omg, g_of<S>(Gr, i + 1), ws * (Sv - Dv));
    // f: P +- R with P = om_f (3 Gamma mu + phi q), R = om_f phi r
    const float P = __builtin_fmaf(fQ, q, fP);
    const float R = fQ * r;
    const float wf = WT(i) * sf;
    const float fp = __builtin_fmaf(omf, f_of<S>(Fr, i), wf * (P + R));
    const float fm = __builtin_fmaf(omf, f_of<S>(Fr, i + 1), wf * (P - R));
    const uint32_t ef = enc_pair<S>(fp, fm);
    outf[j] = ef;
    if constexpr (S == ST_FP16) fsum = dot2_acc(ef, 1.0f, 1.0f, fsum);
    else fsum += lo16<S>(ef) + hi16<S>(ef);
    // g planes 2j-2, 2j-1
    outg[j - 1] = enc_pair_sr<S>(gprev, gp, sr_bits(nkey, 2 * j - 2), sr_bits(nkey, 2 * j - 1));
    gprev = gm;  // plane 2j goes with the next pair
  }
  outg[9] = enc_pair_sr<S>(gprev, 0.0f, sr_bits(nkey, 18), 0u);  // g_18 alone in the low half
  return __builtin_fmaf(-c.inv_scale_f, fsum, ph);
}

}  // namespace d3q19
}  // namespace lbm
