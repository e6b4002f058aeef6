// lbm_dev.h -- device-side definitions shared by the gfx950 kernels of the
// phase-field lattice Boltzmann library: per-case table entry, population
// storage codecs and pull-streaming index helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

enum Storage { ST_FP32 = 0, ST_FP16 = 1, ST_BF16 = 2 };

// One case as the kernels see it.  All physical constants are pre-derived on
// the host in double and rounded once to float.
struct CaseDev {
  int nx, ny, nz;
  int wall_x, wall_y, wall_z;
  int n;            // nodes
  unsigned stride;  // elements per population plane (>= n); a copy is < 4 GiB,
                    // so every byte offset into it fits 32 bits
  char* state[2];   // the two copies of the stored populations
  unsigned* clock;  // step counter of the 16-bit stochastic rounding: a step
                    // reading copy p reads clock[p] and sets clock[1 - p] to
                    // one more (so graph replays need no host update)
  // physics (float)
  // theta'(phi) = th_k phi (phi - th_r1) (phi - th_r2): the asymmetric well
  // beta phi^2 (phi-1)^2 has th_k = 4 beta, roots 1 and 1/2; the symmetric
  // well beta (phi^2 - phi*^2)^2 has th_k = 4 beta, roots phi* and -phi*
  float th_k, th_r1, th_r2;
  float kappa;
  float gamma3;     // 3 Gamma, Gamma = theta_M / (tau_f - 1/2)
  float omega_f;    // 1 / tau_f
  float rho0, drho; // rho = rho0 + drho phi (Eq. 4a: rho_G, rho_L - rho_G;
                    // Eq. 4b: (rho_L + rho_G) / 2, (rho_L - rho_G) / (2 phi*))
  float mu0, dmu;   // dynamic viscosity mu0 + dmu phi, mu_G at the gas value
                    // of phi and mu_L at the liquid value
  float wa, wb;     // diagnostic weight w = wa phi + wb before clamping to [0, 1]:
                    // 0, 1/2, 1 at a quarter, half, three quarters of the way
                    // from the gas to the liquid value of phi
  float gravity, rho_ref;
  float corr;       // drho * theta_M for remove_fa = 1, else 0 (coefficient of lap mu
                    // in -F_a / u)
  float fa_coef;    // drho * theta_M           (F_a dump, whichever model runs)
  float p0;         // rest pressure of the 16-bit g deviations
  float scale_f, inv_scale_f, scale_g, inv_scale_g;
  unsigned phiv;    // remove_fa = 2: byte offset, within a copy, of the float plane
                    // holding phi of the step that wrote the copy; 0 otherwise
};

// theta'(phi) of the double well (Eq. 1a / 1b), with phi = hi + lo carried as
// two floats: phi - th_r1 and phi - th_r2 are formed before rounding to one
// float, so they keep their absolute precision near the roots (the bulk values
// of phi and the interface midpoint).
__device__ __forceinline__ float dtheta(const CaseDev& c, float hi, float lo) {
  const float a = hi + lo;
  const float b = (hi - c.th_r1) + lo;
  const float d = (hi - c.th_r2) + lo;
  return c.th_k * a * b * d;
}

// Per-tile work item: case index and tile origin.
struct TileDev {
  int icase, x0, y0, z0;
};

// ---------------------------------------------------------------- codecs
__device__ __forceinline__ uint16_t enc_bf16(float v) {
  uint32_t b = __float_as_uint(v);
  if ((b & 0x7f800000u) == 0x7f800000u) {  // Inf / NaN: keep, quiet NaN
    return (uint16_t)((b >> 16) | ((b & 0x007fffffu) ? 0x40u : 0u));
  }
  b += 0x7fffu + ((b >> 16) & 1u);          // round to nearest even
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float dec_bf16(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}
__device__ __forceinline__ uint16_t enc_fp16(float v) {
  return __half_as_ushort(__float2half_rn(v));
}
__device__ __forceinline__ float dec_fp16(uint16_t h) {
  return __half2float(__ushort_as_half(h));
}
template <int S>
__device__ __forceinline__ uint16_t enc16(float v) {
  if constexpr (S == ST_BF16) return enc_bf16(v);
  else return enc_fp16(v);
}
template <int S>
__device__ __forceinline__ float dec16(uint16_t h) {
  if constexpr (S == ST_BF16) return dec_bf16(h);
  else return dec_fp16(h);
}

// ---------------------------------------------------------------- stochastic rounding
// The 16-bit g stores of a time step round stochastically: a value between two
// neighbours of the 16-bit format becomes the upper one with probability equal
// to its fractional distance from the lower one, so the rounding error has
// mean zero whatever the value.  Round to nearest returns the same error for
// the same value at every step, and the hydrodynamic populations of a slowly
// varying flow hold nearly the same values from step to step: their rounding
// then acts like a steady spurious force.
//
// Random bits: a counter-based generator, the 32-bit "lowbias32" integer hash
// of C. Wellons (xorshift-multiply rounds with constants 0x7feb352d and
// 0x846ca68b), keyed by the time step once per launch and by the node index
// once per node; the directions of a node take that key plus i times
// 0x9e3779b9 (a Weyl sequence), each value then uniform on 32 bits.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__host__ __device__ __forceinline__ uint32_t sr_step_key(uint32_t t) {
  return mix32(t * 0x9e3779b9u + 0x6a09e667u);
}
__host__ __device__ __forceinline__ uint32_t sr_node_key(uint32_t step_key, unsigned idx) {
  return mix32(idx ^ step_key);
}
__host__ __device__ __forceinline__ uint32_t sr_bits(uint32_t node_key, int i) {
  return node_key + (uint32_t)i * 0x9e3779b9u;
}
// The float bits of v with r's top bits added below the last bit the 16-bit
// format keeps, then cut there: FP16 keeps 10 of the 23 fraction bits (13 bits
// cut, exact in the FP16 normal range), BF16 keeps 7 (16 cut, the upper half is
// the BF16 word).  A carry into the exponent is the rounding up to the next
// binade.  Inf stays Inf and NaN stays NaN: a NaN or Inf that came through the
// 16-bit format has zeros in the cut bits, so the addition cannot carry out of
// its fraction.
template <int S>
__device__ __forceinline__ uint32_t sr_word(float v, uint32_t r) {
  if constexpr (S == ST_BF16) return __float_as_uint(v) + (r >> 16);
  else return (__float_as_uint(v) + (r >> 19)) & 0xffffe000u;
}
template <int S>
__device__ __forceinline__ uint16_t enc16_sr(float v, uint32_t r) {
  const uint32_t b = sr_word<S>(v, r);
  if constexpr (S == ST_BF16) return (uint16_t)(b >> 16);
  else return enc_fp16(__uint_as_float(b));
}
// Read this step's counter; one thread of the launch sets the next step's.
__device__ __forceinline__ uint32_t sr_clock(const CaseDev& c, int parity) {
  const uint32_t t = c.clock[parity];
  if (blockIdx.x == 0 && threadIdx.x == 0) c.clock[parity ^ 1] = t + 1u;
  return t;
}

// Bytes of one copy of the stored populations for q velocities.
//   FP32:       2q float planes (f_0..f_{q-1}, g_0..g_{q-1}), then one BF16
//               plane holding the low part of f_0: f_0 = hi + lo carries the
//               order parameter (f_0 ~ phi ~ 1 in the liquid) to ~1e-9
//               instead of the 6e-8 of one float
//   FP16/BF16:  one float plane (f_0), then 2q-1 16-bit planes
//               (f_1..f_{q-1}, g_0..g_{q-1})
// then, with phi_plane, one float plane of phi (the correction from data needs
// phi one step back; a copy carries the phi of the step that wrote it).
__host__ __device__ inline size_t copy_bytes(int storage, int q, long long stride,
                                             bool phi_plane = false) {
  const size_t pops = storage == ST_FP32 ? (size_t)(2 * q) * 4 * stride + (size_t)2 * stride
                                         : (size_t)4 * stride + (size_t)(2 * q - 1) * 2 * stride;
  return pops + (phi_plane ? (size_t)4 * stride : 0);
}

// Error-free transformation s + e = a + b (round to nearest, no reassociation).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Global-memory access.  The state pointers live in a table, so the compiler
// would treat them as generic (flat) pointers; casting to the global address
// space, with a uniform base and a 32-bit per-lane byte offset, gives
// global_load/global_store in their scalar-base form and keeps memory waits
// apart from LDS waits.
#define LBM_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T gload(const char* base, unsigned byte_off) {
  return *(const LBM_GLOBAL T*)((const LBM_GLOBAL char*)base + byte_off);
}
template <class T>
__device__ __forceinline__ void gstore(char* base, unsigned byte_off, T v) {
  *(LBM_GLOBAL T*)((LBM_GLOBAL char*)base + byte_off) = v;
}
// Store of a population (or of a field plane that the next kernel reads once):
// a word written once per step and read again only after the whole grid has
// been swept.  The non-temporal hint streams it past the caches, so it does
// not displace the lines the kernel re-reads (halo positions, stencil planes).
template <class T>
__device__ __forceinline__ void gstore_nt(char* base, unsigned byte_off, T v) {
  __builtin_nontemporal_store(v, (LBM_GLOBAL T*)((LBM_GLOBAL char*)base + byte_off));
}

// Plane layout of one copy (Q velocities):
//   FP32:      f_0..f_{Q-1}, g_0..g_{Q-1} as float planes, then the BF16 low
//              part of f_0
//   FP16/BF16: f_0 as a float plane, then f_1..f_{Q-1}, g_0..g_{Q-1} as
//              16-bit planes
// Offsets are bytes from the start of the copy.
template <int S, int Q>
struct Pops {
  static __device__ __forceinline__ unsigned fofs(const CaseDev& c, int i, unsigned j) {
    if constexpr (S == ST_FP32) return ((unsigned)i * c.stride + j) * 4u;
    else return i == 0 ? j * 4u : 4u * c.stride + ((unsigned)(i - 1) * c.stride + j) * 2u;
  }
  static __device__ __forceinline__ unsigned gofs(const CaseDev& c, int i, unsigned j) {
    if constexpr (S == ST_FP32) return ((unsigned)(Q + i) * c.stride + j) * 4u;
    else return 4u * c.stride + ((unsigned)(Q - 1 + i) * c.stride + j) * 2u;
  }
  // Stored word of f_i (i > 0) and g_i -> value
  static __device__ __forceinline__ float dec_f(const CaseDev& c, float w) { return w; }
  static __device__ __forceinline__ float dec_f(const CaseDev& c, uint16_t w) {
    return dec16<S>(w) * c.inv_scale_f;
  }
  static __device__ __forceinline__ float dec_g(const CaseDev& c, float w, float wi) { return w; }
  static __device__ __forceinline__ float dec_g(const CaseDev& c, uint16_t w, float wi) {
    return dec16<S>(w) * c.inv_scale_g + wi * c.p0;
  }
  // low part of f_0 from its stored BF16 word (FP32 storage only; zero otherwise)
  static __device__ __forceinline__ float dec_lo(uint16_t w) {
    if constexpr (S == ST_FP32) return dec_bf16(w);
    else return 0.0f;
  }
  // f_i at a byte offset (i only selects the width: f_0 is always a float)
  static __device__ __forceinline__ float f(const CaseDev& c, const char* base, int i,
                                            unsigned ofs) {
    if constexpr (S == ST_FP32) {
      return gload<float>(base, ofs);
    } else {
      if (i == 0) return gload<float>(base, ofs);
      return dec_f(c, gload<uint16_t>(base, ofs));
    }
  }
  static __device__ __forceinline__ float g(const CaseDev& c, const char* base, unsigned ofs,
                                            float wi) {
    if constexpr (S == ST_FP32) return gload<float>(base, ofs);
    else return dec_g(c, gload<uint16_t>(base, ofs), wi);
  }
  // low part of f_0 (FP32 storage only; zero otherwise)
  static __device__ __forceinline__ float f0lo(const CaseDev& c, const char* base, unsigned j) {
    if constexpr (S == ST_FP32) {
      return dec_lo(gload<uint16_t>(base, (unsigned)(2 * Q) * 4u * c.stride + 2u * j));
    } else {
      return 0.0f;
    }
  }
  // Quantise f_i (i > 0) to what the store will hold, store it at node j.
  static __device__ __forceinline__ float put_f(const CaseDev& c, char* base, int i, unsigned j,
                                                float v) {
    if constexpr (S == ST_FP32) {
      gstore_nt<float>(base, fofs(c, i, j), v);
      return v;
    } else {
      const uint16_t h = enc16<S>(v * c.scale_f);
      gstore_nt<uint16_t>(base, fofs(c, i, j), h);
      return Pops<S, Q>::dec_f(c, h);
    }
  }
  // f_0 = hi + lo; the 16-bit layouts keep hi + lo rounded to one float
  static __device__ __forceinline__ void put_f0(const CaseDev& c, char* base, unsigned j,
                                                float hi, float lo) {
    if constexpr (S == ST_FP32) {
      float h, l;
      two_sum(hi, lo, h, l);
      gstore_nt<float>(base, 4u * j, h);
      gstore_nt<uint16_t>(base, (unsigned)(2 * Q) * 4u * c.stride + 2u * j, enc_bf16(l));
    } else {
      gstore_nt<float>(base, 4u * j, hi + lo);
    }
  }
  static __device__ __forceinline__ void put_g(const CaseDev& c, char* base, int i, unsigned j,
                                               float v, float wi) {
    if constexpr (S == ST_FP32) {
      (void)wi;
      gstore_nt<float>(base, gofs(c, i, j), v);
    } else {
      gstore_nt<uint16_t>(base, gofs(c, i, j), enc16<S>((v - wi * c.p0) * c.scale_g));
    }
  }
};

// Uniform per-plane destination pointers of one copy: every store of a node
// then uses the same per-lane offset (4 idx for float planes, 2 idx for
// 16-bit planes).
template <int S, int Q>
struct OutPtrs {
  char* f[Q];
  char* g[Q];
  char* f0lo;
  __device__ __forceinline__ OutPtrs(const CaseDev& c, char* base) {
    using P = Pops<S, Q>;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      f[i] = base + P::fofs(c, i, 0);
      g[i] = base + P::gofs(c, i, 0);
    }
    f0lo = base + (size_t)(2 * Q) * 4 * c.stride;
  }
  // store f_i (i > 0) at node idx; returns what was stored (decoded)
  __device__ __forceinline__ float put_f(const CaseDev& c, int i, unsigned idx, float v) const {
    if constexpr (S == ST_FP32) {
      gstore_nt<float>(f[i], 4u * idx, v);
      return v;
    } else {
      const uint16_t h = enc16<S>(v * c.scale_f);
      gstore_nt<uint16_t>(f[i], 2u * idx, h);
      return Pops<S, Q>::dec_f(c, h);
    }
  }
  // store g_i at node idx; 16-bit: rounded stochastically with the bits r
  __device__ __forceinline__ void put_g(const CaseDev& c, int i, unsigned idx, float v,
                                        float wi, uint32_t r) const {
    if constexpr (S == ST_FP32) gstore_nt<float>(g[i], 4u * idx, v);
    else gstore_nt<uint16_t>(g[i], 2u * idx, enc16_sr<S>((v - wi * c.p0) * c.scale_g, r));
  }
  __device__ __forceinline__ void put_f0(unsigned idx, float hi, float lo) const {
    if constexpr (S == ST_FP32) {
      float h, l;
      two_sum(hi, lo, h, l);
      gstore_nt<float>(f[0], 4u * idx, h);
      gstore_nt<uint16_t>(f0lo, 2u * idx, enc_bf16(l));
    } else {
      gstore_nt<float>(f[0], 4u * idx, hi + lo);
    }
  }
};

// Coordinate of a stencil position on one axis: periodic wrap, or the mirror
// ghost of a wall half a cell beyond the last node (ghost -k <-> node k-1),
// clamped so that positions far outside (never used by a real node) still
// address memory inside the grid.
__device__ __forceinline__ int map_axis(int g, int n, int wall) {
  if (wall) {
    if (g < 0) g = -g - 1;
    else if (g >= n) g = 2 * n - 1 - g;
    return g < 0 ? 0 : (g >= n ? n - 1 : g);
  }
  g %= n;
  return g < 0 ? g + n : g;
}

// Local coordinate (in a region whose first position has global coordinate
// origin) holding the real node that a position mirrors.  Unchanged on
// periodic axes and for positions inside the grid.
__device__ __forceinline__ int mirror_local(int l, int origin, int n, int wall, int width) {
  if (!wall) return l;
  int g = origin + l;
  if (g >= 0 && g < n) return l;
  g = (g < 0) ? -g - 1 : 2 * n - 1 - g;
  int lm = g - origin;
  return lm < 0 ? 0 : (lm >= width ? width - 1 : lm);
}

// Pull source of direction i at node (x, y, z): the neighbour x - e_i (with
// periodic wrap), or the node itself with the opposite direction when x - e_i
// lies beyond a wall (halfway bounce-back).  Returns the source node and sets
// *bb when the opposite direction is to be read.
__device__ __forceinline__ unsigned pull_src(const CaseDev& c, int x, int y, int z, int ex,
                                             int ey, int ez, bool* bb) {
  int sx = x - ex, sy = y - ey, sz = z - ez;
  bool b = false;
  if (sx < 0 || sx >= c.nx) {
    if (c.wall_x) b = true;
    else sx = sx < 0 ? sx + c.nx : sx - c.nx;
  }
  if (sy < 0 || sy >= c.ny) {
    if (c.wall_y) b = true;
    else sy = sy < 0 ? sy + c.ny : sy - c.ny;
  }
  if (sz < 0 || sz >= c.nz) {
    if (c.wall_z) b = true;
    else sz = sz < 0 ? sz + c.nz : sz - c.nz;
  }
  *bb = b;
  if (b) return (unsigned)(x + c.nx * (y + c.ny * z));
  return (unsigned)(sx + c.nx * (sy + c.ny * sz));
}

}  // namespace lbm
