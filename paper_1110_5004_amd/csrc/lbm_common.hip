// lbm_common.hip -- lattice-independent gfx950 kernels: streaming of raw
// words (the exact pull permutation of the step), 16-bit encoding, the
// bandwidth-calibration copies, the paper-experiment diagnostics (spread
// radius, F_a from discrete data and in Lee and Lin's form), and the
// fixed-order FP64 diagnostics reduction.
#include "lbm_dev.h"
#include "lbm_kernels.h"
#include "lbm_lattice.h"

namespace lbm {

template <int LAT>
__global__ void __launch_bounds__(256)
k_stream_words(CaseDev c, const uint32_t* __restrict__ in, uint32_t* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c.n) return;
  const int x = idx % c.nx;
  const int y = (idx / c.nx) % c.ny;
  const int z = idx / (c.nx * c.ny);
  constexpr int Q = LAT == 0 ? d2q9::Q : d3q19::Q;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int ex, ey, ez, op;
    if constexpr (LAT == 0) {
      ex = d2q9::EX(i); ey = d2q9::EY(i); ez = 0; op = d2q9::OPP(i);
    } else {
      ex = d3q19::EX(i); ey = d3q19::EY(i); ez = d3q19::EZ(i); op = d3q19::OPP(i);
    }
    int dir = i;
    unsigned j = idx;
    if (i > 0) {
      bool bb;
      j = pull_src(c, x, y, z, ex, ey, ez, &bb);
      if (bb) dir = op;
    }
    out[(size_t)i * c.n + idx] = in[(size_t)dir * c.n + j];
  }
}

hipError_t stream_words(int lattice, const CaseDev& c, const uint32_t* in, uint32_t* out,
                        hipStream_t stream) {
  const int grid = (c.n + 255) / 256;
  if (lattice == 0)
    hipLaunchKernelGGL(k_stream_words<0>, dim3(grid), dim3(256), 0, stream, c, in, out);
  else
    hipLaunchKernelGGL(k_stream_words<1>, dim3(grid), dim3(256), 0, stream, c, in, out);
  return hipGetLastError();
}

template <int S>
__global__ void __launch_bounds__(256)
k_encode16(const float* __restrict__ in, uint16_t* __restrict__ out, long long n) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    out[k] = enc16<S>(in[k]);
}

// The stochastic rounding of the step's g stores (sr_word) applied to in[k] as
// the step with counter t stores direction dir of node k.
template <int S>
__global__ void __launch_bounds__(256)
k_encode16_sr(const float* __restrict__ in, uint16_t* __restrict__ out, long long n, uint32_t t,
              int dir) {
  const uint32_t sk = sr_step_key(t);
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    out[k] = enc16_sr<S>(in[k], sr_bits(sr_node_key(sk, (unsigned)k), dir));
}

hipError_t encode16_sr(int storage, const float* in, uint16_t* out, long long n, uint32_t t,
                       int dir, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  const int grid = (int)(blocks < 65536 ? blocks : 65536);
  if (storage == ST_BF16)
    hipLaunchKernelGGL(k_encode16_sr<ST_BF16>, dim3(grid), dim3(256), 0, stream, in, out, n, t,
                       dir);
  else
    hipLaunchKernelGGL(k_encode16_sr<ST_FP16>, dim3(grid), dim3(256), 0, stream, in, out, n, t,
                       dir);
  return hipGetLastError();
}

hipError_t encode16(int storage, const float* in, uint16_t* out, long long n,
                    hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  const int grid = (int)(blocks < 65536 ? blocks : 65536);
  if (storage == ST_BF16)
    hipLaunchKernelGGL(k_encode16<ST_BF16>, dim3(grid), dim3(256), 0, stream, in, out, n);
  else
    hipLaunchKernelGGL(k_encode16<ST_FP16>, dim3(grid), dim3(256), 0, stream, in, out, n);
  return hipGetLastError();
}

// Coalesced 16-byte copy; tail handled element-wise.
__global__ void __launch_bounds__(256)
k_copy(const float* __restrict__ in, float* __restrict__ out, long long n) {
  // four 16-byte words per thread and round, non-temporal loads and stores:
  // the fastest plain copy measured here (5.9 TB/s HBM-resident against 4.9
  // for one word per thread and cached accesses)
  typedef float v4f __attribute__((ext_vector_type(4)));
  const long long n4 = n / 4;
  const v4f* i4 = reinterpret_cast<const v4f*>(in);
  v4f* o4 = reinterpret_cast<v4f*>(out);
  constexpr int U = 4;
  const long long step = (long long)gridDim.x * blockDim.x * U;
  for (long long k = blockIdx.x * (long long)blockDim.x * U + threadIdx.x; k < n4; k += step) {
    v4f v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = k + (long long)u * blockDim.x;
      if (j < n4) v[u] = __builtin_nontemporal_load(&i4[j]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = k + (long long)u * blockDim.x;
      if (j < n4) __builtin_nontemporal_store(v[u], &o4[j]);
    }
  }
  for (long long k = n4 * 4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    out[k] = in[k];
}

hipError_t copy_bw(const float* in, float* out, long long n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n / 16 + 255) / 256;
  const int grid = (int)(blocks < 32768 ? (blocks > 0 ? blocks : 1) : 32768);
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, stream, in, out, n);
  return hipGetLastError();
}

// Pull-copy: the data movement of one step without its arithmetic.  Every
// stored word of node idx is read from the node the step pulls it from
// (x - e_i, or idx itself where that leaves the grid) and written to idx,
// with the non-temporal stores of the step kernels.
template <int LAT, int S>
__global__ void __launch_bounds__(256)
k_pull_copy(CaseDev c, const char* __restrict__ src, char* __restrict__ dst) {
  constexpr int Q = LAT == 0 ? d2q9::Q : d3q19::Q;
  using P = Pops<S, Q>;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c.n) return;
  const int x = idx % c.nx;
  const int y = (idx / c.nx) % c.ny;
  const int z = idx / (c.nx * c.ny);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int ex, ey, ez;
    if constexpr (LAT == 0) {
      ex = d2q9::EX(i); ey = d2q9::EY(i); ez = 0;
    } else {
      ex = d3q19::EX(i); ey = d3q19::EY(i); ez = d3q19::EZ(i);
    }
    const bool in = x - ex >= 0 && x - ex < c.nx && y - ey >= 0 && y - ey < c.ny &&
                    z - ez >= 0 && z - ez < c.nz;
    const unsigned j = in ? (unsigned)(idx - ex - c.nx * (ey + c.ny * ez)) : (unsigned)idx;
    if (S == ST_FP32 || i == 0)
      gstore_nt<uint32_t>(dst, P::fofs(c, i, idx), gload<uint32_t>(src, P::fofs(c, i, j)));
    else
      gstore_nt<uint16_t>(dst, P::fofs(c, i, idx), gload<uint16_t>(src, P::fofs(c, i, j)));
    if (S == ST_FP32)
      gstore_nt<uint32_t>(dst, P::gofs(c, i, idx), gload<uint32_t>(src, P::gofs(c, i, j)));
    else
      gstore_nt<uint16_t>(dst, P::gofs(c, i, idx), gload<uint16_t>(src, P::gofs(c, i, j)));
  }
  if (S == ST_FP32) {
    const unsigned lo = (unsigned)(2 * Q) * 4u * c.stride;
    gstore_nt<uint16_t>(dst, lo + 2u * idx, gload<uint16_t>(src, lo + 2u * idx));
  }
}

hipError_t pull_copy(int lattice, int storage, const CaseDev& c, const void* src, void* dst,
                     hipStream_t stream) {
  const int grid = (c.n + 255) / 256;
  const char* s = static_cast<const char*>(src);
  char* d = static_cast<char*>(dst);
  if (lattice == 0) {
    if (storage == ST_FP32)
      hipLaunchKernelGGL((k_pull_copy<0, ST_FP32>), dim3(grid), dim3(256), 0, stream, c, s, d);
    else
      hipLaunchKernelGGL((k_pull_copy<0, ST_FP16>), dim3(grid), dim3(256), 0, stream, c, s, d);
  } else {
    if (storage == ST_FP32)
      hipLaunchKernelGGL((k_pull_copy<1, ST_FP32>), dim3(grid), dim3(256), 0, stream, c, s, d);
    else
      hipLaunchKernelGGL((k_pull_copy<1, ST_FP16>), dim3(grid), dim3(256), 0, stream, c, s, d);
  }
  return hipGetLastError();
}

// Spread radius (the droplet half-width of the paper's falling-droplet
// comparison): one 64-lane workgroup per grid row in x.  Each lane scans a
// strided subset of the node pairs (x, x + 1), x = 0 .. nx - 2, for crossings
// of phi = level (exactly one of the two >= level), located by linear
// interpolation in double; min / max and the count combine across the wave
// (exact operations, so the result does not depend on the order).  Out:
// half the distance between the row's outermost crossings, or -1 when the row
// has fewer than two.
__global__ void __launch_bounds__(64)
k_row_spread(int nx, const float* __restrict__ phi, double level, double* __restrict__ out) {
  const long row = blockIdx.x;
  const float* r = phi + row * nx;
  double lo = 1e300, hi = -1e300;
  int cnt = 0;
  for (int x = threadIdx.x; x + 1 < nx; x += 64) {
    const double a = r[x], b = r[x + 1];
    if ((a >= level) == (b >= level)) continue;
    const double pos = x + (level - a) / (b - a);
    lo = fmin(lo, pos);
    hi = fmax(hi, pos);
    ++cnt;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
    cnt += __shfl_xor(cnt, off, 64);
  }
  if (threadIdx.x == 0) out[row] = cnt >= 2 ? 0.5 * (hi - lo) : -1.0;
}

hipError_t row_spread(const CaseDev& c, const float* phi, double level, double* out,
                      hipStream_t stream) {
  const int rows = c.ny * c.nz;
  hipLaunchKernelGGL(k_row_spread, dim3(rows), dim3(64), 0, stream, c.nx, phi, level, out);
  return hipGetLastError();
}

// Neighbour coordinate g = x + d, |d| <= 1, on an axis of n nodes: the
// periodic image, or the mirror ghost of a wall (ghost -1 -> node 0, ghost n
// -> node n - 1), the neighbour convention of every stencil of the step.
__device__ __forceinline__ int step_axis(int g, int n, int wall) {
  if (g < 0) return wall ? 0 : n - 1;
  if (g >= n) return wall ? n - 1 : 0;
  return g;
}

// Launch shape of the node-parallel diagnostics: one grid row (y, z) per
// blockIdx.x, x across blockIdx.y * blockDim.x + threadIdx.x, so that no
// thread divides by a grid size.
struct RowLaunch {
  dim3 grid, block;
};
inline RowLaunch row_launch(const CaseDev& c) {
  const int bx = c.nx >= 256 ? 256 : ((c.nx + 63) / 64) * 64;
  return {dim3(c.ny * c.nz, (c.nx + bx - 1) / bx), dim3(bx)};
}

// Visits the Q - 1 moving directions of the lattice at node (x, y, z) as
// fn(neighbour index, w_i, e_x, e_y, e_z).
template <int LAT, class Fn>
__device__ __forceinline__ void for_neighbours(const CaseDev& c, int x, int y, int z, Fn&& fn) {
  constexpr int Q = LAT == 0 ? d2q9::Q : d3q19::Q;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    int ex, ey, ez;
    float w;
    if constexpr (LAT == 0) {
      ex = d2q9::EX(i); ey = d2q9::EY(i); ez = 0; w = d2q9::WT(i);
    } else {
      ex = d3q19::EX(i); ey = d3q19::EY(i); ez = d3q19::EZ(i); w = d3q19::WT(i);
    }
    const int mx = step_axis(x + ex, c.nx, c.wall_x);
    const int my = step_axis(y + ey, c.ny, c.wall_y);
    const int mz = LAT == 0 ? 0 : step_axis(z + ez, c.nz, c.wall_z);
    fn((unsigned)(mx + c.nx * (my + c.ny * mz)), w, ex, ey, ez);
  }
}

// F_a of Eq. 12 from discrete data: -u [(rho^n - rho^(n-1)) + div(rho u)^n],
// rho = rho0 + drho phi, the divergence 3 sum_i w_i e_i . (rho u)(x + e_i).
template <int LAT>
__global__ void __launch_bounds__(256)
k_fa_discrete(CaseDev c, const float* __restrict__ phi_prev, const float* __restrict__ phi,
              FieldPtrs f, float* __restrict__ out) {
  constexpr int DIM = LAT == 0 ? 2 : 3;
  const int x = blockIdx.y * blockDim.x + threadIdx.x;
  if (x >= c.nx) return;
  const int row = blockIdx.x;
  const int y = row % c.ny;
  const int z = row / c.ny;
  const unsigned idx = (unsigned)x + (unsigned)c.nx * row;
  float div = 0.0f;
  for_neighbours<LAT>(c, x, y, z, [&](unsigned j, float w, int ex, int ey, int ez) {
    const float rho = c.rho0 + phi[j] * c.drho;
    float eu = ex * f.u[0][j] + ey * f.u[1][j];
    if (DIM == 3) eu += ez * f.u[2][j];
    div += 3.0f * w * rho * eu;
  });
  const float dt_rho = (phi[idx] - phi_prev[idx]) * c.drho;
#pragma unroll
  for (int a = 0; a < DIM; ++a) out[(size_t)a * c.n + idx] = -f.u[a][idx] * (dt_rho + div);
}

hipError_t fa_discrete(int lattice, const CaseDev& c, const float* phi_prev, const FieldPtrs& f,
                       float* out, hipStream_t stream) {
  const RowLaunch L = row_launch(c);
  if (L.grid.y > 65535u) return hipErrorInvalidConfiguration;
  if (lattice == 0)
    hipLaunchKernelGGL(k_fa_discrete<0>, L.grid, L.block, 0, stream, c, phi_prev, f.phi, f, out);
  else
    hipLaunchKernelGGL(k_fa_discrete<1>, L.grid, L.block, 0, stream, c, phi_prev, f.phi, f, out);
  return hipGetLastError();
}

// F_a of Eq. 12 in Lee and Lin's form, Eq. 11: -u div[lambda grad(P - p)],
// expanded as lambda lap q + grad lambda . grad q with q = P - p, the
// isotropic central gradient 3 sum_i w_i e_i g(x + e_i) and Laplacian
// 6 sum_i w_i (g(x + e_i) - g(x)).  P = phi theta' - theta is the equation of
// state of the double well theta = beta (phi - phi_g)^2 (phi - phi_l)^2,
// written as beta a b (2 phi (a + b) - a b) with a = phi - phi_g,
// b = phi - phi_l; lambda = mu_dyn / (rho cs^2) = 3 (mu0 + dmu phi) /
// (rho0 + drho phi).
template <int LAT>
__global__ void __launch_bounds__(256)
k_fa_leelin(CaseDev c, WellArgs wa, FieldPtrs f, float* __restrict__ out) {
  constexpr int DIM = LAT == 0 ? 2 : 3;
  const int x = blockIdx.y * blockDim.x + threadIdx.x;
  if (x >= c.nx) return;
  const int row = blockIdx.x;
  const int y = row % c.ny;
  const int z = row / c.ny;
  const unsigned idx = (unsigned)x + (unsigned)c.nx * row;
  auto q_lam = [&](unsigned j, float& q, float& lam) {
    const float ph = f.phi[j];
    const float a = ph - wa.phi_g;
    const float b = ph - wa.phi_l;
    q = wa.beta * a * b * (2.0f * ph * (a + b) - a * b) - f.p[j];
    lam = 3.0f * (c.mu0 + c.dmu * ph) / (c.rho0 + c.drho * ph);
  };
  float q0, l0;
  q_lam(idx, q0, l0);
  float gq[3] = {0.0f, 0.0f, 0.0f}, gl[3] = {0.0f, 0.0f, 0.0f};
  float lap = 0.0f;
  for_neighbours<LAT>(c, x, y, z, [&](unsigned j, float w, int ex, int ey, int ez) {
    float q, l;
    q_lam(j, q, l);
    lap += w * (q - q0);
    gq[0] += w * ex * q;
    gq[1] += w * ey * q;
    gl[0] += w * ex * l;
    gl[1] += w * ey * l;
    if (DIM == 3) {
      gq[2] += w * ez * q;
      gl[2] += w * ez * l;
    }
  });
  float div = l0 * 6.0f * lap;
#pragma unroll
  for (int a = 0; a < DIM; ++a) div += 9.0f * gl[a] * gq[a];
#pragma unroll
  for (int a = 0; a < DIM; ++a) out[(size_t)a * c.n + idx] = -f.u[a][idx] * div;
}

hipError_t fa_leelin(int lattice, const CaseDev& c, const WellArgs& wa, const FieldPtrs& f,
                     float* out, hipStream_t stream) {
  const RowLaunch L = row_launch(c);
  if (L.grid.y > 65535u) return hipErrorInvalidConfiguration;
  if (lattice == 0)
    hipLaunchKernelGGL(k_fa_leelin<0>, L.grid, L.block, 0, stream, c, wa, f, out);
  else
    hipLaunchKernelGGL(k_fa_leelin<1>, L.grid, L.block, 0, stream, c, wa, f, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- FP64 reductions
// Diagnostics of node fields (phi, u) in two passes: sums (and one max) over
// the nodes, then the second moment about the centroid those sums give.
// Every node goes to a fixed thread of a fixed workgroup; threads combine by
// a fixed shuffle tree, waves by a fixed order through LDS, workgroups by a
// single-workgroup pass.  The result is therefore bit-reproducible.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// Combine one value per slot and thread of a 256-thread workgroup; slot
// DG_U2MAX by max, the others by sum; threads 0..kDiagSlots-1 write out.
__device__ __forceinline__ void block_combine(double* acc, double* sh, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < kDiagSlots; ++s) {
    const double v = (s == DG_U2MAX) ? wave_max(acc[s]) : wave_sum(acc[s]);
    if (lane == 0) sh[wave * kDiagSlots + s] = v;
  }
  __syncthreads();
  if (threadIdx.x < kDiagSlots) {
    const int s = threadIdx.x;
    double v = sh[s];
    for (int w = 1; w < 4; ++w)
      v = (s == DG_U2MAX) ? fmax(v, sh[w * kDiagSlots + s]) : v + sh[w * kDiagSlots + s];
    out[s] = v;
  }
}

__device__ __forceinline__ double centroid_weight(const DiagArgs& a, double ph) {
  const double w = a.wa * ph + a.wb;
  return w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
}

// pass 1: mass, momentum, weight, weighted position and velocity, max u^2,
// non-finite count
__global__ void __launch_bounds__(256) k_diag_sums(DiagArgs a, double* __restrict__ partials) {
  __shared__ double sh[4 * kDiagSlots];
  double acc[kDiagSlots];
#pragma unroll
  for (int s = 0; s < kDiagSlots; ++s) acc[s] = 0.0;
  const int stride = gridDim.x * blockDim.x;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < a.n; idx += stride) {
    const int x = idx % a.nx;
    const int y = (idx / a.nx) % a.ny;
    const int z = idx / (a.nx * a.ny);
    const double ph = a.phi[idx];
    const double rho = a.rho0 + ph * a.drho;
    const double w = centroid_weight(a, ph);
    const double xc[3] = {(double)x, (double)y, (double)z};
    acc[DG_MASS] += ph;
    double u2 = 0.0;
    bool finite = isfinite(ph);
    for (int d = 0; d < a.dim; ++d) {
      const double u = a.u[d][idx];
      acc[DG_MOM + d] += rho * u;
      acc[DG_CEN + d] += w * xc[d];
      acc[DG_CVEL + d] += w * u;
      u2 += u * u;
      finite = finite && isfinite(u);
    }
    acc[DG_WSUM] += w;
    acc[DG_U2MAX] = fmax(acc[DG_U2MAX], u2);
    if (!finite) acc[DG_BAD] += 1.0;
  }
  block_combine(acc, sh, partials + (size_t)blockIdx.x * kDiagSlots);
}

// pass 2: sum w (x - X)^2 per axis about the centroid X of pass 1 (out)
__global__ void __launch_bounds__(256)
k_diag_spread(DiagArgs a, const double* __restrict__ out, double* __restrict__ partials) {
  __shared__ double sh[4 * kDiagSlots];
  double acc[kDiagSlots];
#pragma unroll
  for (int s = 0; s < kDiagSlots; ++s) acc[s] = 0.0;
  const double cen[3] = {out[DG_CEN], out[DG_CEN + 1], out[DG_CEN + 2]};
  const int stride = gridDim.x * blockDim.x;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < a.n; idx += stride) {
    const int xc[3] = {idx % a.nx, (idx / a.nx) % a.ny, idx / (a.nx * a.ny)};
    const double w = centroid_weight(a, a.phi[idx]);
    for (int d = 0; d < a.dim; ++d) {
      const double dx = (double)xc[d] - cen[d];
      acc[DG_M2 + d] += w * dx * dx;
    }
  }
  block_combine(acc, sh, partials + (size_t)blockIdx.x * kDiagSlots);
}

// Combine the workgroup partials and finish: pass 1 writes every slot but
// DG_M2 (centroid and centroid velocity divided by the weight, |u|max), pass
// 2 only DG_M2 (divided by the weight of pass 1).  No weight: 0.
__global__ void __launch_bounds__(256)
k_diag_finish(const double* __restrict__ partials, int nblocks, int pass,
              double* __restrict__ out) {
  __shared__ double sh[4 * kDiagSlots];
  __shared__ double tot[kDiagSlots];
  double acc[kDiagSlots];
#pragma unroll
  for (int s = 0; s < kDiagSlots; ++s) acc[s] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) {
      const double v = partials[(size_t)b * kDiagSlots + s];
      acc[s] = (s == DG_U2MAX) ? fmax(acc[s], v) : acc[s] + v;
    }
  }
  block_combine(acc, sh, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (pass == 1) {
    const double ws = tot[DG_WSUM];
    out[DG_MASS] = tot[DG_MASS];
    out[DG_WSUM] = ws;
    for (int d = 0; d < 3; ++d) {
      out[DG_MOM + d] = tot[DG_MOM + d];
      out[DG_CEN + d] = ws > 0.0 ? tot[DG_CEN + d] / ws : 0.0;
      out[DG_CVEL + d] = ws > 0.0 ? tot[DG_CVEL + d] / ws : 0.0;
      out[DG_M2 + d] = 0.0;
    }
    out[DG_U2MAX] = sqrt(tot[DG_U2MAX]);
    out[DG_BAD] = tot[DG_BAD];
  } else {
    const double ws = out[DG_WSUM];
    for (int d = 0; d < 3; ++d) out[DG_M2 + d] = ws > 0.0 ? tot[DG_M2 + d] / ws : 0.0;
  }
}

hipError_t field_diag(const DiagArgs& a, double* partials, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_diag_sums, dim3(kReduceBlocks), dim3(256), 0, stream, a, partials);
  hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(256), 0, stream, partials, kReduceBlocks, 1,
                     out);
  hipLaunchKernelGGL(k_diag_spread, dim3(kReduceBlocks), dim3(256), 0, stream, a,
                     (const double*)out, partials);
  hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(256), 0, stream, partials, kReduceBlocks, 2,
                     out);
  return hipGetLastError();
}

}  // namespace lbm
