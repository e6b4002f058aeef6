// lbm_kernels.h -- host-side launch interface of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_dev.h"

namespace lbm {

struct TileShape {
  int tx, ty, tz;  // nodes per tile along x, y, z
  int nt;          // threads per workgroup
  int strip;       // width in nodes of the tile-list strips (0: the default)
  int form;        // D3Q19 step form (TileForm); D2Q9: 0
};

// D3Q19 step forms.  THREE: k3_pull, k3_fields_t on tx x ty x tz tiles,
// k3_collide.  FUSED: one kernel, a tx x ty tile of the x-y plane marching
// up a chunk of tz planes.  TWO (16-bit storage, every model): k3_pull, then
// k3_fcm, a tx x ty tile marching up a chunk of tz planes that forms the
// fields and collides.
enum TileForm { FORM_THREE = 0, FORM_FUSED = 1, FORM_TWO = 2 };

// Everything one step / field launch needs.
struct LaunchArgs {
  const CaseDev* cases;  // device case table
  const TileDev* tiles;  // device tile list
  int ntiles;
  int grid;              // workgroups (multiple of 8)
  int parity;            // copy holding the current populations
  int storage;
  int rf;                // 1: some case forms lap mu (corrected model)
  hipStream_t stream;
};

struct FieldPtrs {
  float* phi;
  float* u[3];
  float* p;
  float* mu;
  float* fa[3];
};

extern const TileShape kD2Q9Tiles[];
extern const TileShape kD2Q9FieldShape;  // tile of the D2Q9 field dump
extern const int kD2Q9TileCount;
extern const TileShape kD3Q19Tiles[];
extern const int kD3Q19TileCount;

hipError_t d2q9_step(int variant, const LaunchArgs& a);
hipError_t d2q9_fields(const LaunchArgs& a, const FieldPtrs& f);
hipError_t d2q9_init(const CaseDev& c, int storage, int parity, const double* phi0,
                     const double* u0, const double* p0, hipStream_t stream);

// D3Q19: per case and step either the fused kernel (no field planes) or three
// kernels passing 13 field planes (phi hi/lo, gbar moments, mu (field dump
// only), u, p, lap mu, and the rate D of the correction from data).
constexpr int kField3Planes = 13;
struct Field3Ptrs {
  float* plane[kField3Planes];
};
hipError_t d3q19_step_case(int variant, const CaseDev& c, int storage, int parity,
                           const Field3Ptrs& f, hipStream_t stream);
// The fused D3Q19 step for 16-bit storage (k3_march): tx x ty tiles of the
// x-y plane (32 x 8, 32 x 16 or 64 x 8) marching up chunks of zs planes.
hipError_t d3q19_march(const CaseDev& c, int storage, int tx, int ty, int zs, int parity,
                       hipStream_t stream);
hipError_t d3q19_fields_case(const CaseDev& c, int storage, int parity, const Field3Ptrs& f,
                             const FieldPtrs& out, hipStream_t stream);
hipError_t d3q19_init(const CaseDev& c, int storage, int parity, const double* phi0,
                      const double* u0, const double* p0, hipStream_t stream);

// Common kernels.
hipError_t stream_words(int lattice, const CaseDev& c, const uint32_t* in, uint32_t* out,
                        hipStream_t stream);
hipError_t encode16(int storage, const float* in, uint16_t* out, long long n,
                    hipStream_t stream);
hipError_t encode16_sr(int storage, const float* in, uint16_t* out, long long n, uint32_t t,
                       int dir, hipStream_t stream);
hipError_t copy_bw(const float* in, float* out, long long n, hipStream_t stream);
// F_a = -u [(rho^n - rho^(n-1)) + div(rho u)] from phi at n-1 and the dumped
// fields f (phi, u) at n; out: dim planes of c.n floats.
hipError_t fa_discrete(int lattice, const CaseDev& c, const float* phi_prev, const FieldPtrs& f,
                       float* out, hipStream_t stream);
// F_a = -u div[lambda (grad P - grad p)] (Lee and Lin's form) from the dumped
// fields f (phi, u, p); P = phi theta'(phi) - theta(phi) with theta =
// beta (phi - phi_g)^2 (phi - phi_l)^2, lambda = 3 mu_dyn(phi) / rho(phi).
struct WellArgs {
  float beta, phi_g, phi_l;
};
hipError_t fa_leelin(int lattice, const CaseDev& c, const WellArgs& wa, const FieldPtrs& f,
                     float* out, hipStream_t stream);
// Per row in x of a node field phi: half the distance between the outermost
// phi = level crossings, or -1 (out: c.ny * c.nz doubles).
hipError_t row_spread(const CaseDev& c, const float* phi, double level, double* out,
                      hipStream_t stream);
// One copy of the state (stride c.stride) moved src -> dst with the pull
// shifts of the step and no arithmetic (bandwidth calibration).
hipError_t pull_copy(int lattice, int storage, const CaseDev& c, const void* src, void* dst,
                     hipStream_t stream);

// FP64 diagnostics of node fields: kDiagSlots finished values per call
// (slot layout below, the same as LBM_DIAG_* of lbm.h), reduced in a fixed
// order by kReduceBlocks workgroups whose partial sums (kReduceBlocks *
// kDiagSlots doubles) go through `partials`.
constexpr int kDiagSlots = 16;
constexpr int kReduceBlocks = 512;
enum {
  DG_MASS = 0, DG_MOM = 1,   /* 1..3 */
  DG_WSUM = 4, DG_CEN = 5,   /* 5..7 */
  DG_CVEL = 8,               /* 8..10 */
  DG_M2 = 11,                /* 11..13 */
  DG_U2MAX = 14,             /* |u| max once finished */
  DG_BAD = 15
};
struct DiagArgs {
  int dim, nx, ny, nz, n;
  double rho0, drho;  // rho = rho0 + drho phi
  double wa, wb;      // centroid weight clamp(wa phi + wb, 0, 1)
  const float* phi;
  const float* u[3];
};
hipError_t field_diag(const DiagArgs& a, double* partials, double* out, hipStream_t stream);

}  // namespace lbm
