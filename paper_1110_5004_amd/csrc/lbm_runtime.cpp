// lbm_runtime.cpp -- host runtime behind the C ABI of include/lbm.h:
// parameter validation and derivation, device arena layout, tile lists,
// launch selection, HIP graph capture of repeated steps, field dumps and
// FP64 diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_kernels.h"

using lbm::CaseDev;
static_assert(lbm::kDiagSlots == LBM_DIAG_SLOTS && lbm::DG_MOM == LBM_DIAG_MOMENTUM &&
                  lbm::DG_WSUM == LBM_DIAG_WSUM && lbm::DG_CEN == LBM_DIAG_CENTROID &&
                  lbm::DG_CVEL == LBM_DIAG_CENTROID_VEL && lbm::DG_M2 == LBM_DIAG_SECOND_MOMENT &&
                  lbm::DG_U2MAX == LBM_DIAG_UMAX && lbm::DG_BAD == LBM_DIAG_NONFINITE,
              "diagnostics slot layout");
static_assert(sizeof(double) * lbm::kReduceBlocks * lbm::kDiagSlots == LBM_DIAG_WORKSPACE_BYTES,
              "diagnostics workspace");
using lbm::TileDev;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(LBM_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

int dim_of(int lattice) { return lattice == LBM_D3Q19 ? 3 : 2; }
int q_of(int lattice) { return lattice == LBM_D3Q19 ? 19 : 9; }

long long nodes_of(const lbm_case_params& c) { return (long long)c.nx * c.ny * c.nz; }
long long stride_of(const lbm_case_params& c) {
  return (long long)align_up((size_t)nodes_of(c), 64);
}

bool is_pow2(double s) {
  if (!(s > 0.0) || !std::isfinite(s)) return false;
  int e;
  return std::frexp(s, &e) == 0.5;
}

int validate(const lbm_case_params* cs, int32_t n) {
  if (!cs || n <= 0) return fail(LBM_ERR_ARG, "need at least one case");
  for (int k = 0; k < n; ++k) {
    const lbm_case_params& c = cs[k];
    if (c.lattice != LBM_D2Q9 && c.lattice != LBM_D3Q19)
      return fail(LBM_ERR_ARG, "case %d: unknown lattice %d", k, c.lattice);
    if (c.lattice != cs[0].lattice)
      return fail(LBM_ERR_ARG, "case %d: all cases of a handle must share the lattice", k);
    if ((c.remove_fa == 2) != (cs[0].remove_fa == 2))
      return fail(LBM_ERR_ARG,
                  "case %d: remove_fa = 2 cannot be mixed with 0 / 1 in one handle", k);
    if (c.storage != cs[0].storage)
      return fail(LBM_ERR_ARG, "case %d: all cases of a handle must share the storage", k);
    if (c.storage < LBM_FP32 || c.storage > LBM_BF16)
      return fail(LBM_ERR_ARG, "case %d: unknown storage %d", k, c.storage);
    if (c.nx < 4 || c.ny < 4) return fail(LBM_ERR_ARG, "case %d: nx, ny must be >= 4", k);
    // node indices are formed with 24-bit multiplies
    if (c.nx >= (1 << 24) || c.ny >= (1 << 24) || c.nz >= (1 << 24))
      return fail(LBM_ERR_ARG, "case %d: every side must be < 2^24", k);
    if (c.lattice == LBM_D2Q9 && c.nz != 1)
      return fail(LBM_ERR_ARG, "case %d: nz must be 1 for D2Q9", k);
    if (c.lattice == LBM_D3Q19 && c.nz < 4)
      return fail(LBM_ERR_ARG, "case %d: nz must be >= 4 for D3Q19", k);
    if (nodes_of(c) > (1LL << 30)) return fail(LBM_ERR_ARG, "case %d: too many nodes", k);
    // kernels address one copy of the populations with 32-bit byte offsets
    if (lbm::copy_bytes(c.storage, q_of(c.lattice), stride_of(c), c.remove_fa == 2) >=
        (1ULL << 32))
      return fail(LBM_ERR_ARG, "case %d: one copy of the populations exceeds 4 GiB", k);
    for (int a = 0; a < 3; ++a)
      if (c.bc[a] != LBM_PERIODIC && c.bc[a] != LBM_WALL)
        return fail(LBM_ERR_ARG, "case %d: bc[%d] must be periodic or wall", k, a);
    const double vals[] = {c.beta, c.kappa, c.theta_m, c.tau_f, c.tau_g, c.rho_l, c.rho_g,
                           c.mu_ratio, c.gravity, c.rho_ref, c.p0};
    for (double v : vals)
      if (!std::isfinite(v)) return fail(LBM_ERR_ARG, "case %d: non-finite parameter", k);
    if (!(c.tau_f > 0.5) || !(c.tau_g > 0.5))
      return fail(LBM_ERR_ARG, "case %d: tau_f and tau_g must exceed 1/2", k);
    if (!(c.rho_l > 0.0) || !(c.rho_g > 0.0) || !(c.mu_ratio > 0.0))
      return fail(LBM_ERR_ARG, "case %d: densities and viscosity ratio must be > 0", k);
    if (c.theta_m < 0.0 || c.beta < 0.0 || c.kappa < 0.0)
      return fail(LBM_ERR_ARG, "case %d: theta_m, beta, kappa must be >= 0", k);
    if (c.remove_fa < 0 || c.remove_fa > 2)
      return fail(LBM_ERR_ARG, "case %d: remove_fa must be 0, 1 or 2", k);
    if (c.well != LBM_WELL_ASYMMETRIC && c.well != LBM_WELL_SYMMETRIC)
      return fail(LBM_ERR_ARG, "case %d: well must be LBM_WELL_ASYMMETRIC or LBM_WELL_SYMMETRIC", k);
    if (c.well == LBM_WELL_SYMMETRIC && !(c.phi_star > 0.0 && std::isfinite(c.phi_star)))
      return fail(LBM_ERR_ARG, "case %d: phi_star must be finite and > 0", k);
    if ((c.scale_f != 0.0 && !is_pow2(c.scale_f)) || (c.scale_g != 0.0 && !is_pow2(c.scale_g)))
      return fail(LBM_ERR_ARG, "case %d: 16-bit scales must be powers of two (or 0)", k);
  }
  return LBM_OK;
}

const lbm::TileShape* tiles_for(int lattice, int* count) {
  if (lattice == LBM_D3Q19) {
    *count = lbm::kD3Q19TileCount;
    return lbm::kD3Q19Tiles;
  }
  *count = lbm::kD2Q9TileCount;
  return lbm::kD2Q9Tiles;
}

long long count_tiles(const lbm_case_params& c, const lbm::TileShape& t) {
  const long long tz = c.lattice == LBM_D3Q19 ? (c.nz + t.tz - 1) / t.tz : 1;
  return (long long)((c.nx + t.tx - 1) / t.tx) * ((c.ny + t.ty - 1) / t.ty) * tz;
}

// Tile list, case after case.  Within a case the tiles run in vertical strips
// about kStripNodes (or the shape's own strip) wide (tile rows inside a strip, strips left to right), so
// that consecutive tiles -- which the kernel hands to the same XCD -- share
// their halos.
constexpr int kStripNodes = 512;

std::vector<TileDev> build_tiles(const lbm_case_params* cs, int n, const lbm::TileShape& t,
                                 std::vector<int>* off, std::vector<int>* cnt) {
  std::vector<TileDev> v;
  if (off) off->assign(n, 0);
  if (cnt) cnt->assign(n, 0);
  const int strip = t.strip > 0 ? t.strip : kStripNodes;
  const int sw = std::max(1, strip / t.tx) * t.tx;  // strip width in nodes
  for (int k = 0; k < n; ++k) {
    const lbm_case_params& c = cs[k];
    const int nzt = c.lattice == LBM_D3Q19 ? (c.nz + t.tz - 1) / t.tz : 1;
    if (off) (*off)[k] = (int)v.size();
    for (int xs = 0; xs < c.nx; xs += sw)
      for (int z = 0; z < nzt; ++z)
        for (int y = 0; y < c.ny; y += t.ty)
          for (int x = xs; x < std::min(c.nx, xs + sw); x += t.tx)
            v.push_back(TileDev{k, x, y, z * t.tz});
    if (cnt) (*cnt)[k] = (int)v.size() - (off ? (*off)[k] : 0);
  }
  return v;
}

// Field-dump tile shape: variant 0 of each lattice.
const lbm::TileShape& field_shape(int lattice) {
  int n;
  return lattice == LBM_D2Q9 ? lbm::kD2Q9FieldShape : tiles_for(lattice, &n)[0];
}

struct Layout {
  size_t cases_off, tiles_off, ftiles_off, fld_off, part_off, dout_off, clock_off, total;
  std::vector<size_t> state_off;  // two copies per case, contiguous
  size_t max_tiles, n_ftiles, fld_plane;
};

Layout plan(const lbm_case_params* cs, int n) {
  Layout L{};
  size_t at = 0;
  L.cases_off = at;
  at = align_up(at + sizeof(CaseDev) * n);
  int nv;
  const lbm::TileShape* shapes = tiles_for(cs[0].lattice, &nv);
  size_t mt = 0;
  for (int v = 0; v < nv; ++v) {
    size_t t = 0;
    for (int k = 0; k < n; ++k) t += count_tiles(cs[k], shapes[v]);
    mt = std::max(mt, t);
  }
  L.max_tiles = mt;
  L.tiles_off = at;
  at = align_up(at + sizeof(TileDev) * mt);
  size_t ft = 0;
  for (int k = 0; k < n; ++k) ft += count_tiles(cs[k], field_shape(cs[0].lattice));
  L.n_ftiles = ft;
  L.ftiles_off = at;
  at = align_up(at + sizeof(TileDev) * ft);
  const int q = q_of(cs[0].lattice), dim = dim_of(cs[0].lattice);
  L.state_off.resize(2 * n);
  long long nmax = 0;
  for (int k = 0; k < n; ++k) {
    const size_t cb =
        align_up(lbm::copy_bytes(cs[k].storage, q, stride_of(cs[k]), cs[k].remove_fa == 2));
    L.state_off[2 * k] = at;
    at += cb;
    L.state_off[2 * k + 1] = at;
    at += cb;
    nmax = std::max(nmax, stride_of(cs[k]));
  }
  // field scratch: phi, u (dim), p, mu, fa (dim) floats; also the staging of
  // the FP64 initial fields (2 + dim doubles per node).  D3Q19 steps also pass
  // kField3Planes planes between their kernels, placed after the dump planes.
  L.fld_plane = (size_t)nmax;
  size_t fplanes = std::max<size_t>(3 + 2 * dim, 2 * (2 + dim));
  if (cs[0].lattice == LBM_D3Q19) fplanes = 3 + 2 * dim + lbm::kField3Planes;
  L.fld_off = at;
  at = align_up(at + fplanes * L.fld_plane * sizeof(float));
  L.part_off = at;
  at = align_up(at + sizeof(double) * lbm::kReduceBlocks * lbm::kDiagSlots);
  L.dout_off = at;
  at = align_up(at + sizeof(double) * lbm::kDiagSlots);
  L.clock_off = at;  // the step counter of the stochastic rounding, one per copy
  at = align_up(at + 2 * sizeof(unsigned));
  L.total = at;
  return L;
}

int round8(long long x) { return (int)((std::max(x, 1LL) + 7) / 8 * 8); }

}  // namespace

struct lbm_handle {
  int ncases = 0, lattice = 0, storage = 0, dim = 2, q = 9, rf = 0;
  std::vector<lbm_case_params> prm;
  std::vector<CaseDev> cd;
  Layout L;
  char* arena = nullptr;
  bool own_arena = false;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int check_every = 0;
  int64_t step = 0;
  int parity = 0;
  int64_t since_check = 0;
  int variant = 0, grid_blocks = 0, graph_steps = 16;
  int ntiles = 0;
  std::vector<int> ftile_off, ftile_cnt;
  std::vector<double> mass0;
  hipGraphExec_t gexec = nullptr;
  int g_variant = -1, g_grid = -1, g_steps = 0;

  CaseDev* d_cases() { return reinterpret_cast<CaseDev*>(arena + L.cases_off); }
  TileDev* d_tiles() { return reinterpret_cast<TileDev*>(arena + L.tiles_off); }
  TileDev* d_ftiles() { return reinterpret_cast<TileDev*>(arena + L.ftiles_off); }
  float* fld(int plane) {
    return reinterpret_cast<float*>(arena + L.fld_off) + (size_t)plane * L.fld_plane;
  }
  double* partials() { return reinterpret_cast<double*>(arena + L.part_off); }
  double* dout() { return reinterpret_cast<double*>(arena + L.dout_off); }
  unsigned* clock() { return reinterpret_cast<unsigned*>(arena + L.clock_off); }
};

namespace {

CaseDev derive(const lbm_case_params& p, char* s0, char* s1) {
  CaseDev c{};
  c.nx = p.nx;
  c.ny = p.ny;
  c.nz = p.nz;
  c.wall_x = p.bc[0] == LBM_WALL;
  c.wall_y = p.bc[1] == LBM_WALL;
  c.wall_z = p.lattice == LBM_D3Q19 && p.bc[2] == LBM_WALL;
  c.n = (int)nodes_of(p);
  c.stride = (unsigned)stride_of(p);
  c.state[0] = s0;
  c.state[1] = s1;
  // bulk values of phi: 0 and 1 for the asymmetric well, -phi* and phi* for
  // the symmetric one; rho and the dynamic viscosity are linear in phi
  // between the gas and the liquid value (Eq. 4a / 4b)
  const bool sym = p.well == LBM_WELL_SYMMETRIC;
  const double phi_g = sym ? -p.phi_star : 0.0;
  const double phi_l = sym ? p.phi_star : 1.0;
  const double drho = (p.rho_l - p.rho_g) / (phi_l - phi_g);  // d rho / d phi
  const double gamma = p.theta_m / (p.tau_f - 0.5);  // theta_M = Gamma (tau_f - 1/2)
  const double mu_l = p.rho_l * (p.tau_g - 0.5) / 3.0;  // nu_L = cs^2 (tau_g - 1/2)
  const double mu_g = mu_l / p.mu_ratio;
  const double dmu = (mu_l - mu_g) / (phi_l - phi_g);
  c.th_k = (float)(4.0 * p.beta);
  c.th_r1 = (float)phi_l;
  c.th_r2 = (float)(sym ? phi_g : 0.5);
  c.kappa = (float)p.kappa;
  c.gamma3 = (float)(3.0 * gamma);
  c.omega_f = (float)(1.0 / p.tau_f);
  c.rho0 = (float)(p.rho_g - phi_g * drho);
  c.drho = (float)drho;
  c.mu0 = (float)(mu_g - phi_g * dmu);
  c.dmu = (float)dmu;
  c.wa = (float)(2.0 / (phi_l - phi_g));
  c.wb = (float)(-2.0 * phi_g / (phi_l - phi_g) - 0.5);
  c.gravity = (float)p.gravity;
  c.rho_ref = (float)p.rho_ref;
  c.corr = (float)(p.remove_fa == 1 ? drho * p.theta_m : 0.0);
  c.phiv = p.remove_fa == 2
               ? (unsigned)lbm::copy_bytes(p.storage, q_of(p.lattice), stride_of(p), false)
               : 0u;
  c.fa_coef = (float)(drho * p.theta_m);
  c.p0 = (float)p.p0;
  // 16-bit scales: FP16 keeps deviations down to ~1e-8 normal with 2^13;
  // BF16 has the float exponent range and needs none.
  double sf = p.scale_f, sg = p.scale_g;
  if (sf == 0.0) sf = p.storage == LBM_FP16 ? 8192.0 : 1.0;
  if (sg == 0.0) sg = p.storage == LBM_FP16 ? 8192.0 : 1.0;
  c.scale_f = (float)sf;
  c.inv_scale_f = (float)(1.0 / sf);
  c.scale_g = (float)sg;
  c.inv_scale_g = (float)(1.0 / sg);
  return c;
}

lbm::LaunchArgs step_args(lbm_handle* h, int parity, hipStream_t s) {
  lbm::LaunchArgs a{};
  a.cases = h->d_cases();
  a.tiles = h->d_tiles();
  a.ntiles = h->ntiles;
  a.grid = h->grid_blocks > 0 ? round8(h->grid_blocks) : round8(h->ntiles);
  a.parity = parity;
  a.storage = h->storage;
  a.rf = h->rf;
  a.stream = s;
  return a;
}

lbm::Field3Ptrs step_fields3(lbm_handle* h) {
  lbm::Field3Ptrs f{};
  for (int k = 0; k < lbm::kField3Planes; ++k) f.plane[k] = h->fld(3 + 2 * h->dim + k);
  return f;
}

hipError_t launch_step(lbm_handle* h, int parity, hipStream_t s) {
  if (h->lattice == LBM_D3Q19) {
    const lbm::Field3Ptrs f = step_fields3(h);
    for (int k = 0; k < h->ncases; ++k) {
      hipError_t e = lbm::d3q19_step_case(h->variant, h->cd[k], h->storage, parity, f, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  lbm::LaunchArgs a = step_args(h, parity, s);
  return lbm::d2q9_step(h->variant, a);
}

int upload_tiles(lbm_handle* h) {
  int nv;
  const lbm::TileShape* shapes = tiles_for(h->lattice, &nv);
  std::vector<TileDev> t = build_tiles(h->prm.data(), h->ncases, shapes[h->variant], nullptr,
                                       nullptr);
  h->ntiles = (int)t.size();
  HIPCHK(hipMemcpyAsync(h->d_tiles(), t.data(), t.size() * sizeof(TileDev),
                        hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

void drop_graph(lbm_handle* h) {
  if (h->gexec) hipGraphExecDestroy(h->gexec);
  h->gexec = nullptr;
  h->g_variant = h->g_grid = -1;
  h->g_steps = 0;
}

int ensure_graph(lbm_handle* h) {
  if (h->gexec && h->g_variant == h->variant && h->g_grid == h->grid_blocks &&
      h->g_steps == h->graph_steps)
    return LBM_OK;
  drop_graph(h);
  if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < h->graph_steps && e == hipSuccess; ++k) e = launch_step(h, k & 1, h->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
  if (e != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return fail(LBM_ERR_HIP, "step launch during capture: %s", hipGetErrorString(e));
  }
  if (e2 != hipSuccess) return fail(LBM_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
  e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->gexec = nullptr;
    return fail(LBM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  h->g_variant = h->variant;
  h->g_grid = h->grid_blocks;
  h->g_steps = h->graph_steps;
  return LBM_OK;
}

int dump_fields(lbm_handle* h, int icase, const lbm::FieldPtrs& f) {
  if (h->lattice == LBM_D3Q19) {
    HIPCHK(lbm::d3q19_fields_case(h->cd[icase], h->storage, h->parity, step_fields3(h), f,
                                  h->stream));
    return LBM_OK;
  }
  lbm::LaunchArgs a{};
  a.cases = h->d_cases();
  a.tiles = h->d_ftiles() + h->ftile_off[icase];
  a.ntiles = h->ftile_cnt[icase];
  a.grid = round8(a.ntiles);
  a.parity = h->parity;
  a.storage = h->storage;
  a.rf = h->rf == 2 ? 2 : 1;
  a.stream = h->stream;
  HIPCHK(lbm::d2q9_fields(a, f));
  return LBM_OK;
}

lbm::FieldPtrs scratch_fields(lbm_handle* h) {
  lbm::FieldPtrs f{};
  int k = 0;
  f.phi = h->fld(k++);
  for (int a = 0; a < h->dim; ++a) f.u[a] = h->fld(k++);
  f.p = h->fld(k++);
  f.mu = h->fld(k++);
  for (int a = 0; a < h->dim; ++a) f.fa[a] = h->fld(k++);
  return f;
}

// Centroid weight and density of the diagnostics from the bulk values of phi
// and rho (rho linear in phi between them, Eq. 4a / 4b).
lbm::DiagArgs diag_args(int dim, int nx, int ny, int nz, double phi_g, double phi_l,
                        double rho_g, double rho_l) {
  lbm::DiagArgs a{};
  a.dim = dim;
  a.nx = nx;
  a.ny = ny;
  a.nz = dim == 3 ? nz : 1;
  a.n = a.nx * a.ny * a.nz;
  a.drho = (rho_l - rho_g) / (phi_l - phi_g);
  a.rho0 = rho_g - phi_g * a.drho;
  a.wa = 2.0 / (phi_l - phi_g);
  a.wb = -2.0 * phi_g / (phi_l - phi_g) - 0.5;
  return a;
}

// The finished diagnostics (lbm::DG_* slots) of case icase, on the host.
int diag_sums(lbm_handle* h, int icase, double* s) {
  lbm::FieldPtrs f = scratch_fields(h);
  int rc = dump_fields(h, icase, f);
  if (rc) return rc;
  const lbm_case_params& p = h->prm[icase];
  const bool sym = p.well == LBM_WELL_SYMMETRIC;
  lbm::DiagArgs a = diag_args(h->dim, p.nx, p.ny, p.nz, sym ? -p.phi_star : 0.0,
                              sym ? p.phi_star : 1.0, p.rho_g, p.rho_l);
  a.phi = f.phi;
  for (int d = 0; d < 3; ++d) a.u[d] = d < h->dim ? f.u[d] : f.u[0];
  HIPCHK(lbm::field_diag(a, h->partials(), h->dout(), h->stream));
  HIPCHK(hipMemcpyAsync(s, h->dout(), sizeof(double) * lbm::kDiagSlots, hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

// Arguments of lbm_field_diagnostics (and of its variant without workspace).
int check_field_diag(int32_t dim, int32_t nx, int32_t ny, int32_t nz, const float* phi,
                     const float* u, double phi_g, double phi_l, double rho_g, double rho_l,
                     const double* out) {
  if (dim != 2 && dim != 3) return fail(LBM_ERR_ARG, "dim must be 2 or 3");
  if (dim == 2) nz = 1;
  if (nx < 1 || ny < 1 || nz < 1) return fail(LBM_ERR_ARG, "bad grid %d x %d x %d", nx, ny, nz);
  if ((double)nx * ny * nz >= 2147483648.0) return fail(LBM_ERR_ARG, "grid of 2^31 nodes or more");
  if (!std::isfinite(phi_g) || !std::isfinite(phi_l) || !std::isfinite(rho_g) ||
      !std::isfinite(rho_l) || phi_l == phi_g)
    return fail(LBM_ERR_ARG, "need finite phi_g != phi_l and finite rho_g, rho_l");
  if (!phi || !u || !out) return fail(LBM_ERR_ARG, "NULL field or output");
  return LBM_OK;
}

int check_finite(lbm_handle* h) {
  for (int k = 0; k < h->ncases; ++k) {
    double s[lbm::kDiagSlots];
    int rc = diag_sums(h, k, s);
    if (rc) return rc;
    if (s[lbm::DG_BAD] > 0.0)
      return fail(LBM_ERR_NONFINITE, "case %d: %.0f nodes with non-finite phi or u at step %lld",
                  k, s[lbm::DG_BAD], (long long)h->step);
  }
  return LBM_OK;
}

}  // namespace

// ---- partial sums of lbm_field_diagnostics_noalloc
// A file-scope device array: every GPU the library runs on holds its own copy
// (64 KiB) until the process ends.  Host code never uses its name as an
// address; it takes each device's address from hipGetSymbolAddress, once per
// device with that device current, and keeps it.  Every workgroup of the
// first and third diagnostics kernels writes its whole slot before the
// second and fourth read it, so nothing needs clearing between calls.
static __device__ __align__(256) double scratch[lbm::kReduceBlocks * lbm::kDiagSlots];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices];  // per device; nullptr until its first call

int scratch_of_current_device(double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(LBM_ERR_ARG, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LBM_ERR_HIP, "hipGetSymbolAddress gave a null address");
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return LBM_OK;
}
}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

int lbm_beta_kappa(double sigma, double width, double* beta, double* kappa) {
  if (!beta || !kappa || !(width > 0.0) || !(sigma >= 0.0))
    return fail(LBM_ERR_ARG, "need sigma >= 0, W > 0 and output pointers");
  *beta = 12.0 * sigma / width;
  *kappa = 1.5 * sigma * width;
  return LBM_OK;
}

int lbm_beta_kappa_sym(double sigma, double width, double phi_star, double* beta,
                       double* kappa) {
  if (!beta || !kappa || !(width > 0.0) || !(sigma >= 0.0) || !(phi_star > 0.0))
    return fail(LBM_ERR_ARG, "need sigma >= 0, W > 0, phi_star > 0 and output pointers");
  const double p2 = phi_star * phi_star;
  *beta = 3.0 * sigma / (4.0 * width * p2 * p2);
  *kappa = 3.0 * sigma * width / (8.0 * p2);
  return LBM_OK;
}

int lbm_required_bytes(const lbm_case_params* cases, int32_t ncases, size_t* bytes) {
  int rc = validate(cases, ncases);
  if (rc) return rc;
  if (!bytes) return fail(LBM_ERR_ARG, "bytes is NULL");
  *bytes = plan(cases, ncases).total;
  return LBM_OK;
}

int lbm_init(const lbm_case_params* cases, int32_t ncases, const double* const* phi0,
             const double* const* u0, const double* const* p0, void* dev_arena,
             size_t arena_bytes, void* hip_stream, int32_t check_every, lbm_handle** out) {
  if (!out) return fail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate(cases, ncases);
  if (rc) return rc;
  if (!phi0 || !u0 || !p0) return fail(LBM_ERR_ARG, "initial field arrays are NULL");
  for (int k = 0; k < ncases; ++k)
    if (!phi0[k] || !u0[k] || !p0[k]) return fail(LBM_ERR_ARG, "case %d: NULL initial field", k);
  if (check_every < 0) return fail(LBM_ERR_ARG, "check_every must be >= 0");
  Layout L = plan(cases, ncases);
  if (dev_arena && arena_bytes < L.total)
    return fail(LBM_ERR_OOM, "arena of %zu bytes, need %zu", arena_bytes, L.total);
  if (dev_arena && (reinterpret_cast<uintptr_t>(dev_arena) % kAlign))
    return fail(LBM_ERR_ARG, "arena must be 256-byte aligned");

  lbm_handle* h = new lbm_handle();
  h->ncases = ncases;
  h->lattice = cases[0].lattice;
  h->storage = cases[0].storage;
  h->dim = dim_of(h->lattice);
  h->q = q_of(h->lattice);
  h->prm.assign(cases, cases + ncases);
  h->L = L;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->check_every = check_every;
  // kernel form: 2 (correction from data, every case), 1 (lap mu formed;
  // a case with remove_fa = 0 has corr = 0), or 0
  for (int k = 0; k < ncases; ++k) h->rf = std::max(h->rf, (int)cases[k].remove_fa);
  if (dev_arena) {
    h->arena = reinterpret_cast<char*>(dev_arena);
  } else {
    hipError_t e = hipMalloc(&h->arena, L.total);
    if (e != hipSuccess) {
      delete h;
      return fail(LBM_ERR_OOM, "hipMalloc(%zu): %s", L.total, hipGetErrorString(e));
    }
    h->own_arena = true;
  }
  auto bail = [&](int code) {
    lbm_free(h);
    return code;
  };
  // zero everything once: plane padding and unused tails then read back as
  // zeros, so raw states of equal runs compare equal byte for byte
  {
    hipError_t e = hipMemsetAsync(h->arena, 0, L.total, h->stream);
    if (e != hipSuccess) return bail(fail(LBM_ERR_HIP, "arena clear: %s", hipGetErrorString(e)));
  }
  for (int k = 0; k < ncases; ++k) {
    h->cd.push_back(derive(cases[k], h->arena + L.state_off[2 * k], h->arena + L.state_off[2 * k + 1]));
    h->cd.back().clock = h->clock();  // zero from the clear above: step 0
  }
  {
    hipError_t e = hipMemcpyAsync(h->d_cases(), h->cd.data(), sizeof(CaseDev) * ncases,
                                  hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return bail(fail(LBM_ERR_HIP, "case table upload: %s", hipGetErrorString(e)));
  }
  std::vector<TileDev> ft = build_tiles(cases, ncases, field_shape(h->lattice), &h->ftile_off,
                                        &h->ftile_cnt);
  {
    hipError_t e = hipMemcpyAsync(h->d_ftiles(), ft.data(), ft.size() * sizeof(TileDev),
                                  hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return bail(fail(LBM_ERR_HIP, "tile upload: %s", hipGetErrorString(e)));
  }
  if ((rc = upload_tiles(h))) return bail(rc);

  // initial populations, one case at a time through the FP64 staging area
  for (int k = 0; k < ncases; ++k) {
    const size_t n = (size_t)nodes_of(cases[k]);
    double* st = reinterpret_cast<double*>(h->fld(0));
    double* d_phi = st;
    double* d_u = st + n;
    double* d_p = st + (1 + h->dim) * n;
    hipError_t e = hipMemcpyAsync(d_phi, phi0[k], n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_u, u0[k], h->dim * n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_p, p0[k], n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = h->lattice == LBM_D3Q19
              ? lbm::d3q19_init(h->cd[k], h->storage, 0, d_phi, d_u, d_p, h->stream)
              : lbm::d2q9_init(h->cd[k], h->storage, 0, d_phi, d_u, d_p, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bail(fail(LBM_ERR_HIP, "case %d init: %s", k, hipGetErrorString(e)));
  }
  h->mass0.resize(ncases);
  for (int k = 0; k < ncases; ++k) {
    double s[lbm::kDiagSlots];
    if ((rc = diag_sums(h, k, s))) return bail(rc);
    h->mass0[k] = s[lbm::DG_MASS];
  }
  *out = h;
  return LBM_OK;
}

int lbm_step(lbm_handle* h, int64_t nsteps) {
  if (!h) return fail(LBM_ERR_ARG, "NULL handle");
  if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps must be >= 0");
  while (nsteps > 0) {
    int64_t left_before_check =
        h->check_every > 0 ? h->check_every - h->since_check : nsteps;
    int64_t chunk = std::min<int64_t>(nsteps, left_before_check);
    while (chunk > 0) {
      if (h->graph_steps >= 2 && h->parity == 0 && chunk >= h->graph_steps) {
        int rc = ensure_graph(h);
        if (rc) return rc;
        HIPCHK(hipGraphLaunch(h->gexec, h->stream));
        chunk -= h->graph_steps;
        nsteps -= h->graph_steps;
        h->step += h->graph_steps;
        h->since_check += h->graph_steps;
      } else {
        HIPCHK(launch_step(h, h->parity, h->stream));
        h->parity ^= 1;
        chunk -= 1;
        nsteps -= 1;
        h->step += 1;
        h->since_check += 1;
      }
    }
    if (h->check_every > 0 && h->since_check >= h->check_every) {
      h->since_check = 0;
      int rc = check_finite(h);
      if (rc) return rc;
    }
  }
  return LBM_OK;
}

int lbm_prepare(lbm_handle* h) {
  if (!h) return fail(LBM_ERR_ARG, "NULL handle");
  if (h->graph_steps < 2) return LBM_OK;
  return ensure_graph(h);
}

int lbm_moments_device(lbm_handle* h, int32_t icase, float* phi, float* u, float* p, float* mu,
                       float* fa) {
  if (!h || icase < 0 || icase >= h->ncases) return fail(LBM_ERR_ARG, "bad handle or case");
  lbm::FieldPtrs f = scratch_fields(h);
  const size_t n = (size_t)h->cd[icase].n;
  if (phi) f.phi = phi;
  if (u)
    for (int a = 0; a < h->dim; ++a) f.u[a] = u + a * n;
  if (p) f.p = p;
  if (mu) f.mu = mu;
  if (fa)
    for (int a = 0; a < h->dim; ++a) f.fa[a] = fa + a * n;
  return dump_fields(h, icase, f);
}

int lbm_moments(lbm_handle* h, int32_t icase, float* phi, float* u, float* p, float* mu,
                float* fa) {
  if (!h || icase < 0 || icase >= h->ncases) return fail(LBM_ERR_ARG, "bad handle or case");
  lbm::FieldPtrs f = scratch_fields(h);
  int rc = dump_fields(h, icase, f);
  if (rc) return rc;
  const size_t n = (size_t)h->cd[icase].n, b = n * sizeof(float);
  if (phi) HIPCHK(hipMemcpyAsync(phi, f.phi, b, hipMemcpyDeviceToHost, h->stream));
  for (int a = 0; a < h->dim; ++a) {
    if (u) HIPCHK(hipMemcpyAsync(u + a * n, f.u[a], b, hipMemcpyDeviceToHost, h->stream));
    if (fa) HIPCHK(hipMemcpyAsync(fa + a * n, f.fa[a], b, hipMemcpyDeviceToHost, h->stream));
  }
  if (p) HIPCHK(hipMemcpyAsync(p, f.p, b, hipMemcpyDeviceToHost, h->stream));
  if (mu) HIPCHK(hipMemcpyAsync(mu, f.mu, b, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_diagnostics(lbm_handle* h, int32_t icase, lbm_diag* out) {
  if (!h || !out || icase < 0 || icase >= h->ncases) return fail(LBM_ERR_ARG, "bad arguments");
  double s[lbm::kDiagSlots];
  int rc = diag_sums(h, icase, s);
  if (rc) return rc;
  std::memset(out, 0, sizeof *out);
  out->step = h->step;
  out->mass = s[lbm::DG_MASS];
  out->mass0 = h->mass0[icase];
  out->mass_drift_rel = out->mass0 != 0.0 ? std::fabs(out->mass - out->mass0) / std::fabs(out->mass0)
                                          : std::fabs(out->mass);
  out->wsum = s[lbm::DG_WSUM];
  for (int a = 0; a < h->dim; ++a) {
    out->momentum[a] = s[lbm::DG_MOM + a];
    out->centroid[a] = s[lbm::DG_CEN + a];
    out->centroid_vel[a] = s[lbm::DG_CVEL + a];
    out->second_moment[a] = s[lbm::DG_M2 + a];
  }
  out->umax = s[lbm::DG_U2MAX];
  out->nonfinite = (int64_t)s[lbm::DG_BAD];
  return LBM_OK;
}

int lbm_field_diagnostics(int32_t dim, int32_t nx, int32_t ny, int32_t nz, const float* phi,
                          const float* u, double phi_g, double phi_l, double rho_g,
                          double rho_l, double* out, void* workspace, size_t workspace_bytes,
                          void* hip_stream) {
  int rc = check_field_diag(dim, nx, ny, nz, phi, u, phi_g, phi_l, rho_g, rho_l, out);
  if (rc) return rc;
  if (!workspace || workspace_bytes < LBM_DIAG_WORKSPACE_BYTES ||
      reinterpret_cast<uintptr_t>(workspace) % alignof(double) != 0)
    return fail(LBM_ERR_ARG, "workspace: need %d bytes, 8-byte aligned",
                LBM_DIAG_WORKSPACE_BYTES);
  lbm::DiagArgs a = diag_args(dim, nx, ny, nz, phi_g, phi_l, rho_g, rho_l);
  a.phi = phi;
  for (int d = 0; d < 3; ++d) a.u[d] = u + (size_t)(d < dim ? d : 0) * a.n;
  HIPCHK(lbm::field_diag(a, static_cast<double*>(workspace), out,
                         reinterpret_cast<hipStream_t>(hip_stream)));
  return LBM_OK;
}

int lbm_fa_discrete(lbm_handle* h, int32_t icase, const float* phi_prev, float* fa) {
  if (!h || !phi_prev || !fa || icase < 0 || icase >= h->ncases)
    return fail(LBM_ERR_ARG, "bad arguments");
  lbm::FieldPtrs f = scratch_fields(h);
  int rc = dump_fields(h, icase, f);
  if (rc) return rc;
  HIPCHK(lbm::fa_discrete(h->lattice == LBM_D2Q9 ? 0 : 1, h->cd[icase], phi_prev, f, fa,
                          h->stream));
  return LBM_OK;
}

int lbm_fa_leelin(lbm_handle* h, int32_t icase, float* fa) {
  if (!h || !fa || icase < 0 || icase >= h->ncases) return fail(LBM_ERR_ARG, "bad arguments");
  lbm::FieldPtrs f = scratch_fields(h);
  int rc = dump_fields(h, icase, f);
  if (rc) return rc;
  const lbm_case_params& p = h->prm[icase];
  const bool sym = p.well == LBM_WELL_SYMMETRIC;
  const lbm::WellArgs wa{(float)p.beta, (float)(sym ? -p.phi_star : 0.0),
                         (float)(sym ? p.phi_star : 1.0)};
  HIPCHK(lbm::fa_leelin(h->lattice == LBM_D2Q9 ? 0 : 1, h->cd[icase], wa, f, fa, h->stream));
  return LBM_OK;
}

int lbm_spread_radius(lbm_handle* h, int32_t icase, double level, double* radius) {
  if (!h || !radius || icase < 0 || icase >= h->ncases) return fail(LBM_ERR_ARG, "bad arguments");
  if (!std::isfinite(level)) return fail(LBM_ERR_ARG, "level must be finite");
  lbm::FieldPtrs f = scratch_fields(h);
  int rc = dump_fields(h, icase, f);
  if (rc) return rc;
  const CaseDev& c = h->cd[icase];
  const size_t rows = (size_t)c.ny * c.nz;
  // per-row results (doubles) in the first F_a plane, which the dump just
  // wrote and nothing here reads: one float plane holds nx * rows >= 2 rows
  // floats
  if (2 * rows > (size_t)c.stride) return fail(LBM_ERR_ARG, "grid too narrow in x");
  double* rowbuf = reinterpret_cast<double*>(f.fa[0]);
  HIPCHK(lbm::row_spread(c, f.phi, level, rowbuf, h->stream));
  std::vector<double> host(rows);
  HIPCHK(hipMemcpyAsync(host.data(), rowbuf, rows * sizeof(double), hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  double best = 0.0;
  for (double v : host) best = std::max(best, v);
  *radius = best;
  return LBM_OK;
}

int lbm_info(const lbm_handle* h, int32_t* ncases, int64_t* step, int32_t* storage) {
  if (!h) return fail(LBM_ERR_ARG, "NULL handle");
  if (ncases) *ncases = h->ncases;
  if (step) *step = h->step;
  if (storage) *storage = h->storage;
  return LBM_OK;
}

int lbm_state_bytes(const lbm_handle* h, int32_t icase, size_t* bytes) {
  if (!h || !bytes || icase < 0 || icase >= h->ncases) return fail(LBM_ERR_ARG, "bad arguments");
  *bytes = lbm::copy_bytes(h->storage, h->q, h->cd[icase].stride, h->rf == 2);
  return LBM_OK;
}

int lbm_get_state(lbm_handle* h, int32_t icase, void* host, size_t bytes) {
  size_t need;
  int rc = lbm_state_bytes(h, icase, &need);
  if (rc) return rc;
  if (!host || bytes != need) return fail(LBM_ERR_STATE, "state needs exactly %zu bytes", need);
  HIPCHK(hipMemcpyAsync(host, h->cd[icase].state[h->parity], need, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_set_state(lbm_handle* h, int32_t icase, const void* host, size_t bytes) {
  size_t need;
  int rc = lbm_state_bytes(h, icase, &need);
  if (rc) return rc;
  if (!host || bytes != need) return fail(LBM_ERR_STATE, "state needs exactly %zu bytes", need);
  HIPCHK(hipMemcpyAsync(h->cd[icase].state[h->parity], host, need, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_set_step(lbm_handle* h, int64_t step) {
  if (!h || step < 0) return fail(LBM_ERR_ARG, "bad arguments");
  // the next step reads the counter of the current copy (modulo 2^32)
  const unsigned t = (unsigned)(uint64_t)step;
  HIPCHK(hipMemcpyAsync(h->clock() + h->parity, &t, sizeof t, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->step = step;
  return LBM_OK;
}

int lbm_variant_count(int32_t lattice, int32_t* count) {
  if (!count || (lattice != LBM_D2Q9 && lattice != LBM_D3Q19)) return fail(LBM_ERR_ARG, "bad lattice");
  int n;
  tiles_for(lattice, &n);
  *count = n;
  return LBM_OK;
}

int lbm_variant_info(int32_t lattice, int32_t variant, int32_t* tx, int32_t* ty, int32_t* tz,
                     int32_t* threads) {
  int n;
  if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return fail(LBM_ERR_ARG, "bad lattice");
  const lbm::TileShape* t = tiles_for(lattice, &n);
  if (variant < 0 || variant >= n) return fail(LBM_ERR_ARG, "variant out of range");
  if (tx) *tx = t[variant].tx;
  if (ty) *ty = t[variant].ty;
  if (tz) *tz = t[variant].tz;
  if (threads) *threads = t[variant].nt;
  return LBM_OK;
}

int lbm_variant_form(int32_t lattice, int32_t variant, int32_t* form) {
  int n;
  if (!form) return fail(LBM_ERR_ARG, "NULL form");
  if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return fail(LBM_ERR_ARG, "bad lattice");
  const lbm::TileShape* t = tiles_for(lattice, &n);
  if (variant < 0 || variant >= n) return fail(LBM_ERR_ARG, "variant out of range");
  *form = t[variant].form;
  return LBM_OK;
}

int lbm_set_launch(lbm_handle* h, int32_t variant, int32_t grid_blocks, int32_t graph_steps) {
  if (!h) return fail(LBM_ERR_ARG, "NULL handle");
  int n;
  tiles_for(h->lattice, &n);
  if (variant < 0 || variant >= n) return fail(LBM_ERR_ARG, "variant out of range");
  if (grid_blocks < 0) return fail(LBM_ERR_ARG, "grid_blocks must be >= 0");
  if (graph_steps < 0 || (graph_steps & 1) || graph_steps > 4096)
    return fail(LBM_ERR_ARG, "graph_steps must be 0 or an even number <= 4096");
  const bool retile = variant != h->variant;
  h->variant = variant;
  h->grid_blocks = grid_blocks;
  h->graph_steps = graph_steps;
  if (retile) {
    HIPCHK(hipStreamSynchronize(h->stream));
    int rc = upload_tiles(h);
    if (rc) return rc;
  }
  return LBM_OK;
}

int lbm_get_launch(const lbm_handle* h, int32_t* variant, int32_t* grid_blocks,
                   int32_t* graph_steps) {
  if (!h) return fail(LBM_ERR_ARG, "NULL handle");
  if (variant) *variant = h->variant;
  if (grid_blocks) *grid_blocks = h->grid_blocks;
  if (graph_steps) *graph_steps = h->graph_steps;
  return LBM_OK;
}

void lbm_free(lbm_handle* h) {
  if (!h) return;
  if (h->stream || h->arena) hipStreamSynchronize(h->stream);
  drop_graph(h);
  if (h->cap_stream) hipStreamDestroy(h->cap_stream);
  if (h->own_arena && h->arena) hipFree(h->arena);
  delete h;
}

int lbm_stream_words(int32_t lattice, int32_t nx, int32_t ny, int32_t nz, const int32_t* bc,
                     const uint32_t* in, uint32_t* out, void* hip_stream) {
  if (!bc || !in || !out) return fail(LBM_ERR_ARG, "NULL argument");
  lbm_case_params p{};
  p.lattice = lattice;
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  for (int a = 0; a < 3; ++a) p.bc[a] = bc[a];
  p.tau_f = p.tau_g = 1.0;
  p.rho_l = p.rho_g = p.mu_ratio = 1.0;
  int rc = validate(&p, 1);
  if (rc) return rc;
  CaseDev c = derive(p, nullptr, nullptr);
  HIPCHK(lbm::stream_words(lattice, c, in, out, reinterpret_cast<hipStream_t>(hip_stream)));
  return LBM_OK;
}

int lbm_encode16(int32_t storage, const float* in, uint16_t* out, int64_t n, void* hip_stream) {
  if (storage != LBM_FP16 && storage != LBM_BF16) return fail(LBM_ERR_ARG, "storage must be FP16 or BF16");
  if (n < 0 || (n > 0 && (!in || !out))) return fail(LBM_ERR_ARG, "bad buffers");
  HIPCHK(lbm::encode16(storage, in, out, n, reinterpret_cast<hipStream_t>(hip_stream)));
  return LBM_OK;
}

int lbm_encode16_stochastic(int32_t storage, const float* in, uint16_t* out, int64_t n,
                            uint32_t step, int32_t direction, void* hip_stream) {
  if (storage != LBM_FP16 && storage != LBM_BF16) return fail(LBM_ERR_ARG, "storage must be FP16 or BF16");
  if (n < 0 || n > 4294967296LL || (n > 0 && (!in || !out))) return fail(LBM_ERR_ARG, "bad buffers");
  if (direction < 0 || direction > 18) return fail(LBM_ERR_ARG, "direction must be 0..18");
  HIPCHK(lbm::encode16_sr(storage, in, out, n, step, direction,
                          reinterpret_cast<hipStream_t>(hip_stream)));
  return LBM_OK;
}

int lbm_copy_bw(const float* in, float* out, int64_t n, void* hip_stream) {
  if (n < 0 || (n > 0 && (!in || !out))) return fail(LBM_ERR_ARG, "bad buffers");
  HIPCHK(lbm::copy_bw(in, out, n, reinterpret_cast<hipStream_t>(hip_stream)));
  return LBM_OK;
}

int lbm_field_diagnostics_noalloc(int32_t dim, int32_t nx, int32_t ny, int32_t nz,
                                  const float* phi, const float* u, double phi_g,
                                  double phi_l, double rho_g, double rho_l, double* out,
                                  void* hip_stream) {
  int rc = check_field_diag(dim, nx, ny, nz, phi, u, phi_g, phi_l, rho_g, rho_l, out);
  if (rc) return rc;
  const hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (s) {  // the partial sums must be those of the device the stream runs on
    int dev = -1, sdev = -1;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipStreamGetDevice(s, &sdev));
    if (sdev != dev)
      return fail(LBM_ERR_ARG, "stream of device %d, current device %d", sdev, dev);
  }
  double* partials = nullptr;
  if ((rc = scratch_of_current_device(&partials))) return rc;
  lbm::DiagArgs a = diag_args(dim, nx, ny, nz, phi_g, phi_l, rho_g, rho_l);
  a.phi = phi;
  for (int d = 0; d < 3; ++d) a.u[d] = u + (size_t)(d < dim ? d : 0) * a.n;
  HIPCHK(lbm::field_diag(a, partials, out, s));
  return LBM_OK;
}

int lbm_pull_copy_bw(int32_t lattice, int32_t storage, int32_t nx, int32_t ny, int32_t nz,
                     const void* src, void* dst, void* hip_stream) {
  if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return fail(LBM_ERR_ARG, "bad lattice");
  if (storage != LBM_FP32 && storage != LBM_FP16 && storage != LBM_BF16)
    return fail(LBM_ERR_ARG, "bad storage");
  if (lattice == LBM_D2Q9) nz = 1;
  if (nx < 1 || ny < 1 || nz < 1) return fail(LBM_ERR_ARG, "bad grid");
  const long long n = (long long)nx * ny * nz;
  const int q = lattice == LBM_D2Q9 ? 9 : 19;
  if ((double)lbm::copy_bytes(storage, q, n) >= 4294967296.0)
    return fail(LBM_ERR_ARG, "one copy must stay below 4 GiB");
  if (!src || !dst) return fail(LBM_ERR_ARG, "bad buffers");
  CaseDev c{};
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.n = (int)n;
  c.stride = (unsigned)n;
  HIPCHK(lbm::pull_copy(lattice == LBM_D2Q9 ? 0 : 1, storage == LBM_FP32 ? lbm::ST_FP32 : lbm::ST_FP16,
                        c, src, dst, reinterpret_cast<hipStream_t>(hip_stream)));
  return LBM_OK;
}

}  // extern "C"
