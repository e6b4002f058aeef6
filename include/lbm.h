/*
 * lbm.h -- C ABI of the MI355X (gfx950) phase-field lattice Boltzmann library.
 *
 * The library advances the incompressible two-distribution phase-field LB
 * model analysed by Li, Luo & Gao, "Additional interfacial force in lattice
 * Boltzmann models for incompressible multiphase flows" (arXiv:1110.5004):
 *   - order parameter phi with bulk free energy beta phi^2 (phi-1)^2 (Eq. 1a)
 *     or beta (phi^2 - phi*^2)^2 (Eq. 1b) and gradient coefficient kappa,
 *     chemical potential mu = theta'(phi) - kappa lap phi, convective
 *     Cahn-Hilliard transport with mobility theta_M (Eq. 2) solved by a BGK
 *     order-parameter distribution f;
 *   - density linear in phi (Eq. 4a, or Eq. 4b with the symmetric well);
 *   - pressure distribution g with the forcing K of Eq. 8, surface force
 *     F_s = mu grad phi and body force G = -(rho - rho_ref) g e_vertical;
 *   - a switch that keeps the additional force F_a = -u [d_t rho + div(rho u)]
 *     of Eq. 12 (original model) or cancels it by adding -F_a to the forcing
 *     (corrected model, paragraph after Eq. 12), with d_t rho + div(rho u)
 *     evaluated through Eq. 5 or taken from the data;
 *   - isotropic central stencils for grad and lap (splash-test paragraph);
 *   - diagnostics: FP64 reductions, the spread radius of the paper's Fig. 5,
 *     F_a from discrete data and in Lee and Lin's form (Eq. 11).
 * D2Q9 follows the paper; D3Q19 is the same model on 19 velocities.
 *
 * Conventions for every function:
 *   - The return value is an lbm_status; no C++ exception crosses the ABI.
 *     On a non-OK status lbm_last_error() gives a thread-local message.
 *   - Host pointers are plain CPU memory owned by the caller.  Device
 *     pointers are HIP device memory on the current device.
 *   - Node index of a case: x + nx * (y + ny * z); vector fields are SoA
 *     (all x components, then y, then z), each of length N = nx ny nz.
 *   - Work is enqueued on the HIP stream given to lbm_init (NULL = the null
 *     stream); functions that return host data synchronise that stream.
 *   - A handle is not thread safe; different handles are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,       /* invalid argument; nothing was allocated or enqueued */
  LBM_ERR_HIP = -2,       /* a HIP runtime call failed; message names it */
  LBM_ERR_NONFINITE = -3, /* a periodic check found NaN/Inf in phi or u */
  LBM_ERR_STATE = -4,     /* call not valid for this handle (e.g. wrong size) */
  LBM_ERR_OOM = -5        /* device arena too small or allocation failed */
} lbm_status;

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
enum { LBM_PERIODIC = 0, LBM_WALL = 1 };
/* Population storage.  LBM_FP32 stores every population as float.
 * LBM_FP16 / LBM_BF16 store f_0 as float and the other populations as 16-bit
 * deviations from the rest state:
 *   f_i (i > 0):  half(f_i * scale_f)              (rest value of f_i is 0)
 *   g_i:          half((g_i - w_i p0) * scale_g)   (rest value w_i p0)
 * f_0 is then rebuilt as phi - sum_{i>0} f_i from the stored values, so the
 * 16-bit rounding moves phi only between neighbours and sum phi is kept.
 * The f_i round to nearest even.  The g_i of a time step round
 * stochastically (lbm_encode16_stochastic): to the upper of the two format
 * values around them with probability equal to the fractional distance from
 * the lower one, with random bits from a counter-based generator: the
 * 32-bit "lowbias32" hash of C. Wellons, h(x) = x ^= x >> 16, x *= 0x7feb352d,
 * x ^= x >> 15, x *= 0x846ca68b, x ^= x >> 16; step key h(t * 0x9e3779b9 +
 * 0x6a09e667) for the time level t the step reads; node key h(k ^ step key)
 * for node index k = x + nx (y + ny z); bits r = node key + i * 0x9e3779b9
 * (mod 2^32) for direction i; FP16 adds r >> 19, BF16 r >> 16, to the float
 * bits and cuts the bits the format drops.  Rounding to nearest returns the
 * same error for the same value at every step, which the slowly varying g of
 * a quiet flow turns into a steady spurious force; the stochastic errors have
 * mean zero.  The initial populations (lbm_init) round to nearest. */
enum { LBM_FP32 = 0, LBM_FP16 = 1, LBM_BF16 = 2 };
/* Double well of the free energy.  LBM_WELL_ASYMMETRIC (Eq. 1a):
 * theta = beta phi^2 (phi - 1)^2, gas phi = 0, liquid phi = 1, density Eq. 4a.
 * LBM_WELL_SYMMETRIC (Eq. 1b): theta = beta (phi^2 - phi*^2)^2, gas -phi*,
 * liquid phi*, density Eq. 4b.  In both, rho and the dynamic viscosity are
 * linear in phi between their gas and liquid values. */
enum { LBM_WELL_ASYMMETRIC = 0, LBM_WELL_SYMMETRIC = 1 };

/* Parameters of one case, in lattice units (dx = dt = 1). */
typedef struct {
  int32_t lattice;           /* LBM_D2Q9 or LBM_D3Q19 (same for all cases of a handle) */
  int32_t nx, ny, nz;        /* each >= 4; nz = 1 for D2Q9 */
  int32_t bc[3];             /* per axis LBM_PERIODIC or LBM_WALL (halfway bounce-back,
                                mirror ghosts for the stencils: neutral wetting) */
  double beta, kappa;        /* beta of the double well (Eq. 1a or 1b, see well) and
                                kappa; lbm_beta_kappa() / lbm_beta_kappa_sym()
                                convert sigma, W */
  double theta_m;            /* mobility theta_M of Eq. 2 (> = 0) */
  double tau_f;              /* relaxation time of f (> 1/2); Gamma = theta_M/(tau_f-1/2) */
  double tau_g;              /* relaxation time of g in the liquid (> 1/2);
                                nu_L = (tau_g - 1/2)/3 */
  double rho_l, rho_g;       /* densities of Eq. 4a (> 0) */
  double mu_ratio;           /* mu_L / mu_G (> 0); = rho_l/rho_g gives constant nu */
  double gravity, rho_ref;   /* G = -(rho - rho_ref) gravity along -y (2-D) / -z (3-D) */
  int32_t remove_fa;         /* 0: original model (F_a kept);
                                1: corrected, -F_a = u drho theta_M lap mu added
                                   (F_a evaluated through Eq. 5);
                                2: corrected with the rate of Eq. 12 taken from
                                   the data, -F_a = u [(rho^n - rho^(n-1)) +
                                   div(rho u_o)], u_o the velocity the original
                                   model recovers at the same step (so the
                                   recovery stays closed-form), the time
                                   difference over one step (zero at the first).
                                   Every case of the handle must use it; each
                                   state copy then carries one more float plane
                                   (phi of the step that wrote it). */
  int32_t storage;           /* LBM_FP32 / LBM_FP16 / LBM_BF16 (same for all cases) */
  double p0;                 /* rest pressure of the 16-bit g deviations */
  double scale_f, scale_g;   /* powers of two for 16-bit storage; 0 = automatic */
  int32_t well;              /* LBM_WELL_ASYMMETRIC (0, the zero-initialised default)
                                or LBM_WELL_SYMMETRIC */
  double phi_star;           /* phi* of the symmetric well (> 0); ignored otherwise */
} lbm_case_params;

/* FP64 diagnostics of one case at the current time level. */
typedef struct {
  int64_t step;              /* time level n */
  double mass;               /* sum phi (total order parameter, conserved) */
  double mass0;              /* sum phi at lbm_init */
  double mass_drift_rel;     /* |mass - mass0| / |mass0| */
  double momentum[3];        /* sum rho u */
  double wsum;               /* sum w, w = clamp(2 s - 1/2, 0, 1) with s = (phi - phi_G) /
                                (phi_L - phi_G) the fraction of the way from the
                                gas to the liquid value of phi */
  double centroid[3];        /* sum w x / sum w (node coordinates) */
  double centroid_vel[3];    /* sum w u / sum w */
  double second_moment[3];   /* sum w (x - X)^2 / sum w per axis */
  double umax;               /* max |u| */
  int64_t nonfinite;         /* nodes with a non-finite phi or u component */
} lbm_diag;

typedef struct lbm_handle lbm_handle;

/* sigma, W -> beta = 12 sigma / W, kappa = 3 sigma W / 2: the pair for which
 * the flat interface 1/2 + 1/2 tanh(2 z / W) solves kappa phi'' = theta'(phi)
 * with tension sigma (the paper states that beta and kappa set sigma and W,
 * without the formula). */
int lbm_beta_kappa(double sigma, double width, double* beta, double* kappa);

/* sigma, W, phi* -> beta = 3 sigma / (4 W phi*^4), kappa = 3 sigma W / (8 phi*^2):
 * the pair for which phi* tanh(2 z / W) solves kappa phi'' = theta'(phi) for
 * the symmetric well of Eq. 1b with tension sigma.  LBM_ERR_ARG for sigma < 0,
 * W <= 0, phi* <= 0 or a NULL output. */
int lbm_beta_kappa_sym(double sigma, double width, double phi_star, double* beta,
                       double* kappa);

/* Device bytes lbm_init needs for these cases (state ping-pong, field
 * scratch, reduction partials, tables).  Validates the parameters. */
int lbm_required_bytes(const lbm_case_params* cases, int32_t ncases, size_t* bytes);

/* Create a handle for ncases cases advancing together (one launch per time
 * step covers all of them).  phi0[k], u0[k] (dim*N_k, SoA) and p0[k] are host
 * FP64 initial fields of case k; they are copied.  The initial populations are
 * the equilibria of (phi0, mu(phi0), u0, p0).
 * dev_arena: device memory of arena_bytes >= lbm_required_bytes, owned by the
 * caller and outliving the handle; NULL makes the library allocate its own.
 * hip_stream: hipStream_t for all work (NULL = null stream).
 * check_every > 0: lbm_step checks for non-finite values every that many
 * steps (synchronising) and returns LBM_ERR_NONFINITE when it finds one. */
int lbm_init(const lbm_case_params* cases, int32_t ncases, const double* const* phi0,
             const double* const* u0, const double* const* p0, void* dev_arena,
             size_t arena_bytes, void* hip_stream, int32_t check_every,
             lbm_handle** out);

/* Advance every case by nsteps time steps (fields, collision and streaming in
 * one fused kernel per step, or for D3Q19 in the three-kernel form when the
 * launch variant selects it; repeated steps replay a captured HIP graph).
 * Asynchronous unless check_every triggers a check. */
int lbm_step(lbm_handle* h, int64_t nsteps);

/* Capture and instantiate the HIP graph of graph_steps time steps for the
 * current launch shape (lbm_set_launch) without advancing the state, so that
 * a later lbm_step that replays it pays no capture cost.  Nothing is enqueued
 * on the handle's stream.  No effect with graph_steps = 0.  LBM_ERR_HIP when
 * the capture or the instantiation fails. */
int lbm_prepare(lbm_handle* h);

/* Macroscopic fields of case icase at the current time level, written to
 * caller-allocated host float arrays: phi[N], u[dim*N], p[N] (hydrodynamic
 * pressure), mu[N] (chemical potential), fa[dim*N] (the additional force
 * F_a = -u (d rho / d phi) theta_M lap mu of the current state, whichever
 * model runs).  Any output may be NULL.  Synchronises the stream. */
int lbm_moments(lbm_handle* h, int32_t icase, float* phi, float* u, float* p, float* mu,
                float* fa);

/* Same fields written to device float arrays of the same sizes (no copy to
 * the host, no synchronisation). */
int lbm_moments_device(lbm_handle* h, int32_t icase, float* phi, float* u, float* p,
                       float* mu, float* fa);

/* FP64 diagnostics of case icase, reduced on the GPU in a fixed order (bit
 * reproducible from run to run).  Synchronises the stream. */
int lbm_diagnostics(lbm_handle* h, int32_t icase, lbm_diag* out);

/* Slots of the device output of lbm_field_diagnostics (doubles). */
enum {
  LBM_DIAG_MASS = 0,           /* sum phi */
  LBM_DIAG_MOMENTUM = 1,       /* 1..3: sum rho u per axis */
  LBM_DIAG_WSUM = 4,           /* sum w (w as in lbm_diag) */
  LBM_DIAG_CENTROID = 5,       /* 5..7: sum w x / sum w */
  LBM_DIAG_CENTROID_VEL = 8,   /* 8..10: sum w u / sum w */
  LBM_DIAG_SECOND_MOMENT = 11, /* 11..13: sum w (x - X)^2 / sum w, X the centroid */
  LBM_DIAG_UMAX = 14,          /* max |u| */
  LBM_DIAG_NONFINITE = 15,     /* nodes with a non-finite phi or u component */
  LBM_DIAG_SLOTS = 16
};
/* Partial sums of lbm_field_diagnostics: 512 workgroups x 16 doubles. */
#define LBM_DIAG_WORKSPACE_BYTES 65536

/* The diagnostics of lbm_diagnostics computed from node fields in device
 * memory (those lbm_moments_device writes, say): phi[N] and u[dim*N] (SoA,
 * component a at offset a*N) of an nx x ny x nz grid (nz = 1 for dim = 2),
 * N = nx ny nz, node index x + nx (y + ny z).  The density is linear in phi
 * between (phi_g, rho_g) and (phi_l, rho_l) (Eq. 4a / 4b); the centroid
 * weight is w = clamp(2 s - 1/2, 0, 1), s = (phi - phi_g) / (phi_l - phi_g).
 * Moments with no weight (sum w = 0) are 0.
 * out: device double[LBM_DIAG_SLOTS] in the slot layout above (components
 * beyond dim are 0).  workspace: device memory of at least
 * LBM_DIAG_WORKSPACE_BYTES, 8-byte aligned, for the partial sums; overwritten.
 * Both caller-owned.  Four kernels are enqueued on hip_stream (no
 * synchronisation); the reduction order is fixed, so results are
 * bit-reproducible.  LBM_ERR_ARG for dim not 2 or 3, a grid with a side
 * below 1 or N >= 2^31, phi_l == phi_g, non-finite parameters, null
 * pointers, or a short or misaligned workspace; nothing is enqueued then. */
int lbm_field_diagnostics(int32_t dim, int32_t nx, int32_t ny, int32_t nz, const float* phi,
                          const float* u, double phi_g, double phi_l, double rho_g,
                          double rho_l, double* out, void* workspace, size_t workspace_bytes,
                          void* hip_stream);

/* lbm_field_diagnostics without the workspace argument and with no device
 * allocation at all, for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc).  The partial sums
 * go to a 64 KiB array in device memory that the library holds per GPU for
 * the life of the process; any grid size up to the limit of
 * lbm_field_diagnostics (N < 2^31 nodes) fits it.  Every call on a GPU uses
 * that GPU's one array: calls that overlap in time on the same GPU (two
 * streams, two threads) race and give wrong results; calls on different GPUs
 * do not.  Each call overwrites every partial it reads, so no clearing is
 * needed between calls.  hip_stream must belong to the current device (NULL:
 * its null stream).  Same arguments, results, bit reproducibility and
 * LBM_ERR_ARG cases as lbm_field_diagnostics (the workspace ones aside), plus
 * LBM_ERR_ARG for a stream of another device; LBM_ERR_HIP if the array's
 * address cannot be obtained on the current device. */
int lbm_field_diagnostics_noalloc(int32_t dim, int32_t nx, int32_t ny, int32_t nz,
                                  const float* phi, const float* u, double phi_g,
                                  double phi_l, double rho_g, double rho_l, double* out,
                                  void* hip_stream);

/* Spread radius of case icase at the current time level: the largest half
 * distance between the outermost crossings of phi = level along a grid row in
 * x (every y, z), crossings located by linear interpolation between nodes x
 * and x + 1 (x = 0 .. nx-2).  This is the droplet half-width that the paper
 * compares between the original and the corrected model in its falling-drop
 * test (Fig. 5).  *radius = 0 when no row crosses the level twice.
 * Synchronizes the stream. */
int lbm_spread_radius(lbm_handle* h, int32_t icase, double level, double* radius);

/* The additional interfacial force F_a of Eq. 12 estimated from discrete
 * data rather than through Eq. 5:
 *   F_a = -u^n [ (rho^n - rho^(n-1)) + div(rho u)^n ],
 * rho linear in phi (Eq. 4a or 4b, by the case's well), the time derivative a backward
 * difference over one step, the divergence by the isotropic central scheme
 * with the step's periodic / mirror-ghost neighbours.  It tests the paper's
 * statement that d_t rho + div(rho u) is approximately Eq. 5.  phi_prev: device
 * float[N], phi of case icase one step earlier (e.g. from
 * lbm_moments_device); fa: device float[dim*N] (SoA), written.  Both
 * caller-owned; enqueued on the handle's stream (no synchronization). */
int lbm_fa_discrete(lbm_handle* h, int32_t icase, const float* phi_prev, float* fa);

/* The additional force of Eq. 12 in the form it takes for Lee and Lin's
 * model, where d_t rho + div(rho u) is given by Eq. 11:
 *   F_a = -u div[ lambda (grad P - grad p) ]
 * evaluated on the current fields of case icase (whichever model runs):
 *   lambda = mu / (rho cs^2), mu the dynamic viscosity (linear in phi between
 *            mu_G and mu_L; the reading under which lambda is a time);
 *   P      = phi theta'(phi) - theta(phi), the equation of state of the
 *            free energy of Eq. 1 (the case's well);
 *   p      = the hydrodynamic pressure of the step;
 *   div[lambda grad q] = lambda lap q + grad lambda . grad q, each operator the
 *   isotropic central scheme with the step's periodic / mirror-ghost
 *   neighbours.
 * It is a diagnostic: it compares the Lee-Lin density source with the Eq. 5
 * one on the same flow.  fa: device float[dim*N] (SoA), caller-owned, written.
 * Enqueued on the handle's stream (no synchronization).  LBM_ERR_ARG for a
 * NULL handle or output or a bad case index. */
int lbm_fa_leelin(lbm_handle* h, int32_t icase, float* fa);

/* Number of cases, time level, and bytes of one case's raw state. */
int lbm_info(const lbm_handle* h, int32_t* ncases, int64_t* step, int32_t* storage);
int lbm_state_bytes(const lbm_handle* h, int32_t icase, size_t* bytes);

/* Raw stored populations of case icase (checkpoint / resume, bit exact).
 * The layout is private to the library version; only pass back what
 * lbm_get_state produced for the same parameters.  Synchronous. */
int lbm_get_state(lbm_handle* h, int32_t icase, void* host, size_t bytes);
int lbm_set_state(lbm_handle* h, int32_t icase, const void* host, size_t bytes);
/* Set the time level of all cases (after lbm_set_state). */
int lbm_set_step(lbm_handle* h, int64_t step);

/* Launch shape.  variant indexes the compiled tile shapes (lbm_variant_info);
 * grid_blocks = 0 launches one workgroup per tile, otherwise that many
 * workgroups loop over the tiles (D2Q9; the D3Q19 kernels always launch one
 * workgroup per tile and ignore it).  graph_steps = 0 disables graph capture,
 * otherwise lbm_step replays a graph of that many (even) steps. */
int lbm_set_launch(lbm_handle* h, int32_t variant, int32_t grid_blocks, int32_t graph_steps);
int lbm_get_launch(const lbm_handle* h, int32_t* variant, int32_t* grid_blocks,
                   int32_t* graph_steps);
/* Number of compiled tile variants for a lattice, and the tile (nodes per
 * axis) and workgroup size of one.  For D3Q19 the tile belongs to the step
 * form that lbm_variant_form reports.  Every variant of a lattice computes
 * the same bits, in every model and storage layout. */
int lbm_variant_count(int32_t lattice, int32_t* count);
int lbm_variant_info(int32_t lattice, int32_t variant, int32_t* tx, int32_t* ty, int32_t* tz,
                     int32_t* threads);
/* The D3Q19 step form of a variant (D2Q9: always 0):
 *   0  three kernels: pull, the fields on tx x ty x tz tiles, collision;
 *   1  fused: one kernel, a tx x ty tile of the x-y plane marching up a chunk
 *      of tz planes with the fields in LDS;
 *   2  two kernels (16-bit storage): the pull, then a tx x ty tile marching up
 *      a chunk of tz planes that forms the fields and collides.
 * Form 1 with 16-bit storage on a grid of odd width or with the correction
 * from data, and form 2 with FP32 storage, run the three-kernel step of
 * variant 1.  LBM_ERR_ARG for a NULL form, a bad lattice or a variant out of
 * range. */
int lbm_variant_form(int32_t lattice, int32_t variant, int32_t* form);

void lbm_free(lbm_handle* h);
const char* lbm_last_error(void);

/* ---- test and calibration entry points ------------------------------- */

/* One streaming pass over raw 32-bit words on the device, exactly as the
 * step kernel pulls populations: out_i(x) = in_i(x - e_i), or in_opp(i)(x)
 * when x - e_i lies beyond a wall.  in/out: device arrays of Q*N words,
 * plane i at offset i*N.  Enqueued on hip_stream. */
int lbm_stream_words(int32_t lattice, int32_t nx, int32_t ny, int32_t nz,
                     const int32_t* bc, const uint32_t* in, uint32_t* out, void* hip_stream);

/* Round float values to the 16-bit storage format (LBM_FP16 or LBM_BF16),
 * round to nearest even, on the device: out[k] = bits of format(in[k]).
 * in: device float[n]; out: device uint16[n]. */
int lbm_encode16(int32_t storage, const float* in, uint16_t* out, int64_t n,
                 void* hip_stream);

/* The stochastic rounding of the 16-bit g stores of a time step, on the
 * device: out[k] = bits of the FP16 / BF16 value that the step with counter
 * `step` (the time level it reads) stores for the value in[k] of direction
 * `direction` (0..18) of node k.  The result is one of the two format values
 * around in[k], the upper one with probability equal to the fractional
 * distance from the lower one (exact values stay; FP16 below its normal range
 * rounds to nearest on the remaining bits), so the rounding error has mean
 * zero.  The random bits come from the counter-based generator keyed by step,
 * node and direction that the storage formats above define.
 * in: device float[n]; out: device uint16[n]; n <= 2^32. */
int lbm_encode16_stochastic(int32_t storage, const float* in, uint16_t* out, int64_t n,
                            uint32_t step, int32_t direction, void* hip_stream);

/* Device copy out[k] = in[k] of n floats with the library's streaming access
 * pattern (achievable-bandwidth calibration). */
int lbm_copy_bw(const float* in, float* out, int64_t n, void* hip_stream);

/* Pull-copy calibration: the memory traffic of one step of an nx x ny x nz
 * grid without its arithmetic.  src and dst each hold one copy of the stored
 * populations in the step's plane layout with a plane stride of nx*ny*nz
 * elements (storage LBM_FP32: 2q float planes then one BF16 plane,
 * (8q + 2) bytes per node; LBM_FP16/LBM_BF16: one float plane then 2q - 1
 * 16-bit planes, (4q + 2) bytes per node).  Every word of node x is read from
 * x - e_i (from x itself where that leaves the grid) and written to x.  The
 * output has no meaning beyond the timing.  Device pointers, caller-owned;
 * enqueued on hip_stream.  LBM_ERR_ARG on bad sizes or null buffers. */
int lbm_pull_copy_bw(int32_t lattice, int32_t storage, int32_t nx, int32_t ny, int32_t nz,
                     const void* src, void* dst, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
