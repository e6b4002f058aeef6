/*
 * lbm_oracle.h -- FP64 CPU oracle for the two-distribution phase-field
 * lattice Boltzmann model analysed by Li, Luo & Gao, "Additional interfacial
 * force in lattice Boltzmann models for incompressible multiphase flows"
 * (arXiv:1110.5004).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the HIP path is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product library never
 * links, includes or calls it, and it shares no code with the product.
 *
 * Everything is IEEE double precision, evaluated in the order the equations
 * are written, one full sweep over the lattice per sub-step:
 *   S1a  phi = sum_i f_i, rho(phi)                      (Eq. 4a)
 *   S1b  grad phi, lap phi, mu = theta'(phi) - kappa lap phi   (Eq. 1a, mu def.)
 *   S1c  lap mu                   (only needed by the corrected model, Eq. 5)
 *   S1d  F_s, G, u, F, p          (Eqs. 3, 5, 12 and the moment recovery)
 *   S1e  grad p -> grad psi, tau(x)
 *   S2   BGK collision of f (order parameter) and gbar (pressure, Eq. 8)
 *   S3   streaming with halfway bounce-back on wall axes
 *
 * Node index: x + nx*(y + ny*z).  Vector fields are stored SoA, component
 * after component, each of length N = nx*ny*nz.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1 };

/* Parameters of one simulation case, in lattice units (dx = dt = 1). */
typedef struct {
  int lattice;          /* ORC_D2Q9 or ORC_D3Q19 */
  int nx, ny, nz;       /* nz = 1 for D2Q9 */
  int wall[3];          /* per axis: 0 periodic, 1 halfway bounce-back walls */
  double beta, kappa;   /* bulk free energy beta*phi^2(phi-1)^2 and gradient coefficient */
  double theta_m;       /* mobility of the Cahn-Hilliard equation (Eq. 2) */
  double tau_f;         /* relaxation time of the order-parameter distribution */
  double tau_g;         /* relaxation time of the pressure distribution in the liquid */
  double rho_l, rho_g;  /* saturated liquid / gas densities (Eq. 4a) */
  double mu_ratio;      /* dynamic viscosity ratio mu_L / mu_G */
  double gravity;       /* magnitude g of the body force G = -(rho - rho_ref) g e_vert */
  double rho_ref;       /* reference density of the body force */
  int remove_fa;        /* 0: original model (F_a present), 1: corrected (adds -F_a,
                           F_a by Eq. 5), 2: corrected with F_a taken from the data,
                           -u [(rho^n - rho^(n-1)) + div(rho u_o)], u_o the velocity of
                           the uncorrected recovery at the same step */
  int well;             /* 0: theta = beta phi^2 (phi-1)^2, phi in [0, 1], rho by Eq. 4a;
                           1: symmetric theta = beta (phi^2 - phi*^2)^2 (Eq. 1b), phi in
                           [-phi*, phi*], rho by Eq. 4b */
  double phi_star;      /* phi* of the symmetric well (> 0; unused when well = 0) */
} orc_params;

typedef struct orc_sim orc_sim;

/* Lattice tables.  q receives Q; e receives Q*3 ints; w receives Q doubles;
 * opp receives Q ints.  Returns 0, or -1 for an unknown lattice. */
int orc_lattice(int lattice, int* q, int* e, double* w, int* opp);

/* sigma, W -> beta, kappa for the flat tanh interface of width W. */
void orc_beta_kappa(double sigma, double width, double* beta, double* kappa);
/* The same for the symmetric well of Eq. 1b with minima at +-phi_star. */
void orc_beta_kappa_sym(double sigma, double width, double phi_star, double* beta,
                        double* kappa);

/* Create a simulation from FP64 initial fields phi0[N], u0[dim*N], p0[N].
 * Returns NULL on invalid parameters. */
orc_sim* orc_create(const orc_params* prm, const double* phi0, const double* u0,
                    const double* p0);
void orc_destroy(orc_sim* s);

/* Advance nsteps full time steps (fields, collide, stream). */
void orc_step(orc_sim* s, long nsteps);
long orc_time(const orc_sim* s);

/* Macroscopic fields at the current time level: phi[N], u[dim*N], p[N],
 * mu[N], lapmu[N] (lap mu is always evaluated here), fa[dim*N] (the
 * additional force of Eq. 12 in the reading F_a = -u drho theta_M lap mu).
 * Any pointer may be NULL. */
void orc_fields(orc_sim* s, double* phi, double* u, double* p, double* mu,
                double* lapmu, double* fa);

/* Diagnostics, fixed summation order (node order).  out receives 20 doubles:
 *  [0] mass = sum phi       [1] mass at creation
 *  [2..4] momentum sum rho u
 *  [5] sum w, w = clamp(2 phi01 - 1/2, 0, 1), phi01 = (phi - phi_G) / (phi_L - phi_G)
 *  [6..8] centroid sum w x / sum w
 *  [9..11] centroid velocity sum w u / sum w
 *  [12..14] second moment sum w (x - X)^2 / sum w, per axis
 *  [15] max |u|   [16] number of non-finite phi or u values
 *  [17..19] reserved (0) */
void orc_diag(orc_sim* s, double* out);

/* Spread radius (diagnostic D6: the droplet half-width the paper compares
 * between the two models in its falling-droplet test, Fig. 5).  Along every
 * grid row in x (every y, z) the crossings of phi = level between nodes x and
 * x + 1 (x = 0 .. nx-2, a crossing where exactly one of the two is >= level)
 * are located by linear interpolation; the row's value is half the distance
 * between its outermost crossings; the result is the maximum over rows with
 * two or more crossings, 0 if there is none.  phi[nx*ny*nz], node order. */
/* Diagnostics of orc_diag from given node fields (phi, u), rho linear in phi
 * through (phi_g, rho_g), (phi_l, rho_l); out[16] (see lbm_oracle.c). */
void orc_field_diag(int dim, int nx, int ny, int nz, const double* phi, const double* u,
                    double phi_g, double phi_l, double rho_g, double rho_l, double* out);
double orc_spread_radius(int nx, int ny, int nz, const double* phi, double level);

/* The additional interfacial force of Eq. 12 estimated from discrete data
 * (instead of through Eq. 5):
 *   F_a = -u [ (rho^n - rho^(n-1)) + div(rho u)^n ],
 * the time derivative a backward difference over one step, the divergence by
 * the isotropic central scheme (sum over components of the gradient of the
 * component, with periodic wrap or mirror ghosts), rho linear in phi
 * (Eq. 4a or 4b).  phi_prev, phi: N values at n-1 and n; u: dim*N
 * (SoA) at n; out: dim*N (SoA). */
void orc_fa_discrete(const orc_params* prm, const double* phi_prev, const double* phi,
                     const double* u, double* out);

/* The additional force of Eq. 12 in the form it takes for Lee and Lin's model,
 * where d_t rho + div(rho u) is given by Eq. 11:
 *   F_a = -u div[ lambda (grad P - grad p) ],
 * lambda = mu / (rho cs^2) with mu the dynamic viscosity (the only reading
 * for which lambda has the dimension of a time: mu_L = rho_L cs^2 (tau_g -
 * 1/2), mu_G = mu_L / ratio, linear in phi between the bulk values), P the
 * thermodynamic pressure read as the equation of state of the free energy of
 * Eq. 1, P = phi theta'(phi) - theta(phi), and p the hydrodynamic pressure.
 * The divergence is expanded as lambda lap(P - p) + grad lambda . grad(P - p),
 * each operator the isotropic central scheme.  phi, p: N values; u: dim*N
 * (SoA); out: dim*N (SoA). */
void orc_fa_leelin(const orc_params* prm, const double* phi, const double* u,
                   const double* pr, double* out);

/* Raw pre-collision populations f[Q*N], g[Q*N] (plane i at offset i*N). */
void orc_get_state(const orc_sim* s, double* f, double* g);
void orc_set_state(orc_sim* s, const double* f, const double* g, long time);

/* ---- building blocks, exposed so that tests can pin them ---------------- */

/* Equilibrium of the order-parameter distribution (Q values). */
void orc_feq(int lattice, double phi, double mu, const double* u, double gamma,
             double* out);
/* Equilibrium of the pressure distribution (Q values). */
void orc_geq(int lattice, double p, double rho, const double* u, double* out);
/* Forcing term (e_i - u) . K_i of Eq. 8 (Q values). */
void orc_source(int lattice, const double* u, const double* force,
                const double* gradpsi, double* out);
/* Velocity and pressure recovered from gbar: inputs are the Q populations,
 * rho, Fs+G (dim), c = s*drho*theta_M*lap mu and grad rho (dim).
 * Outputs u (dim), F (dim), p. */
void orc_recover(int lattice, const double* gbar, double rho, const double* fsg,
                 double c, const double* gradrho, double* u, double* force,
                 double* p);
/* Isotropic gradient (dim*N, SoA) and Laplacian (N) of a scalar field on the
 * grid of prm, with periodic wrap or mirror ghosts on wall axes. */
void orc_grad_lap(const orc_params* prm, const double* field, double* grad,
                  double* lap);
/* One streaming pass applied to arbitrary words: out_i(x) = in_i(x - e_i),
 * or in_opp(i)(x) across a wall.  Words are 32-bit patterns so that tests can
 * check that streaming is an exact permutation. */
void orc_stream_words(const orc_params* prm, const unsigned* in, unsigned* out);

#ifdef __cplusplus
}
#endif
#endif
