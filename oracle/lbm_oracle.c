/*
 * lbm_oracle.c -- FP64 CPU oracle (test infrastructure only; see the header).
 *
 * Written from the paper (Li, Luo & Gao, arXiv:1110.5004) and the readings
 * listed with the design notes of this repository:
 *   free energy, double well and chemical potential ..... Eq. 1a and the
 *                                                          definition of mu
 *   density closure ...................................... Eq. 4a
 *   weights, omega(u), g = cs^2 f + psi omega(0) ........ paragraph with Eq. 6
 *   pressure-distribution evolution with forcing K ....... Eq. 8
 *   additional force F_a = -u [d_t rho + div(rho u)] .... Eq. 12, evaluated
 *                                 with Eq. 5 as -u (drho) theta_M lap mu
 *   corrected model: -F_a added to the forcing term ...... paragraph after Eq. 12
 *   symmetric well and its density law .................. Eq. 1b, Eq. 4b
 *   F_a from discrete data; F_a in Lee and Lin's form .... Eq. 12; Eq. 11
 *   isotropic central first derivatives and Laplacian .... splash-test paragraph
 * The order-parameter equation of the cited original model is not printed in
 * the paper; it is read as the plain BGK Cahn-Hilliard LBE whose equilibrium
 * has moments phi, phi u, Gamma mu I + phi u u (so theta_M = Gamma (tau_f - 1/2)).
 *
 * Plain loops, one sweep per sub-step, no blocking or fusion.  OpenMP only
 * splits the independent per-node loops; results do not depend on the number
 * of threads.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define QMAX 19

typedef struct {
  int q, dim;
  int e[QMAX][3];
  double w[QMAX];
  int opp[QMAX];
} lat_t;

/* D2Q9: rest, 4 axis links, 4 diagonals; weights 4/9, 1/9, 1/36 (paragraph
 * with Eq. 6).  D3Q19: rest, 6 axis links, 12 edge diagonals; weights 1/3,
 * 1/18, 1/36 (standard set; the paper works in 2-D only). */
static int lat_fill(int lattice, lat_t* L) {
  static const int e9[9][2] = {{0, 0}, {1, 0},  {0, 1},   {-1, 0}, {0, -1},
                               {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
  static const int e19[19][3] = {
      {0, 0, 0},  {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
      {0, 0, 1},  {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
      {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
      {0, 1, 1},  {0, -1, -1}, {0, 1, -1},  {0, -1, 1}};
  memset(L, 0, sizeof *L);
  if (lattice == ORC_D2Q9) {
    L->q = 9;
    L->dim = 2;
    for (int i = 0; i < 9; ++i) {
      L->e[i][0] = e9[i][0];
      L->e[i][1] = e9[i][1];
      L->e[i][2] = 0;
      L->w[i] = (i == 0) ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  } else if (lattice == ORC_D3Q19) {
    L->q = 19;
    L->dim = 3;
    for (int i = 0; i < 19; ++i) {
      for (int a = 0; a < 3; ++a) L->e[i][a] = e19[i][a];
      L->w[i] = (i == 0) ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
  } else {
    return -1;
  }
  for (int i = 0; i < L->q; ++i) {
    L->opp[i] = -1;
    for (int j = 0; j < L->q; ++j)
      if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] &&
          L->e[j][2] == -L->e[i][2])
        L->opp[i] = j;
  }
  return 0;
}

int orc_lattice(int lattice, int* q, int* e, double* w, int* opp) {
  lat_t L;
  if (lat_fill(lattice, &L)) return -1;
  if (q) *q = L.q;
  for (int i = 0; i < L.q; ++i) {
    if (e)
      for (int a = 0; a < 3; ++a) e[3 * i + a] = L.e[i][a];
    if (w) w[i] = L.w[i];
    if (opp) opp[i] = L.opp[i];
  }
  return 0;
}

/* A flat interface solves kappa phi'' = theta'(phi).  With theta = beta
 * phi^2 (phi-1)^2 the solution is 1/2 + 1/2 tanh(2 z / W) with W^2 = 8 kappa /
 * beta, and its tension sigma = int kappa phi'^2 dz = sqrt(2 kappa beta) / 6.
 * Inverting both gives beta = 12 sigma / W and kappa = 3 sigma W / 2. */
void orc_beta_kappa(double sigma, double width, double* beta, double* kappa) {
  *beta = 12.0 * sigma / width;
  *kappa = 1.5 * sigma * width;
}

/* With theta = beta (phi^2 - phi*^2)^2 (Eq. 1b) the flat interface is
 * phi* tanh(2 z / W) with W^2 = 2 kappa / (beta phi*^2), and its tension
 * sigma = int kappa phi'^2 dz = (4/3) sqrt(2 kappa beta) phi*^3.  Inverting:
 * beta = 3 sigma / (4 W phi*^4), kappa = 3 sigma W / (8 phi*^2) (for
 * phi* = 1/2 these are the values of the asymmetric well). */
void orc_beta_kappa_sym(double sigma, double width, double phi_star, double* beta,
                        double* kappa) {
  const double p2 = phi_star * phi_star;
  *beta = 3.0 * sigma / (4.0 * width * p2 * p2);
  *kappa = 3.0 * sigma * width / (8.0 * p2);
}

/* ------------------------------------------------------------------------ */

struct orc_sim {
  orc_params prm;
  lat_t L;
  long n;
  long time;
  double *f, *g, *fn, *gn;        /* Q*N populations (current / scratch) */
  double *phi, *rho, *gphi, *lphi; /* N, N, dim*N, N */
  double *mu, *lmu, *u, *force, *pr, *gpsi, *tau;
  /* remove_fa = 2: phi of the previous step (phi0 before the first), the
   * velocity of the uncorrected recovery times rho, and the rate D */
  double *phi_prev, *rhou, *grad, *dmass;
  double mass0;
  double gamma, drho, mu_l, mu_g;
  /* phi of the pure gas and liquid (0, 1 or -phi*, phi*) and the slope of
   * the density law, d rho / d phi (Eq. 4a or 4b) */
  double phi_g, phi_l, drho_dphi;
};

static const double CS2 = 1.0 / 3.0;

/* Coordinate on one axis of a stencil neighbour: periodic wrap, or the mirror
 * ghost of a wall half a cell beyond the last node (ghost -k <-> node k-1). */
static int map_axis(int c, int n, int wall) {
  if (wall) {
    if (c < 0) return -c - 1;
    if (c >= n) return 2 * n - 1 - c;
    return c;
  }
  c %= n;
  if (c < 0) c += n;
  return c;
}

static void coords(const orc_params* p, long idx, int* c) {
  c[0] = (int)(idx % p->nx);
  c[1] = (int)((idx / p->nx) % p->ny);
  c[2] = (int)(idx / ((long)p->nx * p->ny));
}

static long nb_stencil(const orc_params* p, const int* c, const int* d) {
  int m0 = map_axis(c[0] + d[0], p->nx, p->wall[0]);
  int m1 = map_axis(c[1] + d[1], p->ny, p->wall[1]);
  int m2 = map_axis(c[2] + d[2], p->nz, p->wall[2]);
  return m0 + (long)p->nx * (m1 + (long)p->ny * m2);
}

static long count_nodes(const orc_params* p) {
  return (long)p->nx * p->ny * p->nz;
}

/* Isotropic central schemes on the lattice stencil:
 *   d_a phi = (1/cs^2) sum_i w_i e_ia phi(x + e_i)
 *   lap phi = (2/cs^2) sum_{i>0} w_i [phi(x + e_i) - phi(x)]            */
static void grad_lap_lat(const orc_params* p, const lat_t* L, const double* fld,
                         double* grad, double* lap) {
  const long n = count_nodes(p);
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < n; ++idx) {
    int c[3];
    coords(p, idx, c);
    double gsum[3] = {0.0, 0.0, 0.0};
    double lsum = 0.0;
    for (int i = 0; i < L->q; ++i) {
      double v = fld[nb_stencil(p, c, L->e[i])];
      for (int a = 0; a < L->dim; ++a) gsum[a] += L->w[i] * L->e[i][a] * v;
      if (i > 0) lsum += L->w[i] * (v - fld[idx]);
    }
    if (grad)
      for (int a = 0; a < L->dim; ++a) grad[a * n + idx] = gsum[a] / CS2;
    if (lap) lap[idx] = 2.0 * lsum / CS2;
  }
}

void orc_grad_lap(const orc_params* prm, const double* field, double* grad,
                  double* lap) {
  lat_t L;
  if (lat_fill(prm->lattice, &L)) return;
  grad_lap_lat(prm, &L, field, grad, lap);
}

/* theta'(phi) for theta = beta phi^2 (phi - 1)^2 (Eq. 1a), or for the
 * symmetric theta = beta (phi^2 - phi*^2)^2 (Eq. 1b). */
static double dtheta_well(const orc_params* p, double phi) {
  if (p->well) return 4.0 * p->beta * phi * (phi * phi - p->phi_star * p->phi_star);
  return 2.0 * p->beta * phi * (phi - 1.0) * (2.0 * phi - 1.0);
}

/* theta(phi) itself: beta phi^2 (phi - 1)^2 (Eq. 1a) or beta (phi^2 - phi*^2)^2
 * (Eq. 1b). */
static double theta_well(const orc_params* p, double phi) {
  if (p->well) {
    const double d = phi * phi - p->phi_star * p->phi_star;
    return p->beta * d * d;
  }
  return p->beta * phi * phi * (phi - 1.0) * (phi - 1.0);
}

/* Density from the order parameter: Eq. 4a, rho_G + phi (rho_L - rho_G), or
 * Eq. 4b, rho_G + (phi + phi*) / (2 phi*) (rho_L - rho_G); both are
 * rho_G + (phi - phi_G) d rho / d phi. */
static double rho_of(const orc_params* p, double phi) {
  if (p->well)
    return p->rho_g + (phi + p->phi_star) / (2.0 * p->phi_star) * (p->rho_l - p->rho_g);
  return p->rho_g + phi * (p->rho_l - p->rho_g);
}
static double drho_dphi_of(const orc_params* p) {
  return p->well ? (p->rho_l - p->rho_g) / (2.0 * p->phi_star) : p->rho_l - p->rho_g;
}

static double dot(const double* a, const double* b, int dim) {
  double s = 0.0;
  for (int k = 0; k < dim; ++k) s += a[k] * b[k];
  return s;
}

static double edot(const lat_t* L, int i, const double* v) {
  double s = 0.0;
  for (int k = 0; k < L->dim; ++k) s += L->e[i][k] * v[k];
  return s;
}

/* omega_i(u) = w_i (1 + e.u/cs^2 + (e.u)^2/(2 cs^4) - u.u/(2 cs^2)) */
static double omega(const lat_t* L, int i, const double* u) {
  double eu = edot(L, i, u);
  double uu = dot(u, u, L->dim);
  return L->w[i] * (1.0 + eu / CS2 + 0.5 * eu * eu / (CS2 * CS2) - 0.5 * uu / CS2);
}

static void feq_lat(const lat_t* L, double phi, double mu, const double* u,
                    double gamma, double* out) {
  double uu = dot(u, u, L->dim);
  double rest = phi;
  for (int i = 1; i < L->q; ++i) {
    double eu = edot(L, i, u);
    out[i] = L->w[i] * (gamma * mu / CS2 +
                        phi * (eu / CS2 + 0.5 * eu * eu / (CS2 * CS2) - 0.5 * uu / CS2));
    rest -= out[i];
  }
  out[0] = rest;
}

/* g^eq_i = c_s^2 rho omega_i(u) + psi omega_i(0) with psi = p - rho c_s^2,
 * i.e. w_i p + c_s^2 rho (omega_i(u) - w_i). */
static void geq_lat(const lat_t* L, double p, double rho, const double* u,
                    double* out) {
  for (int i = 0; i < L->q; ++i)
    out[i] = L->w[i] * p + CS2 * rho * (omega(L, i, u) - L->w[i]);
}

/* (e_i - u) . K_i with K_i = F omega_i(u) - (omega_i(u) - omega_i(0)) grad psi
 * (Eq. 8; F already holds F_s + G and, in the corrected model, -F_a). */
static void source_lat(const lat_t* L, const double* u, const double* force,
                       const double* gpsi, double* out) {
  for (int i = 0; i < L->q; ++i) {
    double om = omega(L, i, u);
    double s = 0.0;
    for (int k = 0; k < L->dim; ++k) {
      double kk = force[k] * om - (om - L->w[i]) * gpsi[k];
      s += (L->e[i][k] - u[k]) * kk;
    }
    out[i] = s;
  }
}

/* First and zeroth moments of gbar give u and p:
 *   rho cs^2 u = sum e gbar + cs^2 F / 2,  F = F_s + G + c u,
 *   p = sum gbar - u . grad psi / 2  ~  sum gbar + cs^2 u . grad rho / 2
 * (u . grad p dropped, as the paper argues after Eq. 10). */
static void recover_lat(const lat_t* L, const double* gbar, double rho,
                        const double* fsg, double c, const double* gradrho,
                        double* u, double* force, double* p) {
  double m0 = 0.0, m1[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < L->q; ++i) {
    m0 += gbar[i];
    for (int k = 0; k < L->dim; ++k) m1[k] += L->e[i][k] * gbar[i];
  }
  double denom = rho - 0.5 * c;
  for (int k = 0; k < L->dim; ++k) {
    u[k] = (m1[k] / CS2 + 0.5 * fsg[k]) / denom;
    force[k] = fsg[k] + c * u[k];
  }
  *p = m0 + 0.5 * CS2 * dot(u, gradrho, L->dim);
}

void orc_feq(int lattice, double phi, double mu, const double* u, double gamma,
             double* out) {
  lat_t L;
  if (lat_fill(lattice, &L)) return;
  feq_lat(&L, phi, mu, u, gamma, out);
}

void orc_geq(int lattice, double p, double rho, const double* u, double* out) {
  lat_t L;
  if (lat_fill(lattice, &L)) return;
  geq_lat(&L, p, rho, u, out);
}

void orc_source(int lattice, const double* u, const double* force,
                const double* gradpsi, double* out) {
  lat_t L;
  if (lat_fill(lattice, &L)) return;
  source_lat(&L, u, force, gradpsi, out);
}

void orc_recover(int lattice, const double* gbar, double rho, const double* fsg,
                 double c, const double* gradrho, double* u, double* force,
                 double* p) {
  lat_t L;
  if (lat_fill(lattice, &L)) return;
  recover_lat(&L, gbar, rho, fsg, c, gradrho, u, force, p);
}

/* Streaming (S3): pull from x - e_i; a source beyond a wall means the
 * population left x towards the wall and came back reversed. */
static long stream_src(const orc_params* p, const lat_t* L, const int* c, int i,
                       int* opp_used) {
  int s[3];
  int n[3] = {p->nx, p->ny, p->nz};
  *opp_used = 0;
  for (int a = 0; a < 3; ++a) {
    s[a] = c[a] - L->e[i][a];
    if (p->wall[a]) {
      if (s[a] < 0 || s[a] >= n[a]) *opp_used = 1;
    } else {
      s[a] = map_axis(s[a], n[a], 0);
    }
  }
  if (*opp_used) return c[0] + (long)p->nx * (c[1] + (long)p->ny * c[2]);
  return s[0] + (long)p->nx * (s[1] + (long)p->ny * s[2]);
}

void orc_stream_words(const orc_params* prm, const unsigned* in, unsigned* out) {
  lat_t L;
  if (lat_fill(prm->lattice, &L)) return;
  const long n = count_nodes(prm);
  for (long idx = 0; idx < n; ++idx) {
    int c[3];
    coords(prm, idx, c);
    for (int i = 0; i < L.q; ++i) {
      int bb;
      long src = stream_src(prm, &L, c, i, &bb);
      out[i * n + idx] = bb ? in[L.opp[i] * n + src] : in[i * n + src];
    }
  }
}

/* ------------------------------------------------------------------------ */

static int params_ok(const orc_params* p, const lat_t* L) {
  if (p->nx < 4 || p->ny < 4) return 0;
  if (L->dim == 2 && p->nz != 1) return 0;
  if (L->dim == 3 && p->nz < 4) return 0;
  if (!(p->tau_f > 0.5) || !(p->tau_g > 0.5)) return 0;
  if (!(p->rho_l > 0.0) || !(p->rho_g > 0.0) || !(p->mu_ratio > 0.0)) return 0;
  if (p->well != 0 && p->well != 1) return 0;
  if (p->well == 1 && !(p->phi_star > 0.0)) return 0;
  if (p->remove_fa < 0 || p->remove_fa > 2) return 0;
  return 1;
}

static double* alloc0(long n) { return (double*)calloc((size_t)n, sizeof(double)); }

orc_sim* orc_create(const orc_params* prm, const double* phi0, const double* u0,
                    const double* p0) {
  lat_t L;
  if (lat_fill(prm->lattice, &L) || !params_ok(prm, &L)) return NULL;
  orc_sim* s = (orc_sim*)calloc(1, sizeof *s);
  s->prm = *prm;
  if (L.dim == 2) s->prm.wall[2] = 0;
  s->L = L;
  const long n = count_nodes(&s->prm);
  const int q = L.q, dim = L.dim;
  s->n = n;
  s->f = alloc0(q * n);
  s->g = alloc0(q * n);
  s->fn = alloc0(q * n);
  s->gn = alloc0(q * n);
  s->phi = alloc0(n);
  s->rho = alloc0(n);
  s->gphi = alloc0(dim * n);
  s->lphi = alloc0(n);
  s->mu = alloc0(n);
  s->lmu = alloc0(n);
  s->u = alloc0(dim * n);
  s->force = alloc0(dim * n);
  s->pr = alloc0(n);
  s->gpsi = alloc0(dim * n);
  s->tau = alloc0(n);
  s->phi_prev = alloc0(n);
  s->rhou = alloc0(dim * n);
  s->grad = alloc0(dim * n);
  s->dmass = alloc0(n);

  /* Theta_M = Gamma (tau_f - 1/2) for the BGK Cahn-Hilliard LBE. */
  s->gamma = prm->theta_m / (prm->tau_f - 0.5);
  s->drho = prm->rho_l - prm->rho_g;
  s->phi_g = prm->well ? -prm->phi_star : 0.0;
  s->phi_l = prm->well ? prm->phi_star : 1.0;
  s->drho_dphi = drho_dphi_of(prm);
  /* Liquid kinematic viscosity nu_L = cs^2 (tau_g - 1/2); dynamic viscosity
   * linear in phi between mu_G = mu_L / ratio (at phi_G) and mu_L (at phi_L). */
  s->mu_l = prm->rho_l * CS2 * (prm->tau_g - 0.5);
  s->mu_g = s->mu_l / prm->mu_ratio;

  /* Initial state: equilibria of the given phi, u, p, with mu from the same
   * stencils as the step. */
  for (long idx = 0; idx < n; ++idx) {
    s->phi[idx] = phi0[idx];
    s->phi_prev[idx] = phi0[idx];
    s->rho[idx] = rho_of(prm, phi0[idx]);
  }
  grad_lap_lat(&s->prm, &L, s->phi, s->gphi, s->lphi);
  for (long idx = 0; idx < n; ++idx) {
    double uu[3] = {0.0, 0.0, 0.0};
    double fe[QMAX], ge[QMAX];
    for (int k = 0; k < dim; ++k) uu[k] = u0[k * n + idx];
    double mu = dtheta_well(prm, s->phi[idx]) - prm->kappa * s->lphi[idx];
    feq_lat(&L, s->phi[idx], mu, uu, s->gamma, fe);
    geq_lat(&L, p0[idx], s->rho[idx], uu, ge);
    for (int i = 0; i < q; ++i) {
      s->f[i * n + idx] = fe[i];
      s->g[i * n + idx] = ge[i];
    }
  }
  double d[20];
  orc_diag(s, d);
  s->mass0 = d[0];
  s->time = 0;
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  double* bufs[] = {s->f,   s->g,      s->fn,   s->gn,   s->phi,  s->rho,
                    s->gphi, s->lphi, s->mu,   s->lmu,  s->u,    s->force,
                    s->pr,  s->gpsi,  s->tau,  s->phi_prev, s->rhou, s->grad, s->dmass};
  for (size_t k = 0; k < sizeof bufs / sizeof bufs[0]; ++k) free(bufs[k]);
  free(s);
}

long orc_time(const orc_sim* s) { return s->time; }

/* Force of Eq. 3 without the correction, F_s + G (F_s = mu grad phi, G along
 * -vert), and grad rho, at node idx from the stencils of S1b. */
static void node_forces(const orc_sim* s, long idx, double* fsg, double* grho) {
  const orc_params* p = &s->prm;
  const long n = s->n;
  const int dim = s->L.dim;
  const int vert = dim - 1; /* gravity acts along -y in 2-D and -z in 3-D */
  for (int k = 0; k < 3; ++k) fsg[k] = grho[k] = 0.0;
  for (int k = 0; k < dim; ++k) {
    fsg[k] = s->mu[idx] * s->gphi[k * n + idx];   /* F_s = mu grad phi */
    grho[k] = s->drho_dphi * s->gphi[k * n + idx];  /* grad rho */
  }
  fsg[vert] += -(s->rho[idx] - p->rho_ref) * p->gravity;   /* G */
}

/* S1a..S1e on the current populations.  want_lmu forces lap mu even for the
 * original model (used by the field dump for the F_a diagnostic). */
static void sweep_fields(orc_sim* s, int want_lmu) {
  const orc_params* p = &s->prm;
  const lat_t* L = &s->L;
  const long n = s->n;
  const int q = L->q, dim = L->dim;

  /* S1a: order parameter and density. */
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < n; ++idx) {
    double sum = 0.0;
    for (int i = 0; i < q; ++i) sum += s->f[i * n + idx];
    s->phi[idx] = sum;
    s->rho[idx] = rho_of(p, sum);
  }
  /* S1b: stencils and chemical potential. */
  grad_lap_lat(p, L, s->phi, s->gphi, s->lphi);
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < n; ++idx)
    s->mu[idx] = dtheta_well(p, s->phi[idx]) - p->kappa * s->lphi[idx];
  /* S1c: Laplacian of mu, the divergence of the diffusive flux in Eq. 5. */
  if (p->remove_fa || want_lmu)
    grad_lap_lat(p, L, s->mu, NULL, s->lmu);
  else
    memset(s->lmu, 0, (size_t)n * sizeof(double));
  /* S1c': remove_fa = 2 takes the rate d_t rho + div(rho u) of Eq. 12 from
   * the data instead of from Eq. 5: D = (rho^n - rho^(n-1)) +
   * div(rho u_o), u_o the velocity the original model recovers at this step
   * (D must not depend on the u it corrects, so that the recovery stays
   * local and closed-form). */
  if (p->remove_fa == 2) {
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < n; ++idx) {
      double gb[QMAX], fsg[3], grho[3], uu[3], ff[3], pp;
      for (int i = 0; i < q; ++i) gb[i] = s->g[i * n + idx];
      node_forces(s, idx, fsg, grho);
      recover_lat(L, gb, s->rho[idx], fsg, 0.0, grho, uu, ff, &pp);
      for (int k = 0; k < dim; ++k) s->rhou[k * n + idx] = s->rho[idx] * uu[k];
    }
    for (long idx = 0; idx < n; ++idx)
      s->dmass[idx] = s->drho_dphi * (s->phi[idx] - s->phi_prev[idx]);
    for (int a = 0; a < dim; ++a) {
      grad_lap_lat(p, L, s->rhou + (long)a * n, s->grad, NULL);
      for (long idx = 0; idx < n; ++idx) s->dmass[idx] += s->grad[(long)a * n + idx];
    }
  }
  /* S1d: forces, velocity, pressure. */
  const double sw = p->remove_fa == 1 ? 1.0 : 0.0;
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < n; ++idx) {
    double gb[QMAX], fsg[3], grho[3], uu[3], ff[3], pp;
    for (int i = 0; i < q; ++i) gb[i] = s->g[i * n + idx];
    node_forces(s, idx, fsg, grho);
    double c = sw * s->drho_dphi * p->theta_m * s->lmu[idx];  /* -F_a = c u */
    if (p->remove_fa == 2) c = s->dmass[idx];
    recover_lat(L, gb, s->rho[idx], fsg, c, grho, uu, ff, &pp);
    for (int k = 0; k < dim; ++k) {
      s->u[k * n + idx] = uu[k];
      s->force[k * n + idx] = ff[k];
    }
    s->pr[idx] = pp;
  }
  /* S1e: grad psi = grad p - cs^2 grad rho, local relaxation time. */
  grad_lap_lat(p, L, s->pr, s->gpsi, NULL);
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < n; ++idx) {
    for (int k = 0; k < dim; ++k)
      s->gpsi[k * n + idx] -= CS2 * s->drho_dphi * s->gphi[k * n + idx];
    double frac = (s->phi[idx] - s->phi_g) / (s->phi_l - s->phi_g);
    double nu = (s->mu_g + frac * (s->mu_l - s->mu_g)) / s->rho[idx];
    s->tau[idx] = 0.5 + nu / CS2;
  }
}

static void collide(orc_sim* s) {
  const lat_t* L = &s->L;
  const long n = s->n;
  const int q = L->q, dim = L->dim;
  const double tf = s->prm.tau_f;
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < n; ++idx) {
    double uu[3] = {0, 0, 0}, ff[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
    double fe[QMAX], ge[QMAX], src[QMAX];
    for (int k = 0; k < dim; ++k) {
      uu[k] = s->u[k * n + idx];
      ff[k] = s->force[k * n + idx];
      gp[k] = s->gpsi[k * n + idx];
    }
    feq_lat(L, s->phi[idx], s->mu[idx], uu, s->gamma, fe);
    geq_lat(L, s->pr[idx], s->rho[idx], uu, ge);
    source_lat(L, uu, ff, gp, src);
    const double tg = s->tau[idx];
    for (int i = 0; i < q; ++i) {
      double fi = s->f[i * n + idx];
      double gi = s->g[i * n + idx];
      s->f[i * n + idx] = fi - (fi - fe[i]) / tf;
      s->g[i * n + idx] = gi - (gi - ge[i]) / tg + (1.0 - 1.0 / (2.0 * tg)) * src[i];
    }
  }
}

static void stream(orc_sim* s) {
  const orc_params* p = &s->prm;
  const lat_t* L = &s->L;
  const long n = s->n;
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < n; ++idx) {
    int c[3];
    coords(p, idx, c);
    for (int i = 0; i < L->q; ++i) {
      int bb;
      long src = stream_src(p, L, c, i, &bb);
      int j = bb ? L->opp[i] : i;
      s->fn[i * n + idx] = s->f[j * n + src];
      s->gn[i * n + idx] = s->g[j * n + src];
    }
  }
  double* t = s->f;
  s->f = s->fn;
  s->fn = t;
  t = s->g;
  s->g = s->gn;
  s->gn = t;
}

void orc_step(orc_sim* s, long nsteps) {
  for (long k = 0; k < nsteps; ++k) {
    sweep_fields(s, 0);
    memcpy(s->phi_prev, s->phi, (size_t)s->n * sizeof(double));
    collide(s);
    stream(s);
    s->time++;
  }
}

void orc_fields(orc_sim* s, double* phi, double* u, double* p, double* mu,
                double* lapmu, double* fa) {
  const long n = s->n;
  const int dim = s->L.dim;
  sweep_fields(s, 1);
  if (phi) memcpy(phi, s->phi, (size_t)n * sizeof(double));
  if (u) memcpy(u, s->u, (size_t)(dim * n) * sizeof(double));
  if (p) memcpy(p, s->pr, (size_t)n * sizeof(double));
  if (mu) memcpy(mu, s->mu, (size_t)n * sizeof(double));
  if (lapmu) memcpy(lapmu, s->lmu, (size_t)n * sizeof(double));
  if (fa)
    for (int k = 0; k < dim; ++k)
      for (long idx = 0; idx < n; ++idx)
        fa[k * n + idx] =
            -s->u[k * n + idx] * s->drho_dphi * s->prm.theta_m * s->lmu[idx];
}

void orc_diag(orc_sim* s, double* out) {
  const orc_params* p = &s->prm;
  const long n = s->n;
  const int dim = s->L.dim;
  sweep_fields(s, 0);
  for (int k = 0; k < 20; ++k) out[k] = 0.0;
  double mass = 0.0, mom[3] = {0, 0, 0}, sw = 0.0, swx[3] = {0, 0, 0},
         swu[3] = {0, 0, 0}, umax = 0.0, bad = 0.0;
  for (long idx = 0; idx < n; ++idx) {
    int c[3];
    coords(p, idx, c);
    double ph = s->phi[idx];
    mass += ph;
    double w = 2.0 * (ph - s->phi_g) / (s->phi_l - s->phi_g) - 0.5;
    w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
    sw += w;
    double uu = 0.0;
    int finite = isfinite(ph);
    for (int k = 0; k < dim; ++k) {
      double uk = s->u[k * n + idx];
      mom[k] += s->rho[idx] * uk;
      swx[k] += w * c[k];
      swu[k] += w * uk;
      uu += uk * uk;
      finite = finite && isfinite(uk);
    }
    if (!finite) bad += 1.0;
    double um = sqrt(uu);
    if (um > umax) umax = um;
  }
  double cen[3] = {0, 0, 0}, m2[3] = {0, 0, 0};
  for (int k = 0; k < dim; ++k) cen[k] = sw > 0.0 ? swx[k] / sw : 0.0;
  for (long idx = 0; idx < n; ++idx) {
    int c[3];
    coords(p, idx, c);
    double w = 2.0 * (s->phi[idx] - s->phi_g) / (s->phi_l - s->phi_g) - 0.5;
    w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
    for (int k = 0; k < dim; ++k) m2[k] += w * (c[k] - cen[k]) * (c[k] - cen[k]);
  }
  out[0] = mass;
  out[1] = s->time == 0 && s->mass0 == 0.0 ? mass : s->mass0;
  for (int k = 0; k < dim; ++k) {
    out[2 + k] = mom[k];
    out[6 + k] = cen[k];
    out[9 + k] = sw > 0.0 ? swu[k] / sw : 0.0;
    out[12 + k] = sw > 0.0 ? m2[k] / sw : 0.0;
  }
  out[5] = sw;
  out[15] = umax;
  out[16] = bad;
}

/* The diagnostics of orc_diag from given node fields phi[n] and u[dim*n]
 * (n = nx ny nz, node x + nx (y + ny z)): rho linear in phi through (phi_g,
 * rho_g) and (phi_l, rho_l) (Eq. 4a / 4b), centroid weight clamp(2 s - 1/2,
 * 0, 1) with s the fraction of the way from phi_g to phi_l.  out[16]: mass,
 * momentum[3], sum w, centroid[3], centroid velocity[3], second moment about
 * the centroid[3], max |u|, number of nodes with a non-finite phi or u. */
void orc_field_diag(int dim, int nx, int ny, int nz, const double* phi, const double* u,
                    double phi_g, double phi_l, double rho_g, double rho_l, double* out) {
  const long n = (long)nx * ny * (dim == 3 ? nz : 1);
  for (int k = 0; k < 16; ++k) out[k] = 0.0;
  double sw = 0.0, sx[3] = {0, 0, 0};
  for (long idx = 0; idx < n; ++idx) {
    const long x[3] = {idx % nx, (idx / nx) % ny, idx / ((long)nx * ny)};
    const double ph = phi[idx];
    const double rho = rho_g + (ph - phi_g) * (rho_l - rho_g) / (phi_l - phi_g);
    double w = 2.0 * (ph - phi_g) / (phi_l - phi_g) - 0.5;
    w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
    double uu = 0.0;
    int finite = isfinite(ph);
    out[0] += ph;
    sw += w;
    for (int k = 0; k < dim; ++k) {
      const double uk = u[k * n + idx];
      out[1 + k] += rho * uk;
      sx[k] += w * x[k];
      out[8 + k] += w * uk;
      uu += uk * uk;
      finite = finite && isfinite(uk);
    }
    if (sqrt(uu) > out[14]) out[14] = sqrt(uu);
    if (!finite) out[15] += 1.0;
  }
  out[4] = sw;
  for (int k = 0; k < dim; ++k) {
    out[5 + k] = sw > 0.0 ? sx[k] / sw : 0.0;
    out[8 + k] = sw > 0.0 ? out[8 + k] / sw : 0.0;
  }
  for (long idx = 0; idx < n; ++idx) {
    const long x[3] = {idx % nx, (idx / nx) % ny, idx / ((long)nx * ny)};
    double w = 2.0 * (phi[idx] - phi_g) / (phi_l - phi_g) - 0.5;
    w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
    for (int k = 0; k < dim; ++k) {
      const double d = x[k] - out[5 + k];
      out[11 + k] += w * d * d;
    }
  }
  for (int k = 0; k < dim; ++k) out[11 + k] = sw > 0.0 ? out[11 + k] / sw : 0.0;
}

double orc_spread_radius(int nx, int ny, int nz, const double* phi, double level) {
  double best = 0.0;
  for (long r = 0; r < (long)ny * nz; ++r) {
    const double* row = phi + r * nx;
    double left = 0.0, right = 0.0;
    int found = 0;
    for (int x = 0; x + 1 < nx; ++x) {
      const double a = row[x], b = row[x + 1];
      if ((a >= level) == (b >= level)) continue;
      const double pos = x + (level - a) / (b - a);
      if (found == 0 || pos < left) left = pos;
      if (found == 0 || pos > right) right = pos;
      ++found;
    }
    if (found >= 2 && 0.5 * (right - left) > best) best = 0.5 * (right - left);
  }
  return best;
}

void orc_fa_discrete(const orc_params* prm, const double* phi_prev, const double* phi,
                     const double* u, double* out) {
  lat_t L;
  if (lat_fill(prm->lattice, &L)) return;
  const long n = count_nodes(prm);
  const double drho = drho_dphi_of(prm);
  double* m = alloc0(n);
  double* grad = alloc0((long)L.dim * n);
  double* div = alloc0(n);
  for (int a = 0; a < L.dim; ++a) {
    for (long idx = 0; idx < n; ++idx) m[idx] = rho_of(prm, phi[idx]) * u[a * n + idx];
    grad_lap_lat(prm, &L, m, grad, NULL);
    for (long idx = 0; idx < n; ++idx) div[idx] += grad[a * n + idx];
  }
  for (long idx = 0; idx < n; ++idx) {
    const double dt_rho = (phi[idx] - phi_prev[idx]) * drho;
    for (int a = 0; a < L.dim; ++a) out[a * n + idx] = -u[a * n + idx] * (dt_rho + div[idx]);
  }
  free(m);
  free(grad);
  free(div);
}

void orc_fa_leelin(const orc_params* prm, const double* phi, const double* u,
                   const double* pr, double* out) {
  lat_t L;
  if (lat_fill(prm->lattice, &L)) return;
  const long n = count_nodes(prm);
  const double phi_g = prm->well ? -prm->phi_star : 0.0;
  const double phi_l = prm->well ? prm->phi_star : 1.0;
  /* dynamic viscosity: mu_L = rho_L nu_L with nu_L = cs^2 (tau_g - 1/2),
   * mu_G = mu_L / ratio, linear in phi between the bulk values */
  const double mu_l = prm->rho_l * CS2 * (prm->tau_g - 0.5);
  const double mu_g = mu_l / prm->mu_ratio;
  double* q = alloc0(n);
  double* lam = alloc0(n);
  double* gq = alloc0((long)L.dim * n);
  double* lq = alloc0(n);
  double* gl = alloc0((long)L.dim * n);
  for (long idx = 0; idx < n; ++idx) {
    const double ph = phi[idx];
    const double thermo = ph * dtheta_well(prm, ph) - theta_well(prm, ph);  /* P */
    q[idx] = thermo - pr[idx];
    const double mud = mu_g + (ph - phi_g) / (phi_l - phi_g) * (mu_l - mu_g);
    lam[idx] = mud / (rho_of(prm, ph) * CS2);
  }
  grad_lap_lat(prm, &L, q, gq, lq);
  grad_lap_lat(prm, &L, lam, gl, NULL);
  for (long idx = 0; idx < n; ++idx) {
    double div = lam[idx] * lq[idx];
    for (int a = 0; a < L.dim; ++a) div += gl[a * n + idx] * gq[a * n + idx];
    for (int a = 0; a < L.dim; ++a) out[a * n + idx] = -u[a * n + idx] * div;
  }
  free(q);
  free(lam);
  free(gq);
  free(lq);
  free(gl);
}

void orc_get_state(const orc_sim* s, double* f, double* g) {
  const size_t bytes = (size_t)(s->L.q * s->n) * sizeof(double);
  if (f) memcpy(f, s->f, bytes);
  if (g) memcpy(g, s->g, bytes);
}

void orc_set_state(orc_sim* s, const double* f, const double* g, long time) {
  const size_t bytes = (size_t)(s->L.q * s->n) * sizeof(double);
  memcpy(s->f, f, bytes);
  memcpy(s->g, g, bytes);
  s->time = time;
}
