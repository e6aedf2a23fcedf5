/*
 * lbm_oracle.c -- CPU FP64 oracle of the coupled lattice step.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow and written to be checked against the
 * paper by eye: array-of-structures populations, two buffers with push
 * streaming, literal Hermite tensors, brute-force near-contact search.  Only
 * the test-suite, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code with the GPU library.  Build: see oracle/build.py
 * (gcc -O2 -fopenmp -ffp-contract=off).
 *
 * One step (all terms from the state at time n, f and g advance together):
 *   1. phi = sum_i g_i                                    (CAC populations)
 *   2. grad phi, lap phi: isotropic stencils, Sec. 2.1 "Discrete derivatives"
 *      (Eqs. grad_iso, lap_iso) with the hydrodynamic lattice weights;
 *      n = grad phi / (|grad phi| + eps_n)                (Sec. 2.3.1, Eq. n_discrete)
 *      q = phic (1 - phic), phic = clamp(phi, 0, 1)       (Sec. 2.3.1, Eq. q_discrete)
 *      mu_phi = 4 beta phi (phi-1)(phi-1/2) - kappa lap phi, beta = 12 sigma/W,
 *      kappa = 3 sigma W / 2 (chemical potential; the paper names it without
 *      defining it, this is the standard conservative Allen-Cahn form)
 *   3. near-contact detection and pairing (Sec. 2.3.2) and force (Sec. 2.3.3)
 *   4. macroscopic fields and forces (Sec. 2.1: Eqs. pstar_moment, u_moment,
 *      mu_mix_linear, nu_from_mu, omega_phi, Fsplit, Fcap, Fp, Fnu)
 *   5. recursive-regularised collision with Guo forcing (Eqs. lbe, feq3, H2,
 *      H3, fneq3, A3rec, guo) and the CAC lattice Boltzmann collision, then
 *      push streaming of both population sets.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Lattices                                                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
  int q;
  int c[27][3];
  double w[27];
  double cs2;
  int opp[27];
} lattice;

static void finish_lattice(lattice* L) {
  for (int i = 0; i < L->q; ++i) {
    L->opp[i] = -1;
    for (int j = 0; j < L->q; ++j)
      if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] && L->c[j][2] == -L->c[i][2])
        L->opp[i] = j;
  }
}

/* D2Q9: rest 4/9, axis 1/9, diagonal 1/36, cs^2 = 1/3 */
static void make_d2q9(lattice* L) {
  static const int c[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                              {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
  L->q = 9;
  L->cs2 = 1.0 / 3.0;
  for (int i = 0; i < 9; ++i) {
    for (int a = 0; a < 3; ++a) L->c[i][a] = c[i][a];
    int s = abs(c[i][0]) + abs(c[i][1]);
    L->w[i] = (s == 0) ? 4.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  finish_lattice(L);
}

/* D3Q19: rest 1/3, axis 1/18, face diagonal 1/36, cs^2 = 1/3 */
static void make_d3q19(lattice* L) {
  int k = 0;
  L->q = 19;
  L->cs2 = 1.0 / 3.0;
  for (int z = -1; z <= 1; ++z)
    for (int y = -1; y <= 1; ++y)
      for (int x = -1; x <= 1; ++x) {
        int s = abs(x) + abs(y) + abs(z);
        if (s == 3) continue;
        L->c[k][0] = x;
        L->c[k][1] = y;
        L->c[k][2] = z;
        L->w[k] = (s == 0) ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        ++k;
      }
  finish_lattice(L);
}

/* D3Q27 (the paper's hydrodynamic lattice): rest 8/27, axis 2/27, face diagonal
 * 1/54, body diagonal 1/216, cs^2 = 1/3 */
static void make_d3q27(lattice* L) {
  int k = 0;
  L->q = 27;
  L->cs2 = 1.0 / 3.0;
  for (int z = -1; z <= 1; ++z)
    for (int y = -1; y <= 1; ++y)
      for (int x = -1; x <= 1; ++x) {
        int s = abs(x) + abs(y) + abs(z);
        L->c[k][0] = x;
        L->c[k][1] = y;
        L->c[k][2] = z;
        L->w[k] = s == 0 ? 8.0 / 27.0 : (s == 1 ? 2.0 / 27.0 : (s == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
        ++k;
      }
  finish_lattice(L);
}

/* D3Q7 (phase field): rest 1/4, axis 1/8, cs^2 = 1/4 */
static void make_d3q7(lattice* L) {
  int k = 0;
  L->q = 7;
  L->cs2 = 0.25;
  for (int z = -1; z <= 1; ++z)
    for (int y = -1; y <= 1; ++y)
      for (int x = -1; x <= 1; ++x) {
        int s = abs(x) + abs(y) + abs(z);
        if (s > 1) continue;
        L->c[k][0] = x;
        L->c[k][1] = y;
        L->c[k][2] = z;
        L->w[k] = (s == 0) ? 0.25 : 0.125;
        ++k;
      }
  finish_lattice(L);
}

int oracle_lattice(int kind, int* q, int* c, double* w, double* cs2) {
  lattice L;
  if (kind == 0) make_d2q9(&L);
  else if (kind == 1) make_d3q19(&L);
  else if (kind == 2) make_d3q7(&L);
  else if (kind == 3) make_d3q27(&L);
  else return -1;
  *q = L.q;
  *cs2 = L.cs2;
  for (int i = 0; i < L.q; ++i) {
    w[i] = L.w[i];
    for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Hermite tensors, equilibrium, Guo source, regularisation (Sec. 2.1)       */
/* ------------------------------------------------------------------------- */

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

/* H2_ab = c_a c_b - cs^2 delta_ab   (Eq. H2) */
static double H2(const int* c, double cs2, int a, int b) { return c[a] * c[b] - cs2 * kd(a, b); }

/* H3_abg = c_a c_b c_g - cs^2 (c_a d_bg + c_b d_ag + c_g d_ab)   (Eq. H3) */
static double H3(const int* c, double cs2, int a, int b, int g) {
  return (double)(c[a] * c[b] * c[g]) - cs2 * (c[a] * kd(b, g) + c[b] * kd(a, g) + c[g] * kd(a, b));
}

/* Third-order equilibrium, Eq. feq3, contracted literally. */
static double feq_i(const lattice* L, int D, int i, double pstar, const double* u) {
  const int* c = L->c[i];
  double cs2 = L->cs2;
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;
  for (int a = 0; a < D; ++a) t1 += c[a] * u[a];
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) t2 += H2(c, cs2, a, b) * u[a] * u[b];
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b)
      for (int g = 0; g < D; ++g) t3 += H3(c, cs2, a, b, g) * u[a] * u[b] * u[g];
  return L->w[i] * (pstar + t1 / cs2 + t2 / (2.0 * cs2 * cs2) + t3 / (6.0 * cs2 * cs2 * cs2));
}

/* Guo source, Eq. guo: S_i = w_i [ (c_i - u)/cs^2 + (c_i.u) c_i / cs^4 ] . F / rho */
static double guo_i(const lattice* L, int D, int i, const double* u, const double* F, double rho) {
  const int* c = L->c[i];
  double cs2 = L->cs2;
  double cu = 0.0;
  for (int a = 0; a < D; ++a) cu += c[a] * u[a];
  double s = 0.0;
  for (int a = 0; a < D; ++a) s += ((c[a] - u[a]) / cs2 + cu * c[a] / (cs2 * cs2)) * F[a] / rho;
  return L->w[i] * s;
}

/* Recursive regularisation, Eqs. fneq3 and A3rec:
 * A2 = sum_i H2_i fneq_i;  A3 = S(u (x) A2);
 * R_i = w_i [ H2_i : A2 / (2 cs^4) + H3_i ... A3 / (6 cs^6) ]. */
static void regularize(const lattice* L, int D, const double* fneq, const double* u, double* out) {
  double cs2 = L->cs2;
  double A2[3][3] = {{0}};
  for (int i = 0; i < L->q; ++i)
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) A2[a][b] += H2(L->c[i], cs2, a, b) * fneq[i];
  double A3[3][3][3];
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b)
      for (int g = 0; g < D; ++g) A3[a][b][g] = u[a] * A2[b][g] + u[b] * A2[a][g] + u[g] * A2[a][b];
  for (int i = 0; i < L->q; ++i) {
    double t2 = 0.0, t3 = 0.0;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) t2 += H2(L->c[i], cs2, a, b) * A2[a][b];
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        for (int g = 0; g < D; ++g) t3 += H3(L->c[i], cs2, a, b, g) * A3[a][b][g];
    out[i] = L->w[i] * (t2 / (2.0 * cs2 * cs2) + t3 / (6.0 * cs2 * cs2 * cs2));
  }
}

/* Hydrodynamic lattice: D2Q9 in 2D; D3Q19 (q = 19, or 0) or D3Q27 (q = 27) in 3D. */
static int hydro_lattice(int dim, int q, lattice* L) {
  if (dim == 2) make_d2q9(L);
  else if (q == 27) make_d3q27(L);
  else if (q == 19 || q == 0) make_d3q19(L);
  else return -1;
  return 0;
}

int oracle_feq(int dim, int q, double pstar, const double* u, double* out) {
  lattice L;
  if (hydro_lattice(dim, q, &L)) return -1;
  for (int i = 0; i < L.q; ++i) out[i] = feq_i(&L, dim, i, pstar, u);
  return 0;
}

int oracle_guo(int dim, int q, const double* u, const double* F, double rho, double* out) {
  lattice L;
  if (hydro_lattice(dim, q, &L)) return -1;
  for (int i = 0; i < L.q; ++i) out[i] = guo_i(&L, dim, i, u, F, rho);
  return 0;
}

int oracle_regularize(int dim, int q, const double* fneq, const double* u, double* out) {
  lattice L;
  if (hydro_lattice(dim, q, &L)) return -1;
  regularize(&L, dim, fneq, u, out);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Near-contact interaction (Sec. 2.3)                                        */
/* ------------------------------------------------------------------------- */

/* h = W arcosh(1 / (2 sqrt(q)))   (Sec. 2.2.4 Eq. h_of_q, Sec. 2.3.3 Eq. h_impl) */
double oracle_film_thickness(const oracle_params* p, double q) {
  return p->width * acosh(1.0 / (2.0 * sqrt(q)));
}

/* w_h = 1 / (1 + (h/h0)^p)   (Eq. wh_general; h0 = 1, p = 4 gives Eq. wh_impl) */
double oracle_thickness_weight(const oracle_params* p, double h) {
  return 1.0 / (1.0 + pow(h / p->h0, p->p_exp));
}

static long wrapi(long i, long n) {
  long r = i % n;
  return r < 0 ? r + n : r;
}

/* Detection and pairing (Sec. 2.3.2) then force construction (Sec. 2.3.3).
 * Candidates y = x + r, r in the cubic (square in 2D) window of radius w, r != 0,
 * scanned with dz outermost, then dy, then dx, each from -w to +w.
 * Accept: q(y) >= q_th; |q(y)-q(x)| <= eta max(q(x), eps_q); n(x).n(y) <= cos_opp.
 * Choose the smallest |r|^2; among equal |r|^2 the largest facing score
 * (smallest n(x).n(y)); scores within tie_eps of that best count as tied and
 * the first of them in scan order is taken, so that rounding-level differences
 * in n cannot flip the choice between mirror-image candidates. */
int oracle_nci_from_qn(const oracle_params* P, const double* q, const double* n, int* chi,
                       int* partner, double* J) {
  const int D = P->dim;
  const long nx = P->nx, ny = P->ny, nz = (D == 2) ? 1 : P->nz;
  const long N = nx * ny * nz;
  const int w = P->nci_window;
  const int wz = (D == 2) ? 0 : w;
#pragma omp parallel for schedule(dynamic, 256)
  for (long idx = 0; idx < N; ++idx) {
    long x = idx % nx, y = (idx / nx) % ny, z = idx / (nx * ny);
    chi[idx] = 0;
    for (int a = 0; a < 3; ++a) partner[a * N + idx] = 0;
    for (int a = 0; a < D; ++a) J[a * N + idx] = 0.0;
    if (P->a_rep == 0.0) continue;
    double qx = q[idx];
    if (!(qx >= P->q_th)) continue; /* interfacial gate, Eq. q_gate */
    double nxv[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) nxv[a] = n[a * N + idx];
    /* Pass 1: accepted candidates (three tests of Sec. 2.3.2); smallest |r|^2 and,
     * among those, the smallest n(x).n(y) (largest facing score). */
    int found = 0, best[3] = {0, 0, 0};
    long best_d2 = 0;
    double best_dot = 0.0;
    long best_idx = -1;
    for (int pass = 0; pass < 2; ++pass) {
      for (int dz = -wz; dz <= wz; ++dz)
        for (int dy = -w; dy <= w; ++dy)
          for (int dx = -w; dx <= w; ++dx) {
            if (dx == 0 && dy == 0 && dz == 0) continue;
            long jdx = wrapi(x + dx, nx) + nx * (wrapi(y + dy, ny) + ny * wrapi(z + dz, nz));
            double qy = q[jdx];
            if (!(qy >= P->q_th)) continue;                                    /* neighbour gate */
            double qmax = qx > P->eps_q ? qx : P->eps_q;
            if (!(fabs(qy - qx) <= P->eta * qmax)) continue;                   /* Eq. q_similarity */
            double dot = 0.0;
            for (int a = 0; a < D; ++a) dot += nxv[a] * n[a * N + jdx];
            if (!(dot <= P->cos_opp)) continue;                                /* Eq. facing_threshold */
            long d2 = (long)dx * dx + (long)dy * dy + (long)dz * dz;
            if (pass == 0) {
              if (!found || d2 < best_d2 || (d2 == best_d2 && dot < best_dot)) {
                found = 1;
                best_d2 = d2;
                best_dot = dot;
              }
            } else if (best_idx < 0 && d2 == best_d2 && dot <= best_dot + P->tie_eps) {
              /* Pass 2: the first candidate in scan order whose facing score ties the
               * best within tie_eps. */
              best[0] = dx;
              best[1] = dy;
              best[2] = dz;
              best_idx = jdx;
              best_dot = dot;
            }
          }
      if (!found) break;
    }
    if (!found) continue;
    chi[idx] = 1; /* Eq. mask_partner_def */
    for (int a = 0; a < 3; ++a) partner[a * N + idx] = best[a];
    double ny_[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) ny_[a] = n[a * N + best_idx];
    /* Eqs. qpair_impl, q_clamp */
    double qpair = 0.5 * (qx + q[best_idx]);
    double qcl = qpair;
    if (qcl < P->eps_q) qcl = P->eps_q;
    if (qcl > 0.25 - P->eps_q) qcl = 0.25 - P->eps_q;
    /* Eq. face_impl */
    double ff = -best_dot > 0.0 ? -best_dot : 0.0;
    if (ff == 0.0) continue;
    /* Eq. nsym_impl with the line-of-centres fallback */
    double rn = sqrt((double)best_d2);
    double rhat[3] = {best[0] / rn, best[1] / rn, best[2] / rn};
    double nt[3] = {0, 0, 0}, nn = 0.0;
    for (int a = 0; a < D; ++a) {
      nt[a] = nxv[a] - ny_[a];
      nn += nt[a] * nt[a];
    }
    nn = sqrt(nn);
    double ns[3] = {0, 0, 0};
    if (nn < 1e-6) {
      for (int a = 0; a < D; ++a) ns[a] = rhat[a];
    } else {
      for (int a = 0; a < D; ++a) ns[a] = nt[a] / (nn + P->eps_n);
    }
    /* orientation */
    double ref = 0.0;
    if (P->rep_orient == 0) {
      for (int a = 0; a < D; ++a) ref += nxv[a] * ns[a];
    } else {
      for (int a = 0; a < D; ++a) ref += rhat[a] * ns[a];
      ref *= (double)P->rep_orient;
    }
    if (ref < 0.0)
      for (int a = 0; a < D; ++a) ns[a] = -ns[a];
    /* Eqs. h_impl, wh_impl, Jrep_impl */
    double h = oracle_film_thickness(P, qcl);
    double wh = oracle_thickness_weight(P, h);
    for (int a = 0; a < D; ++a) J[a * N + idx] = P->a_rep * qcl * wh * ff * ns[a];
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* State                                                                      */
/* ------------------------------------------------------------------------- */

struct oracle_state {
  oracle_params P;
  int D;
  long nx, ny, nz, N;
  lattice LF, LG;
  double *f, *f2, *g, *g2;                     /* AoS: f[idx*q + i] */
  double *phi, *grad, *lap, *nrm, *q, *mu;     /* per cell, vectors SoA [a*N + idx] */
  double *phi2, *acomp;                        /* MUSCL mode: next phi, compressive flux */
  double *J;
  int *chi, *partner;
  double *pstar, *rho, *u, *F, *omega, *nu;
  double rho_l, rho_g, nu_l, nu_g, rho_mean;
  int dispersed;
  long step;
};

static double* dalloc(long n) { return (double*)calloc((size_t)n, sizeof(double)); }

oracle_state* oracle_create(const oracle_params* p) {
  if (!p || (p->dim != 2 && p->dim != 3) || p->nx < 1 || p->ny < 1 || (p->dim == 3 && p->nz < 1))
    return NULL;
  if (p->dim == 3 && p->hydro_q != 0 && p->hydro_q != 19 && p->hydro_q != 27) return NULL;
  oracle_state* s = (oracle_state*)calloc(1, sizeof(oracle_state));
  s->P = *p;
  s->D = p->dim;
  s->nx = p->nx;
  s->ny = p->ny;
  s->nz = (p->dim == 2) ? 1 : p->nz;
  s->P.nz = (int)s->nz;
  s->N = s->nx * s->ny * s->nz;
  if (s->D == 2) {
    make_d2q9(&s->LF);
    make_d2q9(&s->LG);
  } else {
    hydro_lattice(3, p->hydro_q, &s->LF);
    make_d3q7(&s->LG);
  }
  long N = s->N;
  s->f = dalloc(N * s->LF.q);
  s->f2 = dalloc(N * s->LF.q);
  s->g = dalloc(N * s->LG.q);
  s->g2 = dalloc(N * s->LG.q);
  s->phi = dalloc(N);
  s->phi2 = dalloc(N);
  s->acomp = dalloc(3 * N);
  s->grad = dalloc(3 * N);
  s->lap = dalloc(N);
  s->nrm = dalloc(3 * N);
  s->q = dalloc(N);
  s->mu = dalloc(N);
  s->J = dalloc(3 * N);
  s->chi = (int*)calloc((size_t)N, sizeof(int));
  s->partner = (int*)calloc((size_t)(3 * N), sizeof(int));
  s->pstar = dalloc(N);
  s->rho = dalloc(N);
  s->u = dalloc(3 * N);
  s->F = dalloc(3 * N);
  s->omega = dalloc(N);
  s->nu = dalloc(N);
  if (!s->f || !s->f2 || !s->g || !s->g2 || !s->phi || !s->phi2 || !s->acomp || !s->grad || !s->lap ||
      !s->nrm || !s->q ||
      !s->mu || !s->J || !s->chi || !s->partner || !s->pstar || !s->rho || !s->u || !s->F ||
      !s->omega || !s->nu) {
    oracle_destroy(s);
    return NULL;
  }
  /* Mixture parameters (Sec. 2.1 "Mixture properties"): rho_l = 1 in the phi = 1 phase,
   * nu = cs^2 (tau - 1/2) (Eq. nuomega) for the liquid, nu_g = visc_ratio nu_l. */
  s->rho_l = 1.0;
  s->rho_g = 1.0 / p->density_ratio;
  s->nu_l = s->LF.cs2 * (p->tau - 0.5);
  s->nu_g = p->visc_ratio * s->nu_l;
  return s;
}

void oracle_destroy(oracle_state* s) {
  if (!s) return;
  free(s->f); free(s->f2); free(s->g); free(s->g2);
  free(s->phi); free(s->phi2); free(s->acomp);
  free(s->grad); free(s->lap); free(s->nrm); free(s->q); free(s->mu);
  free(s->J); free(s->chi); free(s->partner);
  free(s->pstar); free(s->rho); free(s->u); free(s->F); free(s->omega); free(s->nu);
  free(s);
}

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

static long nb(const oracle_state* s, long idx, const int* c) {
  long x = idx % s->nx, y = (idx / s->nx) % s->ny, z = idx / (s->nx * s->ny);
  return wrapi(x + c[0], s->nx) + s->nx * (wrapi(y + c[1], s->ny) + s->ny * wrapi(z + c[2], s->nz));
}

/* Step 1: phi = sum_i g_i (lattice Boltzmann phase field; with the finite-
 * difference solver phi is itself the stored field and is left as it is). */
static void compute_phi(oracle_state* s) {
  if (s->P.cac_solver != 0) return;
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < s->N; ++idx) {
    double a = 0.0;
    for (int i = 0; i < s->LG.q; ++i) a += s->g[idx * s->LG.q + i];
    s->phi[idx] = a;
  }
}

/* Step 2: isotropic gradient and Laplacian (Eqs. grad_iso, lap_iso), normal, indicator, mu_phi. */
static void compute_gradients(oracle_state* s) {
  const lattice* L = &s->LF;
  const int D = s->D;
  const long N = s->N;
  const double W = s->P.width, sigma = s->P.sigma;
  const double beta = 12.0 * sigma / W, kappa = 1.5 * sigma * W;
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < N; ++idx) {
    double gr[3] = {0, 0, 0}, sum_nb = 0.0;
    for (int i = 0; i < L->q; ++i) {
      double ph = s->phi[nb(s, idx, L->c[i])];
      for (int a = 0; a < D; ++a) gr[a] += L->w[i] * ph * L->c[i][a];
      if (!(L->c[i][0] == 0 && L->c[i][1] == 0 && L->c[i][2] == 0)) sum_nb += L->w[i] * ph;
    }
    double w0 = 0.0;
    for (int i = 0; i < L->q; ++i)
      if (L->c[i][0] == 0 && L->c[i][1] == 0 && L->c[i][2] == 0) w0 = L->w[i];
    double ph = s->phi[idx];
    double lap = 2.0 / L->cs2 * (sum_nb - (1.0 - w0) * ph);
    double mag = 0.0;
    for (int a = 0; a < D; ++a) {
      gr[a] /= L->cs2;
      mag += gr[a] * gr[a];
    }
    mag = sqrt(mag);
    for (int a = 0; a < D; ++a) {
      s->grad[a * N + idx] = gr[a];
      s->nrm[a * N + idx] = gr[a] / (mag + s->P.eps_n);
    }
    s->lap[idx] = lap;
    double pc = ph < 0.0 ? 0.0 : (ph > 1.0 ? 1.0 : ph);
    s->q[idx] = pc * (1.0 - pc);
    s->mu[idx] = 4.0 * beta * ph * (ph - 1.0) * (ph - 0.5) - kappa * lap;
  }
}

/* Step 4: macroscopic fields and the force split of Eq. Fsplit.
 * F' = F_sigma + F_p + F_rep + F_ext, u' = m + F'/(2 rho);
 * F_nu from the second moment of (f - feq(p*, u'));  F = F' + F_nu;  u = m + F/(2 rho). */
static void compute_macro(oracle_state* s) {
  const lattice* L = &s->LF;
  const int D = s->D, Q = L->q;
  const long N = s->N;
  const double cs2 = L->cs2;
  const double drho = s->rho_l - s->rho_g;
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < N; ++idx) {
    const double* f = &s->f[idx * Q];
    double ph = s->phi[idx];
    double rho = s->rho_g + drho * ph;                                     /* linear mixture rule */
    double mu_dyn = s->rho_g * s->nu_g + (s->rho_l * s->nu_l - s->rho_g * s->nu_g) * ph; /* Eq. mu_mix_linear */
    double nu = mu_dyn / rho;                                              /* Eq. nu_from_mu */
    double omega = 1.0 / (0.5 + nu / cs2);                                 /* Eq. omega_phi */
    double pstar = 0.0, m[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      pstar += f[i];                                                       /* Eq. pstar_moment */
      for (int a = 0; a < D; ++a) m[a] += f[i] * L->c[i][a];
    }
    double Fp[3] = {0, 0, 0}, up[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
      double gphi = s->grad[a * N + idx];
      double grho = drho * gphi;
      Fp[a] = s->mu[idx] * gphi                                            /* Eq. Fcap */
              - pstar * cs2 * grho                                         /* Eq. Fp */
              + rho * s->J[a * N + idx]                                    /* Eq. Frep_impl */
              + (rho - s->rho_mean) * s->P.body_force[a];                  /* external body force */
      up[a] = m[a] + Fp[a] / (2.0 * rho);
    }
    /* Eq. Fnu: -(nu omega / cs^2) [sum_i (f_i - feq_i) c_i c_i] . grad rho */
    double Pi[3][3] = {{0}};
    for (int i = 0; i < Q; ++i) {
      double d = f[i] - feq_i(L, D, i, pstar, up);
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) Pi[a][b] += d * L->c[i][a] * L->c[i][b];
    }
    for (int a = 0; a < D; ++a) {
      double fnu = 0.0;
      for (int b = 0; b < D; ++b) fnu += Pi[a][b] * drho * s->grad[b * N + idx];
      fnu *= -(nu * omega / cs2);
      double Ft = Fp[a] + fnu;
      s->F[a * N + idx] = Ft;
      s->u[a * N + idx] = m[a] + Ft / (2.0 * rho);                         /* Eq. u_moment */
    }
    s->pstar[idx] = pstar;
    s->rho[idx] = rho;
    s->omega[idx] = omega;
    s->nu[idx] = nu;
  }
}

static void compute_fields(oracle_state* s) {
  compute_phi(s);
  compute_gradients(s);
  oracle_nci_from_qn(&s->P, s->q, s->nrm, s->chi, s->partner, s->J);
  compute_macro(s);
}

/* Step 5: collisions and push streaming.
 * Hydrodynamics: f*_i = feq_i + (1 - omega) R_i[fneq] + S_i / 2 with fneq = f - feq + S/2;
 * with R = identity this is exactly Eq. lbe.
 * Phase field (CAC lattice Boltzmann): geq_i = w_i [phi + c_i . j / cs^2],
 * j = phi u + M (4/W) phi (1 - phi) n  (Eqs. cace_conservative, kappa_delta),
 * g*_i = g_i - (g_i - geq_i) / tau_phi, tau_phi = 1/2 + M / cs^2. */
static void collide_and_push(oracle_state* s) {
  const lattice* L = &s->LF;
  const lattice* G = &s->LG;
  const int D = s->D, Q = L->q, QG = G->q;
  const long N = s->N;
  const double M = s->P.mobility, W = s->P.width;
  const double tau_phi = 0.5 + M / G->cs2;
  const double comp = s->P.cac_compress ? 1.0 : 0.0;
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < N; ++idx) {
    const double* f = &s->f[idx * Q];
    const double* g = &s->g[idx * QG];
    double u[3] = {0, 0, 0}, F[3] = {0, 0, 0}, nv[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
      u[a] = s->u[a * N + idx];
      F[a] = s->F[a * N + idx];
      nv[a] = s->nrm[a * N + idx];
    }
    double pstar = s->pstar[idx], rho = s->rho[idx], omega = s->omega[idx];
    double feq[27], S[27], fneq[27], R[27];
    for (int i = 0; i < Q; ++i) {
      feq[i] = feq_i(L, D, i, pstar, u);
      S[i] = guo_i(L, D, i, u, F, rho);
      fneq[i] = f[i] - feq[i] + 0.5 * S[i];
    }
    regularize(L, D, fneq, u, R);
    for (int i = 0; i < Q; ++i) {
      double post = feq[i] + (1.0 - omega) * R[i] + 0.5 * S[i];
      s->f2[nb(s, idx, L->c[i]) * Q + i] = post;
    }
    if (s->P.cac_solver != 0) continue;   /* MUSCL mode: no phase-field populations */
    double ph = s->phi[idx];
    double j[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) j[a] = ph * u[a] + comp * M * (4.0 / W) * ph * (1.0 - ph) * nv[a];
    for (int i = 0; i < QG; ++i) {
      double cj = 0.0;
      for (int a = 0; a < D; ++a) cj += G->c[i][a] * j[a];
      double geq = G->w[i] * (ph + cj / G->cs2);
      double post = g[i] - (g[i] - geq) / tau_phi;
      s->g2[nb(s, idx, G->c[i]) * QG + i] = post;
    }
  }
  double* t = s->f;
  s->f = s->f2;
  s->f2 = t;
  t = s->g;
  s->g = s->g2;
  s->g2 = t;
}

/* Test knob (not part of the method): round the stored populations after each
 * step to a narrower format, to measure how the method amplifies storage
 * rounding.  mode 1: float32; 2: IEEE half; 3: bfloat16 (f only for 2 and 3;
 * g stays float32 there).  Round to nearest even in every case. */
static double round_to(double v, int mode) {
  if (mode == 1) return (double)(float)v;
  if (mode == 2) {
    /* IEEE binary16: 11 significant bits, smallest normal 2^-14, subnormal
     * spacing 2^-24; nearbyint rounds half to even. */
    if (v == 0.0 || !isfinite(v)) return v;
    int E;
    double a = fabs(v);
    frexp(a, &E); /* a in [2^(E-1), 2^E) */
    int ue = E - 11;
    if (ue < -24) ue = -24;
    double r = ldexp(nearbyint(ldexp(a, -ue)), ue);
    if (r > 65504.0) r = INFINITY;
    return v < 0 ? -r : r;
  }
  if (mode == 3) {
    float f = (float)v;
    unsigned int b;
    memcpy(&b, &f, 4);
    unsigned int lsb = (b >> 16) & 1u;
    b = (b + 0x7fffu + lsb) & 0xffff0000u;
    memcpy(&f, &b, 4);
    return (double)f;
  }
  return v;
}

static void round_storage(oracle_state* s) {
  const int mode = s->P.store_round;
  if (mode <= 0) return;
  const long nf = s->N * s->LF.q, ng = s->N * s->LG.q;
  for (long i = 0; i < nf; ++i) s->f[i] = round_to(s->f[i], mode);
  for (long i = 0; i < ng; ++i) s->g[i] = round_to(s->g[i], 1);
  if (s->P.cac_solver != 0)   /* MUSCL mode: the stored phase field is the phi array */
    for (long i = 0; i < s->N; ++i) s->phi[i] = round_to(s->phi[i], 1);
}

/* Eq. minmod */
static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return (a > 0.0 ? 1.0 : -1.0) * (fabs(a) < fabs(b) ? fabs(a) : fabs(b));
}

/* Advective flux through the face between cell c0 and its neighbour c1 = c0 + e_ax
 * (Eqs. face_flux_def, slope_minmod_x, recon_lr_x, upwind_select_x): face velocity
 * the mean of the two cells' velocities, phi from the limited linear reconstruction
 * on the upwind side. */
static double face_flux(const oracle_state* s, long c0, int ax) {
  int e[3] = {0, 0, 0};
  e[ax] = 1;
  int me[3] = {0, 0, 0};
  me[ax] = -1;
  const long N = s->N;
  const long c1 = nb(s, c0, e);
  const long cm = nb(s, c0, me);
  const long c2 = nb(s, c1, e);
  const double* p = s->phi;
  const double uf = 0.5 * (s->u[ax * N + c0] + s->u[ax * N + c1]);
  const double s0 = minmod(p[c0] - p[cm], p[c1] - p[c0]);
  const double s1 = minmod(p[c1] - p[c0], p[c2] - p[c1]);
  const double phL = p[c0] + 0.5 * s0;
  const double phR = p[c1] - 0.5 * s1;
  return uf * (uf >= 0.0 ? phL : phR);
}

/* One explicit step of the conservative Allen-Cahn equation by finite differences
 * (Sec. 2.1.1, Eq. phi_update_muscl), every term from time level n:
 *   phi' = phi - div_h(u phi) + D lap_h(phi) + S_comp,
 * div_h(u phi) from the face fluxes above (Eq. divF), D = M, lap_h the isotropic
 * lattice Laplacian (Eq. lap_iso), and S_comp = -kappa div_iso(phi (1 - phi) n) with
 * kappa = 4 M / W (Eq. kappa_delta) and div_iso(a) = (1/cs^2) sum_i w_i c_i . a(x + c_i)
 * the isotropic divergence on the hydrodynamic lattice (Eq. source_sharp). */
static void muscl_update(oracle_state* s) {
  const lattice* L = &s->LF;
  const int D = s->D;
  const long N = s->N;
  const double M = s->P.mobility, W = s->P.width;
  const double kappa = (s->P.cac_compress ? 1.0 : 0.0) * 4.0 * M / W;
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < N; ++idx) {
    const double ph = s->phi[idx];
    for (int a = 0; a < D; ++a) s->acomp[a * N + idx] = ph * (1.0 - ph) * s->nrm[a * N + idx];
  }
#pragma omp parallel for schedule(static)
  for (long idx = 0; idx < N; ++idx) {
    double div = 0.0;
    for (int ax = 0; ax < D; ++ax) {
      int me[3] = {0, 0, 0};
      me[ax] = -1;
      div += face_flux(s, idx, ax) - face_flux(s, nb(s, idx, me), ax);
    }
    double divc = 0.0;
    for (int i = 0; i < L->q; ++i) {
      const long y = nb(s, idx, L->c[i]);
      for (int a = 0; a < D; ++a) divc += L->w[i] * L->c[i][a] * s->acomp[a * N + y];
    }
    divc /= L->cs2;
    s->phi2[idx] = s->phi[idx] - div + M * s->lap[idx] - kappa * divc;
  }
  double* t = s->phi;
  s->phi = s->phi2;
  s->phi2 = t;
}

int oracle_step(oracle_state* s, int n) {
  if (!s || n < 0) return -1;
  for (int k = 0; k < n; ++k) {
    compute_fields(s);
    collide_and_push(s);
    if (s->P.cac_solver != 0) muscl_update(s);
    round_storage(s);
    s->step++;
  }
  return 0;
}

long oracle_step_count(const oracle_state* s) { return s->step; }

static void set_rho_mean(oracle_state* s) {
  double acc = 0.0;
  for (long idx = 0; idx < s->N; ++idx) acc += s->phi[idx];
  double mean_phi = acc / (double)s->N;
  s->rho_mean = s->rho_g + (s->rho_l - s->rho_g) * mean_phi;
  if (s->P.dispersed == 0 || s->P.dispersed == 1) s->dispersed = s->P.dispersed;
  else s->dispersed = (mean_phi < 0.5) ? 1 : 0;
}

/* Initial populations: f = feq(p*, u), g = geq(phi, u, n) with n from the given phi. */
int oracle_init_fields(oracle_state* s, const double* phi, const double* u, const double* pstar) {
  if (!s || !phi) return -1;
  const int D = s->D, Q = s->LF.q, QG = s->LG.q;
  const long N = s->N;
  memcpy(s->phi, phi, sizeof(double) * N);
  compute_gradients(s);
  const double M = s->P.mobility, W = s->P.width;
  const double comp = s->P.cac_compress ? 1.0 : 0.0;
  for (long idx = 0; idx < N; ++idx) {
    double uu[3] = {0, 0, 0};
    if (u)
      for (int a = 0; a < D; ++a) uu[a] = u[a * N + idx];
    double ps = pstar ? pstar[idx] : 0.0;
    for (int i = 0; i < Q; ++i) s->f[idx * Q + i] = feq_i(&s->LF, D, i, ps, uu);
    double ph = phi[idx];
    double j[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a)
      j[a] = ph * uu[a] + comp * M * (4.0 / W) * ph * (1.0 - ph) * s->nrm[a * N + idx];
    for (int i = 0; i < QG; ++i) {
      double cj = 0.0;
      for (int a = 0; a < D; ++a) cj += s->LG.c[i][a] * j[a];
      s->g[idx * QG + i] = s->LG.w[i] * (ph + cj / s->LG.cs2);
    }
  }
  set_rho_mean(s);
  round_storage(s);
  s->step = 0;
  return 0;
}

int oracle_set_populations(oracle_state* s, const double* f, const double* g) {
  const long N = s->N;
  const int Q = s->LF.q, QG = s->LG.q;
  for (long idx = 0; idx < N; ++idx) {
    for (int i = 0; i < Q; ++i) s->f[idx * Q + i] = f[(long)i * N + idx];
    for (int i = 0; i < QG; ++i) s->g[idx * QG + i] = g[(long)i * N + idx];
  }
  compute_phi(s);
  set_rho_mean(s);
  return 0;
}

/* Test knob: the reference density of the buoyancy force, F_ext = (rho - rho_mean) g,
 * is the box mean at initialisation; a sub-box cut from a larger periodic box takes
 * the larger box's value instead. */
int oracle_set_phi(oracle_state* s, const double* phi) {
  if (!s || !phi || s->P.cac_solver == 0) return -1;   /* phi is state only in MUSCL mode */
  for (long idx = 0; idx < s->N; ++idx) s->phi[idx] = phi[idx];
  return 0;
}

int oracle_set_rho_mean(oracle_state* s, double rho_mean) {
  if (!s) return -1;
  s->rho_mean = rho_mean;
  return 0;
}

int oracle_get_populations(const oracle_state* s, double* f, double* g) {
  const long N = s->N;
  const int Q = s->LF.q, QG = s->LG.q;
  for (long idx = 0; idx < N; ++idx) {
    if (f)
      for (int i = 0; i < Q; ++i) f[(long)i * N + idx] = s->f[idx * Q + i];
    if (g)
      for (int i = 0; i < QG; ++i) g[(long)i * N + idx] = s->g[idx * QG + i];
  }
  return 0;
}

int oracle_get_phi(oracle_state* s, double* out) {
  compute_phi(s);
  memcpy(out, s->phi, sizeof(double) * s->N);
  return 0;
}

int oracle_get_rho(oracle_state* s, double* out) {
  compute_fields(s);
  memcpy(out, s->rho, sizeof(double) * s->N);
  return 0;
}

int oracle_get_pstar(oracle_state* s, double* out) {
  compute_fields(s);
  memcpy(out, s->pstar, sizeof(double) * s->N);
  return 0;
}

int oracle_get_u(oracle_state* s, double* out) {
  compute_fields(s);
  memcpy(out, s->u, sizeof(double) * s->D * s->N);
  return 0;
}

int oracle_get_force(oracle_state* s, double* out) {
  compute_fields(s);
  memcpy(out, s->F, sizeof(double) * s->D * s->N);
  return 0;
}

int oracle_get_gradients(oracle_state* s, double* grad, double* lap, double* nrm, double* q,
                         double* mu) {
  compute_phi(s);
  compute_gradients(s);
  if (grad) memcpy(grad, s->grad, sizeof(double) * s->D * s->N);
  if (lap) memcpy(lap, s->lap, sizeof(double) * s->N);
  if (nrm) memcpy(nrm, s->nrm, sizeof(double) * s->D * s->N);
  if (q) memcpy(q, s->q, sizeof(double) * s->N);
  if (mu) memcpy(mu, s->mu, sizeof(double) * s->N);
  return 0;
}

int oracle_get_nci(oracle_state* s, int* chi, int* partner, double* J) {
  compute_fields(s);
  if (chi) memcpy(chi, s->chi, sizeof(int) * s->N);
  if (partner) memcpy(partner, s->partner, sizeof(int) * 3 * s->N);
  if (J) memcpy(J, s->J, sizeof(double) * s->D * s->N);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Diagnostics                                                                */
/* ------------------------------------------------------------------------- */

/* Breadth-first flood fill of the dispersed set with 8- (2D) or 26- (3D)
 * connectivity on the periodic lattice. */
/* Breadth-first search over the dispersed set; sizes[k] (when given, up to
 * max entries) receives the cell count of the k-th component found. */
long oracle_component_sizes(int dim, int nx, int ny, int nz, const double* phi, int dispersed, long* sizes,
                            long max) {
  long NZ = (dim == 2) ? 1 : nz;
  long N = (long)nx * ny * NZ;
  unsigned char* mark = (unsigned char*)calloc((size_t)N, 1);
  long* queue = (long*)malloc(sizeof(long) * (size_t)N);
  long count = 0;
  for (long start = 0; start < N; ++start) {
    int in = dispersed ? (phi[start] > 0.5) : (phi[start] < 0.5);
    if (!in || mark[start]) continue;
    ++count;
    long head = 0, tail = 0;
    queue[tail++] = start;
    mark[start] = 1;
    while (head < tail) {
      long c = queue[head++];
      long x = c % nx, y = (c / nx) % ny, z = c / ((long)nx * ny);
      int dzr = (dim == 2) ? 0 : 1;
      for (int dz = -dzr; dz <= dzr; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            long j = wrapi(x + dx, nx) + nx * (wrapi(y + dy, ny) + (long)ny * wrapi(z + dz, NZ));
            if (mark[j]) continue;
            int jin = dispersed ? (phi[j] > 0.5) : (phi[j] < 0.5);
            if (!jin) continue;
            mark[j] = 1;
            queue[tail++] = j;
          }
    }
    if (sizes && count <= max) sizes[count - 1] = tail;
  }
  free(mark);
  free(queue);
  return count;
}

long oracle_count_components(int dim, int nx, int ny, int nz, const double* phi, int dispersed) {
  return oracle_component_sizes(dim, nx, ny, nz, phi, dispersed, NULL, 0);
}

int oracle_diagnostics(oracle_state* s, oracle_diag* out) {
  compute_fields(s);
  const long N = s->N;
  const int D = s->D;
  memset(out, 0, sizeof(*out));
  out->step = s->step;
  out->finite = 1;
  for (long idx = 0; idx < N; ++idx) {
    double rho = s->rho[idx], sp = 0.0;
    out->mass_phi += s->phi[idx];
    out->sum_pstar += s->pstar[idx];
    for (int a = 0; a < D; ++a) {
      double ua = s->u[a * N + idx];
      out->momentum[a] += rho * ua;
      sp += ua * ua;
    }
    out->kinetic_energy += 0.5 * rho * sp;
    sp = sqrt(sp);
    if (sp > out->max_speed) out->max_speed = sp;
    out->nci_active += s->chi[idx];
    if (!isfinite(s->phi[idx]) || !isfinite(sp) || !isfinite(s->pstar[idx])) out->finite = 0;
    /* film diagnostics of Sec. 3.3 (Eq. RnAbs): F_rep = rho J (Eq. Frep_impl),
     * F_cap = mu grad phi (Eq. Fcap), n = grad phi / (|grad phi| + eps_n) */
    double frep2 = 0.0, frep_n = 0.0, fcap_n = 0.0;
    for (int a = 0; a < D; ++a) {
      const double fr = rho * s->J[a * N + idx];
      const double fc = s->mu[idx] * s->grad[a * N + idx];
      const double na = s->nrm[a * N + idx];
      frep2 += fr * fr;
      frep_n += fr * na;
      fcap_n += fc * na;
    }
    const double frep = sqrt(frep2);
    if (frep > out->max_frep) out->max_frep = frep;
    if (s->chi[idx]) {
      out->film_frep_n += fabs(frep_n);
      out->film_fcap_n += fabs(fcap_n);
      out->film_frep += frep;
    }
  }
  out->n_droplets = oracle_count_components(D, (int)s->nx, (int)s->ny, (int)s->nz, s->phi, s->dispersed);
  return 0;
}
