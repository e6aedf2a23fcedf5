/*
 * lbm_oracle.h -- CPU FP64 oracle of the coupled lattice step (test infrastructure).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Paper: "Adaptive near-contact repulsion in conservative Allen-Cahn
 * phase-field lattice Boltzmann multiphase model" (arXiv:2603.17481).
 * Section numbers below refer to that paper.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int dim, nx, ny, nz;     /* dim 2 => nz = 1; periodic in every direction            */
  double tau;              /* liquid relaxation time, nu_l = cs^2 (tau - 1/2)           */
  double visc_ratio;       /* nu_g / nu_l (kinematic)                                   */
  double mobility;         /* M, the interface diffusivity D of the CAC equation        */
  double width;            /* W, the interface thickness (epsilon = delta in the paper) */
  double sigma;            /* surface tension                                           */
  double density_ratio;    /* rho_l / rho_g with rho_l = 1                              */
  double a_rep;            /* A_rep; 0 switches the near-contact force off              */
  double body_force[3];    /* g; F_ext = (rho - <rho>) g                                */
  int nci_window;          /* w                                                         */
  double q_th, eta, cos_opp, h0, p_exp, eps_n, eps_q;
  double tie_eps;          /* facing scores within tie_eps of the best count as tied  */
  int rep_orient;          /* 0: along n(x); +1: toward partner; -1: away from partner  */
  int dispersed;           /* 1: droplets {phi>1/2}; 0: bubbles {phi<1/2}; -1: auto     */
  int cac_compress;        /* 1: counter-gradient flux on; 0: off (pure diffusion)       */
  int cac_solver;          /* phase field: 0 conservative Allen-Cahn lattice Boltzmann
                              (g populations); 1 finite-difference MUSCL-TVD update of
                              phi (Sec. 2.1.1, Eq. phi_update_muscl)                   */
  int hydro_q;             /* 3D hydrodynamic lattice: 19 (or 0) D3Q19, 27 D3Q27      */
  int store_round;         /* test knob: 0 none; round stored populations after each
                              step to 1 float32, 2 half (f), 3 bfloat16 (f)            */
} oracle_params;

typedef struct {
  long step;
  double mass_phi, sum_pstar, momentum[3], kinetic_energy, max_speed;
  long n_droplets, nci_active;
  int finite;
  /* Sec. 3.3 (self-tuning of the repulsion), over the film region chi = 1:
   * sums of |F_rep . n|, |F_cap . n| (Eq. RnAbs, numerator and denominator)
   * and |F_rep| with F_rep = rho J, F_cap = mu_phi grad phi, n the unit normal;
   * max_frep = max |F_rep| over all cells. */
  double film_frep_n, film_fcap_n, film_frep, max_frep;
} oracle_diag;

typedef struct oracle_state oracle_state;

/* Lattice tables: kind 0 = D2Q9, 1 = D3Q19, 2 = D3Q7, 3 = D3Q27.  c is q x 3 ints, w is q doubles. */
int oracle_lattice(int kind, int* q, int* c, double* w, double* cs2);

oracle_state* oracle_create(const oracle_params* p);
void oracle_destroy(oracle_state* s);
int oracle_threads(void);
/* OpenMP threads of later calls (n > 0); returns the count now in effect. */
int oracle_set_threads(int n);

/* phi, pstar: N doubles or NULL (pstar NULL => 0); u: dim*N SoA or NULL (=> 0). */
int oracle_init_fields(oracle_state* s, const double* phi, const double* u, const double* pstar);
/* Populations in natural layout (incoming populations at each cell), SoA [q][N]. */
int oracle_set_populations(oracle_state* s, const double* f, const double* g);
/* Test knob: override the reference density rho_mean of F_ext = (rho - rho_mean) g
 * (by default the box mean at initialisation), for a sub-box of a larger box. */
int oracle_set_rho_mean(oracle_state* s, double rho_mean);
/* Test knob for the finite-difference phase field (cac_solver 1), whose state is f and
 * phi: replace phi (N doubles).  -1 for the lattice Boltzmann phase field, where phi is
 * the moment of g. */
int oracle_set_phi(oracle_state* s, const double* phi);
int oracle_get_populations(const oracle_state* s, double* f, double* g);
int oracle_step(oracle_state* s, int n);
long oracle_step_count(const oracle_state* s);

/* Fields of the current state (recomputed from the populations). */
int oracle_get_phi(oracle_state* s, double* out);
int oracle_get_rho(oracle_state* s, double* out);
int oracle_get_pstar(oracle_state* s, double* out);
int oracle_get_u(oracle_state* s, double* out);       /* dim*N SoA */
int oracle_get_force(oracle_state* s, double* out);   /* total F, dim*N SoA */
/* grad phi and n: dim*N SoA; lap phi, q, mu_phi: N (step 2 of the update). */
int oracle_get_gradients(oracle_state* s, double* grad, double* lap, double* nrm, double* q, double* mu);
int oracle_get_nci(oracle_state* s, int* chi, int* partner /* 3*N SoA offsets */, double* J /* dim*N */);
int oracle_diagnostics(oracle_state* s, oracle_diag* out);

/* Stand-alone pieces, exposed so that each can be pinned on its own. */
/* Near-contact detection + force (section 2.3) from given q and n fields (n: dim*N SoA). */
int oracle_nci_from_qn(const oracle_params* p, const double* q, const double* n,
                       int* chi, int* partner, double* J);
/* Third-order equilibrium, Guo source and regularised non-equilibrium of one cell (section 2.1). */
int oracle_feq(int dim, int q, double pstar, const double* u, double* out);
int oracle_guo(int dim, int q, const double* u, const double* F, double rho, double* out);
int oracle_regularize(int dim, int q, const double* fneq, const double* u, double* out);
/* Film-thickness map and thickness weight of section 2.3.3 for one paired indicator. */
double oracle_film_thickness(const oracle_params* p, double q_pair);
double oracle_thickness_weight(const oracle_params* p, double h);
/* Connected components of the dispersed set (8-/26-connectivity, periodic). */
long oracle_count_components(int dim, int nx, int ny, int nz, const double* phi, int dispersed);
/* The same search, also giving the cell count of each component (in the order found, at
 * most max of them). */
long oracle_component_sizes(int dim, int nx, int ny, int nz, const double* phi, int dispersed, long* sizes,
                            long max);

#ifdef __cplusplus
}
#endif
#endif
