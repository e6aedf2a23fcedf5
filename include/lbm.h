/*
 * lbm.h -- C ABI of the MI355X (gfx950) coupled lattice step.
 *
 * One time step couples three pieces of arXiv:2603.17481 ("Adaptive
 * near-contact repulsion in conservative Allen-Cahn phase-field lattice
 * Boltzmann multiphase model"):
 *   - recursive-regularised lattice Boltzmann hydrodynamics with a third-order
 *     equilibrium and Guo forcing in the velocity / p* formulation
 *     (Sec. 2.1: Eqs. lbe, nuomega, pstar, pstar_moment, u_moment,
 *     mu_mix_linear, nu_from_mu, omega_phi, feq3, H2, H3, fneq3, A3rec, guo,
 *     Fsplit, Fcap, Fp, Fnu, grad_iso, lap_iso), on D2Q9 (2D) or D3Q19 (3D);
 *   - the conservative Allen-Cahn equation (Sec. 2.1.1, Eqs. cace,
 *     cace_conservative, normal, kappa_delta) advanced by a lattice Boltzmann
 *     equation on D2Q9 (2D) or D3Q7 (3D) whose equilibrium carries the
 *     counter-gradient flux M (4/W) phi (1 - phi) n in its first moment;
 *   - the near-contact repulsion: interfacial gate, windowed partner search
 *     and the closed-form film-thickness weight (Sec. 2.2, Sec. 2.3: Eqs.
 *     n_discrete, q_discrete, q_gate, window, q_similarity, facing_threshold,
 *     facing_score, mask_partner_def, qpair_impl, q_clamp, face_impl,
 *     nsym_impl, h_impl, wh_impl, Jrep_impl, Frep_impl).
 *
 * Conventions for every entry point:
 *   - Cells are indexed idx = x + nx * (y + ny * z); the box is periodic in
 *     every direction; in 2D nz = 1.  Node i sits at coordinate i.
 *   - Host arrays are owned by the caller, are always double precision
 *     whatever the compute precision, and are copied synchronously.
 *     Vector fields are structure-of-arrays: component a of cell idx at
 *     [a * N + idx].
 *   - Every call returns an LBM_* code; the message of the last failure of a
 *     context is returned by lbm_last_error(ctx) (lbm_last_error(NULL) for a
 *     failed lbm_create).  Nothing throws across the ABI and nothing aborts.
 *   - A context is bound to the HIP device that was current at lbm_create and
 *     to one stream; it is not thread-safe.  Separate contexts are independent.
 *   - The library needs a gfx950 device; it never falls back to the CPU.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_E_INVALID = -1,     /* bad argument or parameter                         */
  LBM_E_OOM = -2,         /* device allocation failed / workspace too small    */
  LBM_E_HIP = -3,         /* HIP runtime error                                 */
  LBM_E_UNSUPPORTED = -4, /* combination not built                             */
  LBM_E_DIVERGED = -5,    /* non-finite value seen by a periodic diagnostic    */
  LBM_E_STATE = -6        /* call out of order (e.g. step before init)         */
};

/* Storage / arithmetic of the populations.  FP16 and BF16 store the
 * hydrodynamic populations as d_i = f_i - w_i pstar_ref in 16 bits and do all
 * arithmetic in FP32; the phase-field populations stay FP32. */
enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP32_F16STORE = 2, LBM_FP32_BF16STORE = 3 };

typedef struct {
  int dim, nx, ny, nz;       /* dim 2 => nz must be 1                                      */
  int precision;             /* LBM_FP64 ... LBM_FP32_BF16STORE                            */
  double tau;                /* liquid relaxation time: nu_l = cs^2 (tau - 1/2), Eq. nuomega */
  double visc_ratio;         /* nu_g / nu_l (kinematic)                                     */
  double mobility;           /* M = D of Eq. cace; tau_phi = 1/2 + M / cs_phi^2             */
  double width;              /* W = epsilon = delta, interface thickness                    */
  double sigma;              /* surface tension                                             */
  double density_ratio;      /* rho_l / rho_g with rho_l = 1 (phi = 1 phase)                */
  double a_rep;              /* A_rep of Eq. Jrep_impl; 0 turns the near-contact force off  */
  double body_force[3];      /* g; F_ext = (rho - <rho>) g, <rho> the box mean              */
  int nci_window;            /* w of Eq. window (1, 2 or 3)                                 */
  double q_th, eta, cos_opp; /* Eqs. q_gate, q_similarity, facing_threshold                 */
  double h0, p_exp;          /* w_h = 1 / (1 + (h/h0)^p), Eq. wh_general                    */
  double eps_n, eps_q;       /* regularisations of Eqs. n_discrete, q_similarity, q_clamp   */
  double tie_eps;            /* partner choice: among candidates at the smallest |r|^2,
                                facing scores within tie_eps of the best are tied and the
                                first in scan order (dz, dy, dx from -w) wins              */
  int rep_orient;            /* n_sym orientation: 0 along n(x) (planar-limit form of
                                Sec. 2.2.5), +1 toward the partner, -1 away from it         */
  int dispersed;             /* droplet count of {phi > 1/2} (1) or {phi < 1/2} (0);
                                -1 picks the minority phase at initialisation              */
  int cac_compress;          /* 1: counter-gradient flux on; 0: off (pure diffusion)        */
  int diag_interval;         /* K > 0: on-device diagnostics every K steps inside lbm_step  */
  double pstar_ref;          /* reference p* of the 16-bit population encoding              */
  int cac_solver;            /* phase-field solver: 0 the lattice Boltzmann scheme of
                                Sec. 2.1.2 (populations g, D2Q9 / D3Q7); 1 the explicit
                                finite-difference scheme of Sec. 2.1.1 (Eq.
                                phi_update_muscl: MUSCL reconstruction with the minmod
                                limiter, upwind face fluxes, isotropic Laplacian and
                                sharpening divergence), phi stored and double-buffered.
                                Not supported by lbm_batch_step.                        */
  int hydro_q;               /* 3D hydrodynamic lattice: 0 or 19 D3Q19, 27 D3Q27 (the
                                paper's lattice, Sec. 2.1; also the weights of the
                                isotropic gradient, Laplacian and divergence stencils).
                                2D: 0 or 9 (D2Q9).                                      */
  int hydro_store;           /* storage of the hydrodynamic populations: 0 the Q
                                populations in place (AA pattern); 1 the paper's
                                "thread-safe" update (Sec. 2.1, Eqs. fneq3, A3rec): each
                                cell keeps the 13 coefficients of its post-collision
                                populations (p*, u, F/(2 rho), (1 - omega) A2) in one of
                                two buffers, and the next step rebuilds each incoming
                                population from the coefficients of the cell it streams
                                from.  dim 3, FP64 or FP32, cac_solver 0 only
                                (LBM_E_UNSUPPORTED otherwise); lbm_set_populations and
                                lbm_batch_step return LBM_E_UNSUPPORTED.  Initial state:
                                the coefficients (p*, u, 0, 0), so the first incoming
                                populations of a cell are the equilibria of the cells
                                they stream from.                                        */
} lbm_params;

typedef struct {
  long step;                 /* state the numbers describe                                  */
  double mass_phi;           /* sum phi (FP64 accumulation)                                 */
  double sum_pstar;          /* sum p*                                                      */
  double momentum[3];        /* sum rho u                                                   */
  double kinetic_energy;     /* sum rho |u|^2 / 2                                           */
  double max_speed;          /* max |u|                                                     */
  long n_droplets;           /* connected components of the dispersed set {phi > 1/2}
                                (droplets) or {phi < 1/2} (bubbles), 8-/26-connected on
                                the periodic lattice, by union-find on the device       */
  long nci_active;           /* number of cells with chi_nc = 1                             */
  int finite;                /* 1 if every p*, u and phi is finite                          */
  /* Sec. 3.3 (self-tuning of the repulsion): sums over the film region (cells
   * with a partner, F_rep != 0) of |F_rep . n| and |F_cap . n| (numerator and
   * denominator of Eq. RnAbs) and of |F_rep|, with F_rep = rho J, F_cap =
   * mu_phi grad phi, n = grad phi / (|grad phi| + eps_n); the film volume in
   * cells; the largest |F_rep|.  R_n = film_frep_n / film_fcap_n and
   * <|F_rep|>_film = film_frep / film_cells.  Accumulated in FP64.             */
  double film_cells;
  double film_frep_n;
  double film_fcap_n;
  double film_frep;
  double max_frep;
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* Fill *p with the defaults: 2D 128x128 FP64, tau 1, M 0.1, W 4, sigma 1e-3,
 * density ratio 1, A_rep 1e-3 and the detection parameters of Sec. 2.3.2
 * (w 3, q_th 0.125, eta 0.1, cos_opp -0.8) and Sec. 2.3.3 (h0 1, p 4). */
void lbm_default_params(lbm_params* p);

/* Bytes of device workspace a context with these parameters needs (all state
 * that stays resident: populations, phi, the repulsive flux, tile lists,
 * reduction scratch).  0 if the parameters are invalid. */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Create a context on the current HIP device.  dev_workspace: NULL lets the
 * library allocate; otherwise a device pointer of at least
 * lbm_workspace_bytes(p) bytes, 256-byte aligned, that the caller keeps alive
 * until lbm_destroy (e.g. a torch tensor).  hip_stream: a hipStream_t, or
 * NULL for a stream the library creates.  Returns LBM_E_INVALID,
 * LBM_E_OOM or LBM_E_HIP on failure, with *out = NULL. */
int lbm_create(const lbm_params* p, void* dev_workspace, size_t ws_bytes, void* hip_stream,
               lbm_ctx** out);
void lbm_destroy(lbm_ctx* ctx);
const char* lbm_last_error(const lbm_ctx* ctx);

/* Initial state: f = feq(p*, u) (Eq. feq3), g = geq(phi, u, n).  phi: N
 * doubles; u: dim*N (NULL = at rest); pstar: N (NULL = pstar_ref).  Resets the
 * step count to 0.  Synchronous. */
int lbm_init_fields(lbm_ctx* ctx, const double* phi, const double* u, const double* pstar);

/* Enqueue n coupled steps on the context's stream (asynchronous). */
int lbm_step(lbm_ctx* ctx, int n);
/* Wait for the stream; LBM_E_DIVERGED if a periodic diagnostic saw a
 * non-finite value since the last lbm_init_fields / lbm_load_state. */
int lbm_sync(lbm_ctx* ctx);
long lbm_step_count(const lbm_ctx* ctx);

/* Fields of the current state, recomputed from the populations (synchronous). */
int lbm_get_phi(lbm_ctx* ctx, double* out_N);
int lbm_get_rho(lbm_ctx* ctx, double* out_N);
int lbm_get_pstar(lbm_ctx* ctx, double* out_N);
int lbm_get_u(lbm_ctx* ctx, double* out_dimN);     /* u = m + F / (2 rho), Eq. u_moment */
int lbm_get_force(lbm_ctx* ctx, double* out_dimN); /* total F of Eq. Fsplit            */
/* Near-contact state of the current step: chi (N ints, NULL to skip),
 * partner offsets (3*N ints, SoA dx/dy/dz, NULL to skip) and J_rep (dim*N). */
int lbm_get_nci(lbm_ctx* ctx, int* chi, int* partner, double* J);
/* Diagnostics of the current state (synchronous, FP64). */
int lbm_diagnostics(lbm_ctx* ctx, lbm_diag* out);
/* Diagnostics recorded every diag_interval steps by lbm_step, oldest first;
 * at most max entries (the last 64 are kept).  Returns the count or <0. */
int lbm_diag_history(lbm_ctx* ctx, lbm_diag* out, int max);

/* Swarm statistics of the current state (the curvature and equivalent-diameter
 * PDFs of the bubble-swarm section; not part of the coupled step).  Both
 * synchronise and allocate temporary device memory.
 *
 * lbm_curvature_histogram: the interfacial mean curvature kappa = div n
 * (Eq. kappa_radius; 2/R on a sphere of radius R), n the outward unit normal
 * of the dispersed phase (grad phi / (|grad phi| + eps_n) for bubbles, its
 * negative for droplets) and div the isotropic divergence of the hydrodynamic
 * lattice, at the interface cells q = phi^(1 - phi^) >= q_band (phi^ = phi
 * clamped to [0, 1]; 0 < q_band <= 1/4).  counts (nbins + 2 longs, 1 <= nbins
 * <= 4096): [0] kappa < kmin, [nbins + 1] kappa >= kmax, [1 + b] the b-th of
 * nbins equal bins of [kmin, kmax); the bin is taken in FP64 from kappa.
 *
 * lbm_component_volumes: cell counts of the connected components (8- / 26-
 * connected, periodic) of the dispersed set, largest first; at most max are
 * written to volumes, *count receives the number of components (droplets or
 * bubbles).  Equivalent diameters follow as (6 V / pi)^(1/3) (3D) or
 * (4 V / pi)^(1/2) (2D).  Errors: LBM_E_INVALID, LBM_E_STATE, LBM_E_OOM,
 * LBM_E_HIP. */
int lbm_curvature_histogram(lbm_ctx* ctx, double q_band, double kmin, double kmax, int nbins, long* counts);
int lbm_component_volumes(lbm_ctx* ctx, long* volumes, long max, long* count);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch lbm_step makes (0 phi moment and interface flags, 1
 * near-contact, 2 collide + stream, 3 diagnostics, 4 finite-difference phase
 * field update).  lbm_timing(ctx, 1) starts recording, 0 stops;
 * lbm_kernel_times synchronises, returns the accumulated milliseconds and
 * launch counts since the last call (ms[5], counts[5]) and resets them. */
int lbm_timing(lbm_ctx* ctx, int enable);
int lbm_kernel_times(lbm_ctx* ctx, double* ms, long* counts);

/* Lattice velocity order used by the population calls: which 0 = default
 * hydrodynamic lattice (D2Q9 / D3Q19), 1 = phase-field lattice (D2Q9 / D3Q7),
 * 2 = D3Q27 (dim 3 only); c (may be null) receives 3*q ints (cx, cy, cz per
 * velocity).  Returns q, or LBM_E_INVALID. */
int lbm_lattice(int dim, int which, int* c);
/* Incoming populations of the current state on the periodic box
 * [x0, x0+bx) x [y0, y0+by) x [z0, z0+bz) (wrapped), SoA [q][bz][by][bx]. */
int lbm_get_populations(lbm_ctx* ctx, int x0, int y0, int z0, int bx, int by, int bz,
                        double* f, double* g);
/* Replace the whole state by the given incoming populations (SoA [q][N]); the
 * step count becomes 0.  Synchronous.  LBM_E_UNSUPPORTED with the
 * finite-difference phase field (cac_solver 1), whose state is f and phi; its
 * g, as lbm_get_populations returns them, stay as lbm_init_fields set them. */
int lbm_set_populations(lbm_ctx* ctx, const double* f, const double* g);

/* Raw state (populations in their stored precision and AA layout, step count;
 * with cac_solver 1 also phi) for checkpoint / restart; a restored context
 * continues bit for bit.  The header records a format version, the box, the
 * precision, the hydrodynamic lattice and the phase-field solver:
 * lbm_load_state returns LBM_E_INVALID unless all of them equal the context's
 * and bytes equals lbm_state_bytes(ctx).  lbm_save_state needs at least
 * lbm_state_bytes(ctx) bytes. */
size_t lbm_state_bytes(const lbm_ctx* ctx);
int lbm_save_state(lbm_ctx* ctx, void* host_buf, size_t bytes);
int lbm_load_state(lbm_ctx* ctx, const void* host_buf, size_t bytes);

/* Near-contact tile selection (Sec. 2.3 pruning, exact): before the
 * near-contact pass, tiles whose gated normals cannot face a gated normal
 * within the window are left out.  mode -1 (default): on lattices of at least
 * 16384 near-contact tiles; 0: never; 1: always.  Results do not depend on the
 * mode.  Synchronises the context's stream.  Returns LBM_OK or LBM_E_INVALID /
 * LBM_E_HIP. */
int lbm_nci_select(lbm_ctx* ctx, int mode);

/* Testing hook: on != 0 makes the context's collide launches (k_collide,
 * k_collide_row, and k_collide_multi in every batch that holds the context)
 * use the instantiations that form element offsets in 64 bits, which a box
 * needs once a z plane of populations or a phi plane reaches 4 GiB (e.g. the
 * 1024^3 swarm).  The arithmetic is the same; this lets those kernels be
 * checked on boxes the oracle can step.  Synchronises the context's stream.
 * Returns LBM_OK or LBM_E_INVALID / LBM_E_HIP. */
int lbm_force_wide_offsets(lbm_ctx* ctx, int on);

/* Serving: advance every context by n steps of the coupled update (Sec. 2,
 * the step lbm_step performs) with multi-domain launches that cover all of
 * them at once: one grid spans the blocks of every lattice and each block finds
 * its lattice in a device job table.  Whole groups of 8 steps replay a HIP
 * graph captured on the first call for this ordered set of contexts (cached,
 * at most 8 sets; lbm_destroy drops the sets that hold a context); the
 * remaining n % 8 steps are launched directly.  All contexts must live on the
 * same device, share lattice and precision, be initialised and appear once.
 * Their populations after the call equal bit for bit those of lbm_step on each
 * alone; periodic diagnostics (diag_interval) are not taken inside a batch.
 * Enqueued on the first context's stream after the others' streams have been
 * synchronised; later work on every context's stream waits for it.
 * Asynchronous.  Errors: LBM_E_INVALID for a bad list, LBM_E_STATE for an
 * uninitialised context, LBM_E_OOM / LBM_E_HIP from allocation or launch, with
 * the message on the first context.  Calls on overlapping sets of contexts
 * from several host threads at once are not supported. */
int lbm_batch_step(lbm_ctx* const* ctxs, int count, int n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the steps of
 * lbm_batch_step (same kernels, same results bit for bit, same requirements on
 * the list) with the job table in a fixed device array of the library instead
 * of an allocation, and no graph.  At most 64 contexts per call; a longer list
 * returns LBM_E_INVALID.  Each GPU holds one such table (64 KB) until the
 * process ends, and every call on that GPU rewrites it before its steps read
 * it, so nothing carries over between calls.  The call is synchronous: it
 * returns after the steps have run on the first context's stream, so
 * consecutive calls never share the table; calls from several host threads at
 * once on one GPU race on it and are not supported.  No memory is allocated
 * and no graph is created.  Errors as lbm_batch_step, plus LBM_E_HIP if the
 * table's address cannot be taken. */
int lbm_batch_step_noalloc(lbm_ctx* const* ctxs, int count, int n);

#ifdef __cplusplus
}
#endif
#endif
