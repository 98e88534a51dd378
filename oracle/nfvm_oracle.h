/*
 * Serial FP64 reference ("oracle") for one NeuralFVM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library: every operator is written out again here, in plain
 * loops, from the paper (Sec. 2.1-2.7 and Algorithms 1-4 of the appendix).
 *
 * Arrays are cell-centred, unpadded, C order [nz][ny][nx] (x fastest).
 * In 2D, nz = 1, there are no z faces and w stays zero.
 *
 * Parity status of every function is listed in the design notes; the
 * full turbulent step is "parity unpinned" beyond its parts (no reference
 * field data exists), while its parts are pinned by closed forms in the
 * CPU test-suite.
 */
#ifndef NFVM_ORACLE_H
#define NFVM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_WALL = 0, ORC_INLET = 1, ORC_OUTLET = 2 };
enum { ORC_KOMEGA = 1, ORC_ENERGY = 2, ORC_BUOYANCY = 4 };
enum { ORC_OK = 0, ORC_E_INVAL = -1, ORC_E_DIVERGED = -4, ORC_E_NOTCONV = -5 };

typedef struct {
  int face;          /* 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+ */
  int lo[2], hi[2];  /* tangential half-open cell ranges */
  int kind;          /* ORC_WALL / ORC_INLET / ORC_OUTLET */
  double U[3], T, k, omega, T_wall; /* T_wall NaN = adiabatic */
} orc_patch;

typedef struct {
  int dim, n[3];
  double h[3];
  double nu, alpha_T, Pr_t, sigma_k, sigma_w, dt;
  int physics;
  double gravity[3], T_ref, beta_T, T_solid;
  int n_patches;
  const orc_patch* patches;
  const unsigned char* solid; /* [nz][ny][nx], 1 = solid; may be NULL */
  int n_levels, nu1, nu2;
  double omega_jacobi; /* 0 = 4/5 in 2D, 6/7 in 3D */
  double tol;
  int max_cycles;
  int prolong;         /* 0: linear interpolation (eq. prolongation); 1: nearest
                          (piecewise constant), the plainest reading of the
                          upsampling in Algorithm 1 */
  int rk_order;        /* explicit stage: 1 forward Euler; 2 Heun's method in
                          its strong-stability-preserving form (Sec. 2.6 leaves
                          the Runge-Kutta scheme open) */
  int literal;         /* 1: Algorithm 1 as printed: the residual restricted to
                          every level, one undamped Jacobi sweep per level on the
                          way up with the scalar diagonal 2 sum_d 1/h_d^2 of eq.
                          jacobi_pc (one sweep from zero on the coarsest level),
                          nearest upsampling, one fine sweep, repeated as a plain
                          iteration (no Krylov wrapper); nu1, nu2, omega_jacobi
                          and prolong are then ignored */
  int nu_coarse;       /* pre and post sweeps on the levels below the finest
                          (0: nu1 and nu2 there too); the cycle keeps the
                          V shape of Algorithm 1 (the paper fixes no sweep
                          count) */
} orc_case;

typedef struct { double *u, *v, *w, *p, *T, *k, *omega; } orc_fields;

typedef struct {
  int cycles, status;
  double rel_residual, max_face_div, min_k, min_omega;
} orc_stats;

typedef struct orc_mg orc_mg;

/* closure at one point: out = {alpha*, nu_t, alpha (eq. a), beta*} */
void orc_closure_point(double nu, double k, double omega, double out[4]);
void orc_fixed_omega(const orc_case* c, double* omega);
void orc_nut(const orc_case* c, const double* k, const double* omega, double* nut);
void orc_explicit_rhs(const orc_case* c, const orc_fields* in, orc_fields* rhs);
void orc_explicit(const orc_case* c, const orc_fields* in, orc_fields* out);
void orc_destroy(const orc_case* c, const double* u, const double* v, const double* w,
                 const double* k, const double* omega, double tau, double* k_out,
                 double* omega_out);
void orc_rhs_b(const orc_case* c, const double* us, const double* vs, const double* ws,
               double* b);
void orc_project(const orc_case* c, const double* phi, const double* us, const double* vs,
                 const double* ws, double* p, double* u, double* v, double* w,
                 double* max_face_div);

/* d u_a / d x_b per cell, nine values per cell (row-major); zero on
 * non-fluid cells (post-processing, Sec. 3.2). */
void orc_velocity_gradient(const orc_case* c, const double* u, const double* v,
                           const double* w, double* G9);

/* Boundary classification as tables (see the definition): neighbour index
 * or -1 per cell and face direction, the affine ghost rule of each field,
 * the fixed-omega flag per cell. */
void orc_ghost_table(const orc_case* c, int* nidx, double* a0, double* a1,
                     unsigned char* fixed);

orc_mg* orc_mg_create(const orc_case* c);
void orc_mg_free(orc_mg* mg);
int orc_mg_levels(const orc_mg* mg);
void orc_mg_level_shape(const orc_mg* mg, int l, int n[3], double h[3]);
void orc_mg_level_active(const orc_mg* mg, int l, unsigned char* act);
void orc_mg_apply(const orc_mg* mg, int l, const double* x, double* y);
void orc_mg_smooth(const orc_mg* mg, int l, double* x, const double* b, int sweeps);
void orc_mg_restrict(const orc_mg* mg, int l, const double* r_fine, double* b_coarse);
void orc_mg_prolong_add(const orc_mg* mg, int l, const double* e_coarse, double* x_fine);
void orc_mg_vcycle(const orc_mg* mg, double* x, const double* b);
int orc_mg_solve(const orc_mg* mg, const double* b, double* x, double tol, int max_cycles,
                 int forced_cycles, int* cycles, double* rel_residual);

/* Reverse mode of the pressure step (Sec. 2.4): the map from (u*, p^n) to
 * (u^{n+1}, p^{n+1}) through b = rhs_b(u*), phi = A^-1 b, u = u* - dt
 * grad(phi), p = p^n + phi is affine in u*; its transposed Jacobian applied to
 * the adjoints (ubar, vbar, wbar, pbar) of the outputs gives the adjoint of
 * u* in (usbar, vsbar, wsbar) (that of p^n is pbar itself).  A is symmetric,
 * so A^-T is a second solve with the same multigrid (to tol, or forced
 * cycles); phibar receives A's right-hand side of that solve and lambda its
 * solution when not NULL.  Returns the solve's status. */
int orc_pressure_adjoint(const orc_case* c, const double* ubar, const double* vbar,
                         const double* wbar, const double* pbar, double tol, int max_cycles,
                         int forced_cycles, double* usbar, double* vsbar, double* wsbar,
                         double* phibar, double* lambda, int* cycles, double* rel_residual);

/* warm != 0: each step's pressure solve starts from the previous step's
 * increment (zero at the first step of the call), else from zero. */
int orc_step(const orc_case* c, orc_fields* s, int n_steps, const int* forced_cycles,
             orc_stats* stats, int warm);

#ifdef __cplusplus
}
#endif
#endif
