/*
 * nfvm.h -- C ABI of the MI355X NeuralFVM time-step library (libnfvm.so).
 *
 * The library advances the incompressible RANS equations with the standard
 * k-omega model on a uniform structured grid, as formulated in
 * "NeuralFVM: Neural-physics-based Finite Volume Method for Turbulent Flows
 * Using the k-omega Model" (Xue et al., arXiv 2603.21869):
 *   - explicit first-order-upwind finite-volume update of u, v, w, T, k, omega
 *     (Sec. 2.3; Algorithms 2 and 4; appendix on explicit time stepping),
 *   - semi-implicit destruction of k and omega in two half steps around it
 *     (Sec. 2.5, eqs. k_des_step / o_des_step; Sec. 2.6; Algorithm 3),
 *   - pressure projection with a geometric-multigrid Poisson solve
 *     (Sec. 2.4, eqs. pc_residual to jacobi_pc; Algorithm 1).
 * Every step of the time step runs in HIP kernels built for gfx950.
 *
 * Conventions shared by all entry points:
 *   - Every call returns an nfvm_status; nothing throws across the ABI.  On a
 *     negative status nfvm_last_error() returns a message (thread-local).
 *   - Host arrays are FP64, cell-centred, C order [nz][ny][nx] (x fastest),
 *     nz = 1 in 2D.  The caller owns every host pointer; the library only
 *     reads or writes it during the call.
 *   - Device arrays (the *_device calls) use the same dense layout, in FP64,
 *     and must stay valid until the call returns.
 *   - The library owns all device memory of a grid; nfvm_free_grid releases
 *     it.  Device memory comes from hipMalloc unless nfvm_set_allocator has
 *     installed another allocator (for instance PyTorch's caching allocator).
 *   - Work of a grid is issued on the HIP stream given to nfvm_init_grid
 *     (NULL: a stream the library creates).  A grid handle must not be used
 *     from two threads at once; server calls are thread-safe.
 */
#ifndef NFVM_H
#define NFVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NFVM_OK = 0,
  NFVM_PENDING = 1,       /* nfvm_poll: request not finished yet */
  NFVM_E_INVAL = -1,      /* bad argument or descriptor */
  NFVM_E_NOMEM = -2,      /* device allocation failed or request above the HBM budget */
  NFVM_E_DEVICE = -3,     /* a HIP call failed */
  NFVM_E_DIVERGED = -4,   /* non-finite residual or field */
  NFVM_E_NOTCONV = -5,    /* max_cycles reached before tol; fields stay valid */
  NFVM_E_NOTFOUND = -6    /* unknown ticket */
} nfvm_status;

typedef enum { NFVM_FP64 = 0, NFVM_FP32 = 1, NFVM_MIXED = 2 } nfvm_precision;

/* boundary patch kinds (Sec. 2.7) */
enum { NFVM_WALL = 0, NFVM_INLET = 1, NFVM_OUTLET = 2 };
/* physics switches: k-omega closure, energy equation, Boussinesq buoyancy */
enum { NFVM_PHYS_KOMEGA = 1, NFVM_PHYS_ENERGY = 2, NFVM_PHYS_BUOYANCY = 4 };

/* A rectangle of boundary faces on one side of the box (Sec. 2.7).
 * face: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+.  lo/hi: half-open cell ranges
 * along the two tangential axes (x faces: j, k; y faces: i, k; z faces: i, j).
 * Faces no patch covers are adiabatic no-slip walls; the first patch that
 * covers a face wins.
 *   WALL   no-slip; dk/dn = 0; omega fixed in the wall cell to
 *          6 nu / (beta_i d^2); T = T_wall (NaN: adiabatic).
 *   INLET  Dirichlet U, T, k, omega; zero-gradient pressure.
 *   OUTLET zero-gradient velocity, T, k, omega; zero pressure. */
typedef struct {
  int32_t face;
  int32_t lo[2], hi[2];
  int32_t kind;
  double U[3], T, k, omega, T_wall;
} nfvm_patch;

/* Grid and solver description (the paper's problem statement: uniform
 * grid, fluid properties, boundary patches, optional solid mask, time step).
 *   dim           2 or 3; n = cells per axis (n[2] = 1 in 2D); h = spacing [m]
 *   nu, rho       kinematic viscosity [m^2/s], density (p is kinematic)
 *   alpha_T       thermal diffusivity; Pr_t turbulent Prandtl number (0.85)
 *   sigma_k, sigma_w  turbulent Prandtl numbers of k and omega
 *   dt            time step [s]
 *   physics       NFVM_PHYS_* bits
 *   gravity, T_ref, beta_T   Boussinesq source -beta_T (T - T_ref) g
 *   T_solid       temperature of solid cells (NaN: adiabatic)
 *   solid_mask    [nz][ny][nx], 1 = solid, may be NULL; fluid pockets must
 *                 connect to an OUTLET face (else A is singular)
 *   precision     NFVM_FP64 / NFVM_FP32 / NFVM_MIXED (FP32 fields, BF16
 *                 coarse levels, FP64 pressure, residual and projection)
 *   n_levels      multigrid levels; every axis < dim halves exactly per level;
 *                 the coarsest level holds at most 512 fluid cells
 *   nu1, nu2      pre/post Jacobi sweeps; omega_jacobi (0: 4/5 in 2D, 6/7 in 3D)
 *   tol           relative residual target ||b - A phi|| <= tol ||b||
 *   max_cycles    preconditioner applications per pressure solve
 *   nu_coarse     pre and post sweeps on every level below the finest
 *                 (0: nu1 and nu2 there too).  The V-cycle keeps its shape;
 *                 more work on the cheap coarse levels makes up for their
 *                 rediscretised operators, which approximate the fine one
 *                 less well around solid blocks as the grids coarsen.
 *   coarse_fp32_cells  NFVM_MIXED only: coarse levels with at least this many
 *                 cells are stored in FP32 like the finest level, smaller
 *                 ones in BF16 (0: 131072).  BF16 rounding of a large coarse
 *                 level's iterate puts noise on the cycle's correction at
 *                 that level's scale, where the operator weighs it most, and
 *                 costs iterations that grow with the grid; on the small
 *                 levels it is harmless.  A value above every level's cell
 *                 count keeps all coarse levels in BF16. */
typedef struct {
  int32_t dim, n[3];
  double h[3];
  double nu, rho, alpha_T, Pr_t, sigma_k, sigma_w, dt;
  uint32_t physics;
  double gravity[3], T_ref, beta_T, T_solid;
  int32_t n_patches;
  const nfvm_patch* patches;
  const uint8_t* solid_mask;
  int32_t precision;
  int32_t n_levels, nu1, nu2;
  double omega_jacobi, tol;
  int32_t max_cycles;
  int32_t nu_coarse;
  int32_t coarse_fp32_cells;
} nfvm_grid_desc;

/* Host FP64 fields, [nz][ny][nx].  p is kinematic pressure (Pa / rho). */
typedef struct { double *u, *v, *w, *p, *T, *k, *omega; } nfvm_fields;

typedef struct {
  int32_t cycles;         /* preconditioner (V-cycle) applications */
  int32_t status;         /* nfvm_status of this step */
  double rel_residual;    /* ||r|| / ||b|| at exit of the pressure solve */
  double max_face_div;    /* max cell divergence of the corrected face fluxes */
  double min_k, min_omega;/* over fluid cells after the step */
  double seconds;         /* device time of the step */
} nfvm_step_stats;

typedef struct nfvm_grid* nfvm_grid_t;
typedef struct nfvm_server* nfvm_server_t;

/* Optional device allocator used for all later allocations (NULL, NULL:
 * back to hipMalloc/hipFree).  alloc(bytes, ctx) returns a device pointer or
 * NULL; free(ptr, ctx) releases it.  Not thread-safe against running calls. */
typedef void* (*nfvm_alloc_fn)(size_t bytes, void* ctx);
typedef void (*nfvm_free_fn)(void* ptr, void* ctx);
nfvm_status nfvm_set_allocator(nfvm_alloc_fn alloc, nfvm_free_fn free_fn, void* ctx);

/* Create a grid on the current HIP device, classify its cells (patches,
 * solids, wall-fixed omega cells), build the multigrid hierarchy and upload
 * init (all seven fields required).  stream: hipStream_t or NULL.
 * Errors: NFVM_E_INVAL (descriptor), NFVM_E_NOMEM, NFVM_E_DEVICE. */
nfvm_status nfvm_init_grid(const nfvm_grid_desc* desc, const nfvm_fields* init, void* stream,
                           nfvm_grid_t* out);

/* Advance n_steps time steps (Sec. 2.6): destruction over dt/2, explicit
 * step of the rest terms, projection, destruction over dt/2.  stats: NULL or
 * n_steps entries.  Returns NFVM_E_NOTCONV if a pressure solve hit
 * max_cycles (the step is still completed) and NFVM_E_DIVERGED on
 * non-finite residuals (the step stops; fields are undefined). */
nfvm_status nfvm_step(nfvm_grid_t grid, int32_t n_steps, nfvm_step_stats* stats);

/* Advance n_steps time steps (Sec. 2.6) of several grids together, a
 * batching the paper does not treat: each multigrid level's kernels run as one launch
 * over the tiles of every grid of a precision, the bottom solvers and the
 * CG finalisers as one workgroup per grid, all on grids[0]'s stream (the
 * other grids' streams are joined before and after).  A grid whose pressure
 * solve converges goes on to its next step while the others iterate.
 * Results are bitwise those of nfvm_step on each grid alone.  All grids on
 * the current device, no grid twice.  stats: NULL or n_grids * n_steps
 * entries, grid-major; statuses: NULL or n_grids entries (each as
 * nfvm_step would return).  Returns the first non-OK status in grid order. */
nfvm_status nfvm_step_batch(nfvm_grid_t* grids, int32_t n_grids, int32_t n_steps,
                            nfvm_step_stats* stats, nfvm_status* statuses);

/* Solve A x = b with the grid's pressure operator (eq. pc_discretized:
 * seven/five-point -laplacian, zero-gradient walls, inlets and solids, zero
 * value at outlets) by the multigrid-preconditioned iteration.  b, x: host
 * FP64 [nz][ny][nx]; x is the initial guess on entry and the solution on exit;
 * solid cells are ignored on entry and 0 on exit; b = 0 gives x = 0.
 * forced_cycles >= 0 runs exactly that many cycles (tol ignored).  stats may
 * be NULL.  A domain with no outlet has a singular operator (constant mode):
 * a non-zero b then ends in NFVM_E_NOTCONV or NFVM_E_DIVERGED. */
nfvm_status nfvm_mg_solve(nfvm_grid_t grid, const double* b, double* x, double tol,
                          int32_t max_cycles, int32_t forced_cycles, nfvm_step_stats* stats);

/* As nfvm_mg_solve with device FP64 arrays, on the grid's stream. */
nfvm_status nfvm_mg_solve_device(nfvm_grid_t grid, const double* b_dev, double* x_dev,
                                 double tol, int32_t max_cycles, int32_t forced_cycles,
                                 nfvm_step_stats* stats);

/* Reverse mode of the pressure solve (the paper's solver is differentiable,
 * Sec. 1 and 4): for the adjoint xbar of the solution of A x = b, the adjoint
 * of the right-hand side is bbar = A^-T xbar, and A (eq. pc_discretized) is
 * symmetric, so this is the same multigrid solve with xbar on the right.  The
 * solution is differentiated as the exact A^-1 b (implicit differentiation),
 * not through the iterations that approximate it.  xbar_dev, bbar_dev: device
 * FP64 [nz][ny][nx]; bbar_dev holds the initial guess on entry (zeros for
 * none) and bbar on exit.  Tolerance, forced cycles, stats and errors as
 * nfvm_mg_solve_device. */
nfvm_status nfvm_mg_solve_adjoint_device(nfvm_grid_t grid, const double* xbar_dev,
                                         double* bbar_dev, double tol, int32_t max_cycles,
                                         int32_t forced_cycles, nfvm_step_stats* stats);

/* Reverse mode of the pressure step (Sec. 2.4): the map from the explicit
 * step's velocity u* and the pressure p^n to u = u* - dt G(phi) and
 * p = p^n + phi, where phi = A^-1 b and b = -(1/dt) sum_d D_d L_d BC_d(u*_d)
 * (eq. pc_residual), with the boundary ghosts of Sec. 2.7, is affine in u*.
 * For the adjoints ubar, vbar, wbar, pbar of u, v, w and p it writes the
 * adjoints of u*, v*, w* into usbar, vsbar, wsbar (that of p^n is pbar
 * itself): usbar = ubar + (dB/du*)^T lambda with lambda = A^-T (pbar -
 * dt G^T ubar), one multigrid solve (to tol, or forced_cycles; the solve is
 * differentiated as the exact one).  All arrays device FP64 [nz][ny][nx],
 * all seven required (in 2D w is passed through: wsbar = wbar); outputs may
 * not alias inputs.  Runs on the grid's stream and waits for it; the grid's
 * fields are not touched.  stats: NULL or one entry (the solve's cycles,
 * status, relative residual and time).  Errors as nfvm_mg_solve_device;
 * NFVM_E_INVAL for a null pointer. */
nfvm_status nfvm_pressure_adjoint_device(nfvm_grid_t grid, const double* ubar,
                                         const double* vbar, const double* wbar,
                                         const double* pbar, double* usbar, double* vsbar,
                                         double* wsbar, double tol, int32_t max_cycles,
                                         int32_t forced_cycles, nfvm_step_stats* stats);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation):
 * nfvm_mg_solve_device without any device allocation.  The solve's
 * reduction partials and scalars live in a fixed 2 MiB device array of the
 * library (one copy per device, held until the process ends) instead of the
 * grid's own buffers; the kernels and their order are nfvm_mg_solve_device's,
 * so the results are the same.  Arguments, layout and errors as
 * nfvm_mg_solve_device; NFVM_E_INVAL if the grid's reductions need more
 * partials than the array holds (about 87,000 workgroups; grids up to the
 * 1024 x 512 x 256 room with autotuned tiles fit).  Every call on a device
 * shares its array: calls that overlap on one device (two host threads, or
 * two streams in flight) race and must not be made.  The call waits for the
 * grid's stream (it cannot be captured into a graph). */
nfvm_status nfvm_mg_solve_device_noalloc(nfvm_grid_t grid, const double* b_dev, double* x_dev,
                                         double tol, int32_t max_cycles, int32_t forced_cycles,
                                         nfvm_step_stats* stats);

/* Copy the cell-centred fields u, v, w, p, T, k, omega (the tensors of
 * Sec. 2.2, one value per cell) to host FP64 arrays, [nz][ny][nx] (all seven
 * pointers required; waits for the grid's stream).  Errors: NFVM_E_INVAL for
 * a null pointer. */
nfvm_status nfvm_get_fields(nfvm_grid_t grid, nfvm_fields* out);

/* Vortex criterion of Sec. 3.2 (lambda2 of Jeong and Hussain) for the
 * grid's current velocity: per cell the middle eigenvalue of S^2 + W^2,
 * with S and W the symmetric and antisymmetric parts of the velocity
 * gradient (central differences with the boundary ghosts, as in the
 * destruction step of Algorithm 3); negative values mark vortex cores.
 * Non-fluid cells receive 0.  lambda2: host array of n[0]*n[1]*n[2] FP64
 * values, C order [nz][ny][nx], written before return (the call waits for
 * the grid's stream).  Computed on the device in the velocity's precision.
 * Errors: NFVM_E_INVAL for a null argument. */
nfvm_status nfvm_lambda2(nfvm_grid_t grid, double* lambda2);

/* Reverse mode of the explicit stage (Sec. 2.3, Algorithms 2 and 4, eqs.
 * ko_mom, ko_temp, ko_k, ko_o; the solver is differentiable, Sec. 1 and 4):
 * the forward-Euler step E of the rest terms maps the fields (u, v, w, p, T,
 * k, omega) to (u, v, w, T, k, omega), with nu_t the closure of the input k
 * and omega (eqs. a_star, ko_turb_diff), the boundary ghosts of Sec. 2.7,
 * k and omega clamped at 1e-10 and omega held on wall-adjacent cells.  For
 * the adjoints `bar` of its six outputs (bar->p is not read and may be
 * NULL) this writes the adjoints J^T bar of its seven inputs into `out`,
 * J the Jacobian of E at the input state `state` (upwind selections and
 * clamps as the forward step takes them there).  All arrays device FP64
 * [nz][ny][nx], T absolute; outputs may not alias inputs.  Arithmetic in
 * FP64 whatever the grid's precision; the grid's fields are not touched.
 * The first call of this or nfvm_destroy_adjoint_device allocates 22 FP64
 * values per padded cell of scratch, kept until the grid is freed.  Runs on
 * the grid's stream and waits for it.  Errors: NFVM_E_INVAL for a null
 * pointer, NFVM_E_NOMEM. */
nfvm_status nfvm_explicit_adjoint_device(nfvm_grid_t grid, const nfvm_fields* state,
                                         const nfvm_fields* bar, nfvm_fields* out);

/* Reverse mode of the destruction step (Sec. 2.5, Algorithm 3, eqs.
 * k_des_step, o_des_step, beta_star, o_des): the step over a time tau maps
 * (u, v, w, k, omega) to k' = k / (1 + tau beta* f_beta* omega) and omega' =
 * omega / (1 + tau beta_i f_beta omega), whose coefficients read the central
 * gradients of k, omega and the velocity (boundary ghosts of Sec. 2.7);
 * wall-adjacent cells keep omega and non-fluid cells keep both.  For the
 * adjoints kbar, wbar of k' and omega' this writes the adjoints of the five
 * inputs (state->u, v, w, k, omega; T and p not read, out->T and out->p not
 * written) at the input state.  All arrays device FP64 [nz][ny][nx]; outputs
 * may not alias inputs; FP64 arithmetic; scratch as for
 * nfvm_explicit_adjoint_device (shared).  Runs on the grid's stream and
 * waits for it.  Errors: NFVM_E_INVAL for a null pointer or tau < 0,
 * NFVM_E_NOMEM. */
nfvm_status nfvm_destroy_adjoint_device(nfvm_grid_t grid, const nfvm_fields* state, double tau,
                                        const double* kbar, const double* wbar,
                                        nfvm_fields* out);

/* Reverse mode of one whole time step (nfvm_step; the solver is
 * differentiable, Sec. 1 and 4): the step loads the state as
 * nfvm_set_fields does (omega held on wall-adjacent cells), then
 * destruction over dt/2, the explicit stage, the pressure step and
 * destruction over dt/2 (Sec. 2.3 to 2.5).  For the adjoints `bar` of the
 * seven fields after the step it writes those of the seven fields of
 * `state` into `out`: the step is run forward from `state` on the grid's
 * fields (which hold its result on return), keeping the stage inputs, and
 * the stages' reverse modes (nfvm_destroy_adjoint_device,
 * nfvm_pressure_adjoint_device, nfvm_explicit_adjoint_device) are applied
 * in reverse order; both pressure solves run to tol (or forced_cycles) and
 * the solve is differentiated as the exact A^-1.  With NFVM_OPT_RK_ORDER 2
 * the explicit stage is Heun's (U + E(E(U))) / 2 and its reverse mode
 * (b + J1^T J2^T b) / 2, the forward-Euler reverse mode taken at the first
 * stage's output, then at U.  All arrays device FP64 [nz][ny][nx], T
 * absolute; outputs may not alias inputs.  stats: NULL or two entries, the
 * forward and the adjoint solve.  The first call allocates 35 dense FP64
 * arrays of scratch (20 more with the Heun stage, plus the stage reverse
 * modes' scratch), kept until the grid is freed.  Runs on the grid's stream
 * and waits for it.  Errors: NFVM_E_INVAL for a null pointer; solve
 * statuses as nfvm_mg_solve_device (a diverged forward solve leaves `out`
 * unwritten). */
nfvm_status nfvm_step_adjoint_device(nfvm_grid_t grid, const nfvm_fields* state,
                                     const nfvm_fields* bar, nfvm_fields* out, double tol,
                                     int32_t max_cycles, int32_t forced_cycles,
                                     nfvm_step_stats* stats);

/* Line probes of Sec. 3.1 (the velocity magnitude V, the temperature T, k
 * and omega compared along lines of the channel cases): at n points of the
 * grid's current fields.  pts: host array of 3*n FP64 coordinates in metres
 * (x, y, z per point; z is ignored in 2D), the box spanning [0, n_d h_d].
 * Each field is interpolated trilinearly between the cell centres (the
 * centre of cell i at (i + 1/2) h), over the fluid cells among the eight
 * around the point with their weights renormalised to sum to one; a point
 * is first clamped into the box of cell centres.  V is the magnitude of the
 * interpolated velocity; T is absolute (T_ref added back).  out: host array
 * of 4*n FP64 values {V, T, k, omega} per point, written before return (the
 * call waits for the grid's stream); a point whose eight cells are all
 * non-fluid receives NaN.  Computed on the device in FP64 from the stored
 * fields.  Errors: NFVM_E_INVAL for a null grid, n < 0, null arrays with
 * n > 0, or more than ncells / 7 points (the points and results pass
 * through the grid's staging buffer). */
nfvm_status nfvm_line_probe(nfvm_grid_t grid, const double* pts, int32_t n, double* out);

/* Replace the grid's fields (Sec. 2.2 tensors) from host FP64 arrays,
 * [nz][ny][nx], all seven required; values in solid cells are kept as given
 * and never updated; omega in wall-adjacent cells is reset to the wall value
 * (Sec. 2.7); the pressure solve's initial guess is cleared.  Errors:
 * NFVM_E_INVAL for a null pointer. */
nfvm_status nfvm_set_fields(nfvm_grid_t grid, const nfvm_fields* in);

/* Bytes of device memory a grid with this descriptor allocates. */
nfvm_status nfvm_grid_footprint(const nfvm_grid_desc* desc, size_t* bytes);

/* Host-side check of the reduction scratch (no device work): *needed is the
 * largest number of workgroups any reducing level-0 kernel launches for this
 * descriptor under any tile choice the autotuner can make (each workgroup
 * stores up to three FP64 partials); *capacity is how many workgroups the
 * grid's partial buffer holds.  Every reducing launch also checks this
 * itself and fails with NFVM_E_DEVICE instead of writing past the buffer.
 * Errors: NFVM_E_INVAL (descriptor or null pointer). */
nfvm_status nfvm_reduction_blocks(const nfvm_grid_desc* desc, int32_t* needed,
                                  int32_t* capacity);

/* Release the grid's device memory, stream (if the library created it) and
 * graphs; waits for the grid's pending work.  The handle is invalid after.
 * The grid's buffers come from one allocation with a zeroed guard zone after
 * each; NFVM_E_DEVICE (the grid is released all the same) if a guard zone
 * holds a non-zero byte, naming the buffer an out-of-bounds store ran past. */
nfvm_status nfvm_free_grid(nfvm_grid_t grid);

/* Serving: at most max_slots solves run at once; queued solves are admitted
 * first fit in arrival order while the summed device footprint of running
 * solves stays within hbm_budget_bytes.  Running solves are spread over
 * min(max_slots, 3) lanes, each a host thread with its own HIP stream that
 * advances its solves together as in nfvm_step_batch (at most
 * ceil(max_slots / lanes) per lane); lanes overlap on the device.  A lane
 * admits the next request as soon as it has room (new work joins at the next
 * round of its lane).  A finished solve releases its device memory and keeps
 * its fields on the host until polled.  Every request's fields are bitwise
 * those of nfvm_step on a grid of its own.
 * hbm_budget_bytes <= 0: 90 % of the free device memory. */
nfvm_status nfvm_server_create(double hbm_budget_bytes, int32_t max_slots, nfvm_server_t* out);

/* Queue a solve of n_steps time steps; the descriptor, patches, mask and
 * init are copied before return.  NFVM_E_NOMEM if its footprint alone is
 * above the budget. */
nfvm_status nfvm_submit(nfvm_server_t server, const nfvm_grid_desc* desc,
                        const nfvm_fields* init, int32_t n_steps, uint64_t* ticket);

/* NFVM_PENDING while queued or running.  When done, copies the final fields
 * into out (if non-NULL; all seven pointers) and the last step's stats into
 * last (if non-NULL), releases the request and returns its status. */
nfvm_status nfvm_poll(nfvm_server_t server, uint64_t ticket, nfvm_fields* out,
                      nfvm_step_stats* last);

/* Per-request timestamps in seconds since server creation: submit, admit,
 * first step meeting tol, done (negative: not yet).  Valid until polled. */
nfvm_status nfvm_request_times(nfvm_server_t server, uint64_t ticket, double times[4]);

/* Block until every submitted request is done (not yet polled ones stay). */
nfvm_status nfvm_server_drain(nfvm_server_t server);

nfvm_status nfvm_server_destroy(nfvm_server_t server);

/* Kernel timing.  nfvm_profile(grid, mask) times every later launch of the
 * kernels whose bit (1 << id) is set with HIP events on the grid's stream and
 * resets the totals (mask 0: off); every kernel of a time step belongs to one
 * id.  nfvm_profile_read returns, per id, the number of timed launches, their
 * summed device time and the mean algorithmic bytes of one launch (the
 * minimum traffic of its operands: each input read once, each output written
 * once, at the storage precision; 0 for the finalisers, whose few KB of
 * partials are latency, not bandwidth).  Ids 10 to 12 gather the per-level
 * kernels of every coarse level, so their bytes vary from launch to launch. */
enum {
  NFVM_K_SMOOTH0 = 0,      /* damped-Jacobi sweep on level 0 */
  NFVM_K_SMOOTH0_ZERO = 1, /* first sweep from a zero iterate */
  NFVM_K_RESTRICT0 = 2,    /* residual + restriction, level 0 -> 1 */
  NFVM_K_PROLONG0 = 3,     /* prolongation + correction, level 1 -> 0 */
  NFVM_K_EXPLICIT = 4,     /* explicit step of u, v, w, T, k, omega */
  NFVM_K_DESTROY = 5,      /* semi-implicit destruction half step */
  NFVM_K_RHS = 6,          /* Poisson right-hand side */
  NFVM_K_PROJECT = 7,      /* projection */
  NFVM_K_FCG_APPLY = 8,    /* w = A z and (z, r), (z, q), (z, w) */
  NFVM_K_FCG_UPDATE = 9,   /* p, q, x, r update and ||r|| */
  NFVM_K_SMOOTH_C = 10,    /* damped-Jacobi sweeps on the coarse levels */
  NFVM_K_RESTRICT_C = 11,  /* residual + restriction between coarse levels */
  NFVM_K_PROLONG_C = 12,   /* prolongation + correction between coarse levels */
  NFVM_K_BOTTOM = 13,      /* LDS bottom solver, or the coarsest dense solve */
  NFVM_K_FCG_START = 14,   /* r = b - A x0, ||b||, ||r|| and level 0's first sweep */
  NFVM_K_FINALIZE = 15,    /* one-workgroup finalisers of the reductions */
  NFVM_K_SMOOTH0_PAIR = 16, /* two damped-Jacobi sweeps in one pass on level 0 */
  NFVM_K_COUNT = 17
};
nfvm_status nfvm_profile(nfvm_grid_t grid, uint32_t kernel_mask);
nfvm_status nfvm_profile_read(nfvm_grid_t grid, int32_t kernel, int64_t* launches,
                              double* seconds, double* bytes_per_launch);

/* Grid options.
 *   NFVM_OPT_GRAPHS   1 (default): the time step runs as captured HIP graphs
 *                     (step prefix, one CG iteration replayed, step suffix);
 *                     0: plain stream launches.  Graphs are not used while
 *                     nfvm_profile timing is on.
 *   NFVM_OPT_PREDICT  CG iterations enqueued before the first convergence
 *                     check (default: the count of the previous solve).
 *   NFVM_OPT_BOTTOM   1 (default): the coarse levels whose arrays fit in the
 *                     LDS of one workgroup (160 KiB on MI355X) run as one
 *                     workgroup in one launch; 0: one launch per operator
 *                     and level.
 *   NFVM_OPT_AUTOTUNE 1 (default, applied in nfvm_init_grid): the tile shape
 *                     (workgroups per launch, planes per thread) of every hot
 *                     kernel is chosen per level by timing candidates on the
 *                     grid; results are cached per shape and precision for
 *                     the process.  0: fixed default tiles.
 *   NFVM_OPT_WARM_START 0 (default): every step's pressure solve starts
 *                     from phi = 0, and restarts through nfvm_get_fields /
 *                     nfvm_set_fields are bitwise.  1: each solve starts
 *                     from the previous step's increment phi = p^{n+1} - p^n
 *                     (zero after nfvm_init_grid, nfvm_set_fields and
 *                     nfvm_mg_solve), which saves cycles in a slowly
 *                     varying flow; the increment is not part of the
 *                     fields, so a restarted run then agrees with the
 *                     uninterrupted one to the solver tolerance only.
 *   NFVM_OPT_PROLONG  0 (default): the multigrid correction is prolongated
 *                     by cell-centred linear interpolation (Sec. 2.4, eq.
 *                     prolongation).  1: nearest (piecewise-constant)
 *                     upsampling, the plainest reading of the upsampling in
 *                     Algorithm 1; the coarse levels then run one launch per
 *                     operator and level (the LDS-resident bottom solver
 *                     interpolates linearly).  Grids batch together only
 *                     with grids of the same setting.  Other values:
 *                     NFVM_E_INVAL.
 *   NFVM_OPT_RK_ORDER 1 (default): the explicit stage is one forward-Euler
 *                     step.  2: Heun's second-order Runge-Kutta method
 *                     (Sec. 2.6 leaves the explicit scheme open), as the
 *                     average of the start and a second Euler step taken
 *                     from the first, whose nu_t comes from the first
 *                     stage's k and omega.  The first call with 2 allocates
 *                     one more set of the six transported fields (three
 *                     velocity and three scalar arrays, padded; not counted
 *                     by nfvm_grid_footprint); NFVM_E_NOMEM if that fails.
 *                     Other values: NFVM_E_INVAL.
 *   NFVM_OPT_LITERAL  0 (default).  1: the pressure solve exactly as
 *                     Algorithm 1 prints it (Sec. 2.4): the residual
 *                     restricted to every level, on the way up one undamped
 *                     Jacobi sweep per level with the scalar diagonal of eq.
 *                     jacobi_pc (6/dx^2, 2 sum_d 1/h_d^2 for unequal spacings;
 *                     one sweep from zero on the coarsest level) and nearest
 *                     upsampling, then one fine sweep, repeated as a plain
 *                     iteration p <- p + V(b - A p) without the conjugate-
 *                     gradient wrapper, to tol or max_cycles (forced counts as
 *                     usual).  nu1, nu2 and omega_jacobi of the descriptor
 *                     are set aside while it is on.  Such grids are stepped
 *                     alone: nfvm_step_batch refuses them (NFVM_E_INVAL).
 *                     Other values: NFVM_E_INVAL.
 *   NFVM_OPT_SWEEP_PAIRS  1 (default): consecutive damped-Jacobi sweeps on
 *                     the finest level run two per pass (x, b and the face
 *                     codes read once for both) where its rows are a
 *                     multiple of 4 cells, as many as keep the V-cycle's
 *                     result out of the buffer the next cycle's first sweep
 *                     is fused into; the fields are bitwise those of single
 *                     sweeps.  0: one sweep per pass.  Batched iterations
 *                     (nfvm_step_batch, serving) take single sweeps.
 *                     Other values: NFVM_E_INVAL.
 * Errors: NFVM_E_INVAL for an unknown option. */
enum {
  NFVM_OPT_GRAPHS = 0,
  NFVM_OPT_PREDICT = 1,
  NFVM_OPT_BOTTOM = 2,
  NFVM_OPT_AUTOTUNE = 3,
  NFVM_OPT_WARM_START = 4,
  NFVM_OPT_PROLONG = 5,
  NFVM_OPT_RK_ORDER = 6,
  NFVM_OPT_LITERAL = 7,
  NFVM_OPT_SWEEP_PAIRS = 8
};

/* Tune the tile shapes of a grid shape and precision ahead of serving:
 * creates a grid of the descriptor with the autotuner on, on a stream of its
 * own, and frees it; the choices stay in the process-wide table.  Served
 * grids never tune: a shape that is in the table takes its choices, another
 * takes those of the tuned shape of the same dimension and precision nearest
 * in cell count (log scale), else the defaults.  Errors as nfvm_init_grid. */
nfvm_status nfvm_tune(const nfvm_grid_desc* desc);

/* The autotuner's choices so far: up to max entries of {kernel id, nx, ny,
 * nz, dim, precision, tile target}; *count receives the number written. */
nfvm_status nfvm_tuning_table(int32_t* entries, int32_t max, int32_t* count);
nfvm_status nfvm_set_option(nfvm_grid_t grid, int32_t option, double value);

/* Message for the last non-OK status on this thread. */
const char* nfvm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
