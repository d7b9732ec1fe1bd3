/*
 * sw.h -- C ABI of the MI355X (gfx950) library for the discontinuous-Galerkin
 * shallow-water operator with sub-grid bathymetry of Arpaia, Orlando, Ferrarin
 * and Bonaventura, arXiv:2505.18743.
 *
 * The library advances
 *     dh/dt + div q = 0,  dq/dt + div(q (x) u) + g h grad zeta = -gamma q,
 *     d(hc)/dt + div(q c) = 0                               (Sec. 2, eq:shw)
 * with h = max(zeta - b, 0) evaluated only at quadrature nodes (eq:zeta2depth-2),
 * nodal Q_r elements on GLL support points (Sec. 3.2), Rusanov fluxes with
 * hydrostatic reconstruction (eq:lxf_parameter, eq:hydro_rec_vars), the
 * non-conservative pressure form (eq:discharge_rhs, eq:pressure_tumolo), an
 * element-wise Newton solve for the free surface with a land-sea-mask Jacobian
 * (eq:newton, eq:mass_matrix), degree coarsening to r_K = 0 at wet/dry
 * elements (eq:criteria_p) and an hc-consistent tracer update
 * (eq:algebraic_concentration), in the explicit Butcher form of Sec. 3.1.
 *
 * Conventions (all calls):
 *  - All real data are IEEE double.  "device" pointers are HIP device (or
 *    managed) memory on the device that was current at sw_create; "host"
 *    pointers are ordinary host memory.  Arrays are copied in or out during
 *    the call; the caller keeps ownership of every buffer it passes.
 *  - Nodal fields use the layout [cell][jy][jx] with (r+1)^2 values per cell,
 *    jx, jy indexing the (r+1)-point GLL support points on [0,1] (Sec. 3.2).
 *  - Sample-node fields use [cell][b][a] with S_L^2 values for a cell of
 *    level L: node (a, b) sits at x = x0 + (i + xhat_a) dx_L,
 *    y = y0 + (j + xhat_b) dx_L, xhat the closed S_L-point rule on [0,1].
 *    The same formula gives bitwise-equal coordinates on both sides of every
 *    face, so a single-valued bed yields equal samples there.
 *  - Cells must be given sorted by level (non-decreasing).
 *  - Calls enqueue work on the context's stream and return without waiting,
 *    except where marked "synchronises".
 *  - Every call returns an sw_status; on failure sw_last_error() returns a
 *    message (thread-local, valid until the next failing call on the thread).
 *    No C++ exception crosses this interface.
 *  - A context is not thread-safe; use one context per host thread/stream.
 */
#ifndef SW_H_
#define SW_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sw_ctx sw_ctx;

typedef enum {
  SW_OK = 0,
  SW_EINVAL = -1,       /* invalid argument (message says which)            */
  SW_ENOMEM = -2,       /* device allocation failed                          */
  SW_EHIP = -3,         /* a HIP runtime call failed                         */
  SW_ENONFINITE = -4,   /* a non-finite value appeared in the state          */
  SW_EDEVICE = -5       /* a kernel detected an invalid index and skipped it */
} sw_status;

/* boundary kinds for the four sides of the domain (west, east, south, north) */
enum { SW_BC_WALL = 0,      /* ghost mirrors the normal discharge                  */
       SW_BC_ELEV = 1,      /* ghost imposes zeta = A sin(2 pi t / T + phase),     */
                            /* extrapolates q, takes c_in on inflow                */
       SW_BC_OPEN = 2,      /* ghost copies the interior state                     */
       SW_BC_PERIODIC = 3,  /* opposite sides are joined (must come in pairs)      */
       SW_BC_STATE = 4,     /* ghost is a given (zeta, q, c) per face node (an     */
                            /* exact state at a supercritical inflow, Sec. 4.4)    */
       SW_BC_DISCHARGE = 5 };/* ghost takes a given q per face node, extrapolates  */
                            /* zeta, takes the given c where q.n < 0 (the inflow   */
                            /* discharge of the channel case, Sec. 4.3)            */

enum { SW_RULE_EQ = 0,      /* closed equispaced (composite trapezoid) rule         */
       SW_RULE_GLL = 1 };   /* Gauss-Legendre-Lobatto rule                         */

enum { SW_QUAD_SUBGRID = 0, /* the S x S sample rule serves every element integral  */
       SW_QUAD_PAPER = 1 }; /* Table 1: volume terms (F, G, R, the friction L and  */
                            /* its matrix) on Gauss-Legendre (floor(3r/2)+1)^2     */
                            /* nodes with bathymetry samples of their own; faces, */
                            /* the wet/dry rule and the continuity and tracer     */
                            /* masses on the GLL (r+2)^2 sample rule; discharge   */
                            /* mass exact (GL (r+1)^2).  Needs SW_RULE_GLL with   */
                            /* S = r + 2 on every level.  Every cell then takes   */
                            /* the general element kernel; sw_vjp_operator and    */
                            /* sw_vjp_step reject such a context.                 */

enum { SW_RK_FE = 0, SW_RK_SSP3 = 1, SW_RK_RK32 = 2, SW_RK_RK44 = 3,  /* Appendix A */
       SW_RK_IMEX = 4 };    /* Sec. 3.1 IMEX pair of Appendix A: the explicit     */
                            /* RK32 tableau for everything but the Manning        */
                            /* friction, TR-BDF2 (chi = 1 - sqrt(2)/2, b~ = b)    */
                            /* for the friction.  A stage solves                  */
                            /* (M + a~_ll dt Gam) q = M q^n + dt (sum a G +       */
                            /* sum a~ L) (eq:algebraic_discharge,                 */
                            /* eq:mass_matrix_discharge) with Gam linearised at   */
                            /* the previous stage; the final combination is       */
                            /* explicit.  sw_vjp_step rejects such a context.     */

typedef struct {
  int32_t nx0, ny0;          /* coarse grid, cells of size dx0                     */
  double x0, y0, dx0;        /* lower-left corner and coarse cell size             */
  int32_t n_cells;           /* number of quadtree leaves                          */
  const int32_t *level;      /* host [n_cells]: leaf level L, cell size dx0/2^L    */
  const int32_t *i, *j;      /* host [n_cells]: position in level-L units          */
  int32_t bc[4];             /* west, east, south, north: SW_BC_*                  */
} sw_mesh_desc;

typedef struct {
  int32_t r;                 /* polynomial degree 1..3                             */
  int32_t rule;              /* SW_RULE_*                                          */
  int32_t n_levels;          /* entries used in S                                  */
  int32_t S[8];              /* sample nodes per direction per level, r+2 <= S <= 32 */
  int32_t rk;                /* SW_RK_*                                            */
  double g;                  /* gravity                                            */
  double eps;                /* velocity desingularisation depth (eq:velocity) > 0 */
  double h_lim;              /* degree-coarsening depth (eq:criteria_p)            */
  double eps0;               /* dry-cell lift of the Newton guess (eq:initial_guess)*/
  int32_t newton_max;        /* Newton iteration cap                               */
  double cfl;                /* dt = cfl * min over face nodes of w J_K/(lambda l) */
  int32_t cfl_mode;          /* 0: w = 1; 1: w = end-point weight of the rule      */
  int32_t tracer;            /* 0 or 1 passive tracer                              */
  int32_t adapt_degree;      /* 1: degree coarsening on, 0: always degree r        */
  double tide_amp, tide_period, tide_phase, tide_c_in;   /* SW_BC_ELEV data         */
  /* tracer numerical diffusion (eq:numdiff): R_i gets - int nu_K h grad c .   */
  /* grad psi_i with nu_K = tracer_diff |K| tracer_strain / r^2, the constant C */
  /* and a characteristic strain rate S (1/s) of the resolved flow; and a     */
  /* first-order decay, the reaction phi(c) = -tracer_decay c of eq:shw        */
  /* (1/s), taken explicitly: R_i gets - tracer_decay int h c psi_i.  Zero: off */
  double tracer_diff, tracer_strain, tracer_decay;
  int32_t quadrature;        /* SW_QUAD_*                                          */
} sw_params;

typedef struct {
  double total_mass;         /* sum over cells of int max(zeta - b, 0) (eq:positivity-7) */
  double min_target_mass;    /* min over cells and stages of the element target mass     */
  double dt;                 /* time step of the last step                              */
  double t;                  /* model time                                              */
  int64_t n_pos_viol;        /* (cell, stage) pairs with negative target mass           */
                             /* (a tracer replay forms no flow target: min_target_mass  */
                             /* is 1e300 and n_pos_viol 0 there; the flow's are the     */
                             /* recording context's)                                    */
  int32_t max_newton_it;     /* largest Newton iteration count in the last step          */
  int32_t nonfinite;         /* 1 if a non-finite value was found in the state           */
  int64_t n_r0_cells;        /* cells at degree 0 for the next step (the degree decision  */
                             /* of eq:criteria_p, taken at the end of the last step)       */
  int64_t n_fallback;        /* masked Jacobians replaced by the constant-mode update    */
  int64_t step;              /* steps taken                                              */
} sw_diag;

/* Create a context: validates the mesh (leaves tile the domain, 2:1 balance,
 * level order) and parameters, builds faces and reference tables, allocates
 * device memory.  `stream` is a hipStream_t (NULL: the default stream).
 * Errors: SW_EINVAL (bad mesh/params), SW_ENOMEM, SW_EHIP. */
sw_status sw_create(sw_ctx **out, const sw_mesh_desc *mesh, const sw_params *p, void *stream);
void sw_destroy(sw_ctx *c);
const char *sw_last_error(void);

/* Batched context of n_members independent problems (ensemble members; the
 * paper treats one problem, this packs several into every kernel launch).
 * meshes[m] and params[m] (host arrays of n_members) describe member m; the
 * members may differ in mesh, cell size, boundary kinds, tide (tide_*) and
 * CFL number (cfl), and must agree in r, rule, n_levels, S[0..n_levels), rk,
 * g, eps, h_lim, eps0, newton_max, cfl_mode, tracer and adapt_degree
 * (SW_EINVAL otherwise).  Each member has its own time, CFL time step (the
 * minimum of Prop. 3.2's bound over its own faces) and diagnostics; faces
 * join cells of one member only.  Cells are ordered by level, then member,
 * then the member's own order; every array argument of the calls below uses
 * that order (sw_cell_map gives it; for single-level members it is the
 * members' cells one after the other).  A dt > 0 given to the step calls is
 * used by every member.  sw_create(c, m, p, s) is sw_create_batch(c, 1, m, p, s). */
sw_status sw_create_batch(sw_ctx **out, int32_t n_members, const sw_mesh_desc *meshes, const sw_params *params,
                          void *stream);
/* Host outputs [n_cells]: member of each cell and its index in that member's
 * description (either may be NULL). */
sw_status sw_cell_map(const sw_ctx *c, int32_t *member_host, int32_t *local_host);
/* Point evaluation of nodal fields (gauges): for n points xy_host [n][2] of a
 * member, the containing cell (context numbering, cell_host [n]) and the basis
 * values phi_host [n][(r+1)^2] (layout [jy][jx]), so that a field's value at
 * point g is sum_j phi[g][j] field[cell[g]][j].  Host computation; SW_EINVAL
 * for a point outside the member's mesh (cells are half-open [x, x+dx)). */
sw_status sw_locate_points(const sw_ctx *c, int32_t member, int32_t n, const double *xy_host, int32_t *cell_host,
                           double *phi_host);

/* Given boundary data of the SW_BC_STATE and SW_BC_DISCHARGE sides.  Their
 * face nodes (the S_L nodes of the cell's rule along each boundary face of
 * those sides, faces in the library's order, nodes ascending along the face)
 * number n_nodes; sw_boundary_nodes writes the count and, where not NULL, the
 * coordinates xy_host [n_nodes][2] (member coordinates) and member_host
 * [n_nodes].  sw_set_boundary_state copies ghost_dev (device [4][n_nodes]:
 * zeta, qx, qy, c at each node; a discharge side reads qx, qy and c) into the
 * context, where it holds until the next call: it is the ghost of every stage
 * of the following steps (a time-dependent state is sampled by the caller
 * between steps).  Steps, sw_apply_operator and the adjoint calls return
 * SW_EINVAL on a mesh with such sides until it has been called once;
 * sw_set_boundary_state returns SW_EINVAL on a mesh without them.  Boundary
 * faces use the interior flux formulas with this ghost (Sec. 3.2: jumps and
 * averages on boundary faces are one-sided). */
sw_status sw_boundary_nodes(const sw_ctx *c, int64_t *n_nodes, double *xy_host, int32_t *member_host);
sw_status sw_set_boundary_state(sw_ctx *c, const double *ghost_dev);

/* Sizes: cells, bathymetry nodes (sum over cells of S_L^2, plus, with
 * SW_QUAD_PAPER, (floor(3r/2)+1)^2 volume-rule nodes per cell), nodal values
 * per field. */
sw_status sw_counts(const sw_ctx *c, int64_t *n_cells, int64_t *n_vol_nodes, int64_t *n_dofs);

/* Host outputs: bathymetry-node coordinates [n_vol_nodes][2] and basis
 * support point coordinates [n_dofs][2].  The sample nodes of every cell come
 * first (cells in context order, node q = b S + a at (x_a, y_b)); with
 * SW_QUAD_PAPER the volume-rule nodes of every cell follow in the same
 * layout.  Synchronises. */
sw_status sw_node_coords(const sw_ctx *c, double *xy_host);
sw_status sw_dof_coords(const sw_ctx *c, double *xy_host);

/* Bed ELEVATION b at the nodes of sw_node_coords (device, [n_vol_nodes]).  The library
 * stores the bathymetry depth z_b = -(b + db_K) of Sec. 2 (db: bed offset). */
sw_status sw_set_bathymetry(sw_ctx *c, const double *b_dev);
/* Per-cell Manning coefficient n_K (eq:manning), device [n_cells]. */
sw_status sw_set_manning(sw_ctx *c, const double *n_dev);
/* Per-cell bed-elevation offset db_K added to every sample of cell K, device [n_cells]. */
sw_status sw_set_bed_offset(sw_ctx *c, const double *db_dev);

/* State I/O, device [n_dofs] each; tracer may be NULL (then zero / not copied).
 * sw_set_state also resets every cell to degree r. */
sw_status sw_set_state(sw_ctx *c, const double *eta, const double *qx, const double *qy, const double *tracer);
sw_status sw_get_state(const sw_ctx *c, double *eta, double *qx, double *qy, double *tracer);
/* Definition 3.1: zeta_j = eta_j in cells with a wet sample node
 * (eta(x_q) - b(x_q) > 0), zeta_j = min_q b(x_q) elsewhere; q = 0. */
sw_status sw_init_lake_at_rest(sw_ctx *c, const double *eta_dev);
sw_status sw_set_time(sw_ctx *c, double t);
/* The elevation boundary's data (SW_BC_ELEV, Sec. 4.5's M2 tide) of every
 * member, replacing sw_params.tide_*: zeta = amplitude sin(2 pi t / period +
 * phase) at the face nodes and c_inflow taken by the tracer on inflow.
 * period must be finite and non-zero (SW_EINVAL otherwise). */
sw_status sw_set_tide(sw_ctx *c, double amplitude, double period, double phase, double c_inflow);

/* Weak residuals of the degree-r test functions for the given state (device
 * inputs/outputs, [n_dofs] each; tracer/R may be NULL): F (eq:mass_rhs),
 * Gx, Gy (eq:discharge_rhs with the friction term of eq:discharge_rhs_implicit
 * added explicitly), R (eq:r_concentration).  dtb_dev (device double, may be
 * NULL) receives min over face nodes/sides of w J_K/(lambda l) (Prop. 3.2). */
sw_status sw_apply_operator(sw_ctx *c, const double *eta, const double *qx, const double *qy,
                            const double *tracer, double t, double *F, double *Gx, double *Gy,
                            double *R, double *dtb_dev);
/* The same evaluation for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid it): same
 * arguments, same kernels and results, but the call's scratch (one residual
 * slot of 4 n_dofs doubles, the per-face time-step bounds and their reduction
 * partials, rounded up to 256 bytes each) lives in a fixed 48 MiB device array
 * of the library (6 Mi doubles, one per GPU, held until the process ends)
 * instead of the context's memory; it calls no allocator.  SW_EINVAL when the
 * context needs more scratch than that (above about 1.5 M dofs per field,
 * 165k cells at r = 2; use sw_apply_operator).  Every call on one GPU shares that array:
 * calls that overlap on the device (other streams or threads, other contexts)
 * race and must be ordered by the caller. */
sw_status sw_apply_operator_noalloc(sw_ctx *c, const double *eta, const double *qx, const double *qy,
                                    const double *tracer, double t, double *F, double *Gx, double *Gy,
                                    double *R, double *dtb_dev);

/* One RK step split in its parts (Sec. 3.1, Butcher form):
 *   sw_step_begin: degree adaptation + conservative remap, H(zeta^n), C~^n,
 *                  stage-1 residuals; dt = given dt if dt > 0, else from the
 *                  CFL reduction of the stage-1 fluxes (kept on the device);
 *   sw_rk_stage(l), l = 2..s: stage-l state from the stored residuals
 *                  (Newton, discharge and tracer solves) and its residuals;
 *   sw_step_end:   final combination with the weights b and the solves.
 * sw_step runs the three; sw_run runs n steps. */
sw_status sw_step_begin(sw_ctx *c, double dt);
sw_status sw_rk_stage(sw_ctx *c, int32_t l);
sw_status sw_step_end(sw_ctx *c);
sw_status sw_step(sw_ctx *c, double dt);
sw_status sw_run(sw_ctx *c, int32_t n_steps, double dt);

/* ---- adjoint (vector-Jacobian products; the paper has no adjoint) ----
 * R(u) = (F, Gx, Gy) are the weak residuals of sw_apply_operator (without a
 * tracer); n_K the Manning coefficients and db_K the bed-elevation offsets of
 * sw_set_manning / sw_set_bed_offset.  Kinks take the forward's branch:
 * max(x, 0) has derivative 1 iff x > 0, ties of max/min (Rusanov speed,
 * z*_b = min(zb-, zb+), zeta* = max(zeta, -z*_b)) go to the A (interior) side,
 * d|x|/dx = sign(x) with sign(0) = 0; dry nodes give zero depth derivatives.
 *
 * sw_vjp_operator: for the state (eta, qx, qy) (device [n_dofs] each) and
 * adjoint residuals Fb, Gxb, Gyb (device [n_dofs]), writes
 * eta_b, qx_b, qy_b = (dR/du)^T (Fb, Gxb, Gyb) and n_bar, db_bar
 * (device [n_cells]) = (dR/dn)^T ..., (dR/ddb)^T ...; t is the time of the
 * elevation boundary.  Overwrites its outputs. */
sw_status sw_vjp_operator(sw_ctx *c, const double *eta, const double *qx, const double *qy, double t,
                          const double *Fb, const double *Gxb, const double *Gyb, double *eta_b, double *qx_b,
                          double *qy_b, double *n_bar, double *db_bar);
/* sw_step_record: one step with the fixed dt > 0 (as sw_step) that also
 * stores its stage states u^(1) = u^n, u^(2), ..., u^(s) into stages (device
 * [s][3][n_dofs]: zeta, qx, qy per stage) and, when end is not NULL, the
 * flow u^(n+1) of the final combination into end (device [3][n_dofs]), as it
 * stands before the next step's degree decision and remap (Sec. 3.3).
 * sw_vjp_step: adjoint of that step in the all-wet regime (every rule node wet
 * in every stage, every cell of degree r, no tracer), where the step is the
 * explicit map u^(l) = u^n + dt M^-1 sum_m a_lm R(u^(m)) of Sec. 3.1 with M the
 * all-wet rule mass matrix for zeta (eq:depth_rhs is affine there, so the
 * Newton solve of eq:newton is exact after one iteration) and the exact mass
 * matrix for q.  state_bar (device [3][n_dofs]) holds the adjoint of u^(n+1)
 * on entry and that of u^n on return; n_bar and db_bar (device [n_cells]) are
 * accumulated.  t is the step's start time.  A stage state outside the regime
 * makes the next sw_sync report SW_EDEVICE (code 4).  Uses the context's
 * residual storage: the next step recomputes its start-of-step terms. */
sw_status sw_step_record(sw_ctx *c, double dt, double *stages_dev, double *end_dev);
sw_status sw_vjp_step(sw_ctx *c, const double *stages_dev, double t, double dt, double *state_bar,
                      double *n_bar, double *db_bar);

/* ---- Dynamic h-adaptivity (Sec. 3.3 "Degree and h-adaptivity": refinement
 * criteria; Sec. 3.4: conservative remap, eq:cons-remap, and the mass source
 * Q^n of bathymetry re-sampling, eq:mass-loss) ---- */
enum { SW_AMR_VORTICITY = 0,   /* eta_K = max |curl u| (Sec. 4.4), u = q / h_des    */
                               /* (eq:velocity) by the chain rule with the depth   */
                               /* gradient grad zeta at wet nodes, 0 at dry ones   */
       SW_AMR_TRACER_GRAD = 1 };/* eta_K = max |grad c| (Sec. 5)                    */

typedef struct {
  int32_t indicator;         /* SW_AMR_*                                           */
  double theta_r, theta_c;   /* refine if eta_K > theta_r eta_max, coarsen if      */
                             /* eta_K < theta_c eta_max (eta_max over the mesh)    */
  int32_t n_max;             /* finest level n_K = level + 1 <= n_max (<= n_levels)*/
  double h_min;              /* no refinement of cells of size <= h_min (0: none) */
} sw_amr_params;

typedef struct {
  int64_t n_cells_old, n_cells_new;
  int64_t n_refined;         /* cells split (flagged or for the 2:1 balance)       */
  int64_t n_coarsened;       /* groups of four siblings merged                     */
  double eta_max;
  double mass_old, mass_new; /* sum_K int h before and after (sample rule)         */
  double q_bathy;            /* Q^n of eq:mass-loss: sum_K int z_b l over the new  */
                             /* cells minus the same over the old cells, l the     */
                             /* land-sea mask of the state on each mesh           */
  int32_t boundary_data_kept;/* 1: the given data of state and discharge sides   */
                             /* carried over (their faces are unchanged)          */
} sw_amr_stats;

/* Bathymetry raster: bed ELEVATION b_dev[j][i] (device, nx x ny, nx, ny >= 2)
 * at (x0 + i dx, y0 + j dy).  The library keeps a copy and samples it by
 * bilinear interpolation (clamped to the raster's edge outside it) at every
 * node of sw_node_coords, now and at the new cells of every sw_remesh; this
 * replaces sw_set_bathymetry (the bed offsets still apply). */
sw_status sw_set_bed_grid(sw_ctx *c, int32_t nx, int32_t ny, double x0, double y0, double dx, double dy,
                          const double *b_dev);
/* eta_K of every cell (device [n_cells]) at the state the next step starts
 * from, evaluated at the nodes of the volume integrals (the S x S sample
 * rule, or Table 1's Gauss-Legendre rule with SW_QUAD_PAPER). */
sw_status sw_amr_indicator(sw_ctx *c, int32_t indicator, double *eta_dev);
/* One remesh of a single-member context, between steps.  From the indicator
 * at the state the next step starts from: refine K if eta_K > theta_r eta_max,
 * n_K < n_max and its size exceeds h_min; merge four sibling leaves if all
 * have eta_K < theta_c eta_max and n_K > 1; the mesh stays 2:1 balanced
 * across faces (refinement wins: coarser face neighbours are refined until
 * no leaf faces one two levels finer, and a merge that would face such a
 * leaf is dropped).  The state (zeta, q, c) moves to the new cells by the
 * L2 projection (eq:cons-remap): a child takes its parent's polynomial, a
 * parent the exact-mass projection of its four children.  A child inherits
 * its parent's Manning coefficient and bed offset, a parent takes the mean
 * of its children's.  New cells are ordered by level, then row j, then
 * column i (sw_cells lists them); every cell starts at degree r; the
 * bathymetry of all cells is sampled from the raster of sw_set_bed_grid
 * (SW_EINVAL without one).  Time, time step, tide and CFL number carry over;
 * the boundary data of state and discharge sides carry over when the
 * faces that take them are unchanged (same cells and sides in the same
 * order; out->boundary_data_kept = 1) and must be given again otherwise
 * (sw_set_boundary_state), and the per-launch-shape choices of
 * sw_set_workgroup / sw_autotune return to their defaults.  All arrays sized
 * by the mesh change with it (sw_counts).  out (may be NULL) receives the
 * statistics.  The handle c stays valid; the call synchronises.  Errors:
 * SW_EINVAL (batched context, open step, bad parameters, no raster),
 * SW_ENOMEM, SW_EHIP; the context is unchanged on error. */
sw_status sw_remesh(sw_ctx *c, const sw_amr_params *params, sw_amr_stats *out);
/* Host outputs [n_cells]: level, i and j of every cell (any may be NULL). */
sw_status sw_cells(const sw_ctx *c, int32_t *level_host, int32_t *i_host, int32_t *j_host);
/* The mesh decision of sw_remesh on the host alone (no device work): for a
 * mesh (cells sorted by level) and its indicator values eta_host [n_cells],
 * the new leaves in sw_remesh's order (level_host, i_host, j_host [cap]) and
 * where each takes its state from: type_host [cap] 0 (the same cell,
 * src_host[4n] = its old index), 1 (a child: src_host[4n] = the old parent,
 * src_host[4n+1] = 2 sy + sx of the child) or 2 (a parent: src_host[4n + 2 sy
 * + sx] = the old children).  *n_new receives the new cell count; with cap
 * below it the call returns SW_EINVAL and fills nothing else.  Output arrays
 * may be NULL. */
sw_status sw_amr_plan(const sw_mesh_desc *mesh, const double *eta_host, const sw_amr_params *params, int32_t cap,
                      int32_t *n_new, int32_t *level_host, int32_t *i_host, int32_t *j_host, int32_t *type_host,
                      int32_t *src_host, int64_t *n_refined, int64_t *n_coarsened);

/* sw_tracer_step: advances the context's tracer by one recorded step with
 * the flow given, not solved: the tracer solve of eq:algebraic_concentration
 * with H(zeta^(l)) and the tracer residual R (eq:r_concentration) of every
 * stage, where zeta^(l), q^(l) are read from stages (l = 2..s, as
 * sw_step_record writes them) and the final flow from end; the Newton and
 * discharge solves are skipped.  dt is the recorded step's dt (> 0).  The
 * context's flow must equal the recorded step's start state: set it with
 * sw_set_state (and sw_set_time) where the recording started, then call
 * sw_tracer_step once per recorded step in order; each call leaves the
 * context where the coupled step would (flow = end after the next step's
 * degree decision, tracer advanced, time + dt).  Recorded by a context with
 * a tracer, the replayed tracer equals the coupled run's bit for bit; a
 * record of a flow-only context may differ from it by rounding (its element
 * kernel sums in another order).  Requires params.tracer; the buffers are
 * read only. */
sw_status sw_tracer_step(sw_ctx *c, const double *stages_dev, const double *end_dev, double dt);
/* Several tracers (eq:shw with M > 1 passive tracers, each with its own
 * diffusion and decay): one step of the flow context with the fixed dt > 0,
 * recorded into buffers the flow context keeps (allocated on first use,
 * (s + 1) x 3 x n_dofs doubles), then the n tracer contexts stepped over
 * that record, each as sw_tracer_step would (bit for bit).  They take the
 * step stage by stage together: each stage of up to eight contexts is one
 * launch that factorises H(zeta^(l)) (eq:mass_matrix_concentration) once
 * per cell for all of them, on the sample rule, and so is the final
 * combination on the cells whose degree the end flow leaves unchanged.  The tracer contexts must
 * share the flow's mesh, degree and scheme, one quadrature and one degree
 * rule (h_lim, adapt_degree), and must not repeat (SW_EINVAL otherwise);
 * they start each call with the flow's state, which the call keeps in step
 * with the flow, and carry the flow's bathymetry.  The flow context may
 * carry the first tracer itself.  Every launch of the call runs on the flow
 * context's stream, after the tracer contexts' earlier work; their streams
 * wait for its end. */
sw_status sw_step_tracers(sw_ctx *flow, int32_t n, sw_ctx *const *tracers, double dt);
/* Tracers that react with each other: sw_step_tracers with the reactions
 * h phi_k(c_1, ..., c_n) of eq:shw, phi_k = sum_j B_kj c_j, between the n
 * tracer contexts (1 <= n <= 8), taken explicitly in every stage as
 * eq:imex_shw takes them.  react_host is B, n x n doubles row-major
 * (B_kj at react_host[k n + j], 1/s, finite), read during the call; NULL
 * runs sw_step_tracers.  The tracer contexts step stage by stage together:
 * after each stage's residuals, context k's tracer residual gets
 * sum_j B_kj int h c_j psi_i of that stage's states, integrated on the
 * volume rule with the plain depth, before any context takes the next
 * stage.  The tracer contexts carry the flow's bathymetry and state, so that
 * depth is taken from the first of them.  Each context's own decay (params.tracer_decay) and diffusion still
 * apply.  Every launch of the call runs on the flow context's stream, after
 * the tracer contexts' earlier work; their streams wait for its end (also
 * after a failure).  The contexts' requirements are sw_step_tracers'; the
 * flow context itself as a tracer context is SW_EINVAL. */
sw_status sw_step_tracers_react(sw_ctx *flow, int32_t n, sw_ctx *const *tracers, const double *react_host,
                                double dt);

/* Diagnostics of the last step (host output).  Synchronises.  In a batched
 * context dt and t are member 0's; masses and counts are summed, extrema
 * taken over the members.  sw_member_diagnostics gives one member's. */
sw_status sw_diagnostics(const sw_ctx *c, sw_diag *out_host);
sw_status sw_member_diagnostics(const sw_ctx *c, int32_t member, sw_diag *out_host);
/* Kernel timing.  With profiling on, each launch group of a kernel class is
 * bracketed by HIP events on the context's stream; sw_kernel_time returns the
 * accumulated milliseconds and kernel launches of one class (synchronises):
 *   kind 0: fast element kernel at step begin (degree decision, H^n, stage-1 volume terms)
 *   kind 1: fast element kernel of stages 2..s (solves + volume terms)
 *   kind 2: fast element kernel of the final combination (+ next step's start)
 *   kind 3: face kernel
 *   kind 4: general element kernel (cells the fast kernel leaves, tracer replays)
 *   kind 5: fast tracer kernel of stages 2..s (tracer solve and tracer residual of
 *           the cells the fast element kernel keeps)
 *   kind 6: fast tracer kernel at step begin and of the final combination (+ C~ of
 *           the next step).
 *   kind 7: reaction kernel of sw_step_tracers_react (counted on the first
 *           tracer context).
 * sw_kernel_time_reset clears the totals.  on = 0: off; 1: every class;
 * on = 1 | (mask << 1) with mask != 0: only the classes whose bit is set in
 * mask (fewer events, less perturbation).  The events are timing-only (no
 * system-scope fence at record). */
sw_status sw_profile(sw_ctx *c, int32_t on);
sw_status sw_kernel_time(sw_ctx *c, int32_t kind, double *ms_total, int64_t *launches);
sw_status sw_kernel_time_reset(sw_ctx *c);

/* Wait for the context's stream; reports SW_EDEVICE if a kernel flagged an error. */
sw_status sw_sync(sw_ctx *c);

/* Launch shape on one level (level < 0: all levels).  The element kernel's
 * shape does not change results; the face kernel's changes only the order in
 * which a face's node contributions are summed (rounding).  Kernel 0, the fast
 * element kernel: value = wavefronts per
 * workgroup (1, 2 or 4; a workgroup holds value * 64 / P cells, P the power
 * of two >= S_L; default 1); kernel 1, the face kernel: value = lanes per
 * face (2, 4 or 8; the S_L face nodes are split over them; default 4);
 * kernel 2, the order in which the fast element and tracer kernels hand cells
 * to the 8 XCDs: value = 0 (round robin, workgroup i on XCD i mod 8), 1 (one
 * contiguous range of cells per XCD) or -1 (default: 1 on single-level
 * meshes, 0 on quadtrees; sw_get_workgroup reports the value in effect);
 * results do not depend on it.
 * SW_EINVAL for other values.  sw_get_workgroup reads the current value. */
sw_status sw_set_workgroup(sw_ctx *c, int32_t level, int32_t kernel, int32_t value);
sw_status sw_get_workgroup(const sw_ctx *c, int32_t level, int32_t kernel, int32_t *value);
/* Autotuner of the launch shape: times `steps` steps (after one untimed step)
 * with every triple (fast-kernel wavefronts per workgroup in {1, 2, 4}) x
 * (face lanes per face in {2, 4, 8}) x (element order over the XCDs in
 * {0, 1}, as kernel 2 of sw_set_workgroup) on the context's current state,
 * keeps the fastest triple on every level and puts the state, degrees, times and time
 * steps back as they were (the next step recomputes its start-of-step terms;
 * results are unchanged).  dt as sw_step.  Allocates a snapshot of the state
 * while it runs.  Outputs (host, may be NULL): the chosen pair.  Synchronises. */
sw_status sw_autotune(sw_ctx *c, int32_t steps, double dt, int32_t *wpb_host, int32_t *lanes_host);
/* The element order the last sw_autotune (or sw_set_workgroup kernel 2) set:
 * read it with sw_get_workgroup(c, level, 2, &value). */

/* ---- ensembles of independent members (not part of the paper's method) ----
 * sw_ens_create groups the members into batched contexts (sw_create_batch),
 * one per set of shared parameters listed there, in order of first appearance;
 * the batches are created on `stream` (state I/O and setup calls on a batch use
 * it) and stepped on streams of their own, forked from and joined back to
 * `stream`, so that batches overlap on the device.  Errors as sw_create_batch. */
typedef struct sw_ens sw_ens;
sw_status sw_ens_create(sw_ens **out, int32_t n_members, const sw_mesh_desc *meshes, const sw_params *params,
                        void *stream);
void sw_ens_destroy(sw_ens *e);
/* Number of batches; batch b's context (owned by the ensemble: do not destroy)
 * and member count; batch and index inside the batch of member m. */
sw_status sw_ens_batches(const sw_ens *e, int32_t *n_batches);
sw_status sw_ens_batch(const sw_ens *e, int32_t b, sw_ctx **ctx, int32_t *n_members);
sw_status sw_ens_member(const sw_ens *e, int32_t m, int32_t *batch, int32_t *index);
/* n_steps steps of every member (dt > 0: that step for all, else each member's
 * CFL step).  use_graph = 1: one step of all batches is captured once into a
 * hipGraph (re-captured when dt changes) and replayed n times; a first step is
 * taken eagerly when a batch has just been (re)initialised.  Results equal the
 * eager path's bit for bit.  Work is enqueued on `stream`. */
sw_status sw_ens_run(sw_ens *e, int32_t n_steps, double dt, int32_t use_graph);
/* One step of every member with its CFL time step: sw_ens_run(e, 1, 0, use_graph). */
sw_status sw_ens_step(sw_ens *e, int32_t use_graph);
/* Wait for all work of the ensemble; SW_EDEVICE as sw_sync. */
sw_status sw_ens_sync(sw_ens *e);
/* Launch-shape autotuner of every batch (sw_autotune with `steps` timed
 * steps, on the batch's current state, which is restored).  cache_path (may
 * be NULL or empty): a text file of "<class> <wavefronts per workgroup>
 * <lanes per face>" lines, class "r<r>_S<S>"; classes found there are applied
 * without timing, new ones are timed and written back (the element order over
 * the XCDs is tuned for the timed classes only; cached classes keep the
 * default order).  Synchronises. */
sw_status sw_ens_autotune(sw_ens *e, int32_t steps, const char *cache_path);

#ifdef __cplusplus
}
#endif
#endif /* SW_H_ */
