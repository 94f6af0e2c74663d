/*
 * nmg.h -- C ABI of libnmg, the MI355X (gfx950) Newton multigrid solver for steady shallow
 * water equations with third-order WENO finite volumes and a simplified block Jacobian
 * (Hu, Li, Wang, Wang, "A high-order Newton multigrid method with a simplified Jacobian for
 * steady-state shallow water equations").
 *
 * Every entry point is extern "C", takes plain pointers and sizes, and never throws.  Device
 * pointers are caller-owned device memory (hipMalloc or a torch tensor's data_ptr); host
 * pointers are marked "host".  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  All calls except nmg_newton_solve / nmg_plan_solve are asynchronous on `stream`;
 * errors a kernel produces later surface on the next call that synchronises.  On failure a
 * call returns a negative nmg_status and nmg_last_error() describes the cause (thread-local).
 * Outputs never alias inputs.
 *
 * Data layout (all FP64 unless the precision field says otherwise):
 *  - 1D state U: component-major [2][nx]: U[0*nx + j] = H_j = sigma h, U[1*nx + j] = Q_j
 *    (section 2, eq. 3-4).  2D state: [3][ny][nx] = (h, hu, hv) (eq. 1-2).
 *  - Residual R: same layout as U.  rn[j] = ||R_j||_1 (eq. 13).
 *  - Jacobian J (1D): block-entry-major [nb][2][2][nx]: J[((b*2 + l)*2 + m)*nx + j] =
 *    dR_j^l / dU_i^m with i = j + b - nb/2; nb = 3 (simplified J3) or 5 (full J5).
 *    Blocks whose column cell lies outside the grid are zero.
 *  - 2D Jacobian J9: [9][3][3][ny][nx], blocks ordered (centre, x-2, x-1, x+1, x+2, y-2, y-1,
 *    y+1, y+2) following eq. (21).  J21 (the full stencil): [21][3][3][ny][nx], the nine cross
 *    blocks first, then (x-2, x-1, x+1, x+2) on row y-1, the same on row y+1, then (x-1, y-2),
 *    (x-1, y+2), (x+1, y-2), (x+1, y+2).  Blocks whose column cell lies outside the grid are zero.
 */
#ifndef NMG_H
#define NMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nmg_status;
#define NMG_OK 0
#define NMG_NOT_CONVERGED 1   /* result valid, but res >= tol after n_max Newton steps */
#define NMG_EINVAL (-1)       /* bad argument: null pointer, size not m*2^(levels-1), ... */
#define NMG_ENOMEM_WS (-2)    /* workspace smaller than nmg_workspace_bytes() */
#define NMG_EHIP (-3)         /* HIP launch or runtime error */
#define NMG_ENONFINITE (-4)   /* NaN/Inf residual, or non-positive depth */

/* boundary kinds (per side) */
#define NMG_BC_DISCHARGE 0    /* prescribed discharge q; depth extrapolated unless supercritical (then h if > 0) */
#define NMG_BC_DEPTH 1        /* prescribed depth h when subcritical; discharge extrapolated */
#define NMG_BC_EXTRAP 2       /* zeroth-order extrapolation */
#define NMG_BC_WALL 3         /* reflective: mirror, normal momentum negated */
#define NMG_BC_STATE 4        /* prescribed state (h, u, v) (2D supercritical inflow) */

/* precision of the Jacobian and multigrid */
#define NMG_FP64 0
#define NMG_FP32_MG 1         /* J, D^-1, rhs and dU in FP32; residual, update and test in FP64 */

typedef struct {
    int32_t kind;
    int32_t pad;
    double q, h, u, v;
} nmg_bc;

/* Problem description (host struct; geometry arrays are device pointers).
 * 1D (dim = 1, section 3): nx cells on [x0, x1]; bc[0] left, bc[1] right.
 *   sig_face [nx+1]: channel width sigma at faces x_{j-1/2}, j = 0..nx.
 *   sig_gp, sigx_gp, bx_gp [2*nx]: sigma, d sigma/dx and d b/dx at the two Gauss points
 *   x_j -/+ dx/(2 sqrt 3) of cell j (entries 2j, 2j+1) -- the points of eq. (9).
 * 2D (dim = 2, section 4): nx*ny cells on [x0,x1]x[y0,y1]; bc[0..3] = left, right, bottom, top;
 *   the bottom side is EXTRAP for x < wall_x and WALL beyond when bc[2].kind == NMG_BC_WALL
 *   and wall_x > x0.  bx_gp, by_gp [ny][nx][2][2]: b_x, b_y at the tensor Gauss points
 *   (y point beta, x point gamma) of each cell.
 * levels = L + 1 grid levels (eq. 15 / 23), at most 16: nx (and ny) must be divisible by
 *   2^(levels-1), and the coarsest level may hold at most 256 cells in 1D (so 1D grids have
 *   4 <= nx <= 256 * 2^15 cells) and at most 40 in 2D (2D grids hold at most 2^28 cells);
 *   levels = 1 (1D, jac = 3) solves the regularised system directly (Algorithm 3, step 4).
 *   Newton-SOR plans (params->linear != NMG_LINEAR_MG) build no hierarchy and skip these
 *   level checks.
 * jac = 3 or 5 (1D), 9 or 21 (2D): which Jacobian blocks are assembled (section 3.3 / 4.1; 21
 *   is the full 2D stencil of NMGM-21, whose block SOR on the finest level uses nine colours
 *   (i mod 3) + 3 (j mod 3) since its diagonal neighbours share (i + j) mod 3; the coarse
 *   levels keep the five-point operators of eq. (24) either way).  On very
 *   fine 1D grids the three-block Newton iteration itself can fail where J5 converges: on a
 *   smooth hump flow it converged up to 2^19 cells and ended non-finite from 2^21 cells, where
 *   J5 took 14-16 steps; such a solve reports NMG_ENONFINITE.
 * recon (1D): NMG_RECON_CONSERVED reconstructs H as in section 3.1 (the paper's scheme, not
 *   well balanced).  NMG_RECON_SURFACE, for channels of constant width (the width arrays are
 *   then not read; width 1): WENO3 reconstructs the surface eta = H + zbar, the depths at a face
 *   are eta-/+ minus b at the face, and the source of eq. (9) is evaluated in the exactly equal
 *   split form -g [int (eta_h - eta_j) b_x + eta_j (b_{j+1/2} - b_{j-1/2}) - (b_{j+1/2}^2 -
 *   b_{j-1/2}^2) / 2] (eta_h the cubic through the four face values of eta, the integral by the
 *   same Gauss rule, eta_j = H_j + zbar_j), so a still surface is steady to rounding on any
 *   bottom.  Ghosts copy the surface where the conserved variant copies H (H_g = H_src +
 *   zbar_src - zbar_g).  It needs z_face [nx+1] (b at the faces) and z_avg [nx+4] (cell
 *   averages of b over cells -2..nx+1, ghosts included).
 * recon (2D): NMG_RECON_CONSERVED is the paper's scheme of section 4.1.  NMG_RECON_SURFACE: the
 *   characteristic WENO3 reconstructs (eta, hu, hv) with eta = h + zbar (zbar the cell average
 *   of b; the characteristic basis stays that of the two cells' (h, hu, hv)), the depth at a
 *   face Gauss point is eta there minus b at that point, a ghost that copies a cell's depth
 *   copies its surface instead (h_g = h_src + zbar_src - zbar_g), and the source of each Gauss
 *   line takes the split form -g [int (eta_h - eta_ij) b_x + eta_ij (b_+ - b_-) - (b_+^2 -
 *   b_-^2) / 2] (eta_h the cubic through the line's four face values of eta, b_-+ at the cell's
 *   faces on the line), so still water is steady to rounding on any bottom; with b = 0 it is
 *   the paper's scheme.  It needs z_avg [ny+4][nx+4] (cell averages of b over cells -2..nx+1 x
 *   -2..ny+1) and z_face: b at the two Gauss points y_j -+ dy/(2 sqrt 3) of the x faces
 *   x_{i-1/2}, i = 0..nx ([ny][nx+1][2]), followed by b at the two Gauss points
 *   x_i -+ dx/(2 sqrt 3) of the y faces y_{j-1/2}, j = 0..ny ([ny+1][nx][2]). */
#define NMG_RECON_CONSERVED 0
#define NMG_RECON_SURFACE 1
typedef struct {
    int32_t dim, nx, ny, levels, jac, recon;
    double x0, x1, y0, y1, g;
    nmg_bc bc[4];
    double wall_x;
    const double *sig_face;
    const double *sig_gp;
    const double *sigx_gp;
    const double *bx_gp;
    const double *by_gp;
    const double *z_face;
    const double *z_avg;
} nmg_desc;

/* Solver parameters (section 3.2, 3.4, 5): alpha regularisation (eq. 13), tau damping
 * (eq. 14), eps FD perturbation (eq. 12), omega SOR relaxation (eq. 19/22), nu1/nu2 symmetric
 * smoothing steps, nu3 V-cycles per Newton step, tol on res = mean ||R_j||_1, n_max Newton
 * steps.  check_every: Newton steps between host reads of the convergence state in
 * nmg_newton_solve / nmg_plan_solve (>= 1).
 * linear (2D): NMG_LINEAR_MG: nu3 V-cycles with the multicolour block SOR of eq. (22);
 * NMG_LINEAR_MG_SWEEPS: the same V-cycles smoothed by the paper's four directional sweeps D1-D4
 * of section 4.2 (x ascending with y ascending inside, x descending, both descending, y
 * descending), each a lexicographic block SOR with the oracle's results; a sweep runs the
 * hyperplanes i' + j' = h (3 i' + j' for jac = 21) of its order one after another in one
 * workgroup per level, so it is meant for grids of at most 65536 cells (larger grids return
 * NMG_EINVAL), for comparisons of Newton steps with the paper's smoother.
 * linear (1D): how each Newton step solves the regularised system.  NMG_LINEAR_MG: nu3 V-cycles
 * (Algorithm 2).  NMG_LINEAR_SOR / NMG_LINEAR_SOR_LEX: the Newton-SOR reference solver of
 * section 5.1.1 -- symmetric block SOR steps on the grid itself (multicolour, or the
 * lexicographic forward + backward sweep, which runs one workgroup per instance: one lane sweeps
 * through LDS chunks that the other lanes stage, for iteration-count comparisons), stopped once the l1 norm of the change of dU between two
 * successive steps (summed over cells and components) falls below sor_tol, or after sor_max
 * steps; levels is then ignored. */
#define NMG_LINEAR_MG 0
#define NMG_LINEAR_SOR 1
#define NMG_LINEAR_SOR_LEX 2
#define NMG_LINEAR_MG_SWEEPS 3
typedef struct {
    double alpha, tau, eps, omega, tol;
    int32_t nu1, nu2, nu3, n_max;
    int32_t precision;
    int32_t check_every;
    int32_t linear;
    int32_t sor_max;
    double sor_tol;
    int32_t schedule;   /* 2D launch schedule (NMG_SCHED2D_* bits, 0 the default); 1D ignores it */
    int32_t reserved;
} nmg_params;

/* 2D launch schedules: every choice gives the same results bit for bit (the same operations on
 * the same values in the same order); they differ in speed only, and nmg_autotune2d picks one.
 *   NMG_SCHED2D_ALT_FINEST: the finest level's colour passes take the other of the two forms of
 *     a pass (by default one thread per cell on the cross stencil, whose row loads then issue
 *     together, and three lanes per cell on the 21-cell stencil, one per row of its blocks);
 *   NMG_SCHED2D_ALT_COARSE: the same for the launched five-point levels;
 *   NMG_SCHED2D_NO_STREAM: no non-temporal loads (by default the finest level's passes stream
 *     the rows that the schedule evicts before it returns to them, when its operator is larger
 *     than the memory-side cache);
 *   NMG_SCHED2D_SMALL_BOTTOM: the one-workgroup bottom of the V-cycle starts at levels of at
 *     most 128 cells instead of 512. */
#define NMG_SCHED2D_ALT_FINEST 1
#define NMG_SCHED2D_ALT_COARSE 2
#define NMG_SCHED2D_NO_STREAM 4
#define NMG_SCHED2D_SMALL_BOTTOM 8
#define NMG_TUNE2D_CANDIDATES 16

typedef struct {
    int32_t iters;     /* Newton steps taken */
    int32_t status;    /* NMG_OK, NMG_NOT_CONVERGED or NMG_ENONFINITE */
    double res;        /* final res */
} nmg_stats;

/* The Newton state of a stepwise 2D solve as the device keeps it: res after the last step, the
 * steps taken, whether the iteration is still running (1) and its status (NMG_NOT_CONVERGED
 * while running, then NMG_OK, NMG_NOT_CONVERGED at n_max or NMG_ENONFINITE). */
typedef struct {
    double res;
    int32_t iters, active, status, reserved;
} nmg_newton_state;

/* Bytes of device workspace nmg_mg_vcycle and nmg_newton_solve need for this problem
 * (multigrid hierarchy, Jacobian, residual buffers, tables).  Only sizes and parameters are
 * read: the geometry pointers may be null, so a caller can budget memory before uploading
 * anything.  0 on invalid input. */
size_t nmg_workspace_bytes(const nmg_desc *desc, const nmg_params *params);

/* Residual of eq. (10) (1D, not divided by dx) or eq. (20) (2D) for every cell, the cell norms
 * rn[j] = ||R_j||_1 and res_dev[0] = (1/N) sum_j rn[j] (Algorithm 1).  U, R, rn, res_dev are
 * device pointers.  The 1D kernels divide by depths, widths and wave-speed differences with a
 * refined hardware reciprocal that assumes normal-range operands (a physical state: depths and
 * widths well above 1e-150); a zero or negative depth gives a non-finite residual, which the
 * Newton drivers report as NMG_ENONFINITE. */
nmg_status nmg_residual(const nmg_desc *desc, const double *U, double *R, double *rn,
                        double *res_dev, void *stream);

/* Finite-difference Jacobian of eq. (12) with the regularisation alpha*||R_j||_1*I of eq. (13),
 * assembled on the reduced stencil of section 3.3 (J3; desc->jac = 5 gives J5) or section 4.1
 * (J9; desc->jac = 21 gives the full J21).  R and rn must be nmg_residual's output for the same U.  J (device, FP64) receives the
 * blocks in the layout above. */
nmg_status nmg_jacobian_assemble_simplified(const nmg_desc *desc, const nmg_params *params,
                                            const double *U, const double *R, const double *rn,
                                            double *J, void *stream);

/* One multigrid V-cycle (Algorithm 2) for  sum_i J_ji dU_i = -rhs_j  with the regularised
 * Jacobian J (layout above), multicolour block SOR smoothing (eq. 19/22), restriction and
 * coarse operators of eq. (17)/(24), injection prolongation (eq. 18/25) and a direct solve on
 * the coarsest grid.  setup = 1 copies J into the workspace and builds every coarse operator
 * and diagonal inverse (needed once per J); setup = 0 reuses them.  rhs and dU (in/out) are
 * device arrays in the U layout; precision NMG_FP32_MG makes rhs/dU float arrays. */
nmg_status nmg_mg_vcycle(const nmg_desc *desc, const nmg_params *params, void *ws, size_t ws_bytes,
                         const void *J, const void *rhs, void *dU, int32_t setup, void *stream);

/* Autotuner of the 2D launch schedule: with the operator J (FP64, the 2D layout above) and the
 * right-hand side rhs (device, in params->precision) set up in the workspace once, every schedule
 * 0..NMG_TUNE2D_CANDIDATES-1 (params->schedule is ignored) runs one warm-up V-cycle and then
 * `cycles` timed V-cycles (HIP events on `stream`); ms[c] (host, NMG_TUNE2D_CANDIDATES entries)
 * receives the milliseconds per V-cycle and *best the fastest schedule, to be passed in
 * params->schedule.  2D only; synchronises `stream`; the workspace's correction is overwritten. */
nmg_status nmg_autotune2d(const nmg_desc *desc, const nmg_params *params, void *ws, size_t ws_bytes,
                          const double *J, const void *rhs, int32_t cycles, int32_t *best, double *ms,
                          void *stream);

/* Algorithm 1 driven to res < tol or n_max steps: each step assembles the Jacobian, runs nu3
 * V-cycles from dU = 0, updates U += tau dU (eq. 14) and re-evaluates res.  U (device) is the
 * initial guess on entry and the result on exit.  stats (host) and hist (host, res after each
 * step, up to max_hist entries; may be NULL) are filled on return.  Synchronises `stream`. */
nmg_status nmg_newton_solve(const nmg_desc *desc, const nmg_params *params, void *ws,
                            size_t ws_bytes, double *U, nmg_stats *stats, double *hist,
                            int32_t max_hist, void *stream);

/* Algorithm 1 for one 2D problem in pieces, for callers that interleave it with other work on
 * other streams (a server): nmg_newton2d_begin enqueues the residual of U (device) and the
 * initial Newton state in the workspace (sized by nmg_workspace_bytes); nmg_newton2d_steps
 * enqueues `steps` Newton steps (steps after the iteration has stopped leave U unchanged) and,
 * when state_out (host; pinned memory keeps the copy asynchronous) is not NULL, a copy of the
 * state after them.  Neither call waits for the device: synchronise `stream` (or an event
 * recorded on it) before reading state_out.  The results equal nmg_newton_solve's bit for bit.
 * Errors (bad arguments, NMG_ENOMEM_WS) are returned before anything is enqueued. */
nmg_status nmg_newton2d_begin(const nmg_desc *desc, const nmg_params *params, void *ws, size_t ws_bytes,
                              double *U, void *stream);
nmg_status nmg_newton2d_steps(const nmg_desc *desc, const nmg_params *params, void *ws, size_t ws_bytes,
                              double *U, int32_t steps, nmg_newton_state *state_out, void *stream);

/* ---- Newton solve without allocation ----------------------------------------------------
 * For callers that cannot allocate memory: code next to HIP graph capture, tight serving loops
 * and harnesses that forbid hipMalloc.  nmg_newton_solve_static is nmg_newton_solve with the
 * library's own device workspace instead of the ws argument: a static array of
 * NMG_STATIC_WS_MIB MiB that every GPU the library runs on holds from the library's load until
 * the process ends.  Same arguments and results otherwise (the same kernels, launched without a
 * HIP graph; the result is bitwise that of nmg_newton_solve).  It calls no hipMalloc, hipFree,
 * pinned-memory or other allocating HIP routine.  A problem whose nmg_workspace_bytes exceeds
 * the array returns NMG_ENOMEM_WS (64 MiB covers 1D grids up to about 2e5 cells and 2D grids up
 * to 256 x 128 in FP64, 512 x 256 with NMG_FP32_MG).  Every call on one GPU uses that GPU's one
 * array and leaves its contents behind (each call initialises what it reads): calls that overlap
 * on one GPU, from several threads or streams, race and must be serialised by the caller.
 * Synchronises `stream`. */
#define NMG_STATIC_WS_MIB 64
nmg_status nmg_newton_solve_static(const nmg_desc *desc, const nmg_params *params, double *U,
                                   nmg_stats *stats, double *hist, int32_t max_hist, void *stream);

/* ---- nested iteration (Algorithm 3, Appendix A) -----------------------------------------
 * nmg_interp_coarse_to_fine: the initial cell averages of a 1D grid from the solution on the
 * grid with half as many cells, eq. (A.1)-(A.2): Uc [2][nc] -> Uf [2][2 nc] (device).  The
 * first and last coarse cells (the appendix is silent there) average over their halves the
 * quadratic (A.1) of the neighbouring interior cell.  nc >= 3.
 * nmg_interp2d_coarse_to_fine: the same in two dimensions, eq. (A.3), whose formula the text
 * leaves unfinished: the tensor product of (A.1), so the fine averages are (A.2) along x in each
 * coarse row and then (A.2) along y, the end cells of both directions as in 1D:
 * Uc [3][nyc][nxc] -> Uf [3][2 nyc][2 nxc] (device); nxc, nyc >= 3, nyc <= 32767, nxc nyc <= 2^26;
 * other sizes or null pointers return NMG_EINVAL before any launch.
 * nmg_nested_solve: Algorithm 3 on a 1D or 2D problem given on ngrids nested grids: descs[g]
 * and params[g] describe grid g (g = 0 the finest; grid g has half the cells of grid g-1 in
 * each direction and ngrids - g levels, so the coarsest grid is solved by Newton with the direct
 * coarsest solve).  U[g] (device, [2][nx_g] or [3][ny_g][nx_g]) is grid g's state: U[ngrids-1]
 * holds the initial guess on entry;
 * every other grid starts from the interpolation of the next coarser solution.  stats[g]
 * (host) receives each grid's Newton statistics.  Returns the finest grid's status
 * (NMG_ENONFINITE as soon as a grid breaks down).  The workspace must hold
 * nmg_nested_workspace_bytes() (the largest grid's).  Synchronises `stream`. */
nmg_status nmg_interp_coarse_to_fine(const double *Uc, int32_t nc, double *Uf, void *stream);
nmg_status nmg_interp2d_coarse_to_fine(const double *Uc, int32_t nxc, int32_t nyc, double *Uf, void *stream);
size_t nmg_nested_workspace_bytes(const nmg_desc *descs, int32_t ngrids, const nmg_params *params);
nmg_status nmg_nested_solve(const nmg_desc *descs, int32_t ngrids, const nmg_params *params, void *ws,
                            size_t ws_bytes, double *const *U, nmg_stats *stats, void *stream);

/* ---- batched form: many independent 1D instances (any sizes) per launch ----------------
 * A plan fixes n instances (descs/params host arrays of length n) and the workspace layout.
 * nmg_plan_solve runs Algorithm 1 on all of them together: every kernel launch covers every
 * still-active instance; converged instances drop out without disturbing the others (no
 * cross-instance arithmetic, so each result is bitwise the same alone or in a batch).
 * U[k] (host array of device pointers) is instance k's state, updated in place.  use_graph = 1
 * captures one Newton step as a HIP graph and replays it. */
typedef struct nmg_plan nmg_plan;
nmg_status nmg_plan_create(const nmg_desc *descs, const nmg_params *params, int32_t n,
                           nmg_plan **out);
size_t nmg_plan_workspace_bytes(const nmg_plan *plan);
nmg_status nmg_plan_solve(nmg_plan *plan, void *ws, size_t ws_bytes, double *const *U,
                          nmg_stats *stats, int32_t use_graph, void *stream);
/* Run exactly `steps` Newton steps (or fewer for instances that stop earlier) without
 * re-initialising; nmg_plan_begin evaluates the initial residual.  For step-wise drivers such
 * as a serving loop.  active_out (host, length n; may be NULL) receives 1 for still-active
 * instances; stats (host, may be NULL) the per-instance state. */
nmg_status nmg_plan_begin(nmg_plan *plan, void *ws, size_t ws_bytes, double *const *U, void *stream);
nmg_status nmg_plan_steps(nmg_plan *plan, void *ws, int32_t steps, int32_t use_graph,
                          int32_t *active_out, nmg_stats *stats, void *stream);
/* nmg_plan_begin for instances that have already taken Newton steps under another plan (a
 * serving loop re-plans between steps as requests arrive and retire): n_done (host, length n)
 * holds each instance's step count so far, which must be below its n_max.  The residual is
 * re-evaluated from U[k]; with the same U it equals the value the previous step ended with, so
 * a solve split over several plans takes exactly the steps of an uninterrupted one. */
nmg_status nmg_plan_resume(nmg_plan *plan, void *ws, size_t ws_bytes, double *const *U,
                           const int32_t *n_done, void *stream);
void nmg_plan_destroy(nmg_plan *plan);

/* Kernel timing for benchmarks: with kernel = one of NMG_K_*, every later non-graph step
 * brackets each launch of that kernel with hipEvents on the launch stream (graph replays are
 * not instrumented; NMG_K_NONE switches timing off).  nmg_plan_profile_read returns the summed
 * event time in milliseconds and the number of timed launches since the last read, and resets
 * both.  The read synchronises the stream. */
#define NMG_K_NONE 0
#define NMG_K_JACOBIAN 1      /* finite-difference Jacobian (section 3.2-3.3) */
#define NMG_K_SMOOTH_PRE 2    /* finest-level pre-smoothing + restriction (eq. 17, 19) */
#define NMG_K_SMOOTH_POST 3   /* finest-level prolongation + post-smoothing (eq. 18, 19) */
#define NMG_K_RESIDUAL 4      /* residual (eq. 10) */
#define NMG_K_COARSEN 5       /* coarse operators of all levels (eq. 17) */
#define NMG_K_SMOOTH_FUSED 6  /* finest level: post-smoothing of one V-cycle + pre-smoothing of the next */
nmg_status nmg_plan_profile(nmg_plan *plan, int32_t kernel);
nmg_status nmg_plan_profile_read(nmg_plan *plan, double *ms, int32_t *launches);

/* Tunables of a plan.  They choose between kernels that do the same arithmetic in the same
 * order, so results do not depend on them; a zero-initialised struct (with bottom_cells set)
 * selects the defaults.
 *   bottom_cells: the levels of each instance with at most this many cells (256, 512, 1024 or
 *     2048; the coarsest level always) run in the one-workgroup-per-instance bottom-of-cycle
 *     kernel, whose workgroup size follows (bottom_cells / 2, at least 256, at most 1024); the
 *     larger levels run in the tiled smoothers.  A small value spreads more levels over the
 *     whole GPU, a large one saves launches and synchronisation.  Default 2048.
 *   smooth_tile: cells (= threads) per tile of the tiled smoother, 256 or 512 (0: 256).
 *   split_finest: 0 (default) runs the finest level's post-smoothing of one V-cycle and the
 *     pre-smoothing of the next in one launch where the plan allows it (multigrid plans with
 *     nu3 >= 2 whose instances all use the three-block Jacobian); 1 keeps them apart.
 *   fused_finest: reported by nmg_plan_get_options (1 when that fused launch is in use),
 *     ignored by nmg_plan_set_options.
 *   split_residual: 0 (default) evaluates the residual of eq. (10) and its cell norms inside the
 *     Jacobian launch that ends each Newton step (the Jacobian the next step needs; an instance
 *     that then meets the stopping test leaves it unused); 1 ends each step with a separate
 *     residual launch and starts the next with the Jacobian, which reads it.
 * Setting options refreshes the plan's device tables (and any captured graph) on its next use;
 * the workspace size does not change.  Set them before nmg_plan_begin / nmg_plan_solve.  An
 * invalid set is rejected with NMG_EINVAL and leaves the plan as it was. */
typedef struct {
    int32_t bottom_cells;
    int32_t fused_finest;
    int32_t smooth_tile;
    int32_t split_finest;
    int32_t split_residual;
    int32_t reserved[3];
} nmg_plan_options;
nmg_status nmg_plan_set_options(nmg_plan *plan, const nmg_plan_options *opt);
nmg_status nmg_plan_get_options(const nmg_plan *plan, nmg_plan_options *opt);

/* Autotuner for the batched form: for every candidate option set (NMG_TUNE_CANDIDATES of them,
 * candidate c: bottom_cells = 256 << (c % 4), split_finest = (c / 4) % 2, smooth_tile =
 * 256 << ((c / 8) % 2), split_residual = c / 16) it begins the plan's instances from the states U, runs one untimed Newton step
 * (with use_graph = 1 it also captures the step graph) and times trial_steps more with HIP
 * events; it keeps the fastest set in the plan and returns it in best (host, may be NULL) and
 * the per-step milliseconds of every candidate in times_ms (host, length NMG_TUNE_CANDIDATES,
 * may be NULL).  The states are restored before it returns (it allocates a device copy of them
 * for the duration of the call).  Synchronises `stream`. */
#define NMG_TUNE_CANDIDATES 32
nmg_status nmg_plan_autotune(nmg_plan *plan, void *ws, size_t ws_bytes, double *const *U,
                             int32_t trial_steps, int32_t use_graph, nmg_plan_options *best,
                             double *times_ms, void *stream);

/* A stream for one lane of a server (the batched 1D lane, each 2D worker) on a hardware queue
 * of its own.  The runtime spreads ordinary streams over a few hardware queues (four by
 * default), so two streams can share one and the kernels of one then wait behind those of the
 * other: a long 2D solve would hold up every launch of the latency-bound 1D batch.  A stream
 * made with a compute-unit mask gets a queue that no other stream shares; the mask here enables
 * every compute unit of the current device, so the stream runs anywhere on the GPU.  Like a
 * blocking stream it orders with the null stream: a lane should not share work with the null
 * stream.  *stream (host) receives the handle, owned by the caller and released with
 * nmg_lane_stream_destroy (which waits for its work).  NMG_EHIP if the runtime refuses. */
nmg_status nmg_lane_stream_create(void **stream);
nmg_status nmg_lane_stream_destroy(void *stream);

/* Description of the last error on the calling thread ("" if none). */
const char *nmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NMG_H */
