/*
 * cem.h -- C ABI of the MI355X (gfx950) implementation of one explicit
 * SSP Runge-Kutta stage of the element-based convex limiting scheme for
 * Bernstein continuous Galerkin discretizations with WENO stabilization:
 *
 *   D. Kuzmin, H. Hajduk, J. Vedral, "An element-based convex limiting
 *   framework for continuous Galerkin methods with nonlinear
 *   stabilization", arXiv:2509.04673.  Equation numbers below follow the
 *   order of the arXiv source.
 *
 * Scope: uniform periodic boxes of cube cells in 1, 2 or 3 dimensions,
 * tensor-product Bernstein elements Q_p (p = 1..3, p = 1..2 in 3D), scalar
 * linear advection, the KPP flux (sin u, cos u) in 2D, the nonconvex flux of
 * Sec. 5.1.2 in 1D, and the compressible Euler equations of an ideal gas; in
 * 1D also non-periodic lines with weakly imposed boundary data
 * (cem_mesh_desc.bc).  Arithmetic is IEEE
 * float64.
 *
 * Conventions shared by every call
 *  - Every call returns a cem_status; 0 is success.  A failing call leaves a
 *    message for cem_last_error() (thread-local) and changes no state.
 *  - Device memory is owned by the caller.  The library never allocates or
 *    frees device memory: the state arrays and one workspace (size from
 *    cem_workspace_bytes) are bound with cem_bind.  Host memory passed in is
 *    only read or written during the call.
 *  - All GPU work is enqueued on the stream given to cem_create (a
 *    hipStream_t passed as void*, NULL = default stream) and is asynchronous
 *    unless a call is marked synchronous.  Asynchronous HIP failures surface
 *    at the next synchronous call as CEM_EHIP.
 *  - Nodal arrays are structure-of-arrays, component-major, float64:
 *        u[c * N + node],  node = i0 + L0 * (i1 + L1 * i2),  0 <= ik < Lk,
 *    with Lk = p * n[k] unique nodes per axis of the periodic box (the node
 *    at the upper end of an axis is the node at its lower end), or
 *    L0 = p * n[0] + 1 nodes on a non-periodic line.  Node
 *    (i0, i1, i2) carries the Bernstein coefficient whose nodal point is
 *    lo + h * (i0, i1, i2) / p.  Components: scalar problems m = 1; Euler
 *    m = d + 2 with (rho, rho v_1..rho v_d, rho E).
 */
#ifndef CEM_H
#define CEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CEM_OK = 0,
  CEM_EINVAL = -1, /* invalid argument, unsupported configuration, bad order of calls */
  CEM_EHIP = -2,   /* a HIP runtime call failed */
  CEM_ENOMEM = -3, /* bound workspace smaller than cem_workspace_bytes */
  CEM_ECFL = -4,   /* dt > min_e dt_e at some stage (eq. 23): retry with a smaller dt */
  CEM_EIDP = -5    /* an invariant-domain check failed beyond round-off */
} cem_status;

/* CEM_NONCONVEX: the 1D nonconvex flux of Sec. 5.1.2 (eq. 1dkpp-flux),
 * f(u) = u (1 - u) / 4 for u <= 1/2, u (u - 1) / 2 + 3/16 otherwise; dim 1
 * only (periodic or non-periodic lines). */
typedef enum { CEM_ADVECTION = 0, CEM_KPP = 1, CEM_EULER = 2, CEM_NONCONVEX = 3 } cem_physics_kind;

/* Arithmetic of a stage.  CEM_FP32_MIXED (d = 2, 3): the projected
 * gradient and mass-solve line operators, the WENO sensor (eqs. 7-8) and the
 * residual and element-contribution contractions (eq. 45) run in float with
 * float accumulation, on float copies of g, r, udot and the residual
 * vectors; the state, cell averages, facet fluxes and dt_e (eqs. 18, 40,
 * 42, 51), both limiters (eqs. 44, 53-55, Appendix A) and the update
 * (eq. 49) stay float64, so the invariant domain is kept exactly. */
typedef enum { CEM_FP64 = 0, CEM_FP32_MIXED = 1 } cem_precision;

/* Facet fluxes of the intermediate cell averages (Sec. 4.3, steps 3-4).
 * CEM_FLUX_LIMIT: the flux limiter of eqs. (44), (53) / Appendix A, with
 *   dt_e of eq. (40) (the method as presented).
 * CEM_FLUX_SUBCELL: limiter off, f_ee' = f^H of eq. (42), dt_e the subcell
 *   bound dt_e^max of Lemma 1 (eq. 37): over the boundary nodes i of K_e,
 *   min of m_i / (|c_i| lambda_0i) and m_0 / sum_i |c_i| lambda_0i, with
 *   c_i = int_dK phi_i n, lambda_0i the Riemann speed of (u_0, u_i) along
 *   c_i / |c_i|, u_0 the mean of the interior nodes (m_0 their lumped mass);
 *   for p = 1 (no interior node) u_0 = u^e, m_0 = |K_e| and the bound is
 *   halved.
 * CEM_FLUX_SHRINK: limiter off, f_ee' = f^H, dt_e of eq. (40) reduced to the
 *   largest value that keeps u^e - dt_e |dK|/|K| sum f^H . n admissible (the
 *   Remark after eq. 40; scalar: the global bounds, Euler: Appendix A with
 *   its margin eps_pos).  dt_e may reach 0, which a fixed dt reports as a
 *   CFL violation. */
typedef enum { CEM_FLUX_LIMIT = 0, CEM_FLUX_SUBCELL = 1, CEM_FLUX_SHRINK = 2 } cem_flux_mode;

/* Bounds of the scalar limiters (Sec. 4.1, 4.2 allow local or global ones).
 * CEM_BOUNDS_GLOBAL: [u_min, u_max] for every element.
 * CEM_BOUNDS_LOCAL: per element, [min, max] of the stage input's cell
 *   averages of K_e and its 2d facet neighbours; imposed on the
 *   flux-limited average ubar^e (eq. 53: each facet keeps both of its
 *   elements within their own bounds) and on every slope-limited state of
 *   the element (eq. 55, u_i^min/max taken as the element's bounds).  The
 *   range holds the low-order average ubar^{e,L} (eq. 51), so a zero
 *   limited flux is always admissible, and it lies inside [u_min, u_max].
 *   The flux modes other than CEM_FLUX_LIMIT keep the global bounds for
 *   dt_e (the Remark after eq. 40).  Ignored for Euler. */
typedef enum { CEM_BOUNDS_GLOBAL = 0, CEM_BOUNDS_LOCAL = 1 } cem_bounds_mode;

/* Antidiffusive element contributions f_i^e.
 * CEM_CONTRIB_AEC: eq. (45), the contributions that recover the stabilized
 *   high-order scheme (every degree).
 * CEM_CONTRIB_Q1: the Q1 form of Sec. 5.3, gamma_e (m_i^e (u_i - u^e) -
 *   dt_e [int (phi_i - m_i^e/|K|) div f_h + int phi_i (udot_h^L -
 *   udot_i^L)]), with udot^L the time derivative of the low-order scheme
 *   of Sec. 3 (lumped mass, element-averaged flux divergence and the
 *   Rusanov term with the element's pseudo time step; b_i = 0 on the
 *   periodic box).  Degree 1, scalar problems, float64, single problems
 *   only (CEM_EINVAL otherwise).  The stage still computes g, r and the
 *   consistent-mass solve (debug taps 0, 1), and tap 2 then holds udot^L.
 *   The entropy correction of Sec. 5.3.2 is not provided: its nodal sensors
 *   are defined only in the cited work. */
typedef enum { CEM_CONTRIB_AEC = 0, CEM_CONTRIB_Q1 = 1 } cem_contrib;

/* Boundary conditions of a non-periodic line (eq. ibvp: f(u) . n =
 * F(u, u_hat; n) on the boundary, imposed weakly through the boundary term
 * b of eq. bidef, the boundary facet fluxes f^partial and F(u^e, u_hat^e';
 * n) of Sec. 4 and g_i^e of eq. aecb, with the LLF flux of eq. fluxLLF).
 * CEM_BC_PERIODIC: no boundary (both ends must be periodic together).
 * CEM_BC_STATE: u_hat is the conserved state given in bc_state (inflow or
 *   far-field data; an admissible state for Euler, a value inside the
 *   global bounds for scalar problems).
 * CEM_BC_OUTFLOW: u_hat = u (the boundary flux is f(u) . n).
 * CEM_BC_WALL: Euler only, u_hat = u with reversed momentum (a reflecting
 *   wall: no mass or energy crosses it).
 * At a boundary facet the low-order flux uses u_hat^e' = the boundary data
 * of the element's cell average, the WENO candidate of the missing
 * neighbour is absent, the flux limiter keeps only the element's bounds
 * (eq. 53 for e' > E_h) and local bounds include u_hat^e'. */
typedef enum { CEM_BC_PERIODIC = 0, CEM_BC_STATE = 1, CEM_BC_OUTFLOW = 2, CEM_BC_WALL = 3 } cem_bc_kind;

/* Uniform box [lo, hi] with n[k] cube cells per axis (cell edge h equal on
 * every axis; unused axes ignored).  n[k] >= 2.  Periodic unless bc says
 * otherwise: bc[0], bc[1] (cem_bc_kind) are the conditions at lo[0] and
 * hi[0] of a 1D line, both CEM_BC_PERIODIC (all zero: the periodic box) or
 * both non-periodic.  Non-periodic lines need dim = 1, CEM_FP64,
 * CEM_FLUX_LIMIT or CEM_FLUX_SHRINK and CEM_CONTRIB_AEC (the subcell bound
 * with boundary facets and the periodic Q1 form are not defined); the
 * batched form takes them with any boundary kinds per problem. */
typedef struct {
  int dim;       /* 1, 2 or 3 */
  int degree;    /* Bernstein degree p */
  int n[3];
  double lo[3], hi[3];
  int bc[2];               /* cem_bc_kind at lo[0] and hi[0] */
  double bc_state[2][5];   /* CEM_BC_STATE: conserved state (m values) at each end */
} cem_mesh_desc;

typedef struct {
  int kind;            /* cem_physics_kind */
  double velocity[3];  /* advection velocity (CEM_ADVECTION) */
  double gamma_gas;    /* ratio of specific heats (CEM_EULER), 1 < gamma <= 5/3 */
} cem_physics_desc;

/* Method parameters.  Modes: 0 = the method, 1 = force the factor to 0,
 * 2 = force it to 1 (the LO / HO / WENO / WENO-L switches of Sec. 5.3). */
typedef struct {
  double q;          /* steepening exponent of the sensor (eq. 7), >= 1 */
  double r;          /* exponent of the WENO weights */
  double eps;        /* epsilon of the WENO weights */
  double w_lin;      /* linear weight of each facet-neighbour candidate */
  double eps_pos;    /* strict-positivity margin of the Appendix A limiters */
  double clamp_ulps; /* scalar round-off clamp width in ulps of max|bound| */
  int gamma_mode;    /* WENO sensor gamma_e (eq. 7) */
  int alpha_mode;    /* flux limiter alpha_ee' (eqs. 44, 53 / Appendix A) */
  int beta_mode;     /* slope limiter beta_e (eqs. 54-55 / Appendix A) */
  double u_min, u_max; /* global bounds of scalar problems (Sec. 4.1, 4.2) */
  int precision;       /* cem_precision */
  int flux_mode;       /* cem_flux_mode */
  int bounds;          /* cem_bounds_mode */
  int contrib;         /* cem_contrib */
} cem_params;

typedef struct cem_ctx cem_ctx;

/* Pseudo time step statistics and invariant report.  The invariant domain
 * G is the one Theorem 1 (Sec. 3.3) preserves: u_min <= u <= u_max for
 * scalar problems (global bounds, Sec. 4.1-4.2), rho > 0 and p > 0 for the
 * Euler equations (Sec. 5.2, Appendix A).  Every test is written so that a
 * NaN fails it; extrema propagate NaN. */
typedef struct {
  double dt;             /* global time step of the current/last step (eq. 23) */
  double min_dt_e;       /* min over elements and stages of dt_e (eq. 40 / 37) */
  int cfl_violated;      /* 1 if dt > min_e dt_e at some stage (eq. 23) */
  long long clamped;     /* stage results clamped by <= clamp width (round-off) */
  long long violations;  /* stage results outside G beyond round-off, summed
                            over the stages since the last reset: scalar
                            values outside [u_min - tol, u_max + tol] or NaN;
                            Euler nodes with !(rho > 0), plus nodes with
                            !(p > 0) (each failed condition counts once) */
  int m;                 /* number of components */
  double u_min[5], u_max[5];   /* per-component extrema of the state */
  double mass[5];        /* per-component sum_i m_i u_i (lumped masses) */
  double rho_min, p_min; /* Euler: smallest density and pressure */
  long long nonfinite;   /* state values that are NaN or infinite */
  long long state_violations; /* failed conditions of G in the current state,
                            counted as for violations (at the time of the
                            check, also without any stage run) */
} cem_invariants;

/* Fills p with the defaults: q = 1, r = 2, eps = 1e-12, w_lin = 1e-3,
 * eps_pos = 1e-10, clamp_ulps = 64, all modes 0, bounds (-inf, +inf),
 * precision CEM_FP64, flux_mode CEM_FLUX_LIMIT, bounds CEM_BOUNDS_GLOBAL,
 * contrib CEM_CONTRIB_AEC. */
cem_status cem_params_default(cem_params* p);

/* Creates a context: validates the configuration and builds the element
 * tables on the host (Sec. 2.1: Bernstein basis; Sec. 2.2: semi-norm (8)).
 * Size limits: m * N < 2^31 and m (p+1)^d E < 2^31 (device index arithmetic
 * of the nodal arrays and of the element vectors is 32-bit below them).
 * stream: hipStream_t for all later work.  *out receives the context.
 * No GPU memory is touched until cem_bind. */
cem_status cem_create(const cem_mesh_desc* mesh, const cem_physics_desc* phys,
                      const cem_params* prm, void* stream, cem_ctx** out);

/* Sizes: N unique nodes, E elements, m components, and the workspace bytes
 * needed by cem_bind.  Any pointer may be NULL. */
cem_status cem_sizes(const cem_ctx* ctx, long long* N, long long* E, int* m);
cem_status cem_workspace_bytes(const cem_ctx* ctx, size_t* bytes);

/* Binds caller-owned device memory: u (m*N float64, the state, updated in
 * place by every stage), u_base (m*N float64, the state u^n at the start of
 * a step), workspace (>= cem_workspace_bytes, 256-byte aligned).  Copies the
 * tables into the workspace (asynchronous). */
cem_status cem_bind(cem_ctx* ctx, double* u, double* u_base, void* workspace, size_t ws_bytes);

/* Host <-> device copies of the state (host array m*N float64 in the nodal
 * layout).  upload is asynchronous but waits for the host buffer to be read;
 * download is synchronous. */
cem_status cem_upload_state(cem_ctx* ctx, const double* host_u);
cem_status cem_download_state(cem_ctx* ctx, double* host_u);

/* Global bounds for scalar problems (Sec. 4.1, 4.2).  from_state != 0 takes
 * the min and max of the bound state's coefficients (synchronous); else
 * u_min, u_max are used.  Ignored for Euler. */
cem_status cem_set_bounds(cem_ctx* ctx, int from_state, double u_min, double u_max);

/* One stage of Shu-Osher SSP-RK3 on the bound state (the five steps of
 * Sec. 4.3): stage s = 0, 1, 2 computes u <- a_s u_base + b_s u^FE(u) with
 * (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3) and u^FE the limited forward-Euler
 * update of eq. (49).  At s = 0 the step size is dt if dt > 0, else
 * cfl * min_e dt_e(u) (eq. 40), and it is kept for s = 1, 2.  Stage 0 does
 * not copy u to u_base; cem_step does.  Asynchronous: a CFL violation is
 * reported by cem_check_invariants. */
cem_status cem_rk_stage(cem_ctx* ctx, int stage, double dt, double cfl);

/* One SSP-RK3 step: u_base <- u, then stages 0, 1, 2.  Asynchronous.  By
 * default the three stages are captured once into a HIP graph (on a private
 * stream) and replayed on the context's stream; a new capture happens when
 * dt or cfl change, and after cem_bind / cem_set_bounds.  With kernel timing
 * enabled the stages are launched directly. */
cem_status cem_step(cem_ctx* ctx, double dt, double cfl);

/* Enables (default) or disables graph replay in cem_step. */
cem_status cem_set_graphs(cem_ctx* ctx, int enable);
/* Line kernels of the stage (projected gradient, Sec. 2.2; mass solve,
 * Sec. 4.3 step 2; the results agree to rounding): mode 0 the vector
 * kernels (LDS runs, all gradient axes in one launch), 1 tiles of 16 lines
 * on the matrix cores (the banded line operator as chains of 16x16x4
 * matrix products: float64, or float with float accumulation in the mixed
 * form), 2 (default) the matrix cores when a pass covers at least 2^20
 * values.  The assembly-fused first mass pass and lines too short for the
 * truncated operators keep their kernels.  Drops the captured step. */
cem_status cem_set_line_kernels(cem_ctx* ctx, int mode);
/* 2D Euler: with enable != 0 element pass 2 also performs the update (eq.
 * 49, SSP-RK3 combination, invariant counts) of the nodes whose elements
 * all lie in one of its blocks of consecutive elements, whose update
 * vectors then meet in LDS instead of being stored and re-read; the update
 * kernel handles the other nodes.  Node sums keep the same element order
 * and rounding, so both settings give bitwise the same states.  Off by
 * default: with blocks of 64 consecutive elements about half of the nodes
 * qualify, and the extra barriers of pass 2 cost what the update saves.
 * No effect on other problems.  Drops the captured step. */
cem_status cem_set_fused_update(cem_ctx* ctx, int enable);

/* Call after writing the bound state u by other means than
 * cem_upload_state or the stage calls (e.g. a device copy): derived per-node
 * data kept between stages (nodal fluxes of the KPP flux) is rebuilt. */
cem_status cem_state_modified(cem_ctx* ctx);

/* Synchronous: reads the step size, CFL flag and clamp/violation counters
 * accumulated since the last cem_reset_counters, and the state invariants
 * (Theorem 1: the stage results stay in G when dt <= min_e dt_e, eq. 23).
 * Returns CEM_EIDP when violations, state_violations or nonfinite is
 * nonzero, else CEM_ECFL when the CFL flag is set, else CEM_OK; *out is
 * filled in every case. */
cem_status cem_check_invariants(cem_ctx* ctx, cem_invariants* out);
cem_status cem_reset_counters(cem_ctx* ctx);

/* Copies an intermediate of the last stage into caller device memory dst
 * (asynchronous, count float64 values, count must equal the tap size):
 *   0 g [d][m][N]      1 r [m][N]        2 udot [m][N]    3 gamma [E]
 *   4 nu [E]           5 dt_e [E]        6 u^e [m][E]     7 ubar^{e,L} [m][E]
 *   8 ubar^e [m][E]    9 beta [E]       10 f^A of the +e_k facet [d][m][E]
 *  11 element update vectors [m][(p+1)^d][E]   (tap 1, r, is stored by
 *     cem_rk_stage; cem_step skips it where the assembly is fused with the
 *     first mass pass, as the batched form always does)
 *  12 local bounds of the scalar limiters [2][E] (lower, upper; written by
 *     the element pass only with CEM_BOUNDS_LOCAL) */
cem_status cem_debug_tap(cem_ctx* ctx, int tap, double* dst, size_t count);
size_t cem_tap_size(const cem_ctx* ctx, int tap);

/* Per-kernel timing: every launch of a kernel selected by mask (bit k =
 * kernel id k) is issued with a start and a stop HIP event that take the
 * dispatch's own begin and end timestamps (hipExtLaunchKernelGGL), so the
 * times are kernel execution times without launch latency.  While a mask is
 * set, cem_step launches directly instead of replaying a graph.  Ids:
 *   0 projected-gradient line operator   1 element pass 1 (sensor,
 *   residual, facets)   2 global time step from the per-block minima of
 *   dt_e (a launch of its own only on large meshes; otherwise inside 6)
 *   3 residual gather (fused with the first mass-solve pass on long
 *   x-lines)   4 mass-solve line operator   5 element pass 2 (limiters,
 *   contributions)   6 node update   7 element residual of the 3D Euler
 *   pass 1, a launch of its own there (id 1 is then its sensor and facet
 *   half).
 * cem_kernel_times is synchronous: it returns the summed milliseconds and
 * launch counts per id since the previous call (arrays of n <= 8 entries)
 * and clears them. */
#define CEM_NUM_KERNELS 8
cem_status cem_set_timing(cem_ctx* ctx, unsigned mask);
cem_status cem_kernel_times(cem_ctx* ctx, double* total_ms, long long* launches, int n);

void cem_destroy(cem_ctx* ctx);
const char* cem_last_error(void);

/* ---- No-allocation entry point -------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * cem_step_static runs nsteps SSP-RK3 steps exactly as cem_step does (the
 * same kernels, direct launches, the same results) on the caller's device
 * arrays u (the state, m*N float64, updated in place) and u_base (m*N
 * float64, distinct from u), with the workspace taken from a static device
 * array of CEM_STATIC_WORKSPACE_BYTES inside the library instead of a bound
 * workspace.  ctx needs cem_create only; a binding made with cem_bind, if
 * any, is set aside during the call and left as it was.  The call allocates
 * and frees no memory.  Scalar problems need finite bounds (cem_params
 * u_min/u_max, or an earlier cem_set_bounds).
 * Errors: CEM_ENOMEM when cem_workspace_bytes(ctx) exceeds the static size
 * (nothing is launched); CEM_EINVAL for bad arguments; CEM_EHIP.
 * Every GPU the library runs on holds one copy of the array until the
 * process ends, and every call on that GPU uses it and leaves it holding the
 * last call's data (the call itself sets the tables and zeroes its counters
 * first): calls that overlap on one GPU (other threads, other streams) race
 * and must be serialised by the caller.  The call's counters, dt and CFL
 * flag stay in the array and are not reported.  Asynchronous on the
 * context's stream (the table upload reads host memory before returning). */
#define CEM_STATIC_WORKSPACE_BYTES (64ll << 20)
cem_status cem_step_static(cem_ctx* ctx, double* u, double* u_base, double dt, double cfl, int nsteps);

/* ---- Batched form --------------------------------------------------------
 * count independent problems (uneven mesh sizes; the same dimension, degree,
 * physics, parameters and precision) advance together: every kernel of a
 * stage runs as ONE launch over all problems (blocks mapped to problems by a
 * prefix table), and a whole SSP-RK3 step is captured as one HIP graph and
 * replayed.  Each problem keeps its own time step (fixed dt, or cfl times
 * its own min_e dt_e, eq. 40) and its own counters.  Supported: d = 2 (all
 * physics), 3D Euler, both precisions; d = 1 in float64 (advection, Euler,
 * the nonconvex flux; periodic lines or lines with their own boundary
 * conditions, cem_mesh_desc.bc).
 *
 * State layout: problem k occupies [offsets[k], offsets[k+1]) of the
 * concatenated state arrays (its own component-major SoA block).
 * Ownership as for single problems: u, u_base and the workspace are device
 * memory owned by the caller; the batch allocates none. */
typedef struct cem_batch cem_batch;

/* Validates every problem (as cem_create) and sizes the workspace. */
cem_status cem_batch_create(int count, const cem_mesh_desc* meshes, const cem_physics_desc* phys,
                            const cem_params* prm, void* stream, cem_batch** out);
/* offsets: count + 1 entries (doubles from the start of u). */
cem_status cem_batch_offsets(const cem_batch* b, long long* offsets, int n);
cem_status cem_batch_workspace_bytes(const cem_batch* b, size_t* bytes);
/* u, u_base: device arrays of offsets[count] doubles; workspace 256-aligned. */
cem_status cem_batch_bind(cem_batch* b, double* u, double* u_base, void* workspace, size_t ws_bytes);
/* host arrays of offsets[count] doubles; synchronous. */
cem_status cem_batch_upload_state(cem_batch* b, const double* host_u);
cem_status cem_batch_download_state(cem_batch* b, double* host_u);
/* as cem_set_bounds, for every problem (scalar physics). */
cem_status cem_batch_set_bounds(cem_batch* b, int from_state, double u_min, double u_max);
/* nsteps SSP-RK3 steps of every problem; dt > 0 fixed, else cfl > 0. */
cem_status cem_batch_step(cem_batch* b, double dt, double cfl, int nsteps);
cem_status cem_batch_set_graphs(cem_batch* b, int enable);
cem_status cem_batch_reset_counters(cem_batch* b);
/* Sets the plan's knobs directly (those the autotuner searches): order 0
 * input / 1 largest first; xlines_cap values staged per block of the
 * x-line kernels (256 .. 65536); ytile_lds_bytes LDS bytes of a strided
 * line tile (8192 .. 65536); elem1_kernel 0 the 2D element LDS tile, 1 the
 * system kernels (Euler only; 3D Euler always takes them).  The next step
 * rebuilds the plan. */
cem_status cem_batch_set_plan(cem_batch* b, int order, int xlines_cap, int ytile_lds_bytes, int elem1_kernel);
/* Line kernels of the batch (projected gradient, Sec. 2.2; mass solve,
 * Sec. 4.3 step 2): matrix != 0 runs every fast-operator line pass except
 * the assembly-fused one as matrix-core tiles (the default; float64, or
 * float products with float accumulation in the mixed form), 0 as the
 * vector kernels.  The next step rebuilds the plan. */
cem_status cem_batch_set_line_kernels(cem_batch* b, int matrix);
/* as cem_set_fused_update, for the batched 2D Euler problems. */
cem_status cem_batch_set_fused_update(cem_batch* b, int enable);
/* Per-kernel timing of the batched launches, as cem_set_timing /
 * cem_kernel_times (the same kernel ids; each batched launch is one record,
 * covering every problem it serves).  While a mask is set, cem_batch_step
 * launches directly instead of replaying its graph.  cem_batch_kernel_times
 * is synchronous. */
cem_status cem_batch_set_timing(cem_batch* b, unsigned mask);
cem_status cem_batch_kernel_times(cem_batch* b, double* total_ms, long long* launches, int n);
/* one record per problem (n == count); returns EIDP if any problem failed an
 * invariant-domain check, else ECFL if any set its CFL flag. */
cem_status cem_batch_check_invariants(cem_batch* b, cem_invariants* out, int n);
/* Autotuner of the batched launches: a coordinate search over the plan's
 * knobs from the current plan, each knob in turn over its values with the
 * others at their best so far, timing `steps` steps of each candidate from
 * the current state.  Knobs: problem order (input, largest first); values
 * staged per block of the x-line kernels (512 .. 4096, lines per block);
 * LDS bytes of a strided line tile (20, 40, 56 KiB: one, two or four runs
 * per thread along the line, or the row groups of a matrix-core tile); for
 * 2D Euler the element pass-1 kernel (the 16 x 8 element LDS tile with one
 * thread per element, or element blocks with one thread per element and
 * component); the line kernels (matrix-core tiles or vector runs,
 * cem_batch_set_line_kernels).  Keeps the fastest plan and
 * restores the state.  scratch: caller-owned device memory of at least
 * offsets[count] doubles (the saved state).  report (optional): a JSON
 * record of every trial and the choice, NUL-terminated, truncated to
 * report_cap bytes.  Synchronous; resets the counters. */
cem_status cem_batch_autotune(cem_batch* b, double dt, double cfl, int steps, void* scratch,
                              size_t scratch_bytes, char* report, size_t report_cap);
void cem_batch_destroy(cem_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* CEM_H */
