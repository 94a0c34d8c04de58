/*
 * chanflow: single-GPU (MI355X, gfx950) pressure-Poisson projection solver for
 * incompressible channel flow, after the FFT + tridiagonal method of
 * "A low-communication-overhead parallel method for the 3D incompressible
 * Navier-Stokes equations" (arXiv 2104.08863).
 *
 * Geometry (Section 2, Fig. 1-2): x streamwise and z spanwise are periodic and
 * uniform (lengths lx, lz; nx, nz cells); y is wall-normal, bounded by two
 * no-slip walls, with an arbitrary stretched grid given by its ny+1 face
 * coordinates.  Variables are staggered (Fig. 2): p at cell centres, u on
 * x-faces, v on y-faces, w on z-faces.
 *
 * Every field is a C-order array of shape (ny, nz, nx), x fastest:
 *   p[j][k][i]  at (x_i,       yc_j,        z_k)
 *   u[j][k][i]  at (x_{i+1/2}, yc_j,        z_k)
 *   v[j][k][i]  at (x_i,       y_faces[j+1], z_k)   (v[ny-1] is the top wall:
 *                                                 its stored values are ignored
 *                                                 on input and written as 0)
 *   w[j][k][i]  at (x_i,       yc_j,        z_{k+1/2})
 * Spectral arrays (test hooks only) are complex (re, im interleaved) of shape
 * (nx/2+1, ny, nz), z fastest, holding the unnormalised forward transform: the
 * wall-normal line of wavenumbers (kx, kz) is fhat[kx][:][kz].
 *
 * Conventions for every call:
 *   - Pointers to fields are DEVICE pointers on the plan's device, 16-byte
 *     aligned, contiguous; the caller owns them.  y_faces is a HOST pointer.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the
 *     default stream).  Argument errors are returned synchronously before any
 *     work is enqueued; a failed launch returns CF_ERR_DEVICE.  Nothing aborts
 *     or throws across this interface.  cf_last_error() returns a message for
 *     the last failure on the calling thread.
 *   - A plan owns all device tables and workspace; calls do not allocate.  A
 *     plan must not be used from two streams at once.
 */
#ifndef CHANFLOW_H
#define CHANFLOW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cf_plan cf_plan;

typedef enum {
  CF_OK = 0,
  CF_ERR_ARG = 1,          /* bad pointer, size, alignment or grid */
  CF_ERR_UNSUPPORTED = 2,  /* sizes outside the supported transform/partition set */
  CF_ERR_NOMEM = 3,        /* device allocation failed at plan creation */
  CF_ERR_DEVICE = 4,       /* a HIP call or launch failed */
  CF_ERR_NUMERIC = 5       /* non-finite values detected (cf_plan_numeric_status) */
} cf_status;

enum { CF_FP64 = 0, CF_MIXED = 1 };

typedef struct {
  int precision;      /* CF_FP64 (all arithmetic FP64) or CF_MIXED (FP32 transforms and
                         bulk wall-normal solves, FP64 low-wavenumber lines and residual) */
  int n_parts;        /* PDD partitions P per wall-normal line; 0 = automatic.  Each
                         partition has M = ceil(ny/P) rows, M one of 1,2,3,4,6,8,12,16
                         (CF_MIXED: also 24, 32), with (P-1)*M < ny; when P does not
                         divide ny the last partition is padded with decoupled rows */
  double drop_tol;    /* lines whose PDD corner terms are all <= drop_tol use the dropped
                         (2x2) reduced system; the others the exact one.  < 0 = default
                         (1e-15 FP64, 1e-7 mixed) */
  int fp64_kx;        /* CF_MIXED: lines with kx < fp64_kx and min(kz, nz-kz) < fp64_kz */
  int fp64_kz;        /*   are solved in FP64 (default 4, 4) */
  int refine_passes;  /* CF_MIXED: FP64 residual + correction solves (default 1; one pass
                         reaches <= 1e-6 relative on grids up to ny = 768 as tested, at
                         the largest ny two are needed: 1.3e-6 and 8.5e-9 at ny = 2048) */
  int flags;          /* CF_PLAN_STEP: allocate the projection-step workspace;
                         CF_PLAN_ADJOINT: also the workspace of its adjoint;
                         CF_PLAN_Y_DCT, CF_PLAN_TUNE_PARTS: see below */
  int lines_per_block; /* lines per block of the partitioned solve; 0 = automatic.
                          lines_per_block * n_parts must be <= 512 */
  int drop_parts;     /* G: the dropped reduced system is an outer PDD of G partitions, each a
                         group of n_parts/G consecutive partitions solved exactly inside
                         (Section 2.2 with G partitions); the corner terms of the G-level
                         Eq. (21) are what drop_tol bounds.  Must divide n_parts.  0 =
                         automatic: 4 when 4 divides n_parts, else n_parts */
} cf_options;

/* CF_PLAN_Y_DCT: solve the wall-normal systems by a transform along y instead of
   the partitioned tridiagonal solve (the fully spectral variant for uniform
   spacing, Section 2.1).  Needs uniform y faces (spacing equal to 1e-12
   relative), CF_FP64, and an even ny of the form 2^a or 3*2^a, at most 2048. */
/* CF_PLAN_TUNE_PARTS: choose the partitioning by measurement (Section 2.2 leaves
   the count P and the placement to the solver): at creation the plan times the
   partitioned solve for every admissible P (M = ceil(ny/P) in {1,2,3,4,6,8,12,16},
   in CF_MIXED also 24 and 32, (P-1)*M < ny, P <= 64) and every block of lines_per_block = 4, 8, ..., 256 lines with
   64 <= lines_per_block * P <= 512 that fits in LDS (five launches each, after
   two warm-up launches, in place on zeros in the plan's workspace), keeps the
   fastest and sets the drop threshold for its P (each candidate's accuracy
   follows drop_tol, so the choice affects speed, not the error bound).  Needs
   n_parts = 0, lines_per_block = 0 and the partitioned solve (no CF_PLAN_Y_DCT);
   the timings are read back with cf_plan_tuning.  Takes tens of milliseconds
   on large grids. */
enum { CF_PLAN_STEP = 1, CF_PLAN_ADJOINT = 2, CF_PLAN_Y_DCT = 4, CF_PLAN_TUNE_PARTS = 8 };

typedef struct {
  int nx, ny, nz, precision;
  int n_parts;            /* partitions per line (P) */
  int rows_per_part;      /* M = ceil(ny / P) */
  long long n_lines;      /* (nx/2+1) * nz */
  long long n_drop_lines; /* lines whose corner terms fall below drop_tol */
  long long n_special;    /* lines solved by whole-line FP64 Thomas */
  double k2_threshold;    /* modified-wavenumber^2 above which the drop is allowed */
  size_t workspace_bytes; /* device memory owned by the plan */
  int lines_per_block;    /* lines per block of the partitioned solve */
  size_t slab_iface_bytes; /* device bytes of the interface buffer of cf_solve_spectral_slabs:
                              n_parts * 8 * n_lines values of the plan's precision */
  int drop_parts;         /* G, the outer partitions of the dropped reduced system */
  long long n_dropped_lines; /* lines the partitioned solve drops the corner terms for: those
                              whose block of lines_per_block consecutive lines lies wholly
                              above k2_threshold (the others take the exact reduced system) */
} cf_plan_info;

/* Fill *opt with the defaults. */
void cf_options_default(cf_options* opt);

/*
 * Create a plan on the current HIP device (Section 2 problem setup: Eq. (8)-(9)
 * operator, modified wavenumbers, PDD partitioning of Section 2.2).
 * nx, nz: even, 2^a or 3*2^a, nx/2 and nz in [2, 2048] (nz >= 2).
 * ny >= 2, split into P <= 64 partitions of M = ceil(ny/P) rows with M in
 * {1,2,3,4,6,8,12,16} (CF_MIXED: also 24, 32) and (P-1)*M < ny: any ny up to
 * 1024 (CF_MIXED: 2048).  The automatic P is the fewest partitions that divide
 * ny, preferring powers of two, else the partitioning with the fewest padding
 * rows (the rows P*M - ny that complete the last partition: no-flux rows below
 * the top wall row, decoupled from the line).
 * y_faces: host, ny+1 strictly increasing finite values (walls at both ends).
 * opt: NULL for defaults.  On success *out receives the plan; on failure *out is
 * set to NULL and nothing is leaked.
 */
cf_status cf_plan_create(cf_plan** out, int nx, int ny, int nz, double lx, double lz,
                         const double* y_faces, const cf_options* opt);

/* Release a plan and its device memory (synchronises the device).  NULL-safe. */
void cf_plan_destroy(cf_plan* plan);

cf_status cf_plan_query(const cf_plan* plan, cf_plan_info* info);

/*
 * The timings a CF_PLAN_TUNE_PARTS plan took at creation: *count receives the
 * number of (P, lines_per_block) candidates timed (0 for a plan created without
 * the flag); the first min(cap, *count) entries of the host arrays parts,
 * lines_per_block and us (mean microseconds per launch) receive them, in the
 * order timed.  The arrays may be NULL when cap is 0.
 */
cf_status cf_plan_tuning(const cf_plan* plan, int cap, int* count, int* parts, int* lines_per_block,
                         double* us);

/*
 * Pressure-Poisson solve (Eq. (7)-(9), Section 3.2 steps (2)-(8)):
 * p = the unique solution of L_h p = f - mean_W(f) with mean_W(p) = 0, where
 * L_h = D o G is the staggered 7-point Laplacian (Neumann walls) and
 * mean_W(q) = sum_j dy_j q_j / (nx nz sum_j dy_j).
 * f, p: device double arrays (ny, nz, nx); p may be f itself (in place) but
 * must not overlap it otherwise (CF_ERR_ARG).
 * CF_MIXED plans compute in FP32 with FP64 low-wavenumber lines and the FP64
 * residual-correction passes of the plan; f and p stay double (while the solve
 * runs, p holds intermediate values).
 */
cf_status cf_poisson_solve(cf_plan* plan, const double* f, double* p, void* stream);

/*
 * Divergence right-hand side (Eq. (7), Section 3.2 step (1)):
 * f = scale * [ (u_i - u_{i-1})/dx + (v_j - v_{j-1})/dy_j + (w_k - w_{k-1})/dz ],
 * v = 0 on both walls.  u, v, w, f: device double arrays (ny, nz, nx); f must not
 * overlap u, v or w (CF_ERR_ARG).
 */
cf_status cf_divergence(cf_plan* plan, const double* u, const double* v, const double* w,
                        double* f, double scale, void* stream);

/*
 * One projection step (Section 2, Eq. (3)-(7)): explicit RK2 (Heun, Eq. (5)-(6)) of
 *   du/dt = R(u) = -N(u) + nu lap(u) + fx e_x
 * giving u*, then the pressure solve L_h p = D u* / dt and u1 = u* - dt G p (Eq. (4)),
 * so that D u1 = 0 to round-off.  N(u) = div(u u) in flux form (linear interpolation,
 * the y-interpolation to a face weighted by the two cell heights); lap uses the no-slip
 * ghost mirrored about the wall; v = 0 on both walls.
 * u, v, w: device inputs (ny, nz, nx); u1, v1, w1: outputs (may alias the inputs,
 * must not overlap each other); p: device double output (ny, nz, nx), not
 * overlapping any velocity array, or NULL (pressure kept in the plan workspace).
 * Overlaps that are not allowed return CF_ERR_ARG before anything runs.
 * Velocity arrays are double for CF_FP64 plans and float for CF_MIXED plans.
 * The plan must have been created with CF_PLAN_STEP in opt->flags.
 */
cf_status cf_projection_step(cf_plan* plan, const void* u, const void* v, const void* w, void* u1,
                             void* v1, void* w1, double* p, double dt, double nu, double fx,
                             void* stream);

/*
 * The RK2 predictor of cf_projection_step alone (test hook; Section 2, Eq. (5)-(6)):
 *   ub = u + dt R(u),  u* = (u + ub)/2 + dt/2 R(ub),
 * written to (us, vs, ws); the top-wall v plane of the output is 0.  Arrays and
 * precision as in cf_projection_step; outputs that do not overlap the inputs take
 * the fused single-pass kernel, overlapping ones the two split stages.  The plan
 * must have been created with CF_PLAN_STEP.
 */
cf_status cf_rk2_predictor(cf_plan* plan, const void* u, const void* v, const void* w, void* us, void* vs,
                           void* ws, double dt, double nu, double fx, void* stream);

/*
 * Plane statistics of a velocity field (the quantities a channel-flow run
 * averages, Section 5): for every y-plane j the means over the x-z plane of the
 * stored u, v, w and of their squares, summed in FP64:
 *   stats[6 j + 0..2] = <u>_j, <v>_j, <w>_j,  stats[6 j + 3..5] = <u^2>_j, <v^2>_j, <w^2>_j
 * (v's plane j is the face above cell j; its top-wall plane is taken as stored).
 * u, v, w as in cf_projection_step; stats: device double (ny, 6), overwritten, not
 * overlapping u, v or w (CF_ERR_ARG).
 * Bitwise repeatable (fixed reduction order, no atomics).
 */
cf_status cf_plane_stats(cf_plan* plan, const void* u, const void* v, const void* w, double* stats,
                         void* stream);

/*
 * A time loop of nsteps projection steps (Section 2) starting from (u, v, w).
 * The state alternates between (u, v, w) and the second set (u2, v2, w2) (same
 * shape and precision, not overlapping the first), so every step writes
 * separate arrays and takes the fused RK2 pass; the newest state ends in
 * (u, v, w) when nsteps is even and in (u2, v2, w2) when it is odd.  After every
 * stats_every-th step (0: never) the plane statistics of the new state (the
 * quantities of cf_plane_stats, summed by the step's correction pass itself in
 * a fixed chunk order, so equal to cf_plane_stats up to rounding) are added into
 * stats_acc (device double (ny, 6)); the caller
 * clears it and divides by the number of samples.  p: optional device double
 * (ny, nz, nx) receiving the last step's pressure, or NULL.
 * use_graph != 0 replays the steps from HIP graphs on a plan-owned stream
 * (ordered after earlier work on `stream`, and later work on `stream` after
 * it): one recorded step per parity, with and without the statistics pass, kept
 * in the plan (up to 8, least recently used dropped) and reused by later calls
 * with the same arrays and parameters, which removes the per-launch host cost.
 * Results are identical in both modes.
 * The plan must have been created with CF_PLAN_STEP.
 */
cf_status cf_run_steps(cf_plan* plan, void* u, void* v, void* w, void* u2, void* v2, void* w2, int nsteps,
                       double dt, double nu, double fx, int stats_every, double* stats_acc, double* p,
                       int use_graph, void* stream);

/*
 * Adjoint of cf_projection_step (the differentiated form of Section 2, Eq. (3)-(7)):
 * given the step input (u, v, w) and g1 = dJ/d(u1, v1, w1), returns
 * g = dJ/d(u, v, w) (Euclidean gradient, what autograd expects), with
 *   g* = P^T g1 = W P W^-1 g1          (P = I - G L_h^+ D; W = face volumes: the
 *                                         pressure solve is self-adjoint in the
 *                                         face-volume inner product),
 *   gb = dt/2 J_R(ub)^T g*,  ub = u + dt R(u)   (recomputed),
 *   g  = g* + gb + J_R(u)^T (dt/2 g* + dt gb).
 * Entries of the top-wall v plane are not variables: their gradient is 0.
 * g may alias g1 but not (u, v, w).  Arrays as in cf_projection_step.  The plan
 * must have been created with CF_PLAN_STEP | CF_PLAN_ADJOINT.
 */
cf_status cf_projection_step_adjoint(cf_plan* plan, const void* u, const void* v, const void* w,
                                     const void* gu1, const void* gv1, const void* gw1, void* gu,
                                     void* gv, void* gw, double dt, double nu, double fx, void* stream);

/* Test hook: (gu, gv, gw) = J_R(u, v, w)^T (lu, lv, lw), the transpose of the momentum
 * right-hand side's Jacobian at (u, v, w).  Arrays as in cf_projection_step; gu, gv,
 * gw must not overlap each other or any input (CF_ERR_ARG). */
cf_status cf_rhs_adjoint(cf_plan* plan, const void* u, const void* v, const void* w, const void* lu,
                         const void* lv, const void* lw, void* gu, void* gv, void* gw, double nu,
                         void* stream);

/* Test hook, steps (2)-(4): forward real transform in x then complex transform in z of f
 * (device double (ny, nz, nx)) into fhat (device complex, plan precision: double pairs
 * for CF_FP64, float pairs for CF_MIXED; shape (nx/2+1, ny, nz)). */
cf_status cf_forward_spectral(cf_plan* plan, const double* f, void* fhat, void* stream);

/* Test hook, steps (6)-(8): inverse transforms of phat (layout as above) into p, scaled
 * by 1/(nx nz).  phat is not modified. */
cf_status cf_inverse_spectral(cf_plan* plan, const void* phat, double* p, void* stream);

/* Test hook, step (5): solve every wall-normal line of fhat (Eq. (9) with the PDD of
 * Section 2.2, exact or dropped reduced system per the plan, gauge on the kx=kz=0 line)
 * into phat.  Same layout and precision as cf_forward_spectral; phat may be fhat
 * itself but must not overlap it otherwise (CF_ERR_ARG). */
cf_status cf_solve_spectral(cf_plan* plan, const void* fhat, void* phat, void* stream);

/*
 * The solve of cf_solve_spectral split into y-slabs the way the paper splits it
 * across processes (Section 2.2 PDD; Section 3: each process owns a range of
 * partitions and exchanges only interface values).  The ny rows of every line
 * are cut into n_slabs slabs of n_parts / n_slabs partitions (n_slabs must
 * divide the plan's n_parts).  For every slab a local pass solves its
 * partitions and writes their interface rows (x~_1, x~_M, v_1, v_M, w_1, w_M
 * per partition and line) into iface; then, for every slab, a finishing pass
 * reads all interface rows, solves the reduced system, redoes the slab's local
 * solves and writes the slab's corrected rows.  On several devices the slabs
 * would be the devices and iface the buffer they exchange; here the slabs run
 * one after another on one device.  The result equals cf_solve_spectral's
 * bitwise.  iface: device buffer of cf_plan_info.slab_iface_bytes (layout
 * [n_parts][8][n_lines], plan precision), overwritten.  phat may be fhat itself but
 * must not overlap it otherwise (CF_ERR_ARG).
 * Not available with CF_PLAN_Y_DCT (no partitions).
 */
cf_status cf_solve_spectral_slabs(cf_plan* plan, int n_slabs, const void* fhat, void* phat, void* iface,
                                  void* stream);

/*
 * Failure detection.  Every pressure solve of the partitioned wall-normal solver
 * (cf_poisson_solve, cf_projection_step, its adjoint, cf_run_steps,
 * cf_solve_spectral, cf_solve_spectral_slabs) checks the kx = kz = 0 line of its
 * right-hand side: a non-finite value anywhere in an x-z plane of f (or of the
 * divergence of u*, i.e. in the velocity state) reaches that plane's entry of
 * the line (its sum over the plane), and the solve raises a flag in the plan.
 * This call waits for the work enqueued on `stream` (and the plan's side
 * stream), returns CF_ERR_NUMERIC if the flag is raised and clears it, else
 * CF_OK.  Plans with CF_PLAN_Y_DCT do not check.
 */
cf_status cf_plan_numeric_status(cf_plan* plan, void* stream);

/*
 * cf_solve_spectral_slabs without the iface argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the interface rows go to a fixed device
 * array of the library (32 MiB; each device the library runs on holds its own
 * copy until the process ends, its address taken at plan creation).  The call
 * makes no device allocation and records no per-kernel timing.  Plans whose
 * interface rows (cf_plan_info.slab_iface_bytes) exceed 32 MiB are rejected
 * with CF_ERR_ARG before any work is enqueued.  Every call on a device shares
 * that device's array: calls that overlap on one device (several streams, or
 * several host threads) race and must be serialised by the caller.  The array
 * keeps the last call's contents; every value a call reads from it is written
 * earlier in the same call, so nothing needs clearing.  Other arguments and the
 * result are as for cf_solve_spectral_slabs.
 */
cf_status cf_solve_spectral_slabs_noalloc(cf_plan* plan, int n_slabs, const void* fhat, void* phat, void* stream);

/*
 * Per-kernel timing with HIP events (measurement support).  While enabled, every
 * kernel launch of the plan is bracketed by two events recorded on the launch
 * stream; cf_plan_get_timing synchronises on them and returns the accumulated
 * device time and launch count of one kernel class since the last reset.
 */
enum {
  CF_K_R2C_X = 0,     /* forward real transform along x (+ fused producers) */
  CF_K_FFT_Z_FWD = 1, /* forward complex transform along z */
  CF_K_YSOLVE = 2,    /* PDD wall-normal line solve */
  CF_K_SPECIAL = 3,   /* whole-line FP64 Thomas (kx=kz=0 and the FP64 set) */
  CF_K_FFT_Z_INV = 4, /* inverse complex transform along z */
  CF_K_C2R_X = 5,     /* inverse real transform along x (+ fused consumers) */
  CF_K_DIVERGENCE = 6,
  CF_K_RK1 = 7,       /* RK2 stage 1 (momentum RHS) */
  CF_K_RK2 = 8,       /* RK2 stage 2 (momentum RHS) */
  CF_K_CORRECT = 9,   /* pressure-gradient correction u1 = u* - dt G p */
  CF_K_ADJ_RHS = 10,  /* transposed momentum right-hand side */
  CF_K_ADJ_CORRECT = 11, /* weighted correction of the transposed projection */
  CF_K_RK_FUSED = 12, /* both RK2 stages in one marching pass (forward step) */
  CF_K_SLAB_LOCAL = 13,  /* y-slab solve: local partition solves + interface rows */
  CF_K_SLAB_FINISH = 14, /* y-slab solve: reduced system + correction of one slab */
  CF_K_COUNT = 15
};
cf_status cf_plan_set_timing(cf_plan* plan, int enable);
cf_status cf_plan_reset_timing(cf_plan* plan);
cf_status cf_plan_get_timing(cf_plan* plan, int kernel, double* total_ms, long long* launches);
const char* cf_kernel_name(int kernel);

const char* cf_status_string(cf_status s);

/* Message describing the last error returned on the calling thread ("" if none). */
const char* cf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CHANFLOW_H */
