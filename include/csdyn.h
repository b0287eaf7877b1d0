/*
 * csdyn.h -- C ABI of libcsdyn, an MI355X (gfx950) solver for the two linear
 * systems that the approximate-factorization time step of the spherical-shell
 * dynamo produces (Yin et al., arXiv 2009.02171, Sec. 3.1-3.3).
 *
 * Problem statement (Sec. 3.3, eq. newlinear and the stopping rule after it):
 * solve A x = b by restarted GMRES, right-preconditioned (A M^{-1} x' = b,
 * x = M^{-1} x'), starting from a caller-supplied x0, until
 * ||b - A x|| <= max(atol, rtol * ||b - A x0||).  M^{-1} is restricted
 * additive Schwarz with ILU(0) subdomain solves (eq. onelevel), optionally
 * combined with a coarse-grid solve as the hybrid two-level preconditioner
 * (eq. twolevel, coarsesolve, finesolve).
 *
 * Grid (Sec. 3.2): six panels of N x N x Nr cells of the equiangular gnomonic
 * cubed-sphere shell r_i <= r <= r_o, cell centres
 *   xi_i = -pi/4 + (i+1/2) h_s,  eta_j = -pi/4 + (j+1/2) h_s,
 *   r_k = r_i + (k+1/2) h_r,  h_s = pi/(2N),  h_r = (r_o - r_i)/Nr.
 * Panels 0-3 are centred on +x, +y, -x, -y (xi eastward, eta northward),
 * panel 4 on +z and panel 5 on -z.
 *
 * Vector layout (every x, y, b): double v[6][Nr][N][N][4], contiguous, i
 * fastest within a row, then j, then k, then panel; the 4 components of a
 * cell are its Cartesian vector (x, y, z) and its scalar:
 *   kind VP: (u~, P)   -- velocity-pressure system,
 *   kind BP: (B~, P_b) -- magnetic-field / pseudo-pressure system,
 *   kind VT: (u~, Theta) -- velocity-temperature block of the VTBE.
 * Rows of A (E = Ekman number, Pm = magnetic Prandtl number, Ra = modified
 * Rayleigh number, Pr = Prandtl number, x = r r_hat the cell centre):
 *   VP: u - dt (E lap u - 2 zhat x u);   D(u) - dt lap_N P   (Neumann P)
 *   BP: B - dt (E/Pm) lap B;             D(B) - dt lap_D P_b (Dirichlet P_b)
 *   VT: u - dt (E lap u - 2 zhat x u) - dt (Ra/r_o) Theta x;
 *       Theta - dt (E/Pr) lap_D Theta - dt E (r_i r_o / r^3) (x . u)
 *       (eq. tsvelocity, tstemperature with Delta t / 2 = E dt; R1, R2 and L2
 *       of eq. linearoperator)
 * with finite-volume lap and D (eq. divdiscretization), no-slip u, the
 * pseudo-vacuum condition on B (eq. pvc: tangential B = 0,
 * d(r^2 B_r)/dr = 0 at the walls) and isothermal walls (Theta = 0, eq. utb).
 *
 * Memory: the caller owns every device buffer.  Each *_setup takes a device
 * workspace of at least *_workspace_bytes() bytes; handles are small host
 * structs that point into it, so the workspace must outlive the handle.  No
 * entry point allocates device memory after setup.  Host-side exceptions:
 * the first csdyn_gmres_solve (or two-level csdyn_ras_apply) on a thread
 * allocates, per solve nesting depth (at most two), two small pinned host
 * buffers and two HIP events for the Arnoldi read-backs, kept until the
 * process ends; later calls on that thread reuse them.  opts.timing creates
 * HIP events the same way.
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Apply calls
 * are asynchronous on it; csdyn_gmres_solve returns after the solve.
 * Errors: every call returns an int32 status; csdyn_last_error() gives a
 * thread-local message for the last failure on the calling thread.
 */
#ifndef CSDYN_H
#define CSDYN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSDYN_OK 0
#define CSDYN_ENOTCONV 1      /* outputs valid, tolerance not reached within maxit */
#define CSDYN_EINVAL (-1)     /* null/aliased pointer, bad shape or option */
#define CSDYN_EHIP (-2)       /* a HIP runtime call failed */
#define CSDYN_EZEROPIVOT (-3) /* |pivot| < 1e-300 in an ILU(0) factorization */
#define CSDYN_ENOMEM (-4)     /* workspace smaller than *_workspace_bytes() */
#define CSDYN_EBREAKDOWN (-5) /* NaN or Inf met in the solve */

#define CSDYN_VP 0
#define CSDYN_BP 1
#define CSDYN_VT 2

typedef struct {
    int32_t n;   /* cells per panel edge, N >= 4 */
    int32_t nr;  /* radial cells, Nr >= 1 */
    double ri;   /* inner radius (the paper uses 7/13) */
    double ro;   /* outer radius (the paper uses 20/13) */
} csdyn_grid;

typedef struct {
    int32_t kind;  /* CSDYN_VP, CSDYN_BP or CSDYN_VT */
    double dt;     /* time-step factor of the rows above (> 0 for a nonsingular ILU) */
    double ekman;  /* E */
    double pm;     /* Pm (BP only) */
    double ra;     /* modified Rayleigh number Ra (VT only) */
    double pr;     /* Prandtl number Pr (VT only, > 0) */
} csdyn_op;

/* ---------------------------------------------------------------- operator
 * Matrix-free y = A x (Sec. 3.2): ghost fill across panel edges (cubic
 * interpolation along the neighbour's first cell layer), conservative
 * edge fluxes (mean of the two panels' one-sided fluxes), wall ghosts, and
 * the 11-point finite-volume stencil.  The workspace holds the metric tables
 * (r-independent 2-D tables shared by the six panels) and the edge buffers.
 * csdyn_op_setup uploads the tables (synchronous); csdyn_operator_apply
 * launches three kernels on `stream`.  x and y are device pointers of
 * 24*N*N*Nr doubles and must not alias (CSDYN_EINVAL). */
typedef struct csdyn_opctx csdyn_opctx;
int32_t csdyn_op_workspace_bytes(const csdyn_grid *g, size_t *bytes);
int32_t csdyn_op_setup(const csdyn_grid *g, const csdyn_op *op, void *ws, size_t ws_bytes, void *stream,
                       csdyn_opctx **out);
int32_t csdyn_operator_apply(const csdyn_opctx *ctx, const double *x, double *y, void *stream);
void csdyn_op_destroy(csdyn_opctx *ctx);

/* Workgroup shape of the stencil kernel (a tuning knob): 1 = 32x8,
 * 2 = 16x16, 3 = 64x4, 4 = 16x8, 5 = 32x4 cells (identical results), 6 = the
 * FP64 kernel that requests its layers straight into LDS (16x16 cells, six
 * layer buffers; for N > 16, else 16x8; equal to the others up to rounding,
 * the grouping of the same terms being the compiler's), 0 = default (6 for
 * FP64 shells of at least 6 x 96^3 cells, else 4).  Returns CSDYN_EINVAL
 * outside 0..6. */
int32_t csdyn_op_set_tile(csdyn_opctx *ctx, int32_t tile);

/* Step 3 of the time step (Sec. 3.1, eq. ubtilde) from a solution
 * x = (u~, P) of the VP system (or (B~, P_b) of BP):
 *   out[c] = x[c] - dt (grad_h P)[c],  c = 0..2  (cell-centred gradient:
 *            sum_m g^m dP/dq^m with central differences; panel-edge ghosts
 *            and wall ghosts as in the operator),
 *   out[3] = D_f F: the finite-volume divergence of the corrected face
 *            fluxes F = (flux of u~) - dt (face gradient flux of P), which is
 *            the pressure row of A x; it is zero at faces when the pressure
 *            rows of A x = b hold with b_P = 0.
 * x and out are device vectors in the layout above and must not alias;
 * asynchronous on `stream`. */
int32_t csdyn_project(const csdyn_opctx *ctx, const double *x, double *out, void *stream);

/* ---------------------------------------------------------- preconditioner
 * Restricted additive Schwarz (eq. onelevel): each panel is cut into
 * (N/sub[0]) x (N/sub[1]) x (Nr/sub[2]) boxes; each box is extended by
 * `overlap` (0 or 1) cell layers, across panel edges into the neighbour's
 * first layer; A_i = R_i A R_i^T with the structural stencil pattern is
 * factored by point-wise ILU(0) in box-lexicographic order (i fastest, cell-
 * major, component-minor); the apply gathers x on each extended box, runs the
 * L and U sweeps, and writes y on the owned box only.
 * levels = 2 adds the hybrid coarse correction (eq. twolevel):
 *   w = I_c^f A_c^{-1} I_f^c x  (I_f^c: mean of 8 children, I_c^f: copy;
 *        A_c re-discretised on N/2 x N/2 x Nr/2; A_c^{-1} by GMRES(coarse_restart)
 *        to relative tolerance coarse_rtol from 0, preconditioned by one-level
 *        RAS with sub/2 boxes),
 *   y = w + M_one^{-1}(x - A_f w).
 * levels = 3 repeats the construction on the coarse grid (Sec. 3.3, the
 * multilevel hybrid for larger meshes): A_c^{-1} is then FGMRES(coarse_restart)
 * to coarse_rtol preconditioned by the coarse grid's own two-level hybrid
 * (sub/2 boxes on N/2, sub/4 boxes and the same GMRES settings on N/4); N, Nr
 * and sub must be divisible by 4 and N/4 >= 4.  csdyn_ras_info's coarse fields
 * then describe the one-level RAS of the N/2 grid.
 * For VP the coarse right-hand side's pressure part is projected to zero
 * volume-weighted mean (the coarse Neumann problem's solvability condition).
 * precision = 1 stores the factors in FP32 and runs every operation inside
 * M^{-1} in FP32; x and y stay FP64.
 * Setup assembles and factors on the host, then uploads (synchronous).
 * Errors: CSDYN_EINVAL if N or Nr is not divisible by sub (or by 2*sub for
 * levels = 2); CSDYN_EZEROPIVOT from the factorization. */
typedef struct {
    int32_t sub[3];          /* owned box size in cells (xi, eta, r) */
    int32_t overlap;         /* 0 or 1 */
    int32_t levels;          /* 1, 2 or 3 */
    double coarse_rtol;      /* 0.1 in the paper */
    int32_t coarse_restart;  /* 30 */
    int32_t coarse_maxit;    /* cap on inner iterations per coarse solve */
    int32_t precision;       /* 0 FP64, 1 FP32 inside the preconditioner */
    int32_t storage;         /* where a sweep keeps computed values: 0 automatic (the whole subdomain
                                vector in LDS when its FP64 size is at most 90 KiB, else a ring of
                                recent levels), 1 the ring, 2 the subdomain vector (CSDYN_EINVAL if it
                                does not fit in LDS), 3 as 0 but never folded.  With 0 and
                                2 an FP64 subdomain vector too large for two workgroups per compute
                                unit is folded when the level schedules allow it: its last rows reuse
                                the LDS of its first rows, whose values wait in registers meanwhile.
                                The results do not depend on it */
    int32_t values;          /* layout of the factor values a sweep reads: 0 automatic (packed for
                                FP64 sweeps of at least one subdomain per compute unit, padded
                                otherwise), 1 packed (an odd number of entries per lane stores the
                                last entries unpadded; FP64 only, CSDYN_EINVAL with precision = 1),
                                2 padded pairs.  The results do not depend on it */
} csdyn_ras_opts;

typedef struct csdyn_ras csdyn_ras;
int32_t csdyn_ras_workspace_bytes(const csdyn_opctx *ctx, const csdyn_ras_opts *o, size_t *bytes);
int32_t csdyn_ras_setup(const csdyn_opctx *ctx, const csdyn_ras_opts *o, void *ws, size_t ws_bytes, void *stream,
                        csdyn_ras **out);
/* y = M^{-1} x; x, y device pointers (FP64), must not alias.  The handle keeps
 * a pointer to ctx, which must outlive it.  One-level is
 * asynchronous; two-level synchronises with the host once per inner
 * iteration (convergence test of the coarse GMRES). */
int32_t csdyn_ras_apply(const csdyn_ras *pc, const double *x, double *y, void *stream);
void csdyn_ras_destroy(csdyn_ras *pc);

/* Host-only inspection of one subdomain of the one-level RAS (no device use):
 * the box's global cells in local order, owned flags, and the ILU(0) factors
 * of A_i = R_i A R_i^T as CSR over 4*nloc rows (strict lower part = L with an
 * implied unit diagonal, the rest = U).  Call once with gcell = owned =
 * rowptr = col = val = NULL to get nloc and nnz, then with arrays of
 * nloc, nloc, 4*nloc+1, nnz and nnz entries.  Subdomain s is numbered
 * ((p*nbk + bk)*nbj + bj)*nbi + bi. */
int32_t csdyn_ras_inspect(const csdyn_grid *g, const csdyn_op *op, const int32_t sub[3], int32_t overlap, int32_t s,
                          int64_t *nloc, int64_t *nnz, int32_t *gcell, int32_t *owned, int64_t *rowptr, int32_t *col,
                          double *val);

/* ------------------------------------------------------------------- GMRES
 * Right-preconditioned restarted GMRES(restart) (Sec. 3.3); flexible = 1 is
 * FGMRES, required when M^{-1} contains an inner Krylov solve or FP32
 * arithmetic.  Orthogonalisation (same Krylov space as modified Gram-Schmidt):
 * orth = 0, classical Gram-Schmidt, one pass for the projections and one for
 * the update and norm (PETSc's default GMRES orthogonalisation); orth = 1,
 * classical Gram-Schmidt with one re-orthogonalisation, whose projections are
 * fused into the first update pass (three passes).  The coarse solve inside
 * the two-level preconditioner always uses orth = 0.  Stops when the residual
 * estimate <= max(atol, rtol * ||b - A x0||); then recomputes the true
 * residual.  For VP, b's pressure part is first projected to zero
 * volume-weighted mean and the solution's pressure is returned with zero
 * volume-weighted mean (the Neumann null space).
 * b: device, const; x: device, in x0 / out solution.  pc may be NULL.
 * Blocks until done; returns CSDYN_ENOTCONV if maxit was reached. */
typedef struct {
    int32_t restart;   /* 30 */
    int32_t maxit;     /* total Arnoldi steps */
    int32_t flexible;  /* 0 GMRES, 1 FGMRES */
    double rtol, atol;
    int32_t orth;      /* 0 CGS, 1 CGS2 */
    int32_t rhs_relative; /* 0: stop at max(atol, rtol ||b - A x0||) (Sec. 3.3);
                             1: stop at max(atol, rtol ||b||) */
    int32_t timing;       /* 1: fill stats.t_ms from HIP events recorded on `stream` around each
                             phase (creates the events on first use on a thread); 0: no events */
    int32_t device_steps; /* 0: the host forms each step's Hessenberg column and Givens rotation
                             from the step's read-back (one wait per step); k in [1, 32]: the
                             device forms them and the host reads the convergence state once per
                             k steps, the next k steps already enqueued, so up to 2k - 1 steps
                             past convergence are computed and discarded (for solves whose steps
                             are short next to a host round trip) */
} csdyn_gmres_opts;

/* Phases of stats.t_ms (the breakdown of a preconditioned iteration in Sec. 4.3
 * into the coarse solve, the fine subdomain solves and the fine/coarse
 * transfers, plus the outer solve's own work). */
#define CSDYN_T_OP 0     /* outer operator applies (Arnoldi steps, initial and restart residuals) */
#define CSDYN_T_PCF 1    /* fine one-level RAS sweeps (PC-F) */
#define CSDYN_T_PCC 2    /* the coarse solve: inner GMRES with its operator, RAS and Gram-Schmidt (PC-C) */
#define CSDYN_T_PCI 3    /* restriction, coarse projection, prolongation, x - A_f w, y = w + ...,
                            FP64/FP32 conversions (PC-I) */
#define CSDYN_T_ORTH 4   /* outer Gram-Schmidt (multi-dot, multi-update, normalisation) */
#define CSDYN_T_OTHER 5  /* the rest of the span: vector copies and updates, read-back waits, host
                            Givens steps, launch gaps */

typedef struct {
    int32_t iters, restarts;
    int64_t inner_iters;     /* coarse GMRES iterations summed over the solve */
    double relres_true;      /* ||b - A x|| / ||b - A x0|| recomputed at the end */
    double relres_est;       /* the GMRES estimate at exit */
    double res0;             /* ||b - A x0|| */
    double res_true;         /* ||b - A x|| recomputed at the end */
    double bnorm;            /* ||b|| */
    double t_ms[6];          /* with opts.timing: stream time per phase (CSDYN_T_*), ms; else 0 */
    double t_span_ms;        /* with opts.timing: stream time from the solve's first to its last launch */
    int64_t inner2_iters;    /* three levels: coarsest-grid GMRES iterations summed over the solve */
} csdyn_gmres_stats;

int32_t csdyn_gmres_workspace_bytes(const csdyn_opctx *ctx, const csdyn_gmres_opts *o, size_t *bytes);

/* Batched solves: nshell (<= 64) independent systems, each with its own
 * operator (any grid size) and optional one-level preconditioner (the
 * two-level one synchronises with the host inside), solved by FGMRES
 * (restart = o->restart, CGS orthogonalisation, o->orth must be 0) in lock
 * step: one Arnoldi step of all active shells at a time, one host
 * synchronisation per step for the batch (o->timing and o->device_steps are
 * not used).  use_graph selects how a step runs:
 * 0, the shells' kernels on their own streams; 1, the same captured as a
 * hipGraph per (active set, step index), kept in the handle for later solves;
 * 2, one launch per phase for all active shells together (every shell's RAS
 * subdomains in one launch, then the edge fills, the stencil tiles, the
 * multi-dot, update and normalisation blocks and their reductions: nine
 * launches a step whatever the shell count), captured per (active set, step
 * index); 3, one persistent launch per step (a work-list of the same items,
 * each waiting, bounded, for its shell's previous phase), switched off in this
 * build because its solves did not finish in the time allowed on the GPU.
 * Modes 2 and 3 need one-level FP32 preconditioners on all shells, at most 16
 * shells and N >= 16; csdyn_batch_modes returns a bit mask of the modes a
 * handle can run (bit m for use_graph = m); CSDYN_EINVAL for the others.
 * Modes 0, 1 and 2 give the same results bit for bit.  Stopping rule, projection
 * of the VP pressure and statistics per shell as for csdyn_gmres_solve.
 * b, x: host arrays of nshell device pointers (x holds x0 on entry).  The
 * workspace (csdyn_batch_workspace_bytes) holds every shell's Krylov basis and
 * must outlive the handle; the handle owns its streams, events, graphs and a
 * small pinned host buffer.  Calls on one handle must not overlap.  Returns
 * CSDYN_ENOTCONV if any shell missed its tolerance within maxit. */
typedef struct csdyn_batch csdyn_batch;
int32_t csdyn_batch_workspace_bytes(int32_t nshell, const csdyn_opctx *const *ops, const csdyn_gmres_opts *o,
                                    size_t *bytes);
int32_t csdyn_batch_setup(int32_t nshell, const csdyn_opctx *const *ops, const csdyn_ras *const *pcs,
                          const csdyn_gmres_opts *o, void *ws, size_t ws_bytes, csdyn_batch **out);
int32_t csdyn_gmres_solve_batched(csdyn_batch *batch, const double *const *b, double *const *x, int32_t use_graph,
                                  void *stream, csdyn_gmres_stats *stats);
/* *modes = bit mask of the use_graph values this handle can run (bit m for m). */
int32_t csdyn_batch_modes(const csdyn_batch *batch, int32_t *modes);
void csdyn_batch_destroy(csdyn_batch *batch);

/* ||b - A x|| (b with its pressure part projected for VP, as the solve does):
 * the residual of a candidate initial guess.  ws: at least
 * csdyn_residual_workspace_bytes; blocks until the norm is on the host. */
int32_t csdyn_residual_workspace_bytes(const csdyn_opctx *ctx, size_t *bytes);
int32_t csdyn_residual_norm(const csdyn_opctx *ctx, const double *b, const double *x, void *ws, size_t ws_bytes,
                            void *stream, double *norm);

/* csdyn_residual_norm for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result from the same kernels, with its temporaries (the residual,
 * A x and the reduction partials, about 13 MB) in a static device array of
 * the library instead of a caller workspace.  Shells of at most
 * CSDYN_NOALLOC_MAX_CELLS cells (6 x 32^3), else CSDYN_EINVAL.  Allocates
 * nothing (the array is part of the loaded library, one copy per GPU, kept
 * until the process ends).  Every call on one GPU uses that GPU's array, and
 * every call overwrites all of the array it reads, so nothing carries over;
 * calls that overlap on one GPU (other threads or streams) race and must be
 * serialised by the caller.  Blocks until the norm is on the host. */
#define CSDYN_NOALLOC_MAX_CELLS 196608
int32_t csdyn_residual_norm_noalloc(const csdyn_opctx *ctx, const double *b, const double *x, void *stream,
                                    double *norm);
int32_t csdyn_gmres_solve(const csdyn_opctx *ctx, const csdyn_ras *pc, const csdyn_gmres_opts *o, const double *b,
                          double *x, void *ws, size_t ws_bytes, void *stream, csdyn_gmres_stats *st);

/* Size summary of a preconditioner (for bandwidth accounting).  Entries are
 * ILU(0) factor entries (L and U, diagonal included) before padding. */
typedef struct {
    int32_t nsd_fine, nsd_coarse;
    int64_t nnz_fine, nnz_coarse;             /* factor entries */
    int64_t box_cells_fine, box_cells_coarse; /* cells of all overlapping boxes */
    int64_t owned_cells_fine, owned_cells_coarse;
    int64_t stored_fine, stored_coarse;       /* stored entries incl. slice padding */
    int32_t max_levels_fine, max_levels_coarse; /* L + U sweep levels of the deepest subdomain */
    int32_t precision;
    int32_t lds_fine, lds_coarse;             /* dynamic LDS bytes per workgroup of the sweep kernel */
    int32_t box_in_lds_fine, box_in_lds_coarse; /* where the sweep keeps computed values: 0 a ring of recent
                                                   levels in device memory, 1 that ring in LDS, 2 the whole
                                                   subdomain vector in LDS, 3 that vector folded */
    int32_t threads_fine, threads_coarse;     /* workgroup size of the sweep kernel (256, 512 or 1024) */
    int32_t structures_fine, structures_coarse; /* distinct sweep structures: subdomains with the same
                                                   dependency addresses share one stored copy */
    int32_t blocks_per_cu_fine, blocks_per_cu_coarse; /* sweep workgroups that fit one compute unit */
    int32_t packed_fine, packed_coarse; /* 1 where the sweep reads the packed value layout */
} csdyn_ras_info;
int32_t csdyn_ras_get_info(const csdyn_ras *pc, csdyn_ras_info *info);

/* ------------------------------------------------- learned initial guess
 * The paper starts each time step's GMRES solve from the previous step's
 * solution (Sec. 3.3).  These entries build a panel-wise 3-D convolutional
 * network that predicts the initial guess from the previous two solutions,
 * and train it online on the solutions the solver produces.
 *
 * BF16 tensors are uint16_t bit patterns, channels-last per panel:
 * t[batch][d][h][w][c8] with c8 = round_up(c, 8) and the padded channels
 * zero (the solver's vector layout [6][Nr][N][N][4] is this with 4 FP64
 * channels).  Weights are FP32 w[cout][27][cin], tap t = 9(dz+1) + 3(dy+1) +
 * (dx+1), correlation with zero padding inside each batch entry:
 *   y[b,d,h,w,o] = bias[o] + sum_{t,i} x[b,d+dz,h+dy,w+dx,i] w[o,t,i].
 * Accumulation is FP32 on the matrix cores; outputs are rounded to BF16
 * (round to nearest even) or written as FP32.  cout <= 128 and cin <= 128
 * for the data gradient.  All pointers are device pointers; every call is
 * asynchronous on `stream` and returns CSDYN_EINVAL for null pointers or bad
 * shapes. */
typedef struct {
    int32_t batch, d, h, w; /* batch entries (the six panels) and volume */
    int32_t cin, cout;
} csdyn_conv_shape;

/* Element counts of the two packed BF16 weight copies and the workspace of
 * the weight gradient (host call). */
int32_t csdyn_conv3d_sizes(const csdyn_conv_shape *s, int64_t *wf_elems, int64_t *wb_elems,
                           size_t *bwd_weight_ws_bytes);
/* Pack w into wf (forward) and wb (flipped, transposed: the data gradient's
 * forward weights).  Either output may be NULL. */
int32_t csdyn_conv3d_pack(const csdyn_conv_shape *s, const float *w, uint16_t *wf, uint16_t *wb, void *stream);
/* y = act(conv(x) + bias [+ residual]) with act = relu if relu != 0; y (BF16,
 * cout8 channels) and/or y32 (FP32, cout channels); bias and residual may be
 * NULL. */
int32_t csdyn_conv3d_fwd(const csdyn_conv_shape *s, const uint16_t *x, const uint16_t *wf, const float *bias,
                         const uint16_t *residual, int32_t relu, uint16_t *y, float *y32, void *stream);
/* dx = d loss / d x given dy = d loss / d y (BF16 [..][cout8] -> [..][cin8]);
 * where mask != NULL, dx is zeroed wherever mask <= 0 (the derivative of a
 * relu whose output is mask). */
int32_t csdyn_conv3d_bwd_data(const csdyn_conv_shape *s, const uint16_t *dy, const uint16_t *wb,
                              const uint16_t *mask, uint16_t *dx, void *stream);
/* dw = d loss / d w (FP32 [cout][27][cin], overwritten) and, if db != NULL,
 * db = sum of dy over all voxels; sums run in a fixed order (deterministic).
 * ws: csdyn_conv3d_sizes' bwd_weight_ws_bytes, else CSDYN_ENOMEM. */
int32_t csdyn_conv3d_bwd_weight(const csdyn_conv_shape *s, const uint16_t *x, const uint16_t *dy, float *dw,
                                float *db, void *ws, size_t ws_bytes, void *stream);
/* One Adam step (Kingma and Ba, with bias correction; step >= 1 is the step
 * number): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps), elementwise FP32. */
int32_t csdyn_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, int32_t step, float lr,
                        float beta1, float beta2, float eps, void *stream);

/* The network: widths (c0, c1, c2, c3), four resolution levels (N and Nr
 * multiples of 8), additive skips:
 *   e0 = relu(conv0(x)), e1 = relu(conv1(pool e0)), e2 = relu(conv2(pool e1)),
 *   e3 = relu(conv3(pool e2)), d2 = relu(conv4(up e3) + e2),
 *   d1 = relu(conv5(up d2) + e1), d0 = relu(conv6(up d1) + e0), y = conv7(d0)
 * (pool: mean of 2x2x2 children; up: copy to them), 8 -> c0 -> c1 -> c2 -> c3
 * -> c2 -> c1 -> c0 -> 4 channels.  Inputs x = (x1 / s, (x1 - x2) / sd), s and
 * sd the per-component RMS of x1 and x1 - x2 over all cells; guess =
 * 2 x1 - x2 + sd * y; loss = mean over cells and components of
 * (y - (xn - 2 x1 + x2) / sd)^2.  x1, x2, xn, guess: FP64 solver vectors.
 * Parameters: FP32, flat, layer by layer w[cout][27][cin] then bias[cout]. */
typedef struct csdyn_net csdyn_net;
int32_t csdyn_net_param_count(const int32_t *widths, int64_t *count);
int32_t csdyn_net_workspace_bytes(int32_t n, int32_t nr, const int32_t *widths, size_t *bytes);
/* params: device FP32 initial parameters (copied); Adam moments start at 0. */
int32_t csdyn_net_setup(int32_t n, int32_t nr, const int32_t *widths, const float *params, void *ws,
                        size_t ws_bytes, void *stream, csdyn_net **out);
int32_t csdyn_net_get_params(const csdyn_net *net, float *params, void *stream);
/* guess = 2 x1 - x2 + sd * net(x1, x2); x1 is the latest solution. */
int32_t csdyn_net_predict(csdyn_net *net, const double *x1, const double *x2, double *guess, void *stream);
/* Loss of the sample (x2, x1) -> xn and its gradient (FP32, flat, device;
 * may be NULL).  loss: host pointer or NULL; when given, the call waits for
 * the stream. */
int32_t csdyn_net_loss_grad(csdyn_net *net, const double *x2, const double *x1, const double *xn, float *grads,
                            double *loss, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that sample. */
int32_t csdyn_net_train_step(csdyn_net *net, const double *x2, const double *x1, const double *xn, float lr,
                             double *loss, void *stream);
void csdyn_net_destroy(csdyn_net *net);

/* Initial guess of the next solve from the latest two solutions x1 (newest)
 * and x2 (the paper takes the previous solution, Sec. 3.3):
 *   mode 0: guess = x_e = 2 x1 - x2 (linear extrapolation; net, b and ws
 *           unused, may be NULL);
 *   mode 1: x_n = csdyn_net_predict(net, x1, x2); guess = x_n if
 *           ||b - A x_n|| < ||b - A x_e|| else x_e (the residual fallback);
 *   mode 2: guess = x_e + alpha (x_n - x_e), alpha = <r_e, A d> / <A d, A d>
 *           with r_e = b - A x_e and d = x_n - x_e: the step along the
 *           network's correction that minimises ||b - A guess||, never
 *           larger than ||r_e||.
 * b is projected as the solve projects it (VP pressure part).  Modes 1 and 2
 * apply A twice and synchronise with the host.  info (may be NULL):
 * res_extrap = ||r_e||, res_net = ||b - A x_n||, res_guess = ||b - A guess||
 * (modes 1, 2; -1 for mode 0), alpha (mode 1: 1 when x_n was kept, else 0).
 * All vectors are device FP64 in the solver's layout; guess must not alias
 * x1, x2 or b; ws: csdyn_guess_workspace_bytes, else CSDYN_ENOMEM. */
typedef struct {
    double res_extrap, res_net, res_guess, alpha;
} csdyn_guess_info;
int32_t csdyn_guess_workspace_bytes(const csdyn_opctx *ctx, size_t *bytes);
int32_t csdyn_guess(csdyn_net *net, const csdyn_opctx *ctx, const double *b, const double *x1, const double *x2,
                    int32_t mode, double *guess, void *ws, size_t ws_bytes, void *stream, csdyn_guess_info *info);

/* Right-hand side of one step of the march that feeds the learned guess
 * (the paper's step without its nonlinear terms, Sec. 3.1): b = (v + dt f, 0),
 * v the projected state of the previous step (csdyn_project), f the forcing;
 * all three in the solver's layout on the device; asynchronous. */
int32_t csdyn_march_rhs(const csdyn_opctx *ctx, const double *v, const double *f, double dt, double *b,
                        void *stream);

/* ------------------------------------------------- the semi-implicit step
 * Nonlinear terms of the momentum and induction equations (Sec. 3.1, eq.
 * nonlinearoperator):
 *   f1 = -(u . grad) u + cB (B . grad) B     (cB = 1/(E Pm)),
 *   f3 =  (B . grad) u - (u . grad) B,
 * and, when the velocity-temperature state T = (u, Theta) is given (else
 * NULL), f2 = -(u . grad) Theta in f1's scalar slot (isothermal Theta
 * ghosts), so that f1 is the VT system's explicit vector (f1, f2).
 * Each (a . grad) b is the conservative finite-volume form div(a b_c) of each
 * Cartesian component c (Sec. 3.2, eq. nonlinearint; in Cartesian components
 * the Christoffel source terms of the contravariant form vanish): the sum over
 * the cell's six faces of (a_f . sqrt(g) g^m) (b_c)_f times the face area over
 * the cell volume, a_f and b_f the means of the two cells' values; beyond a
 * panel edge the neighbour is the ghost (cubic interpolation, as in the
 * operator), beyond a wall the wall ghost of the field's own system (u:
 * no-slip, B: pseudo-vacuum); through a panel-edge face the mean of the two
 * panels' one-sided fluxes.
 * vp, bp: the VP and BP contexts of one grid; u, B: device vectors in the
 * solver's layout (component 3, the pressures, is not read); T: device, the
 * VT layout (only component 3 is read), or NULL; f1, f3: device, same
 * layout, component 3 of f3 (and of f1 without T) set to 0; f1 and f3 must
 * not alias each other or the inputs.  ws: csdyn_nonlinear_workspace_bytes
 * (the ghost values of u, B and T), else CSDYN_ENOMEM.  Asynchronous on
 * `stream`. */
int32_t csdyn_nonlinear_workspace_bytes(const csdyn_opctx *ctx, size_t *bytes);
int32_t csdyn_nonlinear(const csdyn_opctx *vp, const csdyn_opctx *bp, const double *u, const double *B,
                        const double *T, double cB, double *f1, double *f3, void *ws, size_t ws_bytes,
                        void *stream);

/* Right-hand side of Step 1 (Sec. 3.1, eqs. tsvelocity, tstemperature and
 * tsmag) in this system's scaling (Delta t = 2 E dt; the vector rows of A are
 * I - (Delta t / 2) L):
 *   rhs[c] = 2 xhat[c] - (A xhat)[c] + c1 fn[c] + c2 fm[c] + c3 gf[c], c < 3,
 *   rhs[3] = 0 (VP, BP: the divergence rows), or the same combination for
 *   the VT system's Theta row (VT: xhat = (\hat u^n, Theta^n), fn = (f1, f2)),
 * i.e. xhat + (Delta t / 2) L xhat + the explicit terms; with the
 * Adams-Bashforth combination c1 = 1.5 Delta t, c2 = -0.5 Delta t (the first
 * step: c1 = Delta t, c2 = 0).  xhat = \hat u^n (or \hat B^n): the vector
 * part of csdyn_project applied to the previous state (eq. ubhat; the vector
 * rows of A do not read the scalar part).  fm and gf may be NULL when their
 * coefficients are 0 (gf: an optional prescribed body force).  rhs must not
 * alias an input.  Asynchronous on `stream`. */
int32_t csdyn_cn_rhs(const csdyn_opctx *ctx, const double *xhat, const double *fn, const double *fm,
                     const double *gf, double c1, double c2, double c3, double *rhs, void *stream);

/* Step 3 (Sec. 3.1, eq. ubtilde) kept as the next step's state: state[c] =
 * x[c] - dt (grad_h P)[c] for c < 3 (as csdyn_project) and state[3] = x[3]
 * (P^{n+1} or P_b^{n+1}).  x and state must not alias.  Asynchronous. */
int32_t csdyn_step3_state(const csdyn_opctx *ctx, const double *x, double *state, void *stream);

/* Right-hand side of Step 2 when Step 1 was the VT solve (Sec. 3.1, eq. tsp):
 * y = ((A x)_vec, 0) for a VP (or BP) context, whose solve then returns
 * x_vec (to its tolerance) with the pressure that satisfies the divergence
 * rows, D(u~) = dt lap_N P.  x and y must not alias; CSDYN_EINVAL for a VT
 * context.  Asynchronous on `stream`. */
int32_t csdyn_vector_rows(const csdyn_opctx *ctx, const double *x, double *y, void *stream);

/* ----------------------------------------------------------------- profile
 * Optional timing of every kernel launch by HIP events recorded on the launch
 * stream.  begin() creates a pool of max_launches event pairs; until end(),
 * each launch records a pair (launches beyond the pool are not timed).
 * end() waits for the recorded events and returns, per kernel name and
 * problem size (cells for the operator, subdomains for RAS, vector length for
 * the Krylov kernels), the launch count, the summed duration and the summed
 * algorithmic bytes (the HBM traffic the launches must cause: operands read
 * once and results written once, no cache effects, no index or padding
 * bytes) and, for the matrix-core kernels of the network, the summed
 * algorithmic flops (2 per multiply-add of the convolution's definition, no
 * padding).  Not thread-safe with concurrent solves on other threads. */
typedef struct {
    char name[32];
    int64_t size;
    int64_t count;
    double total_ms;
    double bytes;
    double flops;
} csdyn_profile_entry;
int32_t csdyn_profile_begin(int32_t max_launches);
/* Restrict the timing of the next begin() .. end() to the launches whose
 * kernel names (as end() reports them) appear in names, a comma-separated
 * list, and of those to one launch in `every` per name (the first, then every
 * every-th); NULL or "" times every launch (the default, every is then
 * ignored).  Fewer timed launches disturb the timed work less.  Returns
 * CSDYN_EINVAL while profiling is active or if every < 1. */
int32_t csdyn_profile_select(const char *names, int32_t every);
int32_t csdyn_profile_end(csdyn_profile_entry *out, int32_t max_entries, int32_t *n_entries);

/* Thread-local text of the last error on this thread ("" if none). */
const char *csdyn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
