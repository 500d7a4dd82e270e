/*
 * rt3d.h -- C ABI of the MI355X (gfx950) hot path of the 3D radiative-transfer scattering solve of
 * Hauschildt & Baron, "A 3D radiative transfer framework XIII: OpenCL implementation".
 *
 * The library computes, with hand-written HIP kernels:
 *   - the formal solution (FS) along characteristics through a Cartesian voxel grid periodic in x
 *     and y, per solid angle (section "Implementation of the formal solution and Lambda*
 *     computation");
 *   - the mean intensity J and the nearest-neighbour (3x3x3 = 27-point) Lambda* operator;
 *   - the non-local operator-splitting (OS) step, solving (1 - Lambda* (1-eps)) dJ = J_fs - J_old
 *     by Jacobi ("Jordan") iterations (section "Implementation of the operator splitting step"),
 *     with the coherent isotropic scattering source S = eps B + (1-eps) J (section "Test case
 *     setup").
 * All state lives on the device; only opacities/eps/B go in and J comes out (section "Method").
 *
 * Environment variables read when a context is created (tuning experiments; the defaults are the
 * measured best): RT3D_SWEEP_SHAPE (index into rt3d_sweep_shapes), RT3D_JACOBI_XCD (Jacobi launch
 * layout 0..4; all give bitwise the same iterates), RT3D_JACOBI_ALTERNATE (0: the column layout walks
 * every sweep bottom first instead of alternating; same iterates), RT3D_JACOBI_COLUMN (voxels per
 * thread of the column layout, 1, 2 or 4; default by grid size; same iterates), RT3D_JACOBI_WALK
 * (1: odd column layers walk top down, 0: never, -1 (default): for float coefficients in columns of 4;
 * same iterates), RT3D_ANCHOR_RATIO (re-anchoring ratio of the RT3D_FP32_SWEEP form, default 1e-2).
 *
 * Discretisation (the paper defers it to earlier papers of its series; these are the readings):
 *   voxels    unit cubes (i,j,k), i fastest; k = 0 is the bottom (inner boundary), k = nz-1 the top;
 *   angles    n_theta-point Gauss-Legendre in mu (n_theta even) x n_phi uniform azimuths
 *             phi_b = 2 pi (b + 1/2) / n_phi (n_phi a multiple of 4), weight w_a / (2 n_phi);
 *             direction index d = a * n_phi + b with the mu nodes ascending (first half downward);
 *   lines     per direction one straight line per column (i,j) through (i+1/2, j+1/2, nz); the
 *             same lines serve Omega and -Omega; chi and S are constant per voxel and every
 *             segment of a line inside a voxel is integrated exactly;
 *   voxel I   the path-length-weighted average over all segments of the direction inside the voxel;
 *   Lambda*   the exact 27-point band of Lambda (S -> J with no boundary light);
 *   OS step   dJ^0 = 0, M Jacobi sweeps, J <- J + dJ^M, c = max_v |dJ_v| / |J_v|; J^0 = B.
 *
 * Layouts: per-voxel fields are float64 [nz][ny][nx] (x fastest).  Lambda* is float64 [27][nz][ny][nx]
 * with neighbour index o = 9 (dk+1) + 3 (dj+1) + (di+1), u = v + (di,dj,dk), periodic in i and j;
 * entries whose u would lie outside 0 <= k+dk < nz are zero.
 *
 * Conventions for every call:
 *   - The return value is an rt3d_status (0 = RT3D_OK, negative = error); nothing throws across the
 *     ABI.  On error the context keeps its previous valid state unless stated otherwise, and
 *     rt3d_last_error() describes the failure.
 *   - ptr_kind selects where a caller buffer lives: RT3D_HOST (0) or RT3D_DEVICE (1).  Device
 *     buffers must be valid on the context's stream; the library does not keep any caller pointer
 *     after the call returns.  Calls with host buffers synchronise the stream before returning.
 *   - The caller owns every buffer it passes; the context owns everything it allocates.
 *   - One context per thread; a context may be used from one host thread at a time.
 */
#ifndef RT3D_H
#define RT3D_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RT3D_OK = 0,
    RT3D_ERR_ARG = -1,           /* invalid argument (sizes, pointers, non-finite or out-of-range data) */
    RT3D_ERR_OOM = -2,           /* device or host allocation failed */
    RT3D_ERR_HIP = -3,           /* a HIP runtime call failed (message in rt3d_last_error) */
    RT3D_ERR_NOT_CONVERGED = -4, /* max_iter reached; J and the last c are valid */
    RT3D_ERR_NONFINITE = -5,     /* a NaN or Inf appeared in dJ or J */
    RT3D_ERR_STATE = -6          /* call out of order (e.g. no medium set, Lambda* not built) */
} rt3d_status;

enum { RT3D_HOST = 0, RT3D_DEVICE = 1 };

typedef enum {
    RT3D_FP64 = 0,        /* every step in float64 */
    RT3D_FP32_SWEEP = 1   /* FS sweeps in float32; J accumulation, Lambda*, OS solve and the
                             convergence test in float64 (see rt3d_os_step) */
} rt3d_precision;

typedef struct {
    int nx, ny, nz;        /* voxels; nx, ny, nz >= 3 */
    int n_theta, n_phi;    /* n_theta even >= 2; n_phi >= 4 and a multiple of 4 */
    double I_top;          /* intensity entering through the top plane (outer boundary), >= 0 */
    int bottom_bc;         /* 0: an upward line enters with I = B of the bottom voxel it enters;
                              1: I = 0 at the bottom plane;
                              2: LTE diffusion, I = B_0 + mu (B_0 - B_1) / ((chi_0 + chi_1) / 2) with B_0,
                                 chi_0 of that voxel and B_1, chi_1 of the voxel above it (the inner
                                 condition of the paper's test; = case 0 for an isothermal slab) */
} rt3d_grid_desc;

typedef struct rt3d_ctx rt3d_ctx;

/* Create a context: validates *g on the host, builds the angle set, the per-direction segment
 * tables and the sweep plan, and then allocates all device buffers on the current HIP device.
 * hip_stream is a hipStream_t (NULL = the default stream); every kernel of this context is launched
 * on it.  Size limit of the sweep: a workgroup holds whole x-rows of lines (nx <= 1024 with the
 * default shape), and a band's LDS -- the deposit window of (rows + the angle set's row spread per
 * layer) nx values and two exchange buffers of rows nx values, in float64 -- fits 48 KB when it can
 * (several workgroups per CU), else up to 156 KB (one per CU); with the default shape nx may reach
 * 1024 for up to 24 x 24 angles, 832 for 32 x 32 and 587 for 48 x 48 (ny and nz are limited by
 * memory only).
 * rt3d_validate checks the same without a device.
 * Errors: RT3D_ERR_ARG (bad descriptor or precision, out == NULL, a grid beyond the sweep's limits),
 * RT3D_ERR_OOM, RT3D_ERR_HIP; the reason is in rt3d_last_error(NULL). */
int rt3d_create(rt3d_ctx **out, const rt3d_grid_desc *g, int precision, void *hip_stream);

/* Free every device buffer and the context.  NULL is ignored. */
void rt3d_destroy(rt3d_ctx *ctx);

/* Set the medium (section "Method": opacities go in, the solution stays on the device; section "Test
 * case setup" for the coherent scattering source S = eps B + (1-eps) J): chi (opacity per unit voxel
 * edge, finite and > 0), eps (thermalisation parameter, 0 < eps <= 1) and B (Planck function, finite),
 * each [nz][ny][nx], caller-owned (host or device per ptr_kind; copied, not kept).  Host data is
 * validated on the host; device data is validated by a device check that reads back one flag.
 * Resets J to B and invalidates Lambda*.  Errors: RT3D_ERR_ARG, RT3D_ERR_HIP. */
int rt3d_set_medium(rt3d_ctx *ctx, const double *chi, const double *eps, const double *B,
                    int ptr_kind);

/* Set the current iterate J ([nz][ny][nx], finite): an initial guess or a resumed state.
 * Errors: RT3D_ERR_STATE (no medium), RT3D_ERR_ARG, RT3D_ERR_HIP. */
int rt3d_set_J(rt3d_ctx *ctx, const double *J, int ptr_kind);

/* Copy the current iterate J out.  Errors: RT3D_ERR_STATE, RT3D_ERR_ARG, RT3D_ERR_HIP. */
int rt3d_get_J(rt3d_ctx *ctx, double *J_out, int ptr_kind);

/* One formal solution for all directions (section "Implementation of the formal solution and
 * Lambda* computation": characteristics started on the inner and outer x-y planes and tracked through
 * the periodic grid, every direction independent; the per-voxel collection of the characteristics'
 * contributions is that section's second pass): J_fs = sum_d W_d Ibar(d) for the source S_or_null
 * ([nz][ny][nx], caller-owned, host or device per ptr_kind) or, when S_or_null is NULL, for
 * S = eps B + (1-eps) J (section "Test case setup").  J_fs_out ([nz][ny][nx], caller-owned) receives
 * J_fs.  Boundary light as in the descriptor.  Also records the top-plane intensities of the upward
 * lines.  With host buffers the call synchronises before returning.
 * Errors: RT3D_ERR_STATE (no medium), RT3D_ERR_ARG (null output, bad ptr_kind, non-finite host S),
 * RT3D_ERR_HIP; on error J and the medium are unchanged. */
int rt3d_formal_solution(rt3d_ctx *ctx, const double *S_or_null, double *J_fs_out, int ptr_kind);

/* Build Lambda* for the current chi (section "Implementation of the formal solution and Lambda*
 * computation": the nearest-neighbour Lambda* operator computed from the same characteristics as the
 * formal solution; section "Method" for its role in the operator splitting): the exact 27-point band
 * of Lambda, Lambda*_vu = dJ_v/dS_u for u in the 3x3x3 block of v, kept in float64 inside the context,
 * and the Jacobi coefficients of the OS step derived from it (see rt3d_set_coef_storage).
 * Idempotent until the next rt3d_set_medium.  Errors: RT3D_ERR_STATE (no medium), RT3D_ERR_HIP. */
int rt3d_build_lstar(rt3d_ctx *ctx);

/* Copy Lambda* (section "Implementation of the formal solution and Lambda* computation") out as
 * float64 [27][nz][ny][nx] in the neighbour order o above into the caller-owned buffer out (host or
 * device per ptr_kind; 27 V doubles).  Synchronises before returning.
 * Errors: RT3D_ERR_STATE (not built), RT3D_ERR_ARG (null output, bad ptr_kind), RT3D_ERR_HIP. */
int rt3d_get_lstar(rt3d_ctx *ctx, double *out, int ptr_kind);

/* One OS step (section "Implementation of the operator splitting step": the OS equations
 * (1 - Lambda* (1-eps)) dJ = J_fs - J_old solved by Jacobi ("Jordan") iterations over the 3D grid;
 * section "Method" for the outer iteration), building Lambda* first if needed: S from J, FS,
 * r = J_fs - J, inner_sweeps >= 1 Jacobi sweeps from dJ = 0 (or Gauss-Seidel sweeps, see
 * rt3d_set_os_method), J <- J + dJ, *max_rel_dJ_out = max_v |dJ_v| / |J_v| (may be NULL).
 * Synchronises before returning (it reads the convergence measure back).
 * In the RT3D_FP32_SWEEP form the context keeps an anchor iterate Ja with its float64 formal
 * solution F_a; a step sweeps the source change (1-eps)(J - Ja) in float32 with no boundary light and
 * uses J_fs = F_a + that sweep, summed in float64, so the float32 error scales with |J - Ja| rather
 * than with J.  A float64 sweep re-anchors at the current J on the first step, after rt3d_set_J or
 * rt3d_set_medium, and whenever the last step's c fell below 1e-2 of max_v |J_v - Ja_v| / |J_v|.  The
 * Jacobi coefficients are stored in float32 in this form by default (rt3d_set_coef_storage); the
 * Jacobi arithmetic is float64.
 * Errors: RT3D_ERR_STATE, RT3D_ERR_ARG, RT3D_ERR_NONFINITE (J is then not trustworthy),
 * RT3D_ERR_HIP. */
int rt3d_os_step(rt3d_ctx *ctx, int inner_sweeps, double *max_rel_dJ_out);

/* The outer OS iteration (sections "Method" and "Implementation of the operator splitting step"):
 * rt3d_os_step until max_rel_dJ < tol or max_iter steps, with Ng acceleration when set
 * (rt3d_set_acceleration).  *iters_out and *final_rel_dJ_out (may be NULL) receive the step count and
 * the last c.  The RT3D_FP32_SWEEP form accepts c < tol only from a
 * step whose formal solution was float64 (a re-anchoring step); a float32 step below tol triggers one.  Returns RT3D_ERR_NOT_CONVERGED when max_iter was
 * reached (J and c remain valid), RT3D_ERR_NONFINITE, RT3D_ERR_ARG, RT3D_ERR_STATE, RT3D_ERR_HIP. */
int rt3d_solve_to_convergence(rt3d_ctx *ctx, double tol, int max_iter, int inner_sweeps,
                              int *iters_out, double *final_rel_dJ_out);

/* Ng acceleration of rt3d_solve_to_convergence (the paper names Ng acceleration among the host-side
 * parts of the method, section "Method"): after every OS step the iterate joins a history that
 * restarts at each extrapolation; once it holds ng_every steps, the newest ng_order + 2 iterates
 * x_n, x_{n-1}, ... are replaced by (1 - sum a_i) x_n + sum_i a_i x_{n-i}, where a minimises
 * sum_v (delta_0 - sum_i a_i (delta_0 - delta_i))_v^2 / x_n,v^2 with delta_i = x_{n-i} - x_{n-i-1}.
 * ng_order 0 switches it off (the default); 1 <= ng_order <= 3 needs ng_every >= ng_order + 1.
 * Dot products are reduced in a fixed order, so runs stay bitwise reproducible.  Allocates
 * (ng_order + 2) history vectors of V float64 on the device.
 * Errors: RT3D_ERR_ARG, RT3D_ERR_OOM, RT3D_ERR_HIP. */
int rt3d_set_acceleration(rt3d_ctx *ctx, int ng_order, int ng_every);

/* Anderson mixing of rt3d_solve_to_convergence, an alternative to Ng's extrapolation (not from the
 * paper; the outer iteration is an affine map of J, and mixing over a sliding window accelerates it
 * like a restarted Krylov method): every OS step x -> g joins a window of the newest depth + 1 pairs
 * (x_i, g_i), and from the second step on the next input is g_k - sum_j gamma_j (g_k - g_{k-j}), where
 * gamma minimises sum_v (f_k - sum_j gamma_j (f_k - f_{k-j}))_v^2 / g_k,v^2, f = g - x (the weights of
 * Ng's method); a singular or non-finite solve keeps g_k.  The window slides; in the RT3D_FP32_SWEEP
 * form a step anchored in float64 restarts it from that step's pair.  depth 0 switches it off (the
 * default); 1 <= depth <= 8.  Setting a depth switches Ng acceleration off and rt3d_set_acceleration
 * with ng_order > 0 switches Anderson mixing off.  Dot products are reduced in a fixed order (bitwise
 * reproducible).  Allocates 2 (depth + 1) V float64 on the device.  rt3d_batch_set_anderson is the
 * batched form's counterpart; the adjoint solve does not mix.  Errors: RT3D_ERR_ARG, RT3D_ERR_OOM,
 * RT3D_ERR_HIP. */
int rt3d_set_anderson(rt3d_ctx *ctx, int depth);

/* Inner solve of the OS step (section "Implementation of the operator splitting step": the Fortran
 * code solves the OS equations by Jordan (Jacobi) or Gauss-Seidel iterations; its GPU version uses
 * Jacobi).  RT3D_OS_JACOBI (the default): inner_sweeps Jacobi sweeps from dJ = 0.
 * RT3D_OS_GAUSS_SEIDEL: inner_sweeps multicolour Gauss-Seidel sweeps from dJ = 0, in place.  The
 * colouring is per axis: index i has colour i mod 2, except on x or y (periodic) of odd length, where
 * the last index has colour 2; z (not periodic) has two colours; a sweep visits the colours in the
 * order (cz * ncy + cy) * ncx + cx (8, 12 or 18 passes, one launch each), and every voxel uses the
 * newest dJ of all its neighbours.  Applies to rt3d_os_step and rt3d_solve_to_convergence of this
 * context (either precision); the batched form and the adjoint solve use Jacobi.
 * Errors: RT3D_ERR_ARG (unknown method). */
enum { RT3D_OS_JACOBI = 0, RT3D_OS_GAUSS_SEIDEL = 1 };
int rt3d_set_os_method(rt3d_ctx *ctx, int method);

/* Storage precision of the Jacobi coefficients of the OS step (section "Implementation of the
 * operator splitting step": the Jacobi sweeps read Lambda* in every iteration, which makes the OS step
 * the second most time-consuming part).  The coefficients chi_v Lambda*_vu of the 13 upper neighbours
 * of each voxel (the lower ones follow by reciprocity) are stored in float64 (RT3D_COEF_FP64, the
 * default of the RT3D_FP64 form) or float32 (RT3D_COEF_FP32, the default of the RT3D_FP32_SWEEP form,
 * half the bytes per sweep); the Jacobi arithmetic, the per-voxel diagonal terms and Lambda* itself
 * stay float64.  The coefficients only precondition the OS step: float32 storage changes the iterates
 * by about 1e-7 of dJ but not the fixed point, which the residual J_fs - J sets.  Allocates the new
 * store (13 V values) on the device before freeing the old one, and re-derives the coefficients from
 * Lambda* when it is built.  Applies to rt3d_os_step, rt3d_solve_to_convergence and the adjoint solve
 * of this context.  Errors: RT3D_ERR_ARG (unknown storage), RT3D_ERR_OOM, RT3D_ERR_HIP (the context
 * keeps its previous storage after RT3D_ERR_OOM). */
enum { RT3D_COEF_FP64 = 0, RT3D_COEF_FP32 = 1 };
int rt3d_set_coef_storage(rt3d_ctx *ctx, int storage);

/* Top-plane intensities of the upward lines from the last formal solution, [n_theta/2 * n_phi][ny][nx]
 * in direction order (the upward directions are d = n_dir/2 .. n_dir-1); entry (j,i) belongs to the
 * line through (i+1/2, j+1/2, nz).  Errors: RT3D_ERR_STATE (no FS yet), RT3D_ERR_ARG, RT3D_ERR_HIP. */
int rt3d_get_emergent_top(rt3d_ctx *ctx, double *out, int ptr_kind);

/* Per-kernel timing with HIP events on the context stream: 0 off; 1 every launch of the source,
 * sweep, reduce, Lambda*, coefficient and Jacobi kernels is bracketed by events; 2 sampled: the same
 * except for the inner sweeps of an OS step, of which the intermediate ones (all but the first, from
 * dJ = 0, and the last, which updates J) are timed as one group by a single pair of events (with two
 * or fewer sweeps the first is timed; Gauss-Seidel: its second sweep).  Mode 2 keeps the events' own
 * cost (about 4% of a step with mode 1) out of the timed work.  Durations are accumulated with the
 * number of launches they cover (rt3d_get_stats: per kernel "launches", "timed", "total_ms");
 * changing the mode clears them.  Errors: RT3D_ERR_ARG. */
int rt3d_set_timing(rt3d_ctx *ctx, int enable);

/* The per-step record since the last rt3d_set_medium, rt3d_set_J or start of
 * rt3d_solve_to_convergence (at most 100000 steps): max |dJ|/|J| (c_out), host wall milliseconds of the
 * step (ms_out) and flags (flags_out: 1 = the step's formal solution was float64, 2 = Ng extrapolated
 * after it, 4 = Anderson mixing after it).  Fills the first min(n, max_n) entries of the arrays (any may be NULL) and returns n, the
 * number of records.  Errors: RT3D_ERR_ARG. */
int rt3d_get_history(rt3d_ctx *ctx, double *c_out, double *ms_out, int *flags_out, int max_n);

/* Statistics as a NUL-terminated JSON object: grid, angles, precision, outer iterations, inner
 * sweeps, device bytes, the sweep plan (workgroups, shape, mean segments per voxel and angle, largest
 * deposit window in rows, LDS bytes of a sweep workgroup), and per-kernel {launches, total_ms} when
 * timing is enabled.
 * Errors: RT3D_ERR_ARG (buffer too small or NULL). */
int rt3d_get_stats(rt3d_ctx *ctx, char *json_buf, int buflen);

/* Static text for a status code. */
const char *rt3d_status_str(int status);

/* Last error message of a context ("" if none); valid until the next call on the context.  With
 * ctx == NULL: the message of the calling thread's last rt3d_create, rt3d_batch_create or
 * rt3d_validate ("" if it succeeded), valid until that thread's next such call. */
const char *rt3d_last_error(const rt3d_ctx *ctx);

/* ---- adjoint: gradients through the converged solution ------------------------------------
 * An extension of the method (the paper computes the forward solution only).  For a loss L of the
 * emergent top intensities I_em (the layout of rt3d_get_emergent_top), given g_em = dL/dI_em
 * ([n_theta/2 * n_phi][ny][nx]), computes dL/dchi and dL/deps per voxel ([nz][ny][nx]) through the
 * fixed point J = Lambda(chi) (eps B + (1-eps) J) + J_bc(chi) at the context's current J, which should
 * be converged (call after rt3d_solve_to_convergence; the gradient is that of the fixed point through
 * the current J, so its accuracy follows that of J).  B, I_top and the bottom light are constants.
 * Method: dL/dS by reverse-mode differentiation of the exact segment integration along the lines;
 * the adjoint fixed point mu = dL/dS + Lambda^T (1-eps) mu, solved through reciprocity
 * (chi_v Lambda_vu = chi_u Lambda_uv) as the forward-form system (1 - Lambda (1-eps)) nu = dL/dS / chi,
 * nu = mu / chi, by the library's operator-splitting iteration (inner_sweeps Jacobi sweeps per step,
 * Ng acceleration as set by rt3d_set_acceleration but with unit weights, stopped when
 * max|d nu| < tol max|nu| or after max_iter steps); then dL/deps = mu (B - J) and dL/dchi
 * from a second reverse-mode pass.  All of it runs in float64 (also in the RT3D_FP32_SWEEP form, whose
 * float32 Jacobi coefficients only precondition).  Overwrites J_fs and the emergent intensities with
 * those of the current J.  *iters_out and *final_rel_out (may be NULL) receive the adjoint steps and
 * the last max|d nu| / max|nu|.  The first call allocates 2 n_dir V + 5 V + n_em float64 on the
 * device (kept until rt3d_destroy).  Deterministic (fixed summation order).
 * Errors: RT3D_ERR_STATE (no medium), RT3D_ERR_ARG (null arrays, non-finite host g_em, bad
 * tol/max_iter/inner_sweeps), RT3D_ERR_NOT_CONVERGED (max_iter reached; the outputs hold the
 * gradients of the last iterate), RT3D_ERR_NONFINITE, RT3D_ERR_OOM, RT3D_ERR_HIP. */
int rt3d_adjoint_emergent(rt3d_ctx *ctx, const double *g_em, double tol, int max_iter, int inner_sweeps,
                          double *dL_dchi, double *dL_deps, int ptr_kind, int *iters_out,
                          double *final_rel_out);

/* ---- sweep workgroup shape and its tuning -------------------------------------------------- */

/* The sweep workgroup shapes: shape i runs threads[i] threads, each carrying lines[i] lines of
 * both directions of an x-mirrored direction pair.  Fills min(count, max_n) entries of the arrays
 * (either may be NULL) and returns the count.  Host-only. */
int rt3d_sweep_shapes(int *threads, int *lines, int max_n);

/* Rebuild the sweep plan (bands and work items) for a shape; medium, J and Lambda* are kept, and
 * the results change only by the summation order of the partial planes.  Errors: RT3D_ERR_ARG
 * (shape out of range, or its bands do not fit the grid; the context is unchanged), RT3D_ERR_OOM,
 * RT3D_ERR_HIP (after these two the context cannot sweep -- RT3D_ERR_STATE -- until a later call
 * succeeds). */
int rt3d_set_sweep_shape(rt3d_ctx *ctx, int shape);

/* Autotuner of the sweep shape.  Times `repeats` formal solutions (from the current J, in the
 * context's precision) for every shape that fits the grid, installs the fastest and, when
 * cache_path is neither NULL nor empty, records it in a JSON cache keyed by device, precision and
 * grid.  When the cache already holds the key, its shape is installed without measuring.
 * *shape_out (may be NULL) receives the shape; ms_out (may be NULL, one entry per shape) the
 * milliseconds per formal solution, -1 where not measured.  Overwrites J_fs and the emergent
 * intensities.  Errors: RT3D_ERR_STATE (no medium), RT3D_ERR_ARG (repeats < 1, unwritable
 * cache), RT3D_ERR_OOM, RT3D_ERR_HIP. */
int rt3d_autotune(rt3d_ctx *ctx, const char *cache_path, int repeats, int *shape_out, double *ms_out);

/* ---- batched form: many problems in one launch per kernel ----------------------------------
 * An extension of the method (the paper solves one wavelength at a time): a batch holds n members,
 * independent problems with grid descriptors of their own (sizes and angle sets may differ), in one
 * precision and one sweep shape -- for instance the wavelengths of a spectrum.  An outer iteration
 * advances every member that has not stopped, with one launch per kernel for all of them; the
 * iteration is captured once in a HIP graph and replayed.  Each member's stopping rule, FP32
 * re-anchoring and Ng schedule are decided on the device with the rules of rt3d_os_step,
 * rt3d_solve_to_convergence and rt3d_set_acceleration, and the arithmetic is that of a single
 * context, so a member's iterates are bitwise those of solving it alone in a context with the same
 * sweep shape.  Member buffers follow the layouts above. */
typedef struct rt3d_batch rt3d_batch;

enum {
    RT3D_MEMBER_RUNNING = 0,     /* still iterating */
    RT3D_MEMBER_CONVERGED = 1,   /* c < tol (in the FP32 form from a float64 formal solution) */
    RT3D_MEMBER_MAX_ITER = 2,    /* stopped after max_iter steps; J and c are valid */
    RT3D_MEMBER_NONFINITE = 3    /* NaN or Inf in dJ or J */
};

/* Create a batch of n_members >= 1 problems: descs[i] (host array) as for rt3d_create, precision
 * and sweep_shape (rt3d_sweep_shapes) shared by all.  hip_stream: a hipStream_t other than the
 * legacy default stream (graphs are captured from it), or NULL for a stream the batch creates (default
 * priority) and destroys.  Errors: RT3D_ERR_ARG (any bad descriptor, n_members < 1, bad precision
 * or shape, a shape whose bands do not fit a grid), RT3D_ERR_OOM, RT3D_ERR_HIP; the reason, prefixed
 * "member i:" when a member failed, is in rt3d_batch_last_error(NULL). */
int rt3d_batch_create(rt3d_batch **out, int n_members, const rt3d_grid_desc *descs, int precision,
                      int sweep_shape, void *hip_stream);

/* Free the batch, its members and (if it created it) its stream.  NULL is ignored. */
void rt3d_batch_destroy(rt3d_batch *b);

/* Number of members (0 for NULL). */
int rt3d_batch_size(const rt3d_batch *b);

/* Last error message of the batch ("" if none), prefixed "member i:" when a member failed.  With
 * b == NULL: as rt3d_last_error(NULL), the calling thread's last failed creation. */
const char *rt3d_batch_last_error(const rt3d_batch *b);

/* Per member, exactly as rt3d_set_medium / rt3d_set_J / rt3d_get_J of a context; member in
 * [0, n).  rt3d_batch_get_Jfs copies the member's last formal solution J_fs out (RT3D_ERR_STATE
 * before the first).  Errors as there, plus RT3D_ERR_ARG for a member out of range. */
int rt3d_batch_set_medium(rt3d_batch *b, int member, const double *chi, const double *eps,
                          const double *B, int ptr_kind);
int rt3d_batch_set_J(rt3d_batch *b, int member, const double *J, int ptr_kind);
int rt3d_batch_get_J(rt3d_batch *b, int member, double *J_out, int ptr_kind);
int rt3d_batch_get_Jfs(rt3d_batch *b, int member, double *Jfs_out, int ptr_kind);

/* Ng acceleration for every member, as rt3d_set_acceleration (order 0 switches all acceleration off,
 * Anderson mixing included).  Errors as there; after an error the batch runs without acceleration
 * until a setter succeeds. */
int rt3d_batch_set_acceleration(rt3d_batch *b, int ng_order, int ng_every);

/* Anderson mixing for every member, as rt3d_set_anderson (depth 0..8; 0 switches all acceleration
 * off).  Like the context calls, this and rt3d_batch_set_acceleration replace each other's setting.
 * Each member keeps its own window in the member state on the device, so its iterates are bitwise
 * those of solving it alone with the same depth.  Errors as there; after an error the batch runs
 * without acceleration until a setter succeeds. */
int rt3d_batch_set_anderson(rt3d_batch *b, int depth);

/* Rebuild every member's plan for a shape, as rt3d_set_sweep_shape.  After RT3D_ERR_ARG from a
 * member the batch cannot sweep (RT3D_ERR_STATE) until a shape change succeeds. */
int rt3d_batch_set_sweep_shape(rt3d_batch *b, int shape);

/* One formal solution of every member from its current J (S = eps B + (1-eps) J, boundary light
 * as in its descriptor, float32 sweeps in the RT3D_FP32_SWEEP form, as rt3d_formal_solution), in
 * one launch per kernel; read the results with rt3d_batch_get_Jfs.
 * Errors: RT3D_ERR_STATE (a member without medium), RT3D_ERR_HIP. */
int rt3d_batch_formal_solution(rt3d_batch *b);

/* Iterate every member with OS steps of inner_sweeps Jacobi sweeps until it stops (see the member
 * states above), replaying the captured iteration and reading the member states back every
 * poll_every >= 1 replays; the iterates do not depend on poll_every.  Lambda* is built first where
 * needed.  Per member (arrays of n entries, each may be NULL): iterations, last c (NaN for a
 * non-finite member) and state.  Returns RT3D_OK when every member converged, else
 * RT3D_ERR_NONFINITE if any member turned non-finite, else RT3D_ERR_NOT_CONVERGED; RT3D_ERR_ARG
 * (tol <= 0, max_iter, inner_sweeps or poll_every < 1), RT3D_ERR_STATE (a member without medium),
 * RT3D_ERR_OOM, RT3D_ERR_HIP. */
int rt3d_batch_solve(rt3d_batch *b, double tol, int max_iter, int inner_sweeps, int poll_every,
                     int *iters_out, double *final_rel_out, int *status_out);

/* Autotuner of the batch's sweep shape: as rt3d_autotune, timing batched formal solutions; the
 * cache key holds the device, the precision and the multiset of member grids. */
int rt3d_batch_autotune(rt3d_batch *b, const char *cache_path, int repeats, int *shape_out,
                        double *ms_out);

/* Statistics of the batch and of its last solve as a NUL-terminated JSON object (members, voxels,
 * voxel-angles, shape, replays, polls, solve milliseconds, iteration counts).
 * Errors: RT3D_ERR_ARG (buffer too small or NULL). */
int rt3d_batch_get_stats(rt3d_batch *b, char *json_buf, int buflen);

/* ---- allocation-free formal solution ------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the formal solution of rt3d_formal_solution without a context.
 * chi, S ([nz][ny][nx]), I_bot ([ny][nx], the intensity entering the bottom plane, e.g. B of the
 * bottom layer; NULL or bottom_bc 1 for none) and J_fs ([nz][ny][nx], the output) are caller-owned
 * device buffers valid on hip_stream (a hipStream_t; NULL = the default stream).  The grid descriptor
 * is taken as for rt3d_create (bottom_bc 0 or 1; the LTE-diffusion condition needs a context), with
 * the default sweep shape (shape 0 of rt3d_sweep_shapes); J_fs is bitwise what rt3d_formal_solution
 * of a context with that shape gives for the same S and boundary light.  The library allocates no
 * device memory for it: the packed medium, the plan's tables and the partial planes live in a
 * file-scope device array of 128 MiB per device (held from the library's load until the process
 * ends); direction pairs are swept in ranges whose partial planes fit.  Host memory is used for the
 * plan.  Calls that overlap on one device (other streams or threads) share that array and race; the
 * call returns after its work on hip_stream has finished.  Errors: RT3D_ERR_ARG (bad descriptor, null
 * pointer, bottom_bc 2, a grid beyond the sweep's limits, or one whose medium and tables or one pair's
 * partial planes exceed the 128 MiB), RT3D_ERR_HIP; the reason is in rt3d_last_error(NULL). */
int rt3d_formal_solution_noalloc(const rt3d_grid_desc *g, const double *chi, const double *S,
                                 const double *I_bot, double *J_fs, void *hip_stream);

/* ---- host-only helpers (no device needed) ------------------------------------------------- */

/* The angle set: mu[d], ox[d], oy[d] (direction cosines) and weights w[d] for d = a*n_phi + b,
 * each array n_theta*n_phi long (caller-owned host memory).  Errors: RT3D_ERR_ARG. */
int rt3d_quadrature(int n_theta, int n_phi, double *mu, double *ox, double *oy, double *w);

/* Segments of the line through (i0+1/2, j0+1/2, nz) for direction d inside layer k, in travel order:
 * voxel column offsets (di[s], dj[s]) relative to (i0, j0) -- not reduced modulo the grid -- and path
 * lengths len[s].  Returns the number of segments (>= 1) or RT3D_ERR_ARG (also when max_seg is too
 * small).  The table is the same for every line of the direction (translation invariance). */
int rt3d_segment_table(const rt3d_grid_desc *g, int d, int k, int *di, int *dj, double *len,
                       int max_seg);

/* Validate a descriptor (including the sweep's size limits for the shape rt3d_create would take)
 * and (optionally, any may be NULL) host medium arrays exactly as rt3d_create / rt3d_set_medium do,
 * on the host only.  Returns RT3D_OK or RT3D_ERR_ARG; the reason is in rt3d_last_error(NULL). */
int rt3d_validate(const rt3d_grid_desc *g, const double *chi, const double *eps, const double *B);

#ifdef __cplusplus
}
#endif

#endif /* RT3D_H */
