// rt3d.hip -- HIP kernels (gfx950) and C ABI of the 3D radiative-transfer scattering hot path:
// formal solution (FS) along characteristics on a grid periodic in x,y, mean intensity J, the
// 27-point Lambda* operator and the operator-splitting (OS) step solved by Jacobi sweeps
// (Hauschildt & Baron, "A 3D radiative transfer framework XIII", sections "Implementation of the
// formal solution and Lambda* computation" and "Implementation of the operator splitting step").
//
// Kernels
//   source_kernel   S = eps B + (1-eps) J packed with chi as {chi, S} per voxel (one 16-byte gather
//                   per segment in the sweep).
//   sweep_kernel    one workgroup per (x-mirrored direction pair, band of line rows): every thread
//                   owns a few slots, each carrying a line of both directions through the same voxel
//                   (the B lines move between slots at x-face crossings), down (or up) through all
//                   layers; the two lines share the voxel's chi,S gather, exponential and deposit.
//                   All lines of a direction share one segment table, so segment s of every slot in
//                   a layer lands in a distinct voxel: the deposits D_s go into an LDS window without
//                   atomics, one segment index at a time, and each layer's window is written once to
//                   a per-band partial plane P.  Deterministic; no float atomics.  The float64
//                   exponential uses a 16-entry table of 2^(j/16) (per context, copied to LDS).
//   reduce_kernel_pair  per voxel (two neighbours of a row per thread), sums the partial planes of
//                   all directions in a fixed order: J_fs = (1/chi) sum_d W_d |mu_d| sum_bands P, and
//                   the OS right-hand side chi (J_fs - J).
//   lstar_kernel    per voxel, the 27 derivatives dJ_v/dS_u along the lines through v (exact band).
//   coef_kernel     the Jacobi coefficients: chi_v Lambda*_vu for the 13 upper neighbours (the
//                   lower ones follow by reciprocity) and the per-voxel scalings.
//   jacobi_kernel_column  one Jacobi sweep of the OS equations (27-point stencil), a thread marching
//                   up a column of 4 voxels; the last sweep also updates J and reduces max |dJ|/|J|
//                   (and flags NaN/Inf).  jacobi_kernel_colour: one colour pass of the multicolour
//                   Gauss-Seidel alternative.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <optional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rt3d.h"
#include "context.h"
#include "geometry.h"
#include "kernels.h"
#include "tune_cache.h"

namespace rt3d_host {

int fail(rt3d_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(rt3d_ctx *c, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (c) c->err = m;
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? RT3D_ERR_OOM : RT3D_ERR_HIP;
}

hipEvent_t get_event(rt3d_ctx *c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct TimedLaunch {
    rt3d_ctx *c;
    int kid;
    hipEvent_t a = nullptr, b = nullptr;
    bool on;
    // chosen: in sampled timing (mode 2) only the chosen launches are bracketed by events
    TimedLaunch(rt3d_ctx *ctx, int id, bool chosen = true)
        : c(ctx), kid(id), on(ctx->timing == 1 || (ctx->timing == 2 && chosen))
    {
        if (on) {
            a = get_event(c);
            b = get_event(c);
            if (a) hipEventRecord(a, c->stream);
        }
    }
    ~TimedLaunch()
    {
        if (on && a && b) {
            hipEventRecord(b, c->stream);
            c->pending.push_back({kid, a, b});
            c->kernel_timed[kid] += 1;
        }
        c->kernel_launches[kid] += 1;
    }
};

// Sampled timing of n consecutive launches of one kernel as a group (one pair of events): the
// launches are counted by their own TimedLaunch objects, constructed with chosen = false.
struct TimedGroup {
    rt3d_ctx *c;
    int kid, n;
    hipEvent_t a = nullptr, b = nullptr;
    TimedGroup(rt3d_ctx *ctx, int id, int count) : c(ctx), kid(id), n(count)
    {
        if (c->timing == 2 && n > 0) {
            a = get_event(c);
            b = get_event(c);
            if (a) hipEventRecord(a, c->stream);
        }
    }
    void end()
    {
        if (a && b) {
            hipEventRecord(b, c->stream);
            c->pending.push_back({kid, a, b});
            c->kernel_timed[kid] += n;
        }
        a = b = nullptr;
    }
    ~TimedGroup() { end(); }
};

// Resolve pending timing events (call after the stream has been synchronised).
void resolve_timing(rt3d_ctx *c)
{
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) c->kernel_ms[p.kid] += ms;
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
}

int sync(rt3d_ctx *c)
{
    HIP_TRY(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    resolve_timing(c);
    return RT3D_OK;
}

int check_launch(rt3d_ctx *c, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, what);
    return RT3D_OK;
}

int validate_desc(const rt3d_grid_desc *g, std::string &msg)
{
    if (!g) { msg = "grid descriptor is NULL"; return RT3D_ERR_ARG; }
    if (g->nx < 3 || g->ny < 3 || g->nz < 3) { msg = "nx, ny, nz must be >= 3"; return RT3D_ERR_ARG; }
    if (long(g->nx) * g->ny * g->nz > (1L << 31) / 27) { msg = "grid too large"; return RT3D_ERR_ARG; }
    if (g->n_theta < 2 || (g->n_theta % 2) != 0) { msg = "n_theta must be even and >= 2"; return RT3D_ERR_ARG; }
    if (g->n_phi < 4 || (g->n_phi % 4) != 0) { msg = "n_phi must be a positive multiple of 4"; return RT3D_ERR_ARG; }
    if (!std::isfinite(g->I_top) || g->I_top < 0.0) { msg = "I_top must be finite and >= 0"; return RT3D_ERR_ARG; }
    if (g->bottom_bc < 0 || g->bottom_bc > 2) { msg = "bottom_bc must be 0, 1 or 2"; return RT3D_ERR_ARG; }
    return RT3D_OK;
}

int validate_medium_host(long V, const double *chi, const double *eps, const double *B, std::string &msg)
{
    for (long v = 0; chi && v < V; ++v)
        if (!std::isfinite(chi[v]) || !(chi[v] > 0.0)) { msg = "chi must be finite and > 0"; return RT3D_ERR_ARG; }
    for (long v = 0; eps && v < V; ++v)
        if (!(eps[v] > 0.0) || !(eps[v] <= 1.0)) { msg = "eps must lie in (0, 1]"; return RT3D_ERR_ARG; }
    for (long v = 0; B && v < V; ++v)
        if (!std::isfinite(B[v])) { msg = "B must be finite"; return RT3D_ERR_ARG; }
    return RT3D_OK;
}

hipMemcpyKind kind_in(int ptr_kind) { return ptr_kind == RT3D_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind kind_out(int ptr_kind) { return ptr_kind == RT3D_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

dim3 plane_grid(const rt3d_ctx *c)
{
    return dim3((c->g.nx * c->g.ny + kPlaneThreads - 1) / kPlaneThreads, c->g.nz);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2) in linear order.
// Padding the chunks of a plane to a multiple of 8 sends a chunk's blocks of every plane to the same
// XCD, so the plane-below data a Jacobi sweep re-reads is in that XCD's L2.  Padding blocks exit.
// the reduction's grid: one thread per pair of neighbouring voxels of a row
dim3 pair_grid(const rt3d_ctx *c)
{
    return dim3(((c->g.nx + 1) / 2 * c->g.ny + kPlaneThreads - 1) / kPlaneThreads, c->g.nz);
}

dim3 plane_grid_xcd(const rt3d_ctx *c)
{
    const unsigned chunks = (c->g.nx * c->g.ny + kPlaneThreads - 1) / kPlaneThreads;
    return dim3((chunks + 7) / 8 * 8, c->g.nz);
}

int launch_source(rt3d_ctx *c, const double *S_given, const double *Ja, bool fp32)
{
    SourceArgs a{};
    a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz;
    a.chi = c->chi; a.eps = c->eps; a.B = c->B; a.J = c->J; a.S_given = S_given; a.Ja = Ja;
    a.cs = c->cs;
    TimedLaunch t(c, K_SOURCE);
    if (!fp32)
        hipLaunchKernelGGL(source_kernel<double>, plane_grid(c), dim3(kPlaneThreads), 0, c->stream, a);
    else
        hipLaunchKernelGGL(source_kernel<float>, plane_grid(c), dim3(kPlaneThreads), 0, c->stream, a);
    return check_launch(c, "source_kernel");
}

// diff: formal solution of a source difference (no boundary light; top-plane light added to the
// anchor's)
int launch_sweep(rt3d_ctx *c, bool fp32, bool diff)
{
    SweepArgs a{};
    a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz;
    a.n_down = c->A.n_dir / 2;
    a.pseg = c->pseg; a.player = c->player;
    a.pairs = c->pairs; a.items = c->items;
    a.cs = c->cs;
    a.Ibot = (c->g.bottom_bc != 1 && !diff) ? c->B : nullptr;
    a.Islope = (c->g.bottom_bc == 2 && !diff) ? c->bot_slope : nullptr;
    a.I_top = diff ? 0.0 : c->g.I_top;
    a.P = c->P;
    a.Iem = c->Iem;
    a.Iem_base = diff ? c->Iem_a : nullptr;
    a.xtab = c->xtab;
    const size_t smem = sweep_smem_bytes(c->plan, fp32);
    const dim3 grid(c->plan.items.size());
    TimedLaunch t(c, K_SWEEP);
    if (fp32) c->fp32_sweeps += 1; else c->fp64_sweeps += 1;
#define RT3D_LAUNCH_SWEEP(NT_, LPT_)                                                           \
    do {                                                                                          \
        if (!fp32)                                                                                \
            hipLaunchKernelGGL((sweep_kernel<double, NT_, LPT_>), grid, dim3(NT_), smem, c->stream, a); \
        else                                                                                      \
            hipLaunchKernelGGL((sweep_kernel<float, NT_, LPT_>), grid, dim3(NT_), smem, c->stream, a);  \
    } while (0)
    switch (c->sweep_shape) {
    case 1: RT3D_LAUNCH_SWEEP(512, 4); break;
    case 2: RT3D_LAUNCH_SWEEP(256, 8); break;
    case 3: RT3D_LAUNCH_SWEEP(1024, 2); break;
    case 4: RT3D_LAUNCH_SWEEP(256, 4); break;
    case 5: RT3D_LAUNCH_SWEEP(256, 2); break;
    default: RT3D_LAUNCH_SWEEP(512, 2); break;
    }
#undef RT3D_LAUNCH_SWEEP
    return check_launch(c, "sweep_kernel");
}

int launch_reduce(rt3d_ctx *c, bool with_residual, bool fp32, const double *base)
{
    ReduceArgs a{};
    a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz; a.n_pair = c->plan.n_pair;
    a.pairs = c->pairs; a.row_min = c->row_min; a.P = c->P; a.chi = c->chi;
    a.J = c->J; a.base = base; a.Jfs = c->Jfs; a.rb = with_residual ? c->r : nullptr;
    TimedLaunch t(c, K_REDUCE);
    if (!fp32)
        hipLaunchKernelGGL(reduce_kernel_pair<double>, pair_grid(c), dim3(kPlaneThreads), 0, c->stream, a);
    else
        hipLaunchKernelGGL(reduce_kernel_pair<float>, pair_grid(c), dim3(kPlaneThreads), 0, c->stream, a);
    return check_launch(c, "reduce_kernel");
}

// S (given, or from J) -> J_fs (and r when with_residual), sweeps in float32 when fp32
int run_fs(rt3d_ctx *c, const double *S_dev, bool with_residual, bool fp32)
{
    if (!c->plan_ok) return fail(c, RT3D_ERR_STATE, "no sweep plan (a shape change failed)");
    int rc = launch_source(c, S_dev, nullptr, fp32);
    if (!rc) rc = launch_sweep(c, fp32, false);
    if (!rc) rc = launch_reduce(c, with_residual, fp32, nullptr);
    if (!rc) c->have_fs = true;
    return rc;
}

// FP32 form, difference step: J_fs = F_a + FS32((1 - eps)(J - Ja)) with no boundary light
int run_fs_difference(rt3d_ctx *c)
{
    if (!c->plan_ok) return fail(c, RT3D_ERR_STATE, "no sweep plan (a shape change failed)");
    int rc = launch_source(c, nullptr, c->Ja, true);
    if (!rc) rc = launch_sweep(c, true, true);
    if (!rc) rc = launch_reduce(c, true, true, c->Fa);
    if (!rc) c->have_fs = true;
    return rc;
}

// FP32 form, anchor refresh: a float64 formal solution at the current J becomes the new anchor
int refresh_anchor(rt3d_ctx *c)
{
    int rc = run_fs(c, nullptr, true, false);
    if (rc) return rc;
    const size_t vb = size_t(c->V) * sizeof(double);
    HIP_TRY(c, hipMemcpyAsync(c->Ja, c->J, vb, hipMemcpyDeviceToDevice, c->stream), "anchor J");
    HIP_TRY(c, hipMemcpyAsync(c->Fa, c->Jfs, vb, hipMemcpyDeviceToDevice, c->stream), "anchor J_fs");
    HIP_TRY(c, hipMemcpyAsync(c->Iem_a, c->Iem, size_t(c->A.n_dir / 2) * c->g.nx * c->g.ny * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream), "anchor top light");
    c->anchor_valid = true;
    c->force_refresh = false;
    return RT3D_OK;
}

int ensure_lstar(rt3d_ctx *c)
{
    if (c->have_lstar) return RT3D_OK;
    if (!c->plan_ok) return fail(c, RT3D_ERR_STATE, "no sweep plan (a shape change failed)");
    LstarArgs a{};
    a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz; a.n_pair = c->plan.n_pair;
    a.early_exit = c->lstar_early_exit;
    a.pairs = c->pairs; a.seg_off = c->seg_off; a.seg_n = c->seg_n; a.seg_ai = c->seg_ai;
    a.seg_bi = c->seg_bi; a.seg_len = c->seg_len64; a.chi = c->chi; a.L = c->L;
    a.xtab = c->xtab;
    {
        TimedLaunch t(c, K_LSTAR);
        const dim3 grid((c->g.nx * c->g.ny + kLstarThreads - 1) / kLstarThreads, c->g.nz);
        hipLaunchKernelGGL(lstar_kernel, grid, dim3(kLstarThreads), 0, c->stream, a);
    }
    int rc = check_launch(c, "lstar_kernel");
    if (rc) return rc;
    return finish_lstar(c);
}

// The Jacobi coefficients from Lambda* (after it was built into c->L)
int finish_lstar(rt3d_ctx *c)
{
    int rc;
    {
        TimedLaunch t(c, K_COEF);
        if (c->coef_fp32)
            hipLaunchKernelGGL(coef_kernel<float>, plane_grid(c), dim3(kPlaneThreads), 0, c->stream, c->g.nx,
                               c->g.ny, c->g.nz, c->L, c->chi, c->eps, c->Kc32, c->invD, c->Ecoef);
        else
            hipLaunchKernelGGL(coef_kernel<double>, plane_grid(c), dim3(kPlaneThreads), 0, c->stream, c->g.nx,
                               c->g.ny, c->g.nz, c->L, c->chi, c->eps, c->Kc, c->invD, c->Ecoef);
    }
    rc = check_launch(c, "coef_kernel");
    if (rc) return rc;
    c->have_lstar = true;
    return RT3D_OK;
}

int launch_jacobi_args(rt3d_ctx *c, const JacobiArgs &a, bool reverse = false);
int gauss_seidel_sweeps(rt3d_ctx *c, int M);

int launch_jacobi(rt3d_ctx *c, const double *w_in, double *w_out, bool update, bool chosen, bool reverse)
{
    JacobiArgs a{};
    const bool f32 = c->precision == RT3D_FP32_SWEEP;
    a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz;
    a.b = c->r; a.w_in = w_in; a.w_out = w_out;
    a.Kc = c->coef_fp32 ? static_cast<const void *>(c->Kc32) : static_cast<const void *>(c->Kc);
    a.invD = c->invD; a.E = c->Ecoef;
    a.J = update ? c->J : nullptr;
    a.maxrel = c->d_maxrel; a.nonfinite = c->d_flag;
    a.Ja = (f32 && update) ? c->Ja : nullptr;
    a.maxdist = c->d_maxdist;
    TimedLaunch t(c, K_JACOBI, chosen);
    return launch_jacobi_args(c, a, reverse);
}

// M multicolour Gauss-Seidel sweeps from dJ = 0, colour after colour in the order
// (cz * ncy + cy) * ncx + cx, with (1 - eps) dJ kept in place in dJa; the colour passes of the last
// sweep also update J and fold in the convergence measures.
int gauss_seidel_sweeps(rt3d_ctx *c, int M)
{
    const bool f32 = c->precision == RT3D_FP32_SWEEP;
    const bool k32 = c->coef_fp32 != 0;
    HIP_TRY(c, hipMemsetAsync(c->dJa, 0, size_t(c->V) * sizeof(double), c->stream), "memset");
    JacobiArgs a{};
    a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz;
    a.b = c->r; a.w_in = c->dJa; a.w_out = c->dJa;
    a.Kc = k32 ? static_cast<const void *>(c->Kc32) : static_cast<const void *>(c->Kc);
    a.invD = c->invD; a.E = c->Ecoef;
    a.maxrel = c->d_maxrel; a.nonfinite = c->d_flag;
    a.maxdist = c->d_maxdist;
    const int ncx = axis_colours(c->g.nx, true), ncy = axis_colours(c->g.ny, true), ncz = axis_colours(c->g.nz, false);
    for (int m = 0; m < M; ++m) {
        TimedLaunch t(c, K_JACOBI, m == std::min(1, M - 1));   // one record per sweep (all its passes)
        const bool last = m == M - 1;
        a.J = last ? c->J : nullptr;
        a.Ja = (f32 && last) ? c->Ja : nullptr;
        for (int cz = 0; cz < ncz; ++cz)
            for (int cy = 0; cy < ncy; ++cy)
                for (int cx = 0; cx < ncx; ++cx) {
                    const int3 col = make_int3(cx, cy, cz);
                    const int3 cnt = make_int3(colour_count(cx, c->g.nx, true), colour_count(cy, c->g.ny, true),
                                               colour_count(cz, c->g.nz, false));
                    const long total = long(cnt.x) * cnt.y * cnt.z;
                    const dim3 grid(unsigned((total + kPlaneThreads - 1) / kPlaneThreads));
                    if (k32)
                        hipLaunchKernelGGL(jacobi_kernel_colour<float>, grid, dim3(kPlaneThreads), 0, c->stream, a, col, cnt);
                    else
                        hipLaunchKernelGGL(jacobi_kernel_colour<double>, grid, dim3(kPlaneThreads), 0, c->stream, a, col, cnt);
                    int rc = check_launch(c, "jacobi_kernel_colour");
                    if (rc) return rc;
                }
    }
    return RT3D_OK;
}

int launch_jacobi_args(rt3d_ctx *c, const JacobiArgs &a, bool reverse)
{
    launch_jacobi_sweep(a, c->jacobi_xcd, c->coef_fp32 != 0, c->stream, reverse && c->jacobi_alternate,
                        c->jacobi_height, c->jacobi_walk);
    return check_launch(c, "jacobi_kernel");
}

// Extrapolate J from the ring entries, newest = index m (ring of ng_order + 2 vectors): dot
// products, the small solve and the combination all run on the device, with no host round trip.
int ng_step(rt3d_ctx *c, int m)
{
    NgArgs a{};
    a.V = c->V;
    a.order = c->ng_order;
    a.hist = c->ng_hist;
    a.work = c->ng_work;
    a.J = c->J;
    hipLaunchKernelGGL(ng_dots_kernel, dim3(kNgBlocks), dim3(kNgThreads), 0, c->stream, a, m);
    int rc = check_launch(c, "ng_dots_kernel");
    if (rc) return rc;
    hipLaunchKernelGGL(ng_solve_kernel, dim3(1), dim3(kNgThreads), 0, c->stream, a);
    rc = check_launch(c, "ng_solve_kernel");
    if (rc) return rc;
    hipLaunchKernelGGL(ng_combine_kernel, dim3((c->V + 255) / 256), dim3(256), 0, c->stream, a, m);
    return check_launch(c, "ng_combine_kernel");
}

// The next input of the outer iteration by Anderson mixing of the window slots[0..k] (oldest first):
// dot products, the small solve and the combination on the device, no host round trip.
int anderson_step(rt3d_ctx *c, int k, const int *slots)
{
    AaArgs a{};
    a.V = c->V;
    a.k = k;
    for (int q = 0; q <= k; ++q) a.slot[q] = slots[q];
    a.X = c->aa_x;
    a.G = c->aa_g;
    a.work = c->aa_work;
    a.J = c->J;
    hipLaunchKernelGGL(aa_dots_kernel, dim3(kAaBlocks), dim3(kAaThreads), 0, c->stream, a);
    int rc = check_launch(c, "aa_dots_kernel");
    if (rc) return rc;
    hipLaunchKernelGGL(aa_solve_kernel, dim3(1), dim3(kAaThreads), 0, c->stream, a);
    rc = check_launch(c, "aa_solve_kernel");
    if (rc) return rc;
    hipLaunchKernelGGL(aa_combine_kernel, dim3(unsigned((c->V + 255) / 256)), dim3(256), 0, c->stream, a);
    return check_launch(c, "aa_combine_kernel");
}

void free_plan(rt3d_ctx *c);

void free_all(rt3d_ctx *c)
{
    free_plan(c);
    void *ptrs[] = {c->chi, c->eps, c->B, c->J, c->Jfs, c->r, c->dJa, c->dJb, c->L, c->Kc, c->invD, c->Ecoef, c->Iem,
                    c->Sbuf, c->bot_slope, c->xtab, c->cs, c->Ja, c->Fa, c->Iem_a, c->Kc32, c->d_scal,
                    c->ng_hist, c->ng_work, c->aa_x, c->aa_g, c->aa_work, c->adj_Ient, c->adj_Qx, c->adj_nu, c->adj_fs, c->adj_r,
                    c->adj_f, c->adj_pull, c->adj_g, c->adj_qs};
    for (void *p : ptrs)
        if (p) hipFree(p);
    for (auto &p : c->pending) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    for (auto e : c->event_pool) hipEventDestroy(e);
}

int n_sweep_shapes() { return int(sizeof(kSweepShapes) / sizeof(kSweepShapes[0])); }

// Ng's history and Anderson's window (whichever is set) with their device buffers
void free_acceleration(rt3d_ctx *c)
{
    size_t bytes = 0;
    if (c->ng_hist) bytes += size_t(c->ng_order + 2) * c->V * sizeof(double) + kNgWork * sizeof(double);
    if (c->aa_x) bytes += 2 * size_t(c->aa_depth + 1) * c->V * sizeof(double) + kAaWork * sizeof(double);
    c->device_bytes -= std::min(bytes, c->device_bytes);
    for (double **p : {&c->ng_hist, &c->ng_work, &c->aa_x, &c->aa_g, &c->aa_work}) {
        if (*p) hipFree(*p);
        *p = nullptr;
    }
    c->ng_order = c->ng_every = 0;
    c->aa_depth = 0;
}

// Sweep shape of new contexts: RT3D_SWEEP_SHAPE indexes the shape table (default 0, 512 x 2).
int env_sweep_shape()
{
    int shape = 0;
    if (const char *e = std::getenv("RT3D_SWEEP_SHAPE")) {
        const int v = std::atoi(e);
        if (v >= 0 && v < n_sweep_shapes()) shape = v;
    }
    return shape;
}

thread_local std::string t_create_error;
void set_thread_error(const std::string &msg) { t_create_error = msg; }
const char *thread_error() { return t_create_error.c_str(); }

int run_fs_plain(rt3d_ctx *c) { return run_fs(c, nullptr, false, c->precision == RT3D_FP32_SWEEP); }

std::string device_key()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string arch = p.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + "/" + std::to_string(p.multiProcessorCount) + "cu";
}

// the device tables built from the sweep plan (segment tables, pairs, work items, partial planes)
void free_plan(rt3d_ctx *c)
{
    void **ptrs[] = {reinterpret_cast<void **>(&c->P), reinterpret_cast<void **>(&c->seg_len64),
                     reinterpret_cast<void **>(&c->seg_len32), reinterpret_cast<void **>(&c->seg_off),
                     reinterpret_cast<void **>(&c->seg_n), reinterpret_cast<void **>(&c->seg_a),
                     reinterpret_cast<void **>(&c->seg_bb), reinterpret_cast<void **>(&c->seg_bm),
                     reinterpret_cast<void **>(&c->seg_ai), reinterpret_cast<void **>(&c->seg_bi),
                     reinterpret_cast<void **>(&c->row_min), reinterpret_cast<void **>(&c->dirs),
                     reinterpret_cast<void **>(&c->items), reinterpret_cast<void **>(&c->pairs),
                     reinterpret_cast<void **>(&c->pseg), reinterpret_cast<void **>(&c->player)};
    for (void **p : ptrs) {
        if (*p) hipFree(*p);
        *p = nullptr;
    }
    c->device_bytes -= c->plan_bytes;
    c->plan_bytes = 0;
    c->plan_ok = false;
}

bool build_plan(const rt3d_grid_desc &g, const rt3d::AngleSet &A, int shape, rt3d::SweepPlan &plan,
                std::string &msg)
{
    if (shape < 0 || shape >= n_sweep_shapes()) { msg = "sweep shape out of range"; return false; }
    const SweepShape sh = kSweepShapes[shape];
    // one plan for both precisions: a band's LDS is budgeted for the larger of the two; a grid whose
    // bands do not fit the usual budget (which keeps several workgroups per CU) takes the wide one
    if (rt3d::build_sweep_plan(g.nx, g.ny, g.nz, A, sh.threads * sh.lines, 16 * sh.threads, kWindowBytes,
                               plan, msg))
        return true;
    std::string msg_wide;
    if (rt3d::build_sweep_plan(g.nx, g.ny, g.nz, A, sh.threads * sh.lines, 16 * sh.threads, kWindowBytesWide,
                               plan, msg_wide))
        return true;
    msg = msg_wide;
    return false;
}

int install_plan(rt3d_ctx *c, int shape, rt3d::SweepPlan *built)
{
    if (shape < 0 || shape >= n_sweep_shapes()) return fail(c, RT3D_ERR_ARG, "sweep shape out of range");
    rt3d::SweepPlan plan;
    if (built) {
        plan = std::move(*built);
    } else {
        std::string msg;
        if (!build_plan(c->g, c->A, shape, plan, msg)) return fail(c, RT3D_ERR_ARG, msg);
    }
    int rc = sync(c);
    if (rc) return rc;
    free_plan(c);
    c->plan = std::move(plan);
    c->sweep_shape = shape;
    const auto &P = c->plan;
    const size_t before = c->device_bytes;
    auto chk = [&](int r) { if (!rc) rc = r; };
    {
        double *Pp = nullptr;
        chk(dev_alloc(c, &Pp, size_t(P.p_elems)));
        c->P = Pp;
    }
    chk(upload(c, &c->seg_len64, P.seg_len));
    chk(upload(c, &c->seg_len32, std::vector<float>(P.seg_len.begin(), P.seg_len.end())));
    chk(upload(c, &c->seg_off, P.seg_off)); chk(upload(c, &c->seg_n, P.seg_n));
    chk(upload(c, &c->seg_a, P.seg_a)); chk(upload(c, &c->seg_bb, P.seg_bb)); chk(upload(c, &c->seg_bm, P.seg_bm));
    chk(upload(c, &c->seg_ai, P.seg_ai)); chk(upload(c, &c->seg_bi, P.seg_bi));
    chk(upload(c, &c->row_min, P.row_min));
    chk(upload(c, &c->dirs, P.dirs)); chk(upload(c, &c->items, P.items)); chk(upload(c, &c->pairs, P.pairs));
    chk(upload(c, &c->pseg, P.pseg)); chk(upload(c, &c->player, P.player));
    c->plan_bytes = c->device_bytes - before;
    if (rc) {
        free_plan(c);
        return rc;
    }
    c->plan_ok = true;
    return RT3D_OK;
}

int create_ctx(rt3d_ctx **out, const rt3d_grid_desc *g, int precision, hipStream_t stream, int shape,
               std::string &msg)
{
    *out = nullptr;
    if (validate_desc(g, msg) != RT3D_OK) return RT3D_ERR_ARG;
    if (precision != RT3D_FP64 && precision != RT3D_FP32_SWEEP) { msg = "bad precision"; return RT3D_ERR_ARG; }
    if (shape < 0 || shape >= n_sweep_shapes()) { msg = "sweep shape out of range"; return RT3D_ERR_ARG; }
    rt3d_ctx *c = new (std::nothrow) rt3d_ctx();
    if (!c) { msg = "out of host memory"; return RT3D_ERR_OOM; }
    c->g = *g;
    c->precision = precision;
    c->stream = stream;
    c->real_size = (precision == RT3D_FP64) ? sizeof(double) : sizeof(float);
    c->V = long(g->nx) * g->ny * g->nz;
    if (!rt3d::make_angle_set(g->n_theta, g->n_phi, c->A)) { delete c; msg = "bad angle set"; return RT3D_ERR_ARG; }
    // the sweep plan first: a grid that does not fit the sweep kernel fails before any allocation
    rt3d::SweepPlan plan;
    if (!build_plan(*g, c->A, shape, plan, msg)) { delete c; return RT3D_ERR_ARG; }
    if (const char *e = std::getenv("RT3D_JACOBI_XCD")) c->jacobi_xcd = std::max(0, std::min(4, std::atoi(e)));
    if (const char *e = std::getenv("RT3D_JACOBI_ALTERNATE")) c->jacobi_alternate = std::atoi(e) != 0;
    if (const char *e = std::getenv("RT3D_JACOBI_COLUMN")) {
        const int h = std::atoi(e);
        c->jacobi_height = (h == 1 || h == 2 || h == 4) ? h : 0;
    }
    if (const char *e = std::getenv("RT3D_JACOBI_WALK")) c->jacobi_walk = std::max(-1, std::min(1, std::atoi(e)));
    if (const char *e = std::getenv("RT3D_ANCHOR_RATIO")) c->anchor_ratio = std::max(0.0, std::atof(e));
    // Lambda* walk may stop at the first non-neighbour only if no line wraps back within two layers
    {
        double tmax_x = 0.0, tmax_y = 0.0;
        for (int d = 0; d < c->A.n_dir; ++d) {
            tmax_x = std::max(tmax_x, std::fabs(c->A.ox[d] / c->A.mu[d]));
            tmax_y = std::max(tmax_y, std::fabs(c->A.oy[d] / c->A.mu[d]));
        }
        c->lstar_early_exit = (g->nx > 2.0 * tmax_x + 4.0 && g->ny > 2.0 * tmax_y + 4.0) ? 1 : 0;
    }
    const long V = c->V;
    int rc = RT3D_OK;
    auto chk = [&](int r) { if (!rc) rc = r; };
    chk(dev_alloc(c, &c->chi, V)); chk(dev_alloc(c, &c->eps, V)); chk(dev_alloc(c, &c->B, V));
    chk(dev_alloc(c, &c->J, V)); chk(dev_alloc(c, &c->Jfs, V)); chk(dev_alloc(c, &c->r, V));
    chk(dev_alloc(c, &c->dJa, V)); chk(dev_alloc(c, &c->dJb, V)); chk(dev_alloc(c, &c->Sbuf, V));
    chk(dev_alloc(c, &c->L, 27 * V));
    chk(dev_alloc(c, &c->invD, V)); chk(dev_alloc(c, &c->Ecoef, V));
    // Jacobi coefficients: float64 in the FP64 form, float32 in the FP32 form (rt3d_set_coef_storage)
    c->coef_fp32 = precision == RT3D_FP32_SWEEP ? 1 : 0;
    if (c->coef_fp32) chk(dev_alloc(c, &c->Kc32, 13 * V));
    else chk(dev_alloc(c, &c->Kc, 13 * V));
    chk(dev_alloc(c, &c->Iem, size_t(c->A.n_dir / 2) * g->nx * g->ny));
    {
        double2 *cs = nullptr;
        chk(dev_alloc(c, &cs, V));
        c->cs = cs;
    }
    if (precision == RT3D_FP32_SWEEP) {
        chk(dev_alloc(c, &c->Ja, V)); chk(dev_alloc(c, &c->Fa, V));
        chk(dev_alloc(c, &c->Iem_a, size_t(c->A.n_dir / 2) * g->nx * g->ny));
    }
    chk(dev_alloc(c, &c->d_scal, kScalarBytes / sizeof(unsigned long long)));
    if (!rc) {
        c->d_maxrel = c->d_scal;
        c->d_maxdist = c->d_scal + 1;
        c->d_flag = reinterpret_cast<int *>(c->d_scal + 2);
    }
    if (g->bottom_bc == 2) chk(dev_alloc(c, &c->bot_slope, size_t(g->nx) * g->ny));
    chk(dev_alloc(c, &c->xtab, kExpTab));
    if (!rc) {
        // 2^(j/kExpTab) rounded to float64 from the 64-bit-mantissa long double exp2
        double tab[kExpTab];
        for (int j = 0; j < kExpTab; ++j) tab[j] = double(std::exp2(static_cast<long double>(j) / kExpTab));
        if (hipMemcpy(c->xtab, tab, sizeof(tab), hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(c, RT3D_ERR_HIP, "upload of the exponential table");
    }
    if (!rc) rc = install_plan(c, shape, &plan);
    if (rc) {
        msg = c->err;
        free_all(c);
        delete c;
        return rc;
    }
    *out = c;
    return RT3D_OK;
}

}  // namespace rt3d_host

using namespace rt3d_host;

// ================================================================================================
// C ABI
// ================================================================================================

extern "C" {

const char *rt3d_status_str(int status)
{
    switch (status) {
    case RT3D_OK: return "ok";
    case RT3D_ERR_ARG: return "invalid argument";
    case RT3D_ERR_OOM: return "out of memory";
    case RT3D_ERR_HIP: return "HIP runtime error";
    case RT3D_ERR_NOT_CONVERGED: return "not converged";
    case RT3D_ERR_NONFINITE: return "non-finite value";
    case RT3D_ERR_STATE: return "invalid call order";
    default: return "unknown status";
    }
}

const char *rt3d_last_error(const rt3d_ctx *ctx) { return ctx ? ctx->err.c_str() : thread_error(); }

int rt3d_quadrature(int n_theta, int n_phi, double *mu, double *ox, double *oy, double *w)
{
    rt3d::AngleSet A;
    if (!mu || !ox || !oy || !w || !rt3d::make_angle_set(n_theta, n_phi, A)) return RT3D_ERR_ARG;
    std::memcpy(mu, A.mu.data(), sizeof(double) * A.n_dir);
    std::memcpy(ox, A.ox.data(), sizeof(double) * A.n_dir);
    std::memcpy(oy, A.oy.data(), sizeof(double) * A.n_dir);
    std::memcpy(w, A.w.data(), sizeof(double) * A.n_dir);
    return RT3D_OK;
}

int rt3d_segment_table(const rt3d_grid_desc *g, int d, int k, int *di, int *dj, double *len, int max_seg)
{
    std::string msg;
    if (validate_desc(g, msg) != RT3D_OK || !di || !dj || !len) return RT3D_ERR_ARG;
    rt3d::AngleSet A;
    if (!rt3d::make_angle_set(g->n_theta, g->n_phi, A)) return RT3D_ERR_ARG;
    if (d < 0 || d >= A.n_dir || k < 0 || k >= g->nz) return RT3D_ERR_ARG;
    rt3d::LayerSegments L;
    rt3d::direction_segments(g->nz, A, d, k, L);
    const int n = int(L.di.size());
    if (n > max_seg) return RT3D_ERR_ARG;
    for (int s = 0; s < n; ++s) {
        di[s] = L.di[s];
        dj[s] = L.dj[s];
        len[s] = L.len[s];
    }
    return n;
}

int rt3d_validate(const rt3d_grid_desc *g, const double *chi, const double *eps, const double *B)
{
    std::string msg;
    int rc = validate_desc(g, msg);
    if (!rc) {
        rt3d::AngleSet A;
        rt3d::SweepPlan plan;
        if (!rt3d::make_angle_set(g->n_theta, g->n_phi, A)) {
            msg = "bad angle set";
            rc = RT3D_ERR_ARG;
        } else if (!build_plan(*g, A, env_sweep_shape(), plan, msg)) {
            rc = RT3D_ERR_ARG;
        }
    }
    if (!rc) rc = validate_medium_host(long(g->nx) * g->ny * g->nz, chi, eps, B, msg);
    set_thread_error(rc ? msg : std::string());
    return rc;
}

int rt3d_create(rt3d_ctx **out, const rt3d_grid_desc *g, int precision, void *hip_stream)
{
    if (!out) {
        set_thread_error("out is NULL");
        return RT3D_ERR_ARG;
    }
    *out = nullptr;
    std::string msg;
    const int rc = create_ctx(out, g, precision, static_cast<hipStream_t>(hip_stream), env_sweep_shape(), msg);
    set_thread_error(rc ? msg : std::string());
    return rc;
}

void rt3d_destroy(rt3d_ctx *ctx)
{
    if (!ctx) return;
    hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
}

int rt3d_set_medium(rt3d_ctx *c, const double *chi, const double *eps, const double *B, int ptr_kind)
{
    if (!c) return RT3D_ERR_ARG;
    if (!chi || !eps || !B || (ptr_kind != RT3D_HOST && ptr_kind != RT3D_DEVICE))
        return fail(c, RT3D_ERR_ARG, "null medium pointer or bad ptr_kind");
    const long V = c->V;
    if (ptr_kind == RT3D_HOST) {
        std::string msg;
        if (validate_medium_host(V, chi, eps, B, msg)) return fail(c, RT3D_ERR_ARG, msg);
    }
    // staged copies: the context state changes only once the new medium is known to be valid
    HIP_TRY(c, hipMemcpyAsync(c->dJa, chi, V * 8, kind_in(ptr_kind), c->stream), "copy chi");
    HIP_TRY(c, hipMemcpyAsync(c->dJb, eps, V * 8, kind_in(ptr_kind), c->stream), "copy eps");
    HIP_TRY(c, hipMemcpyAsync(c->Sbuf, B, V * 8, kind_in(ptr_kind), c->stream), "copy B");
    if (ptr_kind == RT3D_DEVICE) {
        HIP_TRY(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream), "memset flag");
        hipLaunchKernelGGL(check_medium_kernel, dim3((V + 255) / 256), dim3(256), 0, c->stream, V,
                           c->dJa, c->dJb, c->Sbuf, c->d_flag);
        int rc = check_launch(c, "check_medium_kernel");
        if (rc) return rc;
        int flag = 0;
        HIP_TRY(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream), "flag");
        HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
        if (flag) return fail(c, RT3D_ERR_ARG, "device medium: chi must be finite > 0, eps in (0,1], B finite");
    }
    std::swap(c->chi, c->dJa);
    std::swap(c->eps, c->dJb);
    std::swap(c->B, c->Sbuf);
    if (c->g.bottom_bc == 2) {
        const int nxy = c->g.nx * c->g.ny;
        hipLaunchKernelGGL(diffusion_slope_kernel, dim3((nxy + 255) / 256), dim3(256), 0, c->stream, nxy, c->chi,
                           c->B, c->bot_slope);
        int rc = check_launch(c, "diffusion_slope_kernel");
        if (rc) return rc;
    }
    HIP_TRY(c, hipMemcpyAsync(c->J, c->B, V * 8, hipMemcpyDeviceToDevice, c->stream), "J = B");
    c->have_medium = true;
    c->have_lstar = false;
    c->have_fs = false;
    c->history.clear();
    c->anchor_valid = false;
    c->c_last = INFINITY;
    c->outer_iters = 0;
    c->inner_sweeps = 0;
    return sync(c);
}

int rt3d_set_J(rt3d_ctx *c, const double *J, int ptr_kind)
{
    if (!c) return RT3D_ERR_ARG;
    if (!c->have_medium) return fail(c, RT3D_ERR_STATE, "set the medium first");
    if (!J || (ptr_kind != RT3D_HOST && ptr_kind != RT3D_DEVICE)) return fail(c, RT3D_ERR_ARG, "bad J");
    const long V = c->V;
    if (ptr_kind == RT3D_HOST) {
        for (long v = 0; v < V; ++v)
            if (!std::isfinite(J[v])) return fail(c, RT3D_ERR_ARG, "J must be finite");
        HIP_TRY(c, hipMemcpyAsync(c->J, J, V * 8, hipMemcpyHostToDevice, c->stream), "copy J");
        c->anchor_valid = false;
        c->c_last = INFINITY;
        c->history.clear();
        return sync(c);
    }
    HIP_TRY(c, hipMemcpyAsync(c->dJa, J, V * 8, hipMemcpyDeviceToDevice, c->stream), "copy J");
    HIP_TRY(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream), "memset flag");
    hipLaunchKernelGGL(check_finite_kernel, dim3((V + 255) / 256), dim3(256), 0, c->stream, V, c->dJa, c->d_flag);
    int rc = check_launch(c, "check_finite_kernel");
    if (rc) return rc;
    int flag = 0;
    HIP_TRY(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream), "flag");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
    if (flag) return fail(c, RT3D_ERR_ARG, "J must be finite");
    std::swap(c->J, c->dJa);
    c->anchor_valid = false;
    c->c_last = INFINITY;
    c->history.clear();
    return sync(c);
}

int rt3d_get_J(rt3d_ctx *c, double *J_out, int ptr_kind)
{
    if (!c) return RT3D_ERR_ARG;
    if (!c->have_medium) return fail(c, RT3D_ERR_STATE, "no medium");
    if (!J_out || (ptr_kind != RT3D_HOST && ptr_kind != RT3D_DEVICE)) return fail(c, RT3D_ERR_ARG, "bad output");
    HIP_TRY(c, hipMemcpyAsync(J_out, c->J, c->V * 8, kind_out(ptr_kind), c->stream), "copy J out");
    return ptr_kind == RT3D_HOST ? sync(c) : RT3D_OK;
}

int rt3d_formal_solution(rt3d_ctx *c, const double *S_or_null, double *J_fs_out, int ptr_kind)
{
    if (!c) return RT3D_ERR_ARG;
    TraceRange tr("rt3d_formal_solution");
    if (!c->have_medium) return fail(c, RT3D_ERR_STATE, "set the medium first");
    if (!J_fs_out || (ptr_kind != RT3D_HOST && ptr_kind != RT3D_DEVICE)) return fail(c, RT3D_ERR_ARG, "bad output");
    const double *S_dev = nullptr;
    if (S_or_null) {
        if (ptr_kind == RT3D_HOST) {
            for (long v = 0; v < c->V; ++v)
                if (!std::isfinite(S_or_null[v])) return fail(c, RT3D_ERR_ARG, "S must be finite");
        }
        HIP_TRY(c, hipMemcpyAsync(c->Sbuf, S_or_null, c->V * 8, kind_in(ptr_kind), c->stream), "copy S");
        S_dev = c->Sbuf;
    }
    int rc = run_fs(c, S_dev, false, c->precision == RT3D_FP32_SWEEP);
    if (rc) return rc;
    HIP_TRY(c, hipMemcpyAsync(J_fs_out, c->Jfs, c->V * 8, kind_out(ptr_kind), c->stream), "copy J_fs");
    return sync(c);
}

int rt3d_build_lstar(rt3d_ctx *c)
{
    if (!c) return RT3D_ERR_ARG;
    TraceRange tr("rt3d_build_lstar");
    if (!c->have_medium) return fail(c, RT3D_ERR_STATE, "set the medium first");
    int rc = ensure_lstar(c);
    if (rc) return rc;
    return sync(c);
}

int rt3d_get_lstar(rt3d_ctx *c, double *out, int ptr_kind)
{
    if (!c) return RT3D_ERR_ARG;
    if (!c->have_lstar) return fail(c, RT3D_ERR_STATE, "Lambda* not built");
    if (!out || (ptr_kind != RT3D_HOST && ptr_kind != RT3D_DEVICE)) return fail(c, RT3D_ERR_ARG, "bad output");
    HIP_TRY(c, hipMemcpyAsync(out, c->L, 27 * c->V * 8, kind_out(ptr_kind), c->stream), "copy Lambda*");
    return sync(c);
}

int rt3d_os_step(rt3d_ctx *c, int inner_sweeps, double *max_rel_dJ_out)
{
    if (!c) return RT3D_ERR_ARG;
    TraceRange tr("rt3d_os_step");
    const auto t0 = std::chrono::steady_clock::now();
    if (!c->have_medium) return fail(c, RT3D_ERR_STATE, "set the medium first");
    if (inner_sweeps < 1) return fail(c, RT3D_ERR_ARG, "inner_sweeps must be >= 1");
    int rc = ensure_lstar(c);
    if (rc) return rc;
    bool anchored = true;
    if (c->precision == RT3D_FP32_SWEEP) {
        // float32 sweeps of the source change since the anchor; a float64 sweep re-anchors when the
        // step has become small next to the distance travelled since the anchor (the float32 error
        // of a difference step scales with that distance), or when asked to
        const bool refresh = !c->anchor_valid || c->force_refresh || c->c_last < c->anchor_ratio * c->da_last;
        rc = refresh ? refresh_anchor(c) : run_fs_difference(c);
        anchored = refresh;
    } else {
        rc = run_fs(c, nullptr, true, false);
    }
    if (rc) return rc;
    // the three convergence scalars share one allocation: one clear, one read-back per step
    HIP_TRY(c, hipMemsetAsync(c->d_scal, 0, kScalarBytes, c->stream), "memset");
    if (c->os_method == RT3D_OS_GAUSS_SEIDEL) {
        rc = gauss_seidel_sweeps(c, inner_sweeps);
        if (rc) return rc;
    } else {
        // sweep 1 from dJ = 0; sweeps 2..M from the previous one (carried as (1 - eps) dJ); the last
        // also updates J
        const double *in = nullptr;
        double *bufs[2] = {c->dJa, c->dJb};
        std::optional<TimedGroup> group;
        for (int m = 0; m < inner_sweeps; ++m) {
            const bool last = (m == inner_sweeps - 1);
            double *out = last ? nullptr : bufs[m & 1];
            // sampled timing: the intermediate sweeps 1 .. M-2 as one group (the first sweep, from
            // dJ = 0, and the last, which updates J, are cheaper and dearer); with M <= 2 the first
            if (m == 1 && inner_sweeps > 2) group.emplace(c, K_JACOBI, inner_sweeps - 2);
            // even sweeps top first: the first reads the right-hand side the reduction wrote last at the
            // top, and each later sweep starts where the one before ended
            rc = launch_jacobi(c, in, out, last, inner_sweeps <= 2 && m == 0, (m & 1) == 0);
            if (m == inner_sweeps - 2 && group) group->end();
            if (rc) return rc;
            in = out;
        }
    }
    unsigned long long scal[3] = {0, 0, 0};
    HIP_TRY(c, hipMemcpyAsync(scal, c->d_scal, kScalarBytes, hipMemcpyDeviceToHost, c->stream), "scalars");
    rc = sync(c);
    if (rc) return rc;
    const unsigned long long bits = scal[0], dbits = scal[1];
    int flag = 0;
    std::memcpy(&flag, &scal[2], sizeof(flag));
    c->outer_iters += 1;
    c->inner_sweeps += inner_sweeps;
    double cval, dval;
    std::memcpy(&cval, &bits, sizeof(cval));
    std::memcpy(&dval, &dbits, sizeof(dval));
    c->c_last = cval;
    c->da_last = dval;
    c->last_step_anchored = anchored;
    if (c->history.size() < kHistoryMax) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        c->history.push_back({cval, ms, anchored ? 1 : 0});
    }
    if (flag) {
        if (max_rel_dJ_out) *max_rel_dJ_out = NAN;
        return fail(c, RT3D_ERR_NONFINITE, "NaN or Inf in dJ or J");
    }
    if (max_rel_dJ_out) *max_rel_dJ_out = cval;
    return RT3D_OK;
}

int rt3d_solve_to_convergence(rt3d_ctx *c, double tol, int max_iter, int inner_sweeps, int *iters_out,
                              double *final_rel_dJ_out)
{
    if (!c) return RT3D_ERR_ARG;
    if (!(tol > 0.0) || max_iter < 1 || inner_sweeps < 1) return fail(c, RT3D_ERR_ARG, "bad tol/max_iter/inner_sweeps");
    TraceRange tr("rt3d_solve_to_convergence");
    c->history.clear();
    double cval = INFINITY;
    int n = 0, rc = RT3D_OK;
    const int R = c->ng_order + 2;
    const size_t vbytes = size_t(c->V) * sizeof(double);
    int nh = 0;   // iterates in the Ng history since the last extrapolation (the start included)
    if (c->ng_order > 0) {
        HIP_TRY(c, hipMemcpyAsync(c->ng_hist, c->J, vbytes, hipMemcpyDeviceToDevice, c->stream), "ng hist");
        nh = 1;
    }
    // Anderson window: ring entries of the newest pairs (input, output of the OS step), oldest first
    const int cap = c->aa_depth + 1;
    int aa_count = 0, aa_next = 0;
    int aa_slots[kAaMaxDepth + 1];
    while (n < max_iter) {
        if (c->aa_depth > 0) {
            if (aa_count == cap) {            // drop the oldest pair
                for (int q = 0; q + 1 < cap; ++q) aa_slots[q] = aa_slots[q + 1];
                --aa_count;
            }
            aa_slots[aa_count] = aa_next;
            aa_next = (aa_next + 1) % cap;
            HIP_TRY(c, hipMemcpyAsync(c->aa_x + long(aa_slots[aa_count]) * c->V, c->J, vbytes,
                                      hipMemcpyDeviceToDevice, c->stream), "anderson input");
        }
        rc = rt3d_os_step(c, inner_sweeps, &cval);
        ++n;
        if (rc != RT3D_OK) break;
        if (c->aa_depth > 0) {
            HIP_TRY(c, hipMemcpyAsync(c->aa_g + long(aa_slots[aa_count]) * c->V, c->J, vbytes,
                                      hipMemcpyDeviceToDevice, c->stream), "anderson output");
            ++aa_count;
            // FP32 form: an anchored step starts the window afresh from its own pair; the earlier
            // pairs' outputs carry float32 rounding relative to the previous anchor
            if (c->precision == RT3D_FP32_SWEEP && c->last_step_anchored && aa_count > 1) {
                aa_slots[0] = aa_slots[aa_count - 1];
                aa_count = 1;
            }
        }
        if (cval < tol) {
            // the FP32 form accepts convergence only from a step whose residual is float64
            if (c->precision != RT3D_FP32_SWEEP || c->last_step_anchored) break;
            c->force_refresh = true;
            continue;
        }
        if (c->aa_depth > 0 && aa_count >= 2) {
            rc = anderson_step(c, aa_count - 1, aa_slots);
            if (rc) break;
            if (!c->history.empty()) c->history.back().flags |= 4;
        }
        if (c->ng_order > 0) {
            HIP_TRY(c, hipMemcpyAsync(c->ng_hist + long(nh % R) * c->V, c->J, vbytes,
                                      hipMemcpyDeviceToDevice, c->stream), "ng hist");
            ++nh;
            if (nh - 1 >= c->ng_every) {
                rc = ng_step(c, (nh - 1) % R);
                if (rc) break;
                if (!c->history.empty()) c->history.back().flags |= 2;
                HIP_TRY(c, hipMemcpyAsync(c->ng_hist, c->J, vbytes, hipMemcpyDeviceToDevice, c->stream),
                        "ng hist");
                nh = 1;
            }
        }
    }
    if (iters_out) *iters_out = n;
    if (final_rel_dJ_out) *final_rel_dJ_out = cval;
    if (rc != RT3D_OK) return rc;
    const bool accepted = cval < tol && (c->precision != RT3D_FP32_SWEEP || c->last_step_anchored);
    return accepted ? RT3D_OK : fail(c, RT3D_ERR_NOT_CONVERGED, "max_iter reached");
}

int rt3d_set_acceleration(rt3d_ctx *c, int ng_order, int ng_every)
{
    if (!c) return RT3D_ERR_ARG;
    if (ng_order < 0 || ng_order > 3 || (ng_order > 0 && ng_every < ng_order + 1))
        return fail(c, RT3D_ERR_ARG, "ng_order must be 0..3 and ng_every >= ng_order + 1");
    int rc = sync(c);
    if (rc) return rc;
    free_acceleration(c);
    if (ng_order == 0) return RT3D_OK;
    rc = dev_alloc(c, &c->ng_hist, size_t(ng_order + 2) * c->V);
    if (!rc) rc = dev_alloc(c, &c->ng_work, size_t(kNgWork));
    if (rc) return rc;
    c->ng_order = ng_order;
    c->ng_every = ng_every;
    return RT3D_OK;
}

int rt3d_set_anderson(rt3d_ctx *c, int depth)
{
    if (!c) return RT3D_ERR_ARG;
    if (depth < 0 || depth > kAaMaxDepth) return fail(c, RT3D_ERR_ARG, "Anderson depth must be 0..8");
    int rc = sync(c);
    if (rc) return rc;
    free_acceleration(c);
    if (depth == 0) return RT3D_OK;
    rc = dev_alloc(c, &c->aa_x, size_t(depth + 1) * c->V);
    if (!rc) rc = dev_alloc(c, &c->aa_g, size_t(depth + 1) * c->V);
    if (!rc) rc = dev_alloc(c, &c->aa_work, size_t(kAaWork));
    if (rc) {
        free_acceleration(c);
        return rc;
    }
    c->aa_depth = depth;
    return RT3D_OK;
}

int rt3d_set_os_method(rt3d_ctx *c, int method)
{
    if (!c) return RT3D_ERR_ARG;
    if (method != RT3D_OS_JACOBI && method != RT3D_OS_GAUSS_SEIDEL)
        return fail(c, RT3D_ERR_ARG, "method must be RT3D_OS_JACOBI or RT3D_OS_GAUSS_SEIDEL");
    c->os_method = method;
    return RT3D_OK;
}

int rt3d_set_coef_storage(rt3d_ctx *c, int storage)
{
    if (!c) return RT3D_ERR_ARG;
    if (storage != RT3D_COEF_FP64 && storage != RT3D_COEF_FP32)
        return fail(c, RT3D_ERR_ARG, "storage must be RT3D_COEF_FP64 or RT3D_COEF_FP32");
    const int want = storage == RT3D_COEF_FP32 ? 1 : 0;
    if (want == c->coef_fp32) return RT3D_OK;
    int rc = sync(c);
    if (rc) return rc;
    // allocate the new store before freeing the old one, so that a failure leaves the context as it was
    if (want) {
        float *k = nullptr;
        rc = dev_alloc(c, &k, 13 * size_t(c->V));
        if (rc) return rc;
        hipFree(c->Kc);
        c->Kc = nullptr;
        c->device_bytes -= 13 * size_t(c->V) * sizeof(double);
        c->Kc32 = k;
    } else {
        double *k = nullptr;
        rc = dev_alloc(c, &k, 13 * size_t(c->V));
        if (rc) return rc;
        hipFree(c->Kc32);
        c->Kc32 = nullptr;
        c->device_bytes -= 13 * size_t(c->V) * sizeof(float);
        c->Kc = k;
    }
    c->coef_fp32 = want;
    // the coefficients follow from Lambda* (kept in float64); re-derive them in the new precision
    if (c->have_lstar) {
        rc = finish_lstar(c);
        if (rc) return rc;
        return sync(c);
    }
    return RT3D_OK;
}

int rt3d_get_emergent_top(rt3d_ctx *c, double *out, int ptr_kind)
{
    if (!c) return RT3D_ERR_ARG;
    if (!c->have_fs) return fail(c, RT3D_ERR_STATE, "no formal solution yet");
    if (!out || (ptr_kind != RT3D_HOST && ptr_kind != RT3D_DEVICE)) return fail(c, RT3D_ERR_ARG, "bad output");
    const size_t n = size_t(c->A.n_dir / 2) * c->g.nx * c->g.ny;
    HIP_TRY(c, hipMemcpyAsync(out, c->Iem, n * 8, kind_out(ptr_kind), c->stream), "copy emergent");
    return sync(c);
}

int rt3d_set_timing(rt3d_ctx *c, int enable)
{
    if (!c || enable < 0 || enable > 2) return RT3D_ERR_ARG;
    int rc = sync(c);
    if (rc) return rc;
    c->timing = enable;
    for (int k = 0; k < K_COUNT; ++k) {
        c->kernel_ms[k] = 0.0;
        c->kernel_launches[k] = 0;
        c->kernel_timed[k] = 0;
    }
    return RT3D_OK;
}

int rt3d_get_history(rt3d_ctx *c, double *c_out, double *ms_out, int *flags_out, int max_n)
{
    if (!c || max_n < 0) return RT3D_ERR_ARG;
    const int n = int(c->history.size());
    for (int q = 0; q < n && q < max_n; ++q) {
        if (c_out) c_out[q] = c->history[q].c;
        if (ms_out) ms_out[q] = c->history[q].ms;
        if (flags_out) flags_out[q] = c->history[q].flags;
    }
    return n;
}

int rt3d_get_stats(rt3d_ctx *c, char *buf, int buflen)
{
    if (!c || !buf || buflen < 2) return RT3D_ERR_ARG;
    int rc = sync(c);
    if (rc) return rc;
    std::string s = "{";
    char tmp[1024];
    const int jcol = c->jacobi_height > 0 ? c->jacobi_height : jacobi_column_height(c->g.nx, c->g.ny, c->g.nz);
    std::snprintf(tmp, sizeof tmp,
                  "\"nx\":%d,\"ny\":%d,\"nz\":%d,\"n_dir\":%d,\"precision\":\"%s\",\"outer_iters\":%ld,"
                  "\"inner_sweeps\":%ld,\"fp64_sweeps\":%ld,\"fp32_sweeps\":%ld,\"device_bytes\":%zu,\"partial_plane_bytes\":%lld,"
                  "\"sweep_workgroups\":%zu,\"sweep_shape\":%d,\"sweep_threads\":%d,\"sweep_lines\":%d,\"mean_segments\":%.6f,"
                  "\"max_window_rows\":%d,\"sweep_lds_bytes\":%zu,"
                  "\"os_method\":\"%s\",\"coef_storage\":\"%s\",\"jacobi_layout\":%d,\"jacobi_column\":%d,\"jacobi_alt_walk\":%d,"
                  "\"timing\":%d,\"kernels\":{",
                  c->g.nx, c->g.ny, c->g.nz, c->A.n_dir, c->precision == RT3D_FP64 ? "fp64" : "fp32_sweep",
                  c->outer_iters, c->inner_sweeps, c->fp64_sweeps, c->fp32_sweeps, c->device_bytes,
                  (long long)(c->plan.p_elems * (long long)sizeof(double)), c->plan.items.size(),
                  c->sweep_shape, kSweepShapes[c->sweep_shape].threads, kSweepShapes[c->sweep_shape].lines, c->plan.mean_segments,
                  c->plan.max_win_rows, sweep_smem_bytes(c->plan, c->precision != RT3D_FP64),
                  c->os_method == RT3D_OS_GAUSS_SEIDEL ? "gauss_seidel" : "jacobi", c->coef_fp32 ? "fp32" : "fp64",
                  c->jacobi_xcd, jcol,
                  (c->jacobi_xcd == 4 && jacobi_alt_walk(c->jacobi_walk, c->coef_fp32 != 0, jcol)) ? 1 : 0, c->timing);
    s += tmp;
    for (int k = 0; k < K_COUNT; ++k) {
        std::snprintf(tmp, sizeof tmp, "%s\"%s\":{\"launches\":%ld,\"timed\":%ld,\"total_ms\":%.6f}", k ? "," : "",
                      kKernelNames[k], c->kernel_launches[k], c->kernel_timed[k], c->kernel_ms[k]);
        s += tmp;
    }
    s += "}}";
    if (int(s.size()) + 1 > buflen) return fail(c, RT3D_ERR_ARG, "stats buffer too small");
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return RT3D_OK;
}

int rt3d_sweep_shapes(int *threads, int *lines, int max_n)
{
    const int n = n_sweep_shapes();
    for (int i = 0; i < n && i < max_n; ++i) {
        if (threads) threads[i] = kSweepShapes[i].threads;
        if (lines) lines[i] = kSweepShapes[i].lines;
    }
    return n;
}

int rt3d_set_sweep_shape(rt3d_ctx *c, int shape)
{
    if (!c) return RT3D_ERR_ARG;
    return install_plan(c, shape);
}

int rt3d_autotune(rt3d_ctx *c, const char *cache_path, int repeats, int *shape_out, double *ms_out)
{
    if (!c) return RT3D_ERR_ARG;
    TraceRange tr("rt3d_autotune");
    if (!c->have_medium) return fail(c, RT3D_ERR_STATE, "set the medium first");
    if (repeats < 1) return fail(c, RT3D_ERR_ARG, "repeats must be >= 1");
    const int ns = n_sweep_shapes();
    char grid[96];
    std::snprintf(grid, sizeof grid, "%dx%dx%d|%dx%d", c->g.nx, c->g.ny, c->g.nz, c->g.n_theta, c->g.n_phi);
    const std::string key = device_key() + "|" + (c->precision == RT3D_FP64 ? "fp64" : "fp32_sweep") + "|" + grid;
    int cached = -1;
    if (cache_path && *cache_path && rt3d_tune::lookup(cache_path, key, cached) && cached >= 0 && cached < ns) {
        if (cached != c->sweep_shape) {
            const int rc = install_plan(c, cached);
            if (rc) return rc;
        }
        if (shape_out) *shape_out = cached;
        if (ms_out) for (int i = 0; i < ns; ++i) ms_out[i] = -1.0;
        return RT3D_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(c, hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(c, RT3D_ERR_HIP, "hipEventCreate");
    }
    std::vector<double> ms(ns, INFINITY);
    int rc = RT3D_OK;
    for (int s = 0; s < ns && !rc; ++s) {
        const int r = install_plan(c, s);
        if (r == RT3D_ERR_ARG) continue;      // the shape does not fit this grid
        if (r) { rc = r; break; }
        rc = run_fs_plain(c);                 // warm-up
        if (!rc) rc = sync(c);
        if (!rc && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(c, RT3D_ERR_HIP, "hipEventRecord");
        for (int k = 0; k < repeats && !rc; ++k) rc = run_fs_plain(c);
        if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = fail(c, RT3D_ERR_HIP, "hipEventRecord");
        if (!rc) rc = sync(c);
        float t = 0.f;
        if (!rc && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms[s] = double(t) / repeats;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    int best = -1;
    for (int s = 0; s < ns; ++s)
        if (std::isfinite(ms[s]) && (best < 0 || ms[s] < ms[best])) best = s;
    if (best < 0) return fail(c, RT3D_ERR_ARG, "no sweep shape fits this grid");
    rc = install_plan(c, best);
    if (rc) return rc;
    if (shape_out) *shape_out = best;
    if (ms_out) for (int i = 0; i < ns; ++i) ms_out[i] = std::isfinite(ms[i]) ? ms[i] : -1.0;
    if (cache_path && *cache_path) {
        std::string entry = "{\"shape\": " + std::to_string(best) + ", \"threads\": " +
                            std::to_string(kSweepShapes[best].threads) + ", \"lines\": " +
                            std::to_string(kSweepShapes[best].lines) + ", \"ms\": [";
        for (int i = 0; i < ns; ++i) {
            char t[32];
            if (std::isfinite(ms[i])) std::snprintf(t, sizeof t, "%.4f", ms[i]);
            else std::snprintf(t, sizeof t, "null");
            entry += (i ? ", " : "") + std::string(t);
        }
        entry += "]}";
        std::string err;
        if (!rt3d_tune::store(cache_path, key, entry, err)) return fail(c, RT3D_ERR_ARG, err);
    }
    return RT3D_OK;
}

}  // extern "C"
