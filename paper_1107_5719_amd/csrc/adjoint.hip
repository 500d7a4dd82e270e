// adjoint.hip -- gradient of a loss on the emergent top intensities with respect to every voxel's
// opacity chi and thermalisation parameter eps, through the converged operator-splitting fixed point
// J = Lambda(chi) (eps B + (1 - eps) J) + J_bc(chi) of the scattering solve (an extension of the
// paper's method: it computes the forward solution only).
//
// With g = dL/dI_em given, S = eps B + (1 - eps) J, D = diag(1 - eps) and the Lagrangian
// L + lambda^T (Phi(chi, S) - J) (Phi = the formal solution's mean intensity):
//   a      = dL/dS at fixed chi: the transport adjoint of the emergent light along the upward lines;
//   mu     = a + Lambda^T D mu (the total sensitivity to S), lambda = D mu;
//   dL/deps_v = mu_v (B_v - J_v);
//   dL/dchi_v = d/dchi_v [ g . I_em(chi, S) + lambda . Phi(chi, S) ] at fixed S.
// Reciprocity (chi_v Lambda_vu = chi_u Lambda_uv: the lines of Omega and -Omega coincide and carry
// equal weights) turns the transposed system into the forward one: nu = mu / chi solves
// (I - Lambda D) nu = a / chi, which the library's own operator-splitting iteration solves with the
// source (1 - eps) nu, no boundary light and a / chi added to the formal solution.
//
// The derivatives along the lines are reverse-mode differentiation of the exact segment integration
//   e = exp(-dtau), dtau = chi_v l,  I_out = S + (I_in - S) e,  D = S dtau + (I_in - S)(1 - e):
// with the adjoint variable q of I (q = g at the top end of an upward line, 0 at the end of a
// downward one) and the weight c = lambda_v W |mu| / chi_v = (1 - eps_v) nu_v W |mu| of D in
// lambda . Phi, going backwards  q_in = q_out e + c (1 - e),  and each segment contributes
//   l (c S + (c - q_out)(I_in - S) e)  to dL/dchi_v,  plus the explicit -lambda_v Phi_v / chi_v.
// Kernels: a forward pass stores I entering every layer of every line, a backward pass stores q
// leaving every layer; a per-voxel pull kernel recomputes I_in and q_out of the few segments of a
// layer from those and sums the voxel's terms in a fixed order (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rt3d.h"
#include "context.h"
#include "kernels.h"

using namespace rt3d_host;

namespace {

constexpr int kLineThreads = 256;

struct AdjLineArgs {
    int nx, ny, nz, n_dir;
    const DirInfo *dirs;
    const int *seg_off, *seg_n, *seg_ai, *seg_bi;
    const double *seg_len;
    const double *chi, *S;        // opacity and the converged source
    const double *Ibot;           // light entering the bottom plane ([ny][nx]) or null
    const double *Islope;         // LTE-diffusion gradient ([ny][nx]): upward lines add mu * Islope
    double I_top;
    double *Ient;                 // [n_dir][nz][ny*nx]: I entering layer k along line p
    const double *g;              // [n_up][ny*nx]: dL/dI_em at the top end of the upward lines
    const double *nu, *eps;       // weights c = (1 - eps) nu W|mu| of the deposits, or nu == null
    double *Qx;                   // [n_dir][nz][ny*nx]: adjoint q leaving layer k along line p
    double *Qstart;               // [n_up][ny*nx]: q at the start of the upward lines (or null)
};

__device__ inline int wrap_any(int a, int n)
{
    const int r = a % n;
    return r < 0 ? r + n : r;
}

// voxel of segment s (table index t) of the line whose top column is (i0, j0), in layer k
__device__ inline long seg_voxel(const AdjLineArgs &a, int i0, int j0, int k, int t)
{
    const int col = wrap_any(i0 + a.seg_ai[t], a.nx);
    const int row = wrap_any(j0 + a.seg_bi[t], a.ny);
    return (long(k) * a.ny + row) * a.nx + col;
}

// Forward pass: the intensity entering every layer of every line (the formal solution's recurrence).
__global__ __launch_bounds__(kLineThreads) void adj_record_kernel(AdjLineArgs a)
{
    const int p = blockIdx.x * kLineThreads + threadIdx.x;
    const int d = blockIdx.y;
    const int nxy = a.nx * a.ny;
    if (p >= nxy) return;
    const int i0 = p % a.nx, j0 = p / a.nx;
    const bool down = a.dirs[d].down != 0;
    double I = a.I_top;
    if (!down) {
        const long v0 = seg_voxel(a, i0, j0, 0, a.seg_off[d * a.nz]);
        I = a.Ibot ? a.Ibot[v0] + (a.Islope ? a.dirs[d].mu * a.Islope[v0] : 0.0) : 0.0;
    }
    for (int step = 0; step < a.nz; ++step) {
        const int k = down ? a.nz - 1 - step : step;
        a.Ient[(long(d) * a.nz + k) * nxy + p] = I;
        const int off = a.seg_off[d * a.nz + k], n = a.seg_n[d * a.nz + k];
        for (int s = 0; s < n; ++s) {
            const long v = seg_voxel(a, i0, j0, k, off + s);
            const double em1 = expm1(-a.chi[v] * a.seg_len[off + s]);
            I = I + (I - a.S[v]) * em1;
        }
    }
}

__device__ inline double deposit_weight(const AdjLineArgs &a, long v, double wmu)
{
    return a.nu ? (1.0 - a.eps[v]) * a.nu[v] * wmu : 0.0;
}

// Backward pass: q from the end of every line back to its start, stored where it leaves each layer.
__global__ __launch_bounds__(kLineThreads) void adj_back_kernel(AdjLineArgs a)
{
    const int p = blockIdx.x * kLineThreads + threadIdx.x;
    const int d = blockIdx.y;
    const int nxy = a.nx * a.ny;
    if (p >= nxy) return;
    const int i0 = p % a.nx, j0 = p / a.nx;
    const bool down = a.dirs[d].down != 0;
    const double wmu = a.dirs[d].wmu;
    double q = down ? 0.0 : a.g[long(d - a.n_dir / 2) * nxy + p];
    for (int step = 0; step < a.nz; ++step) {
        const int k = down ? step : a.nz - 1 - step;      // reverse travel order
        a.Qx[(long(d) * a.nz + k) * nxy + p] = q;
        const int off = a.seg_off[d * a.nz + k], n = a.seg_n[d * a.nz + k];
        for (int s = n - 1; s >= 0; --s) {
            const long v = seg_voxel(a, i0, j0, k, off + s);
            const double em1 = expm1(-a.chi[v] * a.seg_len[off + s]);
            const double c = deposit_weight(a, v, wmu);
            q = q - (c - q) * em1;                           // q e + c (1 - e)
        }
    }
    if (!down && a.Qstart) a.Qstart[long(d - a.n_dir / 2) * nxy + p] = q;   // sensitivity to the entry light
}

// LTE-diffusion inner condition: the entry light B_0 + mu (B_0 - B_1) / dtau of an upward line
// depends on chi_0 and chi_1 of its entry column through dtau = (chi_0 + chi_1) / 2.  Per bottom
// column, the lines of every upward direction that enter there add q_start mu d(slope)/d(chi) to
// both voxels' chi gradient.
__global__ void adj_bc_kernel(AdjLineArgs a, const double *B, double *pull)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int nxy = a.nx * a.ny;
    if (c >= nxy) return;
    const int i = c % a.nx, j = c / a.nx;
    double acc = 0.0;
    for (int d = a.n_dir / 2; d < a.n_dir; ++d) {
        const int t = a.seg_off[d * a.nz];                  // first segment of layer 0
        const int i0 = wrap_any(i - a.seg_ai[t], a.nx);
        const int j0 = wrap_any(j - a.seg_bi[t], a.ny);
        acc += a.Qstart[long(d - a.n_dir / 2) * nxy + long(j0) * a.nx + i0] * a.dirs[d].mu;
    }
    const double dtau = 0.5 * (a.chi[c] + a.chi[nxy + c]);
    const double dslope = -0.5 * (B[c] - B[nxy + c]) / (dtau * dtau);   // d(slope)/d(chi_0) = d/d(chi_1)
    pull[c] += acc * dslope;
    pull[nxy + c] += acc * dslope;
}

// Per voxel, over all directions and the segments of its layer that lie in it:
//   mode 0:  out = a_v / chi_v,  a_v = sum q_out (1 - e)                  (nu == null)
//   mode 1:  out = sum l (c S + (c - q_out)(I_in - S) e)
__global__ __launch_bounds__(kPlaneThreads) void adj_pull_kernel(AdjLineArgs a, int mode, double *out)
{
    const int p = blockIdx.x * kPlaneThreads + threadIdx.x;
    const int k = blockIdx.y;
    const int nxy = a.nx * a.ny;
    if (p >= nxy) return;
    const int i = p % a.nx, j = p / a.nx;
    const long v = long(k) * nxy + p;
    const double chiv = a.chi[v], Sv = a.S[v];
    double acc = 0.0;
    for (int d = 0; d < a.n_dir; ++d) {
        const double wmu = a.dirs[d].wmu;
        const int off = a.seg_off[d * a.nz + k], n = a.seg_n[d * a.nz + k];
        for (int s = 0; s < n; ++s) {
            // the line whose segment s lies in v
            const int i0 = wrap_any(i - a.seg_ai[off + s], a.nx);
            const int j0 = wrap_any(j - a.seg_bi[off + s], a.ny);
            const long line = long(j0) * a.nx + i0;
            const long lk = (long(d) * a.nz + k) * nxy + line;
            double q = a.Qx[lk];
            for (int s2 = n - 1; s2 > s; --s2) {
                const long v2 = seg_voxel(a, i0, j0, k, off + s2);
                const double em1 = expm1(-a.chi[v2] * a.seg_len[off + s2]);
                q = q - (deposit_weight(a, v2, wmu) - q) * em1;
            }
            const double len = a.seg_len[off + s];
            const double em1 = expm1(-chiv * len);
            if (mode == 0) {
                acc -= q * em1;
            } else {
                double I = a.Ient[lk];
                for (int s2 = 0; s2 < s; ++s2) {
                    const long v2 = seg_voxel(a, i0, j0, k, off + s2);
                    const double em1b = expm1(-a.chi[v2] * a.seg_len[off + s2]);
                    I = I + (I - a.S[v2]) * em1b;
                }
                const double c = deposit_weight(a, v, wmu);
                acc += len * (c * Sv + (c - q) * (I - Sv) * exp(-chiv * len));
            }
        }
    }
    out[v] = (mode == 0) ? acc / chiv : acc;
}

struct AdjFinalArgs {
    long V;
    const double *chi, *eps, *B, *J, *Jfs, *nu, *pull;
    double *dchi, *deps;
};

__global__ void adj_final_kernel(AdjFinalArgs a)
{
    const long v = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= a.V) return;
    const double nu = a.nu[v];
    a.dchi[v] = a.pull[v] - (1.0 - a.eps[v]) * nu * a.Jfs[v];
    a.deps[v] = a.chi[v] * nu * (a.B[v] - a.J[v]);
}

// the converged source S = eps B + (1 - eps) J
__global__ void adj_source_kernel(long V, const double *eps, const double *B, const double *J, double *S)
{
    const long v = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < V) S[v] = eps[v] * B[v] + (1.0 - eps[v]) * J[v];
}

__global__ void adj_zero_kernel(long V, double *x)
{
    const long v = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < V) x[v] = 0.0;
}

AdjLineArgs line_args(rt3d_ctx *c)
{
    AdjLineArgs a{};
    a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz; a.n_dir = c->A.n_dir;
    a.dirs = c->dirs; a.seg_off = c->seg_off; a.seg_n = c->seg_n; a.seg_ai = c->seg_ai; a.seg_bi = c->seg_bi;
    a.seg_len = c->seg_len64;
    a.chi = c->chi; a.S = c->Sbuf;
    a.Ibot = c->g.bottom_bc != 1 ? c->B : nullptr;
    a.Islope = c->g.bottom_bc == 2 ? c->bot_slope : nullptr;
    a.Qstart = c->g.bottom_bc == 2 ? c->adj_qs : nullptr;
    a.I_top = c->g.I_top;
    a.Ient = c->adj_Ient; a.Qx = c->adj_Qx;
    a.g = c->adj_g;
    a.eps = c->eps;
    return a;
}

int ensure_adjoint_buffers(rt3d_ctx *c)
{
    if (c->adj_Ient) return RT3D_OK;
    const size_t lines = size_t(c->A.n_dir) * c->V;
    int rc = RT3D_OK;
    auto chk = [&](int r) { if (!rc) rc = r; };
    chk(dev_alloc(c, &c->adj_Ient, lines)); chk(dev_alloc(c, &c->adj_Qx, lines));
    chk(dev_alloc(c, &c->adj_nu, c->V)); chk(dev_alloc(c, &c->adj_fs, c->V)); chk(dev_alloc(c, &c->adj_r, c->V));
    chk(dev_alloc(c, &c->adj_f, c->V)); chk(dev_alloc(c, &c->adj_pull, c->V));
    chk(dev_alloc(c, &c->adj_g, size_t(c->A.n_dir / 2) * c->g.nx * c->g.ny));
    if (c->g.bottom_bc == 2) chk(dev_alloc(c, &c->adj_qs, size_t(c->A.n_dir / 2) * c->g.nx * c->g.ny));
    if (rc) {
        double **ptrs[] = {&c->adj_Ient, &c->adj_Qx, &c->adj_nu, &c->adj_fs, &c->adj_r, &c->adj_f, &c->adj_pull,
                           &c->adj_g, &c->adj_qs};
        for (double **p : ptrs) {
            if (*p) hipFree(*p);
            *p = nullptr;
        }
    }
    return rc;
}

dim3 planes(const rt3d_ctx *c) { return dim3((c->g.nx * c->g.ny + kPlaneThreads - 1) / kPlaneThreads, c->g.nz); }

// One step of the operator-splitting iteration for (I - Lambda D) nu = f: formal solution of
// (1 - eps) nu with no boundary light, plus f; residual; M Jacobi sweeps; nu += dnu.
// *dmax and *numax receive max |dnu| and max |nu|.
int adjoint_os_step(rt3d_ctx *c, int M, double *dmax, double *numax, int *bad)
{
    SourceArgs sa{};
    sa.nx = c->g.nx; sa.ny = c->g.ny; sa.nz = c->g.nz;
    sa.scatter_only = 1;
    sa.chi = c->chi; sa.eps = c->eps; sa.B = c->B; sa.J = c->adj_nu;
    sa.cs = c->cs;
    hipLaunchKernelGGL(source_kernel<double>, planes(c), dim3(kPlaneThreads), 0, c->stream, sa);
    int rc = check_launch(c, "source_kernel (adjoint)");
    if (rc) return rc;
    SweepArgs w{};
    w.nx = c->g.nx; w.ny = c->g.ny; w.nz = c->g.nz;
    w.n_down = c->A.n_dir / 2;
    w.pseg = c->pseg; w.player = c->player; w.pairs = c->pairs; w.items = c->items;
    w.cs = c->cs;
    w.Ibot = nullptr;
    w.I_top = 0.0;
    w.P = c->P;
    w.Iem = nullptr;
    w.Iem_base = nullptr;
    w.xtab = c->xtab;
    const size_t smem = sweep_smem_bytes(c->plan, false);
    const dim3 grid(c->plan.items.size());
    with_sweep_shape(c->sweep_shape, [&](auto tag) {
        using Tag = decltype(tag);
        hipLaunchKernelGGL((sweep_kernel<double, Tag::threads, Tag::lines>), grid, dim3(Tag::threads), smem,
                           c->stream, w);
    });
    if ((rc = check_launch(c, "sweep_kernel (adjoint)"))) return rc;
    ReduceArgs ra{};
    ra.nx = c->g.nx; ra.ny = c->g.ny; ra.nz = c->g.nz; ra.n_pair = c->plan.n_pair;
    ra.pairs = c->pairs; ra.row_min = c->row_min; ra.P = c->P; ra.chi = c->chi;
    ra.J = c->adj_nu; ra.base = c->adj_f; ra.Jfs = c->adj_fs; ra.rb = c->adj_r;
    hipLaunchKernelGGL(reduce_kernel_pair<double>,
                       dim3(((c->g.nx + 1) / 2 * c->g.ny + kPlaneThreads - 1) / kPlaneThreads, c->g.nz),
                       dim3(kPlaneThreads), 0, c->stream, ra);
    if ((rc = check_launch(c, "reduce_kernel_pair (adjoint)"))) return rc;
    HIP_TRY(c, hipMemsetAsync(c->d_scal, 0, kScalarBytes, c->stream), "memset");
    const double *in = nullptr;
    double *bufs[2] = {c->dJa, c->dJb};
    for (int m = 0; m < M; ++m) {
        const bool last = m == M - 1;
        JacobiArgs ja{};
        ja.nx = c->g.nx; ja.ny = c->g.ny; ja.nz = c->g.nz;
        ja.b = c->adj_r;
        ja.Kc = c->coef_fp32 ? static_cast<const void *>(c->Kc32) : static_cast<const void *>(c->Kc);
        ja.invD = c->invD; ja.E = c->Ecoef;
        ja.w_in = in;
        ja.w_out = last ? nullptr : bufs[m & 1];
        ja.J = last ? c->adj_nu : nullptr;
        ja.maxrel = c->d_maxrel; ja.maxdist = c->d_maxdist; ja.nonfinite = c->d_flag;
        ja.abs_measure = 1;
        launch_jacobi_sweep(ja, c->jacobi_xcd, c->coef_fp32 != 0, c->stream, c->jacobi_alternate && (m & 1) == 0,
                            c->jacobi_height, c->jacobi_walk);
        if ((rc = check_launch(c, "jacobi_kernel (adjoint)"))) return rc;
        in = ja.w_out;
    }
    unsigned long long scal[3] = {0, 0, 0};
    HIP_TRY(c, hipMemcpyAsync(scal, c->d_scal, kScalarBytes, hipMemcpyDeviceToHost, c->stream), "scalars");
    rc = sync(c);
    if (rc) return rc;
    const unsigned long long b1 = scal[0], b2 = scal[1];
    std::memcpy(bad, &scal[2], sizeof(int));
    std::memcpy(dmax, &b1, sizeof(double));
    std::memcpy(numax, &b2, sizeof(double));
    return RT3D_OK;
}

}  // namespace


extern "C" {

int rt3d_adjoint_emergent(rt3d_ctx *c, const double *g_em, double tol, int max_iter, int inner_sweeps,
                          double *dL_dchi, double *dL_deps, int ptr_kind, int *iters_out, double *final_rel_out)
{
    if (!c) return RT3D_ERR_ARG;
    TraceRange tr("rt3d_adjoint_emergent");
    if (!c->have_medium) return fail(c, RT3D_ERR_STATE, "set the medium first");
    if (!g_em || !dL_dchi || !dL_deps || (ptr_kind != RT3D_HOST && ptr_kind != RT3D_DEVICE))
        return fail(c, RT3D_ERR_ARG, "null array or bad ptr_kind");
    if (!(tol > 0.0) || max_iter < 1 || inner_sweeps < 1)
        return fail(c, RT3D_ERR_ARG, "bad tol/max_iter/inner_sweeps");
    const long V = c->V;
    const long nxy = long(c->g.nx) * c->g.ny;
    const long n_em = long(c->A.n_dir / 2) * nxy;
    if (ptr_kind == RT3D_HOST)
        for (long q = 0; q < n_em; ++q)
            if (!std::isfinite(g_em[q])) return fail(c, RT3D_ERR_ARG, "g_em must be finite");
    int rc = ensure_lstar(c);
    if (!rc) rc = ensure_adjoint_buffers(c);
    if (rc) return rc;
    // the converged source S = eps B + (1 - eps) J and its float64 formal solution (J_fs, I_em)
    rc = run_fs(c, nullptr, false, false);
    if (rc) return rc;
    hipLaunchKernelGGL(adj_source_kernel, dim3((V + 255) / 256), dim3(256), 0, c->stream, V, c->eps, c->B, c->J,
                       c->Sbuf);
    if ((rc = check_launch(c, "adj_source_kernel"))) return rc;
    HIP_TRY(c, hipMemcpyAsync(c->adj_g, g_em, n_em * sizeof(double), kind_in(ptr_kind), c->stream), "copy g");
    AdjLineArgs la = line_args(c);
    const dim3 lgrid((nxy + kLineThreads - 1) / kLineThreads, c->A.n_dir);
    // a = dL/dS at fixed chi (the transport adjoint of the emergent light); f = a / chi
    la.nu = nullptr;
    hipLaunchKernelGGL(adj_back_kernel, lgrid, dim3(kLineThreads), 0, c->stream, la);
    if ((rc = check_launch(c, "adj_back_kernel"))) return rc;
    hipLaunchKernelGGL(adj_pull_kernel, planes(c), dim3(kPlaneThreads), 0, c->stream, la, 0, c->adj_f);
    if ((rc = check_launch(c, "adj_pull_kernel"))) return rc;
    hipLaunchKernelGGL(adj_record_kernel, lgrid, dim3(kLineThreads), 0, c->stream, la);
    if ((rc = check_launch(c, "adj_record_kernel"))) return rc;
    // (I - Lambda D) nu = f by operator splitting from nu = 0, until max|dnu| < tol max|nu|
    hipLaunchKernelGGL(adj_zero_kernel, dim3((V + 255) / 256), dim3(256), 0, c->stream, V, c->adj_nu);
    if ((rc = check_launch(c, "adj_zero_kernel"))) return rc;
    // Ng acceleration as configured for the forward solve, with unit weights (nu may vanish)
    const int R = c->ng_order + 2;
    const size_t vbytes = size_t(V) * sizeof(double);
    NgArgs ng{};
    ng.V = V; ng.order = c->ng_order; ng.hist = c->ng_hist; ng.work = c->ng_work; ng.J = c->adj_nu;
    ng.unit_weights = 1;
    int nh = 0;
    if (c->ng_order > 0) {
        HIP_TRY(c, hipMemcpyAsync(c->ng_hist, c->adj_nu, vbytes, hipMemcpyDeviceToDevice, c->stream), "ng hist");
        nh = 1;
    }
    int it = 0;
    double rel = INFINITY;
    while (it < max_iter) {
        double dmax = 0.0, numax = 0.0;
        int bad = 0;
        rc = adjoint_os_step(c, inner_sweeps, &dmax, &numax, &bad);
        ++it;
        if (rc) return rc;
        if (bad) return fail(c, RT3D_ERR_NONFINITE, "NaN or Inf in the adjoint iterate");
        rel = numax > 0.0 ? dmax / numax : 0.0;
        if (rel < tol) break;
        if (c->ng_order > 0) {
            HIP_TRY(c, hipMemcpyAsync(c->ng_hist + long(nh % R) * V, c->adj_nu, vbytes, hipMemcpyDeviceToDevice,
                                      c->stream), "ng hist");
            ++nh;
            if (nh - 1 >= c->ng_every) {
                const int m = (nh - 1) % R;
                hipLaunchKernelGGL(ng_dots_kernel, dim3(kNgBlocks), dim3(kNgThreads), 0, c->stream, ng, m);
                hipLaunchKernelGGL(ng_solve_kernel, dim3(1), dim3(kNgThreads), 0, c->stream, ng);
                hipLaunchKernelGGL(ng_combine_kernel, dim3((V + 255) / 256), dim3(256), 0, c->stream, ng, m);
                if ((rc = check_launch(c, "ng kernels (adjoint)"))) return rc;
                HIP_TRY(c, hipMemcpyAsync(c->ng_hist, c->adj_nu, vbytes, hipMemcpyDeviceToDevice, c->stream),
                        "ng hist");
                nh = 1;
            }
        }
    }
    if (iters_out) *iters_out = it;
    if (final_rel_out) *final_rel_out = rel;
    // the chi terms along the lines with the deposit weights (1 - eps) nu W|mu|, then both gradients
    la.nu = c->adj_nu;
    hipLaunchKernelGGL(adj_back_kernel, lgrid, dim3(kLineThreads), 0, c->stream, la);
    if ((rc = check_launch(c, "adj_back_kernel"))) return rc;
    hipLaunchKernelGGL(adj_pull_kernel, planes(c), dim3(kPlaneThreads), 0, c->stream, la, 1, c->adj_pull);
    if ((rc = check_launch(c, "adj_pull_kernel"))) return rc;
    if (c->g.bottom_bc == 2) {
        hipLaunchKernelGGL(adj_bc_kernel, dim3((nxy + 255) / 256), dim3(256), 0, c->stream, la, c->B, c->adj_pull);
        if ((rc = check_launch(c, "adj_bc_kernel"))) return rc;
    }
    AdjFinalArgs fa{};
    fa.V = V;
    fa.chi = c->chi; fa.eps = c->eps; fa.B = c->B; fa.J = c->J; fa.Jfs = c->Jfs; fa.nu = c->adj_nu;
    fa.pull = c->adj_pull;
    const bool dev = ptr_kind == RT3D_DEVICE;
    fa.dchi = dev ? dL_dchi : c->adj_fs;    // host outputs are staged in the solve's scratch vectors
    fa.deps = dev ? dL_deps : c->adj_r;
    hipLaunchKernelGGL(adj_final_kernel, dim3((V + 255) / 256), dim3(256), 0, c->stream, fa);
    if ((rc = check_launch(c, "adj_final_kernel"))) return rc;
    if (!dev) {
        HIP_TRY(c, hipMemcpyAsync(dL_dchi, c->adj_fs, V * sizeof(double), hipMemcpyDeviceToHost, c->stream), "dchi");
        HIP_TRY(c, hipMemcpyAsync(dL_deps, c->adj_r, V * sizeof(double), hipMemcpyDeviceToHost, c->stream), "deps");
    }
    c->have_fs = true;
    rc = sync(c);
    if (rc) return rc;
    return rel < tol ? RT3D_OK : fail(c, RT3D_ERR_NOT_CONVERGED, "adjoint solve reached max_iter");
}

}  // extern "C"
