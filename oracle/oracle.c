/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the 3D radiative-transfer scattering solve of
 * Hauschildt & Baron, "A 3D radiative transfer framework XIII: OpenCL implementation".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  It shares no code, header, table or helper with the HIP library.
 *
 * What is computed (section "Method" and its two implementation subsections):
 *   - the formal solution (FS) along characteristics through a Cartesian voxel grid that is
 *     periodic in x and y, for every solid angle ("Implementation of the formal solution");
 *   - the mean intensity J and the nearest-neighbour (3x3x3) Lambda* operator;
 *   - the operator-splitting (OS) step that solves (1 - Lambda* (1-eps)) dJ = J_fs - J_old by
 *     Jacobi ("Jordan") iterations ("Implementation of the operator splitting step"),
 *     with S = eps B + (1-eps) J for coherent isotropic scattering ("Test case setup").
 *
 * The paper defers the discretisation to the earlier papers of its series.  The readings used here:
 *   grid      unit voxels (i,j,k), k = 0 at the bottom (inner boundary), k = nz-1 at the top;
 *   angles    Gauss-Legendre in mu (n_theta even) x uniform phi_b = 2 pi (b + 1/2) / n_phi,
 *             weight W = w_a / (2 n_phi), so that the weights sum to one;
 *   lines     for every direction one straight line per column (i,j), through (i+1/2, j+1/2, nz);
 *             the same lines serve Omega and -Omega; downward lines start at the top with I_top,
 *             upward lines start at z = 0 with I_bot of the bottom voxel they enter;
 *   medium    chi and S constant inside a voxel, so each piece of line inside one voxel
 *             ("segment") is integrated exactly;
 *   voxel I   Ibar_v(Omega) is the path-length-weighted average of I over all segments of the
 *             direction's lines inside v; every voxel holds exactly 1/|mu| of path per direction;
 *   Lambda*   the 27-point band of the exact Lambda operator (S -> J with zero boundary light);
 *   OS        dJ^0 = 0, a fixed number M of Jacobi sweeps, J <- J + dJ^M,
 *             convergence measure c = max_v |dJ_v| / |J_v^new|, initial guess J^0 = B;
 *             alternatively M Gauss-Seidel sweeps in a multicolour order (the Fortran code's other
 *             choice, named in the same subsection): see orc_gs_colour.
 *
 * Layout: every per-voxel field is [k][j][i] with i fastest; Lambda* is [27][V] with neighbour
 * offset index o = 9 (dk+1) + 3 (dj+1) + (di+1), u = v + (di, dj, dk), periodic in i and j.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EARG -1
#define ORC_ENOMEM -2

/* ------------------------------------------------------------------------------------------------
 * Angular quadrature.
 * --------------------------------------------------------------------------------------------- */

/* Gauss-Legendre nodes x[0..n-1] (ascending) and weights on [-1,1]: Newton iteration on P_n,
 * evaluated with the three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
int orc_gauss_legendre(int n, double *x, double *w)
{
    if (n < 2 || !x || !w) return ORC_EARG;
    for (int r = 0; r < n; ++r) {
        /* r-th root counted from +1 downwards; Chebyshev-like starting guess */
        double z = cos(M_PI * (r + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            /* derivative: (1 - z^2) P_n' = n (P_{n-1} - z P_n) */
            dp = n * (p0 - z * p1) / (1.0 - z * z);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute P_n' at the converged root for the weight */
        {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (p0 - z * p1) / (1.0 - z * z);
        }
        x[n - 1 - r] = z;
        w[n - 1 - r] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return ORC_OK;
}

/* Direction set: d = a * n_phi + b, a over the Gauss-Legendre mu nodes (ascending), b over phi.
 * Omega_d = (sqrt(1-mu^2) cos phi_b, sqrt(1-mu^2) sin phi_b, mu_a), W_d = w_a / (2 n_phi). */
int orc_quadrature(int n_theta, int n_phi, double *mu, double *ox, double *oy, double *wt)
{
    if (n_theta < 2 || (n_theta & 1) || n_phi < 4 || (n_phi % 4) != 0) return ORC_EARG;
    double *xg = (double *)malloc(sizeof(double) * n_theta);
    double *wg = (double *)malloc(sizeof(double) * n_theta);
    if (!xg || !wg) { free(xg); free(wg); return ORC_ENOMEM; }
    orc_gauss_legendre(n_theta, xg, wg);
    for (int a = 0; a < n_theta; ++a) {
        double st = sqrt(1.0 - xg[a] * xg[a]);
        for (int b = 0; b < n_phi; ++b) {
            int d = a * n_phi + b;
            double phi = 2.0 * M_PI * (b + 0.5) / n_phi;
            mu[d] = xg[a];
            ox[d] = st * cos(phi);
            oy[d] = st * sin(phi);
            wt[d] = wg[a] / (2.0 * n_phi);
        }
    }
    free(xg);
    free(wg);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------
 * Geometry: one line through one layer.
 * --------------------------------------------------------------------------------------------- */

typedef struct {
    int nx, ny, nz, n_theta, n_phi, n_dir;
    double *mu, *ox, *oy, *wt;
} Geom;

static int geom_init(Geom *g, int nx, int ny, int nz, int n_theta, int n_phi)
{
    if (nx < 3 || ny < 3 || nz < 1) return ORC_EARG;
    g->nx = nx; g->ny = ny; g->nz = nz; g->n_theta = n_theta; g->n_phi = n_phi;
    g->n_dir = n_theta * n_phi;
    g->mu = (double *)malloc(sizeof(double) * 4 * g->n_dir);
    if (!g->mu) return ORC_ENOMEM;
    g->ox = g->mu + g->n_dir;
    g->oy = g->ox + g->n_dir;
    g->wt = g->oy + g->n_dir;
    int rc = orc_quadrature(n_theta, n_phi, g->mu, g->ox, g->oy, g->wt);
    if (rc) { free(g->mu); g->mu = NULL; }
    return rc;
}

static void geom_free(Geom *g) { free(g->mu); g->mu = NULL; }

static int imod(long a, int n) { long r = a % n; return (int)(r < 0 ? r + n : r); }

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Upper bound on the number of segments of one line inside one layer. */
static int max_segments(const Geom *g, int d)
{
    double tx = fabs(g->ox[d] / g->mu[d]), ty = fabs(g->oy[d] / g->mu[d]);
    return (int)ceil(tx) + (int)ceil(ty) + 3;
}

/* Segments of line (i,j) of direction d inside layer k, in the order the photon travels.
 * The line is x(z) = i + 1/2 + (z - nz) Omega_x / mu, y(z) likewise.  Breakpoints are the
 * parameters f in (0,1) along the layer path where x or y crosses an integer; each piece between
 * breakpoints lies in the voxel that contains its midpoint and has length (f1 - f0) / |mu|.
 * Returns the number of segments written (zero-length pieces at exact ties are dropped). */
static int trace_layer(const Geom *g, int d, int i, int j, int k, double *fbuf,
                       int *seg_v, double *seg_len)
{
    const double mu = g->mu[d];
    const double tx = g->ox[d] / mu, ty = g->oy[d] / mu;
    const double za = (mu < 0.0) ? (double)(k + 1) : (double)k;   /* entry height */
    const double zb = (mu < 0.0) ? (double)k : (double)(k + 1);   /* exit height  */
    const double xa = i + 0.5 + (za - g->nz) * tx, xb = i + 0.5 + (zb - g->nz) * tx;
    const double ya = j + 0.5 + (za - g->nz) * ty, yb = j + 0.5 + (zb - g->nz) * ty;
    int nf = 0;
    fbuf[nf++] = 0.0;
    {
        double lo = fmin(xa, xb), hi = fmax(xa, xb);
        for (double X = floor(lo) + 1.0; X < hi; X += 1.0) fbuf[nf++] = (X - xa) / (xb - xa);
    }
    {
        double lo = fmin(ya, yb), hi = fmax(ya, yb);
        for (double Y = floor(lo) + 1.0; Y < hi; Y += 1.0) fbuf[nf++] = (Y - ya) / (yb - ya);
    }
    qsort(fbuf + 1, nf - 1, sizeof(double), cmp_double);
    fbuf[nf++] = 1.0;
    int ns = 0;
    const double inv_mu = 1.0 / fabs(mu);
    for (int q = 0; q + 1 < nf; ++q) {
        double f0 = fbuf[q], f1 = fbuf[q + 1];
        if (!(f1 > f0)) continue;
        double fm = 0.5 * (f0 + f1);
        double xm = xa + fm * (xb - xa), ym = ya + fm * (yb - ya);
        int iv = imod((long)floor(xm), g->nx), jv = imod((long)floor(ym), g->ny);
        seg_v[ns] = (k * g->ny + jv) * g->nx + iv;
        seg_len[ns] = (f1 - f0) * inv_mu;
        ++ns;
    }
    return ns;
}

/* Exported for the geometry tests: segments of line (i,j), direction d, layer k. */
int orc_trace_layer(int nx, int ny, int nz, int n_theta, int n_phi, int d, int i, int j, int k,
                    int *seg_v, double *seg_len, int max_seg)
{
    Geom g;
    int rc = geom_init(&g, nx, ny, nz, n_theta, n_phi);
    if (rc) return rc;
    if (d < 0 || d >= g.n_dir || k < 0 || k >= nz) { geom_free(&g); return ORC_EARG; }
    int ms = max_segments(&g, d);
    if (max_seg < ms) { geom_free(&g); return ORC_EARG; }
    double *fbuf = (double *)malloc(sizeof(double) * (ms + 2));
    int ns = trace_layer(&g, d, i, j, k, fbuf, seg_v, seg_len);
    free(fbuf);
    geom_free(&g);
    return ns;
}

/* ------------------------------------------------------------------------------------------------
 * Formal solution.
 * --------------------------------------------------------------------------------------------- */

/* One direction: trace every line from its boundary through all layers, integrate I exactly across
 * each segment and accumulate D_s = chi_v * (integral of I over the segment) per voxel.
 *   dtau = chi_v l,  em1 = expm1(-dtau) = e^{-dtau} - 1,
 *   I_out = I_in + (I_in - S_v) em1,          (exact solution for constant chi, S)
 *   D_s   = S_v dtau - (I_in - S_v) em1.
 * Dsum[v] receives sum_s D_s; Iem (optional) receives I at the top plane of upward lines. */
static void fs_direction(const Geom *g, int d, const double *chi, const double *S, double I_top,
                         const double *I_bot, const double *I_slope, double *Dsum, double *Iem,
                         double *fbuf, int *seg_v, double *seg_len)
{
    const double mu = g->mu[d];
    for (int j = 0; j < g->ny; ++j) {
        for (int i = 0; i < g->nx; ++i) {
            double I = I_top;
            for (int step = 0; step < g->nz; ++step) {
                int k = (mu < 0.0) ? g->nz - 1 - step : step;
                int ns = trace_layer(g, d, i, j, k, fbuf, seg_v, seg_len);
                if (mu > 0.0 && step == 0) {
                    /* upward line: boundary intensity of the bottom voxel it enters (in layer 0
                     * the voxel index equals the column index j*nx + i), plus mu times the slope
                     * of the LTE-diffusion condition when one is given */
                    I = I_bot ? I_bot[seg_v[0]] : 0.0;
                    if (I_slope) I += mu * I_slope[seg_v[0]];
                }
                for (int s = 0; s < ns; ++s) {
                    int v = seg_v[s];
                    double dtau = chi[v] * seg_len[s];
                    double em1 = expm1(-dtau);
                    double D = S[v] * dtau - (I - S[v]) * em1;
                    I = I + (I - S[v]) * em1;
                    Dsum[v] += D;
                }
            }
            if (Iem && mu > 0.0) Iem[j * g->nx + i] = I;
        }
    }
}

static int n_threads_of(int req)
{
#ifdef _OPENMP
    if (req > 0) return req;
    return omp_get_max_threads();
#else
    (void)req;
    return 1;
#endif
}

/* J_v = sum_d W_d Ibar_v(d),  Ibar_v(d) = |mu_d| / chi_v * sum_{s in v} D_s.
 * I_bot: [ny][nx] intensities entering the bottom plane (NULL = zero).
 * Iem (optional): [n_up][ny][nx], I leaving the top plane along the upward directions, in
 * direction order.  Ibar (optional): [n_dir][V] per-direction voxel intensities.
 * Threads split the directions; each thread sums its own directions in order, and the threads'
 * partial sums are added in thread order. */
static int fs_dirs(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi, const double *S,
                   double I_top, const double *I_bot, const double *I_slope, double *J, double *Iem,
                   double *Ibar, int n_threads, const int *dir_list, int n_list);

int orc_formal_solution(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi,
                        const double *S, double I_top, const double *I_bot, double *J,
                        double *Iem, double *Ibar, int n_threads)
{
    return fs_dirs(nx, ny, nz, n_theta, n_phi, chi, S, I_top, I_bot, NULL, J, Iem, Ibar, n_threads,
                   NULL, 0);
}

/* As orc_formal_solution with the LTE-diffusion inner condition: an upward line of direction cosine
 * mu enters with I_bot + mu * I_slope of the bottom voxel it enters (I_slope: [ny][nx], the
 * gradient dB/dtau at the inner boundary). */
int orc_formal_solution_slope(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi,
                              const double *S, double I_top, const double *I_bot,
                              const double *I_slope, double *J, double *Iem, double *Ibar,
                              int n_threads)
{
    return fs_dirs(nx, ny, nz, n_theta, n_phi, chi, S, I_top, I_bot, I_slope, J, Iem, Ibar, n_threads,
                   NULL, 0);
}

/* As orc_formal_solution, restricted to the directions in dir_list[0..n_list-1] (all directions
 * when dir_list is NULL): J then holds only their share of the angle sum. */
int orc_formal_solution_dirs(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi,
                             const double *S, double I_top, const double *I_bot, double *J,
                             double *Iem, double *Ibar, int n_threads, const int *dir_list,
                             int n_list)
{
    return fs_dirs(nx, ny, nz, n_theta, n_phi, chi, S, I_top, I_bot, NULL, J, Iem, Ibar, n_threads,
                   dir_list, n_list);
}

static int fs_dirs(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi, const double *S,
                   double I_top, const double *I_bot, const double *I_slope, double *J, double *Iem,
                   double *Ibar, int n_threads, const int *dir_list, int n_list)
{
    Geom g;
    int rc = geom_init(&g, nx, ny, nz, n_theta, n_phi);
    if (rc) return rc;
    const long V = (long)nx * ny * nz;
    const int nt = n_threads_of(n_threads);
    double *Jt = (double *)calloc((size_t)nt * V, sizeof(double));
    if (!Jt) { geom_free(&g); return ORC_ENOMEM; }
    const int n_down = g.n_dir / 2;   /* mu nodes ascending: the first half of d points down */
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int ms = 0;
        for (int d = 0; d < g.n_dir; ++d) if (max_segments(&g, d) > ms) ms = max_segments(&g, d);
        double *fbuf = (double *)malloc(sizeof(double) * (ms + 2));
        int *seg_v = (int *)malloc(sizeof(int) * ms);
        double *seg_len = (double *)malloc(sizeof(double) * ms);
        double *Dsum = (double *)malloc(sizeof(double) * V);
        if (!fbuf || !seg_v || !seg_len || !Dsum) {
#pragma omp atomic write
            fail = 1;
        } else {
            double *Jmine = Jt + (size_t)tid * V;
            const int n_sel = dir_list ? n_list : g.n_dir;
            for (int q = tid; q < n_sel; q += nt) {
                const int d = dir_list ? dir_list[q] : q;
                if (d < 0 || d >= g.n_dir) continue;
                memset(Dsum, 0, sizeof(double) * V);
                double *Iem_d = (Iem && g.mu[d] > 0.0) ? Iem + (size_t)(d - n_down) * nx * ny : NULL;
                fs_direction(&g, d, chi, S, I_top, I_bot, I_slope, Dsum, Iem_d, fbuf, seg_v, seg_len);
                const double amu = fabs(g.mu[d]);
                for (long v = 0; v < V; ++v) {
                    double ib = amu / chi[v] * Dsum[v];
                    if (Ibar) Ibar[(size_t)d * V + v] = ib;
                    Jmine[v] += g.wt[d] * ib;
                }
            }
        }
        free(fbuf); free(seg_v); free(seg_len); free(Dsum);
    }
    if (!fail) {
        for (long v = 0; v < V; ++v) {
            double s = 0.0;
            for (int t = 0; t < nt; ++t) s += Jt[(size_t)t * V + v];
            J[v] = s;
        }
    }
    free(Jt);
    geom_free(&g);
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------------------------------
 * Lambda*: the 27-point band of Lambda, built along the lines.
 * --------------------------------------------------------------------------------------------- */

/* Neighbour offset index of u relative to v, or -1 if u is not in the 3x3x3 block around v. */
static int nb_index(const Geom *g, int v, int u)
{
    int iv = v % g->nx, jv = (v / g->nx) % g->ny, kv = v / (g->nx * g->ny);
    int iu = u % g->nx, ju = (u / g->nx) % g->ny, ku = u / (g->nx * g->ny);
    int dk = ku - kv;
    if (dk < -1 || dk > 1) return -1;
    int di = imod(iu - iv, g->nx), dj = imod(ju - jv, g->ny);
    if (di == g->nx - 1) di = -1; else if (di > 1) return -1;
    if (dj == g->ny - 1) dj = -1; else if (dj > 1) return -1;
    return 9 * (dk + 1) + 3 * (dj + 1) + (di + 1);
}

/* e^{-x} - 1 + x for x >= 0 (the self term of dD/dS), summed as its Taylor series
 * x^2/2! - x^3/3! + ... below x = 1/2 so that thin segments do not lose digits to cancellation. */
static double self_term(double x)
{
    if (x >= 0.5) return x + expm1(-x);
    double fact = 1.0;                      /* 17! built up, then divided down */
    for (int n = 2; n <= 17; ++n) fact *= n;
    double r = 1.0 / fact;                  /* coefficient of x^15 in the bracket: 1/17! */
    for (int n = 17; n > 2; --n) {
        fact /= n;                          /* now (n-1)! */
        r = 1.0 / fact - x * r;
    }
    return x * x * r;
}

/* Lambda*_{vu} = sum_d W_d dIbar_v(d)/dS_u for u in the 3x3x3 block of v.
 * For segment s in voxel v:  dD_s/dS_u = delta_uv (dtau_s + em1_s) - em1_s dI_in,s/dS_u, and
 * dI_in,s/dS_u = sum over earlier segments s' in u of c_{s'->s} = (1 - e_{s'}) prod_{s'<s''<s} e_{s''},
 * e = exp(-dtau).  Lines are monotone in z, so every earlier segment that can lie in the 3x3x3 block
 * is in the current or the previous layer: a window of those segments with their running c values
 * makes the band exact (all segments in u are included, also when a line wraps around a small grid). */
int orc_lstar(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi, double *L,
              int n_threads)
{
    Geom g;
    int rc = geom_init(&g, nx, ny, nz, n_theta, n_phi);
    if (rc) return rc;
    const long V = (long)nx * ny * nz;
    const int nt = n_threads_of(n_threads);
    double *Lt = (double *)calloc((size_t)nt * 27 * V, sizeof(double));
    if (!Lt) { geom_free(&g); return ORC_ENOMEM; }
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int ms = 0;
        for (int d = 0; d < g.n_dir; ++d) if (max_segments(&g, d) > ms) ms = max_segments(&g, d);
        double *fbuf = (double *)malloc(sizeof(double) * (ms + 2));
        int *seg_v = (int *)malloc(sizeof(int) * ms);
        double *seg_len = (double *)malloc(sizeof(double) * ms);
        /* window: voxel, layer and c of every segment in the current and the previous layer */
        int *win_v = (int *)malloc(sizeof(int) * 2 * ms);
        int *win_k = (int *)malloc(sizeof(int) * 2 * ms);
        double *win_c = (double *)malloc(sizeof(double) * 2 * ms);
        if (!fbuf || !seg_v || !seg_len || !win_v || !win_k || !win_c) {
#pragma omp atomic write
            fail = 1;
        } else {
            double *Lm = Lt + (size_t)tid * 27 * V;
            for (int d = tid; d < g.n_dir; d += nt) {
                const double mu = g.mu[d], amu = fabs(mu), W = g.wt[d];
                for (int j = 0; j < ny; ++j) {
                    for (int i = 0; i < nx; ++i) {
                        int nw = 0;
                        for (int step = 0; step < nz; ++step) {
                            int k = (mu < 0.0) ? nz - 1 - step : step;
                            /* drop window entries two or more layers upstream */
                            int keep = 0;
                            for (int q = 0; q < nw; ++q) {
                                if (abs(win_k[q] - k) <= 1) {
                                    win_v[keep] = win_v[q]; win_k[keep] = win_k[q];
                                    win_c[keep] = win_c[q]; ++keep;
                                }
                            }
                            nw = keep;
                            int ns = trace_layer(&g, d, i, j, k, fbuf, seg_v, seg_len);
                            for (int s = 0; s < ns; ++s) {
                                int v = seg_v[s];
                                double dtau = chi[v] * seg_len[s];
                                double em1 = expm1(-dtau);
                                double fac = W * amu / chi[v];
                                Lm[13 * V + v] += fac * self_term(dtau);
                                for (int q = 0; q < nw; ++q) {
                                    int o = nb_index(&g, v, win_v[q]);
                                    if (o >= 0) Lm[(size_t)o * V + v] += fac * (-em1) * win_c[q];
                                }
                                /* attenuation e^{-dtau} itself: 1 + em1 would lose all relative
                                 * accuracy once dtau >> 1 */
                                const double att = exp(-dtau);
                                for (int q = 0; q < nw; ++q) win_c[q] *= att;
                                win_v[nw] = v; win_k[nw] = k; win_c[nw] = -em1; ++nw;
                            }
                        }
                    }
                }
            }
        }
        free(fbuf); free(seg_v); free(seg_len); free(win_v); free(win_k); free(win_c);
    }
    if (!fail) {
        for (long q = 0; q < 27 * V; ++q) {
            double s = 0.0;
            for (int t = 0; t < nt; ++t) s += Lt[(size_t)t * 27 * V + q];
            L[q] = s;
        }
    }
    free(Lt);
    geom_free(&g);
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* Dense Lambda by brute force (tiny grids only): column u is the mean intensity produced by a unit
 * source in voxel u alone, with zero boundary intensities.  Lam[v * V + u]. */
int orc_lambda_bruteforce(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi,
                          double *Lam, int n_threads)
{
    const long V = (long)nx * ny * nz;
    double *S = (double *)calloc(V, sizeof(double));
    double *J = (double *)malloc(sizeof(double) * V);
    if (!S || !J) { free(S); free(J); return ORC_ENOMEM; }
    int rc = ORC_OK;
    for (long u = 0; u < V && rc == ORC_OK; ++u) {
        S[u] = 1.0;
        rc = orc_formal_solution(nx, ny, nz, n_theta, n_phi, chi, S, 0.0, NULL, J, NULL, NULL,
                                 n_threads);
        for (long v = 0; v < V; ++v) Lam[v * V + u] = J[v];
        S[u] = 0.0;
    }
    free(S);
    free(J);
    return rc;
}

/* ------------------------------------------------------------------------------------------------
 * Operator splitting.
 * --------------------------------------------------------------------------------------------- */

/* The gradient of B at the inner boundary for the LTE-diffusion condition, per column:
 * (B_0 - B_1) / ((chi_0 + chi_1) / 2), layer 0 the bottom voxel and layer 1 the one above it. */
void orc_diffusion_slope(int nx, int ny, const double *chi, const double *B, double *slope)
{
    const long nxy = (long)nx * ny;
    for (long c = 0; c < nxy; ++c) slope[c] = (B[c] - B[nxy + c]) / (0.5 * (chi[c] + chi[nxy + c]));
}

/* One OS step ("Implementation of the operator splitting step"):
 *   S = eps B + (1-eps) J;  J_fs = FS(S);  r = J_fs - J;
 *   M Jacobi sweeps from dJ^0 = 0 of
 *     dJ^{m+1}_v = (r_v + sum_{u != v} Lstar_vu (1-eps_u) dJ^m_u) / (1 - Lstar_vv (1-eps_v));
 *   J <- J + dJ^M;  c = max_v |dJ_v| / |J_v|.
 * Boundary light: I_top at the top; at the bottom (bottom_from_B) 0: zero, 1: I_bot = B of the
 * bottom voxel a line enters, 2: LTE diffusion, I_bot = B + mu dB/dtau with
 * dB/dtau = (B_0 - B_1) / ((chi_0 + chi_1) / 2) from the bottom voxel and the one above it (the
 * optical distance between their centres; tau grows inwards).  Jfs_out (optional) receives J_fs. */
/* Colour of index i (0 <= i < n) in the multicolour ordering of the Gauss-Seidel sweep.  Two voxels
 * are 27-point neighbours when every coordinate differs by at most one (cyclically in x and y), so a
 * colouring per axis in which adjacent indices differ gives, as the triple (cx, cy, cz), a colouring
 * in which no two voxels of a colour are neighbours: along z (not periodic) k mod 2; along a periodic
 * axis i mod 2 when n is even, and when n is odd i mod 2 except colour 2 for i = n - 1 (its
 * neighbours n - 2 and 0 are odd and even).  The number of colours per axis is returned through
 * *n_colours.  The colours are swept in the order c = (cz * ncy + cy) * ncx + cx. */
int orc_gs_colour(int n, int periodic, int i, int *n_colours)
{
    if (!periodic || n % 2 == 0) {
        if (n_colours) *n_colours = 2;
        return i % 2;
    }
    if (n_colours) *n_colours = 3;
    return i == n - 1 ? 2 : i % 2;
}

/* The inner solve of the OS step: M sweeps of
 *   dJ_v <- (r_v + sum_{u != v} Lstar_vu (1-eps_u) dJ_u) / (1 - Lstar_vv (1-eps_v))  from dJ = 0,
 * Jacobi (method 0: every voxel from the previous sweep's dJ) or Gauss-Seidel (method 1: in place,
 * colour after colour in the order of orc_gs_colour, so each voxel sees the newest dJ of every
 * neighbour of an earlier colour). */
static void os_inner(int nx, int ny, int nz, const double *eps, const double *Lstar, const double *r,
                     int M, int method, double *dJ, double *dJn)
{
    const long V = (long)nx * ny * nz;
    int ncx, ncy, ncz;
    orc_gs_colour(nx, 1, 0, &ncx);
    orc_gs_colour(ny, 1, 0, &ncy);
    orc_gs_colour(nz, 0, 0, &ncz);
    const int n_pass = method == 1 ? ncx * ncy * ncz : 1;
    for (int m = 0; m < M; ++m) {
        /* Jacobi reads the previous sweep (dJ) and writes dJn; Gauss-Seidel reads and writes dJ.
         * Within a Jacobi sweep (and within one colour of a Gauss-Seidel pass) no voxel reads a value
         * written in the same pass, so the layers may be updated by several threads at once; each
         * voxel's sum keeps its order, so the result does not depend on the thread count. */
        const double *src = dJ;
        double *dst = method == 1 ? dJ : dJn;
        for (int pass = 0; pass < n_pass; ++pass)
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        if (method == 1) {
                            int c = (orc_gs_colour(nz, 0, k, NULL) * ncy + orc_gs_colour(ny, 1, j, NULL)) * ncx
                                    + orc_gs_colour(nx, 1, i, NULL);
                            if (c != pass) continue;
                        }
                        long v = ((long)k * ny + j) * nx + i;
                        double acc = r[v];
                        for (int dk = -1; dk <= 1; ++dk) {
                            if (k + dk < 0 || k + dk >= nz) continue;
                            for (int dj = -1; dj <= 1; ++dj)
                                for (int di = -1; di <= 1; ++di) {
                                    int o = 9 * (dk + 1) + 3 * (dj + 1) + (di + 1);
                                    if (o == 13) continue;
                                    long u = ((long)(k + dk) * ny + imod(j + dj, ny)) * nx
                                             + imod(i + di, nx);
                                    acc += Lstar[(size_t)o * V + v] * (1.0 - eps[u]) * src[u];
                                }
                        }
                        dst[v] = acc / (1.0 - Lstar[13 * V + v] * (1.0 - eps[v]));
                    }
        if (method != 1) memcpy(dJ, dJn, sizeof(double) * V);
    }
}

/* One OS step with the inner solve of os_inner (method 0 Jacobi, 1 Gauss-Seidel); otherwise as
 * orc_os_step. */
int orc_os_step_method(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi,
                       const double *eps, const double *B, double I_top, int bottom_from_B,
                       const double *Lstar, double *J, int M, int method, double *c_out,
                       double *Jfs_out, int n_threads)
{
    if (M < 1 || method < 0 || method > 1) return ORC_EARG;
    const long V = (long)nx * ny * nz;
    double *S = (double *)malloc(sizeof(double) * V);
    double *Jfs = (double *)malloc(sizeof(double) * V);
    double *r = (double *)calloc(V, sizeof(double));
    double *dJ = (double *)calloc(V, sizeof(double));
    double *dJn = (double *)malloc(sizeof(double) * V);
    if (!S || !Jfs || !r || !dJ || !dJn) {
        free(S); free(Jfs); free(r); free(dJ); free(dJn);
        return ORC_ENOMEM;
    }
    for (long v = 0; v < V; ++v) S[v] = eps[v] * B[v] + (1.0 - eps[v]) * J[v];
    double *slope = NULL;
    if (bottom_from_B == 2) {
        if (nz < 2) { free(S); free(Jfs); free(r); free(dJ); free(dJn); return ORC_EARG; }
        slope = (double *)malloc(sizeof(double) * nx * ny);
        if (!slope) { free(S); free(Jfs); free(r); free(dJ); free(dJn); return ORC_ENOMEM; }
        orc_diffusion_slope(nx, ny, chi, B, slope);
    }
    int rc = fs_dirs(nx, ny, nz, n_theta, n_phi, chi, S, I_top, bottom_from_B ? B : NULL, slope, Jfs,
                     NULL, NULL, n_threads, NULL, 0);
    free(slope);
    if (rc == ORC_OK) {
        for (long v = 0; v < V; ++v) r[v] = Jfs[v] - J[v];
        os_inner(nx, ny, nz, eps, Lstar, r, M, method, dJ, dJn);
        double c = 0.0;
        for (long v = 0; v < V; ++v) {
            J[v] += dJ[v];
            double q = fabs(dJ[v]) / fabs(J[v]);
            if (q > c || q != q) c = q;
        }
        if (c_out) *c_out = c;
        if (Jfs_out) memcpy(Jfs_out, Jfs, sizeof(double) * V);
    }
    free(S); free(Jfs); free(r); free(dJ); free(dJn);
    return rc;
}

int orc_os_step(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi, const double *eps,
                const double *B, double I_top, int bottom_from_B, const double *Lstar, double *J,
                int M, double *c_out, double *Jfs_out, int n_threads)
{
    return orc_os_step_method(nx, ny, nz, n_theta, n_phi, chi, eps, B, I_top, bottom_from_B, Lstar, J, M,
                              0, c_out, Jfs_out, n_threads);
}

/* The inner solve alone, for the pins: M sweeps (method 0 Jacobi, 1 Gauss-Seidel) of the OS
 * equations with right-hand side r; dJ ([V]) receives the result. */
int orc_os_inner(int nx, int ny, int nz, const double *eps, const double *Lstar, const double *r, int M,
                 int method, double *dJ)
{
    if (M < 1 || method < 0 || method > 1) return ORC_EARG;
    const long V = (long)nx * ny * nz;
    double *tmp = (double *)malloc(sizeof(double) * V);
    if (!tmp) return ORC_ENOMEM;
    memset(dJ, 0, sizeof(double) * V);
    os_inner(nx, ny, nz, eps, Lstar, r, M, method, dJ, tmp);
    free(tmp);
    return ORC_OK;
}

/* Ng acceleration of the outer iteration (named among the host-side parts of the method in the
 * "Method" section; the paper does not spell it out -- this is Ng's least-squares extrapolation).
 * hist[0..m] are the m+1 newest iterates, hist[m] the newest.  With delta_i = x_{n-i} - x_{n-i-1}
 * and Q_i = delta_0 - delta_i (i = 1..order), the coefficients a minimise
 * sum_v w_v (delta_0 - sum_i a_i Q_i)_v^2 with w = 1 / x_n^2, and the new iterate is
 * (1 - sum a_i) x_n + sum_i a_i x_{n-i}.  Returns 0 on success, 1 if the normal equations are
 * singular (the caller then keeps x_n). */
static int ng_extrapolate(long V, int order, double *const *hist, int m, double *out)
{
    double A[3][3] = {{0}}, b[3] = {0}, a[3] = {0};
    const double *x0 = hist[m];
    for (long v = 0; v < V; ++v) {
        double w = 1.0 / (x0[v] * x0[v]);
        double d0 = hist[m][v] - hist[m - 1][v];
        double Q[3];
        for (int i = 1; i <= order; ++i) Q[i - 1] = d0 - (hist[m - i][v] - hist[m - i - 1][v]);
        for (int i = 0; i < order; ++i) {
            b[i] += w * d0 * Q[i];
            for (int j = 0; j < order; ++j) A[i][j] += w * Q[i] * Q[j];
        }
    }
    /* Gaussian elimination with partial pivoting on the order x order system */
    int n = order;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r) if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (!(fabs(A[p][c]) > 0.0)) return 1;
        if (p != c) {
            for (int q = 0; q < n; ++q) { double t = A[c][q]; A[c][q] = A[p][q]; A[p][q] = t; }
            double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r][c] / A[c][c];
            for (int q = c; q < n; ++q) A[r][q] -= f * A[c][q];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double t = b[c];
        for (int q = c + 1; q < n; ++q) t -= A[c][q] * a[q];
        a[c] = t / A[c][c];
    }
    double sa = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!isfinite(a[i])) return 1;
        sa += a[i];
    }
    for (long v = 0; v < V; ++v) {
        double x = (1.0 - sa) * x0[v];
        for (int i = 1; i <= n; ++i) x += a[i - 1] * hist[m - i][v];
        out[v] = x;
    }
    return 0;
}

/* Exported for the Ng pins: hist is [m+1][V] (oldest first); writes the extrapolated iterate. */
int orc_ng_extrapolate(long V, int order, const double *hist_flat, int m, double *out)
{
    if (order < 1 || order > 3 || m < order + 1) return ORC_EARG;
    double *ptrs[8];
    if (m >= 8) return ORC_EARG;
    for (int q = 0; q <= m; ++q) ptrs[q] = (double *)(hist_flat + (size_t)q * V);
    return ng_extrapolate(V, order, ptrs, m, out);
}

/* Outer OS iteration with optional Ng acceleration: after every OS step the iterate joins a history
 * that restarts at each extrapolation; once it holds ng_every >= ng_order + 1 steps the newest
 * iterates are extrapolated (ng_order 1..3; 0 = plain iteration).  The convergence test uses c of
 * the OS step that was just taken. */
int orc_solve_ng(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi,
                 const double *eps, const double *B, double I_top, int bottom_from_B,
                 const double *Lstar, double *J, double tol, int max_iter, int M, int ng_order,
                 int ng_every, int *iters, double *c_out, int n_threads)
{
    if (ng_order < 0 || ng_order > 3 || (ng_order > 0 && ng_every < ng_order + 1)) return ORC_EARG;
    const long V = (long)nx * ny * nz;
    double *Lown = NULL;
    if (!Lstar) {
        Lown = (double *)malloc(sizeof(double) * 27 * V);
        if (!Lown) return ORC_ENOMEM;
        int rc = orc_lstar(nx, ny, nz, n_theta, n_phi, chi, Lown, n_threads);
        if (rc) { free(Lown); return rc; }
        Lstar = Lown;
    }
    const int cap = ng_order > 0 ? ng_every + 1 : 0;
    double **hist = NULL;
    if (cap) {
        hist = (double **)calloc(cap, sizeof(double *));
        for (int q = 0; hist && q < cap; ++q) hist[q] = (double *)malloc(sizeof(double) * V);
        if (!hist || !hist[cap - 1]) { free(Lown); return ORC_ENOMEM; }
        memcpy(hist[0], J, sizeof(double) * V);
    }
    int nh = 1;
    double c = INFINITY;
    int n = 0, rc = ORC_OK;
    while (n < max_iter) {
        rc = orc_os_step(nx, ny, nz, n_theta, n_phi, chi, eps, B, I_top, bottom_from_B, Lstar, J, M,
                         &c, NULL, n_threads);
        ++n;
        if (rc != ORC_OK || c < tol) break;
        if (cap) {
            memcpy(hist[nh], J, sizeof(double) * V);
            ++nh;
            if (nh - 1 >= ng_every) {
                if (ng_extrapolate(V, ng_order, hist, nh - 1, J) == 0) { /* J extrapolated */ }
                memcpy(hist[0], J, sizeof(double) * V);
                nh = 1;
            }
        }
    }
    for (int q = 0; q < cap; ++q) free(hist[q]);
    free(hist);
    free(Lown);
    if (iters) *iters = n;
    if (c_out) *c_out = c;
    if (rc != ORC_OK) return rc;
    return (c < tol) ? ORC_OK : 1;
}

/* Anderson mixing (type II) of the outer iteration -- an alternative to Ng's extrapolation, not from
 * the paper: every OS step x -> g = G(x) joins a sliding window of the newest k + 1 pairs (x_i, g_i),
 * i = 0 (oldest) .. k (newest), with residuals f_i = g_i - x_i.  With df_j = f_k - f_{k-j} and
 * dg_j = g_k - g_{k-j} (j = 1..k), gamma minimises sum_v w_v (f_k - sum_j gamma_j df_j)_v^2 with the
 * weights w = 1 / g_k^2 of Ng's extrapolation, and the next input is g_k - sum_j gamma_j dg_j.  For an
 * affine G the residual of that input is the weighted least-squares residual over the window.
 * Returns 0, or 1 if the normal equations are singular or their solution is not finite (out is then
 * g_k). */
static int anderson_mix(long V, int k, double *const *X, double *const *G, double *out)
{
    double A[8][8] = {{0}}, b[8] = {0}, gam[8] = {0};
    if (k < 1 || k > 8) return 1;
    const double *gk = G[k], *xk = X[k];
    for (long v = 0; v < V; ++v) {
        const double w = 1.0 / (gk[v] * gk[v]);
        const double fk = gk[v] - xk[v];
        double df[8];
        for (int j = 1; j <= k; ++j) df[j - 1] = fk - (G[k - j][v] - X[k - j][v]);
        for (int i = 0; i < k; ++i) {
            b[i] += w * df[i] * fk;
            for (int j = 0; j < k; ++j) A[i][j] += w * df[i] * df[j];
        }
    }
    int bad = 0;
    for (int c = 0; c < k && !bad; ++c) {          /* Gaussian elimination, partial pivoting */
        int p = c;
        for (int r = c + 1; r < k; ++r) if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (!(fabs(A[p][c]) > 0.0)) { bad = 1; break; }
        if (p != c) {
            for (int q = 0; q < k; ++q) { double t = A[c][q]; A[c][q] = A[p][q]; A[p][q] = t; }
            double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < k; ++r) {
            double f = A[r][c] / A[c][c];
            for (int q = c; q < k; ++q) A[r][q] -= f * A[c][q];
            b[r] -= f * b[c];
        }
    }
    for (int c = k - 1; c >= 0 && !bad; --c) {
        double t = b[c];
        for (int q = c + 1; q < k; ++q) t -= A[c][q] * gam[q];
        gam[c] = t / A[c][c];
        if (!isfinite(gam[c])) bad = 1;
    }
    for (long v = 0; v < V; ++v) {
        double x = gk[v];
        if (!bad)
            for (int j = 1; j <= k; ++j) x -= gam[j - 1] * (gk[v] - G[k - j][v]);
        out[v] = x;
    }
    return bad;
}

/* Exported for the pins: X_flat, G_flat are [k+1][V] (oldest first). */
int orc_anderson_mix(long V, int k, const double *X_flat, const double *G_flat, double *out)
{
    double *xs[9], *gs[9];
    if (k < 1 || k > 8) return ORC_EARG;
    for (int q = 0; q <= k; ++q) {
        xs[q] = (double *)(X_flat + (size_t)q * V);
        gs[q] = (double *)(G_flat + (size_t)q * V);
    }
    return anderson_mix(V, k, xs, gs, out);
}

/* Outer OS iteration with Anderson mixing of depth m (1..8): the input of every step after the first
 * is the mixing of the newest min(steps, m + 1) pairs; c is that of the OS step just taken, and on
 * c < tol J receives its output g. */
int orc_solve_anderson(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi,
                       const double *eps, const double *B, double I_top, int bottom_from_B,
                       const double *Lstar, double *J, double tol, int max_iter, int M, int depth,
                       int *iters, double *c_out, int n_threads)
{
    if (depth < 1 || depth > 8) return ORC_EARG;
    const long V = (long)nx * ny * nz;
    double *Lown = NULL;
    if (!Lstar) {
        Lown = (double *)malloc(sizeof(double) * 27 * V);
        if (!Lown) return ORC_ENOMEM;
        int rc = orc_lstar(nx, ny, nz, n_theta, n_phi, chi, Lown, n_threads);
        if (rc) { free(Lown); return rc; }
        Lstar = Lown;
    }
    const int cap = depth + 1;
    double *buf = (double *)malloc(sizeof(double) * (size_t)(2 * cap + 1) * V);
    if (!buf) { free(Lown); return ORC_ENOMEM; }
    double *X[9], *G[9];
    for (int q = 0; q < cap; ++q) { X[q] = buf + (size_t)q * V; G[q] = buf + (size_t)(cap + q) * V; }
    double *x = buf + (size_t)2 * cap * V;          /* input of the next step */
    memcpy(x, J, sizeof(double) * V);
    int count = 0, n = 0, rc = ORC_OK;
    double c = INFINITY;
    while (n < max_iter) {
        /* the window, oldest first: shift out the oldest pair when full */
        if (count == cap) {
            double *tx = X[0], *tg = G[0];
            for (int q = 0; q + 1 < cap; ++q) { X[q] = X[q + 1]; G[q] = G[q + 1]; }
            X[cap - 1] = tx; G[cap - 1] = tg;
            --count;
        }
        memcpy(X[count], x, sizeof(double) * V);
        memcpy(G[count], x, sizeof(double) * V);
        rc = orc_os_step(nx, ny, nz, n_theta, n_phi, chi, eps, B, I_top, bottom_from_B, Lstar, G[count], M,
                         &c, NULL, n_threads);
        ++n;
        ++count;
        if (rc != ORC_OK) break;
        if (c < tol) break;
        if (count >= 2) anderson_mix(V, count - 1, X, G, x);
        else memcpy(x, G[0], sizeof(double) * V);
    }
    if (count > 0) memcpy(J, G[count - 1], sizeof(double) * V);
    free(buf);
    free(Lown);
    if (iters) *iters = n;
    if (c_out) *c_out = c;
    if (rc != ORC_OK) return rc;
    return (c < tol) ? ORC_OK : 1;
}

/* Outer OS iteration until c < tol (or max_iter steps).  J holds the initial guess on entry (the
 * usual start is J = B) and the last iterate on exit.  Lstar may be NULL: it is then built here.
 * Returns the number of steps in *iters and the last c in *c_out; the return code is 1 when
 * max_iter was reached without c < tol. */
int orc_solve(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi, const double *eps,
              const double *B, double I_top, int bottom_from_B, const double *Lstar, double *J,
              double tol, int max_iter, int M, int *iters, double *c_out, int n_threads)
{
    const long V = (long)nx * ny * nz;
    double *Lown = NULL;
    if (!Lstar) {
        Lown = (double *)malloc(sizeof(double) * 27 * V);
        if (!Lown) return ORC_ENOMEM;
        int rc = orc_lstar(nx, ny, nz, n_theta, n_phi, chi, Lown, n_threads);
        if (rc) { free(Lown); return rc; }
        Lstar = Lown;
    }
    double c = INFINITY;
    int n = 0, rc = ORC_OK;
    while (n < max_iter) {
        rc = orc_os_step(nx, ny, nz, n_theta, n_phi, chi, eps, B, I_top, bottom_from_B, Lstar, J, M,
                         &c, NULL, n_threads);
        ++n;
        if (rc != ORC_OK || c < tol) break;
    }
    free(Lown);
    if (iters) *iters = n;
    if (c_out) *c_out = c;
    if (rc != ORC_OK) return rc;
    return (c < tol) ? ORC_OK : 1;
}

/* ------------------------------------------------------------------------------------------------
 * Plane-parallel (1D) formal solution, written without any 3D geometry.
 * --------------------------------------------------------------------------------------------- */

/* Layers k = 0 (bottom) .. nz-1 (top) with vertical optical thickness dtau[k] > 0 and source S[k].
 * For each Gauss-Legendre node mu_a the slant thickness is dtau/|mu|; the layer-averaged intensity
 * of an exactly integrated constant-source layer is  Ibar = S - (I_in - S) em1 / (dtau/|mu|),
 * and J_k = sum_a (w_a / 2) Ibar_k(mu_a). */
int orc_pp1d(int nz, int n_theta, const double *dtau, const double *S, double I_top, double I_bot,
             double I_slope, double *J)
{
    if (nz < 1 || n_theta < 2 || (n_theta & 1)) return ORC_EARG;
    double *x = (double *)malloc(sizeof(double) * n_theta);
    double *w = (double *)malloc(sizeof(double) * n_theta);
    if (!x || !w) { free(x); free(w); return ORC_ENOMEM; }
    orc_gauss_legendre(n_theta, x, w);
    for (int k = 0; k < nz; ++k) J[k] = 0.0;
    for (int a = 0; a < n_theta; ++a) {
        double amu = fabs(x[a]);
        /* upward light at the bottom: I_bot + mu I_slope (I_slope = 0 except for LTE diffusion) */
        double I = (x[a] < 0.0) ? I_top : I_bot + x[a] * I_slope;
        for (int step = 0; step < nz; ++step) {
            int k = (x[a] < 0.0) ? nz - 1 - step : step;
            double t = dtau[k] / amu;
            double em1 = expm1(-t);
            J[k] += 0.5 * w[a] * (S[k] - (I - S[k]) * em1 / t);
            I = I + (I - S[k]) * em1;
        }
    }
    free(x);
    free(w);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------
 * Complex-step derivatives (for the adjoint tests).
 *
 * The formal solution above evaluated with complex chi and S.  For a function f analytic in a
 * parameter p, Im f(p + i h) / h equals df/dp up to rounding for tiny h (no difference of nearly
 * equal numbers), so one complex evaluation with an imaginary perturbation of one voxel's chi (or of
 * the source) gives the exact derivative of J and of the emergent intensities with respect to it.
 * Same lines, segments and integration as the real formal solution:
 *   dtau = chi_v l,  em1 = e^{-dtau} - 1,  D = S dtau - (I - S) em1,  I <- I + (I - S) em1,
 *   Ibar_v = |mu| / chi_v * sum D,  J = sum_d W_d Ibar(d).
 * e^{z} - 1 for complex z = x + iy is split as (e^x - 1) cos y - 2 sin^2(y/2) + i e^x sin y so that
 * the real part keeps the accuracy of expm1 for thin segments.
 * --------------------------------------------------------------------------------------------- */

typedef struct { double re, im; } cplx;

static cplx c_add(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static cplx c_sub(cplx a, cplx b) { cplx r = {a.re - b.re, a.im - b.im}; return r; }
static cplx c_mul(cplx a, cplx b)
{
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}
static cplx c_scale(cplx a, double s) { cplx r = {a.re * s, a.im * s}; return r; }
static cplx c_div(cplx a, cplx b)
{
    const double den = b.re * b.re + b.im * b.im;
    cplx r = {(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
    return r;
}
static cplx c_expm1(cplx z)
{
    const double s = sin(0.5 * z.im);
    cplx r = {expm1(z.re) * cos(z.im) - 2.0 * s * s, exp(z.re) * sin(z.im)};
    return r;
}

/* Complex formal solution: chi = chi_re + i chi_im, S = S_re + i S_im (any imaginary part may be
 * NULL = zero).  I_top is real; I_bot ([ny][nx], real, NULL = zero) is the light entering the bottom
 * plane, to which an upward line adds mu times slope ([ny][nx], complex, NULL = none: the
 * LTE-diffusion gradient dB/dtau, which depends on chi).  Outputs J ([V], real and imaginary parts) and, optionally, the emergent top intensities
 * of the upward directions Iem ([n_up][ny][nx], real and imaginary parts).  Single-threaded. */
int orc_fs_complex(int nx, int ny, int nz, int n_theta, int n_phi, const double *chi_re,
                   const double *chi_im, const double *S_re, const double *S_im, double I_top,
                   const double *I_bot, const double *slope_re, const double *slope_im,
                   double *J_re, double *J_im, double *Iem_re, double *Iem_im)
{
    Geom g;
    int rc = geom_init(&g, nx, ny, nz, n_theta, n_phi);
    if (rc) return rc;
    const long V = (long)nx * ny * nz;
    int ms = 0;
    for (int d = 0; d < g.n_dir; ++d) if (max_segments(&g, d) > ms) ms = max_segments(&g, d);
    double *fbuf = (double *)malloc(sizeof(double) * (ms + 2));
    int *seg_v = (int *)malloc(sizeof(int) * ms);
    double *seg_len = (double *)malloc(sizeof(double) * ms);
    cplx *Dsum = (cplx *)malloc(sizeof(cplx) * V);
    if (!fbuf || !seg_v || !seg_len || !Dsum) {
        free(fbuf); free(seg_v); free(seg_len); free(Dsum); geom_free(&g);
        return ORC_ENOMEM;
    }
    for (long v = 0; v < V; ++v) { J_re[v] = 0.0; J_im[v] = 0.0; }
    const int n_down = g.n_dir / 2;
    for (int d = 0; d < g.n_dir; ++d) {
        const double mu = g.mu[d];
        memset(Dsum, 0, sizeof(cplx) * V);
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                cplx In = {I_top, 0.0};
                for (int step = 0; step < nz; ++step) {
                    const int k = (mu < 0.0) ? nz - 1 - step : step;
                    const int ns = trace_layer(&g, d, i, j, k, fbuf, seg_v, seg_len);
                    if (mu > 0.0 && step == 0) {
                        In.re = I_bot ? I_bot[seg_v[0]] : 0.0;
                        In.im = 0.0;
                        if (slope_re) {   /* LTE diffusion: + mu dB/dtau (complex through chi) */
                            In.re += mu * slope_re[seg_v[0]];
                            In.im += slope_im ? mu * slope_im[seg_v[0]] : 0.0;
                        }
                    }
                    for (int s = 0; s < ns; ++s) {
                        const int v = seg_v[s];
                        const cplx chi = {chi_re[v], chi_im ? chi_im[v] : 0.0};
                        const cplx S = {S_re[v], S_im ? S_im[v] : 0.0};
                        const cplx dtau = c_scale(chi, seg_len[s]);
                        const cplx em1 = c_expm1(c_scale(dtau, -1.0));
                        const cplx IS = c_sub(In, S);
                        const cplx D = c_sub(c_mul(S, dtau), c_mul(IS, em1));
                        In = c_add(In, c_mul(IS, em1));
                        Dsum[v] = c_add(Dsum[v], D);
                    }
                }
                if (mu > 0.0 && Iem_re && Iem_im) {
                    const size_t o = (size_t)(d - n_down) * nx * ny + (size_t)j * nx + i;
                    Iem_re[o] = In.re;
                    Iem_im[o] = In.im;
                }
            }
        }
        const double amu = fabs(mu);
        for (long v = 0; v < V; ++v) {
            const cplx chi = {chi_re[v], chi_im ? chi_im[v] : 0.0};
            const cplx ib = c_scale(c_div(Dsum[v], chi), amu);
            J_re[v] += g.wt[d] * ib.re;
            J_im[v] += g.wt[d] * ib.im;
        }
    }
    free(fbuf); free(seg_v); free(seg_len); free(Dsum);
    geom_free(&g);
    return ORC_OK;
}
