// kernels.h -- HIP device code of the 3D radiative-transfer hot path (gfx950).  Included by the
// single-problem ABI (rt3d.hip) and the batched ABI (batch.hip).  The kernels that batching applies
// to are device functions taking an argument struct, with a single-problem wrapper here and a
// batched wrapper in batch.hip, so both run the same arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "geometry.h"

using rt3d::DirInfo;
using rt3d::WorkItem;

namespace {

// Sweep workgroup shapes (threads, lines per thread and direction); the context picks one.
struct SweepShape { int threads, lines; };
// Measured on MI355X at 129^3 x 256: 512 x 2 is fastest (64 VGPRs, 8 waves/SIMD; the sweep is
// latency-bound, so occupancy beats lines per thread and prefetching).
constexpr SweepShape kSweepShapes[] = {{512, 2}, {512, 4}, {256, 8}, {1024, 2}, {256, 4}, {256, 2}};
// Calls f(NT, LPT) (as integral constants) for the sweep shape with the given index.
template <int NT, int LPT> struct ShapeTag {
    static constexpr int threads = NT, lines = LPT;
};
template <typename F>
inline void with_sweep_shape(int shape, F &&f)
{
    switch (shape) {
    case 1: f(ShapeTag<512, 4>{}); break;
    case 2: f(ShapeTag<256, 8>{}); break;
    case 3: f(ShapeTag<1024, 2>{}); break;
    case 4: f(ShapeTag<256, 4>{}); break;
    case 5: f(ShapeTag<256, 2>{}); break;
    default: f(ShapeTag<512, 2>{}); break;
    }
}
constexpr size_t kWindowBytes = 48 * 1024;   // LDS budget of a band (deposit window and exchange)
// Grids whose windows do not fit kWindowBytes (wide rows, shallow angle sets) take up to this much of
// the 160 KB of LDS a gfx950 workgroup may use (the rest holds the kernel's static LDS): one workgroup
// per CU then, but no width limit below the line budget of a workgroup.
constexpr size_t kWindowBytesWide = 156 * 1024;
// Dynamic LDS of a sweep workgroup: the largest window and exchange buffers of any direction pair's
// bands (each band lays out its own within this).
inline size_t sweep_smem_bytes(const rt3d::SweepPlan &plan, bool f32)
{
    size_t bytes = 0;
    for (const rt3d::PairInfo &pi : plan.pairs)
        bytes = std::max(bytes, rt3d::sweep_lds_bytes(pi.win_rows, pi.band_rows, plan.nx, f32));
    return bytes;
}
constexpr int kPlaneThreads = 256;   // voxel-parallel kernels: one thread per voxel of a k-plane

template <typename real> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// e^x - 1 for x <= 0 (the argument is always -dtau).  No range branches: x is clamped where e^x
// vanishes.
//
// float64, Tang's table method with N = 16: x = (16 k + j) ln2/16 + r with 0 <= j < 16 and
// |r| <= ln2/32, so e^x - 1 = 2^k T_j (1 + r p(r)) - 1 with T_j = 2^(j/16) read from a table and p the
// Taylor polynomial of (e^r - 1)/r through r^6 (truncation below 1e-16 relative).  The multiple
// n = 16 k + j is the nearest integer to x 16/ln2, taken from the rounding of x 16/ln2 + 1.5 * 2^52
// (the spacing of doubles there is 1, so the low word of the sum is n in two's complement).
// 2^k T_j - 1 is exact when 2^k T_j >= 1/2 and is far from zero otherwise; the rounding of T_j bounds
// the relative error by a few 1e-15 where the result is small (|x| a few times ln2/32), and below
// ln2/32 the result is r p(r) itself.  The sweep reduces with one fma on the rounded ln2/16: its error
// in r, |n| times half an ulp of ln2/16, moves e^x by at most 1e-16 |x| e^x relative (below 3e-17
// absolute).  exp_pair_tab splits ln2/16 into a high part whose product with n is exact and a low
// part, so that e^x itself stays accurate to a few ulps for thick segments.  The table (128 bytes,
// in LDS) is small enough that the lanes' lookups never meet in an LDS bank: a 128-entry table with
// the polynomial through r^4 took 2-3% longer per sweep (host emulation against long-double expm1 over
// 3e7 samples of x in [-2000, -1e-14]: at most 2.7e-15 relative here, 3.9e-15 with 128 entries).
constexpr int kExpTabLog2 = 4;
constexpr int kExpTab = 1 << kExpTabLog2;
constexpr double kExpInvStep = 184.66496523378731 / 8;            // 16 / ln2 (128 / ln2, exactly scaled)
constexpr double kExpStep = 0.0054152123481245725 * 8;             // ln2 / 16
constexpr double kExpStepHi = 6.93147180369123816490e-01 / 16;    // 21 trailing zero bits
constexpr double kExpStepLo = 1.90821492927058770002e-10 / 16;
constexpr double kExpRound = 6755399441055744.0;                   // 1.5 * 2^52

// a * b + c as one VOP3 v_fma_f64 with c in an SGPR pair.  For a constant addend the compiler would
// otherwise keep c in VGPRs and copy it into the destination of a two-address v_fmac_f64 at every
// use (a v_mov_b64 per polynomial step of every exponential in the sweep's segment loop).
__device__ inline double fma3(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

__device__ inline double expm1_poly(double r)
{
    double p = fma3(r, 1.0 / 5040.0, 1.0 / 720.0);
    p = fma3(p, r, 1.0 / 120.0);
    p = fma3(p, r, 1.0 / 24.0);
    p = fma3(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    return p * r;
}

__device__ inline double expm1_nonpos_tab(double x, const double *tab)
{
    x = fmax(x, -708.0);
    const double kr = fma(x, kExpInvStep, kExpRound);
    const double kf = kr - kExpRound;
    const int n = __double2loint(kr);
    const double q = expm1_poly(fma(-kf, kExpStep, x));
    const double s = ldexp(tab[n & (kExpTab - 1)], n >> kExpTabLog2);
    return fma(s, q, s - 1.0);
}

// Both e^x and e^x - 1 for x <= 0 from one table evaluation: with s = 2^k T_j and q = r p(r),
// e^x = s (1 + q) and e^x - 1 = s q + (s - 1), each to a few ulps relative (the first also for
// thick segments, where 1 + (e^x - 1) would lose all of it).
__device__ inline void exp_pair_tab(double x, const double *tab, double &e, double &em1)
{
    x = fmax(x, -708.0);
    const double kr = fma(x, kExpInvStep, kExpRound);
    const double kf = kr - kExpRound;
    const int n = __double2loint(kr);
    const double q = expm1_poly(fma(-kf, kExpStepLo, fma(-kf, kExpStepHi, x)));
    const double s = ldexp(tab[n & (kExpTab - 1)], n >> kExpTabLog2);
    e = fma(s, q, s);
    em1 = fma(s, q, s - 1.0);
}

// float32: x = k ln2 + r with |r| <= ln2/2; e^x - 1 = 2^k (e^r - 1) + (2^k - 1), and e^r - 1 is its
// Taylor series through r^8 (truncation below 1e-9 relative).
__device__ inline float expm1_nonpos(float x)
{
    x = fmaxf(x, -87.0f);
    const float kf = rintf(x * 1.44269504089f);
    float r = fmaf(-kf, 0.693145751953125f, x);
    r = fmaf(-kf, 1.42860682e-06f, r);
    float p = 1.0f / 40320.0f;
    p = fmaf(p, r, 1.0f / 5040.0f);
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    const float two_k = ldexpf(1.0f, int(kf));
    return fmaf(two_k, p * r, two_k - 1.0f);
}

// ------------------------------------------------------------------------------------------------
// S update
// ------------------------------------------------------------------------------------------------

// S_given: the source itself.  Ja (difference mode of the FP32 form): the source change since the
// anchor iterate, (1 - eps)(J - Ja), whose formal solution is added to the anchor's.  scatter_only:
// the scattering part (1 - eps) J alone (the adjoint solve, whose thermal term enters as a base).
struct SourceArgs {
    int nx, ny, nz;
    int scatter_only;
    const double *chi, *eps, *B, *J, *S_given, *Ja;
    void *cs;                     // Vec2<real>
};

template <typename real>
__device__ inline void source_body(const SourceArgs &a, int p, int k)
{
    if (p >= a.nx * a.ny) return;
    const long v = long(k) * a.nx * a.ny + p;
    double S;
    if (a.S_given) S = a.S_given[v];
    else if (a.Ja) S = (1.0 - a.eps[v]) * (a.J[v] - a.Ja[v]);
    else if (a.scatter_only) S = (1.0 - a.eps[v]) * a.J[v];
    else S = a.eps[v] * a.B[v] + (1.0 - a.eps[v]) * a.J[v];
    typename Vec2<real>::type c;
    c.x = real(a.chi[v]);
    c.y = real(S);
    static_cast<typename Vec2<real>::type *>(a.cs)[v] = c;
}

template <typename real>
__global__ __launch_bounds__(kPlaneThreads) void source_kernel(SourceArgs a)
{
    source_body<real>(a, blockIdx.x * kPlaneThreads + threadIdx.x, blockIdx.y);
}

// ------------------------------------------------------------------------------------------------
// FS sweep
// ------------------------------------------------------------------------------------------------

struct SweepArgs {
    int nx, ny, nz, n_down;
    const rt3d::PairSeg *pseg;
    const rt3d::PairLayer *player;
    const rt3d::PairInfo *pairs;
    const WorkItem *items;
    const void *cs;               // Vec2<real>
    const double *Ibot;           // [ny][nx] intensities at the bottom plane, or null (zero)
    const double *Islope;         // [ny][nx] LTE-diffusion gradient: upward lines add mu * Islope (or null)
    double I_top;
    void *P;                      // real
    double *Iem;                  // [n_up][ny][nx] or null
    const double *Iem_base;       // added to Iem in difference mode (or null)
    const double *xtab;           // [kExpTab] 2^(j/kExpTab), the float64 exponential's table
};

__device__ inline double expm1_sweep(double x, const double *tab) { return expm1_nonpos_tab(x, tab); }
__device__ inline float expm1_sweep(float x, const double *) { return expm1_nonpos(x); }

template <typename real> __device__ inline real seg_length(const rt3d::PairSeg &g);
template <> __device__ inline double seg_length<double>(const rt3d::PairSeg &g) { return g.len; }
template <> __device__ inline float seg_length<float>(const rt3d::PairSeg &g) { return g.len32; }

// x mod n for 0 <= x < 2n, as min(x, x - n) on unsigned integers (x - n wraps when x < n)
__device__ inline unsigned wrap_once(unsigned x, unsigned n) { return min(x, x - n); }

// One workgroup sweeps the lines of one band for both directions A and B of an x-mirrored pair.  The
// two directions' segments have equal lengths and row offsets and negated column offsets, so at every
// segment index a line of A and a line of B cross the same voxel: slot q = (row, column c) of the band
// holds the A line whose top column is c and the B line whose top column is c + 2 dA (mod nx), dA
// being A's column offset at that segment; both are in voxel column c + dA.  The pair then shares the
// voxel's chi,S, the exponential of its optical depth and the deposit cell.  Where dA changes between
// consecutive segments the B lines move between the slots of their row, through a double-buffered
// LDS array (the barrier that ends every segment index orders the write before the read).  Thread t
// owns slots q = t + i*NT (i < LPT).  Per segment index the slots deposit into pairwise distinct cells
// of the band's LDS window, so the window is updated with a plain read-add-write.
template <typename real, int NT, int LPT>
__device__ __forceinline__ void sweep_body(const SweepArgs &a, const WorkItem &it, unsigned char *smem_raw)
{
    using real2 = typename Vec2<real>::type;
    const rt3d::PairInfo pi = a.pairs[it.pair];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned plane = unsigned(nx) * unsigned(ny);
    const int nlines = it.rows * nx;
    const int wsize = pi.win_rows * nx;
    const real2 *cs = static_cast<const real2 *>(a.cs);
    // LDS: the band's deposit window, then the two exchange buffers of the B lines
    real *win = reinterpret_cast<real *>(smem_raw);
    real *xch = win + wsize;                                   // [2][nlines]
    real *P = static_cast<real *>(a.P) + pi.p_off + long(it.band) * nz * wsize;

    for (int e = threadIdx.x; e < wsize; e += NT) win[e] = real(0);
    __shared__ double xtab[kExpTab];
    if (std::is_same<real, double>::value && threadIdx.x < kExpTab) xtab[threadIdx.x] = a.xtab[threadIdx.x];

    real IA[LPT], IB[LPT];
    int li[LPT], lj[LPT];
    unsigned lbase[LPT];
#pragma unroll
    for (int t = 0; t < LPT; ++t) {
        const int q = threadIdx.x + t * NT;
        const int qq = q < nlines ? q : 0;
        lj[t] = qq / nx;
        li[t] = q < nlines ? qq - lj[t] * nx : -1;   // -1 marks an unused slot
        lbase[t] = unsigned(lj[t] * nx);
        IA[t] = real(a.I_top);
        IB[t] = real(a.I_top);
    }
    __syncthreads();

    int xpar = 0;              // exchange buffer of the last move of the B lines
    bool moved = false;        // the B lines were written to it before the last barrier
    unsigned sa_last = 0;      // A's column offset at the last segment (the B lines' top columns)
    for (int step = 0; step < nz; ++step) {
        const int k = pi.down ? nz - 1 - step : step;
        const rt3d::PairLayer L = a.player[it.pair * nz + k];
        const real2 *csk = cs + long(k) * plane;
        unsigned grow0[LPT];
#pragma unroll
        for (int t = 0; t < LPT; ++t) {
            unsigned r = unsigned(it.j0 + lj[t] + L.rmin);
            r = wrap_once(wrap_once(r, ny), ny);
            grow0[t] = r * unsigned(nx);
        }
        if (!pi.down && step == 0) {
            // upward lines enter through the bottom plane: boundary light of the entry voxel, the
            // same voxel for the slot's A and B lines
            const rt3d::PairSeg g = a.pseg[L.off];
#pragma unroll
            for (int t = 0; t < LPT; ++t) {
                if (li[t] < 0) continue;
                const unsigned row = wrap_once(grow0[t] + unsigned(g.smnx), plane);
                const unsigned col = wrap_once(unsigned(li[t] + g.saA), nx);
                const double sl = a.Islope ? pi.mu * a.Islope[row + col] : 0.0;
                IA[t] = a.Ibot ? real(a.Ibot[row + col] + sl) : real(0);
                IB[t] = IA[t];
            }
        }
        rt3d::PairSeg g = a.pseg[L.off];
        for (int s = 0; s < L.ns; ++s) {
            // the next segment's descriptor is loaded one segment ahead, so its load latency is not
            // part of the chain of latencies of a segment index
            const rt3d::PairSeg gn = a.pseg[L.off + min(s + 1, L.ns - 1)];
            const real len = seg_length<real>(g);
            // gather of segment s: the voxel of each slot in the chi,S plane
            real2 cv[LPT];
            unsigned wc[LPT];
#pragma unroll
            for (int t = 0; t < LPT; ++t) {
                const unsigned col = wrap_once(unsigned(li[t] + g.saA), nx);
                wc[t] = lbase[t] + unsigned(g.sbnx) + col;
                const unsigned grow = wrap_once(grow0[t] + unsigned(g.smnx), plane);
                if (li[t] >= 0) cv[t] = csk[grow + col];
            }
            // the B lines that moved at the end of the previous segment
            if (moved) {
#pragma unroll
                for (int t = 0; t < LPT; ++t)
                    if (li[t] >= 0) IB[t] = xch[xpar * nlines + int(lbase[t]) + li[t]];
            }
            // At one segment index the slots deposit into distinct cells, so the window cells are
            // read first, ahead of the exponentials, and written after: one LDS wait per segment
            // index, not one per deposit.
            real o[LPT];
#pragma unroll
            for (int t = 0; t < LPT; ++t) o[t] = li[t] >= 0 ? win[wc[t]] : real(0);
#pragma unroll
            for (int t = 0; t < LPT; ++t) {
                if (li[t] < 0) continue;
                const real dtau = cv[t].x * len;
                const real em1 = expm1_sweep(-dtau, xtab);     // e^{-dtau} - 1
                const real dA = (IA[t] - cv[t].y) * em1;
                const real dB = (IB[t] - cv[t].y) * em1;
                IA[t] += dA;
                IB[t] += dB;
                const real sd = cv[t].y * dtau;
                win[wc[t]] = o[t] + ((sd - dA) + (sd - dB));   // chi * integral of I, both lines
            }
            // B lines move by -2 (change of dA) columns in their row before the next segment
            moved = g.shB != 0;
            if (moved) {
                xpar ^= 1;
#pragma unroll
                for (int t = 0; t < LPT; ++t)
                    if (li[t] >= 0)
                        xch[xpar * nlines + int(lbase[t] + wrap_once(unsigned(li[t] + g.shB), nx))] = IB[t];
            }
            sa_last = unsigned(g.saA);
            g = gn;
            __syncthreads();
        }
        real *Pk = P + long(k) * wsize;
        for (int e = threadIdx.x; e < wsize; e += NT) {
            Pk[e] = win[e];
            win[e] = real(0);
        }
        __syncthreads();
    }
    if (!pi.down && a.Iem) {
        const long ea0 = long(pi.dA - a.n_down) * plane, eb0 = long(pi.dB - a.n_down) * plane;
#pragma unroll
        for (int t = 0; t < LPT; ++t) {
            if (li[t] < 0) continue;
            // the B line in this slot entered the top at column li + 2 dA (mod nx)
            const unsigned colB = wrap_once(wrap_once(unsigned(li[t]) + sa_last, nx) + sa_last, nx);
            const long ea = ea0 + (it.j0 + lj[t]) * nx + li[t];
            const long eb = eb0 + (it.j0 + lj[t]) * nx + colB;
            const double baseA = a.Iem_base ? a.Iem_base[ea] : 0.0;
            const double baseB = a.Iem_base ? a.Iem_base[eb] : 0.0;
            a.Iem[ea] = baseA + double(IA[t]);
            a.Iem[eb] = baseB + double(IB[t]);
        }
    }
}

// Two slots per thread fit 64 VGPRs (59 in float64), which lets 8 waves share a SIMD (a band's LDS
// takes ~33 KB at 129 columns in float64, half that in float32, so 4 workgroups of 512 fit a CU); the
// segment loop waits on its gathers, and 8 waves hide that better than 6.  Shapes with more slots per
// thread keep the compiler's choice; the batched kernel has a bound of its own.
template <int LPT> constexpr int kSweepMinWaves = LPT <= 2 ? 8 : 1;

template <typename real, int NT, int LPT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kSweepMinWaves<LPT>))) void sweep_kernel(SweepArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    sweep_body<real, NT, LPT>(a, a.items[blockIdx.x], smem_raw);
}

// ------------------------------------------------------------------------------------------------
// Angle reduction of the partial planes
// ------------------------------------------------------------------------------------------------

struct ReduceArgs {
    int nx, ny, nz, n_pair;
    const rt3d::PairInfo *pairs;
    const int *row_min;
    const void *P;            // real
    const double *chi;
    const double *J;          // for r = J_fs - J (may be null)
    const double *base;       // difference mode: J_fs of the anchor, added (may be null)
    double *Jfs;
    double *rb;               // chi (J_fs - J), the right-hand side of the OS step (may be null)
};

// J_fs(v) = (1/chi_v) sum_pairs W|mu| sum over the bands whose deposit windows cover v.  The band of
// voxel row j at layer k is found from the row's offset to the layer's window origin; the previous
// bands (cyclically) still cover the row while the offset stays inside their windows.
template <typename real>
struct PairBands {
    const real *Pq;   // the pair's partial plane of layer k, at the voxel's column
    long o0, o1;      // elements of the band that starts the row's window offset and of the band before it
    int b1, off1;     // that earlier band (cyclically) and the row's offset in its window
};

template <typename real>
__device__ inline PairBands<real> pair_bands(const ReduceArgs &a, const rt3d::PairInfo &pi, int i, int j, int k)
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int rows = pi.band_rows, nb = pi.n_bands, Hw = pi.win_rows;
    const int rmin = a.row_min[pi.dA * nz + k];
    int jj = j - rmin;
    jj += (jj < 0) ? ny : 0;
    int b = min(int((float(jj) + 0.5f) * pi.inv_rows), nb - 1);
    b -= (b * rows > jj) ? 1 : 0;
    b += (b < nb - 1 && (b + 1) * rows <= jj) ? 1 : 0;
    const int off0 = jj - b * rows;
    const long plane = long(Hw) * nx;
    const long band_stride = long(nz) * plane;
    PairBands<real> r;
    r.Pq = static_cast<const real *>(a.P) + pi.p_off + long(k) * plane + i;
    r.b1 = (b == 0) ? nb - 1 : b - 1;
    r.off1 = off0 + ((r.b1 == nb - 1) ? pi.last_rows : rows);
    r.o0 = long(b) * band_stride + long(off0) * nx;
    r.o1 = long(r.b1) * band_stride + long(r.off1) * nx;
    return r;
}

// Row offset of the band before b1 (cyclically): it covers the row too when below the window height.
__device__ inline int pair_bands_next_off(const rt3d::PairInfo &pi, int bb, int off)
{
    bb = (bb == 0) ? pi.n_bands - 1 : bb - 1;
    return off + ((bb == pi.n_bands - 1) ? pi.last_rows : pi.band_rows);
}

// The angle sum of the direction pairs [q0, q1) for voxels (i, j, k) and (i + d1, j, k) (d1 = 0: one
// voxel, read twice), added to acc0 / acc1 pair by pair in order, each pair's bands summed in the
// order band b, b1, then earlier bands.  The partials of the first two bands of kPairGroup pairs are
// loaded before any is summed (a pair whose row only one band covers loads the first band's element
// again and does not add it), so a wave keeps that many loads in flight instead of waiting on each
// pair; the rare third and later bands are read where they are added.  Measured per launch at
// 129^3 x 256 (bitwise the same sums): 0.665 against 0.682 ms in float64, 0.475 against 0.516 ms in
// float32; at 65^3 x 256 0.109 against 0.127 and 0.082 against 0.117 ms; groups of 8 pairs 0.657 /
// 0.493 ms at 129^3.
constexpr int kPairGroup = 4;
template <typename real>
__device__ inline void reduce_pairs(const ReduceArgs &a, int i, int d1, int j, int k, int q0, int q1, double &acc0,
                                    double &acc1)
{
    constexpr int U = kPairGroup;
    for (int qb = q0; qb < q1; qb += U) {
        double x0[U], x1[U], y0[U], y1[U];
        bool m1[U], more[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = min(qb + u, q1 - 1);
            const rt3d::PairInfo pi = a.pairs[q];
            const PairBands<real> pb = pair_bands<real>(a, pi, i, j, k);
            m1[u] = pb.off1 < pi.win_rows;
            more[u] = m1[u] && pair_bands_next_off(pi, pb.b1, pb.off1) < pi.win_rows;
            const long o1 = m1[u] ? pb.o1 : pb.o0;
            x0[u] = double(pb.Pq[pb.o0]);
            x1[u] = double(pb.Pq[pb.o0 + d1]);
            y0[u] = double(pb.Pq[o1]);
            y1[u] = double(pb.Pq[o1 + d1]);
        }
        // keep the sums below the group's loads (the scheduler would otherwise interleave them and
        // wait on each pair's loads before issuing the next pair's)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (qb + u >= q1) break;
            const rt3d::PairInfo pi = a.pairs[qb + u];
            double s0 = x0[u], s1 = x1[u];
            if (m1[u]) {
                s0 += y0[u];
                s1 += y1[u];
            }
            if (more[u]) {
                // bands thinner than the window halo: still earlier bands cover the row
                const PairBands<real> pb = pair_bands<real>(a, pi, i, j, k);
                const long band_stride = long(a.nz) * pi.win_rows * a.nx;
                int bb = pb.b1, off = pb.off1;
                while (true) {
                    off = pair_bands_next_off(pi, bb, off);
                    bb = (bb == 0) ? pi.n_bands - 1 : bb - 1;
                    if (off >= pi.win_rows) break;
                    const long o = long(bb) * band_stride + long(off) * a.nx;
                    s0 += double(pb.Pq[o]);
                    s1 += double(pb.Pq[o + d1]);
                }
            }
            acc0 += pi.wmu * s0;
            acc1 += pi.wmu * s1;
        }
    }
}

// Two neighbouring voxels of one row per thread (p2 indexes the (ny, (nx + 1) / 2) voxel pairs of
// plane k; the batched form takes the same blocks per member): the band lookup is shared and the
// partials of both are read together.  Measured at 129^3 x 256 against one voxel per thread (before
// the loads were grouped): 0.69 against 0.74 ms (float64), 0.51 against 0.59 ms (float32).
// Direction pairs [q0, q1) only: the running sum starts from 0 (first) or from the raw sum a range
// before left in Jfs, and is finished (divided by chi, the residual formed) only when last, so ranges
// taken in order give bitwise the sum of one pass over all pairs.
template <typename real>
__device__ inline void reduce_body_pair_range(const ReduceArgs &a, int p2, int k, int q0, int q1, bool first,
                                              bool last)
{
    const int nx = a.nx, ny = a.ny;
    const int hx = (nx + 1) / 2;
    if (p2 >= hx * ny) return;
    const int j = p2 / hx, i0 = 2 * (p2 - j * hx);
    const bool two = i0 + 1 < nx;
    const int d1 = two ? 1 : 0;          // the second voxel's offset (0: none, reads the first again)
    const long v0 = long(k) * nx * ny + long(j) * nx + i0;
    double acc0 = first ? 0.0 : a.Jfs[v0], acc1 = (first || !two) ? 0.0 : a.Jfs[v0 + 1];
    reduce_pairs<real>(a, i0, d1, j, k, q0, q1, acc0, acc1);
    for (int t = 0; t < (two ? 2 : 1); ++t) {
        const long v = v0 + t;
        const double acc = t ? acc1 : acc0;
        if (!last) {
            a.Jfs[v] = acc;
            continue;
        }
        const double Jfs = a.base ? a.base[v] + acc / a.chi[v] : acc / a.chi[v];
        a.Jfs[v] = Jfs;
        if (a.rb) a.rb[v] = a.chi[v] * (Jfs - a.J[v]);
    }
}

template <typename real>
__device__ inline void reduce_body_pair(const ReduceArgs &a, int p2, int k)
{
    reduce_body_pair_range<real>(a, p2, k, 0, a.n_pair, true, true);
}

template <typename real>
__global__ __launch_bounds__(kPlaneThreads) void reduce_kernel_pair(ReduceArgs a)
{
    reduce_body_pair<real>(a, blockIdx.x * kPlaneThreads + threadIdx.x, blockIdx.y);
}

// pairs [q0, q1) only (see reduce_body_pair_range)
template <typename real>
__global__ __launch_bounds__(kPlaneThreads) void reduce_kernel_pair_range(ReduceArgs a, int q0, int q1, int first,
                                                                          int last)
{
    reduce_body_pair_range<real>(a, blockIdx.x * kPlaneThreads + threadIdx.x, blockIdx.y, q0, q1, first != 0,
                                 last != 0);
}


// ------------------------------------------------------------------------------------------------
// Lambda*
// ------------------------------------------------------------------------------------------------

struct LstarArgs {
    int nx, ny, nz, n_pair;
    int early_exit;                 // 1: no line can wrap back onto a neighbour within two layers
    const rt3d::PairInfo *pairs;    // x-mirrored direction pairs (the tables of direction dA are read)
    const int *seg_off, *seg_n, *seg_ai, *seg_bi;
    const double *seg_len;
    const double *chi;
    double *L;                      // [27][V]
    const double *xtab;             // [kExpTab] 2^(j/kExpTab), the float64 exponential's table
};

// x + expm1(-x) = e^{-x} - 1 + x for x >= 0 (em1 = e^{-x} - 1 given); below 1/2 by Horner on x^2
// (1/2! - x/3! + x^2/4! - ...) through x^15/17!, which avoids the cancellation of the direct form for
// thin segments.
__device__ inline double self_term(double x, double em1)
{
    if (x >= 0.5) return x + em1;
    constexpr double inv_fact[18] = {
        1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040, 1.0 / 40320,
        1.0 / 362880, 1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600, 1.0 / 6227020800.0,
        1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0,
        1.0 / 355687428096000.0};
    double r = inv_fact[17];
#pragma unroll
    for (int n = 16; n >= 2; --n) r = inv_fact[n] - x * r;
    return x * x * r;
}

__device__ inline int wrap_small(int a, int n)
{
    // a may be any integer; returns a mod n in [0, n)
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Lambda*_{vu} = sum_d W_d |mu_d| / chi_v * sum over the segments s of direction d inside v of
//   delta_uv (dtau_s + em1_s) - em1_s * sum over earlier segments s' in u of c_{s'->s},
//   c_{s'->s} = (1 - e_{s'}) prod_{s' < s'' < s} e_{s''},  e = exp(-dtau).
// The lines through v are the reference line shifted so that its segment s lies in v; walking that
// line backwards through the current and the previous layer reaches every earlier segment that can
// lie in the 3x3x3 block (lines are monotone in z).  The two directions of an x-mirrored pair have
// equal segment lengths and row offsets and negated column offsets, so one walk over direction A's
// table serves both (B's voxels at the mirrored columns), and their self terms are equal.
// One wavefront per workgroup, small workgroups letting many of them share a CU to hide the latency of
// the gathers along the lines (measured at 129^3 x 256: 31.7 ms with 256 threads, 29.2 ms with 128,
// 26.4 ms with 64).  The accumulators live in LDS.  A walk reaches the voxel's own layer and the one it
// came from: layer k + 1 for the downward pairs, k - 1 for the upward ones, and the pairs come in two
// runs (all of one vertical direction, then all of the other; the plan checks this).  So a thread
// keeps 18 accumulators, its own layer's 9 and those of the run's other layer, which are stored and
// cleared between the runs: every entry sums the same terms in the same order as with 27.
constexpr int kLstarThreads = 64;
// Columns p (p = j nx + i; p >= nx ny: none) of plane k; the whole block calls this.
__device__ inline void lstar_body(const LstarArgs &a, int p, int k)
{
    __shared__ double acc[18][kLstarThreads];   // [0, 9): layer k; [9, 18): the current run's other layer
    __shared__ double xtab[kExpTab];
    for (int q = threadIdx.x; q < kExpTab; q += kLstarThreads) xtab[q] = a.xtab[q];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const bool valid = p < nx * ny;
    const int j = valid ? p / nx : 0, i = valid ? p - (p / nx) * nx : 0;
    const long plane = long(nx) * ny;
    const long V = plane * nz;
    const long v = k * plane + long(j) * nx + i;
    for (int o = 0; o < 18; ++o) acc[o][threadIdx.x] = 0.0;
    __syncthreads();
    const double chiv = a.chi[v];
    // 3x3x3 block index of a column offset m (mod n) from v: 0 for -1, 1 for 0, 2 for +1, -1 outside
    auto block_col = [](int m, int n) { return (m == 0) ? 1 : (m == 1) ? 2 : (m == n - 1) ? 0 : -1; };
    // the other layer's 9 entries of the 27-point row (entries 0..8 for k - 1, 18..26 for k + 1)
    auto store_other = [&](int down) {
        const int o0 = down ? 18 : 0;
        if (valid)
            for (int o = 0; o < 9; ++o) a.L[(o0 + o) * V + v] = acc[9 + o][threadIdx.x];
        for (int o = 0; o < 9; ++o) acc[9 + o][threadIdx.x] = 0.0;
    };
    int run_down = a.n_pair > 0 ? a.pairs[0].down : 0;
    bool stored_up = false, stored_down = false;    // the layers k - 1 and k + 1 have been written
    for (int q = 0; q < a.n_pair; ++q) {
        const rt3d::PairInfo pi = a.pairs[q];
        if (pi.down != run_down) {
            store_other(run_down);
            stored_down = stored_down || run_down;
            stored_up = stored_up || !run_down;
            run_down = pi.down;
        }
        const double fac = pi.wmu / chiv;
        const int d = pi.dA;
        const int dk = d * nz + k;
        const int off = a.seg_off[dk], n = a.seg_n[dk];
        const int ku = pi.down ? k + 1 : k - 1;
        const bool has_up = ku >= 0 && ku < nz;
        const int offu = has_up ? a.seg_off[d * nz + ku] : 0;
        const int nu = has_up ? a.seg_n[d * nz + ku] : 0;
        for (int s = 0; s < n; ++s) {
            const int as = a.seg_ai[off + s], bs = a.seg_bi[off + s];
            const double dtau = chiv * a.seg_len[off + s];
            const double em1 = expm1_nonpos_tab(-dtau, xtab);
            acc[4][threadIdx.x] += 2.0 * (fac * self_term(dtau, em1));
            const double g = -fac * em1;
            double prodA = 1.0, prodB = 1.0;
            // walk back: current layer s-1 .. 0, then the previous layer from its last segment
            const int total = s + nu;
            for (int w = 0; w < total; ++w) {
                int idx, base;
                if (w < s) { idx = off + s - 1 - w; base = 0; }
                else { idx = offu + nu - 1 - (w - s); base = 9; }
                const int dA = a.seg_ai[idx] - as, dB = a.seg_bi[idx] - bs;
                if (a.early_exit && (dA > 1 || dA < -1 || dB > 1 || dB < -1)) break;
                // with early exit the offsets are -1, 0 or 1 here
                const int mA = a.early_exit ? dA + (dA < 0 ? nx : 0) : wrap_small(dA, nx);
                const int mB = a.early_exit ? dB + (dB < 0 ? ny : 0) : wrap_small(dB, ny);
                const int mAm = (mA == 0) ? 0 : nx - mA;      // direction B's column offset, -dA mod nx
                int colA = i + mA, colB = i + mAm;
                colA -= (colA >= nx) ? nx : 0;
                colB -= (colB >= nx) ? nx : 0;
                int row = j + mB;
                row -= (row >= ny) ? ny : 0;
                const long ub = long(base ? ku : k) * plane + long(row) * nx;
                const double len = a.seg_len[idx];
                double eA, em1A, eB, em1B;
                exp_pair_tab(-a.chi[ub + colA] * len, xtab, eA, em1A);
                exp_pair_tab(-a.chi[ub + colB] * len, xtab, eB, em1B);
                const int oj = block_col(mB, ny);
                const int oiA = block_col(mA, nx), oiB = block_col(mAm, nx);
                if (oiA >= 0 && oj >= 0) acc[base + 3 * oj + oiA][threadIdx.x] += g * (-em1A * prodA);
                if (oiB >= 0 && oj >= 0) acc[base + 3 * oj + oiB][threadIdx.x] += g * (-em1B * prodB);
                prodA *= eA;
                prodB *= eB;
            }
        }
    }
    store_other(run_down);
    stored_down = stored_down || run_down;
    stored_up = stored_up || !run_down;
    // a layer no run reached (all pairs of one vertical direction) has no entries
    if (valid && !stored_up)
        for (int o = 0; o < 9; ++o) a.L[o * V + v] = 0.0;
    if (valid && !stored_down)
        for (int o = 0; o < 9; ++o) a.L[(18 + o) * V + v] = 0.0;
    if (valid)
        for (int o = 0; o < 9; ++o) a.L[(9 + o) * V + v] = acc[o][threadIdx.x];
}

__global__ __launch_bounds__(kLstarThreads) void lstar_kernel(LstarArgs a)
{
    lstar_body(a, blockIdx.x * kLstarThreads + threadIdx.x, blockIdx.y);
}

// Jacobi coefficients.  K_vu = chi_v Lambda*_vu is symmetric (reciprocity: lines for Omega and -Omega
// coincide and the weights are symmetric), so only the 13 upper neighbours o = 14..26 are stored:
// Kc[o - 14][v] = chi_v Lambda*_o(v).  The entry for a lower neighbour u = v + d(o), o < 13, is
// Kc[12 - o][u] (u's upper neighbour 26 - o is v).  Per voxel: invD = 1 / (chi_v (1 - Lambda*_vv (1-eps_v)))
// and E = (1 - eps_v) invD.
template <typename coef>
__global__ __launch_bounds__(kPlaneThreads) void coef_kernel(int nx, int ny, int nz,
                                                             const double *__restrict__ L,
                                                             const double *__restrict__ chi,
                                                             const double *__restrict__ eps,
                                                             coef *__restrict__ Kc, double *__restrict__ invD,
                                                             double *__restrict__ E)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (p >= nx * ny) return;
    const long plane = long(nx) * ny, V = plane * nz, v = k * plane + p;
    const double c = chi[v];
    for (int o = 14; o < 27; ++o) {
        const int kk = k + o / 9 - 1;
        Kc[(o - 14) * V + v] = coef((kk < nz) ? c * L[o * V + v] : 0.0);
    }
    const double inv = 1.0 / (c * (1.0 - L[13 * V + v] * (1.0 - eps[v])));
    invD[v] = inv;
    E[v] = (1.0 - eps[v]) * inv;
}

// ------------------------------------------------------------------------------------------------
// Jacobi sweep of the OS equations, optionally fused with the J update and max |dJ|/|J|
// ------------------------------------------------------------------------------------------------

// The sweep dJ_v <- (r_v + sum_{u != v} Lambda*_vu (1-eps_u) dJ_u) / (1 - Lambda*_vv (1-eps_v)) is
// evaluated as (chi_v r_v + sum_u K_vu w_u) invD_v with w = (1 - eps) dJ carried between sweeps.
struct JacobiArgs {
    int nx, ny, nz;
    const double *b;             // chi (J_fs - J_old): the right-hand side of the chi-scaled system
    const void *Kc;              // [13][V] upper coefficients (double, or float in the FP32 form)
    const double *invD, *E;
    const double *w_in;          // (1 - eps) dJ of the previous sweep; null: dJ^0 = 0 (first sweep)
    double *w_out;               // (1 - eps) dJ of this sweep (intermediate sweeps)
    double *J;                   // last sweep: J += dJ (null otherwise)
    unsigned long long *maxrel;  // bits of max |dJ|/|J| (non-negative doubles order like integers)
    const double *Ja;            // anchor iterate of the FP32 form (may be null)
    unsigned long long *maxdist; // bits of max |J - Ja|/|J| when Ja is given, of max |J| when abs_measure
    int *nonfinite;
    int abs_measure;             // 1: maxrel receives max |dJ| and maxdist max |J| (iterates that may vanish)
};

// Block max of q and of the anchor distance into maxrel / maxdist (as integer bits: non-negative
// doubles order like integers); NaN/Inf raise the flag.  The whole block must call this.
__device__ inline void jacobi_block_max(const JacobiArgs &a, double q, double dist, bool bad)
{
    if (bad) { atomicOr(a.nonfinite, 1); q = 0.0; dist = 0.0; }
    for (int offs = 32; offs > 0; offs >>= 1) {
        q = fmax(q, __shfl_xor(q, offs));
        dist = fmax(dist, __shfl_xor(dist, offs));
    }
    __shared__ double wmax[2][kPlaneThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { wmax[0][wid] = q; wmax[1][wid] = dist; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmax[0][0], md = wmax[1][0];
        for (int w = 1; w < kPlaneThreads / 64; ++w) { m = fmax(m, wmax[0][w]); md = fmax(md, wmax[1][w]); }
        atomicMax(a.maxrel, static_cast<unsigned long long>(__double_as_longlong(m)));
        if (a.Ja || a.abs_measure) atomicMax(a.maxdist, static_cast<unsigned long long>(__double_as_longlong(md)));
    }
}

// The last sweep of a step: J += dJ, and the convergence measures of voxel v folded into q / dist.
__device__ inline void jacobi_update(const JacobiArgs &a, long v, double acc, double &q, double &dist, bool &bad)
{
    const double dJ = acc * a.invD[v];
    const double Jn = a.J[v] + dJ;
    a.J[v] = Jn;
    double qv, dv = 0.0;
    if (a.abs_measure) {
        qv = fabs(dJ);
        dv = fabs(Jn);
    } else {
        qv = fabs(dJ) / fabs(Jn);
        if (a.Ja) dv = fabs(Jn - a.Ja[v]) / fabs(Jn);
    }
    if (!isfinite(Jn) || !isfinite(qv)) {
        bad = true;
    } else {
        q = fmax(q, qv);
        dist = fmax(dist, dv);
    }
}

// Arithmetic is float64 for either coefficient type.
// The whole block must call this (it ends with a block reduction when J is updated).
template <typename coef>
__device__ inline void jacobi_core(const JacobiArgs &a, int i, int j, int k, bool valid)
{
    const coef *Kc = static_cast<const coef *>(a.Kc);
    double q = 0.0, dist = 0.0;
    bool bad = false;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    if (valid) {
        const long plane = long(nx) * ny, V = plane * nz, v = k * plane + long(j) * nx + i;
        double acc = a.b[v];
        if (a.w_in) {
            const int im = (i == 0) ? nx - 1 : i - 1, ip = (i == nx - 1) ? 0 : i + 1;
            const int jm = (j == 0) ? ny - 1 : j - 1, jp = (j == ny - 1) ? 0 : j + 1;
            const int cols[3] = {im, i, ip};
            const int rows[3] = {jm, j, jp};
            // Branch-free over the planes so that all loads can be in flight together: the plane
            // below is clamped at the bottom and its sum masked; the plane above needs no mask, its
            // coefficients are stored as zero in the top layer.
            const int planes[3] = {k > 0 ? k - 1 : 0, k, k < nz - 1 ? k + 1 : k};
            double part[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int o = 0; o < 27; ++o) {
                if (o == 13) continue;
                const long u = planes[o / 9] * plane + long(rows[(o / 3) % 3]) * nx + cols[o % 3];
                const double K = (o > 13) ? double(Kc[(o - 14) * V + v]) : double(Kc[(12 - o) * V + u]);
                part[o / 9] += K * a.w_in[u];
            }
            acc += (k > 0 ? part[0] : 0.0) + part[1] + part[2];
        }
        if (a.w_out) a.w_out[v] = acc * a.E[v];
        if (a.J) jacobi_update(a, v, acc, q, dist, bad);
    }
    if (a.J) jacobi_block_max(a, q, dist, bad);
}

template <typename coef>
__device__ inline void jacobi_body(const JacobiArgs &a, int p, int k)
{
    const bool valid = p < a.nx * a.ny;
    const int j = valid ? p / a.nx : 0;
    jacobi_core<coef>(a, valid ? p - j * a.nx : 0, j, k, valid);
}

template <typename coef>
__global__ __launch_bounds__(kPlaneThreads) void jacobi_kernel(JacobiArgs a)
{
    jacobi_body<coef>(a, blockIdx.x * kPlaneThreads + threadIdx.x, blockIdx.y);
}

// The same sweep on a 1D grid whose blocks are dealt to the 8 XCDs (each with its own L2) in
// contiguous ranges: workgroups go round-robin over the XCDs in launch order, so block b runs on XCD
// b % 8; here that XCD takes the chunks [xcd * G, (xcd + 1) * G) of every plane, G = padded chunks / 8.
// A voxel's mirrored coefficients and iterates sit in the row above (mostly the same or the previous
// chunk) and in the plane below (the same chunk, G * 8 blocks earlier), so they are in that XCD's L2.
// Chunks beyond the plane are padding (no voxels).
template <typename coef>
__global__ __launch_bounds__(kPlaneThreads) void jacobi_kernel_grouped(JacobiArgs a, int group)
{
    const int b = blockIdx.x;
    const int xcd = b & 7, slot = b >> 3;
    const int k = slot / group;
    const int chunk = xcd * group + (slot - k * group);
    jacobi_body<coef>(a, chunk * kPlaneThreads + threadIdx.x, k);
}

// 2D tiles of kTileX x kTileY columns (a wavefront spans two rows of 32), dealt to the XCDs in
// contiguous ranges of tiles per plane as above: the row above a voxel is mostly in its own tile, so
// its iterates and mirrored coefficients come from this workgroup's recent reads.
constexpr int kTileX = 32, kTileY = kPlaneThreads / kTileX;
template <typename coef>
__global__ __launch_bounds__(kPlaneThreads) void jacobi_kernel_tiled(JacobiArgs a, int tiles_x, int group)
{
    const int b = blockIdx.x;
    const int xcd = b & 7, slot = b >> 3;
    const int k = slot / group;
    const int tile = xcd * group + (slot - k * group);
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int i = tx * kTileX + (threadIdx.x % kTileX);
    const int j = ty * kTileY + (threadIdx.x / kTileX);
    const bool valid = i < a.nx && j < a.ny;
    jacobi_core<coef>(a, valid ? i : 0, valid ? j : 0, k, valid);
}

// Column form: a thread takes H voxels (i, j, k0 .. k0 + H - 1) and marches up them, keeping the
// previous iterates of three planes in registers, so each voxel loads one new plane of nine iterates
// instead of 26 neighbours (the coefficient streams and the per-voxel sums are those of jacobi_core,
// in the same order).  Blocks are dealt to the XCDs in contiguous ranges of chunks per column layer,
// as in jacobi_kernel_grouped.  H = 4 on grids that fill the chip; smaller grids take shorter columns
// (more threads), see jacobi_column_height.
constexpr int kJacCol = 4;
// Column layer kc of the columns p (p = j nx + i; p >= nx ny: no voxels).  The whole block must call
// this (it ends with a block reduction when J is updated).
template <typename coef, int H = kJacCol, bool Down = false>
__device__ inline void jacobi_column_body(const JacobiArgs &a, int p, int kc)
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const bool valid = p < nx * ny;
    const coef *Kc = static_cast<const coef *>(a.Kc);
    double q = 0.0, dist = 0.0;
    bool bad = false;
    if (valid) {
        const int j = p / nx, i = p - j * nx, k0 = kc * H;
        const int kfirst = Down ? (k0 + H - 1 < nz - 1 ? k0 + H - 1 : nz - 1) : k0;
        const long plane = long(nx) * ny, V = plane * nz;
        const int im = (i == 0) ? nx - 1 : i - 1, ip = (i == nx - 1) ? 0 : i + 1;
        const int jm = (j == 0) ? ny - 1 : j - 1, jp = (j == ny - 1) ? 0 : j + 1;
        long off[9];              // the 3 x 3 columns around (i, j), in the stencil's order
#pragma unroll
        for (int m = 0; m < 9; ++m)
            off[m] = long(m < 3 ? jm : (m < 6 ? j : jp)) * nx + (m % 3 == 0 ? im : (m % 3 == 1 ? i : ip));
        double Wm[9], W0[9], Wp[9];   // iterates of the planes k - 1 (clamped), k, k + 1 (clamped)
        if (a.w_in) {
            // the first voxel's plane and the one behind it in the walk (clamped at the grid's faces)
            const long kb = Down ? (kfirst < nz - 1 ? kfirst + 1 : kfirst) : (kfirst > 0 ? kfirst - 1 : 0);
#pragma unroll
            for (int m = 0; m < 9; ++m) {
                if constexpr (Down) Wp[m] = a.w_in[kb * plane + off[m]];
                else Wm[m] = a.w_in[kb * plane + off[m]];
                W0[m] = a.w_in[long(kfirst) * plane + off[m]];
            }
        }
#pragma unroll
        for (int t = 0; t < H; ++t) {
            const int k = Down ? kfirst - t : k0 + t;
            if (Down ? k < k0 : k >= nz) break;
            const long km = k > 0 ? k - 1 : 0, kp = k < nz - 1 ? k + 1 : k;
            const long v = k * plane + off[4];
            double acc = a.b[v];
            if (a.w_in) {
                // the plane ahead in the walk
#pragma unroll
                for (int m = 0; m < 9; ++m) {
                    if constexpr (Down) Wm[m] = a.w_in[km * plane + off[m]];
                    else Wp[m] = a.w_in[kp * plane + off[m]];
                }
                const long pls[3] = {km * plane, long(k) * plane, kp * plane};
                double part[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int o = 0; o < 27; ++o) {
                    if (o == 13) continue;
                    const long u = pls[o / 9] + off[o % 9];
                    const double K = (o > 13) ? double(Kc[(o - 14) * V + v]) : double(Kc[(12 - o) * V + u]);
                    const double w = o < 9 ? Wm[o % 9] : (o < 18 ? W0[o % 9] : Wp[o % 9]);
                    part[o / 9] += K * w;
                }
                acc += (k > 0 ? part[0] : 0.0) + part[1] + part[2];
#pragma unroll
                for (int m = 0; m < 9; ++m) {
                    if constexpr (Down) { Wp[m] = W0[m]; W0[m] = Wm[m]; }
                    else { Wm[m] = W0[m]; W0[m] = Wp[m]; }
                }
            }
            if (a.w_out) a.w_out[v] = acc * a.E[v];
            if (a.J) jacobi_update(a, v, acc, q, dist, bad);
        }
    }
    if (a.J) jacobi_block_max(a, q, dist, bad);
}

// reverse: the column layers in descending order (top first).  Consecutive sweeps alternate, so each
// starts where the previous one ended and finds its most recent planes still in the caches; the order
// of the blocks does not change any voxel's sum.
// alt_walk: odd column layers walk their voxels top down (the plane two neighbouring layers share is
// then read by both near their start or both near their end); each voxel's sum is unchanged.
template <typename coef, int H = kJacCol>
__global__ __launch_bounds__(kPlaneThreads) void jacobi_kernel_column(JacobiArgs a, int group, int reverse,
                                                                      int alt_walk)
{
    const int blk = blockIdx.x;
    const int xcd = blk & 7, slot = blk >> 3;
    const int kc = slot / group;
    const int kcol = reverse ? int(gridDim.x) / (8 * group) - 1 - kc : kc;
    const int p = (xcd * group + (slot - kc * group)) * kPlaneThreads + threadIdx.x;
    if (alt_walk && (kcol & 1)) jacobi_column_body<coef, H, true>(a, p, kcol);
    else jacobi_column_body<coef, H, false>(a, p, kcol);
}

// Column height of the column form, from the number of workgroups that columns of 4 give: 4 for
// grids that fill the chip with them, 2 for mid-size grids, 1 for small ones.  Measured per float64
// sweep (H = 4 / 2 / 1): 129^3 (2178 workgroups of 4) 67.8 / 67.3 / 70.5 us, 65^3 (289) 13.8 / 13.3 /
// 14.1 us, 17^3 (10) 8.0 / 5.2 / 3.9 us.  Every height gives the same per-voxel sums.
inline int jacobi_column_height(int nx, int ny, int nz)
{
    const long blocks4 = (long(nx) * ny + kPlaneThreads - 1) / kPlaneThreads * ((nz + 3) / 4);
    return blocks4 >= 1024 ? 4 : (blocks4 >= 128 ? 2 : 1);
}

// Walk direction of the column layout (walk: 1 odd layers top down, 0 all bottom up, -1 by coefficient
// type): top-down odd layers pay with float coefficients in columns of 4 and not with float64 ones.
// Measured per sweep (bitwise the same iterates): float coefficients 129^3 38.0 -> 35.8 us,
// 129^2 x 193 55.2 -> 52.9 us, 65^3 (columns of 2) 9.24 against 9.30 us; float64 coefficients 129^3
// 67.4 -> 73.3 us (L2 fetches 389 against 384 MB), 65^3 13.5 -> 13.0 us.
inline bool jacobi_alt_walk(int walk, bool f32, int H) { return walk >= 0 ? walk != 0 : (f32 && H == 4); }

// Gauss-Seidel colour pass.  The voxels are coloured per axis so that no two 27-point neighbours share
// a colour: index i has colour i mod 2, except on a periodic axis of odd length, where the last index
// has colour 2 (its neighbours n-2 and 0 are odd and even); z (not periodic) always has two.  A pass
// updates the voxels of one colour (cx, cy, cz) in place: none of them reads another's value, and
// each reads the newest value of every neighbour.  Member q of colour c on an axis is 2q + c, or
// n - 1 for colour 2; cnt holds the members per axis.
__device__ inline int colour_member(int c, int q, int n) { return c == 2 ? n - 1 : 2 * q + c; }

template <typename coef>
__global__ __launch_bounds__(kPlaneThreads) void jacobi_kernel_colour(JacobiArgs a, int3 col, int3 cnt)
{
    const long t = long(blockIdx.x) * kPlaneThreads + threadIdx.x;
    const bool valid = t < long(cnt.x) * cnt.y * cnt.z;
    int i = 0, j = 0, k = 0;
    if (valid) {
        const long rest = t / cnt.x;
        i = colour_member(col.x, int(t - rest * cnt.x), a.nx);
        j = colour_member(col.y, int(rest % cnt.y), a.ny);
        k = colour_member(col.z, int(rest / cnt.y), a.nz);
    }
    jacobi_core<coef>(a, i, j, k, valid);
}

// Colours on an axis of length n (periodic or not) and the members of colour c.
inline int axis_colours(int n, bool periodic) { return periodic && (n % 2) ? 3 : 2; }
inline int colour_count(int c, int n, bool periodic)
{
    if (periodic && (n % 2)) return c == 2 ? 1 : (n - 1) / 2;
    return c == 0 ? (n + 1) / 2 : n / 2;
}

// One Jacobi sweep in the given grid layout: 0 one block per chunk of a plane, 1 the same padded to
// a multiple of 8 chunks per plane, 2 contiguous chunk ranges per XCD, 3 2D tiles, 4 columns.
// reverse: the column layout walks its column layers top first (see jacobi_kernel_column).
// height: column height of layout 4 (1, 2 or 4; 0: jacobi_column_height); walk: see jacobi_alt_walk.
inline void launch_jacobi_sweep(const JacobiArgs &a, int layout, bool f32, hipStream_t stream, bool reverse = false,
                                int height = 0, int walk = -1)
{
    const int chunks = (a.nx * a.ny + kPlaneThreads - 1) / kPlaneThreads;
    const int group = (chunks + 7) / 8;
    const dim3 blk(kPlaneThreads);
    if (layout == 4) {
        const int H = height > 0 ? height : jacobi_column_height(a.nx, a.ny, a.nz);
        const dim3 grid(unsigned(8 * group) * unsigned((a.nz + H - 1) / H));
        const int rev = reverse ? 1 : 0, md = jacobi_alt_walk(walk, f32, H) ? 1 : 0;
        if (H == 1) {
            if (f32) hipLaunchKernelGGL((jacobi_kernel_column<float, 1>), grid, blk, 0, stream, a, group, rev, md);
            else hipLaunchKernelGGL((jacobi_kernel_column<double, 1>), grid, blk, 0, stream, a, group, rev, md);
        } else if (H == 2) {
            if (f32) hipLaunchKernelGGL((jacobi_kernel_column<float, 2>), grid, blk, 0, stream, a, group, rev, md);
            else hipLaunchKernelGGL((jacobi_kernel_column<double, 2>), grid, blk, 0, stream, a, group, rev, md);
        } else {
            if (f32) hipLaunchKernelGGL((jacobi_kernel_column<float, 4>), grid, blk, 0, stream, a, group, rev, md);
            else hipLaunchKernelGGL((jacobi_kernel_column<double, 4>), grid, blk, 0, stream, a, group, rev, md);
        }
    } else if (layout == 3) {
        const int tiles_x = (a.nx + kTileX - 1) / kTileX, tiles_y = (a.ny + kTileY - 1) / kTileY;
        const int tgroup = (tiles_x * tiles_y + 7) / 8;
        const dim3 grid(unsigned(8 * tgroup) * unsigned(a.nz));
        if (f32) hipLaunchKernelGGL(jacobi_kernel_tiled<float>, grid, blk, 0, stream, a, tiles_x, tgroup);
        else hipLaunchKernelGGL(jacobi_kernel_tiled<double>, grid, blk, 0, stream, a, tiles_x, tgroup);
    } else if (layout == 2) {
        const dim3 grid(unsigned(8 * group) * unsigned(a.nz));
        if (f32) hipLaunchKernelGGL(jacobi_kernel_grouped<float>, grid, blk, 0, stream, a, group);
        else hipLaunchKernelGGL(jacobi_kernel_grouped<double>, grid, blk, 0, stream, a, group);
    } else {
        const dim3 grid(layout == 1 ? unsigned(group * 8) : unsigned(chunks), a.nz);
        if (f32) hipLaunchKernelGGL(jacobi_kernel<float>, grid, blk, 0, stream, a);
        else hipLaunchKernelGGL(jacobi_kernel<double>, grid, blk, 0, stream, a);
    }
}

// ------------------------------------------------------------------------------------------------
// Ng acceleration: weighted dot products (fixed-order two-level reduction), the small normal
// equations solved on the device, and the combination.  The iterates live in a ring of R = order + 2
// vectors; with the newest at ring index m, iterate x_i (i = 0 newest) is entry (m - i) mod R.
// ------------------------------------------------------------------------------------------------

constexpr int kNgSums = 9;          // A00 A01 A02 A11 A12 A22 b0 b1 b2
constexpr int kNgBlocks = 512;      // blocks of the dot-product pass of one problem (fixes the order)
constexpr int kNgThreads = 256;
// layout of the Ng work buffer of one problem
constexpr int kNgSumOff = kNgBlocks * kNgSums;   // the 9 sums
constexpr int kNgCoefOff = kNgSumOff + kNgSums;  // c0..c3 (x_new = sum_i c_i x_i) and a valid flag
constexpr int kNgWork = kNgCoefOff + 5;

struct NgArgs {
    long V;
    int order;
    const double *hist;             // [order + 2][V]
    double *work;                   // [kNgWork]
    double *J;                      // receives the extrapolated iterate
    int unit_weights;               // 1: weights 1 instead of 1/x_0^2 (iterates that may vanish)
};

__device__ inline const double *ng_x(const NgArgs &a, int m, int i)
{
    const int R = a.order + 2;
    return a.hist + long((m - i + 4 * R) % R) * a.V;
}

// One block's share of the weighted dot products (weights 1/x_0^2, or 1).  Whole block.
__device__ inline void ng_dots_body(const NgArgs &a, int m, int blk)
{
    const double *x0 = ng_x(a, m, 0), *x1 = ng_x(a, m, 1);
    double acc[kNgSums];
#pragma unroll
    for (int q = 0; q < kNgSums; ++q) acc[q] = 0.0;
    for (long v = long(blk) * kNgThreads + threadIdx.x; v < a.V; v += long(kNgBlocks) * kNgThreads) {
        const double y0 = x0[v];
        const double w = a.unit_weights ? 1.0 : 1.0 / (y0 * y0);
        const double d0 = y0 - x1[v];
        double Q[3] = {0.0, 0.0, 0.0};
        for (int i = 1; i <= a.order; ++i) Q[i - 1] = d0 - (ng_x(a, m, i)[v] - ng_x(a, m, i + 1)[v]);
        acc[0] += w * Q[0] * Q[0];
        acc[1] += w * Q[0] * Q[1];
        acc[2] += w * Q[0] * Q[2];
        acc[3] += w * Q[1] * Q[1];
        acc[4] += w * Q[1] * Q[2];
        acc[5] += w * Q[2] * Q[2];
        acc[6] += w * d0 * Q[0];
        acc[7] += w * d0 * Q[1];
        acc[8] += w * d0 * Q[2];
    }
    __shared__ double red[kNgSums][kNgThreads];
#pragma unroll
    for (int q = 0; q < kNgSums; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = kNgThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int q = 0; q < kNgSums; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < kNgSums) a.work[blk * kNgSums + threadIdx.x] = red[threadIdx.x][0];
}

// Sums the block partials in a fixed order (one block), then thread 0 solves the order x order
// normal equations by Gaussian elimination with partial pivoting.  A singular system or a
// non-finite solution clears the valid flag (the plain iterate is kept).
__device__ inline void ng_solve_body(const NgArgs &a)
{
    __shared__ double red[kNgSums][kNgThreads];
    for (int q = 0; q < kNgSums; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < kNgBlocks; b += kNgThreads) s += a.work[b * kNgSums + q];
        red[q][threadIdx.x] = s;
    }
    __syncthreads();
    for (int h = kNgThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int q = 0; q < kNgSums; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double sums[kNgSums];
    for (int q = 0; q < kNgSums; ++q) {
        sums[q] = red[q][0];
        a.work[kNgSumOff + q] = sums[q];
    }
    const int n = a.order;
    double A[3][3] = {{sums[0], sums[1], sums[2]}, {sums[1], sums[3], sums[4]}, {sums[2], sums[4], sums[5]}};
    double b[3] = {sums[6], sums[7], sums[8]}, c[3] = {0.0, 0.0, 0.0};
    bool ok = true;
    for (int col = 0; col < n && ok; ++col) {
        int p = col;
        for (int r = col + 1; r < n; ++r) if (fabs(A[r][col]) > fabs(A[p][col])) p = r;
        if (!(fabs(A[p][col]) > 0.0)) { ok = false; break; }
        if (p != col) {
            for (int q = 0; q < n; ++q) { const double t = A[col][q]; A[col][q] = A[p][q]; A[p][q] = t; }
            const double t = b[col]; b[col] = b[p]; b[p] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            const double f = A[r][col] / A[col][col];
            for (int q = col; q < n; ++q) A[r][q] -= f * A[col][q];
            b[r] -= f * b[col];
        }
    }
    for (int r = n - 1; r >= 0 && ok; --r) {
        double t = b[r];
        for (int q = r + 1; q < n; ++q) t -= A[r][q] * c[q];
        c[r] = t / A[r][r];
        if (!isfinite(c[r])) ok = false;
    }
    double sa = 0.0;
    for (int i = 0; i < n; ++i) sa += c[i];
    a.work[kNgCoefOff + 0] = 1.0 - sa;
    for (int i = 0; i < 3; ++i) a.work[kNgCoefOff + 1 + i] = c[i];
    a.work[kNgCoefOff + 4] = ok ? 1.0 : 0.0;
}

// J_v = c0 x_0 + sum_i c_i x_i (only when the solve succeeded)
__device__ inline void ng_combine_body(const NgArgs &a, int m, long v)
{
    const double *cf = a.work + kNgCoefOff;
    if (cf[4] == 0.0) return;
    double r = cf[0] * ng_x(a, m, 0)[v];
    for (int i = 1; i <= a.order; ++i) r += cf[i] * ng_x(a, m, i)[v];
    a.J[v] = r;
}

__global__ __launch_bounds__(kNgThreads) void ng_dots_kernel(NgArgs a, int m)
{
    ng_dots_body(a, m, blockIdx.x);
}

__global__ __launch_bounds__(kNgThreads) void ng_solve_kernel(NgArgs a)
{
    ng_solve_body(a);
}

__global__ __launch_bounds__(256) void ng_combine_kernel(NgArgs a, int m)
{
    const long v = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < a.V) ng_combine_body(a, m, v);
}

// ------------------------------------------------------------------------------------------------
// Anderson mixing of the outer iteration: windows of (input, output) pairs of the OS step in two rings
// of V-vectors; slot[0..k] are the ring entries of the window, oldest first.  The weighted dot products
// use the fixed two-level partition of the Ng kernels (bitwise reproducible).
// ------------------------------------------------------------------------------------------------

constexpr int kAaMaxDepth = 8;
constexpr int kAaSums = kAaMaxDepth * (kAaMaxDepth + 1) / 2 + kAaMaxDepth;   // A (upper) and b
constexpr int kAaBlocks = 512;
constexpr int kAaThreads = 256;
constexpr int kAaSumOff = kAaBlocks * kAaSums;
constexpr int kAaCoefOff = kAaSumOff + kAaSums;     // gamma_1..gamma_8 and a valid flag
constexpr int kAaWork = kAaCoefOff + kAaMaxDepth + 1;

struct AaArgs {
    long V;
    int k;                          // differences in the window (1..kAaMaxDepth)
    int slot[kAaMaxDepth + 1];      // ring entries of the window, oldest first
    const double *X, *G;            // rings [depth + 1][V] of inputs and outputs
    double *work;                   // [kAaWork]
    double *J;                      // receives the mixed input of the next step
};

// Index of the sum A_ij (i <= j < k) and of b_i in a block's partial sums.
__host__ __device__ constexpr int aa_a_index(int i, int j) { return j * (j + 1) / 2 + i; }
__host__ __device__ constexpr int aa_b_index(int i) { return kAaMaxDepth * (kAaMaxDepth + 1) / 2 + i; }

// One block's share of A_ij = sum_v w df_i df_j and b_i = sum_v w df_i f_k, w = 1/g_k^2, f = g - x,
// df_j = f_k - f_{k-j}; the sums of a thread, then of a wavefront (xor tree), then of the block's
// wavefronts in order.  Whole block; blk is the block's index among the kAaBlocks of the pass.
__device__ inline void aa_dots_body(const AaArgs &a, int blk)
{
    const int k = a.k;
    double acc[kAaSums];
#pragma unroll
    for (int q = 0; q < kAaSums; ++q) acc[q] = 0.0;
    const double *gk = a.G + long(a.slot[k]) * a.V, *xk = a.X + long(a.slot[k]) * a.V;
    for (long v = long(blk) * kAaThreads + threadIdx.x; v < a.V; v += long(kAaBlocks) * kAaThreads) {
        const double g = gk[v];
        const double w = 1.0 / (g * g);
        const double fk = g - xk[v];
        double df[kAaMaxDepth];
#pragma unroll
        for (int j = 1; j <= kAaMaxDepth; ++j) {
            if (j > k) break;
            const long o = long(a.slot[k - j]) * a.V + v;
            df[j - 1] = fk - (a.G[o] - a.X[o]);
        }
#pragma unroll
        for (int j = 0; j < kAaMaxDepth; ++j) {
            if (j >= k) break;
#pragma unroll
            for (int i = 0; i <= j; ++i) acc[aa_a_index(i, j)] += w * df[i] * df[j];
            acc[aa_b_index(j)] += w * df[j] * fk;
        }
    }
#pragma unroll
    for (int q = 0; q < kAaSums; ++q)
        for (int offs = 32; offs > 0; offs >>= 1) acc[q] += __shfl_xor(acc[q], offs);
    __shared__ double part[kAaThreads / 64][kAaSums];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int q = 0; q < kAaSums; ++q) part[wid][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < kAaSums) {
        double s = part[0][threadIdx.x];
        for (int w2 = 1; w2 < kAaThreads / 64; ++w2) s += part[w2][threadIdx.x];
        a.work[blk * kAaSums + threadIdx.x] = s;
    }
}

__global__ __launch_bounds__(kAaThreads) void aa_dots_kernel(AaArgs a) { aa_dots_body(a, blockIdx.x); }

// Sums the block partials in a fixed order, then thread 0 solves the k x k normal equations A gamma = b
// by Gaussian elimination with partial pivoting; a singular system or a non-finite solution clears the
// valid flag (the output g_k is then kept as the next input).  Whole block.
__device__ inline void aa_solve_body(const AaArgs &a)
{
    __shared__ double tot[kAaSums];
    if (threadIdx.x < kAaSums) {
        double s = 0.0;
        for (int b = 0; b < kAaBlocks; ++b) s += a.work[b * kAaSums + threadIdx.x];
        tot[threadIdx.x] = s;
        a.work[kAaSumOff + threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int n = a.k;
    double A[kAaMaxDepth][kAaMaxDepth], b[kAaMaxDepth], g[kAaMaxDepth];
    for (int i = 0; i < n; ++i) {
        b[i] = tot[aa_b_index(i)];
        g[i] = 0.0;
        for (int j = 0; j < n; ++j) A[i][j] = i <= j ? tot[aa_a_index(i, j)] : tot[aa_a_index(j, i)];
    }
    bool ok = true;
    for (int c = 0; c < n && ok; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r) if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (!(fabs(A[p][c]) > 0.0)) { ok = false; break; }
        if (p != c) {
            for (int q = 0; q < n; ++q) { const double t = A[c][q]; A[c][q] = A[p][q]; A[p][q] = t; }
            const double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[r][c] / A[c][c];
            for (int q = c; q < n; ++q) A[r][q] -= f * A[c][q];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0 && ok; --r) {
        double t = b[r];
        for (int q = r + 1; q < n; ++q) t -= A[r][q] * g[q];
        g[r] = t / A[r][r];
        if (!isfinite(g[r])) ok = false;
    }
    for (int i = 0; i < kAaMaxDepth; ++i) a.work[kAaCoefOff + i] = i < n ? g[i] : 0.0;
    a.work[kAaCoefOff + kAaMaxDepth] = ok ? 1.0 : 0.0;
}

__global__ __launch_bounds__(kAaThreads) void aa_solve_kernel(AaArgs a) { aa_solve_body(a); }

// J = g_k - sum_j gamma_j (g_k - g_{k-j}) when the solve succeeded, else g_k (voxel v).
__device__ inline void aa_combine_body(const AaArgs &a, long v)
{
    const double *cf = a.work + kAaCoefOff;
    const double gk = a.G[long(a.slot[a.k]) * a.V + v];
    double x = gk;
    if (cf[kAaMaxDepth] != 0.0)
        for (int j = 1; j <= a.k; ++j) x -= cf[j - 1] * (gk - a.G[long(a.slot[a.k - j]) * a.V + v]);
    a.J[v] = x;
}

__global__ __launch_bounds__(256) void aa_combine_kernel(AaArgs a)
{
    const long v = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < a.V) aa_combine_body(a, v);
}

// finiteness / range check of a device medium
__global__ void check_medium_kernel(long V, const double *chi, const double *eps, const double *B,
                                    int *flag)
{
    long v = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const double c = chi[v], e = eps[v], b = B[v];
    const bool ok = isfinite(c) && c > 0.0 && isfinite(e) && e > 0.0 && e <= 1.0 && isfinite(b);
    if (!ok) atomicOr(flag, 1);
}

// LTE-diffusion inner condition: dB/dtau per bottom column, (B_0 - B_1) / ((chi_0 + chi_1) / 2) from
// the bottom voxel and the one above it (the optical distance between their centres)
__global__ void diffusion_slope_kernel(int nxy, const double *chi, const double *B, double *slope)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nxy) slope[c] = (B[c] - B[nxy + c]) / (0.5 * (chi[c] + chi[nxy + c]));
}

__global__ void check_finite_kernel(long V, const double *x, int *flag)
{
    long v = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= V) return;
    if (!isfinite(x[v])) atomicOr(flag, 1);
}

}  // namespace
