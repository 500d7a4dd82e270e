// Host-side geometry of the HIP library: the angle set, the per-direction segment tables of the
// line family and the band plan of the sweep kernel.
//
// Every line of a direction is the same line translated by an integer number of columns (the lines
// go through the voxel centres (i+1/2, j+1/2) on the top plane and the grid is uniform and periodic
// in x,y), so one table per (direction, layer) describes every line: the column offsets of its
// segments relative to the line's own top column, and their lengths.
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace rt3d {

namespace {

// Number of eigenvalues below x of the symmetric tridiagonal matrix with zero diagonal and squared
// off-diagonals b2[1..n-1] (LDL^T pivots of T - x I; Sylvester's law of inertia).
int sturm_count(int n, const std::vector<double> &b2, double x)
{
    int cnt = 0;
    double piv = -x;
    if (piv < 0.0) ++cnt;
    for (int k = 1; k < n; ++k) {
        if (piv == 0.0) piv = 1e-300;
        piv = -x - b2[k] / piv;
        if (piv < 0.0) ++cnt;
    }
    return cnt;
}

}  // namespace

bool gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    if (n < 2) return false;
    // Jacobi matrix of the Legendre polynomials: zero diagonal, off-diagonal k / sqrt(4k^2 - 1).
    std::vector<double> b2(n, 0.0);
    for (int k = 1; k < n; ++k) b2[k] = double(k) * k / (4.0 * k * k - 1.0);
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int r = 0; r < n; ++r) {
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid == lo || mid == hi) break;
            if (sturm_count(n, b2, mid) > r) hi = mid; else lo = mid;
        }
        x[r] = 0.5 * (lo + hi);
    }
    // exact mirror symmetry of the node set
    for (int r = 0; r < n / 2; ++r) {
        double m = 0.5 * (x[n - 1 - r] - x[r]);
        x[r] = -m;
        x[n - 1 - r] = m;
    }
    // Christoffel numbers: 1 / sum_{k<n} (k + 1/2) P_k(x)^2 (orthonormal Legendre polynomials)
    for (int r = 0; r < n; ++r) {
        double p_prev = 1.0, p = x[r];
        double s = 0.5 * p_prev * p_prev + 1.5 * p * p;
        for (int k = 1; k + 1 < n; ++k) {
            double p_next = ((2.0 * k + 1.0) * x[r] * p - k * p_prev) / (k + 1.0);
            p_prev = p;
            p = p_next;
            s += (k + 1.5) * p * p;
        }
        w[r] = 1.0 / s;
    }
    return true;
}

int mirror_x(int b, int n_phi)
{
    return (b < n_phi / 2) ? n_phi / 2 - 1 - b : 3 * n_phi / 2 - 1 - b;
}

bool make_angle_set(int n_theta, int n_phi, AngleSet &out)
{
    if (n_theta < 2 || (n_theta % 2) != 0 || n_phi < 4 || (n_phi % 4) != 0) return false;
    std::vector<double> x, w;
    if (!gauss_legendre(n_theta, x, w)) return false;
    out.n_theta = n_theta;
    out.n_phi = n_phi;
    out.n_dir = n_theta * n_phi;
    out.mu.resize(out.n_dir);
    out.ox.resize(out.n_dir);
    out.oy.resize(out.n_dir);
    out.w.resize(out.n_dir);
    const double two_pi = 2.0 * M_PI;
    for (int a = 0; a < n_theta; ++a) {
        const double sin_t = std::sqrt(1.0 - x[a] * x[a]);
        for (int b = 0; b < n_phi; ++b) {
            const int d = a * n_phi + b;
            const double phi = two_pi * (b + 0.5) / n_phi;
            out.mu[d] = x[a];
            out.ox[d] = sin_t * std::cos(phi);
            out.oy[d] = sin_t * std::sin(phi);
            out.w[d] = w[a] / (2.0 * n_phi);
        }
        // exact mirror symmetry x -> -x (phi -> pi - phi): the mirror of b is
        // n_phi/2 - 1 - b for b < n_phi/2 and 3 n_phi/2 - 1 - b otherwise
        for (int b = 0; b < n_phi; ++b) {
            const int bm = mirror_x(b, n_phi);
            if (bm > b) {
                out.ox[a * n_phi + bm] = -out.ox[a * n_phi + b];
                out.oy[a * n_phi + bm] = out.oy[a * n_phi + b];
            }
        }
    }
    return true;
}

namespace {

// Heights in (z_lo, z_hi) where X(z) = x0 + (z - nz) t is an integer, ordered along the travel
// direction (descending z when going down).
void face_crossings(int nz, double x0, double t, double z_in, double z_out, std::vector<double> &z)
{
    z.clear();
    const double lo = std::min(z_in, z_out), hi = std::max(z_in, z_out);
    const double Xa = x0 + (lo - nz) * t, Xb = x0 + (hi - nz) * t;
    const double m_lo = std::floor(std::min(Xa, Xb)) + 1.0;
    for (double m = m_lo; m < std::max(Xa, Xb); m += 1.0) {
        double zc = nz + (m - x0) / t;
        zc = std::min(std::max(zc, lo), hi);
        z.push_back(zc);
    }
    std::sort(z.begin(), z.end());
    if (z_out < z_in) std::reverse(z.begin(), z.end());
}

}  // namespace

void layer_segments(int nz, double mu, double ox, double oy, int k, LayerSegments &out)
{
    const double tx = ox / mu, ty = oy / mu;                  // horizontal drift per unit height
    const double z_in = (mu < 0.0) ? k + 1.0 : double(k);
    const double z_out = (mu < 0.0) ? double(k) : k + 1.0;
    std::vector<double> zx, zy;
    face_crossings(nz, 0.5, tx, z_in, z_out, zx);
    face_crossings(nz, 0.5, ty, z_in, z_out, zy);
    // merge the two ordered crossing lists along the travel direction; crossings closer than
    // kCornerTol in height are one crossing through a voxel edge (a line through an edge would
    // otherwise leave a rounding-sized sliver between the x and the y crossing)
    constexpr double kCornerTol = 1e-12;
    const bool down = z_out < z_in;
    std::vector<double> zb;
    zb.reserve(zx.size() + zy.size() + 2);
    zb.push_back(z_in);
    size_t p = 0, q = 0;
    while (p < zx.size() || q < zy.size()) {
        bool take_x;
        if (p == zx.size()) take_x = false;
        else if (q == zy.size()) take_x = true;
        else take_x = down ? (zx[p] >= zy[q]) : (zx[p] <= zy[q]);
        const double z = take_x ? zx[p++] : zy[q++];
        if (std::fabs(z - zb.back()) > kCornerTol) zb.push_back(z);
    }
    if (zb.size() > 1 && std::fabs(z_out - zb.back()) <= kCornerTol) zb.back() = z_out;
    else zb.push_back(z_out);
    out.di.clear();
    out.dj.clear();
    out.len.clear();
    const double inv_amu = 1.0 / std::fabs(mu);
    for (size_t s = 0; s + 1 < zb.size(); ++s) {
        const double dz = std::fabs(zb[s + 1] - zb[s]);
        if (!(dz > 0.0)) continue;
        const double zm = 0.5 * (zb[s] + zb[s + 1]);
        out.di.push_back(int(std::floor(0.5 + (zm - nz) * tx)));
        out.dj.push_back(int(std::floor(0.5 + (zm - nz) * ty)));
        out.len.push_back(dz * inv_amu);
    }
}

void direction_segments(int nz, const AngleSet &A, int d, int k, LayerSegments &out)
{
    const int a = d / A.n_phi, b = d % A.n_phi;
    const int bm = mirror_x(b, A.n_phi);
    if (bm >= b) {
        layer_segments(nz, A.mu[d], A.ox[d], A.oy[d], k, out);
        return;
    }
    const int dm = a * A.n_phi + bm;
    layer_segments(nz, A.mu[dm], A.ox[dm], A.oy[dm], k, out);
    for (int &x : out.di) x = -x;
}

static int pos_mod(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

bool build_sweep_plan(int nx, int ny, int nz, const AngleSet &A, int lines_per_wg, int target_seg_per_wg,
                      size_t lds_bytes_max, SweepPlan &P, std::string &err)
{
    P = SweepPlan();
    P.nx = nx;
    P.ny = ny;
    P.nz = nz;
    P.n_dir = A.n_dir;
    P.lines_per_wg = lines_per_wg;
    const int max_rows = lines_per_wg / nx;
    if (max_rows < 1) {
        err = "nx exceeds the lines one sweep workgroup can hold";
        return false;
    }
    P.seg_off.assign(size_t(A.n_dir) * nz, 0);
    P.seg_n.assign(size_t(A.n_dir) * nz, 0);
    P.row_min.assign(size_t(A.n_dir) * nz, 0);
    P.dirs.resize(A.n_dir);
    std::vector<int> span(A.n_dir, 0);
    std::vector<double> seg_per_layer(A.n_dir, 0.0);
    LayerSegments L;
    long total_segments = 0;
    for (int d = 0; d < A.n_dir; ++d) {
        long nseg = 0;
        for (int k = 0; k < nz; ++k) {
            direction_segments(nz, A, d, k, L);
            const int n = int(L.di.size());
            const int bmin = *std::min_element(L.dj.begin(), L.dj.end());
            const int bmax = *std::max_element(L.dj.begin(), L.dj.end());
            span[d] = std::max(span[d], bmax - bmin);
            const size_t dk = size_t(d) * nz + k;
            P.seg_off[dk] = int(P.seg_a.size());
            P.seg_n[dk] = n;
            P.row_min[dk] = pos_mod(bmin, ny);
            for (int s = 0; s < n; ++s) {
                P.seg_a.push_back(pos_mod(L.di[s], nx));
                P.seg_bb.push_back(L.dj[s] - bmin);
                P.seg_bm.push_back(pos_mod(L.dj[s] - bmin, ny));
                P.seg_ai.push_back(L.di[s]);
                P.seg_bi.push_back(L.dj[s]);
                P.seg_len.push_back(L.len[s]);
            }
            nseg += n;
        }
        total_segments += nseg;
        seg_per_layer[d] = double(nseg) / nz;
        P.dirs[d].wmu = A.w[d] * std::fabs(A.mu[d]);
        P.dirs[d].down = A.mu[d] < 0.0 ? 1 : 0;
        P.dirs[d].pad = 0;
        P.dirs[d].mu = A.mu[d];
    }
    P.mean_segments = double(total_segments) / (double(A.n_dir) * nz);
    // pairs mirrored in x: the partner's tables must equal the owner's up to negated columns
    for (int a = 0; a < A.n_theta; ++a) {
        for (int b = 0; b < A.n_phi; ++b) {
            const int bm = mirror_x(b, A.n_phi);
            if (bm < b) continue;
            const int dA = a * A.n_phi + b, dB = a * A.n_phi + bm;
            for (int k = 0; k < nz; ++k) {
                const size_t ka = size_t(dA) * nz + k, kb = size_t(dB) * nz + k;
                if (P.seg_n[ka] != P.seg_n[kb] || P.row_min[ka] != P.row_min[kb]) {
                    err = "mirrored directions do not share their segment structure";
                    return false;
                }
                for (int s = 0; s < P.seg_n[ka]; ++s) {
                    const int ia = P.seg_off[ka] + s, ib = P.seg_off[kb] + s;
                    if (P.seg_ai[ia] != -P.seg_ai[ib] || P.seg_bi[ia] != P.seg_bi[ib] ||
                        P.seg_len[ia] != P.seg_len[ib]) {
                        err = "mirrored directions do not share their segment structure";
                        return false;
                    }
                }
            }
            PairInfo pi{};
            pi.wmu = P.dirs[dA].wmu;
            pi.dA = dA;
            pi.dB = dB;
            pi.down = P.dirs[dA].down;
            pi.mu = A.mu[dA];
            // Band height: about target_seg_per_wg line-segments per layer for the two directions,
            // never thinner than the window's halo, within the line and LDS budgets.
            int rows = int(std::lround(target_seg_per_wg / (2.0 * nx * seg_per_layer[dA])));
            rows = std::max(rows, std::max(1, span[dA]));
            rows = std::min(rows, max_rows);
            auto lds = [&](int r) {
                return std::max(sweep_lds_bytes(r + span[dA], r, nx, false),
                                sweep_lds_bytes(r + span[dA], r, nx, true));
            };
            while (rows > 1 && lds(rows) > lds_bytes_max) --rows;
            rows = std::min(rows, ny);
            if (lds(rows) > lds_bytes_max) {
                err = "the deposit window of one band exceeds the LDS budget";
                return false;
            }
            pi.band_rows = rows;
            pi.n_bands = (ny + rows - 1) / rows;
            pi.win_rows = rows + span[dA];
            pi.last_rows = ny - (pi.n_bands - 1) * rows;
            pi.inv_rows = 1.0f / float(rows);
            P.max_win_rows = std::max(P.max_win_rows, pi.win_rows);
            P.pairs.push_back(pi);
            const size_t pl0 = P.player.size();
            for (int k = 0; k < nz; ++k) {
                const size_t ka = size_t(dA) * nz + k;
                PairLayer pl{int(P.pseg.size()), P.seg_n[ka], P.row_min[ka], 0};
                P.player.push_back(pl);
                for (int s = 0; s < P.seg_n[ka]; ++s) {
                    const int ia = P.seg_off[ka] + s;
                    PairSeg ps{};
                    ps.saA = P.seg_a[ia];
                    ps.shB = 0;
                    ps.smnx = P.seg_bm[ia] * nx;
                    ps.sbnx = P.seg_bb[ia] * nx;
                    ps.len = P.seg_len[ia];
                    ps.len32 = float(P.seg_len[ia]);
                    P.pseg.push_back(ps);
                }
            }
            // moves of the B lines: a slot holds the B line whose top column is its A line's plus
            // 2 dA, so when dA changes by delta to the next segment in sweep order (layers top down
            // for downward pairs) the B line moves by -2 delta columns
            std::vector<int> order;            // the pair's segments in sweep order, unreduced dA
            std::vector<size_t> at;
            for (int st = 0; st < nz; ++st) {
                const int k = pi.down ? nz - 1 - st : st;
                const size_t ka = size_t(dA) * nz + k;
                const size_t base = size_t(P.player[pl0 + k].off);
                for (int s = 0; s < P.seg_n[ka]; ++s) {
                    order.push_back(P.seg_ai[P.seg_off[ka] + s]);
                    at.push_back(base + size_t(s));
                }
            }
            for (size_t i = 0; i + 1 < order.size(); ++i)
                P.pseg[at[i]].shB = pos_mod(-2 * (order[i + 1] - order[i]), nx);
        }
    }
    P.n_pair = int(P.pairs.size());
    // the Lambda* kernel takes the pairs as two runs, all of one vertical direction, then the other
    for (int p = 1, changes = 0; p < P.n_pair; ++p)
        if (P.pairs[p].down != P.pairs[p - 1].down && ++changes > 1) {
            err = "direction pairs are not ordered by their vertical direction";
            return false;
        }
    int64_t off = 0;
    std::vector<std::pair<double, WorkItem>> work;
    for (int p = 0; p < P.n_pair; ++p) {
        PairInfo &pi = P.pairs[p];
        pi.p_off = off;
        off += int64_t(pi.n_bands) * nz * pi.win_rows * nx;
        for (int b = 0; b < pi.n_bands; ++b) {
            WorkItem it;
            it.pair = p;
            it.band = b;
            it.j0 = b * pi.band_rows;
            it.rows = std::min(pi.band_rows, ny - it.j0);
            work.push_back({it.rows * seg_per_layer[pi.dA], it});
        }
    }
    P.p_elems = off;
    // dispatch the most expensive bands first
    std::stable_sort(work.begin(), work.end(),
                     [](const std::pair<double, WorkItem> &x, const std::pair<double, WorkItem> &y) {
                         return x.first > y.first;
                     });
    for (auto &w : work) P.items.push_back(w.second);
    return true;
}

}  // namespace rt3d
