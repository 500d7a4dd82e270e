// Host-side geometry of the HIP library: angle set, per-direction segment tables and the work plan
// of the line sweep.  Internal to the library (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace rt3d {

struct AngleSet {
    int n_theta = 0, n_phi = 0, n_dir = 0;
    std::vector<double> mu, ox, oy, w;   // per direction d = a * n_phi + b
};

// Gauss-Legendre nodes (ascending) by Sturm-sequence bisection on the Jacobi matrix of the Legendre
// polynomials, weights by the Christoffel sum 1 / sum_k (k + 1/2) P_k(x)^2.
bool gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
bool make_angle_set(int n_theta, int n_phi, AngleSet &out);

// Segments of the reference line (through (1/2, 1/2, nz)) of one direction inside layer k, in travel
// order: column offsets (di, dj) relative to the line's top column and path lengths.
struct LayerSegments {
    std::vector<int> di, dj;
    std::vector<double> len;
};
void layer_segments(int nz, double mu, double ox, double oy, int k, LayerSegments &out);

// Index of the azimuth mirrored in x (phi -> pi - phi).
int mirror_x(int b, int n_phi);

// The segments of direction d of an angle set inside layer k.  Of an x-mirrored pair of azimuths
// the lower index is cut by layer_segments and the other is its exact mirror (columns negated):
// lines that pass through voxel edges (every line when n_phi = 4) leave rounding-sized slivers whose
// voxel would otherwise depend on the rounding of each direction separately.
void direction_segments(int nz, const AngleSet &A, int d, int k, LayerSegments &out);

// Per-direction metadata (plain old data, copied to the device).
struct DirInfo {
    double wmu;        // W_d * |mu_d|
    int down;          // 1 if mu < 0 (sweep from the top layer down)
    int pad;
    double mu;         // direction cosine with the z axis
};

// A pair of directions mirrored in x, (mu, phi) and (mu, pi - phi).  Their lines cross the same
// faces at the same heights: the segment lengths and row offsets are identical and the column
// offsets are negated, so one workgroup sweeps both through the same band and one partial plane
// holds both.  W |mu| is the same for both.
struct PairInfo {
    double wmu;        // W |mu| of either direction
    int dA, dB;        // the two directions; dA owns the shared tables
    int down;          // 1 if mu < 0
    int band_rows;     // Bj: line rows per band (last band may be shorter)
    int n_bands;       // nb
    int win_rows;      // Hw = Bj + span: rows of the deposit window of one band
    int last_rows;     // rows of the last band: ny - (nb - 1) * Bj
    float inv_rows;    // 1 / Bj (band lookup; corrected exactly in the kernel)
    int64_t p_off;     // element offset of this pair's partial planes in P
    double mu;         // direction cosine with the z axis (the same for both)
};

// Segment s of a pair in one layer, packed for one scalar load: the column offset of direction A
// (modulo nx; B's is its negative), the move of the B lines between the slots of their row after
// this segment (-2 times the change of A's column offset to the next segment in sweep order, modulo
// nx; 0: none), the row offset modulo ny times nx (global row step), the row offset within the band
// window times nx (LDS row step), and the length in both precisions.
struct PairSeg {
    int saA, shB, smnx, sbnx;
    double len;
    float len32;
    int pad;
};

// Per (pair, layer): first entry in the packed segment list, segment count, window origin row.
struct PairLayer {
    int off, ns, rmin, pad;
};

// One workgroup of the sweep: direction pair p, band of line rows [j0, j0 + rows).
struct WorkItem {
    int pair, band, j0, rows;
};

struct SweepPlan {
    int nx = 0, ny = 0, nz = 0, n_dir = 0, n_pair = 0;
    int lines_per_wg = 0;                 // lines of one direction in one workgroup
    // segment tables, flat; index of (d, k) is d * nz + k
    std::vector<int> seg_off, seg_n;      // per (d, k)
    std::vector<int> seg_a;               // column offset modulo nx, in [0, nx)
    std::vector<int> seg_bb;              // row offset minus the layer's minimum, in [0, span]
    std::vector<int> seg_bm;              // seg_bb modulo ny
    std::vector<int> seg_ai, seg_bi;      // unreduced column / row offsets (for Lambda*)
    std::vector<double> seg_len;
    std::vector<int> row_min;             // per (d, k): minimum row offset modulo ny
    std::vector<DirInfo> dirs;
    std::vector<PairInfo> pairs;
    std::vector<PairSeg> pseg;            // packed per-pair segments
    std::vector<PairLayer> player;        // per (pair, layer): index pair * nz + k
    std::vector<WorkItem> items;          // in dispatch order (most expensive first)
    int64_t p_elems = 0;                  // size of the partial-plane buffer P in elements
    int max_win_rows = 0;
    double mean_segments = 0.0;           // per voxel and angle
};

// LDS of one sweep workgroup for a band of band_rows line rows and a deposit window of win_rows rows:
// the window and two exchange buffers of one value per line, in the sweep's precision.
inline size_t sweep_lds_bytes(int win_rows, int band_rows, int nx, bool f32)
{
    const size_t cells = size_t(win_rows) * size_t(nx), lines = size_t(band_rows) * size_t(nx);
    return (cells + 2 * lines) * (f32 ? sizeof(float) : sizeof(double));
}

// Build segment tables and the band plan.  lines_per_wg bounds the lines of one direction in one
// band; lds_bytes_max bounds a band's LDS in either precision (sweep_lds_bytes).
bool build_sweep_plan(int nx, int ny, int nz, const AngleSet &A, int lines_per_wg, int target_seg_per_wg,
                      size_t lds_bytes_max, SweepPlan &plan, std::string &err);

}  // namespace rt3d
