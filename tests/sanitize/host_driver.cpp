// Host-side code of the library under AddressSanitizer / UndefinedBehaviorSanitizer: angle sets,
// per-direction segment tables, sweep plans for several grids, angle sets and workgroup shapes (with
// the B-line moves of every direction pair followed through the sweep), and the tuning cache's
// write / replace / read round trip.  Built with g++ by tests/test_sanitizers.py.
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_1107_5719_amd/csrc/geometry.h"
#include "../../paper_1107_5719_amd/csrc/tune_cache.h"

int main(int argc, char **argv)
{
    const std::string cache = argc > 1 ? argv[1] : "/tmp/rt3d_sanitize_cache.json";
    struct G { int nx, ny, nz, nt, np; } grids[] = {{3, 3, 3, 2, 4}, {5, 7, 4, 8, 4}, {9, 7, 11, 8, 8},
                                                    {33, 40, 6, 16, 16}, {17, 17, 17, 4, 12}};
    const int shapes[][2] = {{512, 2}, {512, 4}, {256, 8}, {1024, 2}, {256, 4}, {256, 2}};
    long checked = 0;
    for (const G &g : grids) {
        rt3d::AngleSet A;
        if (!rt3d::make_angle_set(g.nt, g.np, A)) return 1;
        rt3d::LayerSegments L;
        for (int d = 0; d < A.n_dir; ++d)
            for (int k = 0; k < g.nz; ++k) {
                rt3d::direction_segments(g.nz, A, d, k, L);
                if (L.di.empty() || L.di.size() != L.len.size()) return 2;
                checked += long(L.di.size());
            }
        for (const auto &sh : shapes) {
            rt3d::SweepPlan P;
            std::string err;
            if (!rt3d::build_sweep_plan(g.nx, g.ny, g.nz, A, sh[0] * sh[1], 16 * sh[0], 48 * 1024, P, err)) {
                std::printf("plan %dx%dx%d %dx%d shape %dx%d: %s\n", g.nx, g.ny, g.nz, g.nt, g.np, sh[0], sh[1],
                            err.c_str());
                return 3;
            }
            if (P.items.empty() || P.pairs.size() * 2 != size_t(A.n_dir)) return 4;
            // every band's LDS fits the budget; following the B-line moves of each pair keeps in
            // slot c the B line whose top column is c + 2 dA (its voxel is then the A line's), and
            // ends with the top columns the sweep writes the emergent B intensities to
            for (size_t p = 0; p < P.pairs.size(); ++p) {
                const rt3d::PairInfo &pi = P.pairs[p];
                for (int f32 = 0; f32 < 2; ++f32)
                    if (rt3d::sweep_lds_bytes(pi.win_rows, pi.band_rows, g.nx, f32) > 48 * 1024) return 11;
                std::vector<int> top(g.nx), next(g.nx);
                bool first = true;
                int sa_last = 0;
                for (int st = 0; st < g.nz; ++st) {
                    const int k = pi.down ? g.nz - 1 - st : st;
                    const rt3d::PairLayer &pl = P.player[p * g.nz + k];
                    const int off_a = P.seg_off[size_t(pi.dA) * g.nz + k];
                    for (int s = 0; s < pl.ns; ++s) {
                        const rt3d::PairSeg &ps = P.pseg[pl.off + s];
                        const int da = P.seg_ai[off_a + s];
                        const int two = ((2 * da) % g.nx + g.nx) % g.nx;
                        if (ps.saA != ((da % g.nx) + g.nx) % g.nx) return 12;
                        if (ps.shB < 0 || ps.shB >= g.nx) return 13;
                        for (int c = 0; c < g.nx; ++c) {
                            if (first) top[c] = (c + two) % g.nx;
                            if (top[c] != (c + two) % g.nx) return 14;
                        }
                        first = false;
                        for (int c = 0; c < g.nx; ++c) next[(c + ps.shB) % g.nx] = top[c];
                        top.swap(next);
                        sa_last = ps.saA;
                        checked += 1;
                    }
                }
                for (int c = 0; c < g.nx; ++c)
                    if (top[c] != ((c + sa_last) % g.nx + sa_last) % g.nx) return 15;
            }
        }
    }
    std::remove(cache.c_str());
    std::string err;
    if (!rt3d_tune::store(cache, "dev|fp64|5x5x5|2x4", "{\"shape\": 3}", err)) return 5;
    if (!rt3d_tune::store(cache, "dev|fp64|9x9x9|2x4", "{\"shape\": 1}", err)) return 6;
    if (!rt3d_tune::store(cache, "dev|fp64|5x5x5|2x4", "{\"shape\": 4}", err)) return 7;
    int s1 = -1, s2 = -1, s3 = -1;
    if (!rt3d_tune::lookup(cache, "dev|fp64|5x5x5|2x4", s1) || s1 != 4) return 8;
    if (!rt3d_tune::lookup(cache, "dev|fp64|9x9x9|2x4", s2) || s2 != 1) return 9;
    if (rt3d_tune::lookup(cache, "dev|fp32_sweep|9x9x9|2x4", s3)) return 10;
    std::remove(cache.c_str());
    std::printf("host driver ok: %ld segments\n", checked);
    return 0;
}
