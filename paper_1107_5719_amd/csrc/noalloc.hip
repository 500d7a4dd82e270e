// noalloc.hip -- the formal solution for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// rt3d_formal_solution_noalloc computes what rt3d_formal_solution computes (same plan, kernels and
// summation order, so bitwise the same J_fs for the same grid and sweep shape), with no context: the
// caller passes chi, S, the bottom-plane light and the output on the device, and everything else the
// kernels need -- the packed {chi, S} field, the exponential's table, the plan's tables and the partial
// planes of the direction pairs -- lives in one file-scope device array of kScratchBytes.  When the
// partial planes of all pairs do not fit beside the rest, the pairs are swept in ranges that do, and
// the angle sum is carried from range to range in J_fs in the order of a single pass.
//
// The array is a host-side stand-in in host code: the kernels get its device address, taken once per
// device with hipGetSymbolAddress while that device is current, never the array's name.  Every call on
// a device shares that device's array, so calls that overlap on one device (other streams or host
// threads) race; each call returns only after its work on the stream has finished.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rt3d.h"
#include "context.h"
#include "geometry.h"
#include "kernels.h"

using namespace rt3d_host;

namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;   // 128 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// failures are reported like a failed context creation: rt3d_last_error(NULL) of the calling thread
int noalloc_fail(int code, const std::string &msg)
{
    set_thread_error(msg);
    return code;
}

// The device address of this device's scratch array (looked up once per device, with it current).
int scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return noalloc_fail(RT3D_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return noalloc_fail(RT3D_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return noalloc_fail(RT3D_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RT3D_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Packs {chi, S} per voxel as the context's source kernel does for a given S.
__global__ __launch_bounds__(kPlaneThreads) void pack_kernel(long V, const double *chi, const double *S, double2 *cs)
{
    const long v = long(blockIdx.x) * kPlaneThreads + threadIdx.x;
    if (v < V) cs[v] = make_double2(chi[v], S[v]);
}

template <typename T>
int upload(unsigned char *dst, const std::vector<T> &h, hipStream_t st)
{
    if (h.empty()) return RT3D_OK;
    hipError_t e = hipMemcpyAsync(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return noalloc_fail(RT3D_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    return RT3D_OK;
}

}  // namespace

extern "C" {

int rt3d_formal_solution_noalloc(const rt3d_grid_desc *g, const double *chi, const double *S, const double *I_bot,
                                 double *J_fs, void *hip_stream)
{
    set_thread_error(std::string());
    std::string msg;
    if (validate_desc(g, msg) != RT3D_OK) return noalloc_fail(RT3D_ERR_ARG, msg);
    if (g->bottom_bc == 2) return noalloc_fail(RT3D_ERR_ARG, "the LTE-diffusion inner condition needs a context");
    if (!chi || !S || !J_fs) return noalloc_fail(RT3D_ERR_ARG, "chi, S and J_fs must be device pointers");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    rt3d::AngleSet A;
    if (!rt3d::make_angle_set(g->n_theta, g->n_phi, A)) return noalloc_fail(RT3D_ERR_ARG, "bad angle set");
    rt3d::SweepPlan plan;
    if (!build_plan(*g, A, 0, plan, msg)) return noalloc_fail(RT3D_ERR_ARG, msg);
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const long V = long(nx) * ny * nz;
    const SweepShape shape = kSweepShapes[0];

    // workspace layout: exponential table, {chi, S}, pair tables, layer table, pair segments, row minima,
    // work items of every range, then the partial planes of one range of pairs
    std::vector<double> tab(kExpTab);
    for (int j = 0; j < kExpTab; ++j) tab[j] = double(std::exp2(static_cast<long double>(j) / kExpTab));
    // ranges of pairs whose partial planes fit what the tables leave of the workspace
    // (one copy of the pair table per range, at most one range per pair, with the partial-plane
    // offsets relative to the range's first pair)
    const size_t fixed = align256(tab.size() * sizeof(double)) + align256(size_t(V) * sizeof(double2)) +
                         align256(plan.pairs.size() * plan.pairs.size() * sizeof(rt3d::PairInfo)) +
                         align256(plan.player.size() * sizeof(rt3d::PairLayer)) +
                         align256(plan.pseg.size() * sizeof(rt3d::PairSeg)) +
                         align256(plan.row_min.size() * sizeof(int)) +
                         align256(plan.items.size() * sizeof(rt3d::WorkItem));
    if (fixed >= kScratchBytes)
        return noalloc_fail(RT3D_ERR_ARG, "grid too large for the allocation-free formal solution: its tables need " +
                                              std::to_string(fixed) + " of " + std::to_string(kScratchBytes) +
                                              " workspace bytes");
    const size_t room = (kScratchBytes - fixed) / sizeof(double);
    std::vector<int> q_begin;             // pair ranges [q_begin[r], q_begin[r + 1])
    for (int q = 0; q < plan.n_pair;) {
        const int64_t base = plan.pairs[q].p_off;
        int q1 = q;
        while (q1 < plan.n_pair) {
            const int64_t end = q1 + 1 < plan.n_pair ? plan.pairs[q1 + 1].p_off : plan.p_elems;
            if (size_t(end - base) > room) break;
            ++q1;
        }
        if (q1 == q)
            return noalloc_fail(RT3D_ERR_ARG, "grid too large for the allocation-free formal solution: the partial "
                                              "planes of one direction pair exceed its workspace");
        q_begin.push_back(q);
        q = q1;
    }
    q_begin.push_back(plan.n_pair);
    const int n_range = int(q_begin.size()) - 1;
    // the work items of each range, in the plan's dispatch order
    std::vector<rt3d::WorkItem> items;
    std::vector<int> item_begin;
    for (int r = 0; r < n_range; ++r) {
        item_begin.push_back(int(items.size()));
        for (const rt3d::WorkItem &it : plan.items)
            if (it.pair >= q_begin[r] && it.pair < q_begin[r + 1]) items.push_back(it);
    }
    item_begin.push_back(int(items.size()));
    // per range, the pair table with the offsets of its partial planes taken from the range's first pair
    std::vector<rt3d::PairInfo> range_pairs;
    for (int r = 0; r < n_range; ++r) {
        const int64_t shift = plan.pairs[q_begin[r]].p_off;
        for (rt3d::PairInfo pi : plan.pairs) {
            pi.p_off -= shift;          // negative for the pairs before the range, which it does not touch
            range_pairs.push_back(pi);
        }
    }

    void *base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    unsigned char *p = static_cast<unsigned char *>(base);
    unsigned char *d_tab = p;        p += align256(tab.size() * sizeof(double));
    unsigned char *d_cs = p;         p += align256(size_t(V) * sizeof(double2));
    unsigned char *d_pairs = p;      p += align256(plan.pairs.size() * plan.pairs.size() * sizeof(rt3d::PairInfo));
    unsigned char *d_player = p;     p += align256(plan.player.size() * sizeof(rt3d::PairLayer));
    unsigned char *d_pseg = p;       p += align256(plan.pseg.size() * sizeof(rt3d::PairSeg));
    unsigned char *d_rowmin = p;     p += align256(plan.row_min.size() * sizeof(int));
    unsigned char *d_items = p;      p += align256(plan.items.size() * sizeof(rt3d::WorkItem));
    double *d_P = reinterpret_cast<double *>(p);
    // from here on an early return first drains the stream: the copies read this call's host tables
    auto drain_fail = [&](int code, const std::string &m) {
        hipStreamSynchronize(st);
        return noalloc_fail(code, m);
    };
    if ((rc = upload(d_tab, tab, st)) || (rc = upload(d_pairs, range_pairs, st)) ||
        (rc = upload(d_player, plan.player, st)) || (rc = upload(d_pseg, plan.pseg, st)) ||
        (rc = upload(d_rowmin, plan.row_min, st)) || (rc = upload(d_items, items, st)))
        return drain_fail(rc, thread_error());
    hipLaunchKernelGGL(pack_kernel, dim3(unsigned((V + kPlaneThreads - 1) / kPlaneThreads)), dim3(kPlaneThreads), 0,
                       st, V, chi, S, reinterpret_cast<double2 *>(d_cs));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return drain_fail(RT3D_ERR_HIP, std::string("pack_kernel: ") + hipGetErrorString(e));

    SweepArgs sa{};
    sa.nx = nx; sa.ny = ny; sa.nz = nz;
    sa.n_down = A.n_dir / 2;
    sa.pseg = reinterpret_cast<const rt3d::PairSeg *>(d_pseg);
    sa.player = reinterpret_cast<const rt3d::PairLayer *>(d_player);
    const rt3d::PairInfo *d_range_pairs = reinterpret_cast<const rt3d::PairInfo *>(d_pairs);
    sa.cs = d_cs;
    sa.Ibot = g->bottom_bc == 1 ? nullptr : I_bot;
    sa.Islope = nullptr;
    sa.I_top = g->I_top;
    sa.P = d_P;
    sa.Iem = nullptr;
    sa.Iem_base = nullptr;
    sa.xtab = reinterpret_cast<const double *>(d_tab);
    ReduceArgs ra{};
    ra.nx = nx; ra.ny = ny; ra.nz = nz; ra.n_pair = plan.n_pair;

    ra.row_min = reinterpret_cast<const int *>(d_rowmin);
    ra.P = d_P;
    ra.chi = chi;
    ra.Jfs = J_fs;
    const size_t smem = sweep_smem_bytes(plan, false);
    const dim3 red_grid(unsigned(((nx + 1) / 2 * ny + kPlaneThreads - 1) / kPlaneThreads), unsigned(nz));
    for (int r = 0; r < n_range; ++r) {
        const int n_items = item_begin[r + 1] - item_begin[r];
        sa.items = reinterpret_cast<const rt3d::WorkItem *>(d_items) + item_begin[r];
        sa.pairs = d_range_pairs + size_t(r) * plan.pairs.size();
        ra.pairs = sa.pairs;
        if (n_items > 0)
            hipLaunchKernelGGL((sweep_kernel<double, 512, 2>), dim3(unsigned(n_items)), dim3(shape.threads), smem, st, sa);
        e = hipGetLastError();
        if (e != hipSuccess) return drain_fail(RT3D_ERR_HIP, std::string("sweep_kernel: ") + hipGetErrorString(e));
        hipLaunchKernelGGL(reduce_kernel_pair_range<double>, red_grid, dim3(kPlaneThreads), 0, st, ra, q_begin[r],
                           q_begin[r + 1], r == 0 ? 1 : 0, r == n_range - 1 ? 1 : 0);
        e = hipGetLastError();
        if (e != hipSuccess) return drain_fail(RT3D_ERR_HIP, std::string("reduce_kernel: ") + hipGetErrorString(e));
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return noalloc_fail(RT3D_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    return RT3D_OK;
}

}  // extern "C"
