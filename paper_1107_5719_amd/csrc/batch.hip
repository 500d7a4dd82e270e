// batch.hip -- batched form of the scattering solve: many independent problems (wavelengths, on
// grids that may differ in size and angle set) iterated together, one launch per kernel per outer
// iteration for all of them, the whole outer iteration captured once in a HIP graph and replayed.
//
// Every member is an ordinary single-problem context (its buffers, plan and Lambda*); the batch
// adds device arrays of per-member kernel arguments, block tables that map each workgroup to
// (member, work unit), and a per-member control state on the device.  Control is device-side, so a
// replay needs no host decision:
//   ctl_pre     picks each member's mode for this iteration: 0 idle (converged or stopped), 1 a
//               float64 formal solution, 2 (FP32 form) a float32 formal solution of the source
//               change since the anchor.  The rule is the one of the single-problem OS step.
//   source / sweep / reduce   one launch per mode; blocks of members in another mode exit at once.
//   anchor copy (FP32 form)   members that ran a float64 formal solution make it their anchor.
//   jacobi x M  the inner sweeps of every active member.
//   ctl_post    reads each member's max |dJ|/|J|, counts the iteration, applies the stopping rule
//               and schedules the Ng history store / extrapolation.
//   Ng          history store, dot products, the small solve, the combination, ring restart.
// The host replays the graph and reads the control states every poll_every replays; converged
// members are masked on the device, so the iterates do not depend on poll_every.  The arithmetic
// and its order are those of the single-problem path (same device bodies, same Ng partition), so a
// member's iterates are bitwise those of solving it alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rt3d.h"
#include "context.h"
#include "kernels.h"
#include "tune_cache.h"

using namespace rt3d_host;

namespace {

struct MemberState {
    int active;          // 1 while the member iterates
    int mode;            // this iteration: 0 idle, 1 float64 formal solution, 2 float32 difference one
    int status;          // RT3D_MEMBER_* of include/rt3d.h
    int iters;
    int anchor_valid, force_refresh, last_anchored;
    int nh;              // iterates in the Ng history since the last extrapolation
    int ng_store;        // ring slot that receives J in this iteration, or -1
    int ng_newest;       // ring index of the newest iterate when extrapolating in this iteration, or -1
    int aa_count;        // Anderson window: (input, output) pairs held, their ring slots oldest first,
    int aa_next;         // the slot the next input takes, and whether this iteration mixes
    int aa_mix;
    int aa_slot[kAaMaxDepth + 1];
    int pad0;
    double c_last, da_last;
};

struct BatchParams {
    double tol;
    double anchor_ratio;  // FP32 form: re-anchor when c < anchor_ratio * max|J - Ja|/|J| (as a context)
    int max_iter, fp32, ng_order, ng_every;
    int aa_depth;         // Anderson mixing window (0: off)
    int pad;
};

struct MemberScalars {
    unsigned long long *maxrel, *maxdist;
    int *flag;
};

struct CopyArgs {
    long V, n_em;
    const double *J, *Jfs, *Iem;
    double *Ja, *Fa, *Iem_a;
    double *hist;
};

struct BatchItem {
    int member;
    WorkItem item;
};

struct PlaneBlock {
    int member, chunk, k, pad;
};

constexpr int kAuxBlocks = 128;      // blocks per member of the grid-stride copy / combine kernels

__global__ void ctl_pre_kernel(int n, MemberState *st, const BatchParams *prm)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    MemberState &s = st[m];
    if (!s.active) { s.mode = 0; return; }
    if (prm->aa_depth > 0) {
        // the step's input joins the Anderson window (the oldest pair leaves a full window)
        const int cap = prm->aa_depth + 1;
        if (s.aa_count == cap) {
            for (int q = 0; q + 1 < cap; ++q) s.aa_slot[q] = s.aa_slot[q + 1];
            --s.aa_count;
        }
        s.aa_slot[s.aa_count] = s.aa_next;
        s.aa_next = (s.aa_next + 1) % cap;
    }
    if (!prm->fp32) { s.mode = 1; return; }
    const bool refresh = !s.anchor_valid || s.force_refresh || s.c_last < prm->anchor_ratio * s.da_last;
    s.mode = refresh ? 1 : 2;
}

// st == nullptr: every member runs (the batched formal solution outside the iteration)
template <typename real>
__global__ __launch_bounds__(kPlaneThreads) void source_kernel_batch(const SourceArgs *args, const PlaneBlock *blocks,
                                                                     const MemberState *st, int want)
{
    const PlaneBlock b = blocks[blockIdx.x];
    if (st && st[b.member].mode != want) return;
    const SourceArgs a = args[b.member];
    source_body<real>(a, b.chunk * kPlaneThreads + threadIdx.x, b.k);
}

// With two slots per thread the float64 batched sweep is held to 80 VGPRs (6 waves per SIMD): 14.4 ->
// 14.0 ms per batched formal solution of 64 wavelengths when it needed 88.  Held to 64 (8 waves) it
// spills per layer and runs 13.7 against 12.4 ms.  With the paired lines it would take 82 and spills
// 20 bytes at 80, yet 5 waves without the spill run slower: 12.1 against 11.7 ms (shape 256 x 2).
template <int LPT> constexpr int kBatchSweepMinWaves = LPT <= 2 ? 6 : 1;

template <typename real, int NT, int LPT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kBatchSweepMinWaves<LPT>))) void sweep_kernel_batch(const SweepArgs *args, const BatchItem *items,
                                                         const MemberState *st, int want)
{
    extern __shared__ unsigned char smem_raw[];
    const BatchItem bi = items[blockIdx.x];
    if (st && st[bi.member].mode != want) return;
    const SweepArgs a = args[bi.member];
    sweep_body<real, NT, LPT>(a, bi.item, smem_raw);
}

template <typename real>
__global__ __launch_bounds__(kPlaneThreads) void reduce_kernel_batch(const ReduceArgs *args, const PlaneBlock *blocks,
                                                                     const MemberState *st, int want)
{
    const PlaneBlock b = blocks[blockIdx.x];
    if (st && st[b.member].mode != want) return;
    const ReduceArgs a = args[b.member];
    reduce_body_pair<real>(a, b.chunk * kPlaneThreads + threadIdx.x, b.k);
}

__global__ void anchor_copy_kernel(const CopyArgs *args, const MemberState *st)
{
    const int m = blockIdx.y;
    if (st[m].mode != 1) return;
    const CopyArgs a = args[m];
    const long n = a.V > a.n_em ? a.V : a.n_em;
    for (long v = long(blockIdx.x) * blockDim.x + threadIdx.x; v < n; v += long(gridDim.x) * blockDim.x) {
        if (v < a.V) {
            a.Ja[v] = a.J[v];
            a.Fa[v] = a.Jfs[v];
        }
        if (v < a.n_em) a.Iem_a[v] = a.Iem[v];
    }
}

// Clears the convergence scalars (a kernel, not a memset, so that it can sit in the graph).
__global__ void clear_scalars_kernel(int n, const MemberScalars *sc)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    *sc[m].maxrel = 0ull;
    *sc[m].maxdist = 0ull;
    *sc[m].flag = 0;
}

// Lambda* of several members in one launch (small grids alone would leave most of the chip idle)
__global__ __launch_bounds__(kLstarThreads) void lstar_kernel_batch(const LstarArgs *args, const PlaneBlock *blocks)
{
    const PlaneBlock b = blocks[blockIdx.x];
    lstar_body(args[b.member], b.chunk * kLstarThreads + threadIdx.x, b.k);
}

// Jacobi sweep of the members, column form (b.k is the column layer of kJacCol planes)
template <typename coef>
__global__ __launch_bounds__(kPlaneThreads) void jacobi_kernel_batch_column(const JacobiArgs *args,
                                                                            const PlaneBlock *blocks,
                                                                            const MemberState *st)
{
    const PlaneBlock b = blocks[blockIdx.x];
    if (st[b.member].mode == 0) return;
    const JacobiArgs a = args[b.member];
    jacobi_column_body<coef>(a, b.chunk * kPlaneThreads + threadIdx.x, b.k);
}

// The stopping rule of the single-problem solve, per member: a step whose max |dJ|/|J| is below tol
// ends the member (in the FP32 form only a step that ran a float64 formal solution; otherwise the
// next step is forced to re-anchor); NaN/Inf ends it; so does max_iter.  Ng: the iterate goes to the
// history ring and every ng_every stored iterates the ring is extrapolated.
__global__ void ctl_post_kernel(int n, MemberState *st, const BatchParams *prm, const MemberScalars *sc)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    MemberState &s = st[m];
    s.ng_store = -1;
    s.ng_newest = -1;
    s.aa_mix = 0;
    if (s.mode == 0) return;
    if (prm->aa_depth > 0) s.aa_count += 1;      // the step's output joins the window (aa_output_kernel)
    const double c = __longlong_as_double(static_cast<long long>(*sc[m].maxrel));
    const double d = __longlong_as_double(static_cast<long long>(*sc[m].maxdist));
    const bool anchored = s.mode == 1;
    // FP32 form: an anchored step starts the Anderson window afresh, as in the single solve
    if (prm->aa_depth > 0 && prm->fp32 && anchored && s.aa_count > 1) {
        s.aa_slot[0] = s.aa_slot[s.aa_count - 1];
        s.aa_count = 1;
    }
    s.iters += 1;
    s.c_last = c;
    s.da_last = d;
    s.last_anchored = anchored ? 1 : 0;
    if (prm->fp32 && anchored) {
        s.anchor_valid = 1;
        s.force_refresh = 0;
    }
    if (*sc[m].flag) {
        s.status = RT3D_MEMBER_NONFINITE;
        s.active = 0;
        return;
    }
    if (c < prm->tol) {
        if (!prm->fp32 || anchored) {
            s.status = RT3D_MEMBER_CONVERGED;
            s.active = 0;
            return;
        }
        s.force_refresh = 1;
    } else if (prm->ng_order > 0) {
        const int R = prm->ng_order + 2;
        s.ng_store = s.nh % R;
        s.nh += 1;
        if (s.nh - 1 >= prm->ng_every) {
            s.ng_newest = (s.nh - 1) % R;
            s.nh = 1;
        }
    } else if (prm->aa_depth > 0 && s.aa_count >= 2) {
        s.aa_mix = 1;
    }
    if (s.iters >= prm->max_iter) {
        s.status = RT3D_MEMBER_MAX_ITER;
        s.active = 0;
    }
}

__global__ void ng_store_kernel(const CopyArgs *args, const MemberState *st)
{
    const int m = blockIdx.y;
    const int slot = st[m].ng_store;
    if (slot < 0) return;
    const CopyArgs a = args[m];
    double *dst = a.hist + long(slot) * a.V;
    for (long v = long(blockIdx.x) * blockDim.x + threadIdx.x; v < a.V; v += long(gridDim.x) * blockDim.x)
        dst[v] = a.J[v];
}

__global__ __launch_bounds__(kNgThreads) void ng_dots_kernel_batch(const NgArgs *args, const MemberState *st)
{
    const int m = blockIdx.y;
    const int newest = st[m].ng_newest;
    if (newest < 0) return;
    const NgArgs a = args[m];
    ng_dots_body(a, newest, blockIdx.x);
}

__global__ __launch_bounds__(kNgThreads) void ng_solve_kernel_batch(const NgArgs *args, const MemberState *st)
{
    const int m = blockIdx.y;
    if (st[m].ng_newest < 0) return;
    const NgArgs a = args[m];
    ng_solve_body(a);
}

__global__ void ng_combine_kernel_batch(const NgArgs *args, const MemberState *st)
{
    const int m = blockIdx.y;
    const int newest = st[m].ng_newest;
    if (newest < 0) return;
    const NgArgs a = args[m];
    for (long v = long(blockIdx.x) * blockDim.x + threadIdx.x; v < a.V; v += long(gridDim.x) * blockDim.x)
        ng_combine_body(a, newest, v);
}

// Anderson window: J enters the input ring before the step (mode != 0) and the output ring after it
__global__ void aa_store_kernel(const AaArgs *args, const MemberState *st, int output)
{
    const int m = blockIdx.y;
    const MemberState &s = st[m];
    if (s.mode == 0) return;
    const AaArgs a = args[m];
    const int slot = output ? s.aa_slot[s.aa_count - 1] : s.aa_slot[s.aa_count];
    double *dst = (output ? const_cast<double *>(a.G) : const_cast<double *>(a.X)) + long(slot) * a.V;
    for (long v = long(blockIdx.x) * blockDim.x + threadIdx.x; v < a.V; v += long(gridDim.x) * blockDim.x)
        dst[v] = a.J[v];
}

// the window of member m as the single-problem mixing takes it
__device__ inline AaArgs aa_member_args(const AaArgs *args, const MemberState &s, int m)
{
    AaArgs a = args[m];
    a.k = s.aa_count - 1;
    for (int q = 0; q <= kAaMaxDepth; ++q) a.slot[q] = q < s.aa_count ? s.aa_slot[q] : 0;
    return a;
}

__global__ __launch_bounds__(kAaThreads) void aa_dots_kernel_batch(const AaArgs *args, const MemberState *st)
{
    const int m = blockIdx.y;
    if (!st[m].aa_mix) return;
    aa_dots_body(aa_member_args(args, st[m], m), blockIdx.x);
}

__global__ __launch_bounds__(kAaThreads) void aa_solve_kernel_batch(const AaArgs *args, const MemberState *st)
{
    const int m = blockIdx.y;
    if (!st[m].aa_mix) return;
    aa_solve_body(aa_member_args(args, st[m], m));
}

__global__ void aa_combine_kernel_batch(const AaArgs *args, const MemberState *st)
{
    const int m = blockIdx.y;
    if (!st[m].aa_mix) return;
    const AaArgs a = aa_member_args(args, st[m], m);
    for (long v = long(blockIdx.x) * blockDim.x + threadIdx.x; v < a.V; v += long(gridDim.x) * blockDim.x)
        aa_combine_body(a, v);
}

// after an extrapolation the ring restarts from the new iterate
__global__ void ng_restart_kernel(const CopyArgs *args, const MemberState *st)
{
    const int m = blockIdx.y;
    if (st[m].ng_newest < 0) return;
    const CopyArgs a = args[m];
    for (long v = long(blockIdx.x) * blockDim.x + threadIdx.x; v < a.V; v += long(gridDim.x) * blockDim.x)
        a.hist[v] = a.J[v];
}

}  // namespace


struct rt3d_batch {
    int n = 0;
    int precision = RT3D_FP64;
    int shape = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<rt3d_ctx *> m;
    int ng_order = 0, ng_every = 0;
    int aa_depth = 0;                  // Anderson mixing instead of Ng (0: off)
    // device tables (owned)
    MemberState *d_state = nullptr;
    BatchParams *d_params = nullptr;
    MemberScalars *d_scalars = nullptr;
    SourceArgs *d_src = nullptr;       // [2][n]: S from J; difference source (FP32 form)
    SweepArgs *d_sw = nullptr;         // [2][n]: with boundary light; difference
    ReduceArgs *d_red = nullptr;       // [3][n]: with residual; difference (FP32 form); no residual
    CopyArgs *d_copy = nullptr;        // [n]
    NgArgs *d_ng = nullptr;            // [n]
    AaArgs *d_aa = nullptr;            // [n] (window slots come from the member state)
    JacobiArgs *d_jac = nullptr;       // [M][n]
    int jac_M = 0;
    BatchItem *d_items = nullptr;
    PlaneBlock *d_planes = nullptr, *d_columns = nullptr;
    PlaneBlock *d_pplanes = nullptr;   // the reduction's blocks: chunks of voxel pairs of a row
    int n_items = 0, n_planes = 0, n_columns = 0, n_pplanes = 0;
    size_t smem64 = 0, smem32 = 0;
    long max_V = 0;
    bool tables_ok = false;            // argument arrays and block tables match the members
    bool plans_ok = true;              // false after a failed shape change
    // the captured outer iteration
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_M = 0;
    // statistics of the last solve
    long replays = 0, polls = 0;
    double solve_ms = 0.0;
    std::vector<MemberState> h_state;
    std::string err;
};

namespace {

int bfail(rt3d_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

#define BHIP_TRY(b, expr, what)                                                                   \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return bfail(b, e_ == hipErrorOutOfMemory ? RT3D_ERR_OOM : RT3D_ERR_HIP, \
                                           std::string(what) + ": " + hipGetErrorString(e_));     \
    } while (0)

// forward the last error of a member to the batch
int member_fail(rt3d_batch *b, int member, int rc)
{
    b->err = "member " + std::to_string(member) + ": " + b->m[member]->err;
    return rc;
}

template <typename T>
void bfree(T *&p)
{
    if (p) hipFree(p);
    p = nullptr;
}

void drop_graph(rt3d_batch *b)
{
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_M = 0;
}

void free_tables(rt3d_batch *b)
{
    drop_graph(b);
    bfree(b->d_state); bfree(b->d_params); bfree(b->d_scalars);
    bfree(b->d_src); bfree(b->d_sw); bfree(b->d_red); bfree(b->d_copy); bfree(b->d_ng); bfree(b->d_aa); bfree(b->d_jac);
    bfree(b->d_items); bfree(b->d_planes); bfree(b->d_columns); bfree(b->d_pplanes);
    b->jac_M = 0;
    b->tables_ok = false;
}

template <typename T>
int bupload(rt3d_batch *b, T *&d, const std::vector<T> &h)
{
    bfree(d);
    BHIP_TRY(b, hipMalloc(reinterpret_cast<void **>(&d), std::max<size_t>(h.size(), 1) * sizeof(T)), "hipMalloc");
    if (!h.empty()) BHIP_TRY(b, hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
    return RT3D_OK;
}

int launch_check(rt3d_batch *b, const char *what);

// Lambda* of every member that lacks it, in one launch over all their planes (64-column blocks,
// the largest members first), then each member's Jacobi coefficients.
int build_lstar_batched(rt3d_batch *b)
{
    std::vector<LstarArgs> args;
    std::vector<PlaneBlock> blocks;
    std::vector<int> who;
    for (int i = 0; i < b->n; ++i) {
        rt3d_ctx *c = b->m[i];
        if (c->have_lstar) continue;
        if (!c->plan_ok) return bfail(b, RT3D_ERR_STATE, "member " + std::to_string(i) + " has no sweep plan");
        LstarArgs a{};
        a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz; a.n_pair = c->plan.n_pair;
        a.early_exit = c->lstar_early_exit;
        a.pairs = c->pairs; a.seg_off = c->seg_off; a.seg_n = c->seg_n; a.seg_ai = c->seg_ai;
        a.seg_bi = c->seg_bi; a.seg_len = c->seg_len64; a.chi = c->chi; a.L = c->L;
        a.xtab = c->xtab;
        args.push_back(a);
        who.push_back(i);
    }
    if (who.empty()) return RT3D_OK;
    std::vector<int> order(who.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = int(q);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return long(args[x].nx) * args[x].ny * args[x].nz * args[x].n_pair >
               long(args[y].nx) * args[y].ny * args[y].nz * args[y].n_pair;
    });
    for (int q : order) {
        const int chunks = (args[q].nx * args[q].ny + kLstarThreads - 1) / kLstarThreads;
        for (int k = 0; k < args[q].nz; ++k)
            for (int ch = 0; ch < chunks; ++ch) blocks.push_back(PlaneBlock{q, ch, k, 0});
    }
    LstarArgs *d_args = nullptr;
    PlaneBlock *d_blocks = nullptr;
    int rc = RT3D_OK;
    if (hipMalloc(reinterpret_cast<void **>(&d_args), args.size() * sizeof(LstarArgs)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&d_blocks), blocks.size() * sizeof(PlaneBlock)) != hipSuccess) {
        rc = bfail(b, RT3D_ERR_OOM, "hipMalloc (Lambda* tables)");
    } else if (hipMemcpy(d_args, args.data(), args.size() * sizeof(LstarArgs), hipMemcpyHostToDevice) != hipSuccess ||
               hipMemcpy(d_blocks, blocks.data(), blocks.size() * sizeof(PlaneBlock), hipMemcpyHostToDevice) !=
                   hipSuccess) {
        rc = bfail(b, RT3D_ERR_HIP, "upload (Lambda* tables)");
    } else {
        hipLaunchKernelGGL(lstar_kernel_batch, dim3(unsigned(blocks.size())), dim3(kLstarThreads), 0, b->stream,
                           d_args, d_blocks);
        rc = launch_check(b, "lstar_kernel_batch");
        if (!rc && hipStreamSynchronize(b->stream) != hipSuccess) rc = bfail(b, RT3D_ERR_HIP, "sync (Lambda*)");
    }
    bfree(d_args);
    bfree(d_blocks);
    if (rc) return rc;
    for (int i : who) {
        rc = finish_lstar(b->m[i]);
        if (rc) return member_fail(b, i, rc);
    }
    return RT3D_OK;
}

// Argument arrays and block tables of all members (rebuilt whenever a plan or an Ng buffer changes).
int build_tables(rt3d_batch *b)
{
    drop_graph(b);
    b->tables_ok = false;
    const int n = b->n;
    std::vector<SourceArgs> src(2 * n);
    std::vector<SweepArgs> sw(2 * n);
    std::vector<ReduceArgs> red(3 * n);
    std::vector<CopyArgs> cp(n);
    std::vector<NgArgs> ng(n);
    std::vector<AaArgs> aa(n);
    std::vector<MemberScalars> sc(n);
    std::vector<std::pair<double, BatchItem>> work;
    std::vector<PlaneBlock> planes, columns, pplanes;
    const SweepShape sh = kSweepShapes[b->shape];
    b->smem64 = b->smem32 = 0;
    b->max_V = 0;
    for (int i = 0; i < n; ++i) {
        rt3d_ctx *c = b->m[i];
        if (!c->plan_ok || c->sweep_shape != b->shape) return bfail(b, RT3D_ERR_STATE, "member plan missing");
        const int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
        b->max_V = std::max(b->max_V, c->V);
        for (int v = 0; v < 2; ++v) {
            SourceArgs &a = src[v * n + i];
            a.nx = nx; a.ny = ny; a.nz = nz;
            a.chi = c->chi; a.eps = c->eps; a.B = c->B; a.J = c->J; a.S_given = nullptr;
            a.Ja = v == 1 ? c->Ja : nullptr;
            a.cs = c->cs;
            const bool diff = v == 1;
            SweepArgs &s = sw[v * n + i];
            s.nx = nx; s.ny = ny; s.nz = nz;
            s.n_down = c->A.n_dir / 2;
            s.pseg = c->pseg; s.player = c->player; s.pairs = c->pairs; s.items = c->items;
            s.cs = c->cs;
            s.Ibot = (c->g.bottom_bc != 1 && !diff) ? c->B : nullptr;
            s.Islope = (c->g.bottom_bc == 2 && !diff) ? c->bot_slope : nullptr;
            s.I_top = diff ? 0.0 : c->g.I_top;
            s.P = c->P;
            s.Iem = c->Iem;
            s.Iem_base = diff ? c->Iem_a : nullptr;
            s.xtab = c->xtab;
        }
        for (int v = 0; v < 3; ++v) {
            ReduceArgs &a = red[v * n + i];
            a.nx = nx; a.ny = ny; a.nz = nz; a.n_pair = c->plan.n_pair;
            a.pairs = c->pairs; a.row_min = c->row_min; a.P = c->P; a.chi = c->chi;
            a.J = c->J; a.Jfs = c->Jfs;
            a.base = v == 1 ? c->Fa : nullptr;
            a.rb = v == 2 ? nullptr : c->r;
        }
        CopyArgs &k = cp[i];
        k.V = c->V;
        k.n_em = long(c->A.n_dir / 2) * nx * ny;
        k.J = c->J; k.Jfs = c->Jfs; k.Iem = c->Iem;
        k.Ja = c->Ja; k.Fa = c->Fa; k.Iem_a = c->Iem_a;
        k.hist = c->ng_hist;
        NgArgs &g = ng[i];
        g.V = c->V; g.order = c->ng_order; g.hist = c->ng_hist; g.work = c->ng_work; g.J = c->J;
        AaArgs &w = aa[i];
        w.V = c->V; w.k = 0; w.X = c->aa_x; w.G = c->aa_g; w.work = c->aa_work; w.J = c->J;
        sc[i] = MemberScalars{c->d_maxrel, c->d_maxdist, c->d_flag};
        b->smem64 = std::max(b->smem64, sweep_smem_bytes(c->plan, false));
        b->smem32 = std::max(b->smem32, sweep_smem_bytes(c->plan, true));
        // sweep work: a band costs about (segments over all layers) x (line slots per thread)
        for (const WorkItem &it : c->plan.items) {
            double segs = 0.0;
            for (int z = 0; z < nz; ++z) segs += c->plan.player[size_t(it.pair) * nz + z].ns;
            const double slots = std::ceil(double(it.rows) * nx / sh.threads);
            work.push_back({segs * slots, BatchItem{i, it}});
        }
        const int chunks = (nx * ny + kPlaneThreads - 1) / kPlaneThreads;
        for (int z = 0; z < nz; ++z)
            for (int ch = 0; ch < chunks; ++ch) planes.push_back(PlaneBlock{i, ch, z, 0});
        // the reduction takes two neighbouring voxels of a row per thread, as for a single problem
        const int pchunks = ((nx + 1) / 2 * ny + kPlaneThreads - 1) / kPlaneThreads;
        for (int z = 0; z < nz; ++z)
            for (int ch = 0; ch < pchunks; ++ch) pplanes.push_back(PlaneBlock{i, ch, z, 0});
        // the Jacobi sweep's column layers, XCD-aware as in the single-problem grid: each member starts
        // on a multiple of 8 blocks; block b of the member runs on XCD b % 8, which takes the contiguous
        // chunk range [xcd * G, (xcd + 1) * G) of every column layer (G = chunks padded to 8, / 8);
        // padding blocks have no voxels
        const int group = (chunks + 7) / 8;
        while (columns.size() % 8) columns.push_back(PlaneBlock{i, chunks, 0, 0});
        const int layers = (nz + kJacCol - 1) / kJacCol;
        for (int bl = 0; bl < 8 * group * layers; ++bl) {
            const int xcd = bl & 7, slot = bl >> 3;
            const int kc = slot / group;
            columns.push_back(PlaneBlock{i, xcd * group + (slot - kc * group), kc, 0});
        }
    }
    // dispatch the most expensive bands of all members first
    std::stable_sort(work.begin(), work.end(), [](const std::pair<double, BatchItem> &x,
                                                  const std::pair<double, BatchItem> &y) { return x.first > y.first; });
    std::vector<BatchItem> items;
    items.reserve(work.size());
    for (auto &w : work) items.push_back(w.second);
    int rc = RT3D_OK;
    auto chk = [&](int r) { if (!rc) rc = r; };
    chk(bupload(b, b->d_src, src)); chk(bupload(b, b->d_sw, sw)); chk(bupload(b, b->d_red, red));
    chk(bupload(b, b->d_copy, cp)); chk(bupload(b, b->d_ng, ng)); chk(bupload(b, b->d_aa, aa));
    chk(bupload(b, b->d_scalars, sc));
    chk(bupload(b, b->d_items, items)); chk(bupload(b, b->d_planes, planes));
    chk(bupload(b, b->d_columns, columns)); chk(bupload(b, b->d_pplanes, pplanes));
    if (rc) return rc;
    if (!b->d_state) BHIP_TRY(b, hipMalloc(reinterpret_cast<void **>(&b->d_state), n * sizeof(MemberState)), "hipMalloc");
    if (!b->d_params) BHIP_TRY(b, hipMalloc(reinterpret_cast<void **>(&b->d_params), sizeof(BatchParams)), "hipMalloc");
    b->n_items = int(items.size());
    b->n_planes = int(planes.size());
    b->n_columns = int(columns.size());
    b->n_pplanes = int(pplanes.size());
    bfree(b->d_jac);
    b->jac_M = 0;
    b->tables_ok = true;
    return RT3D_OK;
}

// Member buffers move (a new medium or J is swapped in from staging buffers, an Ng ring is
// allocated, a plan is rebuilt): the tables are rebuilt before the next launch.
int ensure_tables(rt3d_batch *b)
{
    if (!b->plans_ok) return bfail(b, RT3D_ERR_STATE, "member plans are missing (a shape change failed)");
    return b->tables_ok ? RT3D_OK : build_tables(b);
}

void invalidate_tables(rt3d_batch *b)
{
    drop_graph(b);
    b->tables_ok = false;
}

// Jacobi argument sets of M inner sweeps: sweep 1 from dJ = 0, sweeps 2..M from the previous one
// (ping-pong buffers), the last updating J.
int build_jacobi_args(rt3d_batch *b, int M)
{
    if (b->jac_M == M && b->d_jac) return RT3D_OK;
    const int n = b->n;
    const bool f32 = b->precision == RT3D_FP32_SWEEP;
    std::vector<JacobiArgs> ja(size_t(M) * n);
    for (int i = 0; i < n; ++i) {
        rt3d_ctx *c = b->m[i];
        double *bufs[2] = {c->dJa, c->dJb};
        const double *in = nullptr;
        for (int s = 0; s < M; ++s) {
            const bool last = s == M - 1;
            double *out = last ? nullptr : bufs[s & 1];
            JacobiArgs &a = ja[size_t(s) * n + i];
            a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz;
            a.b = c->r; a.w_in = in; a.w_out = out;
            a.Kc = c->coef_fp32 ? static_cast<const void *>(c->Kc32) : static_cast<const void *>(c->Kc);
            a.invD = c->invD; a.E = c->Ecoef;
            a.J = last ? c->J : nullptr;
            a.maxrel = c->d_maxrel; a.nonfinite = c->d_flag;
            a.Ja = (f32 && last) ? c->Ja : nullptr;
            a.maxdist = c->d_maxdist;
            in = out;
        }
    }
    int rc = bupload(b, b->d_jac, ja);
    if (rc) return rc;
    b->jac_M = M;
    return RT3D_OK;
}

int launch_check(rt3d_batch *b, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, RT3D_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return RT3D_OK;
}

// sweep launch of one precision for the members in mode 'want' (st null: all members)
int launch_sweep_batch(rt3d_batch *b, bool fp32, const SweepArgs *args, const MemberState *st, int want)
{
    const dim3 grid(b->n_items);
    const size_t smem = fp32 ? b->smem32 : b->smem64;
#define RT3D_BATCH_SWEEP(NT_, LPT_)                                                                \
    do {                                                                                           \
        if (!fp32)                                                                                 \
            hipLaunchKernelGGL((sweep_kernel_batch<double, NT_, LPT_>), grid, dim3(NT_), smem,     \
                               b->stream, args, b->d_items, st, want);                             \
        else                                                                                       \
            hipLaunchKernelGGL((sweep_kernel_batch<float, NT_, LPT_>), grid, dim3(NT_), smem,      \
                               b->stream, args, b->d_items, st, want);                             \
    } while (0)
    switch (b->shape) {
    case 1: RT3D_BATCH_SWEEP(512, 4); break;
    case 2: RT3D_BATCH_SWEEP(256, 8); break;
    case 3: RT3D_BATCH_SWEEP(1024, 2); break;
    case 4: RT3D_BATCH_SWEEP(256, 4); break;
    case 5: RT3D_BATCH_SWEEP(256, 2); break;
    default: RT3D_BATCH_SWEEP(512, 2); break;
    }
#undef RT3D_BATCH_SWEEP
    return launch_check(b, "sweep_kernel_batch");
}

// One outer iteration of every active member, enqueued on the batch stream (captured once).
int enqueue_iteration(rt3d_batch *b, int M)
{
    const int n = b->n;
    const bool f32 = b->precision == RT3D_FP32_SWEEP;
    const dim3 ctl((n + 63) / 64), ctl_t(64);
    const dim3 aux(kAuxBlocks, n);
    int rc;
    hipLaunchKernelGGL(ctl_pre_kernel, ctl, ctl_t, 0, b->stream, n, b->d_state, b->d_params);
    if ((rc = launch_check(b, "ctl_pre_kernel"))) return rc;
    if (b->aa_depth > 0) {
        hipLaunchKernelGGL(aa_store_kernel, aux, dim3(256), 0, b->stream, b->d_aa, b->d_state, 0);
        if ((rc = launch_check(b, "aa_store_kernel"))) return rc;
    }
    // formal solution: float64 (mode 1), and in the FP32 form the float32 difference (mode 2)
    hipLaunchKernelGGL(source_kernel_batch<double>, dim3(b->n_planes), dim3(kPlaneThreads), 0, b->stream,
                       b->d_src, b->d_planes, b->d_state, 1);
    if (f32)
        hipLaunchKernelGGL(source_kernel_batch<float>, dim3(b->n_planes), dim3(kPlaneThreads), 0, b->stream,
                           b->d_src + n, b->d_planes, b->d_state, 2);
    if ((rc = launch_check(b, "source_kernel_batch"))) return rc;
    if ((rc = launch_sweep_batch(b, false, b->d_sw, b->d_state, 1))) return rc;
    if (f32 && (rc = launch_sweep_batch(b, true, b->d_sw + n, b->d_state, 2))) return rc;
    hipLaunchKernelGGL(reduce_kernel_batch<double>, dim3(b->n_pplanes), dim3(kPlaneThreads), 0, b->stream,
                       b->d_red, b->d_pplanes, b->d_state, 1);
    if (f32)
        hipLaunchKernelGGL(reduce_kernel_batch<float>, dim3(b->n_pplanes), dim3(kPlaneThreads), 0, b->stream,
                           b->d_red + n, b->d_pplanes, b->d_state, 2);
    if ((rc = launch_check(b, "reduce_kernel_batch"))) return rc;
    if (f32) {
        hipLaunchKernelGGL(anchor_copy_kernel, aux, dim3(256), 0, b->stream, b->d_copy, b->d_state);
        if ((rc = launch_check(b, "anchor_copy_kernel"))) return rc;
    }
    hipLaunchKernelGGL(clear_scalars_kernel, ctl, ctl_t, 0, b->stream, n, b->d_scalars);
    if ((rc = launch_check(b, "clear_scalars_kernel"))) return rc;
    // members keep the coefficient storage of the batch's precision (float32 in the FP32 form)
    const bool k32 = b->m[0]->coef_fp32 != 0;
    for (int s = 0; s < M; ++s) {
        const JacobiArgs *args = b->d_jac + size_t(s) * n;
        if (k32)
            hipLaunchKernelGGL(jacobi_kernel_batch_column<float>, dim3(b->n_columns), dim3(kPlaneThreads), 0,
                               b->stream, args, b->d_columns, b->d_state);
        else
            hipLaunchKernelGGL(jacobi_kernel_batch_column<double>, dim3(b->n_columns), dim3(kPlaneThreads), 0,
                               b->stream, args, b->d_columns, b->d_state);
        if ((rc = launch_check(b, "jacobi_kernel_batch"))) return rc;
    }
    hipLaunchKernelGGL(ctl_post_kernel, ctl, ctl_t, 0, b->stream, n, b->d_state, b->d_params, b->d_scalars);
    if ((rc = launch_check(b, "ctl_post_kernel"))) return rc;
    if (b->ng_order > 0) {
        hipLaunchKernelGGL(ng_store_kernel, aux, dim3(256), 0, b->stream, b->d_copy, b->d_state);
        hipLaunchKernelGGL(ng_dots_kernel_batch, dim3(kNgBlocks, n), dim3(kNgThreads), 0, b->stream, b->d_ng,
                           b->d_state);
        hipLaunchKernelGGL(ng_solve_kernel_batch, dim3(1, n), dim3(kNgThreads), 0, b->stream, b->d_ng, b->d_state);
        hipLaunchKernelGGL(ng_combine_kernel_batch, aux, dim3(256), 0, b->stream, b->d_ng, b->d_state);
        hipLaunchKernelGGL(ng_restart_kernel, aux, dim3(256), 0, b->stream, b->d_copy, b->d_state);
        if ((rc = launch_check(b, "ng kernels"))) return rc;
    }
    if (b->aa_depth > 0) {
        hipLaunchKernelGGL(aa_store_kernel, aux, dim3(256), 0, b->stream, b->d_aa, b->d_state, 1);
        hipLaunchKernelGGL(aa_dots_kernel_batch, dim3(kAaBlocks, n), dim3(kAaThreads), 0, b->stream, b->d_aa,
                           b->d_state);
        hipLaunchKernelGGL(aa_solve_kernel_batch, dim3(1, n), dim3(kAaThreads), 0, b->stream, b->d_aa, b->d_state);
        hipLaunchKernelGGL(aa_combine_kernel_batch, aux, dim3(256), 0, b->stream, b->d_aa, b->d_state);
        if ((rc = launch_check(b, "anderson kernels"))) return rc;
    }
    return RT3D_OK;
}

int capture_graph(rt3d_batch *b, int M)
{
    if (b->exec && b->graph_M == M) return RT3D_OK;
    drop_graph(b);
    int rc = build_jacobi_args(b, M);
    if (rc) return rc;
    BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    rc = enqueue_iteration(b, M);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return bfail(b, RT3D_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        hipGraphDestroy(g);
        return bfail(b, RT3D_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    b->graph = g;
    b->exec = x;
    b->graph_M = M;
    return RT3D_OK;
}

int check_member(rt3d_batch *b, int member)
{
    if (member < 0 || member >= b->n) return bfail(b, RT3D_ERR_ARG, "member index out of range");
    return RT3D_OK;
}

}  // namespace


extern "C" {

int rt3d_batch_create(rt3d_batch **out, int n_members, const rt3d_grid_desc *descs, int precision, int sweep_shape,
                      void *hip_stream)
{
    auto reject = [](int rc, const std::string &msg) {
        set_thread_error(msg);
        return rc;
    };
    if (!out) return reject(RT3D_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_members < 1 || !descs) return reject(RT3D_ERR_ARG, "n_members < 1 or descs is NULL");
    if (precision != RT3D_FP64 && precision != RT3D_FP32_SWEEP) return reject(RT3D_ERR_ARG, "bad precision");
    if (sweep_shape < 0 || sweep_shape >= n_sweep_shapes()) return reject(RT3D_ERR_ARG, "sweep shape out of range");
    for (int i = 0; i < n_members; ++i) {
        std::string msg;
        if (validate_desc(&descs[i], msg) != RT3D_OK)
            return reject(RT3D_ERR_ARG, "member " + std::to_string(i) + ": " + msg);
    }
    rt3d_batch *b = new (std::nothrow) rt3d_batch();
    if (!b) return reject(RT3D_ERR_OOM, "out of host memory");
    b->n = n_members;
    b->precision = precision;
    b->shape = sweep_shape;
    // a graph is captured from a stream of its own; default priority
    if (hip_stream) {
        b->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreate(&b->stream) != hipSuccess) { delete b; return reject(RT3D_ERR_HIP, "hipStreamCreate failed"); }
        b->own_stream = true;
    }
    int rc = RT3D_OK;
    std::string msg;
    b->m.assign(n_members, nullptr);
    for (int i = 0; i < n_members && !rc; ++i) {
        rc = create_ctx(&b->m[i], &descs[i], precision, b->stream, sweep_shape, msg);
        if (rc) msg = "member " + std::to_string(i) + ": " + msg;
    }
    if (!rc) {
        rc = build_tables(b);
        if (rc) msg = b->err;
    }
    if (rc) {
        rt3d_batch_destroy(b);
        return reject(rc, msg);
    }
    b->h_state.assign(n_members, MemberState{});
    *out = b;
    set_thread_error(std::string());
    return RT3D_OK;
}

void rt3d_batch_destroy(rt3d_batch *b)
{
    if (!b) return;
    if (b->stream) hipStreamSynchronize(b->stream);
    free_tables(b);
    for (rt3d_ctx *c : b->m)
        if (c) rt3d_destroy(c);
    if (b->own_stream && b->stream) hipStreamDestroy(b->stream);
    delete b;
}

const char *rt3d_batch_last_error(const rt3d_batch *b) { return b ? b->err.c_str() : thread_error(); }

int rt3d_batch_size(const rt3d_batch *b) { return b ? b->n : 0; }

int rt3d_batch_set_medium(rt3d_batch *b, int member, const double *chi, const double *eps, const double *B,
                          int ptr_kind)
{
    if (!b) return RT3D_ERR_ARG;
    int rc = check_member(b, member);
    if (rc) return rc;
    rc = rt3d_set_medium(b->m[member], chi, eps, B, ptr_kind);
    if (rc) return member_fail(b, member, rc);
    invalidate_tables(b);
    return RT3D_OK;
}

int rt3d_batch_set_J(rt3d_batch *b, int member, const double *J, int ptr_kind)
{
    if (!b) return RT3D_ERR_ARG;
    int rc = check_member(b, member);
    if (rc) return rc;
    rc = rt3d_set_J(b->m[member], J, ptr_kind);
    if (rc) return member_fail(b, member, rc);
    invalidate_tables(b);
    return RT3D_OK;
}

int rt3d_batch_get_J(rt3d_batch *b, int member, double *J_out, int ptr_kind)
{
    if (!b) return RT3D_ERR_ARG;
    int rc = check_member(b, member);
    if (rc) return rc;
    rc = rt3d_get_J(b->m[member], J_out, ptr_kind);
    return rc ? member_fail(b, member, rc) : RT3D_OK;
}

int rt3d_batch_get_Jfs(rt3d_batch *b, int member, double *Jfs_out, int ptr_kind)
{
    if (!b) return RT3D_ERR_ARG;
    int rc = check_member(b, member);
    if (rc) return rc;
    rt3d_ctx *c = b->m[member];
    if (!c->have_fs) return bfail(b, RT3D_ERR_STATE, "no formal solution yet");
    if (!Jfs_out || (ptr_kind != RT3D_HOST && ptr_kind != RT3D_DEVICE)) return bfail(b, RT3D_ERR_ARG, "bad output");
    BHIP_TRY(b, hipMemcpyAsync(Jfs_out, c->Jfs, c->V * sizeof(double), kind_out(ptr_kind), b->stream), "copy J_fs");
    BHIP_TRY(b, hipStreamSynchronize(b->stream), "sync");
    return RT3D_OK;
}

// Either setter replaces the members' acceleration (as on a context, where each frees the other's
// buffers).  The batch runs without acceleration until every member has taken the new setting, so
// that a member failing half-way never leaves the batch pointing at buffers that were freed.
int rt3d_batch_set_acceleration(rt3d_batch *b, int ng_order, int ng_every)
{
    if (!b) return RT3D_ERR_ARG;
    b->ng_order = b->ng_every = 0;
    b->aa_depth = 0;
    invalidate_tables(b);
    for (int i = 0; i < b->n; ++i) {
        const int rc = rt3d_set_acceleration(b->m[i], ng_order, ng_every);
        if (rc) return member_fail(b, i, rc);
    }
    b->ng_order = ng_order;
    b->ng_every = ng_every;
    return RT3D_OK;
}

int rt3d_batch_set_anderson(rt3d_batch *b, int depth)
{
    if (!b) return RT3D_ERR_ARG;
    if (depth < 0 || depth > kAaMaxDepth) return bfail(b, RT3D_ERR_ARG, "depth must be 0..8");
    b->ng_order = b->ng_every = 0;
    b->aa_depth = 0;
    invalidate_tables(b);
    for (int i = 0; i < b->n; ++i) {
        const int rc = rt3d_set_anderson(b->m[i], depth);
        if (rc) return member_fail(b, i, rc);
    }
    b->aa_depth = depth;
    return RT3D_OK;
}

int rt3d_batch_set_sweep_shape(rt3d_batch *b, int shape)
{
    if (!b) return RT3D_ERR_ARG;
    if (shape < 0 || shape >= n_sweep_shapes()) return bfail(b, RT3D_ERR_ARG, "sweep shape out of range");
    invalidate_tables(b);
    for (int i = 0; i < b->n; ++i) {
        const int rc = install_plan(b->m[i], shape);
        if (rc) {
            // members before i already carry the new plan: the batch is unusable until a shape
            // change succeeds
            b->plans_ok = false;
            return member_fail(b, i, rc);
        }
    }
    b->shape = shape;
    b->plans_ok = true;
    return RT3D_OK;
}

// One formal solution of every member from its current J, in one launch per kernel (the FP32 form
// sweeps in float32, as the single-problem formal solution does).
int rt3d_batch_formal_solution(rt3d_batch *b)
{
    if (!b) return RT3D_ERR_ARG;
    TraceRange tr("rt3d_batch_formal_solution");
    for (int i = 0; i < b->n; ++i)
        if (!b->m[i]->have_medium) return bfail(b, RT3D_ERR_STATE, "member " + std::to_string(i) + " has no medium");
    int rc = ensure_tables(b);
    if (rc) return rc;
    const bool f32 = b->precision == RT3D_FP32_SWEEP;
    if (f32)
        hipLaunchKernelGGL(source_kernel_batch<float>, dim3(b->n_planes), dim3(kPlaneThreads), 0, b->stream,
                           b->d_src, b->d_planes, nullptr, 0);
    else
        hipLaunchKernelGGL(source_kernel_batch<double>, dim3(b->n_planes), dim3(kPlaneThreads), 0, b->stream,
                           b->d_src, b->d_planes, nullptr, 0);
    if ((rc = launch_check(b, "source_kernel_batch"))) return rc;
    if ((rc = launch_sweep_batch(b, f32, b->d_sw, nullptr, 0))) return rc;
    if (f32)
        hipLaunchKernelGGL(reduce_kernel_batch<float>, dim3(b->n_pplanes), dim3(kPlaneThreads), 0, b->stream,
                           b->d_red + 2 * b->n, b->d_pplanes, nullptr, 0);
    else
        hipLaunchKernelGGL(reduce_kernel_batch<double>, dim3(b->n_pplanes), dim3(kPlaneThreads), 0, b->stream,
                           b->d_red + 2 * b->n, b->d_pplanes, nullptr, 0);
    if ((rc = launch_check(b, "reduce_kernel_batch"))) return rc;
    BHIP_TRY(b, hipStreamSynchronize(b->stream), "sync");
    for (rt3d_ctx *c : b->m) {
        c->have_fs = true;
        if (f32) c->fp32_sweeps += 1; else c->fp64_sweeps += 1;
    }
    return RT3D_OK;
}

int rt3d_batch_solve(rt3d_batch *b, double tol, int max_iter, int inner_sweeps, int poll_every, int *iters_out,
                     double *final_rel_out, int *status_out)
{
    if (!b) return RT3D_ERR_ARG;
    TraceRange tr("rt3d_batch_solve");
    if (!(tol > 0.0) || max_iter < 1 || inner_sweeps < 1 || poll_every < 1)
        return bfail(b, RT3D_ERR_ARG, "bad tol/max_iter/inner_sweeps/poll_every");
    const int n = b->n;
    const bool f32 = b->precision == RT3D_FP32_SWEEP;
    for (int i = 0; i < n; ++i)
        if (!b->m[i]->have_medium) return bfail(b, RT3D_ERR_STATE, "member " + std::to_string(i) + " has no medium");
    {
        const int rc = build_lstar_batched(b);
        if (rc) return rc;
    }
    // the Ng ring starts from the current iterate; control state from each member's context
    std::vector<MemberState> h(n);
    for (int i = 0; i < n; ++i) {
        rt3d_ctx *c = b->m[i];
        if (b->ng_order > 0)
            BHIP_TRY(b, hipMemcpyAsync(c->ng_hist, c->J, c->V * sizeof(double), hipMemcpyDeviceToDevice, b->stream),
                     "ng history");
        MemberState &s = h[i];
        std::memset(&s, 0, sizeof(s));
        s.active = 1;
        s.status = RT3D_MEMBER_RUNNING;
        s.anchor_valid = c->anchor_valid ? 1 : 0;
        s.force_refresh = c->force_refresh ? 1 : 0;
        s.last_anchored = c->last_step_anchored ? 1 : 0;
        s.nh = b->ng_order > 0 ? 1 : 0;
        s.ng_store = s.ng_newest = -1;
        s.c_last = c->c_last;
        s.da_last = c->da_last;
    }
    int rc = ensure_tables(b);
    if (rc) return rc;
    // the FP32 form's re-anchoring ratio of the members' contexts (read when they were created, so the
    // same for all of them), as a single solve of each member would use it
    const double ratio = b->m[0]->anchor_ratio;
    for (int i = 1; i < n; ++i)
        if (b->m[i]->anchor_ratio != ratio) return bfail(b, RT3D_ERR_ARG, "members differ in their anchoring ratio");
    BatchParams prm{tol, ratio, max_iter, f32 ? 1 : 0, b->ng_order, b->ng_every, b->aa_depth, 0};
    BHIP_TRY(b, hipMemcpyAsync(b->d_state, h.data(), n * sizeof(MemberState), hipMemcpyHostToDevice, b->stream), "state");
    BHIP_TRY(b, hipMemcpyAsync(b->d_params, &prm, sizeof(prm), hipMemcpyHostToDevice, b->stream), "params");
    rc = capture_graph(b, inner_sweeps);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BHIP_TRY(b, hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); return bfail(b, RT3D_ERR_HIP, "hipEventCreate"); }
    hipEventRecord(e0, b->stream);
    b->replays = 0;
    b->polls = 0;
    // every member stops within max_iter iterations, so max_iter replays always suffice
    while (b->replays < max_iter && !rc) {
        for (int r = 0; r < poll_every && b->replays < max_iter; ++r) {
            const hipError_t e = hipGraphLaunch(b->exec, b->stream);
            if (e != hipSuccess) { rc = bfail(b, RT3D_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e)); break; }
            ++b->replays;
        }
        if (rc) break;
        const hipError_t e = hipMemcpyAsync(h.data(), b->d_state, n * sizeof(MemberState), hipMemcpyDeviceToHost, b->stream);
        const hipError_t es = (e == hipSuccess) ? hipStreamSynchronize(b->stream) : e;
        if (es != hipSuccess) { rc = bfail(b, RT3D_ERR_HIP, std::string("poll: ") + hipGetErrorString(es)); break; }
        ++b->polls;
        bool any = false;
        for (int i = 0; i < n; ++i) any = any || h[i].active;
        if (!any) break;
    }
    hipEventRecord(e1, b->stream);
    hipEventSynchronize(e1);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) b->solve_ms = ms;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    b->h_state = h;
    // back into the member contexts, as a single-problem solve leaves them
    int worst = RT3D_OK;
    for (int i = 0; i < n; ++i) {
        rt3d_ctx *c = b->m[i];
        const MemberState &s = h[i];
        c->outer_iters += s.iters;
        c->inner_sweeps += long(s.iters) * inner_sweeps;
        c->c_last = s.c_last;
        c->da_last = s.da_last;
        c->anchor_valid = s.anchor_valid != 0;
        c->force_refresh = s.force_refresh != 0;
        c->last_step_anchored = s.last_anchored != 0;
        if (s.iters > 0) c->have_fs = true;
        const bool nonfinite = s.status == RT3D_MEMBER_NONFINITE;
        if (iters_out) iters_out[i] = s.iters;
        if (final_rel_out) final_rel_out[i] = nonfinite ? NAN : s.c_last;
        if (status_out) status_out[i] = s.status;
        if (nonfinite) worst = RT3D_ERR_NONFINITE;
        else if (s.status != RT3D_MEMBER_CONVERGED && worst == RT3D_OK) worst = RT3D_ERR_NOT_CONVERGED;
    }
    if (worst == RT3D_ERR_NONFINITE) return bfail(b, worst, "NaN or Inf in dJ or J of a member");
    if (worst == RT3D_ERR_NOT_CONVERGED) return bfail(b, worst, "max_iter reached by a member");
    return RT3D_OK;
}

int rt3d_batch_autotune(rt3d_batch *b, const char *cache_path, int repeats, int *shape_out, double *ms_out)
{
    if (!b) return RT3D_ERR_ARG;
    if (repeats < 1) return bfail(b, RT3D_ERR_ARG, "repeats must be >= 1");
    for (int i = 0; i < b->n; ++i)
        if (!b->m[i]->have_medium) return bfail(b, RT3D_ERR_STATE, "member " + std::to_string(i) + " has no medium");
    const int ns = n_sweep_shapes();
    // key: device, precision and the sorted multiset of member grids
    std::vector<std::string> grids;
    for (rt3d_ctx *c : b->m) {
        char t[96];
        std::snprintf(t, sizeof t, "%dx%dx%d/%dx%d", c->g.nx, c->g.ny, c->g.nz, c->g.n_theta, c->g.n_phi);
        grids.push_back(t);
    }
    std::sort(grids.begin(), grids.end());
    std::string key = device_key() + "|batch|" + (b->precision == RT3D_FP64 ? "fp64" : "fp32_sweep") + "|";
    for (size_t i = 0; i < grids.size();) {
        size_t j = i;
        while (j < grids.size() && grids[j] == grids[i]) ++j;
        key += (i ? "," : "") + grids[i] + "*" + std::to_string(j - i);
        i = j;
    }
    int cached = -1;
    if (cache_path && *cache_path && rt3d_tune::lookup(cache_path, key, cached) && cached >= 0 && cached < ns) {
        if (cached != b->shape) {
            const int rc = rt3d_batch_set_sweep_shape(b, cached);
            if (rc) return rc;
        }
        if (shape_out) *shape_out = cached;
        if (ms_out) for (int i = 0; i < ns; ++i) ms_out[i] = -1.0;
        return RT3D_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BHIP_TRY(b, hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); return bfail(b, RT3D_ERR_HIP, "hipEventCreate"); }
    std::vector<double> ms(ns, INFINITY);
    int rc = RT3D_OK;
    for (int s = 0; s < ns && !rc; ++s) {
        const int r = rt3d_batch_set_sweep_shape(b, s);
        if (r == RT3D_ERR_ARG) continue;      // the shape does not fit some member's grid
        if (r) { rc = r; break; }
        rc = rt3d_batch_formal_solution(b);   // warm-up
        if (!rc && hipEventRecord(e0, b->stream) != hipSuccess) rc = bfail(b, RT3D_ERR_HIP, "hipEventRecord");
        for (int k = 0; k < repeats && !rc; ++k) rc = rt3d_batch_formal_solution(b);
        if (!rc && hipEventRecord(e1, b->stream) != hipSuccess) rc = bfail(b, RT3D_ERR_HIP, "hipEventRecord");
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = bfail(b, RT3D_ERR_HIP, "hipEventSynchronize");
        float t = 0.f;
        if (!rc && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms[s] = double(t) / repeats;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    int best = -1;
    for (int s = 0; s < ns; ++s)
        if (std::isfinite(ms[s]) && (best < 0 || ms[s] < ms[best])) best = s;
    if (best < 0) return bfail(b, RT3D_ERR_ARG, "no sweep shape fits every member");
    rc = rt3d_batch_set_sweep_shape(b, best);
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
        if (!rt3d_tune::store(cache_path, key, entry, err)) return bfail(b, RT3D_ERR_ARG, err);
    }
    return RT3D_OK;
}

int rt3d_batch_get_stats(rt3d_batch *b, char *buf, int buflen)
{
    if (!b || !buf || buflen < 2) return RT3D_ERR_ARG;
    long vox = 0, vox_dir = 0, it_min = -1, it_max = 0, it_sum = 0;
    size_t bytes = 0;
    for (int i = 0; i < b->n; ++i) {
        const rt3d_ctx *c = b->m[i];
        vox += c->V;
        vox_dir += c->V * c->A.n_dir;
        bytes += c->device_bytes;
        const long it = b->h_state.empty() ? 0 : b->h_state[i].iters;
        it_min = (it_min < 0 || it < it_min) ? it : it_min;
        it_max = std::max(it_max, it);
        it_sum += it;
    }
    char tmp[768];
    std::snprintf(tmp, sizeof tmp,
                  "{\"members\":%d,\"precision\":\"%s\",\"sweep_shape\":%d,\"sweep_threads\":%d,\"sweep_lines\":%d,"
                  "\"voxels\":%ld,\"voxel_angles\":%ld,\"device_bytes\":%zu,\"sweep_workgroups\":%d,"
                  "\"plane_blocks\":%d,\"graph_inner_sweeps\":%d,\"replays\":%ld,\"polls\":%ld,\"solve_ms\":%.6f,"
                  "\"iters_min\":%ld,\"iters_max\":%ld,\"iters_sum\":%ld}",
                  b->n, b->precision == RT3D_FP64 ? "fp64" : "fp32_sweep", b->shape,
                  b->shape >= 0 ? kSweepShapes[b->shape].threads : 0, b->shape >= 0 ? kSweepShapes[b->shape].lines : 0,
                  vox, vox_dir, bytes, b->n_items, b->n_planes, b->graph_M, b->replays, b->polls, b->solve_ms,
                  it_min < 0 ? 0 : it_min, it_max, it_sum);
    const std::string s = tmp;
    if (int(s.size()) + 1 > buflen) return bfail(b, RT3D_ERR_ARG, "stats buffer too small");
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return RT3D_OK;
}

}  // extern "C"
