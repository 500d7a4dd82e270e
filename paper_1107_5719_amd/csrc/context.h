// context.h -- the context of one problem (grid, angle set, plan, device buffers) and the host
// helpers shared by the single-problem ABI (rt3d.hip) and the batched ABI (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/rt3d.h"
#include "geometry.h"


enum KernelId { K_SOURCE, K_SWEEP, K_REDUCE, K_LSTAR, K_COEF, K_JACOBI, K_COUNT };
constexpr size_t kHistoryMax = 100000;   // step records kept per context
constexpr size_t kScalarBytes = 3 * sizeof(unsigned long long);   // max rel dJ, max distance, flag
// FP32 form: a float64 sweep re-anchors when c < ratio * max|J - Ja|/|J| (the float32 error of a
// difference step scales with the distance travelled since the anchor)
constexpr double kAnchorRatioDefault = 1e-2;
static const char *kKernelNames[K_COUNT] = {"source", "sweep", "reduce", "lstar", "coef", "jacobi"};

struct rt3d_ctx {
    rt3d_grid_desc g{};
    int precision = RT3D_FP64;
    hipStream_t stream = nullptr;
    rt3d::AngleSet A;
    rt3d::SweepPlan plan;
    long V = 0;
    size_t real_size = 8;
    int lstar_early_exit = 0;
    int sweep_shape = 0;       // index into kSweepShapes
    int os_method = RT3D_OS_JACOBI;   // inner solve of the OS step
    double anchor_ratio = kAnchorRatioDefault;   // FP32 form: re-anchor when c < ratio * max|J - Ja|/|J|
    int jacobi_xcd = 4;        // Jacobi grid: 0 plain, 1 chunks padded to 8 per plane, 2 contiguous chunk
                               // ranges per XCD, 3 2D tiles, 4 columns (default) (RT3D_JACOBI_XCD)
    bool jacobi_alternate = true;   // column layout: consecutive sweeps walk the layers in opposite
                                    // orders (RT3D_JACOBI_ALTERNATE=0: always bottom first)
    int jacobi_height = 0;     // column layout: voxels per column, 1, 2 or 4 (0: by grid size;
                               // RT3D_JACOBI_COLUMN)
    int jacobi_walk = -1;      // column layout: odd column layers walk top down (1), never (0), or for
                               // float coefficients in columns of 4 (-1) (RT3D_JACOBI_WALK)
    // device buffers (owned)
    double *chi = nullptr, *eps = nullptr, *B = nullptr, *J = nullptr, *Jfs = nullptr, *r = nullptr;
    double *dJa = nullptr, *dJb = nullptr, *L = nullptr, *Iem = nullptr;
    double *Kc = nullptr, *invD = nullptr, *Ecoef = nullptr;   // Jacobi coefficients (float64 form)
    double *Sbuf = nullptr;
    double *bot_slope = nullptr;        // [ny][nx] LTE-diffusion gradient (bottom_bc 2)
    double *xtab = nullptr;             // [kExpTab] 2^(j/kExpTab) for the float64 exponential of the sweep
    void *cs = nullptr, *P = nullptr;       // sized for float64; float sweeps use the first half
    double *seg_len64 = nullptr;
    float *seg_len32 = nullptr;
    // FP32 form: anchor iterate, its float64 formal solution and top-plane light, float coefficients
    double *Ja = nullptr, *Fa = nullptr, *Iem_a = nullptr;
    float *Kc32 = nullptr;                                     // Jacobi coefficients stored in float32
    int coef_fp32 = 0;          // Jacobi coefficients stored in float32 (Kc32) rather than float64 (Kc)
    unsigned long long *d_maxdist = nullptr;
    bool anchor_valid = false, force_refresh = false, last_step_anchored = false;
    double c_last = INFINITY, da_last = 0.0;
    long fp64_sweeps = 0, fp32_sweeps = 0;
    int *seg_off = nullptr, *seg_n = nullptr, *seg_a = nullptr, *seg_bb = nullptr, *seg_bm = nullptr;
    int *seg_ai = nullptr, *seg_bi = nullptr, *row_min = nullptr;
    rt3d::DirInfo *dirs = nullptr;
    rt3d::PairInfo *pairs = nullptr;
    rt3d::PairSeg *pseg = nullptr;
    rt3d::PairLayer *player = nullptr;
    rt3d::WorkItem *items = nullptr;
    unsigned long long *d_maxrel = nullptr;
    int *d_flag = nullptr;
    unsigned long long *d_scal = nullptr;   // owns d_maxrel, d_maxdist, d_flag (in that order)
    // adjoint (allocated by the first adjoint call): per (direction, layer, line) the intensity entering
    // the layer and the adjoint variable leaving it; per voxel the adjoint iterate nu, its formal
    // solution, residual, right-hand side and the pulled gradient terms
    double *adj_Ient = nullptr, *adj_Qx = nullptr;
    double *adj_nu = nullptr, *adj_fs = nullptr, *adj_r = nullptr, *adj_f = nullptr, *adj_pull = nullptr;
    double *adj_g = nullptr;            // [n_up][ny][nx]: dL/dI_em
    double *adj_qs = nullptr;           // [n_up][ny][nx]: adjoint at the start of upward lines (bottom_bc 2)
    // Anderson mixing (alternative to Ng): rings of the window's OS-step inputs and outputs
    int aa_depth = 0;
    double *aa_x = nullptr, *aa_g = nullptr;   // [aa_depth + 1][V] each
    double *aa_work = nullptr;                 // [kAaWork]
    // Ng acceleration
    int ng_order = 0, ng_every = 0;
    double *ng_hist = nullptr;          // [ng_order + 2][V] ring of iterates
    double *ng_work = nullptr;          // [kNgWork]: block partials, sums, coefficients
    size_t device_bytes = 0;
    size_t plan_bytes = 0;              // the part of device_bytes that belongs to the sweep plan
    bool have_medium = false, have_lstar = false, have_fs = false, plan_ok = false;
    long outer_iters = 0, inner_sweeps = 0;
    // per OS step since the last new medium, new J or start of a solve: max |dJ|/|J|, wall ms,
    // flags (1: float64 formal solution, 2: Ng extrapolation after the step)
    struct StepRecord { double c, ms; int flags; };
    std::vector<StepRecord> history;
    // timing
    int timing = 0;                    // 0 off, 1 every launch, 2 sampled (see rt3d_set_timing)
    struct Pending { int kid; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    double kernel_ms[K_COUNT] = {0};
    long kernel_launches[K_COUNT] = {0};
    long kernel_timed[K_COUNT] = {0};  // launches bracketed by events
    std::string err;
};


namespace rt3d_host {

// A roctx range for the lifetime of the object (shown by rocprofv3 --marker-trace).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

int fail(rt3d_ctx *c, int code, const std::string &msg);
int hip_fail(rt3d_ctx *c, hipError_t e, const char *what);
int sync(rt3d_ctx *c);
int check_launch(rt3d_ctx *c, const char *what);
int ensure_lstar(rt3d_ctx *c);
int finish_lstar(rt3d_ctx *c);
int validate_desc(const rt3d_grid_desc *g, std::string &msg);
int validate_medium_host(long V, const double *chi, const double *eps, const double *B, std::string &msg);
hipMemcpyKind kind_in(int ptr_kind);
hipMemcpyKind kind_out(int ptr_kind);
int n_sweep_shapes();

// New context with the given sweep shape (index into the shape table); stream may be null.
int create_ctx(rt3d_ctx **out, const rt3d_grid_desc *g, int precision, hipStream_t stream, int shape,
               std::string &msg);
// The sweep plan of a grid and angle set for a shape, on the host (no device work); false with the
// reason in msg when the grid does not fit the sweep kernel's line and LDS budgets.
bool build_plan(const rt3d_grid_desc &g, const rt3d::AngleSet &A, int shape, rt3d::SweepPlan &plan,
                std::string &msg);
// (Re)build the sweep plan for a shape (or take the given one) and upload its tables; Lambda* and
// the state are kept.
int install_plan(rt3d_ctx *c, int shape, rt3d::SweepPlan *built = nullptr);
// Message of the calling thread's last failed context or batch creation ("" after a success).
void set_thread_error(const std::string &msg);
const char *thread_error();
// One formal solution from the current J (source, sweep, reduce; no residual), as the context's
// precision sweeps it.
int run_fs_plain(rt3d_ctx *c);
// S (given on the device, or from J when null) -> J_fs (and r = J_fs - J when with_residual).
int run_fs(rt3d_ctx *c, const double *S_dev, bool with_residual, bool fp32);
// Key of a tuning-cache entry: device, precision and grid of a context.
std::string device_key();

#define HIP_TRY(ctx, expr, what)                                      \
    do {                                                              \
        hipError_t e_ = (expr);                                       \
        if (e_ != hipSuccess) return rt3d_host::hip_fail(ctx, e_, what); \
    } while (0)

template <typename T>
int dev_alloc(rt3d_ctx *c, T **p, size_t count)
{
    const size_t bytes = (count ? count : 1) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(c, e, "hipMalloc");
    }
    c->device_bytes += bytes;
    return RT3D_OK;
}

template <typename T>
int upload(rt3d_ctx *c, T **p, const std::vector<T> &h)
{
    int rc = dev_alloc(c, p, h.size());
    if (rc) return rc;
    if (!h.empty()) HIP_TRY(c, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
    return RT3D_OK;
}

}  // namespace rt3d_host
