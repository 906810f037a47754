// Host side of the MI355X multigrid pressure-Poisson solver: level hierarchy,
// V-cycle driver, FP64 defect-correction loop, adjoint, C ABI (include/mgp.h).
#include "mgp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "mgp_kernels.hpp"
#include "mgp_faces.hpp"
#include "mgp_sweep.hpp"
#include "mgp_sweep2.hpp"
#include "mgp_sweep2r.hpp"
#include "mgp_krylov.hpp"
#include "mgp_resid.hpp"
#include "mgp_tail.hpp"
#include "mgp_transfer.hpp"

using namespace mgp;

namespace {

constexpr int kMaxCoarseCells = kCoarseMax;
constexpr int kTimingPairs = 4096;
constexpr int kMaxPartials = 16384;  // partial sums of one reduction (>= blocks of any launch)

template <typename T>
struct LevelBufs {
    T *bx = nullptr, *by = nullptr, *bz = nullptr;  // low-face coefficients
    T *x = nullptr, *t = nullptr, *b = nullptr;     // iterate, ping-pong partner, rhs
};

struct Level {
    Dims d{};
    long n = 0;
    double h = 0.0;
    LevelBufs<double> f64;
    LevelBufs<float> f32;
};

// what one timed launch recorded (MG_FLAG_TIMING)
struct EvSlot {
    int cls, level;
    double bytes;
};

}  // namespace

struct mg_ctx {
    int nlev = 0;
    Level lev[MG_MAX_LEVELS];
    mg_opts opts{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool mixed = false;
    double* G = nullptr;         // coarsest inverse, n_c x n_c
    double* b0 = nullptr;        // projected rhs, finest
    double* ptmp = nullptr;      // ping-pong partner of the caller's p
    double* work = nullptr;      // scratch (verification copies)
    double* fr = nullptr;        // flexible-CG residual, direction and L direction (MG_FLAG_FCG)
    double* fd = nullptr;        // current direction: one of fd_buf
    double* fd_buf[2] = {nullptr, nullptr};
    double* fq = nullptr;
    double* partials = nullptr;  // kReduceBlocks
    double* rho = nullptr;       // cell density (contexts made by mg_setup_density)
    bool use_rho = false;        // finest FP64 passes form coefficients from rho
    double* scal = nullptr;      // device scalars
    double* host_scal = nullptr; // host mirror: pinned (mg_setup) or host_scal_buf (mg_solve_noalloc)
    double host_scal_buf[16];
    bool caller_memory = false;  // context and arena are not the library's to free (mg_solve_noalloc)
    // levels tail_lev..nlev-1 run as one single-workgroup launch (-1: none)
    int tail_lev = -1;
    TailLevel<double>* tail64 = nullptr;  // device tables (arena)
    TailLevel<float>* tail32 = nullptr;
    TailLevel<double> tail64_h[MG_MAX_LEVELS];  // their host images
    TailLevel<float> tail32_h[MG_MAX_LEVELS];
    void* arena = nullptr;
    size_t arena_bytes = 0;
    double setup_ms = 0.0;
    bool valid = false;          // coefficients imported and accepted
    // timing
    hipEvent_t sync_ev = nullptr;  // marks the scalar copy the mixed loop waits for (NULL: wait for the stream)
    hipEvent_t* ev = nullptr;      // 2 * kTimingPairs events and their records (MG_FLAG_TIMING)
    EvSlot* ev_slot = nullptr;
    int ev_used = 0;
    unsigned timing_mask = (1u << MG_K_COUNT) - 1;  // classes timed under MG_FLAG_TIMING
    double kms[MG_K_COUNT], kms0[MG_K_COUNT];
    long long klaunch[MG_K_COUNT], klaunch0[MG_K_COUNT];
    double kbytes[MG_K_COUNT], kbytes0[MG_K_COUNT];
    char err[512];
};

namespace {

thread_local char g_setup_err[512] = "";

void set_err(mg_ctx* c, const char* fmt, ...)
{
    if (!c) return;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
}

#define HIP_TRY(ctx, call)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            set_err((ctx), "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                    __LINE__);                                                              \
            return MG_EHIP;                                                                 \
        }                                                                                   \
    } while (0)

#define CHECK_LAUNCH(ctx) HIP_TRY(ctx, hipGetLastError())

int grid_for(long n)
{
    long g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > kReduceBlocks) g = kReduceBlocks;
    return (int)g;
}

// Grid-stride elementwise kernels without block partials: one element per
// thread, so that every element's loads are in flight at once instead of a few
// per thread at a time.  A dispatch holds at most 2^32 - 1 work-items per
// dimension, so the grid is capped there and the grid-stride loop covers the
// rest (face counts of the largest grids plan() accepts exceed 2^32).
constexpr long kMaxGridBlocks = 0xFFFFFFFFL / kBlock;

constexpr int grid_full(long n)
{
    long g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > kMaxGridBlocks) g = kMaxGridBlocks;
    return (int)g;
}
// 1536 x 1024 x 1024 cells (< 2^31, accepted by plan()) have 4.8e9 faces
static_assert((long)grid_full(3L * 1536 * 1024 * 1024 + 4096L * 1024) * kBlock <= 0xFFFFFFFFL,
              "face-sized grids stay within the dispatch limit");
static_assert(grid_full(1000) == 4 && grid_full(0) == 1, "one element per thread below the cap");

// plan: number of levels; 0 if invalid
int plan(int nx, int ny, int nz, int coarse_max, Dims* out)
{
    if (nx < 1 || ny < 1 || nz < 1 || coarse_max < 1) return 0;
    if ((long)nx * ny * nz >= (1L << 31)) return 0;
    int n = 0;
    for (;;) {
        if (n >= MG_MAX_LEVELS) return 0;
        if (out) out[n] = Dims{nx, ny, nz};
        ++n;
        if (nx <= coarse_max && ny <= coarse_max && nz <= coarse_max) break;
        if ((nx & 1) || (ny & 1) || (nz & 1)) return 0;
        nx /= 2;
        ny /= 2;
        nz /= 2;
    }
    return n;
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// --- timing ---------------------------------------------------------------

// Hands one launch a pair of HIP events when the context times kernels; the
// launch passes them to hipExtLaunchKernelGGL, which stores the kernel's own
// start and end timestamps in them (no marker packets between kernels).  Only
// the tiled kernels are timed (one kernel name per class and precision), on
// every level; the finest level is also totalled on its own.
struct TimedLaunch {
    mg_ctx* c;
    int slot;
    bool on;
    TimedLaunch(mg_ctx* ctx, int level, int k, double bytes, bool tiled = true) : c(ctx), slot(0), on(false)
    {
        if (!c->ev || !tiled || !((c->timing_mask >> k) & 1u) || c->ev_used >= kTimingPairs) return;
        on = true;
        slot = c->ev_used;
        c->ev_slot[slot] = EvSlot{k, level, bytes};
    }
    hipEvent_t start() const { return on ? c->ev[2 * slot] : nullptr; }
    hipEvent_t stop() const { return on ? c->ev[2 * slot + 1] : nullptr; }
    ~TimedLaunch()
    {
        if (on) c->ev_used++;
    }
};

// after a synchronisation: fold the first `ready` recorded event pairs (all of
// them by default) into the totals; later pairs move to the front
void harvest(mg_ctx* c, int ready = -1)
{
    if (ready < 0 || ready > c->ev_used) ready = c->ev_used;
    for (int t = 0; t < ready; ++t) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[2 * t], c->ev[2 * t + 1]) == hipSuccess) {
            const EvSlot& r = c->ev_slot[t];
            c->kms[r.cls] += ms;
            c->klaunch[r.cls] += 1;
            c->kbytes[r.cls] += r.bytes;
            if (r.level == 0) {
                c->kms0[r.cls] += ms;
                c->klaunch0[r.cls] += 1;
                c->kbytes0[r.cls] += r.bytes;
            }
        }
    }
    for (int t = ready; t < c->ev_used; ++t) {
        const int u = t - ready;
        std::swap(c->ev[2 * u], c->ev[2 * t]);
        std::swap(c->ev[2 * u + 1], c->ev[2 * t + 1]);
        c->ev_slot[u] = c->ev_slot[t];
    }
    c->ev_used -= ready;
}

// --- reductions -----------------------------------------------------------

int reduce_to(mg_ctx* c, int nparts, int slot)
{
    k_reduce_final<<<1, kBlock, 0, c->stream>>>(c->partials, nparts, c->scal, slot);
    CHECK_LAUNCH(c);
    return MG_OK;
}

// The same in two halves: queue the copy, then (after queueing more work) wait
// for the copy alone; timing pairs recorded after the copy are kept for later.
int fetch_scalars_begin(mg_ctx* c, int count, int* ready)
{
    HIP_TRY(c, hipMemcpyAsync(c->host_scal, c->scal, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
    if (c->sync_ev) HIP_TRY(c, hipEventRecord(c->sync_ev, c->stream));
    *ready = c->ev_used;
    return MG_OK;
}

// Without an event (mg_solve_noalloc) the wait covers the work queued after the
// copy as well: same results, no overlap of that work with the host's wait.
int fetch_scalars_end(mg_ctx* c, int ready)
{
    if (c->sync_ev) HIP_TRY(c, hipEventSynchronize(c->sync_ev));
    else HIP_TRY(c, hipStreamSynchronize(c->stream));
    harvest(c, ready);
    return MG_OK;
}

int fetch_scalars(mg_ctx* c, int count)
{
    HIP_TRY(c, hipMemcpyAsync(c->host_scal, c->scal, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    harvest(c);
    return MG_OK;
}

// --- level kernels ----------------------------------------------------------

template <typename T>
LevelBufs<T>& bufs(Level& L);
template <>
LevelBufs<double>& bufs<double>(Level& L) { return L.f64; }
template <>
LevelBufs<float>& bufs<float>(Level& L) { return L.f32; }

template <typename T>
int sweep(mg_ctx* c, int l, const T* b, const T* in, T* out, int order, bool zero_in)
{
    Level& L = c->lev[l];
    LevelBufs<T>& B = bufs<T>(L);
    const double bytes = (double)L.n * sweep_bytes_per_cell<T>();
    TimedLaunch tl(c, l, MG_K_SWEEP, bytes, sweep_is_fused(L.d, sizeof(T)));
    const hipError_t e = launch_sweep<T>(B.bx, B.by, B.bz, L.d, (T)(L.h * L.h), b, in, out, order,
                                         zero_in, c->stream, tl.start(), tl.stop());
    if (e != hipSuccess) {
        set_err(c, "sweep launch failed: %s", hipGetErrorString(e));
        return MG_EHIP;
    }
    return MG_OK;
}

// Two sweeps of one order in one launch (grids that sweep2_ok accepts); with
// ec, from in + P ec (the coarse correction of level l + 1 prolongated on the
// fly).
template <typename T>
int sweep_pair(mg_ctx* c, int l, const T* b, const T* in, T* out, int order, bool zero_in, const T* ec = nullptr)
{
    Level& L = c->lev[l];
    LevelBufs<T>& B = bufs<T>(L);
    // algorithmic bytes of the work done: two sweeps, plus (ec) the prolongation + correction pass it replaces
    const double bytes = 2.0 * (double)L.n * sweep_bytes_per_cell<T>() +
                         (ec ? (double)L.n * (2.0 + 1.0 / 8.0) * sizeof(T) : 0.0);
    TimedLaunch tl(c, l, MG_K_SWEEP2, bytes, sweep2_wide(L.d));
    const hipError_t e = launch_sweep2<T>(B.bx, B.by, B.bz, L.d, (T)(L.h * L.h), b, in, out, order, zero_in,
                                          c->stream, tl.start(), tl.stop(), ec);
    if (e != hipSuccess) {
        set_err(c, "sweep launch failed: %s", hipGetErrorString(e));
        return MG_EHIP;
    }
    return MG_OK;
}

// The pre-smoothing pair of level l from a zero iterate (order 0, into out)
// that also writes the restriction of its residual into bc (the rhs of level
// l + 1): the separate residual + restriction pass is not needed.
int sweep_pair_restrict(mg_ctx* c, int l, const float* b, float* out, float* bc)
{
    Level& L = c->lev[l];
    LevelBufs<float>& B = L.f32;
    // algorithmic bytes of the work done: two sweeps, plus the residual + restriction pass it replaces
    const double bytes = 2.0 * (double)L.n * sweep_bytes_per_cell<float>() +
                         (double)L.n * (5.0 + 1.0 / 8.0) * sizeof(float);
    TimedLaunch tl(c, l, MG_K_SWEEP2R, bytes, true);
    const hipError_t e = launch_sweep2_restrict(B.bx, B.by, B.bz, L.d, (float)(L.h * L.h),
                                                (float)(1.0 / (L.h * L.h)), b, out, bc, 0, c->stream, tl.start(),
                                                tl.stop());
    if (e != hipSuccess) {
        set_err(c, "sweep launch failed: %s", hipGetErrorString(e));
        return MG_EHIP;
    }
    return MG_OK;
}

// whether the pre-smoothing of level l runs as one launch with the restriction
bool fused_restrict(const mg_ctx* c, int l)
{
    return c->opts.pre == 2 && l < c->nlev - 1 && !(c->tail_lev >= 0 && l >= c->tail_lev) &&
           !(c->opts.flags & MG_FLAG_LEVEL_LAUNCHES) && sweep2r_ok(c->lev[l].d);
}

// `count` sweeps of one order on level l from *x (zero_in: from 0) with *t as
// the ping-pong partner; on return *x holds the result.  Pairs of sweeps run
// in the two-sweep kernel where the grid allows it.
template <typename T>
int smooth(mg_ctx* c, int l, const T* b, T** x, T** t, int order, int count, bool zero_in)
{
    int done = 0;
    if (sweep2_ok(c->lev[l].d, sizeof(T))) {
        for (; count - done >= 2; done += 2) {
            const int e = sweep_pair<T>(c, l, b, *x, *t, order, zero_in && done == 0);
            if (e != MG_OK) return e;
            std::swap(*x, *t);
        }
    }
    for (; done < count; ++done) {
        const int e = sweep<T>(c, l, b, *x, *t, order, zero_in && done == 0);
        if (e != MG_OK) return e;
        std::swap(*x, *t);
    }
    return MG_OK;
}

// All pre-sweeps of level l from a zero iterate; on return *x holds the result.
// *restricted: the same launch also wrote the restricted residual into the rhs
// of level l + 1 (FP32 levels that fused_restrict accepts).
template <typename T>
int presmooth(mg_ctx* c, int l, const T* b, T** x, T** t, bool* restricted)
{
    *restricted = false;
    if constexpr (sizeof(T) == 4) {
        if (fused_restrict(c, l)) {
            const int e = sweep_pair_restrict(c, l, b, *t, bufs<float>(c->lev[l + 1]).b);
            if (e != MG_OK) return e;
            std::swap(*x, *t);
            *restricted = true;
            return MG_OK;
        }
    }
    return smooth<T>(c, l, b, x, t, 0, c->opts.pre, true);
}

template <typename T>
int residual_restrict(mg_ctx* c, int l, const T* b, const T* x, T* bc)
{
    Level& L = c->lev[l];
    Level& C = c->lev[l + 1];
    LevelBufs<T>& B = bufs<T>(L);
    const bool tiled = res_tiled_ok(L.d, sizeof(T));
    const double arrays = (sizeof(T) == 8 && l == 0 && c->use_rho) ? 3.0 : 5.0;  // x, b, faces or rho
    TimedLaunch tl(c, l, MG_K_RESTRICT, (double)L.n * (arrays + 1.0 / 8.0) * sizeof(T), tiled);
    if (tiled) {
        const ResGeom g = res_geom(L.d);
        if constexpr (sizeof(T) == 8) {
            if (l == 0 && c->use_rho) {
                hipExtLaunchKernelGGL(k_resid<T, RES_RESTRICT, true>, dim3(g.blocks), dim3(kResNT), 0, c->stream,
                                      tl.start(), tl.stop(), 0, B.bx, B.by, B.bz, b, x, (const float*)nullptr, L.d,
                                      (T)(1.0 / (L.h * L.h)), g.zc, g.ntx, g.nty, (T*)nullptr, (float*)nullptr, bc,
                                      (double*)nullptr, (const T*)c->rho);
                CHECK_LAUNCH(c);
                return MG_OK;
            }
        }
        hipExtLaunchKernelGGL(k_resid<T, RES_RESTRICT, false>, dim3(g.blocks), dim3(kResNT), 0, c->stream,
                              tl.start(), tl.stop(), 0, B.bx, B.by, B.bz, b, x, (const float*)nullptr, L.d,
                              (T)(1.0 / (L.h * L.h)), g.zc, g.ntx, g.nty, (T*)nullptr, (float*)nullptr, bc,
                              (double*)nullptr, (const T*)nullptr);
    } else {
        k_residual_restrict<T><<<grid_for(8 * C.n), kBlock, 0, c->stream>>>(B.bx, B.by, B.bz, L.d, C.d,
                                                                           (T)(1.0 / (L.h * L.h)), b, x, bc);
    }
    CHECK_LAUNCH(c);
    return MG_OK;
}

template <typename T>
int prolong_correct(mg_ctx* c, int l, const T* e, T* x)
{
    Level& L = c->lev[l];
    Level& C = c->lev[l + 1];
    const bool tiled = pro_tiled_ok(L.d, sizeof(T));
    TimedLaunch tl(c, l, MG_K_PROLONG, (double)L.n * (2.0 + 1.0 / 8.0) * sizeof(T), tiled);
    if (tiled) {
        const ProGeom g = pro_geom(L.d, C.d);
        hipExtLaunchKernelGGL(k_prolong_tiled<T>, dim3(g.blocks), dim3(kProNT), 0, c->stream, tl.start(), tl.stop(), 0,
                              L.d, C.d, e, x, g.kc, g.ntx, g.nty);
    } else {
        k_prolong_correct<T><<<grid_for(L.n), kBlock, 0, c->stream>>>(L.d, C.d, e, x);
    }
    CHECK_LAUNCH(c);
    return MG_OK;
}

template <typename T>
int coarse_apply(mg_ctx* c, const T* r, T* e)
{
    Level& L = c->lev[c->nlev - 1];
    k_coarse_apply<T><<<1, 64, 0, c->stream>>>(c->G, (int)L.n, r, e);
    CHECK_LAUNCH(c);
    return MG_OK;
}

template <typename T>
TailLevel<T>* tail_tab(mg_ctx* c);
template <>
TailLevel<double>* tail_tab<double>(mg_ctx* c) { return c->tail64; }
template <>
TailLevel<float>* tail_tab<float>(mg_ctx* c) { return c->tail32; }

// The V-cycle from level l (>= tail_lev) down, in one launch; same contract as vcycle().
template <typename T>
int vcycle_tail(mg_ctx* c, int l, T** x, T** t, const T* b, bool zero_init, int pre_done)
{
    const int pre = c->opts.pre, post = c->opts.post;
    long faces = 0;
    for (int k = l; k < c->nlev - 1; ++k) faces += n_fx(c->lev[k].d) + n_fy(c->lev[k].d) + n_fz(c->lev[k].d);
    const int zi = zero_init ? 1 : 0;
    bool p2 = true;  // every level's x and y sizes powers of two: index arithmetic by shifts
    for (int k = l; k < c->nlev; ++k) {
        const Dims& d = c->lev[k].d;
        p2 = p2 && (d.nx & (d.nx - 1)) == 0 && (d.ny & (d.ny - 1)) == 0;
    }
    const bool flds = sizeof(T) == 4 && faces <= kTailFaceLds;
    auto k = flds ? (p2 ? k_vcycle_tail<T, sizeof(T) == 4, true> : k_vcycle_tail<T, sizeof(T) == 4, false>)
                  : (p2 ? k_vcycle_tail<T, false, true> : k_vcycle_tail<T, false, false>);
    k<<<1, kTailNT, 0, c->stream>>>(tail_tab<T>(c), l, c->nlev, c->G, *x, *t, b, pre, post, zi, pre_done);
    CHECK_LAUNCH(c);
    if (((pre - pre_done) + post) & 1) std::swap(*x, *t);
    return MG_OK;
}

template <typename T>
int fill(mg_ctx* c, T* x, long n, T v)
{
    k_fill<T><<<grid_full(n), kBlock, 0, c->stream>>>(x, n, v);
    CHECK_LAUNCH(c);
    return MG_OK;
}

template <typename S, typename D>
int convert(mg_ctx* c, const S* x, long n, D* y)
{
    k_convert<S, D><<<grid_full(n), kBlock, 0, c->stream>>>(x, n, y);
    CHECK_LAUNCH(c);
    return MG_OK;
}

#define TRY(...)                    \
    do {                            \
        int s_ = (__VA_ARGS__);     \
        if (s_ != MG_OK) return s_; \
    } while (0)

// One V-cycle on level l.  *x holds the iterate (zero_init: treat as 0),
// *t is its ping-pong partner; on return *x holds the result (the two
// pointers may have been swapped).  pre_done pre-sweeps have already run
// (by presmooth, when pre_done = pre and zero_init; restricted: that launch
// also wrote the rhs of level l + 1).
template <typename T>
int vcycle(mg_ctx* c, int l, T** x, T** t, const T* b, bool zero_init, int pre_done = 0, bool restricted = false)
{
    Level& L = c->lev[l];
    if (l == c->nlev - 1) return coarse_apply<T>(c, b, *x);
    if (c->tail_lev >= 0 && l >= c->tail_lev) return vcycle_tail<T>(c, l, x, t, b, zero_init, pre_done);
    const int pre = c->opts.pre, post = c->opts.post;
    if (zero_init && pre == 0) TRY(fill<T>(c, *x, L.n, (T)0));
    if (zero_init && pre_done == 0 && pre > 0) TRY(presmooth<T>(c, l, b, x, t, &restricted));
    else TRY(smooth<T>(c, l, b, x, t, 0, pre - pre_done, zero_init && pre_done == 0));
    Level& C = c->lev[l + 1];
    LevelBufs<T>& CB = bufs<T>(C);
    if (!restricted) TRY(residual_restrict<T>(c, l, b, *x, CB.b));
    T* cx = CB.x;
    T* ct = CB.t;
    TRY(vcycle<T>(c, l + 1, &cx, &ct, CB.b, true));
    // the first two-sweep launch of the post-smoothing adds the prolongated correction itself
    if (post >= 2 && sweep2_ok(L.d, sizeof(T)) && !(c->opts.flags & MG_FLAG_LEVEL_LAUNCHES)) {
        TRY(sweep_pair<T>(c, l, b, *x, *t, 1, false, cx));
        std::swap(*x, *t);
        return smooth<T>(c, l, b, x, t, 1, post - 2, false);
    }
    TRY(prolong_correct<T>(c, l, cx, *x));
    TRY(smooth<T>(c, l, b, x, t, 1, post, false));
    return MG_OK;
}

// The first pre-sweep of an FP64 V-cycle on the finest grid (in -> out,
// order 0) that also leaves ||b - L in||^2 in scal[slot]: the residual norm
// of the iterate the cycle starts from.  Only for grids the fused sweep
// kernel covers (sweep_is_fused).
int sweep_first_norm(mg_ctx* c, const double* b, const double* in, double* out, int slot)
{
    Level& L = c->lev[0];
    LevelBufs<double>& B = L.f64;
    int blocks = 0;
    {
        TimedLaunch tl(c, 0, MG_K_NORM, (double)L.n * sweep_bytes_per_cell<double>(), true);
        // 64 x 8 tiles: 1.68 against 1.77 ms at 512^3 with 64 x 16 (the plain sweep is even)
        const hipError_t e = launch_fused<double, 8>(B.bx, B.by, B.bz, L.d, L.h * L.h, b, in, out, 0, false,
                                                      c->stream, c->partials, &blocks, tl.start(), tl.stop());
        if (e != hipSuccess) {
            set_err(c, "sweep launch failed: %s", hipGetErrorString(e));
            return MG_EHIP;
        }
    }
    return reduce_to(c, blocks, slot);
}

int residual_norm_launch(mg_ctx* c, const double* b, const double* p, double* r_out, int slot)
{
    Level& L = c->lev[0];
    const bool tiled = !r_out && res_tiled_ok(L.d, sizeof(double));
    TimedLaunch tl(c, 0, MG_K_NORM, (double)L.n * (c->use_rho ? 3.0 : 5.0) * sizeof(double), tiled);
    if (tiled) {
        const ResGeom g = res_geom(L.d);
        if (c->use_rho)
            hipExtLaunchKernelGGL(k_resid<double, RES_NORM, true>, dim3(g.blocks), dim3(kResNT), 0, c->stream,
                                  tl.start(), tl.stop(), 0, L.f64.bx, L.f64.by, L.f64.bz, b, p,
                                  (const float*)nullptr, L.d, 1.0 / (L.h * L.h), g.zc, g.ntx, g.nty,
                                  (double*)nullptr, (float*)nullptr, (double*)nullptr, c->partials,
                                  (const double*)c->rho);
        else
            hipExtLaunchKernelGGL(k_resid<double, RES_NORM, false>, dim3(g.blocks), dim3(kResNT), 0, c->stream,
                                  tl.start(), tl.stop(), 0, L.f64.bx, L.f64.by, L.f64.bz, b, p,
                                  (const float*)nullptr, L.d, 1.0 / (L.h * L.h), g.zc, g.ntx, g.nty,
                                  (double*)nullptr, (float*)nullptr, (double*)nullptr, c->partials,
                                  (const double*)nullptr);
        CHECK_LAUNCH(c);
        return reduce_to(c, g.blocks, slot);
    }
    k_residual_norm<<<kReduceBlocks, kBlock, 0, c->stream>>>(L.f64.bx, L.f64.by, L.f64.bz, L.d,
                                                             1.0 / (L.h * L.h), b, p, r_out, c->partials);
    CHECK_LAUNCH(c);
    return reduce_to(c, kReduceBlocks, slot);
}

// Mixed-precision outer step on the finest grid: p_out = p_in + e (e FP32, or
// 0 when e is NULL), r32 = (float)(b0 - L p_out), scal[slot] = ||r||^2.
int outer_update(mg_ctx* c, const double* p_in, const float* e, double* p_out, float* r32, int slot)
{
    Level& F = c->lev[0];
    // reads p (unless NULL), b and the faces or rho, e; writes p' and r32
    const double bytes = (double)F.n * ((c->use_rho ? 3 : 5) * 8 - (p_in ? 0 : 8) + (e ? 4 : 0) + 8 + 4);
    const bool tiled = res_tiled_ok(F.d, sizeof(double));
    if (!p_in && !tiled) {
        set_err(c, "internal: a zero iterate needs the tiled outer update");
        return MG_EINVAL;
    }
    TimedLaunch tl(c, 0, MG_K_OUTER, bytes, tiled);
    if (tiled) {
        const ResGeom g = res_geom(F.d);
        if (c->use_rho)
            hipExtLaunchKernelGGL(k_resid<double, RES_OUTER, true>, dim3(g.blocks), dim3(kResNT), 0, c->stream,
                                  tl.start(), tl.stop(), 0, F.f64.bx, F.f64.by, F.f64.bz, c->b0, p_in, e, F.d,
                                  1.0 / (F.h * F.h), g.zc, g.ntx, g.nty, p_out, r32, (double*)nullptr, c->partials,
                                  (const double*)c->rho);
        else
            hipExtLaunchKernelGGL(k_resid<double, RES_OUTER, false>, dim3(g.blocks), dim3(kResNT), 0, c->stream,
                                  tl.start(), tl.stop(), 0, F.f64.bx, F.f64.by, F.f64.bz, c->b0, p_in, e, F.d,
                                  1.0 / (F.h * F.h), g.zc, g.ntx, g.nty, p_out, r32, (double*)nullptr, c->partials,
                                  (const double*)nullptr);
        CHECK_LAUNCH(c);
        return reduce_to(c, g.blocks, slot);
    }
    k_outer_update<<<kReduceBlocks, kBlock, 0, c->stream>>>(F.f64.bx, F.f64.by, F.f64.bz, F.d, 1.0 / (F.h * F.h),
                                                            c->b0, p_in, e, e ? 0 : 1, p_out, r32, c->partials);
    CHECK_LAUNCH(c);
    return reduce_to(c, kReduceBlocks, slot);
}

// ---------------------------------------------------------------------------
// flexible CG preconditioned by one V-cycle (MG_FLAG_FCG)
// ---------------------------------------------------------------------------

constexpr int kSlotRR = 2, kSlotZQ = 6, kSlotDQ = 7, kSlotDR = 8;

template <typename TZ>
int fcg_step(mg_ctx* c, const TZ* z, double* x, float* r32, bool first, double dq_prev)
{
    Level& F = c->lev[0];
    const long n = F.n;
    if (!first) {
        k_fcg_dot<TZ><<<kReduceBlocks, kBlock, 0, c->stream>>>(z, c->fq, n, c->partials);
        CHECK_LAUNCH(c);
        TRY(reduce_to(c, kReduceBlocks, kSlotZQ));
    }
    int nparts = kReduceBlocks;
    if (res_tiled_ok(F.d, sizeof(double)) && 2 * res_geom(F.d).blocks <= kMaxPartials) {
        // d = z - gamma d_prev and q = L d in one tiled pass; d ping-pongs
        // between two buffers because its ring is re-formed from d_prev
        const ResGeom g = res_geom(F.d);
        nparts = g.blocks;
        double* dnew = c->fd == c->fd_buf[0] ? c->fd_buf[1] : c->fd_buf[0];
        if (c->use_rho)
            k_fcg_dir_apply<TZ, true><<<g.blocks, kResNT, 0, c->stream>>>(
                F.f64.bx, F.f64.by, F.f64.bz, z, c->fd, c->fr, F.d, 1.0 / (F.h * F.h), c->scal, kSlotZQ, dq_prev,
                first ? 1 : 0, g.zc, g.ntx, g.nty, dnew, c->fq, c->partials, c->rho);
        else
            k_fcg_dir_apply<TZ><<<g.blocks, kResNT, 0, c->stream>>>(F.f64.bx, F.f64.by, F.f64.bz, z, c->fd, c->fr,
                                                                     F.d, 1.0 / (F.h * F.h), c->scal, kSlotZQ,
                                                                     dq_prev, first ? 1 : 0, g.zc, g.ntx, g.nty, dnew,
                                                                     c->fq, c->partials);
        CHECK_LAUNCH(c);
        c->fd = dnew;
    } else {
        k_fcg_direction<TZ><<<grid_for(n), kBlock, 0, c->stream>>>(z, c->fd, n, c->scal, kSlotZQ, dq_prev,
                                                                    first ? 1 : 0);
        CHECK_LAUNCH(c);
        k_fcg_apply<<<kReduceBlocks, kBlock, 0, c->stream>>>(F.f64.bx, F.f64.by, F.f64.bz, F.d, 1.0 / (F.h * F.h),
                                                             c->fd, c->fr, c->fq, c->partials);
        CHECK_LAUNCH(c);
    }
    TRY(reduce_to(c, nparts, kSlotDQ));
    k_reduce_final<<<1, kBlock, 0, c->stream>>>(c->partials + nparts, nparts, c->scal, kSlotDR);
    CHECK_LAUNCH(c);
    k_fcg_update<<<kReduceBlocks, kBlock, 0, c->stream>>>(x, c->fr, c->fd, c->fq, n, c->scal, kSlotDR, kSlotDQ,
                                                          r32, c->partials);
    CHECK_LAUNCH(c);
    return reduce_to(c, kReduceBlocks, kSlotRR);
}

// Iterates on x (the caller's p) until ||r|| <= tol ||b0||; r is the updated
// residual.  Same statuses and divergence guard as the V-cycle loops.
int fcg_loop(mg_ctx* c, double* x, double bnorm, double tol, bool zero_guess, mg_stats* st, int* cycles_out,
             double* rr_out, int* status_out)
{
    Level& F = c->lev[0];
    const long n = F.n;
    float* r32 = c->mixed ? F.f32.b : nullptr;
    double rr = 1.0;
    if (zero_guess) {
        TRY(fill<double>(c, x, n, 0.0));
        HIP_TRY(c, hipMemcpyAsync(c->fr, c->b0, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    } else {
        TRY(residual_norm_launch(c, c->b0, x, c->fr, kSlotRR));
        TRY(fetch_scalars(c, kSlotRR + 1));
        rr = std::sqrt(c->host_scal[kSlotRR]) / bnorm;
    }
    if (r32) TRY(convert<double, float>(c, c->fr, n, r32));
    if (st) st->hist[0] = rr;
    int status = MG_ENOCONV, it = 0;
    if (!std::isfinite(rr)) status = MG_ENONFINITE;
    else if (rr <= tol) status = MG_OK;
    double best = rr, dq_prev = 0.0;
    // as in the mixed V-cycle loop: the next preconditioner's pre-sweeps are
    // queued while the host waits for the norm, unless it is expected to converge
    const int pre = c->opts.pre;
    bool queued = false, queued_restricted = false;
    double rr_before = -1.0;
    float* zx32 = F.f32.x;
    float* zt32 = F.f32.t;
    double* zx64 = F.f64.x;
    double* zt64 = F.f64.t;
    while (status == MG_ENOCONV && it < c->opts.max_cycles) {
        const bool first = it == 0;
        if (c->mixed) {
            if (!queued) {
                zx32 = F.f32.x;
                zt32 = F.f32.t;
            }
            TRY(vcycle<float>(c, 0, &zx32, &zt32, r32, true, queued ? pre : 0, queued && queued_restricted));
            TRY(fcg_step<float>(c, zx32, x, r32, first, dq_prev));
        } else {
            if (!queued) {
                zx64 = F.f64.x;
                zt64 = F.f64.t;
            }
            TRY(vcycle<double>(c, 0, &zx64, &zt64, c->fr, true, queued ? pre : 0));
            TRY(fcg_step<double>(c, zx64, x, nullptr, first, dq_prev));
        }
        queued = false;
        int ready = 0;
        TRY(fetch_scalars_begin(c, kSlotDR + 1, &ready));
        const double expect = rr_before > 0.0 ? rr * (rr / rr_before) : HUGE_VAL;
        if (pre > 0 && it + 1 < c->opts.max_cycles && expect > 4.0 * tol) {
            if (c->mixed) {
                zx32 = F.f32.x;
                zt32 = F.f32.t;
                TRY(presmooth<float>(c, 0, r32, &zx32, &zt32, &queued_restricted));
            } else {
                zx64 = F.f64.x;
                zt64 = F.f64.t;
                TRY(smooth<double>(c, 0, c->fr, &zx64, &zt64, 0, pre, true));
            }
            queued = true;
        }
        TRY(fetch_scalars_end(c, ready));
        dq_prev = c->host_scal[kSlotDQ];
        ++it;
        rr_before = rr;
        rr = std::sqrt(c->host_scal[kSlotRR]) / bnorm;
        if (st && it < MG_HIST_MAX) st->hist[it] = rr;
        if (!std::isfinite(rr)) { status = MG_ENONFINITE; break; }
        if (rr <= tol) { status = MG_OK; break; }
        best = std::min(best, rr);
        if (rr > 1e3 * best) break;
    }
    *cycles_out = it;
    *rr_out = rr;
    *status_out = status;
    return MG_OK;
}

// ---------------------------------------------------------------------------
// solve driver shared by mg_solve and mg_solve_adjoint
// ---------------------------------------------------------------------------

int check_ctx(mg_ctx* c)
{
    if (!c) return MG_EINVAL;
    HIP_TRY(c, hipSetDevice(c->device));
    return MG_OK;
}

int solve_impl(mg_ctx* c, const double* rhs, double* p, double tol, mg_stats* st)
{
    const double t0 = now_ms();
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->setup_ms = c->setup_ms;
    }
    if (!c->valid) {
        set_err(c, "the context holds rejected face coefficients: call mg_update first");
        return MG_EINVAL;
    }
    if (!rhs || !p || rhs == p) {
        set_err(c, "rhs and p must be distinct non-NULL device pointers");
        return MG_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0) {
        set_err(c, "p must be 16-byte aligned");
        return MG_EINVAL;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        set_err(c, "tol must be finite and > 0 (got %g)", tol);
        return MG_EINVAL;
    }
    for (int k = 0; k < MG_K_COUNT; ++k) {
        c->kms[k] = c->kms0[k] = 0;
        c->klaunch[k] = c->klaunch0[k] = 0;
        c->kbytes[k] = c->kbytes0[k] = 0;
    }
    c->ev_used = 0;
    Level& F = c->lev[0];
    const long n = F.n;
    const bool zero_guess = (c->opts.flags & MG_FLAG_ZERO_GUESS) != 0;

    // b0 = rhs - mean(rhs); ||b0||^2.  A mixed solve from p = 0 starts from the
    // FP32 residual b0 (L 0 = 0 exactly): the same pass writes it.
    const bool cast_b0 = c->mixed && zero_guess && !(c->opts.flags & MG_FLAG_FCG) &&
                         res_tiled_ok(F.d, sizeof(double));
    k_sum<double><<<kReduceBlocks, kBlock, 0, c->stream>>>(rhs, n, c->partials);
    CHECK_LAUNCH(c);
    TRY(reduce_to(c, kReduceBlocks, 0));
    if (cast_b0)
        k_sub_scalar_norm<true><<<kReduceBlocks, kBlock, 0, c->stream>>>(rhs, n, c->scal, 0, 1.0 / (double)n,
                                                                         c->b0, F.f32.b, c->partials);
    else
        k_sub_scalar_norm<false><<<kReduceBlocks, kBlock, 0, c->stream>>>(rhs, n, c->scal, 0, 1.0 / (double)n,
                                                                          c->b0, nullptr, c->partials);
    CHECK_LAUNCH(c);
    TRY(reduce_to(c, kReduceBlocks, 1));
    TRY(fetch_scalars(c, 2));
    const double mu = c->host_scal[0] / (double)n;
    const double bnorm = std::sqrt(c->host_scal[1]);
    if (st) st->rhs_mean_removed = mu;
    if (!std::isfinite(bnorm) || !std::isfinite(mu)) {
        set_err(c, "right-hand side holds NaN or Inf");
        if (st) st->status = MG_ENONFINITE;
        return MG_ENONFINITE;
    }
    if (bnorm == 0.0) {
        TRY(fill<double>(c, p, n, 0.0));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (st) {
            st->solve_ms = now_ms() - t0;
            st->status = MG_OK;
        }
        return MG_OK;
    }

    const int maxc = c->opts.max_cycles;
    double rr = 1.0, best = 1.0;
    int cycles = 0, status = MG_ENOCONV;
    double* cur = p;        // buffer holding the current iterate
    double* other = c->ptmp;

    if (c->opts.flags & MG_FLAG_FCG) {
        TRY(fcg_loop(c, cur, bnorm, tol, zero_guess, st, &cycles, &rr, &status));
    } else if (!c->mixed) {
        // The residual norm of each iterate is taken by the sweep that starts
        // the next cycle (it reads exactly the residual's inputs): one pass
        // fewer per cycle; when the norm says stop, that sweep's output is
        // dropped.  Grids the fused sweep does not cover use a separate pass.
        // Where the pre-sweeps run as pairs in the two-sweep kernel, an even count
        // of them stays in pairs and the norm takes a residual pass of its own.
        const bool pairs = sweep2_ok(c->lev[0].d, sizeof(double)) && c->opts.pre % 2 == 0;
        const bool fuse = c->opts.pre > 0 && !pairs && sweep_is_fused(c->lev[0].d, sizeof(double)) &&
                          fused_geom<8>(c->lev[0].d).blocks <= kMaxPartials;
        bool known = zero_guess;  // the rr of the current iterate is known (1 for p = 0)
        bool swept = false;       // the next cycle's first pre-sweep has run (into `other`)
        rr = 1.0;
        if (st) st->hist[0] = rr;
        while (true) {
            if (!known) {
                if (fuse) {
                    TRY(sweep_first_norm(c, c->b0, cur, other, 2));
                    swept = true;
                } else {
                    TRY(residual_norm_launch(c, c->b0, cur, nullptr, 2));
                }
                TRY(fetch_scalars(c, 3));
                rr = std::sqrt(c->host_scal[2]) / bnorm;
                if (st && cycles < MG_HIST_MAX) st->hist[cycles] = rr;
            }
            if (!std::isfinite(rr)) { status = MG_ENONFINITE; break; }
            if (rr <= tol) { status = MG_OK; break; }
            if (cycles == 0) best = rr;
            best = std::min(best, rr);
            if (rr > 1e3 * best || cycles >= maxc) break;
            if (swept) {
                std::swap(cur, other);
                TRY(vcycle<double>(c, 0, &cur, &other, c->b0, false, 1));
            } else {
                TRY(vcycle<double>(c, 0, &cur, &other, c->b0, zero_guess && cycles == 0));
            }
            swept = false;
            known = false;
            ++cycles;
        }
    } else {
        Level& F0 = c->lev[0];
        float* r32 = F0.f32.b;
        // initial residual in FP64, cast to FP32.  From p = 0 it is b0 itself
        // (L 0 = 0 exactly) and rr = 1: a cast, and the first update reads no p.
        bool p_zero = false;
        if (cast_b0) {  // r32 = b0, written with it
            rr = 1.0;
            p_zero = true;
        } else {
            if (zero_guess) TRY(fill<double>(c, cur, n, 0.0));
            TRY(outer_update(c, cur, nullptr, other, r32, 2));
            std::swap(cur, other);
            TRY(fetch_scalars(c, 3));
            rr = std::sqrt(c->host_scal[2]) / bnorm;
        }
        if (st) st->hist[0] = rr;
        best = rr;
        if (!std::isfinite(rr)) status = MG_ENONFINITE;
        else if (rr <= tol) status = MG_OK;
        // While the host waits for a cycle's norm, the next cycle's pre-sweeps are
        // already queued (they read only the new FP32 residual and write the
        // correction buffers, never p), so the GPU does not idle through the
        // round trip.  They are skipped when the norm is expected to meet the
        // tolerance: rr_k ~ rr_{k-1}^2 / rr_{k-2}, with a margin of 4.
        const int pre = c->opts.pre;
        bool queued = false, queued_restricted = false;
        double rr_before = -1.0;
        float* ex = F0.f32.x;
        float* et = F0.f32.t;
        while (status == MG_ENOCONV && cycles < maxc) {
            if (queued) {
                TRY(vcycle<float>(c, 0, &ex, &et, r32, true, pre, queued_restricted));
            } else {
                ex = F0.f32.x;
                et = F0.f32.t;
                TRY(vcycle<float>(c, 0, &ex, &et, r32, true));
            }
            queued = false;
            TRY(outer_update(c, p_zero ? nullptr : cur, ex, other, r32, 2));
            p_zero = false;
            std::swap(cur, other);
            ++cycles;
            int ready = 0;
            TRY(fetch_scalars_begin(c, 3, &ready));
            const double expect = rr_before > 0.0 ? rr * (rr / rr_before) : HUGE_VAL;
            if (pre > 0 && cycles < maxc && expect > 4.0 * tol) {
                ex = F0.f32.x;
                et = F0.f32.t;
                TRY(presmooth<float>(c, 0, r32, &ex, &et, &queued_restricted));
                queued = true;
            }
            TRY(fetch_scalars_end(c, ready));
            rr_before = rr;
            rr = std::sqrt(c->host_scal[2]) / bnorm;
            if (st && cycles < MG_HIST_MAX) st->hist[cycles] = rr;
            if (!std::isfinite(rr)) { status = MG_ENONFINITE; break; }
            if (rr <= tol) { status = MG_OK; break; }
            best = std::min(best, rr);
            if (rr > 1e3 * best) break;
        }
        if (p_zero) TRY(fill<double>(c, cur, n, 0.0));  // stopped before any update: p = 0
    }

    // zero-mean result in the caller's buffer
    k_sum<double><<<kReduceBlocks, kBlock, 0, c->stream>>>(cur, n, c->partials);
    CHECK_LAUNCH(c);
    TRY(reduce_to(c, kReduceBlocks, 3));
    if (cur != p) HIP_TRY(c, hipMemcpyAsync(p, cur, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    k_sub_scalar<<<grid_full(n), kBlock, 0, c->stream>>>(p, n, c->scal, 3, 1.0 / (double)n);
    CHECK_LAUNCH(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    harvest(c);

    if (status == MG_ENOCONV) set_err(c, "no convergence after %d cycles (rel. residual %.3e)", cycles, rr);
    if (status == MG_ENONFINITE) set_err(c, "non-finite residual norm after %d cycles", cycles);
    if (st) {
        st->cycles = cycles;
        st->status = status;
        st->rel_res = rr;
        st->solve_ms = now_ms() - t0;
        for (int k = 0; k < MG_K_COUNT; ++k) {
            st->kernel_ms[k] = c->kms[k];
            st->kernel_launches[k] = c->klaunch[k];
            st->kernel_bytes[k] = c->kbytes[k];
            st->kernel_ms_finest[k] = c->kms0[k];
            st->kernel_launches_finest[k] = c->klaunch0[k];
            st->kernel_bytes_finest[k] = c->kbytes0[k];
        }
    }
    return status;
}

void free_ctx(mg_ctx* c)
{
    if (!c || c->caller_memory) return;
    if (c->ev) {
        for (int t = 0; t < 2 * kTimingPairs; ++t)
            if (c->ev[t]) (void)hipEventDestroy(c->ev[t]);
        delete[] c->ev;
    }
    delete[] c->ev_slot;
    if (c->sync_ev) (void)hipEventDestroy(c->sync_ev);
    if (c->arena) (void)hipFree(c->arena);
    if (c->host_scal) (void)hipHostFree(c->host_scal);
    delete c;
}

// bump allocator over one device arena
struct Arena {
    char* base;
    size_t off;
    size_t cap;
    template <typename T>
    T* take(long count)
    {
        const size_t bytes = ((size_t)count * sizeof(T) + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

void carve(mg_ctx* c, Arena& a)
{
    const long n0 = c->lev[0].n;
    c->b0 = a.take<double>(n0);
    c->ptmp = a.take<double>(n0);
    const long nc = c->lev[c->nlev - 1].n;
    c->G = a.take<double>(nc * nc);
    c->work = a.take<double>(n0);
    c->partials = a.take<double>(kMaxPartials);
    c->scal = a.take<double>(16);
    c->tail64 = a.take<TailLevel<double>>(MG_MAX_LEVELS);
    if (c->mixed) c->tail32 = a.take<TailLevel<float>>(MG_MAX_LEVELS);
    if (c->use_rho) c->rho = a.take<double>(n0);
    if (c->opts.flags & MG_FLAG_FCG) {
        c->fr = a.take<double>(n0);
        c->fd_buf[0] = a.take<double>(n0);
        c->fd_buf[1] = a.take<double>(n0);
        c->fd = c->fd_buf[0];
        c->fq = a.take<double>(n0);
    }
    for (int l = 0; l < c->nlev; ++l) {
        Level& L = c->lev[l];
        L.f64.bx = a.take<double>(n_fx(L.d));
        L.f64.by = a.take<double>(n_fy(L.d));
        L.f64.bz = a.take<double>(n_fz(L.d));
        L.f64.x = a.take<double>(L.n);
        L.f64.t = a.take<double>(L.n);
        L.f64.b = a.take<double>(L.n);
        if (c->mixed) {
            L.f32.bx = a.take<float>(n_fx(L.d));
            L.f32.by = a.take<float>(n_fy(L.d));
            L.f32.bz = a.take<float>(n_fz(L.d));
            L.f32.x = a.take<float>(L.n);
            L.f32.t = a.take<float>(L.n);
            L.f32.b = a.take<float>(L.n);
        }
    }
}

// First level of the single-workgroup tail: the deepest run of levels, ending
// at the coarsest, that have at most kTailCells cells and that no tiled kernel
// serves in either precision (so the tail repeats exactly the per-level
// kernels), and that fit its LDS together.  -1 if that run is the coarsest
// level alone or MG_FLAG_LEVEL_LAUNCHES asks for one launch per kernel.
int tail_start(const mg_ctx* c)
{
    if (c->opts.flags & MG_FLAG_LEVEL_LAUNCHES) return -1;
    int l0 = c->nlev;
    for (int l = c->nlev - 1; l >= 0; --l) {
        const Dims& d = c->lev[l].d;
        const bool simple = c->lev[l].n <= kTailCells && !sweep_is_fused(d, 4) && !sweep_is_fused(d, 8) &&
                            !sweep2_ok(d, 4) && !sweep2_ok(d, 8) && !res_tiled_ok(d, 4) && !res_tiled_ok(d, 8) &&
                            !pro_tiled_ok(d, 4) &&
                            !pro_tiled_ok(d, 8);
        if (!simple) break;
        l0 = l;
    }
    long cells = 0;
    for (int l = l0; l < c->nlev; ++l) cells += c->lev[l].n;
    if (cells > kTailLds || c->nlev - l0 > kTailMaxLevels) return -1;
    return l0 < c->nlev - 1 ? l0 : -1;
}

// The tail's level tables (their buffers never move after carve()).
int upload_tail(mg_ctx* c)
{
    c->tail_lev = tail_start(c);
    if (c->tail_lev < 0) return MG_OK;
    for (int l = 0; l < c->nlev; ++l) {
        const Level& L = c->lev[l];
        const double h2 = L.h * L.h;
        c->tail64_h[l] = {L.f64.bx, L.f64.by, L.f64.bz, L.d, h2, 1.0 / h2};
        if (c->mixed) c->tail32_h[l] = {L.f32.bx, L.f32.by, L.f32.bz, L.d, (float)h2, (float)(1.0 / h2)};
    }
    HIP_TRY(c, hipMemcpyAsync(c->tail64, c->tail64_h, sizeof(c->tail64_h), hipMemcpyHostToDevice, c->stream));
    if (c->mixed)
        HIP_TRY(c, hipMemcpyAsync(c->tail32, c->tail32_h, sizeof(c->tail32_h), hipMemcpyHostToDevice, c->stream));
    return MG_OK;
}

// Finest-level coefficients from the caller's faces, or (rho != NULL) from a
// cell density copied into the context; then the coarse levels, the FP32
// copies and the coarsest inverse.
int setup_impl(mg_ctx* c, const double* pbx, const double* pby, const double* pbz, const double* rho = nullptr)
{
    Level& F = c->lev[0];
    // up to one face per thread; one partial count of bad faces per block
    const long faces = n_fx(F.d) + n_fy(F.d) + n_fz(F.d);
    int nb = (int)std::min<long>((faces + kBlock - 1) / kBlock, kMaxPartials);
    // every level's FP32 coefficient copies (mixed precision) are written by the
    // pass that forms the FP64 ones
    float* f32x = c->mixed ? F.f32.bx : nullptr;
    float* f32y = c->mixed ? F.f32.by : nullptr;
    float* f32z = c->mixed ? F.f32.bz : nullptr;
    if (rho) {
        // the pass that forms the faces also keeps the context's copy of rho
        const MarchGeom g = march_geom(F.d, kMaxPartials);
        nb = g.blocks;
        k_faces_march<<<g.blocks, kMarchTX * kMarchTY, 0, c->stream>>>(
            DensityFaceOp<true>{rho, c->rho}, F.d, F.d.nx + 2, g.zc, g.ntx, g.nty, g.ntiles, F.f64.bx, F.f64.by,
            F.f64.bz, c->partials, f32x, f32y, f32z);
    } else {
        k_import_faces<<<nb, kBlock, 0, c->stream>>>(pbx, pby, pbz, F.d, F.f64.bx, F.f64.by, F.f64.bz, c->partials,
                                                     f32x, f32y, f32z);
    }
    c->use_rho = rho != nullptr;
    CHECK_LAUNCH(c);
    TRY(reduce_to(c, nb, 4));
    for (int l = 1; l < c->nlev; ++l) {
        Level& A = c->lev[l - 1];
        Level& B = c->lev[l];
        const long nf = n_fx(B.d) + n_fy(B.d) + n_fz(B.d);
        k_coarsen_faces<<<grid_full(nf), kBlock, 0, c->stream>>>(
            A.f64.bx, A.f64.by, A.f64.bz, A.d, B.d, B.f64.bx, B.f64.by, B.f64.bz, c->mixed ? B.f32.bx : nullptr,
            c->mixed ? B.f32.by : nullptr, c->mixed ? B.f32.bz : nullptr);
        CHECK_LAUNCH(c);
    }
    Level& Cl = c->lev[c->nlev - 1];
    k_coarse_inverse<<<1, kCoarseNT, 0, c->stream>>>(Cl.f64.bx, Cl.f64.by, Cl.f64.bz, Cl.d, Cl.h, c->G,
                                                  c->scal + 5);
    CHECK_LAUNCH(c);
    TRY(fetch_scalars(c, 6));
    if (c->host_scal[4] != 0.0) {
        set_err(c, rho ? "%.0f interior face(s) with a density or coefficient that is not finite and > 0"
                       : "%.0f interior face coefficient(s) are not finite and > 0",
                c->host_scal[4]);
        return MG_EINVAL;
    }
    if (c->host_scal[5] != 0.0) {
        set_err(c, "coarsest-grid bordered matrix is singular");
        return MG_EINVAL;
    }
    return MG_OK;
}

mg_ctx* as_ctx(const mg_ctx* c) { return const_cast<mg_ctx*>(c); }

int level_ok(mg_ctx* c, int level, int precision)
{
    if (level < 0 || level >= c->nlev) {
        set_err(c, "level %d out of range [0, %d)", level, c->nlev);
        return MG_EINVAL;
    }
    if (precision != MG_PREC_FP64 && precision != MG_PREC_MIXED) {
        set_err(c, "precision must be MG_PREC_FP64 or MG_PREC_MIXED");
        return MG_EINVAL;
    }
    if (precision == MG_PREC_MIXED && !c->mixed) {
        set_err(c, "FP32 kernels need a context set up with MG_PREC_MIXED");
        return MG_EINVAL;
    }
    return MG_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int mg_plan_levels(const int dims[3], int coarse_max)
{
    if (!dims) return 0;
    return plan(dims[0], dims[1], dims[2], coarse_max, nullptr);
}

}  // extern "C"

namespace {

// Memory a context is built in when the library may not allocate
// (mg_solve_noalloc): the host context and a device arena of `cap` bytes.
struct CallerMemory {
    mg_ctx* host;
    void* arena;
    size_t cap;
};

// mg_setup (rho == NULL) and mg_setup_density (faces NULL); with mem, in that
// memory, without any allocation
int setup_ctx(mg_ctx** out, const double* beta_x, const double* beta_y, const double* beta_z, const double* rho,
              const int dims[3], double h, int bc, const mg_opts* opts, void* hip_stream,
              const CallerMemory* mem = nullptr)
{
    if (!out) return MG_EINVAL;
    *out = nullptr;
    const double t0 = now_ms();
    mg_ctx* c = mem ? new (mem->host) mg_ctx() : new (std::nothrow) mg_ctx();
    if (!c) return MG_ENOMEM;
    c->caller_memory = mem != nullptr;
    c->err[0] = 0;
    c->opts = opts ? *opts : mg_opts{2, 2, 100, 4, MG_PREC_FP64, 0};
    const mg_opts& o = c->opts;
    g_setup_err[0] = 0;
    auto fail = [&](int status) {
        std::snprintf(g_setup_err, sizeof(g_setup_err), "%s", c->err);
        free_ctx(c);
        return status;
    };
    if ((!rho && (!beta_x || !beta_y || !beta_z)) || !dims) {
        set_err(c, "NULL argument");
        return fail(MG_EINVAL);
    }
    c->use_rho = rho != nullptr;  // carve() then reserves the density copy
    if (bc != MG_BC_NEUMANN) {
        set_err(c, "only MG_BC_NEUMANN is supported");
        return fail(MG_EINVAL);
    }
    if (!(h > 0.0) || !std::isfinite(h)) {
        set_err(c, "h must be finite and > 0");
        return fail(MG_EINVAL);
    }
    if (o.pre < 0 || o.pre > 8 || o.post < 0 || o.post > 8 || o.pre + o.post == 0 || o.max_cycles < 1 ||
        o.max_cycles >= MG_HIST_MAX || o.coarse_max < 1 || o.coarse_max > 4 ||
        (o.precision != MG_PREC_FP64 && o.precision != MG_PREC_MIXED) ||
        (o.flags & ~(MG_FLAG_ZERO_GUESS | MG_FLAG_TIMING | MG_FLAG_FCG | MG_FLAG_LEVEL_LAUNCHES))) {
        set_err(c, "invalid options");
        return fail(MG_EINVAL);
    }
    if (mem && (o.flags & MG_FLAG_TIMING)) {
        set_err(c, "MG_FLAG_TIMING creates events: not available without allocation");
        return fail(MG_EINVAL);
    }
    Dims ds[MG_MAX_LEVELS];
    const int nlev = plan(dims[0], dims[1], dims[2], o.coarse_max, ds);
    if (nlev == 0) {
        set_err(c, "dims %d x %d x %d cannot be coarsened to <= %d per dimension by halving", dims[0], dims[1],
                dims[2], o.coarse_max);
        return fail(MG_EINVAL);
    }
    c->nlev = nlev;
    c->mixed = o.precision == MG_PREC_MIXED;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    double hl = h;
    for (int l = 0; l < nlev; ++l) {
        c->lev[l].d = ds[l];
        c->lev[l].n = (long)ds[l].nx * ds[l].ny * ds[l].nz;
        c->lev[l].h = hl;
        hl *= 2.0;
    }
    if (c->lev[nlev - 1].n > kMaxCoarseCells) {
        set_err(c, "coarsest grid has more than %d cells", kMaxCoarseCells);
        return fail(MG_EINVAL);
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        set_err(c, "no HIP device");
        return fail(MG_EHIP);
    }
    Arena sizing{nullptr, 0, 0};
    carve(c, sizing);
    c->arena_bytes = sizing.off;
    if (mem) {
        if (c->arena_bytes > mem->cap) {
            set_err(c, "a %d x %d x %d grid needs %zu bytes of device scratch with these options; the "
                       "no-allocation buffer holds %zu",
                    dims[0], dims[1], dims[2], c->arena_bytes, mem->cap);
            return fail(MG_EINVAL);
        }
        c->arena = mem->arena;
    } else if (hipMalloc(&c->arena, c->arena_bytes) != hipSuccess) {
        set_err(c, "hipMalloc of %zu bytes failed", c->arena_bytes);
        (void)hipGetLastError();
        return fail(MG_ENOMEM);
    }
    Arena a{static_cast<char*>(c->arena), 0, c->arena_bytes};
    carve(c, a);
    if (mem) {
        // pageable mirror and no event: the scalar reads wait for the stream
        c->host_scal = c->host_scal_buf;
    } else {
        if (hipHostMalloc(reinterpret_cast<void**>(&c->host_scal), sizeof(double) * 16, hipHostMallocDefault) !=
            hipSuccess) {
            set_err(c, "pinned host allocation failed");
            return fail(MG_ENOMEM);
        }
        if (hipEventCreateWithFlags(&c->sync_ev, hipEventDisableTiming) != hipSuccess) {
            set_err(c, "hipEventCreate failed");
            return fail(MG_EHIP);
        }
    }
    if (o.flags & MG_FLAG_TIMING) {
        c->ev = new (std::nothrow) hipEvent_t[2 * kTimingPairs]();
        c->ev_slot = new (std::nothrow) EvSlot[kTimingPairs];
        if (!c->ev || !c->ev_slot) return fail(MG_ENOMEM);
        // timing-only events: no system-scope fence (cache write-back and
        // invalidate) at each record, which would stall the next kernel; they are
        // read only after the stream has been synchronised
        for (int t = 0; t < 2 * kTimingPairs; ++t)
            if (hipEventCreateWithFlags(&c->ev[t], hipEventDisableSystemFence) != hipSuccess) {
                set_err(c, "hipEventCreate failed");
                return fail(MG_EHIP);
            }
    }
    const int su = upload_tail(c);
    if (su != MG_OK) return fail(su);
    const int st = setup_impl(c, beta_x, beta_y, beta_z, rho);
    if (st != MG_OK) return fail(st);
    c->valid = true;
    c->setup_ms = now_ms() - t0;
    *out = c;
    return MG_OK;
}

}  // namespace

extern "C" {

int mg_setup(mg_ctx** out, const double* beta_x, const double* beta_y, const double* beta_z, const int dims[3],
             double h, int bc, const mg_opts* opts, void* hip_stream)
{
    return setup_ctx(out, beta_x, beta_y, beta_z, nullptr, dims, h, bc, opts, hip_stream);
}

int mg_setup_density(mg_ctx** out, const double* rho, const int dims[3], double h, int bc, const mg_opts* opts,
                     void* hip_stream)
{
    return setup_ctx(out, nullptr, nullptr, nullptr, rho, dims, h, bc, opts, hip_stream);
}

int mg_update_density(mg_ctx* c, const double* rho)
{
    TRY(check_ctx(c));
    if (!rho) {
        set_err(c, "NULL argument");
        return MG_EINVAL;
    }
    if (!c->rho) {
        set_err(c, "the context was not set up from a density (mg_setup_density)");
        return MG_EINVAL;
    }
    const double t0 = now_ms();
    c->valid = false;
    TRY(setup_impl(c, nullptr, nullptr, nullptr, rho));
    c->valid = true;
    c->setup_ms = now_ms() - t0;
    return MG_OK;
}

int mg_update(mg_ctx* c, const double* beta_x, const double* beta_y, const double* beta_z)
{
    TRY(check_ctx(c));
    if (!beta_x || !beta_y || !beta_z) {
        set_err(c, "NULL argument");
        return MG_EINVAL;
    }
    const double t0 = now_ms();
    c->valid = false;
    TRY(setup_impl(c, beta_x, beta_y, beta_z));
    c->valid = true;
    c->setup_ms = now_ms() - t0;
    return MG_OK;
}

int mg_set_timing_classes(mg_ctx* c, unsigned mask)
{
    TRY(check_ctx(c));
    if (!c->ev) {
        set_err(c, "the context was set up without MG_FLAG_TIMING");
        return MG_EINVAL;
    }
    if (mask >> MG_K_COUNT) {
        set_err(c, "timing class mask 0x%x has bits beyond MG_K_COUNT", mask);
        return MG_EINVAL;
    }
    c->timing_mask = mask;
    return MG_OK;
}

int mg_solve(mg_ctx* c, const double* rhs, double* p, double tol, mg_stats* st)
{
    TRY(check_ctx(c));
    return solve_impl(c, rhs, p, tol, st);
}

int mg_solve_adjoint(mg_ctx* c, const double* g, double* lambda, double tol, mg_stats* st)
{
    TRY(check_ctx(c));
    return solve_impl(c, g, lambda, tol, st);
}

int mg_face_grad(mg_ctx* c, const double* lambda, const double* p, double* g_x, double* g_y, double* g_z)
{
    TRY(check_ctx(c));
    if (!c->valid) {
        set_err(c, "the context holds rejected face coefficients: call mg_update first");
        return MG_EINVAL;
    }
    if (!lambda || !p || !g_x || !g_y || !g_z) {
        set_err(c, "NULL argument");
        return MG_EINVAL;
    }
    Level& F = c->lev[0];
    const MarchGeom g = march_geom(F.d, kMaxGridBlocks);
    k_faces_march<<<g.blocks, kMarchTX * kMarchTY, 0, c->stream>>>(FaceGradOp{lambda, p, 1.0 / (F.h * F.h)}, F.d,
                                                                    F.d.nx + 1, g.zc, g.ntx, g.nty, g.ntiles, g_x,
                                                                    g_y, g_z, nullptr);
    CHECK_LAUNCH(c);
    return MG_OK;
}

int mg_apply(mg_ctx* c, const double* x, double* y)
{
    TRY(check_ctx(c));
    if (!x || !y || x == y) {
        set_err(c, "x and y must be distinct non-NULL device pointers");
        return MG_EINVAL;
    }
    Level& F = c->lev[0];
    k_apply<<<grid_for(F.n), kBlock, 0, c->stream>>>(F.f64.bx, F.f64.by, F.f64.bz, F.d, 1.0 / (F.h * F.h), x, y);
    CHECK_LAUNCH(c);
    return MG_OK;
}

void mg_destroy(mg_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_ctx(c);
}

const char* mg_last_error(const mg_ctx* c)
{
    if (!c) return g_setup_err;
    return c->err;
}

int mg_faces_from_vof(const double* f_drop, const double* f_film, const int dims[3], double rho_drop,
                      double rho_film, double rho_gas, double* beta_x, double* beta_y, double* beta_z,
                      void* hip_stream)
{
    if (!f_drop || !f_film || !dims || !beta_x || !beta_y || !beta_z) return MG_EINVAL;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return MG_EINVAL;
    if (!(rho_drop > 0) || !(rho_film > 0) || !(rho_gas > 0)) return MG_EINVAL;
    const Dims d{dims[0], dims[1], dims[2]};
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const MarchGeom g = march_geom(d, kMaxGridBlocks);
    k_faces_march<<<g.blocks, kMarchTX * kMarchTY, 0, s>>>(VofFaceOp{f_drop, f_film, rho_drop, rho_film, rho_gas}, d,
                                                            d.nx + 1, g.zc, g.ntx, g.nty, g.ntiles, beta_x, beta_y,
                                                            beta_z, nullptr);
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_density_from_vof(const double* f_drop, const double* f_film, const int dims[3], double rho_drop,
                        double rho_film, double rho_gas, double* rho, void* hip_stream)
{
    if (!f_drop || !f_film || !dims || !rho) return MG_EINVAL;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return MG_EINVAL;
    if (!(rho_drop > 0) || !(rho_film > 0) || !(rho_gas > 0)) return MG_EINVAL;
    const long n = (long)dims[0] * dims[1] * dims[2];
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    k_density_from_vof<<<grid_full(n), kBlock, 0, s>>>(f_drop, f_film, n, rho_drop, rho_film, rho_gas, rho);
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_faces_from_density(const double* rho, const int dims[3], double* beta_x, double* beta_y, double* beta_z,
                          void* hip_stream)
{
    if (!rho || !dims || !beta_x || !beta_y || !beta_z) return MG_EINVAL;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return MG_EINVAL;
    const Dims d{dims[0], dims[1], dims[2]};
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const MarchGeom g = march_geom(d, kMaxGridBlocks);
    k_faces_march<<<g.blocks, kMarchTX * kMarchTY, 0, s>>>(DensityFaceOp<false>{rho, nullptr}, d, d.nx + 1, g.zc, g.ntx,
                                                            g.nty, g.ntiles, beta_x, beta_y, beta_z, nullptr);
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_density_grad(const double* rho, const int dims[3], const double* g_x, const double* g_y, const double* g_z,
                    double* g_rho, void* hip_stream)
{
    if (!rho || !dims || !g_x || !g_y || !g_z || !g_rho) return MG_EINVAL;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return MG_EINVAL;
    const Dims d{dims[0], dims[1], dims[2]};
    const long n = (long)d.nx * d.ny * d.nz;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    k_density_grad<<<grid_full(n), kBlock, 0, s>>>(rho, d, g_x, g_y, g_z, g_rho);
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_divergence(const double* u, const double* v, const double* w, const int dims[3], double h, double dt,
                  double* b, void* hip_stream)
{
    if (!u || !v || !w || !dims || !b) return MG_EINVAL;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || !(h > 0) || !(dt > 0)) return MG_EINVAL;
    const Dims d{dims[0], dims[1], dims[2]};
    const long n = (long)d.nx * d.ny * d.nz;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    k_divergence<<<grid_full(n), kBlock, 0, s>>>(u, v, w, d, h, dt, b);
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_vof_grad(const double* f_drop, const double* f_film, const int dims[3], double rho_drop, double rho_film,
                double rho_gas, const double* g_x, const double* g_y, const double* g_z, double* g_drop,
                double* g_film, void* hip_stream)
{
    if (!f_drop || !f_film || !dims || !g_x || !g_y || !g_z || !g_drop || !g_film) return MG_EINVAL;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || !(rho_drop > 0) || !(rho_film > 0) || !(rho_gas > 0))
        return MG_EINVAL;
    const Dims d{dims[0], dims[1], dims[2]};
    const long n = (long)d.nx * d.ny * d.nz;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    k_vof_grad<<<grid_full(n), kBlock, 0, s>>>(f_drop, f_film, d, rho_drop, rho_film, rho_gas, g_x, g_y, g_z, g_drop,
                                             g_film);
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_velocity_correct(const double* beta_x, const double* beta_y, const double* beta_z, const double* p,
                        const int dims[3], double h, double dt, double* u, double* v, double* w, void* hip_stream)
{
    if (!beta_x || !beta_y || !beta_z || !p || !dims || !u || !v || !w) return MG_EINVAL;
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || !(h > 0) || !(dt > 0)) return MG_EINVAL;
    const Dims d{dims[0], dims[1], dims[2]};
    const long nf = (long)d.nz * d.ny * (d.nx + 1) + (long)d.nz * (d.ny + 1) * d.nx + (long)(d.nz + 1) * d.ny * d.nx;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    k_velocity_correct<<<grid_full(nf), kBlock, 0, s>>>(beta_x, beta_y, beta_z, p, d, h, dt, u, v, w);
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_level_info(const mg_ctx* cc, int level, int dims[3], double* h)
{
    mg_ctx* c = as_ctx(cc);
    if (!c) return MG_EINVAL;
    if (level < 0 || level >= c->nlev) return MG_EINVAL;
    if (dims) {
        dims[0] = c->lev[level].d.nx;
        dims[1] = c->lev[level].d.ny;
        dims[2] = c->lev[level].d.nz;
    }
    if (h) *h = c->lev[level].h;
    return MG_OK;
}

int mg_level_faces(mg_ctx* c, int level, double* beta_x, double* beta_y, double* beta_z)
{
    TRY(check_ctx(c));
    TRY(level_ok(c, level, MG_PREC_FP64));
    if (!beta_x || !beta_y || !beta_z) return MG_EINVAL;
    Level& L = c->lev[level];
    const long total = (long)L.d.nz * L.d.ny * (L.d.nx + 1) + (long)L.d.nz * (L.d.ny + 1) * L.d.nx +
                       (long)(L.d.nz + 1) * L.d.ny * L.d.nx;
    k_export_faces<double><<<grid_for(total), kBlock, 0, c->stream>>>(L.f64.bx, L.f64.by, L.f64.bz, L.d, beta_x,
                                                                      beta_y, beta_z);
    CHECK_LAUNCH(c);
    return MG_OK;
}

int mg_smooth(mg_ctx* c, int level, int precision, const double* b, double* p, int nsweeps, int order)
{
    TRY(check_ctx(c));
    TRY(level_ok(c, level, precision));
    if (!b || !p || nsweeps < 0 || (order != 0 && order != 1)) {
        set_err(c, "invalid smoothing arguments");
        return MG_EINVAL;
    }
    Level& L = c->lev[level];
    if (precision == MG_PREC_FP64) {
        double* x = level == 0 ? c->work : L.f64.x;
        double* t = level == 0 ? c->ptmp : L.f64.t;
        HIP_TRY(c, hipMemcpyAsync(x, p, sizeof(double) * L.n, hipMemcpyDeviceToDevice, c->stream));
        TRY(smooth<double>(c, level, b, &x, &t, order, nsweeps, false));
        HIP_TRY(c, hipMemcpyAsync(p, x, sizeof(double) * L.n, hipMemcpyDeviceToDevice, c->stream));
    } else {
        float* x = L.f32.x;
        float* t = L.f32.t;
        float* bb = L.f32.b;
        TRY(convert<double, float>(c, b, L.n, bb));
        TRY(convert<double, float>(c, p, L.n, x));
        TRY(smooth<float>(c, level, bb, &x, &t, order, nsweeps, false));
        TRY(convert<float, double>(c, x, L.n, p));
    }
    return MG_OK;
}

int mg_residual_restrict(mg_ctx* c, int level, int precision, const double* b, const double* p,
                         double* b_coarse)
{
    TRY(check_ctx(c));
    TRY(level_ok(c, level, precision));
    if (level >= c->nlev - 1) {
        set_err(c, "level %d has no coarser level", level);
        return MG_EINVAL;
    }
    if (!b || !p || !b_coarse) return MG_EINVAL;
    Level& L = c->lev[level];
    Level& C = c->lev[level + 1];
    if (precision == MG_PREC_FP64) {
        TRY(residual_restrict<double>(c, level, b, p, b_coarse));
    } else {
        TRY(convert<double, float>(c, b, L.n, L.f32.b));
        TRY(convert<double, float>(c, p, L.n, L.f32.x));
        TRY(residual_restrict<float>(c, level, L.f32.b, L.f32.x, C.f32.b));
        TRY(convert<float, double>(c, C.f32.b, C.n, b_coarse));
    }
    return MG_OK;
}

int mg_presmooth_restrict(mg_ctx* c, int level, int precision, const double* b, double* p, double* b_coarse)
{
    TRY(check_ctx(c));
    TRY(level_ok(c, level, precision));
    if (level >= c->nlev - 1) {
        set_err(c, "level %d has no coarser level", level);
        return MG_EINVAL;
    }
    if (!b || !p || !b_coarse) {
        set_err(c, "invalid pre-smoothing arguments");
        return MG_EINVAL;
    }
    Level& L = c->lev[level];
    Level& C = c->lev[level + 1];
    bool restricted = false;
    if (precision == MG_PREC_FP64) {
        double* x = level == 0 ? c->work : L.f64.x;
        double* t = level == 0 ? c->ptmp : L.f64.t;
        TRY(presmooth<double>(c, level, b, &x, &t, &restricted));
        TRY(residual_restrict<double>(c, level, b, x, b_coarse));
        HIP_TRY(c, hipMemcpyAsync(p, x, sizeof(double) * L.n, hipMemcpyDeviceToDevice, c->stream));
    } else {
        float* x = L.f32.x;
        float* t = L.f32.t;
        TRY(convert<double, float>(c, b, L.n, L.f32.b));
        TRY(presmooth<float>(c, level, L.f32.b, &x, &t, &restricted));
        if (!restricted) TRY(residual_restrict<float>(c, level, L.f32.b, x, C.f32.b));
        TRY(convert<float, double>(c, C.f32.b, C.n, b_coarse));
        TRY(convert<float, double>(c, x, L.n, p));
    }
    return MG_OK;
}

int mg_prolong_correct(mg_ctx* c, int level, int precision, const double* e_coarse, double* p)
{
    TRY(check_ctx(c));
    TRY(level_ok(c, level, precision));
    if (level >= c->nlev - 1) {
        set_err(c, "level %d has no coarser level", level);
        return MG_EINVAL;
    }
    if (!e_coarse || !p) return MG_EINVAL;
    Level& L = c->lev[level];
    Level& C = c->lev[level + 1];
    if (precision == MG_PREC_FP64) {
        TRY(prolong_correct<double>(c, level, e_coarse, p));
    } else {
        TRY(convert<double, float>(c, e_coarse, C.n, C.f32.x));
        TRY(convert<double, float>(c, p, L.n, L.f32.x));
        TRY(prolong_correct<float>(c, level, C.f32.x, L.f32.x));
        TRY(convert<float, double>(c, L.f32.x, L.n, p));
    }
    return MG_OK;
}

int mg_coarse_solve(mg_ctx* c, const double* r, double* e)
{
    TRY(check_ctx(c));
    if (!r || !e) return MG_EINVAL;
    return coarse_apply<double>(c, r, e);
}

int mg_residual_norm2(mg_ctx* c, const double* b, const double* p, double* norm2)
{
    TRY(check_ctx(c));
    if (!b || !p || !norm2) return MG_EINVAL;
    TRY(residual_norm_launch(c, b, p, nullptr, 6));
    HIP_TRY(c, hipMemcpyAsync(c->host_scal + 6, c->scal + 6, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    harvest(c);
    *norm2 = c->host_scal[6];
    return MG_OK;
}

}  // extern "C"

// ===========================================================================
// Solve without allocation (mg_solve_noalloc)
// ===========================================================================

// Device scratch of mg_solve_noalloc: the level hierarchy, copies and reduction
// buffers of one set-up-and-solve.  Each GPU the library runs on holds its own
// copy until the process ends, and every call on that GPU reuses it.  In host
// code `scratch` is only a stand-in for the symbol: its device address comes
// from hipGetSymbolAddress (scratch_address), never from the name.
static __device__ __align__(256) double scratch[MG_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices];  // device address of `scratch` on each device, once looked up

// Address of `scratch` on the current device (looked up on the first call there).
int scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxScratchDevices) {
        std::snprintf(g_setup_err, sizeof(g_setup_err), "device %d beyond the %d devices mg_solve_noalloc serves",
                      dev, kMaxScratchDevices);
        return MG_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            std::snprintf(g_setup_err, sizeof(g_setup_err), "hipGetSymbolAddress(scratch) failed on device %d: %s",
                          dev, hipGetErrorString(e));
            return MG_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MG_OK;
}

}  // namespace

extern "C" {

int mg_solve_noalloc(const double* beta_x, const double* beta_y, const double* beta_z, const int dims[3], double h,
                     int bc, const mg_opts* opts, const double* rhs, double* p, double tol, mg_stats* st,
                     void* hip_stream)
{
    g_setup_err[0] = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        std::snprintf(g_setup_err, sizeof(g_setup_err), "no HIP device");
        return MG_EHIP;
    }
    void* ptr = nullptr;
    TRY(scratch_address(dev, &ptr));
    // the context lives on this call's stack and its arena in `scratch`
    mg_ctx local;
    const CallerMemory mem{&local, ptr, MG_NOALLOC_SCRATCH_BYTES};
    mg_ctx* c = nullptr;
    TRY(setup_ctx(&c, beta_x, beta_y, beta_z, nullptr, dims, h, bc, opts, hip_stream, &mem));
    const int status = solve_impl(c, rhs, p, tol, st);
    if (status != MG_OK) {
        std::snprintf(g_setup_err, sizeof(g_setup_err), "%s", c->err);
        (void)hipStreamSynchronize(c->stream);  // nothing of this call still runs in `scratch`
    }
    return status;
}

}  // extern "C"
