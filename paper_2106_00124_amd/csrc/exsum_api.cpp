// exsum_api.cpp -- planner and C ABI of the plain single-tensor call.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// Excluded sums follow the box-complement algorithm (Sec. 5) in its
// dimension-reduction form.  With R_0 = A and R_{j+1} = the reduction of R_j
// over its first axis, the excluded sum of R_j (rank d_j) is
//
//   Exc_j(x) = Ex1D_0( Inc_{1..}(R_j) )(x) op Exc_{j+1}(x_1, ..., x_{d_j-1})
//
// where Inc_{1..} box-sums every axis but the first (BDBS-Along-Dim, Sec. 5)
// and Ex1D_0 is the op of the prefix before x_0 and the suffix from x_0+k_0
// along the first axis (Prefix-/Suffix-Along-Dim, Sec. 5).  The two components
// of step j+1 in Corollary "Excluded-sum Components" are exactly the prefix
// and suffix terms; the lower-dimensional term carries the components of the
// later steps, broadcast over the reduced axes (Add-Contribution, Sec. 5).
// Included sums are BDBS along every axis (Sec. 3, "Generalizing to
// Arbitrary Dimensions").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "exsum_internal.hpp"
#include "exsum_plan.hpp"

namespace exs {

static thread_local std::string g_last_error;

exs_status set_error(exs_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

size_t dtype_size(int dtype) {
    switch (dtype) {
        case EXS_F32: return 4;
        case EXS_F64: return 8;
        case EXS_I32: return 4;
        case EXS_I64: return 8;
        case EXS_VALIDX: return 8;
    }
    return 0;
}

exs_status validate_job(const exs_job* job, bool check_ptrs) {
    if (!job) return set_error(EXS_EINVAL, "job is NULL");
    if (job->d < 1 || job->d > EXS_MAX_RANK)
        return set_error(EXS_EINVAL, "rank d must be in 1..8");
    if (dtype_size(job->dtype) == 0) return set_error(EXS_EINVAL, "unknown dtype");
    if (job->op != EXS_SUM && job->op != EXS_MAX && job->op != EXS_MIN)
        return set_error(EXS_EINVAL, "unknown op");
    if (job->dtype == EXS_VALIDX && job->op == EXS_SUM)
        return set_error(EXS_EUNSUPPORTED,
                         "(value, index) pairs take EXS_MAX (argmax) or EXS_MIN (argmin)");
    if (job->mode == 0 || (job->mode & ~(EXS_INCLUDED | EXS_EXCLUDED | EXS_WEAK)))
        return set_error(EXS_EINVAL, "mode must be EXS_INCLUDED and/or EXS_EXCLUDED [| EXS_WEAK]");
    if (job->mode & EXS_WEAK) {
        if (!(job->mode & EXS_EXCLUDED))
            return set_error(EXS_EINVAL, "EXS_WEAK needs EXS_EXCLUDED");
        if (job->op != EXS_SUM)
            return set_error(EXS_EUNSUPPORTED,
                             "weak excluded sums subtract; only + has an inverse");
    }
    __int128 N = 1;
    for (int i = 0; i < job->d; ++i) {
        if (job->dims[i] < 1) return set_error(EXS_EINVAL, "every dims[i] must be >= 1");
        if (job->box[i] < 1 || job->box[i] > job->dims[i])
            return set_error(EXS_EINVAL, "every box[i] must satisfy 1 <= box[i] <= dims[i]");
        N *= job->dims[i];
        if (N * (__int128)dtype_size(job->dtype) > ((__int128)1 << 62))
            return set_error(EXS_EINVAL, "tensor too large");
    }
    if (!check_ptrs) return EXS_OK;
    const bool want_inc = job->mode & EXS_INCLUDED, want_exc = job->mode & EXS_EXCLUDED;
    if (!job->in_dev) return set_error(EXS_EINVAL, "in_dev is NULL");
    if (want_inc && !job->inc_out_dev) return set_error(EXS_EINVAL, "inc_out_dev is NULL");
    if (want_exc && !job->exc_out_dev) return set_error(EXS_EINVAL, "exc_out_dev is NULL");
    const uintptr_t es = (uintptr_t)dtype_size(job->dtype);
    if ((uintptr_t)job->in_dev % es || (want_inc && (uintptr_t)job->inc_out_dev % es) ||
        (want_exc && (uintptr_t)job->exc_out_dev % es))
        return set_error(EXS_EINVAL, "tensors must be aligned to their element size");
    const uintptr_t bytes = (uintptr_t)(N * (__int128)dtype_size(job->dtype));
    auto overlap = [bytes](const void* a, const void* b) {
        const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
        return x < y + bytes && y < x + bytes;
    };
    if (want_inc && overlap(job->in_dev, job->inc_out_dev))
        return set_error(EXS_EINVAL, "inc_out_dev overlaps in_dev");
    if (want_exc && overlap(job->in_dev, job->exc_out_dev))
        return set_error(EXS_EINVAL, "exc_out_dev overlaps in_dev");
    if (want_inc && want_exc && overlap(job->inc_out_dev, job->exc_out_dev))
        return set_error(EXS_EINVAL, "inc_out_dev overlaps exc_out_dev");
    return EXS_OK;
}

// ---------------------------------------------------------------------------
// Per-kernel event timing
// ---------------------------------------------------------------------------
struct TimingRec {
    std::string name;
    hipEvent_t a, b;
    bool ended;  // the end event was recorded
};
static std::mutex g_tmu;
static bool g_timing = false;
// set while the allocation-free entry point runs: its launches record no
// timing events (creating one may allocate)
static thread_local bool g_timing_off = false;
static std::vector<TimingRec> g_pending;
static std::vector<hipEvent_t> g_event_pool;
static thread_local int g_tag = -1;

void set_timing_tag(int level) { g_tag = level; }

static hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

KTimer::KTimer(const char* name, hipStream_t stream) : slot(-1), st(stream) {
    if (g_timing_off) return;
    std::lock_guard<std::mutex> g(g_tmu);
    if (!g_timing) return;
    std::string nm(name);
    if (g_tag >= 0) nm += "@L" + std::to_string(g_tag);
    TimingRec r{nm, take_event(), take_event(), false};
    if (!r.a || !r.b || hipEventRecord(r.a, st) != hipSuccess) {
        // timing is best-effort: a launch whose events cannot be recorded is
        // left out of the totals
        if (r.a) g_event_pool.push_back(r.a);
        if (r.b) g_event_pool.push_back(r.b);
        return;
    }
    g_pending.push_back(r);
    slot = (int)g_pending.size() - 1;
}

KTimer::~KTimer() {
    if (slot < 0) return;
    std::lock_guard<std::mutex> g(g_tmu);
    if (slot < (int)g_pending.size())
        g_pending[slot].ended = hipEventRecord(g_pending[slot].b, st) == hipSuccess;
}

// Launches every step at once on one stream (the plain call).
template <typename T, class Op>
struct EagerSink {
    hipStream_t st;
    bool fused_ok = true;
    void level(int j) { set_timing_tag(j); }
    void bdbs(const T* in, T* out, i64 O, i64 n, i64 I, i64 k) {
        launch_bdbs<T, Op>(in, out, O, n, I, k, st);
    }
    void blockagg(const T* X, T* Ga, i64 n0, i64 M, i64 k0, i64 Q) {
        launch_blockagg<T, Op>(X, Ga, n0, M, k0, Q, st);
    }
    bool aggmid_ok() const { return true; }
    void aggmid(const T* A, T* X, T* Ga, T* G1, i64 n0, i64 P, i64 nf, i64 S, i64 k0, i64 kf,
                i64 Q) {
        launch_aggmid<T, Op>(A, X, Ga, G1, n0, P, nf, S, k0, kf, Q, st);
    }
    bool small1d_ok(i64 n) const { return ex1d_small_ok(n); }
    // the one-workgroup rank-2 kernel: numeric types under +, max and min
    static constexpr bool kSmall2d =
        std::is_arithmetic<T>::value &&
        (std::is_same<Op, OpSum>::value || std::is_same<Op, OpMax>::value ||
         std::is_same<Op, OpMin>::value);
    bool small2d_ok(i64 n0, i64 n1, i64 k0, i64 k1) const {
        return kSmall2d && small2d_eligible(n0, n1, k0, k1, (int)sizeof(T));
    }
    void small2d(const T* A, T* exc, T* inc, i64 n0, i64 n1, i64 k0, i64 k1) {
        if constexpr (kSmall2d) launch_small2d<T, Op>(A, exc, inc, n0, n1, k0, k1, st);
    }
    i64 tail_box_max() const { return tail_box_max_elems((int)sizeof(T)); }
    void bdbs_tail(const T* in, T* out, i64 O, int m, const i64* n, const i64* k) {
        launch_bdbs_tail<T, Op>(in, out, O, m, n, k, st);
    }
    bool long1d_ok(i64 n, i64 k) const { return sizeof(T) == 4 && exs::long1d_ok(n, k); }
    void long1d(const T* A, T* exc, T* inc, i64 n, i64 k, T* Tt, T* Ut, T* CP, T* CS) {
        if constexpr (sizeof(T) == 4) launch_long1d<T, Op>(A, exc, inc, n, k, Tt, Ut, CP, CS, st);
    }
    bool tail_ok(i64 Q, i64 n, i64 k) const { return sizeof(T) == 4 && tail_scan_ok(Q, n, k); }
    void tail_scan(const T* A1, T* PX, T* SX, T* exc2, i64 Q, i64 n, i64 k, i64 pxe) {
        if constexpr (sizeof(T) == 4) launch_tail_scan<T, Op>(A1, PX, SX, exc2, Q, n, k, pxe, st);
    }
    bool row_ok(i64 n0, i64 NX, i64 k0, i64 kx) const {
        return sizeof(T) == 4 && row_eligible(n0, NX, k0, kx, (int)sizeof(T));
    }
    void row_axis0(const T* X, const T* PX, const T* SX, const T* Trest, T* exc, T* inc, i64 n0,
                   i64 NX, i64 k0, i64 kx, i64 Q) {
        if constexpr (sizeof(T) == 4)
            launch_row_axis0<T, Op>(X, PX, SX, Trest, exc, inc, n0, NX, k0, kx, Q, st);
    }
    void segtot(const T* Gw, const T* Ga, T* Tw, T* Ta, i64 Q, i64 M, i64 L) {
        launch_segtot<T, Op>(Gw, Ga, Tw, Ta, Q, M, L, st);
    }
    void segexp(const T* Gw, const T* SPX, const T* SSX, T* PX, T* SX, i64 Q, i64 M, i64 L,
                i64 pxe) {
        launch_segexp<T, Op>(Gw, SPX, SSX, PX, SX, Q, M, L, pxe, st);
    }
    // weak excluded sums need an inverse: numeric element types only
    void total(const T* X, i64 N, void* parts, T* tot) {
        if constexpr (std::is_arithmetic<T>::value) launch_total<T>(X, N, parts, tot, st);
    }
    void weak_exc(const T* inc, const T* tot, T* exc, i64 N) {
        if constexpr (std::is_arithmetic<T>::value) launch_weak_exc<T>(inc, tot, exc, N, st);
    }
    void plane_weak(const T* X, T* inc, const T* tot, T* wexc, i64 n0, i64 MID, i64 NY, i64 NX,
                    i64 k0, i64 ky, i64 kx) {
        if constexpr (sizeof(T) == 4 && std::is_same<Op, OpSum>::value)
            launch_plane_weak<T, Op>(X, inc, tot, wexc, n0, MID, NY, NX, k0, ky, kx, st);
    }
    void ex1d_small(const T* R, T* exc, i64 n, i64 k) {
        launch_ex1d_small<T, Op>(R, exc, n, k, st);
    }
    void blockscan(const T* Gw, const T* Ga, T* PX, T* SX, T* R, i64 Q, i64 M, i64 pxe) {
        launch_blockscan<T, Op>(Gw, Ga, PX, SX, R, Q, M, pxe, st);
    }
    void axis0(const T* W, const T* PX, const T* SX, const T* Trest, T* exc, T* inc, i64 n0,
               i64 M, i64 k0, i64 Q, T* ex2t) {
        launch_axis0<T, Op>(W, PX, SX, Trest, exc, inc, n0, M, k0, Q, ex2t, st);
    }
    // the fused kernels are built for 4-byte element types only
    void plane_axis0(const T* X, const T* PX, const T* SX, const T* Trest, T* exc, T* inc, i64 n0,
                     i64 MID, i64 NY, i64 NX, i64 k0, i64 ky, i64 kx, i64 Q) {
        if constexpr (sizeof(T) == 4)
            launch_plane_axis0<T, Op>(X, PX, SX, Trest, exc, inc, n0, MID, NY, NX, k0, ky, kx, Q,
                                      st);
    }
    void plane_scan(const T* G, const T* Ga, T* PX, T* SX, T* R, T* A1, i64 Q, i64 MID, i64 NY,
                    i64 NX, i64 ky, i64 kx, i64 pxe) {
        if constexpr (sizeof(T) == 4)
            launch_plane_scan<T, Op>(G, Ga, PX, SX, R, A1, Q, MID, NY, NX, ky, kx, pxe, st);
    }
    void plane_bdbs(const T* X, T* W, i64 O, i64 NY, i64 NX, i64 ky, i64 kx) {
        if constexpr (sizeof(T) == 4) launch_plane_bdbs<T, Op>(X, W, O, NY, NX, ky, kx, st);
    }
};

// cost of the slowed fp32 + (0: the plain operator); exs_set_op_cost
static std::atomic<int> g_op_cost{0};

template <typename T>
static exs_status run_dtype(const exs_job* job, Arena& ar, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value) {
        if (job->op == EXS_SUM && !(job->mode & EXS_WEAK) && g_op_cost.load() > 0) {
            EagerSink<T, OpSlowSum> sink{st};
            return plan_job<T>(job, ar, sink);
        }
    }
    if (job->op == EXS_SUM) {
        EagerSink<T, OpSum> sink{st};
        return plan_job<T>(job, ar, sink);
    }
    if (job->op == EXS_MAX) {
        EagerSink<T, OpMax> sink{st};
        return plan_job<T>(job, ar, sink);
    }
    EagerSink<T, OpMin> sink{st};
    return plan_job<T>(job, ar, sink);
}

// (value, index) pairs: max and min only
static exs_status run_validx(const exs_job* job, Arena& ar, hipStream_t st) {
    if (job->op == EXS_MAX) {
        EagerSink<ValIdx, OpMax> sink{st};
        return plan_job<ValIdx>(job, ar, sink);
    }
    if (job->op == EXS_MIN) {
        EagerSink<ValIdx, OpMin> sink{st};
        return plan_job<ValIdx>(job, ar, sink);
    }
    return set_error(EXS_EUNSUPPORTED, "(value, index) pairs take EXS_MAX or EXS_MIN");
}

static exs_status dispatch(const exs_job* job, Arena& ar, hipStream_t st) {
    switch (job->dtype) {
        case EXS_F32: return run_dtype<float>(job, ar, st);
        case EXS_F64: return run_dtype<double>(job, ar, st);
        case EXS_I32: return run_dtype<int>(job, ar, st);
        case EXS_I64: return run_dtype<long long>(job, ar, st);
        case EXS_VALIDX: return run_validx(job, ar, st);
    }
    return set_error(EXS_EINVAL, "unknown dtype");
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free entry point: one file-scope device array
// per GPU, found through hipGetSymbolAddress (the array's name in host code
// is only a stand-in, not a device address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[EXS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this GPU's scratch array, looked up once per device
// with that device current.
static exs_status scratch_for_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return set_error(EXS_EDEVICE, "no current HIP device (or device index >= 64)");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(EXS_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                              hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return EXS_OK;
}

}  // namespace exs

using namespace exs;

extern "C" {

exs_status exs_workspace_size(const exs_job* job, size_t* bytes) {
    if (!bytes) return set_error(EXS_EINVAL, "bytes is NULL");
    exs_status s = validate_job(job, false);
    if (s != EXS_OK) return s;
    Arena ar;
    ar.dry = true;
    s = dispatch(job, ar, nullptr);
    if (s != EXS_OK) return s;
    *bytes = (ar.off + 255) & ~(size_t)255;
    return EXS_OK;
}

exs_status exs_run(const exs_job* job, void* ws, size_t ws_bytes, void* stream) {
    exs_status s = validate_job(job, true);
    if (s != EXS_OK) return s;
    size_t need = 0;
    s = exs_workspace_size(job, &need);
    if (s != EXS_OK) return s;
    if (ws_bytes < need)
        return set_error(EXS_ENOMEM, "workspace too small: need " + std::to_string(need) +
                                         " bytes, got " + std::to_string(ws_bytes));
    if (need > 0 && !ws) return set_error(EXS_EINVAL, "ws is NULL");
    if (((uintptr_t)ws & 255) != 0) return set_error(EXS_EINVAL, "ws must be 256-byte aligned");
    Arena ar;
    ar.dry = false;
    ar.base = (char*)ws;
    ar.cap = ws_bytes;
    hipStream_t st = (hipStream_t)stream;
    s = dispatch(job, ar, st);
    set_timing_tag(-1);
    if (s != EXS_OK) return s;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(EXS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return EXS_OK;
}

exs_status exs_run_noalloc(const exs_job* job, void* stream) {
    exs_status s = validate_job(job, true);
    if (s != EXS_OK) return s;
    size_t need = 0;
    s = exs_workspace_size(job, &need);
    if (s != EXS_OK) return s;
    if (need > (size_t)EXS_NOALLOC_SCRATCH_BYTES)
        return set_error(EXS_ENOMEM, "exs_run_noalloc: this job needs " + std::to_string(need) +
                                         " bytes of workspace, more than the " +
                                         std::to_string((long long)EXS_NOALLOC_SCRATCH_BYTES) +
                                         "-byte static scratch; use exs_run with a workspace");
    void* ws = nullptr;
    s = scratch_for_current_device(&ws);
    if (s != EXS_OK) return s;
    // nothing in the workspace has to start at zero: every kernel writes its
    // scratch before reading it
    Arena ar;
    ar.dry = false;
    ar.base = (char*)ws;
    ar.cap = (size_t)EXS_NOALLOC_SCRATCH_BYTES;
    g_timing_off = true;
    s = dispatch(job, ar, (hipStream_t)stream);
    g_timing_off = false;
    set_timing_tag(-1);
    if (s != EXS_OK) return s;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(EXS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return EXS_OK;
}

exs_status exs_set_op_cost(int32_t cost) {
    if (cost < 0 || cost > (1 << 20)) return set_error(EXS_EINVAL, "cost must be in 0..2^20");
    const hipError_t e[5] = {slow_cost_set_kernels(cost), slow_cost_set_plane(cost),
                             slow_cost_set_row(cost), slow_cost_set_ex1d(cost),
                             slow_cost_set_tailbox(cost)};
    for (hipError_t x : e)
        if (x != hipSuccess)
            return set_error(EXS_EDEVICE, std::string("cannot set the operator cost: ") +
                                              hipGetErrorString(x));
    g_op_cost.store(cost);
    return EXS_OK;
}

exs_status exs_op_probe(void* data, int64_t n, int32_t reps, void* stream) {
    if (n < 0 || reps < 0) return set_error(EXS_EINVAL, "n and reps must be >= 0");
    if (n > 0 && !data) return set_error(EXS_EINVAL, "data is NULL");
    if (n == 0) return EXS_OK;
    launch_op_probe((float*)data, n, reps, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(EXS_EDEVICE, std::string("probe launch failed: ") + hipGetErrorString(e));
    return EXS_OK;
}

const char* exs_status_str(exs_status s) {
    switch (s) {
        case EXS_OK: return "EXS_OK";
        case EXS_EINVAL: return "EXS_EINVAL";
        case EXS_EUNSUPPORTED: return "EXS_EUNSUPPORTED";
        case EXS_ENOMEM: return "EXS_ENOMEM";
        case EXS_EDEVICE: return "EXS_EDEVICE";
        case EXS_EAGAIN: return "EXS_EAGAIN";
        case EXS_ENOTREADY: return "EXS_ENOTREADY";
        case EXS_ENOTFOUND: return "EXS_ENOTFOUND";
    }
    return "EXS_UNKNOWN";
}

const char* exs_last_error(void) { return g_last_error.c_str(); }

const char* exs_version(void) { return "exsum 0.1 (gfx950)"; }

exs_status exs_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> g(g_tmu);
    g_timing = on != 0;
    return EXS_OK;
}

exs_status exs_timing_read(int32_t max, char* names, int64_t* launches, double* total_ms,
                           int32_t* count) {
    std::lock_guard<std::mutex> g(g_tmu);
    std::map<std::string, std::pair<int64_t, double>> acc;
    std::vector<std::string> order;
    for (auto& r : g_pending) {
        if (r.ended && hipEventSynchronize(r.b) != hipSuccess)
            return set_error(EXS_EDEVICE, "hipEventSynchronize failed");
        float ms = 0.f;
        if (r.ended && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            if (!acc.count(r.name)) order.push_back(r.name);
            acc[r.name].first += 1;
            acc[r.name].second += ms;
        }
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_pending.clear();
    int32_t c = 0;
    for (auto& nm : order) {
        if (c >= max) break;
        if (names) {
            std::strncpy(names + 64 * c, nm.c_str(), 63);
            names[64 * c + 63] = 0;
        }
        if (launches) launches[c] = acc[nm].first;
        if (total_ms) total_ms[c] = acc[nm].second;
        ++c;
    }
    if (count) *count = c;
    return EXS_OK;
}

exs_status exs_fill(void* out, int64_t count, int32_t dtype, int32_t kind, uint64_t seed,
                    int64_t lo, int64_t hi, void* stream) {
    if (count < 0) return set_error(EXS_EINVAL, "count < 0");
    if (count > 0 && !out) return set_error(EXS_EINVAL, "out is NULL");
    if (kind == 0 || kind == 2) {
        if (dtype != EXS_F32) return set_error(EXS_EINVAL, "fill kinds 0 and 2 produce f32");
    } else if (kind == 1) {
        if (dtype != EXS_I32 && dtype != EXS_I64)
            return set_error(EXS_EINVAL, "fill kind 1 produces i32 or i64");
        if (hi < lo) return set_error(EXS_EINVAL, "hi < lo");
    } else {
        return set_error(EXS_EINVAL, "unknown fill kind");
    }
    if (count == 0) return EXS_OK;
    const float scale = (float)(1.7320508075688772 / 65535.0);  // sqrt(3)/65535
    launch_fill(out, count, dtype, kind, seed, lo, hi, scale, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(EXS_EDEVICE, std::string("fill launch failed: ") + hipGetErrorString(e));
    return EXS_OK;
}

}  // extern "C"
