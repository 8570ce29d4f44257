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
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "exsum_internal.hpp"

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
    }
    return 0;
}

exs_status validate_job(const exs_job* job, bool check_ptrs) {
    if (!job) return set_error(EXS_EINVAL, "job is NULL");
    if (job->d < 1 || job->d > EXS_MAX_RANK)
        return set_error(EXS_EINVAL, "rank d must be in 1..8");
    if (dtype_size(job->dtype) == 0) return set_error(EXS_EINVAL, "unknown dtype");
    if (job->op != EXS_SUM && job->op != EXS_MAX) return set_error(EXS_EINVAL, "unknown op");
    if (job->mode == 0 || (job->mode & ~(EXS_INCLUDED | EXS_EXCLUDED)))
        return set_error(EXS_EINVAL, "mode must be EXS_INCLUDED and/or EXS_EXCLUDED");
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
};
static std::mutex g_tmu;
static bool g_timing = false;
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
    std::lock_guard<std::mutex> g(g_tmu);
    if (!g_timing) return;
    std::string nm(name);
    if (g_tag >= 0) nm += "@L" + std::to_string(g_tag);
    TimingRec r{nm, take_event(), take_event()};
    if (!r.a || !r.b) return;
    hipEventRecord(r.a, st);
    g_pending.push_back(r);
    slot = (int)g_pending.size() - 1;
}

KTimer::~KTimer() {
    if (slot < 0) return;
    std::lock_guard<std::mutex> g(g_tmu);
    if (slot < (int)g_pending.size()) hipEventRecord(g_pending[slot].b, st);
}

// Bump allocator over the caller's workspace.  In "dry" mode it only
// measures, so sizing and execution share one code path.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, off = 0;
    bool dry = true;
    template <typename T>
    T* take(i64 count) {
        off = (off + 255) & ~(size_t)255;
        T* p = dry ? nullptr : (T*)(base + off);
        off += (size_t)count * sizeof(T);
        return p;
    }
};

static i64 prod(const i64* v, int a, int b) {
    i64 p = 1;
    for (int i = a; i < b; ++i) p *= v[i];
    return p;
}

// Box-sum a rank-d tensor over axes last .. first (last axis first: the
// innermost reduction of the nested definition in Sec. 2), ping-ponging
// between wb[0] and wb[1].  Returns the result (src itself if no axis).
template <typename T, class Op>
static const T* filter_axes(const T* src, const i64* n, const i64* k, int d, int first, int last,
                            T* wb0, T* wb1, bool dry, hipStream_t st) {
    const T* cur = src;
    T* wb[2] = {wb0, wb1};
    int which = 0;
    for (int a = last; a >= first; --a) {
        T* dst = wb[which];
        which ^= 1;
        if (!dry) launch_bdbs<T, Op>(cur, dst, prod(n, 0, a), n[a], prod(n, a + 1, d), k[a], st);
        cur = dst;
    }
    return cur;
}

// The LDS-tiled 2-D BDBS kernel is built for 4-byte element types only.
template <typename T, class Op>
static void plane2_call(const T* X, T* W, i64 O, i64 NY, i64 NX, i64 ky, i64 kx, hipStream_t st) {
    if constexpr (sizeof(T) == 4) launch_plane_bdbs<T, Op>(X, W, O, NY, NX, ky, kx, st);
}

// The fused plane kernel is built for 4-byte element types only.
template <typename T, class Op>
static void plane_call(const T* X, const T* PX, const T* SX, const T* Trest, T* exc, T* inc,
                       i64 n0, i64 MID, i64 NY, i64 NX, i64 k0, i64 ky, i64 kx, i64 Q,
                       hipStream_t st) {
    if constexpr (sizeof(T) == 4)
        launch_plane_axis0<T, Op>(X, PX, SX, Trest, exc, inc, n0, MID, NY, NX, k0, ky, kx, Q, st);
}

template <typename T, class Op>
static exs_status run_generic(const exs_job* job, Arena& ar, hipStream_t st) {
    const int d = job->d;
    i64 n[EXS_MAX_RANK], k[EXS_MAX_RANK];
    for (int i = 0; i < d; ++i) { n[i] = job->dims[i]; k[i] = job->box[i]; }
    const T* A = (const T*)job->in_dev;
    T* inc = (job->mode & EXS_INCLUDED) ? (T*)job->inc_out_dev : nullptr;
    T* exc = (job->mode & EXS_EXCLUDED) ? (T*)job->exc_out_dev : nullptr;
    const bool want_exc = job->mode & EXS_EXCLUDED;
    const bool dry = ar.dry;
    const i64 N = prod(n, 0, d);
    // level 0 streams axis 0 with the fused plane kernel when it applies; it
    // box-sums the two trailing axes itself, the middle axes are done first
    const bool fused = sizeof(T) == 4 && plane_eligible(d, n, k, (int)sizeof(T));

    // buffers for box-summed tensors, shared by every level: level j needs
    // (d_j - 1) passes over N_j elements, the fused level 0 only d - 3
    int wb_count = 0;
    i64 wb_elems = 0;
    for (int j = 0; j < (want_exc ? d : 1); ++j) {
        const int passes = (j == 0 && fused) ? std::max(0, d - 3) : d - j - 1;
        if (passes > 0) {
            wb_count = std::max(wb_count, std::min(2, passes));
            wb_elems = std::max(wb_elems, prod(n, j, d));
        }
    }
    T* wb0 = wb_count >= 1 ? ar.take<T>(wb_elems) : nullptr;
    T* wb1 = wb_count >= 2 ? ar.take<T>(wb_elems) : nullptr;

    set_timing_tag(0);
    if (!want_exc) {
        // included sums only: BDBS along every axis
        if (fused) {
            const T* X0 = filter_axes<T, Op>(A, n, k, d, 1, d - 3, wb0, wb1, dry, st);
            if (!dry)
                plane_call<T, Op>(X0, nullptr, nullptr, nullptr, nullptr, inc, n[0],
                                          prod(n, 1, d - 2), n[d - 2], n[d - 1], k[0], k[d - 2],
                                          k[d - 1], (n[0] + k[0] - 1) / k[0], st);
            return EXS_OK;
        }
        const T* W = filter_axes<T, Op>(A, n, k, d, 1, d - 1, wb0, wb1, dry, st);
        if (!dry) launch_bdbs<T, Op>(W, inc, 1, n[0], prod(n, 1, d), k[0], st);
        return EXS_OK;
    }

    // per-level sizes
    i64 Q[EXS_MAX_RANK], M[EXS_MAX_RANK];
    i64 maxQM = 0;
    for (int j = 0; j < d; ++j) {
        Q[j] = (n[j] + k[j] - 1) / k[j];
        M[j] = prod(n, j + 1, d);
        maxQM = std::max(maxQM, Q[j] * M[j]);
    }
    T* Ga = ar.take<T>(maxQM);
    const int ngb = std::min(2, d - 1);
    T* gb0 = ngb >= 1 ? ar.take<T>(maxQM) : nullptr;
    T* gb1 = ngb >= 2 ? ar.take<T>(maxQM) : nullptr;
    T *PX[EXS_MAX_RANK], *SX[EXS_MAX_RANK], *R[EXS_MAX_RANK + 1];
    R[0] = nullptr;
    for (int j = 0; j < d; ++j) {
        PX[j] = ar.take<T>(Q[j] * M[j]);
        SX[j] = ar.take<T>(Q[j] * M[j]);
        R[j + 1] = ar.take<T>(M[j]);
    }
    // lower-level excluded sums: level j >= 1 writes tb[j % 2] (N_j <= N_1)
    T* tb0 = d >= 3 ? ar.take<T>(M[0]) : nullptr;
    T* tb1 = d >= 2 ? ar.take<T>(M[0]) : nullptr;
    T* tb[2] = {tb0, tb1};

    // top-down: block aggregates, their box-sums over the other axes, block
    // scans, and the reduction that feeds the next level
    for (int j = 0; j < d; ++j) {
        const int dj = d - j;
        const T* src = j == 0 ? A : R[j];
        set_timing_tag(j);
        if (!dry) launch_blockagg<T, Op>(src, Ga, n[j], M[j], k[j], Q[j], st);
        i64 gn[EXS_MAX_RANK], gk[EXS_MAX_RANK];
        gn[0] = Q[j];
        gk[0] = 1;
        for (int a = 1; a < dj; ++a) { gn[a] = n[j + a]; gk[a] = k[j + a]; }
        const T* Gw;
        if (j == 0 && fused && plane2_eligible(n[d - 2], n[d - 1], k[d - 2], k[d - 1],
                                               (int)sizeof(T))) {
            // middle axes by the generic passes, the two trailing axes in one
            // LDS-tiled pass
            const T* G1 = filter_axes<T, Op>(Ga, gn, gk, dj, 1, dj - 3, gb0, gb1, dry, st);
            T* G2 = G1 == gb0 ? gb1 : gb0;
            if (!dry)
                plane2_call<T, Op>(G1, G2, Q[0] * prod(n, 1, d - 2), n[d - 2], n[d - 1], k[d - 2],
                                   k[d - 1], st);
            Gw = G2;
        } else {
            Gw = filter_axes<T, Op>(Ga, gn, gk, dj, 1, dj - 1, gb0, gb1, dry, st);
        }
        if (!dry) launch_blockscan<T, Op>(Gw, Ga, PX[j], SX[j], R[j + 1], Q[j], M[j], st);
    }
    // bottom-up: stream the first axis of each level, adding the level below
    for (int j = d - 1; j >= 0; --j) {
        const int dj = d - j;
        const T* src = j == 0 ? A : R[j];
        set_timing_tag(j);
        T* out = j == 0 ? exc : tb[j % 2];
        const T* Trest = j == d - 1 ? nullptr : tb[(j + 1) % 2];
        if (j == 0 && fused) {
            const T* X0 = filter_axes<T, Op>(A, n, k, d, 1, d - 3, wb0, wb1, dry, st);
            if (!dry)
                plane_call<T, Op>(X0, PX[0], SX[0], Trest, exc, inc, n[0],
                                          prod(n, 1, d - 2), n[d - 2], n[d - 1], k[0], k[d - 2],
                                          k[d - 1], Q[0], st);
            continue;
        }
        const T* W = filter_axes<T, Op>(src, n + j, k + j, dj, 1, dj - 1, wb0, wb1, dry, st);
        if (!dry)
            launch_axis0<T, Op>(W, PX[j], SX[j], Trest, out, j == 0 ? inc : nullptr, n[j], M[j],
                                k[j], Q[j], st);
    }
    return EXS_OK;
}

template <typename T>
static exs_status run_dtype(const exs_job* job, Arena& ar, hipStream_t st) {
    if (job->op == EXS_SUM) return run_generic<T, OpSum>(job, ar, st);
    return run_generic<T, OpMax>(job, ar, st);
}

static exs_status dispatch(const exs_job* job, Arena& ar, hipStream_t st) {
    switch (job->dtype) {
        case EXS_F32: return run_dtype<float>(job, ar, st);
        case EXS_F64: return run_dtype<double>(job, ar, st);
        case EXS_I32: return run_dtype<int>(job, ar, st);
        case EXS_I64: return run_dtype<long long>(job, ar, st);
    }
    return set_error(EXS_EINVAL, "unknown dtype");
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
        if (hipEventSynchronize(r.b) != hipSuccess)
            return set_error(EXS_EDEVICE, "hipEventSynchronize failed");
        float ms = 0.f;
        hipEventElapsedTime(&ms, r.a, r.b);
        if (!acc.count(r.name)) order.push_back(r.name);
        acc[r.name].first += 1;
        acc[r.name].second += ms;
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
