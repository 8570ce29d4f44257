// exsum_corners.hip -- the corners algorithm for strong excluded sums in two
// dimensions: the paper's comparison system, beside the box-complement path.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124), Sec. 1 "Corners Algorithm for Strong
// Excluded Sums" and App. A "Analysis of Corners Algorithm".
//
// The complement of the box [x0, x0+k0) x [x1, x1+k1) of an n0 x n1 tensor
// is cut into four disjoint regions, each sharing one corner of the box and
// reaching to the tensor's edge in both directions (a "pinwheel"):
//
//   PP: y0 <  x0,         y1 <  x1+k1        (low rows, up to the box's right edge)
//   PS: y0 <  x0+k0,      y1 >= x1+k1        (right of the box, up to its bottom)
//   SS: y0 >= x0+k0,      y1 >= x1           (below the box, from its left edge)
//   SP: y0 >= x0,         y1 <  x1           (left of the box, from its top)
//
// Every point outside the box is in exactly one of them and none meets the
// box, so no inverse of the operator is needed (a strong excluded sum).  Each
// region is an orthant clipped to the tensor, so its reduction is one entry of
// a full-tensor table: prefix (P) or suffix (S) along axis 0 of a prefix or
// suffix along axis 1 -- the four leaves of the computation tree of App. A for
// d = 2.  The tables take one pass per tree edge and the regions one more
// pass, as the paper describes the algorithm; passes are not fused, so it
// moves about 16 N elements where the fused box-complement path moves 3 to 4.
//
//   1. rows:    Rp = prefix along axis 1, Rs = suffix along axis 1
//               (one wavefront per row, chunks of 64 lanes with a carry);
//   2. columns: PP, SP = prefix, suffix along axis 0 of Rp;
//               PS, SS = prefix, suffix along axis 0 of Rs
//               (segments of L rows: segment totals, their scans per column,
//               then each segment rescanned from its carry; SP and SS
//               overwrite Rp and Rs in place);
//   3. regions: Exc(x) = PP[x0-1][min(x1+k1,n1)-1] op PS[min(x0+k0,n0)-1][x1+k1]
//                        op SS[x0+k0][x1] op SP[x0][x1-1],
//               a term being the identity where its index leaves the tensor.
#include "exsum_device.hpp"
#include "exsum_internal.hpp"

namespace exs {

constexpr int CORNER_U = 4;   // row chunks of 64 per iteration
constexpr i64 CORNER_L = 64;  // rows per column segment

static inline unsigned corner_grid(i64 threads) {
    const i64 g = (threads + 255) / 256;
    return (unsigned)(g < 1 ? 1 : g);
}

template <typename T, class Op>
__global__ __launch_bounds__(256) void k_corner_rows(const T* __restrict__ A, T* __restrict__ Rp,
                                                     T* __restrict__ Rs, i64 n0, i64 n1) {
    const int lane = threadIdx.x & 63;
    const i64 row = (i64)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n0) return;  // the whole wavefront
    const T e = Op::template id<T>();
    const T* __restrict__ a = A + row * n1;
    T* __restrict__ p = Rp + row * n1;
    T* __restrict__ s = Rs + row * n1;
    constexpr i64 W = 64 * CORNER_U;
    T carry = e;
    for (i64 c = 0; c < n1; c += W) {
        T v[CORNER_U];
#pragma unroll
        for (int u = 0; u < CORNER_U; ++u) {
            const i64 i = c + u * 64 + lane;
            v[u] = i < n1 ? a[i] : e;
        }
#pragma unroll
        for (int u = 0; u < CORNER_U; ++u) v[u] = wave_prefix<T, Op>(v[u], lane);
#pragma unroll
        for (int u = 0; u < CORNER_U; ++u) {
            v[u] = Op::apply(carry, v[u]);
            carry = wshfl(v[u], 63);
            const i64 i = c + u * 64 + lane;
            if (i < n1) p[i] = v[u];
        }
    }
    carry = e;
    for (i64 c = ((n1 - 1) / W) * W; c >= 0; c -= W) {
        T v[CORNER_U];
#pragma unroll
        for (int u = 0; u < CORNER_U; ++u) {
            const i64 i = c + u * 64 + lane;
            v[u] = i < n1 ? a[i] : e;
        }
#pragma unroll
        for (int u = 0; u < CORNER_U; ++u) v[u] = wave_suffix<T, Op>(v[u], lane);
#pragma unroll
        for (int u = CORNER_U - 1; u >= 0; --u) {
            v[u] = Op::apply(v[u], carry);
            carry = wshfl(v[u], 0);
            const i64 i = c + u * 64 + lane;
            if (i < n1) s[i] = v[u];
        }
    }
}

// Segment totals of Rp and Rs along axis 0: thread (segment, column).
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_corner_segtot(const T* __restrict__ Rp,
                                                       const T* __restrict__ Rs, T* __restrict__ Tp,
                                                       T* __restrict__ Ts, i64 n0, i64 n1, i64 S) {
    const i64 idx = gtid();
    if (idx >= S * n1) return;
    const i64 j = idx % n1, sg = idx / n1;
    const i64 r0 = sg * CORNER_L, r1 = r0 + CORNER_L < n0 ? r0 + CORNER_L : n0;
    const T e = Op::template id<T>();
    T ap = e, as = e;
#pragma unroll 8
    for (i64 i = r0; i < r1; ++i) {
        ap = Op::apply(ap, Rp[i * n1 + j]);
        as = Op::apply(as, Rs[i * n1 + j]);
    }
    Tp[idx] = ap;
    Ts[idx] = as;
}

// Exclusive prefix and suffix of the segment totals down each column:
// thread (table, column); table 0 is Tp, table 1 is Ts.
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_corner_segscan(const T* __restrict__ Tp,
                                                        const T* __restrict__ Ts,
                                                        T* __restrict__ CPp, T* __restrict__ CSp,
                                                        T* __restrict__ CPs, T* __restrict__ CSs,
                                                        i64 n1, i64 S) {
    const i64 idx = gtid();
    if (idx >= 2 * n1) return;
    const i64 j = idx % n1;
    const bool second = idx >= n1;
    const T* __restrict__ t = second ? Ts : Tp;
    T* __restrict__ cp = second ? CPs : CPp;
    T* __restrict__ cs = second ? CSs : CSp;
    const T e = Op::template id<T>();
    T acc = e;
    for (i64 sg = 0; sg < S; ++sg) {
        cp[sg * n1 + j] = acc;
        acc = Op::apply(acc, t[sg * n1 + j]);
    }
    acc = e;
    for (i64 sg = S - 1; sg >= 0; --sg) {
        cs[sg * n1 + j] = acc;
        acc = Op::apply(t[sg * n1 + j], acc);
    }
}

// Each segment rescanned from its carries: PP, PS forward; SP, SS backward,
// in place over Rp, Rs (this thread alone touches its segment of its column,
// and it has read every element before it overwrites it).
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_corner_colscan(T* __restrict__ Rp, T* __restrict__ Rs,
                                                        T* __restrict__ PP, T* __restrict__ PS,
                                                        const T* __restrict__ CPp,
                                                        const T* __restrict__ CSp,
                                                        const T* __restrict__ CPs,
                                                        const T* __restrict__ CSs, i64 n0, i64 n1,
                                                        i64 S) {
    const i64 idx = gtid();
    if (idx >= S * n1) return;
    const i64 j = idx % n1, sg = idx / n1;
    const i64 r0 = sg * CORNER_L, r1 = r0 + CORNER_L < n0 ? r0 + CORNER_L : n0;
    T ap = CPp[idx], as = CPs[idx];
#pragma unroll 8
    for (i64 i = r0; i < r1; ++i) {
        ap = Op::apply(ap, Rp[i * n1 + j]);
        as = Op::apply(as, Rs[i * n1 + j]);
        PP[i * n1 + j] = ap;
        PS[i * n1 + j] = as;
    }
    ap = CSp[idx];
    as = CSs[idx];
#pragma unroll 8
    for (i64 i = r1 - 1; i >= r0; --i) {
        ap = Op::apply(Rp[i * n1 + j], ap);
        as = Op::apply(Rs[i * n1 + j], as);
        Rp[i * n1 + j] = ap;
        Rs[i * n1 + j] = as;
    }
}

// The four regions of every point.
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_corner_combine(const T* __restrict__ PP,
                                                        const T* __restrict__ PS,
                                                        const T* __restrict__ SS,
                                                        const T* __restrict__ SP,
                                                        T* __restrict__ exc, i64 n0, i64 n1,
                                                        i64 k0, i64 k1) {
    const i64 idx = gtid();
    if (idx >= n0 * n1) return;
    const i64 x1 = idx % n1, x0 = idx / n1;
    const T e = Op::template id<T>();
    const i64 e0 = x0 + k0 < n0 ? x0 + k0 : n0;  // one past the box, clipped
    const i64 e1 = x1 + k1 < n1 ? x1 + k1 : n1;
    T r = e;
    if (x0 >= 1) r = Op::apply(r, PP[(x0 - 1) * n1 + (e1 - 1)]);
    if (x1 + k1 < n1) r = Op::apply(r, PS[(e0 - 1) * n1 + (x1 + k1)]);
    if (x0 + k0 < n0) r = Op::apply(r, SS[(x0 + k0) * n1 + x1]);
    if (x1 >= 1) r = Op::apply(r, SP[x0 * n1 + (x1 - 1)]);
    exc[idx] = r;
}

// Workspace: four n0 x n1 tables and six S x n1 segment arrays, each start
// aligned to 256 bytes.
static size_t corner_ws_bytes(i64 n0, i64 n1, size_t es, size_t offs[10]) {
    const i64 S = (n0 + CORNER_L - 1) / CORNER_L;
    size_t off = 0;
    for (int t = 0; t < 10; ++t) {
        offs[t] = off;
        off += (size_t)(t < 4 ? n0 * n1 : S * n1) * es;
        off = (off + 255) & ~(size_t)255;
    }
    return off;
}

template <typename T, class Op>
static void run_corners_t(const exs_job* job, char* ws, const size_t* offs, hipStream_t st) {
    const i64 n0 = job->dims[0], n1 = job->dims[1];
    const i64 S = (n0 + CORNER_L - 1) / CORNER_L;
    T* PP = (T*)(ws + offs[0]);
    T* PS = (T*)(ws + offs[1]);
    T* Rp = (T*)(ws + offs[2]);  // becomes SP
    T* Rs = (T*)(ws + offs[3]);  // becomes SS
    T* Tp = (T*)(ws + offs[4]);
    T* Ts = (T*)(ws + offs[5]);
    T* CPp = (T*)(ws + offs[6]);
    T* CSp = (T*)(ws + offs[7]);
    T* CPs = (T*)(ws + offs[8]);
    T* CSs = (T*)(ws + offs[9]);
    {
        KTimer t("k_corner_rows", st);
        hipLaunchKernelGGL((k_corner_rows<T, Op>), dim3((unsigned)((n0 + 3) / 4)), dim3(256), 0, st,
                           (const T*)job->in_dev, Rp, Rs, n0, n1);
    }
    {
        KTimer t("k_corner_segtot", st);
        hipLaunchKernelGGL((k_corner_segtot<T, Op>), dim3(corner_grid(S * n1)), dim3(256), 0, st,
                           Rp, Rs, Tp, Ts, n0, n1, S);
    }
    {
        KTimer t("k_corner_segscan", st);
        hipLaunchKernelGGL((k_corner_segscan<T, Op>), dim3(corner_grid(2 * n1)), dim3(256), 0, st,
                           Tp, Ts, CPp, CSp, CPs, CSs, n1, S);
    }
    {
        KTimer t("k_corner_colscan", st);
        hipLaunchKernelGGL((k_corner_colscan<T, Op>), dim3(corner_grid(S * n1)), dim3(256), 0, st,
                           Rp, Rs, PP, PS, CPp, CSp, CPs, CSs, n0, n1, S);
    }
    {
        KTimer t("k_corner_combine", st);
        hipLaunchKernelGGL((k_corner_combine<T, Op>), dim3(corner_grid(n0 * n1)), dim3(256), 0,
                           st, PP, PS, Rs, Rp, (T*)job->exc_out_dev, n0, n1, job->box[0],
                           job->box[1]);
    }
}

template <typename T>
static void run_corners_op(const exs_job* job, char* ws, const size_t* offs, hipStream_t st) {
    if (job->op == EXS_SUM) run_corners_t<T, OpSum>(job, ws, offs, st);
    else if (job->op == EXS_MAX) run_corners_t<T, OpMax>(job, ws, offs, st);
    else run_corners_t<T, OpMin>(job, ws, offs, st);
}

static exs_status validate_corners(const exs_job* job, bool check_ptrs) {
    exs_status s = validate_job(job, check_ptrs);
    if (s != EXS_OK) return s;
    if (job->d != 2)
        return set_error(EXS_EUNSUPPORTED,
                         "the corners algorithm is built for d = 2 (the paper gives no "
                         "construction of its regions beyond that)");
    if (job->mode != EXS_EXCLUDED)
        return set_error(EXS_EINVAL, "the corners algorithm computes strong excluded sums: "
                                     "mode must be EXS_EXCLUDED");
    if (job->dtype == EXS_VALIDX)
        return set_error(EXS_EUNSUPPORTED, "the corners algorithm takes f32, f64, i32 or i64");
    return EXS_OK;
}

}  // namespace exs

using namespace exs;

extern "C" {

exs_status exs_corners_workspace_size(const exs_job* job, size_t* bytes) {
    if (!bytes) return set_error(EXS_EINVAL, "bytes is NULL");
    exs_status s = validate_corners(job, false);
    if (s != EXS_OK) return s;
    size_t offs[10];
    *bytes = corner_ws_bytes(job->dims[0], job->dims[1], dtype_size(job->dtype), offs);
    return EXS_OK;
}

exs_status exs_run_corners(const exs_job* job, void* ws, size_t ws_bytes, void* stream) {
    exs_status s = validate_corners(job, true);
    if (s != EXS_OK) return s;
    size_t offs[10];
    const size_t need = corner_ws_bytes(job->dims[0], job->dims[1], dtype_size(job->dtype), offs);
    if (ws_bytes < need)
        return set_error(EXS_ENOMEM, "workspace too small: need " + std::to_string(need) +
                                         " bytes, got " + std::to_string(ws_bytes));
    if (!ws) return set_error(EXS_EINVAL, "ws is NULL");
    if (((uintptr_t)ws & 255) != 0) return set_error(EXS_EINVAL, "ws must be 256-byte aligned");
    const uintptr_t w0 = (uintptr_t)ws, w1 = w0 + need;
    const uintptr_t tb = (uintptr_t)(job->dims[0] * job->dims[1]) * dtype_size(job->dtype);
    auto hits = [&](const void* p) {
        const uintptr_t a = (uintptr_t)p;
        return a < w1 && w0 < a + tb;
    };
    if (hits(job->in_dev) || hits(job->exc_out_dev))
        return set_error(EXS_EINVAL, "ws overlaps in_dev or exc_out_dev");
    hipStream_t st = (hipStream_t)stream;
    switch (job->dtype) {
        case EXS_F32: run_corners_op<float>(job, (char*)ws, offs, st); break;
        case EXS_F64: run_corners_op<double>(job, (char*)ws, offs, st); break;
        case EXS_I32: run_corners_op<int>(job, (char*)ws, offs, st); break;
        case EXS_I64: run_corners_op<long long>(job, (char*)ws, offs, st); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(EXS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return EXS_OK;
}

}  // extern "C"
