// exsum_ex1d.hip -- excluded (and included) sums of a long 1-D level, for
// 4-byte element types and boxes of at most 16.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// At the last dimension-reduction level (Sec. 5) only the prefix before x and
// the suffix from x + k remain: Exc[x] = P[x - 1] op S[x + k], with P and S the
// inclusive prefix and suffix along the axis.  The axis is cut into chunks of C
// elements (C a multiple of k); three launches:
//   k_l1_tot   per chunk: its total T[c] and U[c], the total without its first
//              k elements;
//   k_l1_scan  one workgroup: the exclusive prefix CP and suffix CS of T;
//   k_l1_out   per chunk, staged in LDS with the first k elements of the next
//              chunk: the workgroup's prefix and suffix scans plus CP[c] and
//              CS[c] give P and S on the chunk; S past the chunk is the next
//              chunk's first k elements op U[c + 1] op CS[c + 1].  The included
//              sum is BDBS (Sec. 3): each thread owns whole k-blocks, so the
//              block's range suffix is a thread-local scan and the next
//              block's range prefix is read from LDS.
#include "exsum_internal.hpp"
#include "exsum_plane.hpp"

namespace exs {

constexpr int L1_THREADS = 256;
constexpr int L1_SCAN_THREADS = 1024, L1_SCAN_PER = 8;
// the chunk-total scan walks tiles of L1_SCAN_THREADS * L1_SCAN_PER totals;
// at 4096 or more elements per chunk, n < 2^31 stays within this
constexpr int L1_MAX_CHUNKS = 1 << 19;

// elements per thread: whole k-blocks, at least 16
static inline int l1_elems(i64 k) { return (int)(k * ((16 + k - 1) / k)); }

template <typename T, class Op>
__device__ __forceinline__ T l1_wg_reduce(T v, T* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = Op::apply(v, __shfl_xor(v, off, 64));
    if (lane == 0) red[wv] = v;
    __syncthreads();
    T r = red[0];
#pragma unroll
    for (int w = 1; w < L1_THREADS / 64; ++w) r = Op::apply(r, red[w]);
    return r;
}

template <typename T, class Op>
__global__ __launch_bounds__(L1_THREADS) void k_l1_tot(const T* __restrict__ A,
                                                       T* __restrict__ Tt, T* __restrict__ Ut,
                                                       i64 n, int C, int k) {
    __shared__ T red[2][L1_THREADS / 64];
    const T e = Op::template id<T>();
    const i64 base = (i64)blockIdx.x * C;
    const int len = n - base < C ? (int)(n - base) : C;
    T s = e, u = e;
#pragma unroll 8
    for (int i = threadIdx.x; i < len; i += L1_THREADS) {
        const T v = A[base + i];
        s = Op::apply(s, v);
        if (i >= k) u = Op::apply(u, v);
    }
    s = l1_wg_reduce<T, Op>(s, red[0]);
    u = l1_wg_reduce<T, Op>(u, red[1]);
    if (threadIdx.x == 0) {
        Tt[blockIdx.x] = s;
        Ut[blockIdx.x] = u;
    }
}

template <typename T, class Op>
__global__ __launch_bounds__(L1_SCAN_THREADS) void k_l1_scan(const T* __restrict__ Tt,
                                                             T* __restrict__ CP,
                                                             T* __restrict__ CS, int nc) {
    // tiles of L1_SCAN_THREADS * L1_SCAN_PER chunk totals: forward over the
    // tiles for the prefixes, backward for the suffixes, each carrying the op
    // of the tiles already passed
    constexpr int TILE = L1_SCAN_THREADS * L1_SCAN_PER;
    constexpr int NW = L1_SCAN_THREADS / 64;
    __shared__ T wt[NW];
    const T e = Op::template id<T>();
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    T carry = e;  // op of the chunk totals before the tile
    for (int base = 0; base < nc; base += TILE) {
        const int b0 = base + t * L1_SCAN_PER;
        T v[L1_SCAN_PER];
#pragma unroll
        for (int r = 0; r < L1_SCAN_PER; ++r) v[r] = b0 + r < nc ? Tt[b0 + r] : e;
        T run = e;
#pragma unroll
        for (int r = 0; r < L1_SCAN_PER; ++r) run = Op::apply(run, v[r]);
        const T ip = wave_prefix<T, Op>(run, lane);
        if (lane == 63) wt[wv] = ip;
        __syncthreads();
        T lo = e, all = e;
        for (int w = 0; w < NW; ++w) {
            if (w < wv) lo = Op::apply(lo, wt[w]);
            all = Op::apply(all, wt[w]);
        }
        const T up = __shfl_up(ip, 1, 64);
        T before = Op::apply(carry, lane > 0 ? Op::apply(lo, up) : lo);
#pragma unroll
        for (int r = 0; r < L1_SCAN_PER; ++r) {
            if (b0 + r < nc) CP[b0 + r] = before;
            before = Op::apply(before, v[r]);
        }
        carry = Op::apply(carry, all);
        __syncthreads();  // wt is rewritten by the next tile
    }
    carry = e;  // op of the chunk totals after the tile
    for (int base = (nc - 1) / TILE * TILE; base >= 0; base -= TILE) {
        const int b0 = base + t * L1_SCAN_PER;
        T v[L1_SCAN_PER];
#pragma unroll
        for (int r = 0; r < L1_SCAN_PER; ++r) v[r] = b0 + r < nc ? Tt[b0 + r] : e;
        T run = e;
#pragma unroll
        for (int r = 0; r < L1_SCAN_PER; ++r) run = Op::apply(run, v[r]);
        const T is = wave_suffix<T, Op>(run, lane);
        if (lane == 0) wt[wv] = is;
        __syncthreads();
        T hi = e, all = e;
        for (int w = NW - 1; w >= 0; --w) {
            if (w > wv) hi = Op::apply(wt[w], hi);
            all = Op::apply(wt[w], all);
        }
        const T dn = __shfl_down(is, 1, 64);
        T after = Op::apply(lane < 63 ? Op::apply(dn, hi) : hi, carry);
#pragma unroll
        for (int r = L1_SCAN_PER - 1; r >= 0; --r) {
            if (b0 + r < nc) CS[b0 + r] = after;
            after = Op::apply(v[r], after);
        }
        carry = Op::apply(all, carry);
        __syncthreads();
    }
}

// E (elements per thread) is a template parameter so that every loop has a
// fixed trip count.  In LDS each thread's run of E elements sits at
// t * (E + 1) (one pad word per run: distinct banks for the lanes, and every
// access of a run is the thread's base plus a constant); the first k elements
// of the next chunk are run L1_THREADS.
template <typename T, class Op, int E>
__global__ __launch_bounds__(L1_THREADS) void k_l1_out(const T* __restrict__ A,
                                                       const T* __restrict__ CP,
                                                       const T* __restrict__ CS,
                                                       const T* __restrict__ Ut,
                                                       T* __restrict__ exc, T* __restrict__ inc,
                                                       i64 n, int k) {
    constexpr int C = L1_THREADS * E, RS = E + 1;
    constexpr int NR = (C + 16 + L1_THREADS - 1) / L1_THREADS;  // staging rounds, halo included
    __shared__ T raw[(L1_THREADS + 1) * RS];
    __shared__ T suf[L1_THREADS * RS];
    __shared__ T wt[2][L1_THREADS / 64];
    __shared__ T hs[16];
    const T e = Op::template id<T>();
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const i64 c = blockIdx.x, base = c * C;
    // elements from the chunk start to the end of the tensor (capped)
    const int rem = n - base < C + 16 ? (int)(n - base) : C + 16;
    const int len = rem < C ? rem : C;
    const int hlen = rem - C <= 0 ? 0 : (rem - C < k ? rem - C : k);
    const int lim = len + hlen;

    // the chunk's offsets (excluded sums only), issued with the chunk loads
    const T cp = exc ? CP[c] : e, cs = exc ? CS[c] : e;
    const T tail = exc && hlen > 0 ? Op::apply(Ut[c + 1], CS[c + 1]) : e;
    // the chunk and the first k elements of the next one (identity past them):
    // coalesced loads, all issued before the first LDS write
    {
        const __amdgpu_buffer_rsrc_t src = buf(A + base, (unsigned)lim * sizeof(T));
        T g[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int i = t + r * L1_THREADS;
            const T x = bload<T>(src, (unsigned)i * sizeof(T));
            g[r] = i < lim ? x : e;
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int i = t + r * L1_THREADS;
            if (i < C + 16) raw[(i / E) * RS + i % E] = g[r];
        }
    }
    __syncthreads();

    const int x0 = t * E;
    T* const my_raw = raw + t * RS;
    T* const my_suf = suf + t * RS;
    T v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = my_raw[r];
    T run = e;
#pragma unroll
    for (int r = 0; r < E; ++r) run = Op::apply(run, v[r]);
    const T ip = wave_prefix<T, Op>(run, lane);
    const T is = wave_suffix<T, Op>(run, lane);
    if (lane == 63) wt[0][wv] = ip;
    if (lane == 0) wt[1][wv] = is;
    if (t == 0 && hlen > 0) {
        // inclusive suffixes inside the next chunk's first k elements
        T s = tail;
        for (int r = k - 1; r >= 0; --r) {
            s = Op::apply(raw[L1_THREADS * RS + r], s);
            hs[r] = s;
        }
    }
    __syncthreads();
    T lo = cp, hi = cs;
#pragma unroll
    for (int w = 0; w < L1_THREADS / 64; ++w)
        if (w < wv) lo = Op::apply(lo, wt[0][w]);
#pragma unroll
    for (int w = L1_THREADS / 64 - 1; w >= 0; --w)
        if (w > wv) hi = Op::apply(wt[1][w], hi);
    const T up = __shfl_up(ip, 1, 64), dn = __shfl_down(is, 1, 64);
    const T pre = lane > 0 ? Op::apply(lo, up) : lo;   // P before x0
    T s = lane < 63 ? Op::apply(dn, hi) : hi;          // S after the run
    // inclusive suffixes S[x0 + r] for the other threads, and the range
    // suffixes of this thread's k-blocks (the first half of BDBS)
    T bs[E];
    T b = e;
    int left = 0;  // elements of the current block below r
#pragma unroll
    for (int r = E - 1; r >= 0; --r) {
        s = Op::apply(v[r], s);
        my_suf[r] = s;
        b = left == 0 ? v[r] : Op::apply(v[r], b);
        left = left == 0 ? k - 1 : left - 1;
        bs[r] = b;
    }
    __syncthreads();
    // Exc[x] = P[x - 1] op S[x + k]; Inc[x] = range suffix op the range prefix
    // of the next block up to x + k - 1.  Position x0 + j (j < 2E) sits at
    // my_raw[j + (j >= E)]: the next run, or the halo after the last run.
    T ex[E];
    T p = pre, q = e;
    int o = 0;  // offset of x0 + r in its block
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int j = r + k;
        T sy;
        if (x0 + j >= rem) sy = e;
        else if (t == L1_THREADS - 1 && j >= E) sy = hs[j - E];
        else sy = my_suf[j + (j >= E ? 1 : 0)];
        ex[r] = Op::apply(p, sy);
        p = Op::apply(p, v[r]);
        const int jp = j - 1;
        q = o == 0 ? e : Op::apply(q, my_raw[jp + (jp >= E ? 1 : 0)]);
        bs[r] = o == 0 ? bs[r] : Op::apply(bs[r], q);
        o = o + 1 == k ? 0 : o + 1;
    }
    // coalesced stores through LDS; the buffer range drops the lanes past the
    // tensor's end
    __syncthreads();
    if (exc) {
#pragma unroll
        for (int r = 0; r < E; ++r) my_raw[r] = ex[r];
        __syncthreads();
        const __amdgpu_buffer_rsrc_t dst = buf(exc + base, (unsigned)len * sizeof(T));
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int i = t + r * L1_THREADS;
            bstore<T>(dst, (unsigned)i * sizeof(T), raw[(i / E) * RS + i % E]);
        }
        __syncthreads();
    }
    if (inc) {
#pragma unroll
        for (int r = 0; r < E; ++r) my_raw[r] = bs[r];
        __syncthreads();
        const __amdgpu_buffer_rsrc_t dst = buf(inc + base, (unsigned)len * sizeof(T));
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int i = t + r * L1_THREADS;
            bstore<T>(dst, (unsigned)i * sizeof(T), raw[(i / E) * RS + i % E]);
        }
    }
}

i64 long1d_chunks(i64 n, i64 k) { return (n + (i64)L1_THREADS * l1_elems(k) - 1) / ((i64)L1_THREADS * l1_elems(k)); }

bool long1d_ok(i64 n, i64 k) {
    return k <= 16 && n < ((i64)1 << 31) - 64 && long1d_chunks(n, k) <= L1_MAX_CHUNKS;
}

template <typename T, class Op>
void launch_long1d(const T* A, T* exc, T* inc, i64 n, i64 k, T* Tt, T* Ut, T* CP, T* CS,
                   hipStream_t st) {
    const int E = l1_elems(k), C = L1_THREADS * E;
    const i64 nc = long1d_chunks(n, k);
    if (exc) {
        // the chunk offsets (the included sums alone need none)
        {
            KTimer timer("k_l1_tot", st);
            hipLaunchKernelGGL((k_l1_tot<T, Op>), dim3((unsigned)nc), dim3(L1_THREADS), 0, st, A,
                               Tt, Ut, n, C, (int)k);
        }
        KTimer timer("k_l1_scan", st);
        hipLaunchKernelGGL((k_l1_scan<T, Op>), dim3(1), dim3(L1_SCAN_THREADS), 0, st, Tt, CP, CS,
                           (int)nc);
    }
    KTimer timer("k_l1_out", st);
    switch (E) {
#define EXS_L1_CASE(EE)                                                                          \
    case EE:                                                                                     \
        hipLaunchKernelGGL((k_l1_out<T, Op, EE>), dim3((unsigned)nc), dim3(L1_THREADS), 0, st, A, \
                           CP, CS, Ut, exc, inc, n, (int)k);                                     \
        break;
        EXS_L1_CASE(16)
        EXS_L1_CASE(18)
        EXS_L1_CASE(20)
        EXS_L1_CASE(21)
        EXS_L1_CASE(22)
        EXS_L1_CASE(24)
        EXS_L1_CASE(26)
        EXS_L1_CASE(28)
        EXS_L1_CASE(30)
#undef EXS_L1_CASE
        default: break;  // not reached: long1d_ok admits k <= 16, whose E are the cases above
    }
}

template void launch_long1d<float, OpSum>(const float*, float*, float*, i64, i64, float*, float*,
                                          float*, float*, hipStream_t);
template void launch_long1d<float, OpMax>(const float*, float*, float*, i64, i64, float*, float*,
                                          float*, float*, hipStream_t);
template void launch_long1d<int, OpSum>(const int*, int*, int*, i64, i64, int*, int*, int*, int*,
                                        hipStream_t);
template void launch_long1d<int, OpMax>(const int*, int*, int*, i64, i64, int*, int*, int*, int*,
                                        hipStream_t);
template void launch_long1d<float, OpMin>(const float*, float*, float*, i64, i64, float*, float*,
                                          float*, float*, hipStream_t);
template void launch_long1d<int, OpMin>(const int*, int*, int*, i64, i64, int*, int*, int*, int*,
                                        hipStream_t);
template void launch_long1d<float, OpSlowSum>(const float*, float*, float*, i64, i64, float*,
                                              float*, float*, float*, hipStream_t);
hipError_t slow_cost_set_ex1d(int c) { return set_slow_cost_here(c); }

}  // namespace exs
