// exsum_small2d.hip -- included and excluded sums of a small rank-2 tensor in
// one workgroup.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// For d = 2 the box-complement method (Sec. 5) is two levels: level 0
// streams axis 0 of W = BDBS of A along axis 1, and level 1 is the 1-D
// excluded sum of R_1 = A reduced over axis 0.  On the general path that is a
// chain of six or more launches (block aggregates, their box sums and scans,
// the row box sums, the axis-0 stream, the 1-D level).  A tensor that fits in
// LDS takes all of it in one workgroup, from one read of A:
//   R1[x1]    = op of A[., x1] over axis 0;
//   W         = BDBS of A along axis 1 (Sec. 3: the range suffix of a k1-block
//               op the range prefix of the next block);
//   Exc1[x1]  = op of R1 before x1 op op of R1 from x1 + k1 (level 1);
//   Exc[x]    = op of W[., x1] before x0 op op of W[., x1] from x0 + k0
//               op Exc1[x1]   (the component pairs of Corollary
//               "Excluded-sum Components": axis 0's pair on the box-summed
//               tensor, axis 1's pair through R1);
//   Inc[x]    = BDBS of W along axis 0 (the included sum).
// Box sums are one task per (row or column, block); the scans along axis 0
// give each column up to 64 threads, each walking a chunk of rows from the
// other chunks' totals.
#include "exsum_internal.hpp"
#include "exsum_tasks.hpp"

namespace exs {

constexpr int S2_THREADS = 1024;

template <typename T, class Op>
__global__ __launch_bounds__(1024) void k_small2d(const T* __restrict__ A, T* __restrict__ exc,
                                                  T* __restrict__ inc, int n0, int n1, int k0,
                                                  int k1) {
    static_assert(sizeof(T) <= 8, "elements of at most 8 bytes");
    __shared__ __align__(16) unsigned char lds[3 * SMALL2D_BYTES + 3 * SMALL2D_MAX_N1 * 8];
    __shared__ T part[S2_THREADS];
    const int N = n0 * n1;
    T* L0 = (T*)lds;   // A, then W
    T* L1 = L0 + N;    // range suffixes; column prefixes
    T* L2 = L1 + N;    // range prefixes; column suffixes
    T* R1 = L2 + N;    // column totals, then Exc1
    T* P1 = R1 + n1;   // scan buffers of the 1-D level
    T* S1 = P1 + n1;
    const T e = Op::template id<T>();
    const int t = threadIdx.x;
    const bool want_exc = exc != nullptr;
    // column walks: G threads per column (a power of two, at most 64), each
    // over a chunk of c consecutive rows; thread t takes column t % n1
    int G = 1;
    while (G < 64 && 2 * G * n1 <= S2_THREADS && G < n0) G *= 2;
    const int c = (n0 + G - 1) / G;
    const int cx = t % n1, cg = t / n1;
    const bool walker = cg < G;
    const int r0 = cg * c, r1 = r0 + c < n0 ? r0 + c : n0;

    for (int i = t; i < N; i += S2_THREADS) L0[i] = A[i];
    __syncthreads();
    // column totals (the reduction of axis 0), before A is replaced by W:
    // chunk totals, then their op per column
    if (want_exc && walker) {
        T r = e;
        for (int x0 = r0; x0 < r1; ++x0) r = Op::apply(r, L0[x0 * n1 + cx]);
        part[cg * n1 + cx] = r;
    }
    // range prefixes (L2) and range suffixes (L1) of every k1-block of every row
    const int nb1 = (n1 + k1 - 1) / k1;
    for (int task = t; task < n0 * nb1; task += S2_THREADS) {
        const int x0 = task / nb1, b = task - x0 * nb1;
        const int lo = b * k1, hi = lo + k1 < n1 ? lo + k1 : n1;
        const T* row = L0 + x0 * n1;
        T p = e;
        for (int y = lo; y < hi; ++y) {
            p = Op::apply(p, row[y]);
            L2[x0 * n1 + y] = p;
        }
        T s = e;
        for (int y = hi - 1; y >= lo; --y) {
            s = Op::apply(row[y], s);
            L1[x0 * n1 + y] = s;
        }
    }
    __syncthreads();
    if (want_exc && t < n1) {
        T r = e;
        for (int g = 0; g < G; ++g) r = Op::apply(r, part[g * n1 + t]);
        R1[t] = r;
    }
    // W[x0, x1] = suffix of x1's block from x1 op prefix of the next block up
    // to x1 + k1 - 1 (clipped at the row's end)
    for (int i = t; i < N; i += S2_THREADS) {
        const int x0 = i / n1, x1 = i - x0 * n1;
        const int r = x1 % k1, nxt = x1 - r + k1;
        T w = L1[i];
        if (r > 0 && nxt < n1) {
            const int y = x1 + k1 - 1 < n1 ? x1 + k1 - 1 : n1 - 1;
            w = Op::apply(w, L2[x0 * n1 + y]);
        }
        L0[i] = w;
    }
    __syncthreads();
    if (want_exc) {
        // level 1: inclusive prefix (P1) and suffix (S1) of R1 by doubling
        // steps over the workgroup (n1 <= 1024, one element per thread)
        const T v = t < n1 ? R1[t] : e;
        if (t < n1) { P1[t] = v; S1[t] = v; }
        // chunk totals of W for the column walks below
        if (walker) {
            T r = e;
            for (int x0 = r0; x0 < r1; ++x0) r = Op::apply(r, L0[x0 * n1 + cx]);
            part[cg * n1 + cx] = r;
        }
        __syncthreads();
        for (int off = 1; off < n1; off <<= 1) {
            T a = e, b = e;
            if (t < n1) {
                a = t >= off ? P1[t - off] : e;
                b = t + off < n1 ? S1[t + off] : e;
            }
            __syncthreads();
            if (t < n1) {
                P1[t] = Op::apply(a, P1[t]);
                S1[t] = Op::apply(S1[t], b);
            }
            __syncthreads();
        }
        if (t < n1)
            R1[t] = Op::apply(t >= 1 ? P1[t - 1] : e, t + k1 < n1 ? S1[t + k1] : e);
        // level 0 along axis 0: op of W's column before each row (L1) and
        // from each row on (L2), each chunk started from the other chunks'
        // totals
        if (walker) {
            T p = e, s = e;
            for (int g = 0; g < cg; ++g) p = Op::apply(p, part[g * n1 + cx]);
            for (int g = G - 1; g > cg; --g) s = Op::apply(part[g * n1 + cx], s);
            for (int x0 = r0; x0 < r1; ++x0) {
                L1[x0 * n1 + cx] = p;
                p = Op::apply(p, L0[x0 * n1 + cx]);
            }
            for (int x0 = r1 - 1; x0 >= r0; --x0) {
                s = Op::apply(L0[x0 * n1 + cx], s);
                L2[x0 * n1 + cx] = s;
            }
        }
        __syncthreads();
        for (int i = t; i < N; i += S2_THREADS) {
            const int x0 = i / n1, x1 = i - x0 * n1;
            const T after = x0 + k0 < n0 ? L2[i + k0 * n1] : e;
            exc[i] = Op::apply(Op::apply(L1[i], after), R1[x1]);
        }
        __syncthreads();
    }
    if (inc) {
        // BDBS along axis 0: range prefixes and suffixes of every k0-block of
        // every column, then the same combine as along the rows
        const int nb0 = (n0 + k0 - 1) / k0;
        for (int task = t; task < n1 * nb0; task += S2_THREADS) {
            const int b = task / n1, x1 = task - b * n1;
            const int lo = b * k0, hi = lo + k0 < n0 ? lo + k0 : n0;
            T p = e;
            for (int y = lo; y < hi; ++y) {
                p = Op::apply(p, L0[y * n1 + x1]);
                L2[y * n1 + x1] = p;
            }
            T s = e;
            for (int y = hi - 1; y >= lo; --y) {
                s = Op::apply(L0[y * n1 + x1], s);
                L1[y * n1 + x1] = s;
            }
        }
        __syncthreads();
        for (int i = t; i < N; i += S2_THREADS) {
            const int x0 = i / n1, x1 = i - x0 * n1;
            const int r = x0 % k0, nxt = x0 - r + k0;
            T v = L1[i];
            if (r > 0 && nxt < n0) {
                const int y = x0 + k0 - 1 < n0 ? x0 + k0 - 1 : n0 - 1;
                v = Op::apply(v, L2[y * n1 + x1]);
            }
            inc[i] = v;
        }
    }
}

bool small2d_eligible(i64 n0, i64 n1, i64 k0, i64 k1, int es) {
    (void)k0;
    return n0 >= 1 && n1 >= 1 && n0 <= SMALL2D_MAX_N0 && n1 <= SMALL2D_MAX_N1 &&
           k1 <= SMALL2D_MAX_K1 && n0 * n1 * es <= SMALL2D_BYTES;
}

template <typename T, class Op>
void launch_small2d(const T* A, T* exc, T* inc, i64 n0, i64 n1, i64 k0, i64 k1, hipStream_t st) {
    KTimer timer("k_small2d", st);
    hipLaunchKernelGGL((k_small2d<T, Op>), dim3(1), dim3(S2_THREADS), 0, st, A, exc, inc, (int)n0,
                       (int)n1, (int)k0, (int)k1);
}

#define EXS_S2(T)                                                                            \
    template void launch_small2d<T, OpSum>(const T*, T*, T*, i64, i64, i64, i64, hipStream_t); \
    template void launch_small2d<T, OpMax>(const T*, T*, T*, i64, i64, i64, i64, hipStream_t); \
    template void launch_small2d<T, OpMin>(const T*, T*, T*, i64, i64, i64, i64, hipStream_t);
EXS_S2(float)
EXS_S2(double)
EXS_S2(int)
EXS_S2(long long)
#undef EXS_S2

}  // namespace exs
