// exsum_tailbox.hip -- BDBS along the last m axes of a tensor in one pass,
// for trailing sub-tensors small enough for LDS.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// BDBS-Along-Dim (Sec. 5; the 1-D algorithm of Sec. 3) applied to axes
// d-1, d-2, ..., d-m in turn, the innermost axis first.  When those axes span
// at most TB_BYTES of elements, each workgroup stages one trailing sub-tensor
// in LDS, runs the m passes there (ping-pong between two buffers) and writes
// the result once: one read and one write of the tensor instead of m of each.
// Per row of an axis: the range suffix within each k-block (a descending
// scan), then the range prefix of the next block up to x + k - 1 (an
// ascending scan) added to every cell that is not a block start.
#include "exsum_internal.hpp"
#include "exsum_device.hpp"

namespace exs {

constexpr int TB_THREADS = 256;
constexpr int TB_BYTES = 16384;  // one staged sub-tensor; the LDS holds two

struct TailDims {
    int m, S;                  // axes, elements of the sub-tensor
    int n[EXS_MAX_RANK];       // extents, outermost first
    int k[EXS_MAX_RANK];       // box sides
    int st[EXS_MAX_RANK];      // strides within the sub-tensor
};

template <typename T, class Op>
__global__ __launch_bounds__(TB_THREADS) void k_bdbs_tail(const T* __restrict__ in,
                                                          T* __restrict__ out, i64 O,
                                                          TailDims td) {
    constexpr int CAP = TB_BYTES / (int)sizeof(T);
    __shared__ T buf0[CAP];
    __shared__ T buf1[CAP];
    const T e = Op::template id<T>();
    const int t = threadIdx.x;
    const int S = td.S;
    for (i64 o = blockIdx.x; o < O; o += gridDim.x) {
        const T* __restrict__ src = in + o * S;
        T* a = buf0;
        T* b = buf1;
        for (int i = t; i < S; i += TB_THREADS) a[i] = src[i];
        __syncthreads();
        for (int ax = td.m - 1; ax >= 0; --ax) {
            const int n = td.n[ax], k = td.k[ax], st = td.st[ax];
            const int rows = S / n;
            for (int r = t; r < rows; r += TB_THREADS) {
                const int base = (r / st) * n * st + r % st;
                // range suffix within each block (blocks end at multiples of
                // k and at the row's end); off is x's offset in its block
                T s = e;
                int off = (n - 1) % k;
                for (int x = n - 1; x >= 0; --x) {
                    const T v = a[base + x * st];
                    s = (off == k - 1 || x == n - 1) ? v : Op::apply(v, s);
                    b[base + x * st] = s;
                    off = off == 0 ? k - 1 : off - 1;
                }
                // op the next block's range prefix up to x + k - 1
                T q = e;
                off = 0;
                for (int x = 0; x < n; ++x, off = off + 1 == k ? 0 : off + 1) {
                    if (off == 0) {
                        q = e;
                        continue;
                    }
                    const int y = x + k - 1;
                    if (y < n) q = Op::apply(q, a[base + y * st]);
                    b[base + x * st] = Op::apply(b[base + x * st], q);
                }
            }
            __syncthreads();
            T* tmp = a;
            a = b;
            b = tmp;
        }
        T* __restrict__ dst = out + o * S;
        for (int i = t; i < S; i += TB_THREADS) dst[i] = a[i];
        __syncthreads();  // the next sub-tensor overwrites the buffers
    }
}

i64 tail_box_max_elems(int es) { return TB_BYTES / es; }

template <typename T, class Op>
void launch_bdbs_tail(const T* in, T* out, i64 O, int m, const i64* n, const i64* k,
                      hipStream_t st) {
    TailDims td{};
    td.m = m;
    i64 S = 1;
    for (int a = m - 1; a >= 0; --a) {
        td.n[a] = (int)n[a];
        td.k[a] = (int)k[a];
        td.st[a] = (int)S;
        S *= n[a];
    }
    td.S = (int)S;
    const i64 grid = O < 65536 ? O : 65536;
    KTimer timer("k_bdbs_tail", st);
    hipLaunchKernelGGL((k_bdbs_tail<T, Op>), dim3((unsigned)grid), dim3(TB_THREADS), 0, st, in,
                       out, O, td);
}

#define EXS_TB_INST(T, OP)                                                                 \
    template void launch_bdbs_tail<T, OP>(const T*, T*, i64, int, const i64*, const i64*, \
                                          hipStream_t);
EXS_TB_INST(float, OpSum)
EXS_TB_INST(double, OpSum)
EXS_TB_INST(int, OpSum)
EXS_TB_INST(long long, OpSum)
EXS_TB_INST(float, OpMax)
EXS_TB_INST(double, OpMax)
EXS_TB_INST(int, OpMax)
EXS_TB_INST(long long, OpMax)
EXS_TB_INST(float, OpMin)
EXS_TB_INST(double, OpMin)
EXS_TB_INST(int, OpMin)
EXS_TB_INST(long long, OpMin)
EXS_TB_INST(float, OpSlowSum)
EXS_TB_INST(ValIdx, OpMax)
EXS_TB_INST(ValIdx, OpMin)
#undef EXS_TB_INST

hipError_t slow_cost_set_tailbox(int c) { return set_slow_cost_here(c); }

}  // namespace exs
