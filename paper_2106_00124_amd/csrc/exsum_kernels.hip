// exsum_kernels.hip -- HIP kernels (gfx950) for included and excluded sums.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// Kernels of the generic path (any rank 1..8, any box):
//   k_bdbs          BDBS along one axis (Sec. 3; "BDBS-Along-Dim", Sec. 5),
//                   one thread per row chunk, block suffixes in registers.
//   k_bdbs_2sweep   the same for boxes longer than 64 (two sweeps per row).
//   k_blockagg      block aggregates along axis 0 (op over each k0-block):
//                   the first half of a prefix/suffix along the axis.
//   k_blockscan     exclusive prefix/suffix over the blocks and the full
//                   reduction over axis 0 ("dimension reduction", Sec. 5).
//   k_axis0         streams axis 0: prefix and suffix along the axis merged
//                   with the box-sum along it and the contribution of the
//                   lower-dimensional excluded sum (Sec. 5, "Adding in the
//                   Contribution").
//   k_ex1d_2sweep   the axis-0 excluded part for boxes longer than 64.
//   k_fill          counter-based input generator (workload support).
#include "exsum_device.hpp"
#include "exsum_internal.hpp"

namespace exs {

// ---------------------------------------------------------------------------
// BDBS along an axis of a tensor viewed as (O, n, I).  Threads map to
// (o, chunk, i) with i fastest, so loads and stores are coalesced whenever
// I >= 64; each thread streams `cb` blocks of its row.
// ---------------------------------------------------------------------------
template <typename T, class Op, int KB>
__global__ __launch_bounds__(256) void k_bdbs(const T* __restrict__ in, T* __restrict__ out,
                                              i64 O, i64 n, i64 I, int k, i64 cb,
                                              i64 nchunks) {
    const i64 idx = gtid();
    if (idx >= O * nchunks * I) return;
    const i64 i = idx % I;
    const i64 rest = idx / I;
    const i64 c = rest % nchunks;
    const i64 o = rest / nchunks;
    const i64 nb = (n + k - 1) / k;
    const i64 b0 = c * cb;
    if (b0 >= nb) return;
    const i64 b1 = b0 + cb < nb ? b0 + cb : nb;
    const i64 off = o * n * I + i;
    bdbs_row<T, Op, KB>(in + off, out + off, n, I, k, b0, b1);
}

// Two-sweep BDBS for k > 64: the backward sweep writes the range suffixes,
// the forward sweep adds the range prefix of the next block (out != in).
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_bdbs_2sweep(const T* __restrict__ in,
                                                     T* __restrict__ out, i64 O, i64 n,
                                                     i64 I, i64 k) {
    const i64 idx = gtid();
    if (idx >= O * I) return;
    const i64 i = idx % I, o = idx / I;
    const T* src = in + o * n * I + i;
    T* dst = out + o * n * I + i;
    const T e = Op::template id<T>();
    T rs = e;
    for (i64 x = n - 1; x >= 0; --x) {
        const bool last = (x % k == k - 1) || (x == n - 1);
        rs = last ? src[x * I] : Op::apply(src[x * I], rs);
        dst[x * I] = rs;
    }
    T rp = e;
    for (i64 t = 0; t < n; ++t) {
        rp = (t % k == 0) ? src[t * I] : Op::apply(rp, src[t * I]);
        const i64 x = t - k + 1;
        if (x >= 0 && x % k != 0) dst[x * I] = Op::apply(dst[x * I], rp);
    }
    // windows whose next block is the partial last block and reach past n
    const i64 L = (n - 1) / k, Ls = L * k;
    if (L >= 1) {
        i64 lo = Ls - k + 1;
        if (n - k + 1 > lo) lo = n - k + 1;
        for (i64 x = lo; x < Ls; ++x) dst[x * I] = Op::apply(dst[x * I], rp);
    }
}

// Ga[q, m] = op over t in block q of X[t, m]; X viewed as (n0, M).
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_blockagg(const T* __restrict__ X, T* __restrict__ Ga,
                                                  i64 n0, i64 M, i64 k0, i64 Q) {
    const i64 idx = gtid();
    if (idx >= Q * M) return;
    const i64 m = idx % M, q = idx / M;
    const i64 t0 = q * k0;
    const i64 t1 = t0 + k0 < n0 ? t0 + k0 : n0;
    T s = Op::template id<T>();
#pragma unroll 8
    for (i64 t = t0; t < t1; ++t) s = Op::apply(s, X[t * M + m]);
    Ga[idx] = s;
}

// The same for 4-byte elements with M % 4 == 0: each thread owns 4
// consecutive points (16-byte loads), 8 planes in flight at a time.
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_blockagg4(const T* __restrict__ X, T* __restrict__ Ga,
                                                   i64 n0, i64 M, i64 k0, i64 Q) {
    static_assert(sizeof(T) == 4, "4-byte elements");
    const i64 M4 = M >> 2;
    const i64 idx = gtid();
    if (idx >= Q * M4) return;
    // blocks in descending order: the planes read last (low axis-0 index) are
    // the ones the streaming kernel reads first, while they may still sit in
    // the last-level cache
    const i64 m4 = idx % M4, q = Q - 1 - idx / M4;
    const i64 t0 = q * k0;
    const i64 t1 = t0 + k0 < n0 ? t0 + k0 : n0;
    const uint4* __restrict__ src = (const uint4*)X + m4;
    const T e = Op::template id<T>();
    T s0 = e, s1 = e, s2 = e, s3 = e;
    i64 t = t0;
    for (; t + 8 <= t1; t += 8) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[(t + u) * M4];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            s0 = Op::apply(s0, __builtin_bit_cast(T, v[u].x));
            s1 = Op::apply(s1, __builtin_bit_cast(T, v[u].y));
            s2 = Op::apply(s2, __builtin_bit_cast(T, v[u].z));
            s3 = Op::apply(s3, __builtin_bit_cast(T, v[u].w));
        }
    }
    for (; t < t1; ++t) {
        const uint4 v = src[t * M4];
        s0 = Op::apply(s0, __builtin_bit_cast(T, v.x));
        s1 = Op::apply(s1, __builtin_bit_cast(T, v.y));
        s2 = Op::apply(s2, __builtin_bit_cast(T, v.z));
        s3 = Op::apply(s3, __builtin_bit_cast(T, v.w));
    }
    uint4 o;
    o.x = __builtin_bit_cast(unsigned, s0);
    o.y = __builtin_bit_cast(unsigned, s1);
    o.z = __builtin_bit_cast(unsigned, s2);
    o.w = __builtin_bit_cast(unsigned, s3);
    ((uint4*)Ga)[q * M4 + m4] = o;
}

// Per point m: PX[q] = op of Gw[q'] for q' < q, SX[q] = op of Gw[q'] for
// q' > q, R[m] = op over all blocks of Ga (the reduction of axis 0).
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_blockscan(const T* __restrict__ Gw,
                                                   const T* __restrict__ Ga,
                                                   T* __restrict__ PX, T* __restrict__ SX,
                                                   T* __restrict__ R, i64 Q, i64 M) {
    const i64 m = gtid();
    if (m >= M) return;
    const T e = Op::template id<T>();
    T p = e, r = e;
#pragma unroll 8
    for (i64 q = 0; q < Q; ++q) {
        PX[q * M + m] = p;
        p = Op::apply(p, Gw[q * M + m]);
        r = Op::apply(r, Ga[q * M + m]);
    }
    T s = e;
#pragma unroll 8
    for (i64 q = Q - 1; q >= 0; --q) {
        SX[q * M + m] = s;
        s = Op::apply(Gw[q * M + m], s);
    }
    if (R) R[m] = r;
}

// Axis-0 stream for the generic path.  Threads map to (segment, m), m
// fastest; each thread owns one point m and a run of blocks [qa, qb) of
// axis 0, reading one block ahead.
template <typename T, class Op, int K0B>
__global__ __launch_bounds__(256) void k_axis0(const T* __restrict__ W, const T* __restrict__ PX,
                                               const T* __restrict__ SX,
                                               const T* __restrict__ Trest, T* __restrict__ exc,
                                               T* __restrict__ inc, i64 n0, i64 M, int k0,
                                               i64 Q, i64 segblocks, i64 nseg) {
    const i64 idx = gtid();
    if (idx >= nseg * M) return;
    const i64 m = idx % M, s = idx / M;
    const i64 qa = s * segblocks;
    if (qa >= Q) return;
    const i64 qb = qa + segblocks < Q ? qa + segblocks : Q;
    const bool do_ex = exc != nullptr, do_inc = inc != nullptr;
    const T e = Op::template id<T>();
    const T* src = W + m;

    Axis0State<T, Op, K0B> st;
    T v[K0B];
#pragma unroll
    for (int r = 0; r < K0B; ++r) {
        const i64 x = qa * k0 + r;
        v[r] = (r < k0 && x < n0) ? src[x * M] : e;
    }
    st.P = e;
    if (do_ex) {
        st.P = PX[qa * M + m];
        if (Trest) st.P = Op::apply(st.P, Trest[m]);
    }
    st.absorb(v, k0, do_ex, do_inc);

    for (i64 q = qa; q < qb; ++q) {
        const i64 nbase = (q + 1) * k0;
#pragma unroll
        for (int r = 0; r < K0B; ++r) {
            const i64 x = nbase + r;
            v[r] = (r < k0 && x < n0) ? src[x * M] : e;
        }
        if (do_ex) {
            T S = (q + 1 < Q) ? SX[(q + 1) * M + m] : e;
#pragma unroll
            for (int r = K0B - 1; r >= 0; --r) {
                if (r < k0) {
                    S = Op::apply(v[r], S);
                    const i64 x = q * k0 + r;
                    if (x < n0) exc[x * M + m] = Op::apply(st.pex[r], S);
                }
            }
        }
        if (do_inc) {
            T p = e;
#pragma unroll
            for (int r = 0; r < K0B; ++r) {
                if (r < k0) {
                    T val = st.rs[r];
                    if (r > 0) { p = Op::apply(p, v[r - 1]); val = Op::apply(val, p); }
                    const i64 x = q * k0 + r;
                    if (x < n0) inc[x * M + m] = val;
                }
            }
        }
        if (q + 1 < qb) st.absorb(v, k0, do_ex, do_inc);
    }
}

// Axis-0 excluded part for k0 > 64, one thread per point, two sweeps:
// the backward sweep stores the suffix from x0 + k0, the forward sweep
// prepends the prefix before x0 and the lower-dimensional term.
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_ex1d_2sweep(const T* __restrict__ W,
                                                     const T* __restrict__ Trest,
                                                     T* __restrict__ exc, i64 n0, i64 M,
                                                     i64 k0) {
    const i64 m = gtid();
    if (m >= M) return;
    const T e = Op::template id<T>();
    for (i64 x = n0 - k0; x < n0; ++x)
        if (x >= 0) exc[x * M + m] = e;
    T S = e;
    for (i64 t = n0 - 1; t >= 0; --t) {
        S = Op::apply(W[t * M + m], S);
        if (t - k0 >= 0) exc[(t - k0) * M + m] = S;
    }
    T P = Trest ? Trest[m] : e;
    for (i64 x = 0; x < n0; ++x) {
        exc[x * M + m] = Op::apply(P, exc[x * M + m]);
        P = Op::apply(P, W[x * M + m]);
    }
}

// ---------------------------------------------------------------------------
// Counter-based input generator (bit-identical host twin in workloads.py).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_fill(void* out, i64 count, int dtype, int kind,
                                              uint64_t seed, i64 lo, i64 hi, float scale) {
    for (i64 i = gtid(); i < count; i += (i64)gridDim.x * blockDim.x) {
        const uint64_t z = splitmix_at(seed, (uint64_t)i);
        if (kind == 0) {
            const i64 s = (i64)(z & 0xFFFF) + (i64)((z >> 16) & 0xFFFF) +
                          (i64)((z >> 32) & 0xFFFF) + (i64)((z >> 48) & 0xFFFF) - 2 * 65535;
            ((float*)out)[i] = __fmul_rn((float)s, scale);
        } else if (kind == 1) {
            const uint64_t span = (uint64_t)(hi - lo + 1);
            const i64 v = (i64)(z % span) + lo;
            if (dtype == 2) ((int*)out)[i] = (int)v;
            else ((long long*)out)[i] = v;
        } else {
            const uint32_t sign = (uint32_t)(z >> 63);
            const i64 ex = (i64)((z >> 32) % 20ULL) - 10;
            const uint32_t mant = (uint32_t)(z & 0x7FFFFFULL);
            const uint32_t bits = (sign << 31) | ((uint32_t)(ex + 127) << 23) | mant;
            ((uint32_t*)out)[i] = bits;
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(i64 threads, int block = 256) {
    i64 g = (threads + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

static inline int bucket_for(i64 k) {
    if (k <= 1) return 1;
    if (k <= 2) return 2;
    if (k <= 4) return 4;
    if (k <= 8) return 8;
    if (k <= 16) return 16;
    if (k <= 32) return 32;
    if (k <= 64) return 64;
    return 0;
}

template <typename T, class Op>
void launch_bdbs(const T* in, T* out, i64 O, i64 n, i64 I, i64 k, hipStream_t st) {
    const int kb = bucket_for(k);
    KTimer timer(kb == 0 ? "k_bdbs_2sweep" : "k_bdbs", st);
    if (kb == 0) {
        hipLaunchKernelGGL((k_bdbs_2sweep<T, Op>), dim3(grid_for(O * I)), dim3(256), 0, st,
                           in, out, O, n, I, k);
        return;
    }
    const i64 nb = (n + k - 1) / k;
    const i64 cols = O * I;
    i64 nchunks = (65536 + cols - 1) / cols;
    if (nchunks > nb) nchunks = nb;
    if (nchunks < 1) nchunks = 1;
    const i64 cb = (nb + nchunks - 1) / nchunks;
    nchunks = (nb + cb - 1) / cb;
    const unsigned g = grid_for(cols * nchunks);
#define EXS_BDBS_CASE(KB)                                                                   \
    case KB:                                                                                \
        hipLaunchKernelGGL((k_bdbs<T, Op, KB>), dim3(g), dim3(256), 0, st, in, out, O, n, I, \
                           (int)k, cb, nchunks);                                            \
        break;
    switch (kb) {
        EXS_BDBS_CASE(1) EXS_BDBS_CASE(2) EXS_BDBS_CASE(4) EXS_BDBS_CASE(8)
        EXS_BDBS_CASE(16) EXS_BDBS_CASE(32) EXS_BDBS_CASE(64)
    }
#undef EXS_BDBS_CASE
}

template <typename T, class Op>
void launch_blockagg(const T* X, T* Ga, i64 n0, i64 M, i64 k0, i64 Q, hipStream_t st) {
    KTimer timer("k_blockagg", st);
    if constexpr (sizeof(T) == 4) {
        if (M % 4 == 0 && ((uintptr_t)X & 15) == 0 && ((uintptr_t)Ga & 15) == 0) {
            hipLaunchKernelGGL((k_blockagg4<T, Op>), dim3(grid_for(Q * (M / 4))), dim3(256), 0, st,
                               X, Ga, n0, M, k0, Q);
            return;
        }
    }
    hipLaunchKernelGGL((k_blockagg<T, Op>), dim3(grid_for(Q * M)), dim3(256), 0, st, X, Ga, n0,
                       M, k0, Q);
}

template <typename T, class Op>
void launch_blockscan(const T* Gw, const T* Ga, T* PX, T* SX, T* R, i64 Q, i64 M,
                      hipStream_t st) {
    KTimer timer("k_blockscan", st);
    hipLaunchKernelGGL((k_blockscan<T, Op>), dim3(grid_for(M)), dim3(256), 0, st, Gw, Ga, PX,
                       SX, R, Q, M);
}

template <typename T, class Op>
void launch_axis0(const T* W, const T* PX, const T* SX, const T* Trest, T* exc, T* inc, i64 n0,
                  i64 M, i64 k0, i64 Q, hipStream_t st) {
    const int kb = bucket_for(k0);
    if (kb == 0) {
        KTimer timer("k_ex1d_2sweep", st);
        if (exc)
            hipLaunchKernelGGL((k_ex1d_2sweep<T, Op>), dim3(grid_for(M)), dim3(256), 0, st, W,
                               Trest, exc, n0, M, k0);
        if (inc) launch_bdbs<T, Op>(W, inc, 1, n0, M, k0, st);
        return;
    }
    i64 nseg = (65536 + M - 1) / M;
    if (nseg > Q) nseg = Q;
    if (nseg < 1) nseg = 1;
    const i64 segblocks = (Q + nseg - 1) / nseg;
    nseg = (Q + segblocks - 1) / segblocks;
    const unsigned g = grid_for(nseg * M);
    KTimer timer("k_axis0", st);
#define EXS_AX0_CASE(KB)                                                                    \
    case KB:                                                                                \
        hipLaunchKernelGGL((k_axis0<T, Op, KB>), dim3(g), dim3(256), 0, st, W, PX, SX, Trest, \
                           exc, inc, n0, M, (int)k0, Q, segblocks, nseg);                   \
        break;
    switch (kb) {
        EXS_AX0_CASE(1) EXS_AX0_CASE(2) EXS_AX0_CASE(4) EXS_AX0_CASE(8)
        EXS_AX0_CASE(16) EXS_AX0_CASE(32) EXS_AX0_CASE(64)
    }
#undef EXS_AX0_CASE
}

void launch_fill(void* out, i64 count, int dtype, int kind, uint64_t seed, i64 lo, i64 hi,
                 float scale, hipStream_t st) {
    i64 g = (count + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    KTimer timer("k_fill", st);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(256), 0, st, out, count, dtype, kind,
                       seed, lo, hi, scale);
}

#define EXS_INSTANTIATE(T, OP)                                                                 \
    template void launch_bdbs<T, OP>(const T*, T*, i64, i64, i64, i64, hipStream_t);           \
    template void launch_blockagg<T, OP>(const T*, T*, i64, i64, i64, i64, hipStream_t);       \
    template void launch_blockscan<T, OP>(const T*, const T*, T*, T*, T*, i64, i64,            \
                                          hipStream_t);                                        \
    template void launch_axis0<T, OP>(const T*, const T*, const T*, const T*, T*, T*, i64, i64, \
                                      i64, i64, hipStream_t);

EXS_INSTANTIATE(float, OpSum)
EXS_INSTANTIATE(double, OpSum)
EXS_INSTANTIATE(int, OpSum)
EXS_INSTANTIATE(long long, OpSum)
EXS_INSTANTIATE(float, OpMax)
EXS_INSTANTIATE(double, OpMax)
EXS_INSTANTIATE(int, OpMax)
EXS_INSTANTIATE(long long, OpMax)

}  // namespace exs
