// exsum_device.hpp -- device building blocks for included and excluded sums
// on gfx950 (CDNA4, wave64).
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// Every routine here works on a tensor viewed as (outer, n, inner): `n` is the
// length of the axis being processed and `inner` its stride.  Elements past
// the end of an axis behave as the monoid identity (Sec. 1: out-of-range
// coordinates contribute e; the footnote of Sec. 3 allows identity padding
// when n is not a multiple of k).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exsum_internal.hpp"

typedef long long i64;

namespace exs {

// ---------------------------------------------------------------------------
// The monoids: + (integer + wraps, done in unsigned arithmetic) and max.
// Both are commutative, which the dimension-reduction reordering relies on.
// ---------------------------------------------------------------------------
struct OpSum {
    template <typename T> static __device__ __forceinline__ T id() { return T(0); }
    // a - b: + has an inverse (weak excluded sums, total - included)
    static __device__ __forceinline__ float inverse(float a, float b) { return a - b; }
    static __device__ __forceinline__ double inverse(double a, double b) { return a - b; }
    static __device__ __forceinline__ int inverse(int a, int b) {
        return (int)((unsigned)a - (unsigned)b);
    }
    static __device__ __forceinline__ long long inverse(long long a, long long b) {
        return (long long)((unsigned long long)a - (unsigned long long)b);
    }
    static __device__ __forceinline__ float apply(float a, float b) { return a + b; }
    static __device__ __forceinline__ double apply(double a, double b) { return a + b; }
    static __device__ __forceinline__ int apply(int a, int b) {
        return (int)((unsigned)a + (unsigned)b);
    }
    static __device__ __forceinline__ long long apply(long long a, long long b) {
        return (long long)((unsigned long long)a + (unsigned long long)b);
    }
};

struct OpMax {
    template <typename T> static __device__ __forceinline__ T id();
    // max has no inverse; never called (weak excluded sums are + only)
    template <typename T> static __device__ __forceinline__ T inverse(T a, T) { return a; }
    // fp32 max as the IEEE 754-2019 maximum (v_maximum3_f32 on gfx950): the
    // same value as maxnum for the finite inputs the library takes, without
    // the operand quieting that maxnum needs for every value read from memory
    // (which cost registers in the unrolled scans), and, unlike inline
    // assembly, free for the scheduler to move loads across.
    static __device__ __forceinline__ float apply(float a, float b) {
        return __builtin_elementwise_maximum(a, b);
    }
    static __device__ __forceinline__ double apply(double a, double b) { return fmax(a, b); }
    static __device__ __forceinline__ int apply(int a, int b) { return a > b ? a : b; }
    static __device__ __forceinline__ long long apply(long long a, long long b) {
        return a > b ? a : b;
    }
    static __device__ __forceinline__ ValIdx apply(ValIdx a, ValIdx b) {
        return (a.v > b.v || (a.v == b.v && a.i < b.i)) ? a : b;
    }
};
template <> __device__ __forceinline__ float OpMax::id<float>() { return -__builtin_inff(); }
template <> __device__ __forceinline__ ValIdx OpMax::id<ValIdx>() {
    return ValIdx{-__builtin_inff(), 0x7fffffff};
}
template <> __device__ __forceinline__ double OpMax::id<double>() { return -__builtin_inf(); }
template <> __device__ __forceinline__ int OpMax::id<int>() { return (int)0x80000000; }
template <> __device__ __forceinline__ long long OpMax::id<long long>() {
    return (long long)0x8000000000000000ULL;
}

struct OpMin {
    template <typename T> static __device__ __forceinline__ T id();
    // min has no inverse; never called (weak excluded sums are + only)
    template <typename T> static __device__ __forceinline__ T inverse(T a, T) { return a; }
    // fp32 min as the IEEE 754-2019 minimum, for the reasons given for max
    static __device__ __forceinline__ float apply(float a, float b) {
        return __builtin_elementwise_minimum(a, b);
    }
    static __device__ __forceinline__ double apply(double a, double b) { return fmin(a, b); }
    static __device__ __forceinline__ int apply(int a, int b) { return a < b ? a : b; }
    static __device__ __forceinline__ long long apply(long long a, long long b) {
        return a < b ? a : b;
    }
    static __device__ __forceinline__ ValIdx apply(ValIdx a, ValIdx b) {
        return (a.v < b.v || (a.v == b.v && a.i < b.i)) ? a : b;
    }
};
template <> __device__ __forceinline__ float OpMin::id<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ ValIdx OpMin::id<ValIdx>() {
    return ValIdx{__builtin_inff(), 0x7fffffff};
}
template <> __device__ __forceinline__ double OpMin::id<double>() { return __builtin_inf(); }
template <> __device__ __forceinline__ int OpMin::id<int>() { return 0x7fffffff; }
template <> __device__ __forceinline__ long long OpMin::id<long long>() {
    return (long long)0x7fffffffffffffffULL;
}

// An artificially expensive + on fp32 (measurement support, after the
// experiment of Sec. 6, "Excluded Sums With Different Operators", which slows
// its operator down with a recursive Fibonacci computation of tunable size).
// apply returns a + b, as OpSum does, after `g_slow_cost` dependent 32-bit
// integer multiply-add steps whose result is kept live and then dropped, so
// every application costs a known number of extra instructions and results
// do not change.  Every translation unit holds its own copy of the cost
// (internal linkage); set_slow_cost_here writes this unit's copy.
static __constant__ int g_slow_cost;
struct OpSlowSum : OpSum {
    static __device__ __forceinline__ float apply(float a, float b) {
        const float r = a + b;
        unsigned h = __float_as_uint(r);
        const int c = g_slow_cost;
        for (int i = 0; i < c; ++i) h = h * 1664525u + 1013904223u;
        asm volatile("" : : "v"(h));
        return r;
    }
};
static inline hipError_t set_slow_cost_here(int c) {
    return hipMemcpyToSymbol(HIP_SYMBOL(g_slow_cost), &c, sizeof(c));
}

__device__ __forceinline__ i64 gtid() {
    return (i64)blockIdx.x * (i64)blockDim.x + (i64)threadIdx.x;
}

// ---------------------------------------------------------------------------
// Raw buffer access: a descriptor (uniform 64-bit base and byte range, in
// SGPRs) plus a per-thread 32-bit byte offset.  Accesses past the range read
// 0 and drop stores.  Word 3 = 0x00020000 is the gfx9-family raw format.
// 4- and 8-byte element types.
// ---------------------------------------------------------------------------
typedef unsigned exs_u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned voff) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte elements");
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0));
}
// The same with a uniform part of the offset in a scalar register (soff).
template <typename T>
__device__ __forceinline__ T bload_s(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte elements");
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned voff, T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte elements");
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(exs_u32x2, v), r, voff, 0, 0);
}
// The same with the non-temporal hint (cache-policy bit NT): for output
// planes that nothing reads again, so that they do not evict from L2 the
// input rows that neighbouring tiles still read as halo.
template <typename T>
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t r, unsigned voff, T v) {
    static_assert(sizeof(T) == 4, "4-byte elements");
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, 0, 2);
}
// Output stores of the streaming kernels, with the hint or without.  The
// hint pays where every output row is a whole number of 64-byte chunks.
// Rows of other lengths leave chunks at tile edges that two workgroups fill
// in parts; stored without the hint, the parts meet in L2 and reach memory
// as one write instead of two partial ones.
template <typename T, bool NT>
__device__ __forceinline__ void bstore_h(__amdgpu_buffer_rsrc_t r, unsigned voff, T v) {
    if constexpr (NT) bstore_nt<T>(r, voff, v);
    else bstore<T>(r, voff, v);
}
inline bool store_hint_ok(long long row_bytes) { return row_bytes % 64 == 0; }
// A byte offset no descriptor of a tensor below 2^31 bytes covers: a store
// there is dropped.
constexpr unsigned NOWHERE = 0x80000000u;
// Tensors below 2^31 bytes take the "narrow" generic tasks: 32-bit byte
// offsets into descriptors over the whole tensor (fewer registers, no
// branches around accesses) instead of 64-bit element addresses; blocks of
// 64 keep the 64-bit form, which needs fewer registers there.
inline bool narrow_ok(long long elems, int es, int kb) {
    return kb <= 32 && elems * (long long)es < (1ll << 31);
}

// ---------------------------------------------------------------------------
// BDBS along one axis for one row (Sec. 3, "Included Sums in 1D"; App. B,
// Fig. "Pseudocode for the 1D included sum", Lemma "Correctness in 1D").
//
// Blocks of k consecutive elements (aligned to multiples of k).  For each
// block b the range suffix rsuf_b[r] = op of the block from r to its end and
// the range prefix rpre_{b+1}[r-1] = op of the next block from its start to
// r-1 give the window at x = b*k + r:
//     out[x] = rsuf_b[0]                      if r == 0 (the whole block)
//     out[x] = rsuf_b[r] op rpre_{b+1}[r-1]   otherwise
// (0-based form of the combine; the proof of the lemma uses x mod k = 1 in
// 1-based terms).  Positions past n are the identity.  The row is streamed
// block by block with the suffixes of the current block in registers, so each
// input is read once and each output written once.  KB >= k is a
// compile-time bound on the block length so the arrays live in VGPRs.
// Blocks [b0, b1) of the row are produced.
// ---------------------------------------------------------------------------
// Scans of the 64 lanes of a wavefront: inclusive prefix (toward higher
// lanes) and inclusive suffix (toward lower lanes) of one value per lane.
// Lane shuffles of 4- and 8-byte element types (struct elements included).
template <typename T>
__device__ __forceinline__ T wshfl(T v, int src) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __shfl(__builtin_bit_cast(int, v), src, 64));
    else
        return __builtin_bit_cast(T, __shfl(__builtin_bit_cast(long long, v), src, 64));
}

template <typename T, class Op>
__device__ __forceinline__ T wave_prefix(T v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T o = __shfl_up(v, off, 64);
        if (lane >= off) v = Op::apply(o, v);
    }
    return v;
}
template <typename T, class Op>
__device__ __forceinline__ T wave_suffix(T v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T o = __shfl_down(v, off, 64);
        if (lane + off < 64) v = Op::apply(v, o);
    }
    return v;
}

template <typename T, class Op, int KB>
__device__ __forceinline__ void bdbs_row(const T* __restrict__ src, T* __restrict__ dst,
                                         i64 n, i64 stride, int k, i64 b0, i64 b1) {
    const T e = Op::template id<T>();
    T cur[KB], nxt[KB];
#pragma unroll
    for (int r = 0; r < KB; ++r) {
        const i64 x = b0 * k + r;
        cur[r] = (r < k && x < n) ? src[x * stride] : e;
    }
    {
        T s = e;
#pragma unroll
        for (int r = KB - 1; r >= 0; --r) {
            if (r < k) { s = Op::apply(cur[r], s); cur[r] = s; }
        }
    }
    for (i64 b = b0; b < b1; ++b) {
        const i64 base = (b + 1) * k;
#pragma unroll
        for (int r = 0; r < KB; ++r) {
            const i64 x = base + r;
            nxt[r] = (r < k && x < n) ? src[x * stride] : e;
        }
        T p = e;
#pragma unroll
        for (int r = 0; r < KB; ++r) {
            if (r < k) {
                const i64 x = b * k + r;
                T v = cur[r];
                if (r > 0) { p = Op::apply(p, nxt[r - 1]); v = Op::apply(v, p); }
                if (x < n) dst[x * stride] = v;
            }
        }
        T s = e;
#pragma unroll
        for (int r = KB - 1; r >= 0; --r) {
            if (r < k) { s = Op::apply(nxt[r], s); cur[r] = s; }
        }
    }
}

// The same for a tensor below 2^31 bytes (narrow_ok): src and dst are
// descriptors over the whole input and output, off0 the byte offset of the
// row's element 0 and sb the byte stride along the axis.  Every element of a
// block is loaded (elements past the row end or the block read whatever their
// offset points at inside the tensor, or 0 past its end) and replaced by the
// identity; their stores go to NOWHERE.
template <typename T, class Op, int KB>
__device__ __forceinline__ void bdbs_row_narrow(__amdgpu_buffer_rsrc_t src,
                                                __amdgpu_buffer_rsrc_t dst, unsigned off0,
                                                int n, unsigned sb, int k, int b0, int b1) {
    const T e = Op::template id<T>();
    T cur[KB], nxt[KB];
    // byte offsets: the block's base (per thread) plus r * sb (uniform)
    {
        const unsigned ob = off0 + (unsigned)(b0 * k) * sb;
        const int lim = min(k, n - b0 * k);  // elements of the block inside the row
#pragma unroll
        for (int r = 0; r < KB; ++r) {
            const T v = bload<T>(src, ob + (unsigned)r * sb);
            cur[r] = r < lim ? v : e;
        }
    }
    {
        T s = e;
#pragma unroll
        for (int r = KB - 1; r >= 0; --r) {
            s = Op::apply(cur[r], s);
            cur[r] = s;
        }
    }
    for (int b = b0; b < b1; ++b) {
        const int base = (b + 1) * k;
        const unsigned onx = off0 + (unsigned)base * sb, ocur = off0 + (unsigned)(b * k) * sb;
        const int limn = min(k, n - base), limc = min(k, n - b * k);
#pragma unroll
        for (int r = 0; r < KB; ++r) {
            const T v = bload<T>(src, onx + (unsigned)r * sb);
            nxt[r] = r < limn ? v : e;
        }
        T p = e;
#pragma unroll
        for (int r = 0; r < KB; ++r) {
            T v = cur[r];
            if (r > 0) {
                p = Op::apply(p, nxt[r - 1]);
                v = Op::apply(v, p);
            }
            bstore<T>(dst, r < limc ? ocur + (unsigned)r * sb : NOWHERE, v);
        }
        T s = e;
#pragma unroll
        for (int r = KB - 1; r >= 0; --r) {
            s = Op::apply(nxt[r], s);
            cur[r] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Streaming along axis 0 for one point m of the remaining axes (the "first
// dimension-reduction step" of the box-complement algorithm, Sec. 5, with the
// prefix and suffix steps merged; see the design notes):
//
//   Exc[x0] = (op over t < x0 of W[t]) op (op over t >= x0+k0 of W[t]) op Trest
//   Inc[x0] = op over t in [x0, x0+k0) of W[t]            (BDBS along axis 0)
//
// W is the input already box-summed over the other axes.  The axis is cut in
// blocks of k0; PX[q] / SX[q] are the op of the block totals of W strictly
// before / after block q (computed from block aggregates of the input, then
// box-summed over the other axes).  For x0 = q*k0 + r:
//   prefix part = PX[q] op rpre_q[r-1]           (running, in registers)
//   suffix part = rsuf_{q+1}[r] op SX[q+1]       (needs block q+1: one-block lag)
// The caller supplies the block values through `nxt` (one block at a time).
// ---------------------------------------------------------------------------
template <typename T, class Op, int K0B>
struct Axis0State {
    T pex[K0B];   // prefix part for each row of the current block (Exc)
    T rs[K0B];    // range suffix of the current block (Inc)
    T P;          // op of everything before the next block (incl. Trest)

    // Absorb a block whose values past k0 are the identity (no masks needed:
    // an identity leaves the running prefix and the suffix unchanged).
    __device__ __forceinline__ void absorb_all(const T (&v)[K0B]) {
        const T e = Op::template id<T>();
#pragma unroll
        for (int r = 0; r < K0B; ++r) { pex[r] = P; P = Op::apply(P, v[r]); }
        T s = e;
#pragma unroll
        for (int r = K0B - 1; r >= 0; --r) { s = Op::apply(v[r], s); rs[r] = s; }
    }

    // Absorb block values v[0..k0) as the new current block.
    __device__ __forceinline__ void absorb(const T (&v)[K0B], int k0, bool do_ex, bool do_inc) {
        const T e = Op::template id<T>();
        if (do_ex) {
#pragma unroll
            for (int r = 0; r < K0B; ++r) {
                if (r < k0) { pex[r] = P; P = Op::apply(P, v[r]); }
            }
        }
        if (do_inc) {
            T s = e;
#pragma unroll
            for (int r = K0B - 1; r >= 0; --r) {
                if (r < k0) { s = Op::apply(v[r], s); rs[r] = s; }
            }
        }
    }
};

}  // namespace exs
