// exsum_tasks.hpp -- per-task device functions of the generic path.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// Each function computes one thread-sized task of one step, identified by a
// flat task index.  The plain kernels (exsum_kernels.hip) map one thread to
// one task; the work-list kernels of the batched form (exsum_worklist.hip)
// walk the tasks of many steps of many tensors with a persistent grid.  Both
// run exactly this code, so a batched job computes what its plain call does.
#pragma once
#include "exsum_device.hpp"

namespace exs {

// Step kinds
enum StepKind : int {
    SK_BDBS = 0,   // BDBS along one axis, block suffixes in registers (k <= 64)
    SK_BDBS2 = 1,  // BDBS along one axis, two sweeps (any k)
    SK_AGG = 2,    // block aggregates along axis 0
    SK_SCAN = 3,   // exclusive block prefix/suffix and the reduction of axis 0
    SK_AX0 = 4,    // axis-0 stream: excluded and/or included sums (k0 <= 64)
    SK_EX2 = 5,    // axis-0 excluded part, two sweeps (any k0)
    SK_BDBSR = 6,  // BDBS along the contiguous axis through LDS (k <= 64; wavefront tasks)
    SK_SEGTOT = 7, // block scans over many blocks for few points: segment totals
    SK_SEGEXP = 8, // ... and the expansion of the scanned segment totals
    SK_BDBSW = 9,  // SK_BDBS for tensors of 2^31 bytes or more (64-bit addressing)
    SK_AX0W = 10,  // SK_AX0 for tensors of 2^31 bytes or more (64-bit addressing)
    SK_BDBSV = 11, // BDBS along the contiguous axis, one wavefront per task (k <= 64,
                   // tensors below 2^31 bytes); its task count is in threads
    SK_BDBSC = 12, // BDBS along a strided axis, boxes of 17 to 64 split over 2 or 4
                   // lanes per column (tensors below 2^31 bytes); count in threads
    SK_AX0C = 13,  // SK_AX0 the same way (boxes of 17 to 64 along axis 0)
    SK_NKINDS = 14
};

// One step of the generic path.  Pointers are device pointers; the meaning
// of each field depends on the kind (see make_* in exsum_plan.hpp).
struct Step {
    int kind;
    int k;             // box length along the processed axis
    const void* in0;   // bdbs/agg/ax0/ex2: input; scan: Gw
    const void* in1;   // scan: Ga;  ax0: PX
    const void* in2;   // ax0: SX
    const void* in3;   // ax0/ex2: lower-dimensional excluded sums (or null)
    void* out0;        // bdbs: out; agg: Ga; scan: PX; ax0/ex2: exc (or null)
    void* out1;        // scan: SX; ax0: inc (or null)
    void* out2;        // scan: R (or null)
    i64 O, n, I;       // bdbs view (outer, axis length, inner); agg/ax0: n = n0, I = M
    i64 Q;             // blocks along axis 0
    i64 cb, nchunks;   // bdbs: blocks per chunk, chunks;  ax0: blocks per run, runs
    i64 ntasks;        // tasks of this step
    i64 task_begin;    // first flat task index of this step in its work list
};

// BDBS along an axis of a (O, n, I) tensor: task = (o, chunk, i), i fastest
// (coalesced whenever I >= 64); each task streams `cb` blocks of its row.
// NARROW: the tensor is below 2^31 bytes (32-bit byte offsets, bdbs_row_narrow).
template <typename T, class Op, int KB, bool NARROW>
__device__ __forceinline__ void task_bdbs(const T* __restrict__ in, T* __restrict__ out, i64 O,
                                          i64 n, i64 I, int k, i64 cb, i64 nchunks, i64 idx) {
    const i64 i = idx % I;
    const i64 rest = idx / I;
    const i64 c = rest % nchunks;
    const i64 o = rest / nchunks;
    const i64 nb = (n + k - 1) / k;
    const i64 b0 = c * cb;
    if (b0 >= nb || o >= O) return;
    const i64 b1 = b0 + cb < nb ? b0 + cb : nb;
    const i64 off = o * n * I + i;
    if constexpr (NARROW) {
        const unsigned bytes = (unsigned)(O * n * I * (i64)sizeof(T));
        bdbs_row_narrow<T, Op, KB>(buf(in, bytes), buf(out, bytes),
                                   (unsigned)(off * (i64)sizeof(T)), (int)n,
                                   (unsigned)(I * (i64)sizeof(T)), k, (int)b0, (int)b1);
    } else {
        bdbs_row<T, Op, KB>(in + off, out + off, n, I, k, b0, b1);
    }
}

// Two-sweep BDBS for any k: the backward sweep writes the range suffixes,
// the forward sweep adds the range prefix of the next block (out != in).
template <typename T, class Op>
__device__ __forceinline__ void task_bdbs2(const T* __restrict__ in, T* __restrict__ out, i64 n,
                                           i64 I, i64 k, i64 idx) {
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

// Ga[q, m] = op over t in block q of X[t, m]; X viewed as (n0, M); task = (q, m).
template <typename T, class Op>
__device__ __forceinline__ void task_agg(const T* __restrict__ X, T* __restrict__ Ga, i64 n0,
                                         i64 M, i64 k0, i64 idx) {
    const i64 m = idx % M, q = idx / M;
    const i64 t0 = q * k0;
    const i64 t1 = t0 + k0 < n0 ? t0 + k0 : n0;
    T s = Op::template id<T>();
#pragma unroll 8
    for (i64 t = t0; t < t1; ++t) s = Op::apply(s, X[t * M + m]);
    Ga[idx] = s;
}

// Per point m (= task): PX[q] = op of Gw[q'] for q' < q, SX[q] = op of Gw[q']
// for q' > q, R[m] = op over all blocks of Ga (the reduction of axis 0).
// PX is stored for the blocks q with q % pxe == 0 only (where the runs of the
// axis-0 stream that reads it start).
template <typename T, class Op>
__device__ __forceinline__ void task_scan(const T* __restrict__ Gw, const T* __restrict__ Ga,
                                          T* __restrict__ PX, T* __restrict__ SX,
                                          T* __restrict__ R, i64 Q, i64 M, i64 m, i64 pxe = 1) {
    const T e = Op::template id<T>();
    T p = e, r = e;
    i64 c = 0;
#pragma unroll 8
    for (i64 q = 0; q < Q; ++q) {
        if (c == 0) PX[q * M + m] = p;
        c = c + 1 == pxe ? 0 : c + 1;
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

// Block scans over Q blocks when there are few points m (the direct scan is
// one serial walk over all Q blocks per point): segments of L blocks.
// Segment totals, task (s, m): Tw[s, m] = op of Gw[q, m], Ta[s, m] = op of
// Ga[q, m] over the segment's blocks q.
template <typename T, class Op>
__device__ __forceinline__ void task_segtot(const T* __restrict__ Gw, const T* __restrict__ Ga,
                                            T* __restrict__ Tw, T* __restrict__ Ta, i64 Q, i64 M,
                                            i64 L, i64 idx) {
    const i64 m = idx % M, sg = idx / M;
    const i64 q0 = sg * L, q1 = q0 + L < Q ? q0 + L : Q;
    const T e = Op::template id<T>();
    T w = e, g = e;
#pragma unroll 8
    for (i64 q = q0; q < q1; ++q) {
        w = Op::apply(w, Gw[q * M + m]);
        g = Op::apply(g, Ga[q * M + m]);
    }
    Tw[idx] = w;
    Ta[idx] = g;
}

// Expansion, task (s, m): from the exclusive prefix SPX[s, m] and suffix
// SSX[s, m] of the segment totals, PX[q, m] and SX[q, m] of the segment's blocks.
template <typename T, class Op>
__device__ __forceinline__ void task_segexp(const T* __restrict__ Gw, const T* __restrict__ SPX,
                                            const T* __restrict__ SSX, T* __restrict__ PX,
                                            T* __restrict__ SX, i64 Q, i64 M, i64 L, i64 idx,
                                            i64 pxe = 1) {
    const i64 m = idx % M, sg = idx / M;
    const i64 q0 = sg * L, q1 = q0 + L < Q ? q0 + L : Q;
    T p = SPX[idx];
    // PX only for blocks q % pxe == 0 (as in task_scan)
    i64 c = q0 % pxe;
#pragma unroll 8
    for (i64 q = q0; q < q1; ++q) {
        if (c == 0) PX[q * M + m] = p;
        c = c + 1 == pxe ? 0 : c + 1;
        p = Op::apply(p, Gw[q * M + m]);
    }
    T s = SSX[idx];
#pragma unroll 8
    for (i64 q = q1 - 1; q >= q0; --q) {
        SX[q * M + m] = s;
        s = Op::apply(Gw[q * M + m], s);
    }
}

// Axis-0 stream (generic path): task = (run, m), m fastest; the task owns
// point m and blocks [qa, qb) of axis 0, reading one block ahead.
// task_axis0 for tensors below 2^31 bytes: descriptors over W (n0 x M), PX
// and SX (Q x M), Trest (M) and the outputs, 32-bit byte offsets; block rows
// past k0 or past the tensor are loaded from wherever their offset points
// and replaced by the identity, their stores go to NOWHERE.
template <typename T, class Op, int K0B>
__device__ __forceinline__ void task_axis0_narrow(const T* __restrict__ W,
                                                  const T* __restrict__ PX,
                                                  const T* __restrict__ SX,
                                                  const T* __restrict__ Trest,
                                                  T* __restrict__ exc, T* __restrict__ inc,
                                                  i64 n0_, i64 M_, int k0, i64 Q_,
                                                  i64 segblocks, i64 idx) {
    const int M = (int)M_, n0 = (int)n0_, Q = (int)Q_;
    const int m = (int)(idx % M_), s = (int)(idx / M_);
    const int qa = s * (int)segblocks;
    if (qa >= Q) return;
    const int qb = qa + (int)segblocks < Q ? qa + (int)segblocks : Q;
    const bool do_ex = exc != nullptr, do_inc = inc != nullptr;
    const T e = Op::template id<T>();
    constexpr unsigned es = sizeof(T);
    const unsigned nbytes = (unsigned)n0 * (unsigned)M * es;
    const unsigned qbytes = (unsigned)Q * (unsigned)M * es;
    const __amdgpu_buffer_rsrc_t rw = buf(W, nbytes);
    const __amdgpu_buffer_rsrc_t rex = buf(exc, do_ex ? nbytes : 0u);
    const __amdgpu_buffer_rsrc_t rin = buf(inc, do_inc ? nbytes : 0u);
    const unsigned rowb = (unsigned)M * es;   // bytes between rows along axis 0
    const unsigned mo = (unsigned)m * es;

    // w: the raw values of the block being held (its range prefixes and
    // suffixes are formed when it is emitted); Pb: op of everything before
    // it, with the lower-dimensional term
    // byte offsets: the thread's base at the block start (per thread) plus
    // r * rowb (uniform, scalar registers)
    T w[K0B];
    {
        const unsigned ob = mo + (unsigned)(qa * k0) * rowb;
        const int lim = min(k0, n0 - qa * k0);  // rows of the block inside the tensor
#pragma unroll
        for (int r = 0; r < K0B; ++r) {
            const T t = bload<T>(rw, ob + (unsigned)r * rowb);
            w[r] = r < lim ? t : e;
        }
    }
    T Pb = e;
    if (do_ex) {
        Pb = bload<T>(buf(PX, qbytes), mo + (unsigned)qa * rowb);
        if (Trest) Pb = Op::apply(Pb, bload<T>(buf(Trest, rowb), mo));
    }
    const __amdgpu_buffer_rsrc_t rsx = buf(SX, do_ex ? qbytes : 0u);

    for (int q = qa; q < qb; ++q) {
        const int nbase = (q + 1) * k0;
        const unsigned onx = mo + (unsigned)nbase * rowb;        // block q + 1
        const unsigned ocur = mo + (unsigned)(q * k0) * rowb;    // block q
        const int limn = min(k0, n0 - nbase), limc = min(k0, n0 - q * k0);
        T v[K0B];
#pragma unroll
        for (int r = 0; r < K0B; ++r) {
            const T t = bload<T>(rw, onx + (unsigned)r * rowb);
            v[r] = r < limn ? t : e;
        }
        T tmp[K0B];
        if (do_ex) {
            // the prefix before each row of block q, then the suffix from the
            // same row of block q + 1 on (identities past k0 change nothing)
#pragma unroll
            for (int r = 0; r < K0B; ++r) { tmp[r] = Pb; Pb = Op::apply(Pb, w[r]); }
            const T sxv = bload<T>(rsx, mo + (unsigned)(q + 1) * rowb);
            T S = (q + 1 < Q) ? sxv : e;
#pragma unroll
            for (int r = K0B - 1; r >= 0; --r) {
                S = Op::apply(v[r], S);
                bstore<T>(rex, r < limc ? ocur + (unsigned)r * rowb : NOWHERE,
                          Op::apply(tmp[r], S));
            }
        }
        if (do_inc) {
            // BDBS along axis 0: range suffix in block q, range prefix of
            // block q + 1 up to the row before
            T sf = e;
#pragma unroll
            for (int r = K0B - 1; r >= 0; --r) { sf = Op::apply(w[r], sf); tmp[r] = sf; }
            T p = e;
#pragma unroll
            for (int r = 0; r < K0B; ++r) {
                T val = tmp[r];
                if (r > 0) { p = Op::apply(p, v[r - 1]); val = Op::apply(val, p); }
                bstore<T>(rin, r < limc ? ocur + (unsigned)r * rowb : NOWHERE, val);
            }
        }
#pragma unroll
        for (int r = 0; r < K0B; ++r) w[r] = v[r];
    }
}

template <typename T, class Op, int K0B, bool NARROW>
__device__ __forceinline__ void task_axis0(const T* __restrict__ W, const T* __restrict__ PX,
                                           const T* __restrict__ SX, const T* __restrict__ Trest,
                                           T* __restrict__ exc, T* __restrict__ inc, i64 n0,
                                           i64 M, int k0, i64 Q, i64 segblocks, i64 idx) {
    if constexpr (NARROW) {
        task_axis0_narrow<T, Op, K0B>(W, PX, SX, Trest, exc, inc, n0, M, k0, Q, segblocks, idx);
        return;
    }
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

// Axis-0 excluded part for any k0, one task per point, two sweeps: the
// backward sweep stores the suffix from x0 + k0, the forward sweep prepends
// the prefix before x0 and the lower-dimensional term.
template <typename T, class Op>
__device__ __forceinline__ void task_ex2(const T* __restrict__ W, const T* __restrict__ Trest,
                                         T* __restrict__ exc, i64 n0, i64 M, i64 k0, i64 m) {
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
// Split-block tasks for boxes longer than 16 along a strided axis and along
// axis 0.  A thread that holds a whole block (and the next) needs two
// registers per slot of the bucket, which at 32 or 64 slots leaves one to
// four wavefronts per SIMD and starves the memory pipeline.  Here G lanes
// share one column, each holding CS consecutive slots of a block: the range
// prefixes and suffixes of the block (Sec. 3) are each lane's own scans over
// its slots combined with the op of the other lanes' segment totals before or
// after it.  A wavefront covers C = 64 / G columns: lanes g * C .. g * C + C - 1
// hold segment g of the C columns, so one load reads C consecutive elements
// in each of G rows.  Slots past the box length or the tensor end are the
// identity; their loads read nothing and their stores land nowhere.  32-bit
// byte offsets: tensors below 2^31 bytes.  From global memory G = 2 where the
// registers allow (rows of 32 elements per load: 128 bytes of 4-byte
// elements), else 4; CS = KB / G.
// ---------------------------------------------------------------------------
constexpr int COOP_CS = 16;  // slots per lane of the LDS-staged row tasks

// lanes per column of the global-memory split-block tasks: 2, or 4 where 32
// slots per lane would spill past half the register file (the axis-0 stream,
// which holds two blocks and a scan, and 8-byte elements) at KB = 64
__host__ __device__ constexpr int coop_g(int kb, int es, bool axis0) {
    return (kb == 64 && (axis0 || es == 8)) ? 4 : 2;
}
// ... for the axis-0 stream with one output (OUT 1: excluded sums, 2:
// included sums), which carries one block array less than with both (OUT 3)
__host__ __device__ constexpr int coop_g_ax0(int kb, int es, int out) {
    return out == 3 ? coop_g(kb, es, true) : coop_g(kb, es, false);
}

// ADJ: the G lanes of a column are adjacent (lane = c * G + g) -- for
// operands staged in LDS, where no load coalescing is at stake.
template <typename T, class Op, int G, bool ADJ = false>
struct CoopLanes {
    static constexpr int C = 64 / G;
    int c, g;  // column within the wavefront's group, segment of the block
    __device__ __forceinline__ explicit CoopLanes(int lane)
        : c(ADJ ? lane / G : lane % C), g(ADJ ? lane % G : lane / C) {}
    // op of the segment totals of this lane's column before and after its
    // own segment (every lane of the wavefront takes part)
    __device__ __forceinline__ void scan(T tot, T& before, T& after) const {
        const T e = Op::template id<T>();
        before = e;
        after = e;
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const T t = G == 1 ? tot : wshfl(tot, ADJ ? c * G + j : c + j * C);
            if (j < g) before = Op::apply(before, t);
            if (j > g) after = Op::apply(after, t);
        }
    }
};

// Load this lane's slots of one block: `lim` = slots of the segment inside
// the box and the tensor (<= 0: none), `ob` = byte offset of its first slot,
// the slot's row in the scalar offset.  A slot past `lim` still issues its
// load -- of an element of this tensor, or past the descriptor's range, which
// reads 0 -- and takes the identity instead of what it read.
template <typename T, class Op, int CS>
__device__ __forceinline__ void coop_load(__amdgpu_buffer_rsrc_t r, unsigned ob, unsigned rowb,
                                          int lim, T (&v)[CS]) {
    const T e = Op::template id<T>();
#pragma unroll
    for (int s = 0; s < CS; ++s) {
        const T t = bload_s<T>(r, ob, (unsigned)s * rowb);
        v[s] = s < lim ? t : e;
    }
}

// BDBS along the contiguous axis (rows of n elements, I == 1).  Lanes that
// each walk their own row would touch 64 rows per load; instead one wavefront
// (a workgroup of 64 threads) owns 64 rows and a run of cb blocks: the tile,
// with the k - 1 columns of the next block, is staged in LDS by coalesced row
// loads, each lane box-sums its row from LDS (block suffixes in registers, as
// in bdbs_row), writes the results in place, and the tile leaves by coalesced
// row stores.  For boxes over 16 a task owns 64 / G rows and G lanes share a
// row (COOP_CS slots of each block per lane, as in the split-block tasks).
// LDS: rows x rows_pitch(cb, k) elements (odd pitch: few bank conflicts
// between lanes reading their rows).
// Rows per task: 64, or 64 / G for boxes of 17 to 64 (G lanes per row, one
// pass over the tile; the smaller tile leaves room in LDS for more tasks).
__host__ __device__ constexpr int rows_per_task_kb(int kb) {
    return kb > COOP_CS ? 64 / (kb / COOP_CS) : 64;
}
inline int rows_per_task(i64 k) { return rows_per_task_kb(bucket_for(k)); }
__host__ __device__ inline int rows_pitch(i64 cb, i64 k) { return (int)((cb * k + k - 1) | 1); }

// Row tasks pay off once they fill the GPU (four wavefronts per CU).
constexpr i64 ROWS_MIN_TASKS = 1024;

inline i64 rows_tasks(i64 O, i64 n, i64 k, i64 cb) {
    const i64 nb = (n + k - 1) / k;
    const i64 rpt = rows_per_task(k);
    return ((O + rpt - 1) / rpt) * ((nb + cb - 1) / cb);
}

// Blocks per row task: at most 64 columns, fewer while there are fewer than
// min_tasks tasks.
inline i64 rows_blocks(i64 O, i64 n, i64 k, i64 min_tasks) {
    const i64 nb = (n + k - 1) / k;
    i64 cb = 64 / k > 1 ? 64 / k : 1;
    if (cb > nb) cb = nb;
    const i64 groups = (O + rows_per_task(k) - 1) / rows_per_task(k);
    while (cb > 1 && groups * ((nb + cb - 1) / cb) < min_tasks) cb = (cb + 1) / 2;
    return cb;
}

template <typename T, class Op, int KB>
__device__ __forceinline__ void task_bdbs_rows(const T* __restrict__ in, T* __restrict__ out,
                                               i64 O, i64 n, int k, i64 cb, i64 nchunks,
                                               i64 task, T* __restrict__ lds) {
    const int lane = threadIdx.x;
    const T e = Op::template id<T>();
    const i64 g = task / nchunks, c = task % nchunks;
    const i64 nb = (n + k - 1) / k;
    const i64 b0 = c * cb;
    const i64 b1 = b0 + cb < nb ? b0 + cb : nb;
    const i64 col0 = b0 * k;
    const int LW = rows_pitch(cb, k);
    const i64 rin = (b1 - b0) * k + k - 1, rout = (b1 - b0) * k;
    const int win = (int)(rin < n - col0 ? rin : n - col0);
    const int wout = (int)(rout < n - col0 ? rout : n - col0);
    constexpr int RPT = rows_per_task_kb(KB);
    const i64 row0 = g * RPT;
    // Whole rows (one run of blocks per row): the task's rows are one
    // contiguous span of the tensor, staged and stored flat (every lane busy
    // however short the rows); lane f of the span goes to (f / n, f % n),
    // tracked incrementally.
    const bool flat = nchunks == 1;
    const int nn = (int)n;
    const int vrows = row0 + RPT <= O ? RPT : (int)(O - row0);
    if (flat) {
        const T* __restrict__ src = in + row0 * n;
        const int span = vrows * nn, dr = 64 / nn, dc = 64 % nn;
        int r = lane / nn, cc = lane % nn;
        constexpr int U = 8;
        for (int f0 = 0; f0 < span; f0 += 64 * U) {
            T v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int f = f0 + 64 * u + lane;
                v[u] = f < span ? src[f] : e;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (f0 + 64 * u + lane < span) lds[r * LW + cc] = v[u];
                r += dr;
                cc += dc;
                if (cc >= nn) { cc -= nn; ++r; }
            }
        }
        // identity in the pitch past the row end and in rows past the tensor
        for (int rr = 0; rr < RPT; ++rr) {
            const int c0 = rr < vrows ? nn : 0;
            for (int c = c0 + lane; c < LW; c += 64) lds[rr * LW + c] = e;
        }
    }
    // otherwise stage the tile (identity past the row end and in the unused
    // pitch); LW <= 127, so two 64-column passes cover a row.  Loads are
    // issued in batches of RB rows before any of them is written to LDS.
    constexpr int RB = RPT < 32 ? RPT : 32;
    if (!flat) {
#pragma unroll
        for (int r0 = 0; r0 < RPT; r0 += RB) {
            T v[RB][2];
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
                const i64 row = row0 + r0 + rr;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int cc = lane + 64 * h;
                    v[rr][h] = (row < O && cc < win) ? in[row * n + col0 + cc] : e;
                }
            }
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int cc = lane + 64 * h;
                    if (cc < LW) lds[(r0 + rr) * LW + cc] = v[rr][h];
                }
            }
        }
    }
    __syncthreads();
    if constexpr (KB > COOP_CS) {
        // boxes of 17 to 64: G adjacent lanes per row (the task's 64 / G
        // rows), COOP_CS slots of each block per lane
        constexpr int G = KB / COOP_CS, CS = COOP_CS;
        static_assert(RPT * G == 64, "one pass over the tile");
        const CoopLanes<T, Op, G, true> ln(lane);
        const int s0 = ln.g * CS;
        {
            T* my = lds + ln.c * LW;
            T rs[CS], v[CS];
#pragma unroll
            for (int s = 0; s < CS; ++s) v[s] = s0 + s < k ? my[s0 + s] : e;
            {
                T tot = e;
#pragma unroll
                for (int s = 0; s < CS; ++s) tot = Op::apply(tot, v[s]);
                T before, after;
                ln.scan(tot, before, after);
                T sf = after;
#pragma unroll
                for (int s = CS - 1; s >= 0; --s) {
                    sf = Op::apply(v[s], sf);
                    rs[s] = sf;
                }
            }
            for (i64 b = b0; b < b1; ++b) {
                const int base = (int)(b - b0) * k;
#pragma unroll
                for (int s = 0; s < CS; ++s) {
                    const int x = base + k + s0 + s;
                    v[s] = (s0 + s < k && x < LW) ? my[x] : e;
                }
                T tot = e;
#pragma unroll
                for (int s = 0; s < CS; ++s) tot = Op::apply(tot, v[s]);
                T before, after;
                ln.scan(tot, before, after);
                T p = before;
#pragma unroll
                for (int s = 0; s < CS; ++s) {
                    if (s0 + s < k) my[base + s0 + s] = Op::apply(rs[s], p);
                    p = Op::apply(p, v[s]);
                }
                T sf = after;
#pragma unroll
                for (int s = CS - 1; s >= 0; --s) {
                    sf = Op::apply(v[s], sf);
                    rs[s] = sf;
                }
            }
        }
    } else {
        T* my = lds + lane * LW;
        T cur[KB], nxt[KB];
#pragma unroll
        for (int r = 0; r < KB; ++r) cur[r] = r < k ? my[r] : e;
        {
            T s = e;
#pragma unroll
            for (int r = KB - 1; r >= 0; --r) {
                if (r < k) { s = Op::apply(cur[r], s); cur[r] = s; }
            }
        }
        for (i64 b = b0; b < b1; ++b) {
            const int base = (int)(b - b0) * k;
#pragma unroll
            for (int r = 0; r < KB; ++r) nxt[r] = (r < k && base + k + r < LW) ? my[base + k + r] : e;
            T p = e;
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                if (r < k) {
                    T v = cur[r];
                    if (r > 0) { p = Op::apply(p, nxt[r - 1]); v = Op::apply(v, p); }
                    my[base + r] = v;
                }
            }
            T s = e;
#pragma unroll
            for (int r = KB - 1; r >= 0; --r) {
                if (r < k) { s = Op::apply(nxt[r], s); cur[r] = s; }
            }
        }
    }
    __syncthreads();
    if (flat) {
        T* __restrict__ dst = out + row0 * n;
        const int span = vrows * nn, dr = 64 / nn, dc = 64 % nn;
        int r = lane / nn, cc = lane % nn;
        for (int f = lane; f < span; f += 64) {
            dst[f] = lds[r * LW + cc];
            r += dr;
            cc += dc;
            if (cc >= nn) { cc -= nn; ++r; }
        }
    } else {
#pragma unroll
        for (int r0 = 0; r0 < RPT; r0 += RB) {
            T v[RB][2];
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int cc = lane + 64 * h;
                    v[rr][h] = cc < LW ? lds[(r0 + rr) * LW + cc] : e;
                }
            }
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
                const i64 row = row0 + r0 + rr;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int cc = lane + 64 * h;
                    if (row < O && cc < wout) out[row * n + col0 + cc] = v[rr][h];
                }
            }
        }
    }
    __syncthreads();  // the tile is reused by the next task of this workgroup
}

// BDBS along the contiguous axis by one wavefront per task, without LDS: a
// task is `rpt` consecutive rows (of n elements, k <= 64), processed RB rows
// at a time in windows of 64 columns.  Lane l holds element c0 + l of the
// window and element c0 + 64 + l of the next one (loaded once: it becomes the
// next window).  Range prefixes and suffixes within k-aligned blocks are
// segmented scans across the lanes (Sec. 3: the combine needs, at x, the
// range suffix of x's block from x and the range prefix of the next block up
// to x + k - 1, which lies within the two windows when k <= 64); the block
// that straddles the two windows gets the missing part of its suffix, and its
// prefix in the second window the part in the first.  Positions past n hold
// the identity.  Loads and stores are whole-row, coalesced.
constexpr int WAVE_RB = 8;

// Rows per wavefront task: enough tasks to fill the GPU (about 4096), a
// multiple of WAVE_RB, at most 64 rows.
inline i64 wave_rows_per_task(i64 O) {
    i64 r = (O + 4095) / 4096;
    r = (r + WAVE_RB - 1) / WAVE_RB * WAVE_RB;
    return r < WAVE_RB ? WAVE_RB : (r > 64 ? 64 : r);
}

template <typename T, class Op>
__device__ __forceinline__ T seg_prefix(T v, int lane, int back) {
    // inclusive prefix over the lanes l' with l - back <= l' <= l
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T o = wshfl(v, lane >= off ? lane - off : lane);
        if (off <= back) v = Op::apply(o, v);
    }
    return v;
}
template <typename T, class Op>
__device__ __forceinline__ T seg_suffix(T v, int lane, int fwd) {
    // inclusive suffix over the lanes l' with l <= l' <= l + fwd
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T o = wshfl(v, lane + off < 64 ? lane + off : lane);
        if (off <= fwd) v = Op::apply(v, o);
    }
    return v;
}

template <typename T, class Op>
__device__ __forceinline__ void task_bdbs_wave(const T* __restrict__ in, T* __restrict__ out,
                                               i64 O, i64 n_, int k, i64 rpt, i64 task) {
    const int lane = threadIdx.x & 63;
    const T e = Op::template id<T>();
    const int n = (int)n_;
    const i64 r_begin = task * rpt;
    const i64 r_end = r_begin + rpt < O ? r_begin + rpt : O;
    const unsigned bytes = (unsigned)(O * n_ * (i64)sizeof(T));
    const __amdgpu_buffer_rsrc_t rin = buf(in, bytes), rout = buf(out, bytes);
    constexpr unsigned es = sizeof(T);
    for (i64 r0 = r_begin; r0 < r_end; r0 += WAVE_RB) {
        unsigned rowoff[WAVE_RB];
        bool live[WAVE_RB];
        T a[WAVE_RB], h[WAVE_RB];
#pragma unroll
        for (int j = 0; j < WAVE_RB; ++j) {
            live[j] = r0 + j < r_end;
            rowoff[j] = (unsigned)((r0 + j) * n_) * es;
            const T t = bload<T>(rin, rowoff[j] + (unsigned)lane * es);
            a[j] = live[j] && lane < n ? t : e;
        }
        for (int c0 = 0; c0 < n; c0 += 64) {
            const int xa = c0 + lane, xh = c0 + 64 + lane;
#pragma unroll
            for (int j = 0; j < WAVE_RB; ++j) {
                const T t = bload<T>(rin, rowoff[j] + (unsigned)xh * es);
                h[j] = live[j] && xh < n ? t : e;
            }
            // block geometry of the two windows (same for every row)
            const int oa = xa % k, oh = xh % k;          // offsets within the blocks
            const int endB = (c0 + 63) - (c0 + 63) % k + k - 1;  // last position of the
            const int eh = endB - (c0 + 64);                      // straddling block
            const int y = xa + k - 1;                    // where the next block's prefix ends
            const int ly = y - c0;                       // its lane in the 128-window
#pragma unroll
            for (int j = 0; j < WAVE_RB; ++j) {
                const T pa = seg_prefix<T, Op>(a[j], lane, oa < lane ? oa : lane);
                const T sa = seg_suffix<T, Op>(a[j], lane, (k - 1 - oa) < 63 - lane ? k - 1 - oa : 63 - lane);
                T ph = seg_prefix<T, Op>(h[j], lane, oh < lane ? oh : lane);
                // the straddling block: suffix part in the second window, prefix
                // part in the first
                const T tailB = wshfl(ph, eh >= 0 ? eh : 0);
                const T headB = wshfl(pa, 63);
                const bool inB = eh >= 0 && xa + (k - 1 - oa) == endB;
                const T rs = inB ? Op::apply(sa, tailB) : sa;
                if (eh >= 0 && lane <= eh) ph = Op::apply(headB, ph);
                const T va = wshfl(pa, ly < 64 ? ly : 63);
                const T vh = wshfl(ph, ly >= 64 ? ly - 64 : 0);
                const T rp = ly < 64 ? va : vh;
                const T o = oa == 0 ? rs : Op::apply(rs, rp);
                bstore<T>(rout, live[j] && xa < n ? rowoff[j] + (unsigned)xa * es : NOWHERE, o);
                a[j] = h[j];
            }
        }
    }
}

// BDBS along the middle axis of an (O, n, I) tensor (I >= 1): task = (run of
// `cb` blocks, group of C columns), the group fastest; one wavefront each.
template <typename T, class Op, int KB>
__device__ __forceinline__ void task_bdbs_coop(const T* __restrict__ in, T* __restrict__ out,
                                               i64 O, i64 n_, i64 I_, int k, i64 cb, i64 task) {
    constexpr int G = coop_g(KB, sizeof(T), false), CS = KB / G;
    using L = CoopLanes<T, Op, G>;
    constexpr int C = L::C;
    const L ln(threadIdx.x & 63);
    const T e = Op::template id<T>();
    const i64 cols = O * I_;
    const i64 ngroups = (cols + C - 1) / C;
    const i64 grp = task % ngroups, run = task / ngroups;
    const int n = (int)n_;
    const int nb = (n + k - 1) / k;
    const int b0 = (int)(run * cb);
    if (b0 >= nb) return;  // the whole wavefront
    const int b1 = b0 + (int)cb < nb ? b0 + (int)cb : nb;
    const i64 col = grp * C + ln.c;
    const bool live = col < cols;
    constexpr unsigned es = sizeof(T);
    const unsigned bytes = (unsigned)(cols * n_ * (i64)es);
    const __amdgpu_buffer_rsrc_t rin = buf(in, bytes), rout = buf(out, bytes);
    const unsigned rowb = (unsigned)(I_ * (i64)es);
    const i64 o = live ? col / I_ : 0, i = live ? col % I_ : 0;
    // byte offset of slot 0 of this lane's segment in block 0
    const unsigned base = (unsigned)((o * n_ * I_ + i) * (i64)es) + (unsigned)(ln.g * CS) * rowb;
    auto lim_of = [&](int b) { return live ? min(k, n - b * k) - ln.g * CS : 0; };

    T rs[CS], v[CS];
    coop_load<T, Op, CS>(rin, base + (unsigned)(b0 * k) * rowb, rowb, lim_of(b0), v);
    {
        T tot = e;
#pragma unroll
        for (int s = 0; s < CS; ++s) tot = Op::apply(tot, v[s]);
        T before, after;
        ln.scan(tot, before, after);
        T sf = after;
#pragma unroll
        for (int s = CS - 1; s >= 0; --s) {
            sf = Op::apply(v[s], sf);
            rs[s] = sf;
        }
    }
    for (int b = b0; b < b1; ++b) {
        const int limn = b + 1 < nb ? lim_of(b + 1) : 0;
        coop_load<T, Op, CS>(rin, base + (unsigned)((b + 1) * k) * rowb, rowb, limn, v);
        T tot = e;
#pragma unroll
        for (int s = 0; s < CS; ++s) tot = Op::apply(tot, v[s]);
        T before, after;
        ln.scan(tot, before, after);
        // block b: range suffix op range prefix of block b + 1 before the slot
        const int limc = lim_of(b);
        const unsigned oc = base + (unsigned)(b * k) * rowb;
        T p = before;
#pragma unroll
        for (int s = 0; s < CS; ++s) {
            bstore<T>(rout, s < limc ? oc + (unsigned)s * rowb : NOWHERE, Op::apply(rs[s], p));
            p = Op::apply(p, v[s]);
        }
        T sf = after;
#pragma unroll
        for (int s = CS - 1; s >= 0; --s) {
            sf = Op::apply(v[s], sf);
            rs[s] = sf;
        }
    }
}

// The axis-0 stream of an (n0, M) tensor W (box-summed over the other axes):
// excluded sums (the op of everything before the row, the rows from the same
// row of the next block on, and SX beyond that; Trest folded into the
// running prefix) and included sums (BDBS along axis 0).  Task = (run of
// `segblocks` blocks, group of C points), the group fastest.
template <typename T, class Op, int KB, int OUT>
__device__ __forceinline__ void task_axis0_coop(const T* __restrict__ W, const T* __restrict__ PX,
                                                const T* __restrict__ SX,
                                                const T* __restrict__ Trest,
                                                T* __restrict__ exc, T* __restrict__ inc,
                                                i64 n0_, i64 M_, int k0, i64 Q_, i64 segblocks,
                                                i64 task) {
    constexpr int G = coop_g_ax0(KB, sizeof(T), OUT), CS = KB / G;
    using L = CoopLanes<T, Op, G>;
    constexpr int C = L::C;
    const L ln(threadIdx.x & 63);
    const T e = Op::template id<T>();
    const int n0 = (int)n0_, Q = (int)Q_;
    const i64 ngroups = (M_ + C - 1) / C;
    const i64 grp = task % ngroups, run = task / ngroups;
    const int qa = (int)(run * segblocks);
    if (qa >= Q) return;  // the whole wavefront
    const int qb = qa + (int)segblocks < Q ? qa + (int)segblocks : Q;
    const i64 m = grp * C + ln.c;
    const bool live = m < M_;
    const bool do_ex = exc != nullptr, do_inc = inc != nullptr;
    constexpr unsigned es = sizeof(T);
    const unsigned rowb = (unsigned)(M_ * (i64)es);
    const unsigned nbytes = (unsigned)n0 * rowb;
    const unsigned qbytes = (unsigned)Q * rowb;
    const __amdgpu_buffer_rsrc_t rw = buf(W, nbytes);
    const __amdgpu_buffer_rsrc_t rex = buf(exc, do_ex ? nbytes : 0u);
    const __amdgpu_buffer_rsrc_t rin = buf(inc, do_inc ? nbytes : 0u);
    const __amdgpu_buffer_rsrc_t rsx = buf(SX, do_ex ? qbytes : 0u);
    const unsigned mo = live ? (unsigned)(m * (i64)es) : 0u;
    const unsigned base = mo + (unsigned)(ln.g * CS) * rowb;
    auto lim_of = [&](int q) { return live ? min(k0, n0 - q * k0) - ln.g * CS : 0; };

    if constexpr (OUT == 1 || OUT == 2) {
        // one output: the held block q is kept as the one scan that output
        // needs of it -- its exclusive prefixes from the block start
        // (excluded sums) or its range suffixes (included sums)
        T h[CS], v[CS];
        T hb, ha, ht;  // op of the held block's segments before / after this lane's, of all
        coop_load<T, Op, CS>(rw, base + (unsigned)(qa * k0) * rowb, rowb, lim_of(qa), v);
        {
            T tot = e;
#pragma unroll
            for (int s = 0; s < CS; ++s) tot = Op::apply(tot, v[s]);
            ln.scan(tot, hb, ha);
            ht = Op::apply(Op::apply(hb, tot), ha);
        }
        T Pb = e;
        if constexpr (OUT == 1) {
            T p = hb;
#pragma unroll
            for (int s = 0; s < CS; ++s) {
                h[s] = p;
                p = Op::apply(p, v[s]);
            }
            Pb = bload<T>(buf(PX, qbytes), mo + (unsigned)qa * rowb);
            if (Trest) Pb = Op::apply(Pb, bload<T>(buf(Trest, rowb), mo));
            if (!live) Pb = e;
        } else {
            T sf = ha;
#pragma unroll
            for (int s = CS - 1; s >= 0; --s) {
                sf = Op::apply(v[s], sf);
                h[s] = sf;
            }
        }
        for (int q = qa; q < qb; ++q) {
            const int limn = q + 1 < Q ? lim_of(q + 1) : 0;
            coop_load<T, Op, CS>(rw, base + (unsigned)((q + 1) * k0) * rowb, rowb, limn, v);
            T vt = e;
#pragma unroll
            for (int s = 0; s < CS; ++s) vt = Op::apply(vt, v[s]);
            T vb, va;
            ln.scan(vt, vb, va);
            const int limc = lim_of(q);
            const unsigned oc = base + (unsigned)(q * k0) * rowb;
            if constexpr (OUT == 1) {
                // everything before the row (Pb, then the held block's prefix),
                // then block q + 1 from the same slot on and the blocks after it
                const T sxv = bload<T>(rsx, mo + (unsigned)(q + 1) * rowb);
                T sf = Op::apply(va, (q + 1 < Q && live) ? sxv : e);
#pragma unroll
                for (int s = CS - 1; s >= 0; --s) {
                    sf = Op::apply(v[s], sf);
                    bstore<T>(rex, s < limc ? oc + (unsigned)s * rowb : NOWHERE,
                              Op::apply(Op::apply(Pb, h[s]), sf));
                }
                Pb = Op::apply(Pb, ht);
                T p = vb;
#pragma unroll
                for (int s = 0; s < CS; ++s) {
                    h[s] = p;
                    p = Op::apply(p, v[s]);
                }
            } else {
                // range suffix of block q op range prefix of block q + 1
                T p = vb;
#pragma unroll
                for (int s = 0; s < CS; ++s) {
                    bstore<T>(rin, s < limc ? oc + (unsigned)s * rowb : NOWHERE,
                              Op::apply(h[s], p));
                    p = Op::apply(p, v[s]);
                }
                T sf = va;
#pragma unroll
                for (int s = CS - 1; s >= 0; --s) {
                    sf = Op::apply(v[s], sf);
                    h[s] = sf;
                }
            }
            ht = Op::apply(Op::apply(vb, vt), va);
        }
        return;
    }
    // both outputs (or either, decided at run time): w holds the raw values
    // of the held block q; wb, wa: op of its other segments before / after
    // this lane's; wt: op of the whole block
    T w[CS], v[CS], t[CS];
    T wb, wa, wt;
    coop_load<T, Op, CS>(rw, base + (unsigned)(qa * k0) * rowb, rowb, lim_of(qa), w);
    {
        T tot = e;
#pragma unroll
        for (int s = 0; s < CS; ++s) tot = Op::apply(tot, w[s]);
        ln.scan(tot, wb, wa);
        wt = Op::apply(Op::apply(wb, tot), wa);
    }
    // Pb: op of every row before the held block, with the lower-dimensional term
    T Pb = e;
    if (do_ex) {
        Pb = bload<T>(buf(PX, qbytes), mo + (unsigned)qa * rowb);
        if (Trest) Pb = Op::apply(Pb, bload<T>(buf(Trest, rowb), mo));
        if (!live) Pb = e;
    }
    for (int q = qa; q < qb; ++q) {
        const int limn = q + 1 < Q ? lim_of(q + 1) : 0;
        coop_load<T, Op, CS>(rw, base + (unsigned)((q + 1) * k0) * rowb, rowb, limn, v);
        T vt = e;
#pragma unroll
        for (int s = 0; s < CS; ++s) vt = Op::apply(vt, v[s]);
        T vb, va;
        ln.scan(vt, vb, va);
        const int limc = lim_of(q);
        const unsigned oc = base + (unsigned)(q * k0) * rowb;
        if (do_inc) {
            // range suffix of block q from the slot on, op range prefix of
            // block q + 1 before the slot
            T p = vb;
#pragma unroll
            for (int s = 0; s < CS; ++s) {
                t[s] = p;
                p = Op::apply(p, v[s]);
            }
            T sf = wa;
#pragma unroll
            for (int s = CS - 1; s >= 0; --s) {
                sf = Op::apply(w[s], sf);
                bstore<T>(rin, s < limc ? oc + (unsigned)s * rowb : NOWHERE, Op::apply(sf, t[s]));
            }
        }
        if (do_ex) {
            // everything before the row, then the rows of block q + 1 from the
            // same slot on and the blocks after it
            T p = Op::apply(Pb, wb);
#pragma unroll
            for (int s = 0; s < CS; ++s) {
                t[s] = p;
                p = Op::apply(p, w[s]);
            }
            const T sxv = bload<T>(rsx, mo + (unsigned)(q + 1) * rowb);
            T sf = Op::apply(va, (q + 1 < Q && live) ? sxv : e);
#pragma unroll
            for (int s = CS - 1; s >= 0; --s) {
                sf = Op::apply(v[s], sf);
                bstore<T>(rex, s < limc ? oc + (unsigned)s * rowb : NOWHERE, Op::apply(t[s], sf));
            }
            Pb = Op::apply(Pb, wt);
        }
#pragma unroll
        for (int s = 0; s < CS; ++s) w[s] = v[s];
        wb = vb;
        wa = va;
        wt = Op::apply(Op::apply(vb, vt), va);
    }
}

// Dispatch one task of a recorded step (KB: the register bucket of the step,
// for the kinds that have one).
template <typename T, class Op, int KIND, int KB>
__device__ __forceinline__ void run_task(const Step& s, i64 i) {
    if constexpr (KIND == SK_BDBS || KIND == SK_BDBSW)
        task_bdbs<T, Op, KB, KIND == SK_BDBS>((const T*)s.in0, (T*)s.out0, s.O, s.n, s.I, s.k,
                                              s.cb, s.nchunks, i);
    else if constexpr (KIND == SK_BDBS2)
        task_bdbs2<T, Op>((const T*)s.in0, (T*)s.out0, s.n, s.I, s.k, i);
    else if constexpr (KIND == SK_AGG)
        task_agg<T, Op>((const T*)s.in0, (T*)s.out0, s.n, s.I, s.k, i);
    else if constexpr (KIND == SK_SCAN)
        task_scan<T, Op>((const T*)s.in0, (const T*)s.in1, (T*)s.out0, (T*)s.out1, (T*)s.out2,
                         s.Q, s.I, i);
    else if constexpr (KIND == SK_SEGTOT)
        task_segtot<T, Op>((const T*)s.in0, (const T*)s.in1, (T*)s.out0, (T*)s.out1, s.Q, s.I,
                           s.cb, i);
    else if constexpr (KIND == SK_SEGEXP)
        task_segexp<T, Op>((const T*)s.in0, (const T*)s.in1, (const T*)s.in2, (T*)s.out0,
                           (T*)s.out1, s.Q, s.I, s.cb, i);
    else if constexpr (KIND == SK_BDBSV)
        task_bdbs_wave<T, Op>((const T*)s.in0, (T*)s.out0, s.O, s.n, s.k, s.cb, i >> 6);
    else if constexpr (KIND == SK_BDBSC)
        task_bdbs_coop<T, Op, KB>((const T*)s.in0, (T*)s.out0, s.O, s.n, s.I, s.k, s.cb,
                                  i >> 6);
    else if constexpr (KIND == SK_AX0C)
        task_axis0_coop<T, Op, KB, 3>(
            (const T*)s.in0, (const T*)s.in1, (const T*)s.in2, (const T*)s.in3, (T*)s.out0,
            (T*)s.out1, s.n, s.I, s.k, s.Q, s.cb, i >> 6);
    else if constexpr (KIND == SK_AX0 || KIND == SK_AX0W)
        task_axis0<T, Op, KB, KIND == SK_AX0>((const T*)s.in0, (const T*)s.in1, (const T*)s.in2,
                                              (const T*)s.in3, (T*)s.out0, (T*)s.out1, s.n, s.I,
                                              s.k, s.Q, s.cb, i);
    else
        task_ex2<T, Op>((const T*)s.in0, (const T*)s.in3, (T*)s.out0, s.n, s.I, s.k, i);
}

// The element type and operator of a part of a work-list launch (uniform
// over the workgroup, so the branch is a scalar one): F receives a value of
// the type and the operator as template arguments.
template <typename T, class Op>
struct TypeOp {
    using type = T;
    using op = Op;
};
template <int ES, class F>
__device__ __forceinline__ void with_type_op(int code, F&& f) {
    if constexpr (ES == 4) {
        switch (code) {
            case EXS_F32 * 4 + EXS_SUM: f(TypeOp<float, OpSum>{}); break;
            case EXS_F32 * 4 + EXS_MAX: f(TypeOp<float, OpMax>{}); break;
            case EXS_F32 * 4 + EXS_MIN: f(TypeOp<float, OpMin>{}); break;
            case EXS_I32 * 4 + EXS_SUM: f(TypeOp<int, OpSum>{}); break;
            case EXS_I32 * 4 + EXS_MAX: f(TypeOp<int, OpMax>{}); break;
            default: f(TypeOp<int, OpMin>{}); break;
        }
    } else {
        switch (code) {
            case EXS_F64 * 4 + EXS_SUM: f(TypeOp<double, OpSum>{}); break;
            case EXS_F64 * 4 + EXS_MAX: f(TypeOp<double, OpMax>{}); break;
            case EXS_F64 * 4 + EXS_MIN: f(TypeOp<double, OpMin>{}); break;
            case EXS_I64 * 4 + EXS_SUM: f(TypeOp<long long, OpSum>{}); break;
            case EXS_I64 * 4 + EXS_MAX: f(TypeOp<long long, OpMax>{}); break;
            default: f(TypeOp<long long, OpMin>{}); break;
        }
    }
}

}  // namespace exs
