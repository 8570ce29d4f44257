// exsum_row.hpp -- fused streaming kernel for a 2-D level (template;
// instantiated per element type in exsum_row.hip).
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// The rank-2 counterpart of k_plane_axis0: for a (n0, NX) tensor, one
// workgroup owns a tile of the row axis for a run of k0-blocks of axis 0 and
// walks axis 0, P rows per round:
//   1. the row segments plus their (kx - 1)-element halo are staged in LDS
//      (blocked layout, identity padding, as in the plane kernel);
//   2. BDBS along the rows (Sec. 3; "BDBS-Along-Dim", Sec. 5), written into a
//      ring of k0 rows in LDS;
//   3. once a k0-block of box-summed rows is in the ring, each thread (one
//      point of the tile) emits the previous block: the excluded sum (prefix
//      before x0, suffix from x0 + k0, the lower-dimensional contribution) and
//      the included sum (BDBS along axis 0).
// It replaces a box-sum pass along the rows plus a separate axis-0 stream
// over the stored result.
#pragma once
#include "exsum_plane.hpp"

namespace exs {

struct RowArgs {
    const void* X;      // (n0, NX)
    const void* PX;     // (Q, NX) op of the box-summed block totals before each block
    const void* SX;     // (Q, NX) ... after each block
    const void* Trest;  // (NX) lower-dimensional excluded sums, or null
    void* exc;          // (n0, NX) or null
    void* inc;          // (n0, NX) or null
    i64 n0, NX, Q;
    int k0, kx;
    int nt;             // output stores carry the non-temporal hint
    i64 tiles, segblocks, nseg;
};

// 256 blocked points per workgroup, one thread each; P rows per round.
template <int KP>
struct RowCfg {
    static constexpr int NT = 256;
    static constexpr int NBX = NT / KP;             // blocks per tile
    static constexpr int COLS = (NBX + 1) * KP;     // blocked halo columns
    static constexpr int PA = COLS + 1;             // odd LDS pitch
    static constexpr int MAXIN = NT + 15;           // real halo elements per row, kx <= 16
    static constexpr int NLOAD = (MAXIN + NT - 1) / NT;
    static constexpr int P = 8;
    static constexpr int RT = (P * NBX + NT - 1) / NT;  // row tasks per thread
};

template <typename T, class Op, int K0B, int KP>
__global__ void __launch_bounds__(256) k_row_axis0(RowArgs a) {
    using C = RowCfg<KP>;
    constexpr int NT = C::NT, P = C::P, PA = C::PA;
    __shared__ T sA[P * PA + 1];  // + a dummy word for writes that must land nowhere
    __shared__ T ring[K0B * NT];

    const T e = Op::template id<T>();
    const int tid = threadIdx.x;
    i64 wg = blockIdx.x;
    const i64 nwg = (i64)gridDim.x;
    if ((nwg & 7) == 0) wg = (wg & 7) * (nwg >> 3) + (wg >> 3);
    const i64 tile = wg % a.tiles;
    const int seg = (int)(wg / a.tiles);
    const int k0 = a.k0, kx = a.kx;
    const int NX = (int)a.NX;
    const int x0 = (int)tile * (C::NBX * kx);
    const int Qn = (int)a.Q;
    const int qa = seg * (int)a.segblocks;
    const int qb = qa + (int)a.segblocks < Qn ? qa + (int)a.segblocks : Qn;
    const int n0 = (int)a.n0;
    const i64 M = a.NX;
    const unsigned row_bytes = (unsigned)(M * (i64)sizeof(T));

    // this thread's point
    const int px = (tid / KP) * kx + tid % KP;
    const bool pvalid = tid % KP < kx && x0 + px < NX;
    const unsigned mb = pvalid ? (unsigned)(x0 + px) * sizeof(T) : (unsigned)K0B * row_bytes;

    for (int i = tid; i < P * PA; i += NT) sA[i] = e;
    for (int r = 0; r < K0B; ++r) ring[r * NT + tid] = e;

    // halo load plan: real element c of the row segment -> blocked LDS slot,
    // byte offset in a row
    const int cols_in = C::NBX * kx + kx - 1;
    int loff[C::NLOAD];
    unsigned goff[C::NLOAD];
#pragma unroll
    for (int j = 0; j < C::NLOAD; ++j) {
        const int c = tid + j * NT;
        const bool inside = c < cols_in && x0 + c < NX;
        loff[j] = inside ? (c / kx) * KP + c % kx : P * PA;
        goff[j] = inside ? (unsigned)(x0 + c) * sizeof(T) : 0u;
    }
    // row tasks (u, b), u outermost; packed u | b << 4; -1 = none
    int rp[C::RT];
#pragma unroll
    for (int i = 0; i < C::RT; ++i) {
        const int task = tid + i * NT;
        rp[i] = task < P * C::NBX ? ((task / C::NBX) | ((task % C::NBX) << 4)) : -1;
    }

    const T* __restrict__ X = (const T*)a.X;
    const int t_begin = qa * k0;
    int t_end = (qb + 1) * k0;  // one block past the run: the suffix/inclusion lag
    if (t_end > n0) t_end = n0;

    const bool do_ex = a.exc != nullptr, do_inc = a.inc != nullptr;
    T* __restrict__ exc = (T*)a.exc;
    T* __restrict__ inc = (T*)a.inc;

    // axis-0 state (as in k_plane_axis0)
    T w[K0B];
#pragma unroll
    for (int r = 0; r < K0B; ++r) w[r] = e;
    T Pb = e;
    if (do_ex) {
        Pb = bload<T>(buf((const T*)a.PX + (i64)qa * M, row_bytes), mb);
        if (a.Trest) Pb = Op::apply(Pb, bload<T>(buf(a.Trest, row_bytes), mb));
    }
    T sx_raw = e;
    bool sx_valid = false;

    auto block_step_h = [&](int q, auto ntc) __attribute__((always_inline)) {
        constexpr bool NTS = decltype(ntc)::value;
        __syncthreads();
        T v[K0B];
#pragma unroll
        for (int r = 0; r < K0B; ++r) v[r] = ring[r * NT + tid];
        if (q != qa) {
            const int xb = (q - 1) * k0;
            const int nrows = n0 - xb < k0 ? n0 - xb : k0;
            const unsigned blk_bytes = (unsigned)nrows * row_bytes;
            T tmp[K0B];
            if (do_ex) {
#pragma unroll
                for (int r = 0; r < K0B; ++r) { tmp[r] = Pb; Pb = Op::apply(Pb, w[r]); }
                const __amdgpu_buffer_rsrc_t ob = buf(exc + (i64)xb * M, blk_bytes);
                T S = sx_valid ? sx_raw : e;
#pragma unroll
                for (int r = K0B - 1; r >= 0; --r) {
                    S = Op::apply(v[r], S);
                    bstore_h<T, NTS>(ob, mb + (unsigned)r * row_bytes, Op::apply(tmp[r], S));
                }
            }
            if (do_inc) {
                T s = e;
#pragma unroll
                for (int r = K0B - 1; r >= 0; --r) { s = Op::apply(w[r], s); tmp[r] = s; }
                const __amdgpu_buffer_rsrc_t ob = buf(inc + (i64)xb * M, blk_bytes);
                T p = e;
#pragma unroll
                for (int r = 0; r < K0B; ++r) {
                    T val = tmp[r];
                    if (r > 0) { p = Op::apply(p, v[r - 1]); val = Op::apply(val, p); }
                    bstore_h<T, NTS>(ob, mb + (unsigned)r * row_bytes, val);
                }
            }
        }
        if (q < qb) {
#pragma unroll
            for (int r = 0; r < K0B; ++r) w[r] = v[r];
        }
    };
    auto block_step = [&](int q) __attribute__((always_inline)) {
        if (a.nt) block_step_h(q, std::true_type{});
        else block_step_h(q, std::false_type{});
    };
    auto ring_fill_identity = [&](int from) {
        for (int r = from; r < K0B; ++r) ring[r * NT + tid] = e;
    };
    auto round_len = [&](int tt, int rr) -> int {
        int n = k0 - rr;
        if (tt + n > t_end) n = t_end - tt;
        return n < P ? n : P;
    };
    // raw halo values prefetched two rounds ahead; the loads are issued
    // unconditionally (past the run they re-read its first row)
    int tf = t_begin, rf = 0;
    auto fetch_next = [&](T (&pre)[P][C::NLOAD]) __attribute__((always_inline)) {
        const bool live = tf < t_end;
        const int np = live ? round_len(tf, rf) : P;
        const int tb = live ? tf : t_begin;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const __amdgpu_buffer_rsrc_t rw = buf(X + (i64)(u < np ? tb + u : tb) * M, row_bytes);
#pragma unroll
            for (int j = 0; j < C::NLOAD; ++j) pre[u][j] = bload<T>(rw, goff[j]);
        }
        if (live) {
            tf += np;
            rf = rf + np == k0 ? 0 : rf + np;
        }
    };

    int qlast = qa - 1;
    int t = t_begin, q = qa, r0 = 0;
    auto step = [&](T (&pre)[P][C::NLOAD]) __attribute__((always_inline)) {
        const int np = round_len(t, r0);
        if (r0 == 0) {
            sx_valid = q < Qn;
            if (do_ex)
                sx_raw = bload<T>(buf((const T*)a.SX + (i64)(q < Qn ? q : Qn - 1) * M, row_bytes),
                                  mb);
        }
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (u < np) {
#pragma unroll
                for (int j = 0; j < C::NLOAD; ++j) {
                    const int o = loff[j] == P * PA ? P * PA : u * PA + loff[j];
                    sA[o] = pre[u][j];
                }
            }
        }
        fetch_next(pre);
        __syncthreads();
        // BDBS along every row of the round, into the ring slots
#pragma unroll
        for (int i = 0; i < C::RT; ++i) {
            const int pk = rp[i];
            if (pk >= 0 && (pk & 15) < np) {
                const int u = pk & 15, b = pk >> 4;
                bdbs_block<T, Op, KP, 1, 1>(sA + u * PA + b * KP, ring + (r0 + u) * NT + b * KP);
            }
        }
        const int tn = t + np;
        const int rn = r0 + np == k0 ? 0 : r0 + np;
        if (r0 + np == k0 || tn == n0) {
            if (r0 + np < k0) ring_fill_identity(r0 + np);  // the tensor ends inside the block
            block_step(q);
            qlast = q;
        } else {
            __syncthreads();  // the staging of the next round overwrites sA
        }
        t = tn;
        if (rn == 0) ++q;
        r0 = rn;
    };

    T pre0[P][C::NLOAD], pre1[P][C::NLOAD];
    fetch_next(pre0);
    fetch_next(pre1);
    __syncthreads();  // identity fill visible before the first staging
    while (t < t_end) {
        step(pre0);
        if (t >= t_end) break;
        step(pre1);
    }
    if (qlast < qb) {
        sx_valid = false;
        ring_fill_identity(0);
        block_step(qb);
    }
}

// Tiles of a row of NX points for row box kx (the KP bucket's tile width).
inline i64 row_tiles(i64 NX, i64 kx) {
    const i64 kp = kx <= 2 ? 2 : kx <= 4 ? 4 : kx <= 8 ? 8 : 16;
    const i64 tx = (256 / kp) * kx;
    return (NX + tx - 1) / tx;
}

// Blocks of axis 0 per workgroup run (about 4 workgroups of 256 per CU).
inline i64 row_run_blocks(i64 Q, i64 NX, i64 kx) {
    const i64 tiles = row_tiles(NX, kx);
    i64 nseg = (1024 + tiles - 1) / tiles;
    if (nseg > Q) nseg = Q;
    if (nseg < 1) nseg = 1;
    return (Q + nseg - 1) / nseg;
}

template <typename T, class Op, int K0B, int KP>
void launch_row_kernel(RowArgs ra, hipStream_t st) {
    ra.tiles = row_tiles(ra.NX, ra.kx);
    ra.segblocks = row_run_blocks(ra.Q, ra.NX, ra.kx);
    ra.nseg = (ra.Q + ra.segblocks - 1) / ra.segblocks;
    hipLaunchKernelGGL((k_row_axis0<T, Op, K0B, KP>), dim3((unsigned)(ra.tiles * ra.nseg)),
                       dim3(RowCfg<KP>::NT), 0, st, ra);
}

template <typename T, class Op, int K0B>
void launch_row_kp(RowArgs ra, hipStream_t st) {
    if (ra.kx <= 2) launch_row_kernel<T, Op, K0B, 2>(ra, st);
    else if (ra.kx <= 4) launch_row_kernel<T, Op, K0B, 4>(ra, st);
    else if (ra.kx <= 8) launch_row_kernel<T, Op, K0B, 8>(ra, st);
    else launch_row_kernel<T, Op, K0B, 16>(ra, st);
}

template <typename T, class Op>
void launch_row_axis0(const T* X, const T* PX, const T* SX, const T* Trest, T* exc, T* inc, i64 n0,
                      i64 NX, i64 k0, i64 kx, i64 Q, hipStream_t st) {
    KTimer timer("k_row_axis0", st);
    RowArgs ra{};
    ra.X = X; ra.PX = PX; ra.SX = SX; ra.Trest = Trest; ra.exc = exc; ra.inc = inc;
    ra.n0 = n0; ra.NX = NX; ra.Q = Q; ra.k0 = (int)k0; ra.kx = (int)kx;
    ra.nt = store_hint_ok(NX * (i64)sizeof(T));
    if (k0 <= 4) launch_row_kp<T, Op, 4>(ra, st);
    else if (k0 <= 8) launch_row_kp<T, Op, 8>(ra, st);
    else launch_row_kp<T, Op, 16>(ra, st);
}

}  // namespace exs
