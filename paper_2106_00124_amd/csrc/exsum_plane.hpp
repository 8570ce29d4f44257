// exsum_plane.hpp -- fused streaming kernel for the first dimension-reduction
// step of included/excluded sums on gfx950 (template; instantiated per element
// type in exsum_plane_*.hip).
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// For a rank >= 3 tensor viewed as (n0, MID, NY, NX) -- MID collects the
// middle axes, already box-summed -- one workgroup owns a tile of the
// (NY, NX) plane for a run of k0-blocks of axis 0 and walks axis 0, P planes
// per round:
//   1. the tiles plus their (ky-1, kx-1) halos are staged in LDS;
//   2. BDBS along x over every halo row (Sec. 3: range suffix of a block,
//      range prefix of the next block, combine);
//   3. BDBS along y over every column, into a ring of k0 planes in LDS:
//      W = each plane box-summed over its two axes ("BDBS-Along-Dim", Sec. 5);
//   4. once a k0-block of W planes is in the ring, each thread (one point of
//      the tile) updates its axis-0 state in registers and emits the previous
//      block: the excluded sum (prefix before x0, suffix from x0+k0, the
//      lower-dimensional contribution) and the included sum (BDBS along
//      axis 0).
//
// Blocked layout.  Along y and x, every k-block of the tile (and of its halo)
// occupies KP slots in LDS, KP the power of two >= k; the slots past k hold
// the identity (written once), so every scan is a fixed-length KP scan with no
// masks: the identities leave the range suffixes and prefixes of the real
// elements unchanged.  Points of the tile use the same layout; padding points
// are simply not stored.
#pragma once
#include "exsum_device.hpp"
#include "exsum_internal.hpp"

namespace exs {

struct PlaneArgs {
    const void* X;      // (n0, MID, NY, NX): input box-summed over the middle axes
    const void* PX;     // (Q, M) op of W-block totals strictly before each block
    const void* SX;     // (Q, M) op of W-block totals strictly after each block
    const void* Trest;  // (M) lower-dimensional excluded sums, or null
    void* exc;          // (n0, M) or null
    void* inc;          // (n0, M) or null
    const void* wtot;   // weak excluded sums: the total of the tensor (one element)
    void* wexc;         // weak excluded sums: (n0, M) total minus included, or null
    i64 n0, MID, NY, NX, M, Q;
    int k0, ky, kx;
    int nt;             // output stores carry the non-temporal hint
    i64 tilesY, tilesX, segblocks, nseg;
};

// 32 x 32 blocked points per workgroup, one thread each; P planes per round.
template <int KP, int PLANES = 4>
struct PlaneCfg {
    static constexpr int NT = 1024;
    static constexpr int TYM = 32, TXM = 32;
    static constexpr int NBY = TYM / KP, NBX = TXM / KP;   // output blocks per tile
    static constexpr int ROWS = (NBY + 1) * KP;            // blocked halo rows
    static constexpr int COLS = (NBX + 1) * KP;            // blocked halo cols
    static constexpr int PA = COLS | 1;                    // odd LDS pitch
    static constexpr int PB = TXM + 1;                     // odd LDS pitch
    static constexpr int SA = ROWS * PA, SB = ROWS * PB;
    // real halo elements of a tile: NB blocks of k <= KP points and k - 1 more
    static constexpr int MAXIN = (TYM + KP - 1) * (TXM + KP - 1);
    static constexpr int NLOAD = (MAXIN + NT - 1) / NT;
    static constexpr int P = PLANES;
    static constexpr int RT = (P * ROWS * NBX + NT - 1) / NT;  // row tasks per thread
    static constexpr int CT = (P * TXM * NBY + NT - 1) / NT;   // column tasks per thread
};

// Blocks of axis 0 per workgroup run of the streaming kernel.  The stream
// kernel fills a CU with one workgroup, so a launch of W workgroups takes
// ceil(W / 256) waves, each as long as one run (its blocks plus the one
// lookahead block every run reads): the split of the tiles' blocks into runs
// that minimises waves x (blocks per run + 1) wins, the fewest runs on ties.
inline i64 plane_run_blocks(i64 Q, i64 tiles) {
    constexpr i64 CUS = 256;
    i64 best = Q > 0 ? Q : 1, best_cost = -1;
    const i64 maxseg = Q < 64 ? Q : 64;
    for (i64 nseg = 1; nseg <= maxseg; ++nseg) {
        const i64 sb = (Q + nseg - 1) / nseg;
        const i64 runs = (Q + sb - 1) / sb;
        const i64 waves = (tiles * runs + CUS - 1) / CUS;
        const i64 cost = waves * (sb + 1);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = sb;
        }
    }
    return best;
}

// Tiles of the (NY, NX) plane for boxes (ky, kx) (the KP bucket's tile shape).
inline i64 plane_tiles(i64 NY, i64 NX, i64 ky, i64 kx) {
    const i64 km = ky > kx ? ky : kx;
    const i64 kp = km <= 2 ? 2 : km <= 4 ? 4 : km <= 8 ? 8 : 16;
    const i64 ty = (32 / kp) * ky, tx = (32 / kp) * kx;
    return ((NY + ty - 1) / ty) * ((NX + tx - 1) / tx);
}

// One BDBS block over KP slots: out[r] = rsuf_b[r] op rpre_{b+1}[r-1]
// (out[0] = rsuf_b[0]); src[0..KP) is the block, src[KP..2KP-1) the next one,
// strided by SS in LDS.  Loads issue back to back; no branches.
template <typename T, class Op, int KP, int SS, int DS>
__device__ __forceinline__ void bdbs_block(const T* __restrict__ src, T* __restrict__ dst) {
    const T e = Op::template id<T>();
    T a0[KP], a1[KP];
#pragma unroll
    for (int r = 0; r < KP; ++r) a0[r] = src[r * SS];
#pragma unroll
    for (int r = 0; r < KP - 1; ++r) a1[r] = src[(KP + r) * SS];
    T sfx = e;
#pragma unroll
    for (int r = KP - 1; r >= 0; --r) {
        sfx = Op::apply(a0[r], sfx);
        a0[r] = sfx;
    }
    T p = e;
#pragma unroll
    for (int r = 1; r < KP; ++r) {
        p = Op::apply(p, a1[r - 1]);
        a0[r] = Op::apply(a0[r], p);
    }
#pragma unroll
    for (int r = 0; r < KP; ++r) dst[r * DS] = a0[r];
}

// WHOLE: every block of the run is exactly K0B planes (k0 == K0B, n0 a
// multiple of k0) and K0B / P is even, so each block is a fixed sequence of
// full rounds; otherwise rounds are sized at run time.
// WEAK: also store total - included (the weak excluded sum, + only).
// K0B <= 8 with boxes up to 8 fits in 64 VGPRs and half the LDS (K0B = 8
// with two planes per round instead of four): two workgroups per CU, so that
// one workgroup's loads overlap the other's scans.
template <typename T, class Op, int K0B, int KP, bool WHOLE, bool WEAK>
__global__ void __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(K0B <= 8 && KP <= 8 ? 8 : 1))) k_plane_axis0(PlaneArgs a) {
    using C = PlaneCfg<KP, K0B == 8 && KP <= 8 ? 2 : 4>;
    constexpr int NT = C::NT, P = C::P, SA = C::SA, SB = C::SB;
    __shared__ T sA[P * SA + 1];  // + a dummy word for writes that must land nowhere
    __shared__ T sB[P * SB];
    __shared__ T ring[K0B * NT];

    const T e = Op::template id<T>();
    const int tid = threadIdx.x;

    // workgroup -> (segment, mid, tile); the workgroups that land on one XCD
    // (ids congruent mod 8) get consecutive tiles of the plane
    i64 wg = blockIdx.x;
    const i64 nwg = (i64)gridDim.x;
    if ((nwg & 7) == 0) wg = (wg & 7) * (nwg >> 3) + (wg >> 3);
    const i64 tiles = a.tilesY * a.tilesX;
    const i64 tile = wg % tiles;
    const i64 rest = wg / tiles;
    const int mid = (int)(rest % a.MID);
    const int seg = (int)(rest / a.MID);
    const int k0 = a.k0, ky = a.ky, kx = a.kx;
    const int NY = (int)a.NY, NX = (int)a.NX;
    // tiles in groups of four tile rows, column by column inside a group, so
    // that one XCD's run of tiles is a compact patch of the plane (its halos
    // are mostly read by the same L2)
    const i64 grow = 4 * a.tilesX;
    const i64 g0 = tile / grow, gin = tile % grow;
    const i64 gh = a.tilesY - g0 * 4 < 4 ? a.tilesY - g0 * 4 : 4;
    const int y0 = (int)(g0 * 4 + gin % gh) * (C::NBY * ky);
    const int x0 = (int)(gin / gh) * (C::NBX * kx);
    // plane and block indices fit in 32 bits (checked by the planner)
    const int Qn = (int)a.Q;
    const int qa = seg * (int)a.segblocks;
    const int qb = qa + (int)a.segblocks < Qn ? qa + (int)a.segblocks : Qn;
    const int n0 = (int)a.n0;
    const i64 M = a.M;
    const unsigned plane_bytes = (unsigned)(M * (i64)sizeof(T));
    const unsigned mid_off = (unsigned)mid * (unsigned)NY * (unsigned)NX;

    // this thread's point in the blocked tile
    const int pyb = tid / C::TXM, pxb = tid % C::TXM;
    const int py = (pyb / KP) * ky + pyb % KP, px = (pxb / KP) * kx + pxb % KP;
    const bool pvalid = pyb % KP < ky && pxb % KP < kx && y0 + py < NY && x0 + px < NX;
    // a point outside the tensor reads and writes past every descriptor's
    // range: its loads return 0 and its stores are dropped
    const unsigned mb = pvalid ? (mid_off + (unsigned)((y0 + py) * NX + x0 + px)) * sizeof(T)
                               : (unsigned)K0B * plane_bytes;

    // LDS: identity everywhere in the plane buffers, then per plane only the
    // real halo elements are overwritten
    for (int i = tid; i < P * SA; i += NT) sA[i] = e;
    for (int r = 0; r < K0B; ++r) ring[r * NT + tid] = e;

    // halo load plan (same for every plane): real element el -> (row, col) of
    // the halo, its blocked LDS slot and its byte offset in a plane
    const int rows_in = C::NBY * ky + ky - 1, cols_in = C::NBX * kx + kx - 1;
    const int count = rows_in * cols_in;
    int loff[C::NLOAD];
    unsigned goff[C::NLOAD];
#pragma unroll
    for (int j = 0; j < C::NLOAD; ++j) {
        const int el = tid + j * NT;
        const int r = el / cols_in, c = el % cols_in;
        const bool inside = el < count && y0 + r < NY && x0 + c < NX;
        loff[j] = inside ? ((r / ky) * KP + r % ky) * C::PA + (c / kx) * KP + c % kx : P * SA;
        goff[j] = inside ? (mid_off + (unsigned)((y0 + r) * NX + x0 + c)) * sizeof(T) : 0u;
    }

    // scan tasks of a round: row task (u, b, row) over every blocked row
    // (padding rows carry identities through), column task (u, b, col) over
    // every blocked column; u outermost, so a round of np < P planes runs the
    // tasks with u < np.  Packed as u | b << 2 | idx << 8; -1 = no task.
    constexpr int rt1 = C::ROWS * C::NBX, ct1 = C::TXM * C::NBY;
    int rp[C::RT], cp[C::CT];
#pragma unroll
    for (int i = 0; i < C::RT; ++i) {
        const int task = tid + i * NT;
        const int u = task / rt1, rem = task % rt1;
        rp[i] = task < P * rt1 ? (u | ((rem / C::ROWS) << 2) | ((rem % C::ROWS) << 8)) : -1;
    }
#pragma unroll
    for (int i = 0; i < C::CT; ++i) {
        const int task = tid + i * NT;
        const int u = task / ct1, rem = task % ct1;
        cp[i] = task < P * ct1 ? (u | ((rem / C::TXM) << 2) | ((rem % C::TXM) << 8)) : -1;
    }

    const T* __restrict__ X = (const T*)a.X;
    const int t_begin = qa * k0;
    int t_end = (qb + 1) * k0;  // one block past the run: the suffix/inclusion lag
    if (t_end > n0) t_end = n0;

    const bool do_ex = a.exc != nullptr, do_inc = a.inc != nullptr;
    T wtot = e;
    if constexpr (WEAK) wtot = *(const T*)a.wtot;
    T* __restrict__ exc = (T*)a.exc;
    T* __restrict__ inc = (T*)a.inc;

    // axis-0 state: the box-summed values of the last complete block (raw;
    // its range prefixes and suffixes are formed when it is emitted) and the
    // op of everything before that block (with the lower-dimensional term)
    T w[K0B];
#pragma unroll
    for (int r = 0; r < K0B; ++r) w[r] = e;
    T Pb = e;
    if (do_ex) {
        Pb = bload<T>(buf((const T*)a.PX + (i64)qa * M, plane_bytes), mb);
        if (a.Trest) Pb = Op::apply(Pb, bload<T>(buf(a.Trest, plane_bytes), mb));
    }
    // SX of the block being filled: loaded when the block starts, from an
    // in-range block index; the identity past the last block is applied at use
    T sx_raw = e;
    bool sx_valid = false;

    // Emit block (q-1) from w and the ring holding block q, then keep block q.
    // Ring slots past k0, and past the end of the tensor, hold the identity;
    // rows of block q-1 past the tensor end fall outside the store range.
    auto block_step_h = [&](int q, auto ntc) __attribute__((always_inline)) {
        constexpr bool NTS = decltype(ntc)::value;
        __syncthreads();
        T v[K0B];
#pragma unroll
        for (int r = 0; r < K0B; ++r) v[r] = ring[r * NT + tid];
        if (q != qa) {
            const int xb = (q - 1) * k0;
            const int nrows = n0 - xb < k0 ? n0 - xb : k0;
            const unsigned blk_bytes = (unsigned)nrows * plane_bytes;
            T tmp[K0B];
            if (do_ex) {
                // prefix before each row of block q-1, then the suffix from
                // the same row of block q on
#pragma unroll
                for (int r = 0; r < K0B; ++r) { tmp[r] = Pb; Pb = Op::apply(Pb, w[r]); }
                const __amdgpu_buffer_rsrc_t ob = buf(exc + (i64)xb * M, blk_bytes);
                T S = sx_valid ? sx_raw : e;
#pragma unroll
                for (int r = K0B - 1; r >= 0; --r) {
                    S = Op::apply(v[r], S);
                    bstore_h<T, NTS>(ob, mb + (unsigned)r * plane_bytes, Op::apply(tmp[r], S));
                }
            }
            if (do_inc || WEAK) {
                // BDBS along axis 0: range suffix in block q-1, range prefix
                // of block q up to the row before
                T s = e;
#pragma unroll
                for (int r = K0B - 1; r >= 0; --r) { s = Op::apply(w[r], s); tmp[r] = s; }
                const __amdgpu_buffer_rsrc_t ob =
                    do_inc ? buf(inc + (i64)xb * M, blk_bytes) : buf(X, 0u);
                const __amdgpu_buffer_rsrc_t ow =
                    WEAK ? buf((T*)a.wexc + (i64)xb * M, blk_bytes) : buf(X, 0u);
                T p = e;
#pragma unroll
                for (int r = 0; r < K0B; ++r) {
                    T val = tmp[r];
                    if (r > 0) { p = Op::apply(p, v[r - 1]); val = Op::apply(val, p); }
                    if (do_inc) bstore_h<T, NTS>(ob, mb + (unsigned)r * plane_bytes, val);
                    if constexpr (WEAK)
                        bstore_h<T, NTS>(ow, mb + (unsigned)r * plane_bytes, Op::inverse(wtot, val));
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
    // Rounds of up to P planes that stay inside one k0-block.  Raw halo
    // values are prefetched two rounds ahead into two register sets used
    // alternately (consumed only when staged into LDS).
    int tf = t_begin, rf = 0;  // the next round to fetch
    // The loads are issued unconditionally (past the run they re-read its
    // first plane), so the number of loads between a load and its use is the
    // same on every path and the compiler's waits stay exact.
    auto fetch_next = [&](T (&pre)[P][C::NLOAD]) __attribute__((always_inline)) {
        const bool live = tf < t_end;
        const int np = live ? round_len(tf, rf) : P;
        const int tb = live ? tf : t_begin;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const __amdgpu_buffer_rsrc_t pl = buf(X + (i64)(u < np ? tb + u : tb) * M, plane_bytes);
#pragma unroll
            for (int j = 0; j < C::NLOAD; ++j) pre[u][j] = bload<T>(pl, goff[j]);
        }
        if (live) {
            tf += np;
            rf = rf + np == k0 ? 0 : rf + np;
        }
    };

    int qlast = qa - 1;
    int t = t_begin, q = qa, r0 = 0;
    // one round: NP planes (NP = P for whole blocks, else run-time np)
    auto round = [&](T (&pre)[P][C::NLOAD], int np) __attribute__((always_inline)) {
        // 1. stage this round's halo tiles; refill the register set two
        //    rounds ahead
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (u < np) {
#pragma unroll
                for (int j = 0; j < C::NLOAD; ++j) {
                    const int o = loff[j] == P * SA ? P * SA : u * SA + loff[j];
                    sA[o] = pre[u][j];
                }
            }
        }
        fetch_next(pre);
        __syncthreads();
        // 2. BDBS along x for every blocked halo row of every plane of the round
#pragma unroll
        for (int i = 0; i < C::RT; ++i) {
            const int pk = rp[i];
            if (pk >= 0 && (pk & 3) < np) {
                const int u = pk & 3, b = (pk >> 2) & 63, row = pk >> 8;
                bdbs_block<T, Op, KP, 1, 1>(sA + u * SA + row * C::PA + b * KP,
                                            sB + u * SB + row * C::PB + b * KP);
            }
        }
        __syncthreads();
        // 3. BDBS along y for every blocked column into the ring slots
#pragma unroll
        for (int i = 0; i < C::CT; ++i) {
            const int pk = cp[i];
            if (pk >= 0 && (pk & 3) < np) {
                const int u = pk & 3, b = (pk >> 2) & 63, col = pk >> 8;
                bdbs_block<T, Op, KP, C::PB, C::TXM>(sB + u * SB + b * KP * C::PB + col,
                                                      ring + (r0 + u) * NT + b * KP * C::TXM + col);
            }
        }
    };
    auto load_sx = [&]() __attribute__((always_inline)) {
        sx_valid = q < Qn;
        if (do_ex)
            sx_raw = bload<T>(buf((const T*)a.SX + (i64)(q < Qn ? q : Qn - 1) * M, plane_bytes), mb);
    };

    T pre0[P][C::NLOAD], pre1[P][C::NLOAD];
    fetch_next(pre0);
    fetch_next(pre1);
    __syncthreads();  // identity fill visible before the first staging
    if constexpr (WHOLE) {
        static_assert(K0B % (2 * P) == 0, "whole blocks take an even number of rounds");
        // blocks qa .. of the run, K0B / P full rounds each
        for (; t < t_end; ++q) {
            load_sx();
#pragma unroll
            for (int rr = 0; rr < K0B / P; rr += 2) {
                r0 = rr * P;
                round(pre0, P);
                r0 = (rr + 1) * P;
                round(pre1, P);
            }
            r0 = 0;
            t += K0B;
            block_step(q);
            qlast = q;
        }
    } else {
        auto step = [&](T (&pre)[P][C::NLOAD]) __attribute__((always_inline)) {
            const int np = round_len(t, r0);
            if (r0 == 0) load_sx();
            round(pre, np);
            // 4. a block of W planes is complete: emit the previous block
            const int tn = t + np;
            const int rn = r0 + np == k0 ? 0 : r0 + np;
            if (r0 + np == k0 || tn == n0) {
                if (r0 + np < k0) ring_fill_identity(r0 + np);  // the tensor ends inside the block
                block_step(q);
                qlast = q;
            }
            t = tn;
            if (rn == 0) ++q;
            r0 = rn;
        };
        while (t < t_end) {
            step(pre0);
            if (t >= t_end) break;
            step(pre1);
        }
    }
    // the block after the run lies past the tensor: emit the last block
    if (qlast < qb) {
        sx_valid = false;
        ring_fill_identity(0);
        block_step(qb);
    }
}

// ---------------------------------------------------------------------------
// 2-D BDBS of every plane of a (O, NY, NX) tensor over its two trailing axes
// (BDBS-Along-Dim along y and x, Sec. 5), with the same blocked LDS tiles as
// the streaming kernel: P planes per round, results staged through LDS so
// each thread stores its own point (coalesced rows).
// ---------------------------------------------------------------------------
struct Plane2Args {
    const void* X;
    void* W;
    i64 O, NY, NX;
    int ky, kx;
    i64 tilesY, tilesX;
};

template <typename T, class Op, int KP>
__global__ void __launch_bounds__(1024) k_plane_bdbs(Plane2Args a) {
    using C = PlaneCfg<KP>;
    constexpr int NT = C::NT, P = C::P, SA = C::SA, SB = C::SB;
    __shared__ T sA[P * SA + 1];
    __shared__ T sB[P * SB];
    __shared__ T sW[P * NT];

    const T e = Op::template id<T>();
    const int tid = threadIdx.x;
    i64 wg = blockIdx.x;
    const i64 nwg = (i64)gridDim.x;
    if ((nwg & 7) == 0) wg = (wg & 7) * (nwg >> 3) + (wg >> 3);
    const i64 tiles = a.tilesY * a.tilesX;
    const i64 tile = wg % tiles;
    const int grp = (int)(wg / tiles);  // which group of planes
    const int ky = a.ky, kx = a.kx;
    const int NY = (int)a.NY, NX = (int)a.NX;
    const int y0 = (int)(tile / a.tilesX) * (C::NBY * ky);
    const int x0 = (int)(tile % a.tilesX) * (C::NBX * kx);
    const unsigned plane_bytes = (unsigned)((i64)NY * NX * (i64)sizeof(T));

    const int pyb = tid / C::TXM, pxb = tid % C::TXM;
    const int py = (pyb / KP) * ky + pyb % KP, px = (pxb / KP) * kx + pxb % KP;
    const bool pvalid = pyb % KP < ky && pxb % KP < kx && y0 + py < NY && x0 + px < NX;
    const unsigned mb = pvalid ? (unsigned)((y0 + py) * NX + x0 + px) * sizeof(T) : plane_bytes;

    for (int i = tid; i < P * SA; i += NT) sA[i] = e;
    const int rows_in = C::NBY * ky + ky - 1, cols_in = C::NBX * kx + kx - 1;
    const int count = rows_in * cols_in;
    int loff[C::NLOAD];
    unsigned goff[C::NLOAD];
#pragma unroll
    for (int j = 0; j < C::NLOAD; ++j) {
        const int el = tid + j * NT;
        const int r = el / cols_in, c = el % cols_in;
        const bool inside = el < count && y0 + r < NY && x0 + c < NX;
        loff[j] = inside ? ((r / ky) * KP + r % ky) * C::PA + (c / kx) * KP + c % kx : P * SA;
        goff[j] = inside ? (unsigned)((y0 + r) * NX + x0 + c) * sizeof(T) : 0u;
    }
    constexpr int rt1 = C::ROWS * C::NBX, ct1 = C::TXM * C::NBY;
    int rp[C::RT], cp[C::CT];
#pragma unroll
    for (int i = 0; i < C::RT; ++i) {
        const int task = tid + i * NT;
        const int u = task / rt1, rem = task % rt1;
        rp[i] = task < P * rt1 ? (u | ((rem / C::ROWS) << 2) | ((rem % C::ROWS) << 8)) : -1;
    }
#pragma unroll
    for (int i = 0; i < C::CT; ++i) {
        const int task = tid + i * NT;
        const int u = task / ct1, rem = task % ct1;
        cp[i] = task < P * ct1 ? (u | ((rem / C::TXM) << 2) | ((rem % C::TXM) << 8)) : -1;
    }
    const T* __restrict__ X = (const T*)a.X;
    T* __restrict__ W = (T*)a.W;
    const i64 plane = (i64)NY * NX;
    __syncthreads();
    // each workgroup walks planes grp, grp + G, ... in rounds of P
    const i64 G = (i64)gridDim.x / tiles;
    for (i64 o0 = (i64)grp * P; o0 < a.O; o0 += G * P) {
        const int np = a.O - o0 < P ? (int)(a.O - o0) : P;
        T v[P][C::NLOAD];
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const __amdgpu_buffer_rsrc_t pl = buf(X + (o0 + (u < np ? u : 0)) * plane, plane_bytes);
#pragma unroll
            for (int j = 0; j < C::NLOAD; ++j) v[u][j] = bload<T>(pl, goff[j]);
        }
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (u < np) {
#pragma unroll
                for (int j = 0; j < C::NLOAD; ++j) {
                    const int o = loff[j] == P * SA ? P * SA : u * SA + loff[j];
                    sA[o] = v[u][j];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < C::RT; ++i) {
            const int pk = rp[i];
            if (pk >= 0 && (pk & 3) < np) {
                const int u = pk & 3, b = (pk >> 2) & 63, row = pk >> 8;
                bdbs_block<T, Op, KP, 1, 1>(sA + u * SA + row * C::PA + b * KP,
                                            sB + u * SB + row * C::PB + b * KP);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < C::CT; ++i) {
            const int pk = cp[i];
            if (pk >= 0 && (pk & 3) < np) {
                const int u = pk & 3, b = (pk >> 2) & 63, col = pk >> 8;
                bdbs_block<T, Op, KP, C::PB, C::TXM>(sB + u * SB + b * KP * C::PB + col,
                                                      sW + u * NT + b * KP * C::TXM + col);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < P; ++u)
            if (u < np) bstore<T>(buf(W + (o0 + u) * plane, plane_bytes), mb, sW[u * NT + tid]);
    }
}

// ---------------------------------------------------------------------------
// Block-level scans of the first dimension-reduction step in one pass: for
// every point m of a (Q, MID, NY, NX) tensor of block aggregates (already
// box-summed over the middle axes), box-sum each plane over its two trailing
// axes (BDBS-Along-Dim along y and x, Sec. 5) and scan the results along the
// block axis q without storing them:
//   PX[q, m] = op of Gw[q', m] for q' < q,  SX[q, m] = op of Gw[q', m] for q' > q,
//   R[m]     = op of Ga[q, m] over all q (the reduction that feeds the next level).
// One workgroup owns a tile for all Q <= QMAX planes (QMAX = 8 to 64); the
// box-summed values of its points stay in registers.
// ---------------------------------------------------------------------------
struct PlaneScanArgs {
    const void* G;   // (Q, MID, NY, NX)
    const void* Ga;  // (Q, M) un-box-summed aggregates (== G when MID has no axes)
    void* PX;
    void* SX;
    void* R;         // (M) or null
    void* A1;        // (ceil(NY / ky), NX): op of R over each ky-row block, or null (MID == 1)
    i64 Q, MID, NY, NX, M;
    int ky, kx;
    int pxe;         // PX is stored for blocks q with q % pxe == 0 only
    i64 tilesY, tilesX;
};

// FULL: exactly QMAX blocks and no middle axes (G == Ga), so every round is
// full and known at compile time: the loads' wait counts are exact.
// QMAX = 8 or 16 (short block axes: small tensors and their lower levels)
// with boxes up to 8 asks for two workgroups per CU (at most 64 VGPRs; the
// LDS fits twice), so that one workgroup's loads overlap the other's scans.
template <typename T, class Op, int KP, int QMAX, bool FULL>
__global__ void __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(QMAX <= 16 && KP <= 8 ? 8 : 1)))
k_plane_scan(PlaneScanArgs a) {
    using C = PlaneCfg<KP>;
    constexpr int NT = C::NT, P = C::P, SA = C::SA, SB = C::SB;
    static_assert(QMAX % (2 * P) == 0, "rounds come in pairs");
    __shared__ T sA[P * SA + 1];
    __shared__ T sB[P * SB];
    __shared__ T sW[P * NT];

    const T e = Op::template id<T>();
    const int tid = threadIdx.x;
    i64 wg = blockIdx.x;
    const i64 nwg = (i64)gridDim.x;
    if ((nwg & 7) == 0) wg = (wg & 7) * (nwg >> 3) + (wg >> 3);
    const i64 tiles = a.tilesY * a.tilesX;
    const i64 tile = wg % tiles;
    const int mid = (int)(wg / tiles);
    const int ky = a.ky, kx = a.kx;
    const int NY = (int)a.NY, NX = (int)a.NX;
    const int Q = FULL ? QMAX : (int)a.Q;
    const int y0 = (int)(tile / a.tilesX) * (C::NBY * ky);
    const int x0 = (int)(tile % a.tilesX) * (C::NBX * kx);
    const i64 plane = (i64)NY * NX;
    const unsigned plane_bytes = (unsigned)(plane * (i64)sizeof(T));
    const bool same = FULL || a.G == a.Ga;

    const int pyb = tid / C::TXM, pxb = tid % C::TXM;
    const int py = (pyb / KP) * ky + pyb % KP, px = (pxb / KP) * kx + pxb % KP;
    const bool pvalid = pyb % KP < ky && pxb % KP < kx && y0 + py < NY && x0 + px < NX;
    const unsigned mb = pvalid ? (unsigned)((y0 + py) * NX + x0 + px) * sizeof(T) : plane_bytes;
    // the point's slot in the staged halo tile (its own, unfiltered value)
    const int own = pyb * C::PA + pxb;

    for (int i = tid; i < P * SA; i += NT) sA[i] = e;
    const int rows_in = C::NBY * ky + ky - 1, cols_in = C::NBX * kx + kx - 1;
    const int count = rows_in * cols_in;
    int loff[C::NLOAD];
    unsigned goff[C::NLOAD];
#pragma unroll
    for (int j = 0; j < C::NLOAD; ++j) {
        const int el = tid + j * NT;
        const int r = el / cols_in, c = el % cols_in;
        const bool inside = el < count && y0 + r < NY && x0 + c < NX;
        loff[j] = inside ? ((r / ky) * KP + r % ky) * C::PA + (c / kx) * KP + c % kx : P * SA;
        goff[j] = inside ? (unsigned)((y0 + r) * NX + x0 + c) * sizeof(T) : 0u;
    }
    constexpr int rt1 = C::ROWS * C::NBX, ct1 = C::TXM * C::NBY;
    int rp[C::RT], cp[C::CT];
#pragma unroll
    for (int i = 0; i < C::RT; ++i) {
        const int task = tid + i * NT;
        const int u = task / rt1, rem = task % rt1;
        rp[i] = task < P * rt1 ? (u | ((rem / C::ROWS) << 2) | ((rem % C::ROWS) << 8)) : -1;
    }
#pragma unroll
    for (int i = 0; i < C::CT; ++i) {
        const int task = tid + i * NT;
        const int u = task / ct1, rem = task % ct1;
        cp[i] = task < P * ct1 ? (u | ((rem / C::TXM) << 2) | ((rem % C::TXM) << 8)) : -1;
    }
    const T* __restrict__ G = (const T*)a.G;
    const T* __restrict__ Ga = (const T*)a.Ga;
    // plane (q, mid) of G; rounds past Q re-read plane 0 (never staged)
    auto fetch = [&](T (&pre)[P][C::NLOAD], int q0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int q = q0 + u < Q ? q0 + u : 0;
            const __amdgpu_buffer_rsrc_t pl = buf(G + ((i64)q * a.MID + mid) * plane, plane_bytes);
#pragma unroll
            for (int j = 0; j < C::NLOAD; ++j) pre[u][j] = bload<T>(pl, goff[j]);
        }
    };
    T gw[QMAX];
    T Rm = e;
    auto round = [&](T (&pre)[P][C::NLOAD], int q0) __attribute__((always_inline)) {
        const int np = Q - q0 < P ? Q - q0 : P;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (u < np) {
#pragma unroll
                for (int j = 0; j < C::NLOAD; ++j) {
                    const int o = loff[j] == P * SA ? P * SA : u * SA + loff[j];
                    sA[o] = pre[u][j];
                }
            }
        }
        if (q0 + 2 * P < Q) fetch(pre, q0 + 2 * P);
        __syncthreads();
        // the reduction over blocks: the point's own aggregate
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (u < np) {
                const T g = same ? sA[u * SA + own]
                                 : bload<T>(buf(Ga + (i64)(q0 + u) * a.M + (i64)mid * plane,
                                                plane_bytes), mb);
                Rm = Op::apply(Rm, g);
            }
        }
#pragma unroll
        for (int i = 0; i < C::RT; ++i) {
            const int pk = rp[i];
            if (pk >= 0 && (pk & 3) < np) {
                const int u = pk & 3, b = (pk >> 2) & 63, row = pk >> 8;
                bdbs_block<T, Op, KP, 1, 1>(sA + u * SA + row * C::PA + b * KP,
                                            sB + u * SB + row * C::PB + b * KP);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < C::CT; ++i) {
            const int pk = cp[i];
            if (pk >= 0 && (pk & 3) < np) {
                const int u = pk & 3, b = (pk >> 2) & 63, col = pk >> 8;
                bdbs_block<T, Op, KP, C::PB, C::TXM>(sB + u * SB + b * KP * C::PB + col,
                                                      sW + u * NT + b * KP * C::TXM + col);
            }
        }
        __syncthreads();
    };
    T pre0[P][C::NLOAD], pre1[P][C::NLOAD];
    fetch(pre0, 0);
    if (P < Q) fetch(pre1, P);
    __syncthreads();
#pragma unroll
    for (int q0 = 0; q0 < QMAX; q0 += 2 * P) {
        if (q0 < Q) {
            round(pre0, q0);
#pragma unroll
            for (int u = 0; u < P; ++u) gw[q0 + u] = q0 + u < Q ? sW[u * NT + tid] : e;
        }
        if (q0 + P < Q) {
            round(pre1, q0 + P);
#pragma unroll
            for (int u = 0; u < P; ++u) gw[q0 + P + u] = q0 + P + u < Q ? sW[u * NT + tid] : e;
        }
    }
    if (a.A1) {
        // the next level's block aggregates: R (the reduction over axis 0)
        // reduced over each ky-row block of the tile; the tile holds whole
        // blocks, and invalid slots hold the identity
        __syncthreads();
        sW[tid] = pvalid ? Rm : e;
        __syncthreads();
        if (tid < C::NBY * C::TXM) {
            const int b = tid / C::TXM, c = tid % C::TXM;
            const int cx = (c / KP) * kx + c % KP;
            T g = e;
            for (int r = 0; r < ky; ++r) g = Op::apply(g, sW[(b * KP + r) * C::TXM + c]);
            if (c % KP < kx && x0 + cx < NX && y0 + b * ky < NY)
                ((T*)a.A1)[(i64)(y0 / ky + b) * NX + x0 + cx] = g;
        }
    }
    if (!pvalid) return;
    const i64 m = (i64)mid * plane + (i64)(y0 + py) * NX + x0 + px;
    T* __restrict__ PX = (T*)a.PX;
    T* __restrict__ SX = (T*)a.SX;
    T pfx = e;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        if (q < Q) {
            if (q % a.pxe == 0) PX[(i64)q * a.M + m] = pfx;
            pfx = Op::apply(pfx, gw[q]);
        }
    }
    T sfx = e;
#pragma unroll
    for (int q = QMAX - 1; q >= 0; --q) {
        if (q < Q) {
            SX[(i64)q * a.M + m] = sfx;
            sfx = Op::apply(gw[q], sfx);
        }
    }
    if (a.R) ((T*)a.R)[m] = Rm;
}

template <typename T, class Op, int KP>
void launch_plane_scan_kp(PlaneScanArgs pa, hipStream_t st) {
    using C = PlaneCfg<KP>;
    const i64 ty = (i64)C::NBY * pa.ky, tx = (i64)C::NBX * pa.kx;
    pa.tilesY = (pa.NY + ty - 1) / ty;
    pa.tilesX = (pa.NX + tx - 1) / tx;
    const i64 grid = pa.tilesY * pa.tilesX * pa.MID;
    if (pa.Q == 32 && pa.G == pa.Ga)
        hipLaunchKernelGGL((k_plane_scan<T, Op, KP, 32, true>), dim3((unsigned)grid), dim3(C::NT),
                           0, st, pa);
    else if (pa.Q <= 8)
        hipLaunchKernelGGL((k_plane_scan<T, Op, KP, 8, false>), dim3((unsigned)grid),
                           dim3(C::NT), 0, st, pa);
    else if (pa.Q <= 16)
        hipLaunchKernelGGL((k_plane_scan<T, Op, KP, 16, false>), dim3((unsigned)grid),
                           dim3(C::NT), 0, st, pa);
    else if (pa.Q <= 32)
        hipLaunchKernelGGL((k_plane_scan<T, Op, KP, 32, false>), dim3((unsigned)grid),
                           dim3(C::NT), 0, st, pa);
    else
        hipLaunchKernelGGL((k_plane_scan<T, Op, KP, 64, false>), dim3((unsigned)grid),
                           dim3(C::NT), 0, st, pa);
}

template <typename T, class Op>
void launch_plane_scan(const T* G, const T* Ga, T* PX, T* SX, T* R, T* A1, i64 Q, i64 MID,
                       i64 NY, i64 NX, i64 ky, i64 kx, i64 pxe, hipStream_t st) {
    KTimer timer("k_plane_scan", st);
    PlaneScanArgs pa{};
    pa.G = G; pa.Ga = Ga; pa.PX = PX; pa.SX = SX; pa.R = R; pa.A1 = MID == 1 ? A1 : nullptr;
    pa.Q = Q; pa.MID = MID; pa.NY = NY; pa.NX = NX; pa.M = MID * NY * NX;
    pa.ky = (int)ky; pa.kx = (int)kx; pa.pxe = (int)pxe;
    const i64 km = ky > kx ? ky : kx;
    if (km <= 2) launch_plane_scan_kp<T, Op, 2>(pa, st);
    else if (km <= 4) launch_plane_scan_kp<T, Op, 4>(pa, st);
    else if (km <= 8) launch_plane_scan_kp<T, Op, 8>(pa, st);
    else launch_plane_scan_kp<T, Op, 16>(pa, st);
}

template <typename T, class Op, int KP>
void launch_plane_bdbs_kp(Plane2Args pa, hipStream_t st) {
    using C = PlaneCfg<KP>;
    const i64 ty = (i64)C::NBY * pa.ky, tx = (i64)C::NBX * pa.kx;
    pa.tilesY = (pa.NY + ty - 1) / ty;
    pa.tilesX = (pa.NX + tx - 1) / tx;
    const i64 tiles = pa.tilesY * pa.tilesX;
    // plane groups so that the grid covers the CUs (each group: P planes per round)
    i64 groups = (512 + tiles - 1) / tiles;
    const i64 maxg = (pa.O + C::P - 1) / C::P;
    if (groups > maxg) groups = maxg;
    if (groups < 1) groups = 1;
    hipLaunchKernelGGL((k_plane_bdbs<T, Op, KP>), dim3((unsigned)(tiles * groups)), dim3(C::NT),
                       0, st, pa);
}

template <typename T, class Op>
void launch_plane_bdbs(const T* X, T* W, i64 O, i64 NY, i64 NX, i64 ky, i64 kx, hipStream_t st) {
    KTimer timer("k_plane_bdbs", st);
    Plane2Args pa{};
    pa.X = X; pa.W = W; pa.O = O; pa.NY = NY; pa.NX = NX; pa.ky = (int)ky; pa.kx = (int)kx;
    const i64 km = ky > kx ? ky : kx;
    if (km <= 2) launch_plane_bdbs_kp<T, Op, 2>(pa, st);
    else if (km <= 4) launch_plane_bdbs_kp<T, Op, 4>(pa, st);
    else if (km <= 8) launch_plane_bdbs_kp<T, Op, 8>(pa, st);
    else launch_plane_bdbs_kp<T, Op, 16>(pa, st);
}

template <typename T, class Op, int K0B, int KP, bool WEAK>
void launch_plane_kernel(PlaneArgs pa, hipStream_t st) {
    using C = PlaneCfg<KP>;
    const i64 ty = (i64)C::NBY * pa.ky, tx = (i64)C::NBX * pa.kx;
    pa.tilesY = (pa.NY + ty - 1) / ty;
    pa.tilesX = (pa.NX + tx - 1) / tx;
    const i64 tiles = pa.tilesY * pa.tilesX * pa.MID;
    pa.segblocks = plane_run_blocks(pa.Q, tiles);
    pa.nseg = (pa.Q + pa.segblocks - 1) / pa.segblocks;
    const i64 grid = tiles * pa.nseg;
    // whole blocks: every block of every run has exactly K0B planes
    if constexpr (K0B % (2 * C::P) == 0) {
        if (pa.k0 == K0B && pa.n0 % K0B == 0) {
            hipLaunchKernelGGL((k_plane_axis0<T, Op, K0B, KP, true, WEAK>), dim3((unsigned)grid),
                               dim3(C::NT), 0, st, pa);
            return;
        }
    }
    hipLaunchKernelGGL((k_plane_axis0<T, Op, K0B, KP, false, WEAK>), dim3((unsigned)grid),
                       dim3(C::NT), 0, st, pa);
}

template <typename T, class Op, int K0B, bool WEAK>
void launch_plane_kp(PlaneArgs pa, hipStream_t st) {
    const int km = pa.ky > pa.kx ? pa.ky : pa.kx;
    if (km <= 2) launch_plane_kernel<T, Op, K0B, 2, WEAK>(pa, st);
    else if (km <= 4) launch_plane_kernel<T, Op, K0B, 4, WEAK>(pa, st);
    else if (km <= 8) launch_plane_kernel<T, Op, K0B, 8, WEAK>(pa, st);
    else launch_plane_kernel<T, Op, K0B, 16, WEAK>(pa, st);
}

template <typename T, class Op, bool WEAK>
void launch_plane_k0(PlaneArgs pa, hipStream_t st) {
    if (pa.k0 <= 4) launch_plane_kp<T, Op, 4, WEAK>(pa, st);
    else if (pa.k0 <= 8) launch_plane_kp<T, Op, 8, WEAK>(pa, st);
    else launch_plane_kp<T, Op, 16, WEAK>(pa, st);
}

template <typename T, class Op>
void launch_plane_axis0(const T* X, const T* PX, const T* SX, const T* Trest, T* exc, T* inc,
                        i64 n0, i64 MID, i64 NY, i64 NX, i64 k0, i64 ky, i64 kx, i64 Q,
                        hipStream_t st) {
    KTimer timer("k_plane_axis0", st);
    PlaneArgs pa{};
    pa.X = X; pa.PX = PX; pa.SX = SX; pa.Trest = Trest; pa.exc = exc; pa.inc = inc;
    pa.n0 = n0; pa.MID = MID; pa.NY = NY; pa.NX = NX; pa.M = MID * NY * NX; pa.Q = Q;
    pa.k0 = (int)k0; pa.ky = (int)ky; pa.kx = (int)kx;
    pa.nt = store_hint_ok(NX * (i64)sizeof(T));
    launch_plane_k0<T, Op, false>(pa, st);
}

// Included sums (into inc, or nowhere) and weak excluded sums total - included
// (into wexc), + only.
template <typename T, class Op>
void launch_plane_weak(const T* X, T* inc, const T* wtot, T* wexc, i64 n0, i64 MID, i64 NY,
                       i64 NX, i64 k0, i64 ky, i64 kx, hipStream_t st) {
    KTimer timer("k_plane_axis0", st);
    PlaneArgs pa{};
    pa.X = X; pa.inc = inc; pa.wtot = wtot; pa.wexc = wexc;
    pa.n0 = n0; pa.MID = MID; pa.NY = NY; pa.NX = NX; pa.M = MID * NY * NX;
    pa.Q = (n0 + k0 - 1) / k0;
    pa.k0 = (int)k0; pa.ky = (int)ky; pa.kx = (int)kx;
    pa.nt = store_hint_ok(NX * (i64)sizeof(T));
    launch_plane_k0<T, Op, true>(pa, st);
}

}  // namespace exs
