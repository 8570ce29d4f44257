// exsum_plane.hip -- fused streaming kernel for the first dimension-reduction
// step of included/excluded sums on gfx950.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// For a rank >= 3 tensor viewed as (n0, MID, NY, NX) -- MID collects the
// middle axes, already box-summed -- one workgroup owns a TY x TX tile of the
// (NY, NX) plane for a run of k0-blocks of axis 0, and walks axis 0 plane by
// plane:
//   1. the tile plus its (ky-1, kx-1) halo is loaded into LDS (coalesced rows);
//   2. BDBS along x (range suffix and range prefix of kx-blocks, then the
//      combine of Sec. 3) over every row of the halo tile, into LDS;
//   3. BDBS along y over every column, into a ring of k0 planes in LDS:
//      W = the plane box-summed over its two axes ("BDBS-Along-Dim", Sec. 5);
//   4. once a k0-block of W planes is in the ring, each thread (one point of
//      the tile) updates its axis-0 state in registers and emits the previous
//      block: the excluded sum (prefix before x0, suffix from x0+k0, the
//      lower-dimensional contribution) and the included sum (BDBS along
//      axis 0).
// The input is read once from HBM (halo re-reads are meant to hit L2: the
// workgroups of one XCD own a contiguous band of tiles), and each output is
// written once.
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
    i64 n0, MID, NY, NX, M, Q;
    int k0, ky, kx, TY, TX;
    i64 tilesY, tilesX, segblocks, nseg;
};

// Workgroup geometry: one thread per point of a 32 x 32 tile; P planes are
// box-summed per round so that every wave has scan work between barriers.
struct PlaneCfg {
    static constexpr int NT = 1024;
    static constexpr int TYM = 32, TXM = 32;
    static constexpr int KPM = 16;               // largest ky, kx
    static constexpr int ROWS = TYM + KPM - 1;   // max halo rows
    static constexpr int COLS = TXM + KPM - 1;   // max halo cols
    static constexpr int PA = (COLS | 1);        // LDS pitch of the input tile (odd)
    static constexpr int PB = TXM + 1;           // LDS pitch of the row-pass output (odd)
    static constexpr int NLOAD = (ROWS * COLS + NT - 1) / NT;
    static constexpr int P = 4;                  // planes per round
};

// One BDBS block of a plane pass: out[r] = rsuf_b[r] op rpre_{b+1}[r-1] for
// r < k (out[0] = rsuf_b[0]), with src[0..k) the block and src[k..2k-1) the
// next block, strided by SS in LDS.  KP >= k is a compile-time bound: the
// loads are unconditional (every address stays inside the LDS tile) and, when
// k < KP, lanes past k are replaced by the identity, so the scan has no
// branches.
template <typename T, class Op, int KP, int SS, int DS>
__device__ __forceinline__ void bdbs_block_lds(const T* __restrict__ src, T* __restrict__ dst,
                                               int k) {
    const T e = Op::template id<T>();
    T a0[KP], a1[KP];
    if (k == KP) {
#pragma unroll
        for (int r = 0; r < KP; ++r) {
            a0[r] = src[r * SS];
            if (r < KP - 1) a1[r] = src[(KP + r) * SS];
        }
    } else {
#pragma unroll
        for (int r = 0; r < KP; ++r) {
            const T v0 = src[r * SS];
            a0[r] = r < k ? v0 : e;
            if (r < KP - 1) {
                const T v1 = src[(k + r) * SS];
                a1[r] = r < k - 1 ? v1 : e;
            }
        }
    }
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
    for (int r = 0; r < KP; ++r)
        if (r < k) dst[r * DS] = a0[r];
}

// Raw buffer access: a resource descriptor (uniform 64-bit base and byte
// range, held in SGPRs) plus a per-thread 32-bit byte offset.  Accesses past
// the range read 0 and drop stores.  Word 3 = 0x00020000 is the gfx9-family
// raw-buffer format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned voff) {
    static_assert(sizeof(T) == 4, "4-byte elements");
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}
template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned voff, T v) {
    static_assert(sizeof(T) == 4, "4-byte elements");
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, 0, 0);
}

template <typename T, class Op, int K0B, int KP>
__global__ void __launch_bounds__(1024) k_plane_axis0(PlaneArgs a) {
    using C = PlaneCfg;
    constexpr int NT = C::NT, P = C::P;
    constexpr int SA = C::ROWS * C::PA, SB = C::ROWS * C::PB;
    __shared__ T sA[P * SA];
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
    const i64 mid = rest % a.MID;
    const i64 s = rest / a.MID;
    const int y0 = (int)((tile / a.tilesX) * a.TY);
    const int x0 = (int)((tile % a.tilesX) * a.TX);
    const i64 qa = s * a.segblocks;
    const i64 qb = qa + a.segblocks < a.Q ? qa + a.segblocks : a.Q;
    const int k0 = a.k0, ky = a.ky, kx = a.kx, TY = a.TY, TX = a.TX;
    const int NY = (int)a.NY, NX = (int)a.NX;
    const i64 M = a.M;
    const i64 n0 = a.n0;

    // this thread's point of the tile; per-thread offsets are 32-bit byte
    // offsets within a plane, the per-plane bases are uniform
    const int py = tid / C::TXM, px = tid % C::TXM;
    const bool pvalid = py < TY && px < TX && y0 + py < NY && x0 + px < NX;
    const unsigned mb = ((unsigned)(mid * NY * NX) + (unsigned)((y0 + py) * NX + x0 + px)) *
                        (unsigned)sizeof(T);

    // halo-tile load plan, identical for every plane: elements outside the
    // tensor read a valid address and are replaced by the identity
    const int rows_in = TY + ky - 1, cols_in = TX + kx - 1;
    const int count = rows_in * cols_in;
    int loff[C::NLOAD];
    unsigned goff[C::NLOAD];
    bool gin[C::NLOAD];
#pragma unroll
    for (int j = 0; j < C::NLOAD; ++j) {
        const int el = tid + j * NT;
        const int r = el / cols_in, c = el % cols_in;
        gin[j] = el < count && y0 + r < NY && x0 + c < NX;
        loff[j] = el < count ? r * C::PA + c : -1;
        goff[j] = gin[j] ? ((unsigned)(mid * NY * NX) + (unsigned)((y0 + r) * NX + x0 + c)) *
                               (unsigned)sizeof(T)
                         : 0u;
    }

    // scan tasks of a full round: row task (u, b, row), column task (u, b,
    // col), flattened with u outermost so a round of np < P planes runs the
    // tasks whose u < np.  The first two of each thread are decoded once and
    // packed as u | b << 2 | idx << 8; any further ones (small boxes only)
    // are decoded per round.  -1 marks no task.
    const int nbx = TX / kx, nby = TY / ky;
    const int rt1 = rows_in * nbx, ct1 = TX * nby;
    const int rtot = P * rt1, ctot = P * ct1;
    auto dec_row = [&](int task) -> int {
        const int u = task / rt1, rem = task - u * rt1;
        const int b = rem / rows_in, row = rem - b * rows_in;
        return u | (b << 2) | (row << 8);
    };
    auto dec_col = [&](int task) -> int {
        const int u = task / ct1, rem = task - u * ct1;
        const int b = rem / TX, col = rem - b * TX;
        return u | (b << 2) | (col << 8);
    };
    const int rp0 = tid < rtot ? dec_row(tid) : -1, rp1 = tid + NT < rtot ? dec_row(tid + NT) : -1;
    const int cp0 = tid < ctot ? dec_col(tid) : -1, cp1 = tid + NT < ctot ? dec_col(tid + NT) : -1;
    auto run_row = [&](int pk, int np) {
        if (pk < 0) return;
        const int u = pk & 3;
        if (u >= np) return;
        const int b = (pk >> 2) & 63, row = pk >> 8;
        bdbs_block_lds<T, Op, KP, 1, 1>(sA + u * SA + row * C::PA + b * kx,
                                        sB + u * SB + row * C::PB + b * kx, kx);
    };
    auto run_col = [&](int pk, int np, int r0) {
        if (pk < 0) return;
        const int u = pk & 3;
        if (u >= np) return;
        const int b = (pk >> 2) & 63, col = pk >> 8;
        bdbs_block_lds<T, Op, KP, C::PB, C::TXM>(sB + u * SB + b * ky * C::PB + col,
                                                  ring + (r0 + u) * NT + b * ky * C::TXM + col,
                                                  ky);
    };

    const T* __restrict__ X = (const T*)a.X;
    const i64 t_begin = qa * k0;
    i64 t_end = (qb + 1) * k0;  // one block past the run: the suffix/inclusion lag
    if (t_end > n0) t_end = n0;

    const bool do_ex = a.exc != nullptr, do_inc = a.inc != nullptr;
    T* __restrict__ exc = (T*)a.exc;
    T* __restrict__ inc = (T*)a.inc;

    const unsigned plane_bytes = (unsigned)(M * (i64)sizeof(T));
    Axis0State<T, Op, K0B> st;
    st.P = e;
    if (do_ex && pvalid) {
        st.P = bload<T>(buf((const T*)a.PX + qa * M, plane_bytes), mb);
        if (a.Trest) st.P = Op::apply(st.P, bload<T>(buf(a.Trest, plane_bytes), mb));
    }
    // SX of the block being filled, loaded when the block starts (from an
    // in-range block index; blocks past the last one use the identity at the
    // point of use, so the register is never overwritten while in flight)
    T sx_raw = e;
    bool sx_valid = false;

    // Emit block (q-1) from the ring holding block q, then absorb block q.
    auto block_step = [&](i64 q) __attribute__((always_inline)) {
        __syncthreads();
        T v[K0B];
#pragma unroll
        for (int r = 0; r < K0B; ++r)
            v[r] = (r < k0 && q * k0 + r < n0) ? ring[r * NT + tid] : e;
        if (q == qa) {
            st.absorb(v, k0, do_ex, do_inc);
            return;
        }
        const i64 xb = (q - 1) * k0;
        if (pvalid) {
            if (do_ex) {
                T S = sx_valid ? sx_raw : e;
#pragma unroll
                for (int r = K0B - 1; r >= 0; --r) {
                    if (r < k0) {
                        S = Op::apply(v[r], S);
                        if (xb + r < n0)
                            bstore<T>(buf(exc + (xb + r) * M, plane_bytes), mb,
                                      Op::apply(st.pex[r], S));
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
                        if (xb + r < n0) bstore<T>(buf(inc + (xb + r) * M, plane_bytes), mb, val);
                    }
                }
            }
        }
        if (q < qb) st.absorb(v, k0, do_ex, do_inc);
    };

    // raw prefetched values; the identity for elements outside the tensor is
    // applied when they are staged, so no load is consumed early
    T pre[P][C::NLOAD];
    auto fetch_round = [&](i64 t, int np) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const __amdgpu_buffer_rsrc_t pl = buf(X + (u < np ? t + u : t) * M, plane_bytes);
#pragma unroll
            for (int j = 0; j < C::NLOAD; ++j) pre[u][j] = bload<T>(pl, goff[j]);
        }
    };

    // rounds of up to P planes that stay inside one k0-block
    i64 qlast = qa - 1;
    i64 t = t_begin;
    i64 q = qa;   // block of plane t
    int r0 = 0;   // position of plane t in its block
    auto round_len = [&](i64 tt, int rr) -> int {
        i64 n = (i64)(k0 - rr);
        if (tt + n > t_end) n = t_end - tt;
        return (int)(n < P ? n : P);
    };
    int np = t < t_end ? round_len(t, 0) : 0;
    if (np > 0) fetch_round(t, np);
    while (t < t_end) {
        if (r0 == 0) {
            sx_valid = q < a.Q;
            if (do_ex)
                sx_raw = bload<T>(buf((const T*)a.SX + (q < a.Q ? q : a.Q - 1) * M, plane_bytes),
                                  mb);
        }
        // 1. stage this round's halo tiles; start loading the next round
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (u < np) {
#pragma unroll
                for (int j = 0; j < C::NLOAD; ++j)
                    if (loff[j] >= 0) sA[u * SA + loff[j]] = gin[j] ? pre[u][j] : e;
            }
        }
        const i64 tn = t + np;
        const int rn = r0 + np == k0 ? 0 : r0 + np;
        const int npn = tn < t_end ? round_len(tn, rn) : 0;
        if (npn > 0) fetch_round(tn, npn);
        __syncthreads();
        // 2. BDBS along x for every halo row of every plane of the round
        run_row(rp0, np);
        run_row(rp1, np);
        for (int task = tid + 2 * NT; task < rtot; task += NT) run_row(dec_row(task), np);
        __syncthreads();
        // 3. BDBS along y for every column into the ring slots of the round
        run_col(cp0, np, r0);
        run_col(cp1, np, r0);
        for (int task = tid + 2 * NT; task < ctot; task += NT) run_col(dec_col(task), np, r0);
        // 4. a block of W planes is complete: emit the previous block
        if (r0 + np == k0 || t + np == n0) {
            block_step(q);
            qlast = q;
        }
        t = tn;
        if (rn == 0) ++q;
        r0 = rn;
        np = npn;
    }
    // the block after the run lies past the tensor: emit the last block
    if (qlast < qb) {
        sx_valid = false;
        block_step(qb);
    }
}

bool plane_eligible(int d, const i64* n, const i64* k, int es) {
    if (d < 3 || es != 4) return false;
    if (k[0] > 16) return false;
    if (k[d - 2] > PlaneCfg::KPM || k[d - 1] > PlaneCfg::KPM) return false;
    // plane offsets are 32-bit inside the kernel
    if (n[d - 2] * n[d - 1] >= ((i64)1 << 31)) return false;
    // per-point byte offsets within a plane of the (middle x plane) space are 32-bit
    i64 M = 1;
    for (int i = 1; i < d; ++i) M *= n[i];
    if (M * es >= ((i64)1 << 32)) return false;
    return true;
}

template <typename T, class Op, int K0B, int KP>
static void launch_plane_kb(PlaneArgs pa, hipStream_t st) {
    using C = PlaneCfg;
    pa.TY = (int)(C::TYM / pa.ky * pa.ky);
    pa.TX = (int)(C::TXM / pa.kx * pa.kx);
    pa.tilesY = (pa.NY + pa.TY - 1) / pa.TY;
    pa.tilesX = (pa.NX + pa.TX - 1) / pa.TX;
    const i64 tiles = pa.tilesY * pa.tilesX * pa.MID;
    // enough workgroups to cover every CU; each run of blocks reads one
    // extra block of planes
    i64 nseg = (256 + tiles - 1) / tiles;
    if (nseg > pa.Q) nseg = pa.Q;
    if (nseg < 1) nseg = 1;
    pa.segblocks = (pa.Q + nseg - 1) / nseg;
    pa.nseg = (pa.Q + pa.segblocks - 1) / pa.segblocks;
    const i64 grid = tiles * pa.nseg;
    hipLaunchKernelGGL((k_plane_axis0<T, Op, K0B, KP>), dim3((unsigned)grid), dim3(C::NT), 0, st,
                       pa);
}

template <typename T, class Op, int K0B>
static void launch_plane_kp(PlaneArgs pa, hipStream_t st) {
    if (pa.ky <= 8 && pa.kx <= 8) launch_plane_kb<T, Op, K0B, 8>(pa, st);
    else launch_plane_kb<T, Op, K0B, 16>(pa, st);
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
    if (k0 <= 4) launch_plane_kp<T, Op, 4>(pa, st);
    else if (k0 <= 8) launch_plane_kp<T, Op, 8>(pa, st);
    else launch_plane_kp<T, Op, 16>(pa, st);
}

#define EXS_INST_PLANE(T, OP)                                                                  \
    template void launch_plane_axis0<T, OP>(const T*, const T*, const T*, const T*, T*, T*,    \
                                            i64, i64, i64, i64, i64, i64, i64, i64, hipStream_t);
EXS_INST_PLANE(float, OpSum)
EXS_INST_PLANE(int, OpSum)
EXS_INST_PLANE(float, OpMax)
EXS_INST_PLANE(int, OpMax)

}  // namespace exs
