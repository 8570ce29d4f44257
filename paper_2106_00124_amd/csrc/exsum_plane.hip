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

template <int K0B, int ES>
struct PlaneCfg {
    // points (= threads) per workgroup so that the k0-ring of W planes stays
    // within 64 KB of LDS (128 KB for the widest case)
    static constexpr int NT = (K0B * ES <= 64) ? 1024 : (K0B * ES <= 128) ? 512 : 256;
    static constexpr int TYM = NT == 1024 ? 32 : 16;
    static constexpr int TXM = NT == 256 ? 16 : 32;
    static constexpr int ROWS = 2 * TYM - 1;     // max halo rows
    static constexpr int COLS = 2 * TXM - 1;     // max halo cols
    static constexpr int PA = 2 * TXM + 1;       // LDS pitch of the input tile (odd)
    static constexpr int PB = TXM + 1;           // LDS pitch of the row-pass output (odd)
    static constexpr int NLOAD = (ROWS * COLS + NT - 1) / NT;
};

template <typename T, class Op, int K0B>
__global__ void __launch_bounds__((PlaneCfg<K0B, sizeof(T)>::NT))
k_plane_axis0(PlaneArgs a) {
    using C = PlaneCfg<K0B, sizeof(T)>;
    constexpr int NT = C::NT;
    __shared__ T sA[C::ROWS * C::PA];
    __shared__ T sB[C::ROWS * C::PB];
    __shared__ T ring[K0B * NT];

    const T e = Op::template id<T>();
    const int tid = threadIdx.x;
    const T* __restrict__ X = (const T*)a.X;

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
    const i64 y0 = (tile / a.tilesX) * a.TY;
    const i64 x0 = (tile % a.tilesX) * a.TX;
    const i64 qa = s * a.segblocks;
    const i64 qb = qa + a.segblocks < a.Q ? qa + a.segblocks : a.Q;
    const int k0 = a.k0, ky = a.ky, kx = a.kx;
    const i64 M = a.M;

    // this thread's point of the tile
    const int py = tid / C::TXM, px = tid % C::TXM;
    const bool pvalid = py < a.TY && px < a.TX && y0 + py < a.NY && x0 + px < a.NX;
    const i64 m = (mid * a.NY + y0 + py) * a.NX + x0 + px;

    // halo-tile load plan (identical for every plane)
    const int rows_in = a.TY + ky - 1, cols_in = a.TX + kx - 1;
    const int count = rows_in * cols_in;
    int loff[C::NLOAD];
    i64 goff[C::NLOAD];
    bool gval[C::NLOAD];
#pragma unroll
    for (int j = 0; j < C::NLOAD; ++j) {
        const int el = tid + j * NT;
        const int r = el / cols_in, c = el % cols_in;
        loff[j] = el < count ? r * C::PA + c : -1;
        gval[j] = el < count && y0 + r < a.NY && x0 + c < a.NX;
        goff[j] = (mid * a.NY + y0 + r) * a.NX + x0 + c;
    }
    const i64 plane_stride = a.MID * a.NY * a.NX;

    T pre[C::NLOAD];
    auto fetch = [&](i64 t) {
        const T* src = X + t * plane_stride;
#pragma unroll
        for (int j = 0; j < C::NLOAD; ++j) pre[j] = gval[j] ? src[goff[j]] : e;
    };

    const i64 t_begin = qa * k0;
    i64 t_end = (qb + 1) * k0;  // one block past the run: the suffix/inclusion lag
    if (t_end > a.n0) t_end = a.n0;

    const bool do_ex = a.exc != nullptr, do_inc = a.inc != nullptr;
    T* __restrict__ exc = (T*)a.exc;
    T* __restrict__ inc = (T*)a.inc;
    const T* __restrict__ PX = (const T*)a.PX;
    const T* __restrict__ SX = (const T*)a.SX;
    const T* __restrict__ Trest = (const T*)a.Trest;

    Axis0State<T, Op, K0B> st;
    st.P = e;
    if (do_ex && pvalid) {
        st.P = PX[qa * M + m];
        if (Trest) st.P = Op::apply(st.P, Trest[m]);
    }
    T sx_next = e;  // SX of the block being filled

    // Emit block (q-1) from the ring holding block q, then absorb block q.
    auto block_step = [&](i64 q) {
        __syncthreads();
        T v[K0B];
#pragma unroll
        for (int r = 0; r < K0B; ++r)
            v[r] = (r < k0 && q * k0 + r < a.n0) ? ring[r * NT + tid] : e;
        if (q == qa) {
            st.absorb(v, k0, do_ex, do_inc);
            return;
        }
        const i64 qe = q - 1;
        if (pvalid) {
            if (do_ex) {
                T S = sx_next;
#pragma unroll
                for (int r = K0B - 1; r >= 0; --r) {
                    if (r < k0) {
                        S = Op::apply(v[r], S);
                        const i64 x = qe * k0 + r;
                        if (x < a.n0) exc[x * M + m] = Op::apply(st.pex[r], S);
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
                        const i64 x = qe * k0 + r;
                        if (x < a.n0) inc[x * M + m] = val;
                    }
                }
            }
        }
        if (q < qb) st.absorb(v, k0, do_ex, do_inc);
    };

    if (t_begin < t_end) fetch(t_begin);
    i64 qlast = qa - 1;
    for (i64 t = t_begin; t < t_end; ++t) {
        const i64 q = t / k0;
        const int r = (int)(t - q * k0);
        if (r == 0 && do_ex && pvalid) sx_next = q < a.Q ? SX[q * M + m] : e;
        // 1. stage the prefetched halo tile, prefetch the next plane
#pragma unroll
        for (int j = 0; j < C::NLOAD; ++j)
            if (loff[j] >= 0) sA[loff[j]] = pre[j];
        if (t + 1 < t_end) fetch(t + 1);
        __syncthreads();
        // 2. BDBS along x for every halo row: range suffix of block b, plus the
        //    range prefix of block b+1 (identity past the tensor edge)
        {
            const int nbx = a.TX / kx;
            const int tasks = rows_in * nbx;
            for (int task = tid; task < tasks; task += NT) {
                const int row = task % rows_in, b = task / rows_in;
                const T* src = sA + row * C::PA + b * kx;
                T* dst = sB + row * C::PB + b * kx;
                T sfx = e;
                for (int rr = kx - 1; rr >= 0; --rr) {
                    sfx = Op::apply(src[rr], sfx);
                    dst[rr] = sfx;
                }
                T p = e;
                for (int rr = 1; rr < kx; ++rr) {
                    p = Op::apply(p, src[kx + rr - 1]);
                    dst[rr] = Op::apply(dst[rr], p);
                }
            }
        }
        __syncthreads();
        // 3. BDBS along y for every column into ring slot r
        {
            const int nby = a.TY / ky;
            const int tasks = a.TX * nby;
            T* slot = ring + r * NT;
            for (int task = tid; task < tasks; task += NT) {
                const int col = task % a.TX, b = task / a.TX;
                const T* src = sB + b * ky * C::PB + col;
                T* dst = slot + b * ky * C::TXM + col;
                T sfx = e;
                for (int rr = ky - 1; rr >= 0; --rr) {
                    sfx = Op::apply(src[rr * C::PB], sfx);
                    dst[rr * C::TXM] = sfx;
                }
                T p = e;
                for (int rr = 1; rr < ky; ++rr) {
                    p = Op::apply(p, src[(ky + rr - 1) * C::PB]);
                    dst[rr * C::TXM] = Op::apply(dst[rr * C::TXM], p);
                }
            }
        }
        // 4. a block of W planes is complete: emit the previous block
        if (r == k0 - 1 || t == a.n0 - 1) {
            block_step(q);
            qlast = q;
        }
    }
    // the block after the run lies past the tensor: emit the last block
    if (qlast < qb) {
        if (do_ex && pvalid) sx_next = e;
        block_step(qb);
    }
}

bool plane_eligible(int d, const i64* n, const i64* k, int es) {
    if (d < 3) return false;
    const i64 k0 = k[0];
    if (k0 > 64) return false;
    int kb = k0 <= 1 ? 1 : k0 <= 2 ? 2 : k0 <= 4 ? 4 : k0 <= 8 ? 8 : k0 <= 16 ? 16 : k0 <= 32 ? 32 : 64;
    const int nt = (kb * es <= 64) ? 1024 : (kb * es <= 128) ? 512 : 256;
    const int tym = nt == 1024 ? 32 : 16, txm = nt == 256 ? 16 : 32;
    return k[d - 2] <= tym && k[d - 1] <= txm;
}

template <typename T, class Op, int K0B>
static void launch_plane_kb(PlaneArgs pa, hipStream_t st) {
    using C = PlaneCfg<K0B, sizeof(T)>;
    pa.TY = (int)(C::TYM / pa.ky * pa.ky);
    pa.TX = (int)(C::TXM / pa.kx * pa.kx);
    pa.tilesY = (pa.NY + pa.TY - 1) / pa.TY;
    pa.tilesX = (pa.NX + pa.TX - 1) / pa.TX;
    const i64 tiles = pa.tilesY * pa.tilesX * pa.MID;
    // enough workgroups to cover the CUs twice; each run of blocks reads
    // one extra block of planes
    i64 nseg = (512 + tiles - 1) / tiles;
    if (nseg > pa.Q) nseg = pa.Q;
    if (nseg < 1) nseg = 1;
    pa.segblocks = (pa.Q + nseg - 1) / nseg;
    pa.nseg = (pa.Q + pa.segblocks - 1) / pa.segblocks;
    const i64 grid = tiles * pa.nseg;
    hipLaunchKernelGGL((k_plane_axis0<T, Op, K0B>), dim3((unsigned)grid), dim3(C::NT), 0, st,
                       pa);
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
    if (k0 <= 1) launch_plane_kb<T, Op, 1>(pa, st);
    else if (k0 <= 2) launch_plane_kb<T, Op, 2>(pa, st);
    else if (k0 <= 4) launch_plane_kb<T, Op, 4>(pa, st);
    else if (k0 <= 8) launch_plane_kb<T, Op, 8>(pa, st);
    else if (k0 <= 16) launch_plane_kb<T, Op, 16>(pa, st);
    else if (k0 <= 32) launch_plane_kb<T, Op, 32>(pa, st);
    else launch_plane_kb<T, Op, 64>(pa, st);
}

#define EXS_INST_PLANE(T, OP)                                                                  \
    template void launch_plane_axis0<T, OP>(const T*, const T*, const T*, const T*, T*, T*,    \
                                            i64, i64, i64, i64, i64, i64, i64, i64, hipStream_t);
EXS_INST_PLANE(float, OpSum)
EXS_INST_PLANE(double, OpSum)
EXS_INST_PLANE(int, OpSum)
EXS_INST_PLANE(long long, OpSum)
EXS_INST_PLANE(float, OpMax)
EXS_INST_PLANE(double, OpMax)
EXS_INST_PLANE(int, OpMax)
EXS_INST_PLANE(long long, OpMax)

}  // namespace exs
