// exsum_plan.hpp -- the planner of included/excluded sums for one tensor.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// Excluded sums follow the box-complement algorithm (Sec. 5) in its
// dimension-reduction form.  With R_0 = A and R_{j+1} = the reduction of R_j
// over its first axis, the excluded sum of R_j (rank d_j) is
//
//   Exc_j(x) = Ex1D_0( Inc_{1..}(R_j) )(x) op Exc_{j+1}(x_1, ..., x_{d_j-1})
//
// where Inc_{1..} box-sums every axis but the first (BDBS-Along-Dim, Sec. 5)
// and Ex1D_0 is the op of the prefix before x_0 and the suffix from x_0+k_0
// along the first axis (Prefix-/Suffix-Along-Dim, Sec. 5).  The two components
// of step j+1 in Corollary "Excluded-sum Components" are exactly the prefix
// and suffix terms; the lower-dimensional term carries the components of the
// later steps, broadcast over the reduced axes (Add-Contribution, Sec. 5).
// Included sums are BDBS along every axis (Sec. 3, "Generalizing to
// Arbitrary Dimensions").
//
// The planner emits its steps into a Sink: EagerSink launches each step on a
// stream (the plain call); the batched form records them into work lists.
// Buffers come from an Arena over the caller's workspace; in "dry" mode the
// arena only measures, so sizing and execution share one code path.
//
// Kernel choice (each special path applies only where the sink offers it and
// its size rules hold; otherwise the generic one-axis passes run): a level of
// rank >= 3 streams its first axis with the fused plane kernels; a rank-2
// level with the fused row stream; the rank-3 level also hands the last two
// levels to one workgroup when their table is small; the last (1-D) level
// runs in one workgroup when short and in chunks when long; trailing axes
// that fit in LDS are box-summed in one staged pass.
#pragma once
#include <algorithm>

#include "exsum_internal.hpp"

namespace exs {

// Bump allocator over the caller's workspace.  In "dry" mode it only
// measures, so sizing and execution share one code path.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, off = 0;
    bool dry = true;
    template <typename T>
    T* take(i64 count) {
        off = (off + 255) & ~(size_t)255;
        T* p = dry ? nullptr : (T*)(base + off);
        off += (size_t)count * sizeof(T);
        return p;
    }
};

inline i64 prod(const i64* v, int a, int b) {
    i64 p = 1;
    for (int i = a; i < b; ++i) p *= v[i];
    return p;
}

// Box-sum a rank-d tensor over axes last .. first (last axis first: the
// innermost reduction of the nested definition in Sec. 2), ping-ponging
// between wb[0] and wb[1].  Axes with k = 1 are skipped (BDBS with k = 1 is
// the identity); when the axes end at the tensor's last axis, the trailing
// ones that fit the sink's staged sub-tensor go in one pass.  Returns the
// result (src itself if no axis).
template <typename T, class Sink>
static const T* filter_axes(const T* src, const i64* n, const i64* k, int d, int first, int last,
                            T* wb0, T* wb1, bool dry, Sink& sink) {
    const T* cur = src;
    T* wb[2] = {wb0, wb1};
    int which = 0;
    int a = last;
    if (last == d - 1) {
        int m = 0, busy = 0;
        i64 S = 1;
        while (last - m >= first && S * n[last - m] <= sink.tail_box_max()) {
            S *= n[last - m];
            busy += k[last - m] > 1;
            ++m;
        }
        if (busy >= 2) {
            T* dst = wb[which];
            which ^= 1;
            if (!dry) sink.bdbs_tail(cur, dst, prod(n, 0, d - m), m, n + d - m, k + d - m);
            cur = dst;
            a = last - m;
        }
    }
    for (; a >= first; --a) {
        if (k[a] == 1) continue;
        T* dst = wb[which];
        which ^= 1;
        if (!dry) sink.bdbs(cur, dst, prod(n, 0, a), n[a], prod(n, a + 1, d), k[a]);
        cur = dst;
    }
    return cur;
}

// Block scans of a level (PX, SX over the Q blocks of each of the M points,
// and R = op of Ga over all blocks).  The direct scan is one serial walk over
// the Q blocks per point; unless the points alone fill the GPU (2^18 threads)
// or the walk is short, the blocks are cut into segments of L, the segment
// totals are scanned the same way (recursively), and the segments are
// expanded in parallel.
// PX is stored only for blocks q % pxe == 0 (the run starts of a fused
// stream); the scan of the segment totals stores all of its own.
template <typename T, class Sink>
static void emit_blockscan(const T* Gw, const T* Ga, T* PX, T* SX, T* R, i64 Q, i64 M, Arena& ar,
                           bool dry, Sink& sink, i64 pxe = 1) {
    constexpr i64 L = 64;
    if (M >= ((i64)1 << 18) || Q <= L) {
        if (!dry) sink.blockscan(Gw, Ga, PX, SX, R, Q, M, pxe);
        return;
    }
    const i64 S = (Q + L - 1) / L;
    T* Tw = ar.take<T>(S * M);
    T* Ta = ar.take<T>(S * M);
    T* SPX = ar.take<T>(S * M);
    T* SSX = ar.take<T>(S * M);
    if (!dry) sink.segtot(Gw, Ga, Tw, Ta, Q, M, L);
    emit_blockscan<T>(Tw, Ta, SPX, SSX, R, S, M, ar, dry, sink);
    if (!dry) sink.segexp(Gw, SPX, SSX, PX, SX, Q, M, L, pxe);
}

template <typename T, class Sink>
static exs_status plan_job(const exs_job* job, Arena& ar, Sink& sink) {
    const int d = job->d;
    i64 n[EXS_MAX_RANK], k[EXS_MAX_RANK];
    for (int i = 0; i < d; ++i) { n[i] = job->dims[i]; k[i] = job->box[i]; }
    const T* A = (const T*)job->in_dev;
    T* inc = (job->mode & EXS_INCLUDED) ? (T*)job->inc_out_dev : nullptr;
    T* exc = (job->mode & EXS_EXCLUDED) ? (T*)job->exc_out_dev : nullptr;
    const bool weak = job->mode & EXS_WEAK;
    const bool want_exc = (job->mode & EXS_EXCLUDED) && !weak;  // strong excluded sums
    const bool dry = ar.dry;
    const i64 N = prod(n, 0, d);
    // a small rank-2 tensor: both levels in one workgroup, no workspace
    if (d == 2 && !weak && sink.small2d_ok(n[0], n[1], k[0], k[1])) {
        if (!dry) sink.small2d(A, exc, inc, n[0], n[1], k[0], k[1]);
        return EXS_OK;
    }
    // a level of rank >= 3 streams its first axis with the fused plane kernel
    // when it applies; it box-sums the two trailing axes itself, the middle
    // axes are done first (levels past 0 exist only for strong excluded sums)
    bool fz[EXS_MAX_RANK] = {};
    for (int j = 0; j < (want_exc ? d : 1); ++j)
        fz[j] = sink.fused_ok && sizeof(T) == 4 &&
                plane_eligible(d - j, n + j, k + j, (int)sizeof(T));
    const bool fused = fz[0];

    // included sums (alone, or for the weak excluded sums) of a rank-1 or
    // rank-2 tensor in one pass: the chunked 1-D kernel or the 2-D stream
    const bool inc1 = !want_exc && d == 1 && sink.long1d_ok(n[0], k[0]);
    const bool inc2 = !want_exc && d == 2 && sink.row_ok(n[0], n[1], k[0], k[1]);
    // buffers for box-summed tensors, shared by every level: level j needs
    // (d_j - 1) passes over N_j elements, a fused level only d_j - 3
    int wb_count = 0;
    i64 wb_elems = 0;
    for (int j = 0; j < (want_exc ? d : 1); ++j) {
        const int passes = fz[j]                        ? std::max(0, d - j - 3)
                           : (j == 0 && (inc1 || inc2)) ? 0
                                                        : d - j - 1;
        if (passes > 0) {
            wb_count = std::max(wb_count, std::min(2, passes));
            wb_elems = std::max(wb_elems, prod(n, j, d));
        }
    }
    T* wb0 = wb_count >= 1 ? ar.take<T>(wb_elems) : nullptr;
    T* wb1 = wb_count >= 2 ? ar.take<T>(wb_elems) : nullptr;

    sink.level(0);
    if (weak) {
        // weak excluded sums for +: total - included (the paper's BDBSC
        // route, Sec. 1 and Sec. 6), the included sums by BDBS along every
        // axis; exc doubles as the included buffer when inc is not wanted
        T* tot = ar.take<T>(1);
        unsigned long long* parts = ar.take<unsigned long long>(TOT_PARTS);
        if (!dry) sink.total(A, N, parts, tot);
        if (fused) {
            const T* X0 = filter_axes<T>(A, n, k, d, 1, d - 3, wb0, wb1, dry, sink);
            if (!dry)
                sink.plane_weak(X0, inc, tot, exc, n[0], prod(n, 1, d - 2), n[d - 2], n[d - 1],
                                k[0], k[d - 2], k[d - 1]);
            return EXS_OK;
        }
        T* incb = inc ? inc : exc;
        if (inc1 || inc2) {
            if (!dry) {
                if (inc1)
                    sink.long1d(A, nullptr, incb, n[0], k[0], nullptr, nullptr, nullptr, nullptr);
                else
                    sink.row_axis0(A, nullptr, nullptr, nullptr, nullptr, incb, n[0], n[1], k[0],
                                   k[1], (n[0] + k[0] - 1) / k[0]);
                sink.weak_exc(incb, tot, exc, N);
            }
            return EXS_OK;
        }
        const T* W = filter_axes<T>(A, n, k, d, 1, d - 1, wb0, wb1, dry, sink);
        if (!dry) {
            sink.bdbs(W, incb, 1, n[0], prod(n, 1, d), k[0]);
            sink.weak_exc(incb, tot, exc, N);
        }
        return EXS_OK;
    }
    if (!want_exc) {
        // included sums only: BDBS along every axis
        if (fused) {
            const T* X0 = filter_axes<T>(A, n, k, d, 1, d - 3, wb0, wb1, dry, sink);
            if (!dry)
                sink.plane_axis0(X0, nullptr, nullptr, nullptr, nullptr, inc, n[0],
                                 prod(n, 1, d - 2), n[d - 2], n[d - 1], k[0], k[d - 2], k[d - 1],
                                 (n[0] + k[0] - 1) / k[0]);
            return EXS_OK;
        }
        if (inc2) {
            if (!dry)
                sink.row_axis0(A, nullptr, nullptr, nullptr, nullptr, inc, n[0], n[1], k[0], k[1],
                               (n[0] + k[0] - 1) / k[0]);
            return EXS_OK;
        }
        if (inc1) {
            if (!dry) sink.long1d(A, nullptr, inc, n[0], k[0], nullptr, nullptr, nullptr, nullptr);
            return EXS_OK;
        }
        const T* W = filter_axes<T>(A, n, k, d, 1, d - 1, wb0, wb1, dry, sink);
        if (!dry) sink.bdbs(W, inc, 1, n[0], prod(n, 1, d), k[0]);
        return EXS_OK;
    }

    // per-level sizes
    i64 Q[EXS_MAX_RANK], M[EXS_MAX_RANK];
    i64 maxQM = 0;
    for (int j = 0; j < d; ++j) {
        Q[j] = (n[j] + k[j] - 1) / k[j];
        M[j] = prod(n, j + 1, d);
        maxQM = std::max(maxQM, Q[j] * M[j]);
    }
    T* Ga = ar.take<T>(maxQM);
    const int ngb = std::min(2, d - 1);
    T* gb0 = ngb >= 1 ? ar.take<T>(maxQM) : nullptr;
    T* gb1 = ngb >= 2 ? ar.take<T>(maxQM) : nullptr;
    T *PX[EXS_MAX_RANK], *SX[EXS_MAX_RANK], *R[EXS_MAX_RANK + 1];
    R[0] = nullptr;
    for (int j = 0; j < d; ++j) {
        PX[j] = ar.take<T>(Q[j] * M[j]);
        SX[j] = ar.take<T>(Q[j] * M[j]);
        R[j + 1] = ar.take<T>(M[j]);
    }
    // lower-level excluded sums: level j >= 1 writes tb[j % 2] (N_j <= N_1)
    T* tb0 = d >= 3 ? ar.take<T>(M[0]) : nullptr;
    T* tb1 = d >= 2 ? ar.take<T>(M[0]) : nullptr;
    T* tb[2] = {tb0, tb1};

    // top-down: block aggregates, their box-sums over the other axes, block
    // scans, and the reduction that feeds the next level
    // the last level is 1-D; when short, one workgroup computes its excluded
    // sums directly from R_{d-1} (no block passes)
    const bool last_small = d >= 2 && sink.small1d_ok(n[d - 1]);
    // when long, in chunks: chunk totals, their scans, one pass over the axis
    const bool last_long = !last_small && sink.long1d_ok(n[d - 1], k[d - 1]);
    T *c_tot = nullptr, *c_rest = nullptr, *c_pre = nullptr, *c_suf = nullptr;
    if (last_long) {
        const i64 nc = long1d_chunks(n[d - 1], k[d - 1]);
        c_tot = ar.take<T>(nc);
        c_rest = ar.take<T>(nc);
        c_pre = ar.take<T>(nc);
        c_suf = ar.take<T>(nc);
    }
    // fused levels with at most 64 blocks take their block scans in the same
    // pass as the box-sums of the trailing axes
    const bool p2ok =
        d >= 3 && plane2_eligible(n[d - 2], n[d - 1], k[d - 2], k[d - 1], (int)sizeof(T));
    bool scan[EXS_MAX_RANK] = {};
    for (int j = 0; j < d; ++j) scan[j] = fz[j] && Q[j] <= 64 && p2ok;
    // a fused level of rank >= 4 takes its block aggregates in the same pass
    // as its box sums along the innermost middle axis f with k > 1 (k <= 16):
    // that pass writes the box-summed tensor for P2 (xa), Ga, and Ga box-summed
    // along f (g1a); the other middle axes stay separate passes
    int amf[EXS_MAX_RANK] = {};  // f relative to the level, 0: not taken
    T* xa[EXS_MAX_RANK] = {};
    T* g1a = nullptr;
    for (int j = 0; j < d; ++j) {
        const int dj = d - j;
        // (4-byte fused levels below 2^31 bytes: 32-bit offsets)
        if (!(fz[j] && p2ok && dj >= 4 && sink.aggmid_ok() &&
              prod(n, j, d) * (i64)sizeof(T) < ((i64)1 << 31)))
            continue;
        for (int a = dj - 3; a >= 1; --a)
            if (k[j + a] > 1) {
                if (k[j + a] <= 16) amf[j] = a;
                break;
            }
        if (amf[j]) {
            xa[j] = ar.take<T>(prod(n, j, d));
            if (!g1a) g1a = ar.take<T>(maxQM);
        }
    }
    // the rank-3 level d - 3, when it takes that pass, also reduces R_{d-2}
    // over the blocks of level d - 2 (its tiles hold whole blocks); when that
    // table is small one workgroup finishes the last two levels from it
    // (box-sums, block scans, the 1-D level), and only the level d - 2
    // stream then reads R_{d-2}
    const bool tail = d >= 3 && scan[d - 3] &&
                      sink.row_ok(n[d - 2], n[d - 1], k[d - 2], k[d - 1]) &&
                      sink.tail_ok(Q[d - 2], n[d - 1], k[d - 1]);
    T* A1 = tail ? ar.take<T>(Q[d - 2] * n[d - 1]) : nullptr;
    for (int j = 0; j < d; ++j) {
        const int dj = d - j;
        const T* src = j == 0 ? A : R[j];
        if (j == d - 1 && (last_small || last_long)) break;
        sink.level(j);
        const int f = amf[j];
        if (!dry) {
            if (f)
                sink.aggmid(src, xa[j], Ga, g1a, n[j], prod(n, j + 1, j + f), n[j + f],
                            prod(n, j + f + 1, d), k[j], k[j + f], Q[j]);
            else
                sink.blockagg(src, Ga, n[j], M[j], k[j], Q[j]);
        }
        i64 gn[EXS_MAX_RANK], gk[EXS_MAX_RANK];
        gn[0] = Q[j];
        gk[0] = 1;
        for (int a = 1; a < dj; ++a) { gn[a] = n[j + a]; gk[a] = k[j + a]; }
        const T* Gw;
        const i64 mid = prod(n, j + 1, d - 2);
        // Ga box-summed over the middle axes
        auto mid_sums = [&]() {
            return f ? filter_axes<T>(g1a, gn, gk, dj, 1, f - 1, gb0, gb1, dry, sink)
                     : filter_axes<T>(Ga, gn, gk, dj, 1, dj - 3, gb0, gb1, dry, sink);
        };
        if (scan[j]) {
            // middle axes by the generic passes; the two trailing axes and the
            // block scans in one pass (the box-summed planes are not stored)
            const T* G1 = mid_sums();
            const bool last3 = tail && j == d - 3;
            // the streaming kernel reads the block prefix only where its runs start
            if (!dry)
                sink.plane_scan(G1, Ga, PX[j], SX[j], R[j + 1], last3 ? A1 : nullptr, Q[j], mid,
                                n[d - 2], n[d - 1], k[d - 2], k[d - 1],
                                plane_axis0_run_blocks(Q[j], mid, n[d - 2], n[d - 1], k[d - 2],
                                                       k[d - 1]));
            if (last3) {
                // the last two levels; Exc_{d-1} goes where the bottom-up
                // pass expects it
                sink.level(d - 2);
                if (!dry)
                    sink.tail_scan(A1, PX[d - 2], SX[d - 2], tb[(d - 1) % 2], Q[d - 2], n[d - 1],
                                   k[d - 1], row_axis0_run_blocks(Q[d - 2], n[d - 1], k[d - 1]));
                break;
            }
            continue;
        }
        if (fz[j] && p2ok) {
            // middle axes by the generic passes, the two trailing axes in one
            // LDS-tiled pass
            const T* G1 = mid_sums();
            T* G2 = G1 == gb0 ? gb1 : gb0;
            if (!dry)
                sink.plane_bdbs(G1, G2, Q[j] * mid, n[d - 2], n[d - 1], k[d - 2], k[d - 1]);
            Gw = G2;
        } else {
            Gw = filter_axes<T>(Ga, gn, gk, dj, 1, dj - 1, gb0, gb1, dry, sink);
        }
        // the fused streams (of a level of rank >= 3, or of a 2-D level) read
        // the block prefix only where their runs start
        const i64 pxe = fz[j] ? plane_axis0_run_blocks(Q[j], mid, n[d - 2], n[d - 1], k[d - 2],
                                                       k[d - 1])
                        : dj == 2 && sink.row_ok(n[j], n[j + 1], k[j], k[j + 1])
                            ? row_axis0_run_blocks(Q[j], n[j + 1], k[j + 1])
                            : 1;
        emit_blockscan<T>(Gw, Ga, PX[j], SX[j], R[j + 1], Q[j], M[j], ar, dry, sink, pxe);
    }
    // bottom-up: stream the first axis of each level, adding the level below
    for (int j = d - 1; j >= 0; --j) {
        const int dj = d - j;
        const T* src = j == 0 ? A : R[j];
        sink.level(j);
        T* out = j == 0 ? exc : tb[j % 2];
        const T* Trest = j == d - 1 ? nullptr : tb[(j + 1) % 2];
        if (j == d - 1 && tail) continue;
        if (j == d - 1 && last_small) {
            if (!dry) sink.ex1d_small(src, out, n[j], k[j]);
            continue;
        }
        if (j == d - 1 && last_long) {
            if (!dry)
                sink.long1d(src, out, j == 0 ? inc : nullptr, n[j], k[j], c_tot, c_rest, c_pre,
                            c_suf);
            continue;
        }
        if (fz[j]) {
            const T* X0 = amf[j] ? filter_axes<T>(xa[j], n + j, k + j, dj, 1, amf[j] - 1, wb0,
                                                  wb1, dry, sink)
                                 : filter_axes<T>(src, n + j, k + j, dj, 1, dj - 3, wb0, wb1,
                                                  dry, sink);
            if (!dry)
                sink.plane_axis0(X0, PX[j], SX[j], Trest, out, j == 0 ? inc : nullptr, n[j],
                                 prod(n, j + 1, d - 2), n[d - 2], n[d - 1], k[j], k[d - 2],
                                 k[d - 1], Q[j]);
            continue;
        }
        if (dj == 2 && sink.row_ok(n[j], n[j + 1], k[j], k[j + 1])) {
            // a 2-D level: the row box-sums and the axis stream in one pass
            if (!dry)
                sink.row_axis0(src, PX[j], SX[j], Trest, out, j == 0 ? inc : nullptr, n[j],
                               n[j + 1], k[j], k[j + 1], Q[j]);
            continue;
        }
        const T* W = filter_axes<T>(src, n + j, k + j, dj, 1, dj - 1, wb0, wb1, dry, sink);
        // boxes longer than 64 with few points: chunk totals for the chunked sweep
        const i64 ch = bucket_for(k[j]) == 0 && out ? ex2_chunks(n[j], M[j]) : 1;
        T* ex2t = ch > 1 ? ar.take<T>(ch * M[j]) : nullptr;
        if (!dry)
            sink.axis0(W, PX[j], SX[j], Trest, out, j == 0 ? inc : nullptr, n[j], M[j], k[j],
                       Q[j], ex2t);
    }
    return EXS_OK;
}


}  // namespace exs
