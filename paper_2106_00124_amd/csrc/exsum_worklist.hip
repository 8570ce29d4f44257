// exsum_worklist.hip -- persistent work-list kernels of the batched form.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// One launch covers one kind of step (with one element size and register
// bucket) for many tensors at once, in parts of one element type and
// operator each.  The steps of the launch sit in a device
// array; every step's tasks start at a multiple of WL_CHUNK in the launch's
// flat task range, so that a chunk of WL_CHUNK consecutive tasks (one
// workgroup's share) belongs to one step, named by the launch's chunk table.
// The workgroups of a part walk its chunks with a stride of their count; the
// step of a chunk is read once per workgroup (uniform: scalar loads) and each
// thread runs the same per-task function as the plain kernels on its task of
// the chunk.
#include "exsum_internal.hpp"
#include "exsum_tasks.hpp"

namespace exs {

// The part of the launch that workgroup w serves.
__device__ __forceinline__ int wl_part(const WlParts& p, int w) {
    int g = 0;
    while (g + 1 < p.n && w >= p.wg0[g + 1]) ++g;
    return g;
}

template <int ES, int KIND, int KB>
__global__ __launch_bounds__(256) void k_worklist(const Step* __restrict__ steps,
                                                  const int* __restrict__ chunk_step, WlParts p) {
    static_assert(WL_CHUNK == 256, "one chunk per workgroup of 256 threads");
    const int w = blockIdx.x;
    const int g = wl_part(p, w);
    const i64 c1 = p.unit0[g + 1], nw = p.wg0[g + 1] - p.wg0[g];
    const i64 c0 = p.unit0[g] + (w - p.wg0[g]);
    with_type_op<ES>(p.code[g], [&](auto to) __attribute__((always_inline)) {
        using T = typename decltype(to)::type;
        using Op = typename decltype(to)::op;
        for (i64 c = c0; c < c1; c += nw) {
            const Step& s = steps[chunk_step[c]];
            const i64 t = c * WL_CHUNK + threadIdx.x - s.task_begin;
            if (t < s.ntasks) run_task<T, Op, KIND, KB>(s, t);
        }
    });
}

// Row BDBS tasks (SK_BDBSR) take a whole wavefront each: workgroups of 64
// threads walk the tasks of their part with a workgroup stride (the chunk
// table has one entry per task here); the LDS tile is dynamic (sized for the
// widest step of the launch).
template <int ES, int KB>
__global__ __launch_bounds__(64) void k_worklist_rows(const Step* __restrict__ steps,
                                                      const int* __restrict__ task_step, WlParts p) {
    extern __shared__ __align__(16) unsigned char exs_wl_lds[];
    const int w = blockIdx.x;
    const int g = wl_part(p, w);
    const i64 t1 = p.unit0[g + 1], nw = p.wg0[g + 1] - p.wg0[g];
    const i64 t0 = p.unit0[g] + (w - p.wg0[g]);
    with_type_op<ES>(p.code[g], [&](auto to) __attribute__((always_inline)) {
        using T = typename decltype(to)::type;
        using Op = typename decltype(to)::op;
        for (i64 t = t0; t < t1; t += nw) {
            const Step& s = steps[task_step[t]];
            task_bdbs_rows<T, Op, KB>((const T*)s.in0, (T*)s.out0, s.O, s.n, s.k, s.cb, s.nchunks,
                                      t - s.task_begin, (T*)exs_wl_lds);
        }
    });
}

template <int ES>
static void launch_rows(int kb, const Step* steps, const int* table, const WlParts& p, size_t lds,
                        hipStream_t st) {
    const int grid = p.wg0[p.n];
#define EXS_WLR(KB)                                                                                \
    case KB:                                                                                       \
        hipLaunchKernelGGL((k_worklist_rows<ES, KB>), dim3(grid), dim3(64), lds, st, steps, table, \
                           p);                                                                     \
        return;
    switch (kb) {
        EXS_WLR(1) EXS_WLR(2) EXS_WLR(4) EXS_WLR(8) EXS_WLR(16) EXS_WLR(32) EXS_WLR(64)
    }
#undef EXS_WLR
}

template <int ES, int KIND>
static void launch_kb(int kb, const Step* steps, const int* table, const WlParts& p,
                      hipStream_t st) {
    const int grid = p.wg0[p.n];
#define EXS_WL(KB)                                                                                 \
    case KB:                                                                                       \
        hipLaunchKernelGGL((k_worklist<ES, KIND, KB>), dim3(grid), dim3(256), 0, st, steps, table, \
                           p);                                                                     \
        return;
    if constexpr (KIND == SK_BDBS || KIND == SK_AX0 || KIND == SK_BDBSW || KIND == SK_AX0W) {
        switch (kb) {
            EXS_WL(1) EXS_WL(2) EXS_WL(4) EXS_WL(8) EXS_WL(16) EXS_WL(32) EXS_WL(64)
        }
    } else if constexpr (KIND == SK_BDBSC || KIND == SK_AX0C) {
        switch (kb) {
            EXS_WL(32) EXS_WL(64)
        }
    } else {
        hipLaunchKernelGGL((k_worklist<ES, KIND, 1>), dim3(grid), dim3(256), 0, st, steps, table,
                           p);
    }
#undef EXS_WL
}

template <int ES>
static void launch_kind(int kind, int kb, const Step* steps, const int* table, const WlParts& p,
                        size_t lds, hipStream_t st) {
    switch (kind) {
        case SK_BDBSR: launch_rows<ES>(kb, steps, table, p, lds, st); break;
        case SK_BDBS: launch_kb<ES, SK_BDBS>(kb, steps, table, p, st); break;
        case SK_BDBS2: launch_kb<ES, SK_BDBS2>(kb, steps, table, p, st); break;
        case SK_AGG: launch_kb<ES, SK_AGG>(kb, steps, table, p, st); break;
        case SK_SCAN: launch_kb<ES, SK_SCAN>(kb, steps, table, p, st); break;
        case SK_SEGTOT: launch_kb<ES, SK_SEGTOT>(kb, steps, table, p, st); break;
        case SK_SEGEXP: launch_kb<ES, SK_SEGEXP>(kb, steps, table, p, st); break;
        case SK_AX0: launch_kb<ES, SK_AX0>(kb, steps, table, p, st); break;
        case SK_EX2: launch_kb<ES, SK_EX2>(kb, steps, table, p, st); break;
        case SK_BDBSW: launch_kb<ES, SK_BDBSW>(kb, steps, table, p, st); break;
        case SK_AX0W: launch_kb<ES, SK_AX0W>(kb, steps, table, p, st); break;
        case SK_BDBSV: launch_kb<ES, SK_BDBSV>(kb, steps, table, p, st); break;
        case SK_BDBSC: launch_kb<ES, SK_BDBSC>(kb, steps, table, p, st); break;
        case SK_AX0C: launch_kb<ES, SK_AX0C>(kb, steps, table, p, st); break;
    }
}

void launch_worklist(int es, int kind, int kb, const void* steps, const int* table,
                     const WlParts& parts, size_t lds, hipStream_t st) {
    const Step* s = (const Step*)steps;
    if (es == 4) launch_kind<4>(kind, kb, s, table, parts, lds, st);
    else launch_kind<8>(kind, kb, s, table, parts, lds, st);
}

}  // namespace exs
