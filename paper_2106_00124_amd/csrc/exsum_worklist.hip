// exsum_worklist.hip -- persistent work-list kernels of the batched form.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// One launch covers one kind of step (with one dtype, operator and register
// bucket) for many tensors at once.  The steps of the launch sit in a device
// array; every step's tasks start at a multiple of WL_CHUNK in the launch's
// flat task range, so that a chunk of WL_CHUNK consecutive tasks (one
// workgroup's share) belongs to one step, named by the launch's chunk table.
// A persistent grid walks the chunks with a grid stride; the step of a chunk
// is read once per workgroup (uniform: scalar loads) and each thread runs the
// same per-task function as the plain kernels on its task of the chunk.
#include "exsum_internal.hpp"
#include "exsum_tasks.hpp"

namespace exs {

template <typename T, class Op, int KIND, int KB>
__global__ __launch_bounds__(256) void k_worklist(const Step* __restrict__ steps,
                                                  const int* __restrict__ chunk_step, i64 nchunks) {
    static_assert(WL_CHUNK == 256, "one chunk per workgroup of 256 threads");
    for (i64 c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const Step& s = steps[chunk_step[c]];
        const i64 t = c * WL_CHUNK + threadIdx.x - s.task_begin;
        if (t < s.ntasks) run_task<T, Op, KIND, KB>(s, t);
    }
}

// Row BDBS tasks (SK_BDBSR) take a whole wavefront each: workgroups of 64
// threads walk the tasks with a workgroup stride (the chunk table has one
// entry per task here); the LDS tile is dynamic (sized for the widest step
// of the launch).
template <typename T, class Op, int KB>
__global__ __launch_bounds__(64) void k_worklist_rows(const Step* __restrict__ steps,
                                                      const int* __restrict__ task_step, i64 total) {
    extern __shared__ __align__(16) unsigned char exs_wl_lds[];
    for (i64 t = blockIdx.x; t < total; t += gridDim.x) {
        const Step& s = steps[task_step[t]];
        task_bdbs_rows<T, Op, KB>((const T*)s.in0, (T*)s.out0, s.O, s.n, s.k, s.cb, s.nchunks,
                                  t - s.task_begin, (T*)exs_wl_lds);
    }
}

template <typename T, class Op>
static void launch_rows(int kb, const Step* steps, const int* table, i64 total, int grid,
                        size_t lds, hipStream_t st) {
#define EXS_WLR(KB)                                                                          \
    case KB:                                                                                 \
        hipLaunchKernelGGL((k_worklist_rows<T, Op, KB>), dim3(grid), dim3(64), lds, st, steps, \
                           table, total);                                                    \
        return;
    switch (kb) {
        EXS_WLR(1) EXS_WLR(2) EXS_WLR(4) EXS_WLR(8) EXS_WLR(16) EXS_WLR(32) EXS_WLR(64)
    }
#undef EXS_WLR
}

template <typename T, class Op, int KIND>
static void launch_kb(int kb, const Step* steps, const int* table, i64 nchunks, int grid,
                      hipStream_t st) {
#define EXS_WL(KB)                                                                            \
    case KB:                                                                                  \
        hipLaunchKernelGGL((k_worklist<T, Op, KIND, KB>), dim3(grid), dim3(256), 0, st, steps, \
                           table, nchunks);                                                   \
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
        hipLaunchKernelGGL((k_worklist<T, Op, KIND, 1>), dim3(grid), dim3(256), 0, st, steps,
                           table, nchunks);
    }
#undef EXS_WL
}

template <typename T, class Op>
static void launch_kind(int kind, int kb, const Step* steps, const int* table, i64 units, int grid,
                        size_t lds, hipStream_t st) {
    switch (kind) {
        case SK_BDBSR: launch_rows<T, Op>(kb, steps, table, units, grid, lds, st); break;
        case SK_BDBS: launch_kb<T, Op, SK_BDBS>(kb, steps, table, units, grid, st); break;
        case SK_BDBS2: launch_kb<T, Op, SK_BDBS2>(kb, steps, table, units, grid, st); break;
        case SK_AGG: launch_kb<T, Op, SK_AGG>(kb, steps, table, units, grid, st); break;
        case SK_SCAN: launch_kb<T, Op, SK_SCAN>(kb, steps, table, units, grid, st); break;
        case SK_SEGTOT: launch_kb<T, Op, SK_SEGTOT>(kb, steps, table, units, grid, st); break;
        case SK_SEGEXP: launch_kb<T, Op, SK_SEGEXP>(kb, steps, table, units, grid, st); break;
        case SK_AX0: launch_kb<T, Op, SK_AX0>(kb, steps, table, units, grid, st); break;
        case SK_EX2: launch_kb<T, Op, SK_EX2>(kb, steps, table, units, grid, st); break;
        case SK_BDBSW: launch_kb<T, Op, SK_BDBSW>(kb, steps, table, units, grid, st); break;
        case SK_AX0W: launch_kb<T, Op, SK_AX0W>(kb, steps, table, units, grid, st); break;
        case SK_BDBSV: launch_kb<T, Op, SK_BDBSV>(kb, steps, table, units, grid, st); break;
        case SK_BDBSC: launch_kb<T, Op, SK_BDBSC>(kb, steps, table, units, grid, st); break;
        case SK_AX0C: launch_kb<T, Op, SK_AX0C>(kb, steps, table, units, grid, st); break;
    }
}

template <typename T>
static void launch_op(int op, int kind, int kb, const Step* steps, const int* table, i64 units,
                      int grid, size_t lds, hipStream_t st) {
    if (op == EXS_SUM) launch_kind<T, OpSum>(kind, kb, steps, table, units, grid, lds, st);
    else if (op == EXS_MAX) launch_kind<T, OpMax>(kind, kb, steps, table, units, grid, lds, st);
    else launch_kind<T, OpMin>(kind, kb, steps, table, units, grid, lds, st);
}

void launch_worklist(int dtype, int op, int kind, int kb, const void* steps, const int* table,
                     i64 units, int grid, size_t lds, hipStream_t st) {
    const Step* s = (const Step*)steps;
    switch (dtype) {
        case EXS_F32: launch_op<float>(op, kind, kb, s, table, units, grid, lds, st); break;
        case EXS_F64: launch_op<double>(op, kind, kb, s, table, units, grid, lds, st); break;
        case EXS_I32: launch_op<int>(op, kind, kb, s, table, units, grid, lds, st); break;
        case EXS_I64: launch_op<long long>(op, kind, kb, s, table, units, grid, lds, st); break;
    }
}

}  // namespace exs
