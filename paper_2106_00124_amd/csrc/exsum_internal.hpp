// exsum_internal.hpp -- declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/exsum.h"

typedef long long i64;

namespace exs {

struct OpSum;
struct OpMax;
struct OpMin;
struct OpSlowSum;  // fp32 + with an artificial cost per application (measurement)

// per translation unit: write that unit's copy of the slowed operator's cost
hipError_t slow_cost_set_kernels(int c);
hipError_t slow_cost_set_plane(int c);
hipError_t slow_cost_set_row(int c);
hipError_t slow_cost_set_ex1d(int c);
hipError_t slow_cost_set_tailbox(int c);
// the slowed operator applied reps times to each of n elements (time per op)
void launch_op_probe(float* data, i64 n, int reps, hipStream_t st);

// A struct element: a value with the index of where it came from.  Ordered
// by value, and among equal values the lower index first; max of that total
// order is "argmax" (the largest value and the first place it occurs), min is
// "argmin".  Both are commutative and associative, so they are monoids in the
// sense of Sec. 2 and the box-complement reordering applies; the identity is
// the pair that comes last: (-inf, INT32_MAX) for max, (+inf, INT32_MAX) for
// min.  Eight bytes, laid out as { float value; int32 index; }.
struct __align__(8) ValIdx {
    float v;
    int i;
};
static_assert(sizeof(ValIdx) == 8, "ValIdx is { float; int32; }");

// register bucket (power of two >= k, up to 64) of a box length; 0 = none
inline int bucket_for(i64 k) {
    if (k <= 1) return 1;
    if (k <= 2) return 2;
    if (k <= 4) return 4;
    if (k <= 8) return 8;
    if (k <= 16) return 16;
    if (k <= 32) return 32;
    if (k <= 64) return 64;
    return 0;
}

// work-list launch of the batched form (exsum_worklist.hip): `steps` is a
// device array of Step (exsum_tasks.hpp) whose tasks start at multiples of
// WL_CHUNK; `table` names the step of each of the `units` chunks (of each
// task, for the row kind SK_BDBSR).  One launch serves the steps of one kind
// and register bucket over every element type of size `es` (4 or 8) and
// every operator: its chunks are sorted by (type, operator) into up to six
// parts, and each part gets its own share of the workgroups, so that a
// workgroup runs the code of one type and operator only.
constexpr int WL_CHUNK = 256;
constexpr int WL_MAX_PARTS = 6;
struct WlParts {
    int n;                       // parts of the launch (1..WL_MAX_PARTS)
    int code[WL_MAX_PARTS];      // dtype * 4 + op of each part (EXS_* codes)
    i64 unit0[WL_MAX_PARTS + 1]; // first chunk (row task) of each part; unit0[n] = all
    int wg0[WL_MAX_PARTS + 1];   // first workgroup of each part; wg0[n] = the grid
};
void launch_worklist(int es, int kind, int kb, const void* steps, const int* table,
                     const WlParts& parts, size_t lds, hipStream_t st);

// generic-path launchers (exsum_kernels.hip)
template <typename T, class Op>
void launch_bdbs(const T* in, T* out, i64 O, i64 n, i64 I, i64 k, hipStream_t st);
// weak excluded sums (+ only): the total of the tensor in two deterministic
// stages (partials in `parts`, TOT_PARTS 8-byte slots), the fused stream kernel
// with the total - included epilogue, and the same epilogue as its own pass
constexpr int TOT_PARTS = 1024;
template <typename T>
void launch_total(const T* X, i64 N, void* parts, T* tot, hipStream_t st);
template <typename T, class Op>
void launch_plane_weak(const T* X, T* inc, const T* wtot, T* wexc, i64 n0, i64 MID, i64 NY,
                       i64 NX, i64 k0, i64 ky, i64 kx, hipStream_t st);
template <typename T>
void launch_weak_exc(const T* inc, const T* tot, T* exc, i64 N, hipStream_t st);
// fused 2-D streaming kernel (exsum_row.hpp)
bool row_eligible(i64 n0, i64 NX, i64 k0, i64 kx, int es);
// blocks of axis 0 per run of the 2-D streaming kernel (it reads the block
// prefix only where its runs start)
i64 row_axis0_run_blocks(i64 Q, i64 NX, i64 kx);
template <typename T, class Op>
void launch_row_axis0(const T* X, const T* PX, const T* SX, const T* Trest, T* exc, T* inc, i64 n0,
                      i64 NX, i64 k0, i64 kx, i64 Q, hipStream_t st);
// segmented block scans (few points, many blocks)
template <typename T, class Op>
void launch_segtot(const T* Gw, const T* Ga, T* Tw, T* Ta, i64 Q, i64 M, i64 L, hipStream_t st);
template <typename T, class Op>
void launch_segexp(const T* Gw, const T* SPX, const T* SSX, T* PX, T* SX, i64 Q, i64 M, i64 L,
                   i64 pxe, hipStream_t st);
// excluded sums of a 1-D tensor of at most 8192 elements in one workgroup
bool ex1d_small_ok(i64 n);
// both levels of a small rank-2 tensor in one workgroup (exsum_small2d.hip):
// at most SMALL2D_MAX_N0 x SMALL2D_MAX_N1 elements and SMALL2D_BYTES bytes,
// boxes along axis 1 of at most SMALL2D_MAX_K1
constexpr int SMALL2D_BYTES = 32768, SMALL2D_MAX_N0 = 128, SMALL2D_MAX_N1 = 1024,
              SMALL2D_MAX_K1 = 64;
bool small2d_eligible(i64 n0, i64 n1, i64 k0, i64 k1, int es);
template <typename T, class Op>
void launch_small2d(const T* A, T* exc, T* inc, i64 n0, i64 n1, i64 k0, i64 k1, hipStream_t st);
template <typename T, class Op>
void launch_ex1d_small(const T* R, T* exc, i64 n, i64 k, hipStream_t st);
template <typename T, class Op>
void launch_blockagg(const T* X, T* Ga, i64 n0, i64 M, i64 k0, i64 Q, hipStream_t st);
// block aggregates along axis 0 fused with BDBS along the middle axis f of an
// (n0, P, nf, S) tensor (kf from 2 to 16): X = BDBS_f(A), Ga, G1 = BDBS_f(Ga)
template <typename T, class Op>
void launch_aggmid(const T* A, T* X, T* Ga, T* G1, i64 n0, i64 P, i64 nf, i64 S, i64 k0, i64 kf,
                   i64 Q, hipStream_t st);
// (PX stored for the blocks q with q % pxe == 0 only)
template <typename T, class Op>
void launch_blockscan(const T* Gw, const T* Ga, T* PX, T* SX, T* R, i64 Q, i64 M, i64 pxe,
                      hipStream_t st);
// Boxes longer than 64 along an axis take per-column sweeps; with few columns
// the sweeps go in chunks of rows (ex2_chunks: chunks per column, 1 for the
// plain per-column sweep), the axis-0 stream's needing C x M chunk totals of
// workspace (ex2t)
inline i64 ex2_chunks(i64 n, i64 cols) {
    if (cols >= ((i64)1 << 20)) return 1;
    i64 c = (((i64)1 << 20) + cols - 1) / cols;
    const i64 cmax = (n + 63) / 64;  // chunks of at least 64 rows
    if (c > cmax) c = cmax;
    return c < 1 ? 1 : c;
}
template <typename T, class Op>
void launch_axis0(const T* W, const T* PX, const T* SX, const T* Trest, T* exc, T* inc, i64 n0,
                  i64 M, i64 k0, i64 Q, T* ex2t, hipStream_t st);
template <typename T, class Op>
void launch_plane_axis0(const T* X, const T* PX, const T* SX, const T* Trest, T* exc, T* inc,
                        i64 n0, i64 MID, i64 NY, i64 NX, i64 k0, i64 ky, i64 kx, i64 Q,
                        hipStream_t st);
bool plane_eligible(int d, const i64* n, const i64* k, int es);
template <typename T, class Op>
void launch_plane_bdbs(const T* X, T* W, i64 O, i64 NY, i64 NX, i64 ky, i64 kx, hipStream_t st);
bool plane2_eligible(i64 NY, i64 NX, i64 ky, i64 kx, int es);
template <typename T, class Op>
void launch_plane_scan(const T* G, const T* Ga, T* PX, T* SX, T* R, T* A1, i64 Q, i64 MID,
                       i64 NY, i64 NX, i64 ky, i64 kx, i64 pxe, hipStream_t st);
// BDBS along the last m axes in one pass, for trailing sub-tensors of at most
// tail_box_max_elems(es) elements (n, k: the m extents and box sides)
i64 tail_box_max_elems(int es);
template <typename T, class Op>
void launch_bdbs_tail(const T* in, T* out, i64 O, int m, const i64* n, const i64* k,
                      hipStream_t st);
// excluded and/or included sums of a long 1-D level in chunks (4-byte
// elements, k <= 16): chunk totals, their scans, the chunk pass; the four
// scratch arrays hold long1d_chunks(n, k) elements each (unused, and may be
// null, when exc is null: the included sums need only the chunk pass)
bool long1d_ok(i64 n, i64 k);
i64 long1d_chunks(i64 n, i64 k);
template <typename T, class Op>
void launch_long1d(const T* A, T* exc, T* inc, i64 n, i64 k, T* Tt, T* Ut, T* CP, T* CS,
                   hipStream_t st);
// the last two levels of a rank-3 tensor from its level-1 block aggregates
// (Q x n table, 4-byte elements) in one workgroup
bool tail_scan_ok(i64 Q, i64 n, i64 k);
template <typename T, class Op>
void launch_tail_scan(const T* A1, T* PX, T* SX, T* exc2, i64 Q, i64 n, i64 k, i64 pxe,
                      hipStream_t st);
// blocks of axis 0 per run of the level-0 streaming kernel (the runs start
// at multiples of it: the only blocks whose prefix it reads)
i64 plane_axis0_run_blocks(i64 Q, i64 MID, i64 NY, i64 NX, i64 ky, i64 kx);
void launch_fill(void* out, i64 count, int dtype, int kind, uint64_t seed, i64 lo, i64 hi,
                 float scale, hipStream_t st);

// per-kernel event timing (exsum_api.cpp); a no-op unless enabled.  The
// planner tags launches with the recursion level they belong to.
void set_timing_tag(int level);
struct KTimer {
    int slot;
    hipStream_t st;
    KTimer(const char* name, hipStream_t stream);
    ~KTimer();
};

// error plumbing (exsum_api.cpp)
exs_status set_error(exs_status s, const std::string& msg);
size_t dtype_size(int dtype);
exs_status validate_job(const exs_job* job, bool check_ptrs);

}  // namespace exs
