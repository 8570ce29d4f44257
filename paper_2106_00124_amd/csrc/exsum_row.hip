// exsum_row.hip -- the fused 2-D streaming kernel instantiated for 4-byte
// element types, and the planner's eligibility test for it.
#include "exsum_row.hpp"

namespace exs {

bool row_eligible(i64 n0, i64 NX, i64 k0, i64 kx, int es) {
    if (es != 4 || k0 > 16 || kx > 16) return false;
    if (n0 + 64 >= ((i64)1 << 31)) return false;
    // byte offsets within two blocks of rows are 32-bit
    if (NX * es * 32 >= ((i64)1 << 32)) return false;
    // rows short against the 256-point tile leave it mostly idle
    return (double)NX / ((double)row_tiles(NX, kx) * 256.0) >= 0.25;
}

i64 row_axis0_run_blocks(i64 Q, i64 NX, i64 kx) { return row_run_blocks(Q, NX, kx); }

template void launch_row_axis0<float, OpSum>(const float*, const float*, const float*, const float*,
                                             float*, float*, i64, i64, i64, i64, i64, hipStream_t);
template void launch_row_axis0<float, OpMax>(const float*, const float*, const float*, const float*,
                                             float*, float*, i64, i64, i64, i64, i64, hipStream_t);
template void launch_row_axis0<int, OpSum>(const int*, const int*, const int*, const int*, int*,
                                           int*, i64, i64, i64, i64, i64, hipStream_t);
template void launch_row_axis0<int, OpMax>(const int*, const int*, const int*, const int*, int*,
                                           int*, i64, i64, i64, i64, i64, hipStream_t);
template void launch_row_axis0<float, OpMin>(const float*, const float*, const float*, const float*,
                                             float*, float*, i64, i64, i64, i64, i64, hipStream_t);
template void launch_row_axis0<int, OpMin>(const int*, const int*, const int*, const int*, int*,
                                           int*, i64, i64, i64, i64, i64, hipStream_t);
template void launch_row_axis0<float, OpSlowSum>(const float*, const float*, const float*,
                                                 const float*, float*, float*, i64, i64, i64, i64,
                                                 i64, hipStream_t);
hipError_t slow_cost_set_row(int c) { return set_slow_cost_here(c); }

}  // namespace exs
