// exsum_plane_f32.hip -- fused plane kernel instantiated for float, and the
// planner's eligibility test for it.
#include "exsum_plane.hpp"

namespace exs {

// Share of the tiles' thread slots that hold a point of the plane: tiny
// planes leave most of a 32 x 32 tile idle, and the generic passes do better.
static double plane_fill(i64 NY, i64 NX, i64 ky, i64 kx) {
    return (double)(NY * NX) / ((double)plane_tiles(NY, NX, ky, kx) * 1024.0);
}

bool plane_eligible(int d, const i64* n, const i64* k, int es) {
    if (d < 3 || es != 4) return false;
    if (k[0] > 16 || k[d - 2] > 16 || k[d - 1] > 16) return false;
    if (plane_fill(n[d - 2], n[d - 1], k[d - 2], k[d - 1]) < 0.25) return false;
    // plane and block indices are 32-bit inside the kernel
    if (n[0] + 64 >= ((i64)1 << 31)) return false;
    if (n[d - 2] * n[d - 1] >= ((i64)1 << 31)) return false;
    // byte offsets within two blocks of planes are 32-bit
    i64 M = 1;
    for (int i = 1; i < d; ++i) M *= n[i];
    if (M * es * 32 >= ((i64)1 << 32)) return false;
    return true;
}

i64 plane_axis0_run_blocks(i64 Q, i64 MID, i64 NY, i64 NX, i64 ky, i64 kx) {
    return plane_run_blocks(Q, plane_tiles(NY, NX, ky, kx) * MID);
}

bool plane2_eligible(i64 NY, i64 NX, i64 ky, i64 kx, int es) {
    return es == 4 && ky <= 16 && kx <= 16 && NY * NX * es < ((i64)1 << 31) &&
           plane_fill(NY, NX, ky, kx) >= 0.25;
}

template void launch_plane_axis0<float, OpSum>(const float*, const float*, const float*,
                                               const float*, float*, float*, i64, i64, i64, i64,
                                               i64, i64, i64, i64, hipStream_t);
template void launch_plane_axis0<float, OpMax>(const float*, const float*, const float*,
                                               const float*, float*, float*, i64, i64, i64, i64,
                                               i64, i64, i64, i64, hipStream_t);
template void launch_plane_axis0<float, OpMin>(const float*, const float*, const float*,
                                               const float*, float*, float*, i64, i64, i64, i64,
                                               i64, i64, i64, i64, hipStream_t);
template void launch_plane_bdbs<float, OpSum>(const float*, float*, i64, i64, i64, i64, i64,
                                             hipStream_t);
template void launch_plane_bdbs<float, OpMax>(const float*, float*, i64, i64, i64, i64, i64,
                                             hipStream_t);
template void launch_plane_bdbs<float, OpMin>(const float*, float*, i64, i64, i64, i64, i64,
                                             hipStream_t);
template void launch_plane_scan<float, OpSum>(const float*, const float*, float*, float*, float*, float*, i64, i64,
                                            i64, i64, i64, i64, i64, hipStream_t);
template void launch_plane_scan<float, OpMax>(const float*, const float*, float*, float*, float*, float*, i64, i64,
                                            i64, i64, i64, i64, i64, hipStream_t);
template void launch_plane_scan<float, OpMin>(const float*, const float*, float*, float*, float*, float*, i64, i64,
                                            i64, i64, i64, i64, i64, hipStream_t);
template void launch_plane_axis0<float, OpSlowSum>(const float*, const float*, const float*,
                                                   const float*, float*, float*, i64, i64, i64,
                                                   i64, i64, i64, i64, i64, hipStream_t);
template void launch_plane_bdbs<float, OpSlowSum>(const float*, float*, i64, i64, i64, i64, i64,
                                                  hipStream_t);
template void launch_plane_scan<float, OpSlowSum>(const float*, const float*, float*, float*,
                                                  float*, float*, i64, i64, i64, i64, i64, i64,
                                                  i64, hipStream_t);
hipError_t slow_cost_set_plane(int c) { return set_slow_cost_here(c); }
template void launch_plane_weak<float, OpSum>(const float*, float*, const float*, float*, i64, i64,
                                              i64, i64, i64, i64, i64, hipStream_t);
}  // namespace exs
