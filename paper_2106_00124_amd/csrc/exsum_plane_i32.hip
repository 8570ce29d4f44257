// exsum_plane_i32.hip -- fused plane kernel instantiated for int32.
#include "exsum_plane.hpp"

namespace exs {
template void launch_plane_axis0<int, OpSum>(const int*, const int*, const int*, const int*, int*,
                                             int*, i64, i64, i64, i64, i64, i64, i64, i64,
                                             hipStream_t);
template void launch_plane_axis0<int, OpMax>(const int*, const int*, const int*, const int*, int*,
                                             int*, i64, i64, i64, i64, i64, i64, i64, i64,
                                             hipStream_t);
template void launch_plane_axis0<int, OpMin>(const int*, const int*, const int*, const int*, int*,
                                             int*, i64, i64, i64, i64, i64, i64, i64, i64,
                                             hipStream_t);
template void launch_plane_bdbs<int, OpSum>(const int*, int*, i64, i64, i64, i64, i64,
                                             hipStream_t);
template void launch_plane_bdbs<int, OpMax>(const int*, int*, i64, i64, i64, i64, i64,
                                             hipStream_t);
template void launch_plane_bdbs<int, OpMin>(const int*, int*, i64, i64, i64, i64, i64,
                                             hipStream_t);
template void launch_plane_scan<int, OpSum>(const int*, const int*, int*, int*, int*, int*, i64, i64,
                                            i64, i64, i64, i64, i64, hipStream_t);
template void launch_plane_scan<int, OpMax>(const int*, const int*, int*, int*, int*, int*, i64, i64,
                                            i64, i64, i64, i64, i64, hipStream_t);
template void launch_plane_scan<int, OpMin>(const int*, const int*, int*, int*, int*, int*, i64, i64,
                                            i64, i64, i64, i64, i64, hipStream_t);
template void launch_plane_weak<int, OpSum>(const int*, int*, const int*, int*, i64, i64, i64, i64,
                                            i64, i64, i64, hipStream_t);
}  // namespace exs
