// vsm_k_f64.hip -- FP64 instantiation of the smoothing kernels.
#include "vsm_kernels_impl.h"

namespace vsm {
template void launch_set_links_t<double>(const Geo&, const void*, void*, hipStream_t);
template void launch_get_links_t<double>(const Geo&, const void*, void*, hipStream_t);
template void launch_load_z3_t<double>(const Geo&, const int8_t*, void*, hipStream_t);
template void launch_centrifuge_t<double>(const Geo&, const int8_t*, const int8_t*, double, void*, int32_t*,
                                     hipStream_t);
template void launch_gauge_t<double>(const Geo&, void*, const void*, hipStream_t);
template void launch_update_t<double>(const Geo&, const void*, void*, const int8_t*, const void*,
                                 const UpdParams&, int, int, int, unsigned long long*, hipStream_t);
template void launch_measure_t<double>(const Geo&, const void*, const int8_t*, const void*, void*, int8_t*,
                                  unsigned long long*, VsmStatsDev*, long long, hipStream_t);
template void launch_update_batch_t<double>(const ServeJob*, const BatchStep&, uint32_t, hipStream_t);
template void launch_serve_small_t<double>(const ServeJob*, const SmallStep&, hipStream_t);
template void launch_clover_t<double>(const Geo&, const void*, void*, double*, double*, double*, hipStream_t);
template void launch_flow_t<double>(const Geo&, const void*, void*, double*, int, double, double, double, hipStream_t);
}  // namespace vsm
