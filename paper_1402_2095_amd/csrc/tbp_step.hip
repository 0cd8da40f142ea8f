// Instantiations of the persistent temporally blocked sparse step.
#include "tbp_step.hpp"

namespace fth {
template <>
int launch_tbp_step<float>(const StepArgs<float>& a, const TbArgs<float>& tb, const StepLaunch& L, int KT, int k,
                           void* stream) {
    return launch_tbp_step_impl<float>(a, tb, L, KT, k, stream);
}
template <>
int launch_tbp_step<double>(const StepArgs<double>& a, const TbArgs<double>& tb, const StepLaunch& L, int KT, int k,
                            void* stream) {
    return launch_tbp_step_impl<double>(a, tb, L, KT, k, stream);
}
template <>
int tbp_resident_grid<float>(int ns, int KT, bool xtra, int block, size_t lds) {
    return tbp_resident_grid_impl<float>(ns, KT, xtra, block, lds);
}
template <>
int tbp_resident_grid<double>(int ns, int KT, bool xtra, int block, size_t lds) {
    return tbp_resident_grid_impl<double>(ns, KT, xtra, block, lds);
}
template <>
int launch_tb_slots<float>(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t N, void* out,
                           void* stream) {
    return launch_tb_slots_impl<float>(row_ptr, col, val, N, out, stream);
}
template <>
int launch_tb_slots<double>(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t N, void* out,
                            void* stream) {
    return launch_tb_slots_impl<double>(row_ptr, col, val, N, out, stream);
}
}  // namespace fth
