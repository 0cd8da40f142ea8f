// Instantiations of the temporally blocked sparse step.
#include "tb_step.hpp"

namespace fth {
template <>
int launch_tb_step<float>(const StepArgs<float>& a, const TbArgs<float>& tb, const StepLaunch& L, int KT, int k,
                          void* stream) {
    return launch_tb_step_impl<float>(a, tb, L, KT, k, stream);
}
template <>
int launch_tb_step<double>(const StepArgs<double>& a, const TbArgs<double>& tb, const StepLaunch& L, int KT, int k,
                           void* stream) {
    return launch_tb_step_impl<double>(a, tb, L, KT, k, stream);
}
template <>
int launch_tb_pairs<float>(const StepArgs<float>& a, const TbArgs<float>& tb, const StepLaunch& L, int KT, int k,
                           void* stream) {
    return launch_tb_pairs_impl<float>(a, tb, L, KT, k, stream);
}
template <>
int launch_tb_pairs<double>(const StepArgs<double>& a, const TbArgs<double>& tb, const StepLaunch& L, int KT, int k,
                            void* stream) {
    return launch_tb_pairs_impl<double>(a, tb, L, KT, k, stream);
}
}  // namespace fth
