// FP64 instantiations of the H.x kernels.
#include "hv_impl.hpp"

namespace ftlm {
template hipError_t launch_hv_typed<double>(const SectorDev&, const BondTable&, const HvLaunch&, hipStream_t);
template hipError_t launch_lanczos_typed<double>(int, int, const LanczosLaunch&, size_t,
                                                 hipStream_t);
}  // namespace ftlm
