// Kernel instantiations of the moment-space collision models for D3Q27
// with f16 population storage.
#include "dispatch.hpp"

namespace lbm {
hipError_t launch_q27_f16_mrt(const Launch& L, hipStream_t s) { return launch_tu_moment_space<27, StoreF16>(L, s); }
}  // namespace lbm
