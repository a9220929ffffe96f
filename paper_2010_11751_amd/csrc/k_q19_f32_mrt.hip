// Kernel instantiations of the moment-space collision models for D3Q19
// with f32 population storage.
#include "dispatch.hpp"

namespace lbm {
hipError_t launch_q19_f32_mrt(const Launch& L, hipStream_t s) { return launch_tu_moment_space<19, StoreF32>(L, s); }
}  // namespace lbm
