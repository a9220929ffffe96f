// Kernel instantiations for D3Q19 with f32 population storage.
#include "dispatch.hpp"

namespace lbm {
hipError_t launch_q19_f32(const Launch& L, hipStream_t s) { return launch_tu<19, StoreF32>(L, s, launch_q19_f32_mrt); }
}  // namespace lbm
