// Kernel instantiations for D3Q19 with f16 population storage.
#include "dispatch.hpp"

namespace lbm {
hipError_t launch_q19_f16(const Launch& L, hipStream_t s) { return launch_tu<19, StoreF16>(L, s, launch_q19_f16_mrt); }
}  // namespace lbm
