// Kernel instantiations for D3Q27 with f16 population storage.
#include "dispatch.hpp"

namespace lbm {
hipError_t launch_q27_f16(const Launch& L, hipStream_t s) { return launch_tu<27, StoreF16>(L, s, launch_q27_f16_mrt); }
}  // namespace lbm
