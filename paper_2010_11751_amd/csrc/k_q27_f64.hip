// Kernel instantiations for D3Q27 with f64 population storage.
#include "dispatch.hpp"

namespace lbm {
hipError_t launch_q27_f64(const Launch& L, hipStream_t s) { return launch_tu<27, StoreF64>(L, s, launch_q27_f64_mrt); }
}  // namespace lbm
