// Kernel instantiations for D3Q19 with f64 population storage.
#include "dispatch.hpp"

namespace lbm {
hipError_t launch_q19_f64(const Launch& L, hipStream_t s) { return launch_tu<19, StoreF64>(L, s, launch_q19_f64_mrt); }
}  // namespace lbm
