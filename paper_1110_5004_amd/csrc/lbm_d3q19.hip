// lbm_d3q19.hip -- gfx950 kernels of the D3Q19 form of the step (not built yet).
#include "lbm_dev.h"
#include "lbm_kernels.h"

namespace lbm {
const TileShape kD3Q19Tiles[] = {{32, 4, 4, 512}};
const int kD3Q19TileCount = 1;

hipError_t d3q19_step(int, const LaunchArgs&) { return hipErrorNotSupported; }
hipError_t d3q19_fields(const LaunchArgs&, const FieldPtrs&) { return hipErrorNotSupported; }
hipError_t d3q19_init(const CaseDev&, int, int, const double*, const double*, const double*,
                      hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace lbm
