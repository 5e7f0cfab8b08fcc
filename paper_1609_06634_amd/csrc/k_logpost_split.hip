// Split-precision (matrix-core) form of the posterior kernel.
#include "common.hpp"

namespace bioem {

bool split_supported(int nx, int ny, int S) { (void)nx; (void)ny; (void)S; return false; }

hipError_t launch_logpost_split(hipStream_t s, const LogpostArgs& a, bool bf16) {
  (void)s; (void)a; (void)bf16;
  return hipErrorNotSupported;
}

}  // namespace bioem
