// Placeholder: mixed-precision and complex GEMM paths.
#include "common.hpp"

namespace ccmi {
void gemm_lowp(const GemmDesc &, int, hipStream_t, int) {
  throw CCError(-6, "FP32 / BF16x3 contractions are not built yet");
}
void gemm_c128(const GemmDesc &, hipStream_t) {
  throw CCError(-6, "complex contractions are not built yet");
}
}  // namespace ccmi
