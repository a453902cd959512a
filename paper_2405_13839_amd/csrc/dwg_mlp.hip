// Learned initial normals: MLP 48 -> 128 -> 128 -> 3 on MFMA (placeholder until the
// kernels land; every entry point reports DWG_E_UNSUPPORTED).
#include "dwg_internal.h"

namespace dwg {

size_t mlp_ws_bytes(int64_t B) { return align256((size_t)B * 4); }

dwg_status mlp_infer_run(const float*, const float*, int64_t, float*, void*, size_t, hipStream_t) {
  set_error("MLP kernels are not available in this build");
  return DWG_E_UNSUPPORTED;
}

dwg_status mlp_train_run(float*, float*, float*, int64_t, float, const float*, const float*,
                         const uint8_t*, int64_t, float*, float*, void*, size_t, hipStream_t) {
  set_error("MLP kernels are not available in this build");
  return DWG_E_UNSUPPORTED;
}

}  // namespace dwg
