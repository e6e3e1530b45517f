// Small-R coupling product (gd_gemv.h) of FP32 solvers whose couplings are
// all exact in FP8 E4M3: J streamed as one byte per coupling (J_FP8N: four per
// lane, where the FP32 kind reads sixteen bytes) and widened exactly to FP32,
// FP32 operands, sums and state: the results of the FP32 couplings bit for
// bit, with a quarter of the HBM traffic.
#include "gd_gemv.h"

namespace gd {

hipError_t launch_gemv_f32_j8(int idx, bool complex_mode, int mode, const DenseStepArgs &a, hipStream_t st) {
    return gemv::launch_variant<gemv::J_FP8N, OP_F32>(idx, complex_mode, mode, a, st);
}

}  // namespace gd
