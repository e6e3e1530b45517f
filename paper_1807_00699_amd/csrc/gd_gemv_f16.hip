// Small-R coupling product (gd_gemv.h) with FP16 operands: J stored in FP8
// E4M3 (exact couplings) or in FP16, widened exactly to FP32, operands read
// from the FP16 copy of the amplitudes, FP32 sums.
#include "gd_gemv.h"

namespace gd {

hipError_t launch_gemv_f16(int idx, bool complex_mode, int mode, bool j_fp8, const DenseStepArgs &a,
                           hipStream_t st) {
    return j_fp8 ? gemv::launch_variant<gemv::J_FP8, OP_F16>(idx, complex_mode, mode, a, st)
                 : gemv::launch_variant<gemv::J_B16, OP_F16>(idx, complex_mode, mode, a, st);
}

}  // namespace gd
