// Small-R coupling product (gd_gemv.h) with BF16 operands: J stored in FP8
// E4M3 (exact couplings) or in BF16, widened exactly to FP32, operands read
// from the BF16 copy of the amplitudes, FP32 sums.  FP16 operands:
// gd_gemv_f16.hip.
#include "gd_gemv.h"

namespace gd {

hipError_t launch_gemv_f16(int idx, bool complex_mode, int mode, bool j_fp8, const DenseStepArgs &a,
                           hipStream_t st);

hipError_t launch_gemv_lp(int idx, bool complex_mode, int mode, int op, bool j_fp8, const DenseStepArgs &a,
                          hipStream_t st) {
    if (op == OP_BF16)
        return j_fp8 ? gemv::launch_variant<gemv::J_FP8, OP_BF16>(idx, complex_mode, mode, a, st)
                     : gemv::launch_variant<gemv::J_B16, OP_BF16>(idx, complex_mode, mode, a, st);
    if (op == OP_F16) return launch_gemv_f16(idx, complex_mode, mode, j_fp8, a, st);
    return hipErrorInvalidValue;
}

}  // namespace gd
