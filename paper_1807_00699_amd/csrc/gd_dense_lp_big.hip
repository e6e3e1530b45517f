// Reduced-precision coupling step, the larger workgroup tiles (variants
// 7-13 of gd_dense_lp.h), in a translation unit of their own.
#include "gd_dense_lp.h"

namespace gd {

hipError_t launch_dense_step_lp_big(const DenseConfig &cfg, bool complex_mode, int mode, int op,
                                    bool j_fp8, const DenseStepArgs &a, hipStream_t st) {
    if (op != OP_BF16 && op != OP_F16) return hipErrorInvalidValue;
#define GD_CASE(id, bm, bn, bk, wm, wn, dl) \
    case id: return launch_lp<bm, bn, bk, wm, wn, dl>(complex_mode, op, j_fp8, mode, a, st);
    switch (cfg.id) { GD_LP_BIG_VARIANTS(GD_CASE) }
#undef GD_CASE
    return hipErrorInvalidValue;
}

}  // namespace gd
