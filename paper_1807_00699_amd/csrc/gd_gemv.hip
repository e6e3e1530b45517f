// Small-R coupling product (gd_gemv.h): FP32 couplings and operands, and the
// host-side variant table.  The reduced-precision instantiations live in
// gd_gemv_lp.hip and gd_gemv_f16.hip, FP8-stored couplings with FP32
// operands in gd_gemv_f8.hip.
#include "gd_gemv.h"

namespace gd {

namespace {
constexpr int kGemvCfg[][5] = {
#define GD_ROW(id, w, rpw, bud, u, ks) {w, rpw, bud, u, ks},
    GD_GEMV_VARIANTS(GD_ROW)
#undef GD_ROW
};
}  // namespace

int gemv_config_count() { return int(sizeof(kGemvCfg) / sizeof(kGemvCfg[0])); }

DenseConfig gemv_config(int idx) {
    DenseConfig c{};
    c.id = kGemvBase + idx;
    c.bm = kGemvCfg[idx][0] / kGemvCfg[idx][4] * kGemvCfg[idx][1];
    c.bn = 16;
    c.bk = 0;
    c.wn = 1;
    c.traj_tile = 0;
    c.threads = 64 * kGemvCfg[idx][0];
    c.min_np = 32;
    return c;
}

bool gemv_fits(int idx, int Np, int R, bool complex_mode, int op, bool j_fp8) {
    if (idx < 0 || idx >= gemv_config_count()) return false;
    const int C = (complex_mode ? 2 : 1) * R;
    if (R < 1 || C > kGemvMaxCols || Np % 32) return false;
    const int jk = op == OP_F32 ? (j_fp8 ? gemv::J_FP8N : gemv::J_F32) : (j_fp8 ? gemv::J_FP8 : gemv::J_B16);
    return gemv::fits_registers(jk, gemv::column_capacity(C), kGemvCfg[idx][0]);
}

hipError_t launch_gemv_lp(int idx, bool complex_mode, int mode, int op, bool j_fp8, const DenseStepArgs &a,
                          hipStream_t st);
hipError_t launch_gemv_f32_j8(int idx, bool complex_mode, int mode, const DenseStepArgs &a, hipStream_t st);

hipError_t launch_gemv_step(const DenseConfig &cfg, bool complex_mode, int mode, int op, bool j_fp8,
                            const DenseStepArgs &a, hipStream_t st) {
    const int idx = cfg.id - kGemvBase;
    if (idx < 0 || idx >= gemv_config_count()) return hipErrorInvalidValue;
    if (op == OP_F32)
        return j_fp8 ? launch_gemv_f32_j8(idx, complex_mode, mode, a, st)
                     : gemv::launch_variant<gemv::J_F32, OP_F32>(idx, complex_mode, mode, a, st);
    return launch_gemv_lp(idx, complex_mode, mode, op, j_fp8, a, st);
}

}  // namespace gd
