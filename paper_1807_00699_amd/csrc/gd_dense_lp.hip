// Reduced-precision coupling step (kernels and their description:
// gd_dense_lp.h): the variant table and the launcher of variants 0-6.
#include "gd_dense_lp.h"

namespace gd {

namespace {

constexpr int kLpCfg[][6] = {
#define GD_ROW(id, bm, bn, bk, wm, wn, dl) {bm, bn, bk, wm, wn, dl},
    GD_LP_VARIANTS(GD_ROW) GD_LP_BIG_VARIANTS(GD_ROW)
#undef GD_ROW
};

}  // namespace

int dense_lp_config_count() { return int(sizeof(kLpCfg) / sizeof(kLpCfg[0])); }

DenseConfig dense_lp_config(bool complex_mode, int idx) {
    DenseConfig c;
    c.id = idx;
    c.bm = kLpCfg[idx][0];
    c.bn = kLpCfg[idx][1];
    c.bk = kLpCfg[idx][2];
    c.wn = kLpCfg[idx][4];
    c.traj_tile = complex_mode ? c.bn / 2 : c.bn;
    c.threads = 64 * kLpCfg[idx][3] * kLpCfg[idx][4];
    if (kLpCfg[idx][5] > 0 && ((kLpCfg[idx][5] - 1) & 15)) c.min_np = 16 * 64;   // operand-load tail
    return c;
}

hipError_t launch_dense_step_lp(const DenseConfig &cfg, bool complex_mode, int mode, int op,
                                bool j_fp8, const DenseStepArgs &a, hipStream_t st) {
    if (op != OP_BF16 && op != OP_F16) return hipErrorInvalidValue;
#define GD_CASE(id, bm, bn, bk, wm, wn, dl) \
    case id: return launch_lp<bm, bn, bk, wm, wn, dl>(complex_mode, op, j_fp8, mode, a, st);
    switch (cfg.id) { GD_LP_VARIANTS(GD_CASE) }
#undef GD_CASE
    return launch_dense_step_lp_big(cfg, complex_mode, mode, op, j_fp8, a, st);
}

}  // namespace gd
