// Interfaces of the learned-proposal kernels (gd_learned.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace gd {

constexpr int kMlpF = 20;       // features per spin
constexpr int kMlpH = 64;       // hidden width
constexpr int kMlpOut = 2;      // outputs: sign logit, confidence logit
constexpr int kMlpNParam = kMlpF * kMlpH + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH * kMlpOut + kMlpOut;
constexpr unsigned long long kFeatKey = 0x5EED5EEDull;

struct FeatArgs {
    const int *inst_n;
    const long long *inst_spin;
    const float *inst_inv_s;
    const int *ell_idx;
    const float *ell_w;
    int dmax, nmax, iters;
    float *feats;    // [sum n][kMlpF]
    float *lambda;   // [K][8] eigenvalues of J/s (nullable)
    float *vecs;     // [sum n][8] sign-fixed Ritz vectors (nullable)
};

struct MlpTrainArgs {
    float *params, *mom, *vel;     // [kMlpNParam]
    const float *X;                // [M][F]
    const float *labels;           // [M] +-1
    const int *seg;                // [K+1] instance boundaries
    const int *spin_inst;          // [M] instance of each row
    int M;
    float *out;                    // [M][2]
    float *sigma;                  // [K]
    float *partial;                // [nparts][kMlpNParam] gradient partials of the training workgroups
    double *loss_part;             // [nparts] their loss partials
    float *grad_out;               // [kMlpNParam] (nullable)
    double *loss;                  // [1]
};

struct ProposeArgs {
    const int *inst_n;
    const long long *inst_spin, *inst_state;
    int K;
    long long total_state;
    const float *out;              // [sum n][2] network outputs
    float *x, *gam, *eps;          // batch solver state and per-spin eps
    unsigned long long seed;
    double amp, alpha, beta, eps0;
    float gamma0;
};

hipError_t launch_features(const FeatArgs &a, int K, hipStream_t st);
hipError_t launch_mlp_forward(const float *params, const float *X, float *out, int M, bool fp16,
                              hipStream_t st);
hipError_t launch_mlp_train_step(const MlpTrainArgs &a, int K, int nparts, float lr, int step,
                                 hipStream_t st);
hipError_t launch_propose(const ProposeArgs &a, hipStream_t st);

}  // namespace gd
