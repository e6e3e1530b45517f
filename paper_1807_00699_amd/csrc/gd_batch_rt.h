// Host interface of the batched sparse solver (gd_batch_rt.hip); used by the
// C ABI in gd_runtime.hip.  Not part of the public header.
#pragma once
#include "../../include/gd.h"

#include <cstdint>

#include <hip/hip_runtime.h>

namespace gd {

struct BatchSolver;

int batch_create(BatchSolver **out, int count, const gd_instance *inst, int model, const gd_params *p);
void batch_destroy(BatchSolver *b);
int batch_set_init(BatchSolver *b, int R, const float *psi0, const float *gamma0, const float *eps);
int batch_run(BatchSolver *b, int R, int64_t steps);
int batch_energy(BatchSolver *b, double *E, int32_t *best);
int batch_spins(BatchSolver *b, void *out, int fmt);
int batch_get_state(BatchSolver *b, float *psi, float *gamma, int64_t *step);
int batch_set_state(BatchSolver *b, int R, const float *psi, const float *gamma, int64_t step);
int batch_stats(BatchSolver *b, gd_run_stats *out);
// out[k * R + r] = 1 if trajectory r of instance k became non-finite, else 0
int batch_trajectory_status(BatchSolver *b, int32_t *out, int64_t count);
int batch_set_targets(BatchSolver *b, const double *targets);
int batch_ttt(BatchSolver *b, double *seconds, int64_t *steps, double *best_energy);
int batch_count(const BatchSolver *b);

// Device view of a batch solver for the learned-proposal kernels.
struct BatchView {
    int K, dmax, nmax, R;
    long long total;
    const int *d_n;
    const long long *d_spin, *d_state;
    const float *d_inv_s;
    const int *d_idx;
    const float *d_w;
    float *d_eps, *d_x, *d_gam;
    hipStream_t stream;
    double eps0, gamma0, amp;
};
int batch_view(BatchSolver *b, BatchView *v);
// allocate the state for R trajectories (contents undefined), reset statistics
int batch_prepare_state(BatchSolver *b, int R);
// after x, gamma and eps were written on the device: pick the kernel variant
int batch_finish_init(BatchSolver *b);
double batch_scale(const BatchSolver *b, int k);

}  // namespace gd
