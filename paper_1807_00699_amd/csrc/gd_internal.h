// Internal interfaces between the host runtime and the gfx950 kernels of
// libgd.so.  Not part of the public ABI (include/gd.h).
#pragma once
#include <vector>
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gd {

// Records `msg` as the calling thread's last error and returns `code`.
int gd_fail(int code, const char *msg);

// Epilogue of the dense coupling kernel.
enum StepMode : int {
    MODE_EULER = 0,   // psi_out = psi + dt f, gamma += dt phi
    MODE_RK1 = 1,     // k1; acc = k1; stage = y + dt/2 k1
    MODE_RK2 = 2,     // k2; acc += 2 k2; stage = y + dt/2 k2
    MODE_RK3 = 3,     // k3; acc += 2 k3; stage = y + dt k3
    MODE_RK4 = 4,     // k4; y += dt/6 (acc + k4)
    MODE_ENERGY = 5,  // per-trajectory partial sums of Eq. (h) over a row tile
};

// Operand precision of the coupling product.
enum OperandKind : int { OP_F32 = 0, OP_BF16 = 1, OP_F16 = 2 };

// Row tile of every dense kernel and the padding unit of n.
constexpr int kRowTile = 64;

// All pointers are device pointers.  Per-trajectory arrays are "planes" of
// [Rp][Np] floats (trajectory-major, spin contiguous, zero padded); complex
// amplitudes use two consecutive planes (re, im) of plane_stride floats.
struct DenseStepArgs {
    const void *J;         // [Np][Np] coupling, operand precision (FP32 / BF16 / FP16)
    const void *B;         // GEMM operand planes (FP32, or BF16/FP16 shadow)
    const float *psi_in;   // stage-input amplitudes at (r, i) (FP32 planes)
    float *psi_out;        // output amplitudes (next stage / next step)
    void *shadow_out;      // reduced-precision copy of psi_out for the next GEMM (or null)
    const float *gam_in;   // stage-input gains
    float *gam_out;        // output gains (may alias gam_in)
    const float *y_psi;    // RK4: amplitudes at the start of the step
    const float *y_gam;    // RK4: gains at the start of the step
    float *acc_psi;        // RK4: k1 + 2 k2 + 2 k3 accumulators
    float *acc_gam;
    const float *eps;      // [Np] per-spin gain rates
    const float *h1;       // [Np] q = 1 resonant term h_1i (zero padded)
    const float *g;        // [Np] external field g_i (energy mode)
    int *flags;            // [Rp] nonzero when trajectory r became non-finite
    double *partial;       // energy mode: [n_row_tiles][Rp]
    long long plane_stride;
    int Np, Rp, n, R;
    float inv_s, dt, gamma_c, rho_th;
    // resonant term h_q conj(Psi)^(q-1) of the complex models (q = 0: none)
    int q;
    float hq;
    // noise of the step's final stage: noise_amp = D sqrt(dt) (0: none),
    // noise_key = SplitMix64 key of this step
    float noise_amp;
    unsigned long long noise_key;
    // energy mode: weight of the second plane's product (3/4 for the q = 3, 6
    // clock states, whose second plane holds sin(theta) / (sqrt(3)/2))
    float im_weight;
};

// Kernel variants of the dense path.  traj_tile = trajectories per workgroup.
struct DenseConfig {
    int id;
    int bm;        // rows per workgroup (the energy partials use row tiles of bm)
    int bn;        // GEMM columns per workgroup
    int bk;        // K chunk per pipeline stage
    int wn;        // waves along the column dimension
    int traj_tile; // trajectories per workgroup
    int threads;
    int min_np = 0; // smallest padded size the variant runs
};

int dense_config_count(bool complex_mode);
DenseConfig dense_config(bool complex_mode, int idx);
bool dense_config_fits(const DenseConfig &c, int Np, int Rp);

hipError_t launch_dense_step(const DenseConfig &cfg, bool complex_mode, int mode, int op,
                             const DenseStepArgs &a, hipStream_t st);

// Reduced-precision variants (gd_dense_lp.hip): BF16/FP16 operands, FP32
// accumulation; J either in the operand type or FP8 E4M3 (j_fp8).
int dense_lp_config_count();
DenseConfig dense_lp_config(bool complex_mode, int idx);
hipError_t launch_dense_step_lp(const DenseConfig &cfg, bool complex_mode, int mode, int op,
                                bool j_fp8, const DenseStepArgs &a, hipStream_t st);

// ---- small-R coupling product (gd_gemv.hip): a J-streaming matrix-vector
// kernel for at most kGemvMaxCols GEMM columns (R real or 2R complex), with
// the same modes and epilogue as the dense kernels.  Its variants carry ids
// kGemvBase + index next to the dense ones; bm = rows per workgroup (16 or
// 32, the row tile of its energy partials).
constexpr int kGemvBase = 100;
constexpr int kGemvMaxCols = 16;
int gemv_config_count();
DenseConfig gemv_config(int idx);
// variant idx runs C = R (real) or 2R (complex) columns at Np spins with
// operand kind op and FP8-stored J
bool gemv_fits(int idx, int Np, int R, bool complex_mode, int op, bool j_fp8);
hipError_t launch_gemv_step(const DenseConfig &cfg, bool complex_mode, int mode, int op, bool j_fp8,
                            const DenseStepArgs &a, hipStream_t st);

// ---- GD-mod (gd_mod.hip): one Euler step with per-trajectory couplings K
// [R][Np][Np] (updated in place); c_hat = dt * eps_hat.  Needs Np % 16 == 0
// and gdmod_lds_bytes <= 64 KiB.
size_t gdmod_lds_bytes(bool complex_mode, int Np);
hipError_t launch_gdmod(bool complex_mode, const DenseStepArgs &a, const float *J, float *K, float c_hat,
                        hipStream_t st);

// ---- batched sparse solver (gd_batch.hip)
struct BatchArgs {
    const int *inst_n;            // [K] spins per instance
    const long long *inst_spin;   // [K] offset of the instance's spins in per-spin arrays
    const long long *inst_state;  // [K] offset of the instance's [R][n] state block
    const float *inst_inv_s;      // [K] 1 / coupling scale
    const int *ell_idx;           // [sum n][dmax] local neighbour indices (padding: 0)
    const float *ell_w;           // [sum n][dmax] couplings (padding: 0)
    // packed form (dmax <= 3, one coupling magnitude per instance, n_max < 2^16 - 1):
    // [sum n][2] words, word 0 = idx0 | idx1 << 16, word 1 = idx2 | neg2 << 29 |
    // neg1 << 30 | neg0 << 31 (neg: coupling -mag, else +mag); a missing
    // coupling has index n_k (the instance's size), an amplitude row that holds zeros
    const unsigned int *ell_pack;
    const float *inst_wmag;       // [K] the magnitude of instance k's couplings
    const int *inst_tlog;         // [K] per-instance-width variants: log2 of instance k's item width
    // per-instance-width variants: spins relabeled per instance for the LDS
    // gathers (label = LDS row and slot of a spin): label of spin i, spin of
    // label p (both [sum n], instance-local values), and the packed
    // neighbours in label order with labels as indices ([sum n][2] words)
    const int *tw_label, *tw_spin;
    const unsigned int *tw_pack;
    const float *eps, *h1, *g;    // [sum n]
    float *x, *gam;               // state [sum_k R n_k]
    double *E;                    // [K][R] energies after the launch
    int *flags;                   // [K][R] non-finite flags
    const int *wg_off;            // [nwg + 1] item ranges per workgroup
    const int *items;             // item = k * nslices + slice (per-instance widths: k * R + first trajectory)
    int nslices, R, dmax, nmax, steps;
    float dt, gamma_c, rho_th;
    float eps0;                   // the rate of every spin, for variants that need uniform eps and no field
};

struct BatchConfig {
    int id;
    int traj;     // trajectories per work item (0: chosen per instance, at most 64)
    int threads;  // workgroup size
    int slots;    // spins per thread (n_max <= slots * threads / traj)
    bool packed;  // neighbours in registers from the packed form (LDS: amplitudes only)
    bool uniform; // one eps for every spin and no field (eps0, h_1 = 0): no per-slot constants
    bool dbuf;    // amplitudes double-buffered in LDS (packed form): one barrier per step
};

int batch_config_count();
BatchConfig batch_config(int idx);
size_t batch_lds_bytes(const BatchConfig &c, int nmax, int dmax);
int batch_item_capacity(const BatchConfig &c);   // spin-trajectories of one item (slots x threads)
// resident workgroups per CU of a variant (registers, LDS and threads)
int batch_occupancy(const BatchConfig &c, int nmax, int dmax);

// ---- persistent tuner cache (gd_tune_cache.hip; GD_AUTOTUNE_CACHE=<file>)
// the variant id stored for (kind, key) by this or an earlier process on the
// same device and library build, or -1
int tune_cache_lookup(const char *kind, const std::vector<long long> &key);
void tune_cache_store(const char *kind, const std::vector<long long> &key, int id);
hipError_t prepare_batch(const BatchConfig &c, int nmax, int dmax);   // once per variant, outside capture
hipError_t launch_batch(const BatchConfig &c, int nwg, const BatchArgs &a, hipStream_t st);
// Per instance k < K: (best_E[k], best_r[k]) takes the lowest E[k * R + r]
// (ties -> lowest r) when it is strictly lower
hipError_t launch_batch_best(const double *E, int K, int R, double *best_E, int *best_r, hipStream_t st);

// ---- auxiliary kernels (gd_aux.hip)
// user [R][n] (or [R][n][2]) -> zero-padded planes [P][Rp][Np]
hipError_t launch_pack_planes(const float *user, float *planes, int n, int R, int Np, int Rp,
                              int nplanes, hipStream_t st);
hipError_t launch_unpack_planes(const float *planes, float *user, int n, int R, int Np, int Rp,
                                int nplanes, hipStream_t st);
// Readout of the amplitudes onto the spin domain of Eq. (h).
enum Readout {
    RO_SIGN = 0,     // real Ising: d = sign(x), sign(+-0) = +1
    RO_PHASOR = 1,   // XY: d = Psi / |Psi| (Psi = 0 -> 1)
    RO_SIGN_RE = 2,  // complex Ising: d = sign(Re Psi)
    RO_CLOCK = 3     // q-state clock: k = floor(q arg(Psi) / 2pi + 1/2) mod q,
                     // d = (cos 2pi k/q, sin 2pi k/q), second plane scaled as
                     // clock_im_weight describes
};
// 3/4 for q = 3 and 6 (the second plane then holds sin / (sqrt(3)/2) in
// {0, +-1}, exact), 1 otherwise
float clock_im_weight(int q);
// Discretised state planes D (and its operand copy), zero outside n x R.
// Optional outputs (null to skip): spins8 [R][n] int8, angle [R][n] float in
// [0, 2pi) of the discretised state, states [R][n] int32 (RO_CLOCK).
// flags[r] set on NaN.
hipError_t launch_discretise(const float *psi, float *D, void *shadowD, int op, int readout, int q,
                             int8_t *spins8, float *angle, int32_t *states, int *flags, int n, int R,
                             int Np, int Rp, int nplanes, long long plane_stride, hipStream_t st);
// E[r] = sum_t partial[t][r] (fixed order), best = argmin (ties -> lowest r),
// E[Rp] = E[best] (E holds Rp + 1 doubles); with run_e, the running best of a
// run's checks (*run_e, *run_i) takes (E[best], best) when E[best] < *run_e;
// with trace, *trace = E[best] as well
hipError_t launch_energy_reduce(const double *partial, int ntiles, int Rp, int R, double *E,
                                int *best, hipStream_t st, double *run_e = nullptr, int *run_i = nullptr,
                                double *trace = nullptr);
// The argmin and running-best part of launch_energy_reduce for E[r] already formed
hipError_t launch_energy_argmin(double *E, int R, int Rp, int *best, double *run_e, int *run_i,
                                hipStream_t st, double *trace = nullptr);
// FP64 re-score from the FP32 amplitudes (unit phasors / signs formed in FP64):
// partial[t][r] = sum_{i in tile t} [-Re(conj(d_i) (J d)_i) + g_i Re(d_i)]
// D64: scratch for the FP64 readout planes, nplanes * Rp * Np doubles
hipError_t launch_energy_fp64(const float *J, const float *psi, const float *g, double *D64,
                              double *partial, int Np, int Rp, int n, int R, int nplanes,
                              long long plane_stride, int readout, int q, hipStream_t st);
// shadow copy of FP32 planes in BF16 / FP16
hipError_t launch_make_shadow(const float *src, void *dst, long long count, int op, hipStream_t st);
// any_flag: out[0] = number of r < R with flags[r] != 0
hipError_t launch_count_flags(const int *flags, int R, int *out, hipStream_t st);
// `steps` Euler or RK4 steps of a small problem (Np 64 or 128; FP32) in one
// launch: psi_in/gam_in -> psi_out/gam_out (gam_out
// may alias gam_in), flags[r] set if trajectory r ends non-finite.  Noise
// (a.noise_amp != 0): step t0 + k uses the key SplitMix64(seed ^
// SplitMix64(t0 + k)), as the step-by-step path does.  With E: the Eq. (h)
// energies of the final state's readout (readout, q) into E[r], r < R.
hipError_t launch_small_steps(bool complex_mode, bool rk4, const DenseStepArgs &a, int steps,
                              unsigned long long seed, long long t0, int readout, int q, double *E,
                              hipStream_t st);
// Running best of a run's device checks: (*run_e, *run_i) = (e0, i0)
hipError_t launch_best_seed(double *run_e, int *run_i, double e0, int i0, hipStream_t st);

}  // namespace gd
