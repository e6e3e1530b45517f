// GD-mod step (Sec. 1): the coupling of Eq. (main) is Delta_ij K_ij with
// Delta_ij = gamma_i + gamma_j, and every trajectory carries its own coupling
// matrix K that follows Eq. (gamma2), dK_ij/dt = eps_hat (J_ij - Delta_ij K_ij).
//
// One explicit Euler step, all right-hand sides at the old state:
//   c_i   = sum_j (gamma_i + gamma_j) K_ij Psi_j          (raw sum; 1/s in the epilogue)
//   K_ij += dt eps_hat (J_ij - (gamma_i + gamma_j) K_ij)
// followed by the pointwise update of Eq. (main, gamma) shared with the dense
// kernels (gd_epilogue.h).  The diagonal needs no test: J_ii = 0 and K_ii(0)
// = 0, so K_ii stays 0 and adds nothing.
//
// Every K element is read and written once per step, so the step streams
// R * Np^2 * 8 bytes through HBM (J rows are shared by all trajectories and
// come from L2): an HBM-bound batched matrix-vector product, not a GEMM.
//
// Launch: grid (Np / 16 row blocks, R trajectories), 256 threads.  The
// workgroup stages its trajectory's amplitudes and gains in LDS, each wave
// sweeps 4 consecutive rows with 16-byte loads (64 lanes x 4 columns per
// instruction, fully coalesced), reduces each row across the wave, and lane 0
// applies the epilogue to the 4 rows.
#include "gd_epilogue.h"

namespace gd {

namespace {

constexpr int kModRowsPerWave = 4;
constexpr int kModWaves = 4;
constexpr int kModRows = kModRowsPerWave * kModWaves;

template <bool CPLX>
__global__ void __launch_bounds__(64 * kModWaves)
gdmod_euler_k(DenseStepArgs a, const float *__restrict__ J, float *__restrict__ K, float c_hat) {
    extern __shared__ float sh[];   // [Np] gamma, [Np] Re Psi, [Np] Im Psi (complex)
    const int Np = a.Np;
    const int r = blockIdx.y;
    const long long ps = a.plane_stride;
    float *sg = sh, *sx = sh + Np, *sy = sh + 2 * Np;
    for (int j = threadIdx.x * 4; j < Np; j += 64 * kModWaves * 4) {
        const long long o = (long long)r * Np + j;
        *reinterpret_cast<f32x4 *>(sg + j) = *reinterpret_cast<const f32x4 *>(a.gam_in + o);
        *reinterpret_cast<f32x4 *>(sx + j) = *reinterpret_cast<const f32x4 *>(a.psi_in + o);
        if (CPLX) *reinterpret_cast<f32x4 *>(sy + j) = *reinterpret_cast<const f32x4 *>(a.psi_in + ps + o);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i0 = blockIdx.x * kModRows + wave * kModRowsPerWave;
    f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < kModRowsPerWave; ++q) {
        const int i = i0 + q;
        const float gi = sg[i];
        float *Kr = K + ((long long)r * Np + i) * Np;
        const float *Jr = J + (long long)i * Np;
        float sre = 0.0f, sim = 0.0f;
        // KU chunks of 256 columns per pass: all their K and J loads are in
        // flight together (K is streamed: non-temporal loads and stores)
        constexpr int KU = 4;
        for (int j0 = lane * 4; j0 < Np; j0 += 256 * KU) {
            f32x4 k[KU], jj[KU];
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int j = j0 + 256 * u;
                if (j < Np) {
                    k[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(Kr + j));
                    jj[u] = *reinterpret_cast<const f32x4 *>(Jr + j);
                }
            }
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int j = j0 + 256 * u;
                if (j >= Np) break;
                const f32x4 gj = *reinterpret_cast<const f32x4 *>(sg + j);
                const f32x4 xj = *reinterpret_cast<const f32x4 *>(sx + j);
                f32x4 yj = {0.f, 0.f, 0.f, 0.f};
                if (CPLX) yj = *reinterpret_cast<const f32x4 *>(sy + j);
                f32x4 kn;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float d = gi + gj[e];
                    const float dk = d * k[u][e];
                    sre += dk * xj[e];
                    if (CPLX) sim += dk * yj[e];
                    kn[e] = k[u][e] + c_hat * (jj[u][e] - dk);
                }
                __builtin_nontemporal_store(kn, reinterpret_cast<f32x4 *>(Kr + j));
            }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            sre += __shfl_xor(sre, m);
            if (CPLX) sim += __shfl_xor(sim, m);
        }
        cr[q] = sre;
        ci[q] = sim;
    }
    if (lane == 0) {
        const bool bad = step_epilogue4<MODE_EULER, CPLX, OP_F32>(a, i0, r, true, cr, ci);
        if (bad) a.flags[r] = 1;
    }
}

}  // namespace

size_t gdmod_lds_bytes(bool complex_mode, int Np) { return size_t(complex_mode ? 3 : 2) * Np * sizeof(float); }

hipError_t launch_gdmod(bool complex_mode, const DenseStepArgs &a, const float *J, float *K, float c_hat,
                        hipStream_t st) {
    if (a.Np % kModRows || a.R < 1) return hipErrorInvalidValue;
    const size_t lds = gdmod_lds_bytes(complex_mode, a.Np);
    if (lds > 65536) return hipErrorInvalidValue;
    const dim3 grid(a.Np / kModRows, a.R), block(64 * kModWaves);
    if (complex_mode)
        gdmod_euler_k<true><<<grid, block, lds, st>>>(a, J, K, c_hat);
    else
        gdmod_euler_k<false><<<grid, block, lds, st>>>(a, J, K, c_hat);
    return hipGetLastError();
}

}  // namespace gd
