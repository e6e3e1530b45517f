// Auxiliary kernels of libgd.so: layout conversion, readout (discretisation)
// of the amplitudes onto the spin domains of Eq. (h), deterministic energy
// reductions and the FP64 re-scoring of Eq. (h).
#include "gd_epilogue.h"

#include <algorithm>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace gd {

namespace {

// user [R][n] or [R][n][2] <-> planes [P][Rp][Np] (zero padded)
__global__ void pack_planes_k(const float *__restrict__ user, float *__restrict__ planes, int n,
                              int R, int Np, int Rp, int P) {
    const long long total = (long long)Rp * Np;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int r = int(t / Np), i = int(t % Np);
        const bool in = (r < R) && (i < n);
        for (int p = 0; p < P; ++p) {
            float v = 0.0f;
            if (in) v = (P == 1) ? user[(long long)r * n + i] : user[((long long)r * n + i) * 2 + p];
            planes[p * total + t] = v;
        }
    }
}

__global__ void unpack_planes_k(const float *__restrict__ planes, float *__restrict__ user, int n,
                                int R, int Np, int Rp, int P) {
    const long long total = (long long)R * n;
    const long long pstride = (long long)Rp * Np;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int r = int(t / n), i = int(t % n);
        const long long src = (long long)r * Np + i;
        if (P == 1) user[t] = planes[src];
        else for (int p = 0; p < P; ++p) user[t * 2 + p] = planes[p * pstride + src];
    }
}

__device__ inline void store_shadow(void *dst, long long k, float v, int op) {
    if (op == OP_BF16) static_cast<__hip_bfloat16 *>(dst)[k] = __float2bfloat16(v);
    else if (op == OP_F16) static_cast<__half *>(dst)[k] = __float2half(v);
}

constexpr double kTwoPi = 6.283185307179586476925286766559;   // nearest double to 2 pi

// q-state clock readout in FP64: theta = arg Psi in [0, 2pi) (Psi = 0 ->
// theta = 0), k = floor(q theta / 2pi + 1/2) mod q.
__device__ inline int clock_state(double x, double y, int q) {
    double th = (x == 0.0 && y == 0.0) ? 0.0 : atan2(y, x);
    if (th < 0.0) th += kTwoPi;
    const long long c = (long long)floor((double)q * th / kTwoPi + 0.5);
    return (int)(((c % q) + q) % q);
}

// Planes of clock state k: d0 = cos(2 pi k / q); d1 = sin(2 pi k / q), held
// as sin / (sqrt(3)/2) in {0, +-1} for q = 3 and 6 so that both planes are
// exact (their product then carries the weight 3/4).
__device__ inline void clock_planes(int k, int q, double &d0, double &d1) {
    switch (q) {
    case 2: d0 = k ? -1.0 : 1.0; d1 = 0.0; return;
    case 3: d0 = k ? -0.5 : 1.0; d1 = k == 0 ? 0.0 : (k == 1 ? 1.0 : -1.0); return;
    case 4: d0 = k == 0 ? 1.0 : (k == 2 ? -1.0 : 0.0); d1 = k == 1 ? 1.0 : (k == 3 ? -1.0 : 0.0); return;
    case 6:   // cos: 1, 1/2, -1/2, -1, -1/2, 1/2; sin / (sqrt(3)/2): 0, 1, 1, 0, -1, -1
        d0 = k == 0 ? 1.0 : (k == 3 ? -1.0 : ((k == 1 || k == 5) ? 0.5 : -0.5));
        d1 = (k == 0 || k == 3) ? 0.0 : (k < 3 ? 1.0 : -1.0);
        return;
    default: sincospi(2.0 * k / q, &d1, &d0); return;
    }
}

// Discretised planes (d0, d1) of one amplitude in FP64 for readout `ro`;
// `k` receives the clock state (RO_CLOCK) or 0/1 for the sign readouts.
__device__ inline void readout_planes(double x, double y, int ro, int q, double &d0, double &d1,
                                      int &k) {
    d1 = 0.0;
    k = 0;
    switch (ro) {
    case RO_SIGN:
    case RO_SIGN_RE:
        d0 = (x < 0.0) ? -1.0 : 1.0;   // sign(+-0) = +1
        k = x < 0.0;
        return;
    case RO_PHASOR: {
        if (x == 0.0 && y == 0.0) {
            d0 = 1.0;
            return;
        }
        const double m = sqrt(x * x + y * y);
        d0 = x / m;
        d1 = y / m;
        return;
    }
    default:
        k = clock_state(x, y, q);
        clock_planes(k, q, d0, d1);
        return;
    }
}

// Readout onto the spin domains of Eq. (h).
__global__ void __launch_bounds__(256)
discretise_k(const float *__restrict__ psi, float *__restrict__ D, void *shadowD,
             int op, int ro, int q, int8_t *__restrict__ spins8,
             float *__restrict__ angle, int32_t *__restrict__ states,
             int *__restrict__ flags, int n, int R, int Np, int Rp, int P,
             long long ps) {
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    // 2-D grid: trajectories along y, groups of 4 consecutive spins along x
    // (Np is a multiple of 4: 16-byte plane loads and stores)
    const int nq = Np / 4;
    for (int r = blockIdx.y; r < Rp; r += gridDim.y)
    for (int iq = blockIdx.x * blockDim.x + threadIdx.x; iq < nq; iq += gridDim.x * blockDim.x) {
        const int i0 = iq * 4;
        const long long t = (long long)r * Np + i0;
        const f32x4 xv = *reinterpret_cast<const f32x4 *>(psi + t);
        const f32x4 yv = P == 2 ? *reinterpret_cast<const f32x4 *>(psi + ps + t) : f32x4{0.f, 0.f, 0.f, 0.f};
        f32x4 d0v = {0.f, 0.f, 0.f, 0.f}, d1v = {0.f, 0.f, 0.f, 0.f};
        bool nan = false;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = i0 + e;
            if (r >= R || i >= n) continue;
            const float x = xv[e], y = yv[e];
            double e0, e1;
            int k;
            readout_planes(x, y, ro, q, e0, e1, k);
            d0v[e] = float(e0);
            d1v[e] = float(e1);
            float th;
            if (ro == RO_PHASOR) {
                th = 0.0f;
                if (!(x == 0.0f && y == 0.0f)) {
                    th = atan2f(y, x);
                    if (th < 0.0f) th += 6.28318530717958647692f;
                    if (th >= 6.28318530717958647692f) th = 0.0f;
                }
            } else if (ro == RO_CLOCK) {
                th = float(kTwoPi * k / q);
            } else {
                th = k ? 3.14159265358979323846f : 0.0f;
            }
            const long long o = (long long)r * n + i;
            if (spins8) spins8[o] = k ? int8_t(-1) : int8_t(1);
            if (angle) angle[o] = th;
            if (states) states[o] = k;
            nan |= __builtin_isnan(x) || __builtin_isnan(y);
        }
        if (nan) flags[r] = 1;
        *reinterpret_cast<f32x4 *>(D + t) = d0v;
        if (P == 2) *reinterpret_cast<f32x4 *>(D + ps + t) = d1v;
        if (shadowD) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                store_shadow(shadowD, t + e, d0v[e], op);
                if (P == 2) store_shadow(shadowD, ps + t + e, d1v[e], op);
            }
        }
    }
}

// E[r] = sum over row tiles in fixed order (one thread per trajectory).
__global__ void energy_sum_k(const double *__restrict__ partial, int ntiles, int Rp, int R,
                             double *__restrict__ E) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double s = 0.0;
    for (int t = 0; t < ntiles; ++t) s += partial[(long long)t * Rp + r];
    E[r] = s;
}

// The same sums for few trajectories and many row tiles: one wave per
// trajectory, lane l adds tiles l, l + 64, ... in order, then a butterfly
// over the wave (a fixed order, so repeated checks give the same sums).
__global__ void __launch_bounds__(64) energy_sum_wide_k(const double *__restrict__ partial, int ntiles,
                                                        int Rp, double *__restrict__ E) {
    const int r = blockIdx.x, lane = threadIdx.x;
    double s = 0.0;
    for (int t = lane; t < ntiles; t += 64) s += partial[(long long)t * Rp + r];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m);
    if (lane == 0) E[r] = s;
}

// best = argmin_r E[r], ties -> lowest r (one workgroup); best_e = E[best]
// (one read-back for the host's check).  With run_e: the running best of a
// run's checks keeps (E[best], best) when E[best] < *run_e.  With trace:
// E[best] is also written there (the check's entry of the energy trace).
__global__ void energy_argmin_k(const double *__restrict__ E, int R, int *__restrict__ best,
                                double *__restrict__ best_e, double *__restrict__ run_e,
                                int *__restrict__ run_i, double *__restrict__ trace) {
    __shared__ double sv[256];
    __shared__ int si[256];
    double bv = __builtin_inf();
    int bi = 0x7fffffff;
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        const double s = E[r];
        if (s < bv || (s == bv && r < bi)) { bv = s; bi = r; }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double ov = sv[threadIdx.x + w];
            const int oi = si[threadIdx.x + w];
            if (ov < sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int b = (si[0] == 0x7fffffff) ? 0 : si[0];
        if (best) best[0] = b;
        if (best_e) best_e[0] = E[b];
        if (trace) trace[0] = E[b];
        if (run_e && E[b] < run_e[0]) {
            run_e[0] = E[b];
            run_i[0] = b;
        }
    }
}

// FP64 re-score of Eq. (h) for the discretised state, formed in FP64 from
// the FP32 amplitudes by the readout of the model.  The readout planes are
// written once in FP64 ([P][Rp][Np], zero outside n x R); then per workgroup
// (row tile t of 64 spins, column tile of 64 trajectories): T = J d over K
// through LDS in FP64, and partial[t][r] = sum_{i in tile} [ -(d0_i T0_i +
// w d1_i T1_i) + g_i d0_i ] (w: weight of the second plane).
constexpr int E64_T = 64;
constexpr int E64_K = 16;

__global__ void __launch_bounds__(256)
planes64_k(const float *__restrict__ psi, double *__restrict__ D64, int n, int R, int Np, int Rp, int P,
           long long ps, int ro, int q) {
    for (int r = blockIdx.y; r < Rp; r += gridDim.y)
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Np; i += gridDim.x * blockDim.x) {
            const long long t = (long long)r * Np + i;
            double d0 = 0.0, d1 = 0.0;
            if (r < R && i < n) {
                int k;
                readout_planes(psi[t], P == 2 ? psi[ps + t] : 0.0f, ro, q, d0, d1, k);
            }
            D64[t] = d0;
            if (P == 2) D64[ps + t] = d1;
        }
}

// T = J d on the FP64 matrix cores (v_mfma_f64_16x16x4_f64): workgroup tile
// 64 rows x 64 trajectories, 2 x 2 waves of 32 x 32 (2 x 2 blocks of 16 x 16),
// K chunks of 16 staged in LDS as [row][k] doubles with a one-double pad (the
// 8-byte operand reads of 16 rows at one k then hit distinct banks).  MFMA
// operands: A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k; result
// D[l / 16 + 4 e][l % 16] in element e of lane l (rows interleaved, unlike
// the FP32 16x16x4 layout).
template <int P>
__global__ void __launch_bounds__(256)
energy_fp64_k(const float *__restrict__ J, const double *__restrict__ D64, const float *__restrict__ g,
              double *__restrict__ partial, int Np, int Rp, long long ps, double w) {
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    constexpr int KP = E64_K + 1;
    __shared__ double sJ[E64_T][KP];
    __shared__ double sD[P][E64_T][KP];
    __shared__ double red[2][E64_T];
    const int mt = blockIdx.x, ct = blockIdx.y;
    const int i0 = mt * E64_T, r0 = ct * E64_T;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int l16 = lane & 15, lq = lane >> 4;
    f64x4 acc[P][2][2];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[p][mb][nb] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < Np; k0 += E64_K) {
        // 64 rows x 16 k of J and of each plane: 4 elements per thread
#pragma unroll
        for (int u = 0; u < E64_K * E64_T / 256; ++u) {
            const int e = tid + u * 256;
            const int row = e / E64_K, kk = e % E64_K;
            sJ[row][kk] = (double)J[(long long)(i0 + row) * Np + k0 + kk];
#pragma unroll
            for (int p = 0; p < P; ++p) sD[p][row][kk] = D64[p * ps + (long long)(r0 + row) * Np + k0 + kk];
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < E64_K / 4; ++k4) {
            const int k = 4 * k4 + lq;
            double av[2], bv[P][2];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) av[mb] = sJ[wm * 32 + mb * 16 + l16][k];
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) bv[p][nb] = sD[p][wn * 32 + nb * 16 + l16][k];
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb)
                        acc[p][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mb], bv[p][nb], acc[p][mb][nb],
                                                                             0, 0, 0);
        }
        __syncthreads();
    }
    // per trajectory column: sum over this wave's rows, then over the lanes
    // that hold the same column, then over the two row waves
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const int rl = wn * 32 + nb * 16 + l16;
        const long long rb = (long long)(r0 + rl) * Np;
        double s = 0.0;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = i0 + wm * 32 + mb * 16 + lq + 4 * e;
                const double d0 = D64[rb + i];
                double t = d0 * acc[0][mb][nb][e];
                if (P == 2) t += w * (D64[ps + rb + i] * acc[P - 1][mb][nb][e]);
                s += -t + (double)g[i] * d0;
            }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (lq == 0) red[wm][rl] = s;
    }
    __syncthreads();
    if (tid < E64_T) partial[(long long)mt * Rp + r0 + tid] = red[0][tid] + red[1][tid];
}

// Device energy check of a small problem, closing the launch of its steps:
// trajectory r's Eq. (h) energy E_r = sum_i [-(d0_i T0_i + w d1_i T1_i) +
// g_i d0_i], d the readout planes of the model (formed in FP64, held in FP32
// as in the coupling kernels' energy mode), T = J d summed in FP32 in j
// order, the Np terms added in FP64 in a fixed tree.  d0s, d1s, reds: this
// trajectory's LDS rows; every thread of the workgroup calls it.
template <bool CPLX, int NPX>
__device__ inline void small_energy(const DenseStepArgs &a, const float *Js, float *d0s, float *d1s,
                                    double *reds, int i, int r, float x, float y, int ro, int q,
                                    double *__restrict__ E) {
    double e0 = 0.0, e1 = 0.0;
    if (r < a.R && i < a.n) {
        int k;
        readout_planes(x, y, ro, q, e0, e1, k);
    }
    const float d0 = float(e0), d1 = float(e1);
    d0s[i] = d0;
    if (CPLX) d1s[i] = d1;
    __syncthreads();
    float t0 = 0.0f, t1 = 0.0f;
    for (int j = 0; j < NPX; ++j) {
        const float w = Js[j * NPX + i];
        t0 = fmaf(w, d0s[j], t0);
        if (CPLX) t1 = fmaf(w, d1s[j], t1);
    }
    double term = -(double)d0 * (double)t0 + (double)a.g[i] * (double)d0;
    if (CPLX) term -= (double)a.im_weight * ((double)d1 * (double)t1);
    reds[i] = term;
    __syncthreads();
    for (int w = NPX / 2; w > 0; w >>= 1) {
        if (i < w) reds[i] += reds[i + w];
        __syncthreads();
    }
    if (i == 0 && r < a.R) E[r] = reds[0];
}

// Many integration steps of a small dense problem in one launch (Np <= 128,
// FP32 operands): a workgroup holds J and the
// amplitudes of 256 / Np trajectories in LDS for all the steps, one thread
// per (spin, trajectory) with its amplitude and gain in registers.  Per
// coupling evaluation: C_ir = sum_j J_ij Psi_jr in j order (J is symmetric,
// so lanes on consecutive i read row j contiguously), then Eq. (main) and
// Eq. (gamma) as in the dense kernels: an explicit Euler step, or the four
// stages of the classical RK4 step on the joint state (Psi, gamma); then the
// noise increment of step t0 + st (amplitude a.noise_amp, key derived from
// `seed` and the step index as on the host).  With E: the energy check of
// the final state (readout ro, clock order q) into E[r].
template <bool CPLX, int NPX, bool RK4>
__global__ void __launch_bounds__(256)
small_step_k(DenseStepArgs a, int steps, unsigned long long seed, long long t0, int ro, int q,
             double *E) {
    constexpr int TR = 256 / NPX;
    constexpr int PL = CPLX ? 2 : 1;
    __shared__ float Js[NPX * NPX];
    __shared__ float xs[PL][TR][NPX];
    __shared__ float ds[PL][TR][NPX];
    __shared__ double red[TR][NPX];
    const int tid = threadIdx.x;
    const int i = tid % NPX, tl = tid / NPX;
    const int r = blockIdx.x * TR + tl;
    const long long idx = (long long)r * NPX + i;
    const long long ps = a.plane_stride;
    const float *J = static_cast<const float *>(a.J);
    for (int q = tid; q < NPX * NPX; q += 256) Js[q] = J[q];
    float x = a.psi_in[idx];
    float y = CPLX ? a.psi_in[ps + idx] : 0.0f;
    float g = a.gam_in[idx];
    const float ep = a.eps[i], hh = a.h1[i];
    const bool valid = r < a.R && i < a.n;
    // sums over the amplitudes in LDS, then the right-hand side at (sx, sy, sg)
    auto rhs = [&](float sx, float sy, float sg, float &fr, float &fi, float &fg) {
        float cr = 0.0f, ci = 0.0f;
        // 16 terms at a time: their LDS reads are issued together, then the
        // multiply-adds run in j order
        for (int j0 = 0; j0 < NPX; j0 += 16) {
            float w[16], v0[16], v1[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                w[u] = Js[(j0 + u) * NPX + i];
                v0[u] = xs[0][tl][j0 + u];
                v1[u] = CPLX ? xs[PL - 1][tl][j0 + u] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                cr = fmaf(w[u], v0[u], cr);
                if (CPLX) ci = fmaf(w[u], v1[u], ci);
            }
        }
        const float rho = CPLX ? sx * sx + sy * sy : sx * sx;
        const float lin = sg - a.gamma_c - rho;
        fr = sx * lin + cr * a.inv_s + hh;
        fi = CPLX ? sy * lin + ci * a.inv_s : 0.0f;
        fg = ep * (a.rho_th - rho);
        if (CPLX && a.q >= 2) {
            // resonant term h_q conj(Psi)^(q-1), as in the dense kernels
            float pr = sx, pi = -sy;
            for (int k = 2; k < a.q; ++k) {
                const float tr = pr * sx + pi * sy;
                const float ti = pi * sx - pr * sy;
                pr = tr;
                pi = ti;
            }
            fr += a.hq * pr;
            fi += a.hq * pi;
        }
    };
    // publish amplitudes (sx, sy) once every thread has read the previous ones
    auto publish = [&](float sx, float sy) {
        __syncthreads();
        xs[0][tl][i] = sx;
        if (CPLX) xs[PL - 1][tl][i] = sy;
        __syncthreads();
    };
    publish(x, y);
    const float dt = a.dt;
    auto add_noise = [&](int st) {
        if (a.noise_amp != 0.0f && valid) {
            float g0, g1;
            noise_pair(mix64(seed ^ mix64((unsigned long long)(t0 + st))), r, i, g0, g1);
            x += a.noise_amp * g0;
            if (CPLX) y += a.noise_amp * g1;
        }
    };
    for (int st = 0; st < steps; ++st) {
        float fr, fi, fg;
        if constexpr (!RK4) {
            rhs(x, y, g, fr, fi, fg);
            if (valid) {
                x = x + dt * fr;
                y = y + dt * fi;
                g = g + dt * fg;
            }
            add_noise(st);
            publish(x, y);
        } else {
            // stage inputs s = y + c k with c = dt/2, dt/2, dt; accumulator
            // k1 + 2 k2 + 2 k3 (rows outside n keep their state)
            float ar, ai, ag, sx, sy, sg;
            rhs(x, y, g, fr, fi, fg);                                    // k1
            ar = fr; ai = fi; ag = fg;
            sx = valid ? x + 0.5f * dt * fr : x;
            sy = valid ? y + 0.5f * dt * fi : y;
            sg = valid ? g + 0.5f * dt * fg : g;
            publish(sx, sy);
            rhs(sx, sy, sg, fr, fi, fg);                                 // k2
            ar += 2.0f * fr; ai += 2.0f * fi; ag += 2.0f * fg;
            sx = valid ? x + 0.5f * dt * fr : x;
            sy = valid ? y + 0.5f * dt * fi : y;
            sg = valid ? g + 0.5f * dt * fg : g;
            publish(sx, sy);
            rhs(sx, sy, sg, fr, fi, fg);                                 // k3
            ar += 2.0f * fr; ai += 2.0f * fi; ag += 2.0f * fg;
            sx = valid ? x + dt * fr : x;
            sy = valid ? y + dt * fi : y;
            sg = valid ? g + dt * fg : g;
            publish(sx, sy);
            rhs(sx, sy, sg, fr, fi, fg);                                 // k4
            const float c6 = dt * (1.0f / 6.0f);
            if (valid) {
                x = x + c6 * (ar + fr);
                y = y + c6 * (ai + fi);
                g = g + c6 * (ag + fg);
            }
            add_noise(st);
            publish(x, y);
        }
    }
    a.psi_out[idx] = x;
    if (CPLX) a.psi_out[ps + idx] = y;
    a.gam_out[idx] = g;
    // non-finite values persist once they appear, so the final state tells
    if (r < a.R && !(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(g))) a.flags[r] = 1;
    if (E) small_energy<CPLX, NPX>(a, Js, ds[0][tl], ds[PL - 1][tl], red[tl], i, r, x, y, ro, q, E);
}

__global__ void make_shadow_k(const float *__restrict__ src, void *dst, long long count, int op) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < count;
         t += (long long)gridDim.x * blockDim.x)
        store_shadow(dst, t, src[t], op);
}

__global__ void count_flags_k(const int *__restrict__ flags, int R, int *out) {
    __shared__ int s[256];
    int c = 0;
    for (int r = threadIdx.x; r < R; r += blockDim.x) c += flags[r] != 0;
    s[threadIdx.x] = c;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

inline int grid_for(long long total) {
    long long b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return int(b);
}

// Running best over the device checks of one run, kept on the device so that
// a run with no target does not wait for every check: seeded with (e0, i0);
// energy_argmin_k keeps the first strict minimum of E[best] (the host rule).
__global__ void best_seed_k(double *__restrict__ run_e, int *__restrict__ run_i, double e0, int i0) {
    if (threadIdx.x == 0) {
        run_e[0] = e0;
        run_i[0] = i0;
    }
}

}  // namespace

hipError_t launch_pack_planes(const float *user, float *planes, int n, int R, int Np, int Rp,
                              int nplanes, hipStream_t st) {
    pack_planes_k<<<grid_for((long long)Rp * Np), 256, 0, st>>>(user, planes, n, R, Np, Rp, nplanes);
    return hipGetLastError();
}

hipError_t launch_unpack_planes(const float *planes, float *user, int n, int R, int Np, int Rp,
                                int nplanes, hipStream_t st) {
    unpack_planes_k<<<grid_for((long long)R * n), 256, 0, st>>>(planes, user, n, R, Np, Rp, nplanes);
    return hipGetLastError();
}

float clock_im_weight(int q) { return (q == 3 || q == 6) ? 0.75f : 1.0f; }

hipError_t launch_discretise(const float *psi, float *D, void *shadowD, int op, int readout, int q,
                             int8_t *spins8, float *angle, int32_t *states, int *flags, int n, int R,
                             int Np, int Rp, int nplanes, long long plane_stride, hipStream_t st) {
    if (readout == RO_CLOCK && (q < 2 || q > 8)) return hipErrorInvalidValue;
    if (Np % 4) return hipErrorInvalidValue;
    const dim3 grid(unsigned(std::min(64, (Np / 4 + 255) / 256)), unsigned(std::min(Rp, 65535)));
    discretise_k<<<grid, 256, 0, st>>>(psi, D, shadowD, op, readout, q, spins8,
                                                              angle, states, flags, n, R, Np, Rp,
                                                              nplanes, plane_stride);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(const double *partial, int ntiles, int Rp, int R, double *E,
                                int *best, hipStream_t st, double *run_e, int *run_i, double *trace) {
    if (R < 1) return hipErrorInvalidValue;
    if (R <= 512 && ntiles >= 32)
        energy_sum_wide_k<<<R, 64, 0, st>>>(partial, ntiles, Rp, E);
    else
        energy_sum_k<<<(R + 255) / 256, 256, 0, st>>>(partial, ntiles, Rp, R, E);
    energy_argmin_k<<<1, 256, 0, st>>>(E, R, best, E + Rp, run_e, run_i, trace);
    return hipGetLastError();
}

hipError_t launch_energy_argmin(double *E, int R, int Rp, int *best, double *run_e, int *run_i,
                                hipStream_t st, double *trace) {
    if (R < 1 || R > Rp) return hipErrorInvalidValue;
    energy_argmin_k<<<1, 256, 0, st>>>(E, R, best, E + Rp, run_e, run_i, trace);
    return hipGetLastError();
}

hipError_t launch_energy_fp64(const float *J, const float *psi, const float *g, double *D64,
                              double *partial, int Np, int Rp, int n, int R, int nplanes,
                              long long plane_stride, int readout, int q, hipStream_t st) {
    if (Np % E64_T || Rp % E64_T) return hipErrorInvalidValue;
    if (readout == RO_CLOCK && (q < 2 || q > 8)) return hipErrorInvalidValue;
    if (nplanes != 1 && nplanes != 2) return hipErrorInvalidValue;
    const double w = readout == RO_CLOCK ? (double)clock_im_weight(q) : 1.0;
    const dim3 pgrid(unsigned(std::min(64, (Np + 255) / 256)), unsigned(std::min(Rp, 65535)));
    planes64_k<<<pgrid, 256, 0, st>>>(psi, D64, n, R, Np, Rp, nplanes, plane_stride, readout, q);
    const dim3 grid(Np / E64_T, Rp / E64_T);
    if (nplanes == 2)
        energy_fp64_k<2><<<grid, 256, 0, st>>>(J, D64, g, partial, Np, Rp, plane_stride, w);
    else
        energy_fp64_k<1><<<grid, 256, 0, st>>>(J, D64, g, partial, Np, Rp, plane_stride, w);
    return hipGetLastError();
}

hipError_t launch_small_steps(bool complex_mode, bool rk4, const DenseStepArgs &a, int steps,
                              unsigned long long seed, long long t0, int readout, int q, double *E,
                              hipStream_t st) {
    if (steps < 1 || (a.Np != 64 && a.Np != 128)) return hipErrorInvalidValue;
    if (E && readout == RO_CLOCK && (q < 2 || q > 8)) return hipErrorInvalidValue;
    const int tr = 256 / a.Np;
    if (a.Rp % tr) return hipErrorInvalidValue;
    const dim3 grid(a.Rp / tr);
#define GD_SMALL(C, N, K) small_step_k<C, N, K><<<grid, 256, 0, st>>>(a, steps, seed, t0, readout, q, E)
    if (a.Np == 64) {
        if (complex_mode) { if (rk4) GD_SMALL(true, 64, true); else GD_SMALL(true, 64, false); }
        else { if (rk4) GD_SMALL(false, 64, true); else GD_SMALL(false, 64, false); }
    } else {
        if (complex_mode) { if (rk4) GD_SMALL(true, 128, true); else GD_SMALL(true, 128, false); }
        else { if (rk4) GD_SMALL(false, 128, true); else GD_SMALL(false, 128, false); }
    }
#undef GD_SMALL
    return hipGetLastError();
}

hipError_t launch_best_seed(double *run_e, int *run_i, double e0, int i0, hipStream_t st) {
    best_seed_k<<<1, 64, 0, st>>>(run_e, run_i, e0, i0);
    return hipGetLastError();
}

hipError_t launch_make_shadow(const float *src, void *dst, long long count, int op, hipStream_t st) {
    make_shadow_k<<<grid_for(count), 256, 0, st>>>(src, dst, count, op);
    return hipGetLastError();
}

hipError_t launch_count_flags(const int *flags, int R, int *out, hipStream_t st) {
    count_flags_k<<<1, 256, 0, st>>>(flags, R, out);
    return hipGetLastError();
}

}  // namespace gd
