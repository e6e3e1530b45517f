// Auxiliary kernels of libgd.so: layout conversion, readout (discretisation)
// of the amplitudes onto the spin domains of Eq. (h), deterministic energy
// reductions and the FP64 re-scoring of Eq. (h).
#include "gd_internal.h"

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

// Readout onto the spin domains of Eq. (h).
__global__ void discretise_k(const float *__restrict__ psi, float *__restrict__ D, void *shadowD,
                             int op, int8_t *__restrict__ spins8, float *__restrict__ angle,
                             int *__restrict__ flags, int n, int R, int Np, int Rp, int P,
                             long long ps) {
    const long long total = (long long)Rp * Np;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int r = int(t / Np), i = int(t % Np);
        const bool in = (r < R) && (i < n);
        float d0 = 0.0f, d1 = 0.0f, th = 0.0f;
        bool nan = false;
        if (in) {
            const float x = psi[t];
            if (P == 1) {
                nan = __builtin_isnan(x);
                d0 = (x < 0.0f) ? -1.0f : 1.0f;        // sign(+-0) = +1
                th = (x < 0.0f) ? 3.14159265358979323846f : 0.0f;
            } else {
                const float y = psi[ps + t];
                nan = __builtin_isnan(x) || __builtin_isnan(y);
                if (x == 0.0f && y == 0.0f) {
                    d0 = 1.0f; d1 = 0.0f; th = 0.0f;
                } else {
                    // unit phasor in double so that |D| = 1 to FP32 rounding
                    const double xd = x, yd = y;
                    const double m = sqrt(xd * xd + yd * yd);
                    d0 = float(xd / m);
                    d1 = float(yd / m);
                    float a = atan2f(y, x);
                    if (a < 0.0f) a += 6.28318530717958647692f;
                    if (a >= 6.28318530717958647692f) a = 0.0f;
                    th = a;
                }
            }
            if (spins8) spins8[(long long)r * n + i] = (d0 < 0.0f && P == 1) ? int8_t(-1) : int8_t(1);
            if (angle) angle[(long long)r * n + i] = th;
            if (nan) flags[r] = 1;
        }
        D[t] = d0;
        if (P == 2) D[ps + t] = d1;
        if (shadowD) {
            store_shadow(shadowD, t, d0, op);
            if (P == 2) store_shadow(shadowD, ps + t, d1, op);
        }
    }
}

// E[r] = sum over row tiles in fixed order; then argmin with ties -> lowest r.
__global__ void energy_reduce_k(const double *__restrict__ partial, int ntiles, int Rp, int R,
                                double *__restrict__ E, int *__restrict__ best) {
    __shared__ double sv[256];
    __shared__ int si[256];
    double bv = __builtin_inf();
    int bi = 0x7fffffff;
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        double s = 0.0;
        for (int t = 0; t < ntiles; ++t) s += partial[(long long)t * Rp + r];
        E[r] = s;
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
    if (threadIdx.x == 0 && best) best[0] = (si[0] == 0x7fffffff) ? 0 : si[0];
}

// FP64 re-score of Eq. (h) for the discretised state, formed in FP64 from
// the FP32 amplitudes: Ising d = sign(x) (sign(+-0) = +1), XY d = psi/|psi|
// (psi = 0 -> 1).  Workgroup (row tile t of 64 spins, column tile of 64
// trajectories): T = J d over K through LDS in FP64, then
// partial[t][r] = sum_{i in tile} [ -Re(conj(d_i) T_i) + g_i Re(d_i) ].
constexpr int E64_T = 64;
constexpr int E64_K = 16;

__device__ inline void unit_phasor(const float *psi, long long ps, int P, long long idx, bool in,
                                   double &dr, double &di) {
    dr = 0.0;
    di = 0.0;
    if (!in) return;
    const double x = psi[idx];
    if (P == 1) {
        dr = (x < 0.0) ? -1.0 : 1.0;
        return;
    }
    const double y = psi[ps + idx];
    if (x == 0.0 && y == 0.0) {
        dr = 1.0;
        return;
    }
    const double m = sqrt(x * x + y * y);
    dr = x / m;
    di = y / m;
}

__global__ void __launch_bounds__(256)
energy_fp64_k(const float *__restrict__ J, const float *__restrict__ psi, const float *__restrict__ g,
              double *__restrict__ partial, int Np, int Rp, int n, int R, int P, long long ps) {
    __shared__ double sJ[E64_K][E64_T + 1];
    __shared__ double sDr[E64_K][E64_T + 1];
    __shared__ double sDi[E64_K][E64_T + 1];
    __shared__ double red[16][E64_T];
    const int mt = blockIdx.x, ct = blockIdx.y;
    const int i0 = mt * E64_T, r0 = ct * E64_T;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;   // 4x4 outputs per thread
    double ar[4][4], ai[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) ar[a][b] = ai[a][b] = 0.0;
    for (int k0 = 0; k0 < Np; k0 += E64_K) {
        for (int q = threadIdx.x; q < E64_K * E64_T; q += 256) {
            const int row = q / E64_K, kk = q % E64_K;
            sJ[kk][row] = (double)J[(long long)(i0 + row) * Np + k0 + kk];
            const int r = r0 + row, j = k0 + kk;
            double dr, di;
            unit_phasor(psi, ps, P, (long long)r * Np + j, r < R && j < n, dr, di);
            sDr[kk][row] = dr;
            sDi[kk][row] = di;
        }
        __syncthreads();
        for (int kk = 0; kk < E64_K; ++kk) {
            double av[4], br[4], bi[4];
            for (int a = 0; a < 4; ++a) av[a] = sJ[kk][ty * 4 + a];
            for (int b = 0; b < 4; ++b) {
                br[b] = sDr[kk][tx * 4 + b];
                bi[b] = sDi[kk][tx * 4 + b];
            }
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    ar[a][b] = fma(av[a], br[b], ar[a][b]);
                    ai[a][b] = fma(av[a], bi[b], ai[a][b]);
                }
        }
        __syncthreads();
    }
    double colsum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + ty * 4 + a;
        for (int b = 0; b < 4; ++b) {
            const int r = r0 + tx * 4 + b;
            double dr, di;
            unit_phasor(psi, ps, P, (long long)r * Np + i, r < R && i < n, dr, di);
            colsum[b] += -(dr * ar[a][b] + di * ai[a][b]) + (double)g[i] * dr;
        }
    }
    for (int b = 0; b < 4; ++b) red[ty][tx * 4 + b] = colsum[b];
    __syncthreads();
    if (threadIdx.x < E64_T) {
        double s = 0.0;
        for (int y = 0; y < 16; ++y) s += red[y][threadIdx.x];
        partial[(long long)mt * Rp + r0 + threadIdx.x] = s;
    }
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

hipError_t launch_discretise(const float *psi, float *D, void *shadowD, int op, int8_t *spins8,
                             float *angle, int *flags, int n, int R, int Np, int Rp, int nplanes,
                             long long plane_stride, hipStream_t st) {
    discretise_k<<<grid_for((long long)Rp * Np), 256, 0, st>>>(psi, D, shadowD, op, spins8, angle,
                                                              flags, n, R, Np, Rp, nplanes,
                                                              plane_stride);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(const double *partial, int ntiles, int Rp, int R, double *E,
                                int *best, hipStream_t st) {
    energy_reduce_k<<<1, 256, 0, st>>>(partial, ntiles, Rp, R, E, best);
    return hipGetLastError();
}

hipError_t launch_energy_fp64(const float *J, const float *psi, const float *g, double *partial,
                              int Np, int Rp, int n, int R, int nplanes, long long plane_stride,
                              hipStream_t st) {
    if (Np % E64_T || Rp % E64_T) return hipErrorInvalidValue;
    dim3 grid(Np / E64_T, Rp / E64_T);
    energy_fp64_k<<<grid, 256, 0, st>>>(J, psi, g, partial, Np, Rp, n, R, nplanes, plane_stride);
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
