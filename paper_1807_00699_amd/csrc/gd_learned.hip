// Learned proposal of initial amplitudes and per-spin gain rates.
//
// The paper suggests site-dependent gain-adjustment rates eps_i(t) as an
// extension of the GD algorithm (Sec. 3); its sub-threshold phase amplifies
// the leading eigenvectors of J (gain rising from below, Sec. 1).  Here a
// small per-spin network reads spectral and local features of J and proposes
// (i) a sign for each spin, used to bias the initial amplitudes, and (ii) a
// confidence, used to set eps_i.  Kernels:
//
//  feat_k      one workgroup per instance: shifted block power iteration on
//              A = J/s + cI (c = max row sum of |J|/s), Cholesky-QR each
//              iteration, Rayleigh-Ritz (8x8 cyclic Jacobi in FP64), sign
//              fix (largest-magnitude entry of each vector positive, ties to
//              the lowest index), then 20 features per spin.
//  mlp_*       20 -> 64 -> 64 -> 2 ReLU network: FP32 forward (vector ALUs,
//              the reference inference), per-instance flip-invariant loss;
//              the training step on the FP32 matrix cores (forward,
//              backward and weight-gradient partials of a workgroup's
//              spins in one kernel), fixed-order reduction fused with Adam;
//              FP16 inference on the matrix cores (FP32 accumulation).
//  propose_k   writes psi0 = a (alpha m_i + (1 - alpha) xi) and eps_i into a
//              batched solver's state, xi from SplitMix64.
#include "gd_internal.h"
#include "gd_learned.h"

#include <hip/hip_fp16.h>

#include <algorithm>

namespace gd {

namespace {

constexpr int F = kMlpF, H = kMlpH, NO = kMlpOut;
constexpr int OFF_W1 = 0, OFF_B1 = F * H, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H * NO, NPAR = OFF_B3 + NO;
static_assert(NPAR == kMlpNParam, "parameter layout");
constexpr float LAMBDA_C = 0.5f;

__host__ __device__ inline unsigned long long splitmix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ inline double uniform01(unsigned long long ctr, unsigned long long key) {
    return double(splitmix64(key ^ splitmix64(ctr)) >> 11) * (1.0 / 9007199254740992.0);
}

// block-wide sum of NV doubles per thread (256 threads); result in out[] of every thread
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *scratch /* [4][NV] */) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        v[q] = x;
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) scratch[w * NV + q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = scratch[q] + scratch[NV + q] + scratch[2 * NV + q] + scratch[3 * NV + q];
    __syncthreads();
}

// 8x8 symmetric eigenproblem by cyclic Jacobi rotations (FP64); eigenvalues
// descending in th, eigenvectors as columns of U.
__device__ inline void jacobi8(double (&A)[8][8], double (&U)[8][8], double (&th)[8]) {
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) U[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < 8; ++p)
            for (int q = p + 1; q < 8; ++q) off += A[p][q] * A[p][q];
        if (off < 1e-30) break;
        for (int p = 0; p < 8; ++p)
            for (int q = p + 1; q < 8; ++q) {
                if (fabs(A[p][q]) < 1e-300) continue;
                const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < 8; ++k) {          // A <- A G  (columns p, q)
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 8; ++k) {          // A <- G^T A (rows p, q)
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 8; ++k) {          // U <- U G
                    const double ukp = U[k][p], ukq = U[k][q];
                    U[k][p] = c * ukp - s * ukq;
                    U[k][q] = s * ukp + c * ukq;
                }
            }
    }
    for (int i = 0; i < 8; ++i) th[i] = A[i][i];
    // selection sort, descending (stable for equal values)
    for (int i = 0; i < 8; ++i) {
        int b = i;
        for (int j = i + 1; j < 8; ++j)
            if (th[j] > th[b]) b = j;
        if (b != i) {
            const double tt = th[i]; th[i] = th[b]; th[b] = tt;
            for (int k = 0; k < 8; ++k) { const double u = U[k][i]; U[k][i] = U[k][b]; U[k][b] = u; }
        }
    }
}

constexpr int FT = 256;   // threads of the feature kernel

__global__ void __launch_bounds__(FT) feat_k(FeatArgs a) {
    extern __shared__ __attribute__((aligned(16))) float fsm[];
    const int k = blockIdx.x;
    const int n = a.inst_n[k];
    const long long spin0 = a.inst_spin[k];
    const int dmax = a.dmax;
    const float inv_s = a.inst_inv_s[k];
    float *V = fsm;                          // [nmax][8]
    float *W = fsm + (size_t)a.nmax * 8;     // [nmax][8]
    __shared__ double red[4 * 36];
    __shared__ double mat[8][8];             // broadcast of L^-1 / U
    __shared__ double shift;
    const int tid = threadIdx.x;
    // shift c = max_i sum_j |J_ij| / s, mean degree
    double cmax = 0.0, degsum = 0.0;
    for (int i = tid; i < n; i += FT) {
        double r = 0.0;
        for (int d = 0; d < dmax; ++d) {
            const float w = a.ell_w[(spin0 + i) * dmax + d];
            r += fabs((double)w) * inv_s;
            degsum += (w != 0.0f);
        }
        cmax = fmax(cmax, r);
    }
    for (int o = 32; o > 0; o >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, o));
    {
        double v[1] = {degsum};
        if ((tid & 63) == 0) red[64 + (tid >> 6)] = cmax;
        block_sum<1>(v, red);
        degsum = v[0];
    }
    if (tid == 0) shift = fmax(fmax(red[64], red[65]), fmax(red[66], red[67]));
    __syncthreads();
    const double c = shift;
    // V0 from SplitMix64
    for (int i = tid; i < n; i += FT)
        for (int q = 0; q < 8; ++q)
            V[i * 8 + q] = float(2.0 * uniform01((unsigned long long)(8 * i + q), kFeatKey) - 1.0);
    __syncthreads();
    auto apply = [&]() {   // W = A V
        for (int i = tid; i < n; i += FT) {
            float acc[8];
            for (int q = 0; q < 8; ++q) acc[q] = float(c) * V[i * 8 + q];
            for (int d = 0; d < dmax; ++d) {
                const float w = a.ell_w[(spin0 + i) * dmax + d] * inv_s;
                const int j = a.ell_idx[(spin0 + i) * dmax + d];
                for (int q = 0; q < 8; ++q) acc[q] += w * V[j * 8 + q];
            }
            for (int q = 0; q < 8; ++q) W[i * 8 + q] = acc[q];
        }
        __syncthreads();
    };
    for (int it = 0; it < a.iters; ++it) {
        apply();
        // G = W^T W (upper triangle, FP64)
        double g[36];
        for (int q = 0; q < 36; ++q) g[q] = 0.0;
        for (int i = tid; i < n; i += FT) {
            int q = 0;
            for (int p = 0; p < 8; ++p)
                for (int r = p; r < 8; ++r) g[q++] += (double)W[i * 8 + p] * (double)W[i * 8 + r];
        }
        block_sum<36>(g, red);
        if (tid == 0) {
            // Cholesky G = L L^T, then L^-1 (lower triangular)
            double G[8][8], L[8][8], Li[8][8];
            int q = 0;
            for (int p = 0; p < 8; ++p)
                for (int r = p; r < 8; ++r) { G[p][r] = g[q]; G[r][p] = g[q]; ++q; }
            for (int i = 0; i < 8; ++i)
                for (int j = 0; j < 8; ++j) L[i][j] = Li[i][j] = 0.0;
            for (int j = 0; j < 8; ++j) {
                double d = G[j][j];
                for (int p = 0; p < j; ++p) d -= L[j][p] * L[j][p];
                L[j][j] = sqrt(fmax(d, 1e-300));
                for (int i = j + 1; i < 8; ++i) {
                    double v = G[i][j];
                    for (int p = 0; p < j; ++p) v -= L[i][p] * L[j][p];
                    L[i][j] = v / L[j][j];
                }
            }
            for (int j = 0; j < 8; ++j) {
                Li[j][j] = 1.0 / L[j][j];
                for (int i = j + 1; i < 8; ++i) {
                    double v = 0.0;
                    for (int p = j; p < i; ++p) v -= L[i][p] * Li[p][j];
                    Li[i][j] = v / L[i][i];
                }
            }
            for (int i = 0; i < 8; ++i)
                for (int j = 0; j < 8; ++j) mat[i][j] = Li[i][j];
        }
        __syncthreads();
        // V = W L^-T: V_i[q] = sum_p W_i[p] Li[q][p]
        for (int i = tid; i < n; i += FT)
            for (int q = 0; q < 8; ++q) {
                double v = 0.0;
                for (int p = 0; p <= q; ++p) v += (double)W[i * 8 + p] * mat[q][p];
                V[i * 8 + q] = float(v);
            }
        __syncthreads();
    }
    // Rayleigh-Ritz: H = V^T A V
    apply();
    {
        double h[36];
        for (int q = 0; q < 36; ++q) h[q] = 0.0;
        for (int i = tid; i < n; i += FT) {
            int q = 0;
            for (int p = 0; p < 8; ++p)
                for (int r = p; r < 8; ++r) h[q++] += (double)V[i * 8 + p] * (double)W[i * 8 + r];
        }
        block_sum<36>(h, red);
        if (tid == 0) {
            double Hm[8][8], U[8][8], th[8];
            int q = 0;
            for (int p = 0; p < 8; ++p)
                for (int r = p; r < 8; ++r) { Hm[p][r] = h[q]; Hm[r][p] = h[q]; ++q; }
            jacobi8(Hm, U, th);
            for (int i = 0; i < 8; ++i)
                for (int j = 0; j < 8; ++j) mat[i][j] = U[i][j];
            for (int j = 0; j < 8; ++j) {
                red[j] = th[j] - c;
                if (a.lambda) a.lambda[(long long)k * 8 + j] = float(th[j] - c);
            }
        }
        __syncthreads();
        double lam[8];
        for (int j = 0; j < 8; ++j) lam[j] = red[j];
        __syncthreads();
        // V <- V U (into W)
        for (int i = tid; i < n; i += FT)
            for (int q = 0; q < 8; ++q) {
                double v = 0.0;
                for (int p = 0; p < 8; ++p) v += (double)V[i * 8 + p] * mat[p][q];
                W[i * 8 + q] = float(v);
            }
        __syncthreads();
        // sign fix: largest magnitude entry positive (ties: lowest index)
        __shared__ float bestv[4][8];
        __shared__ int besti[4][8];
        __shared__ float sgn[8];
        for (int q = 0; q < 8; ++q) {
            float bv = -1.0f;
            int bi = 0x7fffffff;
            for (int i = tid; i < n; i += FT) {
                const float v = fabsf(W[i * 8 + q]);
                if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const float ov = __shfl_xor(bv, o);
                const int oi = __shfl_xor(bi, o);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if ((tid & 63) == 0) { bestv[tid >> 6][q] = bv; besti[tid >> 6][q] = bi; }
        }
        __syncthreads();
        if (tid < 8) {
            float bv = bestv[0][tid];
            int bi = besti[0][tid];
            for (int w = 1; w < 4; ++w)
                if (bestv[w][tid] > bv || (bestv[w][tid] == bv && besti[w][tid] < bi)) {
                    bv = bestv[w][tid];
                    bi = besti[w][tid];
                }
            sgn[tid] = W[bi * 8 + tid] < 0.0f ? -1.0f : 1.0f;
            if (a.lambda) { /* eigenvalues already written */ }
        }
        __syncthreads();
        const double meandeg = degsum / n;
        const float sn = sqrtf(float(n));
        for (int i = tid; i < n; i += FT) {
            double rs = 0.0, ra = 0.0, deg = 0.0;
            for (int d = 0; d < dmax; ++d) {
                const float w = a.ell_w[(spin0 + i) * dmax + d];
                rs += (double)w * inv_s;
                ra += fabs((double)w) * inv_s;
                deg += (w != 0.0f);
            }
            float *f = a.feats + (spin0 + i) * F;
            f[0] = float(rs);
            f[1] = float(deg / fmax(meandeg, 1e-300));
            for (int q = 0; q < 8; ++q) {
                const float v = sgn[q] * W[i * 8 + q];
                f[2 + q] = sn * v;
                f[10 + q] = float(n * lam[q] * (double)v * v);
            }
            f[18] = float(ra);
            f[19] = 1.0f;
            if (a.vecs)
                for (int q = 0; q < 8; ++q) a.vecs[(spin0 + i) * 8 + q] = sgn[q] * W[i * 8 + q];
        }
    }
}

// ---------------------------------------------------------------- MLP

constexpr int MT = 256;

// forward of one spin; z1/z2 pre-activations.  sp: the parameters, read at
// wave-uniform addresses (from global memory the compiler turns them into
// scalar loads feeding the FMAs)
__device__ inline void mlp_fwd1(const float *__restrict__ sp, const float *x, float *z1, float *z2, float *o) {
    for (int j = 0; j < H; ++j) {
        float acc = sp[OFF_B1 + j];
        for (int f = 0; f < F; ++f) acc += x[f] * sp[OFF_W1 + f * H + j];
        z1[j] = acc;
    }
    for (int b = 0; b < H; ++b) {
        float acc = sp[OFF_B2 + b];
        for (int j = 0; j < H; ++j) acc += fmaxf(z1[j], 0.0f) * sp[OFF_W2 + j * H + b];
        z2[b] = acc;
    }
    for (int q = 0; q < NO; ++q) {
        float acc = sp[OFF_B3 + q];
        for (int b = 0; b < H; ++b) acc += fmaxf(z2[b], 0.0f) * sp[OFF_W3 + b * NO + q];
        o[q] = acc;
    }
}

__global__ void __launch_bounds__(MT) mlp_forward_k(const float *__restrict__ p, const float *__restrict__ X,
                                                   float *__restrict__ out, int M) {
    const float *__restrict__ sp = p;
    const int m = blockIdx.x * MT + threadIdx.x;
    if (m >= M) return;
    float x[F], z1[H], z2[H], o[NO];
    for (int f = 0; f < F; ++f) x[f] = X[(long long)m * F + f];
    mlp_fwd1(sp, x, z1, z2, o);
    out[(long long)m * NO] = o[0];
    out[(long long)m * NO + 1] = o[1];
}

// FP16 inference on the matrix cores (v_mfma_f32_32x32x16_f16, FP32
// accumulation).  Each wave takes 32 spins at a time and computes the
// transposed layers, Z1^T = W1^T X^T (features padded from 20 to 32) and
// Z2^T = W2^T relu(Z1)^T, so that a lane holds one spin's column: lane l
// (half h = l / 32) owns the accumulator rows 8q + 4h + e (q, e < 4) of each
// 32-row block for spin l mod 32.  Those 16 values, rectified and rounded to
// FP16, are already the second layer's B operand for two 16-deep K steps if
// the K order of W2^T is permuted to match: step s, slot j of half h reads
// hidden unit 8 (2 s + j / 4) + 4 h + j mod 4 of the block (every product is
// still summed once).  The two outputs take the 32 hidden units of each lane
// on the vector ALUs and add the other lane half.  The weight operands are
// built once per workgroup in LDS in the lane order of the instruction.
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
constexpr int MFT = 256;   // 4 waves

__global__ void __launch_bounds__(MFT) mlp_forward_mfma_k(const float *__restrict__ p, const float *__restrict__ X,
                                                         float *__restrict__ out, int M) {
    static_assert(H == 64 && F <= 32 && NO == 2, "layer shapes of the MFMA forward");
    // A1[rb][s][lane]: W1^T rows 32 rb + l % 32, features 16 s + 8 h + j
    // A2[rb][ib][s][lane]: W2^T rows 32 rb + l % 32, hidden 32 ib + 8 (2 s + j / 4) + 4 h + j % 4
    __shared__ f16x8_t A1[2][2][64], A2[2][2][2][64];
    __shared__ float B1s[2][2][16], B2s[2][2][16], W3s[2][2][16][2];   // [rb][h][4q + e](...)
    const int tid = threadIdx.x;
    for (int q = tid; q < 2 * 2 * 64; q += MFT) {
        const int rb = q / 128, st = (q / 64) % 2, l = q % 64, h = l / 32, row = 32 * rb + l % 32;
        f16x8_t v;
        for (int j = 0; j < 8; ++j) {
            const int f = 16 * st + 8 * h + j;
            v[j] = (_Float16)(f < F ? p[OFF_W1 + f * H + row] : 0.0f);
        }
        A1[rb][st][l] = v;
    }
    for (int q = tid; q < 2 * 2 * 2 * 64; q += MFT) {
        const int rb = q / 256, ib = (q / 128) % 2, st = (q / 64) % 2, l = q % 64, h = l / 32;
        const int row = 32 * rb + l % 32;
        f16x8_t v;
        for (int j = 0; j < 8; ++j) {
            const int hin = 32 * ib + 8 * (2 * st + j / 4) + 4 * h + j % 4;
            v[j] = (_Float16)p[OFF_W2 + hin * H + row];
        }
        A2[rb][ib][st][l] = v;
    }
    for (int q = tid; q < 2 * 2 * 16; q += MFT) {
        const int rb = q / 32, h = (q / 16) % 2, k = q % 16;
        const int row = 32 * rb + 8 * (k / 4) + 4 * h + k % 4;
        B1s[rb][h][k] = p[OFF_B1 + row];
        B2s[rb][h][k] = p[OFF_B2 + row];
        W3s[rb][h][k][0] = p[OFF_W3 + row * NO];
        W3s[rb][h][k][1] = p[OFF_W3 + row * NO + 1];
    }
    __syncthreads();
    const int lane = tid & 63, h = lane >> 5, l32 = lane & 31;
    const float b30 = p[OFF_B3], b31 = p[OFF_B3 + 1];
    const int ntiles = (M + 31) / 32;
    const int stride = gridDim.x * (MFT / 64);
    // the feature words of a tile (rows of F = 20 floats are 16-byte aligned:
    // four-float loads, zeros past feature 19); the next tile's are loaded
    // while the current one is multiplied
    static_assert(F == 20, "feature row of five 16-byte words");
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    auto load_x = [&](int t, float4 &w0, float4 &w1, float4 &w2) {
        const long long m = (long long)t * 32 + l32;
        const bool ok = t < ntiles && m < M;
        const float4 *xr = reinterpret_cast<const float4 *>(X + (ok ? m : 0) * F);
        w0 = ok ? xr[2 * h] : z4;
        w1 = ok ? xr[2 * h + 1] : z4;
        w2 = ok && h == 0 ? xr[4] : z4;
    };
    int t = blockIdx.x * (MFT / 64) + (tid >> 6);
    float4 c0, c1, c2;
    load_x(t, c0, c1, c2);
    for (; t < ntiles; t += stride) {
        const long long m = (long long)t * 32 + l32;
        const bool ok = m < M;
        float4 n0, n1, n2;
        load_x(t + stride, n0, n1, n2);
        // B1: features 16 s + 8 h + j of spin m
        f16x8_t xb[2];
        {
            const float v0[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
            const float v1[4] = {c2.x, c2.y, c2.z, c2.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                xb[0][j] = (_Float16)v0[j];
                xb[1][j] = (_Float16)(j < 4 ? v1[j] : 0.0f);
            }
        }
        c0 = n0;
        c1 = n1;
        c2 = n2;
        f32x16_t z1[2], z2[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
            for (int k = 0; k < 16; ++k) z1[rb][k] = B1s[rb][h][k];
#pragma unroll
            for (int st = 0; st < 2; ++st)
                z1[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A1[rb][st][lane], xb[st], z1[rb], 0, 0, 0);
        }
        // relu(Z1)^T as the B operand of layer 2, in the permuted K order
        f16x8_t hb[2][2];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int st = 0; st < 2; ++st)
#pragma unroll
                for (int j = 0; j < 8; ++j) hb[ib][st][j] = (_Float16)fmaxf(z1[ib][8 * st + j], 0.0f);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
            for (int k = 0; k < 16; ++k) z2[rb][k] = B2s[rb][h][k];
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                for (int st = 0; st < 2; ++st)
                    z2[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A2[rb][ib][st][lane], hb[ib][st], z2[rb], 0, 0, 0);
        }
        float o0 = 0.0f, o1 = 0.0f;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const float r = fmaxf(z2[rb][k], 0.0f);
                o0 = fmaf(r, W3s[rb][h][k][0], o0);
                o1 = fmaf(r, W3s[rb][h][k][1], o1);
            }
        o0 += __shfl_xor(o0, 32);
        o1 += __shfl_xor(o1, 32);
        if (h == 0 && ok) {
            out[m * NO] = o0 + b30;
            out[m * NO + 1] = o1 + b31;
        }
    }
}

// per instance: sigma_k (flip alignment) and loss sums
__global__ void __launch_bounds__(256) mlp_segment_k(const float *__restrict__ out, const float *__restrict__ lab,
                                                    const int *__restrict__ seg, float *__restrict__ sigma,
                                                    double *__restrict__ seg_loss) {
    __shared__ double red[4 * 2];
    const int k = blockIdx.x;
    double v[2] = {0.0, 0.0};
    for (int i = seg[k] + threadIdx.x; i < seg[k + 1]; i += 256) {
        const double m = tanh((double)out[2 * i]);
        const double s = lab[i];
        v[0] += (m - s) * (m - s);
        v[1] += (m + s) * (m + s);
    }
    block_sum<2>(v, red);
    if (threadIdx.x == 0) sigma[k] = v[0] <= v[1] ? 1.0f : -1.0f;
}

// Training step on the matrix cores (v_mfma_f32_32x32x2_f32, FP32 products
// and sums).  Each wave takes 32 spins at a time (one spin per lane column,
// as in the FP16 inference kernel: lane l, half h = l / 32, holds rows
// 8q + 4h + e of each 32-row block for spin l mod 32) and computes
//   Z1^T = W1^T X^T + b1, Z2^T = W2^T relu(Z1)^T + b2   (forward),
//   O = W3^T relu(Z2) + b3 on the vector ALUs, the per-spin loss and dO,
//   dH2 = (W3 dO) * [Z2 > 0], dH1^T = W2 dH2^T * [Z1 > 0]   (backward),
// the K = 2 steps of the layer products taking each lane's rows in the order
// it holds them (the weight operand permuted to match, every product summed
// once).  The weight gradients contract over spins, so each wave transposes
// its tile through two LDS buffers ([spin][feature], rows padded to 65
// words): dW2 = relu(Z1)^T dH2 and dW1 = X^T dH1 on the matrix cores, the
// bias gradients and dW3 = relu(Z2)^T dO as column sums on the vector ALUs.
// The weights are staged in LDS once per workgroup (the operand of a K step
// is then one conflict-free LDS read per lane, W2 in rows of 65 words so that
// both its row and its column order read across banks).
// The accumulators stay in registers over all of the wave's tiles; at the
// end the four waves of a workgroup add theirs into one partial in a fixed
// order (partial[block][param], loss_part[block]).  Without TRAIN the kernel
// only writes the two outputs of every spin.
constexpr int TT = 256;           // 4 waves
constexpr int PS = 65;            // padded row of W2 and of the transposition buffers
// LDS: the weights (W1 [f][j], W2 [j][b] in rows of PS, b1, b2, W3), then
// (training) the transposition buffers of the four waves
constexpr int kWLds = F * H + H * PS + 2 * H + H * NO;
constexpr size_t kFwdLds = (size_t)kWLds * 4;
constexpr size_t kTrainLds = (size_t)(kWLds + 4 * 2 * 32 * PS) * 4;

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool TRAIN>
__device__ __forceinline__ void mlp_mfma32(const MlpTrainArgs &a, float *smem) {
    static_assert(H == 64 && F <= 32 && F % 2 == 0 && NO == 2, "layer shapes of the MFMA training step");
    const float *__restrict__ p = a.params;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, h = lane >> 5, c = lane & 31;
    float *W1s = smem;                                        // W1[f][j] at f H + j
    float *W2s = W1s + F * H;                                 // W2[j][b] at j PS + b
    float *B1s = W2s + H * PS, *B2s = B1s + H, *W3s = B2s + H;
    float *P = smem + kWLds + (size_t)w * 2 * 32 * PS;        // this wave's buffers
    float *Q = P + 32 * PS;
    for (int q = tid; q < F * H; q += TT) W1s[q] = p[OFF_W1 + q];
    for (int q = tid; q < H * H; q += TT) W2s[(q / H) * PS + q % H] = p[OFF_W2 + q];
    for (int q = tid; q < H; q += TT) {
        B1s[q] = p[OFF_B1 + q];
        B2s[q] = p[OFF_B2 + q];
    }
    for (int q = tid; q < H * NO; q += TT) W3s[q] = p[OFF_W3 + q];
    __syncthreads();
    f32x16_t g2[4], g1[2];               // dW2 blocks (j-block, b-block), dW1 blocks (j-block)
    float gb1 = 0.f, gb2 = 0.f, gw30 = 0.f, gw31 = 0.f, gb30 = 0.f, gb31 = 0.f;
    double lsum = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 16; ++k) g2[u][k] = 0.f;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int k = 0; k < 16; ++k) g1[u][k] = 0.f;
    const float invM = 1.0f / float(a.M);
    const float b30 = p[OFF_B3], b31 = p[OFF_B3 + 1];
    const int ntiles = (a.M + 31) / 32;
    const int tstride = gridDim.x * (TT / 64);
    // features 2 i + h of spin 32 t + c (zeros past M); the next tile's are
    // loaded while the current one is multiplied
    auto load_x = [&](int t, float (&xd)[F / 2]) {
        const int m = t * 32 + c;
        const bool ok = t < ntiles && m < a.M;
        const float *xr = a.X + (long long)(ok ? m : 0) * F;
#pragma unroll
        for (int i = 0; i < F / 2; ++i) xd[i] = ok ? xr[2 * i + h] : 0.0f;
    };
    float xn[F / 2];
    int t = blockIdx.x * (TT / 64) + w;
    load_x(t, xn);
    for (; t < ntiles; t += tstride) {
        const int m = t * 32 + c;
        const bool ok = m < a.M;
        float xv[F / 2];
#pragma unroll
        for (int i = 0; i < F / 2; ++i) xv[i] = xn[i];
        load_x(t + tstride, xn);
        // the forward pass alone reads the weights from LDS in every tile (an
        // offset the compiler cannot see through keeps them out of the
        // registers, so that two waves fit a SIMD); the training step keeps
        // them in registers
        int wo = 0;
        if constexpr (!TRAIN) __asm__ volatile("" : "+v"(wo));
        const float *W1t = W1s + wo, *W2t = W2s + wo, *B1t = B1s + wo, *B2t = B2s + wo, *W3t = W3s + wo;
        // the spin's target sigma_k s_i, loaded before the products
        float tg = 0.0f;
        if constexpr (TRAIN)
            if (ok) tg = a.sigma[a.spin_inst[m]] * a.labels[m];
        f32x16_t z1[2], z2[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
            for (int k = 0; k < 16; ++k) z1[rb][k] = B1t[32 * rb + 8 * (k / 4) + 4 * h + k % 4];
#pragma unroll
            for (int i = 0; i < F / 2; ++i)
                z1[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(W1t[(2 * i + h) * H + 32 * rb + c], xv[i],
                                                             z1[rb], 0, 0, 0);
        }
#pragma unroll
        for (int rb2 = 0; rb2 < 2; ++rb2) {
#pragma unroll
            for (int k = 0; k < 16; ++k) z2[rb2][k] = B2t[32 * rb2 + 8 * (k / 4) + 4 * h + k % 4];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int j = 32 * rb + 8 * (k / 4) + 4 * h + k % 4;
                    z2[rb2] = __builtin_amdgcn_mfma_f32_32x32x2f32(W2t[j * PS + 32 * rb2 + c],
                                                                  fmaxf(z1[rb][k], 0.0f), z2[rb2], 0, 0, 0);
                }
        }
        float o0 = 0.0f, o1 = 0.0f;
#pragma unroll
        for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int b = 32 * rb2 + 8 * (k / 4) + 4 * h + k % 4;
                const float r = fmaxf(z2[rb2][k], 0.0f);
                o0 = fmaf(r, W3t[b * NO], o0);
                o1 = fmaf(r, W3t[b * NO + 1], o1);
            }
        o0 += __shfl_xor(o0, 32) + b30;
        o1 += __shfl_xor(o1, 32) + b31;
        if constexpr (!TRAIN) {
            if (h == 0 && ok) {
                a.out[(long long)m * NO] = o0;
                a.out[(long long)m * NO + 1] = o1;
            }
            continue;
        } else {
            // loss of the spin and the output gradient (zero past M)
            float d0 = 0.0f, d1 = 0.0f;
            if (ok) {
                const float mm = tanhf(o0);
                const float cc = 1.0f / (1.0f + expf(-o1));
                const float y = (mm * tg > 0.0f) ? 1.0f : 0.0f;
                d0 = 2.0f * (mm - tg) * (1.0f - mm * mm) * invM;
                d1 = LAMBDA_C * (cc - y) * invM;
                // BCE(sigmoid(o1), y) in the stable logit form softplus(o1) - y o1
                const float bce = fmaxf(o1, 0.0f) - y * o1 + log1pf(expf(-fabsf(o1)));
                if (h == 0) lsum += (double)(((mm - tg) * (mm - tg) + LAMBDA_C * bce) * invM);
            }
            f32x16_t dh2[2], dh1[2];
#pragma unroll
            for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int b = 32 * rb2 + 8 * (k / 4) + 4 * h + k % 4;
                    const float g = d0 * W3t[b * NO] + d1 * W3t[b * NO + 1];
                    dh2[rb2][k] = z2[rb2][k] > 0.0f ? g : 0.0f;
                }
#pragma unroll
            for (int rbj = 0; rbj < 2; ++rbj) {
#pragma unroll
                for (int k = 0; k < 16; ++k) dh1[rbj][k] = 0.0f;
#pragma unroll
                for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int b = 32 * rb2 + 8 * (k / 4) + 4 * h + k % 4;
                        dh1[rbj] = __builtin_amdgcn_mfma_f32_32x32x2f32(W2t[(32 * rbj + c) * PS + b], dh2[rb2][k],
                                                                       dh1[rbj], 0, 0, 0);
                    }
#pragma unroll
                for (int k = 0; k < 16; ++k) dh1[rbj][k] = z1[rbj][k] > 0.0f ? dh1[rbj][k] : 0.0f;
            }
            // dW2 += relu(Z1)^T dH2 over the tile's spins; db2
            wave_sync();
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int j = 32 * rb + 8 * (k / 4) + 4 * h + k % 4;
                    P[c * PS + j] = fmaxf(z1[rb][k], 0.0f);
                    Q[c * PS + j] = dh2[rb][k];
                }
            wave_sync();
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) {
                const int row = (2 * s2 + h) * PS + c;
                const float hj0 = P[row], hj1 = P[row + 32], db0 = Q[row], db1 = Q[row + 32];
                g2[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(hj0, db0, g2[0], 0, 0, 0);
                g2[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(hj0, db1, g2[1], 0, 0, 0);
                g2[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(hj1, db0, g2[2], 0, 0, 0);
                g2[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(hj1, db1, g2[3], 0, 0, 0);
            }
            for (int s = 0; s < 32; ++s) gb2 += Q[s * PS + lane];
            // dW1 += X^T dH1 (features padded to 32 rows with zeros); db1
            wave_sync();
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int k = 0; k < 16; ++k) P[c * PS + 32 * rb + 8 * (k / 4) + 4 * h + k % 4] = dh1[rb][k];
#pragma unroll
            for (int i = 0; i < F / 2; ++i) Q[c * PS + 2 * i + h] = xv[i];
            for (int f = F + h; f < 32; f += 2) Q[c * PS + f] = 0.0f;
            wave_sync();
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) {
                const int row = (2 * s2 + h) * PS + c;
                const float xf = Q[row];
                g1[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(xf, P[row], g1[0], 0, 0, 0);
                g1[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(xf, P[row + 32], g1[1], 0, 0, 0);
            }
            for (int s = 0; s < 32; ++s) gb1 += P[s * PS + lane];
            // dW3 += relu(Z2)^T dO; db3
            wave_sync();
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    P[c * PS + 32 * rb + 8 * (k / 4) + 4 * h + k % 4] = fmaxf(z2[rb][k], 0.0f);
            if (h == 0) {
                Q[2 * c] = d0;
                Q[2 * c + 1] = d1;
            }
            wave_sync();
            for (int s = 0; s < 32; ++s) {
                const float hv = P[s * PS + lane];
                gw30 = fmaf(hv, Q[2 * s], gw30);
                gw31 = fmaf(hv, Q[2 * s + 1], gw31);
                gb30 += Q[2 * s];
                gb31 += Q[2 * s + 1];
            }
        }
    }
    if constexpr (TRAIN) {
        // the workgroup's partial: the waves add theirs in order (wave 0 writes)
        for (int q = 1; q < 64; q <<= 1) lsum += __shfl_xor(lsum, q);
        __syncthreads();
        float *R = smem + kWLds;                        // NPAR floats, then 4 doubles
        double *RL = reinterpret_cast<double *>(R + ((NPAR + 1) & ~1));
        for (int v = 0; v < TT / 64; ++v) {
            if (w == v) {
                auto put = [&](int q, float val) { R[q] = v == 0 ? val : R[q] + val; };
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int j = 32 * (u >> 1) + 8 * (k / 4) + 4 * h + k % 4, b = 32 * (u & 1) + c;
                        put(OFF_W2 + j * H + b, g2[u][k]);
                    }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int f = 8 * (k / 4) + 4 * h + k % 4, j = 32 * u + c;
                        if (f < F) put(OFF_W1 + f * H + j, g1[u][k]);
                    }
                put(OFF_B1 + lane, gb1);
                put(OFF_B2 + lane, gb2);
                put(OFF_W3 + lane * NO, gw30);
                put(OFF_W3 + lane * NO + 1, gw31);
                if (lane == 0) {
                    put(OFF_B3, gb30);
                    put(OFF_B3 + 1, gb31);
                    RL[v] = lsum;
                }
            }
            __syncthreads();
        }
        float *part = a.partial + (long long)blockIdx.x * NPAR;
        for (int q = tid; q < NPAR; q += TT) part[q] = R[q];
        if (tid == 0) a.loss_part[blockIdx.x] = ((RL[0] + RL[1]) + RL[2]) + RL[3];
    }
}

// the training step: one wave per SIMD (its accumulators and operands take
// the whole register file)
__global__ void __launch_bounds__(TT) mlp_train_mfma_k(MlpTrainArgs a) {
    extern __shared__ __attribute__((aligned(16))) float smem[];
    mlp_mfma32<true>(a, smem);
}

// the forward pass alone (outputs for the flip alignment): at least two
// waves per SIMD (the weights are re-read from LDS in every tile)
__global__ void __launch_bounds__(TT, 2) mlp_forward_mfma32_k(MlpTrainArgs a) {
    extern __shared__ __attribute__((aligned(16))) float smem[];
    mlp_mfma32<false>(a, smem);
}

// Fixed-order sum of the workgroup partials, then Adam.  A workgroup of
// 1024 threads (16 waves) takes 64 parameters: wave v sums its sixteenth of
// the partials (eight interleaved running sums, loads in flight), the waves'
// sums are added in wave order.  The last workgroup adds the loss partials.
constexpr int AT = 1024, AP = 64;
__global__ void __launch_bounds__(AT) mlp_adam_k(MlpTrainArgs a, int nparts, float lr, int step) {
    __shared__ float ws[AT / 64][AP];
    __shared__ double ls[AT];
    const int lane = threadIdx.x & 63, v = threadIdx.x >> 6;
    if (blockIdx.x == gridDim.x - 1) {
        double x = 0.0;
        for (int q = threadIdx.x; q < nparts; q += AT) x += a.loss_part[q];
        ls[threadIdx.x] = x;
        __syncthreads();
        for (int s = AT / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) ls[threadIdx.x] += ls[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.loss[0] = ls[0];
        return;
    }
    const int q = blockIdx.x * AP + lane;
    const int per = (nparts + AT / 64 - 1) / (AT / 64);
    const int p0 = min(nparts, v * per), p1 = min(nparts, p0 + per);
    float s8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (q < NPAR) {
        int pp = p0;
        for (; pp + 8 <= p1; pp += 8)
#pragma unroll
            for (int u = 0; u < 8; ++u) s8[u] += a.partial[(long long)(pp + u) * NPAR + q];
        for (; pp < p1; ++pp) s8[(pp - p0) & 7] += a.partial[(long long)pp * NPAR + q];
    }
    ws[v][lane] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    __syncthreads();
    if (v == 0 && q < NPAR) {
        float g = 0.0f;
        for (int u = 0; u < AT / 64; ++u) g += ws[u][lane];
        if (a.grad_out) a.grad_out[q] = g;
        if (lr > 0.0f) {
            const float b1 = 0.9f, b2 = 0.999f;
            const float mo = b1 * a.mom[q] + (1.0f - b1) * g;
            const float ve = b2 * a.vel[q] + (1.0f - b2) * g * g;
            a.mom[q] = mo;
            a.vel[q] = ve;
            const float mh = mo / (1.0f - powf(b1, float(step)));
            const float vh = ve / (1.0f - powf(b2, float(step)));
            a.params[q] -= lr * mh / (sqrtf(vh) + 1e-8f);
        }
    }
}

__global__ void propose_k(ProposeArgs a) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= a.total_state) return;
    // locate instance: binary search over state offsets
    int lo = 0, hi = a.K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (a.inst_state[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const int k = lo;
    const int n = a.inst_n[k];
    const long long rel = t - a.inst_state[k];
    const int r = int(rel / n), i = int(rel % n);
    const long long sp = a.inst_spin[k] + i;
    const float m = tanhf(a.out[sp * NO]);
    const unsigned long long ctr = (((unsigned long long)k << 20) + (unsigned long long)r) * 65536ull + i;
    const double u = uniform01(ctr, a.seed);
    a.x[t] = float(a.amp * (a.alpha * m + (1.0 - a.alpha) * (2.0 * u - 1.0)));
    a.gam[t] = a.gamma0;
    if (r == 0) {
        const float c = 1.0f / (1.0f + expf(-a.out[sp * NO + 1]));
        a.eps[sp] = float(a.eps0 * exp(a.beta * (c - 0.5)));
    }
}

}  // namespace

hipError_t launch_features(const FeatArgs &a, int K, hipStream_t st) {
    const size_t lds = (size_t)a.nmax * 16 * sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&feat_k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    feat_k<<<K, FT, lds, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *params, const float *X, float *out, int M, bool fp16,
                              hipStream_t st) {
    if (M <= 0) return hipSuccess;
    const int g = (M + MT - 1) / MT;
    if (fp16) {
        // the feature rows are read as 16-byte words
        if (reinterpret_cast<uintptr_t>(X) % 16) return hipErrorInvalidValue;
        // one wave per 32 spins at a time; at most the workgroups that are
        // resident at once (two per CU), so each builds the weight operands once
        const int tiles = (M + 31) / 32;
        const int gm = std::min((tiles + MFT / 64 - 1) / (MFT / 64), 512);
        mlp_forward_mfma_k<<<gm, MFT, 0, st>>>(params, X, out, M);
    } else {
        mlp_forward_k<<<g, MT, 0, st>>>(params, X, out, M);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_train_step(const MlpTrainArgs &a, int K, int nparts, float lr, int step,
                                 hipStream_t st) {
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&mlp_train_mfma_k),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       int(kTrainLds));
    if (attr != hipSuccess) return attr;
    const int ntiles = (a.M + 31) / 32;
    const int gw = (ntiles + TT / 64 - 1) / (TT / 64);
    mlp_forward_mfma32_k<<<std::min(gw, 2048), TT, kFwdLds, st>>>(a);
    mlp_segment_k<<<K, 256, 0, st>>>(a.out, a.labels, a.seg, a.sigma, nullptr);
    const int np = std::max(1, std::min(nparts, gw));
    mlp_train_mfma_k<<<np, TT, kTrainLds, st>>>(a);
    mlp_adam_k<<<(NPAR + AP - 1) / AP + 1, AT, 0, st>>>(a, np, lr, step);
    return hipGetLastError();
}

hipError_t launch_propose(const ProposeArgs &a, hipStream_t st) {
    const long long g = (a.total_state + 255) / 256;
    propose_k<<<unsigned(g), 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace gd
