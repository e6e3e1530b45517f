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
//  mlp_*       20 -> 64 -> 64 -> 2 ReLU network: FP32 forward, per-instance
//              flip-invariant loss, backward, weight-gradient partials over
//              spin chunks, fixed-order reduction fused with Adam; FP16
//              inference on the matrix cores (FP32 accumulation).
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

// backward per spin: dO, dH2, dH1 and the activations needed for weight grads
// Activations and their gradients are written feature-major ([H][M]), so the
// stores of a wave (consecutive spins) are contiguous.
__global__ void __launch_bounds__(MT) mlp_backward_k(MlpTrainArgs a) {
    __shared__ float sp[NPAR];
    for (int q = threadIdx.x; q < NPAR; q += MT) sp[q] = a.params[q];
    __syncthreads();
    const int m = blockIdx.x * MT + threadIdx.x;
    if (m >= a.M) return;
    const int k = a.spin_inst[m];
    float x[F], z1[H], z2[H], o[NO];
    for (int f = 0; f < F; ++f) x[f] = a.X[(long long)m * F + f];
    mlp_fwd1(sp, x, z1, z2, o);
    const float mm = tanhf(o[0]);
    const float cc = 1.0f / (1.0f + expf(-o[1]));
    const float t = a.sigma[k] * a.labels[m];
    const float y = (mm * t > 0.0f) ? 1.0f : 0.0f;
    const float invM = 1.0f / float(a.M);
    const float d0 = 2.0f * (mm - t) * (1.0f - mm * mm) * invM;
    const float d1 = LAMBDA_C * (cc - y) * invM;
    // BCE(sigmoid(o1), y) in the stable logit form softplus(o1) - y o1
    const float bce = fmaxf(o[1], 0.0f) - y * o[1] + log1pf(expf(-fabsf(o[1])));
    a.spin_loss[m] = ((mm - t) * (mm - t) + LAMBDA_C * bce) * invM;
    a.dO[(long long)m * NO] = d0;
    a.dO[(long long)m * NO + 1] = d1;
    float dh2[H];
    for (int b = 0; b < H; ++b) {
        const float g = d0 * sp[OFF_W3 + b * NO] + d1 * sp[OFF_W3 + b * NO + 1];
        dh2[b] = z2[b] > 0.0f ? g : 0.0f;
        a.H2[(long long)b * a.M + m] = fmaxf(z2[b], 0.0f);
        a.dH2[(long long)b * a.M + m] = dh2[b];
    }
    for (int j = 0; j < H; ++j) {
        float g = 0.0f;
        for (int b = 0; b < H; ++b) g += dh2[b] * sp[OFF_W2 + j * H + b];
        a.H1[(long long)j * a.M + m] = fmaxf(z1[j], 0.0f);
        a.dH1[(long long)j * a.M + m] = z1[j] > 0.0f ? g : 0.0f;
    }
}

// weight-gradient partials: block p reduces spins [p*chunk, (p+1)*chunk) into
// partial[p][NPAR], each parameter summed over the spins in order.  Tiles of
// WG_TILE spins are staged in LDS; register blocks per thread: a 4 x 4 block
// of W2 (16 products per 8 LDS reads), 5 entries of one W1 column, and one of
// B1 / B2 / W3 (plus B3 for two threads).
constexpr int WG_TILE = 32;
typedef float f32x4 __attribute__((ext_vector_type(4)));
static_assert(MT == 256 && H == 64 && F == 20 && NO == 2, "thread map of mlp_wgrad_k");
__global__ void __launch_bounds__(MT) mlp_wgrad_k(MlpTrainArgs a, int chunk) {
    // rows padded to H + 4 floats: the transposing LDS stores (consecutive
    // spins) spread over banks, the 16-byte reads stay aligned
    constexpr int HP = H + 4;
    __shared__ __attribute__((aligned(16))) float sX[WG_TILE][F], sH1[WG_TILE][HP], sH2[WG_TILE][HP];
    __shared__ __attribute__((aligned(16))) float sD1[WG_TILE][HP], sD2[WG_TILE][HP], sDO[WG_TILE][NO];
    const int t = threadIdx.x;
    const int j0 = (t / 16) * 4, b0 = (t % 16) * 4;    // W2 block
    const int wj = t % 64, f0 = (t / 64) * 5;           // W1: rows f0..f0+4 of column wj
    float w2[4][4], w1[5], one = 0.0f, b3 = 0.0f;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) w2[u][v] = 0.0f;
#pragma unroll
    for (int u = 0; u < 5; ++u) w1[u] = 0.0f;
    const int m0 = blockIdx.x * chunk;
    const int m1 = min(a.M, m0 + chunk);
    for (int r0 = m0; r0 < m1; r0 += WG_TILE) {
        const int cnt = min(WG_TILE, m1 - r0);
        for (int q = t; q < WG_TILE * H; q += MT) {
            const int r = q % WG_TILE, c = q / WG_TILE;     // feature-major sources
            const bool in = r < cnt;
            const long long mc = (long long)c * a.M + r0 + r;
            sH1[r][c] = in ? a.H1[mc] : 0.0f;
            sH2[r][c] = in ? a.H2[mc] : 0.0f;
            sD1[r][c] = in ? a.dH1[mc] : 0.0f;
            sD2[r][c] = in ? a.dH2[mc] : 0.0f;
        }
        for (int q = t; q < WG_TILE * F; q += MT) {
            const int r = q / F, c = q % F;
            sX[r][c] = r < cnt ? a.X[(long long)(r0 + r) * F + c] : 0.0f;
        }
        if (t < WG_TILE * NO) {
            const int r = t / NO, c = t % NO;
            sDO[r][c] = r < cnt ? a.dO[(long long)(r0 + r) * NO + c] : 0.0f;
        }
        __syncthreads();
        for (int r = 0; r < WG_TILE; ++r) {
            const f32x4 h1 = *reinterpret_cast<const f32x4 *>(&sH1[r][j0]);
            const f32x4 d2 = *reinterpret_cast<const f32x4 *>(&sD2[r][b0]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) w2[u][v] = fmaf(h1[u], d2[v], w2[u][v]);
            const float d1 = sD1[r][wj];
#pragma unroll
            for (int u = 0; u < 5; ++u) w1[u] = fmaf(sX[r][f0 + u], d1, w1[u]);
            if (t < 64) one += sD1[r][t];                                      // B1
            else if (t < 128) one += sD2[r][t - 64];                           // B2
            else one = fmaf(sH2[r][(t - 128) / 2], sDO[r][(t - 128) % 2], one);  // W3
            if (t < NO) b3 += sDO[r][t];                                       // B3
        }
        __syncthreads();
    }
    float *part = a.partial + (long long)blockIdx.x * NPAR;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) part[OFF_W2 + (j0 + u) * H + b0 + v] = w2[u][v];
#pragma unroll
    for (int u = 0; u < 5; ++u) part[OFF_W1 + (f0 + u) * H + wj] = w1[u];
    if (t < 64) part[OFF_B1 + t] = one;
    else if (t < 128) part[OFF_B2 + t - 64] = one;
    else part[OFF_W3 + (t - 128)] = one;
    if (t < NO) part[OFF_B3 + t] = b3;
}

// fixed-order sum of the partials, then Adam; loss = fixed-order sum of spin losses
__global__ void __launch_bounds__(MT) mlp_adam_k(MlpTrainArgs a, int nparts, float lr, int step) {
    const int q = blockIdx.x * MT + threadIdx.x;
    if (q < NPAR) {
        // eight interleaved running sums (independent loads in flight),
        // combined in a fixed order
        float s8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int pp = 0;
        for (; pp + 8 <= nparts; pp += 8)
#pragma unroll
            for (int u = 0; u < 8; ++u) s8[u] += a.partial[(long long)(pp + u) * NPAR + q];
        for (; pp < nparts; ++pp) s8[pp & 7] += a.partial[(long long)pp * NPAR + q];
        const float g = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
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

// loss = sum of the per-spin terms, fixed order (strided per thread, then a tree)
__global__ void __launch_bounds__(1024) mlp_loss_k(const float *__restrict__ spin_loss, int M,
                                                  double *__restrict__ loss) {
    __shared__ double s[1024];
    double v = 0.0;
    for (int m = threadIdx.x; m < M; m += 1024) v += spin_loss[m];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = s[0];
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
    const int g = (a.M + MT - 1) / MT;
    mlp_forward_k<<<g, MT, 0, st>>>(a.params, a.X, a.out, a.M);
    mlp_segment_k<<<K, 256, 0, st>>>(a.out, a.labels, a.seg, a.sigma, nullptr);
    mlp_backward_k<<<g, MT, 0, st>>>(a);
    const int chunk = (a.M + nparts - 1) / nparts;
    mlp_wgrad_k<<<nparts, MT, 0, st>>>(a, chunk);
    mlp_adam_k<<<(NPAR + MT - 1) / MT, MT, 0, st>>>(a, nparts, lr, step);
    mlp_loss_k<<<1, 1024, 0, st>>>(a.spin_loss, a.M, a.loss);
    return hipGetLastError();
}

hipError_t launch_propose(const ProposeArgs &a, hipStream_t st) {
    const long long g = (a.total_state + 255) / 256;
    propose_k<<<unsigned(g), 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace gd
