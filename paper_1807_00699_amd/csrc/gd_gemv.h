// Coupling product for a small number of trajectories (R columns, or 2R for
// complex amplitudes, at most 16): C_ir = sum_j J_ij Psi_jr of Eq. (main) as a
// matrix-vector product that streams J from HBM once per evaluation, fused
// with the same pointwise update of Eq. (main, gamma) as the GEMM kernels
// (gd_epilogue.h) and with the same energy mode for Eq. (h).
//
// At small R the product does 2 R flops per coupling read, far below the
// matrix-core ridge, so the work is bound by the bytes of J and belongs on
// the vector ALUs:
//  * a workgroup of W waves owns W x RPW consecutive rows of J; each wave
//    sweeps its RPW rows with one 16-byte load per lane and row (a wave
//    instruction reads 1 KiB of one row: 256 FP32, 512 BF16/FP16 or 1024 FP8
//    couplings), a few loads per row in flight;
//  * the operand columns Psi[c][k] of the R trajectories are staged in LDS as
//    FP32 (widened from the BF16/FP16 copy in the reduced-precision modes),
//    one chunk of K at a time, and shared by the W waves; inside each
//    wave-wide block the 16-byte slots are ordered so that lane l's j-th slot
//    sits at j * 64 + l: every ds_read_b128 of the inner loop reads 64
//    consecutive slots (no bank conflicts);
//  * each lane keeps RPW x CM partial sums in registers (FP32 fused
//    multiply-adds); at the end the wave reduces them with a transposing
//    butterfly: at each xor distance half of the remaining values go to the
//    partner, so RPW x CM sums cost about RPW x CM exchanges instead of six
//    each, and every lane ends with one finished sum;
//  * the sums pass through LDS to lanes r < R, which run the epilogue of four
//    consecutive rows of trajectory r (16-byte state accesses).
// The reduction order is fixed, so results are deterministic.
#pragma once
#include "gd_epilogue.h"

namespace gd {
namespace gemv {

// storage of J: FP32, FP8 E4M3 (exact for couplings such as {-1, 0, +1}),
// or the 16-bit operand type
// J_FP8N: FP8 couplings read four per lane at the positions of J_F32's
// 16-byte loads, so every lane multiplies and sums the couplings J_F32 gives
// it, in the same order: results equal those of FP32 couplings bit for bit
// when every coupling is exact in FP8 (FP32 solvers), with a quarter of the bytes
enum JKind : int { J_F32 = 0, J_FP8 = 1, J_B16 = 2, J_FP8N = 3 };

template <int JK>
constexpr int j_bytes() {
    return JK == J_F32 ? 4 : (JK == J_FP8 || JK == J_FP8N ? 1 : 2);
}

// couplings per lane per load (J_FP8N: the four of J_F32)
template <int JK>
constexpr int j_epl() {
    return JK == J_FP8 ? 16 : (JK == J_B16 ? 8 : 4);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// elements 4j .. 4j + 3 of a 16-byte word of J as FP32 (exact widening)
template <int JK, int OPT>
__device__ inline f32x4 widen_quad(const u32x4 &w, int j) {
    if constexpr (JK == J_F32) {
        (void)j;   // one quad per 16-byte word
        return f32x4{__uint_as_float(w[0]), __uint_as_float(w[1]), __uint_as_float(w[2]), __uint_as_float(w[3])};
    } else if constexpr (JK == J_FP8 || JK == J_FP8N) {
        const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8(int(w[j]), false);
        const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8(int(w[j]), true);
        return f32x4{lo[0], lo[1], hi[0], hi[1]};
    } else if constexpr (OPT == OP_BF16) {
        const unsigned int a = w[2 * j], b = w[2 * j + 1];
        return f32x4{__uint_as_float(a << 16), __uint_as_float(a & 0xFFFF0000u), __uint_as_float(b << 16),
                     __uint_as_float(b & 0xFFFF0000u)};
    } else {
        const unsigned int a = w[2 * j], b = w[2 * j + 1];
        const __half2 x = *reinterpret_cast<const __half2 *>(&a);
        const __half2 y = *reinterpret_cast<const __half2 *>(&b);
        const float2 fx = __half22float2(x), fy = __half22float2(y);
        return f32x4{fx.x, fx.y, fy.x, fy.y};
    }
}

// four consecutive operands k .. k + 3 of one column as FP32
template <int OPT>
__device__ inline f32x4 load_operand4(const void *B, long long off) {
    if constexpr (OPT == OP_F32) {
        return *reinterpret_cast<const f32x4 *>(static_cast<const float *>(B) + off);
    } else {
        const uint2 w = *reinterpret_cast<const uint2 *>(static_cast<const unsigned short *>(B) + off);
        if constexpr (OPT == OP_BF16) {
            return f32x4{__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u), __uint_as_float(w.y << 16),
                         __uint_as_float(w.y & 0xFFFF0000u)};
        } else {
            const __half2 x = *reinterpret_cast<const __half2 *>(&w.x);
            const __half2 y = *reinterpret_cast<const __half2 *>(&w.y);
            const float2 fx = __half22float2(x), fy = __half22float2(y);
            return f32x4{fx.x, fx.y, fy.x, fy.y};
        }
    }
}

// Sum of v[m] over the 64 lanes for every m < M (M a power of two <= 64):
// the value of index (lane >> (6 - log2 M)) is returned in every lane.
template <int M>
__device__ inline float wave_transpose_sum(float (&v)[M], int lane) {
    static_assert(M >= 1 && M <= 64 && (M & (M - 1)) == 0, "M: power of two <= 64");
    int m = 32;
#pragma unroll
    for (int K = M; K > 1; K >>= 1) {
        const bool up = (lane & m) != 0;
#pragma unroll
        for (int k = 0; k < K / 2; ++k) {
            // both values first, as plain register values: otherwise the
            // compiler turns the lane-dependent choice into a lane-dependent
            // index into v, which moves v to scratch memory
            float lo = v[k], hi = v[k + K / 2];
            __asm__("" : "+v"(lo), "+v"(hi));
            const float send = up ? lo : hi;
            const float keep = up ? hi : lo;
            v[k] = keep + __shfl_xor(send, m);
        }
        m >>= 1;
    }
    float s = v[0];
    for (; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    return s;
}

// 512-thread workgroups leave each wave 256 registers, 1024-thread ones
// 128: too few for the widened reduced-precision couplings of many columns,
// or for many columns at all
constexpr bool fits_registers(int jk, int cm, int w) {
    if (w >= 16) return cm <= 2;
    return !(w >= 8 && ((jk == J_FP8 && cm >= 8) || (jk == J_B16 && cm >= 16)));
}

template <int M>
constexpr int ilog2() {
    return M <= 1 ? 0 : 1 + ilog2<M / 2>();
}

// LDS floats per staged column: as much of K as the LDS budget of
// `budget` floats holds for CM columns, a multiple of the wave-wide block
template <int JK, int CM>
constexpr int chunk_width(int budget) {
    constexpr int BW = 64 * j_epl<JK>();
    const int w = budget / CM / BW * BW;
    return w < BW ? BW : w;
}

template <int MODE, bool CPLX, int JK, int OPT, int CM, int W, int RPW, int KCM, int U, int KS>
__global__ void __launch_bounds__(64 * W) gemv_step_k(DenseStepArgs a) {
    constexpr int JB = j_bytes<JK>();
    constexpr int EPL = j_epl<JK>();   // couplings per lane per load
    constexpr int QPL = EPL / 4;   // operand slots (4 floats) per lane per load
    constexpr int BW = 64 * EPL;   // columns of one wave-wide load
    constexpr int SB = BW / 4;     // slots per block
    constexpr int M = RPW * CM;
    constexpr int NG = RPW / 4;    // groups of four rows per wave
    constexpr int WR = W / KS;     // waves along the rows; KS waves split each row group's K
    static_assert(KCM % BW == 0 && RPW % 4 == 0, "chunk of whole blocks; groups of four rows");
    static_assert(W % KS == 0, "K groups of whole waves");
    __shared__ __attribute__((aligned(16))) float sp[CM * KCM];
    __shared__ float so[W][M];
    __shared__ double se[WR][CM];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int Np = a.Np;
    const int R = a.R;
    const int C = (CPLX ? 2 : 1) * R;
    const int wr = wave % WR, kp = wave / WR;   // row group, K part (blocks kp, kp + KS, ...)
    const int i0 = blockIdx.x * (WR * RPW) + wr * RPW;
    const unsigned char *Jb = static_cast<const unsigned char *>(a.J);

    // the state operands of the epilogue do not depend on the sums: lanes
    // r < R load them first, so their latency hides under the J stream
    // (1024-thread workgroups, 128 registers per lane, load them at the end)
    constexpr bool EPI_EARLY = W * 64 <= 512;
    EpiIn pre[NG];
    if constexpr (MODE != MODE_ENERGY && EPI_EARLY) {
        if (kp == 0 && lane < R) {
#pragma unroll
            for (int g = 0; g < NG; ++g) epi_load<MODE, CPLX>(a, i0 + 4 * g, lane, pre[g]);
        }
    }

    float acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0f;

    // U of this K part's wave-wide blocks (t -> block t KS + kp of the chunk)
    // of the wave's RPW rows: U x RPW 16-byte loads per lane
    auto load_batch = [&](u32x4 (&jw)[U][RPW], int k0, int b0, int nb) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + ((b0 + u) * KS + kp) * BW + EPL * lane;
            const bool ok = (b0 + u < nb) && k < Np;
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                if constexpr (JK == J_FP8N)
                    jw[u][q] = u32x4{ok ? *reinterpret_cast<const unsigned int *>(Jb + (long long)(i0 + q) * Np + k)
                                        : 0u, 0u, 0u, 0u};
                else
                    jw[u][q] = ok ? *reinterpret_cast<const u32x4 *>(Jb + ((long long)(i0 + q) * Np + k) * JB)
                                  : u32x4{0u, 0u, 0u, 0u};
            }
        }
    };
    auto fma_batch = [&](const u32x4 (&jw)[U][RPW], int b0, int nb) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (b0 + u < nb) {
#pragma unroll
                for (int j = 0; j < QPL; ++j) {
                    f32x4 jf[RPW];
#pragma unroll
                    for (int q = 0; q < RPW; ++q) jf[q] = widen_quad<JK, OPT>(jw[u][q], j);
                    const int slot = ((b0 + u) * KS + kp) * SB + j * 64 + lane;
#pragma unroll
                    for (int c = 0; c < CM; ++c) {
                        const f32x4 p = *reinterpret_cast<const f32x4 *>(&sp[c * KCM + 4 * slot]);
#pragma unroll
                        for (int q = 0; q < RPW; ++q) {
                            float s = acc[q * CM + c];
                            s = __builtin_fmaf(jf[q][0], p[0], s);
                            s = __builtin_fmaf(jf[q][1], p[1], s);
                            s = __builtin_fmaf(jf[q][2], p[2], s);
                            s = __builtin_fmaf(jf[q][3], p[3], s);
                            acc[q * CM + c] = s;
                        }
                    }
                }
            }
        }
    };

    // operand staging: a chunk is SMAX 16-byte slots per thread.  Up to 8 of
    // them are held in registers: all their loads are issued together and, when
    // the whole chunk fits (SMAX <= 8), the next chunk's loads are issued before
    // the current chunk is multiplied; larger chunks are staged in rounds of 8
    constexpr int NT = 64 * W;
    constexpr int SMAX = (CM * KCM / 4 + NT - 1) / NT;
    constexpr int SREG = SMAX < 8 ? SMAX : 8;
    constexpr int ROUNDS = (SMAX + SREG - 1) / SREG;
    constexpr bool PREFETCH = ROUNDS == 1;
    f32x4 stg[SREG];
    auto chunk_cols = [&](int k0) {
        const int rem = Np - k0;
        return rem >= KCM ? KCM : (rem + BW - 1) / BW * BW;
    };
    auto stage_load = [&](int k0, int kc, int rnd) {
        const int ns = kc / 4;
#pragma unroll
        for (int u = 0; u < SREG; ++u) {
            const int idx = tid + (rnd * SREG + u) * NT;
            stg[u] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (idx < CM * ns) {
                const int c = idx / ns, t = idx - c * ns;
                const int k = k0 + 4 * t;
                if (c < C && k < Np) {
                    const int p = c >= R ? 1 : 0;
                    const int r = c - p * R;
                    stg[u] = load_operand4<OPT>(a.B, p * a.plane_stride + (long long)r * Np + k);
                }
            }
        }
    };
    auto stage_store = [&](int kc, int rnd) {
        const int ns = kc / 4;
#pragma unroll
        for (int u = 0; u < SREG; ++u) {
            const int idx = tid + (rnd * SREG + u) * NT;
            if (idx < CM * ns) {
                const int c = idx / ns, t = idx - c * ns;
                const int blk = t / SB, tin = t - blk * SB;
                const int pos = blk * SB + (tin % QPL) * 64 + tin / QPL;
                *reinterpret_cast<f32x4 *>(&sp[c * KCM + 4 * pos]) = stg[u];
            }
        }
    };

    u32x4 cur[U][RPW], nxt[U][RPW];
    int kc = chunk_cols(0);
    stage_load(0, kc, 0);
    auto part_blocks = [&](int kcols) { return (kcols / BW - kp + KS - 1) / KS; };
    load_batch(cur, 0, 0, part_blocks(kc));
    stage_store(kc, 0);
    for (int rnd = 1; rnd < ROUNDS; ++rnd) {
        stage_load(0, kc, rnd);
        stage_store(kc, rnd);
    }
    __syncthreads();
    for (int k0 = 0; k0 < Np; k0 += KCM) {
        const int nb = part_blocks(kc);
        const int k1 = k0 + KCM;
        const int kc1 = k1 < Np ? chunk_cols(k1) : 0;
        if (PREFETCH && kc1) stage_load(k1, kc1, 0);   // the next chunk's operands, in flight meanwhile
        // software pipeline: the next batch's loads are in flight while the
        // current batch is multiplied
        for (int b0 = 0; b0 < nb; b0 += U) {
            const bool more = b0 + U < nb;
            if (more) load_batch(nxt, k0, b0 + U, nb);
            fma_batch(cur, b0, nb);
            if (more) {
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int q = 0; q < RPW; ++q) cur[u][q] = nxt[u][q];
            }
        }
        if (kc1) {
            load_batch(cur, k1, 0, part_blocks(kc1));   // the next chunk's first loads do not touch LDS
            __syncthreads();                    // every wave is done with this chunk's operands
            for (int rnd = 0; rnd < ROUNDS; ++rnd) {
                if (!PREFETCH) stage_load(k1, kc1, rnd);
                stage_store(kc1, rnd);
            }
            __syncthreads();
        }
        kc = kc1;
    }

    // one finished sum per lane: index (q, c) = lane >> (6 - log2 M)
    const float tot = wave_transpose_sum<M>(acc, lane);
    constexpr int SH = 6 - ilog2<M>();
    if ((lane & ((1 << SH) - 1)) == 0) so[wave][lane >> SH] = tot;
    __syncthreads();

    // the row group's sum over its K parts, in a fixed order
    auto row_sum = [&](int row, int col) {
        float v = so[wr][row * CM + col];
#pragma unroll
        for (int p = 1; p < KS; ++p) v += so[wr + p * WR][row * CM + col];
        return v;
    };
    if constexpr (MODE == MODE_ENERGY) {
        if (kp == 0 && lane < R) {
            double e = 0.0;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                f32x4 tr, ti = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                    tr[e4] = row_sum(4 * g + e4, lane);
                    if (CPLX) ti[e4] = row_sum(4 * g + e4, R + lane);
                }
                e += energy_terms4<CPLX>(a, i0 + 4 * g, lane, tr, ti);
            }
            se[wr][lane] = e;
        }
        __syncthreads();
        if (wave == 0 && lane < R) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < WR; ++w) s += se[w][lane];
            a.partial[(long long)blockIdx.x * a.Rp + lane] = s;
        }
    } else {
        if (kp == 0 && lane < R) {
            bool bad = false;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                f32x4 cr, ci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                    cr[e4] = row_sum(4 * g + e4, lane);
                    if (CPLX) ci[e4] = row_sum(4 * g + e4, R + lane);
                }
                if constexpr (!EPI_EARLY) epi_load<MODE, CPLX>(a, i0 + 4 * g, lane, pre[g]);
                bad |= epi_apply<MODE, CPLX, OPT>(a, i0 + 4 * g, lane, true, pre[g], cr, ci);
            }
            if (bad) a.flags[lane] = 1;
        }
    }
}

// Variants {W waves, RPW rows per wave, LDS budget in floats for the staged
// operand chunk, U blocks of loads in flight per row, KS waves splitting the
// K range of one row group}.  Rows per workgroup (W / KS) x RPW are 16 or 32
// (the row tile of the energy partials); 16 puts 256 workgroups, one per CU,
// on N = 4096, and KS > 1 gives each CU 2 or 4 times the waves (and loads in
// flight) at the price of one more fixed-order sum through LDS.  Variants 5
// and 6 keep 128 KiB of J in flight per CU on N = 4096 (twice the others).
#define GD_GEMV_VARIANTS(X)    \
    X(0, 4, 4, 8192, 2, 1)     \
    X(1, 4, 4, 8192, 4, 1)     \
    X(2, 8, 4, 8192, 2, 1)     \
    X(3, 8, 4, 8192, 2, 2)     \
    X(4, 16, 4, 8192, 1, 4)    \
    X(5, 8, 4, 8192, 4, 2)     \
    X(6, 16, 4, 8192, 2, 4)

template <int MODE, bool CPLX, int JK, int OPT, int CM, int W, int RPW, int BUD, int U, int KS>
hipError_t launch_one(const DenseStepArgs &a, hipStream_t st) {
    constexpr int KCM = chunk_width<JK, CM>(BUD);
    // 16-bit and FP8 couplings widen to 2x / 4x the registers per load: with
    // 8 or more columns one batch in flight keeps the kernel out of scratch
    constexpr int UE = (JK != J_F32 && JK != J_FP8N && CM >= 8) ? 1 : U;
    if constexpr (!fits_registers(JK, CM, W)) {
        return hipErrorInvalidValue;
    } else {
        const dim3 grid(a.Np / (W / KS * RPW)), block(64 * W);
        gemv_step_k<MODE, CPLX, JK, OPT, CM, W, RPW, KCM, UE, KS><<<grid, block, 0, st>>>(a);
    }
    return hipGetLastError();
}

template <bool CPLX, int JK, int OPT, int CM, int W, int RPW, int BUD, int U, int KS>
hipError_t launch_modes(int mode, const DenseStepArgs &a, hipStream_t st) {
    switch (mode) {
    case MODE_EULER: return launch_one<MODE_EULER, CPLX, JK, OPT, CM, W, RPW, BUD, U, KS>(a, st);
    case MODE_RK1: return launch_one<MODE_RK1, CPLX, JK, OPT, CM, W, RPW, BUD, U, KS>(a, st);
    case MODE_RK2: return launch_one<MODE_RK2, CPLX, JK, OPT, CM, W, RPW, BUD, U, KS>(a, st);
    case MODE_RK3: return launch_one<MODE_RK3, CPLX, JK, OPT, CM, W, RPW, BUD, U, KS>(a, st);
    case MODE_RK4: return launch_one<MODE_RK4, CPLX, JK, OPT, CM, W, RPW, BUD, U, KS>(a, st);
    case MODE_ENERGY: return launch_one<MODE_ENERGY, CPLX, JK, OPT, CM, W, RPW, BUD, U, KS>(a, st);
    default: return hipErrorInvalidValue;
    }
}

// columns C = P R -> compiled column capacity CM (power of two)
template <int JK, int OPT, int W, int RPW, int BUD, int U, int KS>
hipError_t launch_cols(bool cplx, int mode, const DenseStepArgs &a, hipStream_t st) {
    const int C = (cplx ? 2 : 1) * a.R;
    if (cplx) {
        if (C <= 2) return launch_modes<true, JK, OPT, 2, W, RPW, BUD, U, KS>(mode, a, st);
        if (C <= 4) return launch_modes<true, JK, OPT, 4, W, RPW, BUD, U, KS>(mode, a, st);
        if (C <= 8) return launch_modes<true, JK, OPT, 8, W, RPW, BUD, U, KS>(mode, a, st);
        if (C <= 16) return launch_modes<true, JK, OPT, 16, W, RPW, BUD, U, KS>(mode, a, st);
    } else {
        if (C <= 1) return launch_modes<false, JK, OPT, 1, W, RPW, BUD, U, KS>(mode, a, st);
        if (C <= 2) return launch_modes<false, JK, OPT, 2, W, RPW, BUD, U, KS>(mode, a, st);
        if (C <= 4) return launch_modes<false, JK, OPT, 4, W, RPW, BUD, U, KS>(mode, a, st);
        if (C <= 8) return launch_modes<false, JK, OPT, 8, W, RPW, BUD, U, KS>(mode, a, st);
        if (C <= 16) return launch_modes<false, JK, OPT, 16, W, RPW, BUD, U, KS>(mode, a, st);
    }
    return hipErrorInvalidValue;
}

// compiled column capacity (a power of two) for C = P R columns
inline int column_capacity(int C) {
    int cm = 1;
    while (cm < C) cm *= 2;
    return cm;
}

template <int JK, int OPT>
hipError_t launch_variant(int idx, bool cplx, int mode, const DenseStepArgs &a, hipStream_t st) {
    if (a.R < 1 || (cplx ? 2 : 1) * a.R > 16 || a.Np % 32) return hipErrorInvalidValue;
#define GD_GEMV_CASE(id, w, rpw, bud, u, ks) \
    case id: return launch_cols<JK, OPT, w, rpw, bud, u, ks>(cplx, mode, a, st);
    switch (idx) { GD_GEMV_VARIANTS(GD_GEMV_CASE) }
#undef GD_GEMV_CASE
    return hipErrorInvalidValue;
}

}  // namespace gemv
}  // namespace gd
