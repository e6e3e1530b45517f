// Reduced-precision coupling step: the coupling product of Eq. (main) with
// BF16 or FP16 operands and FP32 accumulation on the matrix cores
// (v_mfma_f32_32x32x16_bf16 / _f16), the amplitude/gain update in FP32.
//
// J is stored either in the operand type or, when every coupling is exactly
// representable there (e.g. couplings in {-1, 0, +1}), in FP8 (OCP E4M3,
// one byte per coupling) and widened exactly to the operand type: while it is
// staged into LDS in the register-staged variants (v_cvt_pk_f32_fp8, then the
// top 16 bits: FP8 values have at most four significant bits, so the
// truncation is exact), after the LDS read in the direct-to-LDS variants
// further below (J stays FP8 in LDS there).  The operand Psi
// is a BF16/FP16 copy of the FP32 amplitudes that the epilogue of the
// previous step writes next to them; the epilogue itself reads and writes the
// FP32 state (gd_epilogue.h).
//
// Tiling: workgroup BM x BN (GEMM columns), WM x WN waves, each wave a grid of
// 32x32 MFMA blocks.  The register-staged variants hold both tiles in LDS as
// [row][k] in the operand type with an 8-element pad per row; each lane
// fetches the 8 operands of its half-wave K slice with one ds_read_b128.
// Complex tiles pair real and
// imaginary column blocks inside a wave as in the FP32 kernel.
#pragma once
#include "gd_epilogue.h"

namespace gd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline void tile_map_lp(int b, int nblk, int n_mt, int n_ct, int &mt, int &ct) {
    int t = b;
    if ((nblk & 7) == 0) t = (b & 7) * (nblk >> 3) + (b >> 3);
    const int gm = 8;
    const int width = gm * n_ct;
    const int group = t / width;
    const int first = group * gm;
    const int gsz = min(gm, n_mt - first);
    const int in = t - group * width;
    mt = first + in % gsz;
    ct = in / gsz;
}

// four FP8 (E4M3) bytes -> four 16-bit operands packed in two dwords
template <int OPT>
__device__ inline void widen_fp8x4(unsigned int w, unsigned int &lo, unsigned int &hi) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f32x2 a = __builtin_amdgcn_cvt_pk_f32_fp8(int(w), false);
    const f32x2 b = __builtin_amdgcn_cvt_pk_f32_fp8(int(w), true);
    if constexpr (OPT == OP_BF16) {
        lo = (__float_as_uint(a[0]) >> 16) | (__float_as_uint(a[1]) & 0xFFFF0000u);
        hi = (__float_as_uint(b[0]) >> 16) | (__float_as_uint(b[1]) & 0xFFFF0000u);
    } else {
        const __half2 x = __floats2half2_rn(a[0], a[1]);
        const __half2 y = __floats2half2_rn(b[0], b[1]);
        lo = *reinterpret_cast<const unsigned int *>(&x);
        hi = *reinterpret_cast<const unsigned int *>(&y);
    }
}

template <int OPT>
__device__ inline f32x16 mfma32(u32x4 a, u32x4 b, f32x16 c) {
    if constexpr (OPT == OP_BF16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

template <int BM, int BN, int BK, int WM, int WN, bool CPLX, int MODE, int OPT, bool JFP8>
__global__ void __launch_bounds__(64 * WM * WN)
dense_step_lp(DenseStepArgs a) {
    constexpr int LDP = BK + 8;            // LDS row pitch in 16-bit elements
    constexpr int NT = 64 * WM * WN;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int MB = TM / 32, NB = TN / 32;
    constexpr int NP = CPLX ? NB / 2 : NB;
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    static_assert(!CPLX || (NB % 2 == 0), "complex waves pair re/im blocks");
    // global loads are 16 bytes: 16 FP8 couplings or 8 16-bit values
    constexpr int AQ = JFP8 ? BK / 16 : BK / 8;     // 16-byte loads per A row chunk
    constexpr int BQ = BK / 8;                      // 16-byte loads per B row chunk
    constexpr int AL = BM * AQ / NT, BL = BN * BQ / NT;
    static_assert(BM * AQ % NT == 0 && BN * BQ % NT == 0, "load split");

    __shared__ __attribute__((aligned(16))) unsigned short lds[2][(BM + BN) * LDP];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int n_mt = a.Np / BM, n_ct = a.Rp / TRAJ;
    int mt, ct;
    tile_map_lp(blockIdx.x, gridDim.x, n_mt, n_ct, mt, ct);
    const int m0 = mt * BM, r0 = ct * TRAJ;
    const long long Np = a.Np;
    const unsigned char *J8 = static_cast<const unsigned char *>(a.J);
    const unsigned short *J16 = static_cast<const unsigned short *>(a.J);
    const unsigned short *Bop = static_cast<const unsigned short *>(a.B);

    u32x4 ra[AL], rb[BL];
    auto gload = [&](int k0) {
#pragma unroll
        for (int u = 0; u < AL; ++u) {
            const int q = tid + u * NT;
            const int row = q / AQ, kq = q % AQ;
            if constexpr (JFP8)
                ra[u] = *reinterpret_cast<const u32x4 *>(J8 + (m0 + row) * Np + k0 + kq * 16);
            else
                ra[u] = *reinterpret_cast<const u32x4 *>(J16 + (m0 + row) * Np + k0 + kq * 8);
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int q = tid + u * NT;
            const int col = q / BQ, kq = q % BQ;
            const int plane = CPLX ? col / (BN / 2) : 0;
            const int tr = CPLX ? col % (BN / 2) : col;
            rb[u] = *reinterpret_cast<const u32x4 *>(Bop + plane * a.plane_stride + (r0 + tr) * Np +
                                                     k0 + kq * 8);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < AL; ++u) {
            const int q = tid + u * NT;
            const int row = q / AQ, kq = q % AQ;
            if constexpr (JFP8) {
                unsigned int x0, x1, x2, x3, x4, x5, x6, x7;
                widen_fp8x4<OPT>(ra[u][0], x0, x1);
                widen_fp8x4<OPT>(ra[u][1], x2, x3);
                widen_fp8x4<OPT>(ra[u][2], x4, x5);
                widen_fp8x4<OPT>(ra[u][3], x6, x7);
                const u32x4 w0 = {x0, x1, x2, x3}, w1 = {x4, x5, x6, x7};
                *reinterpret_cast<u32x4 *>(&lds[buf][row * LDP + kq * 16]) = w0;
                *reinterpret_cast<u32x4 *>(&lds[buf][row * LDP + kq * 16 + 8]) = w1;
            } else {
                *reinterpret_cast<u32x4 *>(&lds[buf][row * LDP + kq * 8]) = ra[u];
            }
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int q = tid + u * NT;
            const int col = q / BQ, kq = q % BQ;
            *reinterpret_cast<u32x4 *>(&lds[buf][(BM + col) * LDP + kq * 8]) = rb[u];
        }
    };
    auto bcol = [&](int nb) -> int {
        if (CPLX) {
            const int p = nb / NP, tb = nb % NP;
            return p * (BN / 2) + wn * (TN / 2) + tb * 32;
        }
        return wn * TN + nb * 32;
    };
    auto tcol = [&](int tb) -> int { return CPLX ? wn * (TN / 2) + tb * 32 : wn * TN + tb * 32; };

    f32x16 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.0f;

    const int nk = a.Np / BK;
    const int l32 = lane & 31, lh = lane >> 5;
    gload(0);
    lstore(0);
    __syncthreads();
    constexpr int NS = BK / 16;   // 16-wide K slices per chunk
    for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        const bool more = kc + 1 < nk;
        if (more) gload((kc + 1) * BK);
        // operands of slice kk+1 are read from LDS while slice kk multiplies;
        // the next chunk goes to the other buffer half-way through this one
        u32x4 av[2][MB], bv[2][NB];
        auto lread = [&](int kk, int set) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                av[set][mb] = *reinterpret_cast<const u32x4 *>(
                    &lds[buf][(wm * TM + mb * 32 + l32) * LDP + kk * 16 + lh * 8]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                bv[set][nb] = *reinterpret_cast<const u32x4 *>(
                    &lds[buf][(BM + bcol(nb) + l32) * LDP + kk * 16 + lh * 8]);
        };
        lread(0, 0);
#pragma unroll
        for (int kk = 0; kk < NS; ++kk) {
            const int set = kk & 1;
            if (kk + 1 < NS) lread(kk + 1, set ^ 1);
            if (kk == NS / 2 && more) lstore(buf ^ 1);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[mb][nb] = mfma32<OPT>(av[set][mb], bv[set][nb], acc[mb][nb]);
        }
        if (NS == 1 && more) lstore(buf ^ 1);
        __syncthreads();
    }

    // ---------------------------------------------------------------- epilogue
    // acc[mb][nb][4q + e]: row i = m0 + wm*TM + mb*32 + 8q + 4*lh + e, column l32 of block nb
    auto sub4 = [](const f32x16 &v, int q) -> f32x4 {
        return f32x4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
    };
    if constexpr (MODE == MODE_ENERGY) {
        double esum[NP];
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int r = r0 + tcol(tb) + l32;
            double s = 0.0;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    s += energy_terms4<CPLX>(a, m0 + wm * TM + mb * 32 + 8 * q + 4 * lh, r,
                                             sub4(acc[mb][tb], q),
                                             CPLX ? sub4(acc[mb][NP + tb], q) : sub4(acc[mb][tb], q));
            s += __shfl_xor(s, 32);
            esum[tb] = s;
        }
        double *red = reinterpret_cast<double *>(&lds[0][0]);
        if (lh == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) red[(wm * WN + wn) * (NP * 32) + tb * 32 + l32] = esum[tb];
        }
        __syncthreads();
        if (wm == 0 && lh == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) {
                double s = 0.0;
                for (int w = 0; w < WM; ++w) s += red[(w * WN + wn) * (NP * 32) + tb * 32 + l32];
                a.partial[(long long)mt * a.Rp + r0 + tcol(tb) + l32] = s;
            }
        }
    } else if constexpr ((CPLX ? 2 : 1) * TRAJ * (BM + 4) * 4 <= 2 * (BM + BN) * LDP * 2) {
        // The sums are staged through LDS as [trajectory][row] (the main loop
        // is done with it) so that the state update runs with consecutive
        // lanes on consecutive spins of one trajectory: every state load and
        // store of a wave is then a few fully used contiguous runs instead of
        // 16-byte pieces of 32 trajectories.
        constexpr int TP = BM + 4;                          // LDS pitch in floats
        float *st = reinterpret_cast<float *>(&lds[0][0]);
        float *sti = st + TRAJ * TP;                       // imaginary sums (complex)
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int tr = tcol(tb) + l32;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = wm * TM + mb * 32 + 8 * q + 4 * lh;
                    *reinterpret_cast<f32x4 *>(&st[tr * TP + row]) = sub4(acc[mb][tb], q);
                    if (CPLX) *reinterpret_cast<f32x4 *>(&sti[tr * TP + row]) = sub4(acc[mb][NP + tb], q);
                }
        }
        __syncthreads();
        constexpr int NT = 64 * WM * WN;
        constexpr int RG = BM / 4;                          // 4-row groups per trajectory
        static_assert((TRAJ * RG) % NT == 0, "epilogue split");
#pragma unroll 4
        for (int u = 0; u < TRAJ * RG / NT; ++u) {
            const int g = threadIdx.x + u * NT;
            const int tr = g / RG, row = (g % RG) * 4;
            const int r = r0 + tr;
            const bool rvalid = r < a.R;
            const f32x4 cr = *reinterpret_cast<const f32x4 *>(&st[tr * TP + row]);
            const f32x4 ci = CPLX ? *reinterpret_cast<const f32x4 *>(&sti[tr * TP + row]) : cr;
            const bool bad = step_epilogue4<MODE, CPLX, OPT>(a, m0 + row, r, rvalid, cr, ci);
            if (bad && rvalid) a.flags[r] = 1;
        }
    } else {
        // tiles too wide to stage: update straight from the accumulator layout
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int r = r0 + tcol(tb) + l32;
            const bool rvalid = r < a.R;
            bool bad = false;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    bad |= step_epilogue4<MODE, CPLX, OPT>(
                        a, m0 + wm * TM + mb * 32 + 8 * q + 4 * lh, r, rvalid, sub4(acc[mb][tb], q),
                        CPLX ? sub4(acc[mb][NP + tb], q) : sub4(acc[mb][tb], q));
            if (bad && rvalid) a.flags[r] = 1;
        }
    }
}

// Direct-to-LDS variant (BK = 64).  Both chunk tiles are copied from global
// memory into LDS by global_load_lds_dwordx4 (1 KiB per wave instruction,
// rows unpadded), so J stays FP8 in LDS (64-byte rows) and is widened after
// the LDS read: half the LDS bytes of a 16-bit J for its copy and its reads.
// The K order inside each 32-wide block is permuted identically for both
// operands so that one 16-byte LDS read of FP8 J feeds two MFMA K slices:
// lane half h, slice s of the pair, element e takes logical k = 16h + 8s + e.
// 16-byte slots are XOR-swizzled by row (slot ^ ((row >> 2) & 3) for 64-byte
// rows, slot ^ ((row >> 1) & 7) for 128-byte rows), so 16 consecutive rows
// read at one slot hit all 64 banks.  The state update stages the sums of one
// wave column at a time through LDS.
typedef __attribute__((address_space(1))) void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;

template <int ROWB>
__device__ inline int lp_swz(int row) { return ROWB == 64 ? (row >> 2) & 3 : (row >> 1) & 7; }

// 8 FP8 (E4M3) values in two dwords -> 8 16-bit operands (exact)
template <int OPT>
__device__ inline u32x4 widen_fp8x8(unsigned int w0, unsigned int w1) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
    u32x4 r;
    if constexpr (OPT == OP_BF16) {
        r[0] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, false));
        r[1] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, true));
        r[2] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, false));
        r[3] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, true));
    } else {
        r[0] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w0, 1.0f, false));
        r[1] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w0, 1.0f, true));
        r[2] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w1, 1.0f, false));
        r[3] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w1, 1.0f, true));
    }
    return r;
}

// s_waitcnt immediate: at most n vector-memory operations of this wave
// outstanding, all its LDS operations complete (expcnt at its maximum)
constexpr int lp_vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4); }

// PFX = 4096 * S3 + LDS floor (KiB) * 16 + PF.  PF > 0: the state operands
// of the first update groups (at most 16 wave loads per thread, a register
// budget) are loaded during the last K chunks, one per chunk after that
// chunk's copies; a wave then waits for its copies with vmcnt(loads issued
// since), since vector-memory loads complete in issue order, and meets the
// others at a plain barrier, so each load has the chunk's matrix work to
// land in.  S3 = 1: three LDS stages, the copies of chunk k + 2 issued at
// the start of chunk k (two chunks of matrix work to land in), waited for
// the same way.
template <int BM, int BN, int WM, int WN, bool CPLX, int MODE, int OPT, bool JFP8, int PFX>
__global__ void __launch_bounds__(64 * WM * WN)
dense_step_lp_dl(DenseStepArgs a) {
    constexpr int PF = PFX & 15;
    constexpr int LDSMIN = ((PFX >> 4) & 255) * 1024;
    constexpr int BK = 64;
    constexpr int NT = 64 * WM * WN, NW = WM * WN;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int MB = TM / 32, NB = TN / 32;
    constexpr int NP = CPLX ? NB / 2 : NB;
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    static_assert(!CPLX || (NB % 2 == 0), "complex waves pair re/im blocks");
    constexpr int RA = JFP8 ? BK : 2 * BK;            // bytes per A (J) row in LDS
    constexpr int RB = 2 * BK;                        // bytes per B (Psi) row
    constexpr int ABYTES = BM * RA, TILEB = ABYTES + BN * RB;
    constexpr int NIA = ABYTES / 1024, NI = TILEB / 1024;   // 1 KiB copies per chunk
    // three stages where they fit the 160 KiB of LDS (J in 16 bits doubles
    // the A tile), else two
    constexpr int NSTG = ((PFX >> 12) & 1) && 3 * TILEB <= 160 * 1024 ? 3 : 2;
    static_assert(NI % NW == 0 && ABYTES % 1024 == 0, "copy split");
    constexpr int NCW = NI / NW;
    // staged state update: one wave column (TRAJ / WN trajectories) per pass
    constexpr int TP = BM + 4;
    constexpr int TRP = TRAJ / WN;
    constexpr int STB = (CPLX ? 2 : 1) * TRP * TP * 4;
    constexpr int LDSB0 = NSTG * TILEB > STB ? NSTG * TILEB : STB;
    constexpr int LDSB = LDSB0 > LDSMIN ? LDSB0 : LDSMIN;
    __shared__ __attribute__((aligned(1024))) unsigned char lds[LDSB];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int n_mt = a.Np / BM, n_ct = a.Rp / TRAJ;
    int mt, ct;
    tile_map_lp(blockIdx.x, gridDim.x, n_mt, n_ct, mt, ct);
    const int m0 = mt * BM, r0 = ct * TRAJ;
    const long long Np = a.Np;
    const unsigned char *Jb = static_cast<const unsigned char *>(a.J);
    const unsigned char *Bb = static_cast<const unsigned char *>(a.B);

    // this lane's source of each of its copies (fixed across chunks, + k0 bytes)
    const unsigned char *src[NCW];
    int kscale[NCW];                                   // bytes per k of that source
#pragma unroll
    for (int u = 0; u < NCW; ++u) {
        const int j = wave + u * NW;                   // copy index
        if (j < NIA) {
            constexpr int LPR = RA / 16;               // lanes per row
            const int row = j * (64 / LPR) + lane / LPR;
            const int ls = (lane % LPR) ^ lp_swz<RA>(row);
            src[u] = Jb + ((m0 + row) * Np) * (JFP8 ? 1 : 2) + ls * 16;
            kscale[u] = JFP8 ? 1 : 2;
        } else {
            const int row = (j - NIA) * 8 + lane / 8;  // B row = GEMM column
            const int ls = (lane % 8) ^ lp_swz<RB>(row);
            const int plane = CPLX ? row / (BN / 2) : 0;
            const int tr = CPLX ? row % (BN / 2) : row;
            src[u] = Bb + (plane * a.plane_stride + (long long)(r0 + tr) * Np) * 2 + ls * 16;
            kscale[u] = 2;
        }
    }
    auto copy_chunk = [&](int k0, int buf) {
#pragma unroll
        for (int u = 0; u < NCW; ++u) {
            const int j = wave + u * NW;
            __builtin_amdgcn_global_load_lds((gvoid_t *)(src[u] + (long long)k0 * kscale[u]),
                                             (lvoid_t *)&lds[buf * TILEB + j * 1024], 16, 0, 0);
        }
    };
    auto bcol = [&](int nb) -> int {
        if (CPLX) {
            const int p = nb / NP, tb = nb % NP;
            return p * (BN / 2) + wn * (TN / 2) + tb * 32;
        }
        return wn * TN + nb * 32;
    };
    auto tcol = [&](int tb) -> int { return CPLX ? wn * (TN / 2) + tb * 32 : wn * TN + tb * 32; };

    f32x16 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.0f;

    const int nk = a.Np / BK;
    const int l32 = lane & 31, lh = lane >> 5;
    // update groups: pass p (wave column), group u of the thread's groups
    // in that pass; operands loaded ahead for the first NUP groups in
    // (pass, group) order
    constexpr int RG = BM / 4;
    static_assert((TRP * RG) % NT == 0, "epilogue split");
    constexpr int NUPP = TRP * RG / NT;               // groups per thread and pass
    constexpr int NF = PF > 0 ? epi_fields<MODE, CPLX>() : 0;
    constexpr int NUP = NF == 0 ? 0 : (16 / NF < WN * NUPP ? 16 / NF : WN * NUPP);
    constexpr int NPF = NUP * NF;
    f32x4 pf[NPF > 0 ? NPF : 1];
    auto grp_idx = [&](int v) -> long long {          // v = pass * NUPP + u
        const int p = v / NUPP, g = tid + (v % NUPP) * NT;
        return (long long)(r0 + p * TRP + g / RG) * Np + m0 + (g % RG) * 4;
    };
    copy_chunk(0, 0);
    if constexpr (NSTG == 3) {
        // chunk 0 has landed; chunk 1 may still be in flight
        if (nk > 1) {
            copy_chunk(BK, 1);
            __builtin_amdgcn_s_waitcnt(lp_vmcnt_imm(NCW));
        } else {
            __builtin_amdgcn_s_waitcnt(lp_vmcnt_imm(0));
        }
        __asm__ __volatile__("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        __asm__ __volatile__("" ::: "memory");
    } else {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    auto chunk = [&](int kc, auto pslot) {
        constexpr int PS = decltype(pslot)::value;
        const int buf = NSTG == 3 ? kc % 3 : kc & 1;
        const bool ahead = kc + NSTG - 1 < nk;     // copies of chunk kc + NSTG - 1 issued here
        if (ahead) copy_chunk((kc + NSTG - 1) * BK, NSTG == 3 ? (kc + 2) % 3 : buf ^ 1);
        constexpr int NL = PS < 0 ? 0 : 1;
        if constexpr (NL > 0) {
            __builtin_amdgcn_sched_barrier(0);
            pf[PS] = *reinterpret_cast<const f32x4 *>(epi_field_ptr<CPLX>(a, PS % NF) + grp_idx(PS / NF));
            __builtin_amdgcn_sched_barrier(0);
        }
        const unsigned char *At = &lds[buf * TILEB];
        const unsigned char *Bt = At + ABYTES;
        // operands of K-slice pair m (two 16-wide slices): A [MB][2], B [NB][2]
        u32x4 av[2][MB][2], bv[2][NB][2];
        auto lread = [&](int m, int set) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int row = wm * TM + mb * 32 + l32;
                if constexpr (JFP8) {
                    const int slot = (2 * m + lh) ^ lp_swz<RA>(row);
                    const u32x4 w = *reinterpret_cast<const u32x4 *>(At + row * RA + slot * 16);
                    av[set][mb][0] = widen_fp8x8<OPT>(w[0], w[1]);
                    av[set][mb][1] = widen_fp8x8<OPT>(w[2], w[3]);
                } else {
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const int slot = (4 * m + 2 * lh + s) ^ lp_swz<RA>(row);
                        av[set][mb][s] = *reinterpret_cast<const u32x4 *>(At + row * RA + slot * 16);
                    }
                }
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int row = bcol(nb) + l32;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int slot = (4 * m + 2 * lh + s) ^ lp_swz<RB>(row);
                    bv[set][nb][s] = *reinterpret_cast<const u32x4 *>(Bt + row * RB + slot * 16);
                }
            }
        };
        lread(0, 0);
#pragma unroll
        for (int m = 0; m < BK / 32; ++m) {
            const int set = m & 1;
            if (m + 1 < BK / 32) lread(m + 1, set ^ 1);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[mb][nb] = mfma32<OPT>(av[set][mb][s], bv[set][nb][s], acc[mb][nb]);
        }
        // this wave's copies of the next chunk have landed (an operand load
        // and, with three stages, the copies of the chunk after it, issued
        // later, may still be in flight); then a plain workgroup barrier with
        // compiler-only fences (a release fence would wait for those too)
        if (NSTG == 3 && ahead)
            __builtin_amdgcn_s_waitcnt(lp_vmcnt_imm(NCW + NL));
        else
            __builtin_amdgcn_s_waitcnt(lp_vmcnt_imm(NL));
        if constexpr (PF > 0 || NSTG == 3) {
            __asm__ __volatile__("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            __asm__ __volatile__("" ::: "memory");
        } else {
            __syncthreads();
        }
    };
    int kc = 0;
    for (; kc < nk - NPF; ++kc) chunk(kc, std::integral_constant<int, -1>{});
    if constexpr (NPF > 0)   // the launcher guarantees nk >= NPF
        seq_apply([&](auto q) { chunk(kc + decltype(q)::value, q); }, std::make_integer_sequence<int, NPF>{});

    // ---------------------------------------------------------------- epilogue
    // acc[mb][nb][4q + e]: row i = m0 + wm*TM + mb*32 + 8q + 4*lh + e, column l32 of block nb
    auto sub4 = [](const f32x16 &v, int q) -> f32x4 {
        return f32x4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
    };
    if constexpr (MODE == MODE_ENERGY) {
        double esum[NP];
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int r = r0 + tcol(tb) + l32;
            double s = 0.0;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    s += energy_terms4<CPLX>(a, m0 + wm * TM + mb * 32 + 8 * q + 4 * lh, r,
                                             sub4(acc[mb][tb], q),
                                             CPLX ? sub4(acc[mb][NP + tb], q) : sub4(acc[mb][tb], q));
            s += __shfl_xor(s, 32);
            esum[tb] = s;
        }
        double *red = reinterpret_cast<double *>(&lds[0]);
        if (lh == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) red[(wm * WN + wn) * (NP * 32) + tb * 32 + l32] = esum[tb];
        }
        __syncthreads();
        if (wm == 0 && lh == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) {
                double s = 0.0;
                for (int w = 0; w < WM; ++w) s += red[(w * WN + wn) * (NP * 32) + tb * 32 + l32];
                a.partial[(long long)mt * a.Rp + r0 + tcol(tb) + l32] = s;
            }
        }
    } else {
        // pass p: the waves of column p stage their sums as [trajectory][row]
        // (TRP trajectories), then every thread updates 4-row groups of them
        float *st = reinterpret_cast<float *>(&lds[0]);
        float *sti = st + TRP * TP;
#pragma unroll
        for (int p = 0; p < WN; ++p) {
            if (wn == p) {
#pragma unroll
                for (int tb = 0; tb < NP; ++tb) {
                    const int tr = tcol(tb) - p * TRP + l32;
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int row = wm * TM + mb * 32 + 8 * q + 4 * lh;
                            *reinterpret_cast<f32x4 *>(&st[tr * TP + row]) = sub4(acc[mb][tb], q);
                            if (CPLX)
                                *reinterpret_cast<f32x4 *>(&sti[tr * TP + row]) = sub4(acc[mb][NP + tb], q);
                        }
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < NUPP; ++u) {
                const int g = tid + u * NT;
                const int tr = g / RG, row = (g % RG) * 4;
                const int r = r0 + p * TRP + tr;
                const bool rvalid = r < a.R;
                const f32x4 cr = *reinterpret_cast<const f32x4 *>(&st[tr * TP + row]);
                const f32x4 ci = CPLX ? *reinterpret_cast<const f32x4 *>(&sti[tr * TP + row]) : cr;
                const int v = p * NUPP + u;
                bool bad;
                if (v < NUP) {
                    EpiIn in;
                    epi_fill<MODE, CPLX>(a, m0 + row, &pf[(v < NUP ? v : 0) * NF], in);
                    bad = epi_apply<MODE, CPLX, OPT>(a, m0 + row, r, rvalid, in, cr, ci);
                } else {
                    bad = step_epilogue4<MODE, CPLX, OPT>(a, m0 + row, r, rvalid, cr, ci);
                }
                if (bad && rvalid) a.flags[r] = 1;
            }
            if (p + 1 < WN) __syncthreads();
        }
    }
}

template <int BM, int BN, int WM, int WN, bool CPLX, int OPT, bool JFP8, int PFX>
hipError_t launch_lp_dl_modes(int mode, const DenseStepArgs &a, hipStream_t st) {
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    if (a.Np % BM || a.Np % 64 || a.Rp % TRAJ) return hipErrorInvalidValue;
    // the operand-load tail needs at most 16 chunks
    if ((PFX & 15) && a.Np / 64 < 16) return hipErrorInvalidValue;
    const dim3 grid((a.Np / BM) * (a.Rp / TRAJ)), block(64 * WM * WN);
#define GD_LAUNCH(M) dense_step_lp_dl<BM, BN, WM, WN, CPLX, M, OPT, JFP8, PFX><<<grid, block, 0, st>>>(a)
    switch (mode) {
    case MODE_EULER: GD_LAUNCH(MODE_EULER); break;
    case MODE_RK1: GD_LAUNCH(MODE_RK1); break;
    case MODE_RK2: GD_LAUNCH(MODE_RK2); break;
    case MODE_RK3: GD_LAUNCH(MODE_RK3); break;
    case MODE_RK4: GD_LAUNCH(MODE_RK4); break;
    case MODE_ENERGY: GD_LAUNCH(MODE_ENERGY); break;
    default: return hipErrorInvalidValue;
    }
#undef GD_LAUNCH
    return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN, bool CPLX, int OPT, bool JFP8>
hipError_t launch_lp_modes(int mode, const DenseStepArgs &a, hipStream_t st) {
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    if (a.Np % BM || a.Np % BK || a.Rp % TRAJ) return hipErrorInvalidValue;
    const dim3 grid((a.Np / BM) * (a.Rp / TRAJ)), block(64 * WM * WN);
#define GD_LAUNCH(M) dense_step_lp<BM, BN, BK, WM, WN, CPLX, M, OPT, JFP8><<<grid, block, 0, st>>>(a)
    switch (mode) {
    case MODE_EULER: GD_LAUNCH(MODE_EULER); break;
    case MODE_RK1: GD_LAUNCH(MODE_RK1); break;
    case MODE_RK2: GD_LAUNCH(MODE_RK2); break;
    case MODE_RK3: GD_LAUNCH(MODE_RK3); break;
    case MODE_RK4: GD_LAUNCH(MODE_RK4); break;
    case MODE_ENERGY: GD_LAUNCH(MODE_ENERGY); break;
    default: return hipErrorInvalidValue;
    }
#undef GD_LAUNCH
    return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN, int DL>
hipError_t launch_lp(bool cx, int op, bool jfp8, int mode, const DenseStepArgs &a, hipStream_t st) {
#define GD_SEL(C, O, F)                                                                              \
    if (cx == C && op == O && jfp8 == F) {                                                           \
        if constexpr (DL > 0) return launch_lp_dl_modes<BM, BN, WM, WN, C, O, F, DL - 1>(mode, a, st);     \
        else return launch_lp_modes<BM, BN, BK, WM, WN, C, O, F>(mode, a, st);                       \
    }
    GD_SEL(false, OP_BF16, true) GD_SEL(false, OP_BF16, false)
    GD_SEL(false, OP_F16, true) GD_SEL(false, OP_F16, false)
    GD_SEL(true, OP_BF16, true) GD_SEL(true, OP_BF16, false)
    GD_SEL(true, OP_F16, true) GD_SEL(true, OP_F16, false)
#undef GD_SEL
    return hipErrorInvalidValue;
}

// Variants {BM, BN (GEMM columns), BK, WM, WN, DL (0: register-staged; else
// direct-to-LDS copies with J kept FP8 in LDS, DL - 1 = 4096 for three LDS
// stages + LDS floor in KiB * 16 + state-operand loads per tail chunk)}.  Ids 0-6 are instantiated in
// gd_dense_lp.hip, the larger workgroup tiles 7-13 in gd_dense_lp_big.hip
// (two translation units that compile in parallel).  256 x 256 tiles (eight
// waves of 128 x 64) halve the LDS bytes written per flop against 128 x 128
// and put one workgroup on each CU at N = 4096.
#define GD_LP_VARIANTS(X)           \
    X(0, 128, 128, 64, 2, 2, 0)     \
    X(1, 64, 128, 64, 2, 2, 0)      \
    X(2, 128, 256, 64, 2, 2, 0)     \
    X(3, 128, 128, 32, 2, 2, 0)     \
    X(4, 128, 128, 64, 2, 2, 1)     \
    X(5, 128, 128, 64, 2, 2, 1153)  \
    X(6, 128, 128, 64, 2, 2, 1154)
#define GD_LP_BIG_VARIANTS(X)       \
    X(7, 256, 256, 64, 2, 4, 1)     \
    X(8, 256, 128, 64, 2, 2, 1)     \
    X(9, 128, 256, 64, 2, 4, 1)     \
    X(10, 256, 128, 64, 4, 2, 1)    \
    X(11, 256, 256, 64, 2, 4, 4097) \
    X(12, 128, 256, 64, 2, 4, 4097) \
    X(13, 256, 128, 64, 2, 2, 4097)

}  // namespace

// launcher of the larger tiles (gd_dense_lp_big.hip)
hipError_t launch_dense_step_lp_big(const DenseConfig &cfg, bool complex_mode, int mode, int op,
                                    bool j_fp8, const DenseStepArgs &a, hipStream_t st);

}  // namespace gd
