// Dense coupling step of the gain-dissipative method on gfx950.
//
// One launch evaluates, for every spin i and trajectory r of a tile, the
// coupling sum C_ir = (1/s) sum_j J_ij Psi_jr of Eq. (main) as a GEMM on the
// matrix cores (v_mfma_f32_16x16x4_f32, FP32 in and out), and then applies the
// pointwise part of Eq. (main) and Eq. (gamma) in the epilogue, so that the
// coupling result never goes to HBM (it stays in registers, or passes
// through LDS to put consecutive lanes on consecutive spins):
//   f   = Psi (gamma - gamma_c - |Psi|^2) + C + h_1
//   phi = eps_i (rho_th - |Psi|^2)
// followed by an Euler update or one stage of the classical RK4 scheme on
// the joint state (Psi, gamma).  The energy mode reuses the same main loop
// with the discretised spins as operand and reduces the terms of Eq. (h).
//
// Layout: J is [Np][Np] row-major (zero diagonal, zero padding); every
// per-trajectory quantity is a plane [Rp][Np] (trajectory-major, spin index
// contiguous).  The product is C[i][r] = sum_k J[i][k] Psi[r][k]: both
// operands are K-contiguous, so global->LDS copies are plain 16-byte vector
// loads.  The register-staged variants hold both tiles in LDS as [row][k]
// with an 8-float pad per row; the direct-to-LDS variants (further below)
// copy chunks straight into unpadded, XOR-swizzled rows.  Both read 16 bytes
// per lane without bank conflicts.
//
// Tiling: a workgroup owns BM rows x BN GEMM columns, WM x WN waves; a wave
// owns (BM/WM) x (BN/WN) as 16x16 MFMA blocks.  Complex amplitudes use BN/2
// trajectories: the real parts sit in LDS columns [0, BN/2), the imaginary
// parts in [BN/2, BN), and every wave takes matching real/imaginary blocks,
// so the real and imaginary accumulators of one (i, r) live in the same lane
// and register and the epilogue needs no data exchange.
//
// K order inside a 16-wide slice is permuted: lane group q = lane/16 feeds
// k = 4q + t to MFMA number t (A and B use the same permutation), so each
// lane fetches its 4 operands of a slice with one ds_read_b128.
//
// Pipelining: chunk loads are issued LA chunks ahead (register sets), the
// next chunk is written to the other LDS buffer half-way through the current
// one, LDS operand reads run one slice ahead of the MFMAs, and (when they fit)
// the epilogue's state operands are loaded two chunks before the end.  KS > 1
// splits K between KS groups of waves of the same tile (more waves per CU).
#include "gd_epilogue.h"

#include <type_traits>
#include <utility>

namespace gd {

namespace {


// Workgroup -> (row tile, column tile).  Consecutive workgroup ids land on
// different XCDs (round-robin dispatch), so the linear id is first regrouped
// into one contiguous range per XCD, then mapped in column-major groups of
// `gm` row tiles: each XCD works on a compact block of J rows x trajectories
// and keeps it resident in its own L2.
__device__ inline void tile_map(int b, int nblk, int n_mt, int n_ct, int &mt, int &ct) {
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

template <int BM, int BN, int BK, int WM, int WN, bool CPLX, int MODE, int KS, int LA>
__global__ void __launch_bounds__(64 * WM * WN * KS)
dense_step_f32(DenseStepArgs a) {
    // LDS row pitch in floats: an 8-float pad makes the 16-byte operand reads
    // bank-conflict free on gfx950 (a 4-float pad still conflicts)
    constexpr int LDP = BK + 8;
    constexpr int NTG = 64 * WM * WN;   // threads of one K group
    constexpr int TM = BM / WM;     // rows per wave
    constexpr int TN = BN / WN;     // GEMM columns per wave
    constexpr int MB = TM / 16;     // 16-row MFMA blocks per wave
    constexpr int NB = TN / 16;     // 16-column MFMA blocks per wave
    constexpr int NP = CPLX ? NB / 2 : NB;   // trajectory blocks per wave
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    static_assert(!CPLX || (NB % 2 == 0), "complex waves pair re/im blocks");
    constexpr int KQ = BK / 4;                 // float4 per row chunk
    constexpr int AL = BM * KQ / NTG;          // A float4 loads per thread
    constexpr int BL = BN * KQ / NTG;          // B float4 loads per thread
    static_assert(BM * KQ % NTG == 0 && BN * KQ % NTG == 0, "load split");
    constexpr int TILE = (BM + BN) * LDP;
    static_assert(LA == 1 || LA == 2, "load lookahead of one or two chunks");
    // KS > 1: KS groups of WM x WN waves take K chunks g, g + KS, ... of the
    // same output tile (more waves per CU to hide latency); group 0 adds the
    // other groups' partial sums through LDS and runs the epilogue.
    static_assert(KS == 1 || (KS - 1) * NTG * MB * NB * 4 <= KS * 2 * TILE, "reduction fits LDS");

    __shared__ __attribute__((aligned(16))) float lds[KS][2][TILE];

    const int tid = threadIdx.x;
    const int grp = tid / NTG;
    const int tg = tid % NTG;
    const int lane = tid & 63;
    const int wave = tg >> 6;
    const int wm = wave % WM;
    const int wn = wave / WM;
    const int n_mt = a.Np / BM;
    const int n_ct = a.Rp / TRAJ;
    int mt, ct;
    tile_map(blockIdx.x, gridDim.x, n_mt, n_ct, mt, ct);
    const int m0 = mt * BM;
    const int r0 = ct * TRAJ;
    const long long Np = a.Np;

    const float *J = static_cast<const float *>(a.J);
    const float *Bop = static_cast<const float *>(a.B);
    float(*gl)[TILE] = lds[grp];

    // LA > 1: chunk loads are issued LA chunks ahead into LA register sets
    f32x4 ra[LA][AL], rb[LA][BL];
    auto gload = [&](int k0, int set) {
#pragma unroll
        for (int u = 0; u < AL; ++u) {
            const int q = tg + u * NTG;
            const int row = q / KQ, kq = q % KQ;
            ra[set][u] = *reinterpret_cast<const f32x4 *>(J + (m0 + row) * Np + k0 + kq * 4);
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int q = tg + u * NTG;
            const int col = q / KQ, kq = q % KQ;
            const int plane = CPLX ? col / (BN / 2) : 0;
            const int tr = CPLX ? col % (BN / 2) : col;
            rb[set][u] = *reinterpret_cast<const f32x4 *>(Bop + plane * a.plane_stride +
                                                     (r0 + tr) * Np + k0 + kq * 4);
        }
    };
    auto lstore = [&](int buf, int set) {
#pragma unroll
        for (int u = 0; u < AL; ++u) {
            const int q = tg + u * NTG;
            const int row = q / KQ, kq = q % KQ;
            *reinterpret_cast<f32x4 *>(&gl[buf][row * LDP + kq * 4]) = ra[set][u];
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int q = tg + u * NTG;
            const int col = q / KQ, kq = q % KQ;
            *reinterpret_cast<f32x4 *>(&gl[buf][(BM + col) * LDP + kq * 4]) = rb[set][u];
        }
    };
    // LDS column (within the B tile) of column block nb of this wave
    auto bcol = [&](int nb) -> int {
        if (CPLX) {
            const int p = nb / NP, tb = nb % NP;
            return p * (BN / 2) + wn * (TN / 2) + tb * 16;
        }
        return wn * TN + nb * 16;
    };
    // trajectory offset (within the tile) of trajectory block tb of this wave
    auto tcol = [&](int tb) -> int { return CPLX ? wn * (TN / 2) + tb * 16 : wn * TN + tb * 16; };

    f32x4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    // The epilogue's state operands are loaded into registers two K chunks
    // before the end of the main loop (when they fit the register budget), so
    // their HBM latency overlaps the last matrix iterations.
    constexpr bool PREF = KS == 1 && LA == 1 && (MODE != MODE_ENERGY) && (MB * NP * (CPLX ? 44 : 32) <= 96);
    EpiIn pre[PREF ? MB : 1][PREF ? NP : 1];
    auto prefetch = [&]() {
        if constexpr (PREF) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    epi_load<MODE, CPLX>(a, m0 + wm * TM + mb * 16 + 4 * (lane >> 4),
                                         r0 + tcol(tb) + (lane & 15), pre[mb][tb]);
        }
    };

    const int nk = a.Np / BK;
    const int nit = (nk + KS - 1) / KS;        // iterations of every group
    const int itpf = nit >= 2 ? nit - 2 : 0;
    const int l16 = lane & 15;
    const int lq = lane >> 4;
    constexpr int NS = BK / 16;   // 16-wide K slices per chunk
    if (grp < nk) gload(grp * BK, 0);
    if (grp < nk) lstore(0, 0);
#pragma unroll
    for (int j = 1; j < LA; ++j)
        if (grp + j * KS < nk) gload((grp + j * KS) * BK, j);
    __syncthreads();
    // one iteration; SL = it % LA is a compile-time constant so the register
    // sets of the chunk loads are indexed statically
    auto iteration = [&](int it, auto slc) {
        constexpr int SL = decltype(slc)::value;
        const int buf = it & 1;
        const int kc = it * KS + grp;            // this group's chunk
        const bool have = kc < nk;
        const bool more = kc + KS < nk;
        if (kc + LA * KS < nk) gload((kc + LA * KS) * BK, SL);
        if (grp == 0 && it == itpf) prefetch();   // after the chunk load, so that load is not held up
        if (have) {
            // operands of slice kk+1 are read from LDS while slice kk multiplies
            f32x4 av[2][MB], bv[2][NB];
            auto lread = [&](int kk, int set) {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    av[set][mb] = *reinterpret_cast<const f32x4 *>(
                        &gl[buf][(wm * TM + mb * 16 + l16) * LDP + kk * 16 + lq * 4]);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    bv[set][nb] = *reinterpret_cast<const f32x4 *>(
                        &gl[buf][(BM + bcol(nb) + l16) * LDP + kk * 16 + lq * 4]);
            };
            lread(0, 0);
#pragma unroll
            for (int kk = 0; kk < NS; ++kk) {
                const int set = kk & 1;
                if (kk + 1 < NS) lread(kk + 1, set ^ 1);
                // the next chunk goes to the other buffer half-way through this one
                // (that buffer was last read before the previous barrier)
                if (kk == NS / 2 && more) lstore(buf ^ 1, (SL + 1) % LA);
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                av[set][mb][t], bv[set][nb][t], acc[mb][nb], 0, 0, 0);
            }
            if (NS == 1 && more) lstore(buf ^ 1, (SL + 1) % LA);
        }
        __syncthreads();
    };
    for (int it = 0; it < nit; it += LA) {
        iteration(it, std::integral_constant<int, 0>{});
        if constexpr (LA > 1)
            if (it + 1 < nit) iteration(it + 1, std::integral_constant<int, 1>{});
    }
    if constexpr (KS > 1) {
        // partial sums of groups 1..KS-1 -> group 0 (all LDS reads of the loop are done)
        float *xs = &lds[0][0][0];
        if (grp > 0) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    *reinterpret_cast<f32x4 *>(
                        &xs[((((grp - 1) * MB + mb) * NB + nb) * NTG + tg) * 4]) = acc[mb][nb];
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int g = 1; g < KS; ++g)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[mb][nb] += *reinterpret_cast<const f32x4 *>(
                            &xs[((((g - 1) * MB + mb) * NB + nb) * NTG + tg) * 4]);
        }
        __syncthreads();
    }

    // ---------------------------------------------------------------- epilogue
    // acc[mb][nb][e] holds row i = m0 + wm*TM + mb*16 + 4*lq + e, column l16 of
    // block nb; only group 0 holds the full sums.
    if constexpr (MODE == MODE_ENERGY) {
        double esum[NP];
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int r = r0 + tcol(tb) + l16;
            double s = 0.0;
            if (grp == 0) {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    s += energy_terms4<CPLX>(a, m0 + wm * TM + mb * 16 + 4 * lq, r, acc[mb][tb],
                                             CPLX ? acc[mb][NP + tb] : acc[mb][tb]);
            }
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            esum[tb] = s;
        }
        // combine the row waves through LDS (the main loop is done with it)
        double *red = reinterpret_cast<double *>(&lds[0][0][0]);
        if (grp == 0 && lq == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) red[(wm * WN + wn) * (NP * 16) + tb * 16 + l16] = esum[tb];
        }
        __syncthreads();
        if (grp == 0 && wm == 0 && lq == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) {
                double s = 0.0;
                for (int w = 0; w < WM; ++w) s += red[(w * WN + wn) * (NP * 16) + tb * 16 + l16];
                a.partial[(long long)mt * a.Rp + r0 + tcol(tb) + l16] = s;
            }
        }
    } else if constexpr (!PREF && (CPLX ? 2 : 1) * TRAJ * (BM + 4) <= KS * 2 * TILE) {
        // The sums are staged through LDS as [trajectory][row] (the main loop
        // is done with it) so that the state update runs with consecutive
        // lanes on consecutive spins of one trajectory (contiguous runs per
        // wave instead of 64-byte pieces of 16 trajectories); every thread of
        // the workgroup, all K groups included, takes part in the update.
        constexpr int TP = BM + 4;                          // LDS pitch in floats
        float *st = &lds[0][0][0];
        float *sti = st + TRAJ * TP;                       // imaginary sums (complex)
        if (grp == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) {
                const int tr = tcol(tb) + l16;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    const int row = wm * TM + mb * 16 + 4 * lq;
                    *reinterpret_cast<f32x4 *>(&st[tr * TP + row]) = acc[mb][tb];
                    if (CPLX) *reinterpret_cast<f32x4 *>(&sti[tr * TP + row]) = acc[mb][NP + tb];
                }
            }
        }
        __syncthreads();
        constexpr int NT = NTG * KS;
        constexpr int RG = BM / 4;                          // 4-row groups per trajectory
        static_assert((TRAJ * RG) % NT == 0, "epilogue split");
#pragma unroll 4
        for (int u = 0; u < TRAJ * RG / NT; ++u) {
            const int g = tid + u * NT;
            const int tr = g / RG, row = (g % RG) * 4;
            const int r = r0 + tr;
            const bool rvalid = r < a.R;
            const f32x4 cr = *reinterpret_cast<const f32x4 *>(&st[tr * TP + row]);
            const f32x4 ci = CPLX ? *reinterpret_cast<const f32x4 *>(&sti[tr * TP + row]) : cr;
            const bool bad = step_epilogue4<MODE, CPLX, OP_F32>(a, m0 + row, r, rvalid, cr, ci);
            if (bad && rvalid) a.flags[r] = 1;
        }
    } else {
        if (grp != 0) return;
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int r = r0 + tcol(tb) + l16;
            const bool rvalid = r < a.R;
            bool bad = false;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int i0 = m0 + wm * TM + mb * 16 + 4 * lq;
                const f32x4 ci = CPLX ? acc[mb][NP + tb] : acc[mb][tb];
                if constexpr (PREF)
                    bad |= epi_apply<MODE, CPLX, OP_F32>(a, i0, r, rvalid, pre[mb][tb], acc[mb][tb], ci);
                else
                    bad |= step_epilogue4<MODE, CPLX, OP_F32>(a, i0, r, rvalid, acc[mb][tb], ci);
            }
            if (bad && rvalid) a.flags[r] = 1;
        }
    }
}

// Direct-to-LDS variant (BK = 32 or 64): chunk tiles are copied from global
// memory straight into LDS by global_load_lds_dwordx4 (each wave instruction
// fills 1 KiB: 8 rows of 32 floats or 4 rows of 64), with no register staging
// and no LDS store instructions; a wave only waits for its copies at the end
// of the chunk, before the barrier.  Rows are unpadded; the 16-byte slot s of
// row w is stored at slot s ^ ((w >> 1) & 7) (BK = 32) or s ^ (w & 15)
// (BK = 64), which spreads the 16-byte operand reads of 16 consecutive rows
// over all 64 banks.  The state update always uses the LDS-staged sums.
typedef __attribute__((address_space(1))) void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;

template <int BK>
__device__ inline int dl_swz(int row) { return BK == 32 ? (row >> 1) & 7 : row & 15; }

// s_waitcnt immediate: wait until at most n vector-memory operations of this
// wave are outstanding and all its LDS operations have completed (expcnt left
// at its maximum)
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4); }

// PF > 0: the state operands of the update are loaded into registers during
// the last K chunks, PF wave loads per chunk, each issued after that chunk's
// copies.  A wave waits for a chunk's copies with vmcnt(PF): vector-memory
// loads complete in issue order, so the operand loads issued since stay in
// flight and each one has a chunk's matrix work to land in; spreading them
// keeps the HBM burst of all workgroups (which run in step) small.
template <int BM, int BN, int BK, int WM, int WN, bool CPLX, int MODE, int PF>
__global__ void __launch_bounds__(64 * WM * WN)
dense_step_f32_dl(DenseStepArgs a) {
    static_assert(BK == 32 || BK == 64, "chunk width");
    constexpr int SPR = BK / 4;                        // 16-byte slots per row
    constexpr int NT = 64 * WM * WN;
    constexpr int NW = WM * WN;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int MB = TM / 16, NB = TN / 16;
    constexpr int NP = CPLX ? NB / 2 : NB;
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    static_assert(!CPLX || (NB % 2 == 0), "complex waves pair re/im blocks");
    constexpr int TILE = (BM + BN) * BK;               // floats per buffer
    constexpr int NI = TILE / 256;                     // 1 KiB copies per chunk
    static_assert(NI % NW == 0 && BM % 8 == 0, "copy split");
    __shared__ __attribute__((aligned(1024))) float lds[2][TILE];
    // state-update groups (trajectory, 4 rows) of each thread
    constexpr int RG = BM / 4;
    static_assert((TRAJ * RG) % NT == 0, "epilogue split");
    constexpr int NU = TRAJ * RG / NT;
    constexpr int NF = PF > 0 ? epi_fields<MODE, CPLX>() : 0;
    constexpr int NPF = NU * NF;                       // operand loads per wave
    constexpr int TAIL = PF > 0 ? (NPF + PF - 1) / PF : 0;   // chunks that carry them

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int n_mt = a.Np / BM, n_ct = a.Rp / TRAJ;
    int mt, ct;
    tile_map(blockIdx.x, gridDim.x, n_mt, n_ct, mt, ct);
    const int m0 = mt * BM, r0 = ct * TRAJ;
    const long long Np = a.Np;
    const float *J = static_cast<const float *>(a.J);
    const float *Bop = static_cast<const float *>(a.B);

    // this lane's source row offsets for its copies (fixed across chunks)
    const float *src[NI / NW];
#pragma unroll
    for (int u = 0; u < NI / NW; ++u) {
        const int j = wave + u * NW;                   // copy index: 64 / SPR rows
        const int row = j * (64 / SPR) + lane / SPR;
        const int ls = (lane % SPR) ^ dl_swz<BK>(row);  // logical slot stored in this lane's slot
        if (row < BM) {
            src[u] = J + (m0 + row) * Np + ls * 4;
        } else {
            const int col = row - BM;
            const int plane = CPLX ? col / (BN / 2) : 0;
            const int tr = CPLX ? col % (BN / 2) : col;
            src[u] = Bop + plane * a.plane_stride + (r0 + tr) * Np + ls * 4;
        }
    }
    auto copy_chunk = [&](int k0, int buf) {
#pragma unroll
        for (int u = 0; u < NI / NW; ++u) {
            const int j = wave + u * NW;
            __builtin_amdgcn_global_load_lds((gvoid_t *)(src[u] + k0), (lvoid_t *)&lds[buf][j * 256], 16, 0, 0);
        }
    };
    auto bcol = [&](int nb) -> int {
        if (CPLX) {
            const int p = nb / NP, tb = nb % NP;
            return p * (BN / 2) + wn * (TN / 2) + tb * 16;
        }
        return wn * TN + nb * 16;
    };
    auto tcol = [&](int tb) -> int { return CPLX ? wn * (TN / 2) + tb * 16 : wn * TN + tb * 16; };
    // element offset of state-update group u of this thread
    auto grp_idx = [&](int u) -> long long {
        const int g = tid + u * NT;
        return (long long)(r0 + g / RG) * Np + m0 + (g % RG) * 4;
    };

    f32x4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 pf[NPF > 0 ? NPF : 1];

    const int nk = a.Np / BK;
    const int l16 = lane & 15, lq = lane >> 4;
    // one K chunk; P >= 0 issues operand loads P*PF .. P*PF+PF-1
    auto chunk = [&](int kc, auto pslot) {
        constexpr int P = decltype(pslot)::value;
        const int buf = kc & 1;
        // the buffer refilled here was last read before the previous barrier
        if (kc + 1 < nk) copy_chunk((kc + 1) * BK, buf ^ 1);
        constexpr int NL = P < 0 ? 0 : (NPF - P * PF < PF ? NPF - P * PF : PF);
        if constexpr (NL > 0) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const int q = P * PF + l;              // constant after unrolling
                pf[q] = *reinterpret_cast<const f32x4 *>(epi_field_ptr<CPLX>(a, q % NF) + grp_idx(q / NF));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        f32x4 av[2][MB], bv[2][NB];
        auto lread = [&](int kk, int set) {
            const int s = kk * 4 + lq;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int row = wm * TM + mb * 16 + l16;
                av[set][mb] = *reinterpret_cast<const f32x4 *>(&lds[buf][row * BK + (s ^ dl_swz<BK>(row)) * 4]);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int row = BM + bcol(nb) + l16;
                bv[set][nb] = *reinterpret_cast<const f32x4 *>(&lds[buf][row * BK + (s ^ dl_swz<BK>(row)) * 4]);
            }
        };
        lread(0, 0);
#pragma unroll
        for (int kk = 0; kk < BK / 16; ++kk) {
            const int set = kk & 1;
            if (kk + 1 < BK / 16) lread(kk + 1, set ^ 1);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[set][mb][t], bv[set][nb][t],
                                                                          acc[mb][nb], 0, 0, 0);
        }
        // this wave's copies of the next chunk have landed (operand loads
        // issued after them may still be in flight) and its LDS reads of this
        // chunk are done; then a plain workgroup barrier, with compiler-only
        // fences around it (a release fence would also wait for the operand
        // loads)
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(NL));
        __asm__ __volatile__("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        __asm__ __volatile__("" ::: "memory");
    };
    copy_chunk(0, 0);
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    __syncthreads();
    int kc = 0;
    for (; kc < nk - TAIL; ++kc) chunk(kc, std::integral_constant<int, -1>{});
    if constexpr (TAIL > 0) {
        // the launcher guarantees nk >= TAIL
        seq_apply([&](auto p) { chunk(kc + decltype(p)::value, p); }, std::make_integer_sequence<int, TAIL>{});
    }

    if constexpr (MODE == MODE_ENERGY) {
        double esum[NP];
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int r = r0 + tcol(tb) + l16;
            double s = 0.0;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                s += energy_terms4<CPLX>(a, m0 + wm * TM + mb * 16 + 4 * lq, r, acc[mb][tb],
                                         CPLX ? acc[mb][NP + tb] : acc[mb][tb]);
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            esum[tb] = s;
        }
        double *red = reinterpret_cast<double *>(&lds[0][0]);
        if (lq == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) red[(wm * WN + wn) * (NP * 16) + tb * 16 + l16] = esum[tb];
        }
        __syncthreads();
        if (wm == 0 && lq == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) {
                double s = 0.0;
                for (int w = 0; w < WM; ++w) s += red[(w * WN + wn) * (NP * 16) + tb * 16 + l16];
                a.partial[(long long)mt * a.Rp + r0 + tcol(tb) + l16] = s;
            }
        }
    } else if constexpr ((CPLX ? 2 : 1) * TRAJ * (BM + 4) > 2 * TILE) {
        // sums of the whole tile exceed the two chunk buffers: stage and
        // update one wave column (TRAJ / WN trajectories) per pass
        constexpr int TP = BM + 4;
        constexpr int TRP = TRAJ / WN;
        static_assert(NPF == 0, "operand loads ahead follow the one-pass group order");
        static_assert((CPLX ? 2 : 1) * TRP * TP <= 2 * TILE, "staging fits LDS");
        static_assert((TRP * RG) % NT == 0, "epilogue split");
        constexpr int NUPP = TRP * RG / NT;
        float *st = &lds[0][0];
        float *sti = st + TRP * TP;
#pragma unroll
        for (int p = 0; p < WN; ++p) {
            if (wn == p) {
#pragma unroll
                for (int tb = 0; tb < NP; ++tb) {
                    const int tr = tcol(tb) - p * TRP + l16;
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) {
                        const int row = wm * TM + mb * 16 + 4 * lq;
                        *reinterpret_cast<f32x4 *>(&st[tr * TP + row]) = acc[mb][tb];
                        if (CPLX) *reinterpret_cast<f32x4 *>(&sti[tr * TP + row]) = acc[mb][NP + tb];
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
                const bool bad = step_epilogue4<MODE, CPLX, OP_F32>(a, m0 + row, r, rvalid, cr, ci);
                if (bad && rvalid) a.flags[r] = 1;
            }
            if (p + 1 < WN) __syncthreads();
        }
    } else {
        constexpr int TP = BM + 4;
        static_assert((CPLX ? 2 : 1) * TRAJ * TP <= 2 * TILE, "staging fits LDS");
        float *st = &lds[0][0];
        float *sti = st + TRAJ * TP;
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int tr = tcol(tb) + l16;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int row = wm * TM + mb * 16 + 4 * lq;
                *reinterpret_cast<f32x4 *>(&st[tr * TP + row]) = acc[mb][tb];
                if (CPLX) *reinterpret_cast<f32x4 *>(&sti[tr * TP + row]) = acc[mb][NP + tb];
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int g = tid + u * NT;
            const int tr = g / RG, row = (g % RG) * 4;
            const int r = r0 + tr;
            const bool rvalid = r < a.R;
            const f32x4 cr = *reinterpret_cast<const f32x4 *>(&st[tr * TP + row]);
            const f32x4 ci = CPLX ? *reinterpret_cast<const f32x4 *>(&sti[tr * TP + row]) : cr;
            bool bad;
            if constexpr (NPF > 0) {
                EpiIn in;
                epi_fill<MODE, CPLX>(a, m0 + row, &pf[u * NF], in);
                bad = epi_apply<MODE, CPLX, OP_F32>(a, m0 + row, r, rvalid, in, cr, ci);
            } else {
                bad = step_epilogue4<MODE, CPLX, OP_F32>(a, m0 + row, r, rvalid, cr, ci);
            }
            if (bad && rvalid) a.flags[r] = 1;
        }
    }
}

// chunks of the operand-load tail of the direct-to-LDS kernel in this mode
template <bool CPLX, int PF>
inline int dl_tail_chunks(int mode, int nu) {
    if (PF == 0 || mode == MODE_ENERGY) return 0;
    const int per = CPLX ? 3 : 2;
    const int nf = (mode == MODE_RK2 || mode == MODE_RK3 || mode == MODE_RK4) ? 3 * per : per;
    return (nu * nf + PF - 1) / PF;
}

template <int BM, int BN, int BK, int WM, int WN, bool CPLX, int PF>
hipError_t launch_modes_dl(int mode, const DenseStepArgs &a, hipStream_t st) {
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    if (a.Np % BM || a.Np % BK || a.Rp % TRAJ) return hipErrorInvalidValue;
    if (a.Np / BK < dl_tail_chunks<CPLX, PF>(mode, TRAJ * (BM / 4) / (64 * WM * WN))) return hipErrorInvalidValue;
    const int nblk = (a.Np / BM) * (a.Rp / TRAJ);
    const dim3 grid(nblk), block(64 * WM * WN);
#define GD_LAUNCH(M) dense_step_f32_dl<BM, BN, BK, WM, WN, CPLX, M, PF><<<grid, block, 0, st>>>(a)
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

template <int BM, int BN, int BK, int WM, int WN, bool CPLX, int KS, int LA>
hipError_t launch_modes(int mode, const DenseStepArgs &a, hipStream_t st) {
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    if (a.Np % BM || a.Np % BK || a.Rp % TRAJ) return hipErrorInvalidValue;
    const int nblk = (a.Np / BM) * (a.Rp / TRAJ);
    const dim3 grid(nblk), block(64 * WM * WN * KS);
#define GD_LAUNCH(M) dense_step_f32<BM, BN, BK, WM, WN, CPLX, M, KS, LA><<<grid, block, 0, st>>>(a)
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

// Variants {BM, BN (GEMM columns), BK, WM, WN, KS (K groups), LA (load
// lookahead in chunks), DL (0: chunks staged through registers; else
// direct-to-LDS copies with DL - 1 state-operand loads per tail chunk)}; identical for real and
// complex amplitudes (complex tiles hold BN/2 trajectories).  The runtime
// times the variants that tile a problem and keeps the fastest.
#define GD_DENSE_VARIANTS(X)               \
    X(0, 64, 64, 32, 2, 2, 1, 1, 0)        \
    X(1, 64, 128, 32, 2, 2, 1, 1, 0)       \
    X(2, 128, 128, 32, 2, 2, 1, 1, 0)      \
    X(3, 32, 64, 32, 1, 2, 1, 1, 0)        \
    X(4, 64, 64, 64, 2, 2, 1, 1, 0)        \
    X(5, 64, 128, 64, 2, 2, 1, 1, 0)       \
    X(6, 128, 64, 32, 4, 1, 1, 1, 0)       \
    X(7, 64, 64, 32, 2, 2, 2, 1, 0)        \
    X(8, 64, 64, 32, 2, 2, 1, 2, 0)        \
    X(9, 128, 128, 32, 2, 2, 1, 2, 0)      \
    X(10, 64, 64, 32, 2, 2, 1, 1, 1)       \
    X(11, 64, 128, 32, 2, 2, 1, 1, 1)      \
    X(12, 64, 64, 32, 2, 2, 1, 1, 2)       \
    X(13, 64, 64, 32, 2, 2, 1, 1, 3)       \
    X(14, 64, 64, 64, 2, 2, 1, 1, 3)       \
    X(15, 128, 128, 32, 2, 2, 1, 1, 1)

constexpr int kCfg[][8] = {
#define GD_ROW(id, bm, bn, bk, wm, wn, ks, la, dl) {bm, bn, bk, wm, wn, ks, la, dl},
    GD_DENSE_VARIANTS(GD_ROW)
#undef GD_ROW
};

}  // namespace

int dense_config_count(bool) { return int(sizeof(kCfg) / sizeof(kCfg[0])); }

DenseConfig dense_config(bool complex_mode, int idx) {
    DenseConfig c;
    c.id = idx;
    c.bm = kCfg[idx][0];
    c.bn = kCfg[idx][1];
    c.bk = kCfg[idx][2];
    c.wn = kCfg[idx][4];
    c.traj_tile = complex_mode ? c.bn / 2 : c.bn;
    c.threads = 64 * kCfg[idx][3] * kCfg[idx][4] * kCfg[idx][5];
    // direct-to-LDS variants with operand loads need as many K chunks as the
    // longest load tail (RK stages) has chunks
    const int pf = kCfg[idx][7] - 1;
    if (pf > 0) {
        const int nu = c.traj_tile * (c.bm / 4) / c.threads;
        const int nf = 3 * (complex_mode ? 3 : 2);
        c.min_np = c.bk * ((nu * nf + pf - 1) / pf);
    }
    return c;
}

hipError_t launch_dense_step(const DenseConfig &cfg, bool complex_mode, int mode, int op,
                             const DenseStepArgs &a, hipStream_t st) {
    if (op != OP_F32) return hipErrorInvalidValue;
#define GD_CASE(id, bm, bn, bk, wm, wn, ks, la, dl)                                      \
    case id:                                                                             \
        if constexpr (dl > 0)                                                            \
            return complex_mode ? launch_modes_dl<bm, bn, bk, wm, wn, true, dl - 1>(mode, a, st) \
                                : launch_modes_dl<bm, bn, bk, wm, wn, false, dl - 1>(mode, a, st); \
        else                                                                             \
            return complex_mode ? launch_modes<bm, bn, bk, wm, wn, true, ks, la>(mode, a, st) \
                                : launch_modes<bm, bn, bk, wm, wn, false, ks, la>(mode, a, st);
    switch (cfg.id) { GD_DENSE_VARIANTS(GD_CASE) }
#undef GD_CASE
    return hipErrorInvalidValue;
}

bool dense_config_fits(const DenseConfig &c, int Np, int Rp) {
    return Np % c.bm == 0 && Np % c.bk == 0 && Rp % c.traj_tile == 0 && Np >= c.min_np;
}

}  // namespace gd
