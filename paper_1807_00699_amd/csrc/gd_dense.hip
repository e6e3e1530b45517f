// Dense coupling step of the gain-dissipative method on gfx950.
//
// One launch evaluates, for every spin i and trajectory r of a tile, the
// coupling sum C_ir = (1/s) sum_j J_ij Psi_jr of Eq. (main) as a GEMM on the
// matrix cores (v_mfma_f32_32x32x2_f32, FP32 in and out), and then applies the
// pointwise part of Eq. (main) and Eq. (gamma) in the epilogue, so that the
// coupling result never leaves registers:
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
// loads and LDS holds both tiles as [row][k].
//
// Tiling: a workgroup owns 64 rows x BN GEMM columns; two waves along rows
// (32 rows each) and WN waves along columns.  Complex amplitudes use BN/2
// trajectories, real part in LDS columns [0, BN/2) and imaginary part in
// [BN/2, BN), arranged so that each wave holds the real and imaginary
// accumulators of the same (i, r) in the same lane and register.
//
// K order inside a 16-wide slice is permuted so that lane half h feeds
// k = 8h + t to MFMA number t; A and B use the same permutation, so each lane
// fetches 8 contiguous floats with two ds_read_b128 per operand block.
#include "gd_internal.h"

namespace gd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int BM = kRowTile;  // rows per workgroup
constexpr int WM = 2;         // waves along rows
constexpr int BK = 32;        // K chunk per pipeline stage
constexpr int LDP = BK + 4;   // LDS row pitch in floats (conflict-free b128 reads)

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

__device__ inline bool finite4(float a) { return __builtin_isfinite(a); }

template <int BN, int WN, bool CPLX, int MODE>
__global__ void __launch_bounds__(64 * WM * WN)
dense_step_f32(DenseStepArgs a) {
    constexpr int NT = 64 * WM * WN;
    constexpr int TM = BM / WM;     // 32 rows per wave
    constexpr int TN = BN / WN;     // GEMM columns per wave
    constexpr int MB = TM / 32;     // MFMA row blocks per wave
    constexpr int NB = TN / 32;     // MFMA column blocks per wave
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    static_assert(MB == 1, "two waves of 32 rows");
    static_assert(!CPLX || (NB % 2 == 0), "complex waves pair re/im blocks");
    constexpr int KQ = BK / 4;                 // float4 per row chunk
    constexpr int AL = BM * KQ / NT;           // A float4 loads per thread
    constexpr int BL = BN * KQ / NT;           // B float4 loads per thread
    static_assert(BM * KQ % NT == 0 && BN * KQ % NT == 0, "load split");

    __shared__ __attribute__((aligned(16))) float lds[2][(BM + BN) * LDP];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
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

    f32x4 ra[AL], rb[BL];
    auto gload = [&](int k0) {
#pragma unroll
        for (int u = 0; u < AL; ++u) {
            const int q = tid + u * NT;
            const int row = q / KQ, kq = q % KQ;
            ra[u] = *reinterpret_cast<const f32x4 *>(J + (m0 + row) * Np + k0 + kq * 4);
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int q = tid + u * NT;
            const int col = q / KQ, kq = q % KQ;
            const int plane = CPLX ? col / (BN / 2) : 0;
            const int tr = CPLX ? col % (BN / 2) : col;
            rb[u] = *reinterpret_cast<const f32x4 *>(Bop + plane * a.plane_stride +
                                                     (r0 + tr) * Np + k0 + kq * 4);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < AL; ++u) {
            const int q = tid + u * NT;
            const int row = q / KQ, kq = q % KQ;
            *reinterpret_cast<f32x4 *>(&lds[buf][row * LDP + kq * 4]) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int q = tid + u * NT;
            const int col = q / KQ, kq = q % KQ;
            *reinterpret_cast<f32x4 *>(&lds[buf][(BM + col) * LDP + kq * 4]) = rb[u];
        }
    };
    // LDS column of block nb for this wave
    auto bcol = [&](int nb) -> int {
        if (CPLX) {
            constexpr int half = NB / 2;
            const int p = nb / half, tb = nb % half;
            return p * (BN / 2) + wn * (TN / 2) + tb * 32;
        }
        return wn * TN + nb * 32;
    };

    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[nb][v] = 0.0f;

    const int nk = a.Np / BK;
    gload(0);
    lstore(0);
    __syncthreads();
    const int lrow = lane & 31;
    const int lh = lane >> 5;
    for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nk) gload((kc + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK / 16; ++kk) {
            const float *pa = &lds[buf][(wm * TM + lrow) * LDP + kk * 16 + lh * 8];
            const f32x4 a0 = *reinterpret_cast<const f32x4 *>(pa);
            const f32x4 a1 = *reinterpret_cast<const f32x4 *>(pa + 4);
            f32x4 b0[NB], b1[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float *pb = &lds[buf][(BM + bcol(nb) + lrow) * LDP + kk * 16 + lh * 8];
                b0[nb] = *reinterpret_cast<const f32x4 *>(pb);
                b1[nb] = *reinterpret_cast<const f32x4 *>(pb + 4);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[t], b0[nb][t], acc[nb], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[t], b1[nb][t], acc[nb], 0, 0, 0);
        }
        if (kc + 1 < nk) lstore(buf ^ 1);
        __syncthreads();
    }

    // ---------------------------------------------------------------- epilogue
    // acc[nb][4q + e] holds row i = m0 + wm*32 + 8q + 4*lh + e, column lrow of block nb.
    const int ibase = m0 + wm * TM + 4 * lh;
    constexpr int NP = CPLX ? NB / 2 : NB;   // trajectory blocks per wave
    if constexpr (MODE == MODE_ENERGY) {
        // e_ir = -sum_p D_p(i,r) T_p(i,r) + g_i D_0(i,r); reduce over the 64 rows.
        double esum[NP];
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int r = r0 + (CPLX ? wn * (TN / 2) + tb * 32 : bcol(tb)) + lrow;
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i0 = ibase + 8 * q;
                const long long idx = (long long)r * Np + i0;
                const f32x4 d0 = *reinterpret_cast<const f32x4 *>(a.psi_in + idx);
                const f32x4 gg = *reinterpret_cast<const f32x4 *>(a.g + i0);
                f32x4 d1 = {0.f, 0.f, 0.f, 0.f};
                if (CPLX) d1 = *reinterpret_cast<const f32x4 *>(a.psi_in + a.plane_stride + idx);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    double t = -(double)d0[e] * (double)acc[tb][4 * q + e] + (double)gg[e] * (double)d0[e];
                    if (CPLX) t -= (double)d1[e] * (double)acc[NP + tb][4 * q + e];
                    s += t;
                }
            }
            s += __shfl_xor(s, 32);
            esum[tb] = s;
        }
        // combine the two row waves through LDS (main loop is done with it)
        __syncthreads();
        double *red = reinterpret_cast<double *>(&lds[0][0]);
        if (wm == 1 && lh == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) red[(wn * NP + tb) * 32 + lrow] = esum[tb];
        }
        __syncthreads();
        if (wm == 0 && lh == 0) {
#pragma unroll
            for (int tb = 0; tb < NP; ++tb) {
                const int r = r0 + (CPLX ? wn * (TN / 2) + tb * 32 : bcol(tb)) + lrow;
                a.partial[(long long)mt * a.Rp + r] = esum[tb] + red[(wn * NP + tb) * 32 + lrow];
            }
        }
        return;
    } else {
        const float inv_s = a.inv_s, dt = a.dt, gc = a.gamma_c, rho_th = a.rho_th;
#pragma unroll
        for (int tb = 0; tb < NP; ++tb) {
            const int r = r0 + (CPLX ? wn * (TN / 2) + tb * 32 : bcol(tb)) + lrow;
            const bool rvalid = r < a.R;
            bool bad = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i0 = ibase + 8 * q;
                const long long idx = (long long)r * Np + i0;
                const f32x4 ep = *reinterpret_cast<const f32x4 *>(a.eps + i0);
                const f32x4 hh = *reinterpret_cast<const f32x4 *>(a.h1 + i0);
                const f32x4 xr = *reinterpret_cast<const f32x4 *>(a.psi_in + idx);
                f32x4 xi = {0.f, 0.f, 0.f, 0.f};
                if (CPLX) xi = *reinterpret_cast<const f32x4 *>(a.psi_in + a.plane_stride + idx);
                const f32x4 gm = *reinterpret_cast<const f32x4 *>(a.gam_in + idx);
                f32x4 fr, fi, fg;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float rho = CPLX ? xr[e] * xr[e] + xi[e] * xi[e] : xr[e] * xr[e];
                    const float lin = gm[e] - gc - rho;
                    fr[e] = xr[e] * lin + acc[tb][4 * q + e] * inv_s + hh[e];
                    if (CPLX) fi[e] = xi[e] * lin + acc[NP + tb][4 * q + e] * inv_s;
                    fg[e] = ep[e] * (rho_th - rho);
                }
                // rows beyond n keep their (zero) state and gain
                bool rowv[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) rowv[e] = rvalid && (i0 + e < a.n);

                if constexpr (MODE == MODE_EULER) {
                    f32x4 nr, ni, ng;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        nr[e] = rowv[e] ? xr[e] + dt * fr[e] : xr[e];
                        if (CPLX) ni[e] = rowv[e] ? xi[e] + dt * fi[e] : xi[e];
                        ng[e] = rowv[e] ? gm[e] + dt * fg[e] : gm[e];
                        bad |= !(finite4(nr[e]) && finite4(ng[e]) && (!CPLX || finite4(ni[e])));
                    }
                    *reinterpret_cast<f32x4 *>(a.psi_out + idx) = nr;
                    if (CPLX) *reinterpret_cast<f32x4 *>(a.psi_out + a.plane_stride + idx) = ni;
                    *reinterpret_cast<f32x4 *>(a.gam_out + idx) = ng;
                } else {
                    // RK4 stage on y = (psi, gamma); psi_in/gam_in is the stage input
                    f32x4 yr, yi, yg;
                    if constexpr (MODE == MODE_RK1) {
                        yr = xr; yi = xi; yg = gm;
                    } else {
                        yr = *reinterpret_cast<const f32x4 *>(a.y_psi + idx);
                        if (CPLX) yi = *reinterpret_cast<const f32x4 *>(a.y_psi + a.plane_stride + idx);
                        yg = *reinterpret_cast<const f32x4 *>(a.y_gam + idx);
                    }
                    f32x4 ar, ai, ag;
                    if constexpr (MODE == MODE_RK1) {
                        ar = fr; ai = fi; ag = fg;
                    } else {
                        ar = *reinterpret_cast<const f32x4 *>(a.acc_psi + idx);
                        if (CPLX) ai = *reinterpret_cast<const f32x4 *>(a.acc_psi + a.plane_stride + idx);
                        ag = *reinterpret_cast<const f32x4 *>(a.acc_gam + idx);
                    }
                    if constexpr (MODE == MODE_RK4) {
                        const float c6 = dt * (1.0f / 6.0f);
                        f32x4 nr, ni, ng;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            nr[e] = rowv[e] ? yr[e] + c6 * (ar[e] + fr[e]) : yr[e];
                            if (CPLX) ni[e] = rowv[e] ? yi[e] + c6 * (ai[e] + fi[e]) : yi[e];
                            ng[e] = rowv[e] ? yg[e] + c6 * (ag[e] + fg[e]) : yg[e];
                            bad |= !(finite4(nr[e]) && finite4(ng[e]) && (!CPLX || finite4(ni[e])));
                        }
                        *reinterpret_cast<f32x4 *>(a.psi_out + idx) = nr;
                        if (CPLX) *reinterpret_cast<f32x4 *>(a.psi_out + a.plane_stride + idx) = ni;
                        *reinterpret_cast<f32x4 *>(a.gam_out + idx) = ng;
                    } else {
                        if constexpr (MODE != MODE_RK1) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                ar[e] += 2.0f * fr[e];
                                if (CPLX) ai[e] += 2.0f * fi[e];
                                ag[e] += 2.0f * fg[e];
                            }
                        }
                        const float c = (MODE == MODE_RK3) ? dt : 0.5f * dt;
                        f32x4 sr, si, sg;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            sr[e] = rowv[e] ? yr[e] + c * fr[e] : yr[e];
                            if (CPLX) si[e] = rowv[e] ? yi[e] + c * fi[e] : yi[e];
                            sg[e] = rowv[e] ? yg[e] + c * fg[e] : yg[e];
                        }
                        *reinterpret_cast<f32x4 *>(a.acc_psi + idx) = ar;
                        if (CPLX) *reinterpret_cast<f32x4 *>(a.acc_psi + a.plane_stride + idx) = ai;
                        *reinterpret_cast<f32x4 *>(a.acc_gam + idx) = ag;
                        *reinterpret_cast<f32x4 *>(a.psi_out + idx) = sr;
                        if (CPLX) *reinterpret_cast<f32x4 *>(a.psi_out + a.plane_stride + idx) = si;
                        *reinterpret_cast<f32x4 *>(a.gam_out + idx) = sg;
                    }
                }
            }
            if (bad && rvalid) a.flags[r] = 1;
        }
    }
}

template <int BN, int WN, bool CPLX>
hipError_t launch_modes(int mode, const DenseStepArgs &a, hipStream_t st) {
    constexpr int TRAJ = CPLX ? BN / 2 : BN;
    const int nblk = (a.Np / BM) * (a.Rp / TRAJ);
    const dim3 grid(nblk), block(64 * WM * WN);
    switch (mode) {
    case MODE_EULER: dense_step_f32<BN, WN, CPLX, MODE_EULER><<<grid, block, 0, st>>>(a); break;
    case MODE_RK1: dense_step_f32<BN, WN, CPLX, MODE_RK1><<<grid, block, 0, st>>>(a); break;
    case MODE_RK2: dense_step_f32<BN, WN, CPLX, MODE_RK2><<<grid, block, 0, st>>>(a); break;
    case MODE_RK3: dense_step_f32<BN, WN, CPLX, MODE_RK3><<<grid, block, 0, st>>>(a); break;
    case MODE_RK4: dense_step_f32<BN, WN, CPLX, MODE_RK4><<<grid, block, 0, st>>>(a); break;
    case MODE_ENERGY: dense_step_f32<BN, WN, CPLX, MODE_ENERGY><<<grid, block, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Variants: {GEMM columns per workgroup, waves along columns}.
constexpr int kRealCfg[][2] = {{64, 2}, {128, 2}, {128, 4}};
constexpr int kCplxCfg[][2] = {{64, 1}, {128, 2}, {256, 2}};

}  // namespace

int dense_config_count(bool complex_mode) {
    return complex_mode ? int(sizeof(kCplxCfg) / sizeof(kCplxCfg[0]))
                        : int(sizeof(kRealCfg) / sizeof(kRealCfg[0]));
}

DenseConfig dense_config(bool complex_mode, int idx) {
    const int(*t)[2] = complex_mode ? kCplxCfg : kRealCfg;
    DenseConfig c;
    c.id = idx;
    c.bn = t[idx][0];
    c.wn = t[idx][1];
    c.traj_tile = complex_mode ? c.bn / 2 : c.bn;
    c.threads = 64 * WM * c.wn;
    return c;
}

hipError_t launch_dense_step(const DenseConfig &cfg, bool complex_mode, int mode, int op,
                             const DenseStepArgs &a, hipStream_t st) {
    if (op != OP_F32) return hipErrorInvalidValue;
    if (a.Np % BM || a.Rp % cfg.traj_tile) return hipErrorInvalidValue;
    if (complex_mode) {
        switch (cfg.id) {
        case 0: return launch_modes<64, 1, true>(mode, a, st);
        case 1: return launch_modes<128, 2, true>(mode, a, st);
        case 2: return launch_modes<256, 2, true>(mode, a, st);
        }
    } else {
        switch (cfg.id) {
        case 0: return launch_modes<64, 2, false>(mode, a, st);
        case 1: return launch_modes<128, 2, false>(mode, a, st);
        case 2: return launch_modes<128, 4, false>(mode, a, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace gd
