// Pointwise part of one integration step, shared by every coupling kernel.
//
// Given the coupling sums C (already computed by a GEMM, before the 1/s
// scale) for four consecutive spins i0..i0+3 of trajectory r, apply the rest
// of Eq. (main) and Eq. (gamma):
//   f   = Psi (gamma - gamma_c - |Psi|^2) + C / s + h_1 + h_q conj(Psi)^(q-1)
//   phi = eps_i (rho_th - |Psi|^2)
// and an Euler update or one stage of the classical RK4 scheme on the joint
// state (Psi, gamma).  The final stage of a step adds the noise increment
// D sqrt(dt) eta (Euler-Maruyama for the Euler scheme; the same additive
// increment after the deterministic RK4 step).  Optionally writes a BF16/FP16
// copy of the new amplitudes: the operand of the next coupling GEMM.
#pragma once
#include "gd_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <utility>

namespace gd {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline bool gd_finite(float a) { return __builtin_isfinite(a); }

// SplitMix64 (Steele, Lea, Flood 2014): one output of the generator whose
// state was z before the output step.
__device__ inline unsigned long long mix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Two independent standard normal numbers for (trajectory r, spin i) of the
// step keyed by `key`, by the Box-Muller transform of two 24-bit uniforms:
// u1 = (m1 + 1) 2^-24 in (0, 1], u2 = m2 2^-24 in [0, 1) (both exact in FP32).
__device__ inline void noise_pair(unsigned long long key, int r, int i, float &g0, float &g1) {
    const unsigned long long ctr = ((unsigned long long)(unsigned)r << 32) | (unsigned)i;
    const unsigned long long z = mix64(key ^ mix64(ctr));
    const float u1 = float((z >> 40) + 1ull) * 5.9604644775390625e-8f;       // 2^-24
    const float two_u2 = float((z >> 16) & 0xFFFFFFull) * 1.1920928955078125e-7f;  // 2^-23
    const float rad = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincospif(two_u2, &sn, &cs);   // angle 2 pi u2
    g0 = rad * cs;
    g1 = rad * sn;
}

// store four consecutive floats as BF16 / FP16 (round to nearest even)
template <int OPT>
__device__ inline void store_shadow4(void *base, long long idx, f32x4 v) {
    if constexpr (OPT == OP_BF16) {
        __hip_bfloat16 *p = static_cast<__hip_bfloat16 *>(base) + idx;
        __hip_bfloat162 lo = __halves2bfloat162(__float2bfloat16(v[0]), __float2bfloat16(v[1]));
        __hip_bfloat162 hi = __halves2bfloat162(__float2bfloat16(v[2]), __float2bfloat16(v[3]));
        reinterpret_cast<__hip_bfloat162 *>(p)[0] = lo;
        reinterpret_cast<__hip_bfloat162 *>(p)[1] = hi;
    } else if constexpr (OPT == OP_F16) {
        __half *p = static_cast<__half *>(base) + idx;
        reinterpret_cast<__half2 *>(p)[0] = __floats2half2_rn(v[0], v[1]);
        reinterpret_cast<__half2 *>(p)[1] = __floats2half2_rn(v[2], v[3]);
    }
}

// Operands of the pointwise update of four consecutive spins of one
// trajectory, loaded ahead of the update (the dense kernel issues these loads
// during its last GEMM iterations so their latency overlaps the matrix work).
struct EpiIn {
    f32x4 ep, hh, xr, xi, gm, yr, yi, yg, ar, ai, ag;
};

template <int MODE, bool CPLX>
__device__ inline void epi_load(const DenseStepArgs &a, int i0, int r, EpiIn &in) {
    const long long idx = (long long)r * a.Np + i0;
    const long long ps = a.plane_stride;
    in.ep = *reinterpret_cast<const f32x4 *>(a.eps + i0);
    in.hh = *reinterpret_cast<const f32x4 *>(a.h1 + i0);
    in.xr = *reinterpret_cast<const f32x4 *>(a.psi_in + idx);
    in.xi = f32x4{0.f, 0.f, 0.f, 0.f};
    if (CPLX) in.xi = *reinterpret_cast<const f32x4 *>(a.psi_in + ps + idx);
    in.gm = *reinterpret_cast<const f32x4 *>(a.gam_in + idx);
    if constexpr (MODE == MODE_RK2 || MODE == MODE_RK3 || MODE == MODE_RK4) {
        in.yr = *reinterpret_cast<const f32x4 *>(a.y_psi + idx);
        in.yi = CPLX ? *reinterpret_cast<const f32x4 *>(a.y_psi + ps + idx) : f32x4{0.f, 0.f, 0.f, 0.f};
        in.yg = *reinterpret_cast<const f32x4 *>(a.y_gam + idx);
        in.ar = *reinterpret_cast<const f32x4 *>(a.acc_psi + idx);
        in.ai = CPLX ? *reinterpret_cast<const f32x4 *>(a.acc_psi + ps + idx) : f32x4{0.f, 0.f, 0.f, 0.f};
        in.ag = *reinterpret_cast<const f32x4 *>(a.acc_gam + idx);
    }
}

// State operands the pointwise update reads per (trajectory, 4 rows) group:
// Psi (re, im), gamma, and for RK stages 2..4 also the stage base y and the
// slope accumulator.
template <int MODE, bool CPLX>
constexpr int epi_fields() {
    if constexpr (MODE == MODE_ENERGY) return 0;
    constexpr int per = CPLX ? 3 : 2;
    return (MODE == MODE_RK2 || MODE == MODE_RK3 || MODE == MODE_RK4) ? 3 * per : per;
}

// f(integral_constant<P>) for each P of the sequence, in order
template <typename F, int... P>
__device__ inline void seq_apply(F &&f, std::integer_sequence<int, P...>) {
    (f(std::integral_constant<int, P>{}), ...);
}

template <bool CPLX>
__device__ inline const float *epi_field_ptr(const DenseStepArgs &a, int f) {
    constexpr int per = CPLX ? 3 : 2;
    const float *base[3][2] = {{a.psi_in, a.gam_in}, {a.y_psi, a.y_gam}, {a.acc_psi, a.acc_gam}};
    const int blk = f / per, k = f % per;
    if (CPLX && k == 1) return base[blk][0] + a.plane_stride;
    return base[blk][k == 0 ? 0 : 1];
}

// EpiIn of one group from its state fields q[0 .. epi_fields) loaded ahead
// (in epi_field_ptr order) and the per-row eps and h1 loaded here
template <int MODE, bool CPLX>
__device__ inline void epi_fill(const DenseStepArgs &a, int i0, const f32x4 *q, EpiIn &in) {
    constexpr int per = CPLX ? 3 : 2;
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    in.ep = *reinterpret_cast<const f32x4 *>(a.eps + i0);
    in.hh = *reinterpret_cast<const f32x4 *>(a.h1 + i0);
    in.xr = q[0];
    in.xi = CPLX ? q[1] : z;
    in.gm = q[per - 1];
    if constexpr (epi_fields<MODE, CPLX>() > per) {
        in.yr = q[per];
        in.yi = CPLX ? q[per + 1] : z;
        in.yg = q[2 * per - 1];
        in.ar = q[2 * per];
        in.ai = CPLX ? q[2 * per + 1] : z;
        in.ag = q[3 * per - 1];
    }
}

// Returns true if a written value is non-finite.  cr/ci: raw GEMM sums.
template <int MODE, bool CPLX, int OPT>
__device__ inline bool epi_apply(const DenseStepArgs &a, int i0, int r, bool rvalid, const EpiIn &in,
                                 f32x4 cr, f32x4 ci) {
    const long long idx = (long long)r * a.Np + i0;
    const long long ps = a.plane_stride;
    const float inv_s = a.inv_s, dt = a.dt, gc = a.gamma_c, rho_th = a.rho_th;
    const f32x4 ep = in.ep, hh = in.hh, xr = in.xr, xi = in.xi, gm = in.gm;
    f32x4 fr, fi, fg;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float rho = CPLX ? xr[e] * xr[e] + xi[e] * xi[e] : xr[e] * xr[e];
        const float lin = gm[e] - gc - rho;
        fr[e] = xr[e] * lin + cr[e] * inv_s + hh[e];
        fi[e] = CPLX ? xi[e] * lin + ci[e] * inv_s : 0.0f;
        fg[e] = ep[e] * (rho_th - rho);
    }
    if (CPLX && a.q >= 2) {
        // resonant term h_q conj(Psi)^(q-1): repeated products with conj(Psi)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float pr = xr[e], pi = -xi[e];
            for (int k = 2; k < a.q; ++k) {
                const float tr = pr * xr[e] + pi * xi[e];
                const float ti = pi * xr[e] - pr * xi[e];
                pr = tr;
                pi = ti;
            }
            fr[e] += a.hq * pr;
            fi[e] += a.hq * pi;
        }
    }
    // rows beyond n and padded trajectories keep their (zero) state and gain
    bool rowv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) rowv[e] = rvalid && (i0 + e < a.n);
    bool bad = false;
    f32x4 nr, ni, ng;   // values written to psi_out / gam_out
    if constexpr (MODE == MODE_EULER) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            nr[e] = rowv[e] ? xr[e] + dt * fr[e] : xr[e];
            ni[e] = rowv[e] ? xi[e] + dt * fi[e] : xi[e];
            ng[e] = rowv[e] ? gm[e] + dt * fg[e] : gm[e];
        }
    } else {
        // RK4 stage on y = (psi, gamma); psi_in/gam_in is the stage input
        f32x4 yr = xr, yi = xi, yg = gm;
        f32x4 ar = fr, ai = fi, ag = fg;
        if constexpr (MODE != MODE_RK1) {
            yr = in.yr;
            yi = in.yi;
            yg = in.yg;
            ar = in.ar;
            ai = in.ai;
            ag = in.ag;
        }
        if constexpr (MODE == MODE_RK4) {
            const float c6 = dt * (1.0f / 6.0f);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                nr[e] = rowv[e] ? yr[e] + c6 * (ar[e] + fr[e]) : yr[e];
                ni[e] = rowv[e] ? yi[e] + c6 * (ai[e] + fi[e]) : yi[e];
                ng[e] = rowv[e] ? yg[e] + c6 * (ag[e] + fg[e]) : yg[e];
            }
        } else {
            if constexpr (MODE != MODE_RK1) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ar[e] += 2.0f * fr[e];
                    ai[e] += 2.0f * fi[e];
                    ag[e] += 2.0f * fg[e];
                }
            }
            const float c = (MODE == MODE_RK3) ? dt : 0.5f * dt;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                nr[e] = rowv[e] ? yr[e] + c * fr[e] : yr[e];
                ni[e] = rowv[e] ? yi[e] + c * fi[e] : yi[e];
                ng[e] = rowv[e] ? yg[e] + c * fg[e] : yg[e];
            }
            *reinterpret_cast<f32x4 *>(a.acc_psi + idx) = ar;
            if (CPLX) *reinterpret_cast<f32x4 *>(a.acc_psi + ps + idx) = ai;
            *reinterpret_cast<f32x4 *>(a.acc_gam + idx) = ag;
        }
    }
    if constexpr (MODE == MODE_EULER || MODE == MODE_RK4) {
        if (a.noise_amp != 0.0f) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (rowv[e]) {
                    float g0, g1;
                    noise_pair(a.noise_key, r, i0 + e, g0, g1);
                    nr[e] += a.noise_amp * g0;
                    if (CPLX) ni[e] += a.noise_amp * g1;
                }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) bad |= !(gd_finite(nr[e]) && gd_finite(ng[e]) && gd_finite(ni[e]));
    }
    *reinterpret_cast<f32x4 *>(a.psi_out + idx) = nr;
    if (CPLX) *reinterpret_cast<f32x4 *>(a.psi_out + ps + idx) = ni;
    *reinterpret_cast<f32x4 *>(a.gam_out + idx) = ng;
    if constexpr (OPT != OP_F32) {
        store_shadow4<OPT>(a.shadow_out, idx, nr);
        if (CPLX) store_shadow4<OPT>(a.shadow_out, ps + idx, ni);
    }
    return bad;
}

template <int MODE, bool CPLX, int OPT>
__device__ inline bool step_epilogue4(const DenseStepArgs &a, int i0, int r, bool rvalid,
                                      f32x4 cr, f32x4 ci) {
    EpiIn in;
    epi_load<MODE, CPLX>(a, i0, r, in);
    return epi_apply<MODE, CPLX, OPT>(a, i0, r, rvalid, in, cr, ci);
}

// Energy terms of Eq. (h) for four consecutive spins of trajectory r:
// sum_e [ -(D_0 T_0 + w D_1 T_1) + g_i D_0 ] in FP64 (T: raw GEMM sums of
// J D; w = im_weight).
template <bool CPLX>
__device__ inline double energy_terms4(const DenseStepArgs &a, int i0, int r, f32x4 tr, f32x4 ti) {
    const long long idx = (long long)r * a.Np + i0;
    const f32x4 d0 = *reinterpret_cast<const f32x4 *>(a.psi_in + idx);
    const f32x4 gg = *reinterpret_cast<const f32x4 *>(a.g + i0);
    f32x4 d1 = {0.f, 0.f, 0.f, 0.f};
    if (CPLX) d1 = *reinterpret_cast<const f32x4 *>(a.psi_in + a.plane_stride + idx);
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        double t = -(double)d0[e] * (double)tr[e] + (double)gg[e] * (double)d0[e];
        if (CPLX) t -= (double)a.im_weight * ((double)d1[e] * (double)ti[e]);
        s += t;
    }
    return s;
}

}  // namespace gd
