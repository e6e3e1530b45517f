// Batched solver for many instances of uneven size with sparse couplings.
//
// One persistent launch integrates every instance of a batch.  The work is
// split into items (instance k, slice of T trajectories); the host assigns
// items to workgroups by longest-processing-time-first bin packing and each
// workgroup runs its items one after the other, every item for all steps.
// Instances and trajectories are independent (Eq. (main) couples spins of one
// trajectory of one instance only), so no grid-wide synchronisation exists.
//
// Inside an item the amplitudes x_i of the T trajectories sit in LDS as
// [i][T] (the neighbour gathers of the coupling sum read them), each thread
// owns a fixed trajectory r = tid % T and the spins i = tid / T + s * (NT / T)
// for slots s < E, keeping x_ir and gamma_ir in registers across steps.  The
// couplings are an ELL list (dmax neighbours per spin, zero-weight padding),
// copied into LDS at the start of the item.  One step (explicit Euler on
// Eq. (main) and Eq. (gamma), real amplitudes):
//   c   = (1/s_k) sum_d w_id x_{j(i,d)}
//   x  += dt [ x (gamma - gamma_c - x^2) + c + h_1 ]
//   gamma += dt eps_i (rho_th - x^2)
// The update order is fixed (sum over d in list order), so a trajectory's
// result does not depend on T, NT or the rest of the batch.
// After the last step the Eq. (h) energy of the discretised state
// (s_i = sign x_i) is reduced per trajectory in FP64 in a fixed order.
#include "gd_internal.h"

namespace gd {

namespace {

template <int T, int NT, int E>
__global__ void __launch_bounds__(NT)
batch_ell_euler(BatchArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x;
    const int r = tid % T;
    const int ibase = tid / T;
    constexpr int ISTR = NT / T;
    const int dmax = a.dmax;
    float *xl = reinterpret_cast<float *>(smem);                               // [nmax][T]
    float *wl = xl + (size_t)a.nmax * T;                                        // [nmax][dmax]
    unsigned short *il = reinterpret_cast<unsigned short *>(wl + (size_t)a.nmax * dmax);
    double *red = reinterpret_cast<double *>(smem);                             // reuse after the run

    for (int it = a.wg_off[blockIdx.x]; it < a.wg_off[blockIdx.x + 1]; ++it) {
        const int item = a.items[it];
        const int k = item / a.nslices;
        const int rr = (item % a.nslices) * T + r;      // trajectory within the instance
        const int n = a.inst_n[k];
        const long long spin0 = a.inst_spin[k];
        const long long st0 = a.inst_state[k] + (long long)rr * n;   // [R][n] block of instance k
        const float inv_s = a.inst_inv_s[k];
        // couplings of instance k into LDS
        for (int q = tid; q < n * dmax; q += NT) {
            wl[q] = a.ell_w[spin0 * dmax + q];
            il[q] = (unsigned short)a.ell_idx[spin0 * dmax + q];
        }
        float xo[E], go[E], ep[E], hh[E];
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int i = ibase + s * ISTR;
            xo[s] = go[s] = ep[s] = hh[s] = 0.0f;
            if (i < n) {
                xo[s] = a.x[st0 + i];
                go[s] = a.gam[st0 + i];
                ep[s] = a.eps[spin0 + i];
                hh[s] = a.h1[spin0 + i];
                xl[i * T + r] = xo[s];
            }
        }
        __syncthreads();
        const float dt = a.dt, gc = a.gamma_c, rho_th = a.rho_th;
        for (int step = 0; step < a.steps; ++step) {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int i = ibase + s * ISTR;
                if (i < n) {
                    float c = 0.0f;
                    for (int d = 0; d < dmax; ++d) c += wl[i * dmax + d] * xl[il[i * dmax + d] * T + r];
                    const float x = xo[s];
                    const float rho = x * x;
                    const float f = x * (go[s] - gc - rho) + c * inv_s + hh[s];
                    xo[s] = x + dt * f;
                    go[s] = go[s] + dt * (ep[s] * (rho_th - rho));
                }
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int i = ibase + s * ISTR;
                if (i < n) xl[i * T + r] = xo[s];
            }
            __syncthreads();
        }
        // write back the state, flag non-finite trajectories
        bool bad = false;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int i = ibase + s * ISTR;
            if (i < n) {
                a.x[st0 + i] = xo[s];
                a.gam[st0 + i] = go[s];
                bad |= !(__builtin_isfinite(xo[s]) && __builtin_isfinite(go[s]));
            }
        }
        // energy of the discretised state, Eq. (h): -sum_i s_i sum_d w_id s_j + g_i s_i
        double e = 0.0;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int i = ibase + s * ISTR;
            if (i < n) {
                const double si = xo[s] < 0.0f ? -1.0 : 1.0;
                double h = 0.0;
                for (int d = 0; d < dmax; ++d) {
                    const float xj = xl[il[i * dmax + d] * T + r];
                    h += (double)wl[i * dmax + d] * (xj < 0.0f ? -1.0 : 1.0);
                }
                e += -si * h + (double)a.g[spin0 + i] * si;
            }
        }
        __syncthreads();                       // all reads of xl / wl are done
        red[tid] = e;
        __syncthreads();
        if (tid < T) {
            double tot = 0.0;
            for (int q = tid; q < NT; q += T) tot += red[q];   // fixed order
            a.E[(long long)k * a.R + (item % a.nslices) * T + tid] = tot;
        }
        if (bad) a.flags[(long long)k * a.R + rr] = 1;
        __syncthreads();                       // LDS is reused by the next item
    }
}

// Variants {T, NT, E}: T trajectories per item, NT threads, E slots per thread
// (n_max <= E * NT / T).
#define GD_BATCH_VARIANTS(X) \
    X(0, 8, 1024, 16)        \
    X(1, 4, 512, 16)         \
    X(2, 2, 256, 16)         \
    X(3, 8, 512, 32)         \
    X(4, 16, 1024, 16)       \
    X(5, 4, 1024, 8)         \
    X(6, 1, 256, 16)

constexpr int kBatchCfg[][3] = {
#define GD_ROW(id, t, nt, e) {t, nt, e},
    GD_BATCH_VARIANTS(GD_ROW)
#undef GD_ROW
};

}  // namespace

int batch_config_count() { return int(sizeof(kBatchCfg) / sizeof(kBatchCfg[0])); }

BatchConfig batch_config(int idx) {
    BatchConfig c;
    c.id = idx;
    c.traj = kBatchCfg[idx][0];
    c.threads = kBatchCfg[idx][1];
    c.slots = kBatchCfg[idx][2];
    return c;
}

size_t batch_lds_bytes(const BatchConfig &c, int nmax, int dmax) {
    size_t b = (size_t)nmax * c.traj * 4 + (size_t)nmax * dmax * 4 + (size_t)nmax * dmax * 2;
    b = (b + 15) / 16 * 16;
    const size_t red = (size_t)c.threads * 8;
    return b > red ? b : red;
}

hipError_t prepare_batch(const BatchConfig &c, int nmax, int dmax) {
    const int lds = int(batch_lds_bytes(c, nmax, dmax));
#define GD_CASE(id, t, nt, e)                                                                   \
    case id:                                                                                    \
        return hipFuncSetAttribute(reinterpret_cast<const void *>(&batch_ell_euler<t, nt, e>), \
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    switch (c.id) { GD_BATCH_VARIANTS(GD_CASE) }
#undef GD_CASE
    return hipErrorInvalidValue;
}

// Running best of a batch run's checks, one workgroup per instance k: the
// lowest E[k][r] (ties -> lowest r) replaces (best_E[k], best_r[k]) when it
// is strictly lower, as when the host reads every check back.
__global__ void __launch_bounds__(256)
batch_best_k(const double *__restrict__ E, int R, double *__restrict__ best_E, int *__restrict__ best_r) {
    __shared__ double sv[256];
    __shared__ int si[256];
    const int k = blockIdx.x, tid = threadIdx.x;
    double bv = __builtin_inf();
    int bi = 0x7fffffff;
    for (int r = tid; r < R; r += 256) {
        const double s = E[(long long)k * R + r];
        if (s < bv || (s == bv && r < bi)) { bv = s; bi = r; }
    }
    sv[tid] = bv;
    si[tid] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            const double ov = sv[tid + w];
            const int oi = si[tid + w];
            if (ov < sv[tid] || (ov == sv[tid] && oi < si[tid])) {
                sv[tid] = ov;
                si[tid] = oi;
            }
        }
        __syncthreads();
    }
    if (tid == 0 && si[0] != 0x7fffffff && sv[0] < best_E[k]) {
        best_E[k] = sv[0];
        best_r[k] = si[0];
    }
}

hipError_t launch_batch_best(const double *E, int K, int R, double *best_E, int *best_r, hipStream_t st) {
    if (K < 1 || R < 1) return hipErrorInvalidValue;
    batch_best_k<<<K, 256, 0, st>>>(E, R, best_E, best_r);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchConfig &c, int nwg, const BatchArgs &a, hipStream_t st) {
    const size_t lds = batch_lds_bytes(c, a.nmax, a.dmax);
#define GD_CASE(id, t, nt, e)                                           \
    case id:                                                            \
        if (a.nmax > e * nt / t) return hipErrorInvalidValue;           \
        batch_ell_euler<t, nt, e><<<nwg, nt, lds, st>>>(a);             \
        return hipGetLastError();
    switch (c.id) { GD_BATCH_VARIANTS(GD_CASE) }
#undef GD_CASE
    return hipErrorInvalidValue;
}

}  // namespace gd
