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
// The arithmetic is fixed (fused multiply-adds over d in list order, then
// batch_euler_update with contraction off), so a trajectory's result does not
// depend on the variant, T, NT or the rest of the batch.
// After the last step the Eq. (h) energy of the discretised state
// (s_i = sign x_i) is reduced per trajectory in FP64 in a fixed order.
#include "gd_internal.h"

#include <type_traits>

namespace gd {

namespace {

// Coupling term d of a spin from its packed words (word 0: idx0 | idx1 << 16;
// word 1: idx2 | sign2 << 29 | sign1 << 30 | sign0 << 31; a missing coupling
// points at the all-zero row n of its instance): the neighbour's amplitude with the
// coupling's sign applied.  mag * (+-x) equals the ELL product (+-mag) * x
// bit for bit, so fma(+-x, mag, c) reproduces the list's sum.
template <int D, int T>
__device__ inline float signed_nb(const unsigned char *xlb, const uint2 w, int rb) {
    constexpr int SH = T == 1 ? 2 : (T == 2 ? 3 : (T == 4 ? 4 : (T == 8 ? 5 : 6)));   // log2(4 T)
    const unsigned int idx = D == 0 ? (w.x & 0xFFFFu) : (D == 1 ? (w.x >> 16) : (w.y & 0xFFFFu));
    const float v = *reinterpret_cast<const float *>(xlb + (idx << SH) + rb);
    const unsigned int sgn = (w.y << D) & 0x80000000u;      // bit 31 - D
    return __uint_as_float(__float_as_uint(v) ^ sgn);
}

// One explicit Euler step of Eq. (main) and Eq. (gamma) for a real amplitude
// x with gain g and coupling sum c: the operations and their rounding are
// written out (no contraction beyond the written fmas), so every batch kernel
// variant produces the same bits whatever its instruction schedule.
__device__ inline void batch_euler_update(float &x, float &g, float c, float inv_s, float h1, float eps,
                                          float gc, float rho_th, float dt) {
#pragma clang fp contract(off)
    const float rho = x * x;
    const float f = __builtin_fmaf(x, (g - gc) - rho, __builtin_fmaf(c, inv_s, h1));
    const float gn = __builtin_fmaf(dt, eps * (rho_th - rho), g);
    x = __builtin_fmaf(dt, f, x);
    g = gn;
}

// PK: the neighbours of the thread's spins live in registers (two words per
// slot, read once per item from the packed form) instead of LDS, so a
// coupling term costs one LDS read (the neighbour's amplitude) and a few
// integer operations instead of three LDS reads; the products and their
// order are those of the ELL list (three terms; padding reads the zero row).
// UNI: every spin has the rate eps0 and no field term (h_1 = -0, the value
// a zero field maps to), so the slots carry no per-spin constants.
// DB (with PK): the amplitudes are double-buffered in LDS, step t reads one
// copy and writes the other, so a step needs one barrier instead of two.
template <int T, int NT, int E, bool PK, bool UNI, bool DB>
__global__ void __launch_bounds__(NT)
batch_ell_euler(BatchArgs a) {
    static_assert(!DB || PK, "double buffering is a variant of the packed form");
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x;
    const int r = tid % T;
    const int ibase = tid / T;
    constexpr int ISTR = NT / T;
    const int dmax = a.dmax;
    float *xl = reinterpret_cast<float *>(smem);                               // [nmax][T]
    float *wl = xl + (size_t)a.nmax * T;                                        // [nmax][dmax] (not PK)
    unsigned short *il = reinterpret_cast<unsigned short *>(wl + (size_t)a.nmax * dmax);
    double *red = reinterpret_cast<double *>(smem);                             // reuse after the run
    const uint2 *pk = reinterpret_cast<const uint2 *>(a.ell_pack);

    for (int it = a.wg_off[blockIdx.x]; it < a.wg_off[blockIdx.x + 1]; ++it) {
        const int item = a.items[it];
        const int k = item / a.nslices;
        const int rr = (item % a.nslices) * T + r;      // trajectory within the instance
        const int n = a.inst_n[k];
        const long long spin0 = a.inst_spin[k];
        const long long st0 = a.inst_state[k] + (long long)rr * n;   // [R][n] block of instance k
        const float inv_s = a.inst_inv_s[k];
        const float mag = PK ? a.inst_wmag[k] : 0.0f;
        // couplings of instance k into LDS (PK: only the zero row n_max, which
        // the reduction of the previous item may have overwritten)
        if constexpr (!PK) {
            for (int q = tid; q < n * dmax; q += NT) {
                wl[q] = a.ell_w[spin0 * dmax + q];
                il[q] = (unsigned short)a.ell_idx[spin0 * dmax + q];
            }
        } else {
            for (int q = tid; q < T; q += NT) xl[(size_t)n * T + q] = 0.0f;
            if constexpr (DB)
                for (int q = tid; q < T; q += NT) xl[(size_t)(a.nmax + 1 + n) * T + q] = 0.0f;
        }
        // DB: buffer b at xl + b (n_max + 1) T; step t reads buffer t % 2
        float *xl1 = xl + (size_t)(a.nmax + 1) * T;
        const unsigned char *xlb = reinterpret_cast<const unsigned char *>(xl);
        const int rb = r * 4;
        float xo[E], go[E], ep[UNI ? 1 : E], hh[UNI ? 1 : E];
        uint2 nb[PK ? E : 1];
        if constexpr (UNI) {
            ep[0] = a.eps0;
            hh[0] = -0.0f;
        }
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int i = ibase + s * ISTR;
            xo[s] = go[s] = 0.0f;
            if constexpr (!UNI) ep[s] = hh[s] = 0.0f;
            if constexpr (PK) nb[s] = uint2{0u, 0u};
            if (i < n) {
                xo[s] = a.x[st0 + i];
                go[s] = a.gam[st0 + i];
                if constexpr (!UNI) {
                    ep[s] = a.eps[spin0 + i];
                    hh[s] = a.h1[spin0 + i];
                }
                if constexpr (PK) nb[s] = pk[spin0 + i];
                xl[i * T + r] = xo[s];
            }
        }
        __syncthreads();
        const float dt = a.dt, gc = a.gamma_c, rho_th = a.rho_th;
        for (int step = 0; step < a.steps; ++step) {
            const unsigned char *src = DB && (step & 1) ? reinterpret_cast<const unsigned char *>(xl1) : xlb;
            float *dst = DB && !(step & 1) ? xl1 : xl;
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int i = ibase + s * ISTR;
                if (i < n) {
                    float c = 0.0f;
                    if constexpr (PK) {
                        c = __builtin_fmaf(signed_nb<0, T>(src, nb[s], rb), mag, c);
                        c = __builtin_fmaf(signed_nb<1, T>(src, nb[s], rb), mag, c);
                        c = __builtin_fmaf(signed_nb<2, T>(src, nb[s], rb), mag, c);
                    } else {
                        for (int d = 0; d < dmax; ++d)
                            c = __builtin_fmaf(wl[i * dmax + d], xl[il[i * dmax + d] * T + r], c);
                    }
                    batch_euler_update(xo[s], go[s], c, inv_s, hh[UNI ? 0 : s], ep[UNI ? 0 : s], gc, rho_th, dt);
                    if constexpr (DB) dst[i * T + r] = xo[s];
                }
            }
            __syncthreads();
            if constexpr (!DB) {
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    const int i = ibase + s * ISTR;
                    if (i < n) xl[i * T + r] = xo[s];
                }
                __syncthreads();
            }
        }
        // the buffer that holds the final amplitudes (DB: written by the last step)
        const float *xf = DB && (a.steps & 1) ? xl1 : xl;
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
                if constexpr (PK) {
                    // sign(x_j) times the coupling's sign, times mag; the zero row reads +0 (sign +1)
                    // with weight 0, so padding is skipped by its index
                    const uint2 w = nb[s];
                    const unsigned int idx[3] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu};
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        if ((int)idx[d] == n) continue;
                        const float xj = xf[idx[d] * T + r];
                        const double sg = ((w.y << d) & 0x80000000u) ? -1.0 : 1.0;
                        h += (double)mag * sg * (xj < 0.0f ? -1.0 : 1.0);
                    }
                } else {
                    for (int d = 0; d < dmax; ++d) {
                        const float xj = xf[il[i * dmax + d] * T + r];
                        h += (double)wl[i * dmax + d] * (xj < 0.0f ? -1.0 : 1.0);
                    }
                }
                e += -si * h + (double)a.g[spin0 + i] * si;
            }
        }
        // per trajectory: lanes of one trajectory (tid % T) within a wave by a
        // butterfly over the lane bits above T, then the waves in order
        // (a fixed order: the result does not depend on timing)
#pragma unroll
        for (int m = 32; m >= T; m >>= 1) e += __shfl_xor(e, m);
        __syncthreads();                       // all reads of xl / wl are done
        if ((tid & 63) < T) red[(tid >> 6) * T + (tid & 63)] = e;
        __syncthreads();
        if (tid < T) {
            double tot = 0.0;
            for (int w = 0; w < NT / 64; ++w) tot += red[w * T + tid];
            a.E[(long long)k * a.R + (item % a.nslices) * T + tid] = tot;
        }
        if (bad) a.flags[(long long)k * a.R + rr] = 1;
        __syncthreads();                       // LDS is reused by the next item
    }
}

// Per-instance trajectory width (packed form, double-buffered amplitudes):
// instance k runs in items of T_k = 2^tlog_k trajectories, T_k chosen by the
// host so that T_k (n_k + 1) <= E NT + 64 -- small instances get wide items,
// large ones narrow items, every item holds about E NT spin-trajectories.
// The amplitudes of an item sit in LDS as [i][T_k], so one wave instruction
// of the neighbour gathers reads 64 / T_k rows of T_k consecutive words (T_k
// >= 32: whole bank sweeps), and every thread updates E slots per barrier.
// The item's state is staged through LDS at its start and end so that the
// global reads and writes run along the [R][n] rows.  Thread t owns the
// trajectory r = t mod T_k and the spins t / T_k + s NT / T_k; the products,
// their order and the update are those of batch_ell_euler, so a trajectory's
// result does not depend on the variant.
// The spins of an instance are relabeled by the host (label = LDS row and
// position of the slot that updates the spin) so that the d-th neighbours of
// the G = 64 / T_k spins one gather instruction serves fall on different
// banks as far as possible; the state is staged through the labels, the
// per-spin constants are read at the spin's own index.
// The step loop is written for the vector ALU, which bounds it: each slot
// keeps the byte offsets of its three neighbour amplitudes and of its own
// amplitude in buffer 0, and the three couplings as signed magnitudes
// (+-mag times x is bit for bit the product of mag and +-x, so no sign flip
// per term); buffer 1 sits at the fixed offset (E NT + 64) words, and the
// steps run in pairs so that the buffer a step reads or writes is a constant
// offset folded into the LDS instruction.
template <int NT, int E, bool UNI>
__global__ void __launch_bounds__(NT)
batch_ell_tw(BatchArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr unsigned B1 = (unsigned)(E * NT + 64) * 4u;             // byte offset of buffer 1
    static_assert(B1 < 65536, "the offset of buffer 1 fits the LDS instruction's immediate");
    const int tid = threadIdx.x;
    float *xl0 = reinterpret_cast<float *>(smem);
    float *xl1 = reinterpret_cast<float *>(smem + B1);
    double *red = reinterpret_cast<double *>(smem);                   // reuse after the run
    const uint2 *pk = reinterpret_cast<const uint2 *>(a.tw_pack);    // in label order

    for (int it = a.wg_off[blockIdx.x]; it < a.wg_off[blockIdx.x + 1]; ++it) {
        const int item = a.items[it];
        const int k = item / a.R, r0 = item % a.R;
        const int tlog = a.inst_tlog[k];
        const int T = 1 << tlog;
        const int r = tid & (T - 1);
        const int ibase = tid >> tlog;
        const int ISTR = NT >> tlog;
        const int n = a.inst_n[k];
        const long long spin0 = a.inst_spin[k];
        const long long blk = a.inst_state[k] + (long long)r0 * n;      // rows r0 .. r0 + T - 1 of [R][n]
        const float inv_s = a.inst_inv_s[k];
        const float mag = a.inst_wmag[k];
        // stage the item's amplitudes (buffer 0) and gains (buffer 1) as
        // [label][T] from coalesced reads of the [T][n] block
        const int *lab = a.tw_label + spin0;
        const int *spn = a.tw_spin + spin0;
        for (int q = tid; q < T * n; q += NT) {
            const int rr = q / n, i = q - rr * n;
            const int p = lab[i];
            xl0[p * T + rr] = a.x[blk + q];
            xl1[p * T + rr] = a.gam[blk + q];
        }
        __syncthreads();
        float xo[E], go[E], ep[UNI ? 1 : E], hh[UNI ? 1 : E];
        const float *na[E][3];           // in buffer 0: the neighbours' amplitudes (row n if missing)
        float *wa[E];                    // and the own amplitude
        float sm[E][3];                  // couplings as signed magnitudes
        if constexpr (UNI) {
            ep[0] = a.eps0;
            hh[0] = -0.0f;
        }
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int i = ibase + s * ISTR;
            xo[s] = go[s] = 0.0f;
            if constexpr (!UNI) ep[s] = hh[s] = 0.0f;
            wa[s] = xl0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                na[s][d] = xl0;
                sm[s][d] = 0.0f;
            }
            if (i < n) {                      // i: the label of the slot's spin
                xo[s] = xl0[i * T + r];
                go[s] = xl1[i * T + r];
                if constexpr (!UNI) {
                    ep[s] = a.eps[spin0 + spn[i]];
                    hh[s] = a.h1[spin0 + spn[i]];
                }
                const uint2 w = pk[spin0 + i];
                const unsigned idx[3] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    na[s][d] = xl0 + ((int)idx[d] << tlog) + r;
                    sm[s][d] = __uint_as_float(__float_as_uint(mag) ^ ((w.y << d) & 0x80000000u));
                }
                wa[s] = xl0 + (i << tlog) + r;
            }
        }
        __syncthreads();                      // gains read before buffer 1 holds amplitudes
        for (int q = tid; q < T; q += NT) {
            xl0[n * T + q] = 0.0f;
            xl1[n * T + q] = 0.0f;
        }
        __syncthreads();
        const float dt = a.dt, gc = a.gamma_c, rho_th = a.rho_th;
        // one step reading the buffer at byte offset RD, writing the other
        auto step = [&](auto rd) {
            constexpr int RD = decltype(rd)::value / 4;           // in words
            constexpr int WR = RD ? 0 : (int)B1 / 4;
#pragma unroll
            for (int s = 0; s < E; ++s) {
                if (ibase + s * ISTR < n) {
                    const float v0 = na[s][0][RD];
                    const float v1 = na[s][1][RD];
                    const float v2 = na[s][2][RD];
                    float c = __builtin_fmaf(v0, sm[s][0], 0.0f);
                    c = __builtin_fmaf(v1, sm[s][1], c);
                    c = __builtin_fmaf(v2, sm[s][2], c);
                    batch_euler_update(xo[s], go[s], c, inv_s, hh[UNI ? 0 : s], ep[UNI ? 0 : s], gc, rho_th, dt);
                    wa[s][WR] = xo[s];
                }
            }
            __syncthreads();
        };
        int t = 0;
        for (; t + 1 < a.steps; t += 2) {
            step(std::integral_constant<unsigned, 0u>{});
            step(std::integral_constant<unsigned, B1>{});
        }
        if (t < a.steps) step(std::integral_constant<unsigned, 0u>{});
        // final amplitudes in buffer steps % 2 (the last step's target); the
        // other buffer stages the gains for the write-back
        const float *xf = (a.steps & 1) ? xl1 : xl0;
        float *gs = (a.steps & 1) ? xl0 : xl1;
        bool bad = false;
        double e = 0.0;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int i = ibase + s * ISTR;
            if (i < n) {
                gs[i * T + r] = go[s];
                bad |= !(__builtin_isfinite(xo[s]) && __builtin_isfinite(go[s]));
                // Eq. (h) of the discretised state: -s_i sum_d w_id s_j + g_i s_i
                const double si = xo[s] < 0.0f ? -1.0 : 1.0;
                double h = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int j = (int)(na[s][d] - xl0) >> tlog;
                    if (j == n) continue;                                     // missing coupling
                    const float xj = xf[(j << tlog) + r];
                    const double sg = (__float_as_uint(sm[s][d]) & 0x80000000u) ? -1.0 : 1.0;
                    h += (double)mag * sg * (xj < 0.0f ? -1.0 : 1.0);
                }
                e += -si * h + (double)a.g[spin0 + spn[i]] * si;
            }
        }
        __syncthreads();
        for (int q = tid; q < T * n; q += NT) {
            const int rr = q / n, i = q - rr * n;
            const int p = lab[i];
            a.x[blk + q] = xf[p * T + rr];
            a.gam[blk + q] = gs[p * T + rr];
        }
        // per trajectory: lanes of one trajectory within a wave by a butterfly
        // over the lane bits from T up, then the waves in order
        for (int m = 32; m >= T; m >>= 1) e += __shfl_xor(e, m);
        __syncthreads();                       // all reads of the LDS buffers are done
        const int tw = T < 64 ? T : 64;
        if ((tid & 63) < tw) red[(tid >> 6) * tw + (tid & 63)] = e;
        __syncthreads();
        if (tid < T) {
            // T <= 64: waves w hold lanes r of the trajectory tid
            double tot = 0.0;
            for (int w = 0; w < NT / 64; ++w) tot += red[w * tw + tid];
            a.E[(long long)k * a.R + r0 + tid] = tot;
        }
        if (bad) a.flags[(long long)k * a.R + r0 + r] = 1;
        __syncthreads();                       // LDS is reused by the next item
    }
}

// Variants {T, NT, E, PK, UNI, DB}: T trajectories per item, NT threads, E
// slots per thread (n_max <= E * NT / T), PK neighbours in registers (packed
// form; two more registers per slot), UNI uniform eps and no field (two
// fewer), DB amplitudes double-buffered in LDS (one barrier per step); the
// slot count keeps each variant within the register budget of its
// workgroup size.
#define GD_BATCH_VARIANTS(X)                 \
    X(0, 8, 1024, 16, false, false, false)   \
    X(1, 4, 512, 16, false, false, false)    \
    X(2, 2, 256, 16, false, false, false)    \
    X(3, 8, 512, 32, false, false, false)    \
    X(4, 16, 1024, 16, false, false, false)  \
    X(5, 4, 1024, 8, false, false, false)    \
    X(6, 1, 256, 16, false, false, false)    \
    X(7, 4, 512, 16, true, false, false)     \
    X(8, 4, 1024, 8, true, false, false)     \
    X(9, 2, 512, 8, true, false, false)      \
    X(10, 2, 256, 16, true, false, false)    \
    X(11, 4, 1024, 8, true, true, false)     \
    X(12, 4, 1024, 8, true, true, true)      \
    X(13, 4, 1024, 8, true, false, true)     \
    X(14, 2, 512, 8, true, false, true)

// Variants of batch_ell_tw {NT, E, UNI} (ids after the fixed-width ones):
// E NT spin-trajectories per item.
#define GD_BATCH_TW_VARIANTS(X) \
    X(15, 1024, 8, true)        \
    X(16, 1024, 8, false)       \
    X(17, 1024, 4, true)        \
    X(18, 512, 8, true)         \
    X(19, 512, 6, true)         \
    X(20, 256, 8, true)

constexpr int kBatchCfg[][6] = {
#define GD_ROW(id, t, nt, e, pk, uni, db) {t, nt, e, pk, uni, db},
    GD_BATCH_VARIANTS(GD_ROW)
#undef GD_ROW
#define GD_ROW(id, nt, e, uni) {0, nt, e, 1, uni, 1},
    GD_BATCH_TW_VARIANTS(GD_ROW)
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
    c.packed = kBatchCfg[idx][3] != 0;
    c.uniform = kBatchCfg[idx][4] != 0;
    c.dbuf = kBatchCfg[idx][5] != 0;
    return c;
}

int batch_item_capacity(const BatchConfig &c) { return c.slots * c.threads; }

size_t batch_lds_bytes(const BatchConfig &c, int nmax, int dmax) {
    if (c.traj == 0) {
        // two amplitude buffers of (n_k + 1) T_k <= E NT + 64 words; the
        // per-trajectory energy partials of the waves reuse them
        const size_t b = (size_t)(batch_item_capacity(c) + 64) * 4 * 2;
        const size_t red = (size_t)(c.threads / 64) * 64 * 8;
        return b > red ? b : red;
    }
    size_t b = (size_t)(nmax + 1) * c.traj * 4 * (c.dbuf ? 2 : 1);   // + the zero row(s) of the packed form
    if (!c.packed) b += (size_t)nmax * dmax * 4 + (size_t)nmax * dmax * 2;
    b = (b + 15) / 16 * 16;
    const size_t red = (size_t)c.threads * 8;
    return b > red ? b : red;
}

hipError_t prepare_batch(const BatchConfig &c, int nmax, int dmax) {
    const int lds = int(batch_lds_bytes(c, nmax, dmax));
#define GD_CASE(id, t, nt, e, pk, uni, db)                                                                   \
    case id:                                                                                                 \
        return hipFuncSetAttribute(reinterpret_cast<const void *>(&batch_ell_euler<t, nt, e, pk, uni, db>), \
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    switch (c.id) { GD_BATCH_VARIANTS(GD_CASE) }
#undef GD_CASE
#define GD_CASE(id, nt, e, uni)                                                                              \
    case id:                                                                                                 \
        return hipFuncSetAttribute(reinterpret_cast<const void *>(&batch_ell_tw<nt, e, uni>),                \
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    switch (c.id) { GD_BATCH_TW_VARIANTS(GD_CASE) }
#undef GD_CASE
    return hipErrorInvalidValue;
}

int batch_occupancy(const BatchConfig &c, int nmax, int dmax) {
    const size_t lds = batch_lds_bytes(c, nmax, dmax);
    int occ = 0;
    hipError_t e = hipErrorInvalidValue;
#define GD_CASE(id, t, nt, e_, pk, uni, db)                                                               \
    case id:                                                                                              \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_ell_euler<t, nt, e_, pk, uni, db>, nt, lds); \
        break;
    switch (c.id) { GD_BATCH_VARIANTS(GD_CASE) }
#undef GD_CASE
#define GD_CASE(id, nt, e_, uni)                                                                          \
    case id:                                                                                              \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_ell_tw<nt, e_, uni>, nt, lds);       \
        break;
    switch (c.id) { GD_BATCH_TW_VARIANTS(GD_CASE) }
#undef GD_CASE
    return e == hipSuccess && occ > 0 ? occ : 1;
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
#define GD_CASE(id, t, nt, e, pk, uni, db)                              \
    case id:                                                            \
        if (a.nmax > e * nt / t) return hipErrorInvalidValue;           \
        if (pk && (!a.ell_pack || !a.inst_wmag || a.dmax > 3 || a.nmax > 65535)) return hipErrorInvalidValue; \
        batch_ell_euler<t, nt, e, pk, uni, db><<<nwg, nt, lds, st>>>(a); \
        return hipGetLastError();
    switch (c.id) { GD_BATCH_VARIANTS(GD_CASE) }
#undef GD_CASE
    // per-instance widths: the host checked T_k (n_k + 1) <= E NT + 64 and
    // T_k <= 64 for every instance when it built the schedule
#define GD_CASE(id, nt, e, uni)                                                                              \
    case id:                                                                                                 \
        if (!a.tw_pack || !a.tw_label || !a.tw_spin || !a.inst_wmag || !a.inst_tlog || a.dmax > 3 ||          \
            a.nmax > 65535)                                                                                  \
            return hipErrorInvalidValue;                                                                     \
        batch_ell_tw<nt, e, uni><<<nwg, nt, lds, st>>>(a);                                                   \
        return hipGetLastError();
    switch (c.id) { GD_BATCH_TW_VARIANTS(GD_CASE) }
#undef GD_CASE
    return hipErrorInvalidValue;
}

}  // namespace gd
