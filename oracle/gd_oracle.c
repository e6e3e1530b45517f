/*
 * gd_oracle.c -- plain FP64 CPU oracle of the gain-dissipative (GD) method
 * of Kalinin & Berloff, "Global optimization of spin Hamiltonians with
 * gain-dissipative systems" (arXiv:1807.00699).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker for the HIP library,
 * not part of it: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header or constant with
 * the HIP library.
 *
 * Everything is written for clarity, not speed: explicit loops, float64,
 * trajectories independent (an OpenMP loop over trajectories is the only
 * parallelism; it does not change any result).
 *
 * What it computes (paper notation):
 *   Eq. (main), GD form (Delta_ij = 1, K_ij = J_ij, Sec. 1):
 *     dPsi_i/dt = Psi_i (gamma_i - gamma_c - |Psi_i|^2)
 *                 + sum_{j != i} J_ij Psi_j / s
 *                 + sum_{q=1}^{nq} h_qi conj(Psi_i)^(q-1) + D xi_i(t)
 *   Eq. (gamma): dgamma_i/dt = eps_i (rho_th - |Psi_i|^2)
 *   s is a coupling scale (s = 1 is the equation as printed).
 *   Integrators: explicit Euler, and the classical 4th-order Runge-Kutta
 *   scheme (Sec. 2) applied to the joint state (Psi, gamma).
 *   Noise (D > 0): white noise xi_i with independent real and imaginary
 *   parts of unit intensity; after each deterministic step the increment
 *   D sqrt(dt) (eta_re + i eta_im) is added (real mode: D sqrt(dt) eta_re),
 *   which for the Euler scheme is the Euler-Maruyama method.  eta_re, eta_im
 *   are standard normals made by the Box-Muller transform from a
 *   counter-based SplitMix64 stream (see orc_gauss_pair).
 *   Real-amplitude mode integrates the same equations for real Psi.
 *   Readout and energies follow Eq. (h); the diagonal of J is excluded as in
 *   Eq. (main) and Eq. (hs).
 *   GD-mod (Delta_ij = gamma_i + gamma_j, couplings adapted by Eq. (gamma2)):
 *   orc_run_mod, explicit Euler.
 *   Brute-force ground states: Ising by Gray-code enumeration, q-state clock
 *   (planar Potts) model by odometer enumeration.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_NONFINITE -3
#define ORC_E_OOM -4

enum { ORC_EULER = 0, ORC_RK4 = 1 };

/* ------------------------------------------------------------------ */
/* Right-hand side of Eq. (main) and Eq. (gamma), real amplitudes.      */
/* psi, gam: one trajectory's state (length n).  fpsi, fgam: d/dt.      */
/* h1: h_1i (length n) or NULL.  Only q = 1 fields exist on the real    */
/* subspace used here; an h_2 term is a shift of gamma_c (Sec. 3).      */
/* ------------------------------------------------------------------ */
static void rhs_real(int n, const double *J, double s, const double *h1,
                     const double *eps, double rho_th, double gamma_c,
                     const double *psi, const double *gam,
                     double *fpsi, double *fgam)
{
    for (int i = 0; i < n; ++i) {
        double c = 0.0;                       /* sum_{j != i} J_ij psi_j */
        for (int j = 0; j < n; ++j)
            if (j != i) c += J[(size_t)i * n + j] * psi[j];
        double rho = psi[i] * psi[i];
        fpsi[i] = psi[i] * (gam[i] - gamma_c - rho) + c / s + (h1 ? h1[i] : 0.0);
        fgam[i] = eps[i] * (rho_th - rho);
    }
}

/* Complex amplitudes with resonant terms h_qi conj(Psi_i)^(q-1), q=1..nq. */
static void rhs_complex(int n, const double *J, double s, int nq, const double *h,
                        const double *eps, double rho_th, double gamma_c,
                        const double complex *psi, const double *gam,
                        double complex *fpsi, double *fgam)
{
    for (int i = 0; i < n; ++i) {
        double complex c = 0.0;
        for (int j = 0; j < n; ++j)
            if (j != i) c += J[(size_t)i * n + j] * psi[j];
        double rho = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
        double complex f = psi[i] * (gam[i] - gamma_c - rho) + c / s;
        double complex pw = 1.0;            /* conj(psi)^(q-1) */
        for (int q = 1; q <= nq; ++q) {
            f += h[(size_t)(q - 1) * n + i] * pw;
            pw *= conj(psi[i]);
        }
        fpsi[i] = f;
        fgam[i] = eps[i] * (rho_th - rho);
    }
}

/* One Euler or RK4 step of one real trajectory (y = (psi, gamma)). */
static void step_real(int n, const double *J, double s, const double *h1,
                      const double *eps, double rho_th, double gamma_c,
                      double dt, int integrator, double *psi, double *gam,
                      double *w /* workspace 12n */)
{
    double *k1p = w, *k1g = w + n, *k2p = w + 2 * n, *k2g = w + 3 * n;
    double *k3p = w + 4 * n, *k3g = w + 5 * n, *k4p = w + 6 * n, *k4g = w + 7 * n;
    double *yp = w + 8 * n, *yg = w + 9 * n;
    if (integrator == ORC_EULER) {
        rhs_real(n, J, s, h1, eps, rho_th, gamma_c, psi, gam, k1p, k1g);
        for (int i = 0; i < n; ++i) {
            psi[i] += dt * k1p[i];
            gam[i] += dt * k1g[i];
        }
        return;
    }
    rhs_real(n, J, s, h1, eps, rho_th, gamma_c, psi, gam, k1p, k1g);
    for (int i = 0; i < n; ++i) { yp[i] = psi[i] + 0.5 * dt * k1p[i]; yg[i] = gam[i] + 0.5 * dt * k1g[i]; }
    rhs_real(n, J, s, h1, eps, rho_th, gamma_c, yp, yg, k2p, k2g);
    for (int i = 0; i < n; ++i) { yp[i] = psi[i] + 0.5 * dt * k2p[i]; yg[i] = gam[i] + 0.5 * dt * k2g[i]; }
    rhs_real(n, J, s, h1, eps, rho_th, gamma_c, yp, yg, k3p, k3g);
    for (int i = 0; i < n; ++i) { yp[i] = psi[i] + dt * k3p[i]; yg[i] = gam[i] + dt * k3g[i]; }
    rhs_real(n, J, s, h1, eps, rho_th, gamma_c, yp, yg, k4p, k4g);
    for (int i = 0; i < n; ++i) {
        psi[i] += dt / 6.0 * (k1p[i] + 2.0 * k2p[i] + 2.0 * k3p[i] + k4p[i]);
        gam[i] += dt / 6.0 * (k1g[i] + 2.0 * k2g[i] + 2.0 * k3g[i] + k4g[i]);
    }
}

static void step_complex(int n, const double *J, double s, int nq, const double *h,
                         const double *eps, double rho_th, double gamma_c,
                         double dt, int integrator, double complex *psi, double *gam,
                         double complex *wc /* 5n */, double *wg /* 5n */)
{
    double complex *k1p = wc, *k2p = wc + n, *k3p = wc + 2 * n, *k4p = wc + 3 * n, *yp = wc + 4 * n;
    double *k1g = wg, *k2g = wg + n, *k3g = wg + 2 * n, *k4g = wg + 3 * n, *yg = wg + 4 * n;
    rhs_complex(n, J, s, nq, h, eps, rho_th, gamma_c, psi, gam, k1p, k1g);
    if (integrator == ORC_EULER) {
        for (int i = 0; i < n; ++i) { psi[i] += dt * k1p[i]; gam[i] += dt * k1g[i]; }
        return;
    }
    for (int i = 0; i < n; ++i) { yp[i] = psi[i] + 0.5 * dt * k1p[i]; yg[i] = gam[i] + 0.5 * dt * k1g[i]; }
    rhs_complex(n, J, s, nq, h, eps, rho_th, gamma_c, yp, yg, k2p, k2g);
    for (int i = 0; i < n; ++i) { yp[i] = psi[i] + 0.5 * dt * k2p[i]; yg[i] = gam[i] + 0.5 * dt * k2g[i]; }
    rhs_complex(n, J, s, nq, h, eps, rho_th, gamma_c, yp, yg, k3p, k3g);
    for (int i = 0; i < n; ++i) { yp[i] = psi[i] + dt * k3p[i]; yg[i] = gam[i] + dt * k3g[i]; }
    rhs_complex(n, J, s, nq, h, eps, rho_th, gamma_c, yp, yg, k4p, k4g);
    for (int i = 0; i < n; ++i) {
        psi[i] += dt / 6.0 * (k1p[i] + 2.0 * k2p[i] + 2.0 * k3p[i] + k4p[i]);
        gam[i] += dt / 6.0 * (k1g[i] + 2.0 * k2g[i] + 2.0 * k3g[i] + k4g[i]);
    }
}

/* ------------------------------------------------------------------ */
/* Noise numbers                                                         */
/* ------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea, Flood 2014): the output for generator state x
 * (the state first advances by the odd constant 0x9E3779B97F4A7C15, then a
 * xor-shift-multiply finaliser mixes it). */
uint64_t orc_splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/*
 * Two independent standard normals for step t, trajectory r, spin i:
 *   key = SplitMix64(seed ^ SplitMix64(t)),
 *   z   = SplitMix64(key ^ SplitMix64(r * 2^32 + i)),
 *   u1  = (bits 40..63 of z, plus 1) / 2^24   in (0, 1],
 *   u2  = (bits 16..39 of z) / 2^24           in [0, 1),
 *   (g0, g1) = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2)   (Box-Muller).
 */
void orc_gauss_pair(uint64_t seed, int64_t t, int64_t r, int64_t i, double *g0, double *g1)
{
    const uint64_t key = orc_splitmix64(seed ^ orc_splitmix64((uint64_t)t));
    const uint64_t z = orc_splitmix64(key ^ orc_splitmix64(((uint64_t)r << 32) | (uint64_t)i));
    const double u1 = ((double)(z >> 40) + 1.0) / 16777216.0;
    const double u2 = (double)((z >> 16) & 0xFFFFFFull) / 16777216.0;
    const double rad = sqrt(-2.0 * log(u1));
    *g0 = rad * cos(2.0 * M_PI * u2);
    *g1 = rad * sin(2.0 * M_PI * u2);
}

/* The pairs of orc_gauss_pair for step t, trajectories r0..r0+R-1 and spins
 * 0..n-1, written to out [R][n][2]. */
void orc_gauss_block(uint64_t seed, int64_t t, int64_t r0, int R, int n, double *out)
{
    for (int r = 0; r < R; ++r)
        for (int i = 0; i < n; ++i)
            orc_gauss_pair(seed, t, r0 + r, i, &out[((size_t)r * n + i) * 2],
                           &out[((size_t)r * n + i) * 2 + 1]);
}

static int finite_vec(const double *v, size_t m)
{
    for (size_t k = 0; k < m; ++k)
        if (!isfinite(v[k])) return 0;
    return 1;
}

/*
 * orc_run_real: integrate R independent real-amplitude trajectories for
 * `steps` steps.  psi, gamma: [R][n] in/out.  h1: [n] or NULL.  eps: [n].
 * Noise: amplitude D (0: none), seed, index t0 of the first step and index
 * r0 of the first trajectory (the noise numbers depend on the global step
 * and trajectory indices, so any sub-range is an exact sub-problem).
 * Returns ORC_E_NONFINITE if any trajectory's state became non-finite.
 */
int orc_run_real(int n, const double *J, double s, const double *h1,
                 const double *eps, double rho_th, double gamma_c, double dt,
                 int integrator, int R, double *psi, double *gamma,
                 long steps, int nthreads, double D, uint64_t seed, int64_t t0, int64_t r0)
{
    if (n <= 0 || R < 0 || steps < 0 || !(s > 0.0) || !J || !eps || !psi || !gamma) return ORC_E_ARG;
    int bad = 0;
    (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) reduction(| : bad)
    for (int r = 0; r < R; ++r) {
        double *w = malloc(sizeof(double) * 12 * (size_t)n);
        if (!w) { bad |= 2; continue; }
        double *p = psi + (size_t)r * n, *g = gamma + (size_t)r * n;
        for (long t = 0; t < steps; ++t) {
            step_real(n, J, s, h1, eps, rho_th, gamma_c, dt, integrator, p, g, w);
            if (D != 0.0)
                for (int i = 0; i < n; ++i) {
                    double g0, g1;
                    orc_gauss_pair(seed, t0 + t, r0 + r, i, &g0, &g1);
                    p[i] += D * sqrt(dt) * g0;
                }
        }
        if (!finite_vec(p, n) || !finite_vec(g, n)) bad |= 1;
        free(w);
    }
    if (bad & 2) return ORC_E_OOM;
    return bad ? ORC_E_NONFINITE : ORC_OK;
}

/*
 * orc_run_complex: as orc_run_real for complex amplitudes.
 * psi: [R][n][2] (re, im) in/out; gamma [R][n]; h: [nq][n] (h_qi) or NULL.
 */
int orc_run_complex(int n, const double *J, double s, int nq, const double *h,
                    const double *eps, double rho_th, double gamma_c, double dt,
                    int integrator, int R, double *psi, double *gamma,
                    long steps, int nthreads, double D, uint64_t seed, int64_t t0, int64_t r0)
{
    if (n <= 0 || R < 0 || steps < 0 || !(s > 0.0) || !J || !eps || !psi || !gamma) return ORC_E_ARG;
    if (nq < 0 || (nq > 0 && !h)) return ORC_E_ARG;
    int bad = 0;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) reduction(| : bad)
    for (int r = 0; r < R; ++r) {
        double complex *z = malloc(sizeof(double complex) * 6 * (size_t)n);
        double *wg = malloc(sizeof(double) * 5 * (size_t)n);
        if (!z || !wg) { free(z); free(wg); bad |= 2; continue; }
        double *pr = psi + (size_t)r * n * 2, *g = gamma + (size_t)r * n;
        double complex *p = z + 5 * (size_t)n;
        for (int i = 0; i < n; ++i) p[i] = pr[2 * i] + I * pr[2 * i + 1];
        for (long t = 0; t < steps; ++t) {
            step_complex(n, J, s, nq, h, eps, rho_th, gamma_c, dt, integrator, p, g, z, wg);
            if (D != 0.0)
                for (int i = 0; i < n; ++i) {
                    double g0, g1;
                    orc_gauss_pair(seed, t0 + t, r0 + r, i, &g0, &g1);
                    p[i] += D * sqrt(dt) * (g0 + I * g1);
                }
        }
        for (int i = 0; i < n; ++i) { pr[2 * i] = creal(p[i]); pr[2 * i + 1] = cimag(p[i]); }
        if (!finite_vec(pr, 2 * (size_t)n) || !finite_vec(g, n)) bad |= 1;
        free(z);
        free(wg);
    }
    if (bad & 2) return ORC_E_OOM;
    return bad ? ORC_E_NONFINITE : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* GD-mod: Delta_ij = gamma_i + gamma_j with adapted couplings K_ij      */
/* ------------------------------------------------------------------ */

/*
 * orc_run_mod: the GD-mod algorithm (Sec. 1): Eq. (main) with
 * Delta_ij = gamma_i + gamma_j and per-trajectory couplings K_ij that follow
 * Eq. (gamma2), dK_ij/dt = eps_hat (J_ij - Delta_ij K_ij), together with
 * Eq. (gamma); explicit Euler, every right-hand side at the old state:
 *   c_i     = sum_{j != i} (gamma_i + gamma_j) K_ij Psi_j / s
 *   Psi_i  += dt [Psi_i (gamma_i - gamma_c - |Psi_i|^2) + c_i + h1_i]
 *   gamma_i += dt eps_i (rho_th - |Psi_i|^2)
 *   K_ij   += dt eps_hat (J_ij - (gamma_i + gamma_j) K_ij)
 * then the noise increment (as in orc_run_real / orc_run_complex).
 * cplx: 0 real amplitudes psi [R][n], 1 complex psi [R][n][2].
 * K: [R][n][n] in/out (the caller sets K(0)).
 */
int orc_run_mod(int n, int cplx, const double *J, double s, const double *h1,
                const double *eps, double rho_th, double gamma_c, double eps_hat, double dt,
                int R, double *psi, double *gamma, double *K, long steps, int nthreads,
                double D, uint64_t seed, int64_t t0, int64_t r0)
{
    if (n <= 0 || R < 0 || steps < 0 || !(s > 0.0) || !J || !eps || !psi || !gamma || !K)
        return ORC_E_ARG;
    const int P = cplx ? 2 : 1;
    int bad = 0;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) reduction(| : bad)
    for (int r = 0; r < R; ++r) {
        double *x = psi + (size_t)r * n * P, *g = gamma + (size_t)r * n;
        double *Kr = K + (size_t)r * n * n;
        double *nx = malloc(sizeof(double) * (size_t)n * P);
        double *ng = malloc(sizeof(double) * (size_t)n);
        if (!nx || !ng) { free(nx); free(ng); bad |= 2; continue; }
        for (long t = 0; t < steps; ++t) {
            for (int i = 0; i < n; ++i) {
                double cr = 0.0, ci = 0.0;
                for (int j = 0; j < n; ++j) {
                    if (j == i) continue;
                    const double w = (g[i] + g[j]) * Kr[(size_t)i * n + j];
                    cr += w * x[(size_t)j * P];
                    if (cplx) ci += w * x[(size_t)j * P + 1];
                }
                const double xr = x[(size_t)i * P], xi = cplx ? x[(size_t)i * P + 1] : 0.0;
                const double rho = xr * xr + xi * xi;
                const double lin = g[i] - gamma_c - rho;
                nx[(size_t)i * P] = xr + dt * (xr * lin + cr / s + (h1 ? h1[i] : 0.0));
                if (cplx) nx[(size_t)i * P + 1] = xi + dt * (xi * lin + ci / s);
                ng[i] = g[i] + dt * eps[i] * (rho_th - rho);
            }
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    if (j == i) continue;
                    double *k = &Kr[(size_t)i * n + j];
                    *k += dt * eps_hat * (J[(size_t)i * n + j] - (g[i] + g[j]) * *k);
                }
            for (int i = 0; i < n; ++i) {
                x[(size_t)i * P] = nx[(size_t)i * P];
                if (cplx) x[(size_t)i * P + 1] = nx[(size_t)i * P + 1];
                g[i] = ng[i];
            }
            if (D != 0.0)
                for (int i = 0; i < n; ++i) {
                    double g0, g1;
                    orc_gauss_pair(seed, t0 + t, r0 + r, i, &g0, &g1);
                    x[(size_t)i * P] += D * sqrt(dt) * g0;
                    if (cplx) x[(size_t)i * P + 1] += D * sqrt(dt) * g1;
                }
        }
        if (!finite_vec(x, (size_t)n * P) || !finite_vec(g, n)) bad |= 1;
        free(nx);
        free(ng);
    }
    if (bad & 2) return ORC_E_OOM;
    return bad ? ORC_E_NONFINITE : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Readout (Eq. (h) spin domains)                                       */
/* ------------------------------------------------------------------ */

/* Ising: s = -1 if x < 0 else +1 (both zeros give +1).  NaN -> error. */
int orc_ising_spins(long m, const double *x, int8_t *spin)
{
    for (long k = 0; k < m; ++k) {
        if (isnan(x[k])) return ORC_E_NONFINITE;
        spin[k] = (x[k] < 0.0) ? -1 : 1;
    }
    return ORC_OK;
}

/* XY: theta = arg(psi) mapped to [0, 2pi); psi == 0 gives theta = 0. */
int orc_xy_phases(long m, const double *psi /* [m][2] */, double *theta)
{
    const double two_pi = 2.0 * M_PI;
    for (long k = 0; k < m; ++k) {
        double re = psi[2 * k], im = psi[2 * k + 1];
        if (isnan(re) || isnan(im)) return ORC_E_NONFINITE;
        if (re == 0.0 && im == 0.0) { theta[k] = 0.0; continue; }
        double t = atan2(im, re);
        if (t < 0.0) t += two_pi;
        if (t >= two_pi) t -= two_pi;
        theta[k] = t;
    }
    return ORC_OK;
}

/* q-state clock: k = round(q theta / 2pi) mod q, halves rounded up. */
int orc_potts_states(long m, const double *psi, int q, int32_t *state)
{
    if (q < 2) return ORC_E_ARG;
    const double two_pi = 2.0 * M_PI;
    for (long k = 0; k < m; ++k) {
        double re = psi[2 * k], im = psi[2 * k + 1];
        if (isnan(re) || isnan(im)) return ORC_E_NONFINITE;
        double t = (re == 0.0 && im == 0.0) ? 0.0 : atan2(im, re);
        if (t < 0.0) t += two_pi;
        long c = (long)floor(q * t / two_pi + 0.5);
        state[k] = (int32_t)(((c % q) + q) % q);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Energies, Eq. (h) with the diagonal excluded                          */
/*   E = - sum_{i != j} J_ij cos(theta_i - theta_j) + sum_i g_i cos theta_i */
/* ------------------------------------------------------------------ */

/* Ising, integer J and g: exact int64.  spin: [R][n]. */
int orc_energy_ising_i64(int n, const int64_t *J, const int64_t *g, int R,
                         const int8_t *spin, int64_t *E)
{
    for (int r = 0; r < R; ++r) {
        const int8_t *s = spin + (size_t)r * n;
        int64_t e = 0;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j)
                if (j != i) e -= J[(size_t)i * n + j] * s[i] * s[j];
            if (g) e += g[i] * s[i];
        }
        E[r] = e;
    }
    return ORC_OK;
}

/* Ising, real J and g: float64. */
int orc_energy_ising(int n, const double *J, const double *g, int R,
                     const int8_t *spin, double *E)
{
    for (int r = 0; r < R; ++r) {
        const int8_t *s = spin + (size_t)r * n;
        double e = 0.0;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j)
                if (j != i) e -= J[(size_t)i * n + j] * s[i] * s[j];
            if (g) e += g[i] * s[i];
        }
        E[r] = e;
    }
    return ORC_OK;
}

/* XY: float64 with cos of the phase differences. theta: [R][n]. */
int orc_energy_xy(int n, const double *J, const double *g, int R,
                  const double *theta, double *E)
{
    for (int r = 0; r < R; ++r) {
        const double *t = theta + (size_t)r * n;
        double e = 0.0;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j)
                if (j != i) e -= J[(size_t)i * n + j] * cos(t[i] - t[j]);
            if (g) e += g[i] * cos(t[i]);
        }
        E[r] = e;
    }
    return ORC_OK;
}

/* cos(2 pi m / q), exact for the q whose values are binary fractions. */
static double clock_cos(int m, int q)
{
    m = ((m % q) + q) % q;
    if (m == 0) return 1.0;
    if (q == 2) return -1.0;
    if (q == 3) return -0.5;
    if (q == 4) return (m == 2) ? -1.0 : 0.0;
    if (q == 6) {
        static const double c6[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
        return c6[m];
    }
    return cos(2.0 * M_PI * m / q);
}

/* q-state clock model: theta_i = 2 pi k_i / q.  state: [R][n]. */
int orc_energy_potts(int n, const double *J, const double *g, int q, int R,
                     const int32_t *state, double *E)
{
    if (q < 2) return ORC_E_ARG;
    for (int r = 0; r < R; ++r) {
        const int32_t *k = state + (size_t)r * n;
        double e = 0.0;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j)
                if (j != i) e -= J[(size_t)i * n + j] * clock_cos(k[i] - k[j], q);
            if (g) e += g[i] * clock_cos(k[i], q);
        }
        E[r] = e;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Brute force                                                           */
/* ------------------------------------------------------------------ */

/*
 * Ising ground state by Gray-code enumeration with incremental energy
 * updates.  Flipping spin k changes E by
 *     4 s_k sum_{j != k} J_kj s_j - 2 g_k s_k
 * (both ordered pairs (k,j), (j,k) of Eq. (h) change).  When g == NULL the
 * Z2 symmetry fixes the last spin to +1 and 2^(n-1) states are visited.
 * Returns the minimum energy and the first minimiser in enumeration order.
 */
int orc_brute_ising(int n, const double *J, const double *g, double *Emin, int8_t *smin)
{
    if (n <= 0 || n > 30) return ORC_E_ARG;
    int free_bits = g ? n : n - 1;
    int8_t s[32];
    for (int i = 0; i < n; ++i) s[i] = 1;
    double e = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j)
            if (j != i) e -= J[(size_t)i * n + j];
        if (g) e += g[i];
    }
    double best = e;
    memcpy(smin, s, (size_t)n);
    uint64_t total = 1ull << free_bits;
    for (uint64_t t = 1; t < total; ++t) {
        int k = __builtin_ctzll(t);            /* bit that changes in the Gray code */
        double h = 0.0;
        for (int j = 0; j < n; ++j)
            if (j != k) h += J[(size_t)k * n + j] * s[j];
        e += 4.0 * s[k] * h - (g ? 2.0 * g[k] * s[k] : 0.0);
        s[k] = (int8_t)-s[k];
        if (e < best) { best = e; memcpy(smin, s, (size_t)n); }
    }
    *Emin = best;
    return ORC_OK;
}

/* Same enumeration in exact int64 arithmetic for integer J, g. */
int orc_brute_ising_i64(int n, const int64_t *J, const int64_t *g, int64_t *Emin, int8_t *smin)
{
    if (n <= 0 || n > 40) return ORC_E_ARG;
    int free_bits = g ? n : n - 1;
    int8_t s[64];
    for (int i = 0; i < n; ++i) s[i] = 1;
    int64_t e = 0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j)
            if (j != i) e -= J[(size_t)i * n + j];
        if (g) e += g[i];
    }
    int64_t best = e;
    memcpy(smin, s, (size_t)n);
    uint64_t total = 1ull << free_bits;
    for (uint64_t t = 1; t < total; ++t) {
        int k = __builtin_ctzll(t);
        int64_t h = 0;
        for (int j = 0; j < n; ++j)
            if (j != k) h += J[(size_t)k * n + j] * s[j];
        e += 4 * s[k] * h - (g ? 2 * g[k] * s[k] : 0);
        s[k] = (int8_t)-s[k];
        if (e < best) { best = e; memcpy(smin, s, (size_t)n); }
    }
    *Emin = best;
    return ORC_OK;
}

/*
 * q-state clock model ground state by odometer enumeration of all q^n
 * states (state of spin 0 fixed to 0 when g == NULL: the energy is
 * invariant under a global rotation k -> k + c).  Changing spin k from a to b
 * changes E by
 *   -2 sum_{j != k} J_kj [cos(2pi(b-k_j)/q) - cos(2pi(a-k_j)/q)]
 *   + g_k [cos(2pi b/q) - cos(2pi a/q)].
 */
int orc_brute_potts(int n, const double *J, const double *g, int q, double *Emin, int32_t *kmin)
{
    if (n <= 0 || n > 24 || q < 2) return ORC_E_ARG;
    double states = pow((double)q, (double)n);
    if (states > 5e7) return ORC_E_ARG;
    int32_t k[32];
    for (int i = 0; i < n; ++i) k[i] = 0;
    double e = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j)
            if (j != i) e -= J[(size_t)i * n + j];
        if (g) e += g[i];
    }
    double best = e;
    memcpy(kmin, k, sizeof(int32_t) * (size_t)n);
    int first = g ? 0 : 1;                 /* digits that vary */
    for (;;) {
        int d = first;
        /* odometer increment, applying each digit change as a single-spin move */
        while (d < n) {
            int a = k[d], b = (a + 1) % q;
            double dh = 0.0;
            for (int j = 0; j < n; ++j)
                if (j != d) dh += J[(size_t)d * n + j] * (clock_cos(b - k[j], q) - clock_cos(a - k[j], q));
            e += -2.0 * dh + (g ? g[d] * (clock_cos(b, q) - clock_cos(a, q)) : 0.0);
            k[d] = b;
            if (b != 0) break;                 /* no carry */
            ++d;
        }
        if (d >= n) break;                     /* wrapped around: all visited */
        if (e < best) { best = e; memcpy(kmin, k, sizeof(int32_t) * (size_t)n); }
    }
    *Emin = best;
    return ORC_OK;
}
