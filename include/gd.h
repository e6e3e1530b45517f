/*
 * gd.h -- C ABI of libgd.so, a gfx950 (MI355X) implementation of the
 * gain-dissipative (GD) optimiser of Kalinin & Berloff, "Global optimization
 * of spin Hamiltonians with gain-dissipative systems" (arXiv:1807.00699).
 *
 * The library time-steps, for R independent trajectories ("restarts") of one
 * coupling matrix J, the rate equations
 *
 *   dPsi_i/dt   = Psi_i (gamma_i - gamma_c - |Psi_i|^2)
 *                 + (1/s) sum_{j != i} J_ij Psi_j  + h_1i
 *                 + h_q conj(Psi_i)^(q-1) + D xi_i(t)                Eq. (main)
 *   dgamma_i/dt = eps_i (rho_th - |Psi_i|^2)                         Eq. (gamma)
 *
 * (GD form: Delta_ij = 1, K_ij = J_ij) for real amplitudes (Ising, Sec. 3,
 * on the real subspace where the q = 2 penalty is a shift of gamma_c),
 * complex amplitudes without resonant term (XY, Sec. 2), or complex
 * amplitudes with one resonant term h_q (Ising through h_2, and the q-state
 * clock (planar Potts) model, Eq. (hs)), and scores the discretised states
 * with the Hamiltonian of Eq. (h):
 *
 *   H = - sum_{i != j} J_ij cos(theta_i - theta_j) + sum_i g_i cos(theta_i).
 *
 * Conventions shared by every call:
 *  - Every function returns GD_OK (0) or a negative gd_error code; no
 *    exception or abort crosses the ABI.  gd_last_error() returns a
 *    thread-local message for the last failure on the calling thread.
 *  - Pointers are host pointers unless GD_F_DEVICE_PTRS is set in the
 *    solver's params, in which case every array argument (inputs and outputs)
 *    is a device pointer on the solver's device.  The caller always keeps
 *    ownership of its arrays; the library copies what it needs.
 *  - Matrices are row-major.  Per-trajectory arrays are trajectory-major:
 *    element (r, i) of a [batch][n] array is at r*n + i; complex values are
 *    interleaved (re, im), i.e. [batch][n][2].
 *  - A handle is not thread-safe: calls on one handle must not overlap.
 *  - Work is enqueued on params.stream (a hipStream_t; NULL = a stream the
 *    library creates).  Calls synchronise that stream before returning unless
 *    GD_F_ASYNC is set (then only gd_run may return early).
 */
#ifndef GD_H_
#define GD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GD_ABI_VERSION 2

/* Error codes (all negative). */
typedef enum gd_error {
    GD_OK = 0,
    GD_E_INVALID_ARG = -1,   /* bad size, NULL pointer, unknown enum, bad struct_size */
    GD_E_NOT_SYMMETRIC = -2, /* J[i][j] != J[j][i] for some i != j (exact compare) */
    GD_E_NONFINITE = -3,     /* NaN/Inf in J, g, eps or an initial state */
    GD_E_OOM = -4,           /* device allocation failed; the handle stays valid */
    GD_E_DEVICE = -5,        /* HIP runtime error (message in gd_last_error) */
    GD_E_STATE = -6,         /* call out of order (e.g. energy before any state exists) */
    GD_E_DIVERGED = -7,      /* a trajectory became non-finite (see gd_stats.diverged) */
    GD_E_UNSUPPORTED = -8    /* valid request the library does not implement */
} gd_error;

/* Spin model.
 *  GD_ISING          real amplitudes; readout sign(x) (theta in {0, pi}).
 *  GD_XY             complex amplitudes, no resonant term; theta = arg Psi.
 *  GD_ISING_COMPLEX  complex amplitudes with the q = 2 term h_2 conj(Psi)
 *                    (Sec. 3); readout sign(Re Psi).
 *  GD_POTTS          complex amplitudes with the q-th term h_q conj(Psi)^(q-1)
 *                    (Eq. (hs)); readout k = floor(q theta / 2pi + 1/2) mod q
 *                    (theta = arg Psi in [0, 2pi), Psi = 0 -> theta = 0),
 *                    energy of Eq. (h) at theta_i = 2 pi k_i / q. */
typedef enum gd_model { GD_ISING = 0, GD_XY = 1, GD_ISING_COMPLEX = 2, GD_POTTS = 3 } gd_model;

/* Time integrator: explicit Euler, or the classical 4th-order Runge-Kutta
 * scheme on the joint state (Psi, gamma) (Sec. 2 uses RK4 for XY). */
typedef enum gd_integrator { GD_EULER = 0, GD_RK4 = 1 } gd_integrator;

/* Operand precision of the coupling product sum_j J_ij Psi_j.  Accumulation,
 * the amplitude/gain update and the energies are FP32 (energies are also
 * re-scored in FP64) in every mode. */
typedef enum gd_precision {
    GD_PREC_FP32 = 0,  /* J and Psi in FP32 (when every coupling is exact in FP8 E4M3 the
                          few-trajectory kernels stream a one-byte copy of J, widened exactly
                          and summed in the FP32 order: the same results bit for bit;
                          the environment variable GD_J8_COPY=0 turns the copy off) */
    GD_PREC_BF16 = 1,  /* Psi operand rounded to BF16; J in BF16 (FP8 storage when exact) */
    GD_PREC_FP16 = 2   /* Psi operand rounded to FP16; J in FP16 (FP8 storage when exact) */
} gd_precision;

/* Output format of gd_spins. */
typedef enum gd_spin_fmt {
    GD_SPINS_I8 = 0,         /* Ising models: int8 +-1, [batch][n] */
    GD_SPINS_ANGLE_F32 = 1,  /* float theta in [0, 2pi) of the discretised state, [batch][n]
                                (XY: arg Psi; Ising: 0 or pi; Potts: 2 pi k / q) */
    GD_SPINS_STATE_I32 = 2   /* Potts: int32 k in [0, q), [batch][n] */
} gd_spin_fmt;

/* Algorithm (Sec. 1).  GD: Delta_ij = 1, K_ij = J_ij.  GD-mod: Delta_ij =
 * gamma_i + gamma_j with per-trajectory couplings K_ij adapted by Eq. (gamma2),
 *   dK_ij/dt = eps_hat (J_ij - Delta_ij K_ij),  K_ij(0) = J_ij,
 * integrated with explicit Euler (FP32, n <= 4096, dense solvers only).  Every
 * trajectory holds an n x n K (R n^2 floats of device memory).  GD-mod needs
 * positive gains (Delta_ij <= 0 makes Eq. (gamma2) unstable): gamma_c at or
 * above max_i sum_j |J_ij| / s keeps every fixed-point gain >= rho_th. */
typedef enum gd_variant { GD_VARIANT_GD = 0, GD_VARIANT_MOD = 1 } gd_variant;

#define GD_F_DEVICE_PTRS 0x1u  /* array arguments are device pointers */
#define GD_F_ASYNC 0x2u        /* gd_run returns without synchronising the stream */
#define GD_F_PROFILE 0x4u      /* time the coupling launches of every 8th step with one HIP event
                                  pair per step (kernel_ms / kernel_launches = mean launch time);
                                  the fused small-problem kernel is timed per launch and counts
                                  its coupling evaluations (steps x stages, + 1 for an energy
                                  check that closes the launch) as launches; steps replayed from
                                  a captured graph (few-trajectory matrix-vector kernels) are
                                  timed per replay and count their launches; batch solvers time
                                  every persistent launch (a chunk of steps) and count it once */

/* Parameters of a solver.  Fill with gd_default_params(), then override.
 * struct_size must be sizeof(gd_params) of the caller's header. */
typedef struct gd_params {
    uint32_t struct_size;
    int32_t integrator;      /* gd_integrator */
    int32_t precision;       /* gd_precision */
    uint32_t flags;          /* GD_F_* */
    double dt;               /* time step (default 0.05) */
    double eps;              /* gain-adjustment rate epsilon of Eq. (gamma) (default 0.1) */
    double rho_th;           /* threshold density rho_th of Eq. (gamma) (default 1) */
    double gamma_c;          /* loss rate gamma_c of Eq. (main) (default 0) */
    double gamma0;           /* initial gain gamma_i(0) when none is given (default 0) */
    double j_scale;          /* coupling scale s; 0 selects s = sqrt(sum_{i!=j} J_ij^2 / n) */
    double init_amp;         /* amplitude of the default initial state (default 0.1) */
    uint64_t seed;           /* seed of the default initial state */
    int32_t check_interval;  /* steps between device energy checks inside gd_run (0 = none) */
    int32_t has_target;      /* nonzero: gd_run stops at the first check with min_r E_r <= target */
    double target_energy;    /* target of Eq. (h) energy for time-to-target */
    void *stream;            /* hipStream_t or NULL */
    /* noise D xi_i(t) of Eq. (main) (dense solvers; default D = 0).  Each step
     * first takes the deterministic Euler or RK4 step, then adds
     * D sqrt(dt) (eta_re + i eta_im) (real models: D sqrt(dt) eta_re) with
     * eta_re, eta_im independent N(0, 1) drawn by Box-Muller from
     * z = SplitMix64(k_t ^ SplitMix64(r 2^32 + i)), k_t = SplitMix64(noise_seed
     * ^ SplitMix64(t)), t = index of the step since gd_set_init / the step of
     * gd_set_state: u1 = ((z >> 40) + 1) 2^-24, u2 = ((z >> 16) mod 2^24) 2^-24,
     * eta = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).  With D = 0 the
     * dynamics are deterministic. */
    double noise_D;
    uint64_t noise_seed;
    int32_t q;               /* GD_POTTS: number of states, 2 <= q <= 8 */
    int32_t variant;         /* gd_variant: GD (default) or GD-mod */
    double h_q;              /* resonant strength of GD_ISING_COMPLEX and GD_POTTS.  For q = 2,
                                0 selects 1.1 max_i sum_{j != i} |J_ij| / s (the bound of
                                Sec. 1 for the penalty to pin the phases, with a 10% margin).
                                For q > 2 it must be given (> 0): the paper states no value,
                                and the term outgrows the cubic saturation for q > 4 (for
                                q = 4 when h_4 > 1), so large values make the dynamics
                                blow up. */
    double eps_hat;          /* GD-mod: rate eps_hat of Eq. (gamma2) (default 0.1) */
} gd_params;

/* Counters of a solver (cumulative over gd_run calls since the last
 * gd_set_init / gd_set_state). */
typedef struct gd_run_stats {
    uint32_t struct_size;
    int32_t batch;            /* R */
    int64_t steps_done;       /* integration steps of the current trajectories */
    int64_t spin_updates;     /* sum over gd_run calls of n * R * steps */
    double run_seconds;       /* host wall time inside gd_run (synchronous calls) */
    double kernel_ms;         /* summed device time of the sampled coupling launches (GD_F_PROFILE) */
    int64_t kernel_launches;  /* number of coupling launches timed in kernel_ms */
    int32_t diverged;         /* trajectories whose state became non-finite */
    int32_t target_reached;   /* 1 once a check met the target */
    double ttt_seconds;       /* device time (HIP events on the solver's stream) of the gd_run
                                 calls since gd_set_init / gd_set_state, counted from the start
                                 of each call, up to the event recorded after that check */
    int64_t ttt_steps;        /* steps done at that check */
    double best_energy;       /* lowest device-checked energy so far (+inf if none) */
    int32_t best_index;       /* its trajectory */
    int32_t kernel_config;    /* id of the coupling kernel variant in use: when a batch is
                                 set up (gd_set_init, gd_set_state, the first gd_run) the
                                 library times the variants that fit the problem, once per
                                 (model, precision, size, batch, integrator), and keeps the
                                 fastest; the environment variable GD_DENSE_CONFIG=<id>
                                 pins one instead (the set-up call then fails with
                                 GD_E_INVALID_ARG if that id does not fit).  Problems of
                                 at most 128 padded spins (FP32, no pinned variant) use a
                                 fused multi-step kernel instead of the variants.  Batches
                                 of instances: the same with GD_BATCH_CONFIG=<id>; the
                                 variants with per-instance item widths also relabel each
                                 instance's spins at set-up (host threads, deterministic,
                                 results unchanged bit for bit) so that their LDS gathers
                                 avoid bank conflicts; GD_BATCH_RELABEL=0 keeps the
                                 given order.  With
                                 GD_AUTOTUNE_CACHE=<file> the picks persist across
                                 processes: the file names the device and library build
                                 in its first line (a file of another device or build is
                                 ignored, and rewritten at the next pick), a set-up looks
                                 its problem up there first (the file is read again when
                                 it changed) and uses an id from it only when that id fits
                                 the problem */
} gd_run_stats;

typedef struct gd_solver gd_solver;

/* Defaults: Euler, FP32, dt 0.05, eps 0.1, rho_th 1, gamma_c 0, gamma0 0,
 * automatic coupling scale, init_amp 0.1, seed 0, no checks, NULL stream,
 * no noise, q = 2, automatic h_q. */
void gd_default_params(gd_params *p);

/*
 * gd_create: build a solver for one instance.
 *   n      number of spins (1 <= n <= 65536).
 *   J      n*n row-major couplings; must be finite and exactly symmetric; the
 *          diagonal is ignored (the sums of Eq. (main) and Eq. (hs) skip j = i).
 *   g      external field g_i of Eq. (h), length n, or NULL for g = 0.  It
 *          enters Eq. (main) as the q = 1 resonant term h_1i = -g_i sqrt(rho_th)/s,
 *          so that the dynamics minimise Eq. (h) as printed.
 *   model  gd_model.  p: parameters (copied), NULL = defaults.
 * Errors: GD_E_INVALID_ARG, GD_E_NOT_SYMMETRIC, GD_E_NONFINITE, GD_E_OOM,
 * GD_E_DEVICE, GD_E_UNSUPPORTED (reduced precision with J not exactly
 * representable in it).  GD_POTTS needs 2 <= params.q <= 8, and h_q > 0
 * when q > 2.  GD-mod needs Euler steps, FP32 and n <= 4096
 * (GD_E_UNSUPPORTED otherwise).  On error *out is set to NULL.
 */
int gd_create(gd_solver **out, int32_t n, const float *J, const float *g,
              int32_t model, const gd_params *p);

/* gd_destroy: free the handle and its device memory (NULL is a no-op). */
void gd_destroy(gd_solver *s);

/*
 * gd_set_init: set the initial state of `batch` trajectories and reset the
 * step counter and statistics.
 *   psi0   GD_ISING [batch][n], complex models [batch][n][2]; NULL = default
 *          initial state (GD_ISING U(-a, a); complex models a*exp(i*phi),
 *          phi ~ U[0, 2pi); a = init_amp (0 gives Psi(0) = 0, the start of
 *          Sec. 2), drawn from SplitMix64 keyed by seed, trajectory and spin).
 *   gamma0 [batch][n] initial gains, or NULL for params.gamma0.
 *   eps    [n] per-spin gain rates eps_i (the site-dependent rates suggested
 *          in Sec. 3), or NULL for params.eps.
 */
int gd_set_init(gd_solver *s, int32_t batch, const float *psi0, const float *gamma0,
                const float *eps);

/*
 * gd_run: integrate `steps` steps of all trajectories.  If no state exists
 * yet, the default initial state with `batch` trajectories is created first;
 * otherwise `batch` must equal the current batch and the trajectories
 * continue.  With check_interval > 0 the discretised energies are evaluated
 * on the device every check_interval steps; with has_target the run stops at
 * the first check where min_r E_r <= target_energy (gd_stats.ttt_*).  The
 * host waits for each check only with has_target or GD_F_ASYNC.  A target
 * recorded by gd_set_targets is compared one check later, while the next
 * steps run.  Times to target are device time (HIP events) in both cases;
 * with no target the best energy of the checks is kept on the device and
 * reaches gd_stats when the run ends.
 * Returns GD_E_DIVERGED if any trajectory is non-finite at the end.
 */
int gd_run(gd_solver *s, int32_t batch, int64_t steps);

/*
 * gd_energy: Eq. (h) energies of the discretised current state (Ising:
 * s_i = sign(x_i) with sign(+-0) = +1 (complex Ising: of Re Psi_i); XY:
 * theta_i = arg Psi_i, Psi_i = 0 -> theta_i = 0; Potts: the readout of
 * gd_model), evaluated on the device in FP64 from the FP32 state (exact for
 * integer-valued J and g; Potts: exact for q in {2, 3, 4, 6}).
 *   E     [batch] doubles.  best: argmin_r E_r (ties -> lowest r), nullable.
 */
int gd_energy(gd_solver *s, double *E, int32_t *best);

/*
 * gd_energy_device: the same energies as computed by the device check path
 * (FP32 coupling product, FP64 accumulation of the per-spin terms).  Exact,
 * and equal to gd_energy, for integer-valued J and g with n < 2^24.
 */
int gd_energy_device(gd_solver *s, double *E, int32_t *best);

/* gd_spins: discretised current state into caller memory, format gd_spin_fmt
 * (GD_SPINS_I8 needs GD_ISING or GD_ISING_COMPLEX; GD_SPINS_STATE_I32 needs
 * GD_POTTS). */
int gd_spins(gd_solver *s, void *out, int32_t fmt);

/*
 * gd_spins_noalloc: gd_spins for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same output as gd_spins, staged through a fixed device array
 * of 16 MiB (one per GPU, held until the process ends) instead of a buffer
 * allocated per call; it calls no hipMalloc, hipFree or allocating routine.
 * Single-instance solvers only (GD_E_UNSUPPORTED for batches).  Errors as
 * gd_spins, plus GD_E_INVALID_ARG when batch * n * (1 byte for GD_SPINS_I8,
 * 4 otherwise) exceeds 16 MiB.  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU (other threads, other streams) race.
 */
int gd_spins_noalloc(gd_solver *s, void *out, int32_t fmt);

/* gd_get_state / gd_set_state: amplitudes ([batch][n] or [batch][n][2]),
 * gains [batch][n] and step counter; NULL pointers are skipped on get.
 * gd_set_state needs both psi and gamma and keeps the per-spin eps. */
int gd_get_state(gd_solver *s, float *psi, float *gamma, int64_t *step);
int gd_set_state(gd_solver *s, int32_t batch, const float *psi, const float *gamma,
                 int64_t step);

/* gd_mod_couplings (GD-mod): the current coupling matrix K (n*n, row-major)
 * of trajectory `traj` into caller memory.  gd_set_init and gd_set_state
 * reset every K to J. */
int gd_mod_couplings(gd_solver *s, int32_t traj, float *K);

/* gd_stats: copy the counters (out->struct_size must be set). */
int gd_stats(gd_solver *s, gd_run_stats *out);

/* gd_trajectory_status: which trajectories diverged.  out[r] = 1 when the
 * amplitudes or gains of trajectory r became non-finite during a gd_run since
 * gd_set_init / gd_set_state (Eq. (main) and Eq. (gamma) carry a NaN or Inf
 * into every later step, so the state stays so), else 0; gd_stats.diverged is
 * the count of ones.  out: caller's host array of `count` int32, count = R
 * (batch solvers: instances x R, out[k * R + r] for trajectory r of instance
 * k).  GD_E_STATE without a state, GD_E_INVALID_ARG on a NULL pointer or a
 * count that differs. */
int gd_trajectory_status(gd_solver *s, int32_t *out, int64_t count);

/* gd_best_trace: the best-so-far energy (Eq. (h)) at each device check of
 * gd_run since gd_set_init / gd_set_state.  *count = number of checks
 * recorded (the first 65536 are kept); the first min(*count, cap) entries
 * are written: steps[k] = steps done at check k, best[k] = lowest device-
 * checked energy over checks 0..k (min_r E_r at each check, as for the
 * target of time-to-target).  steps and best: caller's host arrays of cap
 * entries (may be NULL when cap is 0, to query the count).  Dense solvers
 * only (batches of instances report per-instance results through gd_ttt:
 * GD_E_INVALID_ARG). */
int gd_best_trace(gd_solver *s, int64_t *steps, double *best, int32_t cap, int32_t *count);

/* gd_coupling_scale: the scale s in use (batch solvers: of instance 0). */
int gd_coupling_scale(gd_solver *s, double *scale);

/*
 * Batches of instances of uneven size (the paper's workloads run many
 * instances, Sec. 2 and 3).  One instance: n spins and either a dense
 * coupling matrix J (n*n, row-major) or CSR arrays (row_ptr [n+1], col/val
 * [nnz]; host memory), plus an optional field g [n].  The same validation
 * as gd_create applies per instance; every instance gets its own coupling
 * scale s_k.  The batched solver integrates the Ising model (real
 * amplitudes) with explicit Euler steps in FP32 and no noise; other
 * combinations return GD_E_UNSUPPORTED.  All instances share params and the trajectory count R.
 */
typedef struct gd_instance {
    int32_t n;
    const float *J;          /* dense couplings or NULL */
    const int32_t *row_ptr;  /* CSR, used when J is NULL */
    const int32_t *col;
    const float *val;
    const float *g;          /* external field or NULL */
} gd_instance;

/*
 * gd_create_batch: one handle for `count` instances.  The calls above then
 * work on the whole batch with concatenated layouts: per-trajectory arrays are
 * the instances' [R][n_k] blocks one after the other (sum_k R*n_k floats);
 * eps of gd_set_init is [sum_k n_k]; gd_energy writes E [count][R] and best
 * [count] (argmin per instance, ties -> lowest r); gd_spins writes int8
 * spins in the state layout.  gd_run makes one persistent launch per chunk
 * of steps (check_interval steps, or all), captured once in a hipGraph and
 * replayed.
 */
int gd_create_batch(gd_solver **out, int32_t count, const gd_instance *inst, int32_t model,
                    const gd_params *p);

/*
 * gd_set_targets: target energies of Eq. (h), [count] (one for a single-
 * instance solver), or NULL to clear.  With check_interval > 0, gd_run
 * records for each instance the wall time and step count of the first check
 * where its best energy is <= its target; with has_target it stops once every
 * instance has reached its target.  For a single-instance solver this sets
 * params.target_energy; gd_run then records the time-to-target and stops
 * there only if params.has_target was set at creation.
 */
int gd_set_targets(gd_solver *s, const double *targets);

/*
 * gd_ttt: per instance [count]: seconds to the check that met the target (-1
 * if not reached) on the clock of gd_run_stats.ttt_seconds (device time of
 * the gd_run calls since the last set-up, from the start of each call), the
 * step count at that check (-1), and the best checked energy so far (+inf).
 * Any pointer may be NULL.
 */
int gd_ttt(gd_solver *s, double *seconds, int64_t *steps, double *best_energy);

const char *gd_error_string(int code);
const char *gd_last_error(void);

/* ------------------------------------------------------------------------
 * Learned proposal.  The paper suggests site-dependent gain-adjustment rates
 * eps_i(t) as an extension (Sec. 3); the sub-threshold phase of the dynamics
 * amplifies the leading eigenvectors of J (Sec. 1).  A per-spin network reads
 * GD_NFEAT features of J and proposes a sign for each spin (biasing the
 * initial amplitudes) and a confidence (setting eps_i).  The random-start
 * solver stays the fallback and judges the energies.
 * ------------------------------------------------------------------------ */
#define GD_NFEAT 20
#define GD_MLP_NPARAM 5634

/*
 * gd_features (batch solvers): per spin, in the concatenated spin order,
 * GD_NFEAT floats: [0] sum_j J_ij/s, [1] degree / mean degree, [2..9]
 * sqrt(n) v_k[i], [10..17] n lambda_k v_k[i]^2, [18] sum_j |J_ij|/s, [19] 1,
 * where (lambda_k, v_k), k < 8, are the Ritz pairs of J/s after `iters`
 * steps of block power iteration on J/s + cI (c = max_i sum_j |J_ij|/s)
 * from a SplitMix64 start block, with Cholesky-QR each step, each v_k
 * sign-fixed so that its largest-magnitude entry is positive (ties: lowest
 * index).  lambda [count][8] and vecs [sum n][8] are optional (NULL).
 * Instances need n <= 2560.  Host output pointers.
 */
int gd_features(gd_solver *s, int32_t iters, float *feats, float *lambda, float *vecs);

/* Network GD_NFEAT -> 64 -> 64 -> 2 (ReLU), parameters (GD_MLP_NPARAM floats):
 * W1 [20][64], b1 [64], W2 [64][64], b2 [64], W3 [64][2], b3 [2].
 * Outputs per spin: o0 (sign logit, m = tanh o0) and o1 (confidence logit,
 * c = sigmoid o1). */
typedef struct gd_mlp gd_mlp;

/* params NULL: He-normal weights from SplitMix64 + Box-Muller keyed by seed,
 * zero biases.  flags: GD_F_DEVICE_PTRS makes X/labels/out/params of the
 * calls below device pointers (seg stays host memory). */
int gd_mlp_create(gd_mlp **out, const float *params, uint64_t seed, uint32_t flags);
void gd_mlp_destroy(gd_mlp *m);
/* replace the parameters (NULL keeps them) and reset the Adam moments */
int gd_mlp_set_params(gd_mlp *m, const float *params);
int gd_mlp_get_params(gd_mlp *m, float *params);

/* outputs [M][2] for features X [M][GD_NFEAT]; fp16 != 0 runs the FP16
 * inference kernel (parameters, features and activations rounded to half
 * precision, products summed in FP32 on the matrix cores).  With
 * GD_F_DEVICE_PTRS the FP16 kernel reads X in 16-byte words: X must be
 * 16-byte aligned (GD_E_INVALID_ARG otherwise). */
int gd_mlp_forward(gd_mlp *m, int32_t M, const float *X, float *out, int32_t fp16);

/*
 * gd_mlp_train_step: one FP32 step on M rows from K instances (rows
 * seg[k]..seg[k+1]-1 belong to instance k; seg host memory) with labels +-1,
 * a low-energy state of each instance.  Loss (per instance the label is
 * aligned to the prediction by the global flip sigma_k of Eq. (h)):
 *   L = (1/M) sum_i [(m_i - sigma_k s_i)^2 + 0.5 BCE(c_i, [m_i sigma_k s_i > 0])].
 * lr > 0 applies Adam (0.9, 0.999, 1e-8, bias-corrected); lr = 0 only
 * evaluates.  loss and grad [GD_MLP_NPARAM] (host, nullable) receive the
 * loss and the gradient at the parameters before the update.  Computed on
 * the FP32 matrix cores (FP32 products and sums; the gradient summed over
 * rows in a fixed order, so repeated calls give the same bits).
 */
int gd_mlp_train_step(gd_mlp *m, int32_t M, const float *X, const float *labels, int32_t K,
                      const int32_t *seg, float lr, double *loss, float *grad);

/*
 * gd_propose (batch solvers): features (feat_iters iterations) -> FP16
 * network -> initial state of R trajectories per instance:
 *   psi0_ir = init_amp (alpha m_i + (1 - alpha) (2u - 1)),
 *   u = SplitMix64 uniform of counter ((k 2^20 + r) 2^16 + i) and `seed`,
 *   gamma_ir(0) = params.gamma0, eps_i = params.eps exp(beta (c_i - 1/2));
 * then behaves as gd_set_init.
 */
int gd_propose(gd_solver *s, gd_mlp *m, int32_t R, int32_t feat_iters, double alpha, double beta,
               uint64_t seed);

#ifdef __cplusplus
}
#endif

#endif /* GD_H_ */
