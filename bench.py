"""Throughput and time-to-target benchmark of the gain-dissipative solver on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload ising4096|xy1024|...]

A step is one integration step (one RK4 step = four coupling launches) of
all R trajectories; the timed steps end on a device energy check
(discretise, energy product, best-of-R), every min(check, K) steps.

Default workload (the dense Ising instance of Sec. 3 at N = 4096): density-0.5
{-1, 0, +1} couplings, R = 4096 random restarts, Euler dt = 0.05, inputs
resident in HBM.  One JSON line:
  * value: spin-updates/s (N * R * steps / s) of the plain FP32 form over K
    timed steps, and the same for the BF16-operand / FP8-stored-J form under
    "legs", each with the roofline position of its coupling kernel (device time
    per launch from one HIP event pair around the coupling launches of every
    8th step of the timed run, on the solver's stream);
  * ttt: time to a target energy (best-known + 0.1%) for both forms, 8 starts
    each over a 10 000-step budget independent of K, checks every 100 steps
    (best-so-far energy of every check kept); best-known = the lowest energy of
    every run made here (longer reference runs and the timed runs); success
    fraction, median (censored runs count as beyond the budget) and TTS99 (time
    to solution with 99% confidence from independent starts);
  * cpu_baseline: the FP64 oracle timed on the host over a bounded sample of
    the same workload, on all cores and on one thread, with the CPU model;
    this leg also scores the returned spins with the oracle's Eq. (h) energies
    (energy error of each form against the oracle).
Other workloads (--workload) print the single-form line of that workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


WORKLOADS = {
    # name: (model, n, R, integrator, dt, steps, generator)
    "xy1024": dict(model="xy", n=1024, R=1024, integrator="rk4", dt=0.02, steps=5000,
                   J="dense_gaussian", desc="XY, N=1024, J~N(0,1/N), R=1024, RK4 dt=0.02, FP32"),
    "ising64": dict(model="ising", n=64, R=100, integrator="euler", dt=0.05, steps=2000,
                    J="dense_pm1", desc="Ising, N=64, J iid {-1,+1}, R=100, Euler dt=0.05, FP32"),
    "ising4096_fp32": dict(model="ising", n=4096, R=4096, integrator="euler", dt=0.05, steps=500,
                           J="sparse_pm1", desc="Ising, N=4096, J in {-1,0,1} density 0.5, "
                                                "R=4096, Euler dt=0.05, FP32 operands"),
    "ising4096_bf16": dict(model="ising", n=4096, R=4096, integrator="euler", dt=0.05, steps=10000,
                           J="sparse_pm1", precision="bf16",
                           desc="Ising, N=4096, J in {-1,0,1} density 0.5 stored FP8, R=4096, "
                                "Euler dt=0.05, BF16 operand, FP32 accumulation/state"),
    "batch256": dict(model="ising", n=None, R=64, integrator="euler", dt=0.05, steps=5000,
                     J="regular3_maxcut", batch=256,
                     desc="256 Ising instances, N_k even uniform in [50,2000], random 3-regular "
                          "max-cut couplings (J=-1 on edges, gauged by a random s*), R=64, "
                          "Euler dt=0.05, FP32, one persistent launch per chunk (hipGraph)"),
    "gemv4096": dict(model="ising", n=4096, R=1, integrator="euler", dt=0.05, steps=20000,
                     J="sparse_pm1", desc="Ising, N=4096, J in {-1,0,1} density 0.5, one trajectory "
                                          "(R=1), Euler dt=0.05, FP32 arithmetic, J streamed per step "
                                          "(stored FP8: the couplings are exact there)"),
    "gemv4096_fp8": dict(model="ising", n=4096, R=1, integrator="euler", dt=0.05, steps=20000,
                         J="sparse_pm1", precision="bf16",
                         desc="Ising, N=4096, J in {-1,0,1} density 0.5 stored FP8, one trajectory "
                              "(R=1), Euler dt=0.05, BF16 operand, FP32 sums and state"),
    "gemv4096_f32j": dict(model="ising", n=4096, R=1, integrator="euler", dt=0.05, steps=20000,
                          J="dense_gaussian", desc="Ising, N=4096, J ~ N(0, 1/N) (not exact in FP8), one "
                                                   "trajectory (R=1), Euler dt=0.05, FP32 J (64 MiB) "
                                                   "streamed per step"),
    "gemv16384": dict(model="ising", n=16384, R=1, integrator="euler", dt=0.05, steps=2000,
                      J="sparse_pm1", desc="Ising, N=16384, J in {-1,0,1} density 0.5, one trajectory "
                                           "(R=1), Euler dt=0.05, FP32 arithmetic, J streamed per step "
                                           "(stored FP8: 256 MiB)"),
    "gdmod1024": dict(model="xy", n=1024, R=256, integrator="euler", dt=0.02, steps=2000,
                      J="dense_gaussian", gdmod=True,
                      desc="GD-mod (Delta_ij = gamma_i + gamma_j, couplings adapted by Eq. (gamma2)), "
                           "XY, N=1024, J~N(0,1/N), R=256, Euler dt=0.02, eps_hat=0.2, FP32"),
}
PEAKS_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}
PEAK_HBM_GBS = 8000.0
PEAK_VALU_F32 = 78.6    # FP32 vector FMA without packed math (256 CUs, 2.4 GHz)


KERNEL_SOURCES = {"dense_step_f32": ("gd_dense.hip", "gd_epilogue.h"),
                  "dense_step_lp": ("gd_dense_lp.h", "gd_epilogue.h"),
                  "gemv_step_k": ("gd_gemv.h", "gd_epilogue.h")}


def fp8_exact(J):
    """True when every coupling is exactly an OCP FP8 E4M3 value: the library
    then stores J in one byte per coupling for the kernels that stream J
    every step (the small-R kernels; at reduced precision all kernels)."""
    m = np.arange(8, dtype=np.float64)
    vals = np.concatenate([m / 8 * 2.0**-6] + [(1 + m / 8) * 2.0**(e - 7) for e in range(1, 16)])[:-1]
    vals = np.concatenate([vals, -vals])
    Jo = np.asarray(J, np.float64).copy()
    np.fill_diagonal(Jo, 0.0)
    return bool(np.isin(Jo, vals).all())


def kernel_traffic(config_id, kern="dense_step_f32", workload="xy1024"):
    """HBM bytes per launch of a coupling kernel from its committed counter
    summary (profiles/<kernel>_<workload>_counters.txt: one
    traffic_bytes_per_launch for kernel_config_id, or one
    traffic_bytes_per_launch_cfg<id> per variant measured), or None when there
    is none, the kernel sources changed since the counters were taken or the
    running variant was not measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kern}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    csrc = os.path.join(ROOT, "paper_1807_00699_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in KERNEL_SOURCES[kern])
    if hashlib.sha256(src).hexdigest()[:16] != kv.get("kernel_source_sha256_16"):
        return None
    if f"traffic_bytes_per_launch_cfg{int(config_id)}" in kv:
        return float(kv[f"traffic_bytes_per_launch_cfg{int(config_id)}"])
    if int(kv.get("kernel_config_id", -1)) != int(config_id):
        return None
    return float(kv["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="ising4096", choices=sorted(WORKLOADS) + ["ising4096"])
    ap.add_argument("--check", type=int, default=50,
                    help="steps between device energy checks (the timed steps end on one)")
    ap.add_argument("--ttt-seeds", type=int, default=8, help="starts per form in the time-to-target runs")
    ap.add_argument("--ttt-budget", type=int, default=10000, help="step budget of a time-to-target run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-target reference run")
    ap.add_argument("--compare-ttt", action="store_true",
                    help="time-to-target comparisons: FP32 vs BF16 (N=4096) and random vs learned start")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB (reference for HBM counters)")
    ap.add_argument("--scaling", action="store_true",
                    help="steps and time to a stationary state vs N (XY, U[-10,10], paper regime)")
    ap.add_argument("--gdmod-scaling", action="store_true",
                    help="steps to a stationary state vs N, GD vs GD-mod (XY, U[-10,10], Euler)")
    ap.add_argument("--learned", action="store_true",
                    help="throughput of the learned proposal's training and inference kernels")
    ap.add_argument("--maxcut800", action="store_true",
                    help="N=800 G(n,0.06) max-cut stand-ins: cut quality and time, 100 runs each")
    return ap.parse_args()


def copy_calibration():
    """A plain 256 MiB device-to-device copy, 5 times: the bytes it must move
    are known (256 MiB read + 256 MiB written per launch), so the FETCH_SIZE /
    WRITE_SIZE counters it produces calibrate those of the solver kernels."""
    import torch
    n = 64 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 4 * n, "launches": 5}), flush=True)


def cpu_baseline(wl, J, psi0, target_s):
    """Oracle (FP64, OpenMP over trajectories) on a bounded sample: a subset
    of trajectories for a few steps, scaled to spin-updates/s."""
    from oracle import oracle as O
    threads = min(16, os.cpu_count() or 1)
    integ = O.RK4 if wl["integrator"] == "rk4" else O.EULER
    n = wl["n"]
    # small instances: all trajectories (the sample is then the workload itself,
    # run for as many steps as fill the time budget)
    R_s = wl["R"] if n * wl["R"] <= 65536 else min(wl["R"], threads * 2)
    steps = 20
    # pilot, then size the sample to ~target_s
    t0 = time.perf_counter()
    O.run(J, psi0[:R_s], model=wl["model"], steps=steps, dt=wl["dt"], eps=0.1,
          integrator=integ, nthreads=threads)
    pilot = time.perf_counter() - t0
    steps = max(1, int(target_s * steps / max(pilot, 1e-6)))
    cap = 100 * wl["steps"]
    steps = min(steps, cap)
    for _ in range(3):          # the pilot includes start-up costs: re-size once or twice
        t0 = time.perf_counter()
        O.run(J, psi0[:R_s], model=wl["model"], steps=steps, dt=wl["dt"], eps=0.1,
              integrator=integ, nthreads=threads)
        el = time.perf_counter() - t0
        if el >= 0.5 * target_s or steps >= cap:
            break
        steps = min(cap, int(steps * target_s / max(el, 1e-6)))
    return {"value": n * R_s * steps / el, "unit": "spin-updates/s", "cores": min(threads, R_s),
            "kind": "oracle",
            "sample": f"{R_s} of {wl['R']} trajectories x {steps} steps, {el:.1f} s"}


def batch_instances(K, seed=1):
    from paper_1807_00699_amd import inputs as I
    return I.maxcut_batch(K, 50, 2000, seed)


# algorithmic FP32 flops of one spin-update of the sparse Euler step:
# 2 per neighbour (multiply-add) + 12 for the pointwise update of Eq. (main, gamma)
SPARSE_FLOPS_PER_UPDATE = lambda d: 2 * d + 12
PEAK_FP32_VALU_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_LDS_GBS = 78643.2         # 256 CU x 128 B per clock x 2.4 GHz


def bench_batch(args, wl, steps):
    import torch

    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I

    K, R = wl["batch"], wl["R"]
    sizes, insts = batch_instances(K)
    x0 = np.concatenate([I.psi0_real(int(n), R, 5000 + k).ravel() for k, n in enumerate(sizes)])
    torch.cuda.init()
    B = gd.BatchSolver(insts, dt=wl["dt"], eps=0.1, check_interval=args.check, flags=gd.GD_F_PROFILE)
    B.set_init(R, x0)
    if args.warmup:
        B.run(args.warmup)
    torch.cuda.synchronize()
    st0 = B.stats()
    t0 = time.perf_counter()
    B.run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = B.stats()
    # device time of the timed persistent launches (HIP events around each)
    kern_s = (st.kernel_ms - st0.kernel_ms) / 1e3
    E, best = B.energy()
    B.close()
    total = int(np.sum(sizes))
    upd = total * R * steps
    flops = upd * SPARSE_FLOPS_PER_UPDATE(3)
    # roofline of the kernel: the LDS traffic of a spin-update (three neighbour
    # amplitudes read, its own written: 16 B) against the LDS bandwidth of the
    # chip (128 B per clock per CU, 256 CUs, 2.4 GHz = 78.6 TB/s)
    lds_bytes = 16.0 * upd
    out = {
        "metric": "spin-updates/s (N*R*steps/s)", "value": upd / el, "unit": "spin-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": el / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "instances": K, "sum_n": total, "R": R,
                   "energy_check_every": args.check, "kernel_config": st.kernel_config},
        "roofline": {"bound": "lds", "achieved": lds_bytes / kern_s / 1e9, "peak": PEAK_LDS_GBS,
                     "unit": "GB/s", "frac": lds_bytes / kern_s / 1e9 / PEAK_LDS_GBS,
                     "traffic": None, "kernel": "batch_ell_tw" if st.kernel_config >= 15 else "batch_ell_euler",
                     "launches": int(st.kernel_launches - st0.kernel_launches),
                     "kernel_seconds": kern_s, "lds_bytes_per_update": 16,
                     "alu_tflops": flops / kern_s / 1e12, "alu_peak_tflops": PEAK_FP32_VALU_TFLOPS},
        "best_energy_sum": float(E.min(1).sum()),
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        threads = min(16, os.cpu_count() or 1)
        # sample: the first 16 instances, 16 trajectories each, as many steps as
        # fill the time budget (a 20-step pilot sizes it)
        mats = []
        for k in range(16):
            n = int(sizes[k])
            e, w, _ = I.regular3_maxcut(n, 1000 + k)
            mats.append((n, I.edges_to_dense(n, e, w), I.psi0_real(n, 16, 5000 + k)))

        def sweep(nsteps):
            t0 = time.perf_counter()
            done = 0
            for n, J, x in mats:
                O.run(J, x, model="ising", steps=nsteps, dt=wl["dt"], eps=0.1, nthreads=threads)
                done += n * 16 * nsteps
            return done, time.perf_counter() - t0

        _, pilot = sweep(20)
        nsteps = max(20, min(20 * steps, int(args.cpu_seconds * 20 / max(pilot, 1e-6))))
        for _ in range(3):
            done, elc = sweep(nsteps)
            if elc >= 0.5 * args.cpu_seconds or nsteps >= 20 * steps:
                break
            nsteps = min(20 * steps, int(nsteps * args.cpu_seconds / max(elc, 1e-6)))
        out["cpu_baseline"] = {"value": done / elc, "unit": "spin-updates/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"16 instances x 16 trajectories x {nsteps} steps "
                                         f"(dense FP64 oracle), {elc:.1f} s"}
    print(json.dumps(out), flush=True)


def bench_gdmod(args, wl, steps):
    """GD-mod throughput: every step streams each trajectory's N x N coupling
    matrix K through HBM once (read and write), so the roofline is HBM
    bandwidth; algorithmic bytes per launch = R Np^2 8 (K) + R Np (2 P + 2) 4
    (amplitudes and gains, read and written).  J rows are shared by all
    trajectories and served from L2 (not counted)."""
    import torch

    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I

    n, R = wl["n"], wl["R"]
    J = getattr(I, wl["J"])(n, 1)
    Jd = J.astype(np.float64)
    np.fill_diagonal(Jd, 0.0)
    gc = float(np.abs(Jd).sum(1).max() / np.sqrt((Jd**2).sum() / n))
    psi0 = I.psi0_complex(n, R, 1)
    torch.cuda.init()
    S = gd.Solver(J, model=gd.GD_XY, dt=wl["dt"], eps=0.1, variant=gd.GD_VARIANT_MOD, eps_hat=0.2,
                  gamma_c=gc, check_interval=args.check, flags=gd.GD_F_PROFILE)
    S.set_init(R, psi0)
    if args.warmup:
        S.run(args.warmup)
    S.set_init(R, psi0)
    torch.cuda.synchronize()
    st0 = S.stats()
    t0 = time.perf_counter()
    S.run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = S.stats()
    E, best = S.energy()
    S.close()
    Np = -(-n // 64) * 64
    launches = st.kernel_launches - st0.kernel_launches
    avg_s = (st.kernel_ms - st0.kernel_ms) / 1e3 / max(launches, 1)
    bytes_launch = R * Np * Np * 8.0 + R * Np * (2 * 2 + 2) * 4.0
    achieved = bytes_launch / avg_s / 1e9
    out = {
        "metric": "spin-updates/s (N*R*steps/s)", "value": n * R * steps / el, "unit": "spin-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": el / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "R": R, "integrator": "euler", "dt": wl["dt"],
                   "gamma_c": gc, "energy_check_every": args.check},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None, "kernel": "gdmod_euler_k",
                     "launches": int(launches), "avg_launch_us": avg_s * 1e6,
                     "bytes_per_launch": bytes_launch},
        "best_energy": float(E[best]),
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        threads = min(16, os.cpu_count() or 1)
        Rs = threads
        t0 = time.perf_counter()
        O.run_mod(J, psi0[:Rs], model="xy", steps=20, dt=wl["dt"], eps=0.1, eps_hat=0.2, gamma_c=gc,
                  nthreads=threads)
        pilot = time.perf_counter() - t0
        ns = max(1, min(10 * steps, int(args.cpu_seconds * 20 / max(pilot, 1e-6))))
        t0 = time.perf_counter()
        O.run_mod(J, psi0[:Rs], model="xy", steps=ns, dt=wl["dt"], eps=0.1, eps_hat=0.2, gamma_c=gc,
                  nthreads=threads)
        elc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n * Rs * ns / elc, "unit": "spin-updates/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{Rs} of {R} trajectories x {ns} steps, {elc:.1f} s"}
    print(json.dumps(out), flush=True)


def compare_ttt(args):
    """Time to target, random vs learned start (one JSON line): 256 held-out
    random 3-regular max-cut instances, N in [512, 2048], R = 64, Euler.
    Target per instance: best-known energy + 0.1%, best-known = best over two
    12 000-step runs from other starts.  (FP32 vs BF16/FP8-J time to target
    is part of the default bench line, over several starts.)"""
    import torch

    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I
    from paper_1807_00699_amd import train_proposal as T

    torch.cuda.init()
    out = {"compare": "time-to-target within 0.1% of best-known energy"}
    here = os.path.join(ROOT, "paper_1807_00699_amd")
    params = np.load(os.path.join(here, "proposal_weights.npy"))
    meta = json.load(open(os.path.join(here, "proposal_meta.json")))
    sizes, insts = I.maxcut_batch(256, 512, 2048, 999)
    refb = T.reference_energies(insts, 64, 12000, seeds=[301, 302])
    targets = refb + 1e-3 * np.abs(refb)
    budget, chk = 3000, 25
    rows = {}
    base, bsec, _, bwall = T.steps_to_target(insts, 64, budget, chk, targets, seed=11)
    with gd.MLP(params) as m:
        lrn, lsec, _, lwall = T.steps_to_target(insts, 64, budget, chk, targets, m, meta["alpha"],
                                                meta["beta"], seed=11)
    for name, st, sec, wall in (("random_start", base, bsec, bwall), ("learned_start", lrn, lsec, lwall)):
        ok = st >= 0
        rows[name] = {"reached": int(ok.sum()), "of": len(st),
                      "median_steps_reached": float(np.median(st[ok])) if ok.any() else None,
                      "mean_steps_censored": float(np.where(ok, st, budget).mean()),
                      "batch_ttt_s_all": float(sec.max()) if ok.all() else None, "run_s": wall}
    out["batch256_learned"] = {"budget_steps": budget, "check_every": chk, **rows}
    print(json.dumps(out), flush=True)


def _lambda_max(J, s):
    """largest algebraic eigenvalue of J/s (host, for gamma_c above it)"""
    from scipy.sparse.linalg import eigsh
    return float(eigsh(np.asarray(J, np.float64) / s, k=1, which="LA", tol=1e-8)[0][0])


def _stationary_steps(S, R, max_steps, check, rho_th=1.0, tol=1e-3):
    """Integrate in chunks of `check` steps; a trajectory is stationary at the
    first check where max_i |rho_i - rho_th| < tol rho_th and no phase moved
    by more than tol (radians) since the previous check.  Returns the step
    count per trajectory (-1 if not reached)."""
    first = np.full(R, -1, np.int64)
    prev = None
    done = 0
    while done < max_steps and np.any(first < 0):
        S.run(check)
        done += check
        p, _, _ = S.state()
        z = p[..., 0].astype(np.float64) + 1j * p[..., 1]
        rho = np.abs(z) ** 2
        th = np.angle(z)
        if prev is not None:
            dth = np.abs(np.angle(np.exp(1j * (th - prev))))
            ok = (np.abs(rho - rho_th).max(1) < tol * rho_th) & (dth.max(1) < tol)
            first[(first < 0) & ok] = done
        prev = th
    return first


def scaling(args):
    """Time per instance to a stationary state vs N on one GPU (the paper
    times 20 runs per size of its GD algorithm on XY problems up to N = 3000
    and fits a power law).  Per N: dense U[-10,10] couplings, XY, RK4
    dt = 0.02, eps = 0.5, Psi(0) = 0 with noise D = 1e-6 (it only seeds the
    symmetry breaking) and gamma_c = lambda_max(J/s) + 0.1 (gain rising from
    below); R = 128 runs in one batch (the trajectory
    tile is 128 wide, so 20 runs would cost the same).  Pass 1 finds each
    run's steps to stationarity (host checks every 100 steps); pass 2 times
    200 steps without checks; time per run = steps x time per step of the
    batch.  The FP64 oracle's time per RK4 step of one run (one core) is
    measured beside it."""
    import torch

    from oracle import oracle as O
    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I

    torch.cuda.init()
    sizes = [250, 500, 1000, 1500, 2000, 3000, 4000]
    R, check, budget = 128, 100, 80000
    rows = []
    for n in sizes:
        J = I.dense_uniform(n, 7000 + n)
        s = float(np.sqrt((J.astype(np.float64) ** 2).sum() / n))
        gc = _lambda_max(J, s) + 0.1
        kw = dict(integrator=gd.GD_RK4, dt=0.02, eps=0.5, gamma_c=gc, noise_D=1e-6,
                  noise_seed=n, init_amp=0.0)
        with gd.Solver(J, model=gd.GD_XY, **kw) as S:
            S.set_init(R)
            first = _stationary_steps(S, R, budget, check)
            S.set_init(R)
            S.run(20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.run(200)
            ms = (time.perf_counter() - t0) / 200 * 1e3
            E, b = S.energy()
        reached = first >= 0
        mean_steps = float(first[reached].mean()) if reached.any() else None
        # median over all runs, unreached ones counted as beyond the budget
        med = float(np.median(np.where(reached, first, budget + 1)))
        median_steps = med if med <= budget else None
        psi = np.zeros((1, n, 2))
        t0 = time.perf_counter()
        O.run(J, psi + 0.1, model="xy", steps=2, dt=0.02, eps=0.5, integrator=O.RK4, nthreads=1)
        oracle_ms = (time.perf_counter() - t0) / 2 * 1e3
        rows.append({"n": n, "runs": R, "reached": int(reached.sum()), "mean_steps": mean_steps,
                     "median_steps": median_steps,
                     "seconds_per_run_median": None if median_steps is None else median_steps * ms / 1e3,
                     "max_steps": int(first[reached].max()) if reached.any() else None,
                     "ms_per_step_batch": ms,
                     "seconds_per_run_mean": None if mean_steps is None else mean_steps * ms / 1e3,
                     "seconds_all_runs": None if not reached.all() else float(first.max()) * ms / 1e3,
                     "oracle_ms_per_step_one_run": oracle_ms})
        print(json.dumps({"progress": rows[-1]}), file=sys.stderr, flush=True)
    ok = [r for r in rows if r["median_steps"]]
    ln = np.log([r["n"] for r in ok])

    def slope(key):
        if len(ok) < 2:
            return None
        return float(np.polyfit(ln, np.log([r[key] for r in ok]), 1)[0])

    print(json.dumps({"scaling": "time to a stationary state vs N (XY, U[-10,10], RK4, eps 0.5, "
                                 "paper regime)",
                      "rows": rows,
                      "fit_exponent": {"seconds_per_run_median": slope("seconds_per_run_median"),
                                       "median_steps": slope("median_steps"),
                                       "ms_per_step_batch": slope("ms_per_step_batch"),
                                       "oracle_ms_per_step_one_run": slope("oracle_ms_per_step_one_run")},
                      "criterion": "max_i |rho_i - 1| < 1e-3 and max_i |dtheta_i| < 1e-3 rad "
                                   "between checks 100 steps apart",
                      "budget_steps": budget}), flush=True)


def gdmod_scaling(args):
    """Steps to a stationary state vs N for GD and GD-mod on the same problems
    (the paper expects GD-mod's iteration count to grow more slowly with N,
    Sec. 4).  XY, dense U[-10,10] couplings, explicit Euler dt = 0.02,
    eps = 0.5, eps_hat = 0.5, Psi(0) = 0 with D = 1e-6, gamma_c = max_i
    sum_j |J_ij| / s for both (GD-mod needs positive gains; the same loss keeps
    the comparison fair), 32 runs per N, stationarity as in --scaling."""
    import torch

    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I

    torch.cuda.init()
    R, check, budget = 32, 100, 60000
    rows = []
    for n in (100, 200, 400, 800, 1600):
        J = I.dense_uniform(n, 9000 + n)
        Jd = J.astype(np.float64)
        s = float(np.sqrt((Jd**2).sum() / n))
        gc = float(np.abs(Jd).sum(1).max() / s)
        row = {"n": n, "runs": R, "gamma_c": gc}
        for name, var in (("gd", gd.GD_VARIANT_GD), ("gdmod", gd.GD_VARIANT_MOD)):
            with gd.Solver(J, model=gd.GD_XY, dt=0.02, eps=0.5, variant=var, eps_hat=0.5,
                           gamma_c=gc, noise_D=1e-6, noise_seed=n, init_amp=0.0) as S:
                S.set_init(R)
                first = _stationary_steps(S, R, budget, check)
                S.set_init(R)
                S.run(20)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                S.run(500)
                ms = (time.perf_counter() - t0) / 500 * 1e3
                E, b = S.energy()
            reached = first >= 0
            med = float(np.median(np.where(reached, first, budget + 1)))
            row[name] = {"reached": int(reached.sum()),
                         "median_steps": med if med <= budget else None,
                         "ms_per_step_batch": ms}
        rows.append(row)
        print(json.dumps({"progress": row}), file=sys.stderr, flush=True)

    def slope(name):
        pts = [(r["n"], r[name]["median_steps"]) for r in rows if r[name]["median_steps"]]
        if len(pts) < 2:
            return None
        return float(np.polyfit(np.log([p[0] for p in pts]), np.log([p[1] for p in pts]), 1)[0])

    print(json.dumps({"gdmod_scaling": "steps to a stationary state vs N, GD vs GD-mod (XY, U[-10,10], "
                                       "Euler dt=0.02, eps=eps_hat=0.5)",
                      "rows": rows, "fit_exponent_median_steps": {"gd": slope("gd"), "gdmod": slope("gdmod")},
                      "budget_steps": budget}), flush=True)


def learned_bench(args):
    """Throughput of the learned proposal's own kernels, one JSON line.
    Data: 256 random 3-regular max-cut instances, N even in [512, 2048]
    (the training distribution), features from gd_features (30 block-power
    iterations), random +-1 labels (the arithmetic does not depend on them);
    all rows and labels resident on the device.  Timed: FP32 training steps
    (forward, backward, Adam) on minibatches of 64 instances; FP16 and FP32
    inference over all spins; gd_propose (features + FP16 network + initial
    state) for the 256 instances x R = 64.  Flops per spin row: forward
    2 (20*64 + 64*64 + 64*2) = 11 008, a training step about three times that
    (forward, activation and weight gradients).  Training runs on the FP32
    matrix cores (157.3 TFLOP/s) and the step's time includes its host round
    trip (the loss is read back every step); FP32 inference, the reference
    form of the network, on the FP32 vector ALUs (78.6 TFLOP/s without packed
    math); FP16 inference on the matrix cores (FP16 MFMA 2.5 PFLOP/s), where
    the features it reads (80 B per row) and the outputs it writes (8 B) make
    HBM (8 TB/s) the bound."""
    import torch

    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I

    torch.cuda.init()
    sizes, insts = I.maxcut_batch(256, 512, 2048, 7)
    sizes = np.asarray(sizes, np.int64)
    with gd.BatchSolver(insts) as B:
        X, _, _ = gd.gd_features(B.h, int(sizes.sum()), len(insts), 30)
    rng = np.random.default_rng(7)
    lab = np.where(rng.random(X.shape[0]) < 0.5, -1.0, 1.0).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Ld = torch.from_numpy(lab).cuda()
    off = np.concatenate([[0], np.cumsum(sizes)])
    fwd = 2 * (20 * 64 + 64 * 64 + 64 * 2)
    peak = 78.6
    out = {"learned": "proposal network throughput (device buffers)", "rows_total": int(X.shape[0]),
           "instances": len(insts), "flops_per_row_forward": fwd, "flops_per_row_train": 3 * fwd,
           "peak_tflops_fp32_valu": peak}
    steps = args.steps or 40
    with gd.MLP(seed=1, device=True) as m:
        batches = []
        for b in range(4):
            r0, r1 = int(off[64 * b]), int(off[64 * (b + 1)])
            seg = (off[64 * b:64 * (b + 1) + 1] - r0).astype(np.int32)
            batches.append((Xd[r0:r1], Ld[r0:r1], seg))
        for w in range(3):
            m.train_step_device(*batches[w % 4], 1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows = 0
        for s in range(steps):
            xb, lb, sg = batches[s % 4]
            m.train_step_device(xb, lb, sg, 1e-3)
            rows += int(xb.shape[0])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["train"] = {"steps": steps, "rows_per_s": rows / el, "instances_per_s": 64 * steps / el,
                        "ms_per_step": 1e3 * el / steps,
                        "tflops": 3 * fwd * rows / el / 1e12,
                        "frac_fp32_mfma": 3 * fwd * rows / el / 1e12 / PEAKS_TFLOPS["fp32"]}
        o = torch.empty((X.shape[0], 2), dtype=torch.float32, device="cuda")
        for name, fp16 in (("infer_fp16", True), ("infer_fp32", False)):
            for _ in range(3):
                m.forward_device(Xd, o, fp16)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(50):
                m.forward_device(Xd, o, fp16)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            r = 50 * X.shape[0] / el
            out[name] = {"rows_per_s": r, "us_per_call": 1e6 * el / 50, "tflops": fwd * r / 1e12,
                         "frac": fwd * r / 1e12 / peak}
            if fp16:
                out[name] = {"rows_per_s": r, "us_per_call": 1e6 * el / 50, "tflops": fwd * r / 1e12,
                             "frac_fp16_mfma": fwd * r / 1e12 / PEAKS_TFLOPS["fp16"],
                             "hbm_gbs": 88 * r / 1e9, "frac_hbm": 88 * r / 1e9 / PEAK_HBM_GBS,
                             "bound": "hbm", "bytes_per_row": 88}
    with gd.BatchSolver(insts) as B, gd.MLP(seed=1) as mh:
        gd.gd_propose(B.h, mh, 64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            gd.gd_propose(B.h, mh, 64)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["propose"] = {"instances_per_s": 10 * len(insts) / el, "ms_per_call": 1e3 * el / 10,
                          "R": 64, "feature_iterations": 30}
    print(json.dumps(out), flush=True)


def maxcut800(args):
    """Max-cut stand-ins shaped like the paper's N = 800 benchmarks (Sec. 3):
    five G(800, 0.06) graphs with unit weights and five with +-1 weights, 100
    runs each (one batch), Ising Euler dt = 0.05, budget 5000 steps, in two
    regimes: random start (U(-0.1, 0.1), gamma_c = 0) and the paper's
    Psi(0) = 0 with noise and gain from below.  Best-known cut per instance:
    best over both regimes and a longer run (1000 runs, 20000 steps).
    Reports mean and best cut, the mean's deviation from the best-known cut,
    and the wall time of the 100-run batch."""
    import torch

    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I

    torch.cuda.init()
    n, p, R, steps = 800, 0.06, 100, 5000
    out = []
    for k in range(10):
        signed = k >= 5
        e, w = I.gnp_maxcut(n, p, 800 + k, signed=signed)
        J = I.edges_to_dense(n, e, -w)
        W = float(w.astype(np.float64).sum())
        s = float(np.sqrt((J.astype(np.float64) ** 2).sum() / n))
        gc = _lambda_max(J, s) + 0.5
        regimes = {"random_start": dict(init_amp=0.1, seed=k),
                   "paper_regime": dict(init_amp=0.0, gamma_c=gc, noise_D=0.01, noise_seed=k)}
        row = {"instance": k, "weights": "+-1" if signed else "1", "edges": int(e.shape[0])}
        best_cut = -np.inf
        for name, kw in regimes.items():
            with gd.Solver(J, model=gd.GD_ISING, dt=0.05, eps=0.1, **kw) as S:
                S.run(10, batch=R)
                S.set_init(R)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                S.run(steps)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                E, b = S.energy()
            cuts = W / 2 - E / 4
            best_cut = max(best_cut, cuts.max())
            row[name] = {"mean_cut": float(cuts.mean()), "best_cut": float(cuts.max()),
                         "seconds_100_runs": el}
            with gd.Solver(J, model=gd.GD_ISING, dt=0.05, eps=0.1,
                           **{**kw, "seed": kw.get("seed", 0) + 100,
                              "noise_seed": kw.get("noise_seed", 0) + 100}) as S:
                S.run(20000, batch=1000)
                E, b = S.energy()
            best_cut = max(best_cut, float((W / 2 - E / 4).max()))
        row["best_known_cut"] = float(best_cut)
        for name in regimes:
            row[name]["mean_deviation_pct"] = 100 * (best_cut - row[name]["mean_cut"]) / best_cut
        out.append(row)
        print(json.dumps({"progress": row}), file=sys.stderr, flush=True)
    summ = {}
    for name in ("random_start", "paper_regime"):
        for grp, sl in (("unit", slice(0, 5)), ("signed", slice(5, 10))):
            devs = [r[name]["mean_deviation_pct"] for r in out[sl]]
            summ[f"{name}_{grp}_mean_deviation_pct"] = [float(min(devs)), float(max(devs))]
    print(json.dumps({"maxcut800": "G(800,0.06) stand-ins, 100 runs x 5000 Euler steps",
                      "summary": summ, "rows": out}), flush=True)


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_rate(J, psi0, model, integrator, dt, threads, target_s, steps_cap):
    """Oracle spin-updates/s on len(psi0) trajectories with `threads` OpenMP
    threads (over trajectories), run long enough to take about target_s."""
    from oracle import oracle as O
    n, Rs = J.shape[0], psi0.shape[0]
    integ = O.RK4 if integrator == "rk4" else O.EULER
    steps = 2
    t0 = time.perf_counter()
    O.run(J, psi0, model=model, steps=steps, dt=dt, eps=0.1, integrator=integ, nthreads=threads)
    pilot = time.perf_counter() - t0
    steps = int(max(2, min(steps_cap, target_s * steps / max(pilot, 1e-6))))
    t0 = time.perf_counter()
    O.run(J, psi0, model=model, steps=steps, dt=dt, eps=0.1, integrator=integ, nthreads=threads)
    el = time.perf_counter() - t0
    return n * Rs * steps / el, steps, el


def headline(args):
    """Dense Ising N = 4096, R = 4096: plain FP32 vs BF16 operand with FP8 J,
    throughput, time to target and the oracle baseline (see the module
    docstring)."""
    import torch

    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I

    n, R, dt = 4096, 4096, 0.05
    K = args.steps if args.steps is not None else 200
    check = max(1, min(args.check, K))
    J = I.sparse_pm1(n, 1)
    x0 = I.psi0_real(n, R, 1)
    torch.cuda.init()
    forms = (("fp32", gd.GD_PREC_FP32, "f32"), ("bf16_fp8j", gd.GD_PREC_BF16, "bf16xf32"))
    legs, results = {}, {}
    for name, prec, dtype in forms:
        S = gd.Solver(J, model=gd.GD_ISING, dt=dt, eps=0.1, precision=prec, check_interval=check,
                      flags=gd.GD_F_PROFILE)
        S.set_init(R, x0)
        if args.warmup:
            S.run(args.warmup)
        S.set_init(R, x0)            # the timed run starts from the initial state
        torch.cuda.synchronize()
        st0 = S.stats()
        t0 = time.perf_counter()
        S.run(K)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = S.stats()
        E, best = S.energy()                       # FP64 re-score of the readout
        Ed, best_d = S.energy(device_path=True)    # the device check's FP32 product, FP64 sums
        spins = S.spins()
        S.close()
        launches = st.kernel_launches - st0.kernel_launches
        avg_s = (st.kernel_ms - st0.kernel_ms) / 1e3 / max(launches, 1)
        flops_launch = 2.0 * n * n * R
        peak = PEAKS_TFLOPS["fp32" if prec == gd.GD_PREC_FP32 else "bf16"]
        achieved = flops_launch / avg_s / 1e12
        legs[name] = {
            "value": n * R * K / el, "ms_per_step": el / K * 1e3, "dtype": dtype,
            "kernel_config": st.kernel_config, "best_energy": float(E[best]),
            "device_check_equals_fp64_rescore": bool(np.array_equal(E, Ed) and best == best_d),
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                         "frac": achieved / peak,
                         "traffic": kernel_traffic(st.kernel_config, "dense_step_f32" if prec == gd.GD_PREC_FP32
                                                    else "dense_step_lp", "ising4096"),
                         "kernel": "dense_step_f32" if prec == gd.GD_PREC_FP32 else "dense_step_lp",
                         "launches": int(launches), "avg_launch_us": avg_s * 1e6,
                         "flops_per_launch": flops_launch},
        }
        results[name] = (E, Ed, spins, best)
        print(json.dumps({"progress": name, "ms_per_step": legs[name]["ms_per_step"]}), file=sys.stderr,
              flush=True)

    ttt = None if args.no_ttt else headline_ttt(args, J, x0, n, R, dt)

    fp = legs["fp32"]
    out = {
        "metric": "spin-updates/s (N*R*steps/s)", "value": fp["value"], "unit": "spin-updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": fp["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Ising, N=4096, J in {-1,0,1} density 0.5 (signs equiprobable), R=4096 "
                               "random restarts, Euler dt=0.05, plain FP32 form (legs: BF16 operand "
                               "with FP8-stored J)",
                   "n": n, "R": R, "integrator": "euler", "dt": dt, "energy_check_every": check,
                   "kernel_config": fp["kernel_config"]},
        "roofline": fp["roofline"],
        "legs": {"bf16_fp8j": legs["bf16_fp8j"]},
        "best_energy": fp["best_energy"],
    }
    if ttt is not None:
        out["ttt"] = ttt
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["energy_vs_oracle"] = headline_cpu_leg(args, J, x0, results)
    print(json.dumps(out), flush=True)


def tts99(reach, horizons):
    """Time to solution with 99% confidence from independent starts: for a
    run length T, p(T) = fraction of starts that reached the target by T and
    TTS99(T) = T ln(0.01) / ln(1 - p(T)) (T itself when every start reached
    it); the minimum over the check times T.  None when no start reached it.
    `reach` and `horizons` share one unit (steps here, so that a start is
    counted at the check where it reached the target whatever its own time
    per step)."""
    best, at = None, None
    m = len(reach)
    for T in horizons:
        p = sum(1 for x in reach if x is not None and x <= T) / m
        if p == 0:
            continue
        v = T if p == 1 else T * np.log(0.01) / np.log(1.0 - p)
        if best is None or v < best:
            best, at = v, T
    return best, at


def headline_ttt(args, J, x0, n, R, dt):
    """Time to target for both forms.  Each form runs `ttt_seeds` batches of R
    trajectories from other starts for the whole step budget, with a device
    energy check every 100 steps, and keeps the best-so-far energy of every
    check (gd_best_trace).  Best-known energy: the lowest energy of every run
    made here -- reference runs from further starts (four BF16 batches over
    twice the budget, one FP32 batch over the budget) and the timed runs
    themselves; target = best-known + 0.1% of its magnitude.  A run's time to
    target = the steps of its first check at or below the target x its time
    per step (device work queued back to back, host wall time of the run /
    its steps); runs that never reach it are censored: success fraction,
    median over the starts (None when half or more are censored) and the time
    to solution with 99% confidence over independent starts (TTS99)."""
    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I

    budget, chk = args.ttt_budget, 100
    t_ref = time.perf_counter()
    ref = []
    for prec, seeds, steps in ((gd.GD_PREC_BF16, (101, 102, 103, 104), 2 * budget),
                               (gd.GD_PREC_FP32, (105,), budget)):
        for sd in seeds:
            with gd.Solver(J, model=gd.GD_ISING, dt=dt, eps=0.1, precision=prec, check_interval=500) as S:
                S.set_init(R, I.psi0_real(n, R, sd))
                S.run(steps)
                ref.append(S.stats().best_energy)
            print(json.dumps({"progress": "reference", "seed": sd, "best": ref[-1]}), file=sys.stderr,
                  flush=True)
    ref_s = time.perf_counter() - t_ref
    runs = {}
    for name, prec in (("fp32", gd.GD_PREC_FP32), ("bf16_fp8j", gd.GD_PREC_BF16)):
        runs[name] = []
        for k in range(args.ttt_seeds):
            with gd.Solver(J, model=gd.GD_ISING, dt=dt, eps=0.1, precision=prec, check_interval=chk) as S:
                S.set_init(R, I.psi0_real(n, R, 1 + k))
                S.run(chk)                    # kernel choice and warm-up, untimed
                S.set_init(R, I.psi0_real(n, R, 1 + k))
                t0 = time.perf_counter()
                S.run(budget)
                wall = time.perf_counter() - t0
                steps, best = S.best_trace()
            runs[name].append((steps, best, wall / budget))
            print(json.dumps({"progress": "ttt", "form": name, "start": 1 + k, "best": float(best[-1]),
                              "s_per_step": wall / budget}), file=sys.stderr, flush=True)
    best_known = float(min(min(ref), *(float(r[1][-1]) for v in runs.values() for r in v)))
    target = best_known + 1e-3 * abs(best_known)
    forms = {}
    for name, rs in runs.items():
        secs, steps_at = [], []
        for steps, best, sps in rs:
            hit = np.nonzero(best <= target)[0]
            steps_at.append(int(steps[hit[0]]) if hit.size else None)
            secs.append(float(steps[hit[0]] * sps) if hit.size else None)
        srt = sorted(x if x is not None else np.inf for x in secs)
        med = srt[len(srt) // 2] if len(srt) % 2 else 0.5 * (srt[len(srt) // 2 - 1] + srt[len(srt) // 2])
        sps_med = float(np.median([r[2] for r in rs]))
        tts, at = tts99(steps_at, range(chk, budget + 1, chk))
        tts = None if tts is None else float(tts * sps_med)
        at = None if at is None else float(at * sps_med)
        forms[name] = {"seconds": secs, "steps": steps_at, "best_energy": [float(r[1][-1]) for r in rs],
                       "seconds_per_step": sps_med,
                       "median_seconds": None if not np.isfinite(med) else float(med),
                       "success_fraction": sum(x is not None for x in secs) / len(secs),
                       "tts99_seconds": tts, "tts99_run_seconds": at}
    t99 = {k: v["tts99_seconds"] for k, v in forms.items()}
    med = {k: v["median_seconds"] for k, v in forms.items()}
    return {"target": target, "best_known": best_known,
            "rule": "best-known = lowest device-checked energy of every run made here (4 BF16 reference "
                    f"batches x {2 * budget} steps, 1 FP32 batch x {budget} steps, and the timed runs; "
                    f"R={R} each); target = best-known + 0.1%",
            "reference_seconds": ref_s, "budget_steps": budget, "check_every": chk,
            "clock": "steps at the first check at the target x the run's time per step (host wall "
                     "time of the whole run / its steps, device work queued back to back)",
            "seeds": args.ttt_seeds, **forms,
            "speedup_bf16_over_fp32": {
                "median": med["fp32"] / med["bf16_fp8j"] if med["fp32"] and med["bf16_fp8j"] else None,
                "tts99": t99["fp32"] / t99["bf16_fp8j"] if t99["fp32"] and t99["bf16_fp8j"] else None}}


def headline_cpu_leg(args, J, x0, results):
    """The oracle on the host: its throughput on a sample of the workload (all
    cores: one trajectory per thread; one thread: one trajectory), and its
    Eq. (h) energies of the spins each form returned (the best trajectory and
    seven others), against the library's FP64 re-score and device check."""
    from oracle import oracle as O
    threads = min(16, os.cpu_count() or 1)
    v_all, st_all, el_all = oracle_rate(J, x0[:threads], "ising", "euler", 0.05, threads, args.cpu_seconds, 2000)
    v_one, st_one, el_one = oracle_rate(J, x0[:1], "ising", "euler", 0.05, 1, args.cpu_seconds / 2, 2000)
    cpu = {"value": v_all, "unit": "spin-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{threads} of {x0.shape[0]} trajectories x {st_all} steps, {el_all:.1f} s",
           "single_thread": {"value": v_one, "cores": 1,
                             "sample": f"1 trajectory x {st_one} steps, {el_one:.1f} s"},
           "host_cpu": host_cpu_model()}
    errs = {}
    for name, (E, Ed, spins, best) in results.items():
        R = spins.shape[0]
        sub = sorted({int(best), 0, 1, R // 3, R // 2, 2 * R // 3, R - 2, R - 1})
        Eo = O.energy_ising(J, spins[sub]).astype(np.float64)
        errs[name] = {"trajectories": sub,
                      "max_abs_fp64_rescore_minus_oracle": float(np.abs(E[sub] - Eo).max()),
                      "max_abs_device_check_minus_oracle": float(np.abs(Ed[sub] - Eo).max()),
                      "best_energy_oracle": float(Eo[sub.index(int(best))]),
                      "max_rel_fp64_rescore_minus_oracle": float((np.abs(E[sub] - Eo) / np.abs(Eo)).max())}
    return cpu, errs


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); restarts are independent, "
              "so N GPUs would each run their own share of trajectories with no communication.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.scaling:
        scaling(args)
        return
    if args.maxcut800:
        maxcut800(args)
        return
    if args.gdmod_scaling:
        gdmod_scaling(args)
        return
    if args.compare_ttt:
        compare_ttt(args)
        return
    if args.learned:
        learned_bench(args)
        return
    import torch

    from paper_1807_00699_amd import gd
    from paper_1807_00699_amd import inputs as I

    if args.workload == "ising4096":
        return headline(args)
    wl = WORKLOADS[args.workload]
    steps = args.steps if args.steps is not None else wl["steps"]
    if wl.get("batch"):
        return bench_batch(args, wl, steps)
    if wl.get("gdmod"):
        return bench_gdmod(args, wl, steps)
    n, R = wl["n"], wl["R"]
    J = getattr(I, wl["J"])(n, 1)
    psi0 = I.psi0_complex(n, R, 1) if wl["model"] == "xy" else I.psi0_real(n, R, 1)
    model = gd.GD_XY if wl["model"] == "xy" else gd.GD_ISING
    integ = gd.GD_RK4 if wl["integrator"] == "rk4" else gd.GD_EULER
    torch.cuda.init()
    # inputs resident in HBM before the timed region; HIP events on the
    # solver's stream around the coupling launches of every 8th step (GD_F_PROFILE)
    prec_name = wl.get("precision", "fp32")
    prec = {"fp32": gd.GD_PREC_FP32, "bf16": gd.GD_PREC_BF16, "fp16": gd.GD_PREC_FP16}[prec_name]
    S = gd.Solver(J, model=model, integrator=integ, dt=wl["dt"], eps=0.1, precision=prec,
                  check_interval=args.check, flags=gd.GD_F_PROFILE)
    target = best_known = None
    if not args.no_ttt:
        # best-known energy: two untimed runs of the same length from other starts
        for seed in (2, 3):
            p0 = I.psi0_complex(n, R, seed) if wl["model"] == "xy" else I.psi0_real(n, R, seed)
            S.set_init(R, p0)
            S.run(steps)
            E, b = S.energy()
            best_known = E[b] if best_known is None else min(best_known, E[b])
        target = best_known + 1e-3 * abs(best_known)
    S.set_init(R, psi0)
    if args.warmup:
        S.run(args.warmup)
    S.set_init(R, psi0)          # the timed run starts from the initial state
    if target is not None:
        gd.gd_set_targets(S.h, [target])     # recorded, not a stopping point
    torch.cuda.synchronize()
    st0 = S.stats()
    t0 = time.perf_counter()
    S.run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = S.stats()
    E, best = S.energy()
    S.close()

    P = 2 if wl["model"] == "xy" else 1
    launches = st.kernel_launches - st0.kernel_launches
    kms = st.kernel_ms - st0.kernel_ms
    avg_s = kms / 1e3 / max(launches, 1)
    flops_launch = 2.0 * n * n * P * R          # coupling GEMM of one launch
    # padded sizes of at most 128 spins, FP32: the runtime runs many steps per
    # launch of its fused small-problem kernel (FP32 vector ALUs); its events
    # then bracket whole launches and count their coupling evaluations (the
    # J d of an energy check closing a launch is one more)
    small = (-(-n // 64) * 64 <= 128 and prec_name == "fp32")
    gemv = st.kernel_config >= 100 and not small
    achieved = flops_launch / avg_s / 1e12
    if gemv:
        # J-streaming matrix-vector kernel: algorithmic HBM bytes of one launch
        # = the couplings once (FP32, or FP8 when stored so) + the state of R
        # trajectories (Euler: amplitudes and gains read and written, FP32;
        # reduced precision adds the 16-bit operand copy, read and written)
        if prec_name == "fp32":
            jb = 1 if fp8_exact(J) and os.environ.get("GD_J8_COPY", "1") != "0" else 4
        else:
            jb = 1 if fp8_exact(J) else 2
        bytes_launch = n * n * jb + R * n * (8 * P + 8) + (0 if prec_name == "fp32" else R * n * P * 4)
        hbm_gbs = bytes_launch / avg_s / 1e9
    out = {
        "metric": "spin-updates/s (N*R*steps/s)",
        "value": n * R * steps / el,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": el / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec_name == "fp32" else f"{prec_name}xf32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "R": R, "integrator": wl["integrator"],
                   "dt": wl["dt"], "energy_check_every": args.check, "kernel_config": st.kernel_config},
        "roofline": ({"bound": "hbm", "achieved": hbm_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": hbm_gbs / PEAK_HBM_GBS,
                      "traffic": (kernel_traffic(st.kernel_config, "gemv_step_k",
                                                 "ising4096_r1_j" + ("fp8" if jb == 1 else "fp32"))
                                  if args.workload in ("gemv4096", "gemv4096_f32j") else None),
                      "j_bytes_per_coupling": jb,
                      "kernel": "gemv_step_k",
                      "launches": int(launches), "avg_launch_us": avg_s * 1e6,
                      "bytes_per_launch": bytes_launch}
                     if gemv else
                     {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_F32,
                      "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_F32, "traffic": None,
                      "kernel": "small_step_k", "coupling_evaluations": int(launches),
                      "avg_evaluation_us": avg_s * 1e6, "flops_per_evaluation": flops_launch}
                     if small else
                     {"bound": "mfma", "achieved": achieved, "peak": PEAKS_TFLOPS[prec_name],
                      "unit": "TFLOP/s", "frac": achieved / PEAKS_TFLOPS[prec_name],
                      "traffic": (kernel_traffic(st.kernel_config, "dense_step_f32")
                                  if args.workload == "xy1024" else None),
                      "kernel": "dense_step_f32" if prec_name == "fp32" else "dense_step_lp",
                      "launches": int(launches),
                      "avg_launch_us": avg_s * 1e6, "flops_per_launch": flops_launch}),
        "best_energy": float(E[best]),
    }
    if target is not None:
        out["ttt"] = {"target": float(target), "best_known": float(best_known),
                      "rule": "best of two untimed runs of the same length from other starts, +0.1%",
                      "final_gap": float((E[best] - best_known) / abs(best_known)),
                      "seconds": float(st.ttt_seconds) if st.target_reached else None,
                      "steps": int(st.ttt_steps) if st.target_reached else None,
                      "check_every": args.check}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, J, psi0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
