"""Training and evaluation of the learned proposal (initial amplitudes and
per-spin gain rates) on solver-generated data; every step runs in libgd.so.

    python -m paper_1807_00699_amd.train_proposal --instances 20000 --out DIR

1. Data: random 3-regular max-cut instances (the batched workload's
   generator) with even N in [512, 2048], in chunks of 256.  Labels: for each
   instance the discretised state of lowest Eq. (h) energy over R = 64
   random-start trajectories after `label_steps` Euler steps (batched solver).
   Features: gd_features (30 block-power iterations).
2. Training: minibatches of 64 instances, FP32 forward/backward/Adam kernels
   (gd_mlp_train_step), a few epochs.
3. Selection: alpha (initial-amplitude mix) and beta (eps_i spread) from a
   small grid on validation instances by the mean number of steps to reach
   within 0.1% of the best energy found by either start.
Writes DIR/proposal_weights.npy (float32, GD_MLP_NPARAM) and
DIR/proposal_meta.json.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import gd
from . import inputs as I

FEAT_ITERS = 30


def _solve_labels(insts, R, steps, seed):
    """best discretised state per instance after `steps` random-start steps"""
    with gd.BatchSolver(insts, seed=seed) as B:
        B.run(steps, R=R)
        E, best = B.energy()
        spins = B.split(B.spins())
    return np.concatenate([spins[k][best[k]].astype(np.float32) for k in range(len(insts))]), E.min(1)


def _features(insts):
    with gd.BatchSolver(insts) as B:
        f, _, _ = gd.gd_features(B.h, int(sum(i["n"] for i in insts)), len(insts), FEAT_ITERS)
    return f


def make_dataset(count, lo, hi, seed, R=64, label_steps=3000, chunk=256, log=print):
    X, Y, segs = [], [], []
    t0 = time.time()
    for c0 in range(0, count, chunk):
        k = min(chunk, count - c0)
        sizes, insts = I.maxcut_batch(k, lo, hi, seed * 100000 + c0)
        lab, _ = _solve_labels(insts, R, label_steps, seed=c0)
        X.append(_features(insts))
        Y.append(lab)
        segs.extend(int(n) for n in sizes)
        if (c0 // chunk) % 10 == 0:
            log(f"data {c0 + k}/{count} instances, {time.time() - t0:.1f} s")
    return np.concatenate(X), np.concatenate(Y), np.array(segs, np.int64)


def train(X, Y, sizes, epochs=3, batch_instances=64, lr=2e-3, seed=0, log=print):
    off = np.concatenate([[0], np.cumsum(sizes)])
    K = len(sizes)
    rng = np.random.default_rng(seed)
    curve = []
    with gd.MLP(seed=seed) as m:
        step = 0
        for ep in range(epochs):
            order = rng.permutation(K)
            for b0 in range(0, K, batch_instances):
                ids = order[b0:b0 + batch_instances]
                rows = np.concatenate([np.arange(off[i], off[i + 1]) for i in ids])
                seg = np.concatenate([[0], np.cumsum(sizes[ids])]).astype(np.int32)
                lr_t = lr * (0.3 if ep == epochs - 1 else 1.0)
                loss = m.train_step(X[rows], Y[rows], seg, lr_t)
                curve.append(loss)
                step += 1
            log(f"epoch {ep}: mean loss {np.mean(curve[-max(1, K // batch_instances):]):.4f}")
        return m.params, curve


def steps_to_target(insts, R, budget, check, targets, mlp=None, alpha=0.5, beta=0.0, seed=0):
    """per-instance steps at the first check with best energy <= target (-1 if
    not reached), and the batch wall time"""
    with gd.BatchSolver(insts, check_interval=check, has_target=1, seed=seed) as B:
        if mlp is None:
            B.set_init(R)
        else:
            gd.gd_propose(B.h, mlp, R, FEAT_ITERS, alpha, beta, seed)
            B.R = R
        B.set_targets(targets)
        t0 = time.perf_counter()
        B.run(budget)
        wall = time.perf_counter() - t0
        sec, steps, best = B.ttt()
    return steps, sec, best, wall


def reference_energies(insts, R, steps, seeds):
    """best energy over several long random-start runs"""
    best = None
    for s in seeds:
        with gd.BatchSolver(insts, seed=s) as B:
            B.run(steps, R=R)
            E, _ = B.energy()
        e = E.min(1)
        best = e if best is None else np.minimum(best, e)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--instances", type=int, default=20000)
    ap.add_argument("--val", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--label-steps", type=int, default=3000)
    ap.add_argument("--out", default="proposal_out", help="folder for the weights, the log and the validation record")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    logf = open(os.path.join(args.out, "train_proposal.log"), "w")

    def log(s):
        print(s, flush=True)
        logf.write(s + "\n")
        logf.flush()

    X, Y, sizes = make_dataset(args.instances, 512, 2048, seed=1, label_steps=args.label_steps, log=log)
    log(f"dataset: {len(sizes)} instances, {X.shape[0]} spins")
    params, curve = train(X, Y, sizes, epochs=args.epochs, log=log)
    np.save(os.path.join(args.out, "proposal_weights.npy"), params.astype(np.float32))
    # validation: choose alpha, beta
    vs, vinst = I.maxcut_batch(args.val, 512, 2048, 777)
    ref = reference_energies(vinst, 64, 4 * args.label_steps, seeds=[101, 102])
    targets = ref + 1e-3 * np.abs(ref)
    R, budget, check = 64, 3000, 25
    base, _, bbest, bwall = steps_to_target(vinst, R, budget, check, targets, seed=5)
    res = {"random": {"reached": int((base >= 0).sum()), "mean_steps": float(np.where(base >= 0, base, budget).mean()),
                      "wall_s": bwall}}
    best_key, best_score = None, None
    with gd.MLP(params) as m:
        for alpha in (0.3, 0.6, 0.9):
            for beta in (-1.0, 0.0, 1.0):
                st, _, _, wall = steps_to_target(vinst, R, budget, check, targets, m, alpha, beta, seed=5)
                score = float(np.where(st >= 0, st, budget).mean())
                res[f"a{alpha}_b{beta}"] = {"reached": int((st >= 0).sum()), "mean_steps": score, "wall_s": wall}
                log(f"alpha {alpha} beta {beta}: reached {(st >= 0).sum()}/{len(st)} mean steps {score:.0f}")
                if best_score is None or score < best_score:
                    best_key, best_score = (alpha, beta), score
    log(f"random start: reached {res['random']['reached']} mean steps {res['random']['mean_steps']:.0f}")
    meta = {"alpha": best_key[0], "beta": best_key[1], "feat_iters": FEAT_ITERS,
            "train_instances": int(len(sizes)), "train_spins": int(X.shape[0]), "epochs": args.epochs,
            "label_steps": args.label_steps, "final_loss": float(np.mean(curve[-50:])),
            "first_loss": float(np.mean(curve[:10])), "validation": res}
    with open(os.path.join(args.out, "proposal_meta.json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(json.dumps({k: meta[k] for k in ("alpha", "beta", "first_loss", "final_loss")}))


if __name__ == "__main__":
    main()
