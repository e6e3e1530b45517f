"""Learned proposal on the GPU (feature kernel, MLP forward/backward/Adam,
FP16 inference, proposal) against the FP64 oracle of oracle/learned.py.

Tolerances: features after 30 FP32 block-power iterations vs the FP64
iteration: Ritz values 1e-4 relative, 8-dimensional subspaces (projectors)
1e-3, single vectors only where the Ritz value is separated from its
neighbours; MLP FP32 forward 1e-4 absolute at O(1) outputs; gradients 1e-4
relative in norm; FP16 inference 3e-2 relative to the output scale.
"""
import os

import numpy as np
import pytest

from oracle import learned as L
from oracle import oracle as O
from paper_1807_00699_amd import gd
from paper_1807_00699_amd import inputs as I

pytestmark = pytest.mark.gpu


def _batch(sizes, seed):
    insts, dense = [], []
    for k, n in enumerate(sizes):
        e, w, _ = I.regular3_maxcut(int(n), seed + k)
        dense.append(I.edges_to_dense(int(n), e, w))
        insts.append(dict(n=int(n), J=dense[-1]))
    return insts, dense


def test_features_match_oracle():
    sizes = [64, 100, 250, 1000]
    insts, dense = _batch(sizes, 3)
    with gd.BatchSolver(insts) as B:
        f, lam, vec = gd.gd_features(B.h, sum(sizes), len(sizes), 30)
    off = 0
    for k, J in enumerate(dense):
        n = sizes[k]
        s = O.coupling_scale(J)
        fo, Vo, lo = L.features(J, s, 30)
        fg, Vg = f[off:off + n], vec[off:off + n].astype(np.float64)
        off += n
        assert np.allclose(lam[k], lo, rtol=1e-4, atol=1e-5), (lam[k], lo)
        assert np.linalg.norm(Vg @ Vg.T - Vo @ Vo.T) < 1e-3
        for c in (0, 1, 18, 19):
            assert np.allclose(fg[:, c], fo[:, c], atol=1e-5)
        for q in range(8):
            gap = min([abs(lo[q] - lo[p]) for p in range(8) if p != q])
            if gap > 0.02:
                assert np.abs(Vg[:, q] - Vo[:, q]).max() < 1e-3, (k, q)
                assert np.abs(fg[:, 2 + q] - fo[:, 2 + q]).max() < 1e-3 * np.sqrt(n)


def _toy(seed=0, M=3000, K=5):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((M, L.F)).astype(np.float32)
    lab = np.where(rng.random(M) < 0.5, -1.0, 1.0).astype(np.float32)
    seg = np.sort(np.concatenate([[0, M], rng.choice(np.arange(1, M), K - 1, replace=False)])).astype(np.int32)
    p = (rng.standard_normal(L.NPARAM) * 0.2).astype(np.float32)
    return p, X, lab, seg


def test_mlp_forward_gradient_and_adam_match_oracle():
    p, X, lab, seg = _toy()
    with gd.MLP(p) as m:
        out = m.forward(X)
        oo, _ = L.forward(p.astype(np.float64), X.astype(np.float64))
        assert np.abs(out - oo).max() < 1e-4 * max(1.0, np.abs(oo).max())
        o16 = m.forward(X, fp16=True)
        assert np.abs(o16 - oo).max() < 3e-2 * max(1.0, np.abs(oo).max())
        loss, g = m.train_step(X, lab, seg, 0.0, want_grad=True)
        Lo, go = L.loss_and_grad(p.astype(np.float64), X.astype(np.float64), lab.astype(np.float64), seg)
        assert loss == pytest.approx(Lo, rel=1e-5)
        assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
        assert np.array_equal(m.params, p)          # lr = 0 leaves the parameters
        lr = 1e-3
        m.train_step(X, lab, seg, lr)
        p1, _, _ = L.adam(p.astype(np.float64), go, np.zeros(L.NPARAM), np.zeros(L.NPARAM), 1, lr)
        big = np.abs(go) > 1e-3 * np.abs(go).max()
        assert np.abs(m.params - p1)[big].max() < 1e-6


@pytest.mark.parametrize("M,K", [(7, 2), (33, 3), (64, 1)])
def test_mlp_gradient_on_small_and_ragged_batches(M, K):
    """The training kernel takes 32 rows per wave: a batch smaller than one
    tile, one row past a tile, and exactly two tiles."""
    p, X, lab, seg = _toy(seed=M, M=M, K=K)
    with gd.MLP(p) as m:
        loss, g = m.train_step(X, lab, seg, 0.0, want_grad=True)
        Lo, go = L.loss_and_grad(p.astype(np.float64), X.astype(np.float64), lab.astype(np.float64), seg)
        assert loss == pytest.approx(Lo, rel=1e-5)
        assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
        # the same bits again (fixed-order sums)
        loss2, g2 = m.train_step(X, lab, seg, 0.0, want_grad=True)
        assert loss2 == loss and np.array_equal(g2, g)


def test_mlp_device_pointer_calls_match_host_calls():
    """GD_F_DEVICE_PTRS handle (device X, labels, outputs and parameters):
    the same outputs, losses and trained parameters as the host handle."""
    import torch

    p, X, lab, seg = _toy()
    pd = torch.from_numpy(p).cuda()
    Xd = torch.from_numpy(X).cuda()
    Ld = torch.from_numpy(lab).cuda()
    od = torch.empty((X.shape[0], 2), dtype=torch.float32, device="cuda")
    with gd.MLP(p) as mh, gd.MLP(pd, device=True) as md:
        for fp16 in (False, True):
            md.forward_device(Xd, od, fp16)
            assert np.array_equal(od.cpu().numpy(), mh.forward(X, fp16=fp16))
        # the FP16 kernel reads feature rows as 16-byte words: a device X off
        # that alignment is refused (the FP32 kernel takes it)
        buf = torch.zeros(X.size + 1, dtype=torch.float32, device="cuda")
        buf[1:] = Xd.reshape(-1)
        Xm = buf[1:].view(X.shape)
        with pytest.raises(gd.GDError) as ei:
            md.forward_device(Xm, od, True)
        assert ei.value.code == gd.GD_E_INVALID_ARG
        md.forward_device(Xm, od, False)
        assert np.array_equal(od.cpu().numpy(), mh.forward(X, fp16=False))
        for _ in range(3):
            lh = mh.train_step(X, lab, seg, 1e-3)
            ld = md.train_step_device(Xd, Ld, seg, 1e-3)
            assert lh == ld
        md.forward_device(Xd, od)
        assert np.array_equal(od.cpu().numpy(), mh.forward(X))
        with pytest.raises(gd.GDError):
            md.params


def test_training_steps_reduce_loss_on_learnable_labels():
    sizes = [128, 200, 256, 300]
    insts, dense = _batch(sizes, 9)
    with gd.BatchSolver(insts) as B:
        f, lam, vec = gd.gd_features(B.h, sum(sizes), len(sizes), 30)
    # labels: sign of the leading Ritz vector (a function of the features)
    lab = np.where(vec[:, 0] >= 0, 1.0, -1.0).astype(np.float32)
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    with gd.MLP(seed=1) as m:
        first = m.train_step(f, lab, seg, 0.0)
        for _ in range(300):
            m.train_step(f, lab, seg, 3e-3)
        last = m.train_step(f, lab, seg, 0.0)
    assert last < 0.5 * first, (first, last)


def test_propose_writes_formula_state_and_eps():
    sizes = [64, 130]
    R = 6
    insts, dense = _batch(sizes, 21)
    p = _toy(2)[0]
    alpha, beta, seed = 0.6, 0.8, 7
    with gd.BatchSolver(insts, dt=0.05, eps=0.1, init_amp=0.1) as B, gd.MLP(p) as m:
        f, _, _ = gd.gd_features(B.h, sum(sizes), len(sizes), 30)
        o16 = m.forward(f, fp16=True)
        gd.gd_propose(B.h, m, R, 30, alpha, beta, seed)
        B.R = R
        x0, g0, _ = B.state()
        B.run(1)
        x1, g1, _ = B.state()
    mm = np.tanh(o16[:, 0].astype(np.float64))
    cc = 1.0 / (1.0 + np.exp(-o16[:, 1].astype(np.float64)))
    off = 0
    for k, n in enumerate(sizes):
        psi, eps = L.propose(mm[off:off + n], cc[off:off + n], k, R, seed, 0.1, alpha, beta, 0.1)
        xk = B.split(x0)[k]
        assert np.abs(xk - psi).max() < 2e-6 * 0.1 + 1e-7
        # one Euler step with the proposed per-spin eps: gamma_1 = dt eps_i (1 - x^2)
        gk = B.split(g1)[k]
        assert np.allclose(gk, 0.05 * eps[None, :] * (1.0 - xk.astype(np.float64) ** 2), rtol=1e-5, atol=1e-8)
        off += n
    assert np.all(g0 == 0.0)


def test_trained_proposal_beats_random_start_on_held_out_instances():
    """A/B on 64 fresh instances (seed never used in training or validation),
    N even in [512, 2048], R = 64, budget 3000 Euler steps, checks every 25:
    steps until the best energy is within 0.1% of the best-known energy
    (best of two 12000-step random-start runs).  The random-start solver
    scores both arms with the same energy path."""
    import json
    from paper_1807_00699_amd import train_proposal as T

    here = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1807_00699_amd")
    params = np.load(os.path.join(here, "proposal_weights.npy"))
    meta = json.load(open(os.path.join(here, "proposal_meta.json")))
    sizes, insts = I.maxcut_batch(64, 512, 2048, 888)
    ref = T.reference_energies(insts, 64, 12000, seeds=[201, 202])
    targets = ref + 1e-3 * np.abs(ref)
    budget, check = 3000, 25
    base, _, bbest, _ = T.steps_to_target(insts, 64, budget, check, targets, seed=9)
    with gd.MLP(params) as m:
        lrn, _, lbest, _ = T.steps_to_target(insts, 64, budget, check, targets, m, meta["alpha"],
                                             meta["beta"], seed=9)
    b_reached, l_reached = int((base >= 0).sum()), int((lrn >= 0).sum())
    b_mean = float(np.where(base >= 0, base, budget).mean())
    l_mean = float(np.where(lrn >= 0, lrn, budget).mean())
    print(f"random start: {b_reached}/64 reached, mean steps {b_mean:.0f}; "
          f"learned start: {l_reached}/64 reached, mean steps {l_mean:.0f}")
    assert l_reached >= 58 and l_reached > b_reached
    assert l_mean < 0.5 * b_mean
