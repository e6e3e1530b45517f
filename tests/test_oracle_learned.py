"""Pins of the learned-proposal oracle (oracle/learned.py) against facts fixed
outside it: published SplitMix64 outputs, central finite differences of the
loss, the closed form of Adam's first step, numpy's symmetric eigensolver on
matrices with a known gap, and the symmetries the definitions must have."""
import numpy as np
import pytest

from oracle import learned as L
from oracle import oracle as O
from paper_1807_00699_amd import inputs as I


def test_splitmix64_published_sequence():
    # SplitMix64 seeded with 0: the state advances by the golden gamma before
    # each mix, so the k-th output is mix(k * gamma); first three outputs:
    seq, state = [], 0
    for _ in range(3):
        seq.append(L.splitmix64(state))
        state = (state + 0x9E3779B97F4A7C15) & L.M64
    assert seq == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = L.uniform_array(np.arange(20000), 12345)
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01


def _toy(seed=0, M=40, K=3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((M, L.F))
    lab = np.where(rng.random(M) < 0.5, -1.0, 1.0)
    seg = np.array([0, 13, 27, M])
    p = rng.standard_normal(L.NPARAM) * 0.3
    return p, X, lab, seg


def test_loss_gradient_matches_central_differences():
    p, X, lab, seg = _toy()
    Lv, g = L.loss_and_grad(p, X, lab, seg)
    h = 1e-6
    fd = np.empty_like(g)
    for q in range(L.NPARAM):
        e = np.zeros(L.NPARAM)
        e[q] = h
        fd[q] = (L.loss_and_grad(p + e, X, lab, seg)[0] - L.loss_and_grad(p - e, X, lab, seg)[0]) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(g), np.abs(g - fd).max()


def test_loss_is_flip_invariant_and_minimal_at_labels():
    p, X, lab, seg = _toy(1)
    L1, _ = L.loss_and_grad(p, X, lab, seg)
    lab2 = lab.copy()
    lab2[seg[1]:seg[2]] *= -1            # flip one instance's labels
    L2, _ = L.loss_and_grad(p, X, lab2, seg)
    assert L1 == pytest.approx(L2, rel=1e-12)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(2)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = L.adam(p, g, np.zeros(50), np.zeros(50), 1, 0.01)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-9)


def test_block_power_finds_top_eigenspace_with_gap():
    # symmetric matrix with a planted top-8 spectrum well separated from the rest
    n = 60
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([np.linspace(3.0, 2.3, 8), rng.uniform(-1.5, 1.0, n - 8)])
    J = Q @ np.diag(lam) @ Q.T
    J = (J + J.T) / 2
    np.fill_diagonal(J, 0.0)      # the method ignores the diagonal: use the zero-diagonal matrix
    w, U = np.linalg.eigh(J)
    V, lv = L.block_power(J, 1.0, 300)
    top = U[:, np.argsort(-w)[:8]]
    assert np.linalg.norm(V @ V.T - top @ top.T) < 1e-8
    assert np.allclose(lv, np.sort(w)[::-1][:8], atol=1e-10)
    assert np.allclose(V.T @ V, np.eye(8), atol=1e-10)
    for k in range(8):                       # sign rule
        i = np.argmax(np.abs(V[:, k]))
        assert V[i, k] > 0


def test_features_definition_on_regular_graph():
    n = 50
    e, w, s_star = I.regular3_maxcut(n, 4)
    J = I.edges_to_dense(n, e, w).astype(np.float64)
    s = O.coupling_scale(J)
    f, V, lam = L.features(J, s, 40)
    assert f.shape == (n, L.F)
    assert np.allclose(f[:, 1], 1.0) and np.allclose(f[:, 19], 1.0)
    assert np.allclose(f[:, 18], 3.0 / s)
    assert np.allclose(f[:, 0], J.sum(1) / s)
    # converged: the Ritz pairs of J and of its gauge D J D are the top-8
    # eigenpairs of numpy's eigh, and the subspaces map by D
    w, U = np.linalg.eigh(J / s)
    top = U[:, np.argsort(-w)[:8]]
    V, lam = L.block_power(J, s, 3000)
    Jg = I.gauge(J.astype(np.float32), s_star).astype(np.float64)
    Vg, lg = L.block_power(Jg, s, 3000)
    assert np.allclose(lam, np.sort(w)[::-1][:8], atol=1e-9)
    assert np.allclose(lg, lam, atol=1e-9)
    D = np.diag(s_star.astype(np.float64))
    assert np.linalg.norm(V @ V.T - top @ top.T) < 1e-6
    assert np.linalg.norm(Vg @ Vg.T - D @ (V @ V.T) @ D) < 1e-6


def test_proposal_limits():
    m = np.tanh(np.linspace(-2, 2, 30))
    c = np.linspace(0.1, 0.9, 30)
    p1, e1 = L.propose(m, c, 3, 5, 99, amp=0.1, alpha=1.0, beta=0.0, eps0=0.1)
    assert np.allclose(p1, 0.1 * m[None, :]) and np.allclose(e1, 0.1)
    p0, e0 = L.propose(m, c, 3, 400, 99, amp=0.1, alpha=0.0, beta=1.0, eps0=0.1)
    assert np.abs(p0).max() < 0.1 and abs(p0.mean()) < 0.005
    assert np.allclose(e0, 0.1 * np.exp(c - 0.5))
