"""FP64 oracle of the learned proposal (features -> MLP -> initial amplitudes
and per-spin gain rates).  TEST INFRASTRUCTURE ONLY (same rules as
oracle.py): plain numpy, float64, written from the definitions below; it
shares no code with the HIP library.

The paper suggests site-dependent gain-adjustment rates eps_i(t) as an
extension (Sec. 3) and notes that the linear (sub-threshold) phase of the
dynamics amplifies the leading eigenvectors of the coupling matrix (the gain
rises from below, Sec. 1).  The learned proposal therefore reads spectral
features of J and emits, per spin, a predicted sign of a low-energy state
(used to bias the initial amplitudes) and a confidence (used to set eps_i).

Definitions (these are the project's own; both sides implement them):

* SplitMix64 (Steele, Lea, Flood 2014): z += 0x9E3779B97F4A7C15;
  z = (z ^ z>>30) * 0xBF58476D1CE4E5B9; z = (z ^ z>>27) * 0x94D049BB133111EB;
  return z ^ z>>31.  uniform(ctr, key) = (splitmix64(key ^ splitmix64(ctr)) >> 11) * 2^-53.
* Features of an instance (J symmetric, zero diagonal, s = coupling scale):
  A = J/s + c I with c = max_i sum_j |J_ij| / s (Gershgorin: A is PSD);
  V0[i][k] = 2 uniform(8 i + k, FEAT_KEY) - 1, k < 8;
  repeat `iters` times: W = A V, V = W L^-T with L L^T = W^T W (Cholesky);
  Rayleigh-Ritz: H = V^T A V = U diag(theta) U^T (descending), V <- V U,
  lambda_k = theta_k - c (eigenvalues of J/s);
  sign fix: the entry of largest magnitude of each column is positive (ties:
  lowest index).  Per spin i (F = 20):
  f0 = sum_j J_ij / s, f1 = deg_i / mean degree, f2+k = sqrt(n) V[i][k],
  f10+k = n lambda_k V[i][k]^2, f18 = sum_j |J_ij| / s, f19 = 1.
* MLP 20 -> 64 -> 64 -> 2, ReLU hidden layers: h1 = relu(f W1 + b1),
  h2 = relu(h1 W2 + b2), o = h2 W3 + b3; m = tanh(o0), c = sigmoid(o1).
  Parameter vector layout: W1 [20][64], b1 [64], W2 [64][64], b2 [64],
  W3 [64][2], b3 [2] (5634 floats).
* Loss over a minibatch of instances with labels s_i in {-1, +1} (a low
  energy state found by the solver), M spins in total:
  sigma_k = +1 if sum_{i in k} (m_i - s_i)^2 <= sum_{i in k} (m_i + s_i)^2 else -1
  (the labels are defined up to the global flip of Eq. (h));
  y_i = 1 if m_i sigma_k s_i > 0 else 0 (taken as a constant);
  L = (1/M) sum_i [ (m_i - sigma_k s_i)^2 + LAMBDA_C * BCE(c_i, y_i) ].
* Adam (Kingma & Ba 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and
  bias correction, step t starting at 1.
* Proposal for trajectory r of an instance: psi0_ir = a (alpha m_i + (1 - alpha)
  (2 uniform(ctr, seed) - 1)), ctr = (k * 2^20 + r) * 2^16 + i, and
  eps_i = eps0 exp(beta (c_i - 1/2)).
"""
from __future__ import annotations

import numpy as np

F = 20
H = 64
NOUT = 2
NPARAM = F * H + H + H * H + H + H * NOUT + NOUT
FEAT_KEY = 0x5EED5EED
LAMBDA_C = 0.5
M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    x = (x + 0x9E3779B97F4A7C15) & M64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & M64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & M64
    return x ^ (x >> 31)


def uniform(ctr: int, key: int) -> float:
    return (splitmix64((key ^ splitmix64(ctr)) & M64) >> 11) * (1.0 / 9007199254740992.0)


def uniform_array(ctrs, key: int) -> np.ndarray:
    return np.array([uniform(int(c), key) for c in np.ravel(ctrs)]).reshape(np.shape(ctrs))


# ---------------------------------------------------------------- features

def block_power(J, s: float, iters: int):
    """Shifted block power iteration with Cholesky-QR, then Rayleigh-Ritz and
    sign fixing.  Returns (V [n][8], lambda [8]) for J/s."""
    J = np.asarray(J, np.float64).copy()
    np.fill_diagonal(J, 0.0)
    n = J.shape[0]
    A = J / s
    c = np.abs(A).sum(1).max()
    A = A + c * np.eye(n)
    ctr = 8 * np.arange(n)[:, None] + np.arange(8)[None, :]
    V = 2.0 * uniform_array(ctr, FEAT_KEY) - 1.0
    for _ in range(iters):
        W = A @ V
        L = np.linalg.cholesky(W.T @ W)
        V = np.linalg.solve(L, W.T).T          # W L^-T
    Hm = V.T @ A @ V
    th, U = np.linalg.eigh((Hm + Hm.T) / 2)
    order = np.argsort(-th, kind="stable")
    th, U = th[order], U[:, order]
    V = V @ U
    for k in range(8):
        i = int(np.argmax(np.abs(V[:, k])))   # first index of the largest magnitude
        if V[i, k] < 0:
            V[:, k] = -V[:, k]
    return V, th - c


def features(J, s: float, iters: int):
    J = np.asarray(J, np.float64).copy()
    np.fill_diagonal(J, 0.0)
    n = J.shape[0]
    V, lam = block_power(J, s, iters)
    deg = (J != 0).sum(1).astype(np.float64)
    f = np.zeros((n, F))
    f[:, 0] = J.sum(1) / s
    f[:, 1] = deg / max(deg.mean(), 1e-300)
    f[:, 2:10] = np.sqrt(n) * V
    f[:, 10:18] = n * lam[None, :] * V**2
    f[:, 18] = np.abs(J).sum(1) / s
    f[:, 19] = 1.0
    return f, V, lam


# ---------------------------------------------------------------- MLP

def unpack(p):
    p = np.asarray(p, np.float64)
    o = 0
    out = []
    for shape in ((F, H), (H,), (H, H), (H,), (H, NOUT), (NOUT,)):
        size = int(np.prod(shape))
        out.append(p[o:o + size].reshape(shape))
        o += size
    return out


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    o = h2 @ W3 + b3
    return o, (X, z1, h1, z2, h2)


def heads(o):
    return np.tanh(o[:, 0]), 1.0 / (1.0 + np.exp(-o[:, 1]))


def loss_and_grad(p, X, labels, seg):
    """seg: instance boundaries [K+1] into the rows of X.  Returns (L, grad)."""
    o, (X, z1, h1, z2, h2) = forward(p, X)
    m, c = heads(o)
    s = np.asarray(labels, np.float64)
    M = X.shape[0]
    sigma = np.empty(M)
    for k in range(len(seg) - 1):
        a, b = seg[k], seg[k + 1]
        ep = np.sum((m[a:b] - s[a:b]) ** 2)
        em = np.sum((m[a:b] + s[a:b]) ** 2)
        sigma[a:b] = 1.0 if ep <= em else -1.0
    t = sigma * s
    y = (m * t > 0).astype(np.float64)
    o1 = o[:, 1]
    bce = np.maximum(o1, 0.0) - y * o1 + np.log1p(np.exp(-np.abs(o1)))   # = BCE(sigmoid(o1), y)
    L = (np.sum((m - t) ** 2) + LAMBDA_C * np.sum(bce)) / M
    do = np.zeros((M, NOUT))
    do[:, 0] = 2.0 * (m - t) * (1.0 - m * m) / M
    do[:, 1] = LAMBDA_C * (c - y) / M
    W1, b1, W2, b2, W3, b3 = unpack(p)
    gW3 = h2.T @ do
    gb3 = do.sum(0)
    dh2 = (do @ W3.T) * (z2 > 0)
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ W2.T) * (z1 > 0)
    gW1 = X.T @ dh1
    gb1 = dh1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam(p, g, mom, vel, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    mom = b1 * mom + (1 - b1) * g
    vel = b2 * vel + (1 - b2) * g * g
    mh = mom / (1 - b1**t)
    vh = vel / (1 - b2**t)
    return p - lr * mh / (np.sqrt(vh) + eps), mom, vel


def propose(m, c, k, R, seed, amp, alpha, beta, eps0):
    n = len(m)
    ctr = ((k * (1 << 20) + np.arange(R)[:, None]) * (1 << 16) + np.arange(n)[None, :])
    u = uniform_array(ctr, seed)
    psi0 = amp * (alpha * np.asarray(m)[None, :] + (1 - alpha) * (2 * u - 1))
    eps = eps0 * np.exp(beta * (np.asarray(c) - 0.5))
    return psi0, eps
