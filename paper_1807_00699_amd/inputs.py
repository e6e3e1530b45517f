"""Seeded synthetic inputs for the gain-dissipative (GD) solver.

This module is shared by the HIP path's tests/benchmark and by the FP64
oracle's tests.  It holds random-number plumbing and the shapes of the
workloads only: none of the method's arithmetic (no coupling scale, no rate
equation, no energy) lives here, so both sides stay independent.

Every generator draws in float64 from numpy's PCG64 stream keyed by
(seed, stream-id, ...) and rounds ONCE to the storage precision (float32).
Consumers must use the returned float32 arrays (the oracle widens them to
float64 exactly), so both sides integrate the same numbers.

Workload shapes follow the paper:
  * Eq. (h) couplings J (real symmetric, Sec. 1) with zero diagonal;
  * the 'dense' U[-10,10] and 'sparse' 3-regular matrices of Sec. 2;
  * dense +-1 Ising matrices, N(0,1/N) XY matrices, density-0.5 {-1,0,+1}
    matrices and batches of random 3-regular max-cut graphs as synthetic
    stand-ins for the Sec. 3 Max-Cut instances (the G-set files are not used).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "sym_from_upper", "dense_pm1", "dense_gaussian", "dense_uniform",
    "sparse_pm1", "regular3_edges", "regular3_maxcut", "regular3_uniform_bounds",
    "edges_to_dense", "even_sizes", "psi0_real", "psi0_complex",
    "planted_signs", "gauge", "edges_to_csr", "maxcut_batch", "gnp_edges", "gnp_maxcut",
]

# stream ids keep independent draws independent when seeds collide
_S_J, _S_PSI, _S_GRAPH, _S_SIZES, _S_PLANT, _S_W, _S_GNP = 11, 12, 13, 14, 15, 16, 17


def rng(seed: int, *stream: int) -> np.random.Generator:
    """PCG64 generator keyed by (seed, *stream); deterministic across hosts."""
    return np.random.default_rng([int(seed) & 0xFFFFFFFF, *[int(s) for s in stream]])


def sym_from_upper(upper: np.ndarray) -> np.ndarray:
    """Symmetric matrix from the strict upper triangle of `upper`; zero diagonal."""
    u = np.triu(upper, 1)
    return (u + u.T).astype(np.float32)


def dense_pm1(n: int, seed: int) -> np.ndarray:
    """Symmetric J, off-diagonal entries iid uniform on {-1,+1}, zero diagonal."""
    g = rng(seed, _S_J, n)
    up = np.where(g.random((n, n)) < 0.5, -1.0, 1.0)
    return sym_from_upper(up)


def dense_gaussian(n: int, seed: int) -> np.ndarray:
    """Symmetric J, off-diagonal entries iid N(0, 1/n) (rounded to float32)."""
    g = rng(seed, _S_J, n, 1)
    up = g.standard_normal((n, n)) / np.sqrt(n)
    return sym_from_upper(up)


def dense_uniform(n: int, seed: int, lo: float = -10.0, hi: float = 10.0) -> np.ndarray:
    """Symmetric J, off-diagonal entries iid U[lo, hi] (the paper's 'dense' XY matrices)."""
    g = rng(seed, _S_J, n, 2)
    up = g.uniform(lo, hi, (n, n))
    return sym_from_upper(up)


def sparse_pm1(n: int, seed: int, density: float = 0.5) -> np.ndarray:
    """Symmetric J in {-1,0,+1}: each pair i<j nonzero with prob. `density`,
    sign +-1 equiprobable; zero diagonal."""
    g = rng(seed, _S_J, n, 3)
    nz = g.random((n, n)) < density
    sg = np.where(g.random((n, n)) < 0.5, -1.0, 1.0)
    return sym_from_upper(nz * sg)


def regular3_edges(n: int, seed: int, max_tries: int = 10000) -> np.ndarray:
    """Uniform random 3-regular simple graph on n (even) nodes by the pairing
    (configuration) model with rejection of loops and multi-edges.
    Returns int32 edges [3n/2, 2] with i < j, sorted."""
    if n % 2 or n < 4:
        raise ValueError("3-regular graphs need an even n >= 4")
    g = rng(seed, _S_GRAPH, n)
    stubs = np.repeat(np.arange(n, dtype=np.int64), 3)
    for _ in range(max_tries):
        p = g.permutation(stubs).reshape(-1, 2)
        a, b = np.minimum(p[:, 0], p[:, 1]), np.maximum(p[:, 0], p[:, 1])
        if np.any(a == b):
            continue
        key = a * n + b
        if np.unique(key).size != key.size:
            continue
        order = np.argsort(key)
        return np.stack([a[order], b[order]], 1).astype(np.int32)
    raise RuntimeError("pairing model did not produce a simple graph")


def edges_to_dense(n: int, edges: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Dense symmetric float32 matrix with J[i,j] = J[j,i] = w[e] on edge e."""
    J = np.zeros((n, n), np.float64)
    J[edges[:, 0], edges[:, 1]] = w
    J[edges[:, 1], edges[:, 0]] = w
    return J.astype(np.float32)


def planted_signs(n: int, seed: int) -> np.ndarray:
    """Random +-1 vector s* (int8)."""
    g = rng(seed, _S_PLANT, n)
    return np.where(g.random(n) < 0.5, -1, 1).astype(np.int8)


def gauge(J: np.ndarray, d: np.ndarray) -> np.ndarray:
    """J_ij -> d_i J_ij d_j for a +-1 vector d (exact sign flips)."""
    d = d.astype(np.float32)
    return (J * d[:, None] * d[None, :]).astype(np.float32)


def regular3_maxcut(n: int, seed: int):
    """Max-cut form of a random 3-regular graph, J_ij = -1 on edges, then the
    gauge J_ij -> J_ij s*_i s*_j with a random s*.  Returns (edges, w, s*)
    with w the per-edge coupling (float32 +-1)."""
    e = regular3_edges(n, seed)
    s = planted_signs(n, seed)
    w = (-1.0 * s[e[:, 0]].astype(np.float64) * s[e[:, 1]]).astype(np.float32)
    return e, w, s


def regular3_uniform_bounds(n: int, seed: int):
    """The paper's 'sparse' matrices: each node joined to exactly three others,
    each coupling drawn from U(a, b) with bounds a != b taken at random from
    {-10,-3,3,10}.  Returns dense float32 J."""
    e = regular3_edges(n, seed)
    g = rng(seed, _S_W, n)
    vals = np.array([-10.0, -3.0, 3.0, 10.0])
    ab = np.stack([g.permutation(vals)[:2] for _ in range(e.shape[0])])
    lo, hi = ab.min(1), ab.max(1)
    w = g.uniform(lo, hi)
    return edges_to_dense(n, e, w)


def even_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """`count` even sizes drawn uniformly from the even integers in [lo, hi]."""
    g = rng(seed, _S_SIZES, count)
    return (2 * g.integers(lo // 2 + (lo % 2), hi // 2 + 1, count)).astype(np.int32)


def psi0_real(n: int, R: int, seed: int, amp: float = 0.1) -> np.ndarray:
    """Real initial amplitudes, [R][n] float32, iid U(-amp, amp)."""
    g = rng(seed, _S_PSI, n, R)
    return g.uniform(-amp, amp, (R, n)).astype(np.float32)


def psi0_complex(n: int, R: int, seed: int, amp: float = 0.1) -> np.ndarray:
    """Complex initial amplitudes amp*exp(i*phi), phi ~ U[0, 2pi);
    returned as [R][n][2] float32 (re, im)."""
    g = rng(seed, _S_PSI, n, R, 1)
    phi = g.uniform(0.0, 2.0 * np.pi, (R, n))
    out = np.empty((R, n, 2), np.float64)
    out[..., 0] = amp * np.cos(phi)
    out[..., 1] = amp * np.sin(phi)
    return out.astype(np.float32)


def edges_to_csr(n: int, edges: np.ndarray, w: np.ndarray) -> dict:
    """Symmetric CSR (both directions of every edge, columns sorted) as the
    dict accepted by the batched solver: n, row_ptr, col, val."""
    rows = np.concatenate([edges, edges[:, ::-1]]).astype(np.int64)
    vals = np.concatenate([w, w]).astype(np.float32)
    order = np.lexsort((rows[:, 1], rows[:, 0]))
    rows, vals = rows[order], vals[order]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows[:, 0] + 1, 1)
    return dict(n=int(n), row_ptr=np.cumsum(rp).astype(np.int32), col=rows[:, 1].astype(np.int32),
                val=vals)


def maxcut_batch(count: int, lo: int, hi: int, seed: int):
    """`count` random 3-regular max-cut instances (J = -1 on edges, gauged by a
    random s*) with even sizes uniform in [lo, hi].  Instance k uses graph seed
    1000 * seed + k.  Returns (sizes, list of CSR dicts)."""
    sizes = even_sizes(count, lo, hi, seed)
    insts = []
    for k, n in enumerate(sizes):
        e, w, _ = regular3_maxcut(int(n), 1000 * seed + k)
        insts.append(edges_to_csr(int(n), e, w))
    return sizes, insts


def gnp_edges(n: int, p: float, seed: int) -> np.ndarray:
    """Erdos-Renyi G(n, p): each pair i < j is an edge independently with
    probability p.  Returns int32 edges [m, 2] with i < j, sorted."""
    g = rng(seed, _S_GNP, n)
    iu, ju = np.triu_indices(n, 1)
    keep = g.random(iu.size) < p
    return np.stack([iu[keep], ju[keep]], 1).astype(np.int32)


def gnp_maxcut(n: int, p: float, seed: int, signed: bool = False):
    """Max-cut instance on G(n, p) with weights w = 1 (or +-1 equiprobable when
    `signed`), in Ising form J_ij = -w_ij (minimising Eq. (h) maximises the
    cut: cut = W/2 - E/4 with W = sum_{i<j} w_ij).  Returns (edges, w) with w
    float32; a synthetic stand-in shaped like the paper's N = 800 Max-Cut
    benchmarks (Sec. 3), not any published instance."""
    e = gnp_edges(n, p, seed)
    if signed:
        g = rng(seed, _S_GNP, n, 1)
        w = np.where(g.random(e.shape[0]) < 0.5, -1.0, 1.0)
    else:
        w = np.ones(e.shape[0])
    return e, w.astype(np.float32)
