"""Seeded generators: determinism and the structural properties of the
workloads (symmetric J with zero diagonal, densities, 3-regularity, gauge)."""
import numpy as np

from paper_1807_00699_amd import inputs as I


def _sym0(J):
    return np.array_equal(J, J.T) and np.all(np.diag(J) == 0)


def test_determinism_and_dtype():
    for f in (I.dense_pm1, I.dense_gaussian, I.dense_uniform, I.sparse_pm1):
        a, b, c = f(33, 5), f(33, 5), f(33, 6)
        assert a.dtype == np.float32 and np.array_equal(a, b) and not np.array_equal(a, c)
        assert _sym0(a)
    assert np.array_equal(I.psi0_real(10, 3, 1), I.psi0_real(10, 3, 1))
    assert np.array_equal(I.psi0_complex(10, 3, 1), I.psi0_complex(10, 3, 1))


def test_value_sets_and_moments():
    J = I.dense_pm1(200, 1)
    off = J[~np.eye(200, dtype=bool)]
    assert set(np.unique(off)) == {-1.0, 1.0} and abs(off.mean()) < 0.02
    G = I.dense_gaussian(400, 1)
    offg = G[~np.eye(400, dtype=bool)].astype(np.float64)
    assert abs(offg.var() * 400 - 1) < 0.02
    S = I.sparse_pm1(400, 2)
    offs = S[np.triu_indices(400, 1)]
    assert set(np.unique(offs)) <= {-1.0, 0.0, 1.0}
    assert abs((offs != 0).mean() - 0.5) < 0.01 and abs(offs.mean()) < 0.01
    U = I.dense_uniform(100, 3)
    assert U.min() >= -10 and U.max() <= 10


def test_initial_amplitudes():
    x = I.psi0_real(100, 50, 2)
    assert x.shape == (50, 100) and np.abs(x).max() < 0.1
    p = I.psi0_complex(100, 50, 2)
    assert p.shape == (50, 100, 2)
    assert np.allclose(np.hypot(p[..., 0], p[..., 1]), 0.1, rtol=1e-6)


def test_regular3_graphs_and_gauge():
    for n in (4, 50, 302):
        e = I.regular3_edges(n, 7)
        assert e.shape == (3 * n // 2, 2) and np.all(e[:, 0] < e[:, 1])
        deg = np.bincount(e.ravel(), minlength=n)
        assert np.all(deg == 3)
        assert np.unique(e[:, 0].astype(np.int64) * n + e[:, 1]).size == e.shape[0]
    e, w, s = I.regular3_maxcut(100, 3)
    J = I.edges_to_dense(100, e, w)
    assert _sym0(J) and np.all((np.abs(J) > 0).sum(1) == 3)
    # undoing the gauge recovers the all -1 max-cut couplings
    Jb = I.gauge(J, s)
    assert np.array_equal(Jb[np.abs(J) > 0], -np.ones(300, np.float32))
    P = I.regular3_uniform_bounds(50, 4)
    assert _sym0(P) and np.all((np.abs(P) > 0).sum(1) == 3) and np.abs(P).max() <= 10


def test_even_sizes():
    n = I.even_sizes(256, 50, 2000, 1)
    assert n.shape == (256,) and np.all(n % 2 == 0) and n.min() >= 50 and n.max() <= 2000
    assert n.min() < 300 and n.max() > 1700


def test_gnp_maxcut_shape_density_and_cut_identity():
    n, p = 800, 0.06
    e, w = I.gnp_maxcut(n, p, 3)
    m = e.shape[0]
    pairs = n * (n - 1) // 2
    assert abs(m / pairs - p) < 5 * np.sqrt(p * (1 - p) / pairs)
    assert np.all(e[:, 0] < e[:, 1]) and np.unique(e[:, 0] * n + e[:, 1]).size == m
    assert np.all(w == 1.0)
    es, ws = I.gnp_maxcut(n, p, 3, signed=True)
    assert np.array_equal(es, e) and set(np.unique(ws)) == {-1.0, 1.0}
    # Ising form J = -w: cut(s) = W/2 - E(s)/4 for a random partition
    J = I.edges_to_dense(n, es, -ws).astype(np.float64)
    s = np.where(np.random.default_rng(0).random(n) < 0.5, -1.0, 1.0)
    E = -s @ J @ s
    cut = sum(ws[k] for k in range(m) if s[es[k, 0]] != s[es[k, 1]])
    assert np.isclose(cut, ws.sum() / 2 - E / 4)
