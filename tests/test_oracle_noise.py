"""Pins of the oracle's noise term D xi_i(t) of Eq. (main) (the regime of
Sec. 2: zero initial condition, noise seeds, gain rising from below).

The noise numbers are pinned to facts outside the oracle: SplitMix64's
published outputs, the standard normal law (moments, Kolmogorov-Smirnov),
independence between components and steps, and the exact variance of the
discrete Ornstein-Uhlenbeck recursion that the Euler and RK4 schemes reduce
to when J = 0, eps = 0 and the amplitudes are small enough for the cubic
term to vanish to working precision."""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_1807_00699_amd import inputs as I


def test_splitmix64_published_outputs():
    gamma = 0x9E3779B97F4A7C15
    seq = [O.splitmix64((k * gamma) & O.M64) for k in range(3)]
    assert seq == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def _first_increment(R, n, model, seed, t0=0, r0=0):
    """One step from Psi = 0 with J = 0, eps = 0, gamma = 0: the state after
    the step is exactly the noise increment D sqrt(dt) eta (dt f(0) = 0).
    With dt = 0.25 and D = 2 the increment is eta itself."""
    J = np.zeros((n, n))
    psi = np.zeros((R, n)) if model == "ising" else np.zeros((R, n, 2))
    p, _ = O.run(J, psi, model=model, steps=1, dt=0.25, eps=0.0, s=1.0, noise_D=2.0,
                 noise_seed=seed, t0=t0, r0=r0)
    return p


def test_noise_numbers_are_standard_normal_and_independent():
    z = _first_increment(200, 500, "xy", seed=7)
    re, im = z[..., 0].ravel(), z[..., 1].ravel()
    for v in (re, im):
        assert abs(v.mean()) < 5 / np.sqrt(v.size)
        assert abs(v.var() - 1.0) < 5 * np.sqrt(2.0 / v.size)
        assert abs(stats.kurtosis(v, fisher=False) - 3.0) < 5 * np.sqrt(24.0 / v.size)
        assert stats.kstest(v, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(re, im)[0, 1]) < 5 / np.sqrt(re.size)
    # the next step draws fresh numbers; so does another seed
    z1 = _first_increment(200, 500, "xy", seed=7, t0=1)
    z2 = _first_increment(200, 500, "xy", seed=8)
    for other in (z1, z2):
        c = np.corrcoef(re, other[..., 0].ravel())[0, 1]
        assert abs(c) < 5 / np.sqrt(re.size)
    # real mode draws the real part of the same pair
    zr = _first_increment(200, 500, "ising", seed=7)
    assert np.array_equal(zr, z[..., 0])


def test_noise_keys_are_global_step_and_trajectory():
    n, R = 12, 10
    J = I.dense_gaussian(n, 3)
    psi = I.psi0_complex(n, R, 4)
    kw = dict(model="xy", dt=0.05, eps=0.1, noise_D=0.3, noise_seed=11, integrator=O.RK4)
    full, gfull = O.run(J, psi, steps=6, **kw)
    # trajectories 4..7 alone, with r0 = 4, are an exact sub-problem
    sub, gsub = O.run(J, psi[4:8], steps=6, r0=4, **kw)
    assert np.array_equal(sub, full[4:8]) and np.array_equal(gsub, gfull[4:8])
    # 2 + 4 steps with t0 = 2 on the second call reproduce the 6-step run
    a, ga = O.run(J, psi, steps=2, **kw)
    b, gb = O.run(J, a, ga, steps=4, t0=2, **kw)
    assert np.array_equal(b, full) and np.array_equal(gb, gfull)
    # the increment is added after the deterministic step: with and without
    # noise the first step differs by exactly D sqrt(dt) eta(t=0)
    det, _ = O.run(J, psi, steps=1, **{**kw, "noise_D": 0.0})
    noisy, _ = O.run(J, psi, steps=1, **kw)
    eta = _first_increment(R, n, "xy", seed=11)
    assert np.allclose(noisy - det, 0.3 * np.sqrt(0.05) * eta, rtol=0, atol=1e-15)


@pytest.mark.parametrize("integrator", [O.EULER, O.RK4])
@pytest.mark.parametrize("model", ["ising", "xy"])
def test_linear_regime_variance_is_the_discrete_ou_value(model, integrator):
    """J = 0, eps = 0, gamma = 0, gamma_c = c: each component follows
    x_{k+1} = a x_k + D sqrt(dt) eta_k with a = 1 - c dt (Euler) or the RK4
    amplification 1 + z + z^2/2 + z^3/6 + z^4/24, z = -c dt, up to the cubic
    term (relative size Var(x) / c ~ 1e-7 here).  Hence
    Var(x_n) = D^2 dt (1 - a^(2n)) / (1 - a^2)."""
    n, R, steps, dt, c, D = 250, 400, 60, 0.1, 4.0, 1e-3
    J = np.zeros((n, n))
    psi = np.zeros((R, n)) if model == "ising" else np.zeros((R, n, 2))
    p, g = O.run(J, psi, model=model, steps=steps, dt=dt, eps=0.0, s=1.0, gamma_c=c,
                 noise_D=D, noise_seed=5, integrator=integrator)
    assert np.all(g == 0.0)
    z = -c * dt
    a = 1 + z if integrator == O.EULER else 1 + z + z * z / 2 + z**3 / 6 + z**4 / 24
    want = D * D * dt * (1 - a ** (2 * steps)) / (1 - a * a)
    comps = [p] if model == "ising" else [p[..., 0], p[..., 1]]
    for v in comps:
        m = v.size
        assert abs(v.var() / want - 1.0) < 5 * np.sqrt(2.0 / m), (v.var(), want)
    # the Euler and RK4 variances differ by more than the tolerance, so the
    # test tells the schemes apart
    if integrator == O.RK4:
        ae = 1 + z
        we = D * D * dt * (1 - ae ** (2 * steps)) / (1 - ae * ae)
        assert abs(we / want - 1.0) > 10 * np.sqrt(2.0 / p.size)


def test_zero_noise_is_the_deterministic_run():
    n, R = 10, 4
    J = I.dense_pm1(n, 2)
    x = I.psi0_real(n, R, 3)
    a, ga = O.run(J, x, model="ising", steps=30, dt=0.05)
    b, gb = O.run(J, x, model="ising", steps=30, dt=0.05, noise_D=0.0, noise_seed=99)
    assert np.array_equal(a, b) and np.array_equal(ga, gb)


def test_paper_regime_reaches_brute_force_ground_state():
    """Sec. 2 operating mode: Psi(0) = 0, noise seeds only, gain rising from
    below (gamma_c above the largest eigenvalue of J/s, so every mode decays
    until the gain has grown).  On the leading 20 x 20 block of the dense
    +-1 N = 64 instance every one of 64 noise seeds ends in a ground state of
    the brute-force enumeration."""
    J = I.dense_pm1(64, 1)[:20, :20].astype(np.float64)
    e_b, _ = O.brute_ising(J)
    s = O.coupling_scale(J)
    gc = np.linalg.eigvalsh(J / s).max() + 0.5
    x, _ = O.run(J, np.zeros((64, 20)), model="ising", steps=3000, dt=0.05, eps=0.1, gamma_c=gc,
                 noise_D=0.01, noise_seed=1)
    E = O.energy_ising(J, O.ising_spins(x))
    assert np.all(E == e_b)
