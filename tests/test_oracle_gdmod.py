"""Pins of the oracle's GD-mod algorithm (Sec. 1: Delta_ij = gamma_i + gamma_j,
couplings adapted by Eq. (gamma2)), against facts fixed outside it: the
closed form of the coupling relaxation when amplitudes and gains are frozen,
the plain GD oracle when the couplings are frozen, exact symmetry of K, the
fixed point Delta_ij K_ij = J_ij with the Eq. (pth) relation, and brute force."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_00699_amd import inputs as I


def test_coupling_relaxation_closed_form():
    """Psi = 0 stays 0 and eps = 0 freezes gamma, so each K_ij follows
    K_{k+1} = (1 - dt eps_hat D) K_k + dt eps_hat J with D = gamma_i + gamma_j:
    K_k = J/D + (K_0 - J/D) (1 - dt eps_hat D)^k."""
    n, R, steps, dt, eh = 9, 3, 37, 0.05, 0.7
    rng = np.random.default_rng(1)
    J = I.dense_uniform(n, 2).astype(np.float64)
    g0 = rng.uniform(0.2, 1.5, (R, n))
    K0 = rng.normal(size=(R, n, n))
    K0 = K0 + K0.transpose(0, 2, 1)
    for r in range(R):
        np.fill_diagonal(K0[r], 0.0)
    x, g, K = O.run_mod(J, np.zeros((R, n)), g0, K0, model="ising", steps=steps, dt=dt, eps=0.0,
                        eps_hat=eh, s=1.0)
    assert np.all(x == 0.0) and np.array_equal(g, g0)
    D = g0[:, :, None] + g0[:, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        want = J[None] / D + (K0 - J[None] / D) * (1 - dt * eh * D) ** steps
    off = ~np.eye(n, dtype=bool)
    assert np.allclose(K[:, off], want[:, off], rtol=1e-12, atol=1e-12)
    assert np.all(K[:, ~off] == 0.0)


@pytest.mark.parametrize("model", ["ising", "xy"])
def test_frozen_couplings_reduce_to_gd_with_scaled_matrix(model):
    """eps_hat = 0 keeps K = J and eps = 0 keeps gamma_i = g0 for all i, so
    the coupling is (2 g0) J Psi / s: plain GD with s' = s / (2 g0)."""
    n, R, g0 = 14, 4, 0.35
    J = I.dense_gaussian(n, 3).astype(np.float64)
    s = O.coupling_scale(J)
    psi = I.psi0_real(n, R, 4) if model == "ising" else I.psi0_complex(n, R, 4)
    gam = np.full((R, n), g0)
    a, ga, K = O.run_mod(J, psi, gam, model=model, steps=300, dt=0.02, eps=0.0, eps_hat=0.0, s=s,
                         gamma_c=0.5)
    b, gb = O.run(J, psi, gam, model=model, steps=300, dt=0.02, eps=0.0, s=s / (2 * g0),
                  gamma_c=0.5)
    assert np.abs(a - b).max() < 1e-12 * max(1.0, np.abs(b).max())
    assert np.array_equal(ga, gb)
    Jz = J.copy()
    np.fill_diagonal(Jz, 0.0)
    assert np.array_equal(K, np.repeat(Jz[None], R, 0))


def _gamma_c(J):
    # GD-mod needs positive gains (Delta_ij > 0; with Delta_ij < 0 Eq. (gamma2)
    # grows K exponentially).  At a fixed point gamma_i = gamma_c + rho_th -
    # s_i (J s)_i / s, so gamma_c = max_i sum_j |J_ij| / s keeps every gain
    # >= rho_th.
    Jz = np.asarray(J, np.float64).copy()
    np.fill_diagonal(Jz, 0.0)
    return float(np.abs(Jz).sum(1).max() / O.coupling_scale(Jz))


@pytest.mark.slow
def test_symmetry_and_fixed_point():
    """K stays exactly symmetric; at convergence Delta_ij K_ij = J_ij and the
    Eq. (pth) relation of plain GD holds: gamma_i - gamma_c = rho_th -
    s_i (J s)_i / s, summing to H(s)/s + N rho_th."""
    n, R = 16, 4
    J = I.dense_pm1(n, 6).astype(np.float64)
    s = O.coupling_scale(J)
    gc = _gamma_c(J)
    x, g, K = O.run_mod(J, I.psi0_real(n, R, 6), model="ising", steps=20000, dt=0.05, eps=0.1,
                        eps_hat=0.2, gamma_c=gc)
    assert np.array_equal(K, K.transpose(0, 2, 1))
    assert np.abs(x**2 - 1.0).max() < 1e-6
    assert g.min() >= 1.0 - 1e-9
    D = g[:, :, None] + g[:, None, :]
    off = ~np.eye(n, dtype=bool)
    assert np.abs((D * K - J[None])[:, off]).max() < 1e-6
    sp = O.ising_spins(x).astype(np.float64)
    local = 1.0 - sp * (sp @ J.T) / s
    assert np.abs(g - gc - local).max() < 1e-6
    H = O.energy_ising(J, sp.astype(np.int8)).astype(np.float64)
    assert np.allclose((g - gc).sum(1) - n, H / s, rtol=0, atol=1e-5)


def test_gdmod_reaches_brute_force_ground_state_n20():
    J = I.dense_pm1(64, 1)[:20, :20].astype(np.float64)
    e_b, _ = O.brute_ising(J)
    x, _, _ = O.run_mod(J, I.psi0_real(20, 32, 3), model="ising", steps=3000, dt=0.05, eps=0.1,
                        eps_hat=0.2, gamma_c=_gamma_c(J))
    E = O.energy_ising(J, O.ising_spins(x))
    assert E.min() == e_b
