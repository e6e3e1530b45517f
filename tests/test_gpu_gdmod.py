"""GPU parity of the GD-mod step (Sec. 1: Delta_ij = gamma_i + gamma_j,
per-trajectory couplings K adapted by Eq. (gamma2), explicit Euler) against
the FP64 oracle (oracle.run_mod) on the same seeded inputs.

Bar: per trajectory, max-norm relative error of Psi, gamma and K <= 1e-4 at
steps {1, 10, 50, 100, 200}.  gamma_c sits at max_i sum_j |J_ij| / s (the
gains then stay positive, which GD-mod needs)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_00699_amd import gd
from paper_1807_00699_amd import inputs as I

pytestmark = pytest.mark.gpu

SNAP = (1, 10, 50, 100, 200)
TOL = 1e-4


def _rel(a, b):
    R = a.shape[0]
    a = a.reshape(R, -1).astype(np.float64)
    b = b.reshape(R, -1).astype(np.float64)
    return np.abs(a - b).max(1) / np.maximum(np.abs(b).max(1), 1e-30)


def _gamma_c(J):
    Jz = np.asarray(J, np.float64).copy()
    np.fill_diagonal(Jz, 0.0)
    s = np.sqrt((Jz**2).sum() / Jz.shape[0])
    return float(np.abs(Jz).sum(1).max() / s)


def _parity(J, psi0, model, dt, eps_hat, k_sample, **kw):
    n = J.shape[0]
    R = psi0.shape[0]
    om = "ising" if model == gd.GD_ISING else "xy"
    okw = {k: v for k, v in kw.items() if k in ("gamma_c", "noise_D", "noise_seed", "eps")}
    with gd.Solver(J, model=model, dt=dt, variant=gd.GD_VARIANT_MOD, eps_hat=eps_hat, **kw) as S:
        s = O.coupling_scale(np.asarray(J, np.float64))
        assert abs(s - S.scale) <= 1e-12 * s, (s, S.scale)
        S.set_init(R, psi0)
        for r in k_sample:
            assert np.array_equal(S.mod_couplings(r), J * (1 - np.eye(n, dtype=np.float32)))
        op = psi0.astype(np.float64)
        og = np.zeros((R, n))
        oK = None
        prev = 0
        worst = []
        for st in SNAP:
            S.run(st - prev)
            op, og, oK = O.run_mod(J, op, og, oK, model=om, steps=st - prev, dt=dt, eps_hat=eps_hat,
                                   s=s, t0=prev, **okw)
            prev = st
            p, gm, step = S.state()
            assert step == st
            ep, eg = _rel(p, op), _rel(gm, og)
            Kg = np.stack([S.mod_couplings(r) for r in k_sample])
            ek = _rel(Kg, oK[list(k_sample)])
            worst.append((st, float(ep.max()), float(eg.max()), float(ek.max())))
            assert ep.max() <= TOL and eg.max() <= TOL and ek.max() <= TOL, worst[-1]
        print("worst per snapshot (step, psi, gamma, K):", worst)


def test_gdmod_ising_parity():
    """Ising N = 64 dense +-1, R = 20, Euler dt = 0.05, eps = 0.1, eps_hat = 0.2."""
    n, R = 64, 20
    J = I.dense_pm1(n, 1)
    _parity(J, I.psi0_real(n, R, 1), gd.GD_ISING, 0.05, 0.2, (0, 7, 19), gamma_c=_gamma_c(J))


def test_gdmod_xy_noise_parity_ragged():
    """XY N = 100 (ragged: Np = 128), N(0, 1/N) couplings, R = 9, Euler dt = 0.02,
    Psi(0) = 0 with noise D = 0.01, eps_hat = 1.0."""
    n, R = 100, 9
    J = I.dense_gaussian(n, 4)
    _parity(J, np.zeros((R, n, 2), np.float32), gd.GD_XY, 0.02, 1.0, (0, 8), gamma_c=_gamma_c(J),
            noise_D=0.01, noise_seed=3)


def test_gdmod_reaches_brute_force_ground_state_n20():
    J = I.dense_pm1(64, 1)[:20, :20].copy()
    e_b, _ = O.brute_ising(J.astype(np.float64))
    with gd.Solver(J, model=gd.GD_ISING, dt=0.05, eps=0.1, variant=gd.GD_VARIANT_MOD, eps_hat=0.2,
                   gamma_c=_gamma_c(J)) as S:
        S.set_init(32, I.psi0_real(20, 32, 3))
        S.run(3000)
        E, _ = S.energy()
        K = S.mod_couplings(5)
        _, gm, _ = S.state()
    assert E.min() == e_b
    # converged couplings: (gamma_i + gamma_j) K_ij = J_ij off the diagonal
    D = gm[5][:, None].astype(np.float64) + gm[5][None, :]
    off = ~np.eye(20, dtype=bool)
    assert np.abs(D * K - J)[off].max() < 1e-3


def test_gdmod_set_state_resets_couplings_and_rejects_bad_calls():
    n, R = 32, 4
    J = I.dense_pm1(n, 2)
    with gd.Solver(J, variant=gd.GD_VARIANT_MOD, gamma_c=_gamma_c(J)) as S:
        S.run(50, batch=R)
        assert not np.array_equal(S.mod_couplings(1), J)
        p, g, _ = S.state()
        S.set_state(p, g, step=50)
        Jz = J * (1 - np.eye(n, dtype=np.float32))
        assert np.array_equal(S.mod_couplings(1), Jz)
        with pytest.raises(gd.GDError):
            S.mod_couplings(R)
    with gd.Solver(J) as S:
        S.run(1, batch=2)
        with pytest.raises(gd.GDError):
            S.mod_couplings(0)


def test_gdmod_full_size_sampled():
    """GD-mod at the benchmark's size: XY N = 1024, R = 256, Euler dt = 0.02,
    eps_hat = 0.2 (the timed launch configuration), 200 steps, trajectories
    0, 131 and 255 against the oracle (Psi, gamma and K)."""
    n, R = 1024, 256
    J = I.dense_gaussian(n, 1)
    psi0 = I.psi0_complex(n, R, 1)
    gc = _gamma_c(J)
    sub = [0, 131, 255]
    with gd.Solver(J, model=gd.GD_XY, dt=0.02, eps=0.1, variant=gd.GD_VARIANT_MOD, eps_hat=0.2,
                   gamma_c=gc) as S:
        S.set_init(R, psi0)
        S.run(200)
        p, gm, _ = S.state()
        Kg = np.stack([S.mod_couplings(r) for r in sub])
    op, og, oK = O.run_mod(J, psi0[sub], model="xy", steps=200, dt=0.02, eps=0.1, eps_hat=0.2,
                           gamma_c=gc, s=float(np.sqrt((J.astype(np.float64) ** 2).sum() / n)))
    assert _rel(p[sub], op).max() <= TOL and _rel(gm[sub], og).max() <= TOL
    assert _rel(Kg, oK).max() <= TOL
