"""Per-trajectory divergence status and the best-so-far energy trace of the
device checks (gd_trajectory_status, gd_best_trace), through the C ABI."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_00699_amd import gd
from paper_1807_00699_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [64, 200])   # fused small-problem kernel; tiled GEMM variants
def test_trajectory_status_marks_exactly_the_blown_up_trajectories(n):
    """Amplitudes of 1e18 overflow FP32 in the cubic term of Eq. (main) on the
    first step; the coupling sum mixes spins of one trajectory only, so every
    other trajectory stays finite."""
    R = 16
    J = I.dense_pm1(n, 3)
    psi = I.psi0_real(n, R, 4)
    bad = np.zeros(R, bool)
    bad[[1, 6, 15]] = True
    psi[bad, 5] = 1e18
    with gd.Solver(J, model=gd.GD_ISING, dt=0.05, eps=0.1) as S:
        S.set_state(psi, np.zeros((R, n), np.float32))
        with pytest.raises(gd.GDError) as ei:
            S.run(20)
        assert ei.value.code == gd.GD_E_DIVERGED
        st = S.trajectory_status()
        assert st.dtype == np.int32 and st.shape == (R,)
        assert np.array_equal(st, bad.astype(np.int32))
        assert S.stats().diverged == int(bad.sum())
        x, _, _ = S.state()
        assert np.array_equal(~np.isfinite(x).all(axis=1), bad)
        # a new state clears it
        S.set_state(I.psi0_real(n, R, 5), np.zeros((R, n), np.float32))
        S.run(10)
        assert not S.trajectory_status().any() and S.stats().diverged == 0


def test_trajectory_status_rejects_bad_calls():
    J = I.dense_pm1(32, 1)
    with gd.Solver(J, model=gd.GD_ISING) as S:
        with pytest.raises(gd.GDError) as ei:
            gd.gd_trajectory_status(S.h, 4)
        assert ei.value.code == gd.GD_E_STATE
        S.set_init(4)
        with pytest.raises(gd.GDError) as ei:
            gd.gd_trajectory_status(S.h, 5)
        assert ei.value.code == gd.GD_E_INVALID_ARG


@pytest.mark.parametrize("n", [64, 200])
def test_best_trace_follows_the_checks(n):
    """One entry per device check across gd_run calls, at the steps of the
    checks, non-increasing, ending at gd_stats.best_energy; the last check's
    minimum is the Eq. (h) energy of the final discretised state (exact for
    integer J, against the oracle); gd_set_state starts a new trace."""
    R = 32
    J = I.dense_pm1(n, 7)
    with gd.Solver(J, model=gd.GD_ISING, dt=0.05, eps=0.1, check_interval=10) as S:
        S.set_init(R, I.psi0_real(n, R, 8))
        S.run(45)
        S.run(25)
        steps, best = S.best_trace()
        assert list(steps) == [10, 20, 30, 40, 50, 60, 70]
        assert np.all(np.diff(best) <= 0)
        assert best[-1] == S.stats().best_energy
        x, g, _ = S.state()
        # same-precision readout of the GPU's own FP32 state at step 70
        e_last = float(O.energy_ising(J, O.ising_spins(x)).min())
        assert best[-1] == min(best[-2], e_last)
        S.set_state(x, g, step=70)
        assert S.best_trace()[0].size == 0 and S.stats().best_energy == np.inf
        S.run(10)
        st2, b2 = S.best_trace()
        x2, _, _ = S.state()
        assert list(st2) == [80]
        assert b2[0] == float(O.energy_ising(J, O.ising_spins(x2)).min())


def test_batch_trajectory_status_shape_and_health():
    """Batches of instances: one flag per (instance, trajectory)."""
    sizes, insts = I.maxcut_batch(5, 50, 300, 17)
    R = 8
    with gd.BatchSolver(insts, check_interval=25) as B:
        B.set_init(R)
        B.run(100)
        st = B.trajectory_status()
        assert st.shape == (5, R) and st.dtype == np.int32
        assert not st.any() and B.stats().diverged == 0
        with pytest.raises(gd.GDError) as ei:
            gd.gd_trajectory_status(B.h, 5 * R + 1)
        assert ei.value.code == gd.GD_E_INVALID_ARG
