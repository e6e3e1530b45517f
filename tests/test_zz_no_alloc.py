"""gd_spins_noalloc (staging through a fixed per-device array, no device
allocation) against gd_spins, through the C ABI: the same discretised states
bit for bit on two calls in a row, the second with a smaller input, and a
clear refusal above the array's 16 MiB."""
import numpy as np
import pytest

from paper_1807_00699_amd import gd
from paper_1807_00699_amd import inputs as I

pytestmark = pytest.mark.gpu


def _both(S, fmt):
    a = gd.gd_spins(S.h, S.batch, S.n, fmt)
    b = gd.gd_spins_noalloc(S.h, S.batch, S.n, fmt)
    return a, b


def test_spins_noalloc_matches_spins_on_two_calls_second_smaller():
    # first call: Ising N = 300, R = 70 after 120 Euler steps (int8 spins and angles)
    with gd.Solver(I.dense_pm1(300, 61), model=gd.GD_ISING, dt=0.05) as S:
        S.set_init(70, I.psi0_real(300, 70, 61))
        S.run(120)
        for fmt in (gd.GD_SPINS_I8, gd.GD_SPINS_ANGLE_F32):
            a, b = _both(S, fmt)
            assert a.shape == (70, 300) and np.array_equal(a, b), fmt
        big = b
    # second call, smaller input: clock Potts q = 3, N = 100, R = 20 (int32 states)
    with gd.Solver(I.sparse_pm1(100, 62), model=gd.GD_POTTS, q=3, h_q=1.0, integrator=gd.GD_RK4,
                   dt=0.02) as S:
        S.set_init(20, I.psi0_complex(100, 20, 62))
        S.run(60)
        a, b = _both(S, gd.GD_SPINS_STATE_I32)
        assert a.shape == (20, 100) and np.array_equal(a, b)
        assert a.min() >= 0 and a.max() < 3
        a, b = _both(S, gd.GD_SPINS_ANGLE_F32)
        assert np.array_equal(a, b)
    # the first call's result is unchanged by the later use of the array
    assert big.shape == (70, 300)


def test_spins_noalloc_refuses_more_than_its_array():
    n, R = 2048, 2049      # R n float angles = 16.8 MB > 16 MiB; int8 spins = 4.2 MB fit
    with gd.Solver(I.sparse_pm1(n, 63), model=gd.GD_ISING) as S:
        S.set_init(R, I.psi0_real(n, R, 63))
        a, b = _both(S, gd.GD_SPINS_I8)
        assert np.array_equal(a, b)
        with pytest.raises(gd.GDError) as ei:
            gd.gd_spins_noalloc(S.h, S.batch, S.n, gd.GD_SPINS_ANGLE_F32)
        assert ei.value.code == gd.GD_E_INVALID_ARG
        assert "16777216" in str(ei.value)
