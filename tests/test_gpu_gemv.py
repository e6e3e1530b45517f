"""The small-R coupling kernel (J streamed once per evaluation, vector ALUs,
variant ids 100 + k) against the FP64 oracle, through the C ABI.

The paper integrates one trajectory at a time (Sec. 3: repeated runs per
instance; Sec. 4: 20 runs per size), where the coupling sum of Eq. (main) is a
matrix-vector product bound by the bytes of J.  Bars as for the GEMM path
(tests/_parity.py): per trajectory 1e-4 relative in Psi and gamma at steps
{1, 50, 200} (a FP32-floor widening reported), integer-J energies of the
device check exact, and the reduced-precision one-step rounding bound of
tests/test_gpu_lowprec.py.  Sizes: N = 4096 (the dense Ising size), a ragged
N = 3001 (3008 padded, last row tile partly empty), R in {1, 3, 8, 16}.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_00699_amd import gd
from paper_1807_00699_amd import inputs as I

import _parity as P
from test_gpu_lowprec import _one_step_check

pytestmark = pytest.mark.gpu

GEMV_IDS = (100, 101, 102, 103, 104)


def max_columns(cid, jk="f32"):
    """GEMM columns (R real, 2R complex) a pinned variant accepts: the
    1024-thread variant (104, 128 registers per lane) takes 2; the 8-wave
    variants (102, 103) take 4 widened FP8 columns and 8 widened 16-bit ones"""
    if cid == 104:
        return 2
    if cid in (102, 103) and jk == "fp8":
        return 4
    if cid in (102, 103) and jk == "b16":
        return 8
    return 16


def _gemv_parity(J, psi0, model, integrator, dt, steps_list=(1, 50, 200), strict=False, check=0,
                 min_strict=0.9):
    """run through the library (variant chosen by the tuner unless pinned)
    and compare every trajectory with the oracle; returns the solver stats"""
    n, R = J.shape[0], psi0.shape[0]
    mdl = gd.GD_ISING if model == "ising" else gd.GD_XY
    s = O.coupling_scale(J.astype(np.float64))
    with gd.Solver(J, model=mdl, integrator=integrator, dt=dt, eps=0.1, check_interval=check) as S:
        assert abs(S.scale - s) <= 1e-12 * s
        S.set_init(R, psi0)
        op, og = psi0.astype(np.float64), np.zeros((R, n))
        fl = P.Floor(J, psi0, None, model=model, dt=dt, eps=0.1, integrator=integrator, s=s)
        prev = 0
        for st in steps_list:
            S.run(st - prev)
            op, og = O.run(J, op, og, model=model, steps=st - prev, dt=dt, eps=0.1, integrator=integrator, s=s)
            fl.advance(st - prev)
            prev = st
            p, gm, step = S.state()
            assert step == st
            P.check(P.rel(p, op), P.rel(gm, og), None if strict else fl.floor(op, og),
                    min_strict=min_strict, label=f"gemv {model} n={n} R={R} step {st}")
        stats = S.stats()
        spins = S.spins() if model == "ising" else None
    return stats, spins, op


@pytest.mark.parametrize("R", [1, 3, 8, 16])
def test_ising_euler_n4096_tuner_picks_gemv(R):
    """Dense Ising size (density-0.5 {-1, 0, +1} couplings), Euler dt = 0.05:
    the tuner takes a matrix-vector variant over the padded 128-column GEMM,
    and all R trajectories meet the oracle bar; with checks every 50 steps
    the best device energy is the exact oracle energy of the best readout.
    Around step 200 this instance leaves the linear regime and amplifies
    single-precision rounding (the oracle's own float32 run is 2.5e-5 or more
    away from FP64 on most trajectories), so every trajectory is held to its
    widened bound but only 75% (not 90%) must also meet 1e-4 outright."""
    n = 4096
    J = I.sparse_pm1(n, 41)
    psi0 = I.psi0_real(n, R, 41 + R)
    st, spins, _ = _gemv_parity(J, psi0, "ising", gd.GD_EULER, 0.05, check=50, min_strict=0.75)
    assert st.kernel_config >= 100, st.kernel_config
    Eo = O.energy_ising(J, spins).astype(np.float64)
    assert st.best_energy <= Eo.min()         # best over the checks at 50, 100, ..., 200
    assert np.isfinite(st.best_energy) and 0 <= st.best_index < R


@pytest.mark.parametrize("R", [1, 3, 8])
def test_xy_rk4_n4096_tuner_picks_gemv(R):
    """XY, N(0, 1/N) couplings, RK4 dt = 0.02 (2R GEMM columns)."""
    n = 4096
    J = I.dense_gaussian(n, 43)
    psi0 = I.psi0_complex(n, R, 43 + R)
    st, _, _ = _gemv_parity(J, psi0, "xy", gd.GD_RK4, 0.02)
    assert st.kernel_config >= 100, st.kernel_config


@pytest.mark.parametrize("cid", GEMV_IDS)
def test_every_gemv_variant_ragged(monkeypatch, cid):
    """Each variant pinned: ragged Ising N = 3001 (R = 5, Euler) and XY
    N = 1000 (R = 8, RK4) (fewer where the variant takes fewer columns), then
    the device energy check of the Ising run against the oracle's exact
    energies of the same readout."""
    monkeypatch.setenv("GD_DENSE_CONFIG", str(cid))
    Ri = min(5, max_columns(cid))
    Rx = min(8, max_columns(cid) // 2)
    J = I.dense_pm1(3001, 47)
    x0 = I.psi0_real(3001, Ri, 47)
    st, _, _ = _gemv_parity(J, x0, "ising", gd.GD_EULER, 0.05)
    assert st.kernel_config == cid
    Jx = I.dense_gaussian(1000, 48)
    p0 = I.psi0_complex(1000, Rx, 48)
    st, _, _ = _gemv_parity(Jx, p0, "xy", gd.GD_RK4, 0.02)
    assert st.kernel_config == cid
    with gd.Solver(J, model=gd.GD_ISING, dt=0.05, eps=0.1) as S:
        S.set_init(Ri, x0)
        S.run(120)
        Ed, bd = S.energy(device_path=True)
        E, b = S.energy()
        sp = S.spins()
    Eo = O.energy_ising(J, sp).astype(np.float64)
    assert np.array_equal(Ed, Eo) and np.array_equal(E, Eo) and bd == b == int(np.argmin(Eo))


def test_gemv_field_per_spin_eps_and_gamma_c(monkeypatch):
    """External field (q = 1 term), per-spin eps_i and gamma_c != 0 through
    the matrix-vector kernel's epilogue: Ising N = 640, R = 2, and XY R = 4."""
    monkeypatch.setenv("GD_DENSE_CONFIG", "100")
    n = 640
    g = ((np.arange(n) % 5) - 2).astype(np.float32)
    eps = np.linspace(0.05, 0.2, n).astype(np.float32)
    for model, J, x0, integ, dt, gs in (
            ("ising", I.dense_pm1(n, 49), I.psi0_real(n, 2, 49), gd.GD_EULER, 0.05, g),
            ("xy", I.dense_gaussian(n, 50), I.psi0_complex(n, 4, 50), gd.GD_RK4, 0.02, 0.1 * g)):
        mdl = gd.GD_ISING if model == "ising" else gd.GD_XY
        s = O.coupling_scale(J.astype(np.float64))
        with gd.Solver(J, gs, model=mdl, integrator=integ, dt=dt, eps=0.1, gamma_c=0.2) as S:
            S.set_init(x0.shape[0], x0, None, eps)
            S.run(200)
            p, gm, _ = S.state()
            assert S.stats().kernel_config == 100
        op, og = O.run(J, x0, model=model, steps=200, dt=dt, eps=eps, g=gs, gamma_c=0.2, s=s,
                       integrator=O.RK4 if integ == gd.GD_RK4 else O.EULER)
        fl = P.Floor(J, x0, None, model=model, dt=dt, eps=eps, g=gs, gamma_c=0.2, s=s,
                     integrator=O.RK4 if integ == gd.GD_RK4 else O.EULER)
        fl.advance(200)
        P.check(P.rel(p, op), P.rel(gm, og), fl.floor(op, og), label=f"gemv field {model}")


def test_gemv_deterministic_and_matches_gemm(monkeypatch):
    """Two runs give the same state bit for bit; a pinned GEMM variant on the
    same problem agrees to FP32 rounding of the sums (different order)."""
    n, R = 1024, 8
    J = I.dense_gaussian(n, 51)
    p0 = I.psi0_complex(n, R, 51)
    out = []
    for cid in ("100", "100", "12"):
        monkeypatch.setenv("GD_DENSE_CONFIG", cid)
        with gd.Solver(J, model=gd.GD_XY, integrator=gd.GD_RK4, dt=0.02) as S:
            S.set_init(R, p0)
            S.run(30)
            out.append(S.state())
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert P.rel(out[0][0], out[2][0]).max() < 1e-5 and P.rel(out[0][1], out[2][1]).max() < 1e-5


@pytest.mark.parametrize("cid", GEMV_IDS)
def test_gemv_reduced_precision_one_step_bound(monkeypatch, cid):
    """BF16 / FP16 operands with FP8-stored {-1, 0, +1} couplings (N = 4096,
    R = 3), 16-bit couplings not exact in FP8 (N = 1000, R = 16) and the
    complex RK4 form (R = 8): the one-step rounding bound of the operand copy.
    Variants with fewer registers per lane take fewer columns (max_columns):
    they run fewer trajectories, and pinning one beyond its limit is refused."""
    monkeypatch.setenv("GD_DENSE_CONFIG", str(cid))
    rng = np.random.default_rng(53)
    J = I.sparse_pm1(4096, 53)
    R8 = min(3, max_columns(cid, "fp8"))
    x = rng.uniform(-1.2, 1.2, (R8, 4096)).astype(np.float32)
    gam = rng.uniform(-0.5, 1.5, (R8, 4096)).astype(np.float32)
    for prec in (gd.GD_PREC_BF16, gd.GD_PREC_FP16):
        _one_step_check(J, x, gam, prec)
    n = 1000
    R16 = max_columns(cid, "b16")
    up = (1.0 + rng.integers(0, 16, (n, n)) / 16.0) * np.where(rng.random((n, n)) < 0.5, -1, 1)
    J16 = I.sym_from_upper(up)
    x = rng.uniform(-1, 1, (R16, n)).astype(np.float32)
    gam = rng.uniform(0, 1, (R16, n)).astype(np.float32)
    _one_step_check(J16, x, gam, gd.GD_PREC_BF16)
    _one_step_check(J16, x, gam, gd.GD_PREC_FP16)
    Rc = min(8, max_columns(cid, "fp8") // 2)   # +-1 couplings are FP8-stored: 2 Rc columns
    p = rng.uniform(-1, 1, (Rc, n, 2)).astype(np.float32)
    _one_step_check(I.dense_pm1(n, 54), p, gam[:Rc], gd.GD_PREC_BF16, model="xy", dt=0.02,
                    integrator=gd.GD_RK4)
    if max_columns(cid, "fp8") < 8:
        with gd.Solver(I.sparse_pm1(n, 56), precision=gd.GD_PREC_BF16) as S:
            with pytest.raises(gd.GDError) as ei:
                S.set_init(8, I.psi0_real(n, 8, 56))
            assert ei.value.code == gd.GD_E_INVALID_ARG


def test_gemv_reduced_precision_energies_exact_n4096():
    """BF16 with FP8 J, N = 4096, R = 4 (the tuner's choice): after 300 steps
    the FP64 re-score, the device check and the oracle give the same integer
    energies of the readout."""
    n, R = 4096, 4
    J = I.sparse_pm1(n, 55)
    with gd.Solver(J, model=gd.GD_ISING, precision=gd.GD_PREC_BF16, check_interval=100) as S:
        S.set_init(R, I.psi0_real(n, R, 55))
        S.run(300)
        E, b = S.energy()
        Ed, bd = S.energy(device_path=True)
        sp = S.spins()
        st = S.stats()
    assert st.kernel_config >= 100 and st.diverged == 0
    Eo = O.energy_ising(J, sp).astype(np.float64)
    assert np.array_equal(E, Eo) and np.array_equal(Ed, Eo) and b == bd == int(np.argmin(Eo))


def test_gemv_graph_replay_matches_eager_bitwise():
    """Matrix-vector steps replay captured 32-step graphs; runs shorter than
    32 steps launch eagerly.  64 steps in one run (two replays) and in 16 runs
    of 4 steps give the same state bit for bit (Ising N = 2048, R = 2)."""
    n, R = 2048, 2
    J = I.sparse_pm1(n, 57)
    x0 = I.psi0_real(n, R, 57)
    out = []
    for chunks in ([64], [4] * 16):
        with gd.Solver(J, model=gd.GD_ISING, dt=0.05, eps=0.1) as S:
            S.set_init(R, x0)
            for c in chunks:
                S.run(c)
            assert S.stats().kernel_config >= 100
            out.append(S.state())
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("cid", GEMV_IDS)
def test_fp32_solver_fp8_copy_of_j_equals_fp32_couplings_bitwise(monkeypatch, cid):
    """An FP32 solver whose couplings are all exact in FP8 streams a one-byte
    copy of J in the few-trajectory kernels, read where the FP32 kind reads its
    16-byte words and summed in the same order: every variant gives, bit for
    bit, the state and energies of the same run on FP32 couplings (the copy
    turned off with GD_J8_COPY=0), for ragged real (Euler) and complex (RK4)
    problems."""
    monkeypatch.setenv("GD_DENSE_CONFIG", str(cid))
    for model, n, integ, dt in (("ising", 1001, gd.GD_EULER, 0.05), ("xy", 999, gd.GD_RK4, 0.02)):
        cx = model == "xy"
        R = min(3, max_columns(cid) // (2 if cx else 1))
        J = I.dense_pm1(n, 61)
        psi0 = I.psi0_complex(n, R, 61) if cx else I.psi0_real(n, R, 61)
        out = []
        for copy in ("1", "0"):
            monkeypatch.setenv("GD_J8_COPY", copy)
            with gd.Solver(J, model=gd.GD_XY if cx else gd.GD_ISING, integrator=integ, dt=dt, eps=0.1,
                           check_interval=25) as S:
                S.set_init(R, psi0)
                S.run(60)
                p, g, _ = S.state()
                E, b = S.energy(device_path=True)
                assert S.stats().kernel_config == cid
                out.append((p, g, E, b, S.stats().best_energy))
        (p1, g1, E1, b1, be1), (p0, g0, E0, b0, be0) = out
        assert np.array_equal(p1, p0) and np.array_equal(g1, g0), (model, cid)
        assert np.array_equal(E1, E0) and b1 == b0 and be1 == be0, (model, cid)
