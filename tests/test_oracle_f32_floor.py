"""Pins of ``oracle.run_f32``, the single-precision integration whose distance
from the FP64 oracle (the "FP32 floor") widens the GPU parity bound of a
trajectory.  A bug that inflated that distance would quietly loosen every
bound, so the floor is tied here to facts that do not come from ``run_f32``:

* closed forms of Eq. (main, gamma) (logistic law of one mode, linear growth of
  the gain at Psi = 0, the matrix exponential of the linear regime), met to
  single-precision accuracy;
* one step of every integrator agrees with the FP64 step of ``oracle.run``
  inside the worst-case rounding envelope of FP32 arithmetic (a dropped term,
  a wrong sign or a wrong step size is many envelopes away);
* over 200 steps the floor of each trajectory stays within a factor of a model
  of FP32 rounding that uses no single-precision code at all: the FP64 oracle
  stepped one step at a time with a random relative kick of rounding size
  after each step, so the dynamics amplify it as they amplify rounding.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_00699_amd import inputs as I

U = 2.0 ** -24   # unit roundoff of IEEE single precision (round to nearest)


def _rel(a, b):
    R = a.shape[0]
    a = a.reshape(R, -1).astype(np.float64)
    b = b.reshape(R, -1).astype(np.float64)
    return np.abs(a - b).max(1) / np.maximum(np.abs(b).max(1), 1e-30)


def _rhs_scale(J, x, gam, s, gamma_c, h1):
    """Per (trajectory, spin, plane) magnitude M of the terms of Eq. (main):
    |Psi| (|gamma| + |gamma_c| + |Psi|^2) + sum_j |J_ij| |Psi_j| / s + |h_1|,
    the size against which one step's rounding is measured."""
    R, n = gam.shape
    a = np.abs(np.asarray(x, np.float64)).reshape(R, n, -1)
    rho = (a * a).sum(-1)
    Ja = np.abs(np.asarray(J, np.float64))
    np.fill_diagonal(Ja, 0.0)
    coup = np.stack([a[..., p] @ Ja.T for p in range(a.shape[-1])], -1) / s
    return a * (np.abs(gam) + abs(gamma_c) + rho)[..., None] + coup + np.abs(h1)[None, :, None]


# ------------------------------------------------------------ closed forms

def test_run_f32_single_mode_logistic_law():
    """J = 0, eps = 0 (gain frozen at gamma = a + gamma_c): each mode obeys
    x(t)^2 = a x0^2 e^{2at} / (a + x0^2 (e^{2at} - 1)) (Eq. (main) with one
    spin).  RK4 at dt = 0.01 over t = 4 leaves a truncation error far below
    single precision, so the float32 run must meet the law to a few hundred
    roundings of |x|."""
    n = 5
    x0 = np.array([[0.05, -0.2, 0.7, 1.6, -0.01]], np.float32)
    a, gc, T, dt = 0.8, 0.3, 4.0, 0.01
    x, g = O.run_f32(np.zeros((n, n)), x0, np.full((1, n), a + gc, np.float32), model="ising",
                     steps=int(T / dt), dt=dt, eps=0.0, gamma_c=gc, s=1.0, integrator=O.RK4)
    x0d = x0[0].astype(np.float64)
    e = np.exp(2 * a * T)
    law = np.sign(x0d) * np.sqrt(a * x0d ** 2 * e / (a + x0d ** 2 * (e - 1)))
    assert np.array_equal(g, np.full((1, n), a + gc, np.float32))
    assert np.all(np.abs(x[0] - law) <= 400 * U * np.abs(law)), np.abs(x[0] - law) / np.abs(law)


@pytest.mark.parametrize("model", ["ising", "xy"])
@pytest.mark.parametrize("integrator", [O.EULER, O.RK4])
def test_run_f32_zero_state_gain_is_linear(model, integrator):
    """Psi == 0, no field: the amplitudes stay exactly 0 and Eq. (gamma) gives
    gamma_n = gamma_0 + n dt eps rho_th, up to one rounding per step."""
    n, R, steps, dt, eps, rho = 7, 3, 50, 0.05, 0.3, 1.7
    J = I.dense_pm1(n, 2)
    shape = (R, n) if model == "ising" else (R, n, 2)
    gam0 = np.linspace(-1, 1, R * n).reshape(R, n).astype(np.float32)
    p, g = O.run_f32(J, np.zeros(shape, np.float32), gam0, model=model, steps=steps, dt=dt, eps=eps,
                     rho_th=rho, integrator=integrator)
    assert np.all(p == 0.0)
    want = gam0.astype(np.float64) + steps * dt * eps * rho
    assert np.all(np.abs(g - want) <= 8 * steps * U * (np.abs(want) + 1.0))


@pytest.mark.parametrize("model", ["ising", "xy"])
def test_run_f32_linear_regime_matrix_exponential(model):
    """Amplitudes of 1e-4, eps = 0, gamma = gamma_0: the cubic term is 1e-8 of
    the linear one, and Eq. (main) is dPsi/dt = ((gamma_0 - gamma_c) I + J/s) Psi,
    solved by the matrix exponential (numpy eigh).  The float32 RK4 run must
    follow it to within 1e-5 relative."""
    n, R, g0, T, dt = 24, 3, -0.4, 2.0, 0.01
    J = I.dense_gaussian(n, 4)
    s = O.coupling_scale(J.astype(np.float64))
    A = J.astype(np.float64)
    np.fill_diagonal(A, 0.0)
    lam, V = np.linalg.eigh(A / s + g0 * np.eye(n))
    E = (V * np.exp(lam * T)) @ V.T
    rng = np.random.default_rng(4)
    if model == "ising":
        x0 = (1e-4 * rng.uniform(-1, 1, (R, n))).astype(np.float32)
        want = x0.astype(np.float64) @ E.T
    else:
        x0 = (1e-4 * rng.uniform(-1, 1, (R, n, 2))).astype(np.float32)
        want = np.stack([x0[..., 0].astype(np.float64) @ E.T, x0[..., 1].astype(np.float64) @ E.T], -1)
    x, _ = O.run_f32(J, x0, np.full((R, n), g0, np.float32), model=model, steps=int(T / dt), dt=dt,
                     eps=0.0, s=s, integrator=O.RK4)
    assert _rel(x, want).max() < 1e-5, _rel(x, want).max()


# ------------------------------------------------------- one-step envelope

CASES = [
    # model, integrator, dt, gamma_c, with field, per-spin eps
    ("ising", O.EULER, 0.05, 0.0, False, False),
    ("ising", O.EULER, 0.05, 0.3, True, True),
    ("ising", O.RK4, 0.05, 0.2, True, False),
    ("xy", O.EULER, 0.02, 0.0, False, True),
    ("xy", O.RK4, 0.02, 0.1, True, True),
]


@pytest.mark.parametrize("model,integrator,dt,gamma_c,field,per_spin", CASES)
def test_run_f32_one_step_within_rounding_envelope(model, integrator, dt, gamma_c, field, per_spin):
    """From the same float32 state (mid-run, amplitudes O(1), gains of both
    signs), one step of run_f32 and of the FP64 oracle differ by at most
    C u (|y_1| + dt M) per element, M the magnitude of the right-hand side
    terms and C = 2 (n + 8) per coupling evaluation (worst-case rounding of an
    n-term sum plus the pointwise operations).  A missing or mis-signed term
    of Eq. (main, gamma), a wrong dt or a mis-scaled coupling moves a step by
    O(dt M), hundreds of envelopes.  The deviation must also be nonzero:
    run_f32 does round."""
    n, R = 96, 12
    cx = model == "xy"
    J = I.dense_gaussian(n, 21) if cx else I.dense_pm1(n, 21)
    rng = np.random.default_rng(21)
    x = (rng.uniform(-1.2, 1.2, (R, n, 2) if cx else (R, n))).astype(np.float32)
    gam = rng.uniform(-0.8, 1.5, (R, n)).astype(np.float32)
    g = ((np.arange(n) % 5) - 2).astype(np.float32) * (0.3 if cx else 1.0) if field else None
    eps = np.linspace(0.05, 0.25, n).astype(np.float32) if per_spin else 0.1
    s = O.coupling_scale(J.astype(np.float64))
    kw = dict(model=model, dt=dt, eps=eps, g=g, gamma_c=gamma_c, s=s, integrator=integrator, steps=1)
    xf, gf = O.run_f32(J, x, gam, **kw)
    xo, go = O.run(J, x.astype(np.float64), gam.astype(np.float64), **kw)
    h1 = np.zeros(n) if g is None else O.field_h1(g, 1.0, s)
    # stage states of RK4 stay within dt M of y; the envelope takes the larger
    # of the right-hand side scales at y and at y_1 and counts 4 evaluations
    M = np.maximum(_rhs_scale(J, x, gam, s, gamma_c, h1), _rhs_scale(J, xo, go, s, gamma_c, h1))
    stages = 4 if integrator == O.RK4 else 1
    C = 2 * (n + 8) * stages
    env_x = C * U * (np.abs(xo).reshape(M.shape) + dt * M)
    epsv = np.broadcast_to(np.asarray(eps, np.float64), (n,))
    rho_scale = (np.abs(np.asarray(x, np.float64)).reshape(R, n, -1) ** 2).sum(-1) + 1.0
    env_g = C * U * (np.abs(go) + dt * epsv * rho_scale)
    dx = np.abs(xf.astype(np.float64) - xo).reshape(M.shape)
    dg = np.abs(gf.astype(np.float64) - go)
    assert np.all(dx <= env_x), (dx / env_x).max()
    assert np.all(dg <= env_g), (dg / env_g).max()
    assert dx.max() > 0 and dg.max() > 0


# ------------------------------------------- 200 steps: rounding model

def _kicked_fp64_run(J, x0, steps, s, rng, model, integrator, dt, eps, g, gamma_c):
    """The FP64 oracle one step at a time; after each step every amplitude and
    gain moves by one rounding of its size, u (|y| + dt M), with a random sign.
    Contains no single-precision arithmetic."""
    R, n = x0.shape[0], J.shape[0]
    x, gm = x0.astype(np.float64), np.zeros((R, n))
    h1 = np.zeros(n) if g is None else O.field_h1(g, 1.0, s)
    epsv = np.broadcast_to(np.asarray(eps, np.float64), (n,))
    for _ in range(steps):
        M = _rhs_scale(J, x, gm, s, gamma_c, h1)
        x, gm = O.run(J, x, gm, model=model, steps=1, dt=dt, eps=eps, g=g, gamma_c=gamma_c, s=s,
                      integrator=integrator)
        x = x + U * (np.abs(x) + dt * M.reshape(x.shape)) * rng.choice([-1.0, 1.0], x.shape)
        rho = (np.abs(x).reshape(R, n, -1) ** 2).sum(-1)
        gm = gm + U * (np.abs(gm) + dt * epsv * (1.0 + rho)) * rng.choice([-1.0, 1.0], gm.shape)
    return x, gm


FLOOR_CASES = [
    # the Ising N = 64, R = 100 parity workload (dense +-1, Euler dt = 0.05)
    ("ising64", "ising", O.EULER, 0.05, 64, 100, None, 0.1),
    # XY, Gaussian couplings, RK4 dt = 0.02
    ("xy64", "xy", O.RK4, 0.02, 64, 40, None, 0.1),
    # field and per-spin eps
    ("ising96_field", "ising", O.EULER, 0.05, 96, 20, "field", "per_spin"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,model,integrator,dt,n,R,field,eps", FLOOR_CASES)
def test_run_f32_floor_follows_rounding_model(name, model, integrator, dt, n, R, field, eps):
    """Per trajectory, after 200 steps: the float32-vs-float64 distance of
    run_f32 (the floor) is at most 4x, and at least 1/300 of, the largest
    distance of three kicked FP64 runs (seeds 0, 1, 2) from the plain FP64
    run.  Trajectories near an unstable point amplify both alike; a floor
    inflated by a bug (or one that does not round at all) leaves the band."""
    cx = model == "xy"
    J = I.dense_gaussian(n, 2) if cx else I.dense_pm1(n, 1 if field is None else 5)
    seed = 2 if cx else (1 if field is None else 5)
    x0 = I.psi0_complex(n, R, seed) if cx else I.psi0_real(n, R, seed)
    g = ((np.arange(n) % 5) - 2).astype(np.float32) if field else None
    epsv = np.linspace(0.05, 0.2, n).astype(np.float32) if eps == "per_spin" else eps
    s = O.coupling_scale(J.astype(np.float64))
    kw = dict(model=model, dt=dt, eps=epsv, g=g, s=s, integrator=integrator)
    xo, go = O.run(J, x0, steps=200, **kw)
    xf, gf = O.run_f32(J, x0, np.zeros((R, n), np.float32), steps=200, **kw)
    floor = np.maximum(_rel(xf, xo), _rel(gf, go))
    kicked = []
    for sd in range(3):
        xk, gk = _kicked_fp64_run(J, x0, 200, s, np.random.default_rng(sd), model, integrator, dt, epsv,
                                  g, 0.0)
        kicked.append(np.maximum(_rel(xk, xo), _rel(gk, go)))
    model_dist = np.max(kicked, 0)
    ratio = floor / model_dist
    assert np.all(ratio <= 4.0), (name, ratio.max(), int(np.argmax(ratio)))
    assert np.all(ratio >= 1.0 / 300), (name, ratio.min(), int(np.argmin(ratio)))


def test_multi_order_floor_is_rounding_only():
    """The parity floor takes the largest distance of float32 runs that differ
    only in the order of the coupling sums (spins relabelled).  Relabelling
    is exact for the FP64 oracle (equivariance to FP64 rounding), each
    relabelled float32 run stays inside the single-precision band of the
    natural one, and the floor over orders is at least the natural floor."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    import _parity as P
    n, R = 120, 6
    J = I.dense_pm1(n, 61)
    x0 = I.psi0_real(n, R, 61)
    rng = np.random.default_rng(61)
    eps = rng.uniform(0.05, 0.2, n)
    g = rng.integers(-2, 3, n).astype(np.float64)
    s = O.coupling_scale(J.astype(np.float64))
    kw = dict(model="ising", dt=0.05, eps=eps, g=g, s=s)
    xo, go = O.run(J, x0.astype(np.float64), None, steps=100, **kw)
    perm = np.random.default_rng(1234 + n).permutation(n)
    xp, gp = O.run(J[np.ix_(perm, perm)], x0[:, perm].astype(np.float64), None, steps=100,
                   model="ising", dt=0.05, eps=eps[perm], g=g[perm], s=s)
    inv = np.argsort(perm)
    assert np.abs(xp[:, inv] - xo).max() <= 1e-10 * np.abs(xo).max()
    fl = P.Floor(J, x0, None, **kw)
    assert len(fl.runs) == 3
    fl.advance(60)
    fl.advance(40)
    floors = [np.maximum(P.rel(x, xo), P.rel(gm, go)) for x, gm in fl.states()]
    assert all(np.all(f < 1e-3) and np.all(f > 0) for f in floors)
    assert np.array_equal(fl.floor(xo, go), np.max(floors, axis=0))
    assert np.all(fl.floor(xo, go) >= floors[0])
    one = P.Floor(J, x0, None, orders=1, **kw)
    one.advance(100)
    xf, gf = O.run_f32(J, x0, None, steps=100, **kw)
    assert np.array_equal(one.states()[0][0], xf)
    noisy = P.Floor(J, x0, None, noise_D=0.01, **kw)
    assert len(noisy.runs) == 1
