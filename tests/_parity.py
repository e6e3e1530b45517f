"""The amplitude/gain parity rule shared by the GPU tests.

Reading of the 1e-4 relative bar: per trajectory,
  max_i |psi_gpu - psi_orc| / max_i |psi_orc| <= 1e-4, and the same for gamma,
at the compared steps.  The GPU integrates in FP32 and the oracle in FP64, so
the bar measures FP32 rounding as the dynamics carry it.  Near an unstable
point the dynamics amplify rounding past 1e-4 within 200 steps; the oracle's
own float32 integration (``oracle.run_f32``, pinned in
tests/test_oracle_f32_floor.py) shows the same excursion on the same
trajectories.  Where rounding is amplified, its outcome depends on the order
in which the coupling sums are rounded: the floor of a trajectory is therefore
the largest distance from the FP64 oracle among float32 integrations that
differ only in that order (``Floor``: the spins relabelled by the identity,
the reversal and one seeded permutation; the sums of Eq. (main) then run in
another order).  Such a trajectory may be held to 4x that floor instead; every
check reports how many trajectories had such a widened bound and how many
needed it, ``strict`` forbids it, and ``max_used`` caps the count that needed it.
"""
import numpy as np

from oracle import oracle as O

TOL = 1e-4


class Floor:
    """float32 integrations (oracle.run_f32) of one problem in several
    summation orders, advanced together; ``floor(op, og)`` is, per
    trajectory, the largest distance of any of them from the FP64 state.
    Per-spin arguments (eps, g, the rows of h) are relabelled with the
    spins; runs with noise use the natural order only (the noise numbers are
    keyed by the spin index)."""

    def __init__(self, J, psi, gamma=None, orders=3, **kw):
        J = np.asarray(J)
        n = J.shape[0]
        psi = np.asarray(psi, np.float32)
        gamma = (np.zeros(psi.shape[:2], np.float32) if gamma is None
                 else np.asarray(gamma, np.float32).reshape(psi.shape[:2]))
        if kw.get("noise_D", 0.0):
            orders = 1
        perms = [np.arange(n), np.arange(n)[::-1].copy(), np.random.default_rng(1234 + n).permutation(n)]
        self.kw = kw
        self.runs = []
        for perm in perms[:orders]:
            pkw = dict(kw)
            for key in ("eps", "g", "h"):
                if key in pkw and pkw[key] is not None and np.ndim(pkw[key]) >= 1:
                    pkw[key] = np.asarray(pkw[key])[..., perm]
            self.runs.append([perm, np.ascontiguousarray(J[np.ix_(perm, perm)]), psi[:, perm].copy(),
                              gamma[:, perm].copy(), pkw])

    def advance(self, steps, **extra):
        """``extra``: arguments that are not per spin (e.g. the noise step t0)"""
        for run in self.runs:
            perm, Jp, x, g, pkw = run
            run[2], run[3] = O.run_f32(Jp, x, g, steps=steps, **pkw, **extra)

    def states(self):
        """the float32 states in the original spin order"""
        out = []
        for perm, _, x, g, _ in self.runs:
            inv = np.argsort(perm)
            out.append((x[:, inv], g[:, inv]))
        return out

    def floor(self, op, og):
        return np.max([np.maximum(rel(x, op), rel(g, og)) for x, g in self.states()], axis=0)


def rel(a, b):
    """per-trajectory max-norm relative error, arrays [R][...]"""
    R = a.shape[0]
    a = a.reshape(R, -1).astype(np.float64)
    b = b.reshape(R, -1).astype(np.float64)
    return np.abs(a - b).max(1) / np.maximum(np.abs(b).max(1), 1e-30)


def check(ep, eg, floor, *, strict=False, max_used=None, min_strict=0.9, label=""):
    """ep, eg: per-trajectory errors of psi and gamma against the FP64 oracle;
    floor: per-trajectory float32 floor (``Floor.floor``; None when no floor
    applies).  Returns (trajectories with a widened bound, trajectories
    that needed it)."""
    ep, eg = np.asarray(ep), np.asarray(eg)
    over = (ep > TOL) | (eg > TOL)
    used = int(over.sum())
    if floor is None:
        widened = 0
        bound = np.full(ep.shape, TOL)
    else:
        bound = np.maximum(TOL, 4 * np.asarray(floor))
        widened = int(np.sum(bound > TOL))
    print(f"parity {label}: max psi {ep.max():.2e}, gamma {eg.max():.2e}; "
          f"widened bounds {widened}/{ep.size}, needed by {used}", flush=True)
    if strict or floor is None:
        assert used == 0, (label, "strict 1e-4", ep.max(), eg.max(), np.flatnonzero(over)[:10])
        return widened, used
    assert np.all(ep <= bound) and np.all(eg <= bound), (label, ep.max(), eg.max(), int(np.argmax(ep / bound)))
    assert np.mean(~over) >= min_strict, (label, used, ep.size)
    if max_used is not None:
        assert used <= max_used, (label, "more trajectories needed the widened bound", used, max_used)
    return widened, used
