"""The amplitude/gain parity rule shared by the GPU tests.

Reading of the 1e-4 relative bar: per trajectory,
  max_i |psi_gpu - psi_orc| / max_i |psi_orc| <= 1e-4, and the same for gamma,
at the compared steps.  The GPU integrates in FP32 and the oracle in FP64, so
the bar measures FP32 rounding as the dynamics carry it.  Near an unstable
point the dynamics amplify rounding past 1e-4 within 200 steps; the oracle's
own float32 integration (``oracle.run_f32``, pinned in
tests/test_oracle_f32_floor.py) shows the same excursion on the same
trajectories.  Such a trajectory may be held to 4x that floor instead; every
check reports how many trajectories had such a widened bound and how many
needed it, ``strict`` forbids it, and ``max_used`` caps the count that needed it.
"""
import numpy as np

TOL = 1e-4


def rel(a, b):
    """per-trajectory max-norm relative error, arrays [R][...]"""
    R = a.shape[0]
    a = a.reshape(R, -1).astype(np.float64)
    b = b.reshape(R, -1).astype(np.float64)
    return np.abs(a - b).max(1) / np.maximum(np.abs(b).max(1), 1e-30)


def check(ep, eg, floor, *, strict=False, max_used=None, min_strict=0.9, label=""):
    """ep, eg: per-trajectory errors of psi and gamma against the FP64 oracle;
    floor: per-trajectory distance of run_f32 from the FP64 oracle (None when
    no floor applies).  Returns (trajectories with a widened bound, trajectories
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
