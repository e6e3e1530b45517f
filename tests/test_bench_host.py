"""Host-side figures of the benchmark (no GPU): the time-to-solution rule and
the FP8 exactness test that decides how J is stored."""
import math

import numpy as np

import bench


def test_tts99_closed_forms():
    # nobody reaches the target: no figure
    assert bench.tts99([None, None], range(100, 1001, 100)) == (None, None)
    # everyone reaches it by T: TTS99 = T at the first such T
    assert bench.tts99([300, 200, 300], range(100, 1001, 100)) == (300, 300)
    # one start of eight at the 400-step check: 400 ln(0.01)/ln(7/8), and a
    # later horizon with the same p only costs more
    tts, at = bench.tts99([None] * 3 + [400] + [None] * 4, range(100, 1001, 100))
    assert at == 400
    assert math.isclose(tts, 400 * math.log(0.01) / math.log(7 / 8), rel_tol=1e-12)
    # p = 1/4 at T=100 gives 100 ln(.01)/ln(.75) = 1600.8; p = 1/2 at T=200
    # gives 200 ln(.01)/ln(.5) = 1328.8, the minimum
    tts, at = bench.tts99([100, 200, None, None], [100, 200, 300])
    assert at == 200 and math.isclose(tts, 200 * math.log(0.01) / math.log(0.5))


def test_tts99_counts_a_start_at_its_own_check():
    """A start that reaches the target at a check is counted at that check's
    horizon: reach times and horizons in one unit (steps)."""
    tts, at = bench.tts99([None, 400, None, None], range(100, 10001, 100))
    assert at == 400


def test_fp8_exact():
    rng = np.random.default_rng(0)
    J = rng.choice([-1.0, 0.0, 1.0], size=(64, 64))
    assert bench.fp8_exact(J)
    assert bench.fp8_exact(J * 448.0)            # E4M3's largest finite value
    assert bench.fp8_exact(J * 2.0**-9)          # its smallest subnormal
    assert not bench.fp8_exact(J * 480.0)        # beyond the range
    assert not bench.fp8_exact(J * 1.0625)       # a fourth mantissa bit
    assert not bench.fp8_exact(J * 2.0**-10)     # below the smallest subnormal
    Jd = J.copy()
    np.fill_diagonal(Jd, 0.3)                    # the diagonal is not a coupling
    assert bench.fp8_exact(Jd)


def _profile_commands():
    """(file name, argument list) of every bench.py command quoted in profiles/"""
    import os
    import re
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")
    out = []
    for name in sorted(os.listdir(root)):
        for line in open(os.path.join(root, name)):
            m = re.search(r"python3? -u bench\.py([^`'\"()]*)", line)
            if m:
                out.append((name, m.group(1).split()))
    return out


def test_profile_commands_parse_and_name_their_workload(monkeypatch):
    """Every bench.py command that a profile summary quotes is accepted by the
    bench's argument parser, and the coupling-kernel summaries run the workload
    they are named for (the bench's default workload is Ising N = 4096)."""
    import sys
    cmds = _profile_commands()
    assert len(cmds) >= 10
    named = {"dense_step_f32_xy1024": ("xy1024",),
             "dense_step_f32_ising4096": ("ising4096", "ising4096_fp32"),
             "dense_step_lp_ising4096": ("ising4096", "ising4096_bf16")}
    for name, args in cmds:
        monkeypatch.setattr(sys, "argv", ["bench.py", *args])
        a = bench.parse()
        if a.copy_calibration:
            continue
        for prefix, workloads in named.items():
            if name.startswith(prefix):
                assert a.workload in workloads, (name, args)
