"""GD_AUTOTUNE_CACHE: the variant tuners' picks kept in a file that names the
device and library build, looked up first by later set-ups (the file is read
again when it changes), used only when they fit the problem."""
import numpy as np
import pytest

from paper_1807_00699_amd import gd
from paper_1807_00699_amd import inputs as I

pytestmark = pytest.mark.gpu


def _cfg(J, R):
    with gd.Solver(J, model=gd.GD_ISING) as S:
        S.set_init(R)
        return S.stats().kernel_config


def test_dense_picks_persist_in_the_cache_file(tmp_path, monkeypatch):
    f = tmp_path / "tune.txt"
    monkeypatch.setenv("GD_AUTOTUNE_CACHE", str(f))
    J = I.dense_pm1(1088, 3)                   # N = 1088 (no other test's size), R = 256: timed tuning
    c1 = _cfg(J, 256)
    lines = f.read_text().splitlines()
    head = lines[0]
    assert head.startswith("gd-autotune 1 ") and " build " in head
    dense = [l for l in lines[1:] if l.startswith("dense ")]
    assert len(dense) == 1 and dense[0].endswith(f" {c1}")
    key = dense[0].rsplit(" ", 1)[0]
    # an entry edited to another fitting variant (64x64, 64x128 or 32x64 tiles;
    # N = 1088 is a multiple of 64, not of 128)
    # is taken without timing
    other = next(c for c in (0, 1, 3) if c != c1)
    f.write_text(f"{head}\n{key} {other}\n")
    assert _cfg(J, 256) == other
    # an id that does not fit the problem is not used
    f.write_text(f"{head}\n{key} 9999\n")
    assert _cfg(J, 256) == other               # this process's own table
    # a file of another device or build is not trusted: the new problem
    # (R = 128) is tuned and the file rewritten with this build's header
    f.write_text(f"gd-autotune 1 another-device\n{key.replace(' 256 ', ' 128 ')} {other}\n")
    c4 = _cfg(J, 128)
    lines = f.read_text().splitlines()
    assert lines[0] == head
    assert any(l.startswith("dense ") and l.endswith(f" {c4}") for l in lines[1:])


def test_batch_picks_persist_in_the_cache_file(tmp_path, monkeypatch):
    f = tmp_path / "tune.txt"
    monkeypatch.setenv("GD_AUTOTUNE_CACHE", str(f))
    sizes, insts = I.maxcut_batch(24, 400, 1200, 5)   # sum n x R >= 2^16: timed tuning
    with gd.BatchSolver(insts) as B:
        B.set_init(64)
        c1 = B.stats().kernel_config
    lines = f.read_text().splitlines()
    batch = [l for l in lines[1:] if l.startswith("batch ")]
    assert len(batch) == 1 and batch[0].endswith(f" {c1}")
    key = batch[0].rsplit(" ", 1)[0]
    other = 5 if c1 != 5 else 0                # 4 or 8 trajectories x 1024 threads, couplings in LDS
    f.write_text(f"{lines[0]}\n{key} {other}\n")
    with gd.BatchSolver(insts) as B:
        B.set_init(64)
        assert B.stats().kernel_config == other
        B.run(10)
        assert B.stats().diverged == 0
