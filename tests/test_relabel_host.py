"""Host side of the batched kernel's spin relabeling (gd_relabel.h), built
with the host compiler: the labels are a permutation, the conflict counts it
reports are those of its labels, and on random 3-regular graphs it removes
nearly every duplicate residue of a gather pass."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1807_00699_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1807_00699_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("relabel") / "relabel_driver")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "relabel_driver.cpp"), "-o", exe], check=True)
    return exe


def run(exe, nb, g, bs, seed=1, moves=None):
    n = nb.shape[0]
    moves = 12 * n if moves is None else moves
    txt = f"{n} {g} {bs} {seed} {moves}\n" + "\n".join(" ".join(map(str, r)) for r in nb) + "\n"
    out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout.split()
    return int(out[0]), int(out[1]), np.array(out[2:], np.int64)


def conflicts(nb, lab, g, bs):
    """Duplicates of (block of the updated spin's label, d, residue of the
    neighbour's label) over present neighbours, counted directly."""
    n = nb.shape[0]
    tot = 0
    for d in range(3):
        j = nb[:, d]
        ok = j < n
        key = (lab[ok] // bs) * g + lab[j[ok]] % g
        _, cnt = np.unique(key, return_counts=True)
        tot += int((cnt - 1).sum())
    return tot


def regular3_lists(n, seed):
    e = I.regular3_edges(n, seed)
    adj = [[] for _ in range(n)]
    for a, b in e:
        adj[a].append(b)
        adj[b].append(a)
    return np.array([sorted(a) for a in adj], np.int64)


@pytest.mark.parametrize("n,g", [(2000, 32), (1000, 16), (600, 8), (300, 4)])
def test_random_regular_graphs(driver, n, g):
    nb = regular3_lists(n, n + g)
    bs = g // 2
    c0, c1, lab = run(driver, nb, g, bs)
    assert np.array_equal(np.sort(lab), np.arange(n))
    assert c0 == conflicts(nb, np.arange(n), g, bs)
    assert c1 == conflicts(nb, lab, g, bs)
    assert c1 <= 0.05 * c0, (c0, c1)
    # deterministic for a seed
    assert np.array_equal(run(driver, nb, g, bs)[2], lab)


def test_identity_without_blocks_and_small_instances(driver):
    nb = regular3_lists(64, 5)
    assert np.array_equal(run(driver, nb, 2, 1)[2], np.arange(64))    # one row per pass
    assert np.array_equal(run(driver, nb, 1, 1)[2], np.arange(64))
    # fewer spins than residues, missing couplings (index n)
    small = np.array([[1, 2, 5], [0, 5, 5], [0, 3, 5], [2, 4, 5], [3, 5, 5]], np.int64)
    c0, c1, lab = run(driver, small, 32, 16)
    assert np.array_equal(np.sort(lab), np.arange(5))
    assert c1 == conflicts(small, lab, 32, 16) and c1 <= c0


def test_many_spins_pointing_at_one(driver):
    """Neighbour lists need not be symmetric: every spin names spin 0 first."""
    n = 200
    rng = np.random.default_rng(3)
    nb = np.stack([np.zeros(n, np.int64), rng.integers(1, n, n), rng.integers(1, n, n)], 1)
    nb[0, 0] = 1
    c0, c1, lab = run(driver, nb, 16, 8)
    assert np.array_equal(np.sort(lab), np.arange(n))
    assert c1 == conflicts(nb, lab, 16, 8) and c1 <= c0
