"""Batched uneven instances (sparse couplings, one persistent launch, hipGraph
replay, autotuned variant) against the FP64 oracle, instance by instance.

The amplitude/gain bar is the one of the dense tests (tests/_parity.py: per
trajectory 1e-4, or 4x the oracle's own float32-vs-float64 distance where the
dynamics amplify rounding; >= 90% of all trajectories under 1e-4; the count
reported).  The oracle computes each instance's coupling scale itself.
Energies of the discretised state are integer-exact.  A trajectory's result
must not depend on the rest of the batch, on the kernel variant or on how the
steps are chunked into graph replays: those comparisons are bitwise.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1807_00699_amd import gd
from paper_1807_00699_amd import inputs as I

import _parity as P

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _instances(sizes, seed, csr=True):
    insts, dense = [], []
    for k, n in enumerate(sizes):
        e, w, _ = I.regular3_maxcut(int(n), seed + k)
        J = I.edges_to_dense(int(n), e, w)
        dense.append(J)
        if csr:
            rows = [[] for _ in range(n)]
            for (a, b), v in zip(e, w):
                rows[a].append((b, v))
                rows[b].append((a, v))
            rp = np.zeros(n + 1, np.int32)
            col, val = [], []
            for i in range(n):
                rows[i].sort()
                col += [c for c, _ in rows[i]]
                val += [v for _, v in rows[i]]
                rp[i + 1] = len(col)
            insts.append(dict(n=int(n), row_ptr=rp, col=np.array(col, np.int32), val=np.array(val, np.float32)))
        else:
            insts.append(dict(n=int(n), J=J))
    return insts, dense


def _psi0(sizes, R, seed):
    return [I.psi0_real(int(n), R, seed + k) for k, n in enumerate(sizes)]


def _rel(a, b):
    a = a.reshape(a.shape[0], -1).astype(np.float64)
    b = b.reshape(b.shape[0], -1).astype(np.float64)
    return np.abs(a - b).max(1) / np.maximum(np.abs(b).max(1), 1e-30)


def test_batch_parity_against_oracle_per_instance():
    sizes = [50, 62, 100, 158, 200, 250, 300]
    R = 8
    insts, dense = _instances(sizes, 10)
    x0 = _psi0(sizes, R, 10)
    with gd.BatchSolver(insts, dt=0.05, eps=0.1) as B:
        B.set_init(R, np.concatenate([x.ravel() for x in x0]))
        prev = 0
        ox = [x.astype(np.float64) for x in x0]
        og = [np.zeros_like(x, np.float64) for x in x0]
        fl = [P.Floor(J, x0[k], None, model="ising", dt=0.05, eps=0.1) for k, J in enumerate(dense)]
        for st in (1, 10, 50, 100, 200):
            B.run(st - prev)
            xs, gs, step = B.state()
            assert step == st
            strict = []
            for k, J in enumerate(dense):
                ox[k], og[k] = O.run(J, ox[k], og[k], model="ising", steps=st - prev, dt=0.05, eps=0.1)
                fl[k].advance(st - prev)
                ep = _rel(B.split(xs)[k], ox[k])
                eg = _rel(B.split(gs)[k], og[k])
                floor = fl[k].floor(ox[k], og[k])
                P.check(ep, eg, floor, min_strict=0.0, label=f"instance {k} n={sizes[k]} step {st}")
                strict.append((ep <= TOL) & (eg <= TOL))
            assert np.mean(np.concatenate(strict)) >= 0.9, st
            prev = st
        E, best = B.energy()
        sp = B.split(B.spins())
        xs, _, _ = B.state()
    for k, J in enumerate(dense):
        assert np.array_equal(sp[k], O.ising_spins(B.split(xs)[k]))
        Eo = O.energy_ising(J, sp[k])
        assert np.array_equal(E[k], Eo.astype(np.float64))
        assert best[k] == int(np.argmin(Eo))


def test_batch_independence_variants_and_graph_chunks_bitwise():
    sizes = [64, 130, 258, 96]
    R = 16
    insts, _ = _instances(sizes, 20)
    x0 = np.concatenate([x.ravel() for x in _psi0(sizes, R, 20)])
    ref = None
    # 0-6: couplings in LDS; 7-14: neighbours in registers (packed form),
    # 11-12 uniform rates, 12-14 double-buffered amplitudes; 15-20: item width
    # chosen per instance (all 16 trajectories in one item at 8192
    # spin-trajectories per item, 15-16; the 258-spin instance in items of 8
    # at 4096, 17-18, and at 3072 and 2048, 19-20), spins relabeled, the
    # state staged through LDS; the energies of the final state (a zero-step
    # launch of the same variant) too
    for cfg in ("0", "1", "2", "6", "7", "8", "9", "10", "11", "12", "13", "14", "15", "16", "17", "18", "19", "20"):
        os.environ["GD_BATCH_CONFIG"] = cfg
        try:
            with gd.BatchSolver(insts, check_interval=25) as B:
                B.set_init(R, x0)
                B.run(200)
                out = B.state() + B.energy()
                assert B.stats().kernel_config == int(cfg)
        finally:
            del os.environ["GD_BATCH_CONFIG"]
        if ref is None:
            ref = out
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), cfg
        assert np.array_equal(out[3], ref[3]) and np.array_equal(out[4], ref[4]), cfg
    # one graph of 200 steps vs 8 replays of a 25-step graph (autotuned variant)
    with gd.BatchSolver(insts) as B:
        B.set_init(R, x0)
        B.run(200)
        one = B.state()
    assert np.array_equal(one[0], ref[0]) and np.array_equal(one[1], ref[1])
    # an instance alone equals the same instance inside the batch
    k = 2
    off = sum(n * R for n in sizes[:k])
    with gd.BatchSolver([insts[k]]) as B:
        B.set_init(R, x0[off:off + sizes[k] * R])
        B.run(200)
        alone = B.state()
    assert np.array_equal(alone[0], ref[0][off:off + sizes[k] * R])


def test_relabeled_gathers_give_the_same_bits():
    """The per-instance-width variants relabel each instance's spins for
    their LDS gathers; with GD_BATCH_RELABEL=0 they keep the given order.
    Same states, gains and energies either way (sizes from one-row items to
    items of two trajectories, where the relabeling has most to do)."""
    sizes = [40, 120, 500, 1000, 2000]
    R = 32
    insts, _ = _instances(sizes, 41)
    x0 = np.concatenate([x.ravel() for x in _psi0(sizes, R, 41)])
    outs = []
    for relabel in ("1", "0"):
        os.environ["GD_BATCH_CONFIG"] = "18"
        if relabel == "0":
            os.environ["GD_BATCH_RELABEL"] = "0"
        try:
            with gd.BatchSolver(insts, check_interval=30) as B:
                B.set_init(R, x0)
                B.run(90)
                outs.append(B.state() + B.energy())
        finally:
            del os.environ["GD_BATCH_CONFIG"]
            os.environ.pop("GD_BATCH_RELABEL", None)
    a, b = outs
    for q in (0, 1, 3, 4):
        assert np.array_equal(a[q], b[q]), q


def test_batch_gauge_symmetry_and_dense_input():
    n, R = 120, 8
    e, w, s = I.regular3_maxcut(n, 33)
    J = I.edges_to_dense(n, e, w)
    Jplain = I.gauge(J, s)          # undo the gauge: all couplings -1
    x0 = I.psi0_real(n, R, 33)
    with gd.BatchSolver([dict(n=n, J=J)]) as A, gd.BatchSolver([dict(n=n, J=Jplain)]) as B:
        A.set_init(R, (x0 * s[None]).ravel())
        B.set_init(R, x0.ravel())
        A.run(300)
        B.run(300)
        xa, ga, _ = A.state()
        xb, gb, _ = B.state()
    assert np.array_equal(xa.reshape(R, n), xb.reshape(R, n) * s[None])
    assert np.array_equal(ga, gb)
    insts, _ = _instances([n], 33, csr=True)
    with gd.BatchSolver(insts) as C:
        C.set_init(R, (x0 * s[None]).ravel())
        C.run(300)
        xc, _, _ = C.state()
    assert np.array_equal(xc, xa)


def test_batch256_full_size_sampled():
    """256 random 3-regular max-cut instances, N_k even in [50, 2000], R = 64,
    the benchmark's configuration: 200 steps, three instances checked against
    the oracle on 4 trajectories each, exact energies on all."""
    K, R = 256, 64
    sizes = I.even_sizes(K, 50, 2000, 1)
    dense = [I.regular3_maxcut(int(n), 1000 + k)[:2] for k, n in enumerate(sizes)]
    insts = []
    for k, n in enumerate(sizes):
        e, w = dense[k]
        rows = np.concatenate([e, e[:, ::-1]])
        vals = np.concatenate([w, w])
        order = np.lexsort((rows[:, 1], rows[:, 0]))
        rows, vals = rows[order], vals[order]
        rp = np.zeros(n + 1, np.int32)
        np.add.at(rp, rows[:, 0] + 1, 1)
        insts.append(dict(n=int(n), row_ptr=np.cumsum(rp).astype(np.int32),
                          col=rows[:, 1].astype(np.int32), val=vals.astype(np.float32)))
    x0 = [I.psi0_real(int(n), R, 5000 + k) for k, n in enumerate(sizes)]
    with gd.BatchSolver(insts, check_interval=50) as B:
        B.set_init(R, np.concatenate([x.ravel() for x in x0]))
        B.run(200)
        xs, gs, _ = B.state()
        E, best = B.energy()
        sp = B.split(B.spins())
        st = B.stats()
    assert st.diverged == 0 and st.steps_done == 200
    xk = B.split(xs)
    for k in (int(np.argmin(sizes)), int(np.argmax(sizes)), 100):
        J = I.edges_to_dense(int(sizes[k]), *dense[k])
        sub = [0, 1, 31, 63]
        xo, go = O.run(J, x0[k][sub], model="ising", steps=200, dt=0.05, eps=0.1)
        fl = P.Floor(J, x0[k][sub], None, model="ising", dt=0.05, eps=0.1)
        fl.advance(200)
        ep = _rel(xk[k][sub], xo)
        assert np.all(ep <= np.maximum(TOL, 4 * fl.floor(xo, go))), (k, ep)
        Eo = O.energy_ising(J, sp[k])
        assert np.array_equal(E[k], Eo.astype(np.float64))


def test_batch_targets_and_ttt():
    sizes = [20, 20]
    R = 32
    insts, dense = _instances(sizes, 40)
    targets = np.array([O.brute_ising(J)[0] for J in dense], np.float64)
    with gd.BatchSolver(insts, check_interval=100, has_target=1) as B:
        B.set_init(R, np.concatenate([x.ravel() for x in _psi0(sizes, R, 40)]))
        B.set_targets(targets)
        B.run(4000)
        sec, steps, best = B.ttt()
        st = B.stats()
    assert np.all(best == targets), (best, targets)
    assert np.all(sec >= 0) and np.all(steps > 0) and np.all(steps % 100 == 0)
    assert st.target_reached == 1 and st.steps_done <= 4000


def test_batch_errors():
    n = 10
    J = np.zeros((n, n), np.float32)
    J[0, 1] = 1.0
    with pytest.raises(gd.GDError) as ei:
        gd.BatchSolver([dict(n=n, J=J)])
    assert ei.value.code == gd.GD_E_NOT_SYMMETRIC
    J[1, 0] = 1.0
    with pytest.raises(gd.GDError) as ei:
        gd.BatchSolver([dict(n=n, J=J)], integrator=gd.GD_RK4)
    assert ei.value.code == gd.GD_E_UNSUPPORTED
    with gd.BatchSolver([dict(n=n, J=J)]) as B:
        with pytest.raises(gd.GDError) as ei:
            B.energy()
        assert ei.value.code == gd.GD_E_STATE


def test_batch_deferred_best_matches_per_check_readback():
    """Without targets the per-instance best of the checks stays on the
    device until the run ends; with targets (here never reached) the host
    reads every check.  Same per-instance best energies and the same overall
    best after each of three runs (130, 75, 200 steps, checks every 25: the
    last chunk of a run is shorter and is checked too)."""
    sizes = [64, 130, 258, 96]
    R = 16
    insts, _ = _instances(sizes, 41)
    x0 = np.concatenate([x.ravel() for x in _psi0(sizes, R, 41)])
    out = []
    for tracked in (False, True):
        seen = []
        with gd.BatchSolver(insts, check_interval=25) as B:
            if tracked:
                B.set_targets(np.full(len(sizes), -1e30))
            B.set_init(R, x0)
            for k in (130, 75, 200):
                B.run(k)
                _, _, be = B.ttt()
                st = B.stats()
                seen.append((be.tolist(), st.best_energy, st.best_index, st.steps_done))
        out.append(seen)
    assert out[0] == out[1], out
    assert all(np.all(np.isfinite(s[0])) for s in out[0])


def test_missing_couplings_pad_to_the_zero_row():
    """Instances of degree 1-3 (3-regular graphs with every fifth edge
    removed): the packed, relabeled variants point a missing coupling at the
    instance's zero row; they agree bit for bit with the ELL variant 0 and
    their readout's energies are the oracle's."""
    sizes = [60, 300, 1500]
    R = 16
    insts, dense = [], []
    for k, n in enumerate(sizes):
        e, w, _ = I.regular3_maxcut(n, 70 + k)
        keep = np.arange(e.shape[0]) % 5 != 0
        insts.append(I.edges_to_csr(n, e[keep], w[keep]))
        dense.append(I.edges_to_dense(n, e[keep], w[keep]))
        assert np.diff(insts[-1]["row_ptr"]).min() < 3
    x0 = np.concatenate([x.ravel() for x in _psi0(sizes, R, 70)])
    outs = {}
    for cfg in ("0", "18", "20"):
        os.environ["GD_BATCH_CONFIG"] = cfg
        try:
            with gd.BatchSolver(insts, check_interval=40) as B:
                B.set_init(R, x0)
                B.run(120)
                outs[cfg] = B.state() + B.energy()
                sp = B.split(B.spins())
        finally:
            del os.environ["GD_BATCH_CONFIG"]
        for k, J in enumerate(dense):
            assert np.array_equal(outs[cfg][3][k], O.energy_ising(J, sp[k]).astype(np.float64)), (cfg, k)
    for cfg in ("18", "20"):
        for q in (0, 1, 3):
            assert np.array_equal(outs[cfg][q], outs["0"][q]), (cfg, q)


def test_packed_variants_need_one_coupling_magnitude_per_instance():
    """A batch whose instance mixes coupling magnitudes (+-1 and +-2) has no
    packed form: pinning a packed variant is refused, a general one runs and
    matches the oracle's energies of its readout."""
    sizes = [80, 96]
    R = 8
    insts, dense = _instances(sizes, 40)
    v = insts[1]["val"].copy()
    v[::5] *= 2.0                       # symmetric: both (i, j) and (j, i) come from one edge value
    rp, col = insts[1]["row_ptr"], insts[1]["col"]
    Jm = np.zeros((96, 96), np.float32)
    for i in range(96):
        for q in range(rp[i], rp[i + 1]):
            Jm[i, col[q]] = v[q]
    if not np.array_equal(Jm, Jm.T):    # keep it symmetric: rebuild values from the dense matrix
        Jm = np.triu(Jm, 1)
        Jm = Jm + Jm.T
        v = np.array([Jm[i, col[q]] for i in range(96) for q in range(rp[i], rp[i + 1])], np.float32)
    insts[1] = dict(n=96, row_ptr=rp, col=col, val=v)
    dense[1] = Jm
    x0 = np.concatenate([x.ravel() for x in _psi0(sizes, R, 40)])
    os.environ["GD_BATCH_CONFIG"] = "7"
    try:
        with pytest.raises(gd.GDError) as ei:
            with gd.BatchSolver(insts) as B:
                B.set_init(R, x0)
        assert ei.value.code == gd.GD_E_INVALID_ARG
    finally:
        del os.environ["GD_BATCH_CONFIG"]
    with gd.BatchSolver(insts) as B:
        B.set_init(R, x0)
        B.run(100)
        assert B.stats().kernel_config < 7
        E, _ = B.energy()
        sp = B.split(B.spins())
    for k, J in enumerate(dense):
        assert np.array_equal(E[k], O.energy_ising(J, sp[k]).astype(np.float64))
