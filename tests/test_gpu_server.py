"""GPU tests of the serving loop (mfs_server_*): continuous batching of
incident-wave solves on a resident factored operator.

Each request's result must be the same alone on an idle server, in a mix of
requests that arrive while others iterate, and as a one-at-a-time plain solve
(mfs_solve_incident with that wave only); the first two incidences are also
checked against the CPU oracle (amplitudes and fields to 1e-10)."""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

import workloads as W
from oracle import geometry, onebody, periodic

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mfs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1506_05083_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def setup(mfs):
    pr = W.small_periodic(nwaves=6)
    b = pr.body
    ctx = mfs.create(0)
    sh = b.shape
    g = mfs.polar_geometry(sh.a, sh.eps, sh.j, b.M, b.N, b.tau, b.colloc)
    op = mfs.build_operator(ctx, [mfs.BodySpec(b.M, b.N, b.P, b.q, b.k, g)])
    op.factor_modes(1e-10)
    L = mfs.lattice(pr.lattice.ex, pr.lattice.ey, pr.lattice.z0, pr.lattice.p, pr.lattice.N0, pr.lattice.M1)
    waves = [(w.theta, w.phi) for w in pr.waves]
    ref = [mfs.solve_incident(ctx, op, L, [w], tol=1e-12, maxit=100, targets=pr.targets, q_field=pr.q_field)[0]
           for w in waves]
    return pr, ctx, op, L, waves, ref


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def same(r, s):
    assert np.array_equal(r.m, s.m) and np.array_equal(r.n, s.n)
    return max(rel(r.a, s.a), rel(r.b, s.b), rel(r.field, s.field))


def test_server_alone_mix_plain(mfs, setup):
    pr, ctx, op, L, waves, ref = setup
    srv = mfs.Server(ctx, op, L, slots=4, admit_batch=2, tol=1e-12, maxit=100, targets=pr.targets,
                     q_field=pr.q_field, hbm_budget=48 << 30)
    try:
        # alone: wave 0 on an idle server
        t = srv.submit(*waves[0])
        alone, lat0, ok = srv.wait(t)
        assert ok
        log(f"[server] alone: iters {alone.iters} latency {lat0:.1f} ms, vs plain solve {same(alone, ref[0]):.2e}")
        # mix: wave 1 first, the others (and wave 0 again) while it iterates
        tickets = [(1, srv.submit(*waves[1]))]
        t0 = time.perf_counter()
        while srv.stats()["iterating"] < 1 and time.perf_counter() - t0 < 120:
            time.sleep(0.0005)
        for i in (2, 3, 0, 4, 5):
            tickets.append((i, srv.submit(*waves[i])))
        peak = 0
        out = []
        for i, tk in tickets:
            while True:
                st = srv.stats()
                peak = max(peak, st["iterating"])
                r = srv.poll(tk)
                if r is not None:
                    break
                time.sleep(0.0005)
            res, lat, ok = r
            assert ok
            out.append((i, res, lat))
        log(f"[server] mix: most iterating at once {peak}")
        worst = 0.0
        for i, res, lat in out:
            d = same(res, ref[i])
            worst = max(worst, d)
            log(f"[server] wave {i}: iters {res.iters} (plain {ref[i].iters}) latency {lat:.1f} ms "
                f"vs plain solve {d:.2e} eps_flux {res.eps_flux:.2e}")
            assert res.eps_flux < 1e-6
        again = [res for i, res, _ in out if i == 0][0]
        d0 = same(again, alone)
        log(f"[server] wave 0 alone vs in the mix: {d0:.2e}")
        assert d0 <= 1e-13
        assert worst <= 1e-12
        # an unknown (or collected) ticket is an error, not a hang
        with pytest.raises(mfs.MfsError):
            srv.poll(tickets[0][1])
    finally:
        srv.close()


def test_server_matches_oracle(mfs, setup):
    pr, ctx, op, L, waves, ref = setup
    b, lat = pr.body, pr.lattice
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    ps = periodic.PeriodicSolver(b, lat, g, A)
    srv = mfs.Server(ctx, op, L, slots=2, admit_batch=2, tol=1e-12, maxit=100, targets=pr.targets,
                     q_field=pr.q_field, hbm_budget=48 << 30)
    try:
        tks = [srv.submit(*waves[i]) for i in (0, 1)]
        got = [srv.wait(t)[0] for t in tks]
    finally:
        srv.close()
    for i, r in enumerate(got):
        w = pr.waves[i]
        ps.set_wave(w)
        fh = onebody.rhs_modes(b, g, w)
        o = ps.solve(fh, tol=1e-12)
        u, _ = ps.field_and_grad(o["c"], o["d"], pr.targets, pr.q_field, want_grad=False)
        o_m, o_n = ps.orders.m, ps.orders.n
        assert np.array_equal(r.m, o_m) and np.array_equal(r.n, o_n)
        ea = rel(r.a, o["a"])
        eb = rel(r.b, o["b"])
        eu = float(np.linalg.norm(r.field - u) / np.linalg.norm(u))
        log(f"[server oracle] wave {i}: a {ea:.2e} b {eb:.2e} u {eu:.2e}")
        assert ea < 1e-10 and eb < 1e-10 and eu < 1e-10


def test_server_queue_full(mfs, setup):
    pr, ctx, op, L, waves, ref = setup
    srv = mfs.Server(ctx, op, L, slots=1, admit_batch=1, queue_cap=1, tol=1e-12, maxit=100,
                     hbm_budget=48 << 30)
    try:
        tks = []
        for i in range(6):
            t = srv.submit(*waves[i % len(waves)])
            tks.append(t)
        assert any(t is None for t in tks), "a queue of one must refuse some of six immediate requests"
        for t in tks:
            if t is not None:
                assert srv.wait(t)[2]
    finally:
        srv.close()


def test_server_transmission_matches_plain(mfs):
    """A transmission operator (2M x 2N mode blocks) behind the server: each
    request's result equals the one-at-a-time plain solve (the plain solve is
    checked against the oracle in the transmission parity tests)."""
    pr = W.small_periodic_transmission(nwaves=3)
    b, lat = pr.body, pr.lattice
    ctx = mfs.create(0)
    g = mfs.transmission_geometry(b.shape, b.M, b.N, b.tau, b.colloc)
    op = mfs.build_operator(ctx, [mfs.BodySpec(b.M, b.N, b.P, b.q, b.k, g, km=pr.km)])
    op.factor_modes(1e-10)
    L = mfs.lattice(lat.ex, lat.ey, lat.z0, lat.p, lat.N0, lat.M1)
    waves = [(w.theta, w.phi) for w in pr.waves]
    ref = [mfs.solve_incident(ctx, op, L, [w], tol=1e-12, maxit=100, targets=pr.targets, q_field=pr.q_field)[0]
           for w in waves]
    srv = mfs.Server(ctx, op, L, slots=2, admit_batch=2, tol=1e-12, maxit=100, targets=pr.targets,
                     q_field=pr.q_field, hbm_budget=48 << 30)
    try:
        tks = [srv.submit(*w) for w in waves]
        got = [srv.wait(t) for t in tks]
    finally:
        srv.close()
    for i, (res, lat_ms, ok) in enumerate(got):
        assert ok
        d = same(res, ref[i])
        log(f"[server trans] wave {i}: iters {res.iters} (plain {ref[i].iters}) vs plain {d:.2e} "
            f"eps_flux {res.eps_flux:.2e}")
        assert d <= 1e-12
        assert res.eps_flux < 1e-6


def test_server_memory_within_budget(mfs, setup):
    """With a budget that leaves room to factor one wave at a time, the
    device memory the library holds (its allocator's count of live buffers,
    peak over the whole run) stays within hbm_budget while six requests are
    admitted, factored, iterated and recovered, and the results are those of
    the one-at-a-time plain solves."""
    pr, ctx, op, L, waves, ref = setup
    budget = 1 << 30
    mfs.reset_memory_peak(0)
    base = mfs.memory_stats(0)["in_use"]
    srv = mfs.Server(ctx, op, L, slots=4, admit_batch=4, tol=1e-12, maxit=100, targets=pr.targets,
                     q_field=pr.q_field, hbm_budget=budget)
    try:
        tks = [srv.submit(*w) for w in waves]
        got = [srv.wait(t) for t in tks]
    finally:
        srv.close()
    st = mfs.memory_stats(0)
    held = st["peak"] - base
    log(f"[server memory] budget {budget / 2**20:.0f} MiB, peak held {held / 2**20:.0f} MiB, "
        f"after close {(st['in_use'] - base) / 2**20:.0f} MiB")
    assert held <= budget
    assert st["in_use"] - base <= 0
    for i, (res, _, ok) in enumerate(got):
        assert ok
        assert same(res, ref[i]) <= 1e-12
