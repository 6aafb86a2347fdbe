"""GPU parity: every step of the libmfs path, called through the C ABI,
against the CPU oracle on the same seeded inputs.

Tolerances (relative to the largest entry / the norm of the reference):
  fill, right-hand sides, point strengths, neighbour sums: 1e-12 -- these are
  direct sums of O(q) terms in FP64, different summation order only;
  singular values: 1e-13 * s_max absolute (backward-stable SVDs);
  fields and Bragg amplitudes: 1e-10 (the target accuracy of the method;
  the coefficient vectors themselves are not unique and are never compared).
"""
import dataclasses
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import geometry, mie, onebody, periodic

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
def ctx(mfs):
    return mfs.create(0)


def make_op(mfs, ctx, body: W.Body):
    g = mfs.body_geometry(body.shape, body.M, body.N, body.tau, body.colloc)
    return mfs.build_operator(ctx, [mfs.BodySpec(body.M, body.N, body.P, body.q, body.k, g)])


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


CASES = {"tiny": W.tiny_free_space, "sphere": W.sphere_free_space, "small_periodic": W.small_periodic,
         "cup": W.cup_free_space}


@pytest.mark.parametrize("name", list(CASES))
def test_fill_parity(mfs, ctx, name):
    pr = CASES[name]()
    b = pr.body
    log(f"[fill] {name} M={b.M} N={b.N} P={b.P} q={b.q}")
    op = make_op(mfs, ctx, b)
    Ag = op.blocks().cpu().numpy().transpose(0, 2, 1)        # [nd][M][N]
    g = geometry.build_geometry(b)
    Ao = onebody.modal_blocks(b, g)[: b.P // 2 + 1]
    err = rel(Ag, Ao)
    log(f"[fill] {name} max rel err {err:.2e}")
    assert err < 1e-12


def test_fill_parity_periodic_k10_sampled(mfs, ctx):
    """Full size of the k = 10 periodic body (240 x 200, 33 blocks, q = 400),
    sampled rows against the oracle's per-row fill."""
    b = W.periodic_k10(1).body
    log("[fill] periodic_k10")
    op = make_op(mfs, ctx, b)
    Ag = op.blocks().cpu().numpy().transpose(0, 2, 1)
    g = geometry.build_geometry(b)
    rows = np.array([0, 1, 57, 119, 120, 201, 238, 239])
    s = onebody.ring_samples_dGdn(b, g, b.q, rows)
    Ao = (np.fft.fft(s, axis=2) / b.q)[:, :, : b.P // 2 + 1]      # [rows][N][nd]
    err = rel(Ag[:, rows, :], np.transpose(Ao, (2, 0, 1)))
    log(f"[fill] periodic_k10 sampled max rel err {err:.2e}")
    assert err < 1e-12


def test_rhs_and_strengths_parity(mfs, ctx):
    import torch
    pr = W.small_periodic()
    b = pr.body
    op = make_op(mfs, ctx, b)
    g = geometry.build_geometry(b)
    kv = np.stack([W.wave_vector(b.k, w) for w in pr.waves])
    fg = mfs.rhs_modes(op, kv).cpu().numpy()
    fo = np.stack([onebody.rhs_modes(b, g, w) for w in pr.waves])
    log(f"[rhs] max rel err {rel(fg, fo):.2e}")
    assert rel(fg, fo) < 1e-12
    rng = np.random.default_rng(9)
    c = rng.standard_normal((2, b.P, b.N)) + 1j * rng.standard_normal((2, b.P, b.N))
    for qs in (b.P, 3 * b.P):
        sg = mfs.point_strengths(op, torch.from_numpy(c).cuda(), qs).cpu().numpy()
        so = np.stack([onebody.point_strengths(c[i], qs) for i in range(2)])
        log(f"[strengths] qs={qs} max rel err {rel(sg, so):.2e}")
        assert rel(sg, so) < 1e-12


def test_factor_singular_values_and_ranks(mfs, ctx):
    pr = W.small_periodic()
    b = pr.body
    op = make_op(mfs, ctx, b)
    ranks = op.factor_modes(1e-10)
    sv = op.singular_values()
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    for n in range(b.P // 2 + 1):
        s = np.linalg.svd(A[n], compute_uv=False)
        err = np.max(np.abs(sv[n] - s)) / s[0]
        assert err < 1e-13, (n, err)
        assert abs(int(ranks[n]) - int(np.sum(s > 1e-10 * s[0]))) <= 1, n
    log(f"[factor] ranks {list(ranks)}")


def test_batched_build_uneven_bodies(mfs, ctx):
    """Several obstacles of uneven M, N, P, q and k filled in one persistent
    launch and factored in one batch: every body's singular values and its
    free-space field (RHS, apply, point-source field) against the oracle."""
    bodies = [W.Body(W.Shape(0.3, 0.1, 3), N=40, M=48, P=24, q=160, k=5.0, tau=0.2),
              W.Body(W.Shape(0.25, 0.05, 2), N=30, M=36, P=16, q=120, k=7.0, tau=0.15),
              W.Body(W.Shape(0.35), N=24, M=30, P=8, q=96, k=3.0, tau=0.2)]
    specs = []
    for b in bodies:
        g = mfs.body_geometry(b.shape, b.M, b.N, b.tau, b.colloc)
        specs.append(mfs.BodySpec(b.M, b.N, b.P, b.q, b.k, g))
    op = mfs.build_operator(ctx, specs)
    ranks = op.factor_modes(1e-10)
    off = 0
    tg = W.fibonacci_sphere(16, 2.0)
    for i, b in enumerate(bodies):
        g = geometry.build_geometry(b)
        A = onebody.modal_blocks(b, g)
        sv = op.singular_values(i)
        worst = 0.0
        for n in range(b.P // 2 + 1):
            s = np.linalg.svd(A[n], compute_uv=False)
            worst = max(worst, float(np.max(np.abs(sv[n] - s)) / s[0]))
            assert abs(int(ranks[off + n]) - int(np.sum(s > 1e-10 * s[0]))) <= 1, (i, n)
        off += b.P // 2 + 1
        w = W.sample_waves(b.k, None, 1, seed=20 + i)[0]
        kv = W.wave_vector(b.k, w)[None, :]
        fh = mfs.rhs_modes(op, kv, body=i)
        c = mfs.apply_solution_op(op, fh, body=i)
        u = mfs.field_free(op, c, 2 * b.P, tg, body=i).cpu().numpy()[0]
        co = onebody.solve_modes(A, onebody.rhs_modes(b, g, w))
        uo = onebody.field(b, g, co, tg, 2 * b.P)
        err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
        log(f"[batch] body {i}: N={b.N} M={b.M} P={b.P} sv err {worst:.2e} field err {err:.2e}")
        assert worst < 1e-13 and err < 1e-10


@pytest.mark.parametrize("name", ["tiny", "sphere", "cup"])
def test_free_space_fields(mfs, ctx, name):
    """Whole one-body path on the GPU (fill, QR + Jacobi truncation, RHS,
    apply, point-source field) against the oracle's field; the sphere also
    against the Mie series."""
    pr = CASES[name]()
    b = pr.body
    log(f"[free] {name}")
    op = make_op(mfs, ctx, b)
    op.factor_modes(1e-10)
    kv = np.stack([W.wave_vector(b.k, w) for w in pr.waves])
    fh = mfs.rhs_modes(op, kv)
    c = mfs.apply_solution_op(op, fh)
    u = mfs.field_free(op, c, pr.q_field, pr.targets).cpu().numpy()[0]
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    co = onebody.solve_modes(A, onebody.rhs_modes(b, g, pr.waves[0]))
    uo = onebody.field(b, g, co, pr.targets, pr.q_field)
    err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    log(f"[free] {name} field rel err vs oracle {err:.2e}")
    assert err < 1e-10
    if name == "sphere":
        um = mie.sound_hard_sphere(b.k, b.shape.a, kv[0], pr.targets)
        em = np.linalg.norm(u - um) / np.linalg.norm(um)
        log(f"[free] sphere rel err vs Mie {em:.2e}")
        assert em < 1e-9


def _small_periodic_unpaired(nwaves=2):
    """The small polar body with M = 44: (P/2) M = 528 is not a multiple of
    64, so the stored surface sums keep all targets (no mirror pairing)."""
    pr = W.small_periodic(nwaves=nwaves)
    return dataclasses.replace(pr, body=dataclasses.replace(pr.body, M=44))


@pytest.fixture(scope="module", params=["polar", "cup", "polar_unpaired"])
def small_oracle(request):
    pr = {"polar": W.small_periodic, "cup": W.small_periodic_cup,
          "polar_unpaired": _small_periodic_unpaired}[request.param](nwaves=2)
    b, lat = pr.body, pr.lattice
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    ps = periodic.PeriodicSolver(b, lat, g, A)
    out = []
    for w in pr.waves:
        ps.set_wave(w)
        fh = onebody.rhs_modes(b, g, w)
        r = ps.solve(fh, tol=1e-12)
        u, _ = ps.field_and_grad(r["c"], r["d"], pr.targets, pr.q_field, want_grad=False)
        out.append(dict(alpha=ps.alpha, beta=ps.beta, Kelse=ps.Kelse.copy(), Cpt=ps.Cpt.copy(),
                        res=r, u=u, m=ps.orders.m.copy(), n=ps.orders.n.copy(),
                        flux=ps.eps_flux(r["a"], r["b"])))
    return pr, g, out


def _lat(mfs, lat):
    return mfs.lattice(lat.ex, lat.ey, lat.z0, lat.p, lat.N0, lat.M1)


def test_neighbour_sum_parity(mfs, ctx, small_oracle):
    import torch
    pr, g, out = small_oracle
    b = pr.body
    op = make_op(mfs, ctx, b)
    rng = np.random.default_rng(4)
    sig = rng.standard_normal((2, b.P, b.N)) + 1j * rng.standard_normal((2, b.P, b.N))
    ab = np.array([[o["alpha"], o["beta"]] for o in out])
    L = _lat(mfs, pr.lattice)
    st = torch.from_numpy(sig).cuda()
    gs = mfs.neighbour_sum(op, L, st, ab, mfs.TARGETS_SURFACE).cpu().numpy()
    gw = mfs.neighbour_sum(op, L, st, ab, mfs.TARGETS_WALLS).cpu().numpy()
    for i in range(2):
        es = rel(gs[i], out[i]["Kelse"] @ sig[i].reshape(-1))
        ew = rel(gw[i], out[i]["Cpt"] @ sig[i].reshape(-1))
        log(f"[nsum] wave {i} surface {es:.2e} walls {ew:.2e}")
        assert es < 1e-12 and ew < 1e-12
    # user targets, value and derivative, all 9 copies
    X = pr.targets[:10]
    d = rng.standard_normal((10, 3))
    user = np.concatenate([X, d], axis=1)
    Y = geometry.source_ring_points(g, b.P).reshape(-1, 3)
    for want in (0, 1):
        gu = mfs.neighbour_sum(op, L, st, ab, mfs.TARGETS_USER, user=user, want=want).cpu().numpy()
        imgs = periodic.image_list(pr.lattice, out[0]["alpha"], out[0]["beta"], periodic.NEAR9)
        Vm, Gm = periodic.near_matrices(b.k, Y, X, imgs)
        ref = (Vm @ sig[0].reshape(-1)) if want == 0 else np.einsum("tsc,tc,s->t", Gm, d, sig[0].reshape(-1))
        log(f"[nsum] user want={want} {rel(gu[0], ref):.2e}")
        assert rel(gu[0], ref) < 1e-12


@pytest.mark.parametrize("near", ["dense", "on_the_fly", "low_rank", "low_rank_halfturn"])
def test_periodic_solve_parity_small(mfs, ctx, small_oracle, near, monkeypatch):
    """Whole periodic path on the GPU (Q fill and factorisation, batched
    GMRES with the neighbour sums, recovery) for two incidences against the
    oracle: Bragg amplitudes and cell fields to 1e-10, with the near-field
    kernel values stored once (default), evaluated every iteration, or (the
    surface sums) from low-rank factors of the image blocks, in the
    quarter-turn form (two classes of four images) and the half-turn form
    (four classes of two)."""
    pr, g, out = small_oracle
    b = pr.body
    op = make_op(mfs, ctx, b)
    if near != "dense":
        op.set_near_field_budget(0)
    if near.startswith("low_rank"):
        monkeypatch.setenv("MFS_NEAR_LOWRANK", "2")
        monkeypatch.setenv("MFS_LOWRANK_HALFTURN", "1" if near.endswith("halfturn") else "0")
    op.factor_modes(1e-10)
    L = _lat(mfs, pr.lattice)
    res = mfs.solve_incident(ctx, op, L, [(w.theta, w.phi) for w in pr.waves], tol=1e-12, maxit=100,
                             targets=pr.targets, q_field=pr.q_field)
    for i, r in enumerate(res):
        o = out[i]
        assert np.array_equal(r.m, o["m"]) and np.array_equal(r.n, o["n"])
        ea = np.max(np.abs(r.a - o["res"]["a"])) / np.max(np.abs(o["res"]["a"]))
        eb = np.max(np.abs(r.b - o["res"]["b"])) / np.max(np.abs(o["res"]["b"]))
        eu = np.linalg.norm(r.field - o["u"]) / np.linalg.norm(o["u"])
        log(f"[periodic {near}] wave {i} iters gpu {r.iters} oracle {o['res']['iters']} a {ea:.2e} b {eb:.2e} "
            f"u {eu:.2e} flux gpu {r.eps_flux:.2e} oracle {o['flux']:.2e}")
        assert ea < 1e-10 and eb < 1e-10 and eu < 1e-10
        # the flux defect is the discretisation's (1.8e-6 for the small cup):
        # the same on both sides, and small
        assert abs(r.eps_flux - o["flux"]) < 1e-12 + 1e-6 * o["flux"]
        assert r.eps_flux < 1e-5


def test_wide_jacobi_blocks(mfs, ctx, small_oracle, monkeypatch):
    """The 32-column Jacobi blocks (matrix-core Gram of the ten Hermitian
    block pairs, 64 x 64 inner sweep, matrix-core apply), which the library
    takes for factors of 2048 columns and more, forced on the small bodies:
    singular values against LAPACK on the GPU's own blocks, the same ranks as
    with 16-column blocks, and the periodic solve (whose Q^+ then uses them
    as well, on a factor of several hundred columns) against the oracle."""
    pr, g, out = small_oracle
    b = pr.body
    op16 = make_op(mfs, ctx, b)
    r16 = list(op16.factor_modes(1e-10))
    monkeypatch.setenv("MFS_JACOBI_WIDE_MIN_COLS", "0")
    op = make_op(mfs, ctx, b)
    blocks = op.blocks().cpu().numpy().transpose(0, 2, 1)   # [P/2+1][M][N]
    r32 = list(op.factor_modes(1e-10))
    sv = op.singular_values(0)
    e = 0.0
    for n in range(blocks.shape[0]):
        s_own = np.linalg.svd(blocks[n], compute_uv=False)
        e = max(e, float(np.max(np.abs(sv[n][: s_own.size] - s_own)) / s_own[0]))
    log(f"[wide jacobi] singular values vs LAPACK {e:.2e} (of s_max); ranks equal {r32 == r16}")
    assert e < 1e-13
    assert r32 == r16
    L = _lat(mfs, pr.lattice)
    res = mfs.solve_incident(ctx, op, L, [(w.theta, w.phi) for w in pr.waves], tol=1e-12, maxit=100,
                             targets=pr.targets, q_field=pr.q_field)
    for i, r in enumerate(res):
        o = out[i]
        ea = np.max(np.abs(r.a - o["res"]["a"])) / np.max(np.abs(o["res"]["a"]))
        eb = np.max(np.abs(r.b - o["res"]["b"])) / np.max(np.abs(o["res"]["b"]))
        eu = np.linalg.norm(r.field - o["u"]) / np.linalg.norm(o["u"])
        log(f"[wide jacobi] wave {i} iters gpu {r.iters} oracle {o['res']['iters']} a {ea:.2e} b {eb:.2e} "
            f"u {eu:.2e}")
        assert ea < 1e-10 and eb < 1e-10 and eu < 1e-10


@pytest.mark.parametrize("nb", [16, 32, 64])
def test_qr_panel_widths(mfs, ctx, small_oracle, monkeypatch, nb):
    """Every panel width the QR tuner can pick (16, 32, 64), forced through
    MFS_QR_NB: the one-body factors' singular values against LAPACK on the
    GPU's own blocks and, with the periodizer Q factored at that width too,
    the periodic solve against the oracle (amplitudes and fields 1e-10)."""
    pr, g, out = small_oracle
    b = pr.body
    monkeypatch.setenv("MFS_QR_NB", str(nb))
    op = make_op(mfs, ctx, b)
    blocks = op.blocks().cpu().numpy().transpose(0, 2, 1)
    op.factor_modes(1e-10)
    sv = op.singular_values(0)
    e = 0.0
    for n in range(blocks.shape[0]):
        s_own = np.linalg.svd(blocks[n], compute_uv=False)
        e = max(e, float(np.max(np.abs(sv[n][: s_own.size] - s_own)) / s_own[0]))
    res = mfs.solve_incident(ctx, op, _lat(mfs, pr.lattice), [(w.theta, w.phi) for w in pr.waves], tol=1e-12,
                             maxit=100, targets=pr.targets, q_field=pr.q_field)
    for i, r in enumerate(res):
        o = out[i]
        ea = np.max(np.abs(r.a - o["res"]["a"])) / np.max(np.abs(o["res"]["a"]))
        eb = np.max(np.abs(r.b - o["res"]["b"])) / np.max(np.abs(o["res"]["b"]))
        eu = np.linalg.norm(r.field - o["u"]) / np.linalg.norm(o["u"])
        log(f"[qr nb={nb}] sv {e:.2e} wave {i} a {ea:.2e} b {eb:.2e} u {eu:.2e}")
        assert ea < 1e-10 and eb < 1e-10 and eu < 1e-10
    assert e < 1e-13


@pytest.mark.parametrize("form", ["blocked", "unblocked", "sketched"])
def test_pivoted_qr_forms(mfs, ctx, monkeypatch, form):
    """The three forms of the column-pivoted QR of the triangles (blocked:
    panels of 32 with the updates deferred and the norms downdated;
    unblocked: one column step at a time, norms recomputed; sketched: the
    pivots of each 32-column block chosen on a Gaussian sketch, the block
    factored unpivoted and the rest updated once), forced on the small periodic
    body and on the k = 10 body (its 200-column blocks need 7 panels):
    singular values against LAPACK on the GPU's own blocks, 1e-13 of the
    largest; the same kept ranks either way."""
    monkeypatch.setenv("MFS_QRCP", form)
    for b in (W.small_periodic().body, W.periodic_k10(1).body):
        op = make_op(mfs, ctx, b)
        blocks = op.blocks().cpu().numpy().transpose(0, 2, 1)
        ranks = op.factor_modes(1e-10)
        sv = op.singular_values(0)
        e = 0.0
        for n in range(blocks.shape[0]):
            s_own = np.linalg.svd(blocks[n], compute_uv=False)
            e = max(e, float(np.max(np.abs(sv[n][: s_own.size] - s_own)) / s_own[0]))
            assert abs(int(ranks[n]) - int(np.sum(s_own > 1e-10 * s_own[0]))) <= 1, n
        log(f"[qrcp {form}] N={b.N} P={b.P}: singular values vs LAPACK {e:.2e}")
        assert e < 1e-13


def test_qpinv_reflectors_match_formed_u(mfs, ctx, monkeypatch):
    """The full-rank periodizer's Q^+ applied from its QR's reflectors (panel
    by panel, MFS_QPINV_REFLECT=1) against the default with U = Q_1 formed,
    k = 10 workload, two incidences: Bragg amplitudes and fields to 1e-12."""
    pr = W.periodic_k10(2)
    b = pr.body
    op = make_op(mfs, ctx, b)
    op.factor_modes(1e-10)
    L = _lat(mfs, pr.lattice)
    waves = [(w.theta, w.phi) for w in pr.waves]
    kw = dict(tol=1e-12, maxit=pr.maxit, targets=pr.targets, q_field=pr.q_field)
    monkeypatch.setenv("MFS_QPINV_REFLECT", "1")
    res_r = mfs.solve_incident(ctx, op, L, waves, **kw)
    monkeypatch.delenv("MFS_QPINV_REFLECT", raising=False)
    res_u = mfs.solve_incident(ctx, op, L, waves, **kw)
    for a, c in zip(res_r, res_u):
        assert a.q_rank == a.nq_cols == c.q_rank   # the direct (full-rank) form
        ea = np.max(np.abs(a.a - c.a)) / np.max(np.abs(c.a))
        eb = np.max(np.abs(a.b - c.b)) / np.max(np.abs(c.b))
        eu = np.linalg.norm(a.field - c.field) / np.linalg.norm(c.field)
        log(f"[qpinv reflectors] a {ea:.2e} b {eb:.2e} u {eu:.2e}, eps_flux {a.eps_flux:.2e} / {c.eps_flux:.2e}")
        assert ea < 1e-12 and eb < 1e-12 and eu < 1e-12


@pytest.mark.parametrize("qrcp", ["default", "sketched"])
def test_cod_operator_fields(mfs, ctx, monkeypatch, qrcp):
    """The one-body factorisation with the truncated complete orthogonal
    decomposition (MFS_OPINV=cod: pivoted QR of the triangle, cut at the
    trailing Frobenius norm, inverse of the LQ factor) in place of the Jacobi
    SVD, on rank-deficient bodies (the k = 10 body and two of the batch's):
    the free-space field against the oracle's truncated-SVD solution, 1e-10;
    the coefficients differ (the kept ranks are not the SVD's) but the field
    the method computes does not.  Also with the sketch-pivoted QR, whose
    pivots are not the deterministic ones."""
    monkeypatch.setenv("MFS_OPINV", "cod")
    if qrcp != "default":
        monkeypatch.setenv("MFS_QRCP", qrcp)
    bodies = [W.periodic_k10(1).body] + W.batch_obstacles(2)
    tg = W.fibonacci_sphere(24, 2.0)
    for i, b in enumerate(bodies):
        op = make_op(mfs, ctx, b)
        ranks = op.factor_modes(1e-10)
        w = W.sample_waves(b.k, None, 1, seed=40 + i)[0]
        kv = W.wave_vector(b.k, w)[None, :]
        c = mfs.apply_solution_op(op, mfs.rhs_modes(op, kv))
        u = mfs.field_free(op, c, 2 * b.P, tg).cpu().numpy()[0]
        g = geometry.build_geometry(b)
        A = onebody.modal_blocks(b, g)
        co = onebody.solve_modes(A, onebody.rhs_modes(b, g, w))
        uo = onebody.field(b, g, co, tg, 2 * b.P)
        err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
        svr = [int(np.sum(s > 1e-10 * s[0])) for s in (np.linalg.svd(A[n], compute_uv=False) for n in range(3))]
        log(f"[cod] body {i}: N={b.N} M={b.M} P={b.P} ranks {list(ranks[:3])} (SVD {svr}) field err {err:.2e}")
        assert err < 1e-10


def test_sixteen_wave_batch_matches_small_batches(mfs, ctx):
    """Twelve incidences in one batched solve (the stored-field sums then run
    with 16 right-hand sides: the matrix-core mirror form with two column
    blocks) against the same incidences in batches of four (8 right-hand
    sides, the form the oracle parity tests cover): Bragg amplitudes and
    fields to 1e-12."""
    pr = W.small_periodic(nwaves=12)
    b = pr.body
    op = make_op(mfs, ctx, b)
    op.factor_modes(1e-10)
    L = _lat(mfs, pr.lattice)
    waves = [(w.theta, w.phi) for w in pr.waves]
    kw = dict(tol=1e-12, maxit=100, targets=pr.targets, q_field=pr.q_field)
    big = mfs.solve_incident(ctx, op, L, waves, **kw)
    small = []
    for i in range(0, 12, 4):
        small += mfs.solve_incident(ctx, op, L, waves[i:i + 4], **kw)
    worst = 0.0
    for r1, r2 in zip(big, small):
        assert np.array_equal(r1.m, r2.m) and np.array_equal(r1.n, r2.n)
        ea = np.max(np.abs(r1.a - r2.a)) / np.max(np.abs(r2.a))
        eb = np.max(np.abs(r1.b - r2.b)) / np.max(np.abs(r2.b))
        eu = np.linalg.norm(r1.field - r2.field) / np.linalg.norm(r2.field)
        worst = max(worst, ea, eb, eu)
    log(f"[16 waves] one batch of 12 vs three of 4: worst relative difference {worst:.2e}")
    assert worst < 1e-12


@pytest.mark.parametrize("tol", [1e-12, 1e-10])
def test_periodic_k10_full_size_vs_golden(mfs, ctx, tol):
    """Full size of the benchmark workload, in the benchmark's launch
    configuration (all 8 incidences in one batched solve), against the
    oracle's stored solution of incidence 0 (tests/golden/make_golden.py,
    GMRES to 1e-12): Bragg amplitudes and cell fields to 1e-10, at the parity
    tolerance 1e-12 and at the benchmark's GMRES tolerance 1e-10 (the
    '@1e-10 rel err' of the throughput figure).  Every incidence's flux
    balance: 1e-11 at GMRES 1e-12; at GMRES 1e-10 the iteration's own
    residual bounds it (1.3e-10 measured), so 3e-10."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "periodic_k10_wave0.json")))
    pr = W.periodic_k10(8)
    b, lat = pr.body, pr.lattice
    assert abs(pr.waves[0].theta - gold["theta"]) < 1e-15 and abs(pr.waves[0].phi - gold["phi"]) < 1e-15
    op = make_op(mfs, ctx, b)
    op.factor_modes(1e-10)
    tg = np.array(gold["targets"])
    res = mfs.solve_incident(ctx, op, _lat(mfs, lat), [(w.theta, w.phi) for w in pr.waves], tol=tol,
                             maxit=100, targets=tg, q_field=gold["q_field"])
    r = res[0]
    assert r.m.tolist() == gold["m"] and r.n.tolist() == gold["n"]
    ga = np.array(gold["a_re"]) + 1j * np.array(gold["a_im"])
    gb = np.array(gold["b_re"]) + 1j * np.array(gold["b_im"])
    gu = np.array(gold["u_re"]) + 1j * np.array(gold["u_im"])
    ea = np.max(np.abs(r.a - ga)) / np.max(np.abs(ga))
    eb = np.max(np.abs(r.b - gb)) / np.max(np.abs(gb))
    eu = np.linalg.norm(r.field - gu) / np.linalg.norm(gu)
    log(f"[k10 tol {tol:g}] iters gpu {r.iters} oracle {gold['iters']} a {ea:.2e} b {eb:.2e} u {eu:.2e} "
        f"flux {max(x.eps_flux for x in res):.2e} (oracle {gold['eps_flux']:.2e})")
    assert ea < 1e-10 and eb < 1e-10 and eu < 1e-10
    assert all(x.eps_flux < (1e-11 if tol < 1e-11 else 3e-10) for x in res)


def test_periodic_k10_low_rank_vs_golden(mfs, ctx, monkeypatch):
    """The benchmark workload with its surface sums from the low-rank image
    blocks (randomised range finder, QR, projection; ranks well below the
    15360 x 12800 blocks, so the truncation is exercised) instead of the
    stored values: all 8 incidences in one batch, incidence 0 against the
    oracle's stored solution, Bragg amplitudes and cell fields to 1e-10."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "periodic_k10_wave0.json")))
    pr = W.periodic_k10(8)
    b, lat = pr.body, pr.lattice
    monkeypatch.setenv("MFS_NEAR_LOWRANK", "2")
    op = make_op(mfs, ctx, b)
    op.set_near_field_budget(0)
    op.factor_modes(1e-10)
    tg = np.array(gold["targets"])
    res, tm = mfs.solve_incident(ctx, op, _lat(mfs, lat), [(w.theta, w.phi) for w in pr.waves], tol=1e-12,
                                 maxit=100, targets=tg, q_field=gold["q_field"], timing=True)
    assert int(tm["near_mode"]) == 3
    r = res[0]
    assert r.m.tolist() == gold["m"] and r.n.tolist() == gold["n"]
    ga = np.array(gold["a_re"]) + 1j * np.array(gold["a_im"])
    gb = np.array(gold["b_re"]) + 1j * np.array(gold["b_im"])
    gu = np.array(gold["u_re"]) + 1j * np.array(gold["u_im"])
    ea = np.max(np.abs(r.a - ga)) / np.max(np.abs(ga))
    eb = np.max(np.abs(r.b - gb)) / np.max(np.abs(gb))
    eu = np.linalg.norm(r.field - gu) / np.linalg.norm(gu)
    log(f"[k10 low rank] build {tm['near_fill_ms']:.1f} ms, sums {tm['nsum_avg']:.3f} ms avg; iters gpu {r.iters} "
        f"oracle {gold['iters']} a {ea:.2e} b {eb:.2e} u {eu:.2e} flux {max(x.eps_flux for x in res):.2e}")
    assert ea < 1e-10 and eb < 1e-10 and eu < 1e-10
    assert all(x.eps_flux < 1e-11 for x in res)


@pytest.mark.parametrize("name", ["sphere", "cup"])
def test_apply_angle_samples_to_point_strengths(mfs, ctx, name):
    """The apply call with its angle-sample input and point-strength output
    (angle DFT, per-mode pseudoinverse, inverse DFT: eq. (fhatquad), Sec. 4.2,
    the point-source form of Sec. 4.1) against the oracle's chain rhs_modes ->
    solve_modes -> point_strengths, compared through the field the strengths
    radiate at the test points (the strengths themselves are not unique);
    and the angle input against the mode input on the GPU's own operator."""
    import torch
    pr = CASES[name]()
    b = pr.body
    op = make_op(mfs, ctx, b)
    op.factor_modes(1e-10)
    g = geometry.build_geometry(b)
    w = pr.waves[0]
    kv = W.wave_vector(b.k, w)
    X, Nn = geometry.surface_points(g, b.P)                        # [P, M, 3]
    f = -1j * (Nn @ kv) * np.exp(1j * (X @ kv))                     # [P, M]
    f_angle = torch.from_numpy(np.ascontiguousarray(f.T)[None]).cuda()   # [1, M, P]
    sig = mfs.apply_solution_op(op, f_angle, in_layout=mfs.LAYOUT_ANGLE,
                                out_layout=mfs.LAYOUT_POINTS).cpu().numpy()[0]   # [P, N]
    A = onebody.modal_blocks(b, g)
    co = onebody.solve_modes(A, onebody.rhs_modes(b, g, w))
    sig_o = onebody.point_strengths(co, b.P)
    Y = geometry.source_ring_points(g, b.P)
    u = onebody.field_from_points(b.k, Y, sig, pr.targets)
    uo = onebody.field_from_points(b.k, Y, sig_o, pr.targets)
    err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    # the mode-layout path on the same operator: the same field up to the
    # rounding of the angle transform
    c_modes = mfs.apply_solution_op(op, mfs.rhs_modes(op, kv[None]))
    c_angle = mfs.apply_solution_op(op, f_angle, in_layout=mfs.LAYOUT_ANGLE)
    u_m = mfs.field_free(op, c_modes, pr.q_field, pr.targets).cpu().numpy()[0]
    u_a = mfs.field_free(op, c_angle, pr.q_field, pr.targets).cpu().numpy()[0]
    ec = float(np.linalg.norm(u_a - u_m) / np.linalg.norm(u_m))
    log(f"[apply layouts] {name}: field of the point strengths vs oracle {err:.2e}; "
        f"angle vs mode input {ec:.2e}")
    assert err < 1e-10
    assert ec < 1e-11
    with pytest.raises(mfs.MfsError):
        mfs.apply_solution_op(op, f_angle, in_layout=7)
