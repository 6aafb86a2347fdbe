"""Pins of the oracle's periodizing scheme (Sec. 4 of the paper): closed
forms of the auxiliary bases, the wall-cancellation identity, energy-flux
balance, quasi-periodicity, lattice symmetry at normal incidence and an
independent dense solve of the full bordered system eq. (full).  CPU only."""
import math

import numpy as np
import pytest
from scipy.special import spherical_jn

import workloads as W
from oracle import geometry, gmres, onebody, periodic


def test_rb_orders_branch_and_enumeration():
    """kappa_z is +real for propagating and +imaginary for evanescent orders,
    and the kept set is exactly the lattice points inside the pi N0 disc."""
    k = 10.0
    lat = W.Lattice(1.0, 1.3, 0.6, p=4, N0=5, M1=4)
    kv = W.wave_vector(k, W.Wave(0.4, 2.0))
    o = periodic.rb_orders(k, kv, lat)
    prop = k * k - o.kx ** 2 - o.ky ** 2 > 0
    assert np.all(o.kz[prop].real > 0) and np.all(np.abs(o.kz[prop].imag) == 0)
    assert np.all(o.kz[~prop].imag > 0) and np.all(o.kz[~prop].real == 0)
    want = {(m, n) for m in range(-40, 41) for n in range(-40, 41)
            if (kv[0] + 2 * math.pi * m) ** 2 + (kv[1] + 2 * math.pi * n / 1.3) ** 2 <= (5 * math.pi) ** 2}
    assert set(zip(o.m.tolist(), o.n.tolist())) == want
    assert np.allclose(o.kz ** 2 + o.kx ** 2 + o.ky ** 2, k * k)


def test_harmonic_closed_forms():
    """H_00 = j_0(kr) / sqrt(4 pi) = sin(kr)/(kr sqrt(4 pi)); H_10 =
    sqrt(3/(4 pi)) j_1(kr) cos(theta)."""
    k = 3.0
    X = np.array([[0.3, 0.2, -0.4], [0.1, -0.5, 0.2]])
    H, _ = periodic.harmonics(k, 2, X)
    r = np.linalg.norm(X, axis=1)
    assert np.allclose(H[:, 0], np.sin(k * r) / (k * r) / math.sqrt(4 * math.pi), atol=1e-15)
    j1 = np.sin(k * r) / (k * r) ** 2 - np.cos(k * r) / (k * r)
    assert np.allclose(H[:, 2], math.sqrt(3 / (4 * math.pi)) * j1 * X[:, 2] / r, atol=1e-15)


def test_harmonics_gradient_and_helmholtz():
    """Chain-rule gradient = central differences; each H_lm solves the
    Helmholtz equation (second differences)."""
    k, p = 6.0, 7
    X = np.array([[0.31, -0.22, 0.47], [-0.5, 0.4, -0.1], [0.05, 0.6, 0.3]])
    H, g = periodic.harmonics(k, p, X)
    h = 1e-5
    for c in range(3):
        e = np.zeros(3); e[c] = h
        Hp, _ = periodic.harmonics(k, p, X + e)
        Hm, _ = periodic.harmonics(k, p, X - e)
        assert np.max(np.abs((Hp - Hm) / (2 * h) - g[..., c])) < 1e-8
    h = 1e-3
    lap = -6 * H
    for c in range(3):
        e = np.zeros(3); e[c] = h
        lap += periodic.harmonics(k, p, X + e)[0] + periodic.harmonics(k, p, X - e)[0]
    assert np.max(np.abs(lap / h ** 2 + k * k * H)) < 1e-4


def test_gmres_matches_direct_solve():
    rng = np.random.default_rng(3)
    n = 60
    A = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, its, hist = gmres.gmres(lambda v: A @ v, b, 1e-13, n)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-11 * np.linalg.norm(x)
    assert hist[-1] <= 1e-13 and its <= n


# ---------------------------------------------------- small periodic solve

@pytest.fixture(scope="module")
def small():
    pr = W.small_periodic(nwaves=1)
    b, lat = pr.body, pr.lattice
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    ps = periodic.PeriodicSolver(b, lat, g, A)
    ps.set_wave(pr.waves[0])
    fh = onebody.rhs_modes(b, g, pr.waves[0])
    res = ps.solve(fh, tol=1e-12)
    return pr, ps, fh, res


def test_wall_cancellation_identity(small):
    """C with the 3x3 cancellation (6 distant terms per wall pair) equals C
    built from all 18 terms (Sec. 4.1)."""
    pr, ps, fh, res = small
    full = ps.c_point_matrix(cancel=False)
    assert np.max(np.abs(full - ps.Cpt)) < 1e-13 * np.max(np.abs(full))


def test_energy_flux_and_quasiperiodicity(small):
    """Real k, sound-hard: incoming flux equals outgoing flux over the
    propagating Bragg orders (eps_flux), and the representation matches
    Cauchy data across L/R and B/F (eps_per); the Neumann condition holds
    (eps_bc).  Thresholds are the converged levels of this small
    discretisation."""
    pr, ps, fh, res = small
    assert res["hist"][-1] <= 1e-12
    assert ps.eps_flux(res["a"], res["b"]) < 1e-6
    assert ps.eps_per(res["c"], res["d"], 2 * pr.body.P) < 1e-6
    assert ps.eps_bc(res["c"], res["d"], pr.body.q, 10, 10) < 1e-4


def test_beta_typo_reading_is_pinned(small):
    """Using e_x's phase for beta (the typo in eq. (bloch)) breaks the
    quasi-periodicity of the solution at an oblique incidence."""
    pr, ps, fh, res = small
    b = pr.body
    g = ps.geom
    ps2 = periodic.PeriodicSolver(b, pr.lattice, g, ps.A, pinv=ps.pinv)
    ps2.set_wave(pr.waves[0])
    ps2.beta = ps2.alpha
    ps2.Cpt = ps2.c_point_matrix(cancel=True)
    ps2.Q = ps2.q_matrix()
    ps2.Qf = periodic.equilibrated_pinv_factors(ps2.Q, 1e-10)
    ps2.Kelse = ps2.aelse_point_matrix()
    r2 = ps2.solve(fh, tol=1e-10)
    ps2.beta = ps.beta        # judge against the true phases
    assert ps2.eps_per(r2["c"], r2["d"], 2 * b.P) > 1e-3


def test_dense_full_system_agrees_with_schur_gmres(small):
    """Dense least squares on eq. (full) (mode space, no Schur complement,
    no preconditioner, no GMRES) gives the same field and Bragg amplitudes
    as the right-preconditioned iteration eq. (iter)."""
    pr, ps, fh, res = small
    c2, xi2 = ps.dense_full_solve(fh)
    NH = (pr.lattice.p + 1) ** 2
    nrb = ps.orders.m.size
    u1, _ = ps.field_and_grad(res["c"], res["d"], pr.targets, pr.q_field, want_grad=False)
    u2, _ = ps.field_and_grad(c2, xi2[:NH], pr.targets, pr.q_field, want_grad=False)
    assert np.linalg.norm(u1 - u2) / np.linalg.norm(u1) < 1e-6
    prop = (np.abs(ps.orders.kz.imag) < 1e-14)
    a2, b2 = xi2[NH:NH + nrb], xi2[NH + nrb:]
    assert np.max(np.abs(res["a"][prop] - a2[prop])) < 1e-6 * np.max(np.abs(res["a"][prop]))
    assert np.max(np.abs(res["b"][prop] - b2[prop])) < 1e-6 * np.max(np.abs(res["b"][prop]))


def test_normal_incidence_lattice_symmetry():
    """At normal incidence on a square lattice of axisymmetric bodies the
    propagating Bragg amplitudes are invariant under (m,n) -> (-m,n) and
    (m,n) -> (n,m) (the D4 symmetry of the problem)."""
    pr = W.small_periodic(nwaves=1)
    b, lat = pr.body, pr.lattice
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    ps = periodic.PeriodicSolver(b, lat, g, A)
    w = W.Wave(0.0, 0.0)
    ps.set_wave(w)
    res = ps.solve(onebody.rhs_modes(b, g, w), tol=1e-12)
    o = ps.orders
    idx = {(m, n): i for i, (m, n) in enumerate(zip(o.m.tolist(), o.n.tolist()))}
    prop = [i for i in range(o.m.size) if abs(o.kz[i].imag) < 1e-14]
    scale = np.max(np.abs(res["a"]))
    for i in prop:
        m, n = int(o.m[i]), int(o.n[i])
        for j in (idx[(-m, n)], idx[(n, m)]):
            assert abs(res["a"][i] - res["a"][j]) < 1e-8 * scale
            assert abs(res["b"][i] - res["b"][j]) < 1e-8 * scale


# ------------------------------------------ the k = 10 workload's accuracy

def _golden_k10():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "periodic_k10_wave0.json")
    with open(path) as f:
        return json.load(f)


def test_k10_golden_meets_paper_accuracy():
    """The oracle's solve of the k = 10 workload (incidence 0, written by
    tests/golden/make_golden.py from oracle/ only) meets the accuracy the
    paper's periodic tables report (Sec. 5, Tables t:reslo and t:reshi:
    eps_flux, eps_per, eps_bc of 1e-11 to 7e-10): energy flux balanced and
    quasi-periodicity and the boundary condition met to 1e-10, with the
    periodizer parameters the workload uses now (a stale golden fails)."""
    gold = _golden_k10()
    lat = W.periodic_k10(1).lattice
    assert gold["lattice"] == {"ex": lat.ex, "ey": lat.ey, "z0": lat.z0, "p": lat.p, "N0": lat.N0, "M1": lat.M1}
    assert gold["gmres_resid"] <= 1e-12
    assert gold["eps_flux"] <= 1e-10
    assert gold["eps_per"] <= 1e-10
    assert gold["eps_bc"] <= 1e-10


@pytest.mark.skipif(not __import__("os").environ.get("MFS_SLOW_ORACLE"),
                    reason="about 10 minutes of CPU; set MFS_SLOW_ORACLE=1 to run")
def test_k10_accuracy_recomputed():
    """The same accuracy recomputed by the oracle (first incidence of the
    k = 10 workload), and the golden's amplitudes reproduced."""
    pr = W.periodic_k10(1)
    b, lat = pr.body, pr.lattice
    g = geometry.build_geometry(b)
    A = onebody.modal_blocks(b, g)
    ps = periodic.PeriodicSolver(b, lat, g, A)
    w = pr.waves[0]
    ps.set_wave(w)
    res = ps.solve(onebody.rhs_modes(b, g, w), tol=1e-12)
    assert ps.eps_flux(res["a"], res["b"]) <= 1e-10
    assert ps.eps_per(res["c"], res["d"], pr.q_field) <= 1e-10
    assert ps.eps_bc(res["c"], res["d"], b.q) <= 1e-10
    gold = _golden_k10()
    ga = np.array(gold["a_re"]) + 1j * np.array(gold["a_im"])
    assert np.max(np.abs(res["a"] - ga)) <= 1e-12 * np.max(np.abs(ga))
