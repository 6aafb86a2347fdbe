"""GPU tests of the C ABI's error statuses: every failure is reported as an
mfs_status (never a crash), bad input writes nothing, and a solve that hits
its iteration or sweep cap still returns its last iterate.  All conditions
are forced from the host (argument values, a lowered sweep cap): every
kernel runs to its normal end."""
from __future__ import annotations

import math
import os
import sys

import numpy as np
import pytest

import workloads as W

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
def small(mfs):
    pr = W.small_periodic(nwaves=2)
    b = pr.body
    ctx = mfs.create(0)
    g = mfs.body_geometry(b.shape, b.M, b.N, b.tau, b.colloc)
    return pr, ctx, g


def spec(mfs, b, g, **kw):
    d = dict(M=b.M, N=b.N, P=b.P, q=b.q, k=b.k)
    d.update(kw)
    return mfs.BodySpec(d["M"], d["N"], d["P"], d["q"], d["k"], g)


def test_gmres_maxit_returns_last_iterate(mfs, small):
    """maxit = 2: ENOTCONV, and the results hold the second iterate (two
    iterations, residual above the tolerance, finite amplitudes)."""
    pr, ctx, g = small
    b, lat = pr.body, pr.lattice
    op = mfs.build_operator(ctx, [spec(mfs, b, g)])
    op.factor_modes(1e-10)
    L = mfs.lattice(lat.ex, lat.ey, lat.z0, lat.p, lat.N0, lat.M1)
    waves = [(w.theta, w.phi) for w in pr.waves]
    with pytest.raises(mfs.MfsError) as ei:
        mfs.solve_incident(ctx, op, L, waves, tol=1e-12, maxit=2)
    assert ei.value.status == mfs.MFS_ENOTCONV
    res = mfs.solve_incident(ctx, op, L, waves, tol=1e-12, maxit=2, allow_notconv=True)
    for r in res:
        log(f"[maxit] iters {r.iters} resid {r.resid:.2e}")
        assert r.iters == 2 and r.resid > 1e-12
        assert np.all(np.isfinite(r.a)) and np.all(np.isfinite(r.b)) and len(r.m) > 0


def test_apply_before_factor_is_estate(mfs, small):
    import torch
    pr, ctx, g = small
    b = pr.body
    op = mfs.build_operator(ctx, [spec(mfs, b, g)])
    x = torch.zeros((1, b.P, b.M), dtype=torch.complex128, device="cuda")
    with pytest.raises(mfs.MfsError) as ei:
        mfs.apply_solution_op(op, x)
    assert ei.value.status == mfs.MFS_ESTATE
    L = mfs.lattice(1.0, 1.0, 0.6, 8, 4, 8)
    ctx2 = mfs.create(0)
    with pytest.raises(mfs.MfsError) as ei:
        mfs.solve_incident(ctx2, op, L, [(0.1, 0.2)])
    assert ei.value.status == mfs.MFS_ESTATE
    op.factor_modes(1e-10)
    with pytest.raises(mfs.MfsError) as ei:
        op.factor_modes(1e-10)
    assert ei.value.status == mfs.MFS_ESTATE


@pytest.mark.parametrize("bad", ["odd_P", "q_below_P", "M_below_N", "nan_rho", "nonpositive_source"])
def test_bad_operator_input_is_einval(mfs, small, bad):
    pr, ctx, g = small
    b = pr.body
    g2 = {k: v.copy() for k, v in g.items()}
    kw = {}
    if bad == "odd_P":
        kw["P"] = b.P + 1
    elif bad == "q_below_P":
        kw["q"] = b.P - 2
    elif bad == "M_below_N":
        kw["M"] = b.N - 1
        for k in ("rho", "z", "nrho", "nz"):
            g2[k] = g2[k][: b.N - 1].copy()
    elif bad == "nan_rho":
        g2["rho"][3] = math.nan
    elif bad == "nonpositive_source":
        g2["srho"][0] = -0.1
    with pytest.raises(mfs.MfsError) as ei:
        mfs.build_operator(ctx, [spec(mfs, b, g2, **kw)])
    assert ei.value.status == mfs.MFS_EINVAL
    log(f"[einval] {bad}: {ei.value}")


def test_bad_apply_and_sum_arguments_write_nothing(mfs, small):
    """An unknown layout, nrhs out of range or a NaN incidence: EINVAL and the
    output buffer keeps its contents."""
    import torch
    pr, ctx, g = small
    b, lat = pr.body, pr.lattice
    op = mfs.build_operator(ctx, [spec(mfs, b, g)])
    op.factor_modes(1e-10)
    x = torch.ones((1, b.P, b.M), dtype=torch.complex128, device="cuda")
    out = torch.full((1, b.P, b.N), 7.0 + 3.0j, dtype=torch.complex128, device="cuda")
    st = mfs.lib().mfs_apply_solution_op(op.h, 0, 1, mfs._dev(x), 5, mfs._dev(out), 0, mfs._stream())
    assert st == mfs.MFS_EINVAL
    st = mfs.lib().mfs_apply_solution_op(op.h, 0, 1, mfs._dev(x), 0, mfs._dev(out), 1, mfs._stream())
    assert st == mfs.MFS_EINVAL
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0 + 3.0j))
    L = mfs.lattice(lat.ex, lat.ey, lat.z0, lat.p, lat.N0, lat.M1)
    sig = torch.ones((17, b.P, b.N), dtype=torch.complex128, device="cuda")
    with pytest.raises(mfs.MfsError) as ei:
        mfs.neighbour_sum(op, L, sig, np.ones((17, 2), dtype=np.complex128), mfs.TARGETS_SURFACE)
    assert ei.value.status == mfs.MFS_EINVAL
    with pytest.raises(mfs.MfsError) as ei:
        mfs.solve_incident(ctx, op, L, [(math.nan, 0.3)])
    assert ei.value.status == mfs.MFS_EINVAL


def test_jacobi_sweep_cap_is_enotconv(mfs, small):
    """With the sweep cap lowered to one sweep the per-mode Jacobi cannot
    finish: factor_modes reports ENOTCONV (and keeps the last factors);
    with the default cap the same operator factors cleanly."""
    pr, ctx, g = small
    b = pr.body
    op = mfs.build_operator(ctx, [spec(mfs, b, g)])
    os.environ["MFS_JACOBI_MAX_SWEEPS"] = "1"
    try:
        with pytest.raises(mfs.MfsError) as ei:
            op.factor_modes(1e-10)
    finally:
        del os.environ["MFS_JACOBI_MAX_SWEEPS"]
    assert ei.value.status == mfs.MFS_ENOTCONV
    log(f"[jacobi cap] {ei.value}")
    op2 = mfs.build_operator(ctx, [spec(mfs, b, g)])
    op2.factor_modes(1e-10)
