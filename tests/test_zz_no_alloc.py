"""GPU test of mfs_apply_solution_op_noalloc, the solution-operator apply
that allocates nothing (its work memory is a static device array): through
the C ABI, against mfs_apply_solution_op on the same inputs, on two calls in
a row (the second with a smaller input, on another operator), in every
layout pair; the library's own allocation count does not move; a size
beyond the static array is refused and writes nothing."""
from __future__ import annotations

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


def make_op(mfs, ctx, b):
    g = mfs.body_geometry(b.shape, b.M, b.N, b.tau, b.colloc)
    op = mfs.build_operator(ctx, [mfs.BodySpec(b.M, b.N, b.P, b.q, b.k, g)])
    op.factor_modes(1e-10)
    return op


def rand_in(b, nrhs, layout, seed):
    import torch
    rng = np.random.default_rng(seed)
    shape = (nrhs, b.P, b.M) if layout == 0 else (nrhs, b.M, b.P)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return torch.from_numpy(x).cuda()


def run_both(mfs, op, b, x, lin, lout):
    """(noalloc result, allocating result, library bytes in use before/after
    the noalloc call and its peak over it)."""
    import torch
    ncol = b.N
    out_na = torch.full((x.shape[0], b.P, ncol), 5.0 - 2.0j, dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    mfs.reset_memory_peak(0)
    before = mfs.memory_stats(0)
    st = mfs.lib().mfs_apply_solution_op_noalloc(op.h, 0, x.shape[0], mfs._dev(x), lin, mfs._dev(out_na), lout,
                                                 mfs._stream())
    torch.cuda.synchronize()
    after = mfs.memory_stats(0)
    assert st == mfs.MFS_OK, mfs.lib().mfs_last_error().decode()
    ref = mfs.apply_solution_op(op, x, in_layout=lin, out_layout=lout)
    torch.cuda.synchronize()
    return out_na.cpu().numpy(), ref.cpu().numpy(), before, after


@pytest.mark.parametrize("lin,lout", [(0, 0), (1, 0), (0, 2), (1, 2)])
def test_noalloc_matches_allocating_apply(mfs, lin, lout):
    ctx = mfs.create(0)
    big = W.periodic_k10(1).body
    small = W.small_periodic(1).body
    op_big = make_op(mfs, ctx, big)
    op_small = make_op(mfs, ctx, small)
    # first call: the k = 10 body, 12 right-hand sides
    x1 = rand_in(big, 12, lin, 1)
    a1, r1, b1, e1 = run_both(mfs, op_big, big, x1, lin, lout)
    # second call: a smaller input, the small body, 3 right-hand sides
    x2 = rand_in(small, 3, lin, 2)
    a2, r2, b2, e2 = run_both(mfs, op_small, small, x2, lin, lout)
    d1 = float(np.max(np.abs(a1 - r1)) / np.max(np.abs(r1)))
    d2 = float(np.max(np.abs(a2 - r2)) / np.max(np.abs(r2)))
    log(f"[noalloc] layouts in {lin} out {lout}: first call {d1:.1e}, second call {d2:.1e}; library bytes in use "
        f"{b1['in_use']} -> {e1['in_use']} (peak {e1['peak']}), {b2['in_use']} -> {e2['in_use']} (peak {e2['peak']})")
    # the same kernels on the same inputs: identical results
    assert d1 == 0.0 and d2 == 0.0
    for b_, e_ in ((b1, e1), (b2, e2)):
        assert e_["in_use"] == b_["in_use"] and e_["peak"] == b_["in_use"]


def test_noalloc_rejects_more_than_its_scratch(mfs):
    import torch
    ctx = mfs.create(0)
    b = W.small_periodic(1).body
    op = make_op(mfs, ctx, b)
    nrhs = 4000            # 4000 x P x M x 16 B of angle-input modes: more than 64 MiB
    x = torch.ones((nrhs, b.M, b.P), dtype=torch.complex128, device="cuda")
    out = torch.full((nrhs, b.P, b.N), 1.0 + 1.0j, dtype=torch.complex128, device="cuda")
    st = mfs.lib().mfs_apply_solution_op_noalloc(op.h, 0, nrhs, mfs._dev(x), 1, mfs._dev(out), 0, mfs._stream())
    torch.cuda.synchronize()
    assert st == mfs.MFS_EINVAL
    log(f"[noalloc] refused: {mfs.lib().mfs_last_error().decode()}")
    assert bool(torch.all(out == 1.0 + 1.0j))
