"""Addressing of the masked loads of the blocked QR (host-side check, no GPU).

The QR kernels read through `ld_or0(base, i, ok)`, which always issues the
load and reads base[0] when `ok` is false, so every base they form must
lie inside its matrix, also for panels with no trailing columns left.  A
column base one past the end of the matrix once made every factorisation
read one element past its buffer (the first batched-build run faulted the
GPU on the buffers ending on a page boundary).

These tests restate, in Python, how the trailing-update kernels of
`csrc/qr.hip` form their column bases (`y_source`, `yel`) for the panel
loop of the two-level blocked QR (outer panels of nb = 16, 32 or 64
columns, inner panels of 16, inner updates ending at the outer panel), and
check every base against the matrix's columns over the shapes the library
factors: the 256-obstacle batch, the k = 10 periodizer Q, the large cups'
blocks and periodizer Q.
"""
import pytest

import workloads as W

NI = 16


def y_source(n, k0, nbp, which, rank=0):
    """(first column of B as a column index of its matrix, columns of B) as
    the kernels form them; which 0: the matrix's trailing columns, 1: the
    first `rank` columns of U, 2: U's columns from k0 on."""
    if which == 0:
        nb_cols = n - k0 - nbp
        return (k0 + nbp if nb_cols > 0 else 0), nb_cols
    if which == 1:
        return 0, rank
    some = k0 < rank
    return (k0 if some else 0), (rank - k0 if some else 0)


def bases(n, nb, which, rank=0, cend=None, k0=0):
    """Every column index a masked load of the panel at k0 may form: V columns
    (yel: clamped to column 0 past the end) and B columns (base + offset,
    the offset clamped to 0 for columns past the end)."""
    nbp = min(nb, n - k0)
    b0, nb_cols = y_source(n, k0, nbp, which, rank)
    if which == 0 and cend is not None:
        nb_cols = min(nb_cols, cend - (k0 + nbp))
    cols = []
    for c in range(nb):                      # V columns of the panel
        vc = k0 + c
        cols.append(vc if vc < n else 0)
    for c in range(max(nb_cols, 0) + 1):     # B columns, and one past (masked)
        cols.append(b0 + (c if c < nb_cols else 0))
    return cols


def check_matrix(n, nb, rank=None):
    """Walk the factorisation's panels (outer, and inner with their column
    end) and U's formation; return the largest column index formed."""
    worst = -1
    for K0 in range(0, n, nb):
        if nb > NI:
            for k0 in range(K0, min(K0 + nb, n), NI):
                for c in bases(n, NI, 0, cend=K0 + nb, k0=k0):
                    worst = max(worst, c)
                    assert 0 <= c < n, (n, nb, K0, k0, c)
        for c in bases(n, nb, 0, k0=K0):
            worst = max(worst, c)
            assert 0 <= c < n, (n, nb, K0, c)
    r = n if rank is None else rank
    for K0 in range(((n - 1) // nb) * nb, -1, -nb):
        for which in (1, 2):
            b0, nb_cols = y_source(n, K0, min(nb, n - K0), which, r)
            for c in (b0, b0 + max(nb_cols - 1, 0)):
                assert 0 <= c < max(r, 1), (n, nb, K0, which, c)
    return worst


SHAPES = {
    "batch_256": sorted({(b.M, b.N) for b in W.batch_obstacles(256)}),
    "periodizer_k10": [(4608, 1275), (4608, 1269)],
    "large_cup_blocks": [(540, 450), (1080, 900)],
    "large_periodizer": [(25088, 10805)],
    "edge": [(16, 1), (17, 16), (64, 17), (100, 64), (65, 65), (33, 32), (48, 47)],
}


@pytest.mark.parametrize("nb", [16, 32, 64])
@pytest.mark.parametrize("name", list(SHAPES))
def test_masked_load_bases_stay_inside(name, nb):
    for m, n in SHAPES[name]:
        worst = check_matrix(n, nb)
        assert worst <= n - 1
        check_matrix(n, nb, rank=max(1, n // 2))


def test_the_old_base_would_fail():
    """The rule this guards against: the trailing columns' base taken as
    k0 + nbp also after the last panel is one column past the end."""
    n, nb = 1275, 16
    k0 = ((n - 1) // nb) * nb
    nbp = min(nb, n - k0)
    assert k0 + nbp == n                       # the unclamped base: past the end
    assert y_source(n, k0, nbp, 0)[0] == 0     # the kernels' base: column 0
