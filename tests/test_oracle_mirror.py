"""Pin of the half-turn symmetry the stored near field relies on (CPU only).

A half-turn R about the z axis maps a body of revolution onto itself: the
surface node at azimuth 2 pi l / P onto the one at l + P/2, the point source
at azimuth 2 pi l / P onto the one at l + P/2, the normal with the node, and
the lattice shift s = a e_x + b e_y onto -s.  The Helmholtz kernel and its
target-normal derivative are invariant under R, so the image (-a, -b) of a
(target, source) pair equals the image (a, b) of the rotated pair.  Checked
here with the oracle's own kernels and geometry (Sec. 3 and 4.1), for every
neighbour image, values and normal derivatives, on the small periodic body
of the k = 10 family; a shift by anything but half a turn breaks it.
"""
import numpy as np

import workloads as W
from oracle import geometry, kernel


def _images():
    return [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]


def _blocks(pr, lt, ls):
    """Values and normal derivatives of every image for target azimuths lt and
    source azimuths ls: dicts keyed by (a, b), arrays [len(lt), M, len(ls), N]."""
    b, lat = pr.body, pr.lattice
    g = geometry.build_geometry(b)
    X, Nn = geometry.surface_points(g, b.P)       # [P, M, 3]
    Y = geometry.source_ring_points(g, b.P)       # [P, N, 3]
    x, n, y = X[lt][:, :, None, None, :], Nn[lt][:, :, None, None, :], Y[ls][None, None, :, :, :]
    val, der = {}, {}
    for (a, c) in _images():
        sh = np.array([a * lat.ex, c * lat.ey, 0.0])
        val[(a, c)] = kernel.G(b.k, x, y + sh)
        der[(a, c)] = kernel.dG_dnx(b.k, x, n, y + sh)
    return val, der


def test_half_turn_maps_image_to_mirror_image():
    pr = W.small_periodic()
    P = pr.body.P
    assert P % 2 == 0
    lt = np.array([0, 1, P // 4, P // 2 - 1])
    ls = np.array([0, 3, P // 2 + 1, P - 1])
    v0, d0 = _blocks(pr, lt, ls)
    v1, d1 = _blocks(pr, (lt + P // 2) % P, (ls + P // 2) % P)
    for (a, c) in _images():
        ref_v, ref_d = v0[(-a, -c)], d0[(-a, -c)]
        sv = np.max(np.abs(ref_v))
        sd = np.max(np.abs(ref_d))
        assert np.max(np.abs(v1[(a, c)] - ref_v)) < 1e-13 * sv, (a, c)
        assert np.max(np.abs(d1[(a, c)] - ref_d)) < 1e-13 * sd, (a, c)


def test_other_rotations_do_not_pair_the_images():
    """A quarter turn, or a half turn applied to the targets only, leaves
    O(1) differences: the identity is specific to the pairing used."""
    pr = W.small_periodic()
    P = pr.body.P
    lt = np.array([0, 5])
    ls = np.array([2, 9])
    v0, _ = _blocks(pr, lt, ls)
    vq, _ = _blocks(pr, (lt + P // 4) % P, (ls + P // 4) % P)
    vt, _ = _blocks(pr, (lt + P // 2) % P, ls)
    ref = v0[(-1, 0)]
    sv = np.max(np.abs(ref))
    assert np.max(np.abs(vq[(1, 0)] - ref)) > 1e-3 * sv
    assert np.max(np.abs(vt[(1, 0)] - ref)) > 1e-3 * sv


def test_half_turn_pairs_the_wall_nodes():
    """The walls of the unit cell (Sec. 4.1): the half-turn takes the right
    wall's Gauss node (a, b) to the left wall's node (M1-1-a, b), the front
    wall's to the back wall's likewise, and the top (bottom) wall's node i to
    its own node M1^2-1-i, the Gauss rule being symmetric.  Values at the
    paired node against the rotated sources and the negated shift agree; an
    x or y derivative changes sign (its direction turns over), a z derivative
    does not."""
    from oracle import periodic
    pr = W.small_periodic()
    b, lat = pr.body, pr.lattice
    P, M1 = b.P, lat.M1
    assert P % 2 == 0 and M1 % 2 == 0
    g = geometry.build_geometry(b)
    Y = geometry.source_ring_points(g, b.P)          # [P, N, 3]
    w = periodic.wall_nodes(lat)
    idx = np.arange(M1 * M1)
    a_, b_ = idx // M1, idx % M1
    cross = (M1 - 1 - a_) * M1 + b_
    own = M1 * M1 - 1 - idx
    ex, ey, ez = np.eye(3)
    cases = [(w.R, w.L, cross, ex), (w.F, w.B, cross, ey), (w.T, w.T, own, ez), (w.D, w.D, own, ez)]
    ls = np.array([0, 2, P // 2 + 3, P - 1])
    ys, ym = Y[ls], Y[(ls + P // 2) % P]
    sel = np.array([0, 7, M1 * M1 // 2 + 1, M1 * M1 - 1])
    for (X0, X1, pair, d) in cases:
        assert np.allclose(X1[pair[sel]], X0[sel] * np.array([-1.0, -1.0, 1.0]), atol=1e-15)
        x0 = X0[sel][:, None, None, :]
        x1 = X1[pair[sel]][:, None, None, :]
        nd = np.broadcast_to(d, x0.shape)
        sgn = -1.0 if d[2] == 0 else 1.0
        for (a, c) in _images():
            s0 = np.array([a * lat.ex, c * lat.ey, 0.0])
            v0 = kernel.G(b.k, x0, ys[None] + s0)
            v1 = kernel.G(b.k, x1, ym[None] - s0)
            d0 = kernel.dG_dnx(b.k, x0, nd, ys[None] + s0)
            d1 = kernel.dG_dnx(b.k, x1, nd, ym[None] - s0)
            assert np.max(np.abs(v1 - v0)) < 1e-13 * np.max(np.abs(v0)), (a, c)
            assert np.max(np.abs(d1 - sgn * d0)) < 1e-13 * np.max(np.abs(d0)), (a, c)
            # without the rotation of the sources the pairing fails
            bad = kernel.G(b.k, x1, ys[None] - s0)
            assert np.max(np.abs(bad - v0)) > 1e-3 * np.max(np.abs(v0)), (a, c)
