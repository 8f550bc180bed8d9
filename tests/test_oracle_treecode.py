"""Pins for the oracle's treecode (the potential of eq. bw03 by barycentric
Lagrange interpolation on Chebyshev proxies).

What fixes the answers: polynomial reproduction of the Lagrange basis (its
values at the nodes and for monomials up to the degree), the moments the
proxies must keep, the tree's partition of the sources, the direct sum when
no cluster is accepted (theta -> 0), and the interpolation error falling with
the degree against the direct sum (the oracle's eq. bw03 sum, pinned
elsewhere against exact solutions).
"""
import numpy as np
import pytest

import dtn_inputs as I
from oracle import patch as P
from oracle import potential as POT
from oracle import treecode as T
from oracle import wos


@pytest.mark.parametrize("n", [0, 1, 2, 5, 8])
def test_lagrange_basis_reproduces_polynomials(n):
    lo, hi = -0.3, 1.7
    nodes, w = T.cheb_nodes(lo, hi, n), T.bary_weights(n)
    rng = np.random.default_rng(n)
    y = np.concatenate([rng.uniform(lo, hi, 50), nodes, [lo, hi]])
    L = T.lagrange_1d(y, nodes, w)
    assert np.all(np.isfinite(L))
    for m in range(n + 1):
        np.testing.assert_allclose(L @ nodes ** m, y ** m, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(T.lagrange_1d(nodes, nodes, w), np.eye(n + 1))
    if n:
        # the extreme nodes are the interval's ends
        assert nodes[0] == hi and abs(nodes[-1] - lo) < 1e-15


def _cube_sources(n_tiles=None):
    gd = I.geometry_cube_sources()
    g = wos.Geometry(gd)
    pd = I.patches_cube_tiles()
    if n_tiles is not None:
        pd = I.subset_patches(pd, list(range(n_tiles)))
    ps = P.patches_from_desc(pd, gd)
    sig = [P.exact_neumann(gd, *P.collocation_points(p)[:2]) for p in ps]
    return ps, sig, g, gd


def test_tree_partitions_the_sources():
    ps, sig, g, _ = _cube_sources()
    y, a, b = T.tile_sources(ps, sig, g)
    tree = T.build_tree(y, T.tile_faces(ps), leaf_size=40, degree=6)
    seen = []

    def walk(C):
        assert np.all(y[C.idx] >= C.lo) and np.all(y[C.idx] <= C.hi)
        if C.children:
            assert len(C.children) >= 2
            joined = np.concatenate([ch.idx for ch in C.children])
            np.testing.assert_array_equal(np.sort(joined), np.sort(C.idx))
            for ch in C.children:
                walk(ch)
        else:
            assert len(C.idx) <= 40
            seen.append(C.idx)

    walk(tree)
    np.testing.assert_array_equal(np.sort(np.concatenate(seen)), np.arange(len(y)))
    # the root's children are the six faces, in label order (2 axis + (outward
    # normal along +axis)): face f holds the tiles on the plane x_axis = f % 2
    assert len(tree.children) == 6
    for f, ch in enumerate(tree.children):
        assert len(ch.idx) == len(y) // 6
        assert np.all(y[ch.idx, f // 2] == float(f % 2))
    # every cluster below the root lies in its face's plane, so its proxy
    # grid is one layer in the normal direction (49 proxies at degree 6)
    below = []

    def collect(C):
        below.append(C)
        for ch in C.children:
            collect(ch)

    for f, ch in enumerate(tree.children):
        below.clear()
        collect(ch)
        for C in below:
            assert np.ptp(y[C.idx, f // 2]) == 0.0
            if len(C.idx) > 1 and np.ptp(y[C.idx], axis=0).max() > 0.0:
                assert C.deg[f // 2] == 0 and C.n_proxy <= 49


def test_proxies_keep_the_moments_up_to_the_degree():
    """sum_k q_k s_k^alpha = sum_j a_j y_j^alpha for every tensor monomial of
    degree <= n per dimension (and likewise for p): interpolation reproduces
    those monomials exactly."""
    ps, sig, g, _ = _cube_sources()
    y, a, b = T.tile_sources(ps, sig, g)
    tree = T.build_tree(y, T.tile_faces(ps), leaf_size=64, degree=4)
    for C in (tree, tree.children[0], tree.children[-1].children[0]):
        S, q, p = C.proxies(y, a, b)
        c = C.center
        for al in [(0, 0, 0), (1, 0, 0), (0, 2, 1), (3, 1, 0), (4, 4, 4), (2, 0, 3)]:
            if any(al[d] > C.deg[d] for d in range(3)):
                continue
            mono_s = np.prod((S - c) ** np.array(al), axis=1)
            mono_y = np.prod((y[C.idx] - c) ** np.array(al), axis=1)
            ref = mono_y @ a[C.idx]
            assert abs(mono_s @ q - ref) <= 1e-11 * np.sum(np.abs(mono_y * a[C.idx])) + 1e-300, (al, C.deg)
            np.testing.assert_allclose(mono_s @ p, mono_y @ b[C.idx], rtol=0,
                                       atol=1e-11 * np.sum(np.abs(mono_y[:, None] * b[C.idx])))


def _targets(n, seed):
    rng = np.random.default_rng(seed)
    inside = rng.uniform(0.125, 0.875, (n, 3))
    outside = rng.normal(0.5, 1.0, (n, 3))
    outside = outside[np.max(np.abs(outside - 0.5), axis=1) > 0.75][: n // 2]
    return np.concatenate([inside, outside])


def test_tiny_theta_is_the_direct_sum():
    ps, sig, g, _ = _cube_sources(200)
    tg = _targets(6, 1)
    u_tree = T.potential_tree(ps, sig, g, tg, theta=1e-12)
    u_dir = POT.potential(ps, sig, g, tg)
    np.testing.assert_allclose(u_tree, u_dir, rtol=1e-12, atol=1e-14)


def test_error_falls_with_the_degree():
    ps, sig, g, _ = _cube_sources()
    y, a, b = T.tile_sources(ps, sig, g)
    tg = _targets(8, 2)
    u_dir = POT.potential(ps, sig, g, tg)
    scale = np.max(np.abs(u_dir))
    errs = []
    for n in (2, 4, 6, 8):
        tree = T.build_tree(y, T.tile_faces(ps), leaf_size=64, degree=n)
        u, cnt = T.evaluate(tree, y, a, b, tg, theta=0.5)
        assert cnt[:, 0].sum() > 0  # the proxies are used
        errs.append(np.max(np.abs(u - u_dir)) / scale)
    assert errs[0] > errs[1] > errs[2] > errs[3], errs
    assert errs[1] < 1e-4 and errs[3] < 1e-7, errs
