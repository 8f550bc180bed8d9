"""Pins for tabulated Dirichlet data on a box (face grids, bilinear
interpolation): exact on data linear in the face coordinates, the grid
values at the nodes, continuity across edges, and walks whose means follow
the tabulated function's harmonic extension."""
import numpy as np

import dtn_inputs as I
from oracle import wos


def _linear_table(gd, n0, n1, c):
    X = I.box_face_grid(gd, n0, n1)
    return c[0] + X[..., 0] * c[1] + X[..., 1] * c[2] + X[..., 2] * c[3]


def _face_points(n, seed):
    rng = np.random.default_rng(seed)
    p = rng.random((n, 3))
    k = rng.integers(0, 3, n)
    side = rng.integers(0, 2, n)
    p[np.arange(n), k] = side
    return p


def test_bilinear_is_exact_on_linear_data():
    c = [0.3, 2.0, -1.0, 0.5]
    gd = I.geometry_cube_sources()
    quad = dict(gd, data_kind="quadratic", quad=c + [0.0] * 6)
    tab = dict(gd, data_kind="table", tab=_linear_table(gd, 5, 7, c))
    x = _face_points(500, 1)
    np.testing.assert_allclose(wos.Geometry(tab).phi(x), wos.Geometry(quad).phi(x), rtol=0, atol=1e-14)


def test_nodes_cells_and_edges():
    gd = I.geometry_cube_sources()
    rng = np.random.default_rng(2)
    T = rng.standard_normal((6, 4, 5))
    g = wos.Geometry(dict(gd, data_kind="table", tab=T))
    X = I.box_face_grid(gd, 4, 5)
    # interior nodes of every face (edges belong to the lowest-index face)
    for f in range(6):
        v = g.phi(X[f, 1:-1, 1:-1].reshape(-1, 3))
        np.testing.assert_allclose(v, T[f, 1:-1, 1:-1].ravel(), rtol=0, atol=1e-15)
    # a cell centre: the mean of its four corners
    p = 0.25 * (X[4, 1, 2] + X[4, 2, 2] + X[4, 1, 3] + X[4, 2, 3])
    want = 0.25 * (T[4, 1, 2] + T[4, 2, 2] + T[4, 1, 3] + T[4, 2, 3])
    assert abs(g.phi(p[None])[0] - want) < 1e-15
    # on the edge x = 0, y = 0 (faces -x and -y) the -x face's table is used
    e = np.array([[0.0, 0.0, 0.25]])  # a node of face -x: axes (y: 4 nodes, z: 5 nodes)
    assert abs(g.phi(e)[0] - T[0, 0, 1]) < 1e-15


def test_walks_follow_the_tabulated_extension():
    """Sampled source data on 257 x 257 face grids: walk means against the
    sources' potential within 4.5 SE (the interpolation error, of order
    (1/256)^2 / 8 times the data's curvature, is far below the SE)."""
    gd = I.tabulated_cube_sources()
    y = I.interior_points_box(6, 3, margin=0.1)
    r = wos.wos_nodes(wos.Geometry(gd), y, 40_000, seed=6)
    exact = wos.Geometry(I.geometry_cube_sources()).phi(y)
    z = (r["mean"] - exact) / r["se"]
    assert np.all(np.abs(z) < 4.5), z


def test_linear_table_gives_the_same_walks_as_the_closed_form():
    c = [0.3, 2.0, -1.0, 0.5]
    gd = I.geometry_cube_sources()
    y = I.interior_points_box(20, 4, margin=0.05)
    a = wos.wos_nodes(wos.Geometry(dict(gd, data_kind="table", tab=_linear_table(gd, 9, 9, c))), y, 500, seed=8)
    b = wos.wos_nodes(wos.Geometry(dict(gd, data_kind="quadratic", quad=c + [0.0] * 6)), y, 500, seed=8)
    np.testing.assert_array_equal(a["steps"], b["steps"])
    np.testing.assert_allclose(a["mean"], b["mean"], rtol=0, atol=1e-13)
