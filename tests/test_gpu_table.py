"""GPU parity of tabulated Dirichlet data (box face grids, bilinear), through
the C-ABI: walks walk for walk against the oracle, linear tables against the
closed-form linear data, the collocation solve on the oracle's statistics,
the pipeline against the sampled function's exact Neumann data, rejections."""
import numpy as np
import pytest
import torch

import dtn_inputs as I
from oracle import patch as OP
from oracle import wos as OW

from test_gpu_wos import _compare, _gpu_wos

pytestmark = pytest.mark.gpu


def _dtn():
    from paper_1210_1491_amd import dtn
    return dtn


def _linear_table(gd, n0, n1, c):
    X = I.box_face_grid(gd, n0, n1)
    return c[0] + X[..., 0] * c[1] + X[..., 1] * c[2] + X[..., 2] * c[3]


def test_tabulated_walks_match_oracle():
    gd = I.tabulated_cube_sources()
    pts = I.interior_points_box(200, 9, margin=1e-3)
    walks = np.random.default_rng(10).integers(2, 2000, size=len(pts))
    gpu = _gpu_wos(gd, pts, walks, seed=31)
    ora = OW.wos_nodes(OW.Geometry(gd), pts, walks, seed=31)
    _compare(gpu, ora)
    g32 = _gpu_wos(gd, pts[:64], 20_000, seed=4, precision="fp32")
    o32 = OW.wos_nodes(OW.Geometry(gd), pts[:64], 20_000, seed=4)
    _compare(g32, o32, exact_walks=False)


def test_linear_table_equals_closed_form_linear_data():
    c = [0.3, 2.0, -1.0, 0.5]
    gd = I.geometry_cube_sources()
    pts = I.interior_points_box(100, 11, margin=1e-3)
    a = _gpu_wos(dict(gd, data_kind="table", tab=_linear_table(gd, 9, 9, c)), pts, 700, seed=2)
    b = _gpu_wos(dict(gd, data_kind="quadratic", quad=c + [0.0] * 6), pts, 700, seed=2)
    np.testing.assert_array_equal(a["steps"], b["steps"])
    np.testing.assert_allclose(a["mean"], b["mean"], rtol=0, atol=1e-13)


def _tiles():
    return I.subset_patches(I.patches_cube_tiles(), I.cube_tile_subset()[:6])


def test_tabulated_solve_matches_oracle_on_oracle_statistics():
    dtn = _dtn()
    gd = I.tabulated_cube_sources(n0=65, n1=65)
    pd = _tiles()
    og = OW.Geometry(gd)
    rows, ref = [], []
    for p in OP.patches_from_desc(pd, gd):
        nodes, _ = OP.nodes_global(p)
        r = OW.wos_nodes(og, nodes, 200, seed=3)
        rows.append(np.column_stack([r["count"], r["mean"], r["m2"], r["steps"]]))
        ref.append(OP.patch_solve(p, og, r["mean"], r["se"])["sigma"])
    plan = dtn.Plan(dtn.Geometry(gd), pd)
    sig, _ = plan.solve(torch.tensor(np.concatenate(rows), device="cuda"))
    ref = np.concatenate(ref)
    K = OP.single_layer_matrix(1.0 / 32.0, None, 4, 16)
    bar = np.abs(np.linalg.inv(K)).sum(1).max() * 1e-11
    assert np.max(np.abs(sig.cpu().numpy() - ref)) < bar


def test_tabulated_pipeline_against_the_sampled_function():
    dtn = _dtn()
    gd = I.tabulated_cube_sources()
    pd = _tiles()
    g = dtn.Geometry(gd)
    plan = dtn.Plan(g, pd)
    nodes = plan.nodes()
    W = torch.full((plan.num_nodes,), 20_000, dtype=torch.int64, device="cuda")
    stats, _ = dtn.wos_eval(g, nodes, W, seed=5)
    sig, se = plan.solve(stats)
    sig, se = sig.cpu().numpy(), se.cpu().numpy()
    xg, ng, area, tr = [], [], [], []
    for p in OP.patches_from_desc(pd, gd):
        a, b, c, d = OP.collocation_points(p)
        xg.append(a)
        ng.append(b)
        area.append(c)
        tr.append(d < 0.7 * p.h)
    xg, ng, area, tr = map(np.concatenate, (xg, ng, area, tr))
    ex = OP.exact_neumann(I.geometry_cube_sources(), xg, ng)
    noise = float(np.sqrt(np.sum(area[tr] * se[tr] ** 2) / np.sum(area[tr] * ex[tr] ** 2)))
    assert OP.rel_l2(sig, ex, area, tr) < 3 * noise + 1e-3


def test_tabulated_rejections():
    dtn = _dtn()
    tab = np.zeros((6, 4, 4))
    with pytest.raises(dtn.DtnError):      # tables need a box
        dtn.Geometry(dict(I.geometry_ball_quadratic(), data_kind="table", tab=tab))
    with pytest.raises(dtn.DtnError):      # at least 2 nodes per axis
        dtn.Geometry(dict(I.geometry_cube_sources(), data_kind="table", tab=np.zeros((6, 1, 4))))
    bad = tab.copy()
    bad[2, 1, 1] = np.nan
    with pytest.raises(dtn.DtnError):
        dtn.Geometry(dict(I.geometry_cube_sources(), data_kind="table", tab=bad))


def test_points_and_server_on_tabulated_data():
    """Single-point queries on box faces and the query server both read the
    face tables: the points against the oracle's reduction of its own walks,
    the server's answers against the sampled function's exact du/dn."""
    from oracle import point as OPt
    dtn = _dtn()
    gd = I.tabulated_cube_sources()
    g = dtn.Geometry(gd)
    og = OW.Geometry(gd)
    x = np.array([[0.5, 0.5, 0.0], [0.3, 0.0, 0.6]])
    nrm = np.array([[0.0, 0.0, -1.0], [0.0, -1.0, 0.0]])
    t1 = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    a = np.array([0.2, 0.25])
    P = dtn.Points(g, x, nrm, t1, a, n_g1=10, n_g2=10)
    nodes = P.nodes()
    W = torch.full((P.num_nodes,), 2000, dtype=torch.int64, device="cuda")
    stats, _ = dtn.wos_eval(g, nodes, W, 3)
    out = P.neumann(stats).cpu().numpy()
    onodes = np.concatenate([OPt.hemisphere_rule(x[i], nrm[i], t1[i], a[i], 10)[0] for i in range(2)])
    r = OW.wos_nodes(og, onodes, 2000, seed=3)
    st = np.column_stack([r["count"], r["mean"], r["m2"], r["steps"]])
    for i in range(2):
        want = OPt.point_neumann(og.phi, x[i], nrm[i], t1[i], a[i], 10, 10, 1e-6, st[i * 100:(i + 1) * 100])
        assert abs(out[i, 0] - want[0]) < 0.05 * want[1], (i, out[i], want)
    # the server on the tabulated data
    S = dtn.Server(g, n_streams=2, precision="fp32", pilot_walks=64, min_walks=64, max_walks=20_000,
                   layout=(8, 16, 4, 8))
    rng = np.random.default_rng(7)
    pts, nn = I.boundary_points(I.geometry_cube_sources(), 6, rng)
    S.submit(1, pts, nn, 0.01, 5)
    done = []
    while not done:
        r = S.wait(timeout=120.0)
        assert r, "server wait timed out"
        done.extend(r)
    S.close()
    assert done[0]["status"] == 0, done[0]
    ans = done[0]["answer"]
    ex = OP.exact_neumann(I.geometry_cube_sources(), pts, nn)
    assert np.all(np.abs(ans[:, 0] - ex) < 4.5 * ans[:, 1] + 5e-3), (ans, ex)
