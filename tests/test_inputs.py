"""Host-side checks of the seeded workload generators (no device)."""
import numpy as np

import dtn_inputs as I
from oracle import wos as OW


def test_boundary_points_lie_on_the_boundary_with_outward_normals():
    gd = I.geometry_box_holes()
    g = OW.Geometry(gd)
    pts, nrm = I.boundary_points(gd, 3000, np.random.default_rng(1))
    d_in, _ = g.dist_proj(pts - 1e-7 * nrm)
    assert np.all(np.abs(d_in - 1e-7) < 1e-12)  # just inside: distance = the step back
    holes = np.asarray(gd["holes"]).reshape(-1, 6)
    out = pts + 1e-7 * nrm  # just outside: in a hole or out of the box
    in_hole = np.zeros(len(pts), bool)
    for h in holes:
        in_hole |= np.all((out > h[:3]) & (out < h[3:]), axis=1)
    out_box = np.any((out < 0) | (out > 4), axis=1)
    assert np.all(in_hole ^ out_box)
    # uniform by area: the share of points on the outer box matches its area
    faces = I.boundary_faces(gd)
    area = [(f[4][(f[0] + 1) % 3] - f[3][(f[0] + 1) % 3]) * (f[4][(f[0] + 2) % 3] - f[3][(f[0] + 2) % 3])
            for f in faces]
    share = sum(area[:6]) / sum(area)
    assert abs(out_box.mean() - share) < 4 * np.sqrt(share * (1 - share) / len(pts))


def test_serving_queries_arrivals_and_sizes():
    gd = I.geometry_box_holes()
    qs = I.serving_queries(gd, n_queries=400, rate=200.0, seed=5, max_points=64)
    t = np.array([q["t"] for q in qs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 200) < 4 * (1 / 200) / np.sqrt(len(gaps))
    m = np.array([len(q["pts"]) for q in qs])
    assert m.min() >= 1 and m.max() <= 64
    # log-uniform sizes: log(m+1) roughly uniform on [0, log 65]
    assert abs(np.mean(np.log(m + 0.5)) / np.log(65) - 0.5) < 0.08
    assert len({q["seed"] for q in qs}) == len(qs)
    # required standard errors log-uniform on [1e-4, 1e-2]
    se = np.log10([q["se"] for q in qs])
    assert se.min() >= -4 and se.max() <= -2
    assert abs(se.mean() + 3) < 4 * (2 / np.sqrt(12)) / np.sqrt(len(se))
    again = I.serving_queries(gd, n_queries=400, rate=200.0, seed=5, max_points=64)
    assert all(np.array_equal(a["pts"], b["pts"]) for a, b in zip(qs, again))
