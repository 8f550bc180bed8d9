"""Pins for the oracle's distance queries and walk-on-spheres estimator.

The WOS estimate of u (Sec. 2, eq. bw13, sampled as in the text after
Fig. fig_wos; node estimator eq. bw87) is checked against exact harmonic
solutions, its Monte Carlo error against the N^-1/2 law, the epsilon-shell
bias against its O(epsilon) size, and the distance/closest-point queries
against brute force over sampled boundary points.
"""
import numpy as np
import pytest

import dtn_inputs as I
from oracle import wos


def _box_surface_samples(lo, hi, m=120):
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    g = np.linspace(0, 1, m)
    A, B = np.meshgrid(g, g, indexing="ij")
    pts = []
    for k in range(3):
        a, b = (k + 1) % 3, (k + 2) % 3
        for side in (lo[k], hi[k]):
            p = np.zeros((m * m, 3))
            p[:, k] = side
            p[:, a] = lo[a] + A.ravel() * (hi[a] - lo[a])
            p[:, b] = lo[b] + B.ravel() * (hi[b] - lo[b])
            pts.append(p)
    return np.concatenate(pts)


def test_distance_ball_closed_form():
    g = wos.Geometry(I.geometry_ball_quadratic())
    x = I.interior_points_ball(500, 1)
    d, p = g.dist_proj(x)
    np.testing.assert_allclose(d, 1 - np.linalg.norm(x, axis=1), atol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(p, axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(x - p, axis=1), d, atol=1e-14)


def test_distance_box_minus_holes_brute_force():
    holes = np.array([[0.2, 0.2, 0.2, 0.45, 0.5, 0.4], [0.6, 0.55, 0.5, 0.8, 0.75, 0.9]])
    desc = dict(I.geometry_cube_sources(), kind="box_minus_boxes", holes=holes)
    g = wos.Geometry(desc)
    rng = np.random.default_rng(4)
    x = rng.random((4000, 3))
    inside_hole = np.zeros(len(x), bool)
    for h in holes:
        inside_hole |= np.all((x >= h[:3]) & (x <= h[3:]), axis=1)
    x = x[~inside_hole][:300]
    d, p = g.dist_proj(x)
    surf = np.concatenate([_box_surface_samples((0, 0, 0), (1, 1, 1))] +
                          [_box_surface_samples(h[:3], h[3:], 60) for h in holes])
    for i in range(len(x)):
        bd = np.min(np.linalg.norm(surf - x[i], axis=1))
        assert d[i] <= bd + 1e-12
        assert bd - d[i] < 0.02  # sample spacing bound
        assert abs(np.linalg.norm(x[i] - p[i]) - d[i]) < 1e-13
    # projections lie on a surface: outer faces or a hole's boundary
    on_outer = np.any(np.isclose(p, 0.0, atol=1e-15) | np.isclose(p, 1.0, atol=1e-15), axis=1)
    on_hole = np.zeros(len(p), bool)
    for h in holes:
        inb = np.all((p >= h[:3] - 1e-15) & (p <= h[3:] + 1e-15), axis=1)
        onf = np.any(np.isclose(p, h[:3], atol=1e-15) | np.isclose(p, h[3:], atol=1e-15), axis=1)
        on_hole |= inb & onf
    assert np.all(on_outer | on_hole)


def test_dirichlet_data_is_harmonic():
    for desc in (I.geometry_ball_quadratic(), I.geometry_cube_sources()):
        g = wos.Geometry(desc)
        x = I.interior_points_box(50, 3, margin=0.1)
        hh = 1e-3
        lap = -6 * g.phi(x)
        for k in range(3):
            e = np.zeros(3)
            e[k] = hh
            lap += g.phi(x + e) + g.phi(x - e)
        assert np.max(np.abs(lap / hh ** 2)) < 1e-4


def test_wos_matches_exact_ball():
    g = wos.Geometry(I.geometry_ball_quadratic(eps=1e-6))
    x = I.interior_points_ball(16, 11, r_max=0.95)
    r = wos.wos_nodes(g, x, 40_000, seed=5)
    z = (r["mean"] - g.phi(x)) / r["se"]
    assert np.all(np.abs(z) < 4.5), z
    assert np.all(r["capped"] == 0)
    assert np.all(r["count"] == 40_000)


def test_wos_matches_exact_cube_sources():
    g = wos.Geometry(I.geometry_cube_sources(eps=1e-6))
    x = I.interior_points_box(16, 12)
    r = wos.wos_nodes(g, x, 40_000, seed=6)
    z = (r["mean"] - g.phi(x)) / r["se"]
    assert np.all(np.abs(z) < 4.5), z


def test_wos_error_decays_as_inverse_sqrt_n():
    g = wos.Geometry(I.geometry_ball_quadratic(eps=1e-6))
    x = I.interior_points_ball(64, 13, r_max=0.9)
    ex = g.phi(x)
    ns = np.array([100, 1000, 10_000])
    rms = []
    for k, n in enumerate(ns):
        r = wos.wos_nodes(g, x, int(n), seed=100 + k)
        rms.append(np.sqrt(np.mean((r["mean"] - ex) ** 2)))
    slope = np.polyfit(np.log(ns), np.log(rms), 1)[0]
    assert -0.62 < slope < -0.38, slope


def test_epsilon_shell_bias_is_order_epsilon():
    """A thick shell biases the estimate by O(eps); a thin one does not."""
    x = np.array([[0.0, 0.0, 0.5]])
    big = wos.Geometry(I.geometry_ball_quadratic(eps=0.1))
    small = wos.Geometry(I.geometry_ball_quadratic(eps=1e-6))
    rb = wos.wos_nodes(big, x, 200_000, seed=8)
    rs = wos.wos_nodes(small, x, 200_000, seed=8)
    ex = small.phi(x)[0]
    bias_big = rb["mean"][0] - ex
    assert abs(bias_big) > 6 * rb["se"][0]
    assert abs(bias_big) < 0.1 * 3.0  # eps times a bound on |grad u| over the ball
    assert abs(rs["mean"][0] - ex) < 4.5 * rs["se"][0]
    # shells end walks earlier
    assert rb["steps"][0] < rs["steps"][0]


def test_walk_ranges_compose_and_seed_determinism():
    """Counter-based streams: walks [0,a) + [a,n) equal walks [0,n)."""
    g = wos.Geometry(I.geometry_cube_sources())
    x = I.interior_points_box(4, 21)
    full = wos.wos_nodes(g, x, 3000, seed=9)
    again = wos.wos_nodes(g, x, 3000, seed=9, threads=1)
    for k in ("count", "mean", "m2", "steps"):
        np.testing.assert_array_equal(full[k], again[k])
    a = wos.wos_nodes(g, x, 1200, seed=9)
    b = wos.wos_nodes(g, x, 1800, seed=9, walk_begin=1200)
    n = a["count"] + b["count"]
    mean = (a["count"] * a["mean"] + b["count"] * b["mean"]) / n
    delta = b["mean"] - a["mean"]
    m2 = a["m2"] + b["m2"] + delta ** 2 * a["count"] * b["count"] / n
    np.testing.assert_allclose(mean, full["mean"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(m2, full["m2"], rtol=1e-10)
    np.testing.assert_array_equal(a["steps"] + b["steps"], full["steps"])
    other = wos.wos_nodes(g, x, 3000, seed=10)
    assert np.all(other["mean"] != full["mean"])
    sid = wos.wos_nodes(g, x, 3000, seed=9, stream_id=np.arange(4) + 7)
    assert np.all(sid["mean"] != full["mean"])


def test_per_walk_scores_match_node_statistics():
    g = wos.Geometry(I.geometry_ball_quadratic())
    y = np.array([0.1, 0.2, 0.3])
    s, st = wos.wos_scores(g, y, seed=4, stream_id=0, walk_begin=0, n_walks=500)
    r = wos.wos_nodes(g, y[None], 500, seed=4)
    assert abs(r["mean"][0] - s.mean()) < 1e-13
    assert abs(r["m2"][0] - np.sum((s - s.mean()) ** 2)) < 1e-11
    assert r["steps"][0] == st.sum()
    # every recorded point is a boundary value of phi: within the data range
    assert np.all(np.abs(s) <= 2.0)


def test_edge_cases_start_in_shell_cap_and_empty():
    desc = I.geometry_ball_quadratic(eps=1e-3)
    g = wos.Geometry(desc)
    y = np.array([[0.0, 0.0, 1.0 - 5e-4], [0.0, 0.5, 0.0], [0.2, 0.0, 0.1]])
    r = wos.wos_nodes(g, y, np.array([10, 0, 1]), seed=1)
    # start inside the shell: zero steps, value = phi at the closest point
    assert r["steps"][0] == 0 and r["count"][0] == 10
    assert r["mean"][0] == pytest.approx(g.phi([[0, 0, 1.0]])[0], abs=1e-15)
    assert r["m2"][0] == 0.0
    # zero walks: empty statistics
    assert r["count"][1] == 0 and r["mean"][1] == 0.0 and r["steps"][1] == 0
    # one walk: zero spread
    assert r["count"][2] == 1 and r["m2"][2] == 0.0
    # a step cap is counted, never silent
    capd = wos.Geometry(dict(desc, max_steps=2))
    rc = wos.wos_nodes(capd, y[1:2], 100, seed=1)
    assert rc["capped"][0] > 50 and rc["steps"][0] <= 200


def test_adaptive_budget_follows_the_exit_variance():
    """From the centre of the unit ball the first jump lands on the sphere
    and its end point is uniform there (the harmonic measure seen from the
    centre), so with phi = z every walk takes one step and the scores have
    variance E[z^2] = 1/3.  The budget must then be close to 1/(3 se^2) and
    the final standard error close to se."""
    desc = dict(I.geometry_ball_quadratic(eps=1e-6), quad=[0.0, 0.0, 0.0, 1.0] + [0.0] * 6)
    g = wos.Geometry(desc)
    x = np.zeros((8, 3))
    se = 0.01
    r = wos.wos_adaptive(g, x, 1000, 100, 10 ** 6, se, seed=3, stream_id=np.arange(8))
    expect = 1.0 / (3.0 * se * se)
    # sd of the pilot variance of z^2, z uniform on [-1,1]: sqrt((1/5 - 1/9) / 1000)
    sd = expect * np.sqrt((1 / 5 - 1 / 9) / 1000) * 3.0
    assert np.all(np.abs(r["walks_used"] - expect) < 5 * sd), r["walks_used"]
    np.testing.assert_array_equal(r["count"], r["walks_used"])
    np.testing.assert_array_equal(r["steps"], r["walks_used"])  # one step per walk
    assert np.all(np.abs(r["se"] / se - 1.0) < 0.1), r["se"]
    assert np.all(np.abs(r["mean"]) < 5 * r["se"])


def test_adaptive_clamps_and_prefix():
    """A point inside the shell has zero spread: it gets min_walks (or the
    pilot if larger); a tiny target hits max_walks; the statistics are those
    of the first walks_used walks of each point."""
    desc = I.geometry_ball_quadratic(eps=1e-3)
    g = wos.Geometry(desc)
    y = np.array([[0.0, 0.0, 1.0 - 5e-4], [0.0, 0.5, 0.0], [0.2, 0.0, 0.1]])
    r = wos.wos_adaptive(g, y, 300, 1500, 4000, 1e-6, seed=2)
    assert list(r["walks_used"]) == [1500, 4000, 4000]
    r2 = wos.wos_adaptive(g, y, 300, 100, 4000, 1e-6, seed=2)
    assert r2["walks_used"][0] == 300  # never fewer than the pilot
    loose = wos.wos_adaptive(g, y, 300, 100, 4000, 10.0, seed=2)
    assert list(loose["walks_used"]) == [300, 300, 300]
    plain = wos.wos_nodes(g, y, r["walks_used"], seed=2)
    for k in ("count", "mean", "m2", "steps"):
        np.testing.assert_array_equal(r[k], plain[k])
