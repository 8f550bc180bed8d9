"""Pins for the single-point flat-boundary oracle (Sec. 5.1) and for the
half-space walks with a truncation sphere that feed it.

What fixes the answers:
  - Table 1's Sigma2' column and Table 2's small-delta rows (printed values,
    fixtures under tests/golden/ with their citation);
  - the identity Sigma1' + Sigma2' = du/dn for the exact u on the hemisphere
    (eq. bw64 with exact node values), against the closed-form derivative of
    point-source data: any dropped term, wrong sign, wrong kernel constant or
    wrong polar-angle map breaks it;
  - closed forms of the rules: nodes on the hemisphere, sum of the weights
    int_Gamma 3 cos(theta) / (2 pi a^3) ds = 3 / (2a);
  - the half-space walks: exact u of point-source data (R -> infinity), the
    exact half-ball escape probability as a bound (a walk that lands outside
    the sphere has crossed it), and a step-by-step re-walk on tiny inputs;
  - Table 1 itself: the Monte Carlo totals at N_path = 1e3 against the
    analytic value within their standard errors.
"""
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as L

import dtn_inputs as I
from oracle import point as P
from oracle import wos

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
X0 = (0.5, 0.0, 0.0)
N_DOWN = (0.0, 0.0, -1.0)
T1 = (1.0, 0.0, 0.0)


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#", dtype=str)


def _geom(**kw):
    return wos.Geometry(dict(I.geometry_halfspace_charge(), **kw))


def _exact_dudn(x, src):
    """-d/dz of sum q / |y - s| at a point of the plane z = 0 (n = -z)."""
    x = np.asarray(x, float)
    out = 0.0
    for s in np.asarray(src, float):
        d = x - s[:3]
        out += s[3] * d[2] / np.linalg.norm(d) ** 3
    return out


def test_table1_sigma2_column():
    g = _geom()
    rows = _load("table1_halfspace.txt").astype(float)
    for a, _s1, s2, _tot, _err in rows:
        v = P.sigma2(g.phi, X0, N_DOWN, T1, a, 20, 1e-6)
        assert abs(v - s2) <= 5e-7, (a, v, s2)


def test_table2_small_delta_rows():
    g = _geom()
    tab = _load("table2_sigma2.txt").astype(float)
    for row in tab:
        drel = row[0]
        if drel > 1e-4:
            continue  # larger delta/a rows: parity unpinned (see the fixture)
        # delta/a <= 1e-5: to the printed digit; 1e-4: the table's values sit
        # about 0.9 delta/a Sigma2' above the ring rule's, as its larger-delta
        # rows do, which adds 1e-5 to the rounding of the printed digit
        tol = 1e-5 if drel <= 1e-5 else 2e-5
        for ng, want in zip((4, 6, 10, 20), row[1:]):
            v = P.sigma2(g.phi, X0, N_DOWN, T1, 0.5, ng, drel)
            assert abs(v - want) <= tol, (drel, ng, v, want)


@pytest.mark.parametrize("a", [0.1, 0.2, 0.5, 0.7, 1.0])
def test_identity_with_exact_u_test1(a):
    g = _geom()
    nodes, W = P.hemisphere_rule(X0, N_DOWN, T1, a, 20)
    st = np.zeros((len(nodes), 4))
    st[:, 0] = 1
    st[:, 1] = g.phi(nodes)
    v, se, s1, s2 = P.point_neumann(g.phi, X0, N_DOWN, T1, a, 20, 20, 1e-6, st)
    assert se == 0.0
    exact = 1.0 / 1.25 ** 1.5
    assert abs(exact - 0.715542) < 5e-7  # the table's analytic column
    assert abs(v - exact) < 1e-6, (a, v, exact)


def test_identity_with_exact_u_general_data():
    """Off-centre point, several sources, a tilted tangent: the identity holds."""
    rng = np.random.default_rng(11)
    src = np.column_stack([rng.uniform(-1, 1, (4, 2)), -rng.uniform(0.6, 1.5, 4), rng.uniform(-1, 1, 4)])
    g = _geom(src=src)
    x = (0.3, -0.2, 0.0)
    ang = 0.7
    t1 = (np.cos(ang), np.sin(ang), 0.0)
    exact = _exact_dudn(x, src)
    for a in (0.15, 0.4):
        nodes, W = P.hemisphere_rule(x, N_DOWN, t1, a, 24)
        st = np.column_stack([np.ones(len(nodes)), g.phi(nodes), np.zeros(len(nodes)), np.zeros(len(nodes))])
        v, *_ = P.point_neumann(g.phi, x, N_DOWN, t1, a, 24, 24, 1e-7, st)
        assert abs(v - exact) < 2e-6 * max(1.0, abs(exact)), (a, v, exact)


def test_rules_closed_forms():
    for a in (0.1, 0.7):
        nodes, W = P.hemisphere_rule(X0, N_DOWN, T1, a, 20)
        r = nodes - np.asarray(X0)
        np.testing.assert_allclose(np.linalg.norm(r, axis=1), a, rtol=1e-14)
        assert np.all(nodes[:, 2] > 0)  # inside the half space z > 0
        np.testing.assert_allclose(W.sum(), 1.5 / a, rtol=1e-13)
        assert np.all(W > 0)
        pts, Wr, rho = P.ring_rule(X0, N_DOWN, T1, a, 20, 1e-6)
        np.testing.assert_allclose(pts[:, 2], 0.0)
        np.testing.assert_allclose(np.linalg.norm(pts - np.asarray(X0), axis=1), rho, rtol=0, atol=1e-15)
        # area of the ring
        np.testing.assert_allclose(Wr.sum(), np.pi * (a * a - (1e-6 * a) ** 2), rtol=1e-13)


def test_standard_error_propagation():
    a = 0.5
    nodes, W = P.hemisphere_rule(X0, N_DOWN, T1, a, 8)
    n, var = 50.0, 0.3
    st = np.column_stack([np.full(len(nodes), n), np.ones(len(nodes)), np.full(len(nodes), var * (n - 1)),
                          np.zeros(len(nodes))])
    g = _geom()
    _, se, _, _ = P.point_neumann(g.phi, X0, N_DOWN, T1, a, 8, 8, 1e-6, st)
    assert abs(se - np.sqrt(var / n * np.sum(W * W))) < 1e-15


# ----------------------------------------------------- half-space walks

def test_half_space_distance_and_projection():
    g = _geom()
    rng = np.random.default_rng(2)
    x = np.column_stack([rng.uniform(-3, 3, (200, 2)), rng.uniform(0, 2, 200)])
    d, p = g.dist_proj(x)
    np.testing.assert_array_equal(d, x[:, 2])
    np.testing.assert_array_equal(p[:, :2], x[:, :2])
    np.testing.assert_array_equal(p[:, 2], 0.0)


def test_half_space_walks_match_exact_u():
    g = _geom()
    y = np.array([[0.5, 0.0, 0.3], [0.1, -0.4, 0.05], [1.2, 0.7, 0.9]])
    r = wos.wos_nodes(g, y, 40_000, seed=5)
    exact = g.phi(y)  # u off the plane is the potential of the source itself
    z = (r["mean"] - exact) / r["se"]
    assert np.all(np.abs(z) < 4.5), z
    assert np.all(r["capped"] == 0)


def test_half_space_start_cases():
    g = _geom(trunc_r=10.0)
    # outside the truncation sphere: gone to infinity at once, score 0
    s, st = wos.wos_scores(g, (0.0, 0.0, 10.0), 1, 0, 0, 5)
    np.testing.assert_array_equal(s, 0.0)
    np.testing.assert_array_equal(st, 0)
    # beyond the sphere and within the shell: the sphere is tested first
    s, st = wos.wos_scores(g, (20.0, 0.0, 0.5e-5), 1, 0, 0, 3)
    np.testing.assert_array_equal(s, 0.0)
    np.testing.assert_array_equal(st, 0)
    # within the shell: scored at the plane point, no step
    s, st = wos.wos_scores(g, (0.2, 0.1, 0.5e-5), 1, 0, 0, 5)
    np.testing.assert_array_equal(s, g.phi([(0.2, 0.1, 0.0)])[0])
    np.testing.assert_array_equal(st, 0)


def _rewalk(desc, y, seed, sid, walk):
    """Step-by-step half-space walk from the rule alone (tiny inputs)."""
    c = np.asarray(desc["ball_c"], float)
    R = desc["trunc_r"]
    x = np.asarray(y, float).copy()
    n = 0
    words = None
    while True:
        if np.dot(x - c, x - c) >= R * R:
            return 0.0, n
        d = x[2]
        if d < desc["eps"]:
            break
        if n >= desc["max_steps"]:
            break
        if n % 2 == 0:
            words = wos.philox([[walk & 0xffffffff, walk >> 32, n >> 1, sid]], seed)[0]
        k = 2 * (n % 2)
        u = (np.array([words[k], words[k + 1]], float) + 0.5) / 2.0 ** 32
        w = wos.direction(u[None, :])[0]
        x = x + d * w
        n += 1
    src = np.asarray(desc["src"], float)
    p = np.array([x[0], x[1], 0.0])
    return float(sum(s[3] / np.linalg.norm(p - s[:3]) for s in src)), n


def test_half_space_rewalk_tiny():
    desc = dict(I.geometry_halfspace_charge(), trunc_r=3.0, max_steps=60)
    g = wos.Geometry(desc)
    y = (0.4, 0.1, 0.8)
    s, st = wos.wos_scores(g, y, 9, 3, 0, 300)
    escaped = 0
    for k in range(300):
        sv, nv = _rewalk(desc, y, 9, 3, k)
        assert nv == st[k]
        assert abs(sv - s[k]) <= 1e-14 * max(1.0, abs(sv))
        escaped += sv == 0.0
    assert escaped > 0  # the sphere is reached by some walks


def _half_ball_escape(z0, R, lmax=401):
    """Exact probability that Brownian motion from (0, 0, z0) reaches the
    hemisphere |x| = R (z > 0) before the plane z = 0: odd Legendre series of
    the half-ball harmonic with data 1 on the hemisphere, 0 on the disk."""
    s = 0.0
    for l in range(1, lmax, 2):
        c = np.zeros(l + 1)
        c[l] = 1.0
        integ = L.legint(c, lbnd=0)
        s += (2 * l + 1) * (L.legval(1.0, integ) - L.legval(0.0, integ)) * (z0 / R) ** l
    return s


def test_half_space_escape_probability_bound():
    # constant data 1 on the plane: the walk mean is the absorbed fraction
    g = _geom(data_kind="quadratic", quad=[1.0] + [0.0] * 9, src=np.zeros((0, 4)), trunc_r=5.0)
    r = wos.wos_nodes(g, [[0.0, 0.0, 0.5]], 200_000, seed=3)
    v = _half_ball_escape(0.5, 5.0)
    assert abs(v - 1.5 * 0.5 / 5.0) < 0.01  # leading dipole term
    # a walk scored 0 has landed outside the sphere, so its path crossed it:
    # escapes are at most the exact first-passage probability
    assert r["mean"][0] >= 1.0 - v - 4 * r["se"][0]
    # and the sphere does take walks away
    assert r["mean"][0] < 1.0 - 0.5 * v


def test_table1_reproduction_monte_carlo():
    g = _geom()
    rows = _load("table1_halfspace.txt").astype(float)
    exact = 1.0 / 1.25 ** 1.5
    for a, s1_paper, s2_paper, tot_paper, err_paper in rows:
        nodes, W = P.hemisphere_rule(X0, N_DOWN, T1, a, 20)
        r = wos.wos_nodes(g, nodes, 1000, seed=7)
        st = np.column_stack([r["count"], r["mean"], r["m2"], r["steps"]])
        v, se, s1, s2 = P.point_neumann(g.phi, X0, N_DOWN, T1, a, 20, 20, 1e-6, st)
        assert abs(s2 - s2_paper) <= 5e-7
        assert abs(v - exact) < 4 * se, (a, v, se)
        # the paper's own estimate lies within the same Monte Carlo spread
        assert abs(tot_paper - exact) < 4 * se, (a, tot_paper, se)
        assert abs(100 * (tot_paper - 0.71554) / 0.71554 - err_paper) < 0.02
        assert int(r["capped"].sum()) == 0


# ------------------------------------------- exterior of a thin disk (Test 4)

def _disk_u(x, b=1.0):
    """Potential of a conducting disk of radius b at u = 1 (closed form in
    oblate spheroidal coordinates): (2/pi) arcsin(2b / (r_+ + r_-)), r_+/-
    the distances to the rim in the meridian plane."""
    x = np.atleast_2d(x)
    rho = np.hypot(x[:, 0], x[:, 1])
    rp = np.sqrt((rho + b) ** 2 + x[:, 2] ** 2)
    rm = np.sqrt((rho - b) ** 2 + x[:, 2] ** 2)
    return 2.0 / np.pi * np.arcsin(np.minimum(1.0, 2.0 * b / (rp + rm)))


def test_disk_potential_closed_form_is_the_disk_potential():
    # 1 on the disk, ~ (2/pi) b / r far away (total charge 8 b, eq. bw95),
    # harmonic off the disk (7-point Laplacian)
    assert abs(_disk_u([[0.3, -0.2, 0.0]])[0] - 1.0) < 1e-15
    far = np.array([[3e3, 1e3, 2e3]])
    r = np.linalg.norm(far)
    assert abs(_disk_u(far)[0] * r / (2.0 / np.pi) - 1.0) < 1e-6
    h = 1e-3
    for p in ([0.4, 0.1, 0.3], [1.3, -0.2, 0.05], [0.2, 0.2, -0.7]):
        p = np.asarray(p)
        lap = sum(_disk_u(p + h * e)[0] + _disk_u(p - h * e)[0] for e in np.eye(3)) - 6 * _disk_u(p)[0]
        assert abs(lap / h ** 2) < 1e-4
    # the density of eq. bw95 is -du/dz on the upper face
    x0 = np.array([-0.5, 0.0, 0.0])
    fd = (1.0 - _disk_u(x0 + [0, 0, 1e-6])[0]) / 1e-6
    assert abs(fd - 8.0 / (4 * np.pi * np.sqrt(0.75))) < 1e-4


def test_disk_distance_and_projection_brute_force():
    g = wos.Geometry(I.geometry_disk())
    rng = np.random.default_rng(8)
    x = rng.uniform(-2, 2, (300, 3))
    x[:50, 2] = rng.uniform(-1e-3, 1e-3, 50)  # next to the faces
    d, p = g.dist_proj(x)
    rr, tt = np.meshgrid(np.sqrt(np.linspace(0, 1, 400)), np.linspace(0, 2 * np.pi, 800, endpoint=False))
    disk = np.column_stack([(rr * np.cos(tt)).ravel(), (rr * np.sin(tt)).ravel(), np.zeros(rr.size)])
    for i in range(len(x)):
        bd = np.min(np.linalg.norm(disk - x[i], axis=1))
        assert d[i] <= bd + 1e-12 and bd - d[i] < 0.01
        assert abs(np.linalg.norm(x[i] - p[i]) - d[i]) < 1e-13
        assert p[i, 2] == 0.0 and np.hypot(p[i, 0], p[i, 1]) <= 1.0 + 1e-15


def test_disk_walks_match_the_disk_potential():
    g = wos.Geometry(I.geometry_disk())
    y = np.array([[-0.5, 0.0, 0.2], [0.9, 0.3, -0.1], [1.5, 0.0, 0.0], [0.0, 0.0, 2.0]])
    r = wos.wos_nodes(g, y, 40_000, seed=9)
    z = (r["mean"] - _disk_u(y)) / r["se"]
    assert np.all(np.abs(z) < 4.5), z
    assert np.all(r["capped"] == 0)


def test_table5_reproduction_monte_carlo():
    """Test 4 / Table 5: x = (-0.5, 0, 0), a = 0.4, 10x10 x 100, 10x10 x 1000,
    20x20 x 1000 paths; Sigma2' is 0 for the constant data."""
    g = wos.Geometry(I.geometry_disk())
    dp = I.DISK_POINT
    exact = 8.0 / (4.0 * np.pi * np.sqrt(1.0 - 0.25))
    assert abs(exact - 0.735105) < 5e-7  # the printed analytic density
    paper = {(10, 100): 0.68888, (10, 1000): 0.73960, (20, 1000): 0.73441}
    for ng, npath in I.TABLE5_RULES:
        nodes, _ = P.hemisphere_rule(dp["x"], dp["n"], dp["t1"], dp["a"], ng)
        r = wos.wos_nodes(g, nodes, npath, seed=3)
        st = np.column_stack([r["count"], r["mean"], r["m2"], r["steps"]])
        v, se, s1, s2 = P.point_neumann(g.phi, dp["x"], dp["n"], dp["t1"], dp["a"], ng, 20, 1e-6, st)
        assert s2 == 0.0
        assert abs(v - exact) < 4 * se, (ng, npath, v, se)
        assert abs(paper[(ng, npath)] - exact) < 4 * se
