"""Pins for the oracle's local BIE (Sec. 4, eqs. bw47-bw51; Sec. 5.2).

Each pin is fixed by mathematics outside the oracle's own code: closed forms
(disk potential via the complete elliptic integral, areas of spherical caps,
the reflection symmetry that makes the Poisson kernel integrate to 1/2 over a
flat patch's hemisphere), identities of the representation formula bw47 with
exact data evaluated by an independent quadrature, special solutions
(u = 1 gives sigma = 0; u linear in the normal coordinate gives sigma = 1),
finite differences of the kernels, and the spread of sigma over seeds
against the propagated standard error.
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy import integrate, special

import dtn_inputs as I
from oracle import patch as P
from oracle import wos

H_FLAT = 1.0 / 32.0


def _cube_patch(idx=0, **kw):
    gd = I.geometry_cube_sources()
    return P.patches_from_desc(I.subset_patches(I.patches_cube_tiles(**kw), [idx]), gd)[0], gd


def _ball_patch():
    gd = I.geometry_ball_quadratic()
    return P.patches_from_desc(I.patches_ball_pole(), gd)[0], gd


def _exterior_patch():
    gd = I.geometry_ball_exterior()
    return P.patches_from_desc(I.patches_big_sphere(), gd)[0], gd


def test_exterior_patch_geometry():
    """Outside a ball (signed radius -3): Gamma is more than a hemisphere
    and outside the ball, S lies on the sphere with the normal pointing to
    the centre, the panel areas add up to the cap's area."""
    p, gd = _exterior_patch()
    assert p.R == -3.0
    h, R = p.h, p.R
    tm = P.theta_max(h, R)
    assert tm == pytest.approx(np.arccos(-1.0 / 6.0)) and tm > 0.5 * np.pi
    Yg, W = P.nodes_global(p)
    assert np.all(np.linalg.norm(Yg, axis=1) > 3.0 - 1e-12)
    np.testing.assert_allclose(np.linalg.norm(Yg - p.c, axis=1), h, rtol=1e-14)
    assert W.sum() == pytest.approx(2 * np.pi * h * h * (1 - np.cos(tm)), rel=1e-13)
    boxes, X, N, area = P.panels(h, R, 4, 16)
    Xg, Ng = p.to_global(X), p.normal_to_global(N)
    np.testing.assert_allclose(np.linalg.norm(Xg, axis=1), 3.0, rtol=1e-14)
    np.testing.assert_allclose(Ng, -Xg / 3.0, atol=1e-14)
    sm = P.s_max(h, R)
    assert np.all(np.linalg.norm(Xg - p.c, axis=1) <= h)
    assert area.sum() == pytest.approx(2 * np.pi * 9.0 * (1 - np.cos(sm)), rel=1e-13)
    # the surface Jacobian integrates to the same area
    s, ws = np.polynomial.legendre.leggauss(40)
    s, ws = 0.5 * sm * (s + 1), 0.5 * sm * ws
    _, _, jac = P.surface(s, 0.0 * s, R)
    assert np.sum(jac * ws) * 2 * np.pi == pytest.approx(area.sum(), rel=1e-13)


def test_node_weights_sum_to_gamma_area():
    for h, R in ((0.2, None), (0.2, 1.0), (0.5, 3.0)):
        _, W, _, _ = P.node_grid(h, R, 8, 16)
        tm = P.theta_max(h, R)
        assert W.sum() == pytest.approx(2 * np.pi * h * h * (1 - np.cos(tm)), rel=1e-13)
    Y, _, th, _ = P.node_grid(0.2, 1.0, 8, 16)
    # on the sphere |y - c| = h and inside the unit ball around (0,0,-1)
    np.testing.assert_allclose(np.linalg.norm(Y, axis=1), 0.2, rtol=1e-14)
    assert np.all(np.linalg.norm(Y - [0, 0, -1.0], axis=1) < 1.0)
    assert P.theta_max(0.2, 1.0) == pytest.approx(np.arccos(0.1))


def test_green_function_properties():
    h = 0.3
    rng = np.random.default_rng(1)
    x = rng.normal(size=(20, 3))
    x *= (0.9 * h * rng.random(20) / np.linalg.norm(x, axis=1))[:, None]
    y = rng.normal(size=(20, 3))
    ys = h * y / np.linalg.norm(y, axis=1)[:, None]
    # vanishes on the sphere |y| = h (one Kelvin image)
    assert np.max(np.abs(P.green_ball(x, ys, h))) < 1e-12
    # symmetric
    yi = 0.8 * ys
    np.testing.assert_allclose(P.green_ball(x, yi, h), P.green_ball(yi, x, h), rtol=1e-12)
    # harmonic in y away from x
    e = 1e-4
    lap = -6 * P.green_ball(x, yi, h)
    for k in range(3):
        d = np.zeros(3)
        d[k] = e
        lap += P.green_ball(x, yi + d, h) + P.green_ball(x, yi - d, h)
    assert np.max(np.abs(lap / e ** 2)) < 1e-3 * np.max(np.abs(P.green_ball(x, yi, h))) / e
    # P = -dG/dn_y on the sphere, and dG/dn_y matches finite differences
    nrm = ys / h
    fd = (P.green_ball(x, ys + 1e-6 * nrm, h) - P.green_ball(x, ys - 1e-6 * nrm, h)) / 2e-6
    np.testing.assert_allclose(P.poisson_ball(x, ys, h), -fd, rtol=1e-6)
    np.testing.assert_allclose(P.dgreen_ball_dny(x, ys, nrm, h), fd, rtol=1e-6)
    tang = np.cross(nrm, [0.0, 0.0, 1.0])
    tang /= np.linalg.norm(tang, axis=1)[:, None]
    fd_t = (P.green_ball(x, yi + 1e-6 * tang, h) - P.green_ball(x, yi - 1e-6 * tang, h)) / 2e-6
    np.testing.assert_allclose(P.dgreen_ball_dny(x, yi, tang, h), fd_t, rtol=1e-5)


def test_poisson_kernel_is_a_probability_density():
    h = 0.7
    xi, w = leggauss(60)
    th = 0.25 * np.pi * (xi + 1)   # upper hemisphere; the lower one by reflection
    wt = 0.25 * np.pi * w
    ph = 2 * np.pi * np.arange(256) / 256
    T, F = np.meshgrid(th, ph, indexing="ij")
    Y = h * np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1)
    dA = h * h * np.sin(T) * wt[:, None] * 2 * np.pi / 256
    for x in ([0, 0, 0], [0.1, -0.2, 0.05], [0.0, 0.0, -0.3]):
        tot = np.sum(P.poisson_ball(np.array(x)[None, None], Y, h) * dA) + \
              np.sum(P.poisson_ball(np.array(x)[None, None], Y * [1, 1, -1], h) * dA)
        assert tot == pytest.approx(1.0, abs=1e-10)


def test_single_layer_row_sums_match_disk_closed_form():
    """sum_j K_ij = int_disk G_B(x_i, .) : free-space part 4h E(rho/h)/(4pi)
    (potential of a uniform disk in its plane), image part by adaptive 2-D
    quadrature."""
    h = 1.0
    K = P.single_layer_matrix(h, None, 4, 16)
    _, X, _, _ = P.panels(h, None, 4, 16)
    for i in (0, 5, 17, 33, 50, 63):
        rho = np.linalg.norm(X[i])
        free = 4 * h * special.ellipe((rho / h) ** 2) / (4 * np.pi)
        bx = X[i]
        f = lambda a, s: s / np.sqrt(s * s * rho * rho / (h * h)
                                     - 2 * s * (np.cos(a) * bx[0] + np.sin(a) * bx[1]) + h * h)
        img, _ = integrate.dblquad(f, 0, h, 0, 2 * np.pi, epsabs=1e-13, epsrel=1e-13)
        assert K[i].sum() == pytest.approx(free - img / (4 * np.pi), abs=2e-12)


def test_single_layer_scales_with_h_and_singular_rule_converges():
    K1 = P.single_layer_matrix(1.0, None, 4, 8)
    Kh = P.single_layer_matrix(0.25, None, 4, 8)
    np.testing.assert_allclose(Kh, 0.25 * K1, rtol=1e-12, atol=1e-15)
    K40 = P.single_layer_matrix(1.0, None, 4, 8, duffy_n=40)
    np.testing.assert_allclose(K40, K1, rtol=0, atol=1e-11)
    Ks = P.single_layer_matrix(0.2, 1.0, 4, 8)
    Ks40 = P.single_layer_matrix(0.2, 1.0, 4, 8, duffy_n=40)
    np.testing.assert_allclose(Ks40, Ks, rtol=0, atol=1e-12)


def test_gamma_operator_rows_and_convergence():
    QI = P.gamma_operator(H_FLAT, None, 16, 32, 4, 16)
    # flat S: the hemisphere carries exactly half of the harmonic measure
    np.testing.assert_allclose(QI.sum(1), 0.5, atol=1e-13)
    fine = P.gamma_operator(H_FLAT, None, 16, 32, 4, 16, n_sub=16, m=24, n_az=1024)
    np.testing.assert_allclose(fine, QI, rtol=0, atol=1e-12)
    QIs = P.gamma_operator(0.2, 1.0, 8, 16, 4, 8)
    fines = P.gamma_operator(0.2, 1.0, 8, 16, 4, 8, n_sub=16, m=24, n_az=1024)
    np.testing.assert_allclose(fines, QIs, rtol=0, atol=1e-12)


def _which(which, flat_idx):
    if which == "flat":
        return _cube_patch(flat_idx)
    return _ball_patch() if which == "ball" else _exterior_patch()


@pytest.mark.parametrize("which", ["flat", "ball", "exterior"])
def test_constant_data_gives_zero_neumann(which):
    p, gd = _which(which, 40)
    const = dict(gd, data_kind="quadratic", quad=[1.0] + [0.0] * 9)
    g = wos.Geometry(const)
    Y, _ = P.nodes_global(p)
    r = P.patch_solve(p, g, np.ones(len(Y)))
    assert np.max(np.abs(r["sigma"])) < 1e-9


def test_linear_normal_data_gives_unit_neumann():
    p, gd = _cube_patch(5 * 256 + 37)   # a tile of the +z face
    assert np.allclose(p.n, [0, 0, 1])
    lin = dict(gd, data_kind="quadratic", quad=[-1.0, 0, 0, 1.0] + [0.0] * 6)  # u = z - 1
    g = wos.Geometry(lin)
    Y, _ = P.nodes_global(p)
    r = P.patch_solve(p, g, g.phi(Y))
    np.testing.assert_allclose(r["sigma"], 1.0, atol=1e-9)


def _representation(p, gd, x_loc, n=48):
    """Right side of eq. bw47 at a local interior point with exact u, sigma,
    by product Gauss rules on Gamma and S (x is off both, so smooth)."""
    h, R = p.h, p.R
    g = wos.Geometry(gd)
    tm = P.theta_max(h, R)
    xi, w = leggauss(n)
    th, wt = 0.5 * tm * (xi + 1), 0.5 * tm * w
    ph = 2 * np.pi * np.arange(2 * n) / (2 * n)
    T, F = np.meshgrid(th, ph, indexing="ij")
    Y = h * np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), -np.cos(T)], -1)
    dA = h * h * np.sin(T) * wt[:, None] * (np.pi / n)
    u_g = g.phi(p.to_global(Y.reshape(-1, 3))).reshape(T.shape)
    gam = np.sum(P.poisson_ball(x_loc[None, None], Y, h) * u_g * dA)
    smax = P.s_max(h, R)
    s, ws = 0.5 * smax * (xi + 1), 0.5 * smax * w
    S, A = np.meshgrid(s, ph, indexing="ij")
    y, ny, jac = P.surface(S, A, R)
    dS = jac * ws[:, None] * (np.pi / n)
    yg = p.to_global(y.reshape(-1, 3))
    nyg = p.normal_to_global(ny.reshape(-1, 3))
    u_s = g.phi(yg).reshape(S.shape)
    sig = P.exact_neumann(gd, yg, nyg).reshape(S.shape)
    sl = np.sum(P.green_ball(x_loc[None, None], y, h) * sig * dS)
    dl = np.sum(P.dgreen_ball_dny(x_loc[None, None], y, ny, h) * u_s * dS)
    return gam - dl + sl, g.phi(p.to_global(x_loc[None]))[0]


@pytest.mark.parametrize("which", ["flat", "ball", "exterior"])
def test_local_representation_identity(which):
    p, gd = _which(which, 3 * 256 + 100)
    h = p.h
    for x_loc in ([0.1 * h, -0.2 * h, -0.4 * h], [-0.3 * h, 0.25 * h, -0.6 * h]):
        rep, exact = _representation(p, gd, np.array(x_loc))
        assert rep == pytest.approx(exact, abs=1e-10 * max(1.0, abs(exact)))


@pytest.mark.parametrize("which", ["flat", "ball", "exterior"])
def test_exact_node_values_give_accurate_neumann(which):
    """The method's deterministic floor: exact u on Gamma, exact phi on S."""
    if which == "flat":
        gd = I.geometry_cube_sources()
        pd = I.subset_patches(I.patches_cube_tiles(), I.cube_tile_subset()[:6])
        ps, bar = P.patches_from_desc(pd, gd), 1e-4
    elif which == "ball":
        p, gd = _ball_patch()
        ps, bar = [p], 2e-3
    else:
        p, gd = _exterior_patch()
        ps, bar = [p], 2e-3
    g = wos.Geometry(gd)
    sig, exs, area, trusted = [], [], [], []
    for p in ps:
        Y, _ = P.nodes_global(p)
        r = P.patch_solve(p, g, g.phi(Y))
        sig.append(r["sigma"])
        exs.append(P.exact_neumann(gd, r["x"], r["normal"]))
        area.append(r["area"])
        trusted.append(r["r"] < 0.7 * P.s_max(p.h, p.R) * (1 if p.R is None else abs(p.R)))
    # global (area-weighted, all patches) error: a per-patch relative error is
    # ill-posed on patches where the Neumann data is nearly zero
    err = P.rel_l2(*map(np.concatenate, (sig, exs, area, trusted)))
    assert err < bar


def test_exact_neumann_matches_finite_differences():
    for gd in (I.geometry_ball_quadratic(), I.geometry_cube_sources()):
        g = wos.Geometry(gd)
        x = I.interior_points_box(10, 2, margin=0.2)
        nrm = np.random.default_rng(0).normal(size=(10, 3))
        nrm /= np.linalg.norm(nrm, axis=1)[:, None]
        fd = (g.phi(x + 1e-6 * nrm) - g.phi(x - 1e-6 * nrm)) / 2e-6
        np.testing.assert_allclose(P.exact_neumann(gd, x, nrm), fd, rtol=1e-6, atol=1e-8)


def test_propagated_se_matches_spread_over_seeds():
    p, gd = _ball_patch()
    g = wos.Geometry(gd)
    Y, _ = P.nodes_global(p)
    sig, ses = [], []
    dl = None
    for seed in range(24):
        r = wos.wos_nodes(g, Y, 1000, seed=1000 + seed)
        s = P.patch_solve(p, g, r["mean"], r["se"], dl=dl)
        dl = s["dl"]
        sig.append(s["sigma"])
        ses.append(s["se"])
    spread = np.std(np.array(sig), axis=0, ddof=1)
    prop = np.mean(np.array(ses), axis=0)
    ratio = spread / prop
    assert 0.75 < np.median(ratio) < 1.3, np.median(ratio)
    # mean z^2 over panels and seeds (panels share node values, so they are
    # correlated and the spread of this mean is wider than for iid panels)
    z2 = ((np.array(sig) - np.mean(sig, axis=0)) / prop) ** 2
    dof = z2.size - z2.shape[1]
    assert 0.7 < z2.sum() / dof < 1.4


def _point_patch(gd, x, nrm, h, layout=(8, 16, 4, 8)):
    k = int(np.argmax(np.abs(nrm)))
    t1 = np.zeros(3)
    t1[(k + 1) % 3] = 1.0
    return P.Patch(x, nrm, t1, h, *layout)


def test_central_disk_answer_matches_exact_neumann():
    """With exact node values the central-disk answer is the exact du/dn at
    the patch centre up to the collocation error and the average over the
    disk of radius h/4, both second order in h."""
    gd = I.geometry_box_holes()
    g = wos.Geometry(gd)
    rng = np.random.default_rng(3)
    pts, nrm = I.boundary_points(gd, 6, rng, edge_gap=0.1)
    for x, n in zip(pts, nrm):
        ex = P.exact_neumann(gd, x[None], n[None])[0]
        scale = np.max(np.abs(P.grad_phi(gd, x[None])))
        err = []
        for h in (0.04, 0.02):
            p = _point_patch(gd, x, n, h)
            Y, _ = P.nodes_global(p)
            v, _ = P.central_disk_answer(p, g, g.phi(Y), np.zeros(len(Y)))
            err.append(abs(v - ex) / scale)
        assert err[1] < 2e-5, err
        # second order: halving h divides the error by about 4
        assert err[1] < 1e-9 or 0.15 < err[1] / err[0] < 0.35, err


def test_central_disk_answer_se_matches_noise_spread():
    """Gaussian noise of known standard deviation on the node values: the
    spread of the answer over draws matches the propagated standard error."""
    gd = I.geometry_box_holes()
    g = wos.Geometry(gd)
    x, n = I.boundary_points(gd, 1, np.random.default_rng(5), edge_gap=0.1)
    p = _point_patch(gd, x[0], n[0], 0.05)
    Y, _ = P.nodes_global(p)
    u = g.phi(Y)
    rng = np.random.default_rng(6)
    sd = 1e-3 * (1.0 + rng.random(len(Y)))
    vals = []
    for _ in range(300):
        v, se = P.central_disk_answer(p, g, u + sd * rng.standard_normal(len(Y)), sd)
        vals.append(v)
    spread = np.std(vals, ddof=1)
    # sd of a sample sd over 300 draws is about 4 %
    assert abs(spread / se - 1.0) < 0.15, (spread, se)


def test_exterior_ball_walks_match_exact_u():
    """Walks outside the sphere of radius 3 with the truncation sphere 1e5:
    the mean is u = 1/|x| of the central charge (a walk gone to infinity
    scores 0, against u ~ 1e-5 there)."""
    gd = I.geometry_ball_exterior()
    g = wos.Geometry(gd)
    y = np.array([[0.0, 0.0, 3.5], [1.0, 2.0, 2.9], [0.0, 0.0, 10.0], [4.0, 0.0, 0.0]])
    r = wos.wos_nodes(g, y, 40_000, seed=4)
    z = (r["mean"] - 1.0 / np.linalg.norm(y, axis=1)) / r["se"]
    assert np.all(np.abs(z) < 4.5), z
    d, pr = g.dist_proj(y)
    np.testing.assert_allclose(d, np.linalg.norm(y, axis=1) - 3.0, rtol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(pr, axis=1), 3.0, rtol=1e-15)


def test_big_sphere_patch_section_5_2():
    """Sec. 5.2: the patch at (0, 0, 3) outside the sphere of radius 3 with
    the unit charge at its centre, a = 1, 1e4 walks per node: the maximal
    relative error over the panels with r < 0.7a is below the paper's 1.25 %
    and within 4 propagated standard errors of the exact 1/9."""
    p, gd = _exterior_patch()
    g = wos.Geometry(gd)
    Y, _ = P.nodes_global(p)
    r = wos.wos_nodes(g, Y, 10_000, seed=5)
    assert int(r["capped"].sum()) == 0
    res = P.patch_solve(p, g, r["mean"], r["se"])
    ex = P.exact_neumann(gd, res["x"], res["normal"])
    np.testing.assert_allclose(ex, 1.0 / 9.0, rtol=1e-14)
    tr = res["r"] < 0.7 * P.s_max(p.h, p.R) * abs(p.R)
    rel = np.abs(res["sigma"] - ex) / np.abs(ex)
    assert rel[tr].max() < 0.0125
    assert np.all(np.abs(res["sigma"][tr] - ex[tr]) < 4 * res["se"][tr] + 2e-3 * ex[tr])
