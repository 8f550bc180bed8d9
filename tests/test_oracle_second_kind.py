"""Pins for the second-kind flat-patch oracle (Sec. 4, eqs. bw53-bw59).

What fixes the answers: harmonic data with known Neumann data at every point
of S (u = n.(y - c) gives 1; tangential linear and quadratic data give 0),
which pin the Gamma kernel's normalisation and the regularised S integral
off the centre; Test 1's closed form at points of S; at the centre the
reduction to the single-point estimate (Table 1's Sigma2' printed values);
the patch-level floor with exact node values; the SE propagation against the
spread over noisy draws.
"""
import os

import numpy as np
import pytest

import dtn_inputs as I
from oracle import patch as P
from oracle import point as OPt
from oracle import second_kind as SK
from oracle import wos

H = 0.5
XS = [(0.0, 0.0, 0.0), (0.1, 0.05, 0.0), (0.3, -0.2, 0.0), (0.0, 0.42, 0.0), (-0.44, 0.0, 0.0)]


@pytest.mark.parametrize("x", XS)
def test_harmonic_data_with_known_neumann(x):
    x = np.asarray(x)
    # u = n.(y - c) (local z): zero on S, du/dn = 1 everywhere on S
    s, g, t = SK.sigma_at(lambda Y: Y[:, 2], lambda Y: Y[:, 2], x, H)
    assert abs(s - 1.0) < 1e-12 and t == 0.0
    # tangential linear and quadratic data: du/dn = 0 on S
    for f in (lambda Y: Y[:, 0], lambda Y: Y[:, 1] - 2 * Y[:, 0], lambda Y: Y[:, 0] ** 2 - Y[:, 1] ** 2,
              lambda Y: Y[:, 0] * Y[:, 1]):
        s, _, _ = SK.sigma_at(f, f, x, H)
        assert abs(s) < 5e-6, s
    # z times a tangential coordinate: du/dn = x_t at the point
    s, _, _ = SK.sigma_at(lambda Y: Y[:, 2] * Y[:, 0], lambda Y: Y[:, 2] * Y[:, 0], x, H)
    assert abs(s - x[0]) < 5e-6


def test_test1_closed_form_at_points_of_s():
    gd = I.geometry_halfspace_charge()
    g = wos.Geometry(gd)
    p = P.Patch((0.5, 0, 0), (0, 0, -1.0), (1, 0, 0), H, 16, 32, 4, 16)
    phi_local = lambda Y: g.phi(p.to_global(Y))
    rng = np.random.default_rng(3)
    pts = [np.asarray(x) for x in XS] + [np.array([*v, 0.0]) for v in rng.uniform(-0.33, 0.33, (6, 2))]
    for xl in pts:
        s, _, _ = SK.sigma_at(phi_local, phi_local, xl, H)
        xg = p.to_global(xl[None])[0]
        exact = 1.0 / np.linalg.norm(xg - [0, 0, -1.0]) ** 3   # -du/dz
        assert abs(s - exact) < 1e-6 * exact, (xl, s, exact)


def test_centre_reduces_to_the_single_point_estimate():
    """At x = c the kernels are twice those of eqs. bw83 / bw68: the S part
    equals Table 1's Sigma2' column (to its printed digits)."""
    gd = I.geometry_halfspace_charge()
    g = wos.Geometry(gd)
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "table1_halfspace.txt"), comments="#")
    for a, _s1, s2, _tot, _err in rows:
        p = P.Patch((0.5, 0, 0), (0, 0, -1.0), (1, 0, 0), a, 16, 32, 4, 16)
        phi_local = lambda Y, p=p: g.phi(p.to_global(Y))
        _, _, t = SK.sigma_at(phi_local, phi_local, np.zeros(3), a)
        assert abs(t - s2) <= 5e-7, (a, t, s2)
        assert abs(t - OPt.sigma2(g.phi, (0.5, 0, 0), (0, 0, -1.0), (1, 0, 0), a, 20, 1e-6)) < 5e-7


def test_patch_floor_with_exact_node_values():
    """Cube tiles (flat): exact u at the nodes, interpolated on Gamma as in
    the first-kind right-hand side: the trusted panels' relative L2 error
    against the exact data is at the interpolation floor, like the first
    kind's."""
    gd = I.geometry_cube_sources()
    g = wos.Geometry(gd)
    pd = I.subset_patches(I.patches_cube_tiles(), I.cube_tile_subset()[:4])
    sig, exs, area, tr = [], [], [], []
    for p in P.patches_from_desc(pd, gd):
        Y, _ = P.nodes_global(p)
        r = SK.patch_solve_2(p, g, g.phi(Y))
        sig.append(r["sigma"])
        exs.append(P.exact_neumann(gd, r["x"], r["normal"]))
        area.append(r["area"])
        tr.append(r["r"] < 0.7 * p.h)
    err = P.rel_l2(*map(np.concatenate, (sig, exs, area, tr)))
    assert err < 1e-4, err


def test_propagated_se_matches_spread():
    gd = I.geometry_cube_sources()
    g = wos.Geometry(gd)
    p = P.patches_from_desc(I.subset_patches(I.patches_cube_tiles(), [100]), gd)[0]
    Y, _ = P.nodes_global(p)
    u = g.phi(Y)
    se = 1e-3 * (1.0 + 0.5 * np.sin(np.arange(len(u))))
    ref = SK.patch_solve_2(p, g, u, se)
    rng = np.random.default_rng(5)
    draws = np.array([SK.patch_solve_2(p, g, u + se * rng.standard_normal(len(u)))["sigma"] for _ in range(200)])
    spread = draws.std(axis=0, ddof=1)
    np.testing.assert_allclose(spread, ref["se"], rtol=0.15)


# ------------------------------------------------------- curved patches
# The second-kind oracle on patches of a sphere (D != 0) uses the first and
# second normal derivatives of the ball's Green's function written out for
# any points and normals.  Pins: finite differences of G_B itself (the
# first-kind oracle's function); the Gamma kernel's value -dP/dn_x there (by
# finite differences of the Poisson kernel) and its reduction to the flat
# oracle's kernel on a plane; the adjoint double layer's rows against a
# polar rule around the collocation point; exact harmonic data on the unit
# ball's pole patch and Sec. 5.2's patch outside the big sphere.


def test_curved_kernels_match_finite_differences_of_green():
    rng = np.random.default_rng(3)
    h, e = 0.7, 1e-5
    G = lambda a, b: P.green_ball(a, b, h)
    for _ in range(20):
        x, y = rng.normal(size=3) * 0.2, rng.normal(size=3) * 0.3
        nx, ny = rng.normal(size=3), rng.normal(size=3)
        nx, ny = nx / np.linalg.norm(nx), ny / np.linalg.norm(ny)
        fd1 = (G(x + e * nx, y) - G(x - e * nx, y)) / (2 * e)
        fd2 = (G(x + e * nx, y + e * ny) - G(x + e * nx, y - e * ny) - G(x - e * nx, y + e * ny)
               + G(x - e * nx, y - e * ny)) / (4 * e * e)
        d1, d2 = SK.dgreen_dnx(x, nx, y, h), SK.d2green(x, nx, y, ny, h)
        assert abs(d1 - fd1) < 1e-7 * (1 + abs(d1))
        assert abs(d2 - fd2) < 1e-4 * (1 + abs(d2))


def test_gamma_kernel_is_minus_dp_dnx_and_reduces_to_flat():
    rng = np.random.default_rng(4)
    h, e = 0.8, 1e-6
    for _ in range(10):
        x = rng.normal(size=3) * 0.2
        nx = rng.normal(size=3)
        nx /= np.linalg.norm(nx)
        v = rng.normal(size=3)
        y = h * v / np.linalg.norm(v)
        fd = (P.poisson_ball(x + e * nx, y, h) - P.poisson_ball(x - e * nx, y, h)) / (2 * e)
        assert abs(SK.d2green(x, nx, y, y / h, h) + fd) < 1e-6 * (1 + abs(fd))
    a = SK.gamma_operator_2c(1.0, None, 8, 16, 4, 8)
    b = SK.gamma_operator_2(1.0, 8, 16, 4, 8)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("R", [5.0, -3.0])
def test_adjoint_double_layer_rows_against_a_polar_rule(R):
    """Sum over panels of D[i, j] = int_S dG_B/dn_x(x_i, y) ds_y, integrated
    independently by the polar rule around x_i (weak singularity 1/rho)."""
    h = 1.0
    D = SK.adjoint_double_layer(h, R, 4, 8)
    _, X, N, _ = P.panels(h, R, 4, 8)
    assert np.max(np.abs(D)) > 1e-3
    # plain polar Gauss around x_i's projection onto the tangent plane at the
    # centre (rho from 0: rho times the 1/rho kernel is smooth), lifted to
    # the sphere with the area element r / sqrt(r^2 - X^2 - Y^2)
    r, e = abs(R), np.sign(R)
    rim = r * np.sin(P.s_max(h, R))
    xp, wp = np.polynomial.legendre.leggauss(64)
    xr, wr = np.polynomial.legendre.leggauss(48)
    psi, wpsi = np.pi * (xp + 1.0), np.pi * wp
    for i in (0, 5, 17, 31):
        x = X[i]
        ev = np.stack([np.cos(psi), np.sin(psi)], axis=-1)
        be = ev @ x[:2]
        rmax = -be + np.sqrt(be * be + rim * rim - x[:2] @ x[:2])
        rho = 0.5 * rmax[:, None] * (xr[None, :] + 1.0)
        w = wpsi[:, None] * 0.5 * rmax[:, None] * wr[None, :] * rho
        PX, PY = x[0] + rho * ev[:, 0:1], x[1] + rho * ev[:, 1:2]
        q = np.sqrt(r * r - PX * PX - PY * PY)
        y = np.stack([PX, PY, e * (q - r)], axis=-1).reshape(-1, 3)
        ref = np.sum((w * r / q).reshape(-1) * SK.dgreen_dnx(x[None, :], N[i][None, :], y, h))
        assert abs(D[i].sum() - ref) < 1e-10 * abs(ref) + 1e-12, (i, D[i].sum(), ref)
    assert np.all(SK.adjoint_double_layer(h, None, 4, 8) == 0.0)


def test_curved_second_kind_with_exact_node_values():
    """The unit ball's pole patch (u = x^2 - y^2 + z, du/dn = 2x^2 - 2y^2 + z)
    and Sec. 5.2's patch outside the big sphere (u = 1/|x|, du/dn = 1/R^2):
    with exact node values the second kind is at its discretisation floor,
    below the first kind's on the ball; constant data gives zero."""
    for gd, pd, bar in ((I.geometry_ball_quadratic(), I.patches_ball_pole(), 5e-5),
                        (I.geometry_ball_exterior(), I.patches_big_sphere(), 1e-9)):
        p = P.patches_from_desc(pd, gd)[0]
        og = wos.Geometry(gd)
        X, _ = P.nodes_global(p)
        r = SK.patch_solve_2(p, og, og.phi(X))
        ex = P.exact_neumann(gd, r["x"], r["normal"])
        tr = r["r"] < 0.7 * p.h
        err = P.rel_l2(r["sigma"], ex, r["area"], tr)
        assert err < bar, err
        if bar > 1e-8:
            assert err < 0.2 * P.rel_l2(P.patch_solve(p, og, og.phi(X))["sigma"], ex, r["area"], tr)
    one = dict(I.geometry_ball_quadratic(), quad=[1.0] + [0.0] * 9)
    og = wos.Geometry(one)
    p = P.patches_from_desc(I.patches_ball_pole(), one)[0]
    r = SK.patch_solve_2(p, og, np.ones(p.n_theta * p.n_phi))
    assert np.max(np.abs(r["sigma"])) < 1e-9
