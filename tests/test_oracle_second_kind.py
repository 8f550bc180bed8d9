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
