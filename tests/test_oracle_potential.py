"""Pin for the oracle's potential (eq. bw03 with G from eq. bw05).

With the exact Neumann data at the panel centres, the tile fits and tile
quadrature must reproduce the exact harmonic u at interior targets away from
the boundary; Green's third identity makes u vanish outside the domain."""
import numpy as np

import dtn_inputs as I
from oracle import patch as P
from oracle import potential as POT
from oracle import wos


def test_potential_from_exact_neumann_reproduces_u():
    gd = I.geometry_cube_sources()
    g = wos.Geometry(gd)
    ps = P.patches_from_desc(I.patches_cube_tiles(), gd)
    sig = []
    for p in ps:
        xg, ng, _, _ = P.collocation_points(p)
        sig.append(P.exact_neumann(gd, xg, ng))
    tg = I.cube_targets(300, seed=3)
    dist = np.min(np.minimum(tg, 1 - tg), axis=1)
    far = tg[dist >= 1.0 / 8]
    u = POT.potential(ps, sig, g, far)
    ex = g.phi(far)
    assert np.max(np.abs(u - ex)) < 1e-6 * np.sqrt(np.mean(ex ** 2))
    # outside the cube the same representation gives zero
    out = np.array([[1.6, 0.5, 0.5], [0.5, -0.7, 0.2], [2.0, 2.0, 2.0]])
    assert np.max(np.abs(POT.potential(ps, sig, g, out))) < 1e-6
