"""Oracle for the final potential (test infrastructure only).

Eq. bw03 of Yan, Cai & Zeng: for x off the boundary,
  u(x) = int_dOmega G(x,y) du/dn_y ds_y - int_dOmega dG/dn_y(x,y) u(y) ds_y,
  G = 1 / (4 pi |x - y|)  (eq. bw05),
with the Neumann data from the patch solves and the Dirichlet data given.

Reading taken (the paper only says the integral is evaluated, e.g. by FMM):
the boundary is covered by square tiles, each with its patch S (the inscribed
disk of radius h); on each tile the Neumann data is the least-squares
quadratic in the tile's tangent coordinates through the panel values whose
centres lie within 0.7 h of the centre (the accuracy region of Sec. 5.2),
and the tile integral is a 4 x 4 Gauss-Legendre product rule.  The sum over
all tiles is evaluated directly.
"""
import numpy as np
from numpy.polynomial.legendre import leggauss

from . import patch as P


def tile_quadrature(p, sigma, geom, trusted=0.7, n_gl=4):
    """Quadrature points, outward normals, weights, Neumann and Dirichlet
    values on the square tile [-h, h]^2 (tangent frame t1, t2) of patch p."""
    xg, _, _, r = P.collocation_points(p)
    loc = np.stack([(xg - p.c) @ p.t1, (xg - p.c) @ p.t2], axis=-1) / p.h
    m = r < trusted * p.h
    X, Y = loc[m, 0], loc[m, 1]
    A = np.stack([np.ones_like(X), X, Y, X * X, X * Y, Y * Y], axis=-1)
    coef, *_ = np.linalg.lstsq(A, np.asarray(sigma)[m], rcond=None)
    xi, w = leggauss(n_gl)
    Xq, Yq = np.meshgrid(xi, xi, indexing="ij")
    Xq, Yq = Xq.ravel(), Yq.ravel()
    Wq = (np.outer(w, w).ravel()) * p.h * p.h
    Aq = np.stack([np.ones_like(Xq), Xq, Yq, Xq * Xq, Xq * Yq, Yq * Yq], axis=-1)
    sig_q = Aq @ coef
    yq = p.c + p.h * (Xq[:, None] * p.t1 + Yq[:, None] * p.t2)
    nq = np.broadcast_to(p.n, yq.shape)
    return yq, nq, Wq, sig_q, geom.phi(yq)


def potential(patches, sigmas, geom, targets):
    """u at ``targets`` [m,3] from the tiles' Neumann data (eq. bw03)."""
    ys, ns, ws, ss, fs = [], [], [], [], []
    for p, s in zip(patches, sigmas):
        y, n, w, sq, fq = tile_quadrature(p, s, geom)
        ys.append(y), ns.append(n), ws.append(w), ss.append(sq), fs.append(fq)
    y = np.concatenate(ys)
    n = np.concatenate(ns)
    w = np.concatenate(ws)
    s = np.concatenate(ss)
    f = np.concatenate(fs)
    targets = np.asarray(targets, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(targets))
    for i, x in enumerate(targets):
        d = x - y
        r = np.linalg.norm(d, axis=-1)
        G = 1.0 / (4.0 * np.pi * r)
        dG = np.sum(d * n, axis=-1) / (4.0 * np.pi * r ** 3)
        out[i] = np.sum(w * (G * s - dG * f))
    return out
