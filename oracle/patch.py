"""Oracle for the local BIE step of the BIE-WOS method (test infrastructure only).

Plain FP64 numpy statement of Sec. 4 and Sec. 5.2 of Yan, Cai & Zeng:

* hemisphere nodes: Gauss-Legendre in the polar angle as in eq. bw85, with an
  equispaced (trapezoid) rule in the azimuth; the polar angle is measured from
  the inward normal, and Gamma is the part of the sphere |y - c| = h inside
  the domain (Sec. 4, definition of Gamma and Omega_S);
* the Green's function of the whole ball B(c, h) with one Kelvin image
  (Sec. 4, first paragraph), written in the symmetric form
  G_B(x,y) = (1/4pi) [ 1/|x-y| - 1/sqrt(|a|^2 |b|^2 / h^2 - 2 a.b + h^2) ],
  a = y - c, b = x - c;  P = -dG_B/dn_y on the sphere is the Poisson kernel
  (h^2 - |b|^2) / (4 pi h |x - y|^3);
* the first-kind local BIE  K sigma = b  (eqs. bw49, bw50, bw51):
  K sigma(x) = int_S G_B(x,y) sigma(y) ds_y,
  b(x) = u(x)/2 + p.v. int_S dG_B/dn_y u ds + int_Gamma dG_B/dn_y u ds;
  with P = -dG_B/dn_y on Gamma the last term is -int_Gamma P u ds;
* piecewise-constant collocation on S (Sec. 5.2): polar rings x sectors,
  collocation at the parametric panel centre, plain (adaptive) Gauss for
  regular entries, a local polar (Duffy) map with 20 x 20 Gauss on a
  physically square neighbourhood of the point for the singular entry;
* the Gamma integral from node values: the node values are interpolated
  (Lagrange in the polar angle through the Gauss nodes, trigonometric in the
  azimuth) and the interpolant is integrated against P with a fine rule
  (Sec. 5.2: values on a regular grid, interpolated to the quadrature points);
* the Neumann data sigma = du/dn with n the outward normal of the domain in
  which the walks run.

Readings of the paper taken here (the paper is silent or its figure is
lost): panels are polar rings x sectors instead of the lost triangular mesh;
on a flat S the double-layer term vanishes identically (a.n = b.n = 0), on a
sphere it is integrated directly (it is weakly singular there); the relative
error is measured over panels whose centre lies within 0.7 h of c
(Sec. 5.2, accuracy region r < 0.7a).
"""
import functools

import numpy as np
from numpy.polynomial.legendre import leggauss

FOUR_PI = 4.0 * np.pi


# ------------------------------------------------------------------ patches


class Patch:
    """A patch S of the boundary with its hemisphere.

    ``sphere`` is (C, R) when the boundary near c is the sphere |x - C| = |R|
    (then n = (c - C)/R): R > 0 when the domain is inside the sphere, R < 0
    when it is outside (the exterior of a ball, Sec. 5.2's big sphere; n then
    points to the centre); None when the boundary is the plane through c
    normal to n."""

    def __init__(self, c, n, t1, h, n_theta, n_phi, n_rings, n_sectors, sphere=None):
        self.c = np.asarray(c, dtype=np.float64)
        self.n = np.asarray(n, dtype=np.float64)
        self.t1 = np.asarray(t1, dtype=np.float64)
        self.t2 = np.cross(self.n, self.t1)
        self.h = float(h)
        self.n_theta, self.n_phi = int(n_theta), int(n_phi)
        self.n_rings, self.n_sectors = int(n_rings), int(n_sectors)
        self.R = None if sphere is None else float(sphere[1])

    def key(self):
        return (self.h, self.R, self.n_theta, self.n_phi, self.n_rings, self.n_sectors)

    def to_global(self, X):
        """Local coordinates (X along t1, Y along t2, Z along n) -> global."""
        X = np.asarray(X)
        return self.c + X[..., 0:1] * self.t1 + X[..., 1:2] * self.t2 + X[..., 2:3] * self.n

    def normal_to_global(self, N):
        N = np.asarray(N)
        return N[..., 0:1] * self.t1 + N[..., 1:2] * self.t2 + N[..., 2:3] * self.n


def patches_from_desc(desc, geom_desc):
    """Patch objects from a ``dtn_inputs`` patch description."""
    sphere = None
    if geom_desc["kind"] == "ball":
        sphere = (np.asarray(geom_desc["ball_c"], dtype=np.float64), float(geom_desc["ball_r"]))
    elif geom_desc["kind"] == "ball_exterior":
        sphere = (np.asarray(geom_desc["ball_c"], dtype=np.float64), -float(geom_desc["ball_r"]))
    out = []
    for i in range(len(desc["h"])):
        out.append(Patch(desc["c"][i], desc["n"][i], desc["t1"][i], desc["h"][i],
                         desc["n_theta"][i], desc["n_phi"][i], desc["n_rings"][i],
                         desc["n_sectors"][i], sphere))
    return out


# In local coordinates the patch centre is the origin, n = e_z, t1 = e_x and
# t2 = e_y; on a sphere of signed radius R its centre sits at (0, 0, -R)
# (below S for a domain inside the sphere, above it for one outside).


def theta_max(h, R):
    """Polar extent of Gamma, measured from the inward normal: pi/2 over a
    plane; arccos(h / 2R) over a sphere of signed radius R (the part of the
    sphere |v| = h on the domain's side: less than a hemisphere inside a
    ball, more outside one)."""
    return 0.5 * np.pi if R is None else float(np.arccos(h / (2.0 * R)))


def node_grid(h, R, n_theta, n_phi):
    """Hemisphere nodes in local coordinates and their quadrature weights.

    theta_i = theta_max (xi_i + 1)/2 with Gauss-Legendre (xi_i, w_i), as in
    eq. bw85 on [0, theta_max]; phi_j = 2 pi j / n_phi.  Node order is
    theta-major, phi-minor.  Returns (Y [n,3], weight [n], theta, phi)."""
    tm = theta_max(h, R)
    xi, w = leggauss(n_theta)
    th = 0.5 * tm * (xi + 1.0)
    wth = 0.5 * tm * w
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    Y = np.stack([h * np.sin(T) * np.cos(Ph), h * np.sin(T) * np.sin(Ph), -h * np.cos(T)], axis=-1)
    W = (h * h) * np.sin(T) * wth[:, None] * (2.0 * np.pi / n_phi)
    return Y.reshape(-1, 3), W.reshape(-1), th, ph


def nodes_global(p):
    Y, W, _, _ = node_grid(p.h, p.R, p.n_theta, p.n_phi)
    return p.to_global(Y), W


# ------------------------------------------------------------------ surface


def s_max(h, R):
    """Parametric radius of S: h over a plane; the geodesic angle
    2 arcsin(h / 2|R|) over a sphere (|y - c| = h on the rim)."""
    return h if R is None else 2.0 * np.arcsin(h / (2.0 * abs(R)))


def surface(s, a, R):
    """Point, unit normal (the domain's outward one) and area Jacobian of S at
    parameters (s, a), local coordinates.  Plane: y = s (cos a, sin a, 0),
    jac = s.  Sphere of signed radius R, r = |R|, side e = sign(R):
    y = (r sin s cos a, r sin s sin a, e r (cos s - 1)), normal
    (e sin s cos a, e sin s sin a, cos s), jac = r^2 sin s; s is the geodesic
    angle from c, so |y - C| = r with C = (0, 0, -R)."""
    s = np.asarray(s, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    if R is None:
        y = np.stack([s * np.cos(a), s * np.sin(a), np.zeros_like(s)], axis=-1)
        nrm = np.broadcast_to(np.array([0.0, 0.0, 1.0]), y.shape)
        return y, nrm, s
    r, e = abs(R), np.sign(R)
    ss, cs = np.sin(s), np.cos(s)
    y = np.stack([r * ss * np.cos(a), r * ss * np.sin(a), e * r * (cs - 1.0)], axis=-1)
    nrm = np.stack([e * ss * np.cos(a), e * ss * np.sin(a), cs], axis=-1)
    return y, nrm, r * r * ss


def panels(h, R, n_rings, n_sectors):
    """Panel parameter boxes [s0, s1, a0, a1] (ring-major, sector-minor),
    their collocation points (parametric centres, local coordinates), normals
    and areas."""
    sm = s_max(h, R)
    se = sm * np.arange(n_rings + 1) / n_rings
    ae = 2.0 * np.pi * np.arange(n_sectors + 1) / n_sectors
    boxes = np.array([[se[k], se[k + 1], ae[m], ae[m + 1]]
                      for k in range(n_rings) for m in range(n_sectors)])
    sc = 0.5 * (boxes[:, 0] + boxes[:, 1])
    ac = 0.5 * (boxes[:, 2] + boxes[:, 3])
    X, N, _ = surface(sc, ac, R)
    if R is None:
        area = 0.5 * (boxes[:, 1] ** 2 - boxes[:, 0] ** 2) * (boxes[:, 3] - boxes[:, 2])
    else:
        area = R * R * (np.cos(boxes[:, 0]) - np.cos(boxes[:, 1])) * (boxes[:, 3] - boxes[:, 2])
    return boxes, X, N, area


# ------------------------------------------------------------------ kernels


def green_ball(x, y, h):
    """G_B(x, y) for the ball B(0, h) (local coordinates, c = 0)."""
    b = x
    a = y
    r = np.linalg.norm(x - y, axis=-1)
    aa = np.sum(a * a, axis=-1)
    bb = np.sum(b * b, axis=-1)
    ab = np.sum(a * b, axis=-1)
    img = np.sqrt(aa * bb / (h * h) - 2.0 * ab + h * h)
    return (1.0 / r - 1.0 / img) / FOUR_PI


def dgreen_ball_dny(x, y, ny, h):
    """dG_B/dn_y(x, y) for the ball B(0, h): the free-space part
    (x - y).n_y / (4 pi |x - y|^3) minus the gradient of the image term,
    -(1/4pi) D^{-3/2} (a |b|^2/h^2 - b).n_y with D the image distance^2."""
    a = y
    b = x
    d = x - y
    r = np.linalg.norm(d, axis=-1)
    aa = np.sum(a * a, axis=-1)
    bb = np.sum(b * b, axis=-1)
    ab = np.sum(a * b, axis=-1)
    D = aa * bb / (h * h) - 2.0 * ab + h * h
    free = np.sum(d * ny, axis=-1) / (FOUR_PI * r ** 3)
    gimg = -(a * (bb / (h * h))[..., None] - b) / (FOUR_PI * D[..., None] ** 1.5)
    return free - np.sum(gimg * ny, axis=-1)


def poisson_ball(x, y, h):
    """P(x, y) = -dG_B/dn_y on |y| = h: (h^2 - |x|^2) / (4 pi h |x - y|^3)."""
    r = np.linalg.norm(x - y, axis=-1)
    return (h * h - np.sum(x * x, axis=-1)) / (FOUR_PI * h * r ** 3)


# --------------------------------------------------------------- quadrature


def _gl(n, lo, hi):
    xi, w = leggauss(n)
    return 0.5 * (hi - lo) * xi + 0.5 * (hi + lo), 0.5 * (hi - lo) * w


def _box_rule(box, m):
    s, ws = _gl(m, box[0], box[1])
    a, wa = _gl(m, box[2], box[3])
    S, A = np.meshgrid(s, a, indexing="ij")
    return S.ravel(), A.ravel(), np.outer(ws, wa).ravel()


def integrate_regular(f, box, m=10, tol=1e-14, depth=0, max_depth=14):
    """Adaptive tensor Gauss over a parameter box: accept when the rule on the
    box and the sum over its four quarters agree to ``tol`` (max norm over
    the components of the vector-valued integrand f(S, A) -> [n_q, k])."""
    S, A, W = _box_rule(box, m)
    whole = W @ f(S, A)
    sm, am = 0.5 * (box[0] + box[1]), 0.5 * (box[2] + box[3])
    kids = [(box[0], sm, box[2], am), (sm, box[1], box[2], am),
            (box[0], sm, am, box[3]), (sm, box[1], am, box[3])]
    parts = []
    for kb in kids:
        S, A, W = _box_rule(kb, m)
        parts.append(W @ f(S, A))
    split = sum(parts)
    if np.max(np.abs(split - whole)) <= tol or depth >= max_depth:
        return split
    return sum(integrate_regular(f, kb, m, tol, depth + 1, max_depth) for kb in kids)


def integrate_singular(f, box, R, n=20, tol=1e-14):
    """Integral of f over a panel whose collocation point (its parametric
    centre) is a singular point of f.  A sub-box around the point that is
    square in physical lengths (metric g_ss, g_aa of the surface) takes the
    Duffy rule; the rest of the panel is regular and takes the adaptive rule.
    Plane: g_ss = 1, g_aa = s^2.  Sphere of radius |R|: g_ss = R^2,
    g_aa = R^2 sin^2 s."""
    sc, ac = 0.5 * (box[0] + box[1]), 0.5 * (box[2] + box[3])
    gs = 1.0 if R is None else abs(R)
    ga = sc if R is None else abs(R) * np.sin(sc)
    w = min(0.5 * (box[1] - box[0]) * gs, 0.5 * (box[3] - box[2]) * ga)
    ds, da = w / gs, w / ga
    core = (sc - ds, sc + ds, ac - da, ac + da)
    total = integrate_duffy(f, core, (sc, ac), n)
    rest = [(box[0], core[0], box[2], box[3]), (core[1], box[1], box[2], box[3]),
            (core[0], core[1], box[2], core[2]), (core[0], core[1], core[3], box[3])]
    fv = lambda S, A: f(S, A)[:, None]
    for rb in rest:
        if rb[1] - rb[0] > 1e-15 * (1.0 + abs(rb[1])) and rb[3] - rb[2] > 1e-15 * (1.0 + abs(rb[3])):
            total = total + integrate_regular(fv, rb, tol=tol)[0]
    return total


def integrate_duffy(f, box, centre, n=20):
    """Integral of f over a parameter box whose integrand is singular at the
    parameter point ``centre``: the box is cut into four triangles with apex
    at the centre, and each is mapped to the unit square by the Duffy
    (local polar) map (u, v) -> P + u (B1 - P + v (B2 - B1)), Jacobian
    u |det(B1 - P, B2 - B1)|; n x n Gauss on each."""
    P = np.asarray(centre, dtype=np.float64)
    c = [np.array([box[0], box[2]]), np.array([box[1], box[2]]),
         np.array([box[1], box[3]]), np.array([box[0], box[3]])]
    xi, w = _gl(n, 0.0, 1.0)
    U, V = np.meshgrid(xi, xi, indexing="ij")
    WU = np.outer(w, w)
    total = 0.0
    for t in range(4):
        B1, B2 = c[t], c[(t + 1) % 4]
        e1, e2 = B1 - P, B2 - B1
        det = abs(e1[0] * e2[1] - e1[1] * e2[0])
        S = P[0] + U * (e1[0] + V * e2[0])
        A = P[1] + U * (e1[1] + V * e2[1])
        total = total + (WU * U * det).ravel() @ f(S.ravel(), A.ravel())
    return total


# ---------------------------------------------------------------- operators


@functools.lru_cache(maxsize=None)
def single_layer_matrix(h, R, n_rings, n_sectors, duffy_n=20, tol=1e-14):
    """K_ij = int_{panel j} G_B(x_i, y) ds_y (eq. bw50, collocation form)."""
    boxes, X, _, _ = panels(h, R, n_rings, n_sectors)
    Np = len(boxes)
    K = np.zeros((Np, Np))
    for j in range(Np):
        box = boxes[j]
        others = np.array([i for i in range(Np) if i != j])

        def f_reg(S, A, _X=X[others]):
            y, _, jac = surface(S, A, R)
            return green_ball(_X[None, :, :], y[:, None, :], h) * jac[:, None]

        K[others, j] = integrate_regular(f_reg, box, tol=tol)

        def f_sing(S, A, _x=X[j]):
            y, _, jac = surface(S, A, R)
            return green_ball(_x[None, :], y, h) * jac

        K[j, j] = integrate_singular(f_sing, box, R, duffy_n)
    return K


def lagrange_basis(nodes, t):
    """L[a, q] = Lagrange cardinal function a through ``nodes`` at t[q]."""
    nodes = np.asarray(nodes)
    t = np.asarray(t)
    L = np.ones((len(nodes), len(t)))
    for a in range(len(nodes)):
        for b in range(len(nodes)):
            if b != a:
                L[a] *= (t - nodes[b]) / (nodes[a] - nodes[b])
    return L


def trig_cardinal(n, phi):
    """T[b, q]: trigonometric cardinal functions of n equispaced nodes
    2 pi b / n (n even), sin(n d/2) / (n tan(d/2)) with d = phi - phi_b."""
    phi = np.asarray(phi)
    T = np.empty((n, len(phi)))
    for b in range(n):
        d = phi - 2.0 * np.pi * b / n
        s = np.sin(0.5 * d)
        with np.errstate(divide="ignore", invalid="ignore"):
            v = np.sin(0.5 * n * d) * np.cos(0.5 * d) / (n * s)
        v[np.abs(s) < 1e-300] = 1.0
        T[b] = v
    return T


@functools.lru_cache(maxsize=None)
def gamma_operator(h, R, n_theta, n_phi, n_rings, n_sectors, n_sub=8, m=16, n_az=512):
    """(Q.I)_ik = int_Gamma P(x_i, y) l_k(y) ds_y: the Poisson-kernel integral
    over Gamma of the interpolant of the node values (cardinal functions l_k
    of the node grid), with ``n_sub`` x ``m`` Gauss points in the polar angle
    and an ``n_az``-point trapezoid rule in the azimuth."""
    _, X, _, _ = panels(h, R, n_rings, n_sectors)
    tm = theta_max(h, R)
    _, _, th_nodes, _ = node_grid(h, R, n_theta, n_phi)
    ths, wts = [], []
    edges = np.linspace(0.0, tm, n_sub + 1)
    for k in range(n_sub):
        t, w = _gl(m, edges[k], edges[k + 1])
        ths.append(t)
        wts.append(w)
    th = np.concatenate(ths)
    wth = np.concatenate(wts)
    ph = 2.0 * np.pi * np.arange(n_az) / n_az
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    Y = np.stack([h * np.sin(T) * np.cos(Ph), h * np.sin(T) * np.sin(Ph), -h * np.cos(T)], axis=-1)
    dA = (h * h) * np.sin(T) * wth[:, None] * (2.0 * np.pi / n_az)
    Lth = lagrange_basis(th_nodes, th)          # [n_theta, nq_theta]
    Tph = trig_cardinal(n_phi, ph)              # [n_phi, n_az]
    Np = X.shape[0]
    QI = np.empty((Np, n_theta * n_phi))
    for i in range(Np):
        V = poisson_ball(X[i][None, None, :], Y, h) * dA   # [nq_theta, n_az]
        QI[i] = (Lth @ V @ Tph.T).reshape(-1)
    return QI


def double_layer_data(p, geom):
    """DL_i = int_S dG_B/dn_y(x_i, y) phi(y) ds_y for a patch on a sphere
    (weakly singular there, so the principal value is the plain integral);
    identically zero on a plane, where a.n = b.n = 0 for every y in S."""
    h, R = p.h, p.R
    boxes, X, _, _ = panels(h, R, p.n_rings, p.n_sectors)
    Np = len(boxes)
    if R is None:
        return np.zeros(Np)
    DL = np.zeros(Np)
    for j in range(Np):
        box = boxes[j]
        others = np.array([i for i in range(Np) if i != j])

        def f_reg(S, A, _X=X[others]):
            y, ny, jac = surface(S, A, R)
            ph = geom.phi(p.to_global(y))
            return dgreen_ball_dny(_X[None, :, :], y[:, None, :], ny[:, None, :], h) * (jac * ph)[:, None]

        DL[others] += integrate_regular(f_reg, box, tol=1e-14)

        def f_sing(S, A, _x=X[j]):
            y, ny, jac = surface(S, A, R)
            return dgreen_ball_dny(_x[None, :], y, ny, h) * jac * geom.phi(p.to_global(y))

        DL[j] += integrate_singular(f_sing, box, R)
    return DL


# -------------------------------------------------------------------- solve


def collocation_points(p):
    boxes, X, N, area = panels(p.h, p.R, p.n_rings, p.n_sectors)
    r = np.linalg.norm(X, axis=-1)
    return p.to_global(X), p.normal_to_global(N), area, r


def patch_solve(p, geom, u_nodes, se_nodes=None, dl=None):
    """Neumann data on one patch from node values (eqs. bw49-bw51).

    b = phi(x)/2 + DL - (Q.I) u ;  K sigma = b by LU with partial pivoting;
    SE(sigma) = sqrt((A*A) SE_u^2) with A = K^-1 (Q.I) (walks are independent
    across nodes).  ``dl`` may pass a DL vector computed earlier for the same
    patch and data.  Returns dict(sigma, se, b, x, normal, area, r, dl)."""
    K = single_layer_matrix(p.h, p.R, p.n_rings, p.n_sectors)
    QI = gamma_operator(p.h, p.R, p.n_theta, p.n_phi, p.n_rings, p.n_sectors)
    xg, ng, area, r = collocation_points(p)
    phi_S = geom.phi(xg)
    DL = double_layer_data(p, geom) if dl is None else np.asarray(dl, dtype=np.float64)
    b = 0.5 * phi_S + DL - QI @ np.asarray(u_nodes, dtype=np.float64)
    sigma = np.linalg.solve(K, b)
    se = None
    if se_nodes is not None:
        A = np.linalg.solve(K, QI)
        se = np.sqrt((A * A) @ (np.asarray(se_nodes, dtype=np.float64) ** 2))
    return {"sigma": sigma, "se": se, "b": b, "x": xg, "normal": ng, "area": area, "r": r, "dl": DL}


def central_disk_answer(p, geom, u_nodes, se_nodes):
    """du/dn averaged over the ring-0 panels of a plane patch (the central
    disk of radius h / n_rings, whose sectors have equal areas) and its
    standard error, propagated through the same linear map as sigma
    (Sec. 4, eqs. bw49-bw51; node errors independent)."""
    r = patch_solve(p, geom, u_nodes)
    K = single_layer_matrix(p.h, p.R, p.n_rings, p.n_sectors)
    QI = gamma_operator(p.h, p.R, p.n_theta, p.n_phi, p.n_rings, p.n_sectors)
    A = np.linalg.solve(K, QI)
    row = A[: p.n_sectors].mean(axis=0)
    value = float(r["sigma"][: p.n_sectors].mean())
    se = float(np.sqrt(np.sum(row ** 2 * np.asarray(se_nodes, dtype=np.float64) ** 2)))
    return value, se


# ----------------------------------------------------------------- exact data


def grad_phi(desc, x):
    """Gradient of the (harmonic) Dirichlet data's extension."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    if desc["data_kind"] == "quadratic":
        c = desc["quad"]
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        gx = c[1] + 2 * c[4] * X + c[7] * Y + c[9] * Z
        gy = c[2] + 2 * c[5] * Y + c[7] * X + c[8] * Z
        gz = c[3] + 2 * c[6] * Z + c[8] * Y + c[9] * X
        return np.stack([gx, gy, gz], axis=-1)
    g = np.zeros_like(x)
    for s in np.asarray(desc["src"]).reshape(-1, 4):
        d = x - s[:3]
        r = np.linalg.norm(d, axis=-1)
        g -= s[3] * d / r[:, None] ** 3
    return g


def exact_neumann(desc, x, normal):
    return np.sum(grad_phi(desc, x) * normal, axis=-1)


def rel_l2(sigma, exact, area, mask=None):
    """Area-weighted relative L2 error over the panels in ``mask``."""
    if mask is None:
        mask = np.ones_like(area, dtype=bool)
    num = np.sum(area[mask] * (sigma[mask] - exact[mask]) ** 2)
    den = np.sum(area[mask] * exact[mask] ** 2)
    return float(np.sqrt(num / den))
