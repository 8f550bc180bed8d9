"""Oracle for the second-kind local BIE (Sec. 4, eqs. bw53-bw59) on flat
patches and on patches of a sphere (inside a ball or outside one).

TEST INFRASTRUCTURE ONLY: plain numpy; only the test suite, the smoke check
and the benchmark's CPU baseline may import it.  It shares nothing with the
HIP library.

Taking the normal derivative of the representation formula (eq. bw47) at x
and letting x tend to S gives (1/2 I - D) sigma = b (eq. bw55) with
D[sigma](x) = int_S dG/dn_x sigma ds (eq. bw57) and
b(x) = - int_Gamma d2G/dn_x dn_y u ds - p.f. int_S d2G/dn_x dn_y phi ds
(eq. bw59), G = G_B the Green's function of the ball B(c, h).

On a flat patch (S in the plane through c) both x and y lie in the plane:
dG_B/dn_x vanishes there (the free-space part because x - y is in-plane,
the image part because a.n = b.n = 0), so D = 0 and sigma = 2 b, with no
linear solve.  In local coordinates (c = 0, n = e_z, Gamma on the z < 0
side), with a = y, b = x, r = |x - y|:
  on Gamma: -d2G/dn_x dn_y = dP/dn_x = 3 (h^2 - |b|^2) (a.n) / (4 pi h r^5)
            (P the Poisson kernel of the ball);
  on S:      d2G/dn_x dn_y = 1/(4 pi r^3) - 1/(4 pi Dimg^{3/2}),
            Dimg = |a|^2 |b|^2 / h^2 - 2 a.b + h^2.
At x = c these are -3 cos(theta)/(4 pi h^3) and (1/4 pi)(1/rho^3 - 1/h^3):
twice them are the kernels of the single-point estimate (eqs. bw83, bw68).

The hypersingular S integral is regularised as in Sec. 5.1 (eqs. bw63-bw68):
the constant solution u = phi(x) has zero Neumann data, so
  sigma(x) = 2 [ int_Gamma dP/dn_x (u - phi(x)) ds
                 - int_S d2G/dn_x dn_y (phi(y) - phi(x)) ds ],
and the remaining S integral excludes the disk of radius delta = delta_rel h
around x (eq. bw82's O(delta) argument: the linear part of phi(y) - phi(x)
integrates to zero over a disk centred at x).  Reading (the paper's ring
rule is for x = c only): in polar coordinates around x, Gauss in the angle
psi on [0, 2 pi], and along each ray rho from delta to the rim rho_max(psi)
the substitution rho = delta (rho_max / delta)^tau, in two pieces split at
the geometric mean, with Gauss in tau: the integrand's leading part
(grad phi . e_psi) / (4 pi rho) becomes a constant in tau, integrated
exactly, so its angle sum cancels as it does analytically.

The Gamma integral of the node values uses the same interpolant of the node
grid as the first-kind right-hand side (Lagrange in theta through the Gauss
nodes x trigonometric in phi), integrated with the graded fine rule.

On a patch of a sphere D does not vanish: (1/2 I - D) sigma = b is
collocated with piecewise constants on the panels and solved by LU (see
patch_solve_2c); the hypersingular S integral is regularised the same way,
with the rule laid out in the projection of S onto the tangent plane at the
centre.
"""
import functools

import numpy as np
from numpy.polynomial.legendre import leggauss

from . import patch as P

FOUR_PI = 4.0 * np.pi


def kernel_gamma(x, y, h):
    """dP/dn_x(x, y) for x on the flat S (local, z = 0) and y on Gamma."""
    r = np.linalg.norm(x - y, axis=-1)
    bb = np.sum(x * x, axis=-1)
    return 3.0 * (h * h - bb) * y[..., 2] / (FOUR_PI * h * r ** 5)


def kernel_s(x, y, h):
    """d2G_B/dn_x dn_y(x, y) for x, y on the flat S (local, z = 0)."""
    r = np.linalg.norm(x - y, axis=-1)
    aa = np.sum(y * y, axis=-1)
    bb = np.sum(x * x, axis=-1)
    ab = np.sum(x * y, axis=-1)
    D = aa * bb / (h * h) - 2.0 * ab + h * h
    return 1.0 / (FOUR_PI * r ** 3) - 1.0 / (FOUR_PI * D ** 1.5)


def gamma_rule(h, R, n_sub=8, m=16, n_az=512):
    """Fine rule on Gamma (graded in theta as the first-kind operator's)."""
    tm = P.theta_max(h, R)
    ths, wts = [], []
    edges = np.linspace(0.0, tm, n_sub + 1)
    for k in range(n_sub):
        xi, w = leggauss(m)
        ths.append(0.5 * (edges[k + 1] - edges[k]) * xi + 0.5 * (edges[k + 1] + edges[k]))
        wts.append(0.5 * (edges[k + 1] - edges[k]) * w)
    th, wth = np.concatenate(ths), np.concatenate(wts)
    ph = 2.0 * np.pi * np.arange(n_az) / n_az
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    Y = np.stack([h * np.sin(T) * np.cos(Ph), h * np.sin(T) * np.sin(Ph), -h * np.cos(T)], axis=-1)
    dA = (h * h) * np.sin(T) * wth[:, None] * (2.0 * np.pi / n_az)
    return th, ph, Y, dA


@functools.lru_cache(maxsize=None)
def gamma_operator_2(h, n_theta, n_phi, n_rings, n_sectors):
    """Q2[i, k] = int_Gamma dP/dn_x(x_i, y) l_k(y) ds_y at the collocation
    points x_i of a flat patch (l_k the cardinal functions of the node grid)."""
    _, X, _, _ = P.panels(h, None, n_rings, n_sectors)
    _, _, th_nodes, _ = P.node_grid(h, None, n_theta, n_phi)
    th, ph, Y, dA = gamma_rule(h, None)
    Lth = P.lagrange_basis(th_nodes, th)
    Tph = P.trig_cardinal(n_phi, ph)
    Q2 = np.empty((X.shape[0], n_theta * n_phi))
    for i in range(X.shape[0]):
        V = kernel_gamma(X[i][None, None, :], Y, h) * dA
        Q2[i] = (Lth @ V @ Tph.T).reshape(-1)
    return Q2


def s_rule(x, h, delta_rel, n_rho=20, n_psi=20):
    """Points (local, z = 0) and weights of the regularised S integral around
    x: the angle psi by Gauss on [0, 2 pi]; along each ray rho on
    [delta, rho_max(psi)], delta = delta_rel h, by rho = delta (rho_max /
    delta)^tau in two pieces (split at sqrt(delta rho_max)), n_rho Gauss
    points each in tau; weight w_psi w_tau rho^2 log(ratio) (the polar
    Jacobian rho times d rho / d tau)."""
    x = np.asarray(x, dtype=np.float64)
    xp, wp = leggauss(n_psi)
    psi, wpsi = np.pi * (xp + 1.0), np.pi * wp
    xt, wt = leggauss(n_rho)
    tau, wtau = 0.5 * (xt + 1.0), 0.5 * wt
    e = np.stack([np.cos(psi), np.sin(psi)], axis=-1)
    be = e @ x[:2]
    bb = float(x[:2] @ x[:2])
    rmax = -be + np.sqrt(be * be + h * h - bb)
    delta = delta_rel * h
    mid = np.sqrt(delta * rmax)
    rows, ws = [], []
    for lo, hi in ((np.full_like(rmax, delta), mid), (mid, rmax)):
        L = np.log(hi / lo)                                   # per ray
        rho = lo[:, None] * np.exp(L[:, None] * tau[None, :])
        rows.append(rho)
        ws.append(wpsi[:, None] * wtau[None, :] * rho * rho * L[:, None])
    rho = np.concatenate(rows, axis=1)
    W = np.concatenate(ws, axis=1)
    pts = np.zeros(rho.shape + (3,))
    pts[..., 0] = x[0] + rho * e[:, 0:1]
    pts[..., 1] = x[1] + rho * e[:, 1:2]
    return pts.reshape(-1, 3), W.reshape(-1)


def sigma_at(phi_local, u_gamma, x, h, delta_rel=1e-6, n_rho=20, n_psi=20, gamma=None):
    """sigma(x) at one local point x of a flat S from u on Gamma.

    phi_local maps local points [m][3] to the Dirichlet data; u_gamma maps
    local points [m][3] of Gamma to u there (exact values, or an
    interpolant); returns (sigma, gamma part, S part)."""
    x = np.asarray(x, dtype=np.float64)
    th, ph, Y, dA = gamma_rule(h, None) if gamma is None else gamma
    fx = phi_local(x[None, :])[0]
    uY = np.asarray(u_gamma(Y.reshape(-1, 3))).reshape(Y.shape[:-1])
    g = 2.0 * np.sum(kernel_gamma(x[None, None, :], Y, h) * (uY - fx) * dA)
    pts, W = s_rule(x, h, delta_rel, n_rho, n_psi)
    s = -2.0 * np.sum(kernel_s(x[None, :], pts, h) * (phi_local(pts) - fx) * W)
    return g + s, g, s


# ------------------------------------------------ curved patches (D != 0)
#
# On a patch of a sphere (signed radius R, local centre (0, 0, -R)) neither
# kernel vanishes: the normals n_x, n_y are the sphere's (the domain's
# outward ones) and x, y are off the tangent plane.  The kernels below are
# the derivatives of G_B = Phi - Psi, Phi = 1/(4 pi |x - y|) and
# Psi = 1/(4 pi sqrt(f)), f = |a|^2 |b|^2 / h^2 - 2 a.b + h^2 (a = y, b = x
# in local coordinates), written out for any points and unit normals:
#   dG_B/dn_x        = [ -(x - y).n_x / r^3 + (1/2) f^{-3/2} f_x.n_x ] / (4 pi)
#   d2G_B/dn_x dn_y  = [ n_x.n_y / r^3 - 3 ((x - y).n_x)((x - y).n_y) / r^5
#                        - (3/4) f^{-5/2} (f_x.n_x)(f_y.n_y)
#                        + (1/2) f^{-3/2} (4 (b.n_x)(a.n_y) / h^2 - 2 n_x.n_y) ] / (4 pi)
# with f_x = 2 |a|^2 b / h^2 - 2 a and f_y = 2 |b|^2 a / h^2 - 2 b.  On
# Gamma (n_y = a / h, the ball's outward normal) G_B = 0, so the second
# one is -dP/dn_x there, P the Poisson kernel.


def dgreen_dnx(x, nx, y, h):
    """dG_B/dn_x(x, y) for the ball B(0, h), any x, y and unit normal n_x."""
    d = x - y
    r = np.linalg.norm(d, axis=-1)
    aa = np.sum(y * y, axis=-1)
    bb = np.sum(x * x, axis=-1)
    f = aa * bb / (h * h) - 2.0 * np.sum(x * y, axis=-1) + h * h
    fx = 2.0 * (aa / (h * h))[..., None] * x - 2.0 * y
    return (-np.sum(d * nx, axis=-1) / r ** 3 + 0.5 * f ** -1.5 * np.sum(fx * nx, axis=-1)) / FOUR_PI


def d2green(x, nx, y, ny, h):
    """d2G_B/dn_x dn_y(x, y) for the ball B(0, h), any points and normals."""
    d = x - y
    r = np.linalg.norm(d, axis=-1)
    aa = np.sum(y * y, axis=-1)
    bb = np.sum(x * x, axis=-1)
    f = aa * bb / (h * h) - 2.0 * np.sum(x * y, axis=-1) + h * h
    fx = 2.0 * (aa / (h * h))[..., None] * x - 2.0 * y
    fy = 2.0 * (bb / (h * h))[..., None] * y - 2.0 * x
    dnx, dny, nn = np.sum(d * nx, axis=-1), np.sum(d * ny, axis=-1), np.sum(nx * ny, axis=-1)
    free = nn / r ** 3 - 3.0 * dnx * dny / r ** 5
    hxy = 4.0 * np.sum(x * nx, axis=-1) * np.sum(y * ny, axis=-1) / (h * h) - 2.0 * nn
    img = 0.75 * f ** -2.5 * np.sum(fx * nx, axis=-1) * np.sum(fy * ny, axis=-1) - 0.5 * f ** -1.5 * hxy
    return (free - img) / FOUR_PI


@functools.lru_cache(maxsize=None)
def gamma_operator_2c(h, R, n_theta, n_phi, n_rings, n_sectors):
    """Q2[i, k] = -int_Gamma d2G_B/dn_x dn_y(x_i, y) l_k(y) ds_y at the
    collocation points of a patch (plane or sphere), n_y = y / h on Gamma."""
    _, X, N, _ = P.panels(h, R, n_rings, n_sectors)
    _, _, th_nodes, _ = P.node_grid(h, R, n_theta, n_phi)
    th, ph, Y, dA = gamma_rule(h, R)
    Lth = P.lagrange_basis(th_nodes, th)
    Tph = P.trig_cardinal(n_phi, ph)
    NY = Y / h
    Q2 = np.empty((X.shape[0], n_theta * n_phi))
    for i in range(X.shape[0]):
        V = -d2green(X[i][None, None, :], N[i][None, None, :], Y, NY, h) * dA
        Q2[i] = (Lth @ V @ Tph.T).reshape(-1)
    return Q2


@functools.lru_cache(maxsize=None)
def adjoint_double_layer(h, R, n_rings, n_sectors, duffy_n=20, tol=1e-14):
    """D[i, j] = int_{panel j} dG_B/dn_x(x_i, y) ds_y (eq. bw57, collocation
    form); weakly singular on the own panel (Duffy), zero on a plane."""
    boxes, X, N, _ = P.panels(h, R, n_rings, n_sectors)
    Np = len(boxes)
    D = np.zeros((Np, Np))
    if R is None:
        return D
    for j in range(Np):
        others = np.array([i for i in range(Np) if i != j])

        def f_reg(S, A, _X=X[others], _N=N[others]):
            y, _, jac = P.surface(S, A, R)
            return dgreen_dnx(_X[None, :, :], _N[None, :, :], y[:, None, :], h) * jac[:, None]

        D[others, j] = P.integrate_regular(f_reg, boxes[j], tol=tol)

        def f_sing(S, A, _x=X[j], _n=N[j]):
            y, _, jac = P.surface(S, A, R)
            return dgreen_dnx(_x[None, :], _n[None, :], y, h) * jac

        D[j, j] = P.integrate_singular(f_sing, boxes[j], R, duffy_n)
    return D


def s_rule_c(x, h, R, delta_rel, n_rho=20, n_psi=20):
    """The regularised S integral's rule around a point x of a patch of the
    sphere of signed radius R (local coordinates): S is parametrised by its
    projection (X, Y) onto the tangent plane at the centre, a disk of radius
    rho_rim = r sin(s_max), r = |R|, with z = e (sqrt(r^2 - X^2 - Y^2) - r),
    e = sign(R), unit normal (e X / r, e Y / r, sqrt(r^2 - X^2 - Y^2) / r)
    and area element r / sqrt(r^2 - X^2 - Y^2) dX dY.  Around x's
    projection, the rays and the graded radial rule of s_rule, with the disk
    of radius delta = delta_rel h excluded (a region symmetric about x to
    first order, so the odd leading part of the integrand still cancels).
    Returns points [m][3], normals [m][3], weights [m]."""
    r, e = abs(R), np.sign(R)
    rim = r * np.sin(P.s_max(h, R))
    xp, wp = leggauss(n_psi)
    psi, wpsi = np.pi * (xp + 1.0), np.pi * wp
    xt, wt = leggauss(n_rho)
    tau, wtau = 0.5 * (xt + 1.0), 0.5 * wt
    ev = np.stack([np.cos(psi), np.sin(psi)], axis=-1)
    be = ev @ x[:2]
    bb = float(x[:2] @ x[:2])
    rmax = -be + np.sqrt(be * be + rim * rim - bb)
    delta = delta_rel * h
    mid = np.sqrt(delta * rmax)
    rows, ws = [], []
    for lo, hi in ((np.full_like(rmax, delta), mid), (mid, rmax)):
        L = np.log(hi / lo)
        rho = lo[:, None] * np.exp(L[:, None] * tau[None, :])
        rows.append(rho)
        ws.append(wpsi[:, None] * wtau[None, :] * rho * rho * L[:, None])
    rho = np.concatenate(rows, axis=1)
    W = np.concatenate(ws, axis=1)
    X = x[0] + rho * ev[:, 0:1]
    Y = x[1] + rho * ev[:, 1:2]
    q = np.sqrt(r * r - X * X - Y * Y)
    pts = np.stack([X, Y, e * (q - r)], axis=-1)
    nrm = np.stack([e * X / r, e * Y / r, q / r], axis=-1)
    return pts.reshape(-1, 3), nrm.reshape(-1, 3), (W * r / q).reshape(-1)


def patch_solve_2c(p, geom, u_nodes, se_nodes=None, delta_rel=1e-6, n_rho=20, n_psi=20):
    """Neumann data at the collocation points of a patch on a sphere by the
    second-kind equation (eq. bw55) collocated with piecewise constants:
      (1/2 I - D) sigma = b,
      b_i = Q2_i u - (sum_k Q2_ik) phi(x_i)
            - int_S d2G_B/dn_x dn_y (x_i, y) (phi(y) - phi(x_i)) ds_y
    (the constant solution's identity regularises the hypersingular part, as
    on a plane), solved by LU; SE(sigma) = sqrt((M^-1 Q2)^2 SE_u^2)."""
    h, R = p.h, p.R
    Q2 = gamma_operator_2c(h, R, p.n_theta, p.n_phi, p.n_rings, p.n_sectors)
    D = adjoint_double_layer(h, R, p.n_rings, p.n_sectors)
    M = 0.5 * np.eye(len(D)) - D
    xg, ng, area, rr = P.collocation_points(p)
    _, X, N, _ = P.panels(h, R, p.n_rings, p.n_sectors)
    phi_x = geom.phi(xg)
    u = np.asarray(u_nodes, dtype=np.float64)
    b = np.empty(len(X))
    for i in range(len(X)):
        pts, nrm, W = s_rule_c(X[i], h, R, delta_rel, n_rho, n_psi)
        k2 = d2green(X[i][None, :], N[i][None, :], pts, nrm, h)
        s = np.sum(k2 * (geom.phi(p.to_global(pts)) - phi_x[i]) * W)
        b[i] = Q2[i] @ u - Q2[i].sum() * phi_x[i] - s
    sig = np.linalg.solve(M, b)
    se = None
    if se_nodes is not None:
        A = np.linalg.solve(M, Q2)
        se = np.sqrt((A * A) @ (np.asarray(se_nodes, dtype=np.float64) ** 2))
    return {"sigma": sig, "se": se, "b": b, "x": xg, "normal": ng, "area": area, "r": rr}


def patch_solve_2(p, geom, u_nodes, se_nodes=None, delta_rel=1e-6, n_rho=20, n_psi=20):
    """Neumann data at the collocation points of a patch by the second-kind
    equation, from node values u_k (interpolated on Gamma as in the
    first-kind right-hand side); SE by propagation.  Flat patches: D = 0, so
    sigma = 2 b with no solve; patches on a sphere: patch_solve_2c."""
    if p.R is not None:
        return patch_solve_2c(p, geom, u_nodes, se_nodes, delta_rel, n_rho, n_psi)
    Q2 = gamma_operator_2(p.h, p.n_theta, p.n_phi, p.n_rings, p.n_sectors)
    xg, ng, area, r = P.collocation_points(p)
    boxes, X, _, _ = P.panels(p.h, None, p.n_rings, p.n_sectors)
    phi_x = geom.phi(xg)
    u = np.asarray(u_nodes, dtype=np.float64)
    sig = np.empty(len(X))
    for i in range(len(X)):
        pts, W = s_rule(X[i], p.h, delta_rel, n_rho, n_psi)
        s = np.sum(kernel_s(X[i][None, :], pts, p.h) * (geom.phi(p.to_global(pts)) - phi_x[i]) * W)
        sig[i] = 2.0 * (Q2[i] @ u - Q2[i].sum() * phi_x[i]) - 2.0 * s
    se = None
    if se_nodes is not None:
        se = np.sqrt((2.0 * Q2) ** 2 @ (np.asarray(se_nodes, dtype=np.float64) ** 2))
    return {"sigma": sig, "se": se, "x": xg, "normal": ng, "area": area, "r": r}
