// Host construction of the per-class collocation operators of step 2
// (Sec. 4, eqs. bw49-bw51; Sec. 5.2).  Everything is built once per class of
// congruent patches, in local coordinates scaled by 1/h (patch centre at the
// origin, n = e_z, t1 = e_x, t2 = e_y; a curved patch lies on the sphere of
// radius rr = R/h centred at (0, 0, -rr)), and uploaded to the device.
//
//   K_ij    = int_{panel j} G_B(x_i, y) ds_y  with the whole-ball Green's
//             function of B(0,1), one Kelvin image (Sec. 4):
//             G_B = (1/4pi) [1/|x-y| - 1/sqrt(|a|^2 |b|^2 - 2 a.b + 1)]
//   (Q.I)_ik= int_Gamma P(x_i, y) l_k(y) ds_y,  P = (1 - |x|^2)/(4pi |x-y|^3)
//             the Poisson kernel of B(0,1) and l_k the cardinal functions of
//             the node grid (Lagrange in theta x trigonometric in phi): the
//             Gamma integral of the interpolated node values (Sec. 5.2)
//   DL rows   quadrature points and weights of int_S dG_B/dn_y phi ds on a
//             sphere (the double-layer term of b, weakly singular there)
//   LU, A2    LU factors of K (partial pivoting), and (K^-1 Q.I)^2 for the
//             propagation of the node standard errors
//   ans_row   mean over the ring-0 panels of the rows of K^-1 Q.I (standard
//             error of the central-disk mean of sigma)
//   fit       tile fit used by the potential (least-squares quadratic through
//             the panels within 0.7 of the centre, at 4x4 Gauss points)
//
// Quadrature: adaptive 8x8 Gauss-Legendre on parameter boxes for regular
// panel integrals; for the singular (own) panel a Duffy map on a
// neighbourhood of the collocation point that is square in arc length, with
// 24x24 Gauss on each of its four triangles, and the adaptive rule on the
// rest of the panel; for Gamma, Gauss-Legendre on polar sub-intervals graded
// towards the rim (where the Poisson kernel of outer collocation points
// peaks) times a 768-point trapezoid rule in the azimuth.
#include <algorithm>
#include <array>
#include <cmath>
#include <functional>
#include <string>
#include <vector>

#include "dtn_internal.h"

namespace dtn {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kInv4Pi = 1.0 / (4.0 * kPi);

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on the
// three-term recurrence of the Legendre polynomials.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) {
                p1 = z;
                p0 = 1.0;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

struct GL {
    std::vector<double> x, w;
    explicit GL(int n) { gauss_legendre(n, x, w); }
};

struct V3 {
    double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

// Surface of S at parameters (s, a): plane (rr = 0) or sphere of signed
// radius rr (rr > 0: the domain inside the sphere, centre (0, 0, -rr);
// rr < 0: outside it, centre (0, 0, |rr|)).  On the sphere s is the
// geodesic angle from the patch centre, so every rule stays positively
// oriented; n is the domain's outward normal (towards the centre outside).
struct Surf {
    double rr;
    double r() const { return std::fabs(rr); }
    double side() const { return rr < 0.0 ? -1.0 : 1.0; }
    double smax() const { return rr == 0.0 ? 1.0 : 2.0 * std::asin(0.5 / r()); }
    void at(double s, double a, V3 &y, V3 &n, double &jac) const
    {
        const double ca = std::cos(a), sa = std::sin(a);
        if (rr == 0.0) {
            y = {s * ca, s * sa, 0.0};
            n = {0.0, 0.0, 1.0};
            jac = s;
        } else {
            const double ss = std::sin(s), cs = std::cos(s), e = side(), R = r();
            n = {e * ss * ca, e * ss * sa, cs};
            y = {R * ss * ca, R * ss * sa, e * R * (cs - 1.0)};
            jac = R * R * ss;
        }
    }
    // arc-length metric factors along s and a at parameter s
    double gs() const { return rr == 0.0 ? 1.0 : r(); }
    double ga(double s) const { return rr == 0.0 ? s : r() * std::sin(s); }
};

inline double green_ball(V3 x, V3 y)
{
    const double r = norm(sub(x, y));
    const double img = std::sqrt(dot(y, y) * dot(x, x) - 2.0 * dot(y, x) + 1.0);
    return (1.0 / r - 1.0 / img) * kInv4Pi;
}

// dG_B/dn_y for B(0,1): free-space part minus the image term's gradient.
inline double dgreen_ball_dny(V3 x, V3 y, V3 ny)
{
    const V3 d = sub(x, y);
    const double r = norm(d);
    const double bb = dot(x, x);
    const double D = dot(y, y) * bb - 2.0 * dot(y, x) + 1.0;
    const double free = dot(d, ny) / (r * r * r);
    const V3 gi = {y.x * bb - x.x, y.y * bb - x.y, y.z * bb - x.z};
    const double img = -dot(gi, ny) / (D * std::sqrt(D));
    return (free - img) * kInv4Pi;
}

inline double poisson_ball(V3 x, V3 y)
{
    const double r = norm(sub(x, y));
    return (1.0 - dot(x, x)) * kInv4Pi / (r * r * r);
}

struct Box {
    double s0, s1, a0, a1;
};

// A quadrature leaf: parameter point and weight (includes the box Jacobian
// but not the surface Jacobian).
struct Leaf {
    double s, a, w;
};

const GL &gl8()
{
    static const GL g(8);
    return g;
}

void box_rule(const Box &b, const GL &g, std::vector<Leaf> &out)
{
    const double hs = 0.5 * (b.s1 - b.s0), ms = 0.5 * (b.s1 + b.s0);
    const double ha = 0.5 * (b.a1 - b.a0), ma = 0.5 * (b.a1 + b.a0);
    for (size_t i = 0; i < g.x.size(); ++i)
        for (size_t j = 0; j < g.x.size(); ++j)
            out.push_back({ms + hs * g.x[i], ma + ha * g.x[j], hs * ha * g.w[i] * g.w[j]});
}

// Adaptive leaves for a vector integrand f(s, a, out[k]): a box is accepted
// when its rule and the sum of its quarters' rules agree to tol in every
// component.
void adapt_leaves(const Box &b, int k, const std::function<void(double, double, double *)> &f, double tol,
                  int depth, std::vector<Leaf> &leaves)
{
    const GL &g = gl8();
    std::vector<Leaf> whole, split;
    box_rule(b, g, whole);
    const double sm = 0.5 * (b.s0 + b.s1), am = 0.5 * (b.a0 + b.a1);
    const Box kids[4] = {{b.s0, sm, b.a0, am}, {sm, b.s1, b.a0, am}, {b.s0, sm, am, b.a1}, {sm, b.s1, am, b.a1}};
    for (const Box &kb : kids) box_rule(kb, g, split);
    std::vector<double> I1(k, 0.0), I2(k, 0.0), v(k);
    for (const Leaf &l : whole) {
        f(l.s, l.a, v.data());
        for (int c = 0; c < k; ++c) I1[c] += l.w * v[c];
    }
    for (const Leaf &l : split) {
        f(l.s, l.a, v.data());
        for (int c = 0; c < k; ++c) I2[c] += l.w * v[c];
    }
    double err = 0.0;
    for (int c = 0; c < k; ++c) err = std::max(err, std::fabs(I2[c] - I1[c]));
    if (err <= tol || depth >= 16) {
        leaves.insert(leaves.end(), split.begin(), split.end());
        return;
    }
    for (const Box &kb : kids) adapt_leaves(kb, k, f, tol, depth + 1, leaves);
}

// Duffy leaves for a box singular at its centre: four triangles with apex at
// the centre, each mapped from the unit square by (u, v) -> P + u (B1 - P +
// v (B2 - B1)) with Jacobian u |det|.
void duffy_leaves(const Box &b, int n, std::vector<Leaf> &leaves)
{
    static thread_local int cached_n = -1;
    static thread_local GL *g = nullptr;
    if (cached_n != n) {
        delete g;
        g = new GL(n);
        cached_n = n;
    }
    const double ps = 0.5 * (b.s0 + b.s1), pa = 0.5 * (b.a0 + b.a1);
    const double cs[4] = {b.s0, b.s1, b.s1, b.s0};
    const double ca[4] = {b.a0, b.a0, b.a1, b.a1};
    for (int t = 0; t < 4; ++t) {
        const double e1s = cs[t] - ps, e1a = ca[t] - pa;
        const double e2s = cs[(t + 1) % 4] - cs[t], e2a = ca[(t + 1) % 4] - ca[t];
        const double det = std::fabs(e1s * e2a - e1a * e2s);
        for (int i = 0; i < n; ++i) {
            const double u = 0.5 * (g->x[i] + 1.0), wu = 0.5 * g->w[i];
            for (int j = 0; j < n; ++j) {
                const double v = 0.5 * (g->x[j] + 1.0), wv = 0.5 * g->w[j];
                leaves.push_back({ps + u * (e1s + v * e2s), pa + u * (e1a + v * e2a), wu * wv * u * det});
            }
        }
    }
}

// Leaves for a panel whose centre is a singular point of the integrand: Duffy
// on a neighbourhood of the centre that is square in arc length, adaptive on
// the rest (driven by the scalar integrand f).
void singular_leaves(const Box &b, const Surf &surf, const std::function<void(double, double, double *)> &f,
                     std::vector<Leaf> &leaves)
{
    const double sc = 0.5 * (b.s0 + b.s1), ac = 0.5 * (b.a0 + b.a1);
    const double gs = surf.gs(), ga = surf.ga(sc);
    const double half = std::min(0.5 * (b.s1 - b.s0) * gs, 0.5 * (b.a1 - b.a0) * ga);
    const double ds = half / gs, da = half / ga;
    const Box core{sc - ds, sc + ds, ac - da, ac + da};
    duffy_leaves(core, 24, leaves);
    const Box rest[4] = {{b.s0, core.s0, b.a0, b.a1},
                         {core.s1, b.s1, b.a0, b.a1},
                         {core.s0, core.s1, b.a0, core.a0},
                         {core.s0, core.s1, core.a1, b.a1}};
    for (const Box &r : rest) {
        if (r.s1 - r.s0 <= 1e-15 * (1.0 + std::fabs(r.s1)) || r.a1 - r.a0 <= 1e-15 * (1.0 + std::fabs(r.a1)))
            continue;
        adapt_leaves(r, 1, f, 1e-14, 0, leaves);
    }
}

// LU with partial pivoting, row-major, in place; piv[k] = row swapped into k.
bool lu_factor(int n, std::vector<double> &A, std::vector<int32_t> &piv)
{
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i * n + k]) > best) {
                best = std::fabs(A[i * n + k]);
                p = i;
            }
        if (best == 0.0) return false;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
        for (int i = k + 1; i < n; ++i) {
            const double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return true;
}

void lu_solve(int n, const std::vector<double> &LU, const std::vector<int32_t> &piv, double *b)
{
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
        b[i] /= LU[i * n + i];
    }
}

}  // namespace

// ---- second-kind equation on a flat patch (eqs. bw53-bw59), at h = 1.
// With S in the plane through the ball's centre, dG_B/dn_x vanishes for x, y
// on S (D = 0), so sigma = 2b.  The Gamma kernel is dP/dn_x =
// 3 (1 - |x|^2) y.n / (4 pi r^5); the S kernel d2G_B/dn_x dn_y =
// 1/(4 pi r^3) - 1/(4 pi Dimg^{3/2}), Dimg = |x|^2 |y|^2 - 2 x.y + 1.  The
// hypersingular S integral is regularised by the constant solution (as in
// Sec. 5.1, eqs. bw63-bw68) and taken outside the disk of radius
// kSecondKindDelta around x: Gauss in the angle, and along each ray a
// logarithmic substitution rho = lo (hi / lo)^tau in two pieces (split at
// the geometric mean of delta and the rim distance), Gauss in tau, so that
// the 1/rho part of the integrand is integrated exactly and its angle sum
// cancels.
constexpr double kSecondKindDelta = 1e-6;
constexpr int kSecondKindRule = 20;  // Gauss points in the angle and per piece along a ray

inline double dpoisson_dnx(V3 x, V3 y)
{
    const double r = norm(sub(x, y));
    return 3.0 * (1.0 - dot(x, x)) * y.z / (4.0 * kPi * r * r * r * r * r);
}

inline double ddgreen_s(V3 x, V3 y)
{
    const double r = norm(sub(x, y));
    const double D = dot(x, x) * dot(y, y) - 2.0 * dot(x, y) + 1.0;
    return 1.0 / (4.0 * kPi * r * r * r) - 1.0 / (4.0 * kPi * D * std::sqrt(D));
}

// ---- second-kind equation on a patch of a sphere (signed radius rr at
// h = 1, centre C = (0, 0, -rr), outward normal (x - C) / rr): D != 0, so
// (1/2 I - D) sigma = b is solved by LU.  The kernels are the derivatives of
// G_B = 1/(4 pi r) - 1/(4 pi sqrt(f)), f = |x|^2 |y|^2 - 2 x.y + 1, for any
// points and unit normals (on Gamma, n_y = y):
//   dG_B/dn_x       = [-(x - y).n_x / r^3 + f^{-3/2} (|y|^2 x - y).n_x] / (4 pi)
//   d2G_B/dn_x dn_y = [n_x.n_y / r^3 - 3 ((x - y).n_x)((x - y).n_y) / r^5
//                      - 3 f^{-5/2} ((|y|^2 x - y).n_x)((|x|^2 y - x).n_y)
//                      + f^{-3/2} (2 (x.n_x)(y.n_y) - n_x.n_y)] / (4 pi)
inline double dgreen_dnx(V3 x, V3 nx, V3 y)
{
    const V3 d = sub(x, y);
    const double r = norm(d), aa = dot(y, y);
    const double f = aa * dot(x, x) - 2.0 * dot(x, y) + 1.0;
    const V3 gx{aa * x.x - y.x, aa * x.y - y.y, aa * x.z - y.z};
    return (-dot(d, nx) / (r * r * r) + dot(gx, nx) / (f * std::sqrt(f))) * kInv4Pi;
}

inline double ddgreen(V3 x, V3 nx, V3 y, V3 ny)
{
    const V3 d = sub(x, y);
    const double r = norm(d), r2 = r * r, aa = dot(y, y), bb = dot(x, x);
    const double f = aa * bb - 2.0 * dot(x, y) + 1.0, sf = std::sqrt(f);
    const V3 gx{aa * x.x - y.x, aa * x.y - y.y, aa * x.z - y.z};
    const V3 gy{bb * y.x - x.x, bb * y.y - x.y, bb * y.z - x.z};
    const double nn = dot(nx, ny);
    const double fr = nn / (r2 * r) - 3.0 * dot(d, nx) * dot(d, ny) / (r2 * r2 * r);
    const double img = 3.0 * dot(gx, nx) * dot(gy, ny) / (f * f * sf) - (2.0 * dot(x, nx) * dot(y, ny) - nn) / (f * sf);
    return (fr - img) * kInv4Pi;
}

// Tables of the curved second kind: Q2 (Gamma kernel -d2G_B/dn_x dn_y against
// the node interpolant), the regularised S rule around each collocation
// point, c2, M = 1/2 I - D with its LU factors, and (M^-1 Q2)^2 for the SE.
// The S rule parametrises S by its projection (X, Y) onto the tangent plane
// at the centre, a disk of radius r sin(s_max) (z = e (sqrt(r^2 - X^2 - Y^2)
// - r), normal (e X, e Y, sqrt(r^2 - X^2 - Y^2)) / r, area element
// r / sqrt(r^2 - X^2 - Y^2)), with the flat rule's rays and radial grading
// around x's projection and the disk of radius kSecondKindDelta excluded.
template <class Rows>
void second_kind_tables_curved(ClassOps &ops, const std::vector<V3> &X, const std::vector<V3> &N,
                               const std::vector<Box> &boxes, const Surf &surf, Rows &gamma_rows)
{
    const int Np = ops.n_rings * ops.n_sectors, Nn = ops.n_theta * ops.n_phi;
    const double rr = ops.rr, r = surf.r(), e = surf.side();
    gamma_rows(
        [rr](V3 x, V3 y) {
            const V3 nx{x.x / rr, x.y / rr, (x.z + rr) / rr};
            return -ddgreen(x, nx, y, y);
        },
        ops.Q2);
    // D (eq. bw57, collocation form): weakly singular on the own panel
    std::vector<double> D((size_t)Np * Np, 0.0);
    for (int j = 0; j < Np; ++j)
        for (int i = 0; i < Np; ++i) {
            auto f = [&](double s, double a, double *out) {
                V3 y, n;
                double jac;
                surf.at(s, a, y, n, jac);
                out[0] = dgreen_dnx(X[i], N[i], y) * jac;
            };
            std::vector<Leaf> lv;
            if (i == j)
                singular_leaves(boxes[j], surf, f, lv);
            else
                adapt_leaves(boxes[j], 1, f, 1e-14, 0, lv);
            double acc = 0.0;
            for (const Leaf &l : lv) {
                double v;
                f(l.s, l.a, &v);
                acc += l.w * v;
            }
            D[(size_t)i * Np + j] = acc;
        }
    ops.M2 = D;
    for (double &v : ops.M2) v = -v;
    for (int i = 0; i < Np; ++i) ops.M2[(size_t)i * Np + i] += 0.5;
    ops.M2_LU = ops.M2;
    // S rule
    const int n = kSecondKindRule;
    std::vector<double> gx, gw;
    gauss_legendre(n, gx, gw);
    ops.n_s = 2 * n * n;
    ops.s_pts.assign((size_t)Np * ops.n_s * 3, 0.0);
    ops.s_w.assign((size_t)Np * ops.n_s, 0.0);
    ops.c2.assign(Np, 0.0);
    const double rim = r * std::sin(surf.smax());
    for (int i = 0; i < Np; ++i) {
        const V3 x = X[i];
        double wsum = 0.0;
        int q = 0;
        for (int l = 0; l < n; ++l) {
            const double psi = kPi * (gx[l] + 1.0), wpsi = kPi * gw[l];
            const double ex = std::cos(psi), ey = std::sin(psi);
            const double be = ex * x.x + ey * x.y, bb = x.x * x.x + x.y * x.y;
            const double rmax = -be + std::sqrt(be * be + rim * rim - bb);
            const double lo0 = kSecondKindDelta, mid = std::sqrt(kSecondKindDelta * rmax);
            const double los[2] = {lo0, mid}, his[2] = {mid, rmax};
            for (int piece = 0; piece < 2; ++piece) {
                const double L = std::log(his[piece] / los[piece]);
                for (int k = 0; k < n; ++k, ++q) {
                    const double tau = 0.5 * (gx[k] + 1.0), wtau = 0.5 * gw[k];
                    const double rho = los[piece] * std::exp(L * tau);
                    const double px = x.x + rho * ex, py = x.y + rho * ey;
                    const double qz = std::sqrt(r * r - px * px - py * py);
                    const V3 y{px, py, e * (qz - r)};
                    const V3 ny{e * px / r, e * py / r, qz / r};
                    const double w = wpsi * wtau * rho * rho * L * (r / qz) * ddgreen(x, N[i], y, ny);
                    double *o = &ops.s_pts[((size_t)i * ops.n_s + q) * 3];
                    o[0] = y.x;
                    o[1] = y.y;
                    o[2] = y.z;
                    ops.s_w[(size_t)i * ops.n_s + q] = w;
                    wsum += w;
                }
            }
        }
        double qsum = 0.0;
        for (int k = 0; k < Nn; ++k) qsum += ops.Q2[(size_t)i * Nn + k];
        ops.c2[i] = qsum - wsum;
    }
}

template <class Rows>
void second_kind_tables(ClassOps &ops, const std::vector<V3> &X, Rows &gamma_rows)
{
    const int Np = ops.n_rings * ops.n_sectors, Nn = ops.n_theta * ops.n_phi;
    gamma_rows([](V3 x, V3 y) { return dpoisson_dnx(x, y); }, ops.Q2);
    const int n = kSecondKindRule;
    std::vector<double> gx, gw;
    gauss_legendre(n, gx, gw);
    ops.n_s = 2 * n * n;
    ops.s_pts.assign((size_t)Np * ops.n_s * 3, 0.0);
    ops.s_w.assign((size_t)Np * ops.n_s, 0.0);
    ops.c2.assign(Np, 0.0);
    for (int i = 0; i < Np; ++i) {
        const V3 x = X[i];
        double wsum = 0.0;
        int q = 0;
        for (int l = 0; l < n; ++l) {
            const double psi = kPi * (gx[l] + 1.0), wpsi = kPi * gw[l];
            const double ex = std::cos(psi), ey = std::sin(psi);
            const double be = ex * x.x + ey * x.y, bb = x.x * x.x + x.y * x.y;
            const double rmax = -be + std::sqrt(be * be + 1.0 - bb);
            const double lo0 = kSecondKindDelta, mid = std::sqrt(kSecondKindDelta * rmax);
            const double los[2] = {lo0, mid}, his[2] = {mid, rmax};
            for (int piece = 0; piece < 2; ++piece) {
                const double L = std::log(his[piece] / los[piece]);
                for (int k = 0; k < n; ++k, ++q) {
                    const double tau = 0.5 * (gx[k] + 1.0), wtau = 0.5 * gw[k];
                    const double rho = los[piece] * std::exp(L * tau);
                    const V3 y{x.x + rho * ex, x.y + rho * ey, 0.0};
                    const double w = wpsi * wtau * rho * rho * L * ddgreen_s(x, y);
                    double *o = &ops.s_pts[((size_t)i * ops.n_s + q) * 3];
                    o[0] = y.x;
                    o[1] = y.y;
                    o[2] = 0.0;
                    ops.s_w[(size_t)i * ops.n_s + q] = w;
                    wsum += w;
                }
            }
        }
        double qsum = 0.0;
        for (int k = 0; k < Nn; ++k) qsum += ops.Q2[(size_t)i * Nn + k];
        ops.c2[i] = qsum - wsum;
    }
}

bool build_class_ops(ClassOps &ops, std::string &err)
{
    const int Nt = ops.n_theta, Nf = ops.n_phi, Nr = ops.n_rings, Ns = ops.n_sectors;
    const int Nn = Nt * Nf, Np = Nr * Ns;
    const Surf surf{ops.rr};
    const double tmax = ops.rr == 0.0 ? 0.5 * kPi : std::acos(0.5 / ops.rr);

    // ---- node grid: Gauss-Legendre in theta on [0, theta_max], equispaced phi
    std::vector<double> xi, wi;
    gauss_legendre(Nt, xi, wi);
    std::vector<double> th(Nt);
    for (int a = 0; a < Nt; ++a) th[a] = 0.5 * tmax * (xi[a] + 1.0);
    ops.node_tab.resize(3 * Nn);
    for (int a = 0; a < Nt; ++a)
        for (int b = 0; b < Nf; ++b) {
            const double ph = 2.0 * kPi * b / Nf;
            double* o = &ops.node_tab[3 * (a * Nf + b)];
            o[0] = std::sin(th[a]) * std::cos(ph);
            o[1] = std::sin(th[a]) * std::sin(ph);
            o[2] = -std::cos(th[a]);
        }

    // ---- panels and collocation points
    const double smax = surf.smax();
    std::vector<Box> boxes(Np);
    std::vector<V3> X(Np);
    ops.col_tab.resize(3 * Np);
    for (int k = 0; k < Nr; ++k)
        for (int m = 0; m < Ns; ++m) {
            Box b{smax * k / Nr, smax * (k + 1) / Nr, 2.0 * kPi * m / Ns, 2.0 * kPi * (m + 1) / Ns};
            boxes[k * Ns + m] = b;
            V3 y, n;
            double jac;
            surf.at(0.5 * (b.s0 + b.s1), 0.5 * (b.a0 + b.a1), y, n, jac);
            X[k * Ns + m] = y;
            ops.col_tab[3 * (k * Ns + m)] = y.x;
            ops.col_tab[3 * (k * Ns + m) + 1] = y.y;
            ops.col_tab[3 * (k * Ns + m) + 2] = y.z;
        }

    // ---- single-layer matrix K (eq. bw50)
    ops.K.assign((size_t)Np * Np, 0.0);
    for (int j = 0; j < Np; ++j) {
        std::vector<int> others;
        for (int i = 0; i < Np; ++i)
            if (i != j) others.push_back(i);
        const int k = (int)others.size();
        auto f = [&](double s, double a, double *out) {
            V3 y, n;
            double jac;
            surf.at(s, a, y, n, jac);
            for (int c = 0; c < k; ++c) out[c] = green_ball(X[others[c]], y) * jac;
        };
        std::vector<Leaf> leaves;
        adapt_leaves(boxes[j], k, f, 1e-14, 0, leaves);
        std::vector<double> v(k);
        for (const Leaf &l : leaves) {
            f(l.s, l.a, v.data());
            for (int c = 0; c < k; ++c) ops.K[(size_t)others[c] * Np + j] += l.w * v[c];
        }
        auto fs = [&](double s, double a, double *out) {
            V3 y, n;
            double jac;
            surf.at(s, a, y, n, jac);
            out[0] = green_ball(X[j], y) * jac;
        };
        std::vector<Leaf> sl;
        singular_leaves(boxes[j], surf, fs, sl);
        double acc = 0.0;
        for (const Leaf &l : sl) {
            double v1;
            fs(l.s, l.a, &v1);
            acc += l.w * v1;
        }
        ops.K[(size_t)j * Np + j] = acc;
    }
    ops.LU = ops.K;
    if (!lu_factor(Np, ops.LU, ops.piv)) {
        err = "singular collocation matrix";
        return false;
    }

    // ---- Gamma operator Q.I
    // theta breakpoints graded towards the rim: theta_max (1 - 2^-k)
    std::vector<double> tb = {0.0};
    for (int k = 1; k <= 9; ++k) tb.push_back(tmax * (1.0 - std::ldexp(1.0, -k)));
    tb.push_back(tmax);
    const GL g12(12);
    std::vector<double> tq, twq;
    for (size_t s = 0; s + 1 < tb.size(); ++s) {
        const double h = 0.5 * (tb[s + 1] - tb[s]), m = 0.5 * (tb[s + 1] + tb[s]);
        for (int q = 0; q < 12; ++q) {
            tq.push_back(m + h * g12.x[q]);
            twq.push_back(h * g12.w[q]);
        }
    }
    const int NA = 768;
    // Lagrange basis in theta (barycentric form) at the fine theta points
    std::vector<double> bw(Nt, 1.0);
    for (int a = 0; a < Nt; ++a)
        for (int b = 0; b < Nt; ++b)
            if (b != a) bw[a] /= (th[a] - th[b]);
    const int NT = (int)tq.size();
    std::vector<double> Lth((size_t)Nt * NT);
    for (int q = 0; q < NT; ++q) {
        double den = 0.0;
        int hit = -1;
        for (int a = 0; a < Nt; ++a) {
            const double d = tq[q] - th[a];
            if (d == 0.0) hit = a;
            den += bw[a] / d;
        }
        for (int a = 0; a < Nt; ++a)
            Lth[(size_t)a * NT + q] = hit >= 0 ? (a == hit ? 1.0 : 0.0) : (bw[a] / (tq[q] - th[a])) / den;
    }
    // trigonometric cardinal functions (Fourier form) at the fine azimuths
    std::vector<double> Tph((size_t)Nf * NA);
    for (int b = 0; b < Nf; ++b)
        for (int q = 0; q < NA; ++q) {
            const double d = 2.0 * kPi * q / NA - 2.0 * kPi * b / Nf;
            double s = 1.0 + std::cos(0.5 * Nf * d);
            for (int k = 1; k < Nf / 2; ++k) s += 2.0 * std::cos(k * d);
            Tph[(size_t)b * NA + q] = s / Nf;
        }
    // rows of a Gamma operator: int_Gamma kernel(x_i, y) l_k(y) ds_y for the
    // cardinal functions l_k of the node grid
    std::vector<double> V((size_t)NT * NA), tmp((size_t)Nt * NA);
    auto gamma_rows = [&](auto kernel, std::vector<double> &out) {
        out.assign((size_t)Np * Nn, 0.0);
        for (int i = 0; i < Np; ++i) {
            for (int q = 0; q < NT; ++q) {
                const double st = std::sin(tq[q]), ct = std::cos(tq[q]);
                for (int p = 0; p < NA; ++p) {
                    const double ph = 2.0 * kPi * p / NA;
                    const V3 y{st * std::cos(ph), st * std::sin(ph), -ct};
                    V[(size_t)q * NA + p] = kernel(X[i], y) * st * twq[q] * (2.0 * kPi / NA);
                }
            }
            std::fill(tmp.begin(), tmp.end(), 0.0);
            for (int a = 0; a < Nt; ++a)
                for (int q = 0; q < NT; ++q) {
                    const double l = Lth[(size_t)a * NT + q];
                    const double *vr = &V[(size_t)q * NA];
                    double *tr = &tmp[(size_t)a * NA];
                    for (int p = 0; p < NA; ++p) tr[p] += l * vr[p];
                }
            for (int a = 0; a < Nt; ++a)
                for (int b = 0; b < Nf; ++b) {
                    double s = 0.0;
                    const double *tr = &tmp[(size_t)a * NA];
                    const double *cr = &Tph[(size_t)b * NA];
                    for (int p = 0; p < NA; ++p) s += tr[p] * cr[p];
                    out[(size_t)i * Nn + a * Nf + b] = s;
                }
        }
    };
    gamma_rows([](V3 x, V3 y) { return poisson_ball(x, y); }, ops.QI);
    if (ops.rr == 0.0) {
        second_kind_tables(ops, X, gamma_rows);
    } else {
        std::vector<V3> N(Np);
        for (int k = 0; k < Np; ++k) {
            const Box &b = boxes[k];
            V3 y;
            double jac;
            surf.at(0.5 * (b.s0 + b.s1), 0.5 * (b.a0 + b.a1), y, N[k], jac);
        }
        second_kind_tables_curved(ops, X, N, boxes, surf, gamma_rows);
        if (!lu_factor(Np, ops.M2_LU, ops.M2_piv)) {
            err = "singular second-kind matrix";
            return false;
        }
        // (M^-1 Q2)^2 for the propagated standard error
        ops.A2s.assign((size_t)Np * Nn, 0.0);
        std::vector<double> c(Np);
        for (int k = 0; k < Nn; ++k) {
            for (int i = 0; i < Np; ++i) c[i] = ops.Q2[(size_t)i * Nn + k];
            lu_solve(Np, ops.M2_LU, ops.M2_piv, c.data());
            for (int i = 0; i < Np; ++i) ops.A2s[(size_t)i * Nn + k] = c[i] * c[i];
        }
    }

    // ---- A2 = (K^-1 Q.I)^2, and the ring-0 row: the mean over the central
    // ring's panels (equal areas on a plane patch) of K^-1 Q.I
    ops.A2.assign((size_t)Np * Nn, 0.0);
    ops.ans_row.assign((size_t)Nn, 0.0);
    std::vector<double> col(Np);
    for (int k = 0; k < Nn; ++k) {
        for (int i = 0; i < Np; ++i) col[i] = ops.QI[(size_t)i * Nn + k];
        lu_solve(Np, ops.LU, ops.piv, col.data());
        for (int i = 0; i < Np; ++i) ops.A2[(size_t)i * Nn + k] = col[i] * col[i];
        double r = 0.0;
        for (int i = 0; i < ops.n_sectors; ++i) r += col[i];
        ops.ans_row[k] = r / ops.n_sectors;
    }

    // ---- double-layer rows (curved patches only)
    ops.n_dl = 0;
    ops.dl_pts.clear();
    ops.dl_w.clear();
    if (ops.rr != 0.0) {
        std::vector<std::vector<Leaf>> rows(Np);
        std::vector<std::vector<double>> roww(Np);
        for (int i = 0; i < Np; ++i) {
            for (int j = 0; j < Np; ++j) {
                auto f = [&](double s, double a, double *out) {
                    V3 y, n;
                    double jac;
                    surf.at(s, a, y, n, jac);
                    out[0] = dgreen_ball_dny(X[i], y, n) * jac;
                };
                std::vector<Leaf> lv;
                if (j == i)
                    singular_leaves(boxes[j], surf, f, lv);
                else
                    adapt_leaves(boxes[j], 1, f, 1e-14, 0, lv);
                for (const Leaf &l : lv) {
                    double v;
                    f(l.s, l.a, &v);
                    rows[i].push_back(l);
                    roww[i].push_back(l.w * v);
                }
            }
            ops.n_dl = std::max(ops.n_dl, (int)rows[i].size());
        }
        ops.dl_pts.assign((size_t)Np * ops.n_dl * 3, 0.0);
        ops.dl_w.assign((size_t)Np * ops.n_dl, 0.0);
        for (int i = 0; i < Np; ++i)
            for (size_t q = 0; q < rows[i].size(); ++q) {
                V3 y, n;
                double jac;
                surf.at(rows[i][q].s, rows[i][q].a, y, n, jac);
                double *o = &ops.dl_pts[((size_t)i * ops.n_dl + q) * 3];
                o[0] = y.x;
                o[1] = y.y;
                o[2] = y.z;
                ops.dl_w[(size_t)i * ops.n_dl + q] = roww[i][q];
            }
    }

    // ---- tile fit (plane classes): quadratic LSQ over panels within 0.7
    ops.fit.assign((size_t)16 * Np, 0.0);
    ops.tile_gl.assign(16 * 3, 0.0);
    {
        std::vector<double> gx, gw;
        gauss_legendre(4, gx, gw);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                ops.tile_gl[3 * (i * 4 + j)] = gx[i];
                ops.tile_gl[3 * (i * 4 + j) + 1] = gx[j];
                ops.tile_gl[3 * (i * 4 + j) + 2] = gw[i] * gw[j];
            }
        if (ops.rr == 0.0) {
            std::vector<int> tr;
            for (int i = 0; i < Np; ++i)
                if (std::sqrt(X[i].x * X[i].x + X[i].y * X[i].y) < 0.7) tr.push_back(i);
            if (tr.size() >= 6) {
                auto basis = [](double u, double v, double *b) {
                    b[0] = 1.0;
                    b[1] = u;
                    b[2] = v;
                    b[3] = u * u;
                    b[4] = u * v;
                    b[5] = v * v;
                };
                // normal equations (A^T A) c = A^T s, solved by LU
                std::vector<double> AtA(36, 0.0);
                for (int i : tr) {
                    double b[6];
                    basis(X[i].x, X[i].y, b);
                    for (int r = 0; r < 6; ++r)
                        for (int c = 0; c < 6; ++c) AtA[r * 6 + c] += b[r] * b[c];
                }
                std::vector<int32_t> p6;
                if (!lu_factor(6, AtA, p6)) {
                    err = "tile fit is singular";
                    return false;
                }
                for (size_t t = 0; t < tr.size(); ++t) {
                    double b[6];
                    basis(X[tr[t]].x, X[tr[t]].y, b);
                    std::vector<double> cvec(b, b + 6);
                    lu_solve(6, AtA, p6, cvec.data());  // column of (A^T A)^-1 A^T
                    for (int q = 0; q < 16; ++q) {
                        double e[6];
                        basis(ops.tile_gl[3 * q], ops.tile_gl[3 * q + 1], e);
                        double v = 0.0;
                        for (int r = 0; r < 6; ++r) v += e[r] * cvec[r];
                        ops.fit[(size_t)q * Np + tr[t]] = v;
                    }
                }
            }
        }
    }
    return true;
}

void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w) { gauss_legendre(n, x, w); }

}  // namespace dtn
