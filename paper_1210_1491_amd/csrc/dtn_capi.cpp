// C-ABI of the library: geometries, plans, argument checks, error strings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "dtn_internal.h"

namespace dtn {

namespace {
thread_local std::string g_last_error;

struct ClassKey {
    int nt, nf, nr, ns;
    double rr;
    bool operator<(const ClassKey &o) const
    {
        return std::tie(nt, nf, nr, ns, rr) < std::tie(o.nt, o.nf, o.nr, o.ns, o.rr);
    }
};

// Device-resident class operators, shared by all plans of a process and
// kept until exit (a class is a few hundred KB at most).
struct ClassEntry {
    DevClass dev{};
    int device = -1;
};
std::mutex g_class_mu;
std::map<std::pair<int, ClassKey>, ClassEntry> g_classes;

template <class T>
hipError_t upload(const std::vector<T> &v, T **out)
{
    *out = nullptr;
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void **)out, sizeof(T) * v.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*out, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

dtn_status get_class(const ClassKey &key, int device, DevClass &out, bool &fresh)
{
    std::lock_guard<std::mutex> lk(g_class_mu);
    auto it = g_classes.find({device, key});
    fresh = false;
    if (it != g_classes.end()) {
        out = it->second.dev;
        return DTN_OK;
    }
    ClassOps ops;
    ops.n_theta = key.nt;
    ops.n_phi = key.nf;
    ops.n_rings = key.nr;
    ops.n_sectors = key.ns;
    ops.rr = key.rr;
    std::string err;
    if (!build_class_ops(ops, err)) return fail(DTN_E_ARG, "dtn_create_plan: " + err);
    DevClass d{};
    d.n_theta = key.nt;
    d.n_phi = key.nf;
    d.n_rings = key.nr;
    d.n_sectors = key.ns;
    d.n_nodes = key.nt * key.nf;
    d.n_panels = key.nr * key.ns;
    d.curved = key.rr != 0.0 ? 1 : 0;
    d.n_dl = ops.n_dl;
    d.rr = key.rr;
    double *p = nullptr;
    int32_t *ip = nullptr;
    hipError_t e = hipSuccess;
#define UP(field, vec)                                   \
    if (e == hipSuccess) {                               \
        e = upload(ops.vec, &p);                         \
        d.field = p;                                     \
    }
    UP(node_tab, node_tab)
    UP(col_tab, col_tab)
    UP(K, K)
    UP(LU, LU)
    UP(QI, QI)
    UP(A2, A2)
    UP(dl_pts, dl_pts)
    UP(dl_w, dl_w)
    UP(fit, fit)
    UP(tile_gl, tile_gl)
    UP(ans_row, ans_row)
    UP(Q2, Q2)
    UP(s_pts, s_pts)
    UP(s_w, s_w)
    UP(c2, c2)
    UP(M2_LU, M2_LU)
    UP(A2s, A2s)
#undef UP
    if (e == hipSuccess && !ops.M2_piv.empty()) {
        e = upload(ops.M2_piv, &ip);
        d.M2_piv = ip;
    }
    d.n_s = ops.n_s;
    d.k_inf = 0.0;
    for (int i = 0; i < d.n_panels; ++i) {
        double row = 0.0;
        for (int j = 0; j < d.n_panels; ++j) row += std::fabs(ops.K[(size_t)i * d.n_panels + j]);
        d.k_inf = std::max(d.k_inf, row);
    }
    if (e == hipSuccess) {
        e = upload(ops.piv, &ip);
        d.piv = ip;
    }
    if (e == hipSuccess) e = hipMalloc((void **)&d.LU32, sizeof(float) * d.n_panels * d.n_panels);
    if (e == hipSuccess) e = hipMalloc((void **)&d.piv32, sizeof(int32_t) * d.n_panels);
    if (e != hipSuccess) return fail(DTN_E_OOM, std::string("dtn_create_plan: ") + hipGetErrorString(e));
    g_classes[{device, key}] = ClassEntry{d, device};
    out = d;
    fresh = true;
    return DTN_OK;
}

// Device arrays of a geometry (hipFree of NULL is a no-op).
void free_geometry(Geometry &g)
{
    (void)hipFree(g.d_hole_ce);
    (void)hipFree(g.d_hole_box);
    (void)hipFree(g.d_hole_f32);
    (void)hipFree(g.d_sincos);
    (void)hipFree(g.d_cell_mask);
    (void)hipFree(g.d_src);
    (void)hipFree(g.d_tab);
    (void)hipFree(g.d_status);
    g.d_hole_ce = g.d_hole_box = g.d_src = g.d_sincos = g.d_tab = nullptr;
    g.d_hole_f32 = nullptr;
    g.d_cell_mask = nullptr;
    g.d_status = nullptr;
}

// The potential's sum (eq. bw03) runs over square tiles [-h, h]^2 about
// each patch centre in its (t1, n x t1) frame.  It is the integral over the
// box boundary only if the tiles cover every face exactly once: each tile
// has an axis-aligned frame and lies inside its face, tiles on a face do not
// overlap, and their areas add up to the face area.
bool tiles_cover_box(const Geometry &G, const std::vector<dtn_patch> &ps)
{
    const double *lo = G.dev.lo, *hi = G.dev.hi;
    double scale = 0.0;
    for (int k = 0; k < 3; ++k) scale = std::max({scale, std::fabs(lo[k]), std::fabs(hi[k]), hi[k] - lo[k]});
    const double tol = 1e-9 * scale;
    struct Sq { double a0, a1, b0, b1; };
    std::vector<Sq> face[6];
    for (const dtn_patch &q : ps) {
        int k = -1, ta = -1;
        for (int d = 0; d < 3; ++d) {
            if (std::fabs(std::fabs(q.n[d]) - 1.0) < 1e-12) k = d;
            if (std::fabs(std::fabs(q.t1[d]) - 1.0) < 1e-12) ta = d;
        }
        if (k < 0 || ta < 0 || ta == k) return false;
        const int f = 2 * k + (q.n[k] > 0 ? 1 : 0);
        const double plane = q.n[k] < 0 ? lo[k] : hi[k];
        if (std::fabs(q.c[k] - plane) > tol) return false;
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        const Sq sq{q.c[a] - q.h, q.c[a] + q.h, q.c[b] - q.h, q.c[b] + q.h};
        if (sq.a0 < lo[a] - tol || sq.a1 > hi[a] + tol || sq.b0 < lo[b] - tol || sq.b1 > hi[b] + tol) return false;
        face[f].push_back(sq);
    }
    for (int f = 0; f < 6; ++f) {
        const int k = f / 2, a = (k + 1) % 3, b = (k + 2) % 3;
        std::vector<Sq> &v = face[f];
        double area = 0.0;
        for (const Sq &q : v) area += (q.a1 - q.a0) * (q.b1 - q.b0);
        const double want = (hi[a] - lo[a]) * (hi[b] - lo[b]);
        if (std::fabs(area - want) > 1e-9 * want) return false;
        // overlap: sweep in order of the lower a edge
        std::sort(v.begin(), v.end(), [](const Sq &x, const Sq &y) { return x.a0 < y.a0; });
        for (size_t i = 0; i < v.size(); ++i)
            for (size_t j = i + 1; j < v.size() && v[j].a0 < v[i].a1 - tol; ++j)
                if (v[j].b0 < v[i].b1 - tol && v[i].b0 < v[j].b1 - tol) return false;
    }
    return true;
}

bool unit(const double *v, double tol = 1e-12) { return std::fabs(std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - 1.0) < tol; }

// distance from a point to a closed axis-aligned box (0 inside)
double box_dist(const double *x, const double *lo, const double *hi)
{
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double q = std::max({lo[k] - x[k], 0.0, x[k] - hi[k]});
        s += q * q;
    }
    return std::sqrt(s);
}

// Candidate-hole grid.  The box is split into about 32^3 cells.  For a cell
// C, expanded by 1e-3 of its width so that the FP32 rounding of the lookup
// (position, one FMA, truncation: a few 1e-7 of a cell) cannot put a point
// outside the cell it is looked up in, U bounds the distance to the
// boundary from above for every point of C: the interior distance to the
// outer box is at most min_k min(hi_C,k - lo_k, hi_k - lo_C,k), and the
// distance to hole j is a convex function, so at most its largest value at
// the corners of C.  A hole j whose distance to C exceeds U can never be the
// nearest surface of a point of C and is left out of the cell's list; the
// minimum over the listed holes (and the outer faces) is then exactly the
// minimum over all of them.
void build_cell_grid(const double lo[3], const double hi[3], const double *holes, int n_holes,
                     std::vector<uint32_t> &mask, DevGeom &dg)
{
    const double L[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    const double side = std::cbrt(L[0] * L[1] * L[2] / 32768.0);
    int32_t n[3];
    for (int k = 0; k < 3; ++k) {
        n[k] = (int32_t)std::min(256.0, std::max(1.0, std::ceil(L[k] / side)));
        dg.cell_inv[k] = (float)(n[k] / L[k]);
        dg.cell_off[k] = (float)(-lo[k] * (n[k] / L[k]));
        dg.cell_top[k] = (float)n[k] - 0.5f;
    }
    dg.cell_stride[0] = n[1] * n[2];
    dg.cell_stride[1] = n[2];
    mask.assign((size_t)n[0] * n[1] * n[2], 0u);
    const double scale = 1.0 + std::max({std::fabs(lo[0]), std::fabs(lo[1]), std::fabs(lo[2]), std::fabs(hi[0]),
                                         std::fabs(hi[1]), std::fabs(hi[2])});
    const double tol = 1e-9 * scale;
    for (int i = 0; i < n[0]; ++i)
        for (int j = 0; j < n[1]; ++j)
            for (int l = 0; l < n[2]; ++l) {
                const int ijk[3] = {i, j, l};
                double a[3], b[3];
                for (int k = 0; k < 3; ++k) {
                    const double w = L[k] / n[k], margin = 1e-3 * w;
                    a[k] = lo[k] + w * ijk[k] - margin;
                    b[k] = lo[k] + w * (ijk[k] + 1) + margin;
                }
                double U = std::min({b[0] - lo[0], hi[0] - a[0], b[1] - lo[1], hi[1] - a[1], b[2] - lo[2],
                                     hi[2] - a[2]});
                for (int h = 0; h < n_holes; ++h) {
                    double far = 0.0;
                    for (int c = 0; c < 8; ++c) {
                        const double x[3] = {(c & 1) ? b[0] : a[0], (c & 2) ? b[1] : a[1], (c & 4) ? b[2] : a[2]};
                        far = std::max(far, box_dist(x, holes + 6 * h, holes + 6 * h + 3));
                    }
                    U = std::min(U, far);
                }
                uint32_t m = 0;
                for (int h = 0; h < n_holes; ++h) {
                    const double *hl = holes + 6 * h, *hh = hl + 3;
                    double s2 = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        const double gap = std::max({hl[k] - b[k], 0.0, a[k] - hh[k]});
                        s2 += gap * gap;
                    }
                    if (std::sqrt(s2) <= U + tol) m |= 1u << h;
                }
                mask[((size_t)i * n[1] + j) * n[2] + l] = m;
            }
}

// Check that a plane patch lies on a face of the box or of a hole, that S
// fits inside that face and that the half ball over it stays in Omega.
bool check_plane_patch(const Geometry &g, const dtn_patch &p, std::string &why)
{
    int k = -1;
    double sgn = 0.0;
    for (int a = 0; a < 3; ++a)
        if (std::fabs(std::fabs(p.n[a]) - 1.0) < 1e-12) {
            k = a;
            sgn = p.n[a] > 0 ? 1.0 : -1.0;
        }
    if (k < 0 || std::fabs(p.n[(k + 1) % 3]) > 1e-12 || std::fabs(p.n[(k + 2) % 3]) > 1e-12) {
        why = "normal is not an axis direction";
        return false;
    }
    const double *lo = g.dev.lo, *hi = g.dev.hi;
    const double scale = 1.0 + std::max({std::fabs(lo[0]), std::fabs(lo[1]), std::fabs(lo[2]), std::fabs(hi[0]),
                                         std::fabs(hi[1]), std::fabs(hi[2])});
    const double tol = 1e-9 * scale;
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    auto fits = [&](const double *flo, const double *fhi) {
        return p.c[a] - p.h >= flo[a] - tol && p.c[a] + p.h <= fhi[a] + tol && p.c[b] - p.h >= flo[b] - tol &&
               p.c[b] + p.h <= fhi[b] + tol;
    };
    int face_hole = -2;  // -1: outer box face, >= 0: hole index
    const double plane = sgn < 0 ? lo[k] : hi[k];
    if (std::fabs(p.c[k] - plane) < tol && fits(lo, hi)) face_hole = -1;
    for (int i = 0; i < g.dev.n_holes && face_hole == -2; ++i) {
        const double *hl = &g.holes[6 * i], *hh = &g.holes[6 * i + 3];
        const double hp = sgn > 0 ? hl[k] : hh[k];  // Omega's outward normal points into the hole
        if (std::fabs(p.c[k] - hp) < tol && fits(hl, hh)) face_hole = i;
    }
    if (face_hole == -2) {
        why = "centre and disk do not lie on a face with this outward normal";
        return false;
    }
    // the half ball on the Omega side must keep clear of every other surface
    for (int a2 = 0; a2 < 3; ++a2) {
        if (face_hole == -1 && a2 == k) {
            const double other = sgn < 0 ? hi[k] : lo[k];
            if (std::fabs(p.c[k] - other) < p.h - tol) {
                why = "hemisphere crosses the opposite face";
                return false;
            }
            continue;
        }
        if (p.c[a2] - lo[a2] < p.h - tol || hi[a2] - p.c[a2] < p.h - tol) {
            if (!(face_hole == -1 && a2 == k)) {
                why = "hemisphere crosses an outer face";
                return false;
            }
        }
    }
    for (int i = 0; i < g.dev.n_holes; ++i) {
        if (i == face_hole) continue;
        if (box_dist(p.c, &g.holes[6 * i], &g.holes[6 * i + 3]) < p.h - tol) {
            why = "hemisphere crosses a hole";
            return false;
        }
    }
    return true;
}

}  // namespace

bool plane_patch_ok(const Geometry &g, const dtn_patch &p, std::string &why) { return check_plane_patch(g, p, why); }

dtn_status plane_class(int nt, int nf, int nr, int ns, DevClass &out)
{
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("plane_class: ") + hipGetErrorString(e));
    bool fresh = false;
    const dtn_status st = get_class(ClassKey{nt, nf, nr, ns, 0.0}, device, out, fresh);
    if (st != DTN_OK || !fresh) return st;
    // FP32 LU factors of the new class on the device
    std::lock_guard<std::mutex> lk(g_class_mu);
    Plan tmp;
    tmp.classes.resize(1);
    tmp.classes[0].dev = out;
    std::vector<DevClass> one{out};
    e = upload(one, &tmp.d_classes);
    if (e != hipSuccess) return fail(DTN_E_OOM, std::string("plane_class: ") + hipGetErrorString(e));
    dtn_status s2 = launch_lu32(tmp, nullptr);
    e = hipStreamSynchronize(nullptr);
    (void)hipFree(tmp.d_classes);
    if (s2 != DTN_OK) return s2;
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("plane_class: ") + hipGetErrorString(e));
    return DTN_OK;
}

void set_error(const std::string &msg) { g_last_error = msg; }
dtn_status fail(dtn_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

}  // namespace dtn

using namespace dtn;

extern "C" {


const char *dtn_last_error(void) { return g_last_error.c_str(); }
// The build passes the digest of the header it compiles against, so that a
// binding can tell a library built against another version of the header.
#ifndef DTN_HEADER_DIGEST
#error "define DTN_HEADER_DIGEST (first 16 hex digits of the SHA-256 of include/dtn.h)"
#endif

const char *dtn_version(void) { return "dtn-wos-mi355x 0.1 (gfx950) dtn.h " DTN_HEADER_DIGEST; }

dtn_status dtn_create_geometry(const dtn_geometry_desc *desc, dtn_geometry *out)
{
    try {
        if (!desc || !out) return fail(DTN_E_ARG, "dtn_create_geometry: NULL argument");
        *out = nullptr;
        const dtn_geometry_desc &d = *desc;
        if (d.kind < DTN_BALL || d.kind > DTN_BALL_EXTERIOR) return fail(DTN_E_ARG, "dtn_create_geometry: bad kind");
        if (d.data_kind != DTN_DATA_HARMONIC_QUADRATIC && d.data_kind != DTN_DATA_POINT_SOURCES &&
            d.data_kind != DTN_DATA_TABULATED)
            return fail(DTN_E_ARG, "dtn_create_geometry: bad data_kind");
        size_t tab_len = 0;
        if (d.data_kind == DTN_DATA_TABULATED) {
            if (d.kind != DTN_BOX) return fail(DTN_E_ARG, "dtn_create_geometry: tabulated data needs a box");
            if (d.tab_n[0] < 2 || d.tab_n[0] > 4096 || d.tab_n[1] < 2 || d.tab_n[1] > 4096 || !d.tab)
                return fail(DTN_E_ARG, "dtn_create_geometry: tab_n outside [2, 4096] or tab NULL");
            tab_len = (size_t)6 * d.tab_n[0] * d.tab_n[1];
            for (size_t q = 0; q < tab_len; ++q)
                if (!std::isfinite(d.tab[q])) return fail(DTN_E_ARG, "dtn_create_geometry: tab holds a non-finite value");
        }
        if (!(d.eps > 0.0)) return fail(DTN_E_ARG, "dtn_create_geometry: eps must be > 0");
        if (d.max_steps < 0 || d.max_steps > (int64_t)0xffffffff)
            return fail(DTN_E_ARG, "dtn_create_geometry: max_steps outside [0, 2^32 - 1] (a walk's step count "
                                   "is 32-bit)");
        const bool unbounded = d.kind == DTN_HALF_SPACE || d.kind == DTN_DISK || d.kind == DTN_BALL_EXTERIOR;
        if ((d.kind == DTN_BALL || d.kind == DTN_BALL_EXTERIOR) && !(d.ball_r > 0.0))
            return fail(DTN_E_ARG, "dtn_create_geometry: ball_r <= 0");
        if (unbounded && !(d.trunc_r > 0.0)) return fail(DTN_E_ARG, "dtn_create_geometry: trunc_r <= 0");
        if (d.kind == DTN_DISK) {
            if (!(d.disk_r > 0.0)) return fail(DTN_E_ARG, "dtn_create_geometry: disk_r <= 0");
            const double cc = std::sqrt(d.ball_c[0] * d.ball_c[0] + d.ball_c[1] * d.ball_c[1] +
                                        d.ball_c[2] * d.ball_c[2]);
            if (!(cc + d.disk_r < d.trunc_r))
                return fail(DTN_E_ARG, "dtn_create_geometry: the truncation sphere must enclose the disk");
        }
        if (d.kind == DTN_BALL_EXTERIOR && !(d.ball_r < d.trunc_r))
            return fail(DTN_E_ARG, "dtn_create_geometry: the truncation sphere must enclose the ball");
        if (d.kind == DTN_BALL_EXTERIOR && d.data_kind == DTN_DATA_POINT_SOURCES)
            for (int k = 0; k < d.n_src; ++k) {
                const double *q = d.src + 4 * k;
                const double dx = q[0] - d.ball_c[0], dy = q[1] - d.ball_c[1], dz = q[2] - d.ball_c[2];
                if (!(dx * dx + dy * dy + dz * dz < d.ball_r * d.ball_r))
                    return fail(DTN_E_ARG, "dtn_create_geometry: a source lies outside the ball");
            }
        if (d.kind == DTN_BOX || d.kind == DTN_BOX_MINUS_BOXES)
            for (int k = 0; k < 3; ++k)
                if (!(d.box_hi[k] > d.box_lo[k])) return fail(DTN_E_ARG, "dtn_create_geometry: empty box");
        if (d.n_holes < 0 || d.n_src < 0) return fail(DTN_E_ARG, "dtn_create_geometry: negative count");
        if (d.kind == DTN_BOX_MINUS_BOXES && d.n_holes > 0 && !d.holes)
            return fail(DTN_E_ARG, "dtn_create_geometry: holes is NULL");
        if (d.data_kind == DTN_DATA_POINT_SOURCES && (d.n_src < 1 || !d.src))
            return fail(DTN_E_ARG, "dtn_create_geometry: point-source data needs sources");
        if (d.kind == DTN_DISK && d.data_kind == DTN_DATA_POINT_SOURCES)
            for (int k = 0; k < d.n_src; ++k) {
                const double *q = d.src + 4 * k;
                if (q[2] == 0.0 && q[0] * q[0] + q[1] * q[1] <= d.disk_r * d.disk_r)
                    return fail(DTN_E_ARG, "dtn_create_geometry: a source lies on the disk");
            }
        if (d.kind == DTN_HALF_SPACE && d.data_kind == DTN_DATA_POINT_SOURCES)
            for (int k = 0; k < d.n_src; ++k)
                if (!(d.src[4 * k + 2] < 0.0))
                    return fail(DTN_E_ARG, "dtn_create_geometry: a source of the half space is not in z < 0");
        if (d.data_kind == DTN_DATA_HARMONIC_QUADRATIC &&
            std::fabs(d.quad_coef[4] + d.quad_coef[5] + d.quad_coef[6]) >
                1e-12 * (1.0 + std::fabs(d.quad_coef[4]) + std::fabs(d.quad_coef[5]) + std::fabs(d.quad_coef[6])))
            return fail(DTN_E_ARG, "dtn_create_geometry: quadratic data is not harmonic");
        std::unique_ptr<dtn_geometry_s> G(new (std::nothrow) dtn_geometry_s());
        if (!G) return fail(DTN_E_OOM, "dtn_create_geometry: out of host memory");
        Geometry &g = G->g;
        g.desc = d;
        g.dev.kind = d.kind;
        g.dev.data_kind = d.data_kind;
        for (int k = 0; k < 3; ++k) {
            g.dev.c[k] = d.ball_c[k];
            g.dev.lo[k] = d.box_lo[k];
            g.dev.hi[k] = d.box_hi[k];
        }
        g.dev.r = d.ball_r;
        for (int k = 0; k < 10; ++k) g.dev.quad[k] = d.quad_coef[k];
        g.dev.eps = d.eps;
        g.dev.disk_r = d.kind == DTN_DISK ? d.disk_r : 0.0;
        g.dev.trunc_r = unbounded ? d.trunc_r : 0.0;
        if (tab_len) {
            g.dev.tab_n[0] = d.tab_n[0];
            g.dev.tab_n[1] = d.tab_n[1];
            for (int k = 0; k < 3; ++k) {
                g.dev.tab_sc[k][0] = (double)(d.tab_n[0] - 1) / (d.box_hi[k] - d.box_lo[k]);
                g.dev.tab_sc[k][1] = (double)(d.tab_n[1] - 1) / (d.box_hi[k] - d.box_lo[k]);
            }
        }
        g.dev.max_steps = d.max_steps;
        const int nh = d.kind == DTN_BOX_MINUS_BOXES ? d.n_holes : 0;
        g.dev.n_holes = nh;
        g.holes.assign(d.holes ? d.holes : nullptr, d.holes ? d.holes + 6 * nh : nullptr);
        std::vector<double> ce(6 * (size_t)nh);
        for (int i = 0; i < nh; ++i) {
            const double *h = &g.holes[6 * i];
            for (int k = 0; k < 3; ++k) {
                if (!(h[3 + k] > h[k]) || h[k] <= d.box_lo[k] || h[3 + k] >= d.box_hi[k])
                    return fail(DTN_E_ARG, "dtn_create_geometry: hole " + std::to_string(i) +
                                               " is empty or not strictly inside the box");
                ce[6 * i + k] = 0.5 * (h[k] + h[3 + k]);
                ce[6 * i + 3 + k] = 0.5 * (h[3 + k] - h[k]);
            }
        }
        std::vector<float> ce32(8 * (size_t)nh, 0.0f);
        for (int i = 0; i < nh; ++i)
            for (int k = 0; k < 6; ++k) ce32[8 * i + k] = (float)ce[6 * i + k];
        const int ns = d.data_kind == DTN_DATA_POINT_SOURCES ? d.n_src : 0;
        g.dev.n_src = ns;
        if (ns) g.src.assign(d.src, d.src + 4 * ns);
        hipError_t e = hipGetDevice(&g.device);
        if (e == hipSuccess) e = upload(ce, &g.d_hole_ce);
        if (e == hipSuccess) e = upload(g.holes, &g.d_hole_box);
        if (e == hipSuccess) e = upload(ce32, &g.d_hole_f32);
        {
            // (sin, cos) of 2 pi j / 256, evaluated in extended precision and rounded once
            std::vector<double> tab(512);
            for (int j = 0; j < 256; ++j) {
                const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)j / 256.0L;
                tab[2 * j] = (double)std::sin(a);
                tab[2 * j + 1] = (double)std::cos(a);
            }
            if (e == hipSuccess) e = upload(tab, &g.d_sincos);
        }
        if (nh >= 1 && nh <= 32) {
            build_cell_grid(d.box_lo, d.box_hi, g.holes.data(), nh, g.cell_mask, g.dev);
            if (e == hipSuccess) e = upload(g.cell_mask, &g.d_cell_mask);
        }
        if (e == hipSuccess) e = upload(g.src, &g.d_src);
        if (e == hipSuccess && tab_len) e = upload(std::vector<double>(d.tab, d.tab + tab_len), &g.d_tab);
        if (e == hipSuccess) e = upload(std::vector<DevStatus>(1, DevStatus{}), &g.d_status);
        if (e != hipSuccess) {
            free_geometry(g);
            return fail(DTN_E_DEVICE, std::string("dtn_create_geometry: ") + hipGetErrorString(e));
        }
        g.dev.hole_ce = g.d_hole_ce;
        g.dev.hole_box = g.d_hole_box;
        g.dev.hole_f32 = g.d_hole_f32;
        g.dev.sincos = g.d_sincos;
        g.dev.cell_mask = g.d_cell_mask;
        g.dev.src = g.d_src;
        g.dev.tab = g.d_tab;
        g.dev.status = g.d_status;
        // keep stream-ordered scratch in the pool between calls
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, g.device) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        *out = G.release();
        return DTN_OK;
    } catch (...) {
        return fail(DTN_E_OOM, "dtn_create_geometry: exception");
    }
}

void dtn_destroy_geometry(dtn_geometry g)
{
    if (!g) return;
    free_geometry(g->g);
    delete g;
}

dtn_status dtn_wos_eval(dtn_geometry g, const double *pts, int64_t n, const int64_t *walks,
                        const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id, int32_t precision,
                        double *stats, int64_t *capped, void *stream)
{
    try {
        if (!g) return fail(DTN_E_ARG, "dtn_wos_eval: NULL geometry");
        if (n < 0) return fail(DTN_E_ARG, "dtn_wos_eval: n < 0");
        if (precision != DTN_FP64 && precision != DTN_FP32_MIXED)
            return fail(DTN_E_ARG, "dtn_wos_eval: unknown precision");
        if (n > 0 && (!pts || !walks || !stats)) return fail(DTN_E_ARG, "dtn_wos_eval: NULL array");
        if (n > ((int64_t)1 << 40)) return fail(DTN_E_ARG, "dtn_wos_eval: n too large");
        if (!stream_id && n > ((int64_t)1 << 32))
            return fail(DTN_E_ARG, "dtn_wos_eval: more than 2^32 points need explicit stream ids");
        return launch_wos(g->g, pts, n, walks, walk_begin, seed, stream_id, precision, stats, capped, Schedule{},
                          (hipStream_t)stream);
    } catch (...) {
        return fail(DTN_E_DEVICE, "dtn_wos_eval: exception");
    }
}

dtn_status dtn_wos_eval_noalloc(dtn_geometry g, const double *pts, int64_t n, const int64_t *walks,
                                const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id,
                                int32_t precision, double *stats, int64_t *capped, void *stream)
{
    try {
        if (!g) return fail(DTN_E_ARG, "dtn_wos_eval_noalloc: NULL geometry");
        if (n < 0) return fail(DTN_E_ARG, "dtn_wos_eval_noalloc: n < 0");
        if (precision != DTN_FP64 && precision != DTN_FP32_MIXED)
            return fail(DTN_E_ARG, "dtn_wos_eval_noalloc: unknown precision");
        if (n > 0 && (!pts || !walks || !stats)) return fail(DTN_E_ARG, "dtn_wos_eval_noalloc: NULL array");
        if (!stream_id && n > ((int64_t)1 << 32))
            return fail(DTN_E_ARG, "dtn_wos_eval_noalloc: more than 2^32 points need explicit stream ids");
        return launch_wos_noalloc(g->g, pts, n, walks, walk_begin, seed, stream_id, precision, stats, capped,
                                  (hipStream_t)stream);
    } catch (...) {
        return fail(DTN_E_DEVICE, "dtn_wos_eval_noalloc: exception");
    }
}

dtn_status dtn_boundary_distance(dtn_geometry g, const double *pts, int64_t n, int32_t precision, double *dist,
                                 void *stream)
{
    try {
        if (!g) return fail(DTN_E_ARG, "dtn_boundary_distance: NULL geometry");
        if (n < 0 || n > ((int64_t)1 << 40)) return fail(DTN_E_ARG, "dtn_boundary_distance: n outside [0, 2^40]");
        if (precision != DTN_FP64 && precision != DTN_FP32_MIXED)
            return fail(DTN_E_ARG, "dtn_boundary_distance: unknown precision");
        if (n > 0 && (!pts || !dist)) return fail(DTN_E_ARG, "dtn_boundary_distance: NULL array");
        return launch_distance(g->g, pts, n, precision, dist, (hipStream_t)stream);
    } catch (...) {
        return fail(DTN_E_DEVICE, "dtn_boundary_distance: exception");
    }
}

static bool schedule_from(const dtn_schedule *in, Schedule &out, std::string &why)
{
    out = Schedule{};
    if (!in) return true;
    if (in->min_chunk < 1 || in->min_chunk > ((int64_t)1 << 40)) {
        why = "min_chunk outside [1, 2^40]";
        return false;
    }
    if (in->oversub < 1 || in->oversub > 64) {
        why = "oversub outside [1, 64]";
        return false;
    }
    if (in->reserved != 0) {
        why = "reserved field is not 0";
        return false;
    }
    out.min_chunk = in->min_chunk;
    out.oversub = in->oversub;
    return true;
}

dtn_status dtn_wos_adaptive(dtn_geometry g, const double *pts, int64_t n, const dtn_adaptive *budget,
                            uint64_t seed, const uint32_t *stream_id, int32_t precision,
                            const dtn_schedule *sched, double *stats, int64_t *walks_used, int64_t *capped,
                            void *stream)
{
    try {
        const std::string at = "dtn_wos_adaptive: ";
        if (!g || !budget) return fail(DTN_E_ARG, at + "NULL geometry or budget");
        if (n < 0 || n > ((int64_t)1 << 40)) return fail(DTN_E_ARG, at + "n outside [0, 2^40]");
        if (precision != DTN_FP64 && precision != DTN_FP32_MIXED) return fail(DTN_E_ARG, at + "unknown precision");
        if (n > 0 && (!pts || !stats || !walks_used)) return fail(DTN_E_ARG, at + "NULL array");
        if (!stream_id && n > ((int64_t)1 << 32))
            return fail(DTN_E_ARG, at + "more than 2^32 points need explicit stream ids");
        const dtn_adaptive &b = *budget;
        if (b.pilot_walks < 2 || b.pilot_walks > ((int64_t)1 << 40))
            return fail(DTN_E_ARG, at + "pilot_walks outside [2, 2^40]");
        if (b.min_walks < 1 || b.min_walks > b.max_walks || b.max_walks > ((int64_t)1 << 40))
            return fail(DTN_E_ARG, at + "need 1 <= min_walks <= max_walks <= 2^40");
        if (!(b.se_target > 0.0) || !std::isfinite(b.se_target) || !std::isfinite(b.se_target * b.se_target) ||
            !(b.se_target * b.se_target > 0.0))
            return fail(DTN_E_ARG, at + "se_target must be positive and finite (with a normal square)");
        Schedule sc;
        std::string why;
        if (!schedule_from(sched, sc, why)) return fail(DTN_E_ARG, at + why);
        const Adaptive a{b.pilot_walks, b.min_walks, b.max_walks, b.se_target};
        return launch_wos_adaptive(g->g, pts, n, a, seed, nullptr, stream_id, precision, stats, walks_used, capped,
                                   sc, (hipStream_t)stream);
    } catch (...) {
        return fail(DTN_E_DEVICE, "dtn_wos_adaptive: exception");
    }
}

dtn_status dtn_wos_time_schedules(dtn_geometry g, const double *pts, int64_t n, const int64_t *walks,
                                  const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id,
                                  int32_t precision, const dtn_schedule *cands, int32_t n_cands, int32_t reps,
                                  double *stats, float *ms_out, void *stream)
{
    const std::string at = "dtn_wos_time_schedules: ";
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto done = [&](dtn_status st) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return st;
    };
    try {
        if (!g || !cands || !ms_out) return fail(DTN_E_ARG, at + "NULL geometry, candidates or output");
        if (n < 1 || n > ((int64_t)1 << 40)) return fail(DTN_E_ARG, at + "n outside [1, 2^40]");
        if (n_cands < 1 || reps < 1) return fail(DTN_E_ARG, at + "n_cands and reps must be >= 1");
        if (precision != DTN_FP64 && precision != DTN_FP32_MIXED) return fail(DTN_E_ARG, at + "unknown precision");
        if (!pts || !walks || !stats) return fail(DTN_E_ARG, at + "NULL array");
        std::vector<Schedule> sc(n_cands);
        std::string why;
        for (int c = 0; c < n_cands; ++c)
            if (!schedule_from(&cands[c], sc[c], why))
                return fail(DTN_E_ARG, at + "candidate " + std::to_string(c) + ": " + why);
        hipStream_t s = (hipStream_t)stream;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return done(fail(DTN_E_DEVICE, at + "hipEventCreate failed"));
        for (int c = 0; c < n_cands; ++c) {
            dtn_status st = launch_wos(g->g, pts, n, walks, walk_begin, seed, stream_id, precision, stats, nullptr,
                                       sc[c], s);
            if (st != DTN_OK) return done(st);
            hipError_t e = hipEventRecord(e0, s);
            for (int r = 0; r < reps && e == hipSuccess && st == DTN_OK; ++r)
                st = launch_wos(g->g, pts, n, walks, walk_begin, seed, stream_id, precision, stats, nullptr, sc[c],
                                s);
            if (st != DTN_OK) return done(st);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) return done(fail(DTN_E_DEVICE, at + hipGetErrorString(e)));
            ms_out[c] = ms / (float)reps;
        }
        return done(DTN_OK);
    } catch (...) {
        return done(fail(DTN_E_DEVICE, at + "exception"));
    }
}

dtn_status dtn_create_plan(dtn_geometry g, const dtn_patch *patches, int64_t n_patches, dtn_plan *out)
{
    try {
        if (!g || !patches || !out) return fail(DTN_E_ARG, "dtn_create_plan: NULL argument");
        *out = nullptr;
        if (n_patches < 1 || n_patches > (1 << 26)) return fail(DTN_E_ARG, "dtn_create_plan: bad n_patches");
        const Geometry &G = g->g;
        std::unique_ptr<dtn_plan_s> P(new (std::nothrow) dtn_plan_s());
        if (!P) return fail(DTN_E_OOM, "dtn_create_plan: out of host memory");
        Plan &p = P->p;
        p.geom = &g->g;
        p.patches.assign(patches, patches + n_patches);
        p.node_off.assign(n_patches + 1, 0);
        p.panel_off.assign(n_patches + 1, 0);
        p.patch_class.resize(n_patches);
        std::map<ClassKey, int> local;
        std::vector<ClassKey> keys;
        if (G.dev.kind == DTN_HALF_SPACE || G.dev.kind == DTN_DISK)
            return fail(DTN_E_ARG, "dtn_create_plan: patch plans need a bounded domain (use dtn_create_points for "
                                   "the half space and the disk)");
        p.tiles_ok = G.dev.kind == DTN_BOX;
        for (int64_t i = 0; i < n_patches; ++i) {
            const dtn_patch &q = p.patches[i];
            const std::string at = "dtn_create_plan: patch " + std::to_string(i) + ": ";
            if (q.n_theta < 2 || q.n_theta > 32 || q.n_phi < 4 || q.n_phi > 64 || (q.n_phi & 1) || q.n_rings < 1 ||
                q.n_rings > 16 || q.n_sectors < 2 || q.n_sectors > 32 || q.n_rings * q.n_sectors > 128)
                return fail(DTN_E_ARG, at + "unsupported node or panel layout");
            if (!(q.h > 0.0) || !unit(q.n) || !unit(q.t1) ||
                std::fabs(q.n[0] * q.t1[0] + q.n[1] * q.t1[1] + q.n[2] * q.t1[2]) > 1e-12)
                return fail(DTN_E_ARG, at + "h <= 0 or frame (n, t1) not orthonormal");
            double rr = 0.0;
            if (G.dev.kind == DTN_BALL || G.dev.kind == DTN_BALL_EXTERIOR) {
                // outside the ball the domain's outward normal points to the
                // centre and the class takes the signed radius -R/h
                const double R = G.dev.r, e = G.dev.kind == DTN_BALL ? 1.0 : -1.0;
                double v[3], rv = 0.0;
                for (int k = 0; k < 3; ++k) {
                    v[k] = q.c[k] - G.dev.c[k];
                    rv += v[k] * v[k];
                }
                rv = std::sqrt(rv);
                if (std::fabs(rv - R) > 1e-12 * R) return fail(DTN_E_ARG, at + "centre is not on the sphere");
                for (int k = 0; k < 3; ++k)
                    if (std::fabs(e * v[k] / rv - q.n[k]) > 1e-12)
                        return fail(DTN_E_ARG, at + "n is not the outward normal of the domain");
                if (!(q.h <= R)) return fail(DTN_E_ARG, at + "h must not exceed the ball radius");
                if (e < 0.0 && !(R + q.h < G.dev.trunc_r))
                    return fail(DTN_E_ARG, at + "the hemisphere reaches the truncation sphere");
                rr = e * R / q.h;
            } else {
                std::string why;
                if (!check_plane_patch(G, q, why)) return fail(DTN_E_ARG, at + why);
                // potential tiles: patches on the outer faces only
                const int k = std::fabs(q.n[0]) > 0.5 ? 0 : (std::fabs(q.n[1]) > 0.5 ? 1 : 2);
                const double plane = q.n[k] < 0 ? G.dev.lo[k] : G.dev.hi[k];
                if (std::fabs(q.c[k] - plane) > 1e-9) p.tiles_ok = false;
            }
            const ClassKey key{q.n_theta, q.n_phi, q.n_rings, q.n_sectors, rr};
            auto it = local.find(key);
            int ci;
            if (it == local.end()) {
                ci = (int)keys.size();
                local[key] = ci;
                keys.push_back(key);
            } else {
                ci = it->second;
            }
            p.patch_class[i] = ci;
            p.node_off[i + 1] = p.node_off[i] + (int64_t)q.n_theta * q.n_phi;
            p.panel_off[i + 1] = p.panel_off[i] + (int64_t)q.n_rings * q.n_sectors;
        }
        p.n_nodes = p.node_off[n_patches];
        p.n_panels = p.panel_off[n_patches];
        if (p.tiles_ok) p.tiles_ok = tiles_cover_box(G, p.patches);
        hipError_t e = hipGetDevice(&p.device);
        if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_create_plan: ") + hipGetErrorString(e));
        std::vector<DevClass> dc(keys.size());
        std::vector<char> fresh(keys.size(), 0);
        for (size_t c = 0; c < keys.size(); ++c) {
            bool f = false;
            const dtn_status s = get_class(keys[c], p.device, dc[c], f);
            if (s != DTN_OK) return s;
            fresh[c] = f;
        }
        p.classes.resize(keys.size());
        for (size_t c = 0; c < keys.size(); ++c) p.classes[c].dev = dc[c];
        if (e == hipSuccess) e = upload(dc, &p.d_classes);
        if (e == hipSuccess) e = upload(p.patches, &p.d_patches);
        if (e == hipSuccess) e = upload(p.patch_class, &p.d_patch_class);
        if (e == hipSuccess) e = upload(p.node_off, &p.d_node_off);
        if (e == hipSuccess) e = upload(p.panel_off, &p.d_panel_off);
        if (e != hipSuccess) return fail(DTN_E_OOM, std::string("dtn_create_plan: ") + hipGetErrorString(e));
        // FP32 LU factors of new classes, on the device (MFMA trailing updates)
        bool any_fresh = false;
        for (char f : fresh) any_fresh = any_fresh || f;
        if (any_fresh) {
            std::lock_guard<std::mutex> lk(g_class_mu);
            const dtn_status s = launch_lu32(p, nullptr);
            if (s != DTN_OK) return s;
            e = hipStreamSynchronize(nullptr);
            if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_create_plan: ") + hipGetErrorString(e));
        }
        *out = P.release();
        return DTN_OK;
    } catch (...) {
        return fail(DTN_E_OOM, "dtn_create_plan: exception");
    }
}

void dtn_destroy_plan(dtn_plan p)
{
    if (!p) return;
    (void)hipFree(p->p.d_classes);
    (void)hipFree(p->p.d_patches);
    (void)hipFree(p->p.d_patch_class);
    (void)hipFree(p->p.d_node_off);
    (void)hipFree(p->p.d_panel_off);
    delete p;
}

dtn_status dtn_check(dtn_geometry g, void *stream)
{
    try {
        if (!g) return fail(DTN_E_ARG, "dtn_check: NULL geometry");
        static std::mutex mu;  // one snapshot word per geometry
        std::lock_guard<std::mutex> lk(mu);
        uint32_t bits = 0;
        const dtn_status st = take_flags(g->g, (hipStream_t)stream, bits);
        if (st != DTN_OK) return st;
        if (bits & kFlagNoConv)
            return fail(DTN_E_NOCONV, std::string("dtn_check: an FP32-mixed solve did not reach its residual "
                                                  "bound") +
                                          (bits & kFlagCapped ? "; walks were ended by the step cap" : ""));
        if (bits & kFlagCapped)
            return fail(DTN_E_MAXSTEPS, "dtn_check: walks were ended by the step cap (see the per-point capped "
                                        "counts)");
        return DTN_OK;
    } catch (...) {
        return fail(DTN_E_OOM, "dtn_check: exception");
    }
}

dtn_status dtn_walk_counters(dtn_geometry g, void *stream, int32_t enable, int64_t out[2])
{
    try {
        if (!g) return fail(DTN_E_ARG, "dtn_walk_counters: NULL geometry");
        if (enable != 0 && enable != 1) return fail(DTN_E_ARG, "dtn_walk_counters: enable must be 0 or 1");
        static std::mutex mu;  // one snapshot per geometry
        std::lock_guard<std::mutex> lk(mu);
        unsigned long long c[2] = {0, 0};
        const dtn_status st = take_counters(g->g, (hipStream_t)stream, c);
        if (out) {
            out[0] = (int64_t)c[0];
            out[1] = (int64_t)c[1];
        }
        g->g.dev.count_walks = enable;
        return st;
    } catch (...) {
        return fail(DTN_E_OOM, "dtn_walk_counters: exception");
    }
}

dtn_status dtn_plan_set_max_sweeps(dtn_plan p, int32_t max_sweeps)
{
    if (!p) return fail(DTN_E_ARG, "dtn_plan_set_max_sweeps: NULL plan");
    if (max_sweeps < 0 || max_sweeps > 64) return fail(DTN_E_ARG, "dtn_plan_set_max_sweeps: outside [0, 64]");
    p->p.max_sweeps = max_sweeps;
    return DTN_OK;
}

int64_t dtn_plan_num_nodes(dtn_plan p) { return p ? p->p.n_nodes : -1; }
int64_t dtn_plan_num_panels(dtn_plan p) { return p ? p->p.n_panels : -1; }

dtn_status dtn_patch_nodes(dtn_plan p, double *nodes, void *stream)
{
    if (!p || !nodes) return fail(DTN_E_ARG, "dtn_patch_nodes: NULL argument");
    return launch_nodes(p->p, nodes, (hipStream_t)stream);
}

dtn_status dtn_patch_solve(dtn_plan p, const double *node_stats, int32_t precision, double *neumann,
                           double *neumann_se, void *stream)
{
    if (!p || !node_stats || !neumann) return fail(DTN_E_ARG, "dtn_patch_solve: NULL argument");
    if (precision != DTN_FP64 && precision != DTN_FP32_MIXED)
        return fail(DTN_E_ARG, "dtn_patch_solve: unknown precision");
    return launch_solve(p->p, node_stats, precision, neumann, neumann_se, (hipStream_t)stream);
}

dtn_status dtn_patch_solve_second_kind(dtn_plan p, const double *node_stats, double *neumann, double *neumann_se,
                                       void *stream)
{
    try {
        if (!p || !node_stats || !neumann) return fail(DTN_E_ARG, "dtn_patch_solve_second_kind: NULL argument");
        for (const PlanClassHost &c : p->p.classes)
            if (!c.dev.Q2 || (c.dev.curved && !c.dev.M2_LU))
                return fail(DTN_E_UNSUPPORTED, "dtn_patch_solve_second_kind: a patch class has no second-kind tables");
        return launch_solve2(p->p, node_stats, neumann, neumann_se, (hipStream_t)stream);
    } catch (...) {
        return fail(DTN_E_DEVICE, "dtn_patch_solve_second_kind: exception");
    }
}

dtn_status dtn_potential(dtn_plan p, const double *neumann, const double *targets, int64_t m, double *u_out,
                         void *stream)
{
    if (!p) return fail(DTN_E_ARG, "dtn_potential: NULL plan");
    if (m < 0) return fail(DTN_E_ARG, "dtn_potential: m < 0");
    if (m > 0 && (!neumann || !targets || !u_out)) return fail(DTN_E_ARG, "dtn_potential: NULL array");
    if (!p->p.tiles_ok)
        return fail(DTN_E_UNSUPPORTED, "dtn_potential: needs square tiles on the faces of a box domain");
    return launch_potential(p->p, neumann, targets, m, u_out, (hipStream_t)stream);
}

dtn_status dtn_class_operators(int32_t n_theta, int32_t n_phi, int32_t n_rings, int32_t n_sectors, double rr,
                               double *node_tab, double *col_tab, double *K, double *QI, double *A2, double *fit)
{
    try {
        ClassOps ops;
        ops.n_theta = n_theta;
        ops.n_phi = n_phi;
        ops.n_rings = n_rings;
        ops.n_sectors = n_sectors;
        ops.rr = rr;
        if (n_theta < 2 || n_theta > 32 || n_phi < 4 || n_phi > 64 || (n_phi & 1) || n_rings < 1 || n_rings > 16 ||
            n_sectors < 2 || n_sectors > 32 || n_rings * n_sectors > 128 || (rr != 0.0 && std::fabs(rr) < 1.0))
            return fail(DTN_E_ARG, "dtn_class_operators: unsupported layout");
        std::string err;
        if (!build_class_ops(ops, err)) return fail(DTN_E_ARG, "dtn_class_operators: " + err);
        auto put = [](const std::vector<double> &v, double *o) {
            if (o) std::copy(v.begin(), v.end(), o);
        };
        put(ops.node_tab, node_tab);
        put(ops.col_tab, col_tab);
        put(ops.K, K);
        put(ops.QI, QI);
        put(ops.A2, A2);
        put(ops.fit, fit);
        return DTN_OK;
    } catch (...) {
        return fail(DTN_E_OOM, "dtn_class_operators: exception");
    }
}

}  // extern "C"

dtn_status dtn_class_second_kind(int32_t n_theta, int32_t n_phi, int32_t n_rings, int32_t n_sectors, double rr,
                                 double *Q2, double *c2, double *M)
{
    try {
        if (!Q2 || !c2) return fail(DTN_E_ARG, "dtn_class_second_kind: NULL argument");
        if (n_theta < 2 || n_theta > 32 || n_phi < 4 || n_phi > 64 || (n_phi & 1) || n_rings < 1 || n_rings > 16 ||
            n_sectors < 2 || n_sectors > 32 || n_rings * n_sectors > 128)
            return fail(DTN_E_ARG, "dtn_class_second_kind: unsupported layout");
        if (!std::isfinite(rr) || (rr != 0.0 && std::fabs(rr) < 1.0))
            return fail(DTN_E_ARG, "dtn_class_second_kind: |rr| must be >= 1 (or 0 for a plane)");
        dtn::ClassOps ops;
        ops.n_theta = n_theta;
        ops.n_phi = n_phi;
        ops.n_rings = n_rings;
        ops.n_sectors = n_sectors;
        ops.rr = rr;
        std::string err;
        if (!dtn::build_class_ops(ops, err)) return dtn::fail(DTN_E_ARG, "dtn_class_second_kind: " + err);
        std::copy(ops.Q2.begin(), ops.Q2.end(), Q2);
        std::copy(ops.c2.begin(), ops.c2.end(), c2);
        if (M) {
            const int P = n_rings * n_sectors;
            if (rr == 0.0) {
                std::fill(M, M + (size_t)P * P, 0.0);
                for (int i = 0; i < P; ++i) M[(size_t)i * P + i] = 0.5;
            } else {
                std::copy(ops.M2.begin(), ops.M2.end(), M);
            }
        }
        return DTN_OK;
    } catch (...) {
        return dtn::fail(DTN_E_OOM, "dtn_class_second_kind: exception");
    }
}
