// Single-point Neumann data on a flat boundary (Sec. 5.1).
//
// For a point x of a flat part of the boundary with outward normal n and the
// hemisphere Gamma of radius a over the disk S_a (Sec. 3, eq. bw20):
//   du/dn(x) = Sigma1' + Sigma2'                                  (eq. bw64)
//   Sigma1' = - sum_ij W_ij (u(y_ij) - phi(x))                    (eq. bw83)
//   Sigma2' = - 1/(2 pi) int_{S_a minus disk(delta)} (1/rho^3 - 1/a^3)
//               (phi(y) - phi(x)) ds                              (eqs. bw68, bw82)
// with the nodes y_ij of eq. bw85 and u there from the walks (eq. bw87).
// Both rules scale with a: the tables hold them at a = 1 (unit offsets and
// weights times a, see below) and the kernels apply a per point.
//
//   k_point_nodes    one thread per node: y = x + a (s cos t1 + s sin t2 - c n)
//   k_point_neumann  one wave per point: lanes stride over the hemisphere
//                    nodes (Sigma1' and the propagated variance) and over the
//                    ring points (phi evaluated in place for Sigma2'); wave
//                    sums by lane shuffles.  All FP64 (a few hundred terms).
#include <hip/hip_runtime.h>

#include <cmath>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "dtn_device.h"
#include "dtn_internal.h"
#include "dtn_point_rule.h"

namespace dtn {

struct Points {
    Geometry *geom = nullptr;
    std::vector<dtn_point> pts;
    PointRule rule;
    dtn_point *d_pts = nullptr;
    int device = 0;
};

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kPointsPerBlock = 4;  // one wave each

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__global__ __launch_bounds__(256) void k_point_nodes(const dtn_point *__restrict__ pts, int64_t n, int nn,
                                                     const double *__restrict__ hemi, double *__restrict__ nodes)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nn) return;
    const int64_t p = i / nn;
    const int k = (int)(i - p * nn);
    const dtn_point q = pts[p];
    const double t2x = q.n[1] * q.t1[2] - q.n[2] * q.t1[1];
    const double t2y = q.n[2] * q.t1[0] - q.n[0] * q.t1[2];
    const double t2z = q.n[0] * q.t1[1] - q.n[1] * q.t1[0];
    const double u = hemi[4 * k], v = hemi[4 * k + 1], w = hemi[4 * k + 2];
    nodes[3 * i] = q.c[0] + q.a * (u * q.t1[0] + v * t2x - w * q.n[0]);
    nodes[3 * i + 1] = q.c[1] + q.a * (u * q.t1[1] + v * t2y - w * q.n[1]);
    nodes[3 * i + 2] = q.c[2] + q.a * (u * q.t1[2] + v * t2z - w * q.n[2]);
}

template <int DATA>
__global__ __launch_bounds__(256) void k_point_neumann(DevGeom g, const dtn_point *__restrict__ pts, int64_t n,
                                                       int nn, const double *__restrict__ hemi, int nr,
                                                       const double *__restrict__ ring,
                                                       const double *__restrict__ stats, double *__restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * kPointsPerBlock + threadIdx.x / kWave;
    if (p >= n) return;  // wave-uniform
    const int lane = __lane_id();
    const dtn_point q = pts[p];
    const double inv_a = 1.0 / q.a;
    const double fx = phi_eval<DATA>(g, q.c[0], q.c[1], q.c[2]);
    // Sigma1' and its variance: W = table weight / a
    double s1 = 0.0, v1 = 0.0;
    const double *st = stats + 4 * p * (int64_t)nn;
    for (int k = lane; k < nn; k += kWave) {
        const double W = hemi[4 * k + 3] * inv_a;
        const double cnt = st[4 * k], mean = st[4 * k + 1], m2 = st[4 * k + 2];
        s1 += W * (mean - fx);
        if (cnt > 1.0) v1 += W * W * (m2 / (cnt - 1.0)) / cnt;
    }
    // Sigma2' on the ring: points x + rho (cos t1 + sin t2)
    const double t2x = q.n[1] * q.t1[2] - q.n[2] * q.t1[1];
    const double t2y = q.n[2] * q.t1[0] - q.n[0] * q.t1[2];
    const double t2z = q.n[0] * q.t1[1] - q.n[1] * q.t1[0];
    double s2 = 0.0;
    for (int k = lane; k < nr; k += kWave) {
        const double rho = q.a * ring[4 * k], cs = ring[4 * k + 1], sn = ring[4 * k + 2];
        const double y0 = q.c[0] + rho * (cs * q.t1[0] + sn * t2x);
        const double y1 = q.c[1] + rho * (cs * q.t1[1] + sn * t2y);
        const double y2 = q.c[2] + rho * (cs * q.t1[2] + sn * t2z);
        s2 += ring[4 * k + 3] * (phi_eval<DATA>(g, y0, y1, y2) - fx);
    }
    s1 = -wave_sum_f64(s1);
    v1 = wave_sum_f64(v1);
    s2 = wave_sum_f64(s2) * inv_a;
    if (lane == 0) {
        out[4 * p] = s1 + s2;
        out[4 * p + 1] = sqrt(v1);
        out[4 * p + 2] = s1;
        out[4 * p + 3] = s2;
    }
}

template <class T>
hipError_t upload_vec(const std::vector<T> &v, T **out)
{
    *out = nullptr;
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void **)out, sizeof(T) * v.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*out, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

bool unit3(const double *v) { return std::fabs(std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - 1.0) < 1e-12; }

__global__ __launch_bounds__(256) void k_point_answer(const dtn_point *__restrict__ pts, int64_t n, int nn,
                                                      const int64_t *__restrict__ used, double *__restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int64_t w = 0;
    for (int k = 0; k < nn; ++k) w += used[p * nn + k];
    out[4 * p + 2] = (double)w;
    out[4 * p + 3] = pts[p].a;
}

}  // namespace

bool point_ok(const Geometry &g, const dtn_point &q, std::string &why)
{
    if (!(q.a > 0.0) || !std::isfinite(q.a)) {
        why = "a <= 0";
        return false;
    }
    if (!unit3(q.n) || !unit3(q.t1) || std::fabs(q.n[0] * q.t1[0] + q.n[1] * q.t1[1] + q.n[2] * q.t1[2]) > 1e-12) {
        why = "frame (n, t1) not orthonormal";
        return false;
    }
    if (g.dev.kind == DTN_HALF_SPACE) {
        if (std::fabs(q.n[0]) > 1e-12 || std::fabs(q.n[1]) > 1e-12 || q.n[2] > -1.0 + 1e-12) {
            why = "the half space's outward normal is (0, 0, -1)";
            return false;
        }
        const double scale = 1.0 + std::fabs(q.c[0]) + std::fabs(q.c[1]);
        if (std::fabs(q.c[2]) > 1e-12 * scale) {
            why = "centre is not on the plane z = 0";
            return false;
        }
        const double dx = q.c[0] - g.dev.c[0], dy = q.c[1] - g.dev.c[1], dz = q.c[2] - g.dev.c[2];
        if (std::sqrt(dx * dx + dy * dy + dz * dz) + q.a >= g.dev.trunc_r) {
            why = "hemisphere reaches the truncation sphere";
            return false;
        }
        return true;
    }
    if (g.dev.kind == DTN_DISK) {
        if (std::fabs(q.n[0]) > 1e-12 || std::fabs(q.n[1]) > 1e-12 || std::fabs(q.n[2]) < 1.0 - 1e-12) {
            why = "the disk's outward normals are (0, 0, -1) on its upper face and (0, 0, 1) on its lower";
            return false;
        }
        if (std::fabs(q.c[2]) > 1e-12 * (1.0 + g.dev.disk_r)) {
            why = "centre is not on the disk's plane z = 0";
            return false;
        }
        if (std::sqrt(q.c[0] * q.c[0] + q.c[1] * q.c[1]) + q.a > g.dev.disk_r * (1.0 + 1e-12)) {
            why = "S_a leaves the disk";
            return false;
        }
        const double dx = q.c[0] - g.dev.c[0], dy = q.c[1] - g.dev.c[1], dz = q.c[2] - g.dev.c[2];
        if (std::sqrt(dx * dx + dy * dy + dz * dz) + q.a >= g.dev.trunc_r) {
            why = "hemisphere reaches the truncation sphere";
            return false;
        }
        return true;
    }
    if (g.dev.kind == DTN_BOX || g.dev.kind == DTN_BOX_MINUS_BOXES) {
        dtn_patch pt{};
        for (int k = 0; k < 3; ++k) {
            pt.c[k] = q.c[k];
            pt.n[k] = q.n[k];
            pt.t1[k] = q.t1[k];
        }
        pt.h = q.a;
        return plane_patch_ok(g, pt, why);
    }
    why = "the single-point estimate needs a flat boundary (half space, disk or box faces)";
    return false;
}

dtn_status make_point_rule(int n_g1, int n_g2, double delta_rel, PointRule &r)
{
    r = PointRule{};
    r.n_g1 = n_g1;
    r.n_g2 = n_g2;
    r.delta_rel = delta_rel;
    // hemisphere rule at a = 1 (eqs. bw83, bw85): theta = pi/4 (xi + 1),
    // psi = pi (xi + 1); W a = (pi/4 w_i)(pi w_j) sin(th) 3 cos(th) / (2 pi)
    std::vector<double> xi, w;
    gauss_legendre_rule(n_g1, xi, w);
    std::vector<double> hemi(4 * (size_t)n_g1 * n_g1);
    for (int i = 0; i < n_g1; ++i) {
        const double th = 0.25 * kPi * (xi[i] + 1.0), wt = 0.25 * kPi * w[i];
        for (int j = 0; j < n_g1; ++j) {
            const double ps = kPi * (xi[j] + 1.0), wp = kPi * w[j];
            double *h = &hemi[4 * ((size_t)i * n_g1 + j)];
            h[0] = std::sin(th) * std::cos(ps);
            h[1] = std::sin(th) * std::sin(ps);
            h[2] = std::cos(th);
            h[3] = wt * wp * std::sin(th) * 3.0 * std::cos(th) / (2.0 * kPi);
        }
    }
    // ring rule at a = 1 (eqs. bw68, bw82): rho / a = r on [delta_rel, 1],
    // psi on [0, 2 pi]; with rho = a r the term
    // -1/(2 pi) w_rho w_psi rho (1/rho^3 - 1/a^3) equals (1/a) times
    // -1/(2 pi) ((1 - delta_rel)/2 w_k)(pi w_l) r (1/r^3 - 1)
    gauss_legendre_rule(n_g2, xi, w);
    std::vector<double> ring(4 * (size_t)n_g2 * n_g2);
    for (int k = 0; k < n_g2; ++k) {
        const double rr = 0.5 * (1.0 - delta_rel) * xi[k] + 0.5 * (1.0 + delta_rel);
        const double wr = 0.5 * (1.0 - delta_rel) * w[k];
        for (int l = 0; l < n_g2; ++l) {
            const double ps = kPi * (xi[l] + 1.0), wp = kPi * w[l];
            double *h = &ring[4 * ((size_t)k * n_g2 + l)];
            h[0] = rr;
            h[1] = std::cos(ps);
            h[2] = std::sin(ps);
            h[3] = -wr * wp * rr * (1.0 / (rr * rr * rr) - 1.0) / (2.0 * kPi);
        }
    }
    hipError_t e = upload_vec(hemi, &r.d_hemi);
    if (e == hipSuccess) e = upload_vec(ring, &r.d_ring);
    if (e != hipSuccess) {
        free_point_rule(r);
        return fail(DTN_E_DEVICE, std::string("point rule: ") + hipGetErrorString(e));
    }
    return DTN_OK;
}

void free_point_rule(PointRule &r)
{
    (void)hipFree(r.d_hemi);
    (void)hipFree(r.d_ring);
    r.d_hemi = r.d_ring = nullptr;
}

dtn_status launch_point_nodes(const dtn_point *pts, int64_t n, const PointRule &r, double *nodes, hipStream_t s)
{
    const int nn = r.n_g1 * r.n_g1;
    const int64_t total = n * nn;
    if (total == 0) return DTN_OK;
    hipLaunchKernelGGL(k_point_nodes, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, pts, n, nn, r.d_hemi,
                       nodes);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("point nodes: ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status launch_point_neumann(const Geometry &g, const dtn_point *pts, int64_t n, const PointRule &r,
                                const double *stats, double *out, hipStream_t s)
{
    if (n == 0) return DTN_OK;
    const dim3 grid((unsigned)((n + kPointsPerBlock - 1) / kPointsPerBlock)), block(kPointsPerBlock * kWave);
    const int nn = r.n_g1 * r.n_g1, nr = r.n_g2 * r.n_g2;
    if (g.dev.data_kind == DTN_DATA_TABULATED)
        hipLaunchKernelGGL(k_point_neumann<DTN_DATA_TABULATED>, grid, block, 0, s, g.dev, pts, n, nn, r.d_hemi, nr,
                           r.d_ring, stats, out);
    else if (g.dev.data_kind == DTN_DATA_POINT_SOURCES)
        hipLaunchKernelGGL(k_point_neumann<DTN_DATA_POINT_SOURCES>, grid, block, 0, s, g.dev, pts, n, nn, r.d_hemi,
                           nr, r.d_ring, stats, out);
    else
        hipLaunchKernelGGL(k_point_neumann<DTN_DATA_HARMONIC_QUADRATIC>, grid, block, 0, s, g.dev, pts, n, nn,
                           r.d_hemi, nr, r.d_ring, stats, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("point neumann: ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status launch_point_answer(const dtn_point *pts, int64_t n, int nn, const int64_t *used, double *out,
                               hipStream_t s)
{
    if (n == 0) return DTN_OK;
    hipLaunchKernelGGL(k_point_answer, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, n, nn, used, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("point answer: ") + hipGetErrorString(e));
    return DTN_OK;
}

}  // namespace dtn

struct dtn_points_s {
    dtn::Points p;
};

using namespace dtn;

dtn_status dtn_create_points(dtn_geometry g, const dtn_point *pts, int64_t n, int32_t n_g1, int32_t n_g2,
                             double delta_rel, dtn_points *out)
{
    const std::string at = "dtn_create_points: ";
    try {
        if (!g || !pts || !out) return fail(DTN_E_ARG, at + "NULL argument");
        *out = nullptr;
        if (n < 1 || n > ((int64_t)1 << 26)) return fail(DTN_E_ARG, at + "n outside [1, 2^26]");
        if (n_g1 < 1 || n_g1 > 64 || n_g2 < 1 || n_g2 > 64) return fail(DTN_E_ARG, at + "n_g1, n_g2 outside [1, 64]");
        if (!(delta_rel > 0.0 && delta_rel < 1.0)) return fail(DTN_E_ARG, at + "delta_rel outside (0, 1)");
        const Geometry &G = g->g;
        for (int64_t i = 0; i < n; ++i) {
            std::string why;
            if (!point_ok(G, pts[i], why)) return fail(DTN_E_ARG, at + "point " + std::to_string(i) + ": " + why);
        }
        std::unique_ptr<dtn_points_s> P(new (std::nothrow) dtn_points_s());
        if (!P) return fail(DTN_E_OOM, at + "out of host memory");
        Points &p = P->p;
        p.geom = &g->g;
        p.pts.assign(pts, pts + n);
        dtn_status st = make_point_rule(n_g1, n_g2, delta_rel, p.rule);
        if (st != DTN_OK) return st;
        hipError_t e = hipGetDevice(&p.device);
        if (e == hipSuccess) e = upload_vec(p.pts, &p.d_pts);
        if (e != hipSuccess) {
            (void)hipFree(p.d_pts);
            free_point_rule(p.rule);
            return fail(DTN_E_DEVICE, at + hipGetErrorString(e));
        }
        *out = P.release();
        return DTN_OK;
    } catch (...) {
        return fail(DTN_E_OOM, at + "exception");
    }
}

void dtn_destroy_points(dtn_points p)
{
    if (!p) return;
    (void)hipFree(p->p.d_pts);
    free_point_rule(p->p.rule);
    delete p;
}

int64_t dtn_points_num_nodes(dtn_points p)
{
    if (!p) return -1;
    return (int64_t)p->p.pts.size() * p->p.rule.n_g1 * p->p.rule.n_g1;
}

dtn_status dtn_points_nodes(dtn_points p, double *nodes, void *stream)
{
    try {
        if (!p || !nodes) return fail(DTN_E_ARG, "dtn_points_nodes: NULL argument");
        const Points &P = p->p;
        return launch_point_nodes(P.d_pts, (int64_t)P.pts.size(), P.rule, nodes, (hipStream_t)stream);
    } catch (...) {
        return fail(DTN_E_DEVICE, "dtn_points_nodes: exception");
    }
}

dtn_status dtn_points_neumann(dtn_points p, const double *node_stats, double *out, void *stream)
{
    try {
        if (!p || !node_stats || !out) return fail(DTN_E_ARG, "dtn_points_neumann: NULL argument");
        const Points &P = p->p;
        return launch_point_neumann(*P.geom, P.d_pts, (int64_t)P.pts.size(), P.rule, node_stats, out,
                                    (hipStream_t)stream);
    } catch (...) {
        return fail(DTN_E_DEVICE, "dtn_points_neumann: exception");
    }
}
