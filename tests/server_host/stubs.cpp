// Stand-ins for the library functions the query server calls, for the
// host-only build (fake_hip.cpp).  Each launcher enqueues a host closure on
// the stream, as the real one enqueues kernels, reading its inputs and
// writing its outputs when the stream runs it.  The values are simple
// deterministic functions of the inputs (not the method's arithmetic), so
// that the driver can check every answer against the query's own points:
//   node k of a patch (c, n):  c + 1e-3 (k + 1) n
//   walk statistics of a node: mean = x + y + z + 1e-3 u(key, sid), u in [0, 1)
//                              count = budget(se^2) (the pilot for an infinite target)
//   answer of a patch:         (mean over its nodes, 1e-3, sum of budgets, h)
// Descriptors are checked where a kernel would read them: a row that is not
// a valid patch or point aborts the run (padding rows included).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "hip/hip_runtime.h"
#include "dtn_internal.h"
#include "dtn_point_rule.h"

namespace dtn {

thread_local std::string g_err;
void set_error(const std::string &m) { g_err = m; }
dtn_status fail(dtn_status s, const std::string &m)
{
    g_err = m;
    return s;
}
int device_cus() { return 256; }

bool plane_patch_ok(const Geometry &, const dtn_patch &, std::string &) { return true; }

dtn_status plane_class(int nt, int nf, int nr, int ns, DevClass &out)
{
    out = DevClass{};
    out.n_theta = nt;
    out.n_phi = nf;
    out.n_rings = nr;
    out.n_sectors = ns;
    out.n_nodes = nt * nf;
    out.n_panels = nr * ns;
    return DTN_OK;
}

dtn_status make_point_rule(int n_g1, int n_g2, double delta_rel, PointRule &r)
{
    r.n_g1 = n_g1;
    r.n_g2 = n_g2;
    r.delta_rel = delta_rel;
    (void)hipMalloc((void **)&r.d_hemi, sizeof(double) * 4 * n_g1 * n_g1);
    (void)hipMalloc((void **)&r.d_ring, sizeof(double) * 4 * n_g2 * n_g2);
    return DTN_OK;
}
void free_point_rule(PointRule &r)
{
    (void)hipFree(r.d_hemi);
    (void)hipFree(r.d_ring);
    r.d_hemi = r.d_ring = nullptr;
}

namespace {

void check_frame(const double *c, const double *n, double h, int64_t row, const char *what)
{
    int axis = 0;
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(c[k]) || !std::isfinite(n[k])) axis = -9;
        if (std::fabs(std::fabs(n[k]) - 1.0) < 1e-12) ++axis;
    }
    if (axis != 1 || !(h > 0.0) || !std::isfinite(h)) {
        std::fprintf(stderr, "stub kernel: row %lld is not a valid %s descriptor\n", (long long)row, what);
        std::abort();
    }
}

uint64_t mix(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

}  // namespace

// shared with the driver, which computes the expected answers
double stub_u01(uint64_t key, uint32_t sid) { return (double)(mix(key ^ mix(sid)) >> 11) * 0x1p-53; }
int64_t stub_budget(const Adaptive &a, double se2)
{
    if (!(se2 < 1e300)) return a.pilot;
    const double want = std::ceil(1e-6 / se2);
    int64_t b = want > (double)a.w_max ? a.w_max : (int64_t)want;
    if (b < a.w_min) b = a.w_min;
    return b < a.pilot ? a.pilot : b;
}

dtn_status launch_nodes(const Plan &P, double *nodes, hipStream_t s)
{
    const int64_t n = (int64_t)P.patches.size();
    const dtn_patch *pp = P.d_patches;
    const int32_t *pc = P.d_patch_class;
    const DevClass *cl = P.d_classes;
    const int64_t *off = P.d_node_off;
    fake_enqueue(s, [=] {
        for (int64_t i = 0; i < n; ++i) {
            const dtn_patch p = pp[i];
            check_frame(p.c, p.n, p.h, i, "patch");
            const int nn = cl[pc[i]].n_nodes;
            for (int k = 0; k < nn; ++k)
                for (int d = 0; d < 3; ++d) nodes[3 * (off[i] + k) + d] = p.c[d] + 1e-3 * (k + 1) * p.n[d];
        }
    });
    return DTN_OK;
}

dtn_status launch_point_nodes(const dtn_point *pts, int64_t n, const PointRule &r, double *nodes, hipStream_t s)
{
    const int nn = r.n_g1 * r.n_g1;
    fake_enqueue(s, [=] {
        for (int64_t i = 0; i < n; ++i) {
            const dtn_point p = pts[i];
            check_frame(p.c, p.n, p.a, i, "point");
            for (int k = 0; k < nn; ++k)
                for (int d = 0; d < 3; ++d) nodes[3 * (i * nn + k) + d] = p.c[d] + 1e-3 * (k + 1) * p.n[d];
        }
    });
    return DTN_OK;
}

dtn_status launch_node_ids(int64_t n_patches, int nn, const uint64_t *pseed, const uint32_t *psid0,
                           const double *pse2, uint64_t *nseed, uint32_t *nsid, double *nse2, hipStream_t s)
{
    fake_enqueue(s, [=] {
        for (int64_t i = 0; i < n_patches * nn; ++i) {
            const int64_t p = i / nn;
            nseed[i] = pseed[p];
            nsid[i] = psid0[p] + (uint32_t)(i % nn);
            nse2[i] = pse2[p];
        }
    });
    return DTN_OK;
}

dtn_status launch_wos_adaptive(const Geometry &, const double *pts, int64_t n, const Adaptive &a, uint64_t,
                               const uint64_t *node_seed, const uint32_t *stream_id, int, double *stats,
                               int64_t *walks_used, int64_t *capped, const Schedule &, hipStream_t s)
{
    // stream-ordered scratch, as the real launcher takes: the budgets go
    // through it
    int64_t *scratch = nullptr;
    hipError_t e = hipMallocAsync((void **)&scratch, sizeof(int64_t) * (size_t)n, s);
    if (e != hipSuccess) return fail(DTN_E_OOM, "stub adaptive: alloc");
    const Adaptive A = a;
    fake_enqueue(s, [=] {
        for (int64_t i = 0; i < n; ++i) scratch[i] = stub_budget(A, A.node_se2[i]);
    });
    fake_enqueue(s, [=] {
        for (int64_t i = 0; i < n; ++i) {
            const double mean = pts[3 * i] + pts[3 * i + 1] + pts[3 * i + 2] + 1e-3 * stub_u01(node_seed[i], stream_id[i]);
            stats[4 * i] = (double)scratch[i];
            stats[4 * i + 1] = mean;
            stats[4 * i + 2] = 1e-4 * (double)scratch[i];
            stats[4 * i + 3] = 20.0 * (double)scratch[i];
            walks_used[i] = scratch[i];
            if (capped) capped[i] = 0;
        }
    });
    e = hipFreeAsync(scratch, s);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, "stub adaptive: free");
    return DTN_OK;
}

dtn_status launch_solve(const Plan &P, const double *stats, int, double *neu, double *nse, hipStream_t s)
{
    const int64_t n = (int64_t)P.patches.size();
    const int32_t *pc = P.d_patch_class;
    const DevClass *cl = P.d_classes;
    const int64_t *noff = P.d_node_off, *poff = P.d_panel_off;
    fake_enqueue(s, [=] {
        for (int64_t i = 0; i < n; ++i) {
            const DevClass &c = cl[pc[i]];
            double m = 0.0;
            for (int k = 0; k < c.n_nodes; ++k) m += stats[4 * (noff[i] + k) + 1];
            m /= c.n_nodes;
            for (int j = 0; j < c.n_panels; ++j) {
                neu[poff[i] + j] = m;
                nse[poff[i] + j] = 1e-3;
            }
        }
    });
    return DTN_OK;
}

dtn_status launch_answer(const Plan &P, const double *neu, const double *stats, const int64_t *used, double *ans,
                         hipStream_t s)
{
    const int64_t n = (int64_t)P.patches.size();
    const dtn_patch *pp = P.d_patches;
    const int32_t *pc = P.d_patch_class;
    const DevClass *cl = P.d_classes;
    const int64_t *noff = P.d_node_off, *poff = P.d_panel_off;
    fake_enqueue(s, [=] {
        for (int64_t i = 0; i < n; ++i) {
            const DevClass &c = cl[pc[i]];
            int64_t w = 0;
            for (int k = 0; k < c.n_nodes; ++k) w += used[noff[i] + k];
            (void)stats;
            ans[4 * i] = neu[poff[i]];
            ans[4 * i + 1] = 1e-3;
            ans[4 * i + 2] = (double)w;
            ans[4 * i + 3] = pp[i].h;
        }
    });
    return DTN_OK;
}

dtn_status launch_point_neumann(const Geometry &, const dtn_point *pts, int64_t n, const PointRule &r,
                                const double *stats, double *out, hipStream_t s)
{
    const int nn = r.n_g1 * r.n_g1;
    fake_enqueue(s, [=] {
        for (int64_t i = 0; i < n; ++i) {
            check_frame(pts[i].c, pts[i].n, pts[i].a, i, "point");
            double m = 0.0;
            for (int k = 0; k < nn; ++k) m += stats[4 * (i * nn + k) + 1];
            out[4 * i] = m / nn;
            out[4 * i + 1] = 1e-3;
            out[4 * i + 2] = out[4 * i + 3] = 0.0;
        }
    });
    return DTN_OK;
}

dtn_status launch_point_answer(const dtn_point *pts, int64_t n, int nn, const int64_t *used, double *out,
                               hipStream_t s)
{
    fake_enqueue(s, [=] {
        for (int64_t i = 0; i < n; ++i) {
            int64_t w = 0;
            for (int k = 0; k < nn; ++k) w += used[i * nn + k];
            out[4 * i + 2] = (double)w;
            out[4 * i + 3] = pts[i].a;
        }
    });
    return DTN_OK;
}

}  // namespace dtn

extern "C" const char *dtn_last_error(void) { return dtn::g_err.c_str(); }
