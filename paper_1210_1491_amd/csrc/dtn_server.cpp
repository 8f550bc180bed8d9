// Query server: continuous batching of Neumann queries over HIP streams.
//
// A query is a set of boundary points.  Each point gets a patch centred on
// it (one patch class for the whole server, h from a ladder h_max 2^-j).  A
// dispatcher thread forms a batch from the queued queries, first come, first
// served: as many as fit in the largest batch (max_points points) and, with
// the batches in flight, under the device-memory budget.  A batch runs the
// whole path on one stream as single launches over all its patches: nodes,
// per-node walk identities (each query's seed, node index within the query,
// SE target), adaptive walks (pilot, budgets, remainder, merge), the
// collocation solve, the central-disk answers and the copy back, all
// stream-ordered, with its device memory from the stream-ordered pool.  A
// host function enqueued behind the batch copies each query's answers out of
// pinned staging, records the completions and releases the stream and the
// memory, so the next batch can start while others are still in flight.
//
// Under graph replay the device pass of a batch is padded to a size bucket
// and recorded once per stream and bucket into a HIP graph (stream capture,
// thread-local mode, on the dispatcher thread); later batches of the bucket
// refill the stream's pinned staging and replay it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "dtn_internal.h"
#include "dtn_point_rule.h"

namespace dtn {
namespace {

using Clock = std::chrono::steady_clock;

// Walk schedule of a batch: small chunks (down to one walk per lane) so that
// a small batch still spreads over many waves and finishes quickly; large
// batches get chunks of total / (resident waves x 8) walks anyway.
const Schedule kBatchSchedule{64, 8};

struct Query {
    uint64_t id = 0;
    std::vector<dtn_patch> patches;
    double se = 0.0;
    uint64_t seed = 0;
    double *out = nullptr;
    double t_submit = 0.0, t_start = 0.0;
};

struct Batch {
    std::vector<Query *> qs;
    int64_t n = 0;      // points (patches)
    int64_t rows = 0;   // n padded to its size bucket (n under direct launches)
    int64_t bytes = 0;  // device memory reserved
    int slot = -1;
};

// Pinned staging of one stream, sized for the largest batch.
struct Slot {
    hipStream_t stream = nullptr;
    dtn_patch *h_patches = nullptr;  // [max_points]
    uint64_t *h_seed = nullptr;      // [max_points] Philox key per patch
    uint32_t *h_sid0 = nullptr;      // [max_points] query-local index of the patch's first node
    double *h_se2 = nullptr;         // [max_points] squared SE target per patch
    double *h_ans = nullptr;         // [max_points][4]
    std::map<int64_t, hipGraphExec_t> graphs;  // captured device pass per size bucket
    hipStream_t capture = nullptr;  // graph replay: records the passes, never runs work
    bool busy = false;
};

// Offsets of one batch's arrays inside its single device allocation.
struct Layout {
    size_t patches, pseed, psid0, pse2, nodes, nseed, nsid, nse2, stats, used, capped, neu, nse, ans, total;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Layout layout(int64_t n, int64_t nn, int64_t np)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    const size_t nodes = (size_t)(n * nn);
    L.patches = take(sizeof(dtn_patch) * (size_t)n);
    L.pseed = take(sizeof(uint64_t) * (size_t)n);
    L.psid0 = take(sizeof(uint32_t) * (size_t)n);
    L.pse2 = take(sizeof(double) * (size_t)n);
    L.nodes = take(sizeof(double) * 3 * nodes);
    L.nseed = take(sizeof(uint64_t) * nodes);
    L.nsid = take(sizeof(uint32_t) * nodes);
    L.nse2 = take(sizeof(double) * nodes);
    L.stats = take(sizeof(double) * 4 * nodes);
    L.used = take(sizeof(int64_t) * nodes);
    L.capped = take(sizeof(int64_t) * nodes);
    L.neu = take(sizeof(double) * (size_t)(n * np));
    L.nse = take(sizeof(double) * (size_t)(n * np));
    L.ans = take(sizeof(double) * 4 * (size_t)n);
    L.total = o;
    return L;
}

// Rows a batch of n points occupies: n itself under direct launches; under
// graph replay the smallest bucket >= n (n up to 8, then m 2^e with m in
// 5..8, so padding stays under a quarter of the batch), at most max_points.
int64_t padded_rows(const dtn_server_config &c, int64_t n)
{
    if (!c.graph_replay || n <= 8) return n;
    int e = 0;
    while ((int64_t)8 << e < n) ++e;  // 4 2^e < n <= 8 2^e
    const int64_t step = (int64_t)1 << e;
    return std::min((n + step - 1) / step * step, c.max_points);
}

// Device bytes of a batch of n points: its (padded) arrays plus the walk
// kernels' stream-ordered scratch (adaptive statistics and budgets; chunk
// table and partials for up to nodes + 256 CUs x 32 waves x oversub chunks,
// MI355X).
int64_t footprint(const dtn_server_config &c, int64_t n_points)
{
    const int64_t n = padded_rows(c, n_points);
    const bool points = c.n_g1 > 0;
    const int64_t nn = points ? (int64_t)c.n_g1 * c.n_g1 : (int64_t)c.n_theta * c.n_phi;
    const int64_t np = points ? 0 : (int64_t)c.n_rings * c.n_sectors;
    const int64_t nodes = n * nn;
    const int64_t adaptive = nodes * (4 * 8 + 5 * 8);
    const int64_t walk = 8 * (nodes + 1) + 80 + 48 * (nodes + 256 * 32 * (int64_t)kBatchSchedule.oversub + 1);
    return (int64_t)layout(n, nn, np).total + adaptive + walk;
}

double box_distance(const double *x, const double *lo, const double *hi)
{
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double q = std::max({lo[k] - x[k], 0.0, x[k] - hi[k]});
        s += q * q;
    }
    return std::sqrt(s);
}

bool valid_config(const dtn_server_config &c, std::string &why)
{
    if (c.n_streams < 1 || c.n_streams > 16) why = "n_streams outside [1, 16]";
    else if (c.precision != DTN_FP64 && c.precision != DTN_FP32_MIXED) why = "unknown precision";
    else if (c.hbm_budget <= 0) why = "hbm_budget must be positive";
    else if (c.pilot_walks < 2 || c.min_walks < 1 || c.min_walks > c.max_walks || c.max_walks > ((int64_t)1 << 40))
        why = "need pilot_walks >= 2 and 1 <= min_walks <= max_walks <= 2^40";
    else if (!(c.h_max > 0.0) || !std::isfinite(c.h_max)) why = "h_max must be positive";
    else if (c.ladder < 1 || c.ladder > 40) why = "ladder outside [1, 40]";
    else if (c.n_theta < 2 || c.n_theta > 32 || c.n_phi < 4 || c.n_phi > 64 || (c.n_phi & 1) || c.n_rings < 1 ||
             c.n_rings > 16 || c.n_sectors < 2 || c.n_sectors > 32 || c.n_rings * c.n_sectors > 128)
        why = "unsupported patch layout";
    else if (c.max_points < 1 || c.max_points > ((int64_t)1 << 20)) why = "max_points outside [1, 2^20]";
    else if (c.graph_replay != 0 && c.graph_replay != 1) why = "graph_replay must be 0 or 1";
    else if (c.max_batch_queries < 0) why = "max_batch_queries must be >= 0";
    else if (c.n_g1 != 0 && (c.n_g1 < 1 || c.n_g1 > 64 || c.n_g2 < 1 || c.n_g2 > 64 ||
                             !(c.delta_rel > 0.0 && c.delta_rel < 1.0)))
        why = "point mode needs n_g1, n_g2 in [1, 64] and delta_rel in (0, 1)";
    else return true;
    return false;
}

}  // namespace
}  // namespace dtn

using namespace dtn;

struct dtn_server_s {
    Geometry *g = nullptr;
    dtn_server_config cfg{};
    int device = 0;
    DevClass *d_class = nullptr;     // the patch class, [1]
    int32_t *d_zero = nullptr;       // class index of every patch, [max_points]
    int64_t *d_node_off = nullptr;   // i * nodes per patch, [max_points + 1]
    int64_t *d_panel_off = nullptr;  // i * panels per patch, [max_points + 1]
    int64_t nn = 0, np = 0;  // nodes and panels per point
    bool points = false;     // point mode: the single-point estimate, no solve
    PointRule rule;          // point mode's quadrature tables
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Query *> pending;
    std::deque<dtn_query_done> done;
    int64_t in_use = 0;
    int busy = 0;
    bool stop = false;
    std::thread dispatcher;
    Clock::time_point t0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

struct Completion {
    dtn_server_s *S;
    Batch *b;
};

// Finish a batch (lock held): record each query, release the stream and the
// memory.
void finish_locked(dtn_server_s *S, Batch *b, int status)
{
    const double t = S->now();
    for (Query *q : b->qs) {
        dtn_query_done d{};
        d.query_id = q->id;
        d.status = status;
        d.n_points = (int64_t)q->patches.size();
        d.t_submit = q->t_submit;
        d.t_start = q->t_start;
        d.t_done = t;
        S->done.push_back(d);
        delete q;
    }
    S->in_use -= b->bytes;
    if (b->slot >= 0) {
        S->slots[b->slot].busy = false;
        --S->busy;
    }
    delete b;
    S->cv.notify_all();
}

// Host function behind a batch's work on its stream (no HIP calls here).
void on_done(void *arg)
{
    std::unique_ptr<Completion> c((Completion *)arg);
    dtn_server_s *S = c->S;
    Batch *b = c->b;
    const double *ans = S->slots[b->slot].h_ans;
    for (Query *q : b->qs) {
        std::memcpy(q->out, ans, sizeof(double) * 4 * q->patches.size());
        ans += 4 * q->patches.size();
    }
    std::lock_guard<std::mutex> lk(S->mu);
    finish_locked(S, b, DTN_OK);
}

// The device pass of a batch of `rows` patches on stream s, from the slot's
// pinned staging to its answers in pinned staging: every call is
// stream-ordered, so the same sequence runs directly or under capture.
dtn_status record_pass(dtn_server_s *S, Slot &sl, int64_t rows, hipStream_t s)
{
    const int64_t n = rows;
    const Layout L = layout(n, S->nn, S->np);
    char *buf = nullptr;
    hipError_t e = hipMallocAsync((void **)&buf, L.total, s);
    if (e != hipSuccess) return fail(DTN_E_OOM, std::string("server: ") + hipGetErrorString(e));
    Plan P;
    P.geom = S->g;
    P.patches.resize(n);  // launch sizes only; the descriptors are on the device
    P.d_patches = (dtn_patch *)(buf + L.patches);
    P.d_patch_class = S->d_zero;
    P.d_classes = S->d_class;
    P.d_node_off = S->d_node_off;
    P.d_panel_off = S->d_panel_off;
    double *nodes = (double *)(buf + L.nodes), *stats = (double *)(buf + L.stats);
    int64_t *used = (int64_t *)(buf + L.used), *capped = (int64_t *)(buf + L.capped);
    double *neu = (double *)(buf + L.neu), *nse = (double *)(buf + L.nse), *ans = (double *)(buf + L.ans);
    uint64_t *pseed = (uint64_t *)(buf + L.pseed), *nseed = (uint64_t *)(buf + L.nseed);
    uint32_t *psid0 = (uint32_t *)(buf + L.psid0), *nsid = (uint32_t *)(buf + L.nsid);
    double *pse2 = (double *)(buf + L.pse2), *nse2 = (double *)(buf + L.nse2);
    dtn_status st = DTN_OK;
    auto copy = [&](void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
        if (st != DTN_OK) return;
        const hipError_t ec = hipMemcpyAsync(dst, src, bytes, kind, s);
        if (ec != hipSuccess) st = fail(DTN_E_DEVICE, std::string("server: ") + hipGetErrorString(ec));
    };
    copy(P.d_patches, sl.h_patches, (S->points ? sizeof(dtn_point) : sizeof(dtn_patch)) * n, hipMemcpyHostToDevice);
    copy(pseed, sl.h_seed, sizeof(uint64_t) * n, hipMemcpyHostToDevice);
    copy(psid0, sl.h_sid0, sizeof(uint32_t) * n, hipMemcpyHostToDevice);
    copy(pse2, sl.h_se2, sizeof(double) * n, hipMemcpyHostToDevice);
    const dtn_point *d_pts = (const dtn_point *)P.d_patches;
    if (st == DTN_OK) st = S->points ? launch_point_nodes(d_pts, n, S->rule, nodes, s) : launch_nodes(P, nodes, s);
    if (st == DTN_OK) st = launch_node_ids(n, (int)S->nn, pseed, psid0, pse2, nseed, nsid, nse2, s);
    if (st == DTN_OK) {
        Adaptive a{S->cfg.pilot_walks, S->cfg.min_walks, S->cfg.max_walks, 1.0};
        a.node_se2 = nse2;
        st = launch_wos_adaptive(*S->g, nodes, n * S->nn, a, 0, nseed, nsid, S->cfg.precision, stats, used, capped,
                                 kBatchSchedule, s);
    }
    if (S->points) {
        if (st == DTN_OK) st = launch_point_neumann(*S->g, d_pts, n, S->rule, stats, ans, s);
        if (st == DTN_OK) st = launch_point_answer(d_pts, n, (int)S->nn, used, ans, s);
    } else {
        if (st == DTN_OK) st = launch_solve(P, stats, S->cfg.precision, neu, nse, s);
        if (st == DTN_OK) st = launch_answer(P, neu, stats, used, ans, s);
    }
    copy(sl.h_ans, ans, sizeof(double) * 4 * n, hipMemcpyDeviceToHost);
    const hipError_t ef = hipFreeAsync(buf, s);
    if (st == DTN_OK && ef != hipSuccess) st = fail(DTN_E_DEVICE, std::string("server: ") + hipGetErrorString(ef));
    return st;
}

// The slot's graph for `rows`, captured on first use.  The capture records
// on the slot's own capture stream, which never runs work: the stream that
// replays the graph may still be finishing the previous batch's host
// function when the dispatcher gets here.
dtn_status slot_graph(dtn_server_s *S, Slot &sl, int64_t rows, hipGraphExec_t *out)
{
    auto it = sl.graphs.find(rows);
    if (it != sl.graphs.end()) {
        *out = it->second;
        return DTN_OK;
    }
    hipError_t e = hipStreamBeginCapture(sl.capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("server capture: ") + hipGetErrorString(e));
    const dtn_status st = record_pass(S, sl, rows, sl.capture);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(sl.capture, &graph);  // ends the capture on every path
    if (st != DTN_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("server capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("server instantiate: ") + hipGetErrorString(e));
    sl.graphs.emplace(rows, exec);
    *out = exec;
    return DTN_OK;
}

dtn_status enqueue(dtn_server_s *S, Batch *b)
{
    Slot &sl = S->slots[b->slot];
    hipStream_t s = sl.stream;
    const int64_t rows = b->rows;
    {
        int64_t at = 0;
        for (const Query *q : b->qs) {
            const int64_t m = (int64_t)q->patches.size();
            if (S->points) {
                // the staging holds dtn_point records (80 B < sizeof(dtn_patch))
                dtn_point *hp = (dtn_point *)sl.h_patches;
                for (int64_t i = 0; i < m; ++i) {
                    const dtn_patch &pq = q->patches[i];
                    dtn_point &o = hp[at + i];
                    for (int k = 0; k < 3; ++k) {
                        o.c[k] = pq.c[k];
                        o.n[k] = pq.n[k];
                        o.t1[k] = pq.t1[k];
                    }
                    o.a = pq.h;
                }
            } else {
                std::memcpy(sl.h_patches + at, q->patches.data(), sizeof(dtn_patch) * m);
            }
            for (int64_t i = 0; i < m; ++i) {
                sl.h_seed[at + i] = q->seed;
                sl.h_sid0[at + i] = (uint32_t)(i * S->nn);
                sl.h_se2[at + i] = q->se * q->se;
            }
            at += m;
        }
        // padding rows: a valid patch with an infinite SE target (budget =
        // the pilot walks); their answers are never read
        for (; at < rows; ++at) {
            if (S->points) {
                dtn_point *hp = (dtn_point *)sl.h_patches;  // records at the dtn_point stride
                hp[at] = hp[0];
            } else {
                sl.h_patches[at] = sl.h_patches[0];
            }
            sl.h_seed[at] = 0;
            sl.h_sid0[at] = 0;
            sl.h_se2[at] = HUGE_VAL;
        }
    }
    dtn_status st;
    if (!S->cfg.graph_replay) {
        st = record_pass(S, sl, rows, s);
    } else {
        hipGraphExec_t exec = nullptr;
        st = slot_graph(S, sl, rows, &exec);
        if (st == DTN_OK) {
            const hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) st = fail(DTN_E_DEVICE, std::string("server graph launch: ") + hipGetErrorString(e));
        }
    }
    if (st != DTN_OK) return st;
    Completion *c = new Completion{S, b};
    const hipError_t e = hipLaunchHostFunc(s, on_done, c);
    if (e != hipSuccess) {
        delete c;
        return fail(DTN_E_DEVICE, std::string("server: ") + hipGetErrorString(e));
    }
    return DTN_OK;
}

void dispatch_loop(dtn_server_s *S)
{
    (void)hipSetDevice(S->device);
    (void)device_cus();  // device properties read here, outside any capture
    std::unique_lock<std::mutex> lk(S->mu);
    const int ns = (int)S->slots.size();
    auto fits = [&](int64_t points) { return S->in_use + footprint(S->cfg, points) <= S->cfg.hbm_budget; };
    for (;;) {
        S->cv.wait(lk, [&] {
            return S->stop ||
                   (!S->pending.empty() && S->busy < ns && fits((int64_t)S->pending.front()->patches.size()));
        });
        if (S->stop) return;
        // first come, first served: the head, then the queries behind it while
        // the batch stays within max_points and the budget
        Batch *b = new Batch();
        const double t = S->now();
        while (!S->pending.empty()) {
            Query *q = S->pending.front();
            const int64_t m = (int64_t)q->patches.size();
            if (!b->qs.empty() && (b->n + m > S->cfg.max_points || !fits(b->n + m) ||
                                   (S->cfg.max_batch_queries > 0 && (int64_t)b->qs.size() >= S->cfg.max_batch_queries)))
                break;
            S->pending.pop_front();
            q->t_start = t;
            b->qs.push_back(q);
            b->n += m;
        }
        b->bytes = footprint(S->cfg, b->n);
        b->rows = padded_rows(S->cfg, b->n);
        int slot = 0;
        while (S->slots[slot].busy) ++slot;
        S->slots[slot].busy = true;
        ++S->busy;
        S->in_use += b->bytes;
        b->slot = slot;
        lk.unlock();
        const dtn_status st = enqueue(S, b);
        lk.lock();
        if (st != DTN_OK) finish_locked(S, b, st);
    }
}

// Patch centred on a boundary point; false with a reason when none fits.
bool place_patch(const dtn_server_s *S, const double *x, const double *nrm, dtn_patch &p, std::string &why)
{
    const Geometry &G = *S->g;
    int k = -1;
    for (int a = 0; a < 3; ++a)
        if (std::fabs(std::fabs(nrm[a]) - 1.0) < 1e-12) k = a;
    if (k < 0 || std::fabs(nrm[(k + 1) % 3]) > 1e-12 || std::fabs(nrm[(k + 2) % 3]) > 1e-12) {
        why = "normal is not an axis direction";
        return false;
    }
    const double sgn = nrm[k] > 0 ? 1.0 : -1.0;
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    const double *lo = G.dev.lo, *hi = G.dev.hi;
    const double scale = 1.0 + std::max({std::fabs(lo[0]), std::fabs(lo[1]), std::fabs(lo[2]), std::fabs(hi[0]),
                                         std::fabs(hi[1]), std::fabs(hi[2])});
    const double tol = 1e-9 * scale;
    auto within = [&](const double *rlo, const double *rhi) {
        return x[a] >= rlo[a] - tol && x[a] <= rhi[a] + tol && x[b] >= rlo[b] - tol && x[b] <= rhi[b] + tol;
    };
    int own = -2;
    double plane = 0.0;
    const double *rlo = nullptr, *rhi = nullptr;
    const double outer = sgn < 0 ? lo[k] : hi[k];
    if (std::fabs(x[k] - outer) <= tol && within(lo, hi)) {
        own = -1;
        plane = outer;
        rlo = lo;
        rhi = hi;
    }
    for (int i = 0; i < G.dev.n_holes && own == -2; ++i) {
        const double *hl = &G.holes[6 * i], *hh = hl + 3;
        const double hp = sgn > 0 ? hl[k] : hh[k];  // the outward normal of Omega points into the hole
        if (std::fabs(x[k] - hp) <= tol && within(hl, hh)) {
            own = i;
            plane = hp;
            rlo = hl;
            rhi = hh;
        }
    }
    if (own == -2) {
        why = "point is not on a face with this outward normal";
        return false;
    }
    double c[3] = {x[0], x[1], x[2]};
    c[k] = plane;
    double cap = std::min({c[a] - rlo[a], rhi[a] - c[a], c[b] - rlo[b], rhi[b] - c[b]});
    for (int k2 = 0; k2 < 3; ++k2) {
        if (!(own == -1 && k2 == k && sgn < 0)) cap = std::min(cap, std::fabs(c[k2] - lo[k2]));
        if (!(own == -1 && k2 == k && sgn > 0)) cap = std::min(cap, std::fabs(hi[k2] - c[k2]));
    }
    for (int i = 0; i < G.dev.n_holes; ++i)
        if (i != own) cap = std::min(cap, box_distance(c, &G.holes[6 * i], &G.holes[6 * i + 3]));
    double h = S->cfg.h_max;
    int j = 0;
    while (j < S->cfg.ladder && !(h <= cap * (1.0 - 1e-9))) {
        h *= 0.5;
        ++j;
    }
    if (j == S->cfg.ladder) {
        why = "too close to an edge or another surface for the smallest patch of the ladder";
        return false;
    }
    for (int q = 0; q < 3; ++q) {
        p.c[q] = c[q];
        p.n[q] = q == k ? sgn : 0.0;
        p.t1[q] = q == a ? 1.0 : 0.0;
    }
    p.h = h;
    p.n_theta = S->cfg.n_theta;
    p.n_phi = S->cfg.n_phi;
    p.n_rings = S->cfg.n_rings;
    p.n_sectors = S->cfg.n_sectors;
    return plane_patch_ok(G, p, why);
}

}  // namespace

extern "C" {

int64_t dtn_server_footprint(const dtn_server_config *cfg, int64_t n_points)
{
    std::string why;
    if (!cfg || n_points < 0 || !valid_config(*cfg, why)) return -1;
    return footprint(*cfg, n_points);
}

dtn_status dtn_server_create(dtn_geometry g, const dtn_server_config *cfg, dtn_server *out)
{
    const std::string at = "dtn_server_create: ";
    try {
        if (!g || !cfg || !out) return fail(DTN_E_ARG, at + "NULL argument");
        *out = nullptr;
        std::string why;
        if (!valid_config(*cfg, why)) return fail(DTN_E_ARG, at + why);
#ifndef DTN_SERVER_GRAPH_REPLAY
        if (cfg->graph_replay)
            return fail(DTN_E_ARG, at + "graph replay is switched off (a serving run with it crashed the host "
                                        "process; the cause is not yet shown)");
#endif
        Geometry *G = &g->g;
        if (G->dev.kind != DTN_BOX && G->dev.kind != DTN_BOX_MINUS_BOXES)
            return fail(DTN_E_ARG, at + "only box domains (with or without holes) are served");
        std::unique_ptr<dtn_server_s> S(new dtn_server_s());
        S->g = G;
        S->cfg = *cfg;
        S->points = cfg->n_g1 > 0;
        S->nn = S->points ? (int64_t)cfg->n_g1 * cfg->n_g1 : (int64_t)cfg->n_theta * cfg->n_phi;
        S->np = S->points ? 0 : (int64_t)cfg->n_rings * cfg->n_sectors;
        hipError_t e = hipGetDevice(&S->device);
        if (e != hipSuccess) return fail(DTN_E_DEVICE, at + hipGetErrorString(e));
        DevClass cls{};
        dtn_status st = plane_class(cfg->n_theta, cfg->n_phi, cfg->n_rings, cfg->n_sectors, cls);
        if (st != DTN_OK) return st;
        const int64_t mp = cfg->max_points;
        std::vector<int64_t> noff(mp + 1), poff(mp + 1);
        for (int64_t i = 0; i <= mp; ++i) {
            noff[i] = i * S->nn;
            poff[i] = i * S->np;
        }
        auto cleanup = [&]() {
            free_point_rule(S->rule);
            (void)hipFree(S->d_class);
            (void)hipFree(S->d_zero);
            (void)hipFree(S->d_node_off);
            (void)hipFree(S->d_panel_off);
            for (Slot &sl : S->slots) {
                for (auto &kv : sl.graphs) (void)hipGraphExecDestroy(kv.second);
                if (sl.stream) (void)hipStreamDestroy(sl.stream);
                if (sl.capture) (void)hipStreamDestroy(sl.capture);
                if (sl.h_patches) (void)hipHostFree(sl.h_patches);
                if (sl.h_seed) (void)hipHostFree(sl.h_seed);
                if (sl.h_sid0) (void)hipHostFree(sl.h_sid0);
                if (sl.h_se2) (void)hipHostFree(sl.h_se2);
                if (sl.h_ans) (void)hipHostFree(sl.h_ans);
            }
        };
        e = hipMalloc((void **)&S->d_class, sizeof(DevClass));
        if (e == hipSuccess) e = hipMemcpy(S->d_class, &cls, sizeof(DevClass), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc((void **)&S->d_zero, sizeof(int32_t) * mp);
        if (e == hipSuccess) e = hipMemset(S->d_zero, 0, sizeof(int32_t) * mp);
        if (e == hipSuccess) e = hipMalloc((void **)&S->d_node_off, sizeof(int64_t) * (mp + 1));
        if (e == hipSuccess)
            e = hipMemcpy(S->d_node_off, noff.data(), sizeof(int64_t) * (mp + 1), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc((void **)&S->d_panel_off, sizeof(int64_t) * (mp + 1));
        if (e == hipSuccess)
            e = hipMemcpy(S->d_panel_off, poff.data(), sizeof(int64_t) * (mp + 1), hipMemcpyHostToDevice);
        S->slots.resize(cfg->n_streams);
        for (Slot &sl : S->slots) {
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e == hipSuccess && cfg->graph_replay) e = hipStreamCreateWithFlags(&sl.capture, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_patches, sizeof(dtn_patch) * mp);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_seed, sizeof(uint64_t) * mp);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_sid0, sizeof(uint32_t) * mp);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_se2, sizeof(double) * mp);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_ans, sizeof(double) * 4 * mp);
        }
        if (e != hipSuccess) {
            cleanup();
            return fail(DTN_E_OOM, at + hipGetErrorString(e));
        }
        if (S->points) {
            st = make_point_rule(cfg->n_g1, cfg->n_g2, cfg->delta_rel, S->rule);
            if (st != DTN_OK) {
                cleanup();
                return st;
            }
        }
        S->t0 = Clock::now();
        dtn_server_s *raw = S.get();
        S->dispatcher = std::thread(dispatch_loop, raw);
        *out = S.release();
        return DTN_OK;
    } catch (...) {
        return fail(DTN_E_OOM, at + "exception");
    }
}

void dtn_server_destroy(dtn_server s)
{
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->dispatcher.joinable()) s->dispatcher.join();
    {
        // queries in flight still complete through their host functions
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv.wait(lk, [&] { return s->busy == 0; });
        for (Query *q : s->pending) delete q;
        s->pending.clear();
    }
    for (Slot &sl : s->slots) {
        (void)hipStreamSynchronize(sl.stream);
        for (auto &kv : sl.graphs) (void)hipGraphExecDestroy(kv.second);
        (void)hipStreamDestroy(sl.stream);
        if (sl.capture) (void)hipStreamDestroy(sl.capture);
        (void)hipHostFree(sl.h_patches);
        (void)hipHostFree(sl.h_seed);
        (void)hipHostFree(sl.h_sid0);
        (void)hipHostFree(sl.h_se2);
        (void)hipHostFree(sl.h_ans);
    }
    free_point_rule(s->rule);
    (void)hipFree(s->d_class);
    (void)hipFree(s->d_zero);
    (void)hipFree(s->d_node_off);
    (void)hipFree(s->d_panel_off);
    delete s;
}

double dtn_server_clock(dtn_server s) { return s ? s->now() : -1.0; }

dtn_status dtn_server_submit(dtn_server s, uint64_t query_id, const double *pts, const double *normals, int64_t n,
                             double se_target, uint64_t seed, double *out)
{
    const std::string at = "dtn_server_submit: ";
    try {
        if (!s || !pts || !normals || !out) return fail(DTN_E_ARG, at + "NULL argument");
        if (n < 1 || n > s->cfg.max_points) return fail(DTN_E_ARG, at + "n outside [1, max_points]");
        if (!(se_target > 0.0) || !std::isfinite(se_target) || !(se_target * se_target > 0.0))
            return fail(DTN_E_ARG, at + "se_target must be positive and finite");
        std::unique_ptr<Query> q(new Query());
        q->id = query_id;
        q->se = se_target;
        q->seed = seed;
        q->out = out;
        q->patches.resize(n);
        std::string why;
        for (int64_t i = 0; i < n; ++i)
            if (!place_patch(s, pts + 3 * i, normals + 3 * i, q->patches[i], why))
                return fail(DTN_E_ARG, at + "point " + std::to_string(i) + ": " + why);
        if (footprint(s->cfg, n) > s->cfg.hbm_budget)
            return fail(DTN_E_OOM, at + "query exceeds the device memory budget");
        std::lock_guard<std::mutex> lk(s->mu);
        q->t_submit = s->now();
        s->pending.push_back(q.release());
        s->cv.notify_all();
        return DTN_OK;
    } catch (...) {
        return fail(DTN_E_OOM, at + "exception");
    }
}

dtn_status dtn_server_wait(dtn_server s, int64_t max_n, double timeout_s, dtn_query_done *done, int64_t *n_out)
{
    if (!s || !done || !n_out || max_n < 1) return fail(DTN_E_ARG, "dtn_server_wait: bad argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] { return !s->done.empty(); };
    if (timeout_s < 0) s->cv.wait(lk, ready);
    else s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    int64_t k = 0;
    while (k < max_n && !s->done.empty()) {
        done[k++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = k;
    return DTN_OK;
}

}  // extern "C"
