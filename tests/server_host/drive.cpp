// Drives the query server's host logic (dtn_server.cpp built against the
// host-only HIP stand-in and the stub launchers) through a serving trace:
// queries of 1..max_points boundary points with seeded Poisson-like gaps,
// several streams, direct launches or graph replay, patch or point mode.
// Every answer is checked against the query's own points (the stub values,
// see stubs.cpp); then a server is destroyed with queries in flight.
//   drive <n_streams> <graph_replay 0|1> <point_mode 0|1> <queries> <seed> <max_points>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"
#include "dtn_internal.h"

namespace dtn {
double stub_u01(uint64_t key, uint32_t sid);
int64_t stub_budget(const Adaptive &a, double se2);
}  // namespace dtn

struct Q {
    uint64_t id = 0;
    std::vector<double> pts, nrm, out;
    double se = 0.0;
    uint64_t seed = 0;
    int64_t n = 0;
};

static void make_geometry(dtn_geometry_s &G)
{
    dtn::Geometry &g = G.g;
    g.dev.kind = DTN_BOX_MINUS_BOXES;
    for (int k = 0; k < 3; ++k) {
        g.dev.lo[k] = 0.0;
        g.dev.hi[k] = 4.0;
    }
    g.holes = {1.0, 1.0, 1.0, 1.5, 1.6, 1.7, 2.5, 2.2, 2.4, 3.0, 3.0, 3.0};
    g.dev.n_holes = 2;
}

static dtn_server_config make_config(int streams, int graph, int point, int64_t max_points)
{
    dtn_server_config c{};
    c.n_streams = streams;
    c.precision = DTN_FP32_MIXED;
    c.pilot_walks = 100;
    c.min_walks = 100;
    c.max_walks = 1000000;
    c.h_max = 0.25;
    c.ladder = 16;
    c.n_theta = 8;
    c.n_phi = 16;
    c.n_rings = 4;
    c.n_sectors = 8;
    c.max_points = max_points;
    c.graph_replay = graph;
    c.max_batch_queries = 0;
    c.n_g1 = point ? 6 : 0;
    c.n_g2 = point ? 6 : 0;
    c.delta_rel = point ? 1e-6 : 0.0;
    // room for about two of the largest batches: admission binds
    c.hbm_budget = (int64_t)1 << 40;
    c.hbm_budget = 2 * dtn_server_footprint(&c, max_points) + 1;
    return c;
}

static void make_queries(std::vector<Q> &qs, int nq, uint64_t seed, int64_t max_points)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    qs.resize(nq);
    for (int i = 0; i < nq; ++i) {
        Q &q = qs[i];
        q.id = 1000 + i;
        q.n = std::min<int64_t>(max_points, (int64_t)std::floor(std::exp(U(rng) * std::log((double)max_points))) + (i % 7 == 0 ? 0 : 0));
        if (q.n < 1) q.n = 1;
        q.se = std::pow(10.0, -4.0 + 2.0 * U(rng));
        q.seed = rng();
        q.pts.resize(3 * q.n);
        q.nrm.assign(3 * q.n, 0.0);
        q.out.assign(4 * q.n, -1.0);
        for (int64_t p = 0; p < q.n; ++p) {
            const int f = (int)(U(rng) * 6) % 6, k = f / 2;
            for (int d = 0; d < 3; ++d) q.pts[3 * p + d] = 0.05 + 3.9 * U(rng);
            q.pts[3 * p + k] = (f & 1) ? 4.0 : 0.0;
            q.nrm[3 * p + k] = (f & 1) ? 1.0 : -1.0;
        }
    }
}

static int check(const Q &q, const dtn_server_config &c, int point)
{
    const int nn = point ? c.n_g1 * c.n_g1 : c.n_theta * c.n_phi;
    dtn::Adaptive A{c.pilot_walks, c.min_walks, c.max_walks, 1.0};
    const int64_t budget = dtn::stub_budget(A, q.se * q.se);
    for (int64_t i = 0; i < q.n; ++i) {
        const double *x = &q.pts[3 * i], *nv = &q.nrm[3 * i], *o = &q.out[4 * i];
        double m = 0.0;
        for (int k = 0; k < nn; ++k) {
            double s = 0.0;
            for (int d = 0; d < 3; ++d) s += x[d] + 1e-3 * (k + 1) * nv[d];
            m += s + 1e-3 * dtn::stub_u01(q.seed, (uint32_t)(i * nn + k));
        }
        m /= nn;
        const double ladder = std::log2(c.h_max / o[3]);
        if (!(std::fabs(o[0] - m) <= 1e-12 * (1.0 + std::fabs(m))) || o[1] != 1e-3 || o[2] != (double)(nn * budget) ||
            !(o[3] > 0.0) || std::fabs(ladder - std::round(ladder)) > 1e-12) {
            std::fprintf(stderr, "query %llu point %lld: got (%.17g %g %g %g) want (%.17g 0.001 %lld h)\n",
                         (unsigned long long)q.id, (long long)i, o[0], o[1], o[2], o[3], m, (long long)(nn * budget));
            return 1;
        }
    }
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 7) {
        std::fprintf(stderr, "usage: drive streams graph point queries seed max_points\n");
        return 2;
    }
    const int streams = std::atoi(argv[1]), graph = std::atoi(argv[2]), point = std::atoi(argv[3]);
    const int nq = std::atoi(argv[4]);
    const uint64_t seed = std::strtoull(argv[5], nullptr, 10);
    const int64_t max_points = std::atoll(argv[6]);
    dtn_geometry_s G;
    make_geometry(G);
    const dtn_server_config cfg = make_config(streams, graph, point, max_points);
    std::vector<Q> qs;
    make_queries(qs, nq, seed, max_points);

    dtn_server S = nullptr;
    if (dtn_server_create(&G, &cfg, &S) != DTN_OK) {
        std::fprintf(stderr, "create: %s\n", dtn_last_error());
        return 1;
    }
    std::mt19937_64 rng(seed ^ 0x5eed);
    std::exponential_distribution<double> gap(5000.0);  // mean 200 us between arrivals
    int bad = 0;
    for (Q &q : qs) {
        std::this_thread::sleep_for(std::chrono::duration<double>(gap(rng)));
        const dtn_status st = dtn_server_submit(S, q.id, q.pts.data(), q.nrm.data(), q.n, q.se, q.seed, q.out.data());
        if (st != DTN_OK) {
            std::fprintf(stderr, "submit %llu: %s\n", (unsigned long long)q.id, dtn_last_error());
            ++bad;
        }
    }
    int got = 0;
    std::vector<dtn_query_done> done(64);
    while (got < nq - bad) {
        int64_t k = 0;
        dtn_server_wait(S, (int64_t)done.size(), 60.0, done.data(), &k);
        if (k == 0) {
            std::fprintf(stderr, "timed out with %d of %d queries done\n", got, nq - bad);
            return 1;
        }
        for (int64_t j = 0; j < k; ++j) {
            if (done[j].status != DTN_OK) {
                std::fprintf(stderr, "query %llu ended with status %d\n", (unsigned long long)done[j].query_id,
                             done[j].status);
                ++bad;
            }
            if (!(done[j].t_submit <= done[j].t_start && done[j].t_start <= done[j].t_done)) ++bad;
        }
        got += (int)k;
    }
    for (const Q &q : qs) bad += check(q, cfg, point);
    dtn_server_destroy(S);

    // destroy with queries queued and in flight: queued ones are dropped,
    // those in flight complete through their host functions first
    std::vector<Q> more;
    make_queries(more, 24, seed + 1, max_points);
    if (dtn_server_create(&G, &cfg, &S) != DTN_OK) return 1;
    for (Q &q : more) dtn_server_submit(S, q.id, q.pts.data(), q.nrm.data(), q.n, q.se, q.seed, q.out.data());
    dtn_server_destroy(S);

    const FakeStats fs = fake_stats();
    std::printf("streams %d graph %d point %d: %d queries, %ld stream ops, %ld graph launches, %ld captures "
                "(%ld on a stream with unfinished work), peak device bytes %ld, failures %d\n",
                streams, graph, point, nq, fs.ops, fs.graph_launches, fs.captures, fs.captures_on_busy_stream,
                fs.max_live_device_bytes, bad);
    return bad ? 1 : 0;
}
