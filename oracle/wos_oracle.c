/*
 * Oracle for the walk-on-spheres (WOS) step of the BIE-WOS method.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, FP64 CPU
 * statement of what the GPU path must compute.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may build or call it.
 * It shares no code, header, table or constant generator with the HIP
 * library, and it includes nothing from it.
 *
 * What it computes (Yan, Cai & Zeng, "A parallel method for solving Laplace
 * equations with Dirichlet data using local boundary integral equations and
 * random walks"):
 *   - the Feynman-Kac / harmonic-measure representation of u (Sec. 2,
 *     eq. bw13): u(x) is the mean of the Dirichlet data phi at the exit point;
 *   - its sampling by walk on spheres with an epsilon absorption shell
 *     (Sec. 2, text after Fig. fig_wos): jump to a uniform point on the largest
 *     sphere that stays in the domain, until the distance to the boundary drops
 *     below epsilon, then record phi there;
 *   - the node estimator of Sec. 5.1.2, eq. bw87 (mean of the recorded phi),
 *     extended with the unbiased variance so that a standard error is known.
 *
 * Readings taken where the paper is silent:
 *   - phi is recorded at the closest boundary point of the absorbed position
 *     (phi only exists on the boundary);
 *   - uniform directions by Archimedes' hat-box theorem:
 *     z = 1 - 2 u1, s = sqrt(1 - z^2) = 2 sqrt(u1 (1 - u1)), angle = 2 pi u2;
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11),
 *     key = seed, counter = (walk index lo, walk index hi, draw index,
 *     stream id); one call feeds two steps (words 0,1 then 2,3);
 *     32-bit word k maps to the FP64 uniform (k + 1/2) 2^-32;
 *   - a walk that reaches max_steps is scored at its closest boundary point
 *     and counted as capped;
 *   - the node statistics are shifted sums (shift = phi at the node's closest
 *     boundary point) accumulated with Neumaier's compensated summation;
 *   - half space z > 0 (the exterior domain of the flat-boundary tests of
 *     Sec. 5.1.3): the distance to the boundary is z; a walk that reaches the
 *     large truncation sphere |x - ball_c| >= trunc_r is taken to have gone
 *     to infinity (Sec. 5.1.3, the sphere of radius 1e5) and scores u = 0
 *     there, the limit of data that decay at infinity.  The sphere is tested first at
 *     every position (start and after every jump), then the shell, then the
 *     step cap;
 *   - the exterior of a thin disk (Sec. 5.1.3, Test 4): all of space minus
 *     the closed disk {z = 0, x^2 + y^2 <= disk_r^2}; the distance is that to
 *     the disk, the closest point its projection, and the truncation sphere
 *     applies as for the half space;
 *   - tabulated Dirichlet data on a box (no closed form): a grid of values on
 *     each face (-x,+x,-y,+y,-z,+z), uniform in the face's two coordinates
 *     a = (k+1) mod 3 (tab_n0 nodes) and b = (k+2) mod 3 (tab_n1 nodes),
 *     bilinear interpolation in the cell holding the point; a point takes the
 *     nearest face (ties: the lowest index), and the cell index is clamped to
 *     the grid;
 *   - the exterior of a ball (Sec. 5.2, the big sphere): |x - ball_c| >
 *     ball_r, distance |x - ball_c| - ball_r, closest point on the sphere,
 *     the truncation sphere as above.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared wos_oracle.c -lm (see build.py).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- geometry */

enum { OG_BALL = 0, OG_BOX = 1, OG_BOX_MINUS_BOXES = 2, OG_HALF_SPACE = 3, OG_DISK = 4, OG_BALL_EXTERIOR = 5 };
enum { OG_DATA_QUADRATIC = 0, OG_DATA_SOURCES = 1, OG_DATA_TABLE = 2 };

typedef struct {
    int32_t kind;
    int32_t data_kind;
    double ball_c[3];
    double ball_r;
    double box_lo[3];
    double box_hi[3];
    int32_t n_holes;
    int32_t n_src;
    const double *holes; /* [n_holes][6] = lo xyz, hi xyz */
    const double *src;   /* [n_src][4]   = x y z q        */
    double quad[10];     /* c0 + c.x + x^T A x, see og_phi  */
    double eps;
    int64_t max_steps;
    double disk_r;       /* OG_DISK: radius of the disk in z = 0 */
    double trunc_r;      /* unbounded kinds: truncation sphere |x - ball_c| = trunc_r */
    int32_t tab_n0, tab_n1;
    const double *tab;   /* OG_DATA_TABLE: [6][tab_n0][tab_n1] */
} og_geom;

/* Dirichlet data phi(x).
 * Quadratic: c0 + c1 x + c2 y + c3 z + c4 x^2 + c5 y^2 + c6 z^2
 *            + c7 xy + c8 yz + c9 xz   (harmonic when c4 + c5 + c6 = 0).
 * Sources:   sum_k q_k / |x - s_k|. */
/* Bilinear interpolation of the face tables (see the header). */
static double og_phi_table(const og_geom *g, const double x[3])
{
    int f = 0;
    double best = INFINITY;
    for (int k = 0; k < 3; ++k) {
        double dlo = fabs(x[k] - g->box_lo[k]), dhi = fabs(g->box_hi[k] - x[k]);
        if (dlo < best) { best = dlo; f = 2 * k; }
        if (dhi < best) { best = dhi; f = 2 * k + 1; }
    }
    const int k = f / 2, a = (k + 1) % 3, b = (k + 2) % 3;
    const int n0 = g->tab_n0, n1 = g->tab_n1;
    const double sa = (double)(n0 - 1) / (g->box_hi[a] - g->box_lo[a]);
    const double sb = (double)(n1 - 1) / (g->box_hi[b] - g->box_lo[b]);
    const double s = (x[a] - g->box_lo[a]) * sa, t = (x[b] - g->box_lo[b]) * sb;
    int i = (int)floor(s), j = (int)floor(t);
    if (i < 0) i = 0;
    if (i > n0 - 2) i = n0 - 2;
    if (j < 0) j = 0;
    if (j > n1 - 2) j = n1 - 2;
    const double fs = s - i, ft = t - j;
    const double *T = g->tab + (size_t)f * n0 * n1;
    const double v00 = T[(size_t)i * n1 + j], v10 = T[(size_t)(i + 1) * n1 + j];
    const double v01 = T[(size_t)i * n1 + j + 1], v11 = T[(size_t)(i + 1) * n1 + j + 1];
    return (1.0 - fs) * ((1.0 - ft) * v00 + ft * v01) + fs * ((1.0 - ft) * v10 + ft * v11);
}

double og_phi(const og_geom *g, const double x[3])
{
    if (g->data_kind == OG_DATA_TABLE) return og_phi_table(g, x);
    if (g->data_kind == OG_DATA_QUADRATIC) {
        const double *c = g->quad;
        return c[0] + c[1] * x[0] + c[2] * x[1] + c[3] * x[2] + c[4] * x[0] * x[0] +
               c[5] * x[1] * x[1] + c[6] * x[2] * x[2] + c[7] * x[0] * x[1] +
               c[8] * x[1] * x[2] + c[9] * x[0] * x[2];
    }
    double s = 0.0;
    for (int k = 0; k < g->n_src; ++k) {
        const double *q = g->src + 4 * k;
        double dx = x[0] - q[0], dy = x[1] - q[1], dz = x[2] - q[2];
        s += q[3] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    return s;
}

/* Distance from x (inside the domain) to the boundary, and the closest
 * boundary point p.  Ties between surfaces go to the lowest surface index:
 * outer faces -x,+x,-y,+y,-z,+z, then holes in input order. */
double og_dist_proj(const og_geom *g, const double x[3], double p[3])
{
    if (g->kind == OG_HALF_SPACE) {
        if (p) { p[0] = x[0]; p[1] = x[1]; p[2] = 0.0; }
        return x[2];
    }
    if (g->kind == OG_DISK) {
        double rho = sqrt(x[0] * x[0] + x[1] * x[1]);
        if (rho <= g->disk_r) {
            if (p) { p[0] = x[0]; p[1] = x[1]; p[2] = 0.0; }
            return fabs(x[2]);
        }
        double e = rho - g->disk_r;
        if (p) { p[0] = x[0] * (g->disk_r / rho); p[1] = x[1] * (g->disk_r / rho); p[2] = 0.0; }
        return sqrt(e * e + x[2] * x[2]);
    }
    if (g->kind == OG_BALL_EXTERIOR) {
        double v[3] = {x[0] - g->ball_c[0], x[1] - g->ball_c[1], x[2] - g->ball_c[2]};
        double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (p)
            for (int k = 0; k < 3; ++k) p[k] = g->ball_c[k] + g->ball_r * v[k] / r;
        return r - g->ball_r;
    }
    if (g->kind == OG_BALL) {
        double v[3] = {x[0] - g->ball_c[0], x[1] - g->ball_c[1], x[2] - g->ball_c[2]};
        double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (p) {
            if (r > 0.0) {
                for (int k = 0; k < 3; ++k) p[k] = g->ball_c[k] + g->ball_r * v[k] / r;
            } else {
                p[0] = g->ball_c[0] + g->ball_r; p[1] = g->ball_c[1]; p[2] = g->ball_c[2];
            }
        }
        return g->ball_r - r;
    }
    /* outer box, interior distance */
    double best = INFINITY;
    int best_face = 0;
    for (int k = 0; k < 3; ++k) {
        double dlo = x[k] - g->box_lo[k];
        double dhi = g->box_hi[k] - x[k];
        if (dlo < best) { best = dlo; best_face = 2 * k; }
        if (dhi < best) { best = dhi; best_face = 2 * k + 1; }
    }
    int best_hole = -1;
    if (g->kind == OG_BOX_MINUS_BOXES) {
        for (int i = 0; i < g->n_holes; ++i) {
            const double *h = g->holes + 6 * i;
            double q2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double c = 0.5 * (h[k] + h[3 + k]);
                double e = 0.5 * (h[3 + k] - h[k]);
                double q = fabs(x[k] - c) - e;
                if (q > 0.0) q2 += q * q;
            }
            double d = sqrt(q2);
            if (d < best) { best = d; best_hole = i; }
        }
    }
    if (p) {
        p[0] = x[0]; p[1] = x[1]; p[2] = x[2];
        if (best_hole < 0) {
            int k = best_face / 2;
            p[k] = (best_face & 1) ? g->box_hi[k] : g->box_lo[k];
        } else {
            const double *h = g->holes + 6 * best_hole;
            int inside = 1;
            for (int k = 0; k < 3; ++k) {
                if (x[k] < h[k]) { p[k] = h[k]; inside = 0; }
                else if (x[k] > h[3 + k]) { p[k] = h[3 + k]; inside = 0; }
            }
            if (inside) {
                /* rounding put x inside the hole: move to the nearest face */
                double bd = INFINITY; int bf = 0;
                for (int k = 0; k < 3; ++k) {
                    double a = x[k] - h[k], b = h[3 + k] - x[k];
                    if (a < bd) { bd = a; bf = 2 * k; }
                    if (b < bd) { bd = b; bf = 2 * k + 1; }
                }
                int k = bf / 2;
                p[k] = (bf & 1) ? h[3 + k] : h[k];
            }
        }
    }
    return best;
}

/* ------------------------------------------------------------------ Philox */

/* Philox4x32-10 as published by Salmon et al. (SC'11): ten rounds of the
 * two-multiplier S-box, the key bumped by the two Weyl constants between
 * rounds. */
#define OG_PHILOX_M0 0xD2511F53u
#define OG_PHILOX_M1 0xCD9E8D57u
#define OG_PHILOX_W0 0x9E3779B9u
#define OG_PHILOX_W1 0xBB67AE85u

void og_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)OG_PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)OG_PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        if (round < 9) { k0 += OG_PHILOX_W0; k1 += OG_PHILOX_W1; }
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double og_u01(uint32_t k) { return ((double)k + 0.5) * (1.0 / 4294967296.0); }

/* Uniform direction on the unit sphere from two uniforms in (0,1). */
void og_direction(double u1, double u2, double w[3])
{
    double z = 1.0 - 2.0 * u1;
    double s = 2.0 * sqrt(u1 * (1.0 - u1));
    double a = 2.0 * M_PI * u2;
    w[0] = s * cos(a);
    w[1] = s * sin(a);
    w[2] = z;
}

/* --------------------------------------------------------------------- WOS */

/* Has x left the truncation sphere of an unbounded domain (gone to infinity)? */
static int og_escaped(const og_geom *g, const double x[3])
{
    if (g->kind != OG_HALF_SPACE && g->kind != OG_DISK && g->kind != OG_BALL_EXTERIOR) return 0;
    double dx = x[0] - g->ball_c[0], dy = x[1] - g->ball_c[1], dz = x[2] - g->ball_c[2];
    return dx * dx + dy * dy + dz * dz >= g->trunc_r * g->trunc_r;
}

/* One walk from x0.  Returns the recorded phi (0 for a walk gone to
 * infinity); *steps and *capped report the walk length and whether the step
 * cap ended it. */
double og_walk(const og_geom *g, const double x0[3], uint64_t seed, uint32_t stream_id,
               uint64_t walk, int64_t *steps, int *capped)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double x[3] = {x0[0], x0[1], x0[2]};
    double p[3];
    uint32_t r[4] = {0, 0, 0, 0};
    int64_t n = 0;
    *capped = 0;
    for (;;) {
        if (og_escaped(g, x)) { *steps = n; return 0.0; }
        double d = og_dist_proj(g, x, p);
        if (d < g->eps) break;
        if (n >= g->max_steps) { *capped = 1; break; }
        if ((n & 1) == 0) {
            uint32_t ctr[4] = {(uint32_t)walk, (uint32_t)(walk >> 32), (uint32_t)(n >> 1), stream_id};
            og_philox4x32_10(ctr, key, r);
        }
        double u1 = og_u01(r[(n & 1) ? 2 : 0]);
        double u2 = og_u01(r[(n & 1) ? 3 : 1]);
        double w[3];
        og_direction(u1, u2, w);
        x[0] += d * w[0];
        x[1] += d * w[1];
        x[2] += d * w[2];
        ++n;
    }
    *steps = n;
    return og_phi(g, p);
}

/* Neumaier's compensated summation. */
typedef struct { double s, c; } og_ksum;
static void og_kadd(og_ksum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double og_kval(const og_ksum *a) { return a->s + a->c; }

/* Node statistics for walks [walk_begin, walk_begin + n_walks) from each
 * point.  Outputs (per point): count, mean, M2 = sum of squared deviations
 * from the mean, total steps, capped walks. */
void og_wos_nodes(const og_geom *g, const double *pts, int64_t n_pts,
                  const int64_t *walk_begin, const int64_t *n_walks, uint64_t seed,
                  const uint32_t *stream_id, double *count, double *mean, double *m2,
                  int64_t *steps, int64_t *capped, int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t i = 0; i < n_pts; ++i) {
        const double *y = pts + 3 * i;
        double p[3];
        og_dist_proj(g, y, p);
        const double shift = og_phi(g, p);
        og_ksum s1 = {0, 0}, s2 = {0, 0};
        int64_t nst = 0, ncap = 0;
        const uint32_t sid = stream_id ? stream_id[i] : (uint32_t)i;
        const int64_t w0 = walk_begin ? walk_begin[i] : 0;
        const int64_t nw = n_walks[i];
        for (int64_t k = 0; k < nw; ++k) {
            int64_t st; int cap;
            double v = og_walk(g, y, seed, sid, (uint64_t)(w0 + k), &st, &cap) - shift;
            og_kadd(&s1, v);
            og_kadd(&s2, v * v);
            nst += st;
            ncap += cap;
        }
        double n = (double)nw;
        double S1 = og_kval(&s1), S2 = og_kval(&s2);
        count[i] = n;
        mean[i] = nw > 0 ? shift + S1 / n : 0.0;
        m2[i] = nw > 0 ? S2 - S1 * S1 / n : 0.0;
        if (m2[i] < 0.0) m2[i] = 0.0;
        steps[i] = nst;
        capped[i] = ncap;
    }
}

/* Scores of individual walks, for distribution tests on small inputs. */
void og_wos_scores(const og_geom *g, const double y[3], uint64_t seed, uint32_t stream_id,
                   int64_t walk_begin, int64_t n_walks, double *score, int64_t *steps)
{
    for (int64_t k = 0; k < n_walks; ++k) {
        int cap;
        score[k] = og_walk(g, y, seed, stream_id, (uint64_t)(walk_begin + k), &steps[k], &cap);
    }
}

/* Batched access for the pins. */
void og_phi_many(const og_geom *g, const double *x, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = og_phi(g, x + 3 * i);
}
void og_dist_proj_many(const og_geom *g, const double *x, int64_t n, double *d, double *p)
{
    for (int64_t i = 0; i < n; ++i) d[i] = og_dist_proj(g, x + 3 * i, p + 3 * i);
}
void og_philox_many(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) og_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}
void og_direction_many(const double *u, int64_t n, double *w)
{
    for (int64_t i = 0; i < n; ++i) og_direction(u[2 * i], u[2 * i + 1], w + 3 * i);
}
int og_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
