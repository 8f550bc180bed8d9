// Single-point estimate (Sec. 5.1): the quadrature tables and kernel
// launchers shared by point sets and by the query server's point mode.
#pragma once

#include <string>

#include "dtn_internal.h"

namespace dtn {

// Tables at a = 1 (device): the hemisphere rule of eqs. bw83/bw85 and the
// ring rule of eqs. bw68/bw82.
struct PointRule {
    int n_g1 = 0, n_g2 = 0;
    double delta_rel = 0.0;
    double *d_hemi = nullptr;  // [n_g1*n_g1][4]: sin(th) cos(ps), sin(th) sin(ps), cos(th), W at a = 1
    double *d_ring = nullptr;  // [n_g2*n_g2][4]: rho / a, cos(ps), sin(ps), ring weight at a = 1
};

// Builds and uploads the tables (n_g1, n_g2 in [1, 64], delta_rel in (0, 1)).
dtn_status make_point_rule(int n_g1, int n_g2, double delta_rel, PointRule &r);
void free_point_rule(PointRule &r);

// Is the point on a flat part of the boundary with its hemisphere in Omega?
bool point_ok(const Geometry &g, const dtn_point &q, std::string &why);

// Hemisphere nodes of n points (device dtn_point [n]) -> nodes [n nn][3].
dtn_status launch_point_nodes(const dtn_point *pts, int64_t n, const PointRule &r, double *nodes, hipStream_t s);
// (Sigma1' + Sigma2', SE, Sigma1', Sigma2') per point from node statistics.
dtn_status launch_point_neumann(const Geometry &g, const dtn_point *pts, int64_t n, const PointRule &r,
                                const double *stats, double *out, hipStream_t s);
// Serving answers in place: out[p] = (value, SE, walks spent by the point's
// nodes, a), from the (value, SE, ...) rows launch_point_neumann wrote.
dtn_status launch_point_answer(const dtn_point *pts, int64_t n, int nn, const int64_t *used, double *out,
                               hipStream_t s);

}  // namespace dtn
