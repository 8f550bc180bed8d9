// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dtn.h"

namespace dtn {

// Geometry as the kernels see it: passed by value (lands in SGPRs), with the
// holes and sources in device memory read at wave-uniform addresses.
struct DevGeom {
    int32_t kind;
    int32_t data_kind;
    double c[3];
    double r;
    double lo[3];
    double hi[3];
    int32_t n_holes;
    int32_t n_src;
    const double *hole_ce;  // [n_holes][6]: centre xyz, half-extent xyz
    const double *hole_box; // [n_holes][6]: lo xyz, hi xyz
    const float *hole_f32;  // [n_holes][8]: centre xyz, half-extent xyz, 0, 0 (FP32)
    const double *sincos;   // [256][2]: sin, cos of 2 pi j / 256
    // Grid over the box listing, per cell, the holes that can be nearest
    // (bit i = hole i); NULL when not built (more than 32 holes).
    const uint32_t *cell_mask;  // [cell_n0][cell_n1][cell_n2]
    float cell_inv[3];          // cells per unit length
    float cell_off[3];          // -lo * cell_inv
    float cell_top[3];          // cell_n - 1/2 (clamp before truncation)
    int32_t cell_stride[2];     // cell_n1 * cell_n2, cell_n2
    const double *src;      // [n_src][4]
    double quad[10];
    double eps;
    int64_t max_steps;
    double disk_r;          // DTN_DISK: radius of the disk
    double trunc_r;         // unbounded kinds: truncation sphere |x - c| = trunc_r
    // DTN_DATA_TABULATED: face tables [6][n0][n1]; tab_sc[k] = (n - 1)/(hi - lo)
    // along axis k for the first and second grid axis
    const double *tab;
    int32_t tab_n[2];
    double tab_sc[3][2];
    // Status of the work on this geometry (device, see DevStatus).
    struct DevStatus *status;
    int32_t count_walks;  // box minus holes: add the walk counters (dtn_walk_counters)
};

// Sticky status bits raised by kernels working on a geometry (kFlag*), read
// and cleared by dtn_check, and the walk counters of box-minus-holes walks,
// read and cleared by dtn_walk_counters; *_taken are the snapshots those
// calls take.
struct DevStatus {
    uint32_t flags, flags_taken;
    unsigned long long iters, visits;  // wave iterations, hole distances computed by waves
    unsigned long long iters_taken, visits_taken;
};
constexpr uint32_t kFlagCapped = 1u;  // some walk was ended by the step cap
constexpr uint32_t kFlagNoConv = 2u;  // an FP32-mixed solve did not reach its residual bound

// Per-class operators on the device.  A class is a set of congruent patches
// (same layout and same curvature relative to h); K scales with h.
struct DevClass {
    int32_t n_theta, n_phi, n_rings, n_sectors;
    int32_t n_nodes, n_panels;
    int32_t curved;       // patch on a sphere (double-layer term present)
    int32_t n_dl;         // double-layer quadrature points per panel row
    double rr;            // R / h for curved classes, 0 for plane ones
    const double *node_tab;   // [n_theta*n_phi][3]: local node offsets / h
    const double *col_tab;    // [n_panels][3]: local collocation points / h
    const double *K;          // [n_panels][n_panels] at h = 1, row-major
    const double *LU;         // [n_panels][n_panels] FP64 LU of K (row-major)
    const int32_t *piv;       // [n_panels] row permutation of the LU
    float *LU32;              // [n_panels][n_panels] FP32 LU (device-built)
    int32_t *piv32;           // [n_panels]
    const double *QI;         // [n_panels][n_nodes]
    const double *A2;         // [n_panels][n_nodes]: (K^-1 QI)^2 at h = 1
    const double *dl_pts;     // [n_panels][n_dl][3] local points / h
    const double *dl_w;       // [n_panels][n_dl] weights (kernel x area) at h = 1
    const double *fit;        // [16][n_panels] tile fit (flat classes)
    const double *tile_gl;    // [16][3]: (xi, eta, weight) on [-1,1]^2
    const double *ans_row;    // [n_nodes]: ring-0 mean of the rows of K^-1 QI at h = 1
    // second-kind equation, at h = 1 (scale 1/h): b_i = Q2 u -
    // sum_q s_w phi(s_pts) - c2 phi(x_i); flat classes: sigma = 2 b; curved
    // ones: (1/2 I - D) sigma = b by the LU factors M2_LU
    const double *Q2;         // [n_panels][n_nodes]: Gamma operator with the kernel -d2G_B/dn_x dn_y
    const double *s_pts;      // [n_panels][n_s][3]: local points / h of the regularised S rule
    const double *s_w;        // [n_panels][n_s]: weights x kernel of that rule
    const double *c2;         // [n_panels]: sum_k Q2_ik - sum_q s_w_iq
    int32_t n_s;
    const double *M2_LU;      // [n_panels][n_panels] LU of 1/2 I - D (curved classes; NULL on flat ones)
    const int32_t *M2_piv;    // [n_panels]
    const double *A2s;        // [n_panels][n_nodes]: (M^-1 Q2)^2 (curved classes)
    double k_inf;             // max row sum of |K| at h = 1 (residual bound of the refinement)
};

struct Geometry {
    DevGeom dev{};
    dtn_geometry_desc desc{};
    std::vector<double> holes, src;
    double *d_hole_ce = nullptr, *d_hole_box = nullptr, *d_src = nullptr;
    float *d_hole_f32 = nullptr;
    double *d_sincos = nullptr;
    uint32_t *d_cell_mask = nullptr;
    double *d_tab = nullptr;
    DevStatus *d_status = nullptr;  // see DevGeom::status
    std::vector<uint32_t> cell_mask;
    int device = 0;
};

struct PlanClassHost {
    DevClass dev{};
    std::vector<void *> allocations;
};

struct Plan {
    Geometry *geom = nullptr;
    std::vector<dtn_patch> patches;
    std::vector<int32_t> patch_class;
    std::vector<int64_t> node_off, panel_off;
    int64_t n_nodes = 0, n_panels = 0;
    std::vector<PlanClassHost> classes;
    DevClass *d_classes = nullptr;     // [n_classes]
    dtn_patch *d_patches = nullptr;    // [n_patches]
    int32_t *d_patch_class = nullptr;  // [n_patches]
    int64_t *d_node_off = nullptr;     // [n_patches+1]
    int64_t *d_panel_off = nullptr;    // [n_patches+1]
    bool tiles_ok = false;             // the patches tile the whole boundary of a box (square tiles)
    int max_sweeps = 8;                // FP32-mixed solve: FP32 solves with FP64 residual at most
    int device = 0;
};

// Error reporting (thread-local last message).
void set_error(const std::string &msg);
dtn_status fail(dtn_status s, const std::string &msg);

// Walk schedule: chunks per resident wave and the smallest chunk (walks).
struct Schedule {
    int64_t min_chunk = 512;
    int32_t oversub = 4;
};

// Adaptive walk budget: pilot walks, clamp of the total, target standard
// error (or per-point squared targets, device [n], when node_se2 is set).
struct Adaptive {
    int64_t pilot, w_min, w_max;
    double se;
    const double *node_se2 = nullptr;
};

// Kernel launchers (dtn_wos.hip).
dtn_status launch_wos(const Geometry &g, const double *pts, int64_t n, const int64_t *walks,
                      const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id,
                      int precision, double *stats, int64_t *capped, const Schedule &sc, hipStream_t stream);
dtn_status launch_distance(const Geometry &g, const double *pts, int64_t n, int precision, double *dist,
                           hipStream_t stream);
// launch_wos with the default schedule, its scratch in the library's static
// per-device workspace (no allocation); DTN_E_ARG when n needs more.
dtn_status launch_wos_noalloc(const Geometry &g, const double *pts, int64_t n, const int64_t *walks,
                              const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id, int precision,
                              double *stats, int64_t *capped, hipStream_t stream);
size_t noalloc_workspace_bytes();
size_t noalloc_bytes(int64_t n);  // workspace bytes of a launch over n points (default schedule)
// node_seed: per-point Philox keys (device [n]) or NULL for `seed` everywhere.
dtn_status launch_wos_adaptive(const Geometry &g, const double *pts, int64_t n, const Adaptive &a, uint64_t seed,
                               const uint64_t *node_seed, const uint32_t *stream_id, int precision, double *stats,
                               int64_t *walks_used, int64_t *capped, const Schedule &sc, hipStream_t stream);

// Read and clear the geometry's status bits, or its walk counters, after
// the stream's work (synchronises the stream).
dtn_status take_flags(const Geometry &g, hipStream_t stream, uint32_t &out);
dtn_status take_counters(const Geometry &g, hipStream_t stream, unsigned long long out[2]);

// Kernel launchers (dtn_patch.hip).
dtn_status launch_nodes(const Plan &p, double *nodes, hipStream_t stream);
dtn_status launch_solve(const Plan &p, const double *node_stats, int precision, double *neumann,
                        double *neumann_se, hipStream_t stream);
dtn_status launch_potential(const Plan &p, const double *neumann, const double *targets, int64_t m,
                            double *u_out, hipStream_t stream);
dtn_status launch_lu32(const Plan &p, hipStream_t stream);
// Second-kind equation on flat patches (sigma = 2b, no solve).
dtn_status launch_solve2(const Plan &p, const double *node_stats, double *neumann, double *neumann_se,
                         hipStream_t stream);

// Plan helpers shared with the query server (dtn_capi.cpp).
bool plane_patch_ok(const Geometry &g, const dtn_patch &p, std::string &why);
dtn_status plane_class(int nt, int nf, int nr, int ns, DevClass &out);  // cached, FP32 LU included

// Central-disk answer per patch (dtn_patch.hip): mean of the ring-0 panels'
// sigma, its standard error, the walks spent on the patch and h.
dtn_status launch_answer(const Plan &p, const double *neumann, const double *node_stats, const int64_t *walks_used,
                         double *ans, hipStream_t stream);

// Per-node Philox keys, stream ids and squared SE targets of a batch of
// queries from per-patch values (dtn_patch.hip).
// Compute units of the current device (cached per thread).
int device_cus();
dtn_status launch_node_ids(int64_t n_patches, int nn, const uint64_t *pseed, const uint32_t *psid0,
                           const double *pse2, uint64_t *nseed, uint32_t *nsid, double *nse2, hipStream_t stream);

// Host operator construction (dtn_operators.cpp).
struct ClassOps {
    int n_theta, n_phi, n_rings, n_sectors;
    double rr;  // R/h (0 = plane)
    std::vector<double> node_tab, col_tab, K, LU, QI, A2, dl_pts, dl_w, fit, tile_gl, ans_row;
    std::vector<double> Q2, s_pts, s_w, c2;  // second kind
    std::vector<double> M2, M2_LU, A2s;       // second kind on a sphere: 1/2 I - D, its LU, (M^-1 Q2)^2
    std::vector<int32_t> M2_piv;
    std::vector<int32_t> piv;
    int n_dl = 0, n_s = 0;
};
bool build_class_ops(ClassOps &ops, std::string &err);
// Gauss-Legendre abscissae and weights on [-1, 1] (Newton on the recurrence).
void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w);

}  // namespace dtn

// The opaque handles of the C-ABI.
struct dtn_geometry_s {
    dtn::Geometry g;
};
struct dtn_plan_s {
    dtn::Plan p;
};
