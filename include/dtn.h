/*
 * dtn.h -- C-ABI of the MI355X library for the local Dirichlet-to-Neumann
 * (DtN) method of Yan, Cai & Zeng, "A parallel method for solving Laplace
 * equations with Dirichlet data using local boundary integral equations and
 * random walks" (BIE-WOS).
 *
 * The problem (Sec. 2, eqs. bw01 and bw03): given Dirichlet data phi on the
 * boundary of a domain Omega, find the Neumann data du/dn on patches of the
 * boundary, then u anywhere from both.  The method (Sec. 4, the two-step
 * BIE-WOS algorithm):
 *   step 1  u at quadrature nodes on a hemisphere over each patch, by the
 *           Feynman-Kac formula sampled with walk on spheres (Sec. 2, eq. bw13;
 *           node estimator eq. bw87)                         -> dtn_wos_eval
 *   step 2  collocation solve of the local first-kind BIE K sigma = b on the
 *           patch (eqs. bw49-bw51; Sec. 5.2)                 -> dtn_patch_solve
 *   then    u at arbitrary points from eq. bw03              -> dtn_potential
 * and the single-point variant on a flat boundary (Sec. 5.1): du/dn at one
 * point from the regularised hypersingular identity, no solve
 *           hemisphere nodes (eq. bw85)                      -> dtn_points_nodes
 *           Sigma1' + Sigma2' (eqs. bw64, bw83, bw68/bw82)   -> dtn_points_neumann
 *
 * Conventions
 *   - Bulk arrays are DEVICE pointers owned by the caller (e.g. the data_ptr
 *     of a torch tensor on the GPU).  They must stay allocated until the work
 *     enqueued on `stream` has completed.  The library never frees them.
 *   - Descriptors (dtn_geometry_desc, dtn_patch arrays given to
 *     dtn_create_plan) are HOST memory, copied during the call.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Compute calls
 *     only enqueue work; results are valid once the stream has synchronised.
 *   - Errors: a call returns DTN_OK or a negative dtn_status; argument and
 *     shape errors are detected before anything is enqueued.  A HIP error
 *     raised while enqueuing is returned as DTN_E_DEVICE.  dtn_last_error()
 *     gives a message for the last failing call on the calling thread.  No
 *     C++ exception crosses this interface.
 *   - Geometries, plans and point sets are immutable after creation and may
 *     be used from several streams and threads at once.  A plan, a point set
 *     and a server refer to the geometry they were created on: destroy them
 *     before that geometry.
 *   - Randomness: walk k from a point with stream id s uses Philox4x32-10
 *     (Salmon et al., SC'11) with key = seed and counter = (k lo, k hi, draw,
 *     s); one block feeds two steps.  A walk's path is thus a pure function
 *     of (seed, s, k), independent of batching and launch configuration.
 *   - The normal n is the OUTWARD normal of Omega, the domain in which the
 *     walks run; dtn_patch_solve returns du/dn for that n.
 */
#ifndef DTN_H
#define DTN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DTN_OK = 0,
    DTN_E_ARG = -1,         /* invalid argument, shape or descriptor      */
    DTN_E_DEVICE = -2,      /* HIP runtime error                          */
    DTN_E_OOM = -3,         /* device or host allocation failed           */
    DTN_E_UNSUPPORTED = -4, /* valid request this build does not support  */
    DTN_E_NOCONV = -5,      /* iterative refinement did not converge (dtn_check) */
    DTN_E_MAXSTEPS = -6     /* walks ended by the step cap (dtn_check)    */
} dtn_status;

/* Domain kinds (walks run inside Omega). */
enum { DTN_BALL = 0, DTN_BOX = 1, DTN_BOX_MINUS_BOXES = 2, DTN_HALF_SPACE = 3, DTN_DISK = 4, DTN_BALL_EXTERIOR = 5 };
/* Dirichlet data kinds. */
enum { DTN_DATA_HARMONIC_QUADRATIC = 0, DTN_DATA_POINT_SOURCES = 1, DTN_DATA_TABULATED = 2 };
/* Arithmetic of the walks and of the collocation solve. */
enum { DTN_FP64 = 0, DTN_FP32_MIXED = 1 };

typedef struct dtn_geometry_s *dtn_geometry; /* opaque, library-owned */
typedef struct dtn_plan_s *dtn_plan;         /* opaque, library-owned */

/* Domain, Dirichlet data and walk parameters (host memory, copied).
 *   kind DTN_BALL:            |x - ball_c| < ball_r
 *   kind DTN_BOX:             box_lo < x < box_hi
 *   kind DTN_BOX_MINUS_BOXES: the box minus n_holes closed axis-aligned
 *                             boxes holes[i] = (lo x,y,z, hi x,y,z), which
 *                             must lie inside it and not overlap.
 *   kind DTN_HALF_SPACE:      z > 0, boundary the plane z = 0 (the exterior
 *                             domain of Sec. 5.1.3).  A walk that reaches
 *                             the truncation sphere |x - ball_c| >= trunc_r
 *                             (tested at its start and after every jump,
 *                             before the shell) has gone to infinity and
 *                             scores 0, the limit of data that vanish there
 *                             (Sec. 5.1.3 uses trunc_r = 1e5).  Point sources
 *                             must lie in z < 0.
 *   kind DTN_DISK:            all of space minus the closed thin disk
 *                             {z = 0, x^2 + y^2 <= disk_r^2} (Sec. 5.1.3,
 *                             Test 4); the truncation sphere as for the
 *                             half space, which must enclose the disk.  Point
 *                             sources must lie off the disk.
 *   kind DTN_BALL_EXTERIOR:   |x - ball_c| > ball_r (Sec. 5.2, the big
 *                             sphere), the truncation sphere as for the half
 *                             space (trunc_r > ball_r).  Point sources must
 *                             lie inside the ball.
 *   data DTN_DATA_HARMONIC_QUADRATIC: phi = q0 + q1 x + q2 y + q3 z + q4 x^2
 *        + q5 y^2 + q6 z^2 + q7 xy + q8 yz + q9 xz, harmonic (q4+q5+q6 = 0).
 *   data DTN_DATA_POINT_SOURCES: phi = sum_k src[k].q / |x - src[k].xyz|,
 *        src rows (x, y, z, q), every source outside the closed domain.
 *   data DTN_DATA_TABULATED (DTN_BOX only): phi given by tables on the six
 *        faces (order -x,+x,-y,+y,-z,+z), tab host [6][tab_n[0]][tab_n[1]]:
 *        face k's value (i, j) sits at coordinate a = (k/2+1) mod 3 equal to
 *        lo_a + i (hi_a - lo_a)/(tab_n[0] - 1) and b = (k/2+2) mod 3 equal to
 *        lo_b + j (hi_b - lo_b)/(tab_n[1] - 1); phi at a boundary point is
 *        the bilinear interpolant on the nearest face (ties: the lowest
 *        face index).  tab_n[0], tab_n[1] in [2, 4096].
 *   eps: width of the absorbing shell (Sec. 2, epsilon-shell WOS), > 0.
 *   max_steps: a walk still alive after max_steps steps is scored at its
 *        closest boundary point and counted as capped (a walk gone to
 *        infinity is neither capped nor absorbed); 0 <= max_steps <= 2^32 - 1
 *        (a walk's step count is 32-bit).  Capped walks are counted per point
 *        (dtn_wos_eval's `capped`) and raise DTN_E_MAXSTEPS at dtn_check. */
typedef struct {
    int32_t kind;
    int32_t data_kind;
    double ball_c[3];
    double ball_r;
    double box_lo[3];
    double box_hi[3];
    int32_t n_holes;
    int32_t n_src;
    const double *holes; /* host [n_holes][6] */
    const double *src;   /* host [n_src][4]   */
    double quad_coef[10];
    double eps;
    int64_t max_steps;
    double disk_r;  /* DTN_DISK: radius of the disk (other kinds: unused) */
    double trunc_r; /* unbounded kinds: radius of the truncation sphere
                       (centre ball_c); bounded kinds: unused */
    int32_t tab_n[2];  /* DTN_DATA_TABULATED: grid nodes per face axis */
    const double *tab; /* DTN_DATA_TABULATED: host [6][tab_n[0]][tab_n[1]] */
} dtn_geometry_desc;

/* One boundary patch S with its hemisphere (Sec. 4, Fig. fig_biewos).
 *   c: centre on the boundary; n: outward unit normal at c; t1: unit tangent
 *   (t2 = n x t1); h: hemisphere radius = radius of S.
 *   Nodes (step 1): n_theta Gauss-Legendre polar angles on [0, theta_max]
 *   measured from -n (as eq. bw85), times n_phi equispaced azimuths from t1;
 *   theta_max = pi/2 on a plane, arccos(h / 2R) on a sphere of radius R.
 *   Node order: patch-major, theta-major, phi-minor.
 *   Panels (step 2): n_rings x n_sectors polar panels of S (ring-major),
 *   collocation at the parametric panel centres; on a sphere the rings are
 *   uniform in geodesic angle.
 *   Supported: n_theta in [2,32], n_phi even in [4,64], n_rings in [1,16],
 *   n_sectors in [2,32], n_rings*n_sectors <= 128.  96 bytes. */
typedef struct {
    double c[3];
    double n[3];
    double t1[3];
    double h;
    int32_t n_theta, n_phi, n_rings, n_sectors;
} dtn_patch;

/* Message of the last failing call on this thread ("" if none). */
const char *dtn_last_error(void);

/* Library version string.  Its last word is the first 16 hex digits of the
 * SHA-256 of the dtn.h the library was built against (a binding compares it
 * with the header it follows before it calls anything else).  Static
 * storage, never NULL. */
const char *dtn_version(void);

/* Create / destroy a geometry.  Uploads the boundary description and data to
 * the current HIP device.  Errors: DTN_E_ARG for an invalid descriptor
 * (negative sizes, eps <= 0, non-harmonic quadratic, holes outside the box),
 * DTN_E_OOM / DTN_E_DEVICE on allocation or copy failure. */
dtn_status dtn_create_geometry(const dtn_geometry_desc *desc, dtn_geometry *out);
void dtn_destroy_geometry(dtn_geometry g);

/* Step 1: u at n points by walk on spheres (Sec. 2 eq. bw13; eq. bw87).
 *   pts        device [n][3] points inside Omega (a point already within
 *              eps of the boundary ends its walks at once, with 0 steps)
 *   walks      device [n] walks per point (values < 0 are taken as 0)
 *   walk_begin device [n] index of each point's first walk, or NULL for 0
 *              (lets a caller extend an estimate: walks [b, b+walks))
 *   seed       Philox key
 *   stream_id  device [n] per-point stream ids, or NULL for the point index
 *              (then n <= 2^32, so that no two points share a stream)
 *   precision  DTN_FP64 (all in FP64) or DTN_FP32_MIXED (the direction in
 *              FP32: uniforms, square root, sin and cos; distance, epsilon
 *              test, jump, position, projection, scores and sums in FP64)
 *   stats      device [n][4] out: (count, mean, M2, steps), M2 = sum of
 *              squared deviations from the mean; count = 0 gives zeros
 *   capped     device [n] out (int64): walks ended by max_steps, or NULL
 * Scratch is taken from the stream-ordered allocator and released on the
 * same stream.  Errors: DTN_E_ARG (n < 0, NULL pts/walks/stats when n > 0,
 * unknown precision).  Walks ended by the step cap are reported by
 * dtn_check once the stream has run them. */
dtn_status dtn_wos_eval(dtn_geometry g, const double *pts, int64_t n, const int64_t *walks,
                        const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id,
                        int32_t precision, double *stats, int64_t *capped, void *stream);

/* dtn_wos_eval for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, same kernels, same default schedule and the same results
 * bit for bit, but the walk kernels' scratch (chunk offsets, chunk partials,
 * plan segments) lives in a static workspace of the library, 64 MiB per
 * device, held from the first call on a device until the process ends.  The
 * call allocates nothing (no hipMalloc, hipMallocAsync or hipFree); the
 * caller still owns every input and output.  The workspace is shared by every
 * call on the device: calls whose work overlaps on one device (two streams,
 * or two threads) race on it and must be serialised by the caller.  Nothing
 * in it needs to start at zero.
 * Errors: DTN_E_ARG as dtn_wos_eval, and when n needs more workspace than
 * 64 MiB (on a 256-CU MI355X: n > 1,170,119 points); DTN_E_DEVICE when the
 * workspace's address cannot be taken. */
dtn_status dtn_wos_eval_noalloc(dtn_geometry g, const double *pts, int64_t n, const int64_t *walks,
                                const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id,
                                int32_t precision, double *stats, int64_t *capped, void *stream);

/* Distance from n points inside Omega to its boundary, computed as the walk
 * kernels of `precision` compute it (the radius of the largest ball of a walk
 * step, Sec. 2): in FP64 for both; the FP32-mixed walks take the distance to
 * a hole as q * rsq(q^2) without refinement (relative error below 6e-8, less
 * than the 2^-22 by which their jumps are shortened).  For a box minus holes
 * the walk kernels look up, per grid cell, the holes that can be nearest;
 * this call lets a caller check that lookup against a plain minimum over all
 * surfaces.
 *   pts device [n][3]; dist device [n] out.  Errors: DTN_E_ARG. */
dtn_status dtn_boundary_distance(dtn_geometry g, const double *pts, int64_t n, int32_t precision, double *dist,
                                 void *stream);

/* Work schedule of the walk kernels.  The walks of all points form one work
 * list of chunks (point, first walk, walk count), one wave per chunk, in a
 * single launch; the chunk size is C = max(min_chunk, ceil(total walks /
 * (resident waves x oversub))), so a launch has at most n + resident waves x
 * oversub chunks.  Results do not depend on the schedule except for the
 * rounding of the sums (a walk's path is fixed by its counter).
 *   min_chunk  smallest chunk, >= 1 (default 512)
 *   oversub    chunks per resident wave slot, 1..64 (default 4)
 *   reserved   must be 0 */
typedef struct {
    int64_t min_chunk;
    int32_t oversub;
    int32_t reserved;
} dtn_schedule;

/* Adaptive walk budget per point: a pilot of pilot_walks walks estimates the
 * variance s^2 of the scores; the point then gets clamp(ceil(s^2 /
 * se_target^2), min_walks, max_walks) walks in all (never fewer than the
 * pilot), so that its standard error sqrt(s^2 / n) (the error of the node
 * estimate of eq. bw87) meets se_target where the clamp allows.
 *   pilot_walks >= 2; 1 <= min_walks <= max_walks <= 2^40; se_target > 0 */
typedef struct {
    int64_t pilot_walks;
    int64_t min_walks;
    int64_t max_walks;
    double se_target;
} dtn_adaptive;

/* Step 1 with adaptive walk counts (see dtn_adaptive), all on the device:
 * the pilot walks of every point in one launch, the budgets, then the
 * remaining walks of every point in one launch over the uneven work list
 * (walks [pilot, total) of each point), and a merge of the two statistics.
 * The result equals dtn_wos_eval over walks [0, walks_used) up to rounding.
 *   sched      NULL for the default schedule
 *   stats      device [n][4] out as for dtn_wos_eval, over all walks
 *   walks_used device [n] out (int64): total walks of each point
 *   capped     device [n] out (int64) or NULL
 * Other arguments as for dtn_wos_eval.  Errors: DTN_E_ARG for a budget or
 * schedule outside the ranges above, and as dtn_wos_eval. */
dtn_status dtn_wos_adaptive(dtn_geometry g, const double *pts, int64_t n, const dtn_adaptive *budget,
                            uint64_t seed, const uint32_t *stream_id, int32_t precision,
                            const dtn_schedule *sched, double *stats, int64_t *walks_used, int64_t *capped,
                            void *stream);

/* Autotuning support: runs dtn_wos_eval's work (same arguments) once per
 * candidate schedule, `reps` times each after one untimed run, and writes the
 * mean device time per run in milliseconds to ms_out[n_cands] (host).  Blocks
 * until the stream has finished.  stats receives the last run's result.
 * Errors: DTN_E_ARG for n_cands < 1, reps < 1 or an invalid candidate. */
dtn_status dtn_wos_time_schedules(dtn_geometry g, const double *pts, int64_t n, const int64_t *walks,
                                  const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id,
                                  int32_t precision, const dtn_schedule *cands, int32_t n_cands, int32_t reps,
                                  double *stats, float *ms_out, void *stream);

/* A plan holds the patches of a DtN request and, per class of congruent
 * patches, the collocation operators of step 2: the single-layer matrix K
 * (eq. bw50) and its LU factors, the Gamma operator (Poisson kernel against
 * the interpolant of the node values, Sec. 5.2), the double-layer table on
 * curved patches, and the tile fit used by dtn_potential.  Built once on the
 * host and uploaded; the FP32 LU factors are computed on the device.
 *   patches  host [n_patches] (copied)
 * On the sphere of DTN_BALL_EXTERIOR, n points to the centre and Gamma is
 * the part of the sphere |y - c| = h outside the ball (more than a
 * hemisphere), which must stay inside the truncation sphere.
 * Errors: DTN_E_ARG for a patch outside the supported layouts, a patch whose
 * hemisphere is not inside Omega's supported shapes (plane faces of a box,
 * or the sphere of a ball, inside or outside), or n_patches < 1. */
dtn_status dtn_create_plan(dtn_geometry g, const dtn_patch *patches, int64_t n_patches, dtn_plan *out);
void dtn_destroy_plan(dtn_plan p);
/* Most FP32 solves of dtn_patch_solve's FP32-mixed refinement, 0..64
 * (default 8; 0 or 1 cannot reach the bound, so they always raise
 * DTN_E_NOCONV).  Set before enqueuing solves on the plan, not while another
 * thread enqueues them.  Errors: DTN_E_ARG. */
dtn_status dtn_plan_set_max_sweeps(dtn_plan p, int32_t max_sweeps);

/* Status of the work done on a geometry (Sec. 2's capped walks; Sec. 5.2's
 * collocation solve).  Waits for the work enqueued on `stream`, then reads
 * and clears the geometry's status bits, raised by any completed work on it
 * (every plan, point set and server of the geometry, every stream: to cover
 * other streams, synchronise them first):
 *   DTN_E_NOCONV    an FP32-mixed solve missed its residual bound
 *   DTN_E_MAXSTEPS  some walk was ended by the step cap
 *   DTN_OK          neither.
 * Not to be called while a stream capture is recording on `stream`.
 * Errors: DTN_E_ARG (NULL), DTN_E_DEVICE. */
dtn_status dtn_check(dtn_geometry g, void *stream);

/* Work counters of the walks on a box minus holes (diagnostic, for the
 * roofline of the walk kernel).  Waits for the work enqueued on `stream`,
 * reads and clears the counters into out (if not NULL), then switches
 * counting on (enable = 1) or off (0, the default) for walk launches
 * enqueued on this geometry afterwards.  While counting is on, each chunk of
 * walks adds, with two device-wide atomics (0.07 % of the walk time measured
 * on the box-with-holes workload),
 *   out[0]  wave iterations (each computes one distance per lane of its wave)
 *   out[1]  hole distances computed per wave: the sum over wave iterations
 *           of the holes listed for the cells of the wave's walking lanes
 *           (every hole for more than 32 holes).
 * Zero for other domains.  Not while another thread enqueues walks on the
 * geometry.  Errors: DTN_E_ARG (NULL geometry, enable not 0 or 1),
 * DTN_E_DEVICE. */
dtn_status dtn_walk_counters(dtn_geometry g, void *stream, int32_t enable, int64_t out[2]);

/* Sizes of a plan: total nodes and total panels over its patches. */
int64_t dtn_plan_num_nodes(dtn_plan p);
int64_t dtn_plan_num_panels(dtn_plan p);

/* Hemisphere nodes of every patch of the plan (device [num_nodes][3] out). */
dtn_status dtn_patch_nodes(dtn_plan p, double *nodes, void *stream);

/* Step 2: Neumann data on every panel of every patch (eqs. bw49-bw51):
 *   b = phi(x)/2 + DL(x) - sum_k (Q.I)_k u_k,  K sigma = b,
 * DL the double-layer integral of phi over S (zero on plane patches), u_k the
 * node means, and SE(sigma) = sqrt(sum_k A_k^2 SE_k^2), A = K^-1 (Q.I).
 *   node_stats device [num_nodes][4] from dtn_wos_eval, node order
 *   precision  DTN_FP64: FP64 LU solve; DTN_FP32_MIXED: FP32 LU factors
 *              (computed on the device with MFMA) + iterative refinement
 *              with the residual b - K sigma in FP64, until the norm-wise
 *              backward error |r|_inf <= P 2^-53 (|K|_inf |sigma|_inf +
 *              |b|_inf) (P panels), at most max_sweeps FP32 solves (default
 *              8, see dtn_plan_set_max_sweeps); a patch that misses the bound
 *              (or whose residual is not finite) keeps its last iterate and
 *              raises DTN_E_NOCONV at dtn_check
 *   neumann    device [num_panels] out, patch-major, ring-major
 *   neumann_se device [num_panels] out, or NULL */
dtn_status dtn_patch_solve(dtn_plan p, const double *node_stats, int32_t precision, double *neumann,
                           double *neumann_se, void *stream);

/* Step 2 by the second-kind equation (Sec. 4, eqs. bw53-bw59), at the same
 * collocation points as dtn_patch_solve:
 *   (1/2 I - D) sigma = b,   D[sigma](x) = int_S dG/dn_x sigma ds (eq. bw57),
 *   b(x) = - int_Gamma d2G/dn_x dn_y (u - phi(x)) ds
 *          - int_S d2G/dn_x dn_y (phi - phi(x)) ds,
 * G the ball's Green's function, u on Gamma the interpolant of the node
 * means; the hypersingular S integral (eq. bw59's finite part) is
 * regularised by the constant solution and taken outside the disk of radius
 * 1e-6 h around x (its projection onto the tangent plane at the centre, on a
 * sphere), an O(delta) error as in eq. bw82.  On flat patches D = 0 and
 * sigma = 2b with no solve; on a sphere (inside a ball or outside one) D is
 * collocated with piecewise constants (Duffy on the own panel) and the
 * system solved with the class's FP64 LU factors.  SE(sigma) =
 * sqrt(sum_k A_ik^2 SE_k^2) with A = 2 Q2 / h (flat) or (1/2 I - D)^-1 Q2 / h.
 * FP64.  node_stats device [num_nodes][4]; neumann device [num_panels] out;
 * neumann_se device [num_panels] out, or NULL.
 * Errors: DTN_E_ARG (NULL). */
dtn_status dtn_patch_solve_second_kind(dtn_plan p, const double *node_stats, double *neumann, double *neumann_se,
                                       void *stream);

/* u at m targets off the boundary by eq. bw03 (G = 1/(4 pi |x - y|)).
 * Requires the patches to tile the boundary of a box: square tiles
 * [-h,h]^2 in their (t1, n x t1) frame with t1 along an axis, inside their
 * face, not overlapping, and adding up to each face's area (checked when the
 * plan is created; a partial or overlapping tiling is rejected here):
 * per tile, the Neumann data is the least-squares quadratic through the
 * panels within 0.7 h of the centre and the tile integral a 4 x 4 Gauss rule
 * with the exact Dirichlet data.  DTN_E_UNSUPPORTED for other plans.
 *   neumann device [num_panels]; targets device [m][3]; u_out device [m] */
dtn_status dtn_potential(dtn_plan p, const double *neumann, const double *targets, int64_t m,
                         double *u_out, void *stream);

/* ------------------------------------------------- treecode potential
 * The same sum as dtn_potential (same sources: the tiles' 4 x 4 Gauss points
 * with their fitted Neumann and exact Dirichlet weights), evaluated by a
 * kernel-independent treecode, the fast summation the paper names for this
 * step (Sec. 6): barycentric Lagrange interpolation on Chebyshev points
 * (Wang, Krasny & Tlupova 2020).
 *   tree      the root's children are the box's faces (a tile's face: the
 *             axis of its normal's largest component and that component's
 *             sign, label 2 axis + (sign > 0), in label order), so every
 *             cluster below the root lies in one plane; below them clusters
 *             split at the midpoint of their tight bounding box along every
 *             dimension with extent >= the largest / sqrt(2), children in
 *             octant-code order (bit d: upper half in dimension d), down to
 *             <= leaf_size sources;
 *   proxies   per cluster a tensor grid of Chebyshev points of the second
 *             kind on its box padded by 1e-12 of the root extent, `degree`
 *             in each dimension whose extent exceeds 1e-9 of the largest
 *             (one point, the centre, otherwise); charges
 *             q_k = sum_j L_k(y_j) w_j sigma_j and vectors
 *             p_k = -sum_j L_k(y_j) w_j phi_j n_j (L_k the tensor Lagrange
 *             basis), so far away u = sum_k [q_k/r + p_k.(x - s_k)/r^3]/(4 pi);
 *   traversal a cluster of centre c and radius r (half the padded box's
 *             diagonal) is taken whole when r < theta |x - c|: by its
 *             proxies if it has more sources than proxies, else directly;
 *             otherwise its children are visited (a leaf is summed directly).
 * The tree is built on the host from the plan's tile geometry and kept with
 * the handle; the proxies are rebuilt from the Neumann data on every call.
 * Targets are evaluated in Morton order of their position (sorted on the
 * device), so a wave's 64 targets share most of their traversal; a node that
 * at most 32 of a wave's targets take is evaluated by the whole wave
 * repacked, 64/k lanes per taking target, so a target's sum depends on its
 * wave companions only through rounding.  Each face's subtree is walked by
 * its own wave per group of 64 targets, the faces' sums added per target in
 * face order.  Proxies are built only for clusters that some target of the
 * call could take (the test against the targets' bounding box), so interior
 * targets pay nothing for the root's and the faces' proxies.
 * Create: degree in [1, 8], leaf_size in [8, 4096].  Errors: DTN_E_ARG,
 * DTN_E_UNSUPPORTED (a plan dtn_potential rejects), DTN_E_OOM.
 * The tree refers to the plan: destroy it before the plan. */
typedef struct dtn_tree_s *dtn_tree; /* opaque, library-owned */
dtn_status dtn_create_tree(dtn_plan p, int32_t degree, int32_t leaf_size, dtn_tree *out);
void dtn_destroy_tree(dtn_tree t);
/* Clusters, clusters with proxies, proxies in total, sources (host ints). */
dtn_status dtn_tree_info(dtn_tree t, int64_t info[4]);
/* Host only (no device work): the tree dtn_create_tree builds for these
 * patches (host array).  nodes [cap][8] out, in depth-first pre-order: first
 * and end source in tree order, end of the subtree (node index), leaf flag,
 * degrees per axis, first proxy (-1: none); perm [16 n_patches] out: tree
 * position -> source index 16 i + 4 a + b (tile i, Gauss point (xi_a, xi_b)
 * along (t1, n x t1)); n_nodes out.  DTN_E_ARG when cap is too small (n_nodes
 * is still set). */
dtn_status dtn_tree_layout(const dtn_patch *patches, int64_t n_patches, int32_t degree, int32_t leaf_size,
                           int64_t cap, int32_t *nodes, int32_t *perm, int64_t *n_nodes);

/* u at m targets (as dtn_potential) by the treecode with MAC parameter theta
 * in (0, 1).  counts: device [m][2] out (proxy and direct interactions of
 * each target), or NULL.  Device scratch is allocated stream-ordered: the
 * tile sources, proxies and their partials, the sort, and the faces' partial
 * sums for up to 2^22 targets at a time (8 B per face and target, 24 B with
 * counts).
 *   neumann device [num_panels]; targets device [m][3]; u_out device [m].
 * Errors: DTN_E_ARG (NULL arrays with m > 0, theta out of range), DTN_E_OOM. */
dtn_status dtn_tree_potential(dtn_tree t, const double *neumann, const double *targets, int64_t m,
                              double theta, double *u_out, int64_t *counts, void *stream);

/* ------------------------------------------------ single point (Sec. 5.1)
 * du/dn at a point x of a flat part of the boundary with no collocation
 * solve.  Over the hemisphere Gamma of radius a centred at x (Sec. 3,
 * eq. bw20; its Green's function by three images, eq. bw26, gives the kernel
 * 3 cos(theta) / (2 pi a^3) of eq. bw33),
 *   du/dn(x) = Sigma1' + Sigma2'                                     (eq. bw64)
 *   Sigma1' = - sum_ij W_ij (u(y_ij) - phi(x))                       (eq. bw83)
 *     y_ij = x + a (sin th_i cos ps_j t1 + sin th_i sin ps_j t2 - cos th_i n),
 *     th_i = pi/4 (xi_i + 1), ps_j = pi (xi_j + 1)  (eq. bw85, N_g1 Gauss
 *     points xi, weights w), W_ij = (pi/4 w_i)(pi w_j) a^2 sin th_i
 *     3 cos th_i / (2 pi a^3); u(y_ij) from the walks (eq. bw87);
 *   Sigma2' = -1/(2 pi) int over S_a minus the disk of radius
 *     delta = delta_rel a of (1/rho^3 - 1/a^3)(phi(y) - phi(x))
 *     (eqs. bw68, bw82), by an N_g2 x N_g2 Gauss rule in rho on [delta, a]
 *     (Jacobian rho) and angle on [0, 2 pi].
 * The standard error propagates the node variances:
 * se^2 = sum_ij W_ij^2 var_ij / count_ij. */
typedef struct dtn_points_s *dtn_points; /* opaque, library-owned */

/* One query point: x on the boundary, n the outward unit normal there, t1 a
 * unit tangent (t2 = n x t1), a the hemisphere radius.  80 bytes. */
typedef struct {
    double c[3];
    double n[3];
    double t1[3];
    double a;
} dtn_point;

/* Create / destroy a set of query points (host array, copied).
 * Supported: a half space (n = (0,0,-1), c on z = 0, the hemisphere inside
 * the truncation sphere), either face of a thin disk (n = (0,0,-1) on the
 * upper face, (0,0,1) on the lower; S_a inside the disk), or a face of a
 * box / box minus boxes with the disk inside the face and the half ball
 * inside Omega (as for plane patches).
 * n_g1, n_g2 in [1, 64]; delta_rel in (0, 1).  Errors: DTN_E_ARG (n < 1,
 * bad rule sizes, a point off a flat face, a ball domain). */
dtn_status dtn_create_points(dtn_geometry g, const dtn_point *pts, int64_t n, int32_t n_g1, int32_t n_g2,
                             double delta_rel, dtn_points *out);
void dtn_destroy_points(dtn_points p);
/* Number of hemisphere nodes: n x n_g1 x n_g1. */
int64_t dtn_points_num_nodes(dtn_points p);

/* Hemisphere nodes y_ij of every point (device [num_nodes][3] out; point-
 * major, theta-major, psi-minor), to be walked by dtn_wos_eval. */
dtn_status dtn_points_nodes(dtn_points p, double *nodes, void *stream);

/* du/dn at every point from the node statistics.
 *   node_stats device [num_nodes][4] from dtn_wos_eval, node order
 *   out        device [n][4] out: (Sigma1' + Sigma2', its standard error,
 *              Sigma1', Sigma2'), all FP64.  Errors: DTN_E_ARG. */
dtn_status dtn_points_neumann(dtn_points p, const double *node_stats, double *out, void *stream);

/* ------------------------------------------------------------ serving
 * A query server answers Neumann queries at boundary points: for every point
 * of a query it places a patch centred on the point (step 2's layout below,
 * h = h_max 2^-j for the smallest j that keeps the patch and its half ball
 * inside Omega), runs step 1 with adaptive walks (dtn_adaptive with the
 * query's se_target) and step 2, and answers with du/dn averaged over the
 * patch's central ring of panels (the disk of radius h / n_rings), its
 * standard error, the walks spent and h.  Continuous batching: a
 * dispatcher thread joins the queued queries, first come, first served, into
 * a batch of at most max_points points whose device memory fits under the
 * budget next to the batches in flight, and runs it on a free HIP stream of
 * the current device as single launches over all its patches; up to
 * n_streams batches are in flight.  A query's walks are a function of its
 * seed and its nodes only (Philox key = its seed, stream id = node index
 * within the query), so its walk set does not depend on what it is batched
 * with (its sums may round differently).
 * Graph replay (graph_replay = 1): a batch of n points is padded to the
 * smallest size bucket B >= n (B = n up to 8, then m 2^e with m in 5..8, at
 * most max_points), and its whole device pass (copies in, walks, solve,
 * answers, copy out, stream-ordered alloc and free) is one HIP graph,
 * captured once per stream and bucket (recorded on a capture stream of its
 * own, which runs no work) and replayed for every later batch of
 * that bucket.  Padding rows repeat the batch's first patch with an infinite
 * SE target, so they take only the pilot walks; their answers are dropped.
 * Budgets and footprints are those of the padded batch.  This mode is
 * switched off: its tests pass, but a serving run with four streams crashed
 * the host process with a cause not yet shown, so dtn_server_create rejects
 * it (DTN_E_ARG); dtn_server_footprint still reports its padded sizes.
 * Only box domains (with or without holes) are served: every point must lie
 * on a face, with the face's outward normal.
 * Point mode (n_g1 > 0): the single-point estimate of Sec. 5.1 with no
 * collocation solve.  Each point gets the hemisphere of radius a = the rung
 * h chosen as above (the same half ball, so it lies inside Omega), its
 * n_g1 x n_g1 nodes walked with the adaptive budgets, and the answer
 * (Sigma1' + Sigma2', its standard error, walks spent, a) as
 * dtn_points_neumann computes it; stream ids are node indices within the
 * query (point-major, theta-major, psi-minor).  The patch layout fields must
 * still be valid; they place nothing in this mode. */
typedef struct dtn_server_s *dtn_server; /* opaque, library-owned */

typedef struct {
    int32_t n_streams;   /* batches in flight at once, 1..16 */
    int32_t precision;   /* DTN_FP64 or DTN_FP32_MIXED (walks and solve) */
    int64_t hbm_budget;  /* bytes of device memory the batches in flight may hold */
    int64_t pilot_walks, min_walks, max_walks; /* adaptive budget (dtn_adaptive) */
    double h_max;        /* largest patch radius of the ladder, > 0 */
    int32_t ladder;      /* number of rungs h_max 2^-j, j = 0..ladder-1, 1..40 */
    int32_t n_theta, n_phi, n_rings, n_sectors; /* patch layout (as dtn_patch) */
    int64_t max_points;  /* largest query and batch (points), 1..2^20; sizes pinned staging */
    int32_t graph_replay;       /* 0: direct launches; 1: replay a HIP graph per size bucket
                                   (rows padded, see below) -- switched off: rejected by
                                   dtn_server_create with DTN_E_ARG, see below */
    int32_t max_batch_queries;  /* queries joined into one batch at most; 0 = no limit,
                                   1 = one query per batch (no batching across requests) */
    int32_t n_g1, n_g2;  /* point mode when n_g1 > 0 (see below): hemisphere and ring rules, [1, 64] */
    double delta_rel;    /* point mode: excluded disk radius / a, in (0, 1) */
} dtn_server_config;

/* Completion record of a query; times in seconds on the server's clock. */
typedef struct {
    uint64_t query_id;
    int32_t status;      /* DTN_OK or the error that ended the query */
    int32_t reserved;
    int64_t n_points;
    double t_submit, t_start, t_done;
} dtn_query_done;

/* Create / destroy a server on the current device.  Builds the patch class
 * once.  Destroy waits for the queries in flight; queued ones are dropped.
 * Errors: DTN_E_ARG for an invalid configuration or a geometry other than a
 * box or a box with holes. */
dtn_status dtn_server_create(dtn_geometry g, const dtn_server_config *cfg, dtn_server *out);
void dtn_server_destroy(dtn_server s);

/* Device bytes a batch of n_points reserves under this configuration (of
 * its padded size under graph replay). */
int64_t dtn_server_footprint(const dtn_server_config *cfg, int64_t n_points);

/* Seconds since the server was created (the clock of dtn_query_done). */
double dtn_server_clock(dtn_server s);

/* Queue a query.  pts, normals: host [n][3] (copied); out: host [n][4]
 * (value, standard error, walks, h per point), written when the query
 * completes and owned by the caller, who keeps it allocated until then.
 * Errors (synchronous, nothing queued): DTN_E_ARG for n outside [1, max_points],
 * se_target <= 0, a point not on a face with that outward normal, or a point
 * so close to an edge or another surface that no rung fits; DTN_E_OOM when
 * the query alone exceeds the budget. */
dtn_status dtn_server_submit(dtn_server s, uint64_t query_id, const double *pts, const double *normals,
                             int64_t n, double se_target, uint64_t seed, double *out);

/* Wait up to timeout_s seconds (< 0: forever) for completions and return up
 * to max_n of them in completion order; *n_out = 0 on timeout. */
dtn_status dtn_server_wait(dtn_server s, int64_t max_n, double timeout_s, dtn_query_done *done, int64_t *n_out);

/* Diagnostic, host only (no device needed): the class operators that
 * dtn_create_plan builds for patches with this layout and curvature, in local
 * coordinates scaled by 1/h (rr = R/h on a sphere of radius R, -R/h outside
 * a ball, 0 on a plane).
 * Outputs are host arrays (any may be NULL):
 *   node_tab [n_theta*n_phi][3], col_tab [P][3], K [P][P] (at h = 1),
 *   QI [P][n_theta*n_phi], A2 [P][n_theta*n_phi], fit [16][P];
 *   P = n_rings*n_sectors.  Lets a caller inspect or test step 2's operators. */
dtn_status dtn_class_operators(int32_t n_theta, int32_t n_phi, int32_t n_rings, int32_t n_sectors, double rr,
                               double *node_tab, double *col_tab, double *K, double *QI, double *A2, double *fit);

/* Host diagnostic: the second-kind tables of a class at h = 1 (no device),
 * rr as for dtn_class_operators (0: plane): Q2 [P][N] (the Gamma operator
 * with the kernel -d2G_B/dn_x dn_y, dP/dn_x on a plane), c2 [P] (sum_k Q2_ik
 * minus the sum of the regularised S rule's weights) and M [P][P] = 1/2 I - D
 * (D the adjoint double layer of eq. bw57; zero on a plane), or NULL.  Host
 * arrays.  Errors: DTN_E_ARG (NULL Q2 or c2, bad layout, 0 < |rr| < 1). */
dtn_status dtn_class_second_kind(int32_t n_theta, int32_t n_phi, int32_t n_rings, int32_t n_sectors, double rr,
                                 double *Q2, double *c2, double *M);

#ifdef __cplusplus
}
#endif
#endif /* DTN_H */
