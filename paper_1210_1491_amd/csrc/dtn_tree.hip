// Treecode evaluation of the final potential (eq. bw03; the paper names a
// fast summation as the way to scale this step, Sec. 6).  Kernel-independent
// treecode with barycentric Lagrange interpolation on Chebyshev points (Wang,
// Krasny & Tlupova, Commun. Comput. Phys. 28, 2020).  With the tile sources
// y_j, a_j = w_j sigma_j and b_j = -w_j phi_j n_j,
//   u(x) = sum_j [a_j / |x - y_j| + b_j . (x - y_j) / |x - y_j|^3] / (4 pi),
// and a cluster's proxies s_k carry q_k = sum_j L_k(y_j) a_j and
// p_k = sum_j L_k(y_j) b_j, which interpolate y -> 1/|x - y| and its gradient.
//
//   host, per handle       tree over the tile sources in depth-first
//                          pre-order: the root's children are the box's
//                          faces (flat clusters: 2-D proxy grids below
//                          them), then octant splits; node j's subtree is
//                          nodes [j, skip_j), its sources [b, e) in tree
//                          order; proxy grids and the proxy pass's work
//                          items (cluster, source chunk)
//   k_tree_tbox_*          bounding box of the targets: clusters that no
//                          target in it can take get no proxies this call
//   k_tree_proxy_partial   one block per work item: 1-D Lagrange values of 64
//                          sources at a time in LDS, each thread accumulates
//                          up to 3 proxies of the cluster (flat clusters:
//                          2 or 4 thread groups over alternate sources)
//   k_tree_proxy_reduce    per cluster: chunk partials summed in order, proxy
//                          points written beside their charges (in-plane
//                          clusters: a row/column table in the plane's
//                          frame)
//   k_tree_keys            Morton keys of the targets (10 bits per axis in the
//                          sources' bounding box, clamped), then a radix sort
//                          of (key, target) pairs (hipCUB)
//   k_tree_eval            one wave per 64 consecutive sorted targets and
//                          face subtree: a stackless walk of the subtree's
//                          node range under wave-uniform control.  Each
//                          lane keeps the node index below which it is
//                          done (it took an ancestor whole); a node is
//                          opened when a lane still inside it needs it
//                          opened, else the walk jumps past its subtree.
//                          Proxies and sources are read at wave-uniform
//                          addresses (a node few lanes take: by the wave
//                          repacked over those lanes' targets).  All FP64.
//   k_tree_sum             per target: the face subtrees' sums in order
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <limits>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "dtn_device.h"
#include "dtn_internal.h"
#include "dtn_potential.h"
#include "dtn_xcd.h"

namespace dtn {
namespace {

constexpr int kMaxDegree = 8;
constexpr int kProxyChunk = 1024;  // sources per proxy work item
constexpr int kProxyThreads = 256;
constexpr int kProxySlots = 3;     // (kMaxDegree + 1)^3 = 729 <= kProxyThreads * kProxySlots
constexpr double kPadRel = 1e-12;  // box padding, relative to the root extent
constexpr double kFlatRel = 1e-9;  // extents below this (relative) get degree 0

struct TreeNode {
    double c[3];   // centre of the padded box
    double r2;     // squared radius (half the padded box's diagonal)
    double lo[3];  // padded box: the Chebyshev grid's interval per axis
    double hi[3];
    int32_t b, e;     // sources [b, e) in tree order
    int32_t skip;     // first node after this subtree
    int32_t leaf;     // 1 for a leaf
    int32_t proxy;    // first proxy, -1 without proxies
    int32_t n_proxy;  // (deg0 + 1)(deg1 + 1)(deg2 + 1)
    int32_t deg[3];
    // In-plane cluster: its sources lie on one plane x_axis = c[axis] and
    // their normals are exactly +-e_axis (so is every proxy vector); -1
    // otherwise.  Such a cluster's proxies are stored in its plane's frame.
    int32_t axis;
    int32_t pad[2];
};

// A proxy: position, charge and vector.
struct Proxy {
    double x, y, z, q, px, py, pz, pad;
};

// An in-plane cluster (axis a, in-plane axes b = a + 1 and c = a + 2 mod 3)
// keeps its proxies in its plane's frame, as a table over its proxies' 64-byte
// slots: the proxies form an nb x nc grid (nb, nc the Chebyshev point counts
// along b and c), so with pb_i, pc_j the grid's offsets from the cluster's
// centre the table holds, in doubles, the column terms (-2 pc_j, pc_j^2) for
// j < nc, then per row i its row terms (-2 pb_i, pb_i^2) followed by, per
// proxy (i, j), its charge and its vector's component along a (the others
// are 0).  16 (nb + nc + nb nc) bytes of the 64 nb nc; a row is 2 + 2 nc
// contiguous doubles, read with one wait.
__host__ __device__ __forceinline__ int plane_row(int nc, int i)
{
    return 2 * nc + i * (2 + 2 * nc);
}

struct Item {      // proxy pass work item: one cluster's sources [b, e)
    int32_t node, b, e, pad;
    int64_t part;  // offset of its partials (4 doubles per proxy)
};

struct ProxyCluster {
    int32_t node, item_b, item_e, pad;
};

static_assert(sizeof(TreeNode) == 128, "node layout");
static_assert((kMaxDegree + 1) * (kMaxDegree + 1) * (kMaxDegree + 1) <= kProxyThreads * kProxySlots, "slots");

// Node ranges the traversal is split into: the root's subtrees (the
// faces), each walked by its own wave per target group, so that a target
// group's work is spread over several waves; their sums are added per
// target, in range order, by k_tree_sum.
constexpr int kMaxParts = 8;
constexpr int64_t kEvalBatch = (int64_t)1 << 22;  // targets per traversal launch
struct TreeParts {
    int32_t n;
    int32_t lo[kMaxParts], hi[kMaxParts];
};

struct HostTree {
    TreeParts parts;
    std::vector<TreeNode> nodes;
    std::vector<int32_t> perm;  // tree position -> source index (16 patch + q)
    std::vector<int32_t> slot;  // source index -> tree position
    std::vector<Item> items;
    std::vector<ProxyCluster> pcl;
    int64_t n_proxies = 0, part_len = 0;
    double box_lo[3], box_ext[3];  // tight box of all sources (Morton frame)
};

// Recursive build of node [b, e) of perm (depth-first pre-order).  With
// `face` (the root only) the children are the boundary's faces, one per
// face label present, in label order; otherwise the octants of the split.
void build_node(const std::vector<double> &pos, const int8_t *face, int32_t b, int32_t e, int degree,
                int leaf_size, double pad, HostTree &T, std::vector<int32_t> &tmp)
{
    double tlo[3], thi[3];
    for (int d = 0; d < 3; ++d) {
        tlo[d] = std::numeric_limits<double>::infinity();
        thi[d] = -tlo[d];
    }
    for (int32_t i = b; i < e; ++i)
        for (int d = 0; d < 3; ++d) {
            const double v = pos[3 * (size_t)T.perm[i] + d];
            tlo[d] = std::min(tlo[d], v);
            thi[d] = std::max(thi[d], v);
        }
    double ext[3], big = 0.0;
    for (int d = 0; d < 3; ++d) {
        ext[d] = thi[d] - tlo[d];
        big = std::max(big, ext[d]);
    }
    TreeNode nd{};
    double diag2 = 0.0;
    nd.n_proxy = 1;
    for (int d = 0; d < 3; ++d) {
        nd.lo[d] = tlo[d] - pad;
        nd.hi[d] = thi[d] + pad;
        nd.c[d] = 0.5 * (nd.lo[d] + nd.hi[d]);
        diag2 += (nd.hi[d] - nd.lo[d]) * (nd.hi[d] - nd.lo[d]);
        nd.deg[d] = ext[d] > kFlatRel * big ? degree : 0;
        nd.n_proxy *= nd.deg[d] + 1;
    }
    nd.r2 = 0.25 * diag2;
    nd.b = b;
    nd.e = e;
    nd.proxy = -1;
    const bool split = face || (e - b > leaf_size && big > 0.0);
    nd.leaf = split ? 0 : 1;
    const int32_t j = (int32_t)T.nodes.size();
    T.nodes.push_back(nd);
    if (split) {
        double mid[3];
        bool cut[3];
        for (int d = 0; d < 3; ++d) {
            mid[d] = 0.5 * (tlo[d] + thi[d]);
            cut[d] = ext[d] >= big / std::sqrt(2.0);
        }
        // stable counting sort of the sources by octant code (face label at the root)
        int32_t cnt[9] = {0};
        auto code = [&](int32_t s) {
            if (face) return (int)face[s];
            int c = 0;
            for (int d = 0; d < 3; ++d)
                if (cut[d] && pos[3 * (size_t)s + d] >= mid[d]) c |= 1 << d;
            return c;
        };
        for (int32_t i = b; i < e; ++i) ++cnt[code(T.perm[i]) + 1];
        for (int c = 0; c < 8; ++c) cnt[c + 1] += cnt[c];
        int32_t at[8];
        for (int c = 0; c < 8; ++c) at[c] = b + cnt[c];
        for (int32_t i = b; i < e; ++i) tmp[at[code(T.perm[i])]++] = T.perm[i];
        std::copy(tmp.begin() + b, tmp.begin() + e, T.perm.begin() + b);
        for (int c = 0; c < 8; ++c)
            if (cnt[c + 1] > cnt[c])
                build_node(pos, nullptr, b + cnt[c], b + cnt[c + 1], degree, leaf_size, pad, T, tmp);
    }
    T.nodes[j].skip = (int32_t)T.nodes.size();
}

// The tree over the sources at `pos` with face labels `face` (one per
// source, 0..5).  The root's children are the faces, so that no cluster
// below it straddles an edge of the box: each lies in one plane and its
// proxy grid is two-dimensional (degree 0 along the normal), 49 proxies at
// degree 6 where a cluster across an edge needs 343.
void build_tree(const std::vector<double> &pos, const std::vector<int8_t> &face, const std::vector<int8_t> &along,
                int degree, int leaf_size, HostTree &T)
{
    const int32_t n = (int32_t)(pos.size() / 3);
    double lo[3], hi[3], big = 0.0;
    for (int d = 0; d < 3; ++d) {
        lo[d] = std::numeric_limits<double>::infinity();
        hi[d] = -lo[d];
    }
    for (int32_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], pos[3 * (size_t)i + d]);
            hi[d] = std::max(hi[d], pos[3 * (size_t)i + d]);
        }
    for (int d = 0; d < 3; ++d) {
        T.box_lo[d] = lo[d];
        T.box_ext[d] = hi[d] - lo[d];
        big = std::max(big, hi[d] - lo[d]);
    }
    T.perm.resize(n);
    for (int32_t i = 0; i < n; ++i) T.perm[i] = i;
    std::vector<int32_t> tmp(n);
    build_node(pos, face.data(), 0, n, degree, leaf_size, kPadRel * big, T, tmp);
    T.slot.resize(n);
    for (int32_t i = 0; i < n; ++i) T.slot[T.perm[i]] = i;
    // in-plane clusters: every source's normal exactly along one axis a, and
    // every source on one plane x_a = const (then the cluster's degree along
    // a is 0 and its proxies' coordinate along a is the box centre's)
    for (TreeNode &nd : T.nodes) {
        nd.axis = -1;
        const int a = along[T.perm[nd.b]];
        if (a < 0 || nd.deg[a] != 0) continue;
        const double xa = pos[3 * (size_t)T.perm[nd.b] + a];
        bool ok = true;
        for (int32_t i = nd.b; i < nd.e && ok; ++i)
            ok = along[T.perm[i]] == a && pos[3 * (size_t)T.perm[i] + a] == xa;
        if (ok) nd.axis = a;
    }
    // the root's subtrees as traversal parts (sibling subtrees are
    // contiguous in pre-order, so any overflow joins the last part)
    TreeParts &P = T.parts;
    P.n = 0;
    const int32_t nn = (int32_t)T.nodes.size();
    for (int32_t c = 1; c < nn; c = T.nodes[c].skip) {
        if (P.n == kMaxParts) {
            P.hi[kMaxParts - 1] = nn;
            break;
        }
        P.lo[P.n] = c;
        P.hi[P.n] = T.nodes[c].skip;
        ++P.n;
    }
    if (P.n == 0) {  // the root is a leaf: nothing below it
        P.n = 1;
        P.lo[0] = P.hi[0] = nn;
    }
    // proxies of every cluster holding more sources than proxies, in node order
    for (int32_t j = 0; j < (int32_t)T.nodes.size(); ++j) {
        TreeNode &nd = T.nodes[j];
        if (nd.e - nd.b <= nd.n_proxy) continue;
        nd.proxy = (int32_t)T.n_proxies;
        T.n_proxies += nd.n_proxy;
        ProxyCluster pc{j, (int32_t)T.items.size(), 0, 0};
        for (int32_t s = nd.b; s < nd.e; s += kProxyChunk) {
            T.items.push_back(Item{j, s, std::min(nd.e, s + kProxyChunk), 0, T.part_len});
            T.part_len += 4 * (int64_t)nd.n_proxy;
        }
        pc.item_e = (int32_t)T.items.size();
        T.pcl.push_back(pc);
    }
}

// Lagrange basis at y through the Chebyshev points of the second kind on
// [lo, hi] (degree n; the centre alone for n = 0), second barycentric form;
// the unit vector when y equals a node.
// cosk[k] = cos(pi k / n), the points on [-1, 1].
__device__ void lagrange_1d(double y, double lo, double hi, int n, const double *cosk, double *L)
{
    if (n == 0) {
        L[0] = 1.0;
        return;
    }
    const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    double sum = 0.0;
    int hit = -1;
    for (int k = 0; k <= n; ++k) {
        const double d = y - (c + h * cosk[k]);
        const double w = ((k & 1) ? -1.0 : 1.0) * ((k == 0 || k == n) ? 0.5 : 1.0);
        if (d == 0.0) hit = k;
        const double t = d == 0.0 ? 0.0 : w / d;
        L[k] = t;
        sum += t;
    }
    const double inv = 1.0 / sum;
    for (int k = 0; k <= n; ++k) L[k] = hit >= 0 ? (k == hit ? 1.0 : 0.0) : L[k] * inv;
}

__device__ __forceinline__ double cheb_point(const TreeNode &nd, int d, int k)
{
    if (nd.deg[d] == 0) return 0.5 * (nd.lo[d] + nd.hi[d]);
    return 0.5 * (nd.lo[d] + nd.hi[d]) + 0.5 * (nd.hi[d] - nd.lo[d]) * cos(M_PI * k / nd.deg[d]);
}

// Can any target accept node nd?  The acceptance test r^2 < theta^2 |x - c|^2
// fails for every x in the targets' box when r^2 exceeds theta^2 times the
// squared distance from c to the box's farthest corner (a relative margin
// covers the rounding of the per-target distances).  Proxies of clusters
// no target can accept are never read, so they are not built.
__device__ __forceinline__ bool acceptable(const TreeNode &nd, const double *__restrict__ tbox, double theta2)
{
    double d2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double a = fmax(fabs(nd.c[d] - tbox[d]), fabs(tbox[3 + d] - nd.c[d]));
        d2 += a * a;
    }
    return !(nd.r2 > theta2 * d2 * (1.0 + 1e-12));
}

// Bounding box of the targets: per-block partial (lo, hi) rows, then one
// block folds them into tbox[6].  Min and max are exact, so the order is
// immaterial.
__global__ __launch_bounds__(256) void k_tree_tbox_partial(const double *__restrict__ targets, int64_t m,
                                                           double *__restrict__ rows)
{
    __shared__ double r[6][256];
    const int tid = threadIdx.x;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    for (int64_t t = (int64_t)blockIdx.x * 256 + tid; t < m; t += (int64_t)gridDim.x * 256)
        for (int d = 0; d < 3; ++d) {
            const double v = targets[3 * t + d];
            lo[d] = fmin(lo[d], v);
            hi[d] = fmax(hi[d], v);
        }
    for (int d = 0; d < 3; ++d) {
        r[d][tid] = lo[d];
        r[3 + d][tid] = hi[d];
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            for (int d = 0; d < 3; ++d) {
                r[d][tid] = fmin(r[d][tid], r[d][tid + h]);
                r[3 + d][tid] = fmax(r[3 + d][tid], r[3 + d][tid + h]);
            }
        __syncthreads();
    }
    if (tid < 6) rows[6 * (int64_t)blockIdx.x + tid] = r[tid][0];
}

__global__ __launch_bounds__(64) void k_tree_tbox_final(const double *__restrict__ rows, int32_t n_rows,
                                                        double *__restrict__ tbox)
{
    const int q = threadIdx.x;
    if (q >= 6) return;
    double v = q < 3 ? INFINITY : -INFINITY;
    for (int i = 0; i < n_rows; ++i) v = q < 3 ? fmin(v, rows[6 * i + q]) : fmax(v, rows[6 * i + q]);
    tbox[q] = v;
}

// Proxy partials of one work item (a cluster's sources [b, e), at most
// kProxyChunk).  Per batch of 64 sources, 192 threads compute the 1-D
// Lagrange values (one source and axis each) and 64 the charge and vector
// weights into LDS; then each proxy accumulates over the batch.  Clusters
// with at most 64 (128) proxies split the block into 4 (2) groups that take
// alternate sources of each batch, their sums added in group order at the
// end, so that the block's threads stay busy on flat clusters.
__global__ __launch_bounds__(kProxyThreads) void k_tree_proxy_partial(const TreeNode *__restrict__ nodes,
                                                                      const Item *__restrict__ items,
                                                                      const TileSource *__restrict__ src,
                                                                      const double *__restrict__ tbox,
                                                                      double theta2, double *__restrict__ part)
{
    __shared__ double sl[3][64][kMaxDegree + 1];
    __shared__ double sw[64][4];
    __shared__ double red[kProxyThreads][4];
    __shared__ double cosk[kMaxDegree + 1];
    const Item it = items[blockIdx.x];
    const TreeNode &nd = nodes[it.node];
    if (!acceptable(nd, tbox, theta2)) return;  // uniform per block
    const int tid = threadIdx.x;
    const int n1 = nd.deg[1] + 1, n2 = nd.deg[2] + 1, np = nd.n_proxy;
    // the Chebyshev points' cosines, once per block (every axis with
    // points uses the same degree)
    const int nmax = max(nd.deg[0], max(nd.deg[1], nd.deg[2]));
    if (tid <= nmax && nmax > 0) cosk[tid] = cos(M_PI * tid / nmax);
    const int ng = np > 128 ? 1 : (np > 64 ? 2 : 4);
    const int gs = kProxyThreads / ng, gi = tid / gs, kt = tid - gi * gs;
    int k0[kProxySlots], k1[kProxySlots], k2[kProxySlots];
    double acc[kProxySlots][4];
    for (int s = 0; s < kProxySlots; ++s) {
        const int k = kt + gs * s;
        k2[s] = k % n2;
        k1[s] = (k / n2) % n1;
        k0[s] = k / (n1 * n2);
        for (int c = 0; c < 4; ++c) acc[s][c] = 0.0;
    }
    for (int32_t base = it.b; base < it.e; base += 64) {
        const int cnt = min(64, it.e - base);
        __syncthreads();
        {
            const int j = tid & 63, d = tid >> 6;
            if (j < cnt) {
                const TileSource q = src[base + j];
                if (d == 3) {
                    sw[j][0] = q.ws;
                    sw[j][1] = -q.wf * q.nx;
                    sw[j][2] = -q.wf * q.ny;
                    sw[j][3] = -q.wf * q.nz;
                } else {
                    lagrange_1d(d == 0 ? q.x : (d == 1 ? q.y : q.z), nd.lo[d], nd.hi[d], nd.deg[d], cosk, sl[d][j]);
                }
            }
        }
        __syncthreads();
        for (int s = 0; s < kProxySlots; ++s) {
            if (kt + gs * s >= np) break;
            for (int j = gi; j < cnt; j += ng) {
                const double L = sl[0][j][k0[s]] * sl[1][j][k1[s]] * sl[2][j][k2[s]];
                for (int c = 0; c < 4; ++c) acc[s][c] += L * sw[j][c];
            }
        }
    }
    if (ng == 1) {
        for (int s = 0; s < kProxySlots; ++s) {
            const int k = kt + gs * s;
            if (k < np)
                for (int c = 0; c < 4; ++c) part[it.part + 4 * (int64_t)k + c] = acc[s][c];
        }
        return;
    }
    for (int c = 0; c < 4; ++c) red[tid][c] = acc[0][c];
    __syncthreads();
    if (gi == 0 && kt < np)
        for (int c = 0; c < 4; ++c) {
            double v = red[kt][c];
            for (int g = 1; g < ng; ++g) v += red[g * gs + kt][c];
            part[it.part + 4 * (int64_t)kt + c] = v;
        }
}

__global__ __launch_bounds__(kProxyThreads) void k_tree_proxy_reduce(const TreeNode *__restrict__ nodes,
                                                                     const ProxyCluster *__restrict__ pcl,
                                                                     const Item *__restrict__ items,
                                                                     const double *__restrict__ part,
                                                                     const double *__restrict__ tbox,
                                                                     double theta2, Proxy *__restrict__ prox)
{
    const ProxyCluster pc = pcl[blockIdx.x];
    const TreeNode &nd = nodes[pc.node];
    if (!acceptable(nd, tbox, theta2)) return;
    const int n1 = nd.deg[1] + 1, n2 = nd.deg[2] + 1;
    for (int k = threadIdx.x; k < nd.n_proxy; k += kProxyThreads) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int32_t i = pc.item_b; i < pc.item_e; ++i)
            for (int c = 0; c < 4; ++c) v[c] += part[items[i].part + 4 * (int64_t)k + c];
        const double pt[3] = {cheb_point(nd, 0, k / (n1 * n2)), cheb_point(nd, 1, (k / n2) % n1),
                              cheb_point(nd, 2, k % n2)};
        if (nd.axis >= 0) {  // the plane's table
            const int a = nd.axis, ib = (a + 1) % 3, ic = (a + 2) % 3;
            const int idx[3] = {k / (n1 * n2), (k / n2) % n1, k % n2};
            const int nb = nd.deg[ib] + 1, nc = nd.deg[ic] + 1, i = idx[ib], j = idx[ic];
            double *D = reinterpret_cast<double *>(prox + nd.proxy);
            double *R = D + plane_row(nc, i);
            R[2 + 2 * j] = v[0];
            R[3 + 2 * j] = v[1 + a];
            if (j == 0) {
                const double pb = pt[ib] - nd.c[ib];
                R[0] = -2.0 * pb;
                R[1] = pb * pb;
            }
            if (i == 0) {
                const double pc = pt[ic] - nd.c[ic];
                D[2 * j] = -2.0 * pc;
                D[2 * j + 1] = pc * pc;
            }
        } else {
            Proxy o;
            o.x = pt[0];
            o.y = pt[1];
            o.z = pt[2];
            o.q = v[0];
            o.px = v[1];
            o.py = v[2];
            o.pz = v[3];
            o.pad = 0.0;
            prox[nd.proxy + k] = o;
        }
    }
}

__device__ __forceinline__ uint32_t spread10(uint32_t v)
{
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ __launch_bounds__(256) void k_tree_keys(const double *__restrict__ targets, int64_t m, double lo0,
                                                   double lo1, double lo2, double sc0, double sc1, double sc2,
                                                   uint32_t *__restrict__ keys, uint32_t *__restrict__ ids)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const double lo[3] = {lo0, lo1, lo2}, sc[3] = {sc0, sc1, sc2};
    uint32_t key = 0;
    for (int d = 0; d < 3; ++d) {
        const double u = fmin(fmax((targets[3 * t + d] - lo[d]) * sc[d], 0.0), 1023.0);
        key |= spread10((uint32_t)u) << d;
    }
    keys[t] = key;
    ids[t] = (uint32_t)t;
}

enum : int { kNone = 0, kTakeProxy = 1, kTakeDirect = 2, kOpen = 3 };

// 1/|x - y| and 1/|x - y|^2 from q = |x - y|^2 for the interactions: the
// hardware reciprocal square root r (relative error below 6e-8) and its
// residual e = 1 - q r^2, then r (1 + e/2) and r^2 (1 + e), the first-order
// corrections (relative errors ~5e-15 and ~1.5e-14, far below the
// interpolation error that sets the treecode's accuracy).  Six instructions
// for both; a correctly rounded root alone takes nine.
struct InvPowers {
    double r1, r2;
};
__device__ __forceinline__ InvPowers inv_powers(double q)
{
    const double r = __builtin_amdgcn_rsq(q);
    const double s = r * r, e = fma(-q, s, 1.0);
    return {r * fma(e, 0.5, 1.0), fma(s, e, s)};
}

// Every interaction is (q + (m . (x - y)) / |x - y|^2) / |x - y| for a
// charge q and a vector m at y (a source's m is -wf n).
__device__ __forceinline__ double proxy_term(double x, double y, double z, const Proxy &p)
{
    const double ex = x - p.x, ey = y - p.y, ez = z - p.z;
    const InvPowers v = inv_powers(ex * ex + ey * ey + ez * ez);
    return fma(p.px * ex + p.py * ey + p.pz * ez, v.r2, p.q) * v.r1;
}

// In-plane clusters: the target enters as its offsets from the cluster's
// centre (tb, tc in the plane, h above it) and d2 = tb^2 + tc^2 + h^2, and
// |x - y|^2 for the proxy (i, j) is expanded as d2 + (pb_i^2 - 2 pb_i tb) +
// (pc_j^2 - 2 pc_j tc): per target, a row term per row and a column term per
// column, then one add per proxy.  Acceptance keeps |y - c| <= r <
// theta |x - c|, so |x - y|^2 >= (1 - theta)^2 d2 while the summands stay
// below (1 + theta)^2 d2: the expansion costs a few roundings times
// (1 + theta)^2 / (1 - theta)^2 (9 at theta = 0.5).
struct PlaneEntry {
    double b2, c2, p2, q, pn;  // -2 pb_i, -2 pc_j, pb_i^2 + pc_j^2, charge, vector
};

// a b + c with c in scalar registers (the wave-uniform charge): the
// compiler's own choice copies c into vector registers first.
__device__ __forceinline__ double fma_uniform_addend(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// acc += (q + pn h / |x - y|^2) / |x - y| for |x - y|^2 = q2; q and pn are
// wave-uniform.
__device__ __forceinline__ void plane_add(double q2, double h, double q, double pn, double &acc)
{
    const InvPowers v = inv_powers(q2);
    acc = fma(fma_uniform_addend(pn * h, v.r2, q), v.r1, acc);
}

// All proxies of an in-plane cluster with NC columns for the taking lanes
// of a wave, with wave-uniform (scalar) loads: the column terms once, then
// a row per iteration, read whole, so that the row's NC interactions follow
// one wait.
template <int NC>
__device__ __forceinline__ void plane_rows_n(const double *__restrict__ D, int nb, double tb, double tc, double h,
                                             double d2, double &acc)
{
    double cv[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) cv[j] = fma(D[2 * j], tc, D[2 * j + 1]);
    for (int i = 0; i < nb; ++i) {
        const double *R = D + plane_row(NC, i);
        double rv[2 + 2 * NC];
#pragma unroll
        for (int k = 0; k < 2 + 2 * NC; ++k) rv[k] = R[k];
        const double bi = d2 + fma(rv[0], tb, rv[1]);
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            plane_add(bi + cv[j], h, rv[2 + 2 * j], rv[3 + 2 * j], acc);
            // at most two interactions interleaved by the scheduler (a
            // whole row interleaved needs 127 registers)
            if (j % 2 == 1) __builtin_amdgcn_sched_barrier(0);
        }
    }
}

__device__ __forceinline__ void plane_rows(const double *__restrict__ D, int nb, int nc, double tb, double tc,
                                           double h, double d2, double &acc)
{
    static_assert(kMaxDegree + 1 == 9, "one case per column count");
    switch (nc) {
    case 1: plane_rows_n<1>(D, nb, tb, tc, h, d2, acc); break;
    case 2: plane_rows_n<2>(D, nb, tb, tc, h, d2, acc); break;
    case 3: plane_rows_n<3>(D, nb, tb, tc, h, d2, acc); break;
    case 4: plane_rows_n<4>(D, nb, tb, tc, h, d2, acc); break;
    case 5: plane_rows_n<5>(D, nb, tb, tc, h, d2, acc); break;
    case 6: plane_rows_n<6>(D, nb, tb, tc, h, d2, acc); break;
    case 7: plane_rows_n<7>(D, nb, tb, tc, h, d2, acc); break;
    case 8: plane_rows_n<8>(D, nb, tb, tc, h, d2, acc); break;
    default: plane_rows_n<9>(D, nb, tb, tc, h, d2, acc); break;
    }
}

__device__ __forceinline__ double source_term(double x, double y, double z, const TileSource &s)
{
    const double ex = x - s.x, ey = y - s.y, ez = z - s.z;
    const InvPowers v = inv_powers(ex * ex + ey * ey + ez * ez);
    return fma(-s.wf * (ex * s.nx + ey * s.ny + ez * s.nz), v.r2, s.ws) * v.r1;
}

__device__ __forceinline__ void tree_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Entries 0 .. count - 1 of a node (fetch(e) reads entry e) taken by the
// k <= 32 lanes of `mask`: the wave is repacked so that g = 64 / k lanes
// work on each taking lane's target (lane l on the target of rank l / g,
// entries l mod g, l mod g + g, ...), each reading its own entries; the g
// partial sums of a target are then added, in lane order, to its lane's
// sum.  With k > 32 the whole wave walks the entries together instead
// (wave-uniform loads).
template <bool kAhead = true, class Fetch, class Term>
__device__ __forceinline__ void packed_sum(uint64_t mask, int32_t count, Fetch fetch, double x, double y, double z,
                                           double &acc, Term term, double *lx, double *ly, double *lz, double *part)
{
    const int lane = __lane_id();
    const int k = __popcll(mask), g = 64 / k;
    const bool mine = (mask >> lane) & 1ull;
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    if (mine) {
        lx[rank] = x;
        ly[rank] = y;
        lz[rank] = z;
    }
    tree_wave_sync();
    const int t = lane / g, sub = lane - t * g;
    double a = 0.0;
    if (t < k) {
        const double px = lx[t], py = ly[t], pz = lz[t];
        // entries sub, sub + g, ... two per iteration, the next two loaded
        // before the current two are summed (kAhead; else one at a time,
        // for entries whose registers would crowd the wave's)
        int32_t e = sub;
        if (kAhead && e + g < count) {
            auto ea = fetch(e), eb = fetch(e + g);
            for (e += 2 * g; e + g < count; e += 2 * g) {
                const auto ec = fetch(e), ed = fetch(e + g);
                a += term(px, py, pz, ea);
                a += term(px, py, pz, eb);
                ea = ec;
                eb = ed;
            }
            a += term(px, py, pz, ea);
            a += term(px, py, pz, eb);
        }
        if (kAhead) {
            if (e < count) a += term(px, py, pz, fetch(e));
        } else {
            for (; e < count; e += g) a += term(px, py, pz, fetch(e));
        }
    }
    part[lane] = a;
    tree_wave_sync();
    if (mine) {
        double sum = 0.0;
        for (int q = 0; q < g; ++q) sum += part[rank * g + q];
        acc += sum;
    }
    tree_wave_sync();
}

// What a lane does at node nd (kNone for lanes outside it).
__device__ __forceinline__ int node_action(const TreeNode &nd, bool inside, double x, double y, double z,
                                           double theta2)
{
    if (!inside) return kNone;
    const double dx = x - nd.c[0], dy = y - nd.c[1], dz = z - nd.c[2];
    const double R2 = dx * dx + dy * dy + dz * dz;
    return nd.r2 < theta2 * R2 ? (nd.proxy >= 0 ? kTakeProxy : kTakeDirect) : (nd.leaf ? kTakeDirect : kOpen);
}

// Node nd summed into acc for the lanes that take it: by the whole wave
// (wave-uniform loads, lanes that do not take it masked) when more than 32
// lanes take it, else by the repacked wave.
__device__ __forceinline__ void take_node(const TreeNode &nd, int act, const Proxy *__restrict__ prox,
                                          const TileSource *__restrict__ src, double x, double y, double z,
                                          double &acc, int64_t &n_prox, int64_t &n_dir, double *lx, double *ly,
                                          double *lz, double *part)
{
    const auto pterm = [](double a, double b, double c, const Proxy &q) { return proxy_term(a, b, c, q); };
    const auto sterm = [](double a, double b, double c, const TileSource &q) { return source_term(a, b, c, q); };
    const uint64_t mp = __ballot(act == kTakeProxy), md = __ballot(act == kTakeDirect);
    if (mp && nd.axis >= 0) {
        // in-plane cluster: the target in the plane's frame, the proxies
        // from the plane's table
        const int a = nd.axis, ib = a == 2 ? 0 : a + 1, ic = a == 0 ? 2 : a - 1;
        const double ta = a == 0 ? x : (a == 1 ? y : z);
        const double tb = (a == 0 ? y : (a == 1 ? z : x)) - nd.c[ib];
        const double tc = (a == 0 ? z : (a == 1 ? x : y)) - nd.c[ic];
        const double ea = ta - nd.c[a];
        const double *D = reinterpret_cast<const double *>(prox + nd.proxy);
        const int nb = nd.deg[ib] + 1, nc = nd.deg[ic] + 1;
        if (64 / __popcll(mp) < 3) {
            // the row loop costs the wave 10.7 instructions per proxy, the
            // repacked loop 28 per iteration (each lane one entry of its
            // target's): repacking pays from three lanes per target (21
            // or fewer taking lanes), not from two
            if (act == kTakeProxy) plane_rows(D, nb, nc, tb, tc, ea, fma(tb, tb, fma(tc, tc, ea * ea)), acc);
        } else {
            // entry e is proxy (e / nc, e mod nc); the row by a multiply
            // and shift, exact for e < 65536 / (nc - 1) (>= 8192)
            const uint32_t inv = (65536u + (uint32_t)nc - 1u) / (uint32_t)nc;
            const auto fetch = [=](int32_t e) {
                const int32_t i = (int32_t)(((uint32_t)e * inv) >> 16), j = e - i * nc;
                const double *R = D + plane_row(nc, i);
                return PlaneEntry{R[0], D[2 * j], R[1] + D[2 * j + 1], R[2 + 2 * j], R[3 + 2 * j]};
            };
            const auto fterm = [](double b, double c, double h, const PlaneEntry &q) {
                const double d2 = fma(b, b, fma(c, c, h * h));
                const InvPowers v = inv_powers(fma(q.b2, b, fma(q.c2, c, d2 + q.p2)));
                return fma(q.pn * h, v.r2, q.q) * v.r1;
            };
            packed_sum<false>(mp, nb * nc, fetch, tb, tc, ea, acc, fterm, lx, ly, lz, part);
        }
        if (act == kTakeProxy) n_prox += nd.n_proxy;
    } else if (mp) {
        if (__popcll(mp) > 32) {
            // the taking lanes walk the proxies at wave-uniform addresses
            // (scalar loads), two per iteration
            if (act == kTakeProxy) {
                const int32_t k_end = nd.proxy + nd.n_proxy;
                int32_t k = nd.proxy;
                for (; k + 1 < k_end; k += 2) {
                    const Proxy a = prox[k], b = prox[k + 1];
                    acc += proxy_term(x, y, z, a);
                    acc += proxy_term(x, y, z, b);
                }
                if (k < k_end) acc += proxy_term(x, y, z, prox[k]);
            }
        } else {
            const Proxy *P = prox + nd.proxy;
            packed_sum(mp, nd.n_proxy, [=](int32_t e) { return P[e]; }, x, y, z, acc, pterm, lx, ly, lz, part);
        }
        if (act == kTakeProxy) n_prox += nd.n_proxy;
    }
    if (md) {
        if (__popcll(md) > 32) {
            if (act == kTakeDirect) {
                int32_t k = nd.b;
                for (; k + 1 < nd.e; k += 2) {
                    const TileSource a = src[k], b = src[k + 1];
                    acc += source_term(x, y, z, a);
                    acc += source_term(x, y, z, b);
                }
                if (k < nd.e) acc += source_term(x, y, z, src[k]);
            }
        } else {
            const TileSource *S = src + nd.b;
            packed_sum(md, nd.e - nd.b, [=](int32_t e) { return S[e]; }, x, y, z, acc, sterm, lx, ly, lz, part);
        }
        if (act == kTakeDirect) n_dir += nd.e - nd.b;
    }
}

// One wave per (group of 64 consecutive sorted targets, part).  The root
// is decided first: lanes that take it whole are done in every part (part
// 0 sums it); the others walk the part's node range.  With one part the
// wave writes u (and the counts) itself, else its part's sums.  A block
// holds kEvalWaves independent waves, each with its own LDS rows: one per
// block measured fastest (blocks of 4 waves issued VALU work 45 % of the
// cycles instead of 61 %, 5.2-5.5 ms instead of 4.1-4.7 ms per launch).
constexpr int kEvalWaves = 1;

// Target groups per part in the launch: the groups rounded up to a whole
// number of blocks per XCD (the surplus waves exit at once).
__host__ __device__ __forceinline__ int64_t eval_groups_padded(int64_t nt)
{
    const int64_t q = (int64_t)kXcds * kEvalWaves;
    return ((nt + 63) / 64 + q - 1) / q * q;
}

// Seven waves per SIMD (71 registers; the compiler's own choice, 75, allows
// six, measured ~1 % slower).
__global__ __launch_bounds__(64 * kEvalWaves) __attribute__((amdgpu_waves_per_eu(7))) void k_tree_eval(
    const TreeNode *__restrict__ nodes, const Proxy *__restrict__ prox, const TileSource *__restrict__ src,
    const double *__restrict__ targets, const uint32_t *__restrict__ order, int64_t t0, int64_t nt, int32_t n_nodes,
    double theta2, TreeParts parts, double *__restrict__ upart, int64_t *__restrict__ cpart, double *__restrict__ u,
    int64_t *__restrict__ counts)
{
    __shared__ double lx_[kEvalWaves][64], ly_[kEvalWaves][64], lz_[kEvalWaves][64], part_[kEvalWaves][64];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    // Waves in dispatch order: every group's nearest part first, then every
    // group's second nearest, ... (the nearest parts carry most of the
    // work, so the long waves start early and the short ones fill the
    // tail).  Nearness: the group's first target to the part's box centre.
    // Within a rank, the XCD that runs a block (blocks go to the XCDs in
    // turn) takes one contiguous eighth of the groups, in order: sorted
    // targets are spatially compact, so each XCD's L2 holds the clusters
    // near its own region instead of every region's.
    const int64_t n_grp = (nt + 63) / 64, n_pad = eval_groups_padded(nt);
    const int64_t per_rank = n_pad / kEvalWaves;  // blocks per rank, a multiple of kXcds
    const int r = (int)(blockIdx.x / per_rank);
    const int64_t ib = blockIdx.x - (int64_t)r * per_rank;
    const int64_t grp = xcd_contiguous(ib, wv, n_pad, kEvalWaves);
    if (grp >= n_grp) return;  // the whole wave
    double *lx = lx_[wv], *ly = ly_[wv], *lz = lz_[wv], *part = part_[wv];
    int p = 0;
    {
        const int64_t id0 = (int64_t)order[t0 + grp * 64];
        const double x0 = targets[3 * id0], y0 = targets[3 * id0 + 1], z0 = targets[3 * id0 + 2];
        double dist[kMaxParts];
        for (int q = 0; q < parts.n; ++q) {
            const TreeNode &c = nodes[min(parts.lo[q], n_nodes - 1)];
            const double dx = x0 - c.c[0], dy = y0 - c.c[1], dz = z0 - c.c[2];
            const double d2 = dx * dx + dy * dy + dz * dz;
            dist[q] = d2 == d2 ? d2 : INFINITY;  // a NaN target ranks by index (ties below)
        }
        for (int q = 0; q < parts.n; ++q) {
            int rank = 0;
            for (int o = 0; o < parts.n; ++o) rank += dist[o] < dist[q] || (dist[o] == dist[q] && o < q);
            if (rank == r) p = q;
        }
        p = __builtin_amdgcn_readfirstlane(p);
    }
    const int64_t lt = grp * 64 + __lane_id();  // position in this batch of sorted targets
    const bool valid = lt < nt;
    const int64_t id = valid ? (int64_t)order[t0 + lt] : 0;
    double x = 0.0, y = 0.0, z = 0.0;
    if (valid) {
        x = targets[3 * id];
        y = targets[3 * id + 1];
        z = targets[3 * id + 2];
    }
    double acc = 0.0;
    int64_t n_prox = 0, n_dir = 0;
    int32_t done_below = valid ? 0 : INT32_MAX;  // the lane is inside node j iff j >= done_below
    int32_t j = parts.lo[p];
    const int32_t j_end = parts.hi[p];
    if (p == 0) {
        // part 0's wave walks the root first (then its first child, node 1,
        // is part 0's first node; lanes that take the root skip everything)
        j = 0;
    } else {
        // lanes that take the root whole are done in every part
        const int act = node_action(nodes[0], valid, x, y, z, theta2);
        if (act == kTakeProxy || act == kTakeDirect) done_below = INT32_MAX;
    }
    while (j < j_end) {
        const TreeNode &nd = nodes[j];
        const int act = node_action(nd, j >= done_below, x, y, z, theta2);
        take_node(nd, act, prox, src, x, y, z, acc, n_prox, n_dir, lx, ly, lz, part);
        if (act == kTakeProxy || act == kTakeDirect) done_below = nd.skip;
        j = __any(act == kOpen) ? j + 1 : nd.skip;
    }
    if (!valid) return;
    if (parts.n == 1) {
        u[id] = acc * (1.0 / (4.0 * M_PI));
        if (counts) {
            counts[2 * id] = n_prox;
            counts[2 * id + 1] = n_dir;
        }
    } else {
        upart[p * nt + lt] = acc;
        if (cpart) {
            cpart[2 * (p * nt + lt)] = n_prox;
            cpart[2 * (p * nt + lt) + 1] = n_dir;
        }
    }
}

// Per target: the parts' sums added in part order.
__global__ __launch_bounds__(256) void k_tree_sum(const double *__restrict__ upart,
                                                  const int64_t *__restrict__ cpart, int32_t n_parts,
                                                  const uint32_t *__restrict__ order, int64_t t0, int64_t nt,
                                                  double *__restrict__ u, int64_t *__restrict__ counts)
{
    const int64_t lt = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (lt >= nt) return;
    const int64_t id = order[t0 + lt];
    double s = 0.0;
    for (int p = 0; p < n_parts; ++p) s += upart[p * nt + lt];
    u[id] = s * (1.0 / (4.0 * M_PI));
    if (counts) {
        int64_t a = 0, b = 0;
        for (int p = 0; p < n_parts; ++p) {
            a += cpart[2 * (p * nt + lt)];
            b += cpart[2 * (p * nt + lt) + 1];
        }
        counts[2 * id] = a;
        counts[2 * id + 1] = b;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Tile sources on the host: c + h (xi t1 + eta t2) for the 4 x 4 Gauss points
// (xi, eta), t2 = n x t1, source 4 a + b of a tile at (xi_a, xi_b).
// Face label of every tile source (16 per tile): 2 axis + (sign > 0) for the
// axis of the largest component of the tile's normal (the first on ties).
std::vector<int8_t> tile_faces(const dtn_patch *patches, int64_t n)
{
    std::vector<int8_t> f((size_t)n * 16);
    for (int64_t i = 0; i < n; ++i) {
        const double *nv = patches[i].n;
        int k = 0;
        for (int d = 1; d < 3; ++d)
            if (std::fabs(nv[d]) > std::fabs(nv[k])) k = d;
        std::fill(f.begin() + 16 * i, f.begin() + 16 * (i + 1), (int8_t)(2 * k + (nv[k] > 0.0 ? 1 : 0)));
    }
    return f;
}

// Per tile source: the axis its tile's normal lies exactly along (the other
// two components exactly 0), else -1.
std::vector<int8_t> tile_axes(const dtn_patch *patches, int64_t n)
{
    std::vector<int8_t> f((size_t)n * 16);
    for (int64_t i = 0; i < n; ++i) {
        const double *nv = patches[i].n;
        int a = -1;
        for (int d = 0; d < 3; ++d)
            if (nv[d] != 0.0 && nv[(d + 1) % 3] == 0.0 && nv[(d + 2) % 3] == 0.0) a = d;
        std::fill(f.begin() + 16 * i, f.begin() + 16 * (i + 1), (int8_t)a);
    }
    return f;
}

std::vector<double> tile_positions(const dtn_patch *patches, int64_t n)
{
    std::vector<double> gx, gw;
    gauss_legendre_rule(4, gx, gw);
    std::vector<double> pos((size_t)n * 16 * 3);
    for (int64_t i = 0; i < n; ++i) {
        const dtn_patch &q = patches[i];
        const double t2[3] = {q.n[1] * q.t1[2] - q.n[2] * q.t1[1], q.n[2] * q.t1[0] - q.n[0] * q.t1[2],
                              q.n[0] * q.t1[1] - q.n[1] * q.t1[0]};
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                for (int d = 0; d < 3; ++d)
                    pos[3 * (16 * (size_t)i + 4 * a + b) + d] = q.c[d] + q.h * (gx[a] * q.t1[d] + gx[b] * t2[d]);
    }
    return pos;
}

}  // namespace

struct TreeHandle {
    const Plan *plan = nullptr;
    HostTree host;
    TreeNode *d_nodes = nullptr;
    int32_t *d_slot = nullptr;
    Item *d_items = nullptr;
    ProxyCluster *d_pcl = nullptr;
    int device = 0;
};

}  // namespace dtn

struct dtn_tree_s {
    dtn::TreeHandle t;
};

using namespace dtn;

namespace {

template <class T>
hipError_t upload_vec(const std::vector<T> &v, T **out)
{
    *out = nullptr;
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void **)out, sizeof(T) * v.size());
    if (e == hipSuccess) e = hipMemcpy(*out, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
    return e;
}

void free_tree(dtn_tree t)
{
    (void)hipFree(t->t.d_nodes);
    (void)hipFree(t->t.d_slot);
    (void)hipFree(t->t.d_items);
    (void)hipFree(t->t.d_pcl);
}

}  // namespace

dtn_status dtn_create_tree(dtn_plan p, int32_t degree, int32_t leaf_size, dtn_tree *out)
{
    const std::string at = "dtn_create_tree: ";
    try {
        if (!p || !out) return fail(DTN_E_ARG, at + "NULL argument");
        *out = nullptr;
        if (degree < 1 || degree > kMaxDegree) return fail(DTN_E_ARG, at + "degree outside [1, 8]");
        if (leaf_size < 8 || leaf_size > 4096) return fail(DTN_E_ARG, at + "leaf_size outside [8, 4096]");
        const Plan &P = p->p;
        if (!P.tiles_ok)
            return fail(DTN_E_UNSUPPORTED, at + "needs square tiles on the faces of a box domain");
        if ((int64_t)P.patches.size() * 16 > (int64_t)INT32_MAX / 2) return fail(DTN_E_ARG, at + "too many tiles");
        const std::vector<double> pos = tile_positions(P.patches.data(), (int64_t)P.patches.size());
        std::unique_ptr<dtn_tree_s> T(new dtn_tree_s());
        T->t.plan = &P;
        build_tree(pos, tile_faces(P.patches.data(), (int64_t)P.patches.size()),
                   tile_axes(P.patches.data(), (int64_t)P.patches.size()), degree, leaf_size, T->t.host);
        hipError_t e = hipGetDevice(&T->t.device);
        if (e == hipSuccess) e = upload_vec(T->t.host.nodes, &T->t.d_nodes);
        if (e == hipSuccess) e = upload_vec(T->t.host.slot, &T->t.d_slot);
        if (e == hipSuccess) e = upload_vec(T->t.host.items, &T->t.d_items);
        if (e == hipSuccess) e = upload_vec(T->t.host.pcl, &T->t.d_pcl);
        if (e != hipSuccess) {
            free_tree(T.get());
            return fail(DTN_E_OOM, at + hipGetErrorString(e));
        }
        *out = T.release();
        return DTN_OK;
    } catch (const std::bad_alloc &) {
        return fail(DTN_E_OOM, at + "host allocation failed");
    } catch (...) {
        return fail(DTN_E_OOM, at + "exception");
    }
}

void dtn_destroy_tree(dtn_tree t)
{
    if (!t) return;
    free_tree(t);
    delete t;
}

dtn_status dtn_tree_layout(const dtn_patch *patches, int64_t n_patches, int32_t degree, int32_t leaf_size,
                           int64_t cap, int32_t *nodes, int32_t *perm, int64_t *n_nodes)
{
    const std::string at = "dtn_tree_layout: ";
    try {
        if (!patches || !nodes || !perm || !n_nodes) return fail(DTN_E_ARG, at + "NULL argument");
        if (n_patches < 1 || n_patches * 16 > (int64_t)INT32_MAX / 2) return fail(DTN_E_ARG, at + "bad n_patches");
        if (degree < 1 || degree > kMaxDegree) return fail(DTN_E_ARG, at + "degree outside [1, 8]");
        if (leaf_size < 8 || leaf_size > 4096) return fail(DTN_E_ARG, at + "leaf_size outside [8, 4096]");
        HostTree H;
        build_tree(tile_positions(patches, n_patches), tile_faces(patches, n_patches), tile_axes(patches, n_patches),
                   degree, leaf_size, H);
        *n_nodes = (int64_t)H.nodes.size();
        if ((int64_t)H.nodes.size() > cap) return fail(DTN_E_ARG, at + "cap below the number of nodes");
        for (size_t j = 0; j < H.nodes.size(); ++j) {
            const TreeNode &nd = H.nodes[j];
            const int32_t row[8] = {nd.b, nd.e, nd.skip, nd.leaf, nd.deg[0], nd.deg[1], nd.deg[2], nd.proxy};
            std::copy(row, row + 8, nodes + 8 * j);
        }
        std::copy(H.perm.begin(), H.perm.end(), perm);
        return DTN_OK;
    } catch (...) {
        return fail(DTN_E_OOM, at + "exception");
    }
}

dtn_status dtn_tree_info(dtn_tree t, int64_t info[4])
{
    if (!t || !info) return fail(DTN_E_ARG, "dtn_tree_info: NULL argument");
    info[0] = (int64_t)t->t.host.nodes.size();
    info[1] = (int64_t)t->t.host.pcl.size();
    info[2] = t->t.host.n_proxies;
    info[3] = (int64_t)t->t.host.perm.size();
    return DTN_OK;
}

dtn_status dtn_tree_potential(dtn_tree t, const double *neumann, const double *targets, int64_t m, double theta,
                              double *u_out, int64_t *counts, void *stream)
{
    const std::string at = "dtn_tree_potential: ";
    try {
        if (!t) return fail(DTN_E_ARG, at + "NULL tree");
        if (m < 0 || m > (int64_t)INT32_MAX) return fail(DTN_E_ARG, at + "m outside [0, 2^31)");
        if (!(theta > 0.0 && theta < 1.0)) return fail(DTN_E_ARG, at + "theta outside (0, 1)");
        if (m > 0 && (!neumann || !targets || !u_out)) return fail(DTN_E_ARG, at + "NULL array");
        if (m == 0) return DTN_OK;
        const hipStream_t s = (hipStream_t)stream;
        const HostTree &H = t->t.host;
        const int64_t n_src = (int64_t)H.perm.size();
        size_t sort_bytes = 0;
        hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (const uint32_t *)nullptr,
                                                          (uint32_t *)nullptr, (const uint32_t *)nullptr,
                                                          (uint32_t *)nullptr, (int)m, 0, 30, s);
        if (e != hipSuccess) return fail(DTN_E_DEVICE, at + hipGetErrorString(e));
        // targets per eval batch: the parts' partial sums of a batch stay
        // within a few hundred MB
        const TreeParts &P = H.parts;
        const int64_t batch = std::min<int64_t>(m, kEvalBatch);
        const int64_t n_up = P.n > 1 ? (int64_t)P.n * batch : 1;
        const int nb_box = (int)std::min<int64_t>(64, (m + 255) / 256);
        const size_t o_src = 0;
        const size_t o_part = o_src + align256(sizeof(TileSource) * (size_t)n_src);
        const size_t o_prox = o_part + align256(sizeof(double) * (size_t)std::max<int64_t>(H.part_len, 1));
        const size_t o_keys = o_prox + align256(sizeof(Proxy) * (size_t)std::max<int64_t>(H.n_proxies, 1));
        const size_t o_sorted = o_keys + align256(sizeof(uint32_t) * (size_t)m);
        const size_t o_ids = o_sorted + align256(sizeof(uint32_t) * (size_t)m);
        const size_t o_order = o_ids + align256(sizeof(uint32_t) * (size_t)m);
        const size_t o_rows = o_order + align256(sizeof(uint32_t) * (size_t)m);
        const size_t o_tbox = o_rows + align256(sizeof(double) * 6 * (size_t)nb_box);
        const size_t o_up = o_tbox + align256(sizeof(double) * 6);
        const size_t o_cp = o_up + align256(sizeof(double) * (size_t)n_up);
        const size_t o_tmp = o_cp + (counts && P.n > 1 ? align256(2 * sizeof(int64_t) * (size_t)n_up) : 0);
        const size_t bytes = o_tmp + align256(std::max<size_t>(sort_bytes, 1));
        char *w = nullptr;
        e = hipMallocAsync((void **)&w, bytes, s);
        if (e != hipSuccess) return fail(DTN_E_OOM, at + hipGetErrorString(e));
        TileSource *src = (TileSource *)(w + o_src);
        double *part = (double *)(w + o_part);
        Proxy *prox = (Proxy *)(w + o_prox);
        uint32_t *keys = (uint32_t *)(w + o_keys), *sorted = (uint32_t *)(w + o_sorted);
        uint32_t *ids = (uint32_t *)(w + o_ids), *order = (uint32_t *)(w + o_order);
        double *rows = (double *)(w + o_rows), *tbox = (double *)(w + o_tbox);
        double *upart = P.n > 1 ? (double *)(w + o_up) : nullptr;
        int64_t *cpart = counts && P.n > 1 ? (int64_t *)(w + o_cp) : nullptr;
        dtn_status st = launch_tile_sources(*t->t.plan, neumann, t->t.d_slot, src, s);
        if (st != DTN_OK) {
            (void)hipFreeAsync(w, s);
            return st;
        }
        const double theta2 = theta * theta;
        hipLaunchKernelGGL(k_tree_tbox_partial, dim3((unsigned)nb_box), dim3(256), 0, s, targets, m, rows);
        hipLaunchKernelGGL(k_tree_tbox_final, dim3(1), dim3(64), 0, s, rows, (int32_t)nb_box, tbox);
        if (!H.items.empty()) {
            hipLaunchKernelGGL(k_tree_proxy_partial, dim3((unsigned)H.items.size()), dim3(kProxyThreads), 0, s,
                               t->t.d_nodes, t->t.d_items, src, tbox, theta2, part);
            hipLaunchKernelGGL(k_tree_proxy_reduce, dim3((unsigned)H.pcl.size()), dim3(kProxyThreads), 0, s,
                               t->t.d_nodes, t->t.d_pcl, t->t.d_items, part, tbox, theta2, prox);
        }
        double sc[3];
        for (int d = 0; d < 3; ++d) sc[d] = H.box_ext[d] > 0.0 ? 1024.0 / H.box_ext[d] : 0.0;
        hipLaunchKernelGGL(k_tree_keys, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, targets, m, H.box_lo[0],
                           H.box_lo[1], H.box_lo[2], sc[0], sc[1], sc[2], keys, ids);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipcub::DeviceRadixSort::SortPairs((void *)(w + o_tmp), sort_bytes, keys, sorted, ids, order, (int)m,
                                                   0, 30, s);
        for (int64_t t0 = 0; e == hipSuccess && t0 < m; t0 += batch) {
            const int64_t nt = std::min(batch, m - t0);
            const int64_t blocks = eval_groups_padded(nt) / kEvalWaves * P.n;
            hipLaunchKernelGGL(k_tree_eval, dim3((unsigned)blocks),
                               dim3(64 * kEvalWaves), 0, s, t->t.d_nodes, prox, src, targets, order, t0, nt,
                               (int32_t)H.nodes.size(), theta2, P, upart, cpart, u_out, counts);
            if (P.n > 1)
                hipLaunchKernelGGL(k_tree_sum, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, upart, cpart,
                                   P.n, order, t0, nt, u_out, counts);
            e = hipGetLastError();
        }
        const hipError_t ef = hipFreeAsync(w, s);
        if (e == hipSuccess) e = ef;
        if (e != hipSuccess) return fail(DTN_E_DEVICE, at + hipGetErrorString(e));
        return DTN_OK;
    } catch (...) {
        return fail(DTN_E_OOM, at + "exception");
    }
}
