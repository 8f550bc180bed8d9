"""Oracle for the treecode evaluation of the potential (test infrastructure only).

TEST INFRASTRUCTURE ONLY: plain numpy; only the test suite, the smoke check
and the benchmark's CPU baseline may import it.  It shares nothing with the
HIP library.

The paper evaluates the final potential (eq. bw03) directly and names a
fast multipole method as the way to scale it (Sec. 6, conclusion); it fixes
no algorithm.  The reading taken is a kernel-independent treecode with
barycentric Lagrange interpolation on Chebyshev points (Wang, Krasny &
Tlupova, Commun. Comput. Phys. 28, 2020), stated here in its plain form:

  sources    the tile quadrature points y_j of the direct sum, each with a
             single-layer weight a_j = w_j sigma_j and a double-layer vector
             b_j = -w_j phi_j n_j, so that
               u(x) = sum_j [a_j / |x - y_j| + b_j . (x - y_j) / |x - y_j|^3] / (4 pi);
  tree       the root's children are the boundary's faces: one cluster per
             face label of the sources (the face of a tile is the axis of
             its normal's largest component and that component's sign,
             label 2 axis + (sign > 0)), in increasing label order, each
             keeping its sources in input order.  Below them, clusters
             split at the midpoint of their tight bounding box along every
             dimension whose extent is at least the largest extent /
             sqrt(2), children ordered by their octant code (bit d set for
             the upper half in dimension d), until a cluster holds at most
             leaf_size sources (or cannot be split).  A face cluster lies in
             one plane, so its proxy grid and those of all its descendants
             are two-dimensional (degree 0 along the normal): the reading
             taken for this design choice, which the paper leaves open, is
             that clusters never straddle an edge of the box;
  proxies    per cluster, a tensor grid of Chebyshev points of the second
             kind on the box padded by 1e-12 of the root extent, degree n in
             each dimension whose tight extent exceeds 1e-9 of the largest
             (degree 0, the box centre, otherwise).  With L_k the tensor
             Lagrange basis of that grid (barycentric second form),
               q_k = sum_j L_k(y_j) a_j,   p_k = sum_j L_k(y_j) b_j,
             which interpolates y -> 1/|x - y| and its y-gradient;
  traversal  for a target x and a cluster C with centre c (of the padded
             box) and radius r (half its diagonal): if r < theta |x - c|,
             use the proxies when C has more sources than proxies, else its
             sources directly; otherwise recurse into the children (a leaf
             is summed directly).
"""
import numpy as np

from . import potential as POT

FOUR_PI = 4.0 * np.pi
PAD_REL = 1e-12
FLAT_REL = 1e-9


def cheb_nodes(lo, hi, n):
    """Chebyshev points of the second kind on [lo, hi] (the centre for n = 0)."""
    if n == 0:
        return np.array([0.5 * (lo + hi)])
    return 0.5 * (lo + hi) + 0.5 * (hi - lo) * np.cos(np.pi * np.arange(n + 1) / n)


def bary_weights(n):
    """Barycentric weights of those points: (-1)^k, halved at both ends."""
    if n == 0:
        return np.ones(1)
    w = (-1.0) ** np.arange(n + 1)
    w[0] *= 0.5
    w[-1] *= 0.5
    return w


def lagrange_1d(y, nodes, w):
    """Lagrange basis values [m][n+1] at the points y (second barycentric
    form; exactly the unit vector at a point that equals a node)."""
    y = np.asarray(y, dtype=np.float64)
    d = y[:, None] - nodes[None, :]
    hit = d == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        t = w[None, :] / d
        L = t / np.sum(t, axis=1, keepdims=True)
    rows = np.any(hit, axis=1)
    L[rows] = hit[rows].astype(np.float64)
    return L


class Cluster:
    def __init__(self, idx, y, pad, degree, leaf_size, groups=None):
        self.idx = idx
        P = y[idx]
        tlo, thi = P.min(axis=0), P.max(axis=0)
        ext = thi - tlo
        self.lo, self.hi = tlo - pad, thi + pad
        self.center = 0.5 * (self.lo + self.hi)
        self.radius = 0.5 * np.linalg.norm(self.hi - self.lo)
        big = ext.max()
        self.deg = [degree if ext[d] > FLAT_REL * big else 0 for d in range(3)]
        self.n_proxy = int(np.prod([k + 1 for k in self.deg]))
        self.children = []
        if groups is not None:
            for c in np.unique(groups):
                self.children.append(Cluster(idx[groups == c], y, pad, degree, leaf_size))
        elif len(idx) > leaf_size and big > 0.0:
            mid = 0.5 * (tlo + thi)
            code = np.zeros(len(idx), dtype=np.int64)
            for d in range(3):
                if ext[d] >= big / np.sqrt(2.0):
                    code |= (P[:, d] >= mid[d]).astype(np.int64) << d
            for c in np.unique(code):
                self.children.append(Cluster(idx[code == c], y, pad, degree, leaf_size))
        self.has_proxy = len(idx) > self.n_proxy

    def proxies(self, y, a, b):
        """Proxy points [K][3], charges q [K] and vectors p [K][3]."""
        grids, Ls = [], []
        for d in range(3):
            nodes = cheb_nodes(self.lo[d], self.hi[d], self.deg[d])
            grids.append(nodes)
            Ls.append(lagrange_1d(y[self.idx, d], nodes, bary_weights(self.deg[d])))
        L = np.einsum("ja,jb,jc->jabc", Ls[0], Ls[1], Ls[2]).reshape(len(self.idx), -1)
        S = np.stack(np.meshgrid(*grids, indexing="ij"), axis=-1).reshape(-1, 3)
        return S, L.T @ a[self.idx], L.T @ b[self.idx]


def build_tree(y, faces, leaf_size=64, degree=6):
    """The tree over the sources y with face labels `faces` (one per source)."""
    y = np.asarray(y, dtype=np.float64)
    pad = PAD_REL * float((y.max(axis=0) - y.min(axis=0)).max())
    return Cluster(np.arange(len(y)), y, pad, degree, leaf_size, groups=np.asarray(faces))


def face_label(n):
    """Face label of a tile with normal n: 2 axis + (sign > 0) for the axis
    of the largest component (the first such axis on ties)."""
    n = np.asarray(n, dtype=np.float64)
    k = int(np.argmax(np.abs(n)))
    return 2 * k + int(n[k] > 0.0)


def _direct(x, y, a, b):
    d = x[None, :] - y
    r = np.linalg.norm(d, axis=-1)
    return np.sum(a / r + np.sum(b * d, axis=-1) / r ** 3)


def evaluate(tree, y, a, b, targets, theta):
    """u at the targets by the traversal above; also the number of proxy and
    direct interactions per target."""
    y = np.asarray(y, dtype=np.float64)
    cache = {}
    out = np.empty(len(targets))
    counts = np.zeros((len(targets), 2), dtype=np.int64)

    def visit(C, x, k):
        if C.radius < theta * np.linalg.norm(x - C.center):
            if C.has_proxy:
                if id(C) not in cache:
                    cache[id(C)] = C.proxies(y, a, b)
                S, q, p = cache[id(C)]
                counts[k, 0] += len(q)
                return _direct(x, S, q, p)
            counts[k, 1] += len(C.idx)
            return _direct(x, y[C.idx], a[C.idx], b[C.idx])
        if not C.children:
            counts[k, 1] += len(C.idx)
            return _direct(x, y[C.idx], a[C.idx], b[C.idx])
        return sum(visit(ch, x, k) for ch in C.children)

    for k, x in enumerate(np.asarray(targets, dtype=np.float64).reshape(-1, 3)):
        out[k] = visit(tree, x, k) / FOUR_PI
    return out, counts


def tile_sources(patches, sigmas, geom):
    """The direct sum's sources: points, single-layer weights a, double-layer
    vectors b (the oracle's tile quadrature of eq. bw03)."""
    ys, As, Bs = [], [], []
    for p, s in zip(patches, sigmas):
        yq, nq, wq, sq, fq = POT.tile_quadrature(p, s, geom)
        ys.append(yq)
        As.append(wq * sq)
        Bs.append(-(wq * fq)[:, None] * nq)
    return np.concatenate(ys), np.concatenate(As), np.concatenate(Bs)


def tile_faces(patches):
    """Face label of every source of tile_sources (its tile's label)."""
    return np.concatenate([np.full(16, face_label(p.n)) for p in patches])


def potential_tree(patches, sigmas, geom, targets, theta=0.5, degree=6, leaf_size=64):
    """u at the targets from the tiles' Neumann data, by the treecode."""
    y, a, b = tile_sources(patches, sigmas, geom)
    tree = build_tree(y, tile_faces(patches), leaf_size, degree)
    return evaluate(tree, y, a, b, targets, theta)[0]
