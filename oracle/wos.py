"""Python face of the oracle's walk-on-spheres code (test infrastructure only).

Thin ctypes marshalling around ``wos_oracle.c``; all arithmetic is in the C
file.  See that file's header for the passages of the paper it follows
(Sec. 2 eq. bw13 and the epsilon-shell WOS; Sec. 5.1.2 eq. bw87).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int64)
        up = C.POINTER(C.c_uint32)
        gp = C.POINTER(OgGeom)
        L.og_wos_nodes.argtypes = [gp, dp, C.c_int64, ip, ip, C.c_uint64, up, dp, dp, dp, ip, ip, C.c_int]
        L.og_wos_nodes.restype = None
        L.og_wos_scores.argtypes = [gp, dp, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, dp, ip]
        L.og_phi_many.argtypes = [gp, dp, C.c_int64, dp]
        L.og_dist_proj_many.argtypes = [gp, dp, C.c_int64, dp, dp]
        L.og_philox_many.argtypes = [up, C.c_int64, C.c_uint64, up]
        L.og_direction_many.argtypes = [dp, C.c_int64, dp]
        L.og_max_threads.restype = C.c_int
        _lib = L
    return _lib


class OgGeom(C.Structure):
    _fields_ = [
        ("kind", C.c_int32),
        ("data_kind", C.c_int32),
        ("ball_c", C.c_double * 3),
        ("ball_r", C.c_double),
        ("box_lo", C.c_double * 3),
        ("box_hi", C.c_double * 3),
        ("n_holes", C.c_int32),
        ("n_src", C.c_int32),
        ("holes", C.POINTER(C.c_double)),
        ("src", C.POINTER(C.c_double)),
        ("quad", C.c_double * 10),
        ("eps", C.c_double),
        ("max_steps", C.c_int64),
        ("disk_r", C.c_double),
        ("trunc_r", C.c_double),
        ("tab_n0", C.c_int32),
        ("tab_n1", C.c_int32),
        ("tab", C.POINTER(C.c_double)),
    ]


KIND = {"ball": 0, "box": 1, "box_minus_boxes": 2, "half_space": 3, "disk": 4, "ball_exterior": 5}


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _uptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


class Geometry:
    """Domain, Dirichlet data, epsilon and step cap, as a plain description.

    ``desc`` is the dictionary produced by ``dtn_inputs`` (keys ``kind``,
    ``ball_c``, ``ball_r``, ``box_lo``, ``box_hi``, ``holes``, ``data_kind``,
    ``quad``, ``src``, ``eps``, ``max_steps``).
    """

    def __init__(self, desc):
        self.desc = desc
        g = OgGeom()
        g.kind = KIND[desc["kind"]]
        g.data_kind = {"quadratic": 0, "sources": 1, "table": 2}[desc["data_kind"]]
        for k in range(3):
            g.ball_c[k] = float(desc.get("ball_c", (0, 0, 0))[k])
            g.box_lo[k] = float(desc.get("box_lo", (0, 0, 0))[k])
            g.box_hi[k] = float(desc.get("box_hi", (1, 1, 1))[k])
        g.ball_r = float(desc.get("ball_r", 1.0))
        self._holes = np.ascontiguousarray(np.asarray(desc.get("holes", np.zeros((0, 6))), dtype=np.float64).reshape(-1, 6))
        self._src = np.ascontiguousarray(np.asarray(desc.get("src", np.zeros((0, 4))), dtype=np.float64).reshape(-1, 4))
        g.n_holes = self._holes.shape[0]
        g.n_src = self._src.shape[0]
        g.holes = _dptr(self._holes)
        g.src = _dptr(self._src)
        q = desc.get("quad", [0.0] * 10)
        for k in range(10):
            g.quad[k] = float(q[k])
        g.eps = float(desc["eps"])
        g.max_steps = int(desc["max_steps"])
        g.disk_r = float(desc.get("disk_r", 0.0))
        g.trunc_r = float(desc.get("trunc_r", 0.0))
        self._tab = np.ascontiguousarray(np.asarray(desc.get("tab", np.zeros((6, 2, 2))), dtype=np.float64))
        if self._tab.ndim != 3 or self._tab.shape[0] != 6:
            raise ValueError("tab must be [6][n0][n1]")
        g.tab_n0, g.tab_n1 = int(self._tab.shape[1]), int(self._tab.shape[2])
        g.tab = _dptr(self._tab)
        self.g = g

    def ref(self):
        return C.byref(self.g)

    def phi(self, x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3))
        out = np.empty(x.shape[0])
        lib().og_phi_many(self.ref(), _dptr(x), x.shape[0], _dptr(out))
        return out

    def dist_proj(self, x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3))
        d = np.empty(x.shape[0])
        p = np.empty_like(x)
        lib().og_dist_proj_many(self.ref(), _dptr(x), x.shape[0], _dptr(d), _dptr(p))
        return d, p


def philox(ctr, seed):
    """Philox4x32-10 blocks for counters ``ctr`` [n,4] (uint32) and a 64-bit seed."""
    ctr = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    out = np.empty_like(ctr)
    lib().og_philox_many(_uptr(ctr), ctr.shape[0], C.c_uint64(int(seed)), _uptr(out))
    return out


def direction(u):
    """Uniform directions from uniform pairs ``u`` [n,2]."""
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1, 2))
    w = np.empty((u.shape[0], 3))
    lib().og_direction_many(_dptr(u), u.shape[0], _dptr(w))
    return w


def wos_nodes(geom, pts, walks, seed, stream_id=None, walk_begin=None, threads=0):
    """Node statistics from WOS walks (eq. bw87 plus variance).

    Returns a dict of arrays: count, mean, m2, steps, capped, se.
    ``stream_id`` defaults to the point index; ``walk_begin`` to 0.
    """
    pts = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
    n = pts.shape[0]
    walks = np.ascontiguousarray(np.broadcast_to(np.asarray(walks, dtype=np.int64), (n,)).copy())
    wb = None if walk_begin is None else np.ascontiguousarray(
        np.broadcast_to(np.asarray(walk_begin, dtype=np.int64), (n,)).copy())
    sid = None if stream_id is None else np.ascontiguousarray(np.asarray(stream_id, dtype=np.uint32).reshape(n))
    count = np.empty(n)
    mean = np.empty(n)
    m2 = np.empty(n)
    steps = np.empty(n, dtype=np.int64)
    capped = np.empty(n, dtype=np.int64)
    lib().og_wos_nodes(geom.ref(), _dptr(pts), n, None if wb is None else _iptr(wb), _iptr(walks),
                       C.c_uint64(int(seed)), None if sid is None else _uptr(sid),
                       _dptr(count), _dptr(mean), _dptr(m2), _iptr(steps), _iptr(capped), int(threads))
    with np.errstate(invalid="ignore", divide="ignore"):
        var = np.where(count > 1, m2 / np.maximum(count - 1, 1), np.nan)
        se = np.sqrt(var / count)
    return {"count": count, "mean": mean, "m2": m2, "steps": steps, "capped": capped, "se": se}


def wos_adaptive(geom, pts, pilot_walks, min_walks, max_walks, se_target, seed, stream_id=None, threads=0):
    """Node statistics with an adaptive walk count per node.

    The standard error of the node estimate (eq. bw87) is sqrt(var / n).  A
    pilot of ``pilot_walks`` walks estimates var (unbiased); the node then
    gets n = clamp(ceil(var / se_target^2), min_walks, max_walks) walks in
    all, never fewer than the pilot, and the statistics are those of walks
    [0, n) of the node, in one pass.  Returns wos_nodes' dict plus
    ``walks_used``.
    """
    pts = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
    pilot = wos_nodes(geom, pts, pilot_walks, seed, stream_id=stream_id, threads=threads)
    var = np.where(pilot["count"] > 1, pilot["m2"] / (pilot["count"] - 1.0), 0.0)
    want = np.ceil(var / (float(se_target) * float(se_target)))
    total = np.empty(pts.shape[0], dtype=np.int64)
    for i, w in enumerate(want):
        if not (w < max_walks):
            total[i] = max_walks
        elif w <= min_walks:
            total[i] = min_walks
        else:
            total[i] = int(w)
    total = np.maximum(total, int(pilot_walks))
    r = wos_nodes(geom, pts, total, seed, stream_id=stream_id, threads=threads)
    r["walks_used"] = total
    return r


def wos_scores(geom, y, seed, stream_id, walk_begin, n_walks):
    """Per-walk recorded phi and step counts from one start point."""
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(3))
    score = np.empty(int(n_walks))
    steps = np.empty(int(n_walks), dtype=np.int64)
    lib().og_wos_scores(geom.ref(), _dptr(y), C.c_uint64(int(seed)), C.c_uint32(int(stream_id)),
                        int(walk_begin), int(n_walks), _dptr(score), _iptr(steps))
    return score, steps


def max_threads():
    return int(lib().og_max_threads())
