"""Python binding of libdtn (the HIP library for the local DtN method).

Argument marshalling only: every step runs in the library's HIP kernels, on
torch's current HIP stream, with device memory owned by torch tensors.  The
library must have been built (``paper_1210_1491_amd.build``); importing this
module fails loudly when it has not.  There is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np
import torch

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdtn.so")

DTN_OK = 0
STATUS = {0: "DTN_OK", -1: "DTN_E_ARG", -2: "DTN_E_DEVICE", -3: "DTN_E_OOM", -4: "DTN_E_UNSUPPORTED",
          -5: "DTN_E_NOCONV", -6: "DTN_E_MAXSTEPS"}
KIND = {"ball": 0, "box": 1, "box_minus_boxes": 2, "half_space": 3, "disk": 4, "ball_exterior": 5}
DATA = {"quadratic": 0, "sources": 1, "table": 2}
PRECISION = {"fp64": 0, "fp32": 1, "fp32_mixed": 1}


class DtnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GeometryDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("data_kind", C.c_int32), ("ball_c", C.c_double * 3),
                ("ball_r", C.c_double), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
                ("n_holes", C.c_int32), ("n_src", C.c_int32), ("holes", C.POINTER(C.c_double)),
                ("src", C.POINTER(C.c_double)), ("quad_coef", C.c_double * 10), ("eps", C.c_double),
                ("max_steps", C.c_int64), ("disk_r", C.c_double), ("trunc_r", C.c_double),
                ("tab_n", C.c_int32 * 2), ("tab", C.POINTER(C.c_double))]


class PatchDesc(C.Structure):
    _fields_ = [("c", C.c_double * 3), ("n", C.c_double * 3), ("t1", C.c_double * 3), ("h", C.c_double),
                ("n_theta", C.c_int32), ("n_phi", C.c_int32), ("n_rings", C.c_int32), ("n_sectors", C.c_int32)]


assert C.sizeof(PatchDesc) == 96


class PointDesc(C.Structure):
    _fields_ = [("c", C.c_double * 3), ("n", C.c_double * 3), ("t1", C.c_double * 3), ("a", C.c_double)]


class ScheduleDesc(C.Structure):
    _fields_ = [("min_chunk", C.c_int64), ("oversub", C.c_int32), ("reserved", C.c_int32)]


class AdaptiveDesc(C.Structure):
    _fields_ = [("pilot_walks", C.c_int64), ("min_walks", C.c_int64), ("max_walks", C.c_int64),
                ("se_target", C.c_double)]


class ServerConfigDesc(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("precision", C.c_int32), ("hbm_budget", C.c_int64),
                ("pilot_walks", C.c_int64), ("min_walks", C.c_int64), ("max_walks", C.c_int64),
                ("h_max", C.c_double), ("ladder", C.c_int32), ("n_theta", C.c_int32), ("n_phi", C.c_int32),
                ("n_rings", C.c_int32), ("n_sectors", C.c_int32), ("max_points", C.c_int64),
                ("graph_replay", C.c_int32), ("max_batch_queries", C.c_int32), ("n_g1", C.c_int32),
                ("n_g2", C.c_int32), ("delta_rel", C.c_double)]


class QueryDoneDesc(C.Structure):
    _fields_ = [("query_id", C.c_uint64), ("status", C.c_int32), ("reserved", C.c_int32),
                ("n_points", C.c_int64), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double)]


def schedule_struct(sched):
    """dict(min_chunk=..., oversub=...) (or None) -> ScheduleDesc (or None)."""
    if sched is None:
        return None
    return ScheduleDesc(int(sched.get("min_chunk", 512)), int(sched.get("oversub", 4)), 0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (python -c "
                              "'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.dtn_last_error.restype = C.c_char_p
        L.dtn_version.restype = C.c_char_p
        # the argument lists below follow the header beside the package: a
        # library built against another version of it is refused
        if os.path.exists(_build.HEADER):
            want, got = _build.header_digest(), L.dtn_version().decode().rsplit(" ", 1)[-1]
            if got != want:
                raise ImportError(f"{LIB_PATH} was built against another include/dtn.h (digest {got}, the header "
                                  f"has {want}): rebuild it (python -c 'import __graft_entry__ as g; g.build()')")
        L.dtn_create_geometry.argtypes = [C.POINTER(GeometryDesc), C.POINTER(vp)]
        L.dtn_destroy_geometry.argtypes = [vp]
        L.dtn_destroy_geometry.restype = None
        L.dtn_wos_eval.argtypes = [vp, vp, C.c_int64, vp, vp, C.c_uint64, vp, C.c_int32, vp, vp, vp]
        L.dtn_wos_adaptive.argtypes = [vp, vp, C.c_int64, C.POINTER(AdaptiveDesc), C.c_uint64, vp, C.c_int32,
                                       C.POINTER(ScheduleDesc), vp, vp, vp, vp]
        L.dtn_wos_time_schedules.argtypes = [vp, vp, C.c_int64, vp, vp, C.c_uint64, vp, C.c_int32,
                                             C.POINTER(ScheduleDesc), C.c_int32, C.c_int32, vp,
                                             C.POINTER(C.c_float), vp]
        L.dtn_boundary_distance.argtypes = [vp, vp, C.c_int64, C.c_int32, vp, vp]
        L.dtn_server_create.argtypes = [vp, C.POINTER(ServerConfigDesc), C.POINTER(vp)]
        L.dtn_server_destroy.argtypes = [vp]
        L.dtn_server_destroy.restype = None
        L.dtn_server_footprint.argtypes = [C.POINTER(ServerConfigDesc), C.c_int64]
        L.dtn_server_footprint.restype = C.c_int64
        L.dtn_server_clock.argtypes = [vp]
        L.dtn_server_clock.restype = C.c_double
        L.dtn_server_submit.argtypes = [vp, C.c_uint64, vp, vp, C.c_int64, C.c_double, C.c_uint64, vp]
        L.dtn_server_wait.argtypes = [vp, C.c_int64, C.c_double, C.POINTER(QueryDoneDesc), C.POINTER(C.c_int64)]
        L.dtn_create_plan.argtypes = [vp, C.POINTER(PatchDesc), C.c_int64, C.POINTER(vp)]
        L.dtn_destroy_plan.argtypes = [vp]
        L.dtn_destroy_plan.restype = None
        L.dtn_plan_num_nodes.argtypes = [vp]
        L.dtn_plan_num_nodes.restype = C.c_int64
        L.dtn_plan_num_panels.argtypes = [vp]
        L.dtn_plan_num_panels.restype = C.c_int64
        L.dtn_patch_nodes.argtypes = [vp, vp, vp]
        L.dtn_patch_solve.argtypes = [vp, vp, C.c_int32, vp, vp, vp]
        L.dtn_potential.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
        L.dtn_patch_solve_second_kind.argtypes = [vp, vp, vp, vp, vp]
        L.dtn_class_second_kind.argtypes = [C.c_int32] * 4 + [C.c_double] + [C.POINTER(C.c_double)] * 3
        L.dtn_create_points.argtypes = [vp, C.POINTER(PointDesc), C.c_int64, C.c_int32, C.c_int32, C.c_double,
                                        C.POINTER(vp)]
        L.dtn_destroy_points.argtypes = [vp]
        L.dtn_destroy_points.restype = None
        L.dtn_points_num_nodes.argtypes = [vp]
        L.dtn_points_num_nodes.restype = C.c_int64
        L.dtn_points_nodes.argtypes = [vp, vp, vp]
        L.dtn_points_neumann.argtypes = [vp, vp, vp, vp]
        L.dtn_create_tree.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(vp)]
        L.dtn_destroy_tree.argtypes = [vp]
        L.dtn_destroy_tree.restype = None
        L.dtn_tree_info.argtypes = [vp, C.POINTER(C.c_int64)]
        L.dtn_tree_potential.argtypes = [vp, vp, vp, C.c_int64, C.c_double, vp, vp, vp]
        L.dtn_tree_layout.argtypes = [C.POINTER(PatchDesc), C.c_int64, C.c_int32, C.c_int32, C.c_int64, vp, vp,
                                      C.POINTER(C.c_int64)]
        dp = C.POINTER(C.c_double)
        L.dtn_class_operators.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                          dp, dp, dp, dp, dp, dp]
        L.dtn_check.argtypes = [vp, vp]
        L.dtn_walk_counters.argtypes = [vp, vp, C.c_int32, C.POINTER(C.c_int64)]
        L.dtn_wos_eval_noalloc.argtypes = [vp, vp, C.c_int64, vp, vp, C.c_uint64, vp, C.c_int32, vp, vp, vp]
        L.dtn_plan_set_max_sweeps.argtypes = [vp, C.c_int32]
        for f in ("dtn_create_geometry", "dtn_wos_eval", "dtn_wos_adaptive", "dtn_wos_time_schedules",
                  "dtn_boundary_distance", "dtn_server_create", "dtn_server_submit", "dtn_server_wait",
                  "dtn_create_plan", "dtn_patch_nodes",
                  "dtn_patch_solve", "dtn_patch_solve_second_kind", "dtn_class_second_kind", "dtn_potential",
                  "dtn_create_tree", "dtn_tree_info", "dtn_tree_potential", "dtn_tree_layout",
                  "dtn_class_operators",
                  "dtn_create_points",
                  "dtn_points_nodes", "dtn_points_neumann", "dtn_check", "dtn_plan_set_max_sweeps", "dtn_walk_counters",
                  "dtn_wos_eval_noalloc"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(status, what):
    if status != DTN_OK:
        raise DtnError(status, f"{what}: {lib().dtn_last_error().decode()}")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_tensor(t, dtype, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def version():
    return lib().dtn_version().decode()


class Geometry:
    """Domain, Dirichlet data, eps and step cap on the current device."""

    def __init__(self, desc):
        d = GeometryDesc()
        d.kind = KIND[desc["kind"]]
        d.data_kind = DATA[desc["data_kind"]]
        for k in range(3):
            d.ball_c[k] = float(desc.get("ball_c", (0, 0, 0))[k])
            d.box_lo[k] = float(desc.get("box_lo", (0, 0, 0))[k])
            d.box_hi[k] = float(desc.get("box_hi", (1, 1, 1))[k])
        d.ball_r = float(desc.get("ball_r", 1.0))
        self._holes = np.ascontiguousarray(np.asarray(desc.get("holes", np.zeros((0, 6))), np.float64).reshape(-1, 6))
        self._src = np.ascontiguousarray(np.asarray(desc.get("src", np.zeros((0, 4))), np.float64).reshape(-1, 4))
        d.n_holes = self._holes.shape[0]
        d.n_src = self._src.shape[0]
        d.holes = self._holes.ctypes.data_as(C.POINTER(C.c_double))
        d.src = self._src.ctypes.data_as(C.POINTER(C.c_double))
        for k, v in enumerate(desc.get("quad", [0.0] * 10)):
            d.quad_coef[k] = float(v)
        d.eps = float(desc["eps"])
        d.max_steps = int(desc["max_steps"])
        d.disk_r = float(desc.get("disk_r", 0.0))
        d.trunc_r = float(desc.get("trunc_r", 0.0))
        if desc["data_kind"] == "table":
            self._tab = np.ascontiguousarray(np.asarray(desc["tab"], np.float64))
            d.tab_n[0], d.tab_n[1] = int(self._tab.shape[1]), int(self._tab.shape[2])
            d.tab = self._tab.ctypes.data_as(C.POINTER(C.c_double))
        self.desc = desc
        self.handle = C.c_void_p()
        _check(lib().dtn_create_geometry(C.byref(d), C.byref(self.handle)), "dtn_create_geometry")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.dtn_destroy_geometry(h)
            self.handle = None


def wos_eval(geom, pts, walks, seed, walk_begin=None, stream_id=None, precision="fp64", stats=None,
             capped=None):
    """Step 1: node statistics (count, mean, M2, steps) from WOS walks.

    pts [n,3] f64, walks [n] int64, walk_begin [n] int64 or None,
    stream_id [n] int32 (bit pattern of uint32) or None; all on the device.
    Returns (stats [n,4] f64, capped [n] int64)."""
    n = pts.shape[0]
    _dev_tensor(pts, torch.float64, (n, 3))
    _dev_tensor(walks, torch.int64, (n,))
    if walk_begin is not None:
        _dev_tensor(walk_begin, torch.int64, (n,))
    if stream_id is not None:
        _dev_tensor(stream_id, torch.int32, (n,))
    if stats is None:
        stats = torch.empty((n, 4), dtype=torch.float64, device=pts.device)
    if capped is None:
        capped = torch.empty((n,), dtype=torch.int64, device=pts.device)
    _check(lib().dtn_wos_eval(geom.handle, _ptr(pts), n, _ptr(walks), _ptr(walk_begin),
                              C.c_uint64(int(seed) & (2 ** 64 - 1)), _ptr(stream_id), PRECISION[precision],
                              _ptr(stats), _ptr(capped), _stream()), "dtn_wos_eval")
    return stats, capped


def wos_eval_noalloc(geom, pts, walks, seed, stats, capped, walk_begin=None, stream_id=None, precision="fp64"):
    """wos_eval with the library's static workspace: allocates nothing, so the
    caller passes the outputs (stats [n,4] f64, capped [n] int64)."""
    n = pts.shape[0]
    _dev_tensor(pts, torch.float64, (n, 3))
    _dev_tensor(walks, torch.int64, (n,))
    _dev_tensor(stats, torch.float64, (n, 4))
    _dev_tensor(capped, torch.int64, (n,))
    if walk_begin is not None:
        _dev_tensor(walk_begin, torch.int64, (n,))
    if stream_id is not None:
        _dev_tensor(stream_id, torch.int32, (n,))
    _check(lib().dtn_wos_eval_noalloc(geom.handle, _ptr(pts), n, _ptr(walks), _ptr(walk_begin),
                                      C.c_uint64(int(seed) & (2 ** 64 - 1)), _ptr(stream_id), PRECISION[precision],
                                      _ptr(stats), _ptr(capped), _stream()), "dtn_wos_eval_noalloc")
    return stats, capped


def walk_counters(geom, enable=False):
    """(wave iterations, hole distances computed by waves) of the counted
    walks on a box minus holes since the last call (waits for torch's
    current stream); counting stays on for later launches when enable."""
    out = (C.c_int64 * 2)()
    _check(lib().dtn_walk_counters(geom.handle, _stream(), 1 if enable else 0, out), "dtn_walk_counters")
    return int(out[0]), int(out[1])


def check(geom):
    """Status of the work done on `geom` (waits for torch's current stream,
    then reads and clears the geometry's status bits): "ok", "maxsteps"
    (walks ended by the step cap) or "noconv" (an FP32-mixed solve missed its
    residual bound)."""
    st = lib().dtn_check(geom.handle, _stream())
    if st == DTN_OK:
        return "ok"
    if st == -6:
        return "maxsteps"
    if st == -5:
        return "noconv"
    _check(st, "dtn_check")


def boundary_distance(geom, pts, precision="fp64", out=None):
    """Distance to the boundary as the walk kernels compute it (device [n])."""
    n = pts.shape[0]
    _dev_tensor(pts, torch.float64, (n, 3))
    if out is None:
        out = torch.empty((n,), dtype=torch.float64, device=pts.device)
    _dev_tensor(out, torch.float64, (n,))
    _check(lib().dtn_boundary_distance(geom.handle, _ptr(pts), n, PRECISION[precision], _ptr(out), _stream()),
           "dtn_boundary_distance")
    return out


def wos_adaptive(geom, pts, seed, pilot_walks, min_walks, max_walks, se_target, stream_id=None,
                 precision="fp64", schedule=None, stats=None, walks_used=None, capped=None):
    """Step 1 with adaptive walk counts: pilot, per-point budget
    clamp(ceil(var / se_target^2), min_walks, max_walks), remainder, merge.

    Returns (stats [n,4] f64, walks_used [n] int64, capped [n] int64)."""
    n = pts.shape[0]
    _dev_tensor(pts, torch.float64, (n, 3))
    if stream_id is not None:
        _dev_tensor(stream_id, torch.int32, (n,))
    dev = pts.device
    if stats is None:
        stats = torch.empty((n, 4), dtype=torch.float64, device=dev)
    if walks_used is None:
        walks_used = torch.empty((n,), dtype=torch.int64, device=dev)
    if capped is None:
        capped = torch.empty((n,), dtype=torch.int64, device=dev)
    _dev_tensor(stats, torch.float64, (n, 4))
    _dev_tensor(walks_used, torch.int64, (n,))
    _dev_tensor(capped, torch.int64, (n,))
    b = AdaptiveDesc(int(pilot_walks), int(min_walks), int(max_walks), float(se_target))
    sc = schedule_struct(schedule)
    _check(lib().dtn_wos_adaptive(geom.handle, _ptr(pts), n, C.byref(b), C.c_uint64(int(seed) & (2 ** 64 - 1)),
                                  _ptr(stream_id), PRECISION[precision], None if sc is None else C.byref(sc),
                                  _ptr(stats), _ptr(walks_used), _ptr(capped), _stream()), "dtn_wos_adaptive")
    return stats, walks_used, capped


def time_schedules(geom, pts, walks, seed, schedules, reps=1, walk_begin=None, stream_id=None,
                   precision="fp64", stats=None):
    """Mean device milliseconds of dtn_wos_eval's work under each schedule
    (list of dicts); blocks until done.  Returns (ms list, stats)."""
    n = pts.shape[0]
    _dev_tensor(pts, torch.float64, (n, 3))
    _dev_tensor(walks, torch.int64, (n,))
    if walk_begin is not None:
        _dev_tensor(walk_begin, torch.int64, (n,))
    if stream_id is not None:
        _dev_tensor(stream_id, torch.int32, (n,))
    if stats is None:
        stats = torch.empty((n, 4), dtype=torch.float64, device=pts.device)
    cands = (ScheduleDesc * len(schedules))(*[schedule_struct(s) for s in schedules])
    ms = (C.c_float * len(schedules))()
    _check(lib().dtn_wos_time_schedules(geom.handle, _ptr(pts), n, _ptr(walks), _ptr(walk_begin),
                                        C.c_uint64(int(seed) & (2 ** 64 - 1)), _ptr(stream_id),
                                        PRECISION[precision], cands, len(schedules), int(reps), _ptr(stats), ms,
                                        _stream()), "dtn_wos_time_schedules")
    return [float(v) for v in ms], stats


def patches_struct(pdesc):
    P = len(pdesc["h"])
    arr = (PatchDesc * P)()
    for i in range(P):
        for k in range(3):
            arr[i].c[k] = float(pdesc["c"][i][k])
            arr[i].n[k] = float(pdesc["n"][i][k])
            arr[i].t1[k] = float(pdesc["t1"][i][k])
        arr[i].h = float(pdesc["h"][i])
        arr[i].n_theta = int(pdesc["n_theta"][i])
        arr[i].n_phi = int(pdesc["n_phi"][i])
        arr[i].n_rings = int(pdesc["n_rings"][i])
        arr[i].n_sectors = int(pdesc["n_sectors"][i])
    return arr


class Plan:
    """The patches of a DtN request with their class operators (device)."""

    def __init__(self, geom, pdesc):
        self.geom = geom
        arr = patches_struct(pdesc)
        self.n_patches = len(arr)
        self.handle = C.c_void_p()
        _check(lib().dtn_create_plan(geom.handle, arr, len(arr), C.byref(self.handle)), "dtn_create_plan")
        self.num_nodes = int(lib().dtn_plan_num_nodes(self.handle))
        self.num_panels = int(lib().dtn_plan_num_panels(self.handle))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.dtn_destroy_plan(h)
            self.handle = None

    def set_max_sweeps(self, n):
        """Most FP32 solves of the FP32-mixed refinement (default 8)."""
        _check(lib().dtn_plan_set_max_sweeps(self.handle, int(n)), "dtn_plan_set_max_sweeps")

    def nodes(self, out=None, device="cuda"):
        if out is None:
            out = torch.empty((self.num_nodes, 3), dtype=torch.float64, device=device)
        _dev_tensor(out, torch.float64, (self.num_nodes, 3))
        _check(lib().dtn_patch_nodes(self.handle, _ptr(out), _stream()), "dtn_patch_nodes")
        return out

    def solve(self, node_stats, precision="fp64", neumann=None, neumann_se=None):
        _dev_tensor(node_stats, torch.float64, (self.num_nodes, 4))
        dev = node_stats.device
        if neumann is None:
            neumann = torch.empty(self.num_panels, dtype=torch.float64, device=dev)
        if neumann_se is None:
            neumann_se = torch.empty(self.num_panels, dtype=torch.float64, device=dev)
        _check(lib().dtn_patch_solve(self.handle, _ptr(node_stats), PRECISION[precision], _ptr(neumann),
                                     _ptr(neumann_se), _stream()), "dtn_patch_solve")
        return neumann, neumann_se

    def solve_second_kind(self, node_stats, neumann=None, neumann_se=None):
        """Neumann data by the second-kind equation (flat patches: sigma = 2b)."""
        _dev_tensor(node_stats, torch.float64, (self.num_nodes, 4))
        dev = node_stats.device
        if neumann is None:
            neumann = torch.empty(self.num_panels, dtype=torch.float64, device=dev)
        if neumann_se is None:
            neumann_se = torch.empty(self.num_panels, dtype=torch.float64, device=dev)
        _check(lib().dtn_patch_solve_second_kind(self.handle, _ptr(node_stats), _ptr(neumann), _ptr(neumann_se),
                                                 _stream()), "dtn_patch_solve_second_kind")
        return neumann, neumann_se

    def potential(self, neumann, targets, out=None):
        m = targets.shape[0]
        _dev_tensor(neumann, torch.float64, (self.num_panels,))
        _dev_tensor(targets, torch.float64, (m, 3))
        if out is None:
            out = torch.empty(m, dtype=torch.float64, device=targets.device)
        _check(lib().dtn_potential(self.handle, _ptr(neumann), _ptr(targets), m, _ptr(out), _stream()),
               "dtn_potential")
        return out


class Tree:
    """Treecode for the potential of a tile plan (same sum as Plan.potential):
    the tree over the tile sources is built once; each call rebuilds the
    Chebyshev proxies from the Neumann data and walks the tree per wave of
    Morton-sorted targets."""

    def __init__(self, plan, degree=6, leaf_size=64):
        self.plan = plan
        self.handle = C.c_void_p()
        _check(lib().dtn_create_tree(plan.handle, int(degree), int(leaf_size), C.byref(self.handle)),
               "dtn_create_tree")
        info = (C.c_int64 * 4)()
        _check(lib().dtn_tree_info(self.handle, info), "dtn_tree_info")
        self.n_clusters, self.n_proxy_clusters, self.n_proxies, self.n_sources = (int(v) for v in info)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.dtn_destroy_tree(h)
            self.handle = None

    def potential(self, neumann, targets, theta=0.5, out=None, counts=None):
        """u at the targets; counts (int64 [m][2], optional) receives each
        target's proxy and direct interactions."""
        m = targets.shape[0]
        _dev_tensor(neumann, torch.float64, (self.plan.num_panels,))
        _dev_tensor(targets, torch.float64, (m, 3))
        if out is None:
            out = torch.empty(m, dtype=torch.float64, device=targets.device)
        _dev_tensor(out, torch.float64, (m,))
        if counts is not None:
            _dev_tensor(counts, torch.int64, (m, 2))
        _check(lib().dtn_tree_potential(self.handle, _ptr(neumann), _ptr(targets), m, float(theta), _ptr(out),
                                        _ptr(counts), _stream()), "dtn_tree_potential")
        return out


class Points:
    """Single-point queries on a flat boundary (Sec. 5.1): hemisphere nodes
    and du/dn = Sigma1' + Sigma2' from the node statistics."""

    def __init__(self, geom, x, normals, t1, a, n_g1=20, n_g2=20, delta_rel=1e-6):
        self.geom = geom
        x = np.asarray(x, np.float64).reshape(-1, 3)
        normals = np.asarray(normals, np.float64).reshape(-1, 3)
        t1 = np.asarray(t1, np.float64).reshape(-1, 3)
        a = np.broadcast_to(np.asarray(a, np.float64), (x.shape[0],))
        self.n = x.shape[0]
        arr = (PointDesc * max(self.n, 1))()
        for i in range(self.n):
            for k in range(3):
                arr[i].c[k] = float(x[i, k])
                arr[i].n[k] = float(normals[i, k])
                arr[i].t1[k] = float(t1[i, k])
            arr[i].a = float(a[i])
        self.handle = C.c_void_p()
        _check(lib().dtn_create_points(geom.handle, arr, self.n, int(n_g1), int(n_g2), float(delta_rel),
                                       C.byref(self.handle)), "dtn_create_points")
        self.num_nodes = int(lib().dtn_points_num_nodes(self.handle))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.dtn_destroy_points(h)
            self.handle = None

    def nodes(self, out=None, device="cuda"):
        if out is None:
            out = torch.empty((self.num_nodes, 3), dtype=torch.float64, device=device)
        _dev_tensor(out, torch.float64, (self.num_nodes, 3))
        _check(lib().dtn_points_nodes(self.handle, _ptr(out), _stream()), "dtn_points_nodes")
        return out

    def neumann(self, node_stats, out=None):
        """(du/dn, standard error, Sigma1', Sigma2') per point, [n][4]."""
        _dev_tensor(node_stats, torch.float64, (self.num_nodes, 4))
        if out is None:
            out = torch.empty((self.n, 4), dtype=torch.float64, device=node_stats.device)
        _dev_tensor(out, torch.float64, (self.n, 4))
        _check(lib().dtn_points_neumann(self.handle, _ptr(node_stats), _ptr(out), _stream()), "dtn_points_neumann")
        return out


def tree_layout(pdesc, degree=6, leaf_size=64):
    """Host diagnostic: the treecode's tree for these patches (no device):
    nodes [n][8] (first, end source, subtree end, leaf, degrees, first proxy)
    and the source permutation."""
    arr = patches_struct(pdesc)
    n = len(pdesc["h"])
    cap = 4 * 16 * n + 16
    nodes = np.empty((cap, 8), dtype=np.int32)
    perm = np.empty(16 * n, dtype=np.int32)
    nn = C.c_int64()
    _check(lib().dtn_tree_layout(arr, n, int(degree), int(leaf_size), cap, nodes.ctypes.data_as(C.c_void_p),
                                 perm.ctypes.data_as(C.c_void_p), C.byref(nn)), "dtn_tree_layout")
    return nodes[: nn.value].copy(), perm


def class_operators(n_theta, n_phi, n_rings, n_sectors, rr=0.0):
    """Host diagnostic: the class operators the library builds (no device)."""
    Nn, Np = n_theta * n_phi, n_rings * n_sectors
    out = {"node_tab": np.empty((Nn, 3)), "col_tab": np.empty((Np, 3)), "K": np.empty((Np, Np)),
           "QI": np.empty((Np, Nn)), "A2": np.empty((Np, Nn)), "fit": np.empty((16, Np))}
    dp = C.POINTER(C.c_double)
    args = [out[k].ctypes.data_as(dp) for k in ("node_tab", "col_tab", "K", "QI", "A2", "fit")]
    _check(lib().dtn_class_operators(n_theta, n_phi, n_rings, n_sectors, float(rr), *args), "dtn_class_operators")
    return out


class Server:
    """Query server (continuous batching over HIP streams, native dispatcher).

    Each query is a set of boundary points; the answer per point is du/dn
    averaged over the central ring of panels of a patch centred on it, with
    its standard error, the walks spent and the patch radius h."""

    def __init__(self, geom, n_streams=4, precision="fp64", hbm_budget=2 << 30, pilot_walks=100, min_walks=100,
                 max_walks=1_000_000, h_max=0.25, ladder=16, layout=(8, 16, 4, 8), max_points=4096, graphs=False,
                 max_batch_queries=0, point_rule=None):
        """point_rule = (n_g1, n_g2, delta_rel) switches to point mode: the
        single-point estimate (Sec. 5.1) on the hemisphere of radius a = h,
        answers (Sigma1' + Sigma2', SE, walks, a), no collocation solve."""
        self.geom = geom
        g1, g2, dr = (0, 0, 0.0) if point_rule is None else point_rule
        self.cfg = ServerConfigDesc(int(n_streams), PRECISION[precision], int(hbm_budget), int(pilot_walks),
                                    int(min_walks), int(max_walks), float(h_max), int(ladder), *map(int, layout),
                                    int(max_points), 1 if graphs else 0, int(max_batch_queries), int(g1), int(g2),
                                    float(dr))
        self.handle = C.c_void_p()
        _check(lib().dtn_server_create(geom.handle, C.byref(self.cfg), C.byref(self.handle)), "dtn_server_create")
        self._out = {}

    def footprint(self, n_points):
        return int(lib().dtn_server_footprint(C.byref(self.cfg), int(n_points)))

    def clock(self):
        return float(lib().dtn_server_clock(self.handle))

    def submit(self, query_id, pts, normals, se_target, seed):
        pts = np.ascontiguousarray(np.asarray(pts, np.float64).reshape(-1, 3))
        nrm = np.ascontiguousarray(np.asarray(normals, np.float64).reshape(-1, 3))
        if nrm.shape != pts.shape:
            raise ValueError("pts and normals must have the same shape")
        out = np.full((pts.shape[0], 4), np.nan)
        qid = int(query_id)
        if qid in self._out:
            raise ValueError(f"query id {qid} is still in flight")
        self._out[qid] = (out, pts, nrm)
        st = lib().dtn_server_submit(self.handle, C.c_uint64(qid), pts.ctypes.data, nrm.ctypes.data,
                                     pts.shape[0], float(se_target), C.c_uint64(int(seed) & (2 ** 64 - 1)),
                                     out.ctypes.data)
        if st != DTN_OK:
            del self._out[qid]
            _check(st, "dtn_server_submit")
        return out

    def wait(self, max_n=64, timeout=-1.0):
        """Completed queries (up to max_n), each a dict with the answers."""
        buf = (QueryDoneDesc * int(max_n))()
        n = C.c_int64(0)
        _check(lib().dtn_server_wait(self.handle, int(max_n), float(timeout), buf, C.byref(n)), "dtn_server_wait")
        res = []
        for i in range(n.value):
            d = buf[i]
            out, _, _ = self._out.pop(int(d.query_id))
            res.append({"id": int(d.query_id), "status": int(d.status), "n_points": int(d.n_points),
                        "t_submit": d.t_submit, "t_start": d.t_start, "t_done": d.t_done, "answer": out})
        return res

    def in_flight(self):
        return len(self._out)

    def close(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.dtn_server_destroy(h)
            self.handle = None

    def __del__(self):
        self.close()


def class_second_kind(n_theta, n_phi, n_rings, n_sectors, rr=0.0):
    """Host diagnostic: the second-kind tables of a class at h = 1 (rr = R/h
    on a sphere, -R/h outside a ball, 0 on a plane): Q2, c2 and M = 1/2 I - D."""
    Np, Nn = n_rings * n_sectors, n_theta * n_phi
    Q2, c2, M = np.empty((Np, Nn)), np.empty(Np), np.empty((Np, Np))
    dp = C.POINTER(C.c_double)
    _check(lib().dtn_class_second_kind(n_theta, n_phi, n_rings, n_sectors, float(rr), Q2.ctypes.data_as(dp),
                                       c2.ctypes.data_as(dp), M.ctypes.data_as(dp)), "dtn_class_second_kind")
    return {"Q2": Q2, "c2": c2, "M": M}

