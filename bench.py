"""Benchmark of the local DtN hot path on one MI355X.

One step is one pass of the whole path over the unit-cube workload: the
hemisphere nodes of all 6 x 16 x 16 = 1536 patches (h = 1/32, 16 x 32 nodes
each, 786,432 nodes), 1e5 walk-on-spheres walks per node (eps = 1e-5, eight
exterior point sources), the collocation solve for the Neumann data on 64
panels per patch with propagated standard errors, and the potential at 1e4
interior targets from the integral representation.

Prints one JSON line.  `value` is walks per second of the whole step; the
line also carries DtN patches/s, the Neumann error against the exact data
(which fixes the error level the throughput is quoted at), the ALU roofline
of the walk kernel and the oracle's CPU throughput on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# ALU roofline.  Peak: one lane-op slot per lane per cycle, 256 CUs x 4 SIMDs
# x 16 lanes x 2.4 GHz.  Each instruction kind costs the slots measured for it
# by the issue-rate microbenchmarks (``--calibrate``): a kind issued at one
# lane-op per lane per cycle costs 1.
ALU_PEAK = 256 * 4 * 16 * 2.4e9
SLOT_COST = {
    "f64": 1.10,     # v_add/mul/min/max/cmp_f64
    "f64fma": 1.17,  # v_fma_f64
    "f32": 0.69,     # v_fma/add/mul/min/max_f32
    "i32": 1.05,     # 32-bit integer and bit operations (v_bitop3_b32, v_mul_hi_u32)
    "mad64": 0.96,   # v_mad_u64_u32 (32x32->64)
    "cvt": 1.02,     # conversions between f32, f64 and u32
    "trans32": 2.10,  # v_sin_f32, v_cos_f32, v_sqrt_f32
    "rsq64": 4.06,   # v_rsq_f64
}
# Algorithmic work (operation counts by kind) of one walk step and of one walk
# for the box domain with point-source data, counted from what the step
# definition requires, not from what the compiler emits.
STEP_OPS = {
    # distance (11), eps test (1), u1 = ldexp(k + 1/2, -32) (2), u(1-u) (2), x2 (1),
    # square root: -x/2, and three more products (4), sin/cos: x^2, x^3 and the two
    # products of the angle addition (4), s cos / s sin (2)
    "fp64": {"f64": 27,
             # z (1), square root: one Newton step and the residual correction (4),
             # sin/cos: remainder scaling (1), Taylor series (6), angle addition (2); jump (3)
             "f64fma": 17,
             # cap test, Philox xors (half block: 10), counter word, table index and
             # remainder bits (3), step counter
             "i32": 16, "mad64": 10, "cvt": 2, "rsq64": 1},
    # FP64 distance (11), eps test (1), jump shortening (1); FP32 uniforms (2 subtractions
    # after a bit alignment each, counted in i32), z (1), u(1-u) (2), x2 (1), s cos / s sin
    # (2); sqrt, sin, cos on the transcendental unit; conversions: 3 direction components;
    # 3 FP64 FMAs of the jump
    "fp32": {"f64": 13, "f64fma": 3, "f32": 8, "trans32": 3, "cvt": 3, "i32": 15, "mad64": 10},
}
# projection, 8 sources (sub, FMA, rsq + two Newton steps each), shift,
# two compensated adds, square, counters
WALK_OPS = {"f64": 52, "f64fma": 72, "rsq64": 8, "i32": 8}
# Half space with the truncation sphere: the distance is z itself (no work);
# the sphere test (3 differences, a product, 2 FMAs, a compare) replaces the
# 11 operations of the box distance; the rest of the step is the box's.  Per
# walk: one source (differences, square, rsq + two Newton steps, the scaled
# add), the shift and the compensated sums.
HS_STEP_OPS = {
    "fp64": {"f64": 27 - 11 + 5, "f64fma": 17 + 2, "i32": 16, "mad64": 10, "cvt": 2, "rsq64": 1},
    "fp32": {"f64": 13 - 11 + 5, "f64fma": 3 + 2, "f32": 8, "trans32": 3, "cvt": 3, "i32": 15, "mad64": 10},
}
HS_WALK_OPS = {"f64": 10, "f64fma": 9, "rsq64": 1, "i32": 8}
# Exterior of a disk: the distance is rho = sqrt(x^2 + y^2) (a product and an
# FMA, a clamp, the correctly rounded root: 4 f64 + 4 FMA + rsq), e = rho - b
# and its clamp, e^2 + z^2 (a product, an FMA) and its clamp, and the root
# again (FP32-mixed: unrefined, a product and rsq); the sphere test as for
# the half space.  Per walk: the projection onto the disk (root, quotient,
# two products, compare), the constant data, the shift and the sums.
DISK_STEP_OPS = {
    "fp64": {"f64": 27 - 11 + 14 + 5, "f64fma": 17 + 10 + 2, "i32": 16, "mad64": 10, "cvt": 2, "rsq64": 1 + 2},
    "fp32": {"f64": 13 - 11 + 11 + 5, "f64fma": 3 + 6 + 2, "f32": 8, "trans32": 3, "cvt": 3, "i32": 15,
             "mad64": 10, "rsq64": 2},
}
DISK_WALK_OPS = {"f64": 14, "f64fma": 12, "rsq64": 2, "i32": 8}
# Exterior of a ball: the distance is |x - c| - R (3 differences, a product
# and 2 FMAs, the correctly rounded root: 4 f64 + 4 FMA + rsq, the
# difference), the sphere test as for the half space.  Per walk: the
# projection onto the sphere (root, quotient, 3 FMAs), one source, the shift
# and the sums.
EXT_STEP_OPS = {
    "fp64": {"f64": 27 - 11 + 9 + 5, "f64fma": 17 + 6 + 2, "i32": 16, "mad64": 10, "cvt": 2, "rsq64": 1 + 1},
    "fp32": {"f64": 13 - 11 + 9 + 5, "f64fma": 3 + 6 + 2, "f32": 8, "trans32": 3, "cvt": 3, "i32": 15,
             "mad64": 10, "rsq64": 1},
}
EXT_WALK_OPS = {"f64": 16, "f64fma": 14, "rsq64": 2, "i32": 8}
# Box minus holes, FP32-mixed step: the cube's step (its box distance is the
# outer-box part), plus the cell lookup (position to FP32: 3 conversions,
# 3 FMAs, 3 clamps, 3 truncations, 2 index products and 2 adds), the root of
# the nearest hole's squared distance (clamp, rsq, product, min), and per
# hole whose distance the wave computes: 3 differences, 3 differences of
# absolute values, 3 clamps at 0, a product and 2 FMAs for the square, and
# the running min.  The holes per wave iteration are counted by the kernel
# (dtn_walk_counters).  Per walk: the cube's per-walk work with 20 sources
# instead of 8 (each: differences, square, rsq with Newton refinement, the
# scaled add) and the projection's candidate holes at the mean count.
HOLES_STEP_OPS = {k: dict(v) for k, v in STEP_OPS.items()}
for _k in HOLES_STEP_OPS:
    _o = HOLES_STEP_OPS[_k]
    _o["cvt"] = _o.get("cvt", 0) + 3 + 3
    _o["f32"] = _o.get("f32", 0) + 6
    _o["i32"] = _o.get("i32", 0) + 4
    _o["f64"] = _o.get("f64", 0) + 3
    _o["rsq64"] = _o.get("rsq64", 0) + 1
HOLE_OPS = {"f64": 11, "f64fma": 2}
HOLES_WALK_OPS = {"f64": 52 + 12 * 5, "f64fma": 72 + 12 * 9, "rsq64": 8 + 12, "i32": 8}


def slots(ops):
    return sum(SLOT_COST[k] * n for k, n in ops.items())


SLOTS_PER_STEP = {k: slots(v) for k, v in STEP_OPS.items()}
HOLES_SLOTS_PER_STEP = {k: slots(v) for k, v in HOLES_STEP_OPS.items()}
HOLE_SLOTS = slots(HOLE_OPS)
HOLES_SLOTS_PER_WALK = slots(HOLES_WALK_OPS)
SLOTS_PER_WALK = slots(WALK_OPS)
HS_SLOTS_PER_STEP = {k: slots(v) for k, v in HS_STEP_OPS.items()}
HS_SLOTS_PER_WALK = slots(HS_WALK_OPS)
DISK_SLOTS_PER_STEP = {k: slots(v) for k, v in DISK_STEP_OPS.items()}
DISK_SLOTS_PER_WALK = slots(DISK_WALK_OPS)
EXT_SLOTS_PER_STEP = {k: slots(v) for k, v in EXT_STEP_OPS.items()}
EXT_SLOTS_PER_WALK = slots(EXT_WALK_OPS)
# Treecode interactions, counted from what an interaction needs: a proxy of
# an in-plane cluster (r^2 as the target's row sum plus its column term, one
# add; 1/r and 1/r^2 from the hardware estimate y of 1/r and its residual
# e = 1 - r^2 y^2: y^2 (a product), e (an FMA), y (1 + e/2) (an FMA and a
# product), y^2 (1 + e) (an FMA); the dipole product, the charge term's FMA
# and the accumulating FMA) and a tile source taken directly (three
# differences, r^2 (a product, two FMAs), the two powers as above, the
# normal product (a product, two FMAs) and its scaling, the charge term's
# FMA, the accumulating FMA).  The row sums and column terms are per target
# and row or column, not per interaction.  Targets inside the cube take only
# in-plane clusters' proxies.
TREE_PROXY_SLOTS = slots({"f64": 4, "f64fma": 5, "rsq64": 1})
TREE_SOURCE_SLOTS = slots({"f64": 8, "f64fma": 9, "rsq64": 1})

# HBM traffic of the walk kernel on the unit-cube workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs, each scaled by the same counter on a plain
# 256 MiB device copy in the same run (fetch 2.00, write 1.00).  Valid only for
# the kernel sources it was measured on (SHA-256 of these files).
TRAFFIC = {"files": ["paper_1210_1491_amd/csrc/dtn_wos.hip", "paper_1210_1491_amd/csrc/dtn_device.h",
                     "paper_1210_1491_amd/csrc/dtn_internal.h"],
           "sha256": ["87e9164055f41ec601b7f142fabe11c48a5f850b56c6bfd2515da790ea038347",
                      "19671560cc811f1b8a60b74d4037267882fa3f71950dead4aab4cc74733a45da",
                      "3ba5aaa8cff36fcabd3602a4f75e1f6a528fc5a5cd5d175510ed3897d9d2cf24"],
           "fetch_bytes": 41790.938 * 1024 * (262144 / 131088.688), "write_bytes": 38400.0 * 1024 * 1.00,
           # the half-space point workload's walk kernel (same sources), scaled
           # by the copy in its own run (fetch 131086.375 KiB for 262144)
           "halfspace_fetch_bytes": 92472.438 * 1024 * (262144 / 131086.375),
           "halfspace_write_bytes": 80000.0 * 1024 * 1.00}


# ------------------------------------------------- exact data, panel layout
# The accuracy figures compare the library's output with the exact solution
# of the synthetic problems (closed forms of their harmonic data), at the
# collocation points of the panel layout that include/dtn.h documents for
# plane patches: n_rings uniform rings x n_sectors sectors of the disk of
# radius h, ring-major, collocation at the parametric centres.


def exact_grad(gd, x):
    """Gradient of the harmonic extension of the Dirichlet data."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    if gd["data_kind"] == "quadratic":
        c = gd["quad"]
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        return np.stack([c[1] + 2 * c[4] * X + c[7] * Y + c[9] * Z,
                         c[2] + 2 * c[5] * Y + c[7] * X + c[8] * Z,
                         c[3] + 2 * c[6] * Z + c[8] * Y + c[9] * X], axis=-1)
    g = np.zeros_like(x)
    for q in np.asarray(gd["src"]).reshape(-1, 4):
        d = x - q[:3]
        g -= q[3] * d / np.linalg.norm(d, axis=-1)[:, None] ** 3
    return g


def exact_u(gd, x):
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    if gd["data_kind"] == "quadratic":
        c = gd["quad"]
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        return (c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * X + c[5] * Y * Y + c[6] * Z * Z
                + c[7] * X * Y + c[8] * Y * Z + c[9] * X * Z)
    return sum(q[3] / np.linalg.norm(x - q[:3], axis=-1) for q in np.asarray(gd["src"]).reshape(-1, 4))


def plane_panels(pd):
    """Collocation points, outward normals, areas and centre distances of the
    panels of plane patches, patch-major as the solve returns them."""
    X, N, A, R = [], [], [], []
    for i in range(len(pd["h"])):
        c, n, t1, h = (np.asarray(pd[k][i], np.float64) for k in ("c", "n", "t1", "h"))
        t2 = np.cross(n, t1)
        nr, ns = int(pd["n_rings"][i]), int(pd["n_sectors"][i])
        se = h * np.arange(nr + 1) / nr
        ae = 2 * np.pi * np.arange(ns + 1) / ns
        s0, s1 = np.repeat(se[:-1], ns), np.repeat(se[1:], ns)
        a0, a1 = np.tile(ae[:-1], nr), np.tile(ae[1:], nr)
        sc, ac = 0.5 * (s0 + s1), 0.5 * (a0 + a1)
        X.append(c + (sc * np.cos(ac))[:, None] * t1 + (sc * np.sin(ac))[:, None] * t2)
        N.append(np.tile(n, (nr * ns, 1)))
        A.append(0.5 * (s1 ** 2 - s0 ** 2) * (a1 - a0))
        R.append(sc)
    return np.concatenate(X), np.concatenate(N), np.concatenate(A), np.concatenate(R)


def rel_l2(sigma, exact, area, mask):
    """Area-weighted relative L2 error over the panels in ``mask``."""
    return float(np.sqrt(np.sum(area[mask] * (sigma[mask] - exact[mask]) ** 2)
                         / np.sum(area[mask] * exact[mask] ** 2)))


def traffic_if_current():
    import hashlib

    for f, h in zip(TRAFFIC["files"], TRAFFIC["sha256"]):
        with open(os.path.join(ROOT, f), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != h:
                return None
    return TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]


def halfspace_traffic_if_current():
    if traffic_if_current() is None or TRAFFIC["halfspace_fetch_bytes"] is None:
        return None
    return TRAFFIC["halfspace_fetch_bytes"] + TRAFFIC["halfspace_write_bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--walks", type=int, default=100_000)
    ap.add_argument("--tiles", type=int, default=16, help="tiles per cube edge (16 -> 1536 patches)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the other precision's run")
    ap.add_argument("--cpu-walks", type=int, default=100_000, help="walks per node in the CPU sample")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (reference for HBM counters)")
    ap.add_argument("--no-box-holes", action="store_true", help="skip the uneven-batching workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the query-serving workload")
    ap.add_argument("--serving-window", type=int, default=12, help="arrivals in the serving window")
    ap.add_argument("--serving-sweep-window", type=int, default=6,
                    help="arrivals of the half-capacity run (half as many at a quarter); 0 skips both")
    ap.add_argument("--serving-se-range", type=float, nargs=2, default=[1e-4, 1e-2],
                    help="range of the per-query required node standard error (log-uniform)")
    ap.add_argument("--serving-rate", type=float, default=200.0, help="offered load, queries/s")
    ap.add_argument("--serving-stable-only", action="store_true",
                    help="with --only serving: one window at --serving-rate only (a latency distribution at a "
                         "rate the GPU sustains)")
    ap.add_argument("--no-halfspace", action="store_true", help="skip the single-point half-space workload")
    ap.add_argument("--no-disk", action="store_true", help="skip the thin-disk workload (Table 5)")
    ap.add_argument("--no-exterior", action="store_true", help="skip the exterior-sphere workload (Sec. 5.2)")
    ap.add_argument("--no-tabulated", action="store_true", help="skip the tabulated-data workload")
    ap.add_argument("--no-treecode", action="store_true", help="skip the treecode-potential workload")
    ap.add_argument("--only", choices=["cube", "box_holes", "serving", "halfspace", "disk", "exterior", "treecode"],
                    default=None,
                    help="run one workload only (for profiling)")
    ap.add_argument("--box-holes-se", type=float, default=None,
                    help="target standard error of the uneven-batching workload (default: its 1e-3)")
    ap.add_argument("--no-tune", action="store_true", help="default walk schedule, no autotuning")
    ap.add_argument("--calibrate", action="store_true",
                    help="measure the issue cost of the instruction kinds the roofline table charges")
    return ap.parse_args()


# Instruction kinds of the issue-rate microbenchmarks (paper_1210_1491_amd/
# csrc/calib.hip), in library order, with the instructions one chain step issues.
CALIB_KINDS = [("v_fma_f32", 1), ("v_fma_f64", 1), ("v_mad_u64_u32 + v_xor_b32", 2),
               ("v_sqrt_f32 + v_mul_f32", 2), ("v_sin_f32", 1), ("v_rsq_f64", 1),
               ("v_cvt_f64_f32 + v_cvt_f32_f64", 2), ("v_bitop3_b32", 1), ("v_fma_f32 | v_sin_f32 (two chains)", 2),
               ("v_fma_f64 | v_fma_f32 (two chains)", 2), ("v_min_f64 + 2 v_max_f64", 3), ("v_cos_f32", 1),
               ("v_sqrt_f32", 1), ("v_add_f64", 1), ("v_mad_u64_u32", 1), ("v_mul_hi_u32", 1)]


def calibrate():
    """Issue slots per instruction kind: the full-rate lane-slot rate of the
    chip divided by the measured rate of chain steps, per instruction."""
    import ctypes as C

    from paper_1210_1491_amd import build as B

    L = C.CDLL(B.CALIB)
    L.dtn_calib_rate.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_float)]
    rows = {}
    for op, (name, n_instr) in enumerate(CALIB_KINDS):
        rate, ms = C.c_double(), C.c_float()
        st = L.dtn_calib_rate(op, 8192, 16384, C.byref(rate), C.byref(ms))
        if st != 0:
            raise RuntimeError(f"calibration kernel {name} failed: {st}")
        slots_per_step = ALU_PEAK / rate.value
        rows[name] = {"ms": ms.value, "steps_per_s": rate.value, "slots_per_step": slots_per_step,
                      "slots_per_instruction": slots_per_step / n_instr}
        print(f"[calib] {name:40s} {ms.value:8.2f} ms  {slots_per_step:6.2f} slots/step", file=sys.stderr, flush=True)
    return rows


def box_holes(precision, steps, with_cpu=True, se_target=None, tune=True, with_fp64=False):
    """Uneven batching: the box [0,4]^3 minus 20 holes, 5994 patches in five
    panel classes (8..128 panels), adaptive walks 1e3..2e5 per node at a
    target standard error of 1e-3, all in one adaptive call (pilot launch,
    budgets, one launch over the uneven remainder, merge), then the solve,
    captured in a HIP graph and replayed per step.  The walk schedule comes
    from the autotuner (timed on a sample of the remainder's work list as a
    pilot estimates it).  The Neumann data are checked against the exact data
    (global area-weighted relative L2 over the trusted panels, beside the
    same norm of the propagated standard errors).  with_fp64: one more step
    of the plain FP64 path (eager, same budgets rule) for the comparison at
    equal error."""
    import torch

    import dtn_inputs as I
    from paper_1210_1491_amd import autotune, dtn

    cfg = I.CONFIGS["box_holes"]
    gd = cfg["geometry"]()
    pd = cfg["patches"](gd)
    g = dtn.Geometry(gd)
    plan = dtn.Plan(g, pd)
    nodes = plan.nodes()
    N = plan.num_nodes
    stats = torch.empty((N, 4), dtype=torch.float64, device="cuda")
    used = torch.empty(N, dtype=torch.int64, device="cuda")
    capped = torch.empty(N, dtype=torch.int64, device="cuda")
    se_t = cfg["se_target"] if se_target is None else float(se_target)
    budget = (cfg["pilot_walks"], cfg["min_walks"], cfg["max_walks"], se_t)
    # the tuner times a sample of the remainder's work list, estimated from a
    # pilot (the library recomputes the budgets itself in the timed steps)
    pw = torch.full((N,), cfg["pilot_walks"], dtype=torch.int64, device="cuda")
    ps, _ = dtn.wos_eval(g, nodes, pw, cfg["seed"], precision=precision)
    p = ps.cpu().numpy()
    var = p[:, 2] / (p[:, 0] - 1)
    tot = np.clip(np.ceil(var / se_t ** 2), cfg["min_walks"], cfg["max_walks"]).astype(np.int64)
    rem = torch.tensor(np.maximum(tot - cfg["pilot_walks"], 0), device="cuda")
    wb = torch.full_like(rem, cfg["pilot_walks"])
    if tune:
        sched, table = autotune.tune(g, nodes, rem, precision=precision, seed=cfg["seed"], walk_begin=wb)
    else:
        sched, table = dict(autotune.DEFAULT), {}
    print(f"[bench] box_holes schedule {sched}", file=sys.stderr, flush=True)
    # one step (adaptive walks over all patches + solve) captured once in a
    # HIP graph and replayed per timed step
    neu = torch.empty(plan.num_panels, dtype=torch.float64, device="cuda")
    nse = torch.empty(plan.num_panels, dtype=torch.float64, device="cuda")
    cap_stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cap_stream):
        dtn.wos_adaptive(g, nodes, cfg["seed"], *budget, precision=precision, schedule=sched, stats=stats,
                         walks_used=used, capped=capped)
        plan.solve(stats, precision=precision, neumann=neu, neumann_se=nse)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(f"[bench] box_holes step {times[-1]:.2f} s", file=sys.stderr, flush=True)
    # one more step, untimed and eager, with the walk counters on (their
    # atomics are kept out of the timed steps): holes per wave iteration.
    # Same seed and budgets, so it walks exactly the timed steps' walks
    dtn.walk_counters(g, enable=True)
    dtn.wos_adaptive(g, nodes, cfg["seed"], *budget, precision=precision, schedule=sched, stats=torch.empty_like(stats),
                     walks_used=torch.empty_like(used), capped=torch.empty_like(capped))
    iters, visits = dtn.walk_counters(g, enable=False)
    print(f"[bench] box_holes counted step: {visits / max(iters, 1):.3f} holes per wave iteration",
          file=sys.stderr, flush=True)
    st = stats.cpu().numpy()
    u = used.cpu().numpy()
    se = np.sqrt(st[:, 2] / np.maximum(st[:, 0] - 1, 1) / st[:, 0])
    free = (u > cfg["min_walks"]) & (u < cfg["max_walks"])
    sec = float(np.mean(times))
    # exact Neumann data at the collocation points (sources inside the holes)
    xg, ng, area, rc = plane_panels(pd)
    ex = np.sum(exact_grad(gd, xg) * ng, axis=-1)
    tr = rc < 0.7 * np.repeat(np.asarray(pd["h"], np.float64),
                              np.asarray(pd["n_rings"]) * np.asarray(pd["n_sectors"]))

    def errors(neumann, neumann_se):
        sig, sse = neumann.cpu().numpy(), neumann_se.cpu().numpy()
        noise = float(np.sqrt(np.sum(area[tr] * sse[tr] ** 2) / np.sum(area[tr] * ex[tr] ** 2)))
        return rel_l2(sig, ex, area, tr), noise

    err, noise = errors(neu, nse)
    # ALU roofline of the step (both walk launches; the solve and the
    # planning kernels are under 0.1 % of it, counted in the time)
    holes_per_iter = visits / max(iters, 1)
    steps_n, walks_n = float(st[:, 3].sum()), float(u.sum())
    n_counted = 1
    slots_step = HOLES_SLOTS_PER_STEP[precision] + holes_per_iter * HOLE_SLOTS
    slots_walk = HOLES_SLOTS_PER_WALK + holes_per_iter * HOLE_SLOTS
    achieved = (slots_step * steps_n + slots_walk * walks_n) / sec
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK / 1e12, "unit": "T lane-op slots/s",
            "frac": achieved / ALU_PEAK, "traffic": None, "slots_per_step": slots_step, "slots_per_walk": slots_walk,
            "holes_per_wave_iteration": holes_per_iter, "wave_iterations_per_step": iters / n_counted,
            "walking_lanes_per_wave_iteration": steps_n * n_counted / max(iters, 1),
            "counted": "one extra untimed step with the walk counters on"}
    fp64 = None
    if with_fp64:
        stats64, used64 = torch.empty_like(stats), torch.empty_like(used)
        n64, s64 = torch.empty_like(neu), torch.empty_like(nse)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dtn.wos_adaptive(g, nodes, cfg["seed"], *budget, precision="fp64", schedule=sched, stats=stats64,
                         walks_used=used64, capped=capped)
        plan.solve(stats64, precision="fp64", neumann=n64, neumann_se=s64)
        torch.cuda.synchronize()
        sec64 = time.perf_counter() - t0
        print(f"[bench] box_holes plain FP64 step {sec64:.2f} s", file=sys.stderr, flush=True)
        e64, noise64 = errors(n64, s64)
        w64 = float(used64.sum().item())
        fp64 = {"seconds_per_step": sec64, "walks": w64, "walks_per_s": w64 / sec64,
                "patches_per_s": len(pd["h"]) / sec64, "neumann_rel_l2_vs_exact": e64,
                "propagated_noise_rel_l2": noise64, "patches_per_s_ratio": sec64 / sec}
    cpu = box_holes_cpu_baseline(gd, pd, cfg, budget) if with_cpu else None
    return {"workload": f"box [0,4]^3 minus 20 holes, {len(pd['h'])} patches (8..128 panels), {N} nodes, "
                        f"adaptive {cfg['min_walks']}..{cfg['max_walks']} walks/node at SE {se_t}",
            "precision": precision, "seconds_per_step": sec, "walks": float(u.sum()),
            "walks_per_s": float(u.sum()) / sec, "patches_per_s": len(pd["h"]) / sec,
            "walk_steps_per_s": float(st[:, 3].sum()) / sec, "steps_per_walk": float(st[:, 3].sum() / u.sum()),
            "share_at_max_walks": float(np.mean(u == cfg["max_walks"])),
            "median_se_unclamped_nodes": float(np.median(se[free])) if free.any() else None,
            "neumann_rel_l2_vs_exact": err, "propagated_noise_rel_l2": noise,
            "capped_walks": int(capped.sum().item()), "schedule": sched, "schedule_ms": table,
            "roofline": roof, "plain_fp64": fp64, "cpu_baseline": cpu}


def box_holes_cpu_baseline(gd, pd, cfg, budget):
    """CPU baseline of the box-with-holes workload: the oracle's adaptive
    walks (FP64) on 64 seeded nodes of patches of every panel class."""
    import dtn_inputs as I
    from oracle import patch as OP
    from oracle import wos as OW
    idx = I.box_holes_sample(pd, per_class=2, seed=cfg["seed"])
    X = np.concatenate([OP.nodes_global(q)[0] for q in OP.patches_from_desc(I.subset_patches(pd, idx), gd)])
    X = X[np.random.default_rng(cfg["seed"]).choice(len(X), 64, replace=False)]
    t0 = time.perf_counter()
    r = OW.wos_adaptive(OW.Geometry(gd), X, *budget[:3], budget[3], seed=cfg["seed"])
    dt = time.perf_counter() - t0
    return {"value": float(r["count"].sum()) / dt, "unit": "walks/s", "cores": OW.max_threads(), "kind": "oracle",
            "sample": f"64 nodes of {len(idx)} patches (2 per panel class), adaptive walks "
                      f"({int(r['count'].sum())} walks, {int(r['steps'].sum())} steps) in {dt:.1f} s"}


def halfspace_points(precision, steps, warmup, with_cpu=True, cpu_points=128):
    """Single-point Neumann data on a flat boundary (Sec. 5.1), Test 1 scaled
    to many points: the half space z > 0 over a unit charge at (0, 0, -1),
    truncation sphere 1e5, eps 1e-5; 4096 points uniform in the disk of
    radius 2 on z = 0 with a = 0.1 .. 1.0 (Table 1's radii), 20 x 20
    hemisphere nodes x 1e3 walks each (Table 1's rule), Sigma2' by 20 x 20 on
    the ring with delta/a = 1e-6.  A step: nodes, walks, Sigma1' + Sigma2'.
    Accuracy against the exact -du/dz; Table 1 itself (x = (0.5, 0, 0), the
    five radii) from one more call; the oracle on a bounded sample with the
    same seeds and stream ids (so the GPU's values for those points are
    compared with the oracle's)."""
    import torch

    import dtn_inputs as I
    from paper_1210_1491_amd import dtn

    cfg = I.CONFIGS["halfspace_points"]
    gd = cfg["geometry"]()
    g = dtn.Geometry(gd)
    x, nrm, t1, a = cfg["points"](cfg["n_points"], cfg["seed"])
    P = dtn.Points(g, x, nrm, t1, a, cfg["n_g1"], cfg["n_g2"], cfg["delta_rel"])
    N = P.num_nodes
    nodes = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    stats = torch.empty((N, 4), dtype=torch.float64, device="cuda")
    capped = torch.empty(N, dtype=torch.int64, device="cuda")
    out = torch.empty((len(a), 4), dtype=torch.float64, device="cuda")
    walks = torch.full((N,), cfg["walks"], dtype=torch.int64, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    seed = cfg["seed"]

    def step(record):
        P.nodes(out=nodes)
        if record:
            ev0.record()
        dtn.wos_eval(g, nodes, walks, seed, precision=precision, stats=stats, capped=capped)
        if record:
            ev1.record()
        P.neumann(stats, out=out)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    wos_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
        torch.cuda.synchronize()
        wos_ms.append(ev0.elapsed_time(ev1))
    sec = (time.perf_counter() - t0) / steps
    print(f"[bench] halfspace points {precision}: {sec * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    st = stats.cpu().numpy()
    o = out.cpu().numpy()
    walks_n, steps_n = float(st[:, 0].sum()), float(st[:, 3].sum())
    wos_s = float(np.mean(wos_ms)) / 1e3
    achieved = (HS_SLOTS_PER_STEP[precision] * steps_n + HS_SLOTS_PER_WALK * walks_n) / wos_s
    exact = np.sum(exact_grad(gd, x) * nrm, axis=-1)
    z = (o[:, 0] - exact) / o[:, 1]
    res = {"workload": f"half space over a unit charge, {len(a)} points x {cfg['n_g1']}x{cfg['n_g1']} nodes x "
                       f"{cfg['walks']} walks, a in 0.1..1.0, ring rule {cfg['n_g2']}x{cfg['n_g2']}, "
                       f"truncation 1e5, eps 1e-5",
           "precision": precision, "ms_per_step": sec * 1e3, "points_per_s": len(a) / sec,
           "walks_per_s": walks_n / sec, "walk_steps_per_s": steps_n / sec, "steps_per_walk": steps_n / walks_n,
           "wos_kernel_ms": float(np.mean(wos_ms)), "capped_walks": int(capped.sum().item()),
           "rel_l2_vs_exact": float(np.linalg.norm(o[:, 0] - exact) / np.linalg.norm(exact)),
           "se_rel_l2": float(np.linalg.norm(o[:, 1]) / np.linalg.norm(exact)),
           "mean_abs_z": float(np.mean(np.abs(z))), "share_within_3_se": float(np.mean(np.abs(z) < 3)),
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK / 1e12,
                        "unit": "T lane-op slots/s", "frac": achieved / ALU_PEAK,
                        "traffic": halfspace_traffic_if_current() if precision == "fp64" else None,
                        "slots_per_step": HS_SLOTS_PER_STEP[precision], "slots_per_walk": HS_SLOTS_PER_WALK}}
    # Table 1: x = (0.5, 0, 0), the five radii, 20 x 20 nodes x 1e3 walks
    radii = np.array([0.1, 0.2, 0.5, 0.7, 1.0])
    T = dtn.Points(g, np.tile([0.5, 0.0, 0.0], (5, 1)), np.tile([0.0, 0.0, -1.0], (5, 1)),
                   np.tile([1.0, 0.0, 0.0], (5, 1)), radii, 20, 20, 1e-6)
    tn = T.nodes()
    ts, _ = dtn.wos_eval(g, tn, torch.full((T.num_nodes,), 1000, dtype=torch.int64, device="cuda"), 7,
                         precision=precision)
    to = T.neumann(ts).cpu().numpy()
    ex1 = 1.0 / 1.25 ** 1.5
    res["table1"] = {"a": radii.tolist(), "sigma1": to[:, 2].tolist(), "sigma2": to[:, 3].tolist(),
                     "total": to[:, 0].tolist(), "se": to[:, 1].tolist(),
                     "err_pct": (100 * (to[:, 0] - ex1) / ex1).tolist(), "analytic": ex1}
    # Table 2: Sigma2' at x = (0.5, 0, 0), a = 0.5, by rule size and delta/a
    t2 = {}
    zero = torch.zeros((1, 4), dtype=torch.float64, device="cuda")
    for drel in (1e-4, 1e-5, 1e-6):
        t2[f"{drel:g}"] = [float(dtn.Points(g, [[0.5, 0.0, 0.0]], [[0.0, 0.0, -1.0]], [[1.0, 0.0, 0.0]], [0.5], 1,
                                            ng, drel).neumann(zero).cpu().numpy()[0, 3]) for ng in (4, 6, 10, 20)]
    res["table2"] = {"n_g2": [4, 6, 10, 20], "sigma2_by_delta_rel": t2,
                     "paper_1e-6": [0.10087, 0.09338, 0.09306, 0.09305]}
    if with_cpu:
        res["cpu_baseline"] = halfspace_cpu_baseline(gd, x, nrm, t1, a, cfg, o, cpu_points)
    return res


def disk(precision, steps, warmup, with_cpu=True, cpu_points=64, reps=20):
    """Exterior of a thin disk (Sec. 5.1.3, Test 4).  Table 5: the density at
    (-0.5, 0, 0) with a = 0.4 by its three rules (10x10 x 100, 10x10 x 1000,
    20x20 x 1000 paths), each timed end to end (nodes, walks, Sigma1' +
    Sigma2') over `reps` calls, beside the paper's CPU times; then 4096
    points on both faces (20x20 x 1e3 walks) for throughput, accuracy against
    the exact density 2/(pi sqrt(1 - rho^2)) and the walk kernel's ALU
    fraction; the oracle on a sample with the GPU's stream ids."""
    import torch

    import dtn_inputs as I
    from paper_1210_1491_amd import dtn

    cfg = I.CONFIGS["disk_points"]
    gd = cfg["geometry"]()
    g = dtn.Geometry(gd)
    dp = I.DISK_POINT
    exact5 = 8.0 / (4.0 * np.pi * np.sqrt(0.75))
    paper = {(10, 100): (0.68888, 30.0), (10, 1000): (0.73960, 307.0), (20, 1000): (0.73441, 1218.0)}
    table5 = []
    for ng, npath in I.TABLE5_RULES:
        T = dtn.Points(g, [dp["x"]], [dp["n"]], [dp["t1"]], [dp["a"]], ng, 20, 1e-6)
        tn = torch.empty((T.num_nodes, 3), dtype=torch.float64, device="cuda")
        ts = torch.empty((T.num_nodes, 4), dtype=torch.float64, device="cuda")
        to = torch.empty((1, 4), dtype=torch.float64, device="cuda")
        tw = torch.full((T.num_nodes,), npath, dtype=torch.int64, device="cuda")

        def call(seed):
            T.nodes(out=tn)
            dtn.wos_eval(g, tn, tw, seed, precision=precision, stats=ts)
            T.neumann(ts, out=to)

        call(3)
        torch.cuda.synchronize()
        v = to.cpu().numpy()[0]
        t0 = time.perf_counter()
        for r in range(reps):
            call(100 + r)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        pv, pcpu = paper[(ng, npath)]
        table5.append({"rule": f"{ng}x{ng} x {npath}", "paths": ng * ng * npath, "value": float(v[0]),
                       "se": float(v[1]), "sigma2": float(v[3]), "err_pct": float(100 * (v[0] - exact5) / exact5),
                       "gpu_ms": ms, "paper_value": pv, "paper_err_pct": 100 * (pv - exact5) / exact5,
                       "paper_cpu_s": pcpu, "paper_cpu_s_over_gpu_s": pcpu / (ms / 1e3)})
        print(f"[bench] table 5 {ng}x{ng} x {npath}: {v[0]:.5f} +- {v[1]:.5f}, {ms:.3f} ms", file=sys.stderr,
              flush=True)
    x, nrm, t1, a = cfg["points"](cfg["n_points"], cfg["seed"])
    P = dtn.Points(g, x, nrm, t1, a, cfg["n_g1"], cfg["n_g2"], cfg["delta_rel"])
    N = P.num_nodes
    nodes = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    stats = torch.empty((N, 4), dtype=torch.float64, device="cuda")
    capped = torch.empty(N, dtype=torch.int64, device="cuda")
    out = torch.empty((len(a), 4), dtype=torch.float64, device="cuda")
    walks = torch.full((N,), cfg["walks"], dtype=torch.int64, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def step(record):
        P.nodes(out=nodes)
        if record:
            ev0.record()
        dtn.wos_eval(g, nodes, walks, cfg["seed"], precision=precision, stats=stats, capped=capped)
        if record:
            ev1.record()
        P.neumann(stats, out=out)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    wos_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
        torch.cuda.synchronize()
        wos_ms.append(ev0.elapsed_time(ev1))
    sec = (time.perf_counter() - t0) / steps
    print(f"[bench] disk points {precision}: {sec * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    st = stats.cpu().numpy()
    o = out.cpu().numpy()
    walks_n, steps_n = float(st[:, 0].sum()), float(st[:, 3].sum())
    wos_s = float(np.mean(wos_ms)) / 1e3
    achieved = (DISK_SLOTS_PER_STEP[precision] * steps_n + DISK_SLOTS_PER_WALK * walks_n) / wos_s
    exact = 2.0 / (np.pi * np.sqrt(1.0 - (x[:, 0] ** 2 + x[:, 1] ** 2)))
    z = (o[:, 0] - exact) / o[:, 1]
    res = {"workload": f"exterior of a thin disk (b = 1) at u = 1, {len(a)} points on both faces x "
                       f"{cfg['n_g1']}x{cfg['n_g1']} nodes x {cfg['walks']} walks, a <= 0.4, truncation 1e5, "
                       f"eps 1e-5",
           "precision": precision, "ms_per_step": sec * 1e3, "points_per_s": len(a) / sec,
           "walks_per_s": walks_n / sec, "walk_steps_per_s": steps_n / sec, "steps_per_walk": steps_n / walks_n,
           "wos_kernel_ms": float(np.mean(wos_ms)), "capped_walks": int(capped.sum().item()),
           "rel_l2_vs_exact": float(np.linalg.norm(o[:, 0] - exact) / np.linalg.norm(exact)),
           "se_rel_l2": float(np.linalg.norm(o[:, 1]) / np.linalg.norm(exact)),
           "mean_abs_z": float(np.mean(np.abs(z))), "share_within_3_se": float(np.mean(np.abs(z) < 3)),
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK / 1e12,
                        "unit": "T lane-op slots/s", "frac": achieved / ALU_PEAK,
                        "slots_per_step": DISK_SLOTS_PER_STEP[precision], "slots_per_walk": DISK_SLOTS_PER_WALK},
           "table5": table5}
    if with_cpu:
        res["cpu_baseline"] = halfspace_cpu_baseline(gd, x, nrm, t1, a, cfg, o, cpu_points)
    return res


def sphere_exterior(precision, steps, warmup, with_cpu=True, cpu_patches=8):
    """Patches outside a ball (Sec. 5.2's big sphere: R = 3, unit charge at
    the centre, exact du/dn = 1/9 with the domain's normal).  Sec. 5.2 itself:
    the patch at (0, 0, 3) with a = 1, 16x32 nodes x 1e4 walks, 64 panels,
    its maximal relative error over r < 0.7a (the paper: below 1.25 %).
    Throughput: 2048 patches (h = 0.5, 8x16 nodes, 4x8 panels) on a
    Fibonacci lattice of the sphere, 1e4 walks per node, walks + solve per
    step; the walk kernel's ALU fraction; the oracle on a sample of patches
    with the GPU's stream ids."""
    import torch

    import dtn_inputs as I
    from paper_1210_1491_amd import dtn

    cfg = I.CONFIGS["sphere_exterior"]
    gd = cfg["geometry"]()
    g = dtn.Geometry(gd)
    # Sec. 5.2
    pd1 = I.patches_big_sphere()
    plan1 = dtn.Plan(g, pd1)
    n1 = plan1.nodes()
    st1, _ = dtn.wos_eval(g, n1, torch.full((plan1.num_nodes,), 10_000, dtype=torch.int64, device="cuda"), 5,
                          precision=precision)
    s1, e1 = plan1.solve(st1, precision=precision)
    x1, _, a1, r1 = plane_or_sphere_panels(pd1, -gd["ball_r"])
    # the second-kind equation on the same walks ((1/2 I - D) sigma = b, D != 0 on the sphere)
    s2, e2 = plan1.solve_second_kind(st1)
    s1, s2 = s1.cpu().numpy(), s2.cpu().numpy()
    tr1 = r1 < 0.7 * 1.0
    ex1 = np.full_like(s1, 1.0 / 9.0)

    def noise(e):
        return float(np.sqrt(np.sum(a1[tr1] * e.cpu().numpy()[tr1] ** 2) / np.sum(a1[tr1] * ex1[tr1] ** 2)))

    sec52 = {"max_rel_err_r_lt_0.7a": float(np.max(np.abs(s1[tr1] - 1.0 / 9.0)) * 9.0),
             "rel_l2_r_lt_0.7a": rel_l2(s1, ex1, a1, tr1),
             "median_se_rel": float(np.median(e1.cpu().numpy()[tr1]) * 9.0), "paper_bar": 0.0125,
             "propagated_noise_rel_l2": noise(e1),
             "second_kind": {"max_rel_err_r_lt_0.7a": float(np.max(np.abs(s2[tr1] - 1.0 / 9.0)) * 9.0),
                             "rel_l2_r_lt_0.7a": rel_l2(s2, ex1, a1, tr1),
                             "propagated_noise_rel_l2": noise(e2),
                             "max_abs_diff_vs_first_kind": float(np.max(np.abs(s2 - s1)))}}
    print(f"[bench] sec 5.2 max rel err {sec52['max_rel_err_r_lt_0.7a']:.4f}", file=sys.stderr, flush=True)
    # throughput
    pd = cfg["patches"](cfg["n_patches"], seed=cfg["seed"])
    plan = dtn.Plan(g, pd)
    N, Pn = plan.num_nodes, plan.num_panels
    nodes = plan.nodes()
    walks = torch.full((N,), cfg["walks"], dtype=torch.int64, device="cuda")
    stats = torch.empty((N, 4), dtype=torch.float64, device="cuda")
    capped = torch.empty(N, dtype=torch.int64, device="cuda")
    neu = torch.empty(Pn, dtype=torch.float64, device="cuda")
    nse = torch.empty(Pn, dtype=torch.float64, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def step(record):
        plan.nodes(out=nodes)
        if record:
            ev0.record()
        dtn.wos_eval(g, nodes, walks, cfg["seed"], precision=precision, stats=stats, capped=capped)
        if record:
            ev1.record()
        plan.solve(stats, precision=precision, neumann=neu, neumann_se=nse)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    wos_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
        torch.cuda.synchronize()
        wos_ms.append(ev0.elapsed_time(ev1))
    sec = (time.perf_counter() - t0) / steps
    print(f"[bench] sphere exterior {precision}: {sec * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    st = stats.cpu().numpy()
    walks_n, steps_n = float(st[:, 0].sum()), float(st[:, 3].sum())
    wos_s = float(np.mean(wos_ms)) / 1e3
    achieved = (EXT_SLOTS_PER_STEP[precision] * steps_n + EXT_SLOTS_PER_WALK * walks_n) / wos_s
    _, _, area, rc = plane_or_sphere_panels(pd, -gd["ball_r"])
    hh = np.repeat(np.asarray(pd["h"], np.float64), np.asarray(pd["n_rings"]) * np.asarray(pd["n_sectors"]))
    tr = rc < 0.7 * hh
    sig = neu.cpu().numpy()
    res = {"workload": f"outside the sphere R = 3 (unit charge at the centre), {cfg['n_patches']} patches (h = 0.5, "
                       f"8x16 nodes, 32 panels) x {cfg['walks']} walks, truncation 1e5, eps 1e-5",
           "precision": precision, "ms_per_step": sec * 1e3, "patches_per_s": cfg["n_patches"] / sec,
           "walks_per_s": walks_n / sec, "walk_steps_per_s": steps_n / sec, "steps_per_walk": steps_n / walks_n,
           "wos_kernel_ms": float(np.mean(wos_ms)), "capped_walks": int(capped.sum().item()),
           "neumann_rel_l2_vs_exact": rel_l2(sig, np.full_like(sig, 1.0 / 9.0), area, tr),
           "propagated_noise_rel_l2": float(np.sqrt(np.sum(area[tr] * nse.cpu().numpy()[tr] ** 2)
                                                    / np.sum(area[tr] / 81.0))),
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK / 1e12,
                        "unit": "T lane-op slots/s", "frac": achieved / ALU_PEAK,
                        "slots_per_step": EXT_SLOTS_PER_STEP[precision], "slots_per_walk": EXT_SLOTS_PER_WALK},
           "section_5_2": sec52}
    if with_cpu:
        res["cpu_baseline"] = exterior_cpu_baseline(gd, pd, cfg, st, cpu_patches)
    return res


def cube_tabulated(walks_per_node=10_000, n_grid=257):
    """The unit-cube tiling (1536 patches x 512 nodes) with its data given as
    257 x 257 face tables (bilinear), against the closed-form data with the
    same seed (the same walks): walk and solve time, and the Neumann error
    against the exact data for both (their difference is the interpolation's
    share)."""
    import torch

    import dtn_inputs as I
    from paper_1210_1491_amd import dtn

    pd = I.patches_cube_tiles()
    xg, ng, area, rc = plane_panels(pd)
    gd0 = I.geometry_cube_sources()
    ex = np.sum(exact_grad(gd0, xg) * ng, axis=-1)
    tr = rc < 0.7 * np.repeat(np.asarray(pd["h"], np.float64), np.asarray(pd["n_rings"]) * np.asarray(pd["n_sectors"]))
    out = {"workload": f"unit cube, 1536 patches x 512 nodes x {walks_per_node} walks, data as "
                       f"{n_grid}x{n_grid} face tables vs closed form"}
    for name, gd in (("tabulated", I.tabulated_cube_sources(n_grid, n_grid)), ("closed_form", gd0)):
        g = dtn.Geometry(gd)
        plan = dtn.Plan(g, pd)
        nodes = plan.nodes()
        W = torch.full((plan.num_nodes,), walks_per_node, dtype=torch.int64, device="cuda")
        stats, _ = dtn.wos_eval(g, nodes, W, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, _ = dtn.wos_eval(g, nodes, W, 2)
        sig, se = plan.solve(stats)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[name] = {"seconds": sec, "walks_per_s": float(plan.num_nodes) * walks_per_node / sec,
                     "neumann_rel_l2_vs_exact": rel_l2(sig.cpu().numpy(), ex, area, tr)}
    print(f"[bench] cube tabulated: {out['tabulated']['seconds']:.3f} s vs closed form "
          f"{out['closed_form']['seconds']:.3f} s", file=sys.stderr, flush=True)
    return out


def treecode_potential(m_tiles=96, n_targets=1_000_000, degree=6, theta=0.5, leaf=64, reps=3):
    """The potential (eq. bw03) of a finer cube tiling (m_tiles^2 tiles per
    face, 16 sources each: 884,736 at 96) at 1e6 targets uniform in the cube,
    by the treecode and by the direct sum, from the exact du/dn at the
    collocation points (the potential is linear in the Neumann data; this
    leg measures the summation).  Times of whole calls (tile sources,
    proxies, target sort and traversal for the treecode), interactions per
    target, the treecode's error against the direct sum on every target and
    both sums' error against the exact u at targets at least two tile sides
    from the boundary."""
    import torch

    import dtn_inputs as I
    from paper_1210_1491_amd import dtn

    gd = I.geometry_cube_sources()
    pd = I.patches_cube_tiles(m_tiles)
    xg, ng, _, _ = plane_panels(pd)
    neu = torch.tensor(np.sum(exact_grad(gd, xg) * ng, axis=-1), device="cuda")
    tg_np = np.random.default_rng([5, m_tiles]).random((n_targets, 3))
    tg = torch.tensor(tg_np, device="cuda")
    g = dtn.Geometry(gd)
    plan = dtn.Plan(g, pd)
    t0 = time.perf_counter()
    tree = dtn.Tree(plan, degree, leaf)
    t_build = time.perf_counter() - t0
    counts = torch.empty((n_targets, 2), dtype=torch.int64, device="cuda")
    u_t = tree.potential(neu, tg, theta, counts=counts)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        tree.potential(neu, tg, theta, out=u_t)
    ev[1].record()
    torch.cuda.synchronize()
    ms_tree = ev[0].elapsed_time(ev[1]) / reps
    u_d = plan.potential(neu, tg)
    torch.cuda.synchronize()
    ev[0].record()
    plan.potential(neu, tg, out=u_d)
    ev[1].record()
    torch.cuda.synchronize()
    ms_direct = ev[0].elapsed_time(ev[1])
    # speed against accuracy: other degrees and acceptance parameters, the
    # same targets, error against the direct sum
    u_dev = u_d
    sweep = []
    for deg, th in ((2, 0.7), (4, 0.7), (4, 0.5), (6, 0.7), (8, 0.5)):
        tr = dtn.Tree(plan, deg, leaf)
        u_s = tr.potential(neu, tg, th)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            tr.potential(neu, tg, th, out=u_s)
        ev[1].record()
        torch.cuda.synchronize()
        err = float(torch.max(torch.abs(u_s - u_dev)) / torch.max(torch.abs(u_dev)))
        sweep.append({"degree": deg, "theta": th, "ms": ev[0].elapsed_time(ev[1]) / reps,
                      "max_rel_diff_vs_direct": err})
        del tr
    # whole calls at other target counts (seeded uniform targets, the same
    # tree): the share of fixed work and of the traversal's tail
    scaling = []
    for n_s in (250_000, 4_000_000):
        tg_s = torch.tensor(np.random.default_rng([6, n_s]).random((n_s, 3)), device="cuda")
        u_s = tree.potential(neu, tg_s, theta)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            tree.potential(neu, tg_s, theta, out=u_s)
        ev[1].record()
        torch.cuda.synchronize()
        scaling.append({"targets": n_s, "ms": ev[0].elapsed_time(ev[1]) / reps})
        del tg_s, u_s
    scaling.insert(1, {"targets": n_targets, "ms": ms_tree})
    u_t, u_d, cnt = u_t.cpu().numpy(), u_d.cpu().numpy(), counts.cpu().numpy()
    far = np.min(np.minimum(tg_np, 1.0 - tg_np), axis=1) >= 2.0 / m_tiles
    ex = exact_u(gd, tg_np[far])
    inter = float(cnt.sum()) / n_targets
    # ALU roofline of the whole call (proxies, sort and traversal in the
    # time; the traversal's interactions as the work)
    tree_slots = float(cnt[:, 0].sum()) * TREE_PROXY_SLOTS + float(cnt[:, 1].sum()) * TREE_SOURCE_SLOTS
    tree_achieved = tree_slots / (ms_tree * 1e-3)
    out = {
        "workload": f"unit cube, {m_tiles}x{m_tiles} tiles per face ({tree.n_sources} sources), "
                    f"{n_targets} targets uniform in the cube, exact du/dn",
        "degree": degree, "theta": theta, "leaf_size": leaf,
        "clusters": tree.n_clusters, "proxies": tree.n_proxies, "tree_build_s": t_build,
        "ms_treecode": ms_tree, "ms_direct": ms_direct, "speedup": ms_direct / ms_tree,
        "interactions_per_target": inter, "direct_pairs_per_target": tree.n_sources,
        "treecode_interactions_per_s": inter * n_targets / (ms_tree * 1e-3),
        "direct_pairs_per_s": float(tree.n_sources) * n_targets / (ms_direct * 1e-3),
        "max_rel_diff_treecode_vs_direct": float(np.max(np.abs(u_t - u_d)) / np.max(np.abs(u_d))),
        "max_err_vs_exact_treecode": float(np.max(np.abs(u_t[far] - ex))),
        "max_err_vs_exact_direct": float(np.max(np.abs(u_d[far] - ex))),
        "targets_vs_exact": int(far.sum()),
        "sweep": sweep,
        "scaling": scaling,
        "roofline": {"bound": "alu", "achieved": tree_achieved / 1e12, "peak": ALU_PEAK / 1e12,
                     "unit": "T lane-op slots/s", "frac": tree_achieved / ALU_PEAK, "traffic": None,
                     "slots_per_proxy_interaction": TREE_PROXY_SLOTS,
                     "slots_per_source_interaction": TREE_SOURCE_SLOTS, "time": "whole call"},
    }
    print(f"[bench] treecode potential: {ms_tree:.1f} ms vs direct {ms_direct:.1f} ms "
          f"({out['speedup']:.1f}x), {inter:.0f} interactions per target", file=sys.stderr, flush=True)
    return out


def plane_or_sphere_panels(pd, R):
    """Panel areas and centre chord distances for patches on a sphere of
    radius |R| (the layout of include/dtn.h: uniform rings in the geodesic
    angle, parametric centres); returns (None, None, area, r)."""
    A, Rc = [], []
    r = abs(R)
    for i in range(len(pd["h"])):
        h = float(pd["h"][i])
        nr, ns = int(pd["n_rings"][i]), int(pd["n_sectors"][i])
        sm = 2.0 * np.arcsin(h / (2.0 * r))
        se = sm * np.arange(nr + 1) / nr
        s0, s1 = np.repeat(se[:-1], ns), np.repeat(se[1:], ns)
        sc = 0.5 * (s0 + s1)
        A.append(r * r * (np.cos(s0) - np.cos(s1)) * (2 * np.pi / ns))
        Rc.append(2.0 * r * np.sin(0.5 * sc))
    return None, None, np.concatenate(A), np.concatenate(Rc)


def exterior_cpu_baseline(gd, pd, cfg, gpu_stats, n_sample):
    """CPU baseline of the exterior workload: the oracle's walks at the nodes
    of the first n_sample patches with the stream ids the GPU run gave them
    (node index), so the node means can be compared one by one."""
    from oracle import patch as OP
    from oracle import wos as OW
    import dtn_inputs as I
    sub = I.subset_patches(pd, list(range(n_sample)))
    nodes = np.concatenate([OP.nodes_global(p)[0] for p in OP.patches_from_desc(sub, gd)])
    sid = np.arange(len(nodes), dtype=np.uint32)
    t0 = time.perf_counter()
    r = OW.wos_nodes(OW.Geometry(gd), nodes, cfg["walks"], seed=cfg["seed"], stream_id=sid)
    dt = time.perf_counter() - t0
    g = gpu_stats[: len(nodes)]
    gse = np.sqrt(g[:, 2] / (g[:, 0] - 1) / g[:, 0])
    z = np.abs(g[:, 1] - r["mean"]) / np.sqrt(gse ** 2 + r["se"] ** 2)
    walks = float(r["count"].sum())
    return {"value": walks / dt, "unit": "walks/s", "cores": OW.max_threads(), "kind": "oracle",
            "sample": f"nodes of the first {n_sample} patches ({len(nodes)} nodes, {walks:.3g} walks) in {dt:.1f} s",
            "gpu_same_sample": {"max_z": float(z.max()),
                                "median_rel_diff": float(np.median(np.abs(g[:, 1] - r["mean"]) / r["mean"]))}}


def halfspace_cpu_baseline(gd, x, nrm, t1, a, cfg, gpu_out, n_sample):
    """CPU baseline of a single-point workload (half space or disk): the oracle on the first
    n_sample points with the stream ids the GPU run gave their nodes (node
    index), so the oracle's walks are the GPU's (FP64) and the values of the
    sampled points can be compared one by one."""
    from oracle import point as OPt
    from oracle import wos as OW
    og = OW.Geometry(gd)
    nn = cfg["n_g1"] ** 2
    nodes = np.concatenate([OPt.hemisphere_rule(x[i], nrm[i], t1[i], a[i], cfg["n_g1"])[0] for i in range(n_sample)])
    sid = np.arange(n_sample * nn, dtype=np.uint32)
    t0 = time.perf_counter()
    r = OW.wos_nodes(og, nodes, cfg["walks"], seed=cfg["seed"], stream_id=sid)
    dt = time.perf_counter() - t0
    st = np.column_stack([r["count"], r["mean"], r["m2"], r["steps"]])
    want = np.array([OPt.point_neumann(og.phi, x[i], nrm[i], t1[i], a[i], cfg["n_g1"], cfg["n_g2"],
                                       cfg["delta_rel"], st[i * nn:(i + 1) * nn]) for i in range(n_sample)])
    d = np.abs(gpu_out[:n_sample, 0] - want[:, 0]) / want[:, 1]
    walks = float(r["count"].sum())
    return {"value": n_sample / dt, "unit": "points/s", "cores": OW.max_threads(), "kind": "oracle",
            "sample": f"first {n_sample} points ({walks:.3g} walks, {int(r['steps'].sum())} steps) in {dt:.1f} s",
            "walks_per_s": walks / dt,
            "gpu_same_sample": {"max_diff_in_se": float(d.max()),
                                "max_rel_diff": float(np.max(np.abs(gpu_out[:n_sample, 0] - want[:, 0])
                                                             / np.abs(want[:, 0])))}}


# Point-mode rule of the serving workload: 8 x 8 hemisphere nodes (half the
# patch layout's 8 x 16), the 20 x 20 ring rule and delta / a of Table 1.
POINT_RULE = (8, 20, 1e-6)


def serving(precision, window, rate, se_range, sweep_fraction=0.5, sweep_window=6, stable_only=False):
    """Query serving on the box-with-holes geometry: Poisson arrivals, each
    query 1..4096 boundary points (log-uniform) with a required standard
    error per node log-uniform on se_range, one patch per point, adaptive
    walks.  The served path: FP32-mixed walks, continuous batching across
    requests over 4 streams under a 2 GB budget.  The plain path: FP64, one
    query at a time (one stream, one query per batch), on the same arrival
    trace.  The point mode: the served path answering each point by the
    single-point estimate (no patch solve), same trace.  Latency =
    completion - arrival; patches/s = points answered / makespan.  Shorter
    runs offer a half and a quarter of the served path's measured capacity."""
    import dtn_inputs as I
    from paper_1210_1491_amd import dtn

    cfg = I.CONFIGS["serving"]
    gd = cfg["geometry"]()
    g = dtn.Geometry(gd)

    def run(rate_qps, n, prec=precision, plain=False, point=False):
        qs = I.serving_queries(gd, n_queries=n, rate=rate_qps, seed=cfg["seed"], se_range=tuple(se_range))
        mode = dict(n_streams=1, max_batch_queries=1) if plain else dict(n_streams=4)
        if point:
            mode["point_rule"] = POINT_RULE
        S = dtn.Server(g, precision=prec, hbm_budget=cfg["hbm_budget"], pilot_walks=cfg["pilot_walks"],
                       min_walks=cfg["min_walks"], max_walks=cfg["max_walks"], h_max=cfg["h_max"],
                       ladder=cfg["ladder"], layout=cfg["layout"], **mode)
        t0 = S.clock()
        done = []
        last = [time.perf_counter()]

        def progress():
            if time.perf_counter() - last[0] > 30.0:
                last[0] = time.perf_counter()
                print(f"[bench] serving: {len(done)} of {n} queries done at {S.clock() - t0:.0f} s",
                      file=sys.stderr, flush=True)

        for i, q in enumerate(qs):
            while S.clock() - t0 < q["t"]:
                done.extend(S.wait(timeout=max(0.0, min(30.0, q["t"] - (S.clock() - t0)))))
                progress()
            S.submit(i, q["pts"], q["normals"], q["se"], q["seed"])
        while len(done) < n:
            done.extend(S.wait(timeout=30.0))
            progress()
        S.close()
        assert all(d["status"] == 0 for d in done)
        lat = np.array([d["t_done"] - (t0 + qs[d["id"]]["t"]) for d in done])
        walks = sum(float(d["answer"][:, 2].sum()) for d in done)
        points = sum(len(q["pts"]) for q in qs)
        # achieved SE of each answer over its query's node SE target; points
        # whose nodes all ran the walk cap (their answers cannot meet it)
        ratio = np.concatenate([d["answer"][:, 1] / qs[d["id"]]["se"] for d in done])
        nn = cfg["layout"][0] * cfg["layout"][1]
        at_cap = np.concatenate([d["answer"][:, 2] >= nn * cfg["max_walks"] for d in done])
        q_ok = np.array([bool(np.all(d["answer"][:, 1] <= qs[d["id"]]["se"])) for d in done])
        busy = max(d["t_done"] for d in done) - t0
        out = {"rate_qps": rate_qps, "queries": n, "completions": len(done), "points": points,
               "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "percentile_samples": len(lat), "walks": walks, "makespan_s": busy,
               "served_qps": n / busy, "patches_per_s": points / busy, "walks_per_s": walks / busy,
               "median_answer_se_over_target": float(np.median(ratio)),
               "share_points_answer_se_within_target": float(np.mean(ratio <= 1.0)),
               "share_queries_every_answer_within_target": float(np.mean(q_ok)),
               "share_points_all_nodes_at_walk_cap": float(np.mean(at_cap))}
        print(f"[bench] serving {'plain fp64' if plain else prec}{' point mode' if point else ''} at "
              f"{rate_qps:.3g} q/s, {n} queries: "
              f"{out['patches_per_s']:.0f} patches/s, p50 {out['p50_ms']:.0f} ms p99 {out['p99_ms']:.0f} ms "
              f"(over {len(lat)} completions)", file=sys.stderr, flush=True)
        return out

    if stable_only:
        return {"workload": f"box_holes geometry resident; Poisson arrivals at {rate:g} q/s; 1..4096 points per "
                            f"query (log-uniform); patch per point; adaptive walks {cfg['min_walks']}.."
                            f"{cfg['max_walks']} at a per-query node SE log-uniform on [{se_range[0]:g}, "
                            f"{se_range[1]:g}]; 2 GB budget",
                "precision": precision, "stable": run(rate, window)}
    main = run(rate, window)
    plain = run(rate, window, prec="fp64", plain=True)
    point = run(rate, window, point=True)
    stable = run(sweep_fraction * main["served_qps"], sweep_window) if sweep_window > 0 else None
    low = run(0.5 * sweep_fraction * main["served_qps"], max(sweep_window // 2, 1)) if sweep_window > 0 else None
    return {"workload": f"box_holes geometry resident; Poisson arrivals at {rate:g} q/s; 1..4096 points per query "
                        f"(log-uniform); patch per point (h = 0.25 * 2^-j, 8x16 nodes, 32 panels); adaptive walks "
                        f"{cfg['min_walks']}..{cfg['max_walks']} at a per-query node SE log-uniform on "
                        f"[{se_range[0]:g}, {se_range[1]:g}]; 2 GB budget",
            "precision": precision, "served": main, "plain_fp64_per_query": plain,
            "patches_per_s_vs_plain_fp64": main["patches_per_s"] / plain["patches_per_s"],
            "point_mode": dict(point, rule={"n_g1": POINT_RULE[0], "n_g2": POINT_RULE[1],
                                            "delta_rel": POINT_RULE[2]},
                               answer="du/dn at the point by Sigma1' + Sigma2' (Sec. 5.1), no solve; a = h"),
            "points_per_s_point_mode_vs_served": point["patches_per_s"] / main["patches_per_s"],
            "stable": stable, "low": low}


def cpu_baseline(gd, pd_all, walks_per_node, g, full_walks, sigmas=None, full_walks_per_node=None):
    """The oracle on a bounded sample: the 16-tile subset of the cube tiling
    (face centres, edges, corners, 4 seeded tiles), walks_per_node each, every
    node with the stream id it has in the full launch (its global node
    index).  The FP64 GPU path then runs the identical sample (its own nodes,
    the same seed and stream ids) for a like-for-like rate and per-node
    parity: z = |mean_gpu - mean_oracle| / sqrt(se_gpu^2 + se_oracle^2).

    sigmas: the timed runs' Neumann data {(walk precision, solve precision):
    [panels]}; when the sample ran at their walk count, the oracle's own
    Neumann data on the sample (FP64 walks, FP64 solve) is the reference
    each pairing is compared with.  Also times the unit-ball workload (one
    patch, 128 nodes x 1e4 walks) on the oracle in full, beside the GPU."""
    import torch

    import dtn_inputs as I
    from oracle import patch as OP
    from oracle import wos as OW
    from paper_1210_1491_amd import dtn

    sub = I.cube_tile_subset()
    pd = I.subset_patches(pd_all, sub)
    ps = OP.patches_from_desc(pd, gd)
    nodes = np.concatenate([OP.nodes_global(p)[0] for p in ps])
    npp = nodes.shape[0] // len(sub)
    sid = (np.asarray(sub)[:, None] * npp + np.arange(npp)[None, :]).reshape(-1).astype(np.uint32)
    og = OW.Geometry(gd)
    print(f"[bench] oracle: {nodes.shape[0]} nodes x {walks_per_node} walks", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    r = OW.wos_nodes(og, nodes, walks_per_node, seed=2, stream_id=sid)
    dt = time.perf_counter() - t0
    walks = float(r["count"].sum())
    cores = OW.max_threads()
    # the GPU on the same sample
    plan = dtn.Plan(g, pd)
    nd = plan.nodes()
    n = plan.num_nodes
    w = torch.full((n,), walks_per_node, dtype=torch.int64, device=nd.device)
    st = torch.empty((n, 4), dtype=torch.float64, device=nd.device)
    S = torch.tensor(sid.view(np.int32), device=nd.device)
    dtn.wos_eval(g, nd, w, seed=2, precision="fp64", stats=st, stream_id=S)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dtn.wos_eval(g, nd, w, seed=2, precision="fp64", stats=st, stream_id=S)
    torch.cuda.synchronize()
    dt_gpu = time.perf_counter() - t1
    sg = st.cpu().numpy()
    se_g = np.sqrt(sg[:, 2] / (sg[:, 0] - 1) / sg[:, 0])
    se = np.sqrt(se_g ** 2 + r["se"] ** 2)
    diff = np.abs(sg[:, 1] - r["mean"])
    # nodes that start inside the shell: every walk ends at once, no spread on
    # either side; the means differ only by the rounding of the data there
    flat = se == 0
    z = diff[~flat] / se[~flat]
    rel_flat = diff[flat] / np.maximum(np.abs(r["mean"][flat]), 1e-300)
    out = {"value": walks / dt, "unit": "walks/s", "cores": cores, "kind": "oracle",
           "sample": f"{len(sub)} tiles x {npp} nodes x {walks_per_node} walks "
                     f"({int(walks)} walks, {int(r['steps'].sum())} steps) in {dt:.1f} s",
           "steps_per_s": float(r["steps"].sum()) / dt, "walks_per_s_per_core": walks / dt / cores,
           "extrapolated_full_workload_s": full_walks / (walks / dt),
           "gpu_same_sample": {"walks_per_s": walks / dt_gpu, "seconds": dt_gpu,
                               "ratio_gpu_over_oracle": dt / dt_gpu, "parity_max_z": float(z.max()),
                               "nodes_over_4_sigma": int((z > 4).sum()),
                               "nodes_in_shell": int(flat.sum()),
                               "in_shell_max_rel_diff": float(rel_flat.max()) if flat.any() else 0.0,
                               "identical_node_means": int((sg[:, 1] == r["mean"]).sum()), "nodes": int(n)}}
    # each walks x solve pairing of the timed runs against the oracle's own
    # Neumann data on the sample (same walks when the counts agree)
    if sigmas and full_walks_per_node == walks_per_node:
        npan = ps[0].n_rings * ps[0].n_sectors
        ref, exact, area, tr, nse = [], [], [], [], []
        for k, p in enumerate(ps):
            o = OP.patch_solve(p, og, r["mean"][k * npp:(k + 1) * npp], r["se"][k * npp:(k + 1) * npp])
            xg, ng, ar, rc = OP.collocation_points(p)
            ref.append(o["sigma"])
            nse.append(o["se"])
            exact.append(OP.exact_neumann(gd, xg, ng))
            area.append(ar)
            tr.append(rc < 0.7 * p.h)
        ref, exact, area, tr, nse = map(np.concatenate, (ref, exact, area, tr, nse))
        cols = (np.asarray(sub)[:, None] * npan + np.arange(npan)[None, :]).reshape(-1)
        den = np.sum(area[tr] * exact[tr] ** 2)
        pairs = {}
        for (wp, sp), sig in sigmas.items():
            s = sig[cols]
            pairs[f"walks_{wp}_solve_{sp}"] = {
                "rel_l2_vs_oracle": float(np.sqrt(np.sum(area[tr] * (s[tr] - ref[tr]) ** 2) / den)),
                "max_abs_vs_oracle": float(np.max(np.abs(s - ref))),
                "rel_l2_vs_exact": float(np.sqrt(np.sum(area[tr] * (s[tr] - exact[tr]) ** 2) / den))}
        out["precision_vs_oracle"] = {
            "sample": f"{len(sub)} tiles x {npan} panels, oracle FP64 walks ({walks_per_node}/node, same counters) "
                      "and FP64 solve",
            "oracle_rel_l2_vs_exact": float(np.sqrt(np.sum(area[tr] * (ref[tr] - exact[tr]) ** 2) / den)),
            "propagated_noise_rel_l2": float(np.sqrt(np.sum(area[tr] * nse[tr] ** 2) / den)),
            "pairings": pairs}
    # the unit-ball workload in full on the oracle, and on the GPU
    bd, bp = I.geometry_ball_quadratic(), I.patches_ball_pole()
    bps = OP.patches_from_desc(bp, bd)[0]
    bn, _ = OP.nodes_global(bps)
    bg = OW.Geometry(bd)
    t0 = time.perf_counter()
    br = OW.wos_nodes(bg, bn, 10_000, seed=1)
    bsol = OP.patch_solve(bps, bg, br["mean"], br["se"])
    dtb = time.perf_counter() - t0
    xg, ng, ar, _ = OP.collocation_points(bps)
    bex = OP.exact_neumann(bd, xg, ng)
    gb = dtn.Geometry(bd)
    bplan = dtn.Plan(gb, bp)
    bnodes = bplan.nodes()
    bw = torch.full((bplan.num_nodes,), 10_000, dtype=torch.int64, device=bnodes.device)
    bst, _ = dtn.wos_eval(gb, bnodes, bw, seed=1)
    bsig, _ = bplan.solve(bst)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bst, _ = dtn.wos_eval(gb, bnodes, bw, seed=1)
    bsig, _ = bplan.solve(bst)
    torch.cuda.synchronize()
    dtg = time.perf_counter() - t1
    bsig = bsig.cpu().numpy()
    bsig2 = bplan.solve_second_kind(bst)[0].cpu().numpy()

    def rel(a):
        return float(np.sqrt(np.sum(ar * (a - bex) ** 2) / np.sum(ar * bex ** 2)))

    out["unit_ball"] = {"workload": "unit ball, one patch (h 0.2) x 128 nodes x 1e4 walks, eps 1e-4, 32 panels",
                        "oracle_seconds": dtb, "oracle_walks_per_s": 1.28e6 / dtb, "gpu_seconds": dtg,
                        "gpu_walks_per_s": 1.28e6 / dtg, "oracle_rel_l2_vs_exact": rel(bsol["sigma"]),
                        "gpu_rel_l2_vs_exact": rel(bsig), "gpu_second_kind_rel_l2_vs_exact": rel(bsig2),
                        "gpu_vs_oracle_max_abs": float(np.max(np.abs(bsig - bsol["sigma"]))),
                        "neumann_se_median": float(np.median(bsol["se"]))}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the patches are independent; see the design notes for how the path would shard)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import dtn_inputs as I
    from paper_1210_1491_amd import dtn

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    gd = I.geometry_cube_sources()
    pd = I.patches_cube_tiles(m=args.tiles)
    g = dtn.Geometry(gd)
    plan = dtn.Plan(g, pd)
    N, Pn = plan.num_nodes, plan.num_panels
    walks = torch.full((N,), args.walks, dtype=torch.int64, device=dev)
    targets = torch.tensor(I.cube_targets(), device=dev)
    nodes = torch.empty((N, 3), dtype=torch.float64, device=dev)
    stats = torch.empty((N, 4), dtype=torch.float64, device=dev)
    capped = torch.empty((N,), dtype=torch.int64, device=dev)
    neumann = torch.empty(Pn, dtype=torch.float64, device=dev)
    neumann_se = torch.empty(Pn, dtype=torch.float64, device=dev)
    u = torch.empty(targets.shape[0], dtype=torch.float64, device=dev)
    xg, ng, area, rc = plane_panels(pd)
    ex = np.sum(exact_grad(gd, xg) * ng, axis=-1)
    trusted = rc < 0.7 * np.repeat(np.asarray(pd["h"], np.float64),
                                   np.asarray(pd["n_rings"]) * np.asarray(pd["n_sectors"]))
    n_patches = len(pd["h"])
    tg = targets.cpu().numpy()
    u_ex = exact_u(gd, tg)
    far = np.min(np.minimum(tg, 1 - tg), axis=1) >= 1.0 / 8

    if args.copy_probe_mib > 0:
        a = torch.empty(args.copy_probe_mib * 2 ** 17, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def measure(precision, steps, warmup):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        wos_ms = []

        def step(record):
            plan.nodes(out=nodes)
            if record:
                ev0.record()
            dtn.wos_eval(g, nodes, walks, seed=2, precision=precision, stats=stats, capped=capped)
            if record:
                ev1.record()
            plan.solve(stats, precision=precision, neumann=neumann, neumann_se=neumann_se)
            plan.potential(neumann, targets, out=u)

        for _ in range(warmup):
            step(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(True)
            torch.cuda.synchronize()
            wos_ms.append(ev0.elapsed_time(ev1))
        ms = (time.perf_counter() - t0) * 1e3 / steps
        st = stats.cpu().numpy()
        walks_n, steps_n = float(st[:, 0].sum()), float(st[:, 3].sum())
        wos_s = float(np.mean(wos_ms)) / 1e3
        slots = SLOTS_PER_STEP[precision] * steps_n + SLOTS_PER_WALK * walks_n
        sig = neumann.cpu().numpy()
        # the other solve precision on the same node statistics (walks x solve matrix)
        other = "fp32" if precision == "fp64" else "fp64"
        n2, s2 = torch.empty_like(neumann), torch.empty_like(neumann_se)
        plan.solve(stats, precision=other, neumann=n2, neumann_se=s2)
        sig_other = n2.cpu().numpy()
        solves = {precision: rel_l2(sig, ex, area, trusted), other: rel_l2(sig_other, ex, area, trusted),
                  "max_abs_diff_fp32_vs_fp64_solve": float(np.max(np.abs(sig_other - sig)))}
        # the second-kind equation (flat patches: sigma = 2b, no solve) on the
        # timed run's statistics, timed on the stream beside a first-kind solve
        second = None
        if precision == "fp64":
            n2, s2 = torch.empty_like(neumann), torch.empty_like(neumann_se)
            n1, s1 = torch.empty_like(neumann), torch.empty_like(neumann_se)
            plan.solve_second_kind(stats, neumann=n2, neumann_se=s2)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.solve_second_kind(stats, neumann=n2, neumann_se=s2)
            e1.record()
            f0.record()
            plan.solve(stats, precision="fp64", neumann=n1, neumann_se=s1)
            f1.record()
            torch.cuda.synchronize()
            sig2, sse2, sse1 = n2.cpu().numpy(), s2.cpu().numpy(), s1.cpu().numpy()
            den = np.sum(area[trusted] * ex[trusted] ** 2)
            second = {"neumann_rel_l2_vs_exact": rel_l2(sig2, ex, area, trusted),
                      "first_kind_rel_l2_vs_exact": rel_l2(n1.cpu().numpy(), ex, area, trusted),
                      "propagated_noise_rel_l2": float(np.sqrt(np.sum(area[trusted] * sse2[trusted] ** 2) / den)),
                      "first_kind_noise_rel_l2": float(np.sqrt(np.sum(area[trusted] * sse1[trusted] ** 2) / den)),
                      "solve_ms": e0.elapsed_time(e1), "first_kind_solve_ms": f0.elapsed_time(f1)}
        return {"sigma": {precision: sig, other: sig_other}, "second_kind": second, "ms_per_step": ms,
                "rel_l2_by_solve_precision": solves, "walks_per_s": walks_n / (ms / 1e3), "patches_per_s": n_patches / (ms / 1e3),
                "neumann_rel_l2_vs_exact": rel_l2(sig, ex, area, trusted),
                "neumann_se_median": float(np.median(neumann_se.cpu().numpy())),
                "potential_max_err_far": float(np.max(np.abs(u.cpu().numpy()[far] - u_ex[far]))
                                               / np.sqrt(np.mean(u_ex ** 2))),
                "steps_per_walk": steps_n / walks_n, "walk_steps_per_s": steps_n / (ms / 1e3),
                "capped_walks": int(capped.sum().item()), "wos_kernel_ms": float(np.mean(wos_ms)),
                "alu_achieved": slots / wos_s, "total_walks": walks_n}

    if args.calibrate:
        print(json.dumps({"calibration": calibrate(), "peak_lane_slots_per_s": ALU_PEAK}), flush=True)
        return
    if args.only == "box_holes":
        print(json.dumps({"box_holes": box_holes("fp32", args.steps, not args.no_cpu_baseline, args.box_holes_se,
                                                 not args.no_tune, not args.no_variants)}), flush=True)
        return
    if args.only == "serving":
        print(json.dumps({"serving": serving("fp32", args.serving_window, args.serving_rate, args.serving_se_range,
                                             sweep_window=args.serving_sweep_window,
                                             stable_only=args.serving_stable_only)}), flush=True)
        return
    if args.only == "exterior":
        print(json.dumps({"sphere_exterior": sphere_exterior(args.precision, args.steps, args.warmup,
                                                             not args.no_cpu_baseline)}), flush=True)
        return
    if args.only == "disk":
        print(json.dumps({"disk": disk(args.precision, args.steps, args.warmup, not args.no_cpu_baseline)}),
              flush=True)
        return
    if args.only == "treecode":
        print(json.dumps({"treecode_potential": treecode_potential()}), flush=True)
        return
    if args.only == "halfspace":
        print(json.dumps({"halfspace_points": halfspace_points(args.precision, args.steps, args.warmup,
                                                               not args.no_cpu_baseline)}), flush=True)
        return
    m = measure(args.precision, args.steps, args.warmup)
    variants = {}
    if not args.no_variants:
        other = "fp32" if args.precision == "fp64" else "fp64"
        v = measure(other, 1, 0)
        variants[other] = {k: v[k] for k in ("walks_per_s", "patches_per_s", "neumann_rel_l2_vs_exact",
                                              "neumann_se_median", "steps_per_walk", "wos_kernel_ms",
                                              "rel_l2_by_solve_precision")}
        variants[other]["alu_frac"] = v["alu_achieved"] / ALU_PEAK
    curve = None
    if not args.no_variants:
        # Neumann error against the walk budget, both walk precisions (each
        # with its own solve); the last point is the timed run's
        full = {args.precision: m["neumann_rel_l2_vs_exact"], other: v["neumann_rel_l2_vs_exact"]}
        budgets = [b for b in (1000, 10000) if b < args.walks] + [args.walks]
        curve = {"walks_per_node": budgets, "fp64": [], "fp32": []}
        for prec in ("fp64", "fp32"):
            for b in budgets[:-1]:
                walks.fill_(b)
                plan.nodes(out=nodes)
                dtn.wos_eval(g, nodes, walks, seed=2, precision=prec, stats=stats, capped=capped)
                plan.solve(stats, precision=prec, neumann=neumann, neumann_se=neumann_se)
                curve[prec].append(rel_l2(neumann.cpu().numpy(), ex, area, trusted))
            curve[prec].append(full[prec])
        walks.fill_(args.walks)
    ms_per_step = m["ms_per_step"]
    achieved = m["alu_achieved"]
    value = m["walks_per_s"]
    line = {
        "metric": "WOS walks/s + DtN patches/s at fixed Neumann error; p50/p99 query latency",
        "value": value,
        "unit": "walks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"unit cube, {6 * args.tiles ** 2} patches x {N // n_patches} nodes x {args.walks} walks, "
                               f"eps 1e-5, 8 point sources, 64 panels, 1e4 potential targets",
                   "patches": n_patches, "nodes": N, "walks_per_node": args.walks, "precision": args.precision},
        "patches_per_s": m["patches_per_s"],
        "neumann_rel_l2_vs_exact": m["neumann_rel_l2_vs_exact"],
        "rel_l2_by_solve_precision": m["rel_l2_by_solve_precision"],
        "neumann_se_median": m["neumann_se_median"],
        "potential_max_err_far": m["potential_max_err_far"],
        "steps_per_walk": m["steps_per_walk"],
        "walk_steps_per_s": m["walk_steps_per_s"],
        "capped_walks": m["capped_walks"],
        "wos_kernel_ms": m["wos_kernel_ms"],
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK / 1e12,
                     "unit": "T lane-op slots/s", "frac": achieved / ALU_PEAK,
                     "traffic": traffic_if_current() if args.walks == 100_000 and args.tiles == 16 else None,
                     "slots_per_step": SLOTS_PER_STEP[args.precision], "slots_per_walk": SLOTS_PER_WALK},
        "variants": variants,
        "error_vs_walks": curve,
        "second_kind": m.get("second_kind"),
    }
    if args.only is None and not args.no_box_holes:
        line["box_holes"] = box_holes("fp32", 1, not args.no_cpu_baseline, with_fp64=not args.no_variants)
    if args.only is None and not args.no_halfspace:
        line["halfspace_points"] = halfspace_points("fp64", 1, 1, not args.no_cpu_baseline)
    if args.only is None and not args.no_disk:
        line["disk"] = disk("fp64", 1, 1, not args.no_cpu_baseline)
    if args.only is None and not args.no_exterior:
        line["sphere_exterior"] = sphere_exterior("fp64", 1, 1, not args.no_cpu_baseline)
    if args.only is None and not args.no_tabulated:
        line["cube_tabulated"] = cube_tabulated()
    if args.only is None and not args.no_treecode:
        line["treecode_potential"] = treecode_potential()
    if args.only is None and not args.no_serving:
        line["serving"] = serving("fp32", args.serving_window, args.serving_rate, args.serving_se_range,
                                  sweep_window=args.serving_sweep_window)
        line["p50_latency_ms"] = line["serving"]["served"]["p50_ms"]
        line["p99_latency_ms"] = line["serving"]["served"]["p99_ms"]
    if not args.no_cpu_baseline:
        sigmas = {(args.precision, sp): a for sp, a in m["sigma"].items()}
        if not args.no_variants:
            sigmas.update({(other, sp): a for sp, a in v["sigma"].items()})
        cb = cpu_baseline(gd, pd, args.cpu_walks, g, float(N) * args.walks, sigmas, args.walks)
        if "precision_vs_oracle" in cb:
            line["precision_vs_oracle"] = cb.pop("precision_vs_oracle")
        line["unit_ball"] = cb.pop("unit_ball")
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
