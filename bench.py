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

# Full-rate lane-op slots of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
ALU_PEAK = 256 * 4 * 16 * 2.4e9
# Algorithmic work, in full-rate lane-op slots (a quarter-rate op such as a
# 32x32->64 multiply or a square root counts 4), per walk step and per walk,
# for the box domain with point-source data.  The table behind these numbers
# is in the design notes; it counts what the step definition requires, not
# what the compiler emits.
SLOTS_PER_STEP = {"fp64": 108, "fp32": 87}
SLOTS_PER_WALK = 158


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
    ap.add_argument("--cpu-walks", type=int, default=40000, help="walks per node in the CPU sample")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (reference for HBM counters)")
    return ap.parse_args()


def cpu_baseline(gd, pd_all, walks_per_node):
    """The oracle on a bounded sample: the 16-tile subset of the cube tiling
    (face centres, edges, corners, 4 seeded tiles), walks_per_node each."""
    import dtn_inputs as I
    from oracle import patch as OP
    from oracle import wos as OW

    sub = I.cube_tile_subset()
    pd = I.subset_patches(pd_all, sub)
    ps = OP.patches_from_desc(pd, gd)
    nodes = np.concatenate([OP.nodes_global(p)[0] for p in ps])
    g = OW.Geometry(gd)
    t0 = time.perf_counter()
    r = OW.wos_nodes(g, nodes, walks_per_node, seed=2)
    dt = time.perf_counter() - t0
    walks = float(r["count"].sum())
    return {"value": walks / dt, "unit": "walks/s", "cores": OW.max_threads(), "kind": "oracle",
            "sample": f"{len(sub)} tiles x {nodes.shape[0] // len(sub)} nodes x {walks_per_node} walks "
                      f"({int(walks)} walks, {int(r['steps'].sum())} steps) in {dt:.1f} s",
            "steps_per_s": float(r["steps"].sum()) / dt}


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
    from oracle import patch as OP  # exact data and panel geometry only
    from oracle import wos as OW

    ps = OP.patches_from_desc(pd, gd)
    ex, area, trusted = [], [], []
    for p in ps:
        xg, ng, ar, r = OP.collocation_points(p)
        ex.append(OP.exact_neumann(gd, xg, ng))
        area.append(ar)
        trusted.append(r < 0.7 * p.h)
    ex, area, trusted = map(np.concatenate, (ex, area, trusted))
    tg = targets.cpu().numpy()
    u_ex = OW.Geometry(gd).phi(tg)
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
        return {"ms_per_step": ms, "walks_per_s": walks_n / (ms / 1e3), "patches_per_s": len(ps) / (ms / 1e3),
                "neumann_rel_l2_vs_exact": OP.rel_l2(sig, ex, area, trusted),
                "neumann_se_median": float(np.median(neumann_se.cpu().numpy())),
                "potential_max_err_far": float(np.max(np.abs(u.cpu().numpy()[far] - u_ex[far]))
                                               / np.sqrt(np.mean(u_ex ** 2))),
                "steps_per_walk": steps_n / walks_n, "walk_steps_per_s": steps_n / (ms / 1e3),
                "capped_walks": int(capped.sum().item()), "wos_kernel_ms": float(np.mean(wos_ms)),
                "alu_achieved": slots / wos_s, "total_walks": walks_n}

    m = measure(args.precision, args.steps, args.warmup)
    variants = {}
    if not args.no_variants:
        other = "fp32" if args.precision == "fp64" else "fp64"
        v = measure(other, 1, 0)
        variants[other] = {k: v[k] for k in ("walks_per_s", "patches_per_s", "neumann_rel_l2_vs_exact",
                                              "neumann_se_median", "steps_per_walk", "wos_kernel_ms")}
        variants[other]["alu_frac"] = v["alu_achieved"] / ALU_PEAK
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
        "config": {"workload": f"unit cube, {6 * args.tiles ** 2} patches x {N // len(ps)} nodes x {args.walks} walks, "
                               f"eps 1e-5, 8 point sources, 64 panels, 1e4 potential targets",
                   "patches": len(ps), "nodes": N, "walks_per_node": args.walks, "precision": args.precision},
        "patches_per_s": m["patches_per_s"],
        "neumann_rel_l2_vs_exact": m["neumann_rel_l2_vs_exact"],
        "neumann_se_median": m["neumann_se_median"],
        "potential_max_err_far": m["potential_max_err_far"],
        "steps_per_walk": m["steps_per_walk"],
        "walk_steps_per_s": m["walk_steps_per_s"],
        "capped_walks": m["capped_walks"],
        "wos_kernel_ms": m["wos_kernel_ms"],
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK / 1e12,
                     "unit": "TOP/s (full-rate lane-op slots)", "frac": achieved / ALU_PEAK,
                     "traffic": None},
        "variants": variants,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(gd, pd, args.cpu_walks)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
