"""GPU parity of step 1 (walk on spheres) against the oracle, through the C-ABI.

The same Philox counters drive both sides, so the FP64 path follows the
oracle walk for walk: node means agree far inside the statistical bar (the
bar itself is 4 combined standard errors per node), step counts agree as
integers.  The FP32-mixed path draws the same counters but rounds its
directions and jumps differently, so only the statistical bar applies.
"""
import numpy as np
import pytest
import torch

import dtn_inputs as I
from oracle import patch as OP
from oracle import wos as OW

pytestmark = pytest.mark.gpu


def _dtn():
    from paper_1210_1491_amd import dtn
    return dtn


def _gpu_wos(desc, pts, walks, seed, precision="fp64", walk_begin=None, stream_id=None):
    dtn = _dtn()
    g = dtn.Geometry(desc)
    dev = torch.device("cuda:0")
    n = len(pts)
    P = torch.tensor(np.asarray(pts, np.float64).reshape(n, 3), device=dev)
    W = torch.tensor(np.broadcast_to(np.asarray(walks, np.int64), (n,)).copy(), device=dev)
    B = None if walk_begin is None else torch.tensor(np.broadcast_to(np.asarray(walk_begin, np.int64), (n,)).copy(), device=dev)
    S = None if stream_id is None else torch.tensor(np.asarray(stream_id, np.uint32).view(np.int32), device=dev)
    print(f"[gpu] wos n={n} seed={seed} precision={precision}", flush=True)
    stats, capped = dtn.wos_eval(g, P, W, seed, walk_begin=B, stream_id=S, precision=precision)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    return {"count": st[:, 0], "mean": st[:, 1], "m2": st[:, 2], "steps": st[:, 3].astype(np.int64),
            "capped": capped.cpu().numpy()}


def _se(r):
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.sqrt(r["m2"] / (r["count"] - 1) / r["count"])


def _compare(gpu, ora, exact_walks=True):
    diff = np.abs(gpu["mean"] - ora["mean"])
    se = np.sqrt(_se(gpu) ** 2 + ora["se"] ** 2)
    # a point already inside the shell has zero spread on both sides: then
    # the two means must be equal outright
    z = np.where(se > 0, diff / np.where(se > 0, se, 1.0), np.where(diff == 0, 0.0, np.inf))
    assert np.all(z < 4.0), f"max z {z.max()}"
    np.testing.assert_array_equal(gpu["count"], ora["count"])
    if exact_walks:
        # walk-for-walk agreement: means to rounding, steps as integers
        rel = np.abs(gpu["mean"] - ora["mean"]) / np.maximum(np.abs(ora["mean"]), 1e-300)
        assert np.median(rel) < 1e-12, np.median(rel)
        assert np.mean(gpu["steps"] == ora["steps"]) >= 0.99
    return z


def test_fp64_parity_ball_patch_nodes():
    gd = I.geometry_ball_quadratic()
    p = OP.patches_from_desc(I.patches_ball_pole(), gd)[0]
    nodes, _ = OP.nodes_global(p)
    walks = 10_000
    gpu = _gpu_wos(gd, nodes, walks, seed=1)
    ora = OW.wos_nodes(OW.Geometry(gd), nodes, walks, seed=1)
    _compare(gpu, ora)
    assert np.all(gpu["capped"] == 0)


def test_fp64_parity_cube_sources_ragged():
    gd = I.geometry_cube_sources()
    pts = I.interior_points_box(300, 7)
    walks = np.random.default_rng(3).integers(1, 3000, size=300)  # ragged chunks
    gpu = _gpu_wos(gd, pts, walks, seed=11)
    ora = OW.wos_nodes(OW.Geometry(gd), pts, walks, seed=11)
    _compare(gpu, ora)


def test_fp64_parity_box_minus_holes():
    holes = np.array([[0.2, 0.2, 0.2, 0.45, 0.5, 0.4], [0.6, 0.55, 0.5, 0.8, 0.75, 0.9]])
    gd = dict(I.geometry_cube_sources(), kind="box_minus_boxes", holes=holes)
    rng = np.random.default_rng(4)
    x = rng.random((2000, 3))
    keep = np.ones(len(x), bool)
    for h in holes:
        keep &= ~np.all((x >= h[:3]) & (x <= h[3:]), axis=1)
    pts = x[keep][:200]
    gpu = _gpu_wos(gd, pts, 2000, seed=12)
    ora = OW.wos_nodes(OW.Geometry(gd), pts, 2000, seed=12)
    _compare(gpu, ora)


@pytest.mark.parametrize("which", ["ball", "cube"])
def test_fp32_mixed_parity(which):
    if which == "ball":
        gd = I.geometry_ball_quadratic()
        pts = I.interior_points_ball(128, 5, r_max=0.97)
    else:
        gd = I.geometry_cube_sources()
        pts = I.interior_points_box(128, 5)
    gpu = _gpu_wos(gd, pts, 20_000, seed=3, precision="fp32")
    ora = OW.wos_nodes(OW.Geometry(gd), pts, 20_000, seed=3)
    _compare(gpu, ora, exact_walks=False)
    # same number of walks; the FP32 path measures distances in FP64 as the
    # oracle does and only its directions carry FP32 rounding, so the walks
    # take the same number of steps on average
    ratio = gpu["steps"].sum() / ora["steps"].sum()
    assert 0.99 <= ratio <= 1.01, ratio


def test_edge_cases_empty_zero_walks_shell_and_one_walk():
    gd = I.geometry_ball_quadratic(eps=1e-3)
    pts = np.array([[0.0, 0.0, 1.0 - 5e-4], [0.0, 0.5, 0.0], [0.2, 0.0, 0.1], [0.1, 0.1, 0.1]])
    walks = np.array([10, 0, 1, 65])
    gpu = _gpu_wos(gd, pts, walks, seed=1)
    ora = OW.wos_nodes(OW.Geometry(gd), pts, walks, seed=1)
    np.testing.assert_array_equal(gpu["count"], walks)
    np.testing.assert_array_equal(gpu["steps"], ora["steps"])
    assert gpu["steps"][0] == 0 and gpu["m2"][0] == 0.0
    assert gpu["mean"][1] == 0.0 and gpu["m2"][1] == 0.0
    assert gpu["m2"][2] == 0.0
    np.testing.assert_allclose(gpu["mean"], ora["mean"], rtol=1e-12, atol=1e-14)
    # n = 0 is a no-op
    dtn = _dtn()
    g = dtn.Geometry(gd)
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    s, c = dtn.wos_eval(g, e, torch.empty(0, dtype=torch.int64, device="cuda"), 1)
    assert s.shape == (0, 4)


def test_step_cap_counts_match_oracle_exactly():
    gd = I.geometry_cube_sources(max_steps=3)
    pts = I.interior_points_box(64, 9)
    gpu = _gpu_wos(gd, pts, 500, seed=2)
    ora = OW.wos_nodes(OW.Geometry(gd), pts, 500, seed=2)
    np.testing.assert_array_equal(gpu["capped"], ora["capped"])
    np.testing.assert_array_equal(gpu["steps"], ora["steps"])
    assert gpu["capped"].sum() > 0


def test_walk_ranges_compose_and_runs_are_deterministic():
    gd = I.geometry_cube_sources()
    pts = I.interior_points_box(40, 13)
    full = _gpu_wos(gd, pts, 4000, seed=5)
    again = _gpu_wos(gd, pts, 4000, seed=5)
    for k in ("count", "mean", "m2", "steps"):
        np.testing.assert_array_equal(full[k], again[k])
    a = _gpu_wos(gd, pts, 1500, seed=5)
    b = _gpu_wos(gd, pts, 2500, seed=5, walk_begin=1500)
    n = a["count"] + b["count"]
    mean = (a["count"] * a["mean"] + b["count"] * b["mean"]) / n
    np.testing.assert_allclose(mean, full["mean"], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(a["steps"] + b["steps"], full["steps"])
    # a different batch (so a different chunking) gives the same walks
    big = np.concatenate([pts, I.interior_points_box(3000, 14)])
    mixed = _gpu_wos(gd, big, 4000, seed=5, stream_id=np.arange(len(big)))
    np.testing.assert_allclose(mixed["mean"][:40], full["mean"], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(mixed["steps"][:40], full["steps"])


def test_boundary_distance_with_hole_grid_matches_oracle():
    """The walk kernels find the nearest hole through a per-cell candidate
    list; the distance must equal the plain minimum over all surfaces (to a
    few ulps), also on cell faces and next to hole faces, edges and corners."""
    dtn = _dtn()
    gd = I.geometry_box_holes()
    holes = np.asarray(gd["holes"]).reshape(-1, 6)
    rng = np.random.default_rng(12)
    pts = [rng.uniform(0.0, 4.0, (20000, 3))]
    grid = np.arange(1, 32) * 0.125  # cell faces of the 32^3 grid
    q = rng.uniform(0.0, 4.0, (6000, 3))
    k = rng.integers(0, 3, 6000)
    q[np.arange(6000), k] = rng.choice(grid, 6000) + rng.choice([-1e-7, 0.0, 1e-7], 6000)
    pts.append(q)
    for h in holes:  # next to faces, edges and corners of every hole
        lo, hi = h[:3], h[3:]
        c = rng.uniform(lo, hi, (300, 3))
        for m in range(300):
            ax = rng.permutation(3)[: 1 + m % 3]
            for a in ax:
                c[m, a] = (lo[a] - 10 ** rng.uniform(-9, -1)) if rng.random() < 0.5 else (hi[a] + 10 ** rng.uniform(-9, -1))
        pts.append(c)
    pts = np.concatenate(pts)
    inside = np.zeros(len(pts), bool)
    for h in holes:
        inside |= np.all((pts > h[:3]) & (pts < h[3:]), axis=1)
    pts = pts[~inside & np.all((pts > 0) & (pts < 4), axis=1)]
    d_ora, _ = OW.Geometry(gd).dist_proj(pts)
    g = dtn.Geometry(gd)
    P = torch.tensor(pts, device="cuda:0")
    print(f"[gpu] boundary distance n={len(pts)}", flush=True)
    d64 = dtn.boundary_distance(g, P, "fp64").cpu().numpy()
    d32 = dtn.boundary_distance(g, P, "fp32").cpu().numpy()
    assert np.max(np.abs(d64 - d_ora) / np.maximum(d_ora, 1e-300)) < 1e-14
    # the FP32-mixed walks use an unrefined rsq for hole distances: within
    # 6e-8 relative, below the 2^-22 by which their jumps are shortened
    assert np.max(np.abs(d32 - d64) / d64) < 6e-8
    assert np.all(d32 <= d64 * (1.0 + 2.0 ** -22))


def _lattice_holes():
    """40 cubes of side 0.3 on a 5 x 4 x 2 lattice in [0,4]^3: more holes than
    the candidate grid's 32-bit masks hold, so the kernels visit every hole."""
    cs = [(x, y, z) for x in (0.5, 1.25, 2.0, 2.75, 3.5) for y in (0.6, 1.55, 2.45, 3.4) for z in (1.3, 2.7)]
    return np.array([[x - 0.15, y - 0.15, z - 0.15, x + 0.15, y + 0.15, z + 0.15] for x, y, z in cs])


def test_many_holes_without_grid_match_oracle():
    dtn = _dtn()
    holes = _lattice_holes()
    assert len(holes) > 32
    rng = np.random.default_rng(14)
    src = np.column_stack([(holes[:, :3] + holes[:, 3:]) / 2, rng.normal(size=len(holes))])
    gd = dict(I.geometry_box_holes(), holes=holes, src=src)
    # distances: uniform points and points next to faces, edges and corners
    pts = [rng.uniform(0.0, 4.0, (4000, 3))]
    for h in holes[::4]:
        c = rng.uniform(h[:3], h[3:], (100, 3))
        for m in range(100):
            for a in rng.permutation(3)[: 1 + m % 3]:
                c[m, a] = (h[a] - 10 ** rng.uniform(-9, -1)) if rng.random() < 0.5 else (h[3 + a] + 10 ** rng.uniform(-9, -1))
        pts.append(c)
    pts = np.concatenate(pts)
    inside = np.zeros(len(pts), bool)
    for h in holes:
        inside |= np.all((pts > h[:3]) & (pts < h[3:]), axis=1)
    pts = pts[~inside & np.all((pts > 0) & (pts < 4), axis=1)]
    d_ora, _ = OW.Geometry(gd).dist_proj(pts)
    g = dtn.Geometry(gd)
    P = torch.tensor(pts, device="cuda:0")
    print(f"[gpu] many holes: distance n={len(pts)}", flush=True)
    d64 = dtn.boundary_distance(g, P, "fp64").cpu().numpy()
    d32 = dtn.boundary_distance(g, P, "fp32").cpu().numpy()
    assert np.max(np.abs(d64 - d_ora) / np.maximum(d_ora, 1e-300)) < 1e-14
    assert np.max(np.abs(d32 - d64) / d64) < 6e-8
    # walks, walk for walk against the oracle
    wp = pts[:150]
    print(f"[gpu] many holes: walks n={len(wp)}", flush=True)
    gpu = _gpu_wos(gd, wp, 1500, seed=15)
    ora = OW.wos_nodes(OW.Geometry(gd), wp, 1500, seed=15)
    _compare(gpu, ora)


def test_many_points_plan_in_segments_matches_oracle():
    """More than 16384 points take the multi-block plan (segment sums,
    counts, offsets): ragged walk counts with zeros; every point's count and
    walks must match the oracle's, as with the one-workgroup plan."""
    gd = I.geometry_cube_sources()
    n = 40_000
    # a margin keeps starts out of the shell (there every walk scores phi at
    # one boundary point, so the two sides' phi must agree to the bit)
    pts = I.interior_points_box(n, 31, margin=1e-3)
    # 0 or at least 2 walks (one walk has no spread on either side, and its
    # score may differ in the last bit)
    walks = np.random.default_rng(32).integers(2, 9, size=n)
    walks[:100] = 0
    walks[-50:] = 0
    walks[np.random.default_rng(33).random(n) < 0.1] = 0
    gpu = _gpu_wos(gd, pts, walks, seed=21)
    ora = OW.wos_nodes(OW.Geometry(gd), pts, walks, seed=21)
    np.testing.assert_array_equal(gpu["count"], walks)
    _compare(gpu, ora)
