"""GPU parity of adaptive walk budgets (uneven batching) through the C-ABI.

The library runs a pilot over every point in one launch, sets each point's
budget clamp(ceil(var / se^2), min, max) on the device, runs the remaining
walks of every point in one launch over the uneven work list and merges the
two statistics.  The oracle takes the same budget decision in FP64 and then
walks [0, budget) in one pass.  With the same Philox counters the FP64 path
follows the oracle walk for walk, so budgets agree as integers and means to
rounding; the FP32-mixed path is held to the statistical bar.
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


def _nodes_of(gd, pd, idx):
    ps = OP.patches_from_desc(I.subset_patches(pd, idx), gd)
    return np.concatenate([OP.nodes_global(p)[0] for p in ps])


def _gpu_adaptive(desc, pts, budget, seed, precision="fp64", schedule=None):
    dtn = _dtn()
    g = dtn.Geometry(desc)
    P = torch.tensor(np.asarray(pts, np.float64).reshape(-1, 3), device="cuda:0")
    print(f"[gpu] adaptive n={len(P)} budget={budget} seed={seed} precision={precision}", flush=True)
    stats, used, capped = dtn.wos_adaptive(g, P, seed, *budget, precision=precision, schedule=schedule)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    return {"count": st[:, 0], "mean": st[:, 1], "m2": st[:, 2], "steps": st[:, 3].astype(np.int64),
            "walks_used": used.cpu().numpy(), "capped": capped.cpu().numpy()}


def _z(gpu, ora):
    se_g = np.sqrt(gpu["m2"] / (gpu["count"] - 1) / gpu["count"])
    se = np.sqrt(se_g ** 2 + ora["se"] ** 2)
    diff = np.abs(gpu["mean"] - ora["mean"])
    return np.where(se > 0, diff / np.where(se > 0, se, 1.0), np.where(diff == 0, 0.0, np.inf))


@pytest.fixture(scope="module")
def box_holes():
    gd = I.geometry_box_holes()
    pd = I.patches_box_holes(gd)
    return gd, pd


def test_adaptive_fp64_parity_every_class(box_holes):
    gd, pd = box_holes
    pts = _nodes_of(gd, pd, I.box_holes_sample(pd, per_class=1))
    budget = (200, 300, 20_000, 0.02)  # pilot, min, max, se target
    gpu = _gpu_adaptive(gd, pts, budget, seed=4)
    ora = OW.wos_adaptive(OW.Geometry(gd), pts, *budget, seed=4)
    # the budget is an integer decided in FP64 on both sides from the same walks
    same = gpu["walks_used"] == ora["walks_used"]
    assert np.mean(same) >= 0.99, np.mean(same)
    assert np.all(np.abs(gpu["walks_used"] - ora["walks_used"]) <= 1 + 1e-3 * ora["walks_used"])
    assert len(set(ora["walks_used"].tolist())) > 10  # the budgets really are uneven
    assert ora["walks_used"].min() == 300 and ora["walks_used"].max() > 3000
    s = same
    rel = np.abs(gpu["mean"][s] - ora["mean"][s]) / np.maximum(np.abs(ora["mean"][s]), 1e-300)
    assert np.median(rel) < 1e-12, np.median(rel)
    assert np.mean(gpu["steps"][s] == ora["steps"][s]) >= 0.99
    assert np.all(_z(gpu, ora) < 4.0)
    np.testing.assert_array_equal(gpu["count"], gpu["walks_used"])
    assert np.all(gpu["capped"] == 0)


def test_adaptive_equals_plain_walks_over_the_budget(box_holes):
    """Pilot + remainder + merge = the same walks run in one pass."""
    gd, pd = box_holes
    dtn = _dtn()
    pts = _nodes_of(gd, pd, I.box_holes_sample(pd, per_class=1, seed=5))
    for precision in ("fp64", "fp32"):
        a = _gpu_adaptive(gd, pts, (128, 100, 8000, 0.03), seed=6, precision=precision)
        g = dtn.Geometry(gd)
        P = torch.tensor(pts, device="cuda:0")
        W = torch.tensor(a["walks_used"], device="cuda:0")
        st, _ = dtn.wos_eval(g, P, W, 6, precision=precision)
        st = st.cpu().numpy()
        np.testing.assert_array_equal(st[:, 0], a["count"])
        np.testing.assert_array_equal(st[:, 3].astype(np.int64), a["steps"])  # identical walks
        np.testing.assert_allclose(a["mean"], st[:, 1], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(a["m2"], st[:, 2], rtol=1e-9, atol=1e-13)


def _gpu_plain(desc, pts, walks, seed, precision):
    dtn = _dtn()
    g = dtn.Geometry(desc)
    P = torch.tensor(np.asarray(pts, np.float64).reshape(-1, 3), device="cuda:0")
    W = torch.tensor(np.asarray(walks, np.int64), device="cuda:0")
    print(f"[gpu] plain walks n={len(P)} seed={seed} precision={precision}", flush=True)
    stats, capped = dtn.wos_eval(g, P, W, seed, precision=precision)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    return {"count": st[:, 0], "mean": st[:, 1], "m2": st[:, 2], "steps": st[:, 3].astype(np.int64),
            "capped": capped.cpu().numpy()}


def test_adaptive_fp32_mixed_statistical(box_holes):
    """FP32-mixed adaptive walks against the oracle's FP64 adaptive walks.

    The two sides decide their budgets from different pilots (FP32 against
    FP64 directions), so their walk sets differ; the 4-SE bar is applied to
    the same walk set: the GPU's FP32-mixed walks over the oracle's own
    budgets (walks [0, budget) per node, the walks the adaptive path runs;
    that the adaptive path equals plain walks over its budget is tested
    above).  The budgets themselves are compared separately."""
    gd, pd = box_holes
    pts = _nodes_of(gd, pd, I.box_holes_sample(pd, per_class=1, seed=7))[::3]
    budget = (500, 500, 50_000, 0.01)
    gpu = _gpu_adaptive(gd, pts, budget, seed=8, precision="fp32")
    ora = OW.wos_adaptive(OW.Geometry(gd), pts, *budget, seed=8)
    same = _gpu_plain(gd, pts, ora["walks_used"], 8, "fp32")
    np.testing.assert_array_equal(same["count"], ora["walks_used"])
    z = _z(same, ora)
    print(f"[gpu] fp32 vs oracle on the oracle's budgets: max z {z.max():.2f}", flush=True)
    assert np.all(z < 4.0), z.max()
    # The FP32 walks follow the FP64 ones closely (same counters), so most
    # budgets agree; the pilot variance is heavy-tailed (scores near a source
    # are large), so a walk that ends differently can move a budget a lot.
    ratio = gpu["walks_used"] / ora["walks_used"]
    assert np.median(np.abs(ratio - 1.0)) < 0.02, np.median(np.abs(ratio - 1.0))
    assert np.mean((ratio > 0.8) & (ratio < 1.25)) >= 0.95, ratio
    # budgets that were not clamped meet the target
    free = (gpu["walks_used"] > budget[1]) & (gpu["walks_used"] < budget[2])
    se_g = np.sqrt(gpu["m2"] / (gpu["count"] - 1) / gpu["count"])
    assert np.median(se_g[free] / budget[3]) == pytest.approx(1.0, abs=0.1)


def test_adaptive_edge_cases(box_holes):
    gd, _ = box_holes
    dtn = _dtn()
    g = dtn.Geometry(gd)
    # empty input: nothing to do, no error
    E = torch.empty((0, 3), dtype=torch.float64, device="cuda:0")
    dtn.wos_adaptive(g, E, 1, 100, 100, 1000, 0.1)
    # a point inside the shell has zero spread: min walks (or the pilot)
    holes = np.asarray(gd["holes"]).reshape(-1, 6)
    p_shell = holes[0, :3] + np.array([0.5, 0.5, 0.0]) * (holes[0, 3:] - holes[0, :3]) - np.array([0, 0, 2e-6])
    pts = np.array([p_shell, [2.0, 2.0, 3.99]])
    gpu = _gpu_adaptive(gd, pts, (64, 1000, 5000, 1e-9), seed=1)
    assert gpu["walks_used"][0] == 1000 and gpu["steps"][0] == 0 and gpu["m2"][0] == 0.0
    assert gpu["walks_used"][1] == 5000
    ora = OW.wos_adaptive(OW.Geometry(gd), pts, 64, 1000, 5000, 1e-9, seed=1)
    np.testing.assert_array_equal(gpu["walks_used"], ora["walks_used"])
    # budget errors are argument errors, raised before any work
    P = torch.tensor(pts, device="cuda:0")
    for bad in ((1, 10, 100, 0.1), (10, 0, 100, 0.1), (10, 200, 100, 0.1), (10, 10, 100, 0.0),
                (10, 10, 100, float("nan"))):
        with pytest.raises(dtn.DtnError) as ei:
            dtn.wos_adaptive(g, P, 1, *bad)
        assert ei.value.status == -1
    with pytest.raises(dtn.DtnError):
        dtn.wos_adaptive(g, P, 1, 10, 10, 100, 0.1, schedule={"min_chunk": 0})
    with pytest.raises(dtn.DtnError):
        dtn.wos_adaptive(g, P, 1, 10, 10, 100, 0.1, schedule={"oversub": 65})


def test_schedules_change_timing_not_walks(box_holes):
    """Every schedule runs the same walks: identical step counts, means equal
    up to the rounding of the sums."""
    gd, pd = box_holes
    dtn = _dtn()
    g = dtn.Geometry(gd)
    pts = _nodes_of(gd, pd, I.box_holes_sample(pd, per_class=1, seed=9))
    rng = np.random.default_rng(9)
    P = torch.tensor(pts, device="cuda:0")
    W = torch.tensor(rng.integers(0, 6000, len(pts)), device="cuda:0")
    scheds = [{"min_chunk": 512, "oversub": 4}, {"min_chunk": 64, "oversub": 64}, {"min_chunk": 1 << 20, "oversub": 1}]
    ref = None
    for sc in scheds:
        ms, st = dtn.time_schedules(g, P, W, 3, [sc], reps=1)
        assert ms[0] > 0
        st = st.cpu().numpy()
        if ref is None:
            ref = st
        else:
            np.testing.assert_array_equal(st[:, 0], ref[:, 0])
            np.testing.assert_array_equal(st[:, 3], ref[:, 3])
            np.testing.assert_allclose(st[:, 1], ref[:, 1], rtol=1e-13, atol=1e-15)
