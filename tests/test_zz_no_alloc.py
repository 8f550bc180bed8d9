"""dtn_wos_eval_noalloc (the walks with the library's static workspace)
against dtn_wos_eval (stream-ordered scratch), through the C-ABI.

Both run the same kernels under the same default schedule on the same
Philox counters, so every output must be identical: counts, steps and
capped counts as integers, means and M2 bit for bit.  Two calls in a row
share the workspace, the second with a smaller input (it must not see the
first call's chunk table or partials), and a call with many points uses the
multi-block plan's segment arrays.  Sizes beyond the workspace are refused
on the host before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import dtn_inputs as I

pytestmark = pytest.mark.gpu


def _dtn():
    from paper_1210_1491_amd import dtn
    return dtn


def _both(g, pts, walks, seed, precision, walk_begin=None):
    dtn = _dtn()
    n = pts.shape[0]
    ref, ref_cap = dtn.wos_eval(g, pts, walks, seed, walk_begin=walk_begin, precision=precision)
    st = torch.full((n, 4), float("nan"), dtype=torch.float64, device="cuda")
    cap = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    dtn.wos_eval_noalloc(g, pts, walks, seed, st, cap, walk_begin=walk_begin, precision=precision)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), ref_cap.cpu().numpy(), st.cpu().numpy(), cap.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_wos_eval_on_two_calls_in_a_row(precision):
    dtn = _dtn()
    dev = torch.device("cuda:0")
    # call 1: the cube tiles' sample, 16 patches x 512 nodes, ragged walk counts
    gd = I.geometry_cube_sources()
    g = dtn.Geometry(gd)
    plan = dtn.Plan(g, I.subset_patches(I.patches_cube_tiles(), I.cube_tile_subset()))
    nodes = plan.nodes()
    n1 = nodes.shape[0]
    rng = np.random.default_rng(11)
    w1 = torch.tensor(rng.integers(0, 700, n1), dtype=torch.int64, device=dev)
    print(f"[gpu] noalloc call 1: {n1} points {precision}", flush=True)
    a = _both(g, nodes, w1, 5, precision)
    # call 2: fewer points, other counts and a walk offset, same workspace
    n2 = 77
    pts = nodes[:n2].contiguous()
    w2 = torch.tensor(rng.integers(1, 300, n2), dtype=torch.int64, device=dev)
    b0 = torch.tensor(rng.integers(0, 1000, n2), dtype=torch.int64, device=dev)
    print(f"[gpu] noalloc call 2: {n2} points {precision}", flush=True)
    b = _both(g, pts, w2, 6, precision, walk_begin=b0)
    for ref, ref_cap, got, cap in (a, b):
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(cap, ref_cap)
    assert np.all(a[0][:, 0] == w1.cpu().numpy()) and np.all(b[0][:, 0] == w2.cpu().numpy())
    assert dtn.check(g) == "ok"


def test_noalloc_multi_block_plan_and_capped_walks():
    dtn = _dtn()
    dev = torch.device("cuda:0")
    g = dtn.Geometry(I.geometry_cube_sources(max_steps=12))
    n = 20_000  # above the single-block plan's limit: segment arrays in the workspace
    pts = torch.tensor(I.interior_points_box(n, 21), device=dev)
    w = torch.full((n,), 40, dtype=torch.int64, device=dev)
    print(f"[gpu] noalloc multi-block {n} points", flush=True)
    ref, ref_cap, got, cap = _both(g, pts, w, 9, "fp64")
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(cap, ref_cap)
    assert cap.sum() > 0
    assert dtn.check(g) == "maxsteps"
    # then a small call again: the shared workspace holds the large call's data
    small = pts[:5].contiguous()
    ref, ref_cap, got, cap = _both(g, small, w[:5].contiguous(), 10, "fp64")
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(cap, ref_cap)


def test_noalloc_refuses_sizes_beyond_its_workspace():
    dtn = _dtn()
    L = dtn.lib()
    g = dtn.Geometry(I.geometry_cube_sources())
    t = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(t.data_ptr())
    # refused on the host before any device work: the arrays are never read
    st = L.dtn_wos_eval_noalloc(g.handle, p, 2_000_000, p, None, 1, None, 0, p, None,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -1
    assert "workspace" in L.dtn_last_error().decode()
    st = L.dtn_wos_eval_noalloc(g.handle, p, 0, None, None, 1, None, 0, None, None, None)
    assert st == 0
