"""HIP-graph capture of the adaptive walk pipeline through the C-ABI.

The adaptive call enqueues only stream-ordered work (allocations from the
stream-ordered pool, kernels, frees; no memsets), so a caller can capture it
into a HIP graph and replay it.  Every replay must reproduce the eager result
bit for bit (the walks are counter-based and the chunking is fixed by the
inputs), also with other eager work on the device between the replays."""
import numpy as np
import pytest
import torch

import dtn_inputs as I
from oracle import patch as OP

pytestmark = pytest.mark.gpu


def test_adaptive_pipeline_replays_from_a_captured_graph():
    from paper_1210_1491_amd import dtn
    gd = I.geometry_box_holes()
    pd = I.patches_box_holes(gd)
    idx = I.box_holes_sample(pd, per_class=1, seed=12)
    ps = OP.patches_from_desc(I.subset_patches(pd, idx), gd)
    X = np.concatenate([OP.nodes_global(p)[0] for p in ps])
    g = dtn.Geometry(gd)
    P = torch.tensor(X, device="cuda")
    n = len(X)
    budget = (64, 64, 4000, 0.05)
    s = torch.cuda.Stream()
    out = [torch.empty((n, 4), dtype=torch.float64, device="cuda"), torch.empty(n, dtype=torch.int64, device="cuda"),
           torch.empty(n, dtype=torch.int64, device="cuda")]
    with torch.cuda.stream(s):
        dtn.wos_adaptive(g, P, 3, *budget, precision="fp32", stats=out[0], walks_used=out[1], capped=out[2])
    torch.cuda.synchronize()
    eager = [t.clone() for t in out]
    print("[gpu] capture", flush=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        dtn.wos_adaptive(g, P, 3, *budget, precision="fp32", stats=out[0], walks_used=out[1], capped=out[2])
    torch.cuda.synchronize()
    W = torch.full((n,), 100, dtype=torch.int64, device="cuda")
    for rep in range(3):
        for t in out:
            t.fill_(-7)
        torch.cuda.synchronize()
        print(f"[gpu] replay {rep}", flush=True)
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, eager):
            assert torch.equal(a, b)
        dtn.wos_eval(g, P, W, 9)  # eager work between the replays
        torch.cuda.synchronize()
