"""The unit-cube workload at its full size (1536 patches x 512 nodes x 1e5
walks, eps = 1e-5), in the launch configuration the benchmark times.

Sampled nodes are recomputed one by one by the oracle at the full walk count
(same counters); the Neumann data must meet the relative L2 bar of 2e-2
against the exact data over the trusted panels; the potential must match the
exact u at interior targets away from the boundary."""
import numpy as np
import pytest
import torch

import dtn_inputs as I
from oracle import patch as OP
from oracle import wos as OW

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_cube_1536_full_size():
    from paper_1210_1491_amd import dtn
    gd = I.geometry_cube_sources()
    pd = I.patches_cube_tiles()
    print("[gpu] full cube workload", flush=True)
    g = dtn.Geometry(gd)
    plan = dtn.Plan(g, pd)
    nodes = plan.nodes()
    W = torch.full((plan.num_nodes,), 100_000, dtype=torch.int64, device="cuda")
    stats, capped = dtn.wos_eval(g, nodes, W, seed=2)
    sig, se = plan.solve(stats)
    tg = I.cube_targets()
    u = plan.potential(sig, torch.tensor(tg, device="cuda"))
    torch.cuda.synchronize()
    st, sig, se, u = stats.cpu().numpy(), sig.cpu().numpy(), se.cpu().numpy(), u.cpu().numpy()
    assert int(capped.sum()) == 0
    # sampled nodes against the oracle (identical counters: walk for walk)
    ps = OP.patches_from_desc(pd, gd)
    rng = np.random.default_rng(17)
    sample = np.sort(rng.choice(plan.num_nodes, 16, replace=False))
    on = np.concatenate([OP.nodes_global(ps[i // 512])[0][[i % 512]] for i in sample])
    assert np.max(np.abs(on - nodes.cpu().numpy()[sample])) < 1e-14
    o = OW.wos_nodes(OW.Geometry(gd), on, 100_000, seed=2, stream_id=sample.astype(np.uint32))
    gse = np.sqrt(st[sample, 2] / (st[sample, 0] - 1) / st[sample, 0])
    z = np.abs(st[sample, 1] - o["mean"]) / np.sqrt(gse ** 2 + o["se"] ** 2)
    assert np.all(z < 4), z
    assert np.median(np.abs(st[sample, 1] - o["mean"])) < 1e-12
    np.testing.assert_array_equal(st[sample, 3].astype(np.int64), o["steps"])
    # Neumann data against the exact data
    ex, area, tr = [], [], []
    for p in ps:
        xg, ng, ar, r = OP.collocation_points(p)
        ex.append(OP.exact_neumann(gd, xg, ng))
        area.append(ar)
        tr.append(r < 0.7 * p.h)
    err = OP.rel_l2(sig, *map(np.concatenate, (ex, area, tr)))
    print(f"[gpu] neumann rel-L2 vs exact {err:.3e}", flush=True)
    assert err < 2e-2
    # potential at targets at least two tile sides from the boundary
    far = np.min(np.minimum(tg, 1 - tg), axis=1) >= 1.0 / 8
    ue = OW.Geometry(gd).phi(tg)
    assert np.max(np.abs(u[far] - ue[far])) < 1e-3 * np.sqrt(np.mean(ue ** 2))
