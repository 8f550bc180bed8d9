"""GPU tests of the query server (continuous batching) through the C-ABI.

Each answer is checked against the oracle run on the same patch (centred on
the query point, h from the same ladder, which the test recomputes on its
own), the same seed and the same per-node stream ids; a query's walks must
not depend on the queries it is batched with; admission must hold the
device memory of the batches in flight under the budget.
"""
import numpy as np
import pytest

import dtn_inputs as I
from oracle import patch as OP
from oracle import point as OPt
from oracle import wos as OW

pytestmark = pytest.mark.gpu

LAYOUT = (8, 16, 4, 8)


def _dtn():
    from paper_1210_1491_amd import dtn
    return dtn


def _ladder_h(gd, x, nrm, h_max=0.25, ladder=16):
    """Independent statement of the server's rung choice."""
    k = int(np.argmax(np.abs(nrm)))
    a, b = (k + 1) % 3, (k + 2) % 3
    lo, hi = np.asarray(gd["box_lo"], float), np.asarray(gd["box_hi"], float)
    holes = np.asarray(gd["holes"]).reshape(-1, 6)
    own = None
    for j, h in enumerate(holes):
        plane = h[k] if nrm[k] > 0 else h[3 + k]
        if abs(x[k] - plane) < 1e-9 and h[a] <= x[a] <= h[3 + a] and h[b] <= x[b] <= h[3 + b]:
            own = j
    rlo, rhi = (lo, hi) if own is None else (holes[own, :3], holes[own, 3:])
    cap = min(x[a] - rlo[a], rhi[a] - x[a], x[b] - rlo[b], rhi[b] - x[b])
    for k2 in range(3):
        for s, plane in ((-1.0, lo[k2]), (1.0, hi[k2])):
            if own is None and k2 == k and s == nrm[k]:
                continue
            cap = min(cap, abs(x[k2] - plane))
    for j, h in enumerate(holes):
        if j != own:
            q = np.maximum(np.maximum(h[:3] - x, x - h[3:]), 0.0)
            cap = min(cap, float(np.linalg.norm(q)))
    for j in range(ladder):
        hh = h_max * 2.0 ** -j
        if hh <= cap * (1 - 1e-9):
            return hh
    return None


def _run(server, queries, timeout=120.0):
    outs = {}
    for qid, (pts, nrm, se, seed) in queries.items():
        server.submit(qid, pts, nrm, se, seed)
    done = []
    while len(done) < len(queries):
        r = server.wait(timeout=timeout)
        assert r, "server wait timed out"
        done.extend(r)
    for d in done:
        assert d["status"] == 0, d
        outs[d["id"]] = d
    return outs


def test_server_answers_match_oracle_fp64():
    dtn = _dtn()
    gd = I.geometry_box_holes()
    rng = np.random.default_rng(21)
    pts, nrm = I.boundary_points(gd, 5, rng)
    budget = (64, 64, 4000, 0.05)  # pilot, min, max, se target
    S = dtn.Server(dtn.Geometry(gd), n_streams=2, precision="fp64", pilot_walks=budget[0], min_walks=budget[1],
                   max_walks=budget[2], layout=LAYOUT)
    print(f"[gpu] server fp64 parity n={len(pts)}", flush=True)
    out = _run(S, {7: (pts, nrm, budget[3], 77)})[7]["answer"]
    S.close()
    ps = []
    for i in range(len(pts)):
        h = _ladder_h(gd, pts[i], nrm[i])
        assert out[i, 3] == h
        k = int(np.argmax(np.abs(nrm[i])))
        t1 = np.zeros(3)
        t1[(k + 1) % 3] = 1.0
        ps.append(OP.Patch(pts[i], nrm[i], t1, h, *LAYOUT))
    nodes = np.concatenate([OP.nodes_global(p)[0] for p in ps])
    g = OW.Geometry(gd)
    r = OW.wos_adaptive(g, nodes, *budget[:3], budget[3], seed=77, stream_id=np.arange(len(nodes)))
    nn = LAYOUT[0] * LAYOUT[1]
    for i, p in enumerate(ps):
        s = slice(i * nn, (i + 1) * nn)
        se_nodes = np.sqrt(r["m2"][s] / (r["count"][s] - 1) / r["count"][s])
        value, se = OP.central_disk_answer(p, g, r["mean"][s], se_nodes)
        assert abs(out[i, 2] - r["walks_used"][s].sum()) <= 0.001 * out[i, 2]
        assert abs(out[i, 0] - value) < 0.01 * se, (i, out[i], value, se)
        assert out[i, 1] == pytest.approx(se, rel=1e-3)


def test_point_mode_answers_match_oracle_fp64():
    """Point mode (Sec. 5.1, no solve): every answer against the oracle's
    single-point estimate on its own hemisphere nodes (a = the ladder's h),
    walked with the same seed, stream ids and adaptive budgets."""
    dtn = _dtn()
    gd = I.geometry_box_holes()
    rng = np.random.default_rng(31)
    pts, nrm = I.boundary_points(gd, 6, rng)
    budget = (64, 64, 4000, 0.05)
    rule = (8, 12, 1e-6)
    S = dtn.Server(dtn.Geometry(gd), n_streams=2, precision="fp64", pilot_walks=budget[0], min_walks=budget[1],
                   max_walks=budget[2], layout=LAYOUT, point_rule=rule)
    print(f"[gpu] server point mode n={len(pts)}", flush=True)
    out = _run(S, {9: (pts, nrm, budget[3], 99)})[9]["answer"]
    S.close()
    g = OW.Geometry(gd)
    frames, nodes = [], []
    for i in range(len(pts)):
        h = _ladder_h(gd, pts[i], nrm[i])
        assert out[i, 3] == h
        k = int(np.argmax(np.abs(nrm[i])))
        t1 = np.zeros(3)
        t1[(k + 1) % 3] = 1.0
        frames.append((pts[i], nrm[i], t1, h))
        nodes.append(OPt.hemisphere_rule(pts[i], nrm[i], t1, h, rule[0])[0])
    r = OW.wos_adaptive(g, np.concatenate(nodes), *budget[:3], budget[3], seed=99,
                        stream_id=np.arange(len(pts) * rule[0] ** 2))
    nn = rule[0] ** 2
    for i, (x, n, t1, a) in enumerate(frames):
        s = slice(i * nn, (i + 1) * nn)
        st = np.stack([r["count"][s], r["mean"][s], r["m2"][s], r["steps"][s]], axis=-1)
        value, se, _, _ = OPt.point_neumann(g.phi, x, n, t1, a, rule[0], rule[1], rule[2], st)
        bound = OPt.sigma2_rounding_bound(g.phi, x, n, t1, a, rule[1], rule[2])
        assert out[i, 2] == r["walks_used"][s].sum()
        assert abs(out[i, 0] - value) < 0.01 * se + bound, (i, out[i], value, se)
        assert out[i, 1] == pytest.approx(se, rel=1e-3)


def test_point_mode_fp32_mixed_agrees_with_fp64():
    """The serving benchmark's precision: FP32-mixed walks in point mode give
    answers within 4 sqrt(SE_32^2 + SE_64^2) of the FP64 ones (same seeds and
    stream ids: the paths differ only where FP32 rounding moves a walk), with
    the same a and a comparable walk count."""
    dtn = _dtn()
    gd = I.geometry_box_holes()
    rng = np.random.default_rng(32)
    pts, nrm = I.boundary_points(gd, 40, rng)
    g = dtn.Geometry(gd)
    res = {}
    for prec in ("fp64", "fp32"):
        S = dtn.Server(g, n_streams=2, precision=prec, pilot_walks=64, min_walks=64, max_walks=20000,
                       layout=LAYOUT, point_rule=(8, 20, 1e-6))
        print(f"[gpu] server point mode {prec}", flush=True)
        res[prec] = _run(S, {5: (pts, nrm, 0.02, 55)})[5]["answer"]
        S.close()
    a, b = res["fp64"], res["fp32"]
    np.testing.assert_array_equal(a[:, 3], b[:, 3])
    z = np.abs(a[:, 0] - b[:, 0]) / np.sqrt(a[:, 1] ** 2 + b[:, 1] ** 2)
    assert np.all(z < 4.0), z.max()
    assert np.all(np.abs(b[:, 2] / a[:, 2] - 1.0) < 0.5)


def test_answer_does_not_depend_on_the_batch():
    dtn = _dtn()
    gd = I.geometry_box_holes()
    rng = np.random.default_rng(22)
    qs = {}
    for qid, m in zip(range(10, 15), (3, 40, 17, 1, 60)):
        p, n = I.boundary_points(gd, m, rng)
        qs[qid] = (p, n, 0.05, 1000 + qid)
    g = dtn.Geometry(gd)
    kw = dict(precision="fp32", pilot_walks=64, min_walks=64, max_walks=3000, layout=LAYOUT)
    alone = dtn.Server(g, n_streams=1, **kw)
    print("[gpu] server alone", flush=True)
    a = _run(alone, {12: qs[12]})[12]["answer"]
    alone.close()
    mix = dtn.Server(g, n_streams=3, **kw)
    print("[gpu] server mix", flush=True)
    res = _run(mix, qs)
    mix.close()
    # the same walks (the pilot walks fit in one chunk per node either way,
    # so the budgets agree exactly); the remainder's chunks depend on the
    # batch, so the sums may round differently
    b = res[12]["answer"]
    np.testing.assert_array_equal(b[:, 2:], a[:, 2:])  # walks and h
    np.testing.assert_allclose(b[:, :2], a[:, :2], rtol=1e-11, atol=1e-14)
    for d in res.values():
        assert np.all(np.isfinite(d["answer"]))


def test_admission_keeps_memory_under_budget():
    dtn = _dtn()
    gd = I.geometry_box_holes()
    rng = np.random.default_rng(23)
    g = dtn.Geometry(gd)
    kw = dict(precision="fp32", pilot_walks=32, min_walks=32, max_walks=256, layout=LAYOUT)
    probe = dtn.Server(g, n_streams=1, **kw)
    fp = probe.footprint(300)
    probe.close()
    S = dtn.Server(g, n_streams=4, hbm_budget=int(1.5 * fp), **kw)
    qs = {}
    for qid in range(4):
        p, n = I.boundary_points(gd, 300, rng)
        qs[qid] = (p, n, 0.2, 50 + qid)
    print("[gpu] server admission", flush=True)
    res = sorted(_run(S, qs).values(), key=lambda d: d["t_start"])
    S.close()
    for prev, nxt in zip(res, res[1:]):
        assert nxt["t_start"] >= prev["t_done"]  # only one query fits at a time
    # with room for all of them, several run at once
    S = dtn.Server(g, n_streams=4, hbm_budget=8 * fp, **kw)
    res = sorted(_run(S, qs).values(), key=lambda d: d["t_start"])
    S.close()
    assert any(nxt["t_start"] < prev["t_done"] for prev, nxt in zip(res, res[1:]))


def test_server_rejects_bad_queries():
    dtn = _dtn()
    gd = I.geometry_box_holes()
    g = dtn.Geometry(gd)
    S = dtn.Server(g, n_streams=1, pilot_walks=32, min_walks=32, max_walks=64, layout=LAYOUT, max_points=16)
    good, n = I.boundary_points(gd, 2, np.random.default_rng(24))
    bad = good.copy()
    bad[0] += 0.01 * n[0] - 0.013  # off the boundary
    with pytest.raises(dtn.DtnError):
        S.submit(1, bad, n, 0.1, 1)
    edge = np.array([[0.0, 2.0, 1e-9]])  # on an outer face, at an edge
    with pytest.raises(dtn.DtnError):
        S.submit(2, edge, np.array([[-1.0, 0.0, 0.0]]), 0.1, 1)
    with pytest.raises(dtn.DtnError):
        S.submit(3, good, -n, 0.1, 1)  # wrong normal
    with pytest.raises(dtn.DtnError):
        S.submit(4, np.repeat(good[:1], 17, 0), np.repeat(n[:1], 17, 0), 0.1, 1)  # over max_points
    with pytest.raises(dtn.DtnError):
        S.submit(5, good, n, 0.0, 1)
    assert S.in_flight() == 0
    S.close()
    with pytest.raises(dtn.DtnError):
        dtn.Server(g, n_streams=0)
    with pytest.raises(dtn.DtnError):
        dtn.Server(dtn.Geometry(I.geometry_ball_quadratic()))


def test_one_query_per_batch_matches_batching_across_requests():
    """The per-query mode (one query per batch, one stream) gives the walks
    and answers of batching across requests, and runs the queries one after
    another."""
    dtn = _dtn()
    gd = I.geometry_box_holes()
    rng = np.random.default_rng(25)
    qs = {}
    for qid, m in zip(range(30, 35), (9, 10, 3, 17, 10)):
        p, n = I.boundary_points(gd, m, rng)
        qs[qid] = (p, n, 0.05, 500 + qid)
    g = dtn.Geometry(gd)
    kw = dict(precision="fp32", pilot_walks=64, min_walks=64, max_walks=3000, layout=LAYOUT)
    res = {}
    for name, extra in (("per_query", dict(n_streams=1, max_batch_queries=1)), ("batched", dict(n_streams=2))):
        S = dtn.Server(g, **kw, **extra)
        print(f"[gpu] server {name}", flush=True)
        res[name] = _run(S, qs)
        S.close()
    for qid in qs:
        a, b = res["per_query"][qid]["answer"], res["batched"][qid]["answer"]
        np.testing.assert_array_equal(b[:, 2:], a[:, 2:])  # walks and h
        np.testing.assert_allclose(b[:, :2], a[:, :2], rtol=1e-11, atol=1e-14)
    per = sorted(res["per_query"].values(), key=lambda d: d["t_start"])
    for prev, nxt in zip(per, per[1:]):
        assert nxt["t_start"] >= prev["t_done"]


def test_graph_replay_is_rejected_while_switched_off():
    dtn = _dtn()
    g = dtn.Geometry(I.geometry_box_holes())
    with pytest.raises(dtn.DtnError, match="graph replay"):
        dtn.Server(g, graphs=True, layout=LAYOUT)


@pytest.mark.skip(reason="server graph replay is switched off: a four-stream serving run with it ended in a host "
                         "segmentation fault whose cause is not yet shown; the server rejects the mode")
def test_graph_replay_matches_direct_launches():
    """Batches replayed from captured graphs (padded to their size bucket)
    give the direct launches' walks and answers; a bucket's graph replayed
    for a later batch reads that batch's own staging."""
    dtn = _dtn()
    gd = I.geometry_box_holes()
    rng = np.random.default_rng(25)
    qs = {}
    # 9 and 10 share the 10-row bucket (captured once, replayed for the
    # later one); 17 pads to 20; 3 is unpadded
    for qid, m in zip(range(30, 35), (9, 10, 3, 17, 10)):
        p, n = I.boundary_points(gd, m, rng)
        qs[qid] = (p, n, 0.05, 500 + qid)
    g = dtn.Geometry(gd)
    kw = dict(precision="fp32", pilot_walks=64, min_walks=64, max_walks=3000, layout=LAYOUT)
    res = {}
    for name, extra in (("direct", dict(graphs=False, n_streams=1, max_batch_queries=1)),
                        ("graph", dict(graphs=True, n_streams=1, max_batch_queries=1))):
        S = dtn.Server(g, **kw, **extra)
        print(f"[gpu] server {name}", flush=True)
        res[name] = _run(S, qs)
        S.close()
    for qid in qs:
        a, b = res["direct"][qid]["answer"], res["graph"][qid]["answer"]
        np.testing.assert_array_equal(b[:, 2:], a[:, 2:])  # walks and h
        np.testing.assert_allclose(b[:, :2], a[:, :2], rtol=1e-11, atol=1e-14)
