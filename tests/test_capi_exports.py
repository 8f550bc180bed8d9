"""The C-ABI library loads on the CPU and exports every function that
include/dtn.h declares; its host-side operator builder agrees with the
oracle's (independent code) to rounding."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dtn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dtn_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1210_1491_amd import dtn
    lib = ctypes.CDLL(dtn.LIB_PATH)
    names = _declared()
    assert "dtn_wos_eval" in names and "dtn_patch_solve" in names and "dtn_potential" in names
    assert "dtn_create_points" in names and "dtn_points_neumann" in names
    for n in names:
        assert hasattr(lib, n), n
    assert "gfx950" in dtn.version()


@pytest.mark.parametrize("layout", [(16, 32, 4, 16, 0.0), (8, 16, 4, 8, 5.0), (6, 12, 2, 8, 0.0),
                                    (16, 32, 4, 16, -3.0), (8, 16, 4, 8, -5.0)])
def test_host_operators_agree_with_oracle(layout):
    from oracle import patch as OP
    from paper_1210_1491_amd import dtn
    nt, nf, nr, ns, rr = layout
    ops = dtn.class_operators(nt, nf, nr, ns, rr)
    h, R = (1.0, None) if rr == 0.0 else (0.2, 0.2 * rr)
    K = OP.single_layer_matrix(h, R, nr, ns)
    QI = OP.gamma_operator(h, R, nt, nf, nr, ns)
    assert np.max(np.abs(ops["K"] * h - K)) < 1e-12 * np.max(np.abs(K))
    assert np.max(np.abs(ops["QI"] - QI)) < 1e-12
    Y, _, _, _ = OP.node_grid(h, R, nt, nf)
    assert np.max(np.abs(ops["node_tab"] * h - Y)) < 1e-15
    A = np.linalg.solve(K, QI) * h
    np.testing.assert_allclose(ops["A2"], A * A, rtol=1e-9, atol=1e-14)
    _, X, _, _ = OP.panels(h, R, nr, ns)
    assert np.max(np.abs(ops["col_tab"] * h - X)) < 1e-15


def test_host_operator_arguments_are_checked():
    from paper_1210_1491_amd import dtn
    with pytest.raises(dtn.DtnError):
        dtn.class_operators(1, 16, 4, 8)
    with pytest.raises(dtn.DtnError):
        dtn.class_operators(8, 15, 4, 8)
    with pytest.raises(dtn.DtnError):  # |R| < h on either side of a sphere
        dtn.class_operators(8, 16, 4, 8, -0.5)


def test_server_footprint_is_host_side_and_checked():
    """The device footprint the server's admission uses is a host function:
    affine in the number of points (per-node arrays plus a fixed walk
    scratch), at least the bytes of the batch's own arrays, and -1 for an
    invalid configuration."""
    from paper_1210_1491_amd import dtn
    L = dtn.lib()
    cfg = dtn.ServerConfigDesc(4, 1, 2 << 30, 100, 100, 1_000_000, 0.25, 16, 8, 16, 4, 8, 4096, 0, 0)
    f = [L.dtn_server_footprint(ctypes.byref(cfg), n) for n in (1, 2, 100, 4096)]
    nodes = 8 * 16
    per_point = f[2] - f[1]
    assert per_point > 0 and abs((f[3] - f[2]) - 3996 * per_point / 98) <= 4096 * 256
    # the per-node arrays alone: nodes (24 B), stats (32), budgets and counts (8 + 8),
    # walk identities (8 + 4 + 8); panels: Neumann data and SE (2 x 8 x 32)
    assert per_point >= nodes * (24 + 32 + 16 + 20) + 32 * 16
    for bad in (dtn.ServerConfigDesc(0, 1, 2 << 30, 100, 100, 1_000_000, 0.25, 16, 8, 16, 4, 8, 4096, 0, 0),
                dtn.ServerConfigDesc(4, 1, 2 << 30, 1, 100, 1_000_000, 0.25, 16, 8, 16, 4, 8, 4096, 0, 0),
                dtn.ServerConfigDesc(4, 1, 2 << 30, 100, 100, 1_000_000, 0.25, 16, 8, 16, 4, 8, 4096, 2, 0),
                dtn.ServerConfigDesc(4, 1, 2 << 30, 100, 100, 1_000_000, 0.25, 16, 8, 16, 4, 8, 4096, 0, -1)):
        assert L.dtn_server_footprint(ctypes.byref(bad), 10) == -1


def test_server_footprint_in_point_mode():
    """Point mode: n_g1^2 nodes per point and no panels; invalid rules give -1."""
    from paper_1210_1491_amd import dtn
    L = dtn.lib()
    base = (4, 1, 2 << 30, 100, 100, 1_000_000, 0.25, 16, 8, 16, 4, 8, 4096, 0, 0)
    pm = dtn.ServerConfigDesc(*base, 20, 20, 1e-6)
    f = [L.dtn_server_footprint(ctypes.byref(pm), n) for n in (1, 2, 100)]
    per_point = f[2] - f[1]
    assert per_point > 0 and abs((f[2] - f[1]) - 98 * (f[1] - f[0])) <= 98 * 256 * 16
    assert per_point >= 400 * (24 + 32 + 16 + 20)
    patch = L.dtn_server_footprint(ctypes.byref(dtn.ServerConfigDesc(*base)), 100)
    assert patch != f[2]
    for bad in ((20, 0, 1e-6), (65, 20, 1e-6), (20, 20, 0.0), (20, 20, 1.0), (-1, 20, 1e-6)):
        assert L.dtn_server_footprint(ctypes.byref(dtn.ServerConfigDesc(*base, *bad)), 10) == -1, bad
    # n_g1 = 0 is patch mode: the other point fields are not read
    assert L.dtn_server_footprint(ctypes.byref(dtn.ServerConfigDesc(*base, 0, 0, 0.0)), 100) == patch


def _bucket(n, max_points):
    """Size buckets of graph replay, stated independently: n itself up to 8,
    then the smallest m 2^e >= n with m in 5..8, capped at max_points."""
    if n <= 8:
        return n
    cands = [m << e for e in range(0, 21) for m in (5, 6, 7, 8) if (m << e) >= n]
    return min(min(cands), max_points)


@pytest.mark.parametrize("max_points", [4096, 4000])
def test_server_footprint_under_graph_replay_is_that_of_the_padded_batch(max_points):
    from paper_1210_1491_amd import dtn
    L = dtn.lib()
    direct = dtn.ServerConfigDesc(4, 1, 2 << 30, 100, 100, 1_000_000, 0.25, 16, 8, 16, 4, 8, max_points, 0, 0)
    graph = dtn.ServerConfigDesc(4, 1, 2 << 30, 100, 100, 1_000_000, 0.25, 16, 8, 16, 4, 8, max_points, 1, 0)
    sizes = list(range(1, 70)) + [99, 100, 101, 129, 1000, 3000, 3999, 4000]
    for n in sizes:
        b = _bucket(n, max_points)
        assert n <= b <= max(n, min(max_points, int(n * 1.25) + 1))
        got = L.dtn_server_footprint(ctypes.byref(graph), n)
        assert got == L.dtn_server_footprint(ctypes.byref(direct), b), (n, b)


def test_points_arguments_are_checked_before_any_device_work():
    """NULL handles and arrays are refused on the host (no GPU needed)."""
    from paper_1210_1491_amd import dtn
    L = dtn.lib()
    h = ctypes.c_void_p()
    assert L.dtn_create_points(None, None, 1, 20, 20, 1e-6, ctypes.byref(h)) == -1
    assert "NULL" in L.dtn_last_error().decode()
    assert L.dtn_points_nodes(None, None, None) == -1
    assert L.dtn_points_neumann(None, None, None, None) == -1
    assert L.dtn_points_num_nodes(None) == -1


@pytest.mark.parametrize("layout", [(16, 32, 4, 16), (8, 16, 4, 8)])
def test_second_kind_tables_agree_with_oracle(layout):
    """The library's second-kind tables of a flat class (Gamma operator with
    dP/dn_x, and the constant term of the regularised S rule) against the
    oracle's independent functions."""
    from oracle import patch as OP
    from oracle import second_kind as SK
    from paper_1210_1491_amd import dtn
    nt, nf, nr, ns = layout
    t = dtn.class_second_kind(nt, nf, nr, ns)
    Q2 = SK.gamma_operator_2(1.0, nt, nf, nr, ns)
    assert np.max(np.abs(t["Q2"] - Q2)) < 1e-10 * np.max(np.abs(Q2))
    _, X, _, _ = OP.panels(1.0, None, nr, ns)
    for i in range(len(X)):
        pts, W = SK.s_rule(X[i], 1.0, 1e-6)
        wsum = np.sum(W * SK.kernel_s(X[i][None, :], pts, 1.0))
        assert abs(t["c2"][i] - (Q2[i].sum() - wsum)) < 1e-9 * max(1.0, abs(wsum))


def test_geometry_step_cap_is_checked_on_the_host():
    """A walk's step count is 32-bit: caps above 2^32 - 1 (e.g. INT64_MAX for
    'no cap') are refused before any device work, so the kernels' iteration
    bound can never be computed from a cap they do not honour."""
    from paper_1210_1491_amd import dtn
    L = dtn.lib()
    for cap in (2 ** 32, 2 ** 63 - 1, -1):
        d = dtn.GeometryDesc()
        d.kind, d.data_kind = 0, 0
        d.ball_r, d.eps, d.max_steps = 1.0, 1e-4, cap
        h = ctypes.c_void_p()
        assert L.dtn_create_geometry(ctypes.byref(d), ctypes.byref(h)) == -1, cap
        assert "max_steps" in L.dtn_last_error().decode()
        assert not h.value


def test_status_entry_points_check_their_arguments_on_the_host():
    from paper_1210_1491_amd import dtn
    L = dtn.lib()
    assert L.dtn_check(None, None) == -1
    assert L.dtn_plan_set_max_sweeps(None, 4) == -1
    assert L.dtn_walk_counters(None, None, 0, None) == -1
    assert "NULL" in L.dtn_last_error().decode()


def _lu32(K):
    """FP32 LU with partial pivoting (row swaps), as a plain loop."""
    A = K.astype(np.float32).copy()
    piv = []
    for k in range(A.shape[0]):
        p = k + int(np.argmax(np.abs(A[k:, k])))
        piv.append(p)
        A[[k, p]] = A[[p, k]]
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:]).astype(np.float32)
    return A, piv


def _solve32(A, piv, r):
    f = r.astype(np.float32)
    for k, p in enumerate(piv):
        f[[k, p]] = f[[p, k]]
    n = len(f)
    for i in range(n):
        f[i] -= np.float32(np.dot(A[i, :i], f[:i]))
    for i in range(n - 1, -1, -1):
        f[i] = (f[i] - np.float32(np.dot(A[i, i + 1:], f[i + 1:]))) / A[i, i]
    return f.astype(np.float64)


@pytest.mark.parametrize("layout", [(4, 8, 2, 4, 0.0), (8, 16, 4, 8, 0.0), (16, 32, 4, 16, 0.0),
                                    (16, 32, 8, 16, 0.0), (8, 16, 4, 8, 5.0)])
def test_refinement_bound_is_met_after_three_sweeps(layout):
    """The FP32-mixed solve stops once |r|_inf <= P 2^-53 (|K|_inf |y|_inf +
    |b|_inf).  With the library's own class matrices, FP32 factors and an
    FP64 residual, that bound is out of reach after one FP32 solve (so a
    limit of one sweep must report no convergence) and met, with margin,
    from the third on: the default limit of 8 sweeps is never the one that
    stops a supported layout."""
    from paper_1210_1491_amd import dtn
    K = dtn.class_operators(*layout[:4], rr=layout[4])["K"]
    P = K.shape[0]
    A, piv = _lu32(K)
    kinf = np.abs(K).sum(1).max()
    rng = np.random.default_rng(7)
    for _ in range(6):
        b = rng.standard_normal(P) * 10.0 ** rng.uniform(-3, 3)
        y, r, ratio = np.zeros(P), b.copy(), []
        for _ in range(4):
            y = y + _solve32(A, piv, r)
            r = b - K @ y
            ratio.append(np.abs(r).max() / (P * 2.0 ** -53 * (kinf * np.abs(y).max() + np.abs(b).max())))
        assert ratio[0] > 1e3
        assert ratio[2] < 0.5 and ratio[3] < 0.5, ratio


@pytest.mark.parametrize("layout", [(8, 16, 4, 8, 5.0), (16, 32, 4, 16, -3.0)])
def test_curved_second_kind_tables_agree_with_oracle(layout):
    """The library's second-kind tables of a class on a sphere (Gamma
    operator with -d2G_B/dn_x dn_y, 1/2 I - D, and the regularised S rule's
    constant term) against the oracle's independent functions."""
    from oracle import patch as OP
    from oracle import second_kind as SK
    from paper_1210_1491_amd import dtn
    nt, nf, nr, ns, rr = layout
    t = dtn.class_second_kind(nt, nf, nr, ns, rr)
    Q2 = SK.gamma_operator_2c(1.0, rr, nt, nf, nr, ns)
    M = 0.5 * np.eye(nr * ns) - SK.adjoint_double_layer(1.0, rr, nr, ns)
    assert np.max(np.abs(t["Q2"] - Q2)) < 1e-10 * np.max(np.abs(Q2))
    assert np.max(np.abs(t["M"] - M)) < 1e-10
    _, X, N, _ = OP.panels(1.0, rr, nr, ns)
    for i in (0, len(X) // 2, len(X) - 1):
        pts, nrm, W = SK.s_rule_c(X[i], 1.0, rr, 1e-6)
        wsum = np.sum(W * SK.d2green(X[i][None, :], N[i][None, :], pts, nrm, 1.0))
        assert abs(t["c2"][i] - (Q2[i].sum() - wsum)) < 1e-9 * max(1.0, abs(wsum))


def test_binding_refuses_a_library_built_against_another_header(tmp_path, monkeypatch):
    """The library's version string carries the digest of the header it was
    built against; the binding loads it only when that matches the header
    beside the package (a stale library called with a newer header's
    argument lists would read its arguments wrongly)."""
    from paper_1210_1491_amd import build, dtn
    assert dtn.version().endswith(" dtn.h " + build.header_digest())
    other = tmp_path / "dtn.h"
    other.write_bytes(open(build.HEADER, "rb").read() + b"\n/* changed */\n")
    monkeypatch.setattr(build, "HEADER", str(other))
    monkeypatch.setattr(dtn, "_lib", None)
    with pytest.raises(ImportError, match="another include/dtn.h"):
        dtn.lib()
