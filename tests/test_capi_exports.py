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
    for n in names:
        assert hasattr(lib, n), n
    assert "gfx950" in dtn.version()


@pytest.mark.parametrize("layout", [(16, 32, 4, 16, 0.0), (8, 16, 4, 8, 5.0), (6, 12, 2, 8, 0.0)])
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


def test_host_operator_arguments_are_checked():
    from paper_1210_1491_amd import dtn
    with pytest.raises(dtn.DtnError):
        dtn.class_operators(1, 16, 4, 8)
    with pytest.raises(dtn.DtnError):
        dtn.class_operators(8, 15, 4, 8)
