"""The library's treecode tree (built on the host) against the oracle's
independent tree: integer work, so exactly equal — node order (depth-first
pre-order), source ranges (their order within leaves), subtree ends, leaf flags, proxy
degrees and which clusters carry proxies.  No GPU needed."""
import numpy as np
import pytest

import dtn_inputs as I
from oracle import patch as P
from oracle import treecode as T
from oracle import wos


def _preorder(C, out):
    out.append(C)
    for ch in C.children:
        _preorder(ch, out)
    return out


@pytest.mark.parametrize("degree,leaf", [(6, 64), (3, 8), (8, 300), (1, 4096)])
@pytest.mark.parametrize("tiles", ["cube", "box_holes_outer", "subset"])
def test_tree_layout_equals_oracle(degree, leaf, tiles):
    from paper_1210_1491_amd import dtn
    if tiles == "cube":
        gd, pd = I.geometry_cube_sources(), I.patches_cube_tiles()
    elif tiles == "subset":
        gd = I.geometry_cube_sources()
        pd = I.subset_patches(I.patches_cube_tiles(), list(range(5, 1536, 7)))
    else:
        gd = I.geometry_cube_sources()
        pd = I.subset_patches(I.patches_cube_tiles(), list(range(0, 1536, 3)))
    nodes, perm = dtn.tree_layout(pd, degree, leaf)
    ps = P.patches_from_desc(pd, gd)
    y, _, _ = T.tile_sources(ps, [np.zeros(p.n_rings * p.n_sectors) for p in ps], wos.Geometry(gd))
    pre = _preorder(T.build_tree(y, T.tile_faces(ps), leaf, degree), [])
    assert len(pre) == len(nodes)
    pos = {id(C): j for j, C in enumerate(pre)}

    def subtree_end(C):
        while C.children:
            C = C.children[-1]
        return pos[id(C)] + 1

    for j, C in enumerate(pre):
        b, e, skip, is_leaf, d0, d1, d2, proxy = nodes[j]
        if C.children:  # the children's ranges in order; the oracle keeps input order here
            np.testing.assert_array_equal(np.sort(perm[b:e]), np.sort(C.idx))
        else:
            np.testing.assert_array_equal(perm[b:e], C.idx)
        assert skip == subtree_end(C) and skip > j
        assert bool(is_leaf) == (not C.children)
        assert [d0, d1, d2] == C.deg
        assert (proxy >= 0) == C.has_proxy


def test_tree_layout_arguments_are_checked():
    from paper_1210_1491_amd import dtn
    pd = I.subset_patches(I.patches_cube_tiles(), [0, 1, 2])
    for deg, leaf in ((0, 64), (9, 64), (6, 7), (6, 5000)):
        with pytest.raises(dtn.DtnError):
            dtn.tree_layout(pd, deg, leaf)
