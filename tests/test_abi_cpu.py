"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/h2.h, and its host-side tree and block lists are bit-exact
with the oracle (integer work: exact equality)."""
import os
import re

import numpy as np
import pytest

import seeded_inputs as si
from oracle.tree import Tree as OTree
from tests.h2_helpers import ROOT

h2 = pytest.importorskip("paper_2003_10173_amd")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "h2.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(h2_[a-z0-9_]+)\s*\(", text))
    return sorted(n for n in names if not n.endswith("_fn"))


def test_library_exports_every_declared_symbol():
    L = h2.lib()
    names = declared_functions()
    assert len(names) > 20
    missing = [n for n in names if not L.has(n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2003_10173_amd._lib import SIGNATURES
    assert set(declared_functions()) <= set(SIGNATURES)


CASES = [
    ("kernel1d", lambda: si.points_1d_cell_centres(1024), 32),
    ("diffusion2d", lambda: si.points_grid_interior(64), 64),
    ("cells64", lambda: si.points_grid_cell_centres(64, 64), 64),
    ("advdiff128", lambda: si.points_grid_interior(128), 64),
    ("random2d", lambda: np.random.Generator(np.random.PCG64(9)).uniform(size=(3001, 2)), 40),
    ("random3d", lambda: np.random.Generator(np.random.PCG64(4)).uniform(size=(2000, 3)), 32),
    ("ragged1d", lambda: np.random.Generator(np.random.PCG64(1)).uniform(size=1000), 17),
    ("tiny", lambda: np.array([0.3, 0.1, 0.2]), 8),
    ("batch_member", lambda: si.batch_problem(7)["points"], 64),
]


@pytest.mark.parametrize("name,pts_fn,leaf", CASES, ids=[c[0] for c in CASES])
def test_tree_and_lists_bit_exact(name, pts_fn, leaf):
    pts = pts_fn()
    ot = OTree(pts, leaf, 0.7)
    gt = h2.Tree(pts, leaf, 0.7)
    assert gt.L == ot.L
    assert np.array_equal(gt.perm, ot.perm)
    for l in range(ot.L + 1):
        assert np.array_equal(gt.offsets(l), ot.offsets[l])
        want = np.array(ot.far[l], dtype=np.int32).reshape(-1, 2)
        assert np.array_equal(gt.pairs(l), want)
    assert np.array_equal(gt.pairs(-1), np.array(ot.near, dtype=np.int32).reshape(-1, 2))


def test_tree_rejects_bad_arguments():
    with pytest.raises(h2.H2Error):
        h2.Tree(np.array([[np.nan, 0.0]]), 8)
    with pytest.raises(h2.H2Error):
        h2.Tree(np.zeros((10, 2)), 0)
    with pytest.raises(h2.H2Error):
        h2.Tree(np.zeros((10, 4)), 8)
