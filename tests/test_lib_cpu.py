"""Host-side checks of the HIP library (no GPU needed): it loads, exports every function
include/fmmlu.h declares, builds the same octree as the oracle (bit-exact integer work),
and rejects invalid input with the documented status codes."""
import numpy as np
import pytest

import synth
import paper_2201_07325_amd as fm
from oracle.tree import Tree as OracleTree


def test_library_exports_every_declared_symbol():
    L = fm.lib()
    names = fm.header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name


def test_trim_caches_with_nothing_cached():
    # no factorization has run in this process: nothing to free, no device call needed
    fm.trim_caches()
    fm.trim_caches()


def _compare_trees(points, leaf):
    ot = OracleTree(points, leaf)
    gt = fm.Tree(points, leaf).export()
    rows = sorted((int(l), *map(int, c), int(p), int(f)) for l, c, p, f in
                  zip(gt["level"], gt["coord"], gt["npts"], gt["is_leaf"]))
    assert rows == ot.summary()
    assert gt["nlevels"] == ot.nlevels
    assert np.array_equal(gt["order"], ot.order)


@pytest.mark.parametrize("leaf", [16, 64])
def test_tree_matches_oracle_sphere(leaf):
    _compare_trees(synth.unit_sphere(3000).points, leaf)


def test_tree_matches_oracle_graded():
    _compare_trees(synth.graded_ellipsoid(6000, seed=2).points, 16)


def test_tree_matches_oracle_single_box_and_tiny():
    _compare_trees(synth.unit_sphere(10).points, 64)
    _compare_trees(synth.unit_sphere(1).points, 1)


def test_invalid_inputs():
    pts = synth.unit_sphere(100).points.copy()
    with pytest.raises(fm.FmmluError) as e:
        fm.Tree(pts[:, :0], 16)
    assert e.value.code == "EINVAL"
    bad = pts.copy()
    bad[0, 5] = np.nan
    with pytest.raises(fm.FmmluError) as e:
        fm.Tree(bad, 16)
    assert e.value.code == "EINVAL"
    dup = pts.copy()
    dup[:, 7] = dup[:, 3]
    with pytest.raises(fm.FmmluError) as e:
        fm.Tree(dup, 16)
    assert "duplicate" in str(e.value)
    with pytest.raises(fm.FmmluError):
        fm.Tree(pts, 0)
