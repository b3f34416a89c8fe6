"""Pins for the oracle's cluster tree, block tree and partition validator
(Def. 2.1, Def. 2.2; geometric bisection and eta = 2 admissibility)."""
import numpy as np
import pytest

from oracle import trees
from synth import sphere_points


def line_points(xs):
    p = np.zeros((len(xs), 3))
    p[:, 0] = xs
    return p


def test_hand_built_line_tree():
    # x = [5,2,7,0,3,6,1,4]: root box [0,7] splits at 3.5, then at 1.5 / 5.5.
    st = trees.build_structure(line_points([5, 2, 7, 0, 3, 6, 1, 4]), leaf_size=2)
    assert st.perm.tolist() == [3, 6, 1, 4, 0, 7, 2, 5]
    assert st.nnodes == 7
    assert st.level.tolist() == [0, 1, 2, 2, 1, 2, 2]
    leaves = [(int(st.begin[v]), int(st.end[v])) for v in st.leaves()]
    assert leaves == [(0, 2), (2, 4), (4, 6), (6, 8)]
    # level-1 boxes [0,3] and [4,7]: diam 3 > 2 * dist 1 -> not admissible.
    # level-2 leaf pairs: admissible iff distinct (diam 1 <= 2 * dist >= 2).
    blocks = sorted(zip(st.blk_tau.tolist(), st.blk_sigma.tolist(), st.blk_adm.tolist()))
    lv2 = [v for v in range(7) if st.level[v] == 2]
    expect = sorted((t, s, t != s) for t in lv2 for s in lv2)
    assert blocks == expect
    trees.validate_partition(st, leaf_size=2)


def test_single_leaf_and_first_split():
    st = trees.build_structure(sphere_points(64, 5))
    assert st.nnodes == 1 and st.nblocks == 1 and not st.blk_adm[0]
    st = trees.build_structure(sphere_points(65, 5))
    assert st.nnodes == 3
    trees.validate_partition(st)


def test_identical_points_split_at_half():
    st = trees.build_structure(np.ones((130, 3)), leaf_size=64)
    assert st.perm.tolist() == list(range(130))
    sizes = sorted(int(st.end[v] - st.begin[v]) for v in st.leaves())
    assert sizes == [32, 32, 33, 33]
    assert not st.blk_adm.any()          # zero distance: never admissible
    trees.validate_partition(st)


def test_collinear_and_clustered_points():
    rng = np.random.default_rng(7)
    p = np.concatenate([line_points(rng.uniform(0, 1, 300)),
                        rng.normal(size=(200, 3)) * 1e-3 + 5.0,
                        np.tile([[2.0, 2.0, 2.0]], (70, 1))])
    st = trees.build_structure(p, leaf_size=16)
    trees.validate_partition(st, leaf_size=16)
    assert (trees.coverage_bitmap(st) == 1).all()


@pytest.mark.parametrize("n", [100, 777, 2048])
def test_exact_cover_bitmap(n):
    st = trees.build_structure(sphere_points(n, 1000 + n))
    trees.validate_partition(st)
    cnt = trees.coverage_bitmap(st)
    assert cnt.min() == 1 and cnt.max() == 1


def test_admissibility_hand_values():
    lo_t, hi_t = np.array([0.0, 0, 0]), np.array([1.0, 1, 0])     # diam^2 = 2
    lo_s, hi_s = np.array([2.0, 0, 0]), np.array([3.0, 1, 0])     # dist^2 = 1
    # min diam^2 = 2 <= 4 * 1
    assert trees.admissible(lo_t, hi_t, lo_s, hi_s)
    lo_s, hi_s = np.array([1.5, 0, 0]), np.array([2.5, 4, 0])     # dist^2 = .25
    assert not trees.admissible(lo_t, hi_t, lo_s, hi_s)           # 2 > 1
    # touching boxes: dist 0 is never admissible, even for points (diam 0)
    z = np.zeros(3)
    assert not trees.admissible(z, z, z, z)
    assert trees.admissible(z, z, np.array([1.0, 0, 0]), np.array([1.0, 0, 0]))


def test_validator_catches_planted_errors():
    st = trees.build_structure(sphere_points(700, 3))
    trees.validate_partition(st)
    # drop a block -> gap
    bad = trees.build_structure(sphere_points(700, 3))
    bad.blk_tau = bad.blk_tau[1:]; bad.blk_sigma = bad.blk_sigma[1:]; bad.blk_adm = bad.blk_adm[1:]
    with pytest.raises(AssertionError):
        trees.validate_partition(bad)
    # duplicate a block -> overlap
    bad = trees.build_structure(sphere_points(700, 3))
    bad.blk_tau = np.append(bad.blk_tau, bad.blk_tau[0])
    bad.blk_sigma = np.append(bad.blk_sigma, bad.blk_sigma[0])
    bad.blk_adm = np.append(bad.blk_adm, bad.blk_adm[0])
    with pytest.raises(AssertionError):
        trees.validate_partition(bad)
