"""Pins of the multiresolution oracle (Sec. 2.4: projection and 5th-order
prediction of cell averages, level-dependent thresholding of the details,
and the block structure with the interface position identifier).

* projection conserves the mean;
* the prediction reproduces the cell averages of every polynomial of degree
  <= 4 in x and y (tensor products) away from the edges, fails for degree 5
  with details that fall by 2^5 when the grid is halved, and keeps
  constants exactly up to the edges; the sign convention is pinned by the
  linear data (a flipped sign leaves details of h/2);
* the thresholds scale by 1/4 per coarser level;
* the tree (safety zone, grading, existence, leaves, counts) on a case
  derived by hand;
* interface identifiers refine to the finest level.
"""
import numpy as np
import pytest

from oracle import mr


def cell_avg_poly(n, a, b, L=1.0):
    """Exact averages of x^a y^b over the n x n cells of [0, L]^2."""
    e = np.linspace(0.0, L, n + 1)
    ax = (e[1:] ** (a + 1) - e[:-1] ** (a + 1)) / ((a + 1) * (e[1:] - e[:-1]))
    ay = (e[1:] ** (b + 1) - e[:-1] ** (b + 1)) / ((b + 1) * (e[1:] - e[:-1]))
    return np.outer(ay, ax)


def test_projection_conserves_the_mean():
    u = np.random.default_rng(1).random((64, 128))
    c = mr.project(u)
    assert c.shape == (32, 64)
    assert abs(c.mean() - u.mean()) <= 1e-15
    assert c[3, 5] == 0.25 * ((u[6, 10] + u[6, 11]) + (u[7, 10] + u[7, 11]))


@pytest.mark.parametrize("a,b", [(a, b) for a in range(5) for b in range(5)])
def test_prediction_exact_for_degree_four(a, b):
    fine = cell_avg_poly(64, a, b)
    coarse = cell_avg_poly(32, a, b)
    d = fine - mr.predict(coarse)
    inner = d[4:-4, 4:-4]  # two coarse cells from every edge
    assert np.abs(inner).max() <= 1e-14 * max(1.0, np.abs(fine).max()), (a, b)


@pytest.mark.parametrize("a,b", [(5, 0), (0, 5)])
def test_prediction_fifth_order(a, b):
    errs = []
    for n in (32, 64):
        d = cell_avg_poly(2 * n, a, b) - mr.predict(cell_avg_poly(n, a, b))
        errs.append(np.abs(d[4:-4, 4:-4]).max())
    assert errs[0] > 1e-9
    ratio = errs[0] / errs[1]
    assert 30.0 < ratio < 34.0, ratio


def test_constants_and_sign_convention():
    c = np.full((16, 16), 2.5)
    assert np.array_equal(mr.predict(c), np.full((32, 32), 2.5))
    # linear data: the left child of a coarse cell of width h has mean
    # u - h/4; a flipped sign would predict u + h/4 there
    x = cell_avg_poly(32, 1, 0)
    p = mr.predict(x)
    h = 1.0 / 32
    assert abs(p[10, 10] - (x[5, 5] - h / 4)) <= 1e-15
    assert abs(p[10, 11] - (x[5, 5] + h / 4)) <= 1e-15


def test_thresholds_per_level():
    """One detail of known size at each level: flagged against eps at the
    finest level and eps/4 one level up."""
    L, B = 2, 4
    n = B << L  # 16 x 16 solver cells
    u = np.full((n, n), 1.0)
    # a bump in one fine cell: its detail at level L is 3/4 of it; the
    # level-(L-1) detail of its parent is smaller by the averaging
    for bump, want in ((0.9e-3 / 0.75, False), (1.1e-3 / 0.75, True)):
        v = u.copy()
        v[5, 6] += bump
        Q = np.zeros((1, 4, n, n))
        Q[0, 0] = v
        Q[0, 3] = 1.0
        r = mr.analyse(Q, np.full((n, n), 1.0), 0.5, B=B, L=L, eps=1e-3)
        assert bool(r["detail"][L - 1].any()) == want, bump
    lev = mr.pyramid(np.arange(64.0).reshape(8, 8) ** 2, 2)
    assert [x.shape for x in lev] == [(2, 2), (4, 4), (8, 8)]


def test_tree_by_hand():
    """L = 2, 3 x 3 blocks at level 0: one block with significant details at
    level 1 in the top-right corner (row 0, column 5).  Safety zone: level-1
    blocks (0..1, 4..5); grading: their 3 x 3 neighbourhood (rows 0..2,
    columns 3..5) needs its parents, level-0 blocks (0..1, 1..2), refined.
    Leaves: level 2 at level-2 rows 0..3, columns 8..11; level 1 in the rest
    of level-2 rows 0..7, columns 4..11; level 0 elsewhere."""
    d0 = np.zeros((3, 3), bool)
    d1 = np.zeros((6, 6), bool)
    d1[0, 5] = True
    iface = [np.zeros((3, 3), bool), np.zeros((6, 6), bool), np.zeros((12, 12), bool)]
    r = mr.build_tree([d0, d1], iface, 2, B=8)
    want = np.zeros((12, 12), np.int32)
    want[0:8, 4:12] = 1
    want[0:4, 8:12] = 2
    assert np.array_equal(r["leaf"], want)
    assert r["counts"] == [(9, 5), (16, 12), (16, 16)]
    assert r["compression"] == pytest.approx(33 / 144, abs=0)


def test_interface_blocks_reach_the_finest_level():
    L, B = 3, 4
    n = 4 * (B << L)  # 128 x 128: 4 x 4 blocks at level 0
    Q = np.zeros((2, 4, n, n))
    Q[:, 0] = 1.0
    Q[:, 3] = 2.5
    phi = np.full((n, n), 1.0)
    phi[17, 9] = 0.0  # one cell of the band, in solver block (4, 2)
    r = mr.analyse(Q, phi, 0.5, B=B, L=L)
    assert not any(d.any() for d in r["detail"])  # a uniform state
    assert r["leaf"][4, 2] == L
    assert r["iface"][0][0, 0] and r["iface"][1][1, 0] and r["iface"][2][2, 1]
    assert r["iface"][0].sum() == 1 and r["iface"][3].sum() == 1
    # the safety zone and grading keep levels of neighbouring leaves within one
    leaf = r["leaf"]
    assert np.abs(np.diff(leaf, axis=0)).max() <= 1 and np.abs(np.diff(leaf, axis=1)).max() <= 1
    # far from the interface the coarsest level suffices
    assert leaf[31, 31] == 0 and leaf[0, 31] == 0 and leaf[31, 0] == 0
