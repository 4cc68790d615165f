"""Pins of the oracle's generator, Morton order and neighbour search.

Each check compares the oracle with something other than itself: published
known-answer vectors, an independently written decoder, scipy's KD-tree, and a
numpy full sort of all pair distances.
"""
import os

import numpy as np
import pytest
from scipy import spatial, stats

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox ----
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt")) if not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert list(oracle.philox4x32_10(v[:4], v[4:6])) == v[6:]


def test_uniforms_ranges_and_independence():
    u = np.array([oracle.uniforms(12345, i, 7, e) for i in range(300) for e in range(10)])
    assert (u[:, 0] > 0).all() and (u[:, 0] <= 1).all()
    assert (u[:, 1:] >= 0).all() and (u[:, 1:] < 1).all()
    for c in range(4):
        assert stats.kstest(u[:, c], "uniform").pvalue > 1e-4
    # the four streams are not correlated with each other
    cc = np.corrcoef(u.T)
    assert np.abs(cc - np.eye(4)).max() < 0.08
    # different seed / interval / event give different draws
    a = oracle.uniforms(1, 5, 0, 0)
    assert not np.array_equal(a, oracle.uniforms(2, 5, 0, 0))
    assert not np.array_equal(a, oracle.uniforms(1, 5, 1, 0))
    assert not np.array_equal(a, oracle.uniforms(1, 5, 0, 1))


# ---------------------------------------------------------------- Morton ----
def _decode(key):
    """Independent de-interleave: collect every third bit."""
    q = [0, 0, 0]
    for bit in range(30):
        q[bit % 3] |= ((key >> bit) & 1) << (bit // 3)
    return q


def test_morton_small_values():
    assert oracle.morton3_10(0, 0, 0) == 0
    assert oracle.morton3_10(1, 0, 0) == 1
    assert oracle.morton3_10(0, 1, 0) == 2
    assert oracle.morton3_10(0, 0, 1) == 4
    assert oracle.morton3_10(1, 1, 1) == 7
    assert oracle.morton3_10(2, 0, 0) == 8
    assert oracle.morton3_10(1023, 1023, 1023) == (1 << 30) - 1


def test_morton_roundtrip_and_cells():
    g = np.random.default_rng(1)
    for _ in range(500):
        q = [int(v) for v in g.integers(0, 1024, 3)]
        assert _decode(oracle.morton3_10(*q)) == q
    # every level-l cell is one contiguous key range: keys sharing the top 3l bits
    q = g.integers(0, 1024, (2000, 3))
    keys = np.array([oracle.morton3_10(*map(int, r)) for r in q], dtype=np.int64)
    for lev in (1, 3, 5):
        cell = q >> (10 - lev)
        prefix = keys >> (3 * (10 - lev))
        for c in np.unique(prefix):
            sel = prefix == c
            assert (cell[sel] == cell[sel][0]).all()


def test_morton_keys_quantisation_and_inactive():
    st = workloads.const_box(3, 500)
    M = st["M"].copy()
    M[::7] = 0.0
    keys = oracle.morton_keys(st["x"], st["y"], st["z"], M)
    assert (keys[M == 0] == 0xFFFFFFFF).all()
    act = M > 0
    q = np.array([_decode(int(k)) for k in keys[act]])
    pos = np.stack([st["x"][act], st["y"][act], st["z"][act]], 1)
    lo = pos.min(0)
    ext = (pos.max(0) - lo).max()
    expect = np.minimum(((pos - lo) * (1024.0 / ext)).astype(np.int64), 1023)
    assert (q == expect).all()
    perm = oracle.sort_perm(keys)
    assert (np.diff(keys[perm].astype(np.int64)) >= 0).all()


# ------------------------------------------------------------------- kNN ----
def _knn_by_full_sort(x, y, z, M, k, L=None, rmax=np.inf):
    """Reference: numpy distance matrix and a full lexicographic sort."""
    pos = np.stack([x, y, z], 1)
    n = len(x)
    d = pos[None, :, :] - pos[:, None, :]
    if L is not None:
        for a in range(3):
            if L[a]:
                da = d[:, :, a]
                da[da > 0.5 * L[a]] -= L[a]
                da[da < -0.5 * L[a]] += L[a]
    d2 = (d[:, :, 0] * d[:, :, 0] + d[:, :, 1] * d[:, :, 1]) + d[:, :, 2] * d[:, :, 2]
    out = []
    for i in range(n):
        if M[i] <= 0:
            out.append(None)
            continue
        j = np.arange(n)
        ok = (j != i) & (M > 0) & (d2[i] <= rmax * rmax)
        jj = j[ok]
        order = np.lexsort((jj, d2[i, ok]))
        sel = jj[order[: k - 1]]
        out.append((np.sort(sel), d2[i, sel].max() if len(sel) else 0.0))
    return out


@pytest.mark.parametrize("case", ["box", "column", "inactive", "rmax"])
def test_knn_matches_full_sort(case):
    k = 32
    if case in ("box", "inactive", "rmax"):
        st = workloads.const_box(11, 700)
        L = (1.0, 1.0, 1.0)
        per = (1, 1, 1)
    else:
        st = workloads.additive_col(11, 700)
        L = (1.0, 1.0, 0.0)
        per = (1, 1, 0)
    M = st["M"].copy()
    rmax = np.inf
    if case == "inactive":
        M[::5] = 0.0
    if case == "rmax":
        rmax = 0.13
    P = oracle.make_problem(dict(kernel="const", k=k, periodic=per, L=(1.0, 1.0, 1.0), rmax=rmax))
    nbr, cnt, dmax = oracle.knn(P, st["x"], st["y"], st["z"], M)
    ref = _knn_by_full_sort(st["x"], st["y"], st["z"], M, k, L=L, rmax=rmax)
    for i, r in enumerate(ref):
        if r is None:
            assert cnt[i] == 0 and (nbr[i] == -1).all()
            continue
        sel, d2max = r
        assert nbr[i, 0] == i
        assert cnt[i] == 1 + len(sel)
        assert np.array_equal(nbr[i, 1:cnt[i]], sel)
        assert (nbr[i, cnt[i]:] == -1).all()
        assert dmax[i] == np.sqrt(d2max)
    if case == "rmax":
        assert (cnt < k).any() and (dmax <= rmax).all()


def test_knn_distances_match_kdtree():
    st = workloads.const_box(5, 4096)
    P = oracle.make_problem(dict(kernel="const", k=32, periodic=(1, 1, 1), L=(1.0, 1.0, 1.0)))
    q = np.arange(0, 4096, 37)
    nbr, cnt, dmax = oracle.knn(P, st["x"], st["y"], st["z"], st["M"], queries=q)
    pos = np.stack([st["x"], st["y"], st["z"]], 1)
    tree = spatial.cKDTree(pos, boxsize=1.0)
    dd, _ = tree.query(pos[q], k=32)
    np.testing.assert_allclose(dmax, dd[:, -1], rtol=1e-12)
    assert (cnt == 32).all()


def test_knn_lattice_ties():
    # 8^3 lattice: the 31 nearest others cut through a shell of equal distances;
    # ties must go to the lower index.
    st = workloads.lattice_box(8)
    P = oracle.make_problem(dict(kernel="const", k=32, periodic=(1, 1, 1), L=(1.0, 1.0, 1.0)))
    nbr, cnt, dmax = oracle.knn(P, st["x"], st["y"], st["z"], st["M"])
    ref = _knn_by_full_sort(st["x"], st["y"], st["z"], st["M"], 32, L=(1.0, 1.0, 1.0))
    for i in range(len(ref)):
        assert np.array_equal(nbr[i, 1:], ref[i][0])
    # shells on a cubic lattice: 6 at a, 12 at sqrt2 a, 8 at sqrt3 a, 6 at 2a; the
    # 31st other is on the 2a shell, where 5 of the 6 equal-distance sites are kept
    a = 1.0 / 8
    np.testing.assert_array_equal(dmax, 2.0 * a)
