"""Pins of the oracle's neighbour reshuffling (product-kernel test, Sect. 3.3):
the relabelling is a bijection of the active slots for any N, changes with the
refresh and the seed, spreads over [0, N), and leaves slot 0 (the particle
itself) and the unused tail of every row alone.  The particular bijection is
this build's reading (a Feistel network with Philox rounds, cycle-walked to
[0, N)); beyond these properties it is parity unpinned."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("N", [1, 2, 3, 7, 64, 1000, 4099, 65539])
def test_bijection(N):
    im = np.array([oracle.reshuffle_index(N, 11, 2, j) for j in range(N)])
    assert np.array_equal(np.sort(im), np.arange(N))


def test_refresh_and_seed_change_it():
    N = 1000
    a = [oracle.reshuffle_index(N, 11, 2, j) for j in range(64)]
    assert a == [oracle.reshuffle_index(N, 11, 2, j) for j in range(64)]  # deterministic
    assert a != [oracle.reshuffle_index(N, 11, 3, j) for j in range(64)]
    assert a != [oracle.reshuffle_index(N, 12, 2, j) for j in range(64)]
    assert sum(x == j for j, x in enumerate(a)) < 5  # few fixed points


def test_spread():
    # the image of one slot over 2000 refreshes: roughly uniform over [0, N)
    N = 1000
    im = np.array([oracle.reshuffle_index(N, 5, r, 0) for r in range(2000)])
    h = np.histogram(im, bins=10, range=(0, N))[0]
    chi2 = ((h - 200.0) ** 2 / 200.0).sum()
    assert chi2 < 30.0  # 9 degrees of freedom; p < 1e-3 above ~27.9


def test_rows():
    rng = np.random.default_rng(3)
    n, k, N = 50, 8, 40
    nbr = rng.integers(0, N, (n, k)).astype(np.int32)
    nbr[:, 0] = np.arange(n) % N
    cnt = rng.integers(0, k + 1, n).astype(np.int32)
    out = oracle.reshuffle(nbr, cnt, N, 9, 1)
    for i in range(n):
        assert out[i, 0] == nbr[i, 0]
        assert np.array_equal(out[i, max(cnt[i], 1):], nbr[i, max(cnt[i], 1):])
        for s in range(1, cnt[i]):
            v = oracle.reshuffle_index(N, 9, 1, int(nbr[i, s]))
            if v == i:
                v = oracle.reshuffle_index(N, 9, 1, i)
            assert out[i, s] == v
    # rows stay free of repeats among the relabelled entries (pi is injective)
    row = np.arange(1, 30, dtype=np.int32)
    nb2 = np.concatenate([[0], row]).astype(np.int32)[None, :]
    o2 = oracle.reshuffle(nb2, np.array([30], np.int32), N, 9, 4)
    assert len(set(o2[0, 1:].tolist())) == 29


def test_rows_stay_distinct_and_free_of_self():
    # real neighbour rows (distinct others, none equal to the row's particle):
    # after relabelling they are still distinct and still exclude the particle,
    # which pi sends onto itself from exactly one slot; that slot takes pi(i)
    import workloads
    N = 2000
    params, st = workloads.by_name("const_box", seed=4, n=N)
    P = oracle.make_problem(params)
    nbr, cnt, _ = oracle.knn(P, st["x"], st["y"], st["z"], st["M"])
    hit = 0
    for refresh in range(3):
        out = oracle.reshuffle(nbr, cnt, N, 17, refresh)
        for i in range(N):
            others = out[i, 1:cnt[i]]
            assert out[i, 0] == i
            assert i not in others
            assert len(set(others.tolist())) == cnt[i] - 1
            pi_row = [oracle.reshuffle_index(N, 17, refresh, int(j)) for j in nbr[i, 1:cnt[i]]]
            if i in pi_row:
                hit += 1
                assert oracle.reshuffle_index(N, 17, refresh, i) in others
    # rows where pi sends an other onto i occur about (k - 1)/N of the time
    assert 20 < hit < 200
