"""Host logic of the batched form (no GPU): the ef-class split and order."""
import numpy as np

from paper_1804_09996_amd.batched import class_limits_options, class_permutation


def test_class_limits_options():
    assert class_limits_options(512, 100) == [[512], [128, 512], [128, 256, 512]]
    assert class_limits_options(300, 32) == [[320], [128, 320], [128, 256, 320]]
    assert class_limits_options(64, 32) == [[64]]
    assert class_limits_options(100, 200) == [[256]]  # no cut below the short-list


def test_class_permutation_orders_and_bounds():
    rs = np.random.default_rng(3)
    S = 40
    ef = rs.integers(1, 513, 5000)
    for limits in ([512], [128, 512], [128, 256, 512], [64, 128, 192, 256, 320, 512]):
        perm, ranges = class_permutation(ef, S, limits)
        assert np.array_equal(np.sort(perm), np.arange(ef.size))  # a permutation
        assert ranges[0][0] == 0 and ranges[-1][1] == ef.size
        for (r0, r1, top), nxt in zip(ranges, ranges[1:] + [None]):
            if nxt is not None:
                assert r1 == nxt[0]  # contiguous classes
            pools = np.maximum(ef[perm[r0:r1]], S)
            assert top == pools.max()  # the launch is sized for the class's largest pool
            assert np.all(np.diff(ef[perm[r0:r1]]) <= 0)  # longest ef first within a class
            lim = min(l for l in limits if l >= pools.max()) if pools.max() <= max(limits) else max(limits)
            assert np.all(pools <= lim)
        # classes ascend: every pool of a class is above the previous class's limit
        for (a0, a1, _), (b0, b1, _) in zip(ranges, ranges[1:]):
            assert np.maximum(ef[perm[a0:a1]], S).max() < np.maximum(ef[perm[b0:b1]], S).min()


def test_one_class_is_longest_first():
    ef = np.array([5, 300, 17, 300, 1, 64])
    perm, ranges = class_permutation(ef, 10, [512])
    assert list(perm) == [1, 3, 5, 2, 0, 4] and ranges == [(0, 6, 300)]
