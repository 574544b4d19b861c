"""Autotuner bucketing (CPU only): width class of the largest out-degree
and band of k; every pair lands in exactly one bucket."""
from paper_2502_00317_amd import autotune as at


def test_width_class_matches_the_library_classes():
    assert [at.width_class(d) for d in (0, 1, 64, 65, 128, 129, 320, 321, 384, 385, 512, 513, 1024)] == \
        [1, 1, 1, 2, 2, 3, 5, 6, 6, 8, 8, 16, 16]


def test_k_bands_cover_every_k_once():
    seen = [at.k_band(k) for k in range(1, 65)]
    assert seen[0] == 0 and seen[-1] == len(at.K_BANDS) - 1
    assert all(a <= b for a, b in zip(seen, seen[1:]))
    for i, (lo, hi) in enumerate(at.K_BANDS):
        assert all(at.k_band(k) == i for k in range(lo, hi + 1))


def test_bucket_pairs_partition():
    degs = [10, 100, 10, 300, 70, 10]
    ks = [3, 7, 12, 13, 8, 4]
    b = at.bucket_pairs(degs, ks)
    assert sorted(i for idx in b.values() for i in idx) == list(range(len(ks)))
    assert b["w1/k1-5"] == [0, 5] and b["w2/k6-8"] == [1, 4] and b["w1/k9-12"] == [2]
    assert b["w5/k13-64"] == [3]
