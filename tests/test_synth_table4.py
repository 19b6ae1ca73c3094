"""The six training data sets of Section 3.2 (Table 4): the class mixture of each set is drawn with
Table 4's probabilities, and every class has the structure the text gives it."""
import numpy as np
import pytest

from synth import (C_REF, TABLE4, rng_for, table4_classes, table4_sample, table4_set)

EXPECTED = {   # Table 4: (source classes, probabilities), (velocity classes, probabilities)
    "D0": ({"normal": 0.6, "dirac": 0.3, "dirac1": 0.05, "dirac4": 0.05}, {"uniform": 0.5, "skull": 0.5}),
    "D1": ({"normal": 1.0}, {"uniform": 0.5, "skull": 0.5}),
    "D2": ({"normal": 0.6, "dirac": 0.3, "dirac1": 0.05, "dirac4": 0.05},
           {"uniform": 0.4, "skull": 0.4, "rand_constant": 0.1, "square": 0.1}),
    "D3": ({"normal": 1.0}, {"uniform": 0.4, "skull": 0.4, "rand_constant": 0.1, "square": 0.1}),
    "D4": ({"normal": 1.0}, {"skull": 1.0}),
    "D5": ({"normal": 1.0}, {"uniform": 1.0}),
}


@pytest.mark.parametrize("ds", sorted(EXPECTED))
def test_class_frequencies_follow_table4(ds):
    n = 20000
    rng = rng_for(99, int(ds[1]), 0)
    draws = [table4_classes(ds, rng) for _ in range(n)]
    for which, expect in enumerate(EXPECTED[ds]):
        counts = {}
        for d in draws:
            counts[d[which]] = counts.get(d[which], 0) + 1
        assert set(counts) == set(expect), (ds, counts)
        for k, p in expect.items():
            sd = np.sqrt(p * (1 - p) / n)
            assert abs(counts[k] / n - p) <= 5 * sd + 1e-12, (ds, k, counts[k] / n, p)
    # the table itself is the paper's
    assert {k: dict(zip(*v)) for k, v in zip(("b", "c"), TABLE4[ds])} == {"b": EXPECTED[ds][0], "c": EXPECTED[ds][1]}


def test_class_structure():
    nt, p = 48, 8
    seen = set()
    for i in range(400):
        rng = rng_for(98, 2, i)
        kinds = table4_classes("D2", rng_for(98, 2, i))
        c, b = table4_sample("D2", nt, p, rng)
        assert c.shape == (nt, nt) and b.shape == (nt, nt) and b.dtype == np.complex128
        bk, ck = kinds
        seen.add(kinds)
        cn = c / C_REF
        if ck == "uniform":
            assert cn.min() >= 1.0 and cn.max() <= 2.0 and np.unique(cn).size > nt   # i.i.d. entries
        elif ck == "rand_constant":
            assert np.unique(cn).size == 1 and 1.0 <= cn[0, 0] <= 2.0
        elif ck == "square":
            assert set(np.unique(cn)) == {1.0, 2.0} and cn[nt // 2, nt // 2] == 2.0 and cn[0, 0] == 1.0
        else:   # skull rings on a water background with 5 % noise
            assert 0.7 < np.median(cn) < 1.3 and cn.max() > 1.4
        nz = np.flatnonzero(b)
        if bk == "normal":
            assert nz.size == nt * nt and abs(np.std(b.real) - 1) < 0.15
        elif bk == "dirac":
            assert nz.size == 1 and b.flat[nz[0]] == 60.0
        elif bk == "dirac1":
            assert nz.size == 1 and b[nt // 2, nt // 2] == 60.0
        else:
            assert nz.size == 4 and np.all(b.flat[nz] == 30.0)
    assert len({k[0] for k in seen}) == 4 and len({k[1] for k in seen}) == 4


def test_sets_are_reproducible_and_disjoint():
    c1, b1 = table4_set("D0", 3, 24, 4)
    c2, b2 = table4_set("D0", 3, 24, 4)
    c3, b3 = table4_set("D0", 3, 24, 4, first=3)
    assert np.array_equal(c1, c2) and np.array_equal(b1, b2)
    assert not np.array_equal(b1, b3)
    c4, b4 = table4_set("D1", 3, 24, 4)
    assert not np.array_equal(b1, b4)
