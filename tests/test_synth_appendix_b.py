"""Structure of the second synthetic workload's inputs (the paper's simplified spherical-wave and
seismic settings): speeds within U[1, 2], one constant speed for gamma-constant, four aligned
layers (each row constant; four distinct values; boundaries inside the central band) and a
fault (the layers shifted by one offset to the right of one column), m entries of +-1 away from
the PML, and reproducibility by seed."""
import numpy as np
import pytest

from synth import APPB_KINDS, C_REF, appendix_b_system, layered_velocity, m_dirac_source, rng_for


@pytest.mark.parametrize("kind", APPB_KINDS)
def test_speeds_in_range_and_reproducible(kind):
    s = appendix_b_system(kind, 3, nx=96, npml=12)
    assert s.c.shape == (120, 120) and s.b.shape == (120, 120)
    v = s.c / C_REF
    assert v.min() >= 1.0 and v.max() <= 2.0
    t = appendix_b_system(kind, 3, nx=96, npml=12)
    assert np.array_equal(s.c, t.c) and np.array_equal(s.b, t.b)
    assert not np.array_equal(s.c, appendix_b_system(kind, 4, nx=96, npml=12).c)


def test_gamma_constant_and_m_dirac():
    for kind, m in (("gamma_dirac", 1), ("gamma_2dirac", 2)):
        s = appendix_b_system(kind, 1, nx=64, npml=8)
        assert np.unique(s.c).size == 1
        nz = np.argwhere(s.b != 0)
        assert len(nz) == m and set(np.unique(s.b[s.b != 0]).real) <= {-1.0, 1.0}
        assert np.all(s.b.imag == 0)
        assert nz.min() >= 8 + 4 and nz.max() <= 80 - 1 - 8 - 4
    b = m_dirac_source(60, 6, rng_for(8, 9, 0), 25)
    assert np.count_nonzero(b) == 25


def test_layered_structure():
    nt = 128
    c = layered_velocity(nt, rng_for(8, 9, 1), layers=4)
    assert np.all(c == c[:, :1])                      # aligned: each row is constant
    vals, first = np.unique(c[:, 0], return_index=True)
    assert vals.size == 4
    change = np.flatnonzero(np.diff(c[:, 0]) != 0) + 1
    assert change.size == 3 and change.min() >= nt // 8 and change.max() < nt - nt // 8
    assert np.all(np.diff(np.concatenate([[0], change, [nt]])) >= nt // 16)


def test_faulted_structure():
    nt = 128
    c = layered_velocity(nt, rng_for(8, 9, 2), layers=4, faulted=True)
    cols = [tuple(c[:, i]) for i in range(nt)]
    kinds = sorted(set(cols), key=cols.index)
    assert len(kinds) == 2                            # one column profile each side of the fault
    xf = cols.index(kinds[1])
    assert nt // 4 <= xf <= 3 * nt // 4
    left, right = np.array(kinds[0]), np.array(kinds[1])
    cl = np.flatnonzero(np.diff(left) != 0) + 1
    cr = np.flatnonzero(np.diff(right) != 0) + 1
    shift = cr[: len(cl)] - cl[: len(cr)]
    assert shift.size > 0 and np.all(shift == shift[0]) and nt // 16 <= shift[0] <= nt // 8
    assert np.array_equal(np.unique(left), np.unique(right)) or set(np.unique(right)) <= set(np.unique(left))
