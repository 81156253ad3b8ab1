"""The host statement of the column-offset qualification rule (tests/offset_rule.py), pinned on hand-built
matrices whose qualifying slices are known by construction."""
import numpy as np
import scipy.sparse as sp

from offset_rule import expected_offset_slices


def _csr(Q):
    Q = sp.csr_matrix(Q)
    Q.sort_indices()
    return Q.indptr.astype(np.int32), Q.indices.astype(np.int32)


def _tridiag(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])


def test_tridiagonal_interior_slices_qualify():
    # offsets {-1, 0, 1}: the first slice would gather at row -1, the last at row n
    rp, ci = _csr(_tridiag(256))
    assert expected_offset_slices(rp, ci) == (2, 2 * 64 * 3)


def test_partial_last_slice_never_qualifies():
    rp, ci = _csr(_tridiag(256 + 10))
    assert expected_offset_slices(rp, ci) == (3, 3 * 64 * 3)


def test_a_decreasing_row_disqualifies_its_slice():
    rp, ci = _csr(_tridiag(256))
    r = 100                                   # in slice 1
    ci[rp[r]:rp[r + 1]] = ci[rp[r]:rp[r + 1]][::-1].copy()
    assert expected_offset_slices(rp, ci) == (1, 64 * 3)


def test_more_than_fifteen_offsets_disqualify():
    n = 256
    band = sp.diags([np.ones(n - abs(k)) for k in range(-8, 8)], list(range(-8, 8)))   # 16 offsets
    rp, ci = _csr(band)
    assert expected_offset_slices(rp, ci) == (0, 0)
    band15 = sp.diags([np.ones(n - abs(k)) for k in range(-7, 8)], list(range(-7, 8)))  # 15 offsets
    rp, ci = _csr(band15)
    assert expected_offset_slices(rp, ci) == (2, 2 * 64 * 15)


def test_offset_list_longer_than_the_longest_row_disqualifies():
    n = 256
    rows = np.arange(n - 1)
    cols = rows + (rows % 2)                  # one entry per row, at offset 0 or 1: |S| = 2 > w = 1
    Q = sp.csr_matrix((np.ones(n - 1), (rows, cols)), shape=(n, n))
    rp, ci = _csr(Q)
    assert expected_offset_slices(rp, ci) == (0, 0)


def test_rows_lacking_offsets_still_qualify():
    # a 2D 5-point stencil on a 64-wide grid: boundary rows lack -1 / +1 / -64 / +64, the union is 5 offsets
    m = 64
    T = _tridiag(m)
    Q = sp.kronsum(T, T)
    rp, ci = _csr(Q)
    c, z = expected_offset_slices(rp, ci)
    assert c == m - 2 and z == int(rp[(m - 1) * 64] - rp[64])
