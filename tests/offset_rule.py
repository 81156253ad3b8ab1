"""The column-offset qualification rule of the sliced layout, restated on the host for the tests.

The library decides on the device which 64-row slices store their column indices as one offset list; the
GPU tests compare its count with this independent statement of the rule.
"""
import numpy as np


def expected_offset_slices(rowptr, colidx):
    """The qualification rule restated on the host: a full slice of 64 rows whose rows have strictly
    increasing columns, whose offsets (column - row) have at most 15 distinct values, no more than the
    slice's longest row, and with row + offset inside [0, n) for every row and offset of the union."""
    rowptr = np.asarray(rowptr, np.int64)
    colidx = np.asarray(colidx, np.int64)
    n = len(rowptr) - 1
    count = nnz = 0
    for s in range(n // 64):
        r0, r1 = 64 * s, 64 * s + 64
        rows = np.repeat(np.arange(r0, r1), np.diff(rowptr[r0:r1 + 1]))
        cols = colidx[rowptr[r0]:rowptr[r1]]
        offs = cols - rows
        same_row = rows[1:] == rows[:-1]
        if np.any(cols[1:][same_row] <= cols[:-1][same_row]):
            continue
        u = np.unique(offs)
        w = int(np.diff(rowptr[r0:r1 + 1]).max())
        if len(u) == 0 or len(u) > 15 or len(u) > w or r0 + u[0] < 0 or r1 - 1 + u[-1] >= n:
            continue
        count += 1
        nnz += int(rowptr[r1] - rowptr[r0])
    return count, nnz
