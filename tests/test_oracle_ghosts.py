"""The oracle's ghost fill (periodic wrap / zero-gradient outflow, axis by
axis over the full extent of the previous axes) against a per-axis image
rule: for faces that are periodic or outflow, a ghost cell holds the interior
cell whose index along each axis is the periodic image or the nearest
interior index, axis by axis independently.  The GPU stages read such images
instead of ghost cells between the stages of a step; this checks the rule
itself against the fill it stands in for, on every face combination."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2110_01792_amd import inputs

P, O = inputs.PERIODIC, inputs.OUTFLOW


def _image(i, n, lo, hi):
    if i < 0:
        return 0 if lo == O else i + n
    if i >= n:
        return n - 1 if hi == O else i - n
    return i


@pytest.mark.parametrize("n", [(4, 5, 6), (9, 4, 7)])
def test_ghost_fill_equals_per_axis_images(n):
    rng = np.random.default_rng(3)
    axis_kinds = [(P, P), (O, O)]  # a periodic face pairs with a periodic one
    ng = 4
    for kinds in itertools.product(axis_kinds, repeat=3):
        b = inputs.Box(n, ng, (1.0, 1.0, 1.0), tuple(kinds))
        U = rng.uniform(1.0, 2.0, size=(2,) + b.shape)
        oracle.fill_ghosts(b, U)
        nz, ny, nx = b.shape
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    ii, jj, kk = i - ng, j - ng, k - ng
                    si = _image(ii, n[0], *kinds[0])
                    sj = _image(jj, n[1], *kinds[1])
                    sk = _image(kk, n[2], *kinds[2])
                    src = U[:, sk + ng, sj + ng, si + ng]
                    assert np.array_equal(U[:, k, j, i], src), (kinds, (ii, jj, kk))
