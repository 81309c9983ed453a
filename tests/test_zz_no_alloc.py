"""The allocation-free Gram (``ope_gram_noalloc``) against ``ope_gram``.

Two calls in a row, the second with smaller operands: integer-valued blocks
(every partial sum exact, so both entry points give identical results), then
random blocks within the FP64 rounding bound of the two summation orders; and
the size limit of the fixed scratch is refused with OPE_EINVAL.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import EPS, empty_dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _pair(rng, n, lda, na, ldb, nb, integer):
    if integer:
        A = rng.integers(-8, 9, size=(n, lda)).astype(np.float64)
        B = rng.integers(-8, 9, size=(n, ldb)).astype(np.float64)
    else:
        A = rng.standard_normal((n, lda))
        B = rng.standard_normal((n, ldb))
    return A, B


@pytest.mark.parametrize("integer", [True, False])
def test_noalloc_gram_matches_ope_gram(integer):
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=16, N=128, seed=0, with_u0=False)
    rng = np.random.default_rng(7 if integer else 8)
    with ope.Context(p.grid, p.V, 128) as ctx:
        for (n, lda, na, ldb, nb) in ((5003, 128, 128, 96, 96), (777, 20, 17, 5, 5)):
            A, B = _pair(rng, n, lda, na, ldb, nb, integer)
            Ad, Bd = to_dev(A), to_dev(B)
            o1, o2 = empty_dev(na, nb), empty_dev(na, nb)
            say(f"gram noalloc n={n} na={na} nb={nb} integer={integer}")
            ope.ope_gram(ctx.handle, Ad, lda, na, Bd, ldb, nb, n, o1)
            ope.ope_gram_noalloc(Ad, lda, na, Bd, ldb, nb, n, o2)
            g1, g2 = to_host(o1), to_host(o2)
            ref = A[:, :na].T @ B[:, :nb]
            if integer:
                assert np.array_equal(g2, g1) and np.array_equal(g2, ref)
            else:
                bound = 2 * n * EPS * (np.abs(A[:, :na]).T @ np.abs(B[:, :nb]))
                assert np.all(np.abs(g2 - g1) <= bound)
                assert np.all(np.abs(g2 - ref) <= bound)


def test_noalloc_gram_refuses_sizes_beyond_its_scratch():
    from paper_2511_06788_amd import ope
    A = to_dev(np.zeros((64, 129)))
    out = empty_dev(129, 129)
    with pytest.raises(ope.OpeError) as ei:
        ope.ope_gram_noalloc(A, 129, 129, A, 129, 129, 64, out)
    assert ei.value.status == ope.OPE_EINVAL
