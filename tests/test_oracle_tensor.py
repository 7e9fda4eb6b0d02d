"""Pins for the oracle's tensor algebra (oracle.tensor_ops), Section 2.

The unfolding is checked against its index formula written out with loops,
the mode-n product against its defining sum, and both together against the
identity eq. TMM-M and the Kronecker form of a Tucker unfolding
(eq. TuckerUnfold).
"""
import itertools

import numpy as np

from oracle.tensor_ops import fold, frob2, ttm, tucker_to_full, unfold


def _unfold_loops(x, n):
    dims = x.shape
    N = len(dims)
    J = int(np.prod([d for k, d in enumerate(dims) if k != n]))
    out = np.zeros((dims[n], J))
    for idx in itertools.product(*[range(d) for d in dims]):
        j = 0
        for k in range(N):
            if k == n:
                continue
            jk = 1
            for m in range(k):
                if m != n:
                    jk *= dims[m]
            j += idx[k] * jk
        out[idx[n], j] = x[idx]
    return out


def test_unfold_matches_index_formula():
    rng = np.random.default_rng(0)
    for dims in [(3, 4, 2), (2, 3, 2, 3), (5, 1, 4), (4, 3)]:
        x = rng.standard_normal(dims)
        for n in range(len(dims)):
            np.testing.assert_array_equal(unfold(x, n), _unfold_loops(x, n))
            np.testing.assert_array_equal(fold(unfold(x, n), n, dims), x)


def test_unfold_of_fortran_memory():
    # first-index-fastest storage: X_(0) is the raw buffer read column-major
    x = np.asfortranarray(np.random.default_rng(1).standard_normal((4, 3, 5)))
    flat = x.reshape(-1, order="F")
    np.testing.assert_array_equal(unfold(x, 0), flat.reshape(4, 15, order="F"))


def test_ttm_matches_definition():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4, 2))
    b = rng.standard_normal((5, 4))
    y = ttm(x, b, 1)
    want = np.zeros((3, 5, 2))
    for i1, j, i3 in itertools.product(range(3), range(5), range(2)):
        want[i1, j, i3] = sum(x[i1, i2, i3] * b[j, i2] for i2 in range(4))
    np.testing.assert_allclose(y, want, rtol=1e-14, atol=1e-14)


def test_ttm_composition_identity():
    # X x_n B x_n A = X x_n (A B)   (eq. TMM-M)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 5, 3, 2))
    b = rng.standard_normal((6, 3))
    a = rng.standard_normal((2, 6))
    np.testing.assert_allclose(ttm(ttm(x, b, 2), a, 2), ttm(x, a @ b, 2), rtol=1e-12, atol=1e-12)


def test_tucker_unfolding_kronecker_form():
    # X = S x_1 Q1 ... x_N QN  <=>  X_(n) = Qn S_(n) (QN kron .. Q(n+1) kron Q(n-1) .. Q1)^T
    rng = np.random.default_rng(4)
    ranks, dims = (2, 3, 2, 2), (4, 5, 3, 3)
    s = rng.standard_normal(ranks)
    qs = [rng.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    x = tucker_to_full(s, qs)
    for n in range(4):
        kr = np.ones((1, 1))
        for k in reversed(range(4)):
            if k != n:
                kr = np.kron(kr, qs[k])
        np.testing.assert_allclose(unfold(x, n), qs[n] @ unfold(s, n) @ kr.T, rtol=1e-11, atol=1e-11)


def test_frob2():
    x = np.arange(12.0).reshape(3, 4)
    assert frob2(x) == float(np.sum(np.arange(12.0) ** 2))
