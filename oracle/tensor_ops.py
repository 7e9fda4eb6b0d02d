"""Tensor algebra of Section 2 (oracle side).

Indices are 0-based here; the paper's are 1-based.  A tensor is a NumPy
array of shape (I_1, ..., I_N) addressed logically, whatever its memory
order.

* n-unfolding (Section 2): X_(n)(i_n, j) = X(i_1, ..., i_N) with
  j = sum_{k != n} i_k J_k and J_k = prod_{m < k, m != n} I_m.  The
  remaining indices therefore run first-index-fastest across columns.
* mode-n product (Section 2): (X x_n B)(..., j, ...) = sum_{i_n} X(..., i_n, ...) B(j, i_n)
  for B of shape (J, I_n).
"""
import numpy as np


def unfold(x, n):
    """n-unfolding X_(n), shape (I_n, prod_{k != n} I_k)."""
    x = np.asarray(x)
    return np.moveaxis(x, n, 0).reshape(x.shape[n], -1, order="F")


def fold(mat, n, dims):
    """Inverse of unfold: the tensor of shape dims whose n-unfolding is mat."""
    dims = tuple(int(d) for d in dims)
    rest = dims[:n] + dims[n + 1:]
    t = np.asarray(mat).reshape((dims[n],) + rest, order="F")
    return np.moveaxis(t, 0, n)


def ttm(x, b, n):
    """Mode-n product X x_n B, with B of shape (J, I_n)."""
    b = np.asarray(b)
    dims = list(np.shape(x))
    dims[n] = b.shape[0]
    return fold(b @ unfold(x, n), n, dims)


def tucker_to_full(core, factors):
    """[[S; Q_1, ..., Q_N]] = S x_1 Q_1 x_2 ... x_N Q_N (Section 4, eq. HOSVD)."""
    x = np.asarray(core)
    for n, q in enumerate(factors):
        x = ttm(x, q, n)
    return x


def frob2(x):
    """Squared Frobenius norm, accumulated in float64."""
    v = np.asarray(x, dtype=np.float64).reshape(-1)
    return float(v @ v)
