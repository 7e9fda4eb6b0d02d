"""Basic randomized SVD with oversampling and power iteration (oracle side).

Algorithm 1 (Section 3.1), after Halko, Martinsson and Tropp:
  1. draw Omega, J x (R + p);
  2. Y = (X X^T)^q X Omega;
  3. economic QR, Y = Q R;
  4. B = Q^T X;
  5. SVD of B = Ubar Sbar Vbar^T;
  6. U~ = Q Ubar;
  7. keep the leading R columns / values.
The remark on stability after Algorithm 1 says the powers must not be formed
explicitly but applied one factor at a time with a QR in between; the oracle
re-orthonormalises after every half-step (X^T Q, then X Q_z).

Readings where the paper is silent (listed with the others in the design
notes): the sketch width is K = min(R + p, I, J) so that a small mode or a
short row dimension caps it; "economic QR" is taken with a non-negative
diagonal in R, which makes Q unique for a full-column-rank Y.
"""
from dataclasses import dataclass

import numpy as np


def qr_pos(y):
    """Economic Householder QR (LAPACK), columns signed so diag(R) >= 0."""
    q, r = np.linalg.qr(y, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def canonical_signs(u):
    """+-1 per column so that each column's largest-magnitude entry is
    positive; ties go to the lowest row index."""
    u = np.asarray(u)
    if u.size == 0:
        return np.ones(u.shape[1] if u.ndim == 2 else 0)
    idx = np.argmax(np.abs(u), axis=0)
    s = np.sign(u[idx, np.arange(u.shape[1])])
    s[s == 0] = 1.0
    return s


@dataclass
class BRSVDResult:
    U: np.ndarray       # I x R, leading left singular vectors (approx.)
    s: np.ndarray       # R leading singular values of B
    Vt: np.ndarray      # R x J
    K: int              # sketch width actually used
    Q: np.ndarray       # I x K orthonormal range basis
    s_all: np.ndarray   # all K singular values of B


def brsvd(x, rank, p, q, omega_fn):
    """Algorithm 1 on the matrix x (I x J).

    omega_fn(J, K) must return the J x K test matrix (see oracle.philox).
    """
    x = np.asarray(x, dtype=np.float64)
    I, J = x.shape
    if not (1 <= rank <= min(I, J)):
        raise ValueError("target rank must satisfy 1 <= R <= min(I, J)")
    K = min(rank + p, I, J)
    om = np.asarray(omega_fn(J, K), dtype=np.float64)        # step 1
    y = x @ om                                                # step 2, q = 0 part
    qm = qr_pos(y)                                            # step 3
    for _ in range(q):                                        # step 2, powers
        z = x.T @ qm
        qz = qr_pos(z)
        y = x @ qz
        qm = qr_pos(y)
    b = qm.T @ x                                              # step 4
    ub, sb, vbt = np.linalg.svd(b, full_matrices=False)       # step 5
    ut = qm @ ub                                              # step 6
    return BRSVDResult(U=ut[:, :rank], s=sb[:rank], Vt=vbt[:rank],  # step 7
                       K=K, Q=qm, s_all=sb)
