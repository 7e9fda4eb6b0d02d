"""Tucker / HOSVD algorithms of Sections 4-5 and the error measure of Section 8.

Deterministic references (used only to pin the randomized ones):
  thosvd   truncated HOSVD: Q_n = leading R_n left singular vectors of X_(n)
           (eq. UnfoldHOSVD), core S = X x_1 Q_1^T ... x_N Q_N^T (eq. Core).
  sthosvd  sequentially truncated HOSVD (Algorithm 4) at fixed ranks.

Randomized algorithms (the path the GPU implements):
  rp_hosvd   Algorithm 6: every Q_n from a Gaussian sketch of X_(n), then
             the core X x_n Q_n^T.  With oversampling (K_n > R_n) the K-sized
             core is brought back to rank R by a THOSVD of that small core
             (the reading used where the algorithm is silent).
  r_sthosvd  Algorithm 8: for each mode in turn, Algorithm 1 on the current
             S_(n) with target rank R_n, then S <- S x_n Q_n^T.

Every factor has its columns sign-canonicalised (largest-magnitude entry
positive) and the core carries the matching signs; this changes nothing in
the approximation and makes factors comparable entry by entry.

Relative error (Section 8, eq. Relativeerror): E = ||X - Xhat||_F / ||X||_F.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .philox import TAG_RP_HOSVD, TAG_R_STHOSVD, omega_unfolding
from .rsvd import brsvd, canonical_signs, qr_pos
from .tensor_ops import frob2, ttm, tucker_to_full, unfold


@dataclass
class TuckerResult:
    core: np.ndarray
    factors: List[np.ndarray]
    sigma: List[np.ndarray]            # per mode, leading R_n singular values
    k_used: List[int]                  # per mode sketch width (R_n for deterministic)
    norm_x2: float                     # ||X||^2
    norm_core2: float                  # ||G||^2
    rel_error: float                   # explicit ||X - Xhat|| / ||X||
    trace: Optional[list] = field(default=None, repr=False)

    @property
    def rel_error_identity(self):
        """sqrt(max(0, ||X||^2 - ||G||^2)) / ||X||, valid for orthonormal factors."""
        return float(np.sqrt(max(0.0, self.norm_x2 - self.norm_core2) / self.norm_x2))


def rel_error(x, core, factors):
    """E = ||X - [[G; U_1..U_N]]||_F / ||X||_F, everything in float64."""
    x = np.asarray(x, dtype=np.float64)
    xh = tucker_to_full(np.asarray(core, dtype=np.float64),
                        [np.asarray(u, dtype=np.float64) for u in factors])
    return float(np.sqrt(frob2(x - xh) / frob2(x)))


def _check_ranks(dims, ranks):
    if len(ranks) != len(dims):
        raise ValueError("one rank per mode is required")
    for d, r in zip(dims, ranks):
        if not (1 <= r <= d):
            raise ValueError("ranks must satisfy 1 <= R_n <= I_n")


def _finish(x, core, factors, sigma, k_used, trace=None):
    return TuckerResult(core=core, factors=factors, sigma=sigma, k_used=k_used,
                        norm_x2=frob2(x), norm_core2=frob2(core),
                        rel_error=rel_error(x, core, factors), trace=trace)


def _leading_left(mat, r):
    u, s, _ = np.linalg.svd(mat, full_matrices=False)
    return u[:, :r], s[:r]


def thosvd(x, ranks):
    """Truncated HOSVD by brute-force SVD of every unfolding."""
    x = np.asarray(x, dtype=np.float64)
    _check_ranks(x.shape, ranks)
    factors, sigma = [], []
    for n in range(x.ndim):
        u, s = _leading_left(unfold(x, n), ranks[n])
        factors.append(u * canonical_signs(u))
        sigma.append(s)
    core = x
    for n, u in enumerate(factors):
        core = ttm(core, u.T, n)
    return _finish(x, core, factors, sigma, list(ranks))


def sthosvd(x, ranks, mode_order=None):
    """Algorithm 4 with fixed ranks, brute-force SVD per step."""
    x = np.asarray(x, dtype=np.float64)
    _check_ranks(x.shape, ranks)
    order = list(range(x.ndim)) if mode_order is None else list(mode_order)
    factors, sigma = [None] * x.ndim, [None] * x.ndim
    s_t = x
    for n in order:
        u, s = _leading_left(unfold(s_t, n), ranks[n])
        u = u * canonical_signs(u)
        factors[n], sigma[n] = u, s
        s_t = ttm(s_t, u.T, n)
    return _finish(x, s_t, factors, sigma, list(ranks))


def r_sthosvd(x, ranks, p, q, seed, mode_order=None, keep_trace=False, omega_fn=None):
    """Algorithm 8: randomized sequentially truncated HOSVD.

    S starts as the whole tensor X (the first step of the printed algorithm
    writes the unfolding, which cannot be meant before n is bound).  For each
    mode n in mode_order (ascending by default): Algorithm 1 on S_(n) with
    target rank R_n, oversampling p and q power steps, using the test matrix
    Omega(seed, mode=n, tag=2) of the current S (rows in the paper's order,
    see oracle.philox); then S <- S x_n Q_n^T with the rank-R_n factor.
    omega_fn(n, shape, K), when given, supplies the test matrix of mode n for
    the current tensor's shape instead (the structured sketch).
    """
    x = np.asarray(x, dtype=np.float64)
    _check_ranks(x.shape, ranks)
    order = list(range(x.ndim)) if mode_order is None else list(mode_order)
    if sorted(order) != list(range(x.ndim)):
        raise ValueError("mode_order must be a permutation of the modes")
    factors, sigma, k_used = [None] * x.ndim, [None] * x.ndim, [None] * x.ndim
    trace = [] if keep_trace else None
    s_t = x
    for n in order:
        a = unfold(s_t, n)
        if ranks[n] > a.shape[1]:
            raise ValueError("R_n exceeds the column count of the current unfolding")
        if omega_fn is None:
            om_fn = lambda J, K, n=n, sh=s_t.shape: omega_unfolding(seed, n, TAG_R_STHOSVD, sh, K)
        else:
            om_fn = lambda J, K, n=n, sh=s_t.shape: omega_fn(n, sh, K)
        res = brsvd(a, ranks[n], p, q, om_fn)
        u = res.U * canonical_signs(res.U)
        factors[n], sigma[n], k_used[n] = u, res.s, res.K
        if keep_trace:
            trace.append((n, s_t, res))
        s_t = ttm(s_t, u.T, n)                      # Algorithm 8, S x_n Q^T
    return _finish(x, s_t, factors, sigma, k_used, trace)


def rp_hosvd(x, ranks, p, q, seed, omega_fn=None):
    """Algorithm 6: random-projection HOSVD.

    For every mode n independently: K_n = min(R_n + p, I_n, J_n),
    W = X_(n) Omega_n (Omega(seed, mode=n, tag=1)), Q_n an orthonormal basis
    of W, refined by q power steps as in Algorithm 1.  Core H = X x_n Q_n^T.
    When some K_n > R_n the K-sized core is truncated by a THOSVD of H:
    W_n = leading R_n left singular vectors of H_(n), U_n = Q_n W_n,
    G = H x_n W_n^T.
    """
    x = np.asarray(x, dtype=np.float64)
    _check_ranks(x.shape, ranks)
    N = x.ndim
    qs, k_used = [], []
    for n in range(N):
        a = unfold(x, n)
        I, J = a.shape
        K = min(ranks[n] + p, I, J)
        if ranks[n] > J:
            raise ValueError("R_n exceeds the column count of the unfolding")
        om = (omega_unfolding(seed, n, TAG_RP_HOSVD, x.shape, K) if omega_fn is None
              else omega_fn(n, x.shape, K))
        y = a @ om
        qm = qr_pos(y)
        for _ in range(q):
            qz = qr_pos(a.T @ qm)
            qm = qr_pos(a @ qz)
        qs.append(qm)
        k_used.append(K)
    h = x
    for n in range(N):
        h = ttm(h, qs[n].T, n)                      # Algorithm 6, core
    if all(k == r for k, r in zip(k_used, ranks)):
        ws = [np.eye(r) for r in ranks]
        sigma = [np.linalg.svd(unfold(h, n), compute_uv=False)[:ranks[n]]
                 for n in range(N)]
    else:
        ws, sigma = [], []
        for n in range(N):
            w, s = _leading_left(unfold(h, n), ranks[n])
            ws.append(w)
            sigma.append(s)
    factors = []
    g = h
    for n in range(N):
        u = qs[n] @ ws[n]
        sg = canonical_signs(u)
        factors.append(u * sg)
        g = ttm(g, (ws[n] * sg).T, n)
    return _finish(x, g, factors, sigma, k_used)
