"""Further randomized Tucker algorithms of Section 5 (oracle side, FP64).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

  r_sthosvd_adaptive  R-STHOSVD at a tolerance instead of fixed ranks: the
                      fixed-precision use of Algorithm 1 inside Algorithm 8
                      that Section 5.1 describes (ranks not known in advance),
                      with the per-mode split of the error of Algorithm 4 and
                      eq. SubProEQ.
  rp_hooi             random projection HOOI, Algorithm 7.
  r_pet               the pass-efficient randomized Tucker algorithm R-PET,
                      Algorithm 9 (factor sketches and a core sketch from one
                      pass over X, core recovered by least squares).
  omega_kr            the memory-efficient structured test matrix of Section
                      5.1 (a Khatri-Rao product of small Gaussian matrices,
                      one per other mode), and r_sthosvd_kr / rp_hosvd_kr,
                      Algorithms 8 and 6 sketching with it.

Readings where the paper is silent or garbled (listed with the others in the
design notes):
* Adaptive tolerance: the printed bounds mix eps, eps/N and sqrt(N) eps on
  squared and unsquared norms.  Taken here: for a relative target eps, mode
  n keeps the smallest R_n with ||S_(n) - U U^T S_(n)||_F^2 <= eps^2
  ||X||_F^2 / N, so that the whole error (a sum of these per-mode residuals
  for sequential truncation) is at most eps ||X||_F.
* RP-HOOI: Algorithm 7 starts from HOSVD factors or Gaussian matrices; here
  from the orthonormalised Gaussian matrices (a Householder QR of an I_n x R_n
  draw of the Omega stream with tag 5, mode n), a fixed number of sweeps, the
  test matrix of sweep s and mode n drawn with tag 6 and mode s N + n; the
  core is X x_1 Q_1^T ... x_N Q_N^T after the last sweep.
* R-PET: K_n = min(R_n + p, I_n, J_n) and S_n = min(2 K_n + 1, I_n) (the
  paper asks only R_n <= K_n <= S_n; 2K + 1 is the usual choice of the
  one-pass sketching literature); the factor sketches use the RP-HOSVD stream
  (tag 1), the core sketch matrices Omega~_n (S_n x I_n) the tag 3 stream
  (generator rows = i_n, columns = s); the truncation of the recovered K-sized
  core to rank R is the small THOSVD used for oversampled RP-HOSVD.
* Structured sketch: the paper writes W = Z x_{p != n} Omega_p^(n) and calls
  the unfolding of W a product with the Kronecker product of the Omega_p^(n)
  (the dimensions it prints are garbled); a Kronecker product would make the
  sketch width the product of the per-mode widths, so the Khatri-Rao form of
  its footnote is taken, which keeps the width K_n of Algorithm 1: column k
  of Omega_n is the Kronecker product of the k-th columns of Gaussian
  Gamma_q (extent of mode q x K_n), q != n, i.e. the entry for the other
  modes' indices (i_q) is prod_q Gamma_q(i_q, k).  Gamma_q of mode n is the
  stream (seed, counter mode word n N + q, tag 4) over the current extent of
  mode q; no cyclic reordering is needed since the tables are indexed by the
  mode indices themselves.
"""
from dataclasses import dataclass
from typing import List

import numpy as np

from .philox import TAG_RP_HOSVD, TAG_R_STHOSVD, cyclic_position, omega, omega_unfolding
from .rsvd import canonical_signs, qr_pos
from .tensor_ops import frob2, ttm, unfold
from .tucker import TuckerResult, _finish, r_sthosvd, rp_hosvd

TAG_RPET_CORE = 3
TAG_KR = 4
TAG_HOOI_INIT = 5
TAG_HOOI_SKETCH = 6


@dataclass
class AdaptiveResult:
    result: TuckerResult
    ranks: List[int]
    met: List[bool]          # per mode: the tolerance was reached within K


def r_sthosvd_adaptive(x, eps, kmax, q, seed, mode_order=None):
    """Fixed-precision R-STHOSVD.

    For each mode n in order: sketch the current S_(n) with
    K = min(kmax, I_n, J_n) columns (Omega(seed, n, tag 2)), q power steps,
    B = Q^T S_(n) and its SVD; the residual of keeping R columns of
    U = Q Ubar is ||S_(n) - Q B||^2 + sum_{i > R} sigma_i(B)^2 (the part
    outside range(Q) plus the discarded spectrum of B), so R_n
    is the smallest R whose residual is at most eps^2 ||X||^2 / N; if no
    R <= K reaches it, R_n = K and the mode is marked unmet.  Then
    S <- S x_n U_n^T.
    """
    x = np.asarray(x, dtype=np.float64)
    N = x.ndim
    order = list(range(N)) if mode_order is None else list(mode_order)
    budget = eps * eps * frob2(x) / N
    factors, sigma, k_used = [None] * N, [None] * N, [None] * N
    ranks, met = [None] * N, [None] * N
    s_t = x
    for n in order:
        a = unfold(s_t, n)
        I, J = a.shape
        K = min(int(kmax), I, J)
        om = omega_unfolding(seed, n, TAG_R_STHOSVD, s_t.shape, K)
        qm = qr_pos(a @ om)
        for _ in range(q):
            qz = qr_pos(a.T @ qm)
            qm = qr_pos(a @ qz)
        b = qm.T @ a
        ub, sb, _ = np.linalg.svd(b, full_matrices=False)
        # residual after keeping 1..K columns: the part of S_(n) outside
        # range(Q), formed explicitly (no cancellation), plus the tail of
        # B's spectrum
        outside = frob2(a - qm @ b)
        tail = np.concatenate([np.cumsum((sb ** 2)[::-1])[::-1][1:], [0.0]])
        resid = outside + tail
        ok = np.flatnonzero(resid <= budget)
        r = int(ok[0]) + 1 if ok.size else K
        met[n] = bool(ok.size)
        u = qm @ ub[:, :r]
        u = u * canonical_signs(u)
        factors[n], sigma[n], k_used[n], ranks[n] = u, sb[:r], K, r
        s_t = ttm(s_t, u.T, n)
    return AdaptiveResult(result=_finish(x, s_t, factors, sigma, k_used), ranks=ranks, met=met)


def _omega_for(seed, word, tag, shape, n, K):
    """The Omega stream (seed, counter mode word `word`, tag) laid out for the
    n-unfolding of a tensor of `shape`: paper row j = l + L t holds generator
    row c = t + T l, as for the per-mode sketches."""
    L = int(np.prod(shape[:n], dtype=np.int64))
    T = int(np.prod(shape[n + 1:], dtype=np.int64))
    om = omega(seed, word, tag, L * T, K)
    return om[cyclic_position(np.arange(L * T), L, T)]


def _hooi_init(x, ranks, seed):
    return [qr_pos(omega(seed, n, TAG_HOOI_INIT, x.shape[n], r)) for n, r in enumerate(ranks)]


def rp_hooi(x, ranks, sweeps, seed):
    """Algorithm 7: for each sweep and mode n, S = X x_{p != n} Q_p^T,
    W = S_(n) Omega (Omega: prod_{p != n} R_p x R_n Gaussian), Q_n = QR(W);
    the core is X x_1 Q_1^T ... x_N Q_N^T at the end (factor signs then
    made canonical, the core carrying them)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.ndim
    for d, r in zip(x.shape, ranks):
        if not (1 <= r <= d):
            raise ValueError("ranks must satisfy 1 <= R_n <= I_n")
    qs = _hooi_init(x, ranks, seed)
    for s in range(int(sweeps)):
        for n in range(N):
            st = x
            for p_ in range(N):
                if p_ != n:
                    st = ttm(st, qs[p_].T, p_)
            om = _omega_for(seed, s * N + n, TAG_HOOI_SKETCH, st.shape, n, ranks[n])
            qs[n] = qr_pos(unfold(st, n) @ om)
    core = x
    for n in range(N):
        core = ttm(core, qs[n].T, n)
    # as for the other algorithms: each factor's signs canonical, the core
    # carrying them; sigma from the core's unfoldings
    sigma = [np.linalg.svd(unfold(core, n), compute_uv=False)[:ranks[n]] for n in range(N)]
    factors = []
    for n in range(N):
        sg = canonical_signs(qs[n])
        factors.append(qs[n] * sg)
        core = ttm(core, np.diag(sg), n)
    return _finish(x, core, factors, sigma, list(ranks))


def r_pet(x, ranks, p, seed):
    """Algorithm 9 (R-PET): Y_n = X_(n) Omega_n, Q_n = QR(Y_n); core sketch
    H = X x_1 Omega~_1 ... x_N Omega~_N; S = H x_n (Omega~_n Q_n)^+ for all n;
    then the K-sized S and the Q_n are truncated to rank R by the THOSVD of S
    (W_n leading left singular vectors of S_(n), U_n = Q_n W_n,
    G = S x_n W_n^T), signs canonical."""
    x = np.asarray(x, dtype=np.float64)
    N = x.ndim
    qs, ks, ss = [], [], []
    for n in range(N):
        a = unfold(x, n)
        I, J = a.shape
        if not (1 <= ranks[n] <= min(I, J)):
            raise ValueError("ranks must satisfy 1 <= R_n <= min(I_n, J_n)")
        K = min(ranks[n] + p, I, J)
        S = min(2 * K + 1, I)
        qs.append(qr_pos(a @ omega_unfolding(seed, n, TAG_RP_HOSVD, x.shape, K)))
        ks.append(K)
        ss.append(S)
    # core sketch from the same pass over X
    h = x
    for n in range(N):
        omt = omega(seed, n, TAG_RPET_CORE, x.shape[n], ss[n]).T      # S_n x I_n
        h = ttm(h, omt, n)
    core = h
    for n in range(N):
        omt = omega(seed, n, TAG_RPET_CORE, x.shape[n], ss[n]).T
        core = ttm(core, np.linalg.pinv(omt @ qs[n]), n)
    factors, sigma, g = [], [], core
    for n in range(N):
        u, s, _ = np.linalg.svd(unfold(core, n), full_matrices=False)
        w = u[:, :ranks[n]]
        un = qs[n] @ w
        sg = canonical_signs(un)
        factors.append(un * sg)
        sigma.append(s[:ranks[n]])
        g = ttm(g, (w * sg).T, n)
    return _finish(x, g, factors, sigma, ks)


def kr_tables(seed, n, shape, K):
    """The Gaussian tables Gamma_q (shape[q] x K) of mode n's structured
    sketch, q != n (stream word n N + q, tag 4)."""
    N = len(shape)
    return {q: omega(seed, n * N + q, TAG_KR, int(shape[q]), int(K)) for q in range(N) if q != n}


def omega_kr(seed, n, shape, K):
    """Structured test matrix for the n-unfolding of a tensor of `shape`, rows
    in the paper's column order j = l + L t (the other modes' indices in
    storage order, first fastest): Omega(j, k) = prod_{q != n} Gamma_q(i_q(j), k)."""
    shape = tuple(int(d) for d in shape)
    tabs = kr_tables(seed, n, shape, K)
    other = [q for q in range(len(shape)) if q != n]
    J = int(np.prod([shape[q] for q in other], dtype=np.int64))
    idx = np.unravel_index(np.arange(J), [shape[q] for q in other], order="F")
    om = np.ones((J, int(K)))
    for pos, q in enumerate(other):
        om *= tabs[q][idx[pos], :]
    return om


def r_sthosvd_kr(x, ranks, p, q, seed):
    """Algorithm 8 in the natural mode order with Algorithm 1 sketching by
    omega_kr of the current tensor."""
    return r_sthosvd(x, ranks, p, q, seed, omega_fn=lambda n, sh, K: omega_kr(seed, n, sh, K))


def rp_hosvd_kr(x, ranks, p, q, seed):
    """Algorithm 6 with every sketch W = X_(n) omega_kr(seed, n, X.shape, K_n)."""
    return rp_hosvd(x, ranks, p, q, seed, omega_fn=lambda n, sh, K: omega_kr(seed, n, sh, K))
