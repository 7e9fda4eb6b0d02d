"""Pins for the oracle's HOSVD algorithms (oracle.rsvd, oracle.tucker).

Each check is fixed by the mathematics, not by the oracle itself:
* exact recovery of tensors whose multilinear rank is at most the target
  (Table 1 prints errors near 1e-13..1e-12 for RP-HOSVD and R-STHOSVD on
  exact-rank data);
* orthonormal factors, including sketches that are rank deficient;
* ||X - Xhat||^2 = ||X||^2 - ||G||^2 (orthogonal projections, Section 5.1);
* the R-STHOSVD error split into per-mode residuals of the current tensor,
  and the RP-HOSVD per-mode error-sum bound (Section 5.1);
* the full-width special case K = I_n, where the randomized algorithms reduce
  to the deterministic THOSVD / STHOSVD computed by brute-force SVD;
* lower bound E ||X|| >= max_n tau_n, quasi-optimality sum_n tau_n^2;
* the expected spectral error bound of Algorithm 1 (Section 3.1), over 200 seeds;
* noisy data at 20 dB reach a fit near 90 percent (Section 8);
* the sign rule on hand-built matrices (largest magnitude, ties to the lower row);
* the power step against its definition (X X^T)^q X Omega (Algorithm 1
  step 2), formed without the intermediate QRs on a well-conditioned matrix,
  for Algorithm 1, RP-HOSVD and the first mode of R-STHOSVD.
"""
import numpy as np
import pytest

from oracle import philox
from oracle.rsvd import brsvd, canonical_signs, qr_pos
from oracle.tensor_ops import frob2, ttm, tucker_to_full, unfold
from oracle.tucker import r_sthosvd, rel_error, rp_hosvd, sthosvd, thosvd
from paper_2001_07124_amd.inputs import tucker_tensor


def _tau(x, n, r):
    s = np.linalg.svd(unfold(x, n), compute_uv=False)
    return float(np.sqrt(np.sum(s[r:] ** 2)))


def _orth_err(u):
    return float(np.linalg.norm(u.T @ u - np.eye(u.shape[1]), 2))


SHAPES = [((12, 10, 8), (3, 4, 2)), ((8, 7, 6, 5), (2, 3, 2, 2)), ((30, 6, 9), (5, 6, 3))]


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("p,q", [(0, 0), (3, 0), (5, 1), (2, 2)])
def test_exact_recovery(dims, ranks, p, q):
    x, _, _ = tucker_tensor(dims, ranks, seed=5, factors="gaussian", dtype=np.float64)
    for algo in (r_sthosvd, rp_hosvd):
        res = algo(x, ranks, p, q, seed=9)
        assert res.rel_error <= 1e-12, (algo.__name__, res.rel_error)
        for u in res.factors:
            assert _orth_err(u) <= 1e-12


def test_rank_deficient_sketch_still_orthonormal():
    x, _, _ = tucker_tensor((20, 18, 16), (2, 2, 2), seed=1, dtype=np.float64)
    a = unfold(x, 0)
    res = brsvd(a, 2, 8, 1, lambda J, K: philox.omega(0, 0, 2, J, K))
    assert res.K == 10
    assert _orth_err(res.Q) <= 1e-12       # Y has rank 2 but Q is still orthonormal
    assert np.linalg.norm(a - res.U @ (res.U.T @ a)) <= 1e-12 * np.linalg.norm(a)


@pytest.mark.parametrize("algo", [r_sthosvd, rp_hosvd])
def test_projection_identity(algo):
    x, _, _ = tucker_tensor((15, 12, 10, 6), (3, 3, 2, 2), seed=2, noise=0.05, dtype=np.float64)
    res = algo(x, (3, 3, 2, 2), 4, 1, seed=3)
    lhs = res.rel_error ** 2 * res.norm_x2
    rhs = res.norm_x2 - res.norm_core2
    assert abs(lhs - rhs) <= 1e-12 * res.norm_x2
    assert abs(res.rel_error - res.rel_error_identity) <= 1e-9


def test_r_sthosvd_error_split():
    x, _, _ = tucker_tensor((14, 11, 9), (4, 3, 3), seed=4, noise=0.1, dtype=np.float64)
    res = r_sthosvd(x, (4, 3, 3), 2, 0, seed=1, keep_trace=True)
    total = 0.0
    for n, s_prev, _ in res.trace:
        a = unfold(s_prev, n)
        u = res.factors[n]
        total += frob2(a - u @ (u.T @ a))
    err2 = res.rel_error ** 2 * res.norm_x2
    assert abs(err2 - total) <= 1e-10 * err2


def test_rp_hosvd_error_sum_bound():
    x, _, _ = tucker_tensor((14, 11, 9), (4, 3, 3), seed=6, noise=0.1, dtype=np.float64)
    for seed in range(5):
        res = rp_hosvd(x, (4, 3, 3), 2, 0, seed=seed)
        bound = sum(frob2(ttm(x, np.eye(u.shape[0]) - u @ u.T, n)) for n, u in enumerate(res.factors))
        assert res.rel_error ** 2 * res.norm_x2 <= bound * (1 + 1e-12)


def test_full_width_reduces_to_deterministic():
    # p large enough that K_n = I_n: the sketch spans the whole column space.
    x, _, _ = tucker_tensor((9, 8, 7), (3, 3, 3), seed=7, noise=0.2, dtype=np.float64)
    ranks = (3, 2, 4)
    rst = r_sthosvd(x, ranks, 50, 0, seed=2)
    st = sthosvd(x, ranks)
    assert rst.k_used == [9, 8, 6]        # mode 3: J = 3*2 < I_3 caps K at J
    assert abs(rst.rel_error - st.rel_error) <= 1e-12
    for u, v in zip(rst.factors, st.factors):
        np.testing.assert_allclose(u @ u.T, v @ v.T, atol=1e-11)
    for s1, s2 in zip(rst.sigma, st.sigma):
        np.testing.assert_allclose(s1, s2, rtol=1e-11)
    rp = rp_hosvd(x, ranks, 50, 0, seed=2)
    th = thosvd(x, ranks)
    assert abs(rp.rel_error - th.rel_error) <= 1e-12
    for u, v in zip(rp.factors, th.factors):
        np.testing.assert_allclose(u @ u.T, v @ v.T, atol=1e-11)


def test_signs_are_canonical():
    x, _, _ = tucker_tensor((10, 9, 8), (3, 3, 3), seed=8, noise=0.1, dtype=np.float64)
    for res in (r_sthosvd(x, (3, 3, 3), 3, 1, seed=0), rp_hosvd(x, (3, 3, 3), 3, 1, seed=0),
                thosvd(x, (3, 3, 3)), sthosvd(x, (3, 3, 3))):
        for u in res.factors:
            np.testing.assert_array_equal(canonical_signs(u), np.ones(u.shape[1]))
        # the signs travel with the core: the approximation is unchanged
        xh = tucker_to_full(res.core, res.factors)
        assert abs(np.sqrt(frob2(x - xh) / frob2(x)) - res.rel_error) < 1e-14


def test_error_lower_and_quasi_optimal_bounds():
    x, _, _ = tucker_tensor((12, 10, 9), (4, 4, 3), seed=9, noise=0.3, dtype=np.float64)
    ranks = (3, 3, 2)
    taus = [_tau(x, n, r) for n, r in enumerate(ranks)]
    nx = np.sqrt(frob2(x))
    for res in (thosvd(x, ranks), sthosvd(x, ranks), r_sthosvd(x, ranks, 3, 1, seed=1),
                rp_hosvd(x, ranks, 3, 1, seed=1)):
        assert res.rel_error * nx >= max(taus) * (1 - 1e-12)
    for res in (thosvd(x, ranks), sthosvd(x, ranks)):
        assert (res.rel_error * nx) ** 2 <= sum(t * t for t in taus) * (1 + 1e-12)


def test_brsvd_expected_spectral_bound():
    rng = np.random.default_rng(10)
    I, J, R = 60, 90, 5
    u, _ = np.linalg.qr(rng.standard_normal((I, I)))
    v, _ = np.linalg.qr(rng.standard_normal((J, I)))
    sig = 0.8 ** np.arange(I)
    a = (u * sig) @ v.T
    for p in (2, 5, 10):
        for q in (0, 1, 2):
            errs = []
            for seed in range(200):
                res = brsvd(a, R, p, q, lambda JJ, KK, s=seed: philox.omega(s, 0, 2, JJ, KK))
                errs.append(np.linalg.norm(a - res.Q @ (res.Q.T @ a), 2))
            bound = (1 + np.sqrt(R / (p - 1)) + np.e * np.sqrt(R + p) / p
                     * np.sqrt(min(I, J) - R)) ** (1.0 / (2 * q + 1)) * sig[R]
            assert np.mean(errs) <= bound, (p, q, np.mean(errs), bound)
            # and never better than the optimum sigma_{R+p+1}
            assert min(errs) >= sig[R + p] * (1 - 1e-9)


def test_truncated_factor_bound():
    x, _, _ = tucker_tensor((25, 20, 15), (6, 5, 5), seed=11, noise=0.2, dtype=np.float64)
    a = unfold(x, 0)
    for seed in range(5):
        res = brsvd(a, 4, 3, 0, lambda J, K, s=seed: philox.omega(s, 0, 2, J, K))
        lhs = np.linalg.norm(a - res.U @ (res.U.T @ a))
        rhs = np.linalg.norm(a - res.Q @ (res.Q.T @ a)) + _tau(x, 0, 4)
        assert lhs <= rhs * (1 + 1e-12)


def test_qr_pos_convention():
    y = np.random.default_rng(12).standard_normal((20, 6))
    q = qr_pos(y)
    r = q.T @ y
    assert np.all(np.diag(r) > 0)
    np.testing.assert_allclose(np.tril(r, -1), 0, atol=1e-12)


def test_noisy_fit_near_ninety_percent():
    # Section 8: random low-rank tensor at 20 dB SNR, fit = 1 - E close to 0.9
    dims, ranks = (60, 60, 60), (4, 8, 6)
    x0, _, _ = tucker_tensor(dims, ranks, seed=13, factors="gaussian", dtype=np.float64)
    noise = np.random.default_rng(14).standard_normal(dims)
    gamma = np.sqrt(frob2(x0) / frob2(noise) / 10 ** (20 / 10))
    x = x0 + gamma * noise
    for res in (r_sthosvd(x, ranks, 10, 2, seed=0), rp_hosvd(x, ranks, 10, 2, seed=0),
                sthosvd(x, ranks)):
        assert 0.89 <= 1 - res.rel_error <= 0.91


def test_mode_order_permutation():
    x, _, _ = tucker_tensor((10, 9, 8, 7), (3, 2, 3, 2), seed=15, dtype=np.float64)
    res = r_sthosvd(x, (3, 2, 3, 2), 2, 1, seed=4, mode_order=(2, 0, 3, 1))
    assert res.rel_error <= 1e-12
    with pytest.raises(ValueError):
        r_sthosvd(x, (3, 2, 3, 2), 2, 1, seed=4, mode_order=(0, 0, 1, 2))


def test_canonical_signs_hand_built():
    # column 0: the largest magnitude (-5) is negative -> flip; column 1: the
    # largest (+4) positive -> keep; column 2: a tie |-3| = |3| between rows 1
    # and 3 goes to the lower row, whose entry is negative -> flip; column 3: a
    # zero column keeps +1
    u = np.array([[1.0, 4.0, 0.5, 0.0],
                  [-5.0, -2.0, -3.0, 0.0],
                  [2.0, 1.0, 1.0, 0.0],
                  [0.0, 0.0, 3.0, 0.0]])
    np.testing.assert_array_equal(canonical_signs(u), [-1.0, 1.0, -1.0, 1.0])
    # the tie resolved the other way when the lower row holds the positive entry
    np.testing.assert_array_equal(canonical_signs(np.array([[3.0], [-3.0]])), [1.0])
    np.testing.assert_array_equal(canonical_signs(np.array([[-3.0], [3.0]])), [-1.0])
    # after applying the signs every column's largest-magnitude entry is positive
    rng = np.random.default_rng(31)
    v = rng.standard_normal((9, 6))
    w = v * canonical_signs(v)
    for k in range(6):
        i = int(np.flatnonzero(np.abs(w[:, k]) == np.abs(w[:, k]).max())[0])
        assert w[i, k] > 0


def _projector(m):
    qm, _ = np.linalg.qr(m)
    return qm @ qm.T


def test_power_step_spans_the_definition():
    # Algorithm 1 step 2 defines the sketch as (X X^T)^q X Omega; the oracle
    # applies it one factor at a time with a QR in between.  On a small, well
    # conditioned matrix the unstabilised product is accurate, so both ranges
    # must coincide, and differ from the q = 0 range.
    rng = np.random.default_rng(32)
    I, J, R, p = 30, 40, 5, 3
    u, _ = np.linalg.qr(rng.standard_normal((I, I)))
    v, _ = np.linalg.qr(rng.standard_normal((J, I)))
    a = (u * np.linspace(1.0, 0.3, I)) @ v.T
    om = philox.omega(3, 0, 2, J, R + p)
    for q in (1, 2):
        res = brsvd(a, R, p, q, lambda JJ, KK: philox.omega(3, 0, 2, JJ, KK))
        y = np.linalg.matrix_power(a @ a.T, q) @ a @ om
        np.testing.assert_allclose(res.Q @ res.Q.T, _projector(y), atol=1e-10)
    res0 = brsvd(a, R, p, 0, lambda JJ, KK: philox.omega(3, 0, 2, JJ, KK))
    np.testing.assert_allclose(res0.Q @ res0.Q.T, _projector(a @ om), atol=1e-10)
    res1 = brsvd(a, R, p, 1, lambda JJ, KK: philox.omega(3, 0, 2, JJ, KK))
    assert np.linalg.norm(res1.Q @ res1.Q.T - res0.Q @ res0.Q.T) > 0.1


def test_rp_hosvd_power_step_spans_the_definition():
    # with p = 0 every K_n = R_n, so U_n spans the range of Q_n itself:
    # (X_(n) X_(n)^T)^q X_(n) Omega_n with Omega_n = Omega(seed, n, tag 1)
    x, _, _ = tucker_tensor((12, 10, 9), (4, 4, 3), seed=33, noise=0.3, dtype=np.float64)
    ranks = (3, 3, 2)
    for q in (0, 1):
        res = rp_hosvd(x, ranks, 0, q, seed=5)
        for n in range(3):
            a = unfold(x, n)
            om = philox.omega_unfolding(5, n, philox.TAG_RP_HOSVD, x.shape, ranks[n])
            y = np.linalg.matrix_power(a @ a.T, q) @ a @ om
            u = res.factors[n]
            np.testing.assert_allclose(u @ u.T, _projector(y), atol=1e-10)


def test_r_sthosvd_power_step_spans_the_definition():
    # the first mode of Algorithm 8 is Algorithm 1 on X_(1) with Omega(seed, 0, tag 2)
    x, _, _ = tucker_tensor((12, 10, 9), (4, 4, 3), seed=34, noise=0.3, dtype=np.float64)
    res = r_sthosvd(x, (3, 3, 2), 2, 1, seed=6, keep_trace=True)
    n, s0, r0 = res.trace[0]
    a = unfold(s0, n)
    om = philox.omega_unfolding(6, n, philox.TAG_R_STHOSVD, s0.shape, 5)
    y = (a @ a.T) @ a @ om
    np.testing.assert_allclose(r0.Q @ r0.Q.T, _projector(y), atol=1e-10)
