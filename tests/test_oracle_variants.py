"""Pins for the oracle's further randomized Tucker algorithms (oracle.variants).

* fixed-precision R-STHOSVD: the error bound E <= eps that the per-mode
  split gives; at full sketch width it is deterministic STHOSVD with each
  rank the smallest whose tail energy (brute-force SVD of the current
  unfolding) fits eps^2 ||X||^2 / N; exact-rank data return the true ranks;
* RP-HOOI (Algorithm 7): exact recovery, orthonormal factors, the projection
  identity, the lower bound max_n tau_n, and improvement over its Gaussian
  start;
* R-PET (Algorithm 9): exact recovery; without oversampling it shares its
  factor ranges with RP-HOSVD (q = 0), whose core is the orthogonal
  projection onto their Tucker subspace, so the two errors differ by exactly
  the distance between the reconstructions (Pythagoras); and it stays within
  a small factor of RP-HOSVD on noisy data (Table 1).
"""
import numpy as np
import pytest

from oracle.tensor_ops import frob2, ttm, tucker_to_full, unfold
from oracle.tucker import rp_hosvd
from oracle.variants import _hooi_init, r_pet, r_sthosvd_adaptive, rp_hooi
from paper_2001_07124_amd.inputs import tucker_tensor


def _orth(u):
    return float(np.linalg.norm(u.T @ u - np.eye(u.shape[1]), 2))


@pytest.mark.parametrize("eps", [0.3, 0.1, 0.05])
def test_adaptive_meets_tolerance(eps):
    x, _, _ = tucker_tensor((30, 25, 20), (6, 5, 4), seed=50, noise=0.02, factors="gaussian",
                            dtype=np.float64)
    ad = r_sthosvd_adaptive(x, eps, kmax=20, q=1, seed=3)
    assert all(ad.met)
    assert ad.result.rel_error <= eps * (1 + 1e-12)
    for u in ad.result.factors:
        assert _orth(u) <= 1e-12


def test_adaptive_full_width_is_deterministic_sthosvd():
    x, _, _ = tucker_tensor((9, 8, 7), (4, 3, 3), seed=51, noise=0.1, dtype=np.float64)
    eps = 0.08
    ad = r_sthosvd_adaptive(x, eps, kmax=100, q=0, seed=1)
    # brute force: smallest rank whose tail energy fits the per-mode budget
    budget = eps * eps * frob2(x) / 3
    s_t, want = x, []
    for n in range(3):
        a = unfold(s_t, n)
        u, s, _ = np.linalg.svd(a, full_matrices=False)
        tail = np.array([np.sum(s[r:] ** 2) for r in range(1, len(s) + 1)])
        r = int(np.flatnonzero(tail <= budget)[0]) + 1
        want.append(r)
        s_t = ttm(s_t, u[:, :r].T, n)
    assert ad.ranks == want
    e_det = np.sqrt(frob2(s_t) and max(0.0, frob2(x) - frob2(s_t)) / frob2(x))
    assert abs(ad.result.rel_error - e_det) <= 1e-12
    assert ad.result.rel_error <= eps


def test_adaptive_finds_exact_ranks():
    x, _, _ = tucker_tensor((24, 20, 18), (5, 4, 3), seed=52, factors="gaussian", dtype=np.float64)
    ad = r_sthosvd_adaptive(x, 1e-8, kmax=12, q=0, seed=2)
    assert ad.ranks == [5, 4, 3]
    assert ad.result.rel_error <= 1e-12


def test_adaptive_reports_unmet_mode():
    x = np.random.default_rng(53).standard_normal((20, 19, 18))     # no low-rank structure
    ad = r_sthosvd_adaptive(x, 0.01, kmax=6, q=1, seed=4)
    assert ad.ranks[0] == 6 and not ad.met[0]


@pytest.mark.parametrize("dims,ranks", [((20, 18, 16), (4, 3, 5)), ((10, 9, 8, 7), (3, 2, 3, 2))])
def test_rp_hooi_exact_recovery(dims, ranks):
    x, _, _ = tucker_tensor(dims, ranks, seed=54, factors="gaussian", dtype=np.float64)
    res = rp_hooi(x, ranks, sweeps=2, seed=5)
    assert res.rel_error <= 1e-12
    for u in res.factors:
        assert _orth(u) <= 1e-12


def test_rp_hooi_identity_bounds_and_improvement():
    x, _, _ = tucker_tensor((25, 22, 20), (5, 5, 5), seed=55, noise=0.01, dtype=np.float64)
    ranks = (5, 5, 5)
    res = rp_hooi(x, ranks, sweeps=3, seed=6)
    assert abs(res.rel_error ** 2 * res.norm_x2 - (res.norm_x2 - res.norm_core2)) <= 1e-12 * res.norm_x2
    taus = []
    for n, r in enumerate(ranks):
        s = np.linalg.svd(unfold(x, n), compute_uv=False)
        taus.append(np.sqrt(np.sum(s[r:] ** 2)))
    assert res.rel_error * np.sqrt(res.norm_x2) >= max(taus) * (1 - 1e-12)
    # the Gaussian start projects far worse than the iterated factors
    g0 = x
    for n, q in enumerate(_hooi_init(x, ranks, 6)):
        g0 = ttm(g0, q.T, n)
    e0 = np.sqrt(max(0.0, res.norm_x2 - frob2(g0)) / res.norm_x2)
    assert res.rel_error < 0.5 * e0


def test_r_pet_exact_recovery():
    x, _, _ = tucker_tensor((30, 26, 22), (4, 5, 3), seed=56, factors="gaussian", dtype=np.float64)
    res = r_pet(x, (4, 5, 3), p=3, seed=7)
    assert res.rel_error <= 1e-10
    for u in res.factors:
        assert _orth(u) <= 1e-12


def test_r_pet_core_is_in_the_rp_hosvd_subspace():
    # with p = 0 (K = R, no truncation) R-PET and RP-HOSVD (q = 0) share the
    # factor sketches, hence the factor ranges; RP-HOSVD's core X x_n Q_n^T
    # is the orthogonal projection of X onto the Tucker subspace of those
    # ranges and R-PET's reconstruction lies in the same subspace, so
    # ||X - Xpet||^2 = ||X - Xrp||^2 + ||Xpet - Xrp||^2 (Pythagoras)
    x, _, _ = tucker_tensor((12, 11, 10), (3, 3, 3), seed=57, noise=0.2, dtype=np.float64)
    ranks = (3, 2, 4)
    a = r_pet(x, ranks, p=0, seed=8)
    b = rp_hosvd(x, ranks, 0, 0, seed=8)
    for u, v in zip(a.factors, b.factors):
        np.testing.assert_allclose(u @ u.T, v @ v.T, atol=1e-10)
    xa, xb = tucker_to_full(a.core, a.factors), tucker_to_full(b.core, b.factors)
    lhs = frob2(x - xa)
    rhs = frob2(x - xb) + frob2(xa - xb)
    assert abs(lhs - rhs) <= 1e-10 * frob2(x)
    assert frob2(xa - xb) > 1e-6 * frob2(x)         # the oblique core really differs


def test_r_pet_within_reach_of_rp_hosvd_on_noisy_data():
    # Table 1: the one-pass algorithm is less accurate, but of the same order
    x, _, _ = tucker_tensor((40, 36, 30), (5, 5, 5), seed=58, noise=0.05, dtype=np.float64)
    a = r_pet(x, (5, 5, 5), p=5, seed=9)
    b = rp_hosvd(x, (5, 5, 5), 5, 0, seed=9)
    assert b.rel_error <= a.rel_error * (1 + 1e-12) or abs(a.rel_error - b.rel_error) < 1e-3
    assert a.rel_error <= 3 * b.rel_error


# ---- structured (Khatri-Rao) sketch, Section 5.1 ---------------------------

from oracle.philox import omega as _omega  # noqa: E402
from oracle.variants import TAG_KR, kr_tables, omega_kr, r_sthosvd_kr, rp_hosvd_kr  # noqa: E402


@pytest.mark.parametrize("shape", [(5, 4, 3), (4, 3, 5, 2)])
def test_omega_kr_is_the_contraction_with_the_tables(shape):
    # the sketch W = Z x_{q != n} Gamma_q^T taken column by column: column k
    # of X_(n) Omega_n contracts every other mode q of X with column k of
    # Gamma_q (the paper's tensor form, no unfolding or index arithmetic)
    rng = np.random.default_rng(70)
    x = rng.standard_normal(shape)
    K = 3
    for n in range(len(shape)):
        tabs = kr_tables(11, n, shape, K)
        y = unfold(x, n) @ omega_kr(11, n, shape, K)
        for k in range(K):
            t = x
            for q in reversed(range(len(shape))):
                if q != n:
                    t = np.tensordot(t, tabs[q][:, k], axes=([q], [0]))
            np.testing.assert_allclose(y[:, k], t, rtol=1e-12, atol=1e-12)


def test_kr_tables_come_from_their_own_streams():
    shape = (6, 5, 4)
    t01 = kr_tables(3, 0, shape, 4)[1]
    np.testing.assert_array_equal(t01, _omega(3, 0 * 3 + 1, TAG_KR, 5, 4))
    t10 = kr_tables(3, 1, shape, 4)[0]
    np.testing.assert_array_equal(t10, _omega(3, 1 * 3 + 0, TAG_KR, 6, 4))
    assert not np.allclose(kr_tables(3, 1, shape, 4)[2], kr_tables(3, 0, shape, 4)[2])
    assert not np.allclose(kr_tables(4, 0, shape, 4)[1], t01)


def test_omega_kr_moments_factor_over_the_tables():
    # the rows of Omega_n enumerate every combination of table rows once, so
    # a column's mean and mean square are the products of the tables' own
    # (a mistake in the index mapping that repeats or skips rows breaks this)
    shape = (40, 3, 30, 25)
    K = 6
    om = omega_kr(5, 1, shape, K)
    tabs = kr_tables(5, 1, shape, K)
    for k in range(K):
        m1 = np.prod([tabs[q][:, k].mean() for q in tabs])
        m2 = np.prod([(tabs[q][:, k] ** 2).mean() for q in tabs])
        assert abs(om[:, k].mean() - m1) <= 1e-12
        assert abs((om[:, k] ** 2).mean() - m2) <= 1e-12 * m2
    # and the tables themselves are standard normal draws
    allv = np.concatenate([t.ravel() for t in tabs.values()])
    assert abs(allv.mean()) < 0.1 and abs(allv.var() - 1.0) < 0.15


@pytest.mark.parametrize("dims,ranks", [((14, 12, 10), (3, 4, 2)), ((9, 8, 7, 6), (2, 3, 2, 3))])
@pytest.mark.parametrize("p,q", [(0, 0), (3, 1)])
def test_kr_sketch_exact_recovery(dims, ranks, p, q):
    # a Khatri-Rao sketch of generic tables has full column rank on the range
    # of a low-rank unfolding, so both algorithms recover exactly
    x, _, _ = tucker_tensor(dims, ranks, seed=71, factors="gaussian", dtype=np.float64)
    for res in (r_sthosvd_kr(x, ranks, p, q, seed=3), rp_hosvd_kr(x, ranks, p, q, seed=3)):
        assert res.rel_error <= 1e-12
        for u in res.factors:
            assert np.linalg.norm(u.T @ u - np.eye(u.shape[1]), 2) <= 1e-12


def test_kr_sketch_close_to_gaussian_on_noisy_data():
    # the structured sketch spans the dominant subspace about as well as the
    # dense Gaussian one (Section 5.1 offers it as a drop-in)
    from oracle.tucker import r_sthosvd
    x, _, _ = tucker_tensor((40, 36, 30), (5, 5, 5), seed=72, noise=0.02, dtype=np.float64)
    a = r_sthosvd_kr(x, (5, 5, 5), 5, 1, seed=3)
    b = r_sthosvd(x, (5, 5, 5), 5, 1, seed=3)
    assert abs(a.rel_error - b.rel_error) <= 0.02 * b.rel_error
