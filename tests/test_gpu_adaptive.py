"""Fixed-precision R-STHOSVD on the GPU against the FP64 oracle (GPU only).

rhosvd_decompose_adaptive chooses R_n per mode from the tolerance (Section
5.1 with Algorithm 4's per-mode share eps^2 ||X||^2 / N) and
oracle.variants.r_sthosvd_adaptive does the same in FP64 with the part
outside range(Q) formed explicitly.  The rank is an integer decided by
floating point, so each case is chosen (and checked here, on the oracle's
residuals) to sit away from the threshold: the oracle's residual at the
chosen rank is at most 0.8 of the budget and the one at the rank below at
least 1.25 times it, margins far above the residual's rounding (about
1e-7 ||S||^2 in FP32, 1e-5 with split-bf16 operands, against a budget of
at least 7e-4 ||X||^2).  Compared: ranks, the met flags, E, the leading singular
values and the projectors U U^T, to the tolerances of the fixed-rank
end-to-end cases.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.tensor_ops import frob2, ttm, unfold  # noqa: E402
from oracle.variants import r_sthosvd_adaptive  # noqa: E402
from paper_2001_07124_amd import api  # noqa: E402
from paper_2001_07124_amd.inputs import tucker_tensor  # noqa: E402

# (dims, true ranks, factor decay, noise, eps, kmax, q)
CASES = [
    ((60, 50, 40), (5, 6, 4), None, 1e-3, 0.1, 16, 1),
    ((20, 18, 16, 14), (3, 4, 2, 5), None, 1e-3, 0.1, 12, 1),
    ((48, 40, 36), (12, 12, 12), 0.6, 1e-4, 0.046, 20, 2),
]
# (E, projectors and sigma).  bf16: the split-bf16 Gram carries about 1e-5
# of sigma_1^2; a projector then moves by that over the relative gap at the
# cut, (sigma_R^2 - sigma_{R+1}^2) / sigma_1^2, which the decaying case puts
# near 1.4e-3, so 2e-2 bounds it
TOL = {"f64": (1e-9, 1e-8), "f32": (1e-5, 1e-4), "bf16": (1e-3, 2e-2)}


def _oracle_margins(x, eps, res):
    """Per mode, the oracle's residual at R_n and at R_n - 1 over the budget
    (recomputed along the oracle's own sequence of truncations)."""
    budget = eps * eps * frob2(x) / x.ndim
    out = []
    s_t = x
    for n, r in enumerate(res.ranks):
        a = unfold(s_t, n)
        u = res.result.factors[n]
        # with U = Q Ubar the residual of R columns is ||S_(n)||^2 - ||U^T S_(n)||^2
        full = frob2(a)
        at_r = full - frob2(u.T @ a)
        below = full - frob2(u[:, : r - 1].T @ a) if r > 1 else full
        out.append((at_r / budget, below / budget))
        s_t = ttm(s_t, u.T, n)
    return out


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", ["f64", "f32", "bf16"])
def test_adaptive_matches_oracle(case, precision):
    dims, true_ranks, decay, noise, eps, kmax, q = case
    dt = np.float64 if precision == "f64" else np.float32
    x, _, _ = tucker_tensor(dims, true_ranks, seed=31, decay=decay, noise=noise, dtype=dt)
    x64 = x.astype(np.float64)
    ref = r_sthosvd_adaptive(x64, eps, kmax, q, seed=0)
    margins = _oracle_margins(x64, eps, ref)
    for n, (at_r, below) in enumerate(margins):
        # the case is decided far from the threshold (else it is a bad case)
        assert at_r <= 0.8 and (ref.ranks[n] == 1 or below >= 1.25), (n, at_r, below)
    xd = api.to_device(x)
    got = api.decompose_adaptive(xd, eps, kmax=kmax, q=q, seed=0, precision=precision)
    print(f"[adaptive] {dims} {precision}: ranks {got.ranks} (oracle {tuple(ref.ranks)}), "
          f"E {got.rel_error:.8f} (oracle {ref.result.rel_error:.8f})", flush=True)
    assert got.ranks == tuple(ref.ranks)
    assert got.met == tuple(ref.met)
    tol_e, tol_p = TOL[precision]
    assert abs(got.rel_error - ref.result.rel_error) <= tol_e
    for n in range(len(dims)):
        u = got.factors[n].cpu().numpy().astype(np.float64)
        uo = ref.result.factors[n]
        assert np.linalg.norm(u @ u.T - uo @ uo.T, 2) <= tol_p
        s = got.sigma(n)
        np.testing.assert_allclose(s, ref.result.sigma[n], rtol=tol_p, atol=0)
    assert got.k_used == [min(kmax, d) for d in dims]


def test_adaptive_unreachable_tolerance_keeps_kmax():
    # the tolerance is below the noise floor: every mode keeps K_n = kmax
    # columns and reports its share unmet, as the oracle does
    dims = (30, 28, 26)
    x, _, _ = tucker_tensor(dims, (4, 4, 4), seed=32, noise=1e-2, dtype=np.float64)
    ref = r_sthosvd_adaptive(x, 1e-6, 5, 1, seed=0)
    got = api.decompose_adaptive(api.to_device(x), 1e-6, kmax=5, q=1, seed=0, precision="f64")
    assert got.ranks == (5, 5, 5) == tuple(ref.ranks)
    assert got.met == (False, False, False) == tuple(ref.met)
    assert abs(got.rel_error - ref.result.rel_error) <= 1e-9


def test_adaptive_rejects_bad_parameters():
    x = api.to_device(np.ones((4, 4, 4), dtype=np.float32, order="F"))
    for eps, kmax in ((0.0, 4), (-1.0, 4), (0.1, 0), (0.1, 65)):
        with pytest.raises(api.L.RhosvdError):
            api.decompose_adaptive(x, eps, kmax=kmax)
