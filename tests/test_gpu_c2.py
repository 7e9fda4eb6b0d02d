"""Parity at the full size of the order-3 workload (GPU only).

500^3 FP32 (500 MB), exact Tucker rank (20, 20, 20) with factor scales
0.9^k and 1e-4 noise; R-STHOSVD with R = 20, p = 10 (K = 30), q = 1, modes
1 -> 2 -> 3, Omega seed 0 (Algorithm 8 with Algorithm 1 per mode).  Its modes
have 500 rows, so this size takes the wave-private streaming kernels and
CholeskyQR2 rather than the column kernel and the Householder QR of the
200^4 workload.  The FP64 oracle decomposes the upcast tensor with the same
Omega; compared as in the small end-to-end cases: E, per-mode sigma, the
projectors U U^T, orthonormality, the sketch widths, and the identity-based E
against the explicit residual of the GPU's own factors.  The bf16 path is
checked against the same oracle E within 1e-3 and against the FP32 path.
"""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.tensor_ops import frob2, tucker_to_full  # noqa: E402
from oracle.tucker import r_sthosvd as o_rst  # noqa: E402
from paper_2001_07124_amd import api  # noqa: E402
from paper_2001_07124_amd.inputs import make_workload  # noqa: E402

NAME = "r_sthosvd_500x3_r20_f32"


@pytest.fixture(scope="module")
def case():
    print(f"[c2] generating {NAME}", flush=True)
    x, w = make_workload(NAME)
    print("[c2] oracle", flush=True)
    ref = o_rst(x.astype(np.float64), w["target"], w["p"], w["q"], seed=w["seed"])
    xd = api.to_device(x)
    torch.cuda.synchronize()
    return x, w, ref, xd


def _decompose(xd, w, precision):
    dec = api.Decomposer(w["dims"], w["target"], algo="r_sthosvd", p=w["p"], q=w["q"],
                         seed=w["seed"], dtype=torch.float32, precision=precision)
    dec.run(xd)
    torch.cuda.synchronize()
    res = dec.result()
    core = api.to_numpy_fortran(res.core).astype(np.float64)
    facs = [f.cpu().numpy().astype(np.float64) for f in res.factors]
    return res, core, facs


def test_c2_fp32_matches_oracle(case):
    x, w, ref, xd = case
    res, core, facs = _decompose(xd, w, "f32")
    print(f"[c2] f32: E {res.rel_error:.8f}, oracle {ref.rel_error:.8f}", flush=True)
    # FP32 data and accumulation over 250000-column unfoldings: as the small
    # FP32 cases (E 1e-5, sigma 1e-5 relative, projectors 1e-4)
    assert abs(res.rel_error - ref.rel_error) <= 1e-5
    assert abs(res.norm_x2 - ref.norm_x2) <= 1e-6 * ref.norm_x2
    for n, (u, v) in enumerate(zip(facs, ref.factors)):
        r = u.shape[1]
        np.testing.assert_allclose(res.sigma(n), ref.sigma[n], rtol=1e-5, atol=1e-5 * ref.sigma[n][0])
        assert np.linalg.norm(u @ u.T - v @ v.T, 2) <= 1e-4
        assert np.linalg.norm(u.T @ u - np.eye(r), 2) <= 1e-5
        assert res.k_used[n] == ref.k_used[n] == 30
    x64 = x.astype(np.float64)
    e_exp = np.sqrt(frob2(x64 - tucker_to_full(core, facs)) / frob2(x64))
    assert abs(e_exp - res.rel_error) <= 1e-5


def test_c2_bf16_path(case):
    x, w, ref, xd = case
    res, _, facs = _decompose(xd, w, "bf16")
    res32, _, _ = _decompose(xd, w, "f32")
    print(f"[c2] bf16: E {res.rel_error:.8f}, f32 {res32.rel_error:.8f}, oracle {ref.rel_error:.8f}",
          flush=True)
    assert abs(res.rel_error - ref.rel_error) <= 1e-3
    assert abs(res.rel_error - res32.rel_error) <= 1e-4
    for u in facs:
        assert np.linalg.norm(u.T @ u - np.eye(u.shape[1]), 2) <= 1e-5
