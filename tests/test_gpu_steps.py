"""Per-step parity of the HIP kernels against the FP64 oracle (GPU only).

Each step is called through the C ABI on seeded inputs that span several
tiles and a ragged tail, and compared element by element with the oracle's
definition of the same step:
  Omega fill      oracle.philox.omega
  sketch          unfold(X, n) @ omega(...)            (Algorithm 1 step 2, q = 0)
  power step      A (A^T Q)                             (Algorithm 1 step 2, q > 0)
  mode-n product  oracle.tensor_ops.ttm, Gram B B^T     (Algorithm 1 step 4)
  CholeskyQR2     oracle.rsvd.qr_pos (diag(R) > 0)      (Algorithm 1 step 3)
  symmetric EVD   numpy.linalg.eigh                     (Algorithm 1 step 5)
Tolerances: FP64 paths 1e-11 relative; FP32 paths are set from the
accumulation length (J terms of fp32 products): 2e-5 of the column scale.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import philox  # noqa: E402
from oracle.rsvd import qr_pos  # noqa: E402
from oracle.tensor_ops import ttm as o_ttm, unfold  # noqa: E402
from paper_2001_07124_amd import api  # noqa: E402
from paper_2001_07124_amd.inputs import tucker_tensor  # noqa: E402


def _views(dims):
    out = []
    for n in range(len(dims)):
        L = int(np.prod(dims[:n]))
        T = int(np.prod(dims[n + 1:]))
        out.append((n, (L, dims[n], T)))
    return out


def _flat(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x.reshape(-1, order="F").astype(dtype))).cuda()


def _close_cols(got, want, rtol):
    scale = np.maximum(np.max(np.abs(want), axis=0, keepdims=True), 1e-300)
    err = np.max(np.abs(got - want) / scale)
    assert err <= rtol, err


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("J,K", [(37, 9), (1000, 35), (4096, 16)])
def test_omega_fill(dtype, J, K):
    got = api.omega_fill(7, 2, 2, J, K, dtype).cpu().numpy()
    want = philox.omega(7, 2, 2, J, K)
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    np.testing.assert_allclose(got, want, rtol=tol, atol=tol)


DIMS = [(37, 23, 19), (16, 9, 130), (5, 6, 7, 8), (200, 3, 70)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_sketch(dims, dtype):
    x, _, _ = tucker_tensor(dims, tuple(min(3, d) for d in dims), seed=21, noise=0.3, dtype=dtype)
    src = _flat(x, dtype)
    x64 = x.astype(np.float64)
    for n, view in _views(dims):
        J = view[0] * view[2]
        K = min(11, dims[n], J)
        y, nrm = api.sketch(src, view, K, seed=5, mode=n, tag=2, want_norm=True)
        want = unfold(x64, n) @ philox.omega_unfolding(5, n, 2, x64.shape, K)
        tol = 1e-11 if dtype == np.float64 else 2e-5
        _close_cols(y.cpu().numpy(), want, tol)
        assert abs(nrm.item() - float(np.sum(x64 ** 2))) <= (1e-12 if dtype == np.float64 else 1e-6) * np.sum(x64 ** 2)


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_power_step(dims, dtype):
    x, _, _ = tucker_tensor(dims, tuple(min(3, d) for d in dims), seed=22, noise=0.3, dtype=dtype)
    src = _flat(x, dtype)
    x64 = x.astype(np.float64)
    rng = np.random.default_rng(3)
    for n, view in _views(dims):
        K = min(10, dims[n])
        q, _ = np.linalg.qr(rng.standard_normal((dims[n], K)))
        q = q.astype(dtype)
        qt = torch.from_numpy(q).cuda()
        y = api.power(src, view, qt).cpu().numpy()
        a = unfold(x64, n)
        want = a @ (a.T @ q.astype(np.float64))
        _close_cols(y, want, 1e-11 if dtype == np.float64 else 3e-5)


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_ttm_and_gram(dims, dtype):
    x, _, _ = tucker_tensor(dims, tuple(min(3, d) for d in dims), seed=23, noise=0.3, dtype=dtype)
    src = _flat(x, dtype)
    x64 = x.astype(np.float64)
    rng = np.random.default_rng(4)
    for n, view in _views(dims):
        kout = min(13, dims[n] + 2)
        m = rng.standard_normal((dims[n], kout)).astype(dtype)
        out, gram, nrm = api.ttm(src, view, kout, torch.from_numpy(m).cuda(), want_gram=True,
                                 want_norm=True)
        want = o_ttm(x64, m.astype(np.float64).T, n)
        got = out.cpu().numpy().reshape(want.shape, order="F")
        tol = 1e-11 if dtype == np.float64 else 2e-5
        _close_cols(unfold(got, n).T, unfold(want, n).T, tol)
        b = unfold(want, n)
        _close_cols(gram.cpu().numpy(), b @ b.T, tol)
        assert abs(nrm.item() - float(np.sum(want ** 2))) <= tol * np.sum(want ** 2)
    # identity operand on the smallest mode
    n, view = min(_views(dims), key=lambda nv: nv[1][1])
    out, _, _ = api.ttm(src, view, dims[n], None)
    np.testing.assert_array_equal(out.cpu().numpy(), x.reshape(-1, order="F"))


@pytest.mark.parametrize("I,K", [(200, 35), (37, 11), (500, 30), (64, 64), (15, 15), (256, 64), (257, 64),
                                 (1, 1), (512, 32), (513, 32), (300, 40), (700, 30)])
def test_orthonormalize(I, K):
    rng = np.random.default_rng(I * 100 + K)
    y = rng.standard_normal((I, K)) @ np.diag(np.logspace(0, -3, K))
    yt = torch.from_numpy(y).cuda()
    q, q64, flags = api.orthonormalize(yt, torch.float32)
    want = qr_pos(y)
    np.testing.assert_allclose(q64.cpu().numpy(), want, atol=1e-10)
    np.testing.assert_allclose(q.cpu().numpy(), want, atol=2e-7)
    assert flags.item() == 0


def test_orthonormalize_rank_deficient_shifts():
    # taller than 512 rows: CholeskyQR2, whose Gram is singular here
    rng = np.random.default_rng(9)
    base = rng.standard_normal((600, 6))
    y = base @ rng.standard_normal((6, 20))          # rank 6, K = 20
    q, q64, flags = api.orthonormalize(torch.from_numpy(y).cuda(), torch.float64)
    q = q64.cpu().numpy()
    assert flags.item() & api.L.FLAG_CQR_SHIFTED
    assert np.linalg.norm(q.T @ q - np.eye(20), 2) <= 1e-10
    # the range of Y is inside span(Q)
    assert np.linalg.norm(y - q @ (q.T @ y)) <= 1e-10 * np.linalg.norm(y)


def test_orthonormalize_rank_deficient_householder():
    # up to 256 rows (512 for K <= 32): Householder QR, no breakdown to report
    rng = np.random.default_rng(9)
    base = rng.standard_normal((120, 6))
    y = base @ rng.standard_normal((6, 20))          # rank 6, K = 20
    q, q64, flags = api.orthonormalize(torch.from_numpy(y).cuda(), torch.float64)
    q = q64.cpu().numpy()
    assert flags.item() == 0
    assert np.linalg.norm(q.T @ q - np.eye(20), 2) <= 1e-12
    assert np.linalg.norm(y - q @ (q.T @ y)) <= 1e-12 * np.linalg.norm(y)
    np.testing.assert_array_equal(q, q64.cpu().numpy())


@pytest.mark.parametrize("K", [1, 2, 7, 35, 64])
def test_sym_evd(K):
    rng = np.random.default_rng(K)
    a = rng.standard_normal((K, K))
    c = a @ a.T + np.diag(np.logspace(3, -2, K))
    v, lam, flags = api.sym_evd(torch.from_numpy(c).cuda())
    w, u = np.linalg.eigh(c)
    w, u = w[::-1], u[:, ::-1]
    np.testing.assert_allclose(lam.cpu().numpy(), w, rtol=1e-12, atol=1e-12 * w[0])
    vv = v.cpu().numpy()
    assert np.all(np.abs(np.abs(np.sum(vv * u, axis=0)) - 1) < 1e-9)
    assert flags.item() == 0


def _spectrum(kind, K, rng):
    """Eigenvalues with repeated or clustered values (descending)."""
    if kind == "repeated":            # blocks of three equal eigenvalues
        w = np.repeat(np.linspace(10.0, 1.0, (K + 2) // 3), 3)[:K]
    elif kind == "clustered":         # pairs 1e-9 apart, well inside the 1e-3 cluster distance
        base = np.repeat(np.linspace(5.0, 1.0, (K + 1) // 2), 2)[:K]
        w = base + 1e-9 * (np.arange(K) % 2)
    else:                             # an exact zero cluster: a Gram of rank K // 2
        w = np.concatenate([np.linspace(4.0, 1.0, K // 2), np.zeros(K - K // 2)])
    return np.sort(w)[::-1]


@pytest.mark.parametrize("K", [8, 35, 64])
@pytest.mark.parametrize("kind", ["repeated", "clustered", "zero"])
def test_sym_evd_clusters(K, kind):
    # eigenvectors of a repeated or clustered eigenvalue are not unique, so
    # the check is the decomposition itself: eigenvalues, orthonormality of
    # V and the residual norm(C V - V diag(lambda)) against norm(C)
    rng = np.random.default_rng(100 + K)
    w = _spectrum(kind, K, rng)
    u, _ = np.linalg.qr(rng.standard_normal((K, K)))
    c = (u * w) @ u.T
    c = 0.5 * (c + c.T)
    v, lam, flags = api.sym_evd(torch.from_numpy(c).cuda())
    lam, vv = lam.cpu().numpy(), v.cpu().numpy()
    nc = np.linalg.norm(c, 2)
    np.testing.assert_allclose(lam, np.linalg.eigvalsh(c)[::-1], rtol=0, atol=1e-12 * nc)
    assert np.linalg.norm(vv.T @ vv - np.eye(K), 2) <= 1e-10
    assert np.linalg.norm(c @ vv - vv * lam, 2) <= 1e-10 * nc
    assert flags.item() == 0


# ---- precision variants of the FP32-tensor kernels ---------------------------
# bf16 inputs carry a relative rounding error u = 2^-9 per entry; a J-term
# contraction with random signs then errs by about u/sqrt(3) ~ 2.3e-3 of its
# column scale, so 1e-2 bounds it; the split-bf16 power step keeps about 16
# mantissa bits (5e-5).
@pytest.mark.parametrize("dims", DIMS)
def test_bf16_sketch_power_ttm(dims):
    x, _, _ = tucker_tensor(dims, tuple(min(3, d) for d in dims), seed=24, noise=0.3, dtype=np.float32)
    src = _flat(x, np.float32)
    x64 = x.astype(np.float64)
    rng = np.random.default_rng(5)
    for n, view in _views(dims):
        J = view[0] * view[2]
        K = min(11, dims[n], J)
        y, _ = api.sketch(src, view, K, seed=5, mode=n, tag=2, precision="bf16")
        want = unfold(x64, n) @ philox.omega_unfolding(5, n, 2, x64.shape, K)
        _close_cols(y.cpu().numpy(), want, 1e-2)
        q, _ = np.linalg.qr(rng.standard_normal((dims[n], K)))
        y = api.power(src, view, torch.from_numpy(q.astype(np.float32)).cuda(), precision="bf16").cpu().numpy()
        a = unfold(x64, n)
        # the tensor enters both products rounded to bf16 (unit roundoff 2^-9)
        _close_cols(y, a @ (a.T @ q.astype(np.float32).astype(np.float64)), 2.0 ** -8)
        m = rng.standard_normal((dims[n], K)).astype(np.float32)
        out, gram, _ = api.ttm(src, view, K, torch.from_numpy(m).cuda(), want_gram=True, precision="bf16")
        want = o_ttm(x64, m.astype(np.float64).T, n)
        got = out.cpu().numpy().reshape(want.shape, order="F")
        _close_cols(unfold(got, n).T, unfold(want, n).T, 1e-2)
        b = unfold(want, n)
        _close_cols(gram.cpu().numpy(), b @ b.T, 1e-2)


@pytest.mark.parametrize("dims", DIMS)
def test_tiled_kernels_fp32(dims):
    # the workgroup-tiled kernels (used when a shape does not fit the
    # wave-private ones) against the same oracle definitions
    with api.kernel_family("tiled"):
        _tiled_kernels_fp32(dims)


def _tiled_kernels_fp32(dims):
    x, _, _ = tucker_tensor(dims, tuple(min(3, d) for d in dims), seed=25, noise=0.3, dtype=np.float32)
    src = _flat(x, np.float32)
    x64 = x.astype(np.float64)
    rng = np.random.default_rng(6)
    for n, view in _views(dims):
        J = view[0] * view[2]
        K = min(11, dims[n], J)
        y, _ = api.sketch(src, view, K, seed=5, mode=n, tag=2)
        _close_cols(y.cpu().numpy(), unfold(x64, n) @ philox.omega_unfolding(5, n, 2, x64.shape, K), 2e-5)
        q, _ = np.linalg.qr(rng.standard_normal((dims[n], K)))
        q = q.astype(np.float32)
        y = api.power(src, view, torch.from_numpy(q).cuda()).cpu().numpy()
        a = unfold(x64, n)
        _close_cols(y, a @ (a.T @ q.astype(np.float64)), 3e-5)


# e4m3 sketch: every product x w is formed from e4m3 inputs (unit roundoff
# u = 2^-4 for both operands, the tensor scaled by a power of two per
# 32-column block, which is exact), so |dY_ik| <= (2u + u^2) (|X| |Omega|)_ik
# plus the subnormal floors: 2^-10 absolute for Omega entries below 2^-6 and
# 2^-10 / 128 of the block's largest magnitude for the scaled tensor, and
# FP32 accumulation (2^-20 of the same sum at these lengths).
@pytest.mark.parametrize("dims", DIMS)
def test_fp8_sketch_within_rounding_bound(dims):
    x, _, _ = tucker_tensor(dims, tuple(min(3, d) for d in dims), seed=26, noise=0.3, dtype=np.float32)
    src = _flat(x, np.float32)
    x64 = x.astype(np.float64)
    n, view = _views(dims)[0]                   # contiguous: the e4m3 column kernel
    K = min(11, dims[0], view[2])
    y, _ = api.sketch(src, view, K, seed=5, mode=n, tag=2, precision="fp8")
    a = unfold(x64, n)
    om = philox.omega_unfolding(5, n, 2, x64.shape, K)
    want = a @ om
    u = 2.0 ** -4
    bound = ((2 * u + u * u + 2.0 ** -20) * (np.abs(a) @ np.abs(om))
             + 2.0 ** -10 * (np.abs(a) @ np.ones_like(om))
             + 2.0 ** -17 * np.max(np.abs(a)) * (np.ones_like(a) @ np.abs(om)))
    got = y.cpu().numpy()
    assert np.all(np.abs(got - want) <= bound)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"[fp8] sketch {dims}: relative error {rel:.3e}", flush=True)
    assert rel <= 0.05                          # about u / sqrt(3) for random-sign rounding


# ---- modes of 257-512 rows: four waves share each column block -------------
# Shapes whose mode has more rows than one wave holds (256): the row-split
# variants of the wave kernels, each wave on its own rows, Z = S^T M summed
# across the waves.  (300, 9, 40): I = 300 contiguous; (7, 420, 11): I = 420
# strided (L = 7); (500, 13, 9): the exact 500-row variant at K = 30.
TALL = [((300, 9, 40), 0, 11), ((300, 9, 40), 0, 40), ((7, 420, 11), 1, 30), ((500, 13, 9), 0, 30)]


@pytest.mark.parametrize("dims,n,K", TALL)
@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_tall_mode_steps(dims, n, K, precision):
    x, _, _ = tucker_tensor(dims, tuple(min(3, d) for d in dims), seed=27, noise=0.3, dtype=np.float32)
    src = _flat(x, np.float32)
    x64 = x.astype(np.float64)
    view = _views(dims)[n][1]
    rng = np.random.default_rng(7)
    a = unfold(x64, n)
    # f32: FP32 products over J terms; bf16: as test_bf16_sketch_power_ttm
    t_sk, t_pw, t_tt = (2e-5, 3e-5, 2e-5) if precision == "f32" else (1e-2, 2.0 ** -8, 1e-2)
    y, nrm = api.sketch(src, view, K, seed=5, mode=n, tag=2, want_norm=True, precision=precision)
    _close_cols(y.cpu().numpy(), a @ philox.omega_unfolding(5, n, 2, x64.shape, K), t_sk)
    assert abs(nrm.item() - float(np.sum(x64 ** 2))) <= 1e-6 * np.sum(x64 ** 2)
    q, _ = np.linalg.qr(rng.standard_normal((dims[n], K)))
    q = q.astype(np.float32)
    y = api.power(src, view, torch.from_numpy(q).cuda(), precision=precision).cpu().numpy()
    _close_cols(y, a @ (a.T @ q.astype(np.float64)), t_pw)
    m = rng.standard_normal((dims[n], K)).astype(np.float32)
    out, gram, _ = api.ttm(src, view, K, torch.from_numpy(m).cuda(), want_gram=True, precision=precision)
    want = o_ttm(x64, m.astype(np.float64).T, n)
    got = out.cpu().numpy().reshape(want.shape, order="F")
    _close_cols(unfold(got, n).T, unfold(want, n).T, t_tt)
    b = unfold(want, n)
    _close_cols(gram.cpu().numpy(), b @ b.T, t_tt)


# (K, R, J): every row-tile count (R up to 16, 32, 48, 64) and step bound
# (K up to 16, 32, 48, 64), a ragged last chunk, one column, one whole
# chunk, and enough columns for several chunks per wave of the full grid
TRUNC_CASES = [(35, 25, 8013), (16, 16, 1000), (32, 20, 777), (48, 40, 3001), (64, 64, 5000),
               (64, 50, 64), (7, 3, 1), (35, 25, 600011), (13, 13, 129)]


@pytest.mark.parametrize("K,R,J", TRUNC_CASES + [(32, 30, 2500), (12, 5, 130), (3, 1, 70)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_truncate_rotated(K, R, J, dtype):
    """Algorithm 8 step 4 in the rotated layout: out = M^T B, row r of out
    contiguous, on the truncation kernel, against the float64 product."""
    if dtype == np.float64 and K > 32:
        pytest.skip("FP64 truncation kernel takes K <= 32")
    rng = np.random.default_rng(K * 1000 + R + J)
    b = rng.standard_normal((K, J)).astype(dtype)
    m = rng.standard_normal((K, R)).astype(dtype)
    bd = torch.from_numpy(np.ascontiguousarray(b.reshape(-1, order="F"))).cuda()
    out = api.truncate_rotated(bd, K, J, torch.from_numpy(m).cuda())
    got = out.cpu().numpy().astype(np.float64).reshape(R, J)
    want = m.astype(np.float64).T @ b.astype(np.float64)
    # a sum of K products in the data's precision: K eps sum |m| |b| bounds it
    bound = K * (6e-8 if dtype == np.float32 else 1.2e-16) * (np.abs(m).T @ np.abs(b)) + 1e-300
    assert np.all(np.abs(got - want) <= bound)


def test_truncate_rotated_rejects():
    b = torch.zeros(65 * 10, dtype=torch.float32, device="cuda")
    with pytest.raises(api.L.RhosvdError):
        api.truncate_rotated(b, 65, 10, torch.zeros(65, 3, dtype=torch.float32, device="cuda"))
    b = torch.zeros(33 * 10, dtype=torch.float64, device="cuda")
    with pytest.raises(api.L.RhosvdError):
        api.truncate_rotated(b, 33, 10, torch.zeros(33, 3, dtype=torch.float64, device="cuda"))
