"""Python binding of the randomized HOSVD library (argument marshalling only).

PyTorch supplies device memory and the stream; every arithmetic step runs in
the HIP kernels of librhosvd.so.  Tensors follow the library layout: an
order-N tensor of extents (I_1, ..., I_N) is first-index-fastest, i.e. a torch
tensor with Fortran strides (see `to_device`), or a flat 1-D buffer plus
explicit `dims`.  Column-major matrices are returned as transposed views of
contiguous tensors, so `U.shape == (I_n, R_n)` with strides (1, I_n).
"""
import contextlib
import ctypes
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import _lib as L

_ctx_cache = {}


def _context(device_index):
    lib = L.load()
    c = _ctx_cache.get(device_index)
    if c is None:
        c = ctypes.c_void_p()
        L.check(lib.rhosvd_create(ctypes.byref(c), int(device_index)), "rhosvd_create")
        _ctx_cache[device_index] = c
    return c


@contextlib.contextmanager
def kernel_family(name, device_index=0):
    """Within the block, the context of `device_index` runs only the given
    streaming-kernel family ("tiled": the workgroup-tiled FP32/FP64 kernels;
    "auto": the default choice)."""
    code = {"auto": L.KERNELS_AUTO, "tiled": L.KERNELS_TILED}[name]
    lib = L.load()
    ctx = _context(device_index)
    L.check(lib.rhosvd_set_option(ctx, L.OPTION_KERNELS, code), "rhosvd_set_option")
    try:
        yield
    finally:
        L.check(lib.rhosvd_set_option(ctx, L.OPTION_KERNELS, L.KERNELS_AUTO), "rhosvd_set_option")


def _dtype_code(dt):
    if dt == torch.float32:
        return L.F32
    if dt == torch.float64:
        return L.F64
    raise TypeError("tensor dtype must be float32 or float64")


_PREC = {"f64": L.PREC_F64, "f32": L.PREC_F32, "bf16": L.PREC_BF16, "fp8": L.PREC_FP8}


def _prec_code(precision, dt):
    if precision is None:
        return L.PREC_F64 if dt == torch.float64 else L.PREC_F32
    return _PREC[precision]


def fortran_strides(dims):
    s, out = 1, []
    for d in dims:
        out.append(s)
        s *= int(d)
    return tuple(out)


def to_device(a, device="cuda"):
    """Copy a NumPy array to the device as a first-index-fastest torch tensor."""
    a = np.asarray(a)
    flat = torch.from_numpy(np.ascontiguousarray(a.reshape(-1, order="F")))
    dev = flat.to(device)
    return dev.as_strided(tuple(a.shape), fortran_strides(a.shape))


def empty_fortran(dims, dtype, device):
    n = int(np.prod(dims)) if len(dims) else 1
    flat = torch.empty(max(n, 1), dtype=dtype, device=device)
    return flat.as_strided(tuple(int(d) for d in dims), fortran_strides(dims))


def empty_colmajor(rows, cols, dtype, device):
    return torch.empty((int(cols), int(rows)), dtype=dtype, device=device).t()


def to_numpy_fortran(t):
    """Host copy of a first-index-fastest device tensor (shape preserved)."""
    dims = tuple(t.shape)
    n = int(np.prod(dims))
    flat = t.as_strided((n,), (1,)).cpu().numpy()
    return flat.reshape(dims, order="F")


def _check_fortran(x, dims):
    if not x.is_cuda:
        raise ValueError("x must be a device tensor")
    if dims is None:
        dims = tuple(x.shape)
        if x.dim() > 1 and x.stride() != fortran_strides(dims) and x.numel() > 1:
            raise ValueError("x must be first-index-fastest (Fortran strides); use to_device()")
    else:
        dims = tuple(int(d) for d in dims)
        if x.numel() != int(np.prod(dims)) or not (x.is_contiguous() or x.dim() == 1):
            raise ValueError("flat x must hold prod(dims) contiguous elements")
    return dims


def _stream(stream, device):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class Decomposition:
    core: torch.Tensor
    factors: List[torch.Tensor]
    report_buf: torch.Tensor
    order: int
    _report: Optional[L.Report] = field(default=None, repr=False)

    def report(self):
        """Host copy of the device report (synchronises the device)."""
        if self._report is None:
            torch.cuda.synchronize(self.report_buf.device)
            raw = self.report_buf.cpu().numpy().tobytes()
            self._report = L.Report.from_buffer_copy(raw)
        return self._report

    @property
    def rel_error(self):
        """E of Section 8: the explicit residual when the library computed
        it (see explicit_error), else the projection identity."""
        return float(L.load().rhosvd_report_rel_error(ctypes.byref(self.report())))

    @property
    def rel_error_identity(self):
        r = self.report()
        d = r.norm_x2 - r.norm_core2
        return float(np.sqrt(max(d, 0.0) / r.norm_x2))

    @property
    def explicit(self):
        return bool(self.report().flags & L.FLAG_E_EXPLICIT)

    @property
    def norm_x2(self):
        return self.report().norm_x2

    @property
    def norm_core2(self):
        return self.report().norm_core2

    @property
    def flags(self):
        return int(self.report().flags)

    @property
    def k_used(self):
        return [int(self.report().k_used[n]) for n in range(self.order)]

    def sigma(self, n):
        r = self.factors[n].shape[1]
        return np.array([self.report().sigma[n][i] for i in range(r)])


class Decomposer:
    """A reusable decomposition: validates once, owns workspace and outputs.

    run() enqueues the whole pipeline on the stream and returns at once;
    result() returns the output tensors and the report."""

    def __init__(self, dims, ranks, *, algo="r_sthosvd", p=10, q=1, seed=0,
                 dtype=torch.float32, precision=None, mode_order=None, device=None,
                 explicit_error=False, kr_sketch=False):
        self.lib = L.load()
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self.dev_index = self.device.index if self.device.index is not None else 0
        self.ctx = _context(self.dev_index)
        self.dims = tuple(int(d) for d in dims)
        self.ranks = tuple(int(r) for r in ranks)
        self.N = len(self.dims)
        self.dtype = dtype
        self._dims_c = (ctypes.c_int64 * self.N)(*self.dims)
        self._ranks_c = (ctypes.c_int32 * self.N)(*self.ranks)
        self._order_c = None if mode_order is None else (ctypes.c_int32 * self.N)(*mode_order)
        self.tensor = L.Tensor(self.N, self._dims_c, _dtype_code(dtype), None)
        algo_code = {"r_sthosvd": L.R_STHOSVD, "rp_hosvd": L.RP_HOSVD, "rp_hooi": L.RP_HOOI,
                     "r_pet": L.R_PET}[algo]
        flags = (L.OPT_EXPLICIT_ERROR if explicit_error else 0) | (L.OPT_KR_SKETCH if kr_sketch else 0)
        self.params = L.Params(algo_code, self._ranks_c, int(p), int(q), int(seed),
                               self._order_c, _prec_code(precision, dtype), flags)
        ws = ctypes.c_size_t(0)
        L.check(self.lib.rhosvd_workspace_size(ctypes.byref(self.tensor),
                                                ctypes.byref(self.params), ctypes.byref(ws)),
                "rhosvd_workspace_size")
        self.ws_bytes = int(ws.value)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.core = empty_fortran(self.ranks, dtype, self.device)
        self.factors = [empty_colmajor(i, r, dtype, self.device) for i, r in zip(self.dims, self.ranks)]
        self.report_buf = torch.zeros(ctypes.sizeof(L.Report), dtype=torch.uint8, device=self.device)
        self._fac_c = (ctypes.c_void_p * self.N)(*[f.data_ptr() for f in self.factors])
        self.out = L.Output(self.core.data_ptr(), self._fac_c, self.report_buf.data_ptr())

    def run(self, x, stream=None):
        _check_fortran(x, self.dims if x.dim() == 1 else None)
        if x.dtype != self.dtype or x.device != self.device:
            raise ValueError("x dtype/device differ from the planned ones")
        self.tensor.data = x.data_ptr()
        L.check(self.lib.rhosvd_decompose(self.ctx, ctypes.byref(self.tensor),
                                          ctypes.byref(self.params),
                                          ctypes.c_void_p(self.workspace.data_ptr()),
                                          self.ws_bytes, ctypes.byref(self.out),
                                          _stream(stream, self.device)),
                "rhosvd_decompose")

    def run_noalloc(self, x, stream=None):
        """The same decomposition through rhosvd_decompose_noalloc (the
        library's fixed per-device scratch instead of this object's
        workspace)."""
        _check_fortran(x, self.dims if x.dim() == 1 else None)
        if x.dtype != self.dtype or x.device != self.device:
            raise ValueError("x dtype/device differ from the planned ones")
        self.tensor.data = x.data_ptr()
        L.check(self.lib.rhosvd_decompose_noalloc(self.ctx, ctypes.byref(self.tensor),
                                                  ctypes.byref(self.params), ctypes.byref(self.out),
                                                  _stream(stream, self.device)),
                "rhosvd_decompose_noalloc")

    def result(self):
        return Decomposition(core=self.core, factors=self.factors, report_buf=self.report_buf,
                             order=self.N)


def decompose(x, ranks, *, algo="r_sthosvd", p=10, q=1, seed=0, precision=None,
              mode_order=None, dims=None, stream=None, explicit_error=False, kr_sketch=False):
    """One decomposition of x (device tensor, first-index-fastest);
    kr_sketch selects the structured (Khatri-Rao) test matrix of Section 5.1."""
    dims = _check_fortran(x, dims)
    d = Decomposer(dims, ranks, algo=algo, p=p, q=q, seed=seed, dtype=x.dtype,
                   precision=precision, mode_order=mode_order, device=x.device,
                   explicit_error=explicit_error, kr_sketch=kr_sketch)
    d.run(x, stream)
    return d.result()


def r_sthosvd(x, ranks, p=10, q=1, seed=0, **kw):
    """R-STHOSVD (Algorithm 8 with Algorithm 1 per mode)."""
    return decompose(x, ranks, algo="r_sthosvd", p=p, q=q, seed=seed, **kw)


def rp_hosvd(x, ranks, p=10, q=0, seed=0, **kw):
    """RP-HOSVD (Algorithm 6; the K-sized core is truncated by a small THOSVD)."""
    return decompose(x, ranks, algo="rp_hosvd", p=p, q=q, seed=seed, **kw)


def r_pet(x, ranks, p=10, seed=0, **kw):
    """R-PET (Algorithm 9): factor sketches and a core sketch of width
    S_n = min(2 K_n + 1, I_n), the core recovered by least squares."""
    return decompose(x, ranks, algo="r_pet", p=p, q=0, seed=seed, **kw)


def rp_hooi(x, ranks, sweeps=2, seed=0, **kw):
    """RP-HOOI (Algorithm 7) with `sweeps` sweeps from a Gaussian start."""
    return decompose(x, ranks, algo="rp_hooi", p=0, q=sweeps, seed=seed, **kw)


@dataclass
class AdaptiveDecomposition(Decomposition):
    ranks: tuple = ()
    met: tuple = ()


def decompose_adaptive(x, eps, *, kmax=32, q=1, seed=0, precision=None, dims=None, stream=None,
                       explicit_error=False, kr_sketch=False):
    """Fixed-precision R-STHOSVD: the ranks from the tolerance eps (Section
    5.1 with Algorithm 4's per-mode share eps^2 ||X||^2 / N), each mode
    sketched with K_n = min(kmax, I_n, J_n) columns.  Returns the core and
    factors at the chosen ranks plus `ranks` and `met` (per mode, whether its
    share of the tolerance was reached).  Synchronises the stream once per
    mode (the rank choice reads the eigenvalues on the host)."""
    lib = L.load()
    dims = _check_fortran(x, dims)
    dev = x.device
    N = len(dims)
    dims_c = (ctypes.c_int64 * N)(*dims)
    tensor = L.Tensor(N, dims_c, _dtype_code(x.dtype), x.data_ptr())
    flags = (L.OPT_EXPLICIT_ERROR if explicit_error else 0) | (L.OPT_KR_SKETCH if kr_sketch else 0)
    prm = L.AdaptiveParams(float(eps), int(kmax), int(q), int(seed), _prec_code(precision, x.dtype),
                           flags)
    ws = ctypes.c_size_t(0)
    L.check(lib.rhosvd_adaptive_workspace_size(ctypes.byref(tensor), ctypes.byref(prm),
                                               ctypes.byref(ws)), "rhosvd_adaptive_workspace_size")
    workspace = torch.empty(int(ws.value), dtype=torch.uint8, device=dev)
    caps = [min(int(kmax), d) for d in dims]
    fac_bufs = [torch.empty(d * c, dtype=x.dtype, device=dev) for d, c in zip(dims, caps)]
    core_buf = torch.empty(int(np.prod(caps)), dtype=x.dtype, device=dev)
    report_buf = torch.zeros(ctypes.sizeof(L.Report), dtype=torch.uint8, device=dev)
    fac_c = (ctypes.c_void_p * N)(*[f.data_ptr() for f in fac_bufs])
    out = L.Output(core_buf.data_ptr(), fac_c, report_buf.data_ptr())
    ranks_c = (ctypes.c_int32 * N)()
    met_c = (ctypes.c_int32 * N)()
    L.check(lib.rhosvd_decompose_adaptive(_context(dev.index or 0), ctypes.byref(tensor),
                                          ctypes.byref(prm), ctypes.c_void_p(workspace.data_ptr()),
                                          int(ws.value), ctypes.byref(out), ranks_c, met_c,
                                          _stream(stream, dev)),
            "rhosvd_decompose_adaptive")
    ranks = tuple(int(r) for r in ranks_c)
    factors = [f[: d * r].as_strided((d, r), (1, d)) for f, d, r in zip(fac_bufs, dims, ranks)]
    core = core_buf[: int(np.prod(ranks))].as_strided(ranks, fortran_strides(ranks))
    return AdaptiveDecomposition(core=core, factors=factors, report_buf=report_buf, order=N,
                                 ranks=ranks, met=tuple(bool(m) for m in met_c))


# ---- step-level calls (one hot-path step each) -------------------------------

def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _step_ws(I, K, J, device):
    n = L.load().rhosvd_step_workspace_size(int(I), int(K), int(J))
    return torch.empty(int(n), dtype=torch.uint8, device=device), int(n)


def omega_fill(seed, mode, tag, J, K, dtype=torch.float32, device="cuda"):
    lib = L.load()
    dev = torch.device(device)
    out = empty_colmajor(J, K, dtype, dev)
    L.check(lib.rhosvd_omega_fill(_context(dev.index or 0), int(seed), int(mode), int(tag), int(J),
                                  int(K), _dtype_code(dtype), _ptr(out), _stream(None, dev)),
            "rhosvd_omega_fill")
    return out


def sketch(src, view, K, seed, mode, tag, want_norm=False, precision=None):
    """Y = S_(n) Omega for the view (L, I, T) of the flat device tensor src."""
    lib = L.load()
    Lv, I, T = (int(v) for v in view)
    dev = src.device
    y = empty_colmajor(I, K, torch.float64, dev)
    nrm = torch.zeros(1, dtype=torch.float64, device=dev) if want_norm else None
    ws, nb = _step_ws(I, K, Lv * T, dev)
    L.check(lib.rhosvd_sketch(_context(dev.index or 0), _ptr(src), _dtype_code(src.dtype),
                              _prec_code(precision, src.dtype), Lv, I, T, int(K), int(seed), int(mode),
                              int(tag), _ptr(y), _ptr(nrm), _ptr(ws), nb, _stream(None, dev)),
            "rhosvd_sketch")
    return y, nrm


def sketch_kr(src, view, K, tables, ext, want_norm=False, precision=None):
    """Y = S_(n) Omega with the structured test matrix: the view's column
    index split over ext (fastest first), Omega(j, k) = prod_q tables[q](i_q, k)
    with tables[q] device ext[q] x K column-major in src's dtype."""
    lib = L.load()
    Lv, I, T = (int(v) for v in view)
    dev = src.device
    y = empty_colmajor(I, K, torch.float64, dev)
    nrm = torch.zeros(1, dtype=torch.float64, device=dev) if want_norm else None
    ws, nb = _step_ws(I, K, Lv * T, dev)
    nq = len(tables)
    tabs_c = (ctypes.c_void_p * nq)(*[t.data_ptr() for t in tables])
    ext_c = (ctypes.c_int64 * nq)(*[int(e) for e in ext])
    L.check(lib.rhosvd_sketch_kr(_context(dev.index or 0), _ptr(src), _dtype_code(src.dtype),
                                 _prec_code(precision, src.dtype), Lv, I, T, int(K), tabs_c, ext_c,
                                 nq, _ptr(y), _ptr(nrm), _ptr(ws), nb, _stream(None, dev)),
            "rhosvd_sketch_kr")
    return y, nrm


def sketch_all(src, dims, K, seed, tag=1, want_norm=False):
    """Y_n = X_(n) Omega_n for every mode n from one read of the flat device
    tensor src (dims first-index-fastest).  Returns ([Y_n], norm2)."""
    lib = L.load()
    N = len(dims)
    dev = src.device
    dims_c = (ctypes.c_int64 * N)(*[int(d) for d in dims])
    k_c = (ctypes.c_int32 * N)(*[int(k) for k in K])
    nb = int(lib.rhosvd_sketch_all_workspace_size(N, dims_c, k_c, _dtype_code(src.dtype)))
    if nb == 0:
        raise L.RhosvdError(L.EUNSUPPORTED, "rhosvd_sketch_all_workspace_size")
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    total = sum(int(d) * int(k) for d, k in zip(dims, K))
    y = torch.empty(total, dtype=torch.float64, device=dev)
    nrm = torch.zeros(1, dtype=torch.float64, device=dev) if want_norm else None
    L.check(lib.rhosvd_sketch_all(_context(dev.index or 0), _ptr(src), _dtype_code(src.dtype), N,
                                  dims_c, k_c, int(seed), int(tag), _ptr(y), _ptr(nrm), _ptr(ws), nb,
                                  _stream(None, dev)), "rhosvd_sketch_all")
    out, off = [], 0
    for d, k in zip(dims, K):
        out.append(y[off: off + int(d) * int(k)].view(int(k), int(d)).t())
        off += int(d) * int(k)
    return out, nrm


def power(src, view, q_mat, precision=None):
    """Y = S_(n) (S_(n)^T Q) for Q (I x K, column-major device matrix)."""
    lib = L.load()
    Lv, I, T = (int(v) for v in view)
    K = int(q_mat.shape[1])
    dev = src.device
    qc = q_mat.t().contiguous()
    y = empty_colmajor(I, K, torch.float64, dev)
    ws, nb = _step_ws(I, K, Lv * T, dev)
    L.check(lib.rhosvd_power(_context(dev.index or 0), _ptr(src), _dtype_code(src.dtype),
                             _prec_code(precision, src.dtype), Lv, I, T, K, _ptr(qc), _ptr(y), _ptr(ws),
                             nb, _stream(None, dev)), "rhosvd_power")
    return y


def ttm(src, view, kout, m=None, want_gram=False, want_norm=False, precision=None):
    """out = S x_n M^T (folded), optional Gram of its unfolding and ||out||^2."""
    lib = L.load()
    Lv, I, T = (int(v) for v in view)
    dev = src.device
    mc = m.t().contiguous() if m is not None else None
    out = torch.empty(Lv * int(kout) * T, dtype=src.dtype, device=dev)
    gram = empty_colmajor(kout, kout, torch.float64, dev) if want_gram else None
    nrm = torch.zeros(1, dtype=torch.float64, device=dev) if want_norm else None
    ws, nb = _step_ws(I, kout, Lv * T, dev)
    L.check(lib.rhosvd_ttm(_context(dev.index or 0), _ptr(src), _dtype_code(src.dtype),
                           _prec_code(precision, src.dtype), Lv, I, T, int(kout), _ptr(mc), _ptr(out),
                           _ptr(gram), _ptr(nrm), _ptr(ws), nb, _stream(None, dev)), "rhosvd_ttm")
    return out, gram, nrm


def truncate_rotated(b, K, J, m):
    """out (R x J row-major) = M^T B for B = K x J column-major (flat device
    tensor) and M = K x R (a device matrix), on the rotated truncation
    kernel."""
    lib = L.load()
    dev = b.device
    R = int(m.shape[1])
    mc = m.t().contiguous()
    out = torch.empty(R * int(J), dtype=b.dtype, device=dev)
    L.check(lib.rhosvd_truncate_rotated(_context(dev.index or 0), _dtype_code(b.dtype), _ptr(b), int(K),
                                        int(J), _ptr(mc), R, _ptr(out), _stream(None, dev)),
            "rhosvd_truncate_rotated")
    return out


def orthonormalize(y, dtype=torch.float32):
    """Q of CholeskyQR2 for Y (I x K float64 column-major device matrix)."""
    lib = L.load()
    I, K = (int(v) for v in y.shape)
    dev = y.device
    yc = y.t().contiguous()
    q = empty_colmajor(I, K, dtype, dev)
    work = torch.empty(2 * I * K, dtype=torch.float64, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    L.check(lib.rhosvd_orthonormalize(_context(dev.index or 0), _ptr(yc), I, K, _dtype_code(dtype),
                                      _ptr(q), _ptr(work), _ptr(flags), _stream(None, dev)),
            "rhosvd_orthonormalize")
    q64 = work[: I * K].view(K, I).t()
    return q, q64, flags


def sym_evd(c):
    """Eigen-decomposition of a symmetric K x K float64 device matrix."""
    lib = L.load()
    K = int(c.shape[0])
    dev = c.device
    cc = c.t().contiguous()
    v = empty_colmajor(K, K, torch.float64, dev)
    lam = torch.empty(K, dtype=torch.float64, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    L.check(lib.rhosvd_sym_evd(_context(dev.index or 0), _ptr(cc), K, _ptr(v), _ptr(lam),
                               _ptr(flags), _stream(None, dev)), "rhosvd_sym_evd")
    return v, lam, flags


# ---- batched decomposition ----------------------------------------------------

class Batch:
    """R-STHOSVD of many small tensors, one launch per step for the whole
    batch, replayed from a HIP graph (rhosvd_batch_*).

    items: list of (x, ranks, p, q, seed, precision) with x a
    first-index-fastest device tensor; outputs are allocated here."""

    def __init__(self, items, autotune=True, stream=None):
        self.lib = L.load()
        if not items:
            raise ValueError("empty batch")
        dev = items[0][0].device
        self.device = dev
        self.ctx = _context(dev.index or 0)
        n = len(items)
        self._keep = []
        tens = (L.Tensor * n)()
        prms = (L.Params * n)()
        outs = (L.Output * n)()
        self.results = []
        for i, (x, ranks, p, q, seed, prec) in enumerate(items):
            dims = _check_fortran(x, None)
            N = len(dims)
            dims_c = (ctypes.c_int64 * N)(*dims)
            ranks_c = (ctypes.c_int32 * N)(*[int(r) for r in ranks])
            tens[i] = L.Tensor(N, dims_c, _dtype_code(x.dtype), x.data_ptr())
            prms[i] = L.Params(L.R_STHOSVD, ranks_c, int(p), int(q), int(seed), None,
                               _prec_code(prec, x.dtype), 0)
            core = empty_fortran(tuple(int(r) for r in ranks), x.dtype, dev)
            facs = [empty_colmajor(d, r, x.dtype, dev) for d, r in zip(dims, ranks)]
            rep = torch.zeros(ctypes.sizeof(L.Report), dtype=torch.uint8, device=dev)
            fac_c = (ctypes.c_void_p * N)(*[f.data_ptr() for f in facs])
            outs[i] = L.Output(core.data_ptr(), fac_c, rep.data_ptr())
            self._keep += [x, dims_c, ranks_c, fac_c]
            self.results.append(Decomposition(core=core, factors=facs, report_buf=rep, order=N))
        self._tens, self._prms, self._outs = tens, prms, outs
        self.handle = ctypes.c_void_p()
        ws = ctypes.c_size_t(0)
        L.check(self.lib.rhosvd_batch_create(self.ctx, n, tens, prms, outs,
                                             ctypes.byref(self.handle), ctypes.byref(ws)),
                "rhosvd_batch_create")
        self.ws_bytes = int(ws.value)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        L.check(self.lib.rhosvd_batch_bind(self.handle, ctypes.c_void_p(self.workspace.data_ptr()),
                                           self.ws_bytes, 1 if autotune else 0,
                                           _stream(stream, dev)), "rhosvd_batch_bind")

    @property
    def launches(self):
        return int(self.lib.rhosvd_batch_launches(self.handle))

    def run(self, stream=None, use_graph=True):
        L.check(self.lib.rhosvd_batch_run(self.handle, 1 if use_graph else 0,
                                          _stream(stream, self.device)), "rhosvd_batch_run")

    def close(self):
        if self.handle:
            self.lib.rhosvd_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving --------------------------------------------------------------------

class Server:
    """Continuous-batching request loop (rhosvd_server_*): requests queue in
    arrival order and run on `slots` streams as slots and pool memory free up.

    pool_bytes of device memory are allocated here (torch) and handed to the
    library as the workspace budget."""

    def __init__(self, pool_bytes, slots=8, device=None):
        self.lib = L.load()
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        idx = self.device.index if self.device.index is not None else 0
        self.ctx = _context(idx)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        self.handle = ctypes.c_void_p()
        L.check(self.lib.rhosvd_server_create(self.ctx, idx, ctypes.c_void_p(self.pool.data_ptr()),
                                              int(pool_bytes), int(slots), ctypes.byref(self.handle)),
                "rhosvd_server_create")
        self._live = {}

    def submit(self, x, ranks, *, algo="r_sthosvd", p=10, q=1, seed=0, precision=None,
               explicit_error=False, outputs=None):
        """Queue a decomposition of the device tensor x; returns (ticket,
        Decomposition) whose buffers are filled when the ticket is done."""
        dims = _check_fortran(x, None)
        N = len(dims)
        dims_c = (ctypes.c_int64 * N)(*dims)
        ranks_c = (ctypes.c_int32 * N)(*[int(r) for r in ranks])
        t = L.Tensor(N, dims_c, _dtype_code(x.dtype), x.data_ptr())
        algo_code = {"r_sthosvd": L.R_STHOSVD, "rp_hosvd": L.RP_HOSVD, "rp_hooi": L.RP_HOOI,
                     "r_pet": L.R_PET}[algo]
        prm = L.Params(algo_code, ranks_c, int(p), int(q), int(seed), None,
                       _prec_code(precision, x.dtype), L.OPT_EXPLICIT_ERROR if explicit_error else 0)
        if outputs is None:
            core = empty_fortran(tuple(int(r) for r in ranks), x.dtype, self.device)
            facs = [empty_colmajor(d, r, x.dtype, self.device) for d, r in zip(dims, ranks)]
            rep = torch.zeros(ctypes.sizeof(L.Report), dtype=torch.uint8, device=self.device)
            outputs = Decomposition(core=core, factors=facs, report_buf=rep, order=N)
        fac_c = (ctypes.c_void_p * N)(*[f.data_ptr() for f in outputs.factors])
        out = L.Output(outputs.core.data_ptr(), fac_c, outputs.report_buf.data_ptr())
        ticket = ctypes.c_uint64(0)
        L.check(self.lib.rhosvd_server_submit(self.handle, ctypes.byref(t), ctypes.byref(prm),
                                              ctypes.byref(out), ctypes.byref(ticket)),
                "rhosvd_server_submit")
        self._live[int(ticket.value)] = (x, outputs)
        return int(ticket.value), outputs

    def poll(self, ticket):
        """(state, (t_submit, t_start, t_done) in ms); state is L.REQ_*."""
        st = ctypes.c_int32(0)
        times = (ctypes.c_double * 3)()
        L.check(self.lib.rhosvd_server_poll(self.handle, int(ticket), ctypes.byref(st), times),
                "rhosvd_server_poll")
        return int(st.value), (times[0], times[1], times[2])

    def release(self, ticket):
        L.check(self.lib.rhosvd_server_release(self.handle, int(ticket)), "rhosvd_server_release")
        self._live.pop(int(ticket), None)

    def drain(self):
        L.check(self.lib.rhosvd_server_drain(self.handle), "rhosvd_server_drain")

    def close(self):
        if self.handle:
            self.lib.rhosvd_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
