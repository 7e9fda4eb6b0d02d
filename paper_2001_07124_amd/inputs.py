"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only *draws data*; it holds none of the decomposition's
arithmetic, and neither the GPU binding nor the oracle imports it.

Tensors are returned as NumPy arrays of shape (I_1, ..., I_N) in Fortran
(first-index-fastest) memory order, the layout the library consumes.

Recipes (Section 8 describes the paper's synthetic data):
* Low multilinear rank plus noise (eqs. noiselesstensor and noisytensor):
  X = G x_1 A_1 ... x_N A_N + gamma * N, with G ~ N(0,1) of shape ranks,
  A_n either orthonormal (Q of a Householder QR of an I_n x R_n Gaussian) or
  plain Gaussian, optionally scaled column-wise by decay**k, and N ~ N(0,1).
  Core and factors come from one generator seeded with [seed, 0]; the noise
  of the last-mode slab s comes from its own generator seeded with
  [seed, 1, s], so large tensors are produced slab by slab, in parallel,
  with a result independent of the chunking.
* Function tensor 1 / (i^5 + j^5 + k^5)^(1/5) (eq. funtensor) and the
  Hilbert tensor 1 / (i_1 + ... + i_N - N + 1) (eq. HilbertTensor), 1-based.
"""
from concurrent.futures import ThreadPoolExecutor
import math
import os

import numpy as np


def _factors(rng, dims, ranks, kind, decay):
    facs = []
    for d, r in zip(dims, ranks):
        m = rng.standard_normal((d, r))
        if kind == "orthonormal":
            m, _ = np.linalg.qr(m, mode="reduced")
        elif kind != "gaussian":
            raise ValueError("factor kind must be 'orthonormal' or 'gaussian'")
        if decay is not None:
            m = m * (float(decay) ** np.arange(r))
        facs.append(m)
    return facs


def tucker_tensor(dims, ranks, *, seed, factors="orthonormal", decay=None,
                  noise=0.0, dtype=np.float32, workers=None):
    """Low-multilinear-rank tensor plus i.i.d. Gaussian noise (see module doc).

    Returns (X, core, factor_list); X is Fortran-ordered of dtype `dtype`,
    core and factors are float64.
    """
    dims = tuple(int(d) for d in dims)
    ranks = tuple(int(r) for r in ranks)
    if len(dims) != len(ranks) or len(dims) < 2:
        raise ValueError("need matching dims and ranks, order >= 2")
    rng = np.random.default_rng([int(seed), 0])
    core = rng.standard_normal(ranks)
    facs = _factors(rng, dims, ranks, factors, decay)
    # t = core x_1 A_1 ... x_{N-1} A_{N-1}, kept with its last mode at rank R_N
    t = core
    for n in range(len(dims) - 1):
        t = np.moveaxis(np.tensordot(facs[n], t, axes=([1], [n])), 0, n)
    lead = int(np.prod(dims[:-1]))
    t_flat = np.asfortranarray(t).reshape(lead, ranks[-1], order="F")
    out = np.empty(dims, dtype=dtype, order="F")
    flat = out.reshape(lead, dims[-1], order="F")   # a view: Fortran order
    a_last = facs[-1]

    def slab(s):
        col = t_flat @ a_last[s]
        if noise:
            g = np.random.default_rng([int(seed), 1, s])
            col = col + float(noise) * g.standard_normal(lead)
        flat[:, s] = col

    nw = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=nw) as ex:
        list(ex.map(slab, range(dims[-1])))
    return out, core, facs


def function_tensor(n, dtype=np.float64):
    """X(i, j, k) = 1 / (i^5 + j^5 + k^5)^(1/5), i, j, k = 1..n."""
    i = np.arange(1, n + 1, dtype=np.float64)
    p = i ** 5
    x = (p[:, None, None] + p[None, :, None] + p[None, None, :]) ** -0.2
    return np.asfortranarray(x.astype(dtype))


def hilbert_tensor(dims, dtype=np.float64):
    """X(i_1..i_N) = 1 / (i_1 + ... + i_N - N + 1), 1-based indices."""
    grids = np.meshgrid(*[np.arange(1, d + 1, dtype=np.float64) for d in dims],
                        indexing="ij")
    x = 1.0 / (sum(grids) - len(dims) + 1.0)
    return np.asfortranarray(x.astype(dtype))


def snr_db(signal, noise_term):
    """SNR[dB] = 10 log10(||X||^2 / ||gamma N||^2) (Section 8)."""
    s = float(np.vdot(signal, signal))
    n = float(np.vdot(noise_term, noise_term))
    return 10.0 * math.log10(s / n)


# Named workloads.  Each returns the kwargs of tucker_tensor plus the
# decomposition parameters; the names describe the problem, not a run.
WORKLOADS = {
    # order-3 100^3, rank (10,10,10), orthonormal factors, 1e-3 noise, FP64,
    # random-projection HOSVD with p=5, q=0, Omega seed 0.
    "rp_hosvd_100x3_r10_f64": dict(
        dims=(100, 100, 100), ranks=(10, 10, 10), factors="orthonormal",
        decay=None, noise=1e-3, dtype=np.float64, data_seed=11,
        algo="rp_hosvd", target=(10, 10, 10), p=5, q=0, seed=0, prec="f64"),
    # order-3 500^3 FP32, exact rank 20 with factor scales 0.9^k, 1e-4 noise,
    # R-STHOSVD with R=20, p=10, q=1, modes 1->2->3.
    "r_sthosvd_500x3_r20_f32": dict(
        dims=(500, 500, 500), ranks=(20, 20, 20), factors="orthonormal",
        decay=0.9, noise=1e-4, dtype=np.float32, data_seed=12,
        algo="r_sthosvd", target=(20, 20, 20), p=10, q=1, seed=0, prec="f32"),
    # order-4 200^4 FP32 (6.4 GB), rank 25, orthonormal factors, 1e-3 noise,
    # R-STHOSVD with R=25, p=10, q=1.
    "r_sthosvd_200x4_r25": dict(
        dims=(200, 200, 200, 200), ranks=(25, 25, 25, 25), factors="orthonormal",
        decay=None, noise=1e-3, dtype=np.float32, data_seed=13,
        algo="r_sthosvd", target=(25, 25, 25, 25), p=10, q=1, seed=0, prec="f32"),
}


def make_workload(name, scale_dims=None):
    """Draw the tensor of a named workload; scale_dims overrides dims (for
    reduced-size parity runs with the same recipe)."""
    w = dict(WORKLOADS[name])
    dims = tuple(scale_dims) if scale_dims is not None else w["dims"]
    ranks = tuple(min(r, d) for r, d in zip(w["ranks"], dims))
    x, core, facs = tucker_tensor(dims, ranks, seed=w["data_seed"],
                                  factors=w["factors"], decay=w["decay"],
                                  noise=w["noise"], dtype=w["dtype"])
    return x, w


def batch_specs(count=512, seed=1, dim_range=(32, 256), rank_range=(4, 32), order=3):
    """Shapes of a batch of independent order-3 problems: every extent uniform
    in dim_range and every exact rank uniform in rank_range, capped by the
    extent and by the product of the other ranks (a multilinear rank cannot
    exceed it), drawn from one generator seeded with [seed, 2]."""
    rng = np.random.default_rng([int(seed), 2])
    out = []
    for _ in range(int(count)):
        dims = tuple(int(v) for v in rng.integers(dim_range[0], dim_range[1] + 1, size=order))
        ranks = [min(int(r), d) for r, d in
                 zip(rng.integers(rank_range[0], rank_range[1] + 1, size=order), dims)]
        changed = True
        while changed:
            changed = False
            for n in range(order):
                cap = int(np.prod([ranks[m] for m in range(order) if m != n]))
                if ranks[n] > cap:
                    ranks[n] = cap
                    changed = True
        out.append((dims, tuple(ranks)))
    return out


def batch_tensors(specs, *, seed=1, noise=1e-4, dtype=np.float32):
    """One low-rank-plus-noise tensor per spec (orthonormal factors), item i
    drawn with data seed 1000 seed + i."""
    return [tucker_tensor(d, r, seed=1000 * int(seed) + i, noise=noise, dtype=dtype, workers=4)[0]
            for i, (d, r) in enumerate(specs)]
