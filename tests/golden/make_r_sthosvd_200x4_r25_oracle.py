"""Write the FP64 oracle's result for the 200^4 R-STHOSVD workload.

    python tests/golden/make_r_sthosvd_200x4_r25_oracle.py OUT.npz

The workload: 200^4 FP32 (6.4 GB), core 25^4 ~ N(0,1), orthonormal factors,
noise 1e-3, data seed 13; R-STHOSVD (Algorithm 8 with Algorithm 1 per mode)
with ranks 25, p = 10 (K = 35), q = 1, Omega seed 0.  The tensor is drawn by
paper_2001_07124_amd.inputs and upcast to FP64; everything else is the
unmodified oracle (oracle.tucker.r_sthosvd, oracle.philox): the explicit
relative error of Section 8, the per-mode singular values and the
sign-canonical factors, plus the whole mode-1 sketch Y = X_(1) Omega_1 (all
35 columns) and a fingerprint of the input (its squared norm, sum and 64
sampled entries) so that a reader can check it drew the same tensor.

The oracle needs about 60 GB of host memory at this size (the FP64 tensor,
its reconstruction and their difference inside the explicit residual), more
than a 64 GB build host can spare, so the file is produced on a machine with
more memory; the stored values come from this script and the oracle only.
"""
import sys
import time

import numpy as np

sys.path.insert(0, __file__.rsplit("/tests/", 1)[0])

from oracle import philox  # noqa: E402
from oracle.tensor_ops import unfold  # noqa: E402
from oracle.tucker import r_sthosvd  # noqa: E402
from paper_2001_07124_amd.inputs import make_workload  # noqa: E402

NAME = "r_sthosvd_200x4_r25"


def main(out):
    t0 = time.time()
    print(f"[golden] drawing {NAME}", flush=True)
    x32, w = make_workload(NAME)
    dims = tuple(w["dims"])
    rng = np.random.default_rng(77)
    idx = [tuple(int(rng.integers(0, d)) for d in dims) for _ in range(64)]
    samples = np.array([float(x32[i]) for i in idx])
    x = x32.astype(np.float64)
    del x32
    fp_norm2 = float(np.vdot(x.reshape(-1, order="F"), x.reshape(-1, order="F")))
    fp_sum = float(np.sum(x))
    K = w["target"][0] + w["p"]
    print(f"[golden] mode-1 sketch, {time.time() - t0:.0f} s", flush=True)
    om = philox.omega_unfolding(w["seed"], 0, philox.TAG_R_STHOSVD, dims, K)
    y1 = unfold(x, 0) @ om
    del om
    print(f"[golden] oracle R-STHOSVD, {time.time() - t0:.0f} s", flush=True)
    ref = r_sthosvd(x, w["target"], w["p"], w["q"], seed=w["seed"])
    print(f"[golden] E = {ref.rel_error:.10f} (identity {ref.rel_error_identity:.10f}), "
          f"{time.time() - t0:.0f} s", flush=True)
    np.savez(out, rel_error=ref.rel_error, rel_error_identity=ref.rel_error_identity,
             norm_x2=ref.norm_x2, norm_core2=ref.norm_core2,
             sigma=np.array(ref.sigma), factors=np.array(ref.factors), k_used=np.array(ref.k_used),
             y1=y1, fp_norm2=fp_norm2, fp_sum=fp_sum, fp_index=np.array(idx), fp_samples=samples,
             dims=np.array(dims), ranks=np.array(w["target"]), p=w["p"], q=w["q"], seed=w["seed"])
    print(f"[golden] wrote {out}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "r_sthosvd_200x4_r25_oracle.npz")
