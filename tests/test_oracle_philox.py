"""Pins for the oracle's Gaussian test matrices (oracle.philox).

* Philox4x32-10 against the published known-answer vectors (SC'11 /
  Random123) and against rocRAND's independent open-source engine.
* The 23-bit uniform map at its end points (exact in binary32).
* Box-Muller: the pair identity z0^2 + z1^2 = -2 ln u0 and the N(0,1)
  distribution (moments, Kolmogorov-Smirnov, column correlations).
* The Omega layout: e = k*J + j, prefix property, entry-wise access.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _read_kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(w, 16) for w in line.split()])
    return rows


def test_published_known_answers():
    rows = _read_kat()
    assert len(rows) == 3
    for r in rows:
        c, k, want = r[0:4], r[4:6], r[6:10]
        got = philox.philox4x32_10(*[np.array([v]) for v in c], k[0], k[1])
        assert [int(g[0]) for g in got] == want


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    out = tmp_path_factory.mktemp("rocrand") / "philox_ref"
    src = os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp")
    res = subprocess.run([hipcc, "-O1", src, "-o", str(out)], capture_output=True, text=True)
    if res.returncode != 0:
        pytest.skip("could not build rocRAND reference: " + res.stderr[-400:])
    return str(out)


def test_against_rocrand_engine(rocrand_ref):
    rng = np.random.default_rng(1234)
    n = 2000
    c = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    k = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    # a few structured counters as well: the ones the sketches actually use
    c[:10] = np.array([[q, 0, m, t] for q, m, t in
                       [(0, 0, 1), (1, 0, 2), (2, 3, 2), (5, 1, 1), (2**32 - 1, 2, 2),
                        (7, 15, 2), (123456, 0, 1), (99, 4, 2), (3, 3, 3), (4, 0, 0)]])
    lines = "\n".join(" ".join(str(int(v)) for v in list(c[i]) + list(k[i])) for i in range(n))
    res = subprocess.run([rocrand_ref], input=lines, capture_output=True, text=True, check=True)
    want = np.array([[int(w) for w in l.split()] for l in res.stdout.strip().splitlines()],
                    dtype=np.uint64)
    assert want.shape == (n, 4)
    for i in range(n):
        got = philox.philox4x32_10(*[np.array([c[i, j]]) for j in range(4)], int(k[i, 0]), int(k[i, 1]))
        assert [int(g[0]) for g in got] == [int(w) for w in want[i]]


def test_uniform_map_end_points():
    u = philox.uniform01(np.array([0, 511, 512, 0xFFFFFFFF], dtype=np.uint32))
    assert u[0] == 2.0 ** -24
    assert u[1] == 2.0 ** -24                 # low 9 bits are dropped
    assert u[2] == 3 * 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24
    # every value is exactly representable in binary32
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    w = np.random.default_rng(0).integers(0, 2**32, 100000, dtype=np.uint64).astype(np.uint32)
    uw = philox.uniform01(w)
    assert np.all(uw.astype(np.float32).astype(np.float64) == uw)
    assert np.all((uw > 0) & (uw < 1))


def test_box_muller_pair_identity():
    q = np.arange(1000, dtype=np.uint64)
    x0, x1, x2, x3 = philox.philox4x32_10(q, q * 0, q * 0 + 1, q * 0 + 2, 7, 0)
    z = philox.normals_for_quads(q, seed=7, mode=1, tag=2)
    u0, u2 = philox.uniform01(x0), philox.uniform01(x2)
    np.testing.assert_allclose(z[:, 0] ** 2 + z[:, 1] ** 2, -2 * np.log(u0), rtol=1e-12)
    np.testing.assert_allclose(z[:, 2] ** 2 + z[:, 3] ** 2, -2 * np.log(u2), rtol=1e-12)
    # angle comes from the second word of each pair
    u1 = philox.uniform01(x1)
    ang = np.mod(np.arctan2(z[:, 1], z[:, 0]), 2 * np.pi)
    np.testing.assert_allclose(ang, 2 * np.pi * u1, atol=1e-9)


def test_omega_is_standard_normal():
    om = philox.omega(seed=42, mode=0, tag=2, J=20000, K=20)
    v = om.reshape(-1)
    assert abs(v.mean()) < 4 / np.sqrt(v.size)
    assert abs(v.var() - 1.0) < 6 * np.sqrt(2.0 / v.size)
    assert stats.kstest(v, "norm").pvalue > 1e-3
    c = np.corrcoef(om.T)
    off = c[~np.eye(20, dtype=bool)]
    assert np.max(np.abs(off)) < 5 / np.sqrt(om.shape[0])


def test_omega_layout_and_prefix():
    J, K = 37, 9                       # J not a multiple of 4: quads straddle columns
    om = philox.omega(seed=3, mode=2, tag=2, J=J, K=K)
    assert om.shape == (J, K)
    small = philox.omega(seed=3, mode=2, tag=2, J=J, K=4)
    np.testing.assert_array_equal(small, om[:, :4])
    jj, kk = np.meshgrid(np.arange(J), np.arange(K), indexing="ij")
    ent = philox.omega_entries(3, 2, 2, J, jj.reshape(-1), kk.reshape(-1)).reshape(J, K)
    np.testing.assert_array_equal(ent, om)
    # linear index e = k*J + j: entry (j, k) is word e & 3 of quad e >> 2
    e = 5 * J + 11
    z = philox.normals_for_quads(np.array([e >> 2]), 3, 2, 2)[0]
    assert om[11, 5] == z[e & 3]


def test_omega_streams_differ():
    a = philox.omega(seed=0, mode=0, tag=2, J=500, K=8)
    b = philox.omega(seed=0, mode=1, tag=2, J=500, K=8)
    c = philox.omega(seed=0, mode=0, tag=1, J=500, K=8)
    d = philox.omega(seed=1, mode=0, tag=2, J=500, K=8)
    for other in (b, c, d):
        r = np.corrcoef(a.reshape(-1), other.reshape(-1))[0, 1]
        assert abs(r) < 0.1


def test_omega_unfolding_row_order():
    """Row j of omega_unfolding is generator row c, c the cyclic position of
    unfolding column j, both indices written out from their definitions
    (the paper's n-unfolding column index, Section 2, and the cyclic order
    i_{n+1}, ..., i_N, i_1, ..., i_{n-1})."""
    import itertools
    shape = (3, 4, 2, 5)
    K = 3
    for n in range(len(shape)):
        om = philox.omega_unfolding(11, n, 2, shape, K)
        J = int(np.prod(shape)) // shape[n]
        assert om.shape == (J, K)
        others = [m for m in range(len(shape)) if m != n]
        cyc = list(range(n + 1, len(shape))) + list(range(n))
        for idx in itertools.product(*[range(d) for d in shape]):
            j, stride = 0, 1
            for m in others:                     # paper: i_1 fastest, skipping n
                j += idx[m] * stride
                stride *= shape[m]
            c, stride = 0, 1
            for m in cyc:                        # cyclic: i_{n+1} fastest
                c += idx[m] * stride
                stride *= shape[m]
            for k in range(K):
                want = philox.omega_entries(11, n, 2, J, c, k)
                assert om[j, k] == want
    # mode 0 and the last mode: cyclic order equals the paper's order
    assert np.array_equal(philox.omega_unfolding(11, 0, 2, shape, K),
                          philox.omega(11, 0, 2, 40, K))
