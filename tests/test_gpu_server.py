"""The continuous-batching request loop (GPU only).

Requests of uneven shape, order, precision and power count are submitted
while others run; each result must equal, bit for bit, what a single
rhosvd_decompose of the same request computes alone, and match the FP64
oracle within the stated tolerances.  Admission respects the pool: a pool
that holds one request at a time still finishes everything, in order.
"""
import time

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.tucker import r_sthosvd as o_rst  # noqa: E402
from paper_2001_07124_amd import _lib as L  # noqa: E402
from paper_2001_07124_amd import api  # noqa: E402
from paper_2001_07124_amd.inputs import tucker_tensor  # noqa: E402

REQS = [
    # dims, ranks, q, precision
    ((90, 70, 60), (8, 7, 6), 1, "f32"),
    ((48, 40, 36, 30), (5, 4, 4, 3), 0, "bf16"),
    ((120, 64, 50), (10, 8, 9), 1, "bf16"),
    ((33, 29, 31), (6, 5, 4), 0, "f32"),
    ((64, 64, 64, 16), (8, 8, 6, 4), 1, "f32"),
    ((150, 40, 40), (12, 6, 6), 1, "bf16"),
]


def _tensors():
    return [tucker_tensor(d, r, seed=70 + i, noise=1e-2, dtype=np.float32)[0]
            for i, (d, r, _, _) in enumerate(REQS)]


def _same(a, b):
    assert torch.equal(a.core, b.core)
    for fa, fb in zip(a.factors, b.factors):
        assert torch.equal(fa, fb)
    assert torch.equal(a.report_buf, b.report_buf)


def test_server_results_equal_alone_and_match_oracle():
    xs = _tensors()
    xds = [api.to_device(x) for x in xs]
    srv = api.Server(pool_bytes=1 << 30, slots=4)
    tickets = []
    for i, (xd, (d, r, q, prec)) in enumerate(zip(xds, REQS)):
        tickets.append(srv.submit(xd, r, p=6, q=q, seed=i, precision=prec))
        time.sleep(0.002)                         # arrivals spread while earlier ones run
    srv.drain()
    for i, ((ticket, res), xd, x, (d, r, q, prec)) in enumerate(zip(tickets, xds, xs, REQS)):
        state, (t0, t1, t2) = srv.poll(ticket)
        assert state == L.REQ_DONE and t0 <= t1 <= t2
        alone = api.decompose(xd, r, p=6, q=q, seed=i, precision=prec)
        torch.cuda.synchronize()
        _same(res, alone)
        ref = o_rst(x.astype(np.float64), r, 6, q, seed=i)
        tol = 1e-5 if prec == "f32" else 1e-4
        assert abs(res.rel_error - ref.rel_error) <= tol, (i, res.rel_error, ref.rel_error)
        srv.release(ticket)
    srv.close()


def test_server_admits_by_pool_footprint():
    xs = _tensors()[:3]
    xds = [api.to_device(x) for x in xs]
    sizes = []
    for xd, (d, r, q, prec) in zip(xds, REQS[:3]):
        dec = api.Decomposer(d, r, p=6, q=q, precision=prec)
        sizes.append(dec.ws_bytes)
    # room for the largest request only: whatever runs together fits the pool
    pool = (max(sizes) + 4095) // 4096 * 4096
    srv = api.Server(pool_bytes=pool, slots=4)
    tickets = [srv.submit(xd, r, p=6, q=q, seed=i, precision=prec)
               for i, (xd, (d, r, q, prec)) in enumerate(zip(xds, REQS[:3]))]
    srv.drain()
    spans = [srv.poll(t)[1] for t, _ in tickets]
    for t0, t1, t2 in spans:
        assert t0 <= t1 <= t2
    for _, start, _ in spans:
        live = sum((sz + 255) // 256 * 256 for sz, (_, s1, s2) in zip(sizes, spans) if s1 <= start < s2)
        assert live <= pool
    with pytest.raises(L.RhosvdError):            # a request larger than the whole pool
        big = api.to_device(tucker_tensor((200, 200, 200), (8, 8, 8), seed=1, dtype=np.float32)[0])
        srv.submit(big, (8, 8, 8), p=6, q=1)
    srv.close()
