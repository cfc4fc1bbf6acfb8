"""The QR entry point that allocates nothing (its scratch is a static device
array) against the context-based kdqmc_qr_f64 whose kernels it shares: two
calls in a row, the second smaller, each bitwise equal; and its limits."""
import numpy as np
import pytest

import seeded_inputs as si
from gpu_helpers import chain, dev, say, torch

pytestmark = pytest.mark.gpu


def test_noalloc_qr_equals_context_qr(gpu_lib):
    from paper_2608_03894_amd import kdqmc
    t = torch()
    ch = chain(12, -4.0, 1.0)           # N = 432: the context QR's row stride
    N = ch.N
    for n in (432, 100):                # two calls in a row, the second smaller
        say("noalloc QR n", n)
        a = si.random_dense(N, 500 + n)
        A1, A2 = dev(a), dev(a)
        Q1 = t.zeros((N, N), dtype=t.float64, device="cuda:0")
        Q2 = t.full((N, N), 7.0, dtype=t.float64, device="cuda:0")
        ch.qr_f64(n, A1, Q1)
        kdqmc.qr_f64_noalloc(n, N, A2, Q2)
        t.cuda.synchronize()
        r1, r2 = A1.cpu().numpy()[:n, :n], A2.cpu().numpy()[:n, :n]
        q1, q2 = Q1.cpu().numpy()[:n, :n], Q2.cpu().numpy()[:n, :n]
        assert np.array_equal(r1, r2)
        assert np.array_equal(q1, q2)
        # and it is a QR of the input (not two equal wrong answers)
        assert np.abs(q2 @ np.triu(r2) - a[:n, :n]).max() < 1e-12
        assert np.abs(q2.T @ q2 - np.eye(n)).max() < 1e-12
    ch.close()


def test_noalloc_qr_packed_and_limits(gpu_lib):
    from paper_2608_03894_amd import kdqmc
    t = torch()
    say("noalloc QR packed")
    n = 200
    a = si.random_dense(n, 77)
    A, Q = dev(a), t.zeros((n, n), dtype=t.float64, device="cuda:0")
    kdqmc.qr_f64_noalloc(n, n, A, Q)
    t.cuda.synchronize()
    r, q = np.triu(A.cpu().numpy()), Q.cpu().numpy()
    assert np.abs(q @ r - a).max() < 1e-12
    big = t.zeros((513, 513), dtype=t.float64, device="cuda:0")
    with pytest.raises(kdqmc.KdqmcError) as e:
        kdqmc.qr_f64_noalloc(513, 513, big, big)
    assert e.value.code == kdqmc.EINVAL and "512" in str(e.value)
