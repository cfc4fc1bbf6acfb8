"""GPU parity of the building blocks through the C ABI: MFMA GEMM, Householder
QR, and the FFT wrap (column pass exp(-dtau K), row pass exp(+dtau K)) against
the oracle's dense matrix exponentials."""
import numpy as np
import pytest
import scipy.linalg

import seeded_inputs as si
from gpu_helpers import chain, dev, say, torch
from oracle import dqmc, lattice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ch6(gpu_lib):
    return chain(6, -4.0, 1.0)   # N = 108 context for the GEMM / QR calls


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (70, 45, 33), (64, 64, 64), (108, 100, 97)])
def test_gemm_f64(ch6, ta, tb, M, N, K):
    say("gemm", ta, tb, M, N, K)
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C = rng.standard_normal((M, N))
    want = 1.5 * ((A.T if ta else A) @ (B.T if tb else B)) - 0.5 * C
    a, b, c = dev(A), dev(B), dev(C)
    ch6.gemm_f64(ta, tb, M, N, K, 1.5, a, A.shape[1], b, B.shape[1], -0.5, c, N)
    ch6.sync()
    got = c.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(want).max()) * K


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("L,M,N,K", [(12, 432, 432, 432), (24, 1728, 1728, 1728), (24, 1100, 1700, 37)])
def test_gemm_f64_large(gpu_lib, ta, tb, L, M, N, K):
    """Both tile sizes (32 x 32 where 64 x 64 tiles would give under one
    workgroup per CU), ragged edges, slabs of K in flight."""
    say("gemm-large", L, M, N, K, ta, tb)
    ch = chain(L, 0.0, 1.0)
    rng = np.random.default_rng(M + N + K + 2 * ta + tb)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C = rng.standard_normal((M, N))
    want = 0.5 * ((A.T if ta else A) @ (B.T if tb else B)) + 2.0 * C
    a, b, c = dev(A), dev(B), dev(C)
    ch.gemm_f64(ta, tb, M, N, K, 0.5, a, A.shape[1], b, B.shape[1], 2.0, c, N)
    ch.sync()
    got = c.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(want).max()) * K


def test_gemm_f64_k0(ch6):
    """K = 0: no slab is read and C = beta C."""
    C = np.random.default_rng(5).standard_normal((20, 30))
    a, b, c = dev(np.zeros((20, 1))), dev(np.zeros((1, 30))), dev(C)
    ch6.gemm_f64(0, 0, 20, 30, 0, 1.0, a, 1, b, 30, -2.0, c, 30)
    ch6.sync()
    assert np.array_equal(c.cpu().numpy(), -2.0 * C)


@pytest.mark.parametrize("n", [1, 17, 100, 108])
def test_qr_f64(ch6, n):
    say("qr", n)
    N = ch6.N
    rng = np.random.default_rng(n)
    A = np.zeros((N, N))
    A[:n, :n] = rng.standard_normal((n, n)) * np.logspace(0, -8, n)[None, :]
    a = dev(A)
    q = dev(np.zeros((N, N)))
    ch6.qr_f64(n, a, q)
    ch6.sync()
    R = a.cpu().numpy()[:n, :n]
    Q = q.cpu().numpy()[:n, :n]
    assert np.abs(np.tril(R, -1)).max() == 0.0
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-13
    # column-wise backward error (graded columns keep their relative accuracy)
    err = np.abs(Q @ R - A[:n, :n]).max(axis=0) / np.abs(A[:n, :n]).max(axis=0)
    assert err.max() < 1e-12
    # |diag R| equals LAPACK's up to sign
    r_ref = scipy.linalg.qr(A[:n, :n], mode="r")[0]
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(r_ref)), rtol=1e-10, atol=0)


@pytest.mark.parametrize("L,n", [(12, 432), (12, 300), (24, 1728), (24, 1100)])
def test_qr_f64_large(gpu_lib, L, n):
    """16-column panels with 2 or 4 rows per thread (up to 512, 1024 and 2048
    rows), ragged tails."""
    say("qr-large", L, n)
    ch = chain(L, 0.0, 1.0)
    N = ch.N
    rng = np.random.default_rng(n)
    A = np.zeros((N, N))
    A[:n, :n] = rng.standard_normal((n, n)) * np.logspace(0, -6, n)[None, :]
    a = dev(A)
    q = dev(np.zeros((N, N)))
    ch.qr_f64(n, a, q)
    ch.sync()
    R = a.cpu().numpy()[:n, :n]
    Q = q.cpu().numpy()[:n, :n]
    assert np.abs(np.tril(R, -1)).max() == 0.0
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-12
    err = np.abs(Q @ R - A[:n, :n]).max(axis=0) / np.abs(A[:n, :n]).max(axis=0)
    assert err.max() < 1e-11


@pytest.mark.parametrize("L", [3, 6, 9, 12, 15, 18, 24])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed_f16", 2e-6)])
def test_wrap_free(gpu_lib, L, prec, tol):
    """U = 0 (fields drop out): G <- exp(-dtau K) G exp(dtau K) on a random G."""
    say("wrap", L, prec)
    ch = chain(L, 0.0, 1.0, prec=prec)
    m = dqmc.Model(L=L, t=1.0, U=0.0, beta=1.0, dtau=0.1, mu=-1.0)
    G = si.random_dense(ch.N, seed=L)
    ch.set_G(dev(G), 0)
    ch.wrap_slice(1)
    got = ch.G().cpu().numpy()
    want = m.EK @ G @ m.EKinv
    rel = np.abs(got - want).max() / np.abs(want).max()
    say("wrap", L, prec, "rel err", rel)
    assert rel < tol
    assert ch.current_slice() == 1


@pytest.mark.parametrize("L", [3, 12])
def test_wrap_tiles(gpu_lib, L):
    """Every FFT tile width gives the same result (ragged last workgroup)."""
    say("wrap-tiles", L)
    m = dqmc.Model(L=L, t=1.0, U=0.0, beta=1.0, dtau=0.1, mu=-1.0)
    G = si.random_dense(3 * L * L, seed=100 + L)
    want = m.EK @ G @ m.EKinv
    for P in (1, 2, 3, 5, 8):
        ch = chain(L, 0.0, 1.0, fft_tile=P)
        ch.set_G(dev(G), 0)
        ch.wrap_slice(1)
        got = ch.G().cpu().numpy()
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max(), P


@pytest.mark.parametrize("L", [3, 12, 24])
def test_expK_matches_dense_expm(gpu_lib, L):
    """kdqmc_expK_f64 (the product of Eq. (5) by the three steps of Eq. (6))
    against the oracle's dense scipy expm(-+dtau K) times M, on all columns
    and on a ragged leading block of columns."""
    import numpy as np
    import scipy.linalg
    from gpu_helpers import chain, dev, say
    from oracle import lattice
    say("expK", L)
    ch = chain(L, -4.0, 1.0, delay_k=1 if L == 3 else 32)
    N = ch.N
    K = lattice.kagome_K(L)
    m = si.random_dense(N, 300 + L)
    for sign, nc in ((-1, N), (1, N), (-1, N // 2 + 1)):
        a = dev(m)
        ch.expK_f64(a, N, nc, sign)
        got = a.cpu().numpy()
        want = m.copy()
        want[:, :nc] = scipy.linalg.expm(sign * 0.1 * K) @ m[:, :nc]
        say("expK", L, sign, nc, np.abs(got - want).max())
        assert np.abs(got - want).max() < 1e-12 * max(1.0, np.abs(want).max())
    ch.close()
