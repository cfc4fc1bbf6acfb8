"""Pins of the equal-time estimators (Secs. IV-V) in oracle/measure.py:
the Wick contractions against a Fock-space brute force under a Gaussian
weight operator with a non-symmetric G (the configurations' G is not
symmetric), the site geometry against the bonds of K, and the classical
limits of S_Pair and of the CDW field by hand."""
import numpy as np
import pytest
import scipy.linalg

from oracle import brute, lattice, measure


@pytest.fixture(scope="module")
def gaussian():
    """Weight operator U = e^{c^+ A1 c} e^{c^+ A2 c} on 3 sites x 2 spins (64 states)
    with random non-symmetric A1, A2; returns (G from its single-particle form,
    expectation function, annihilators)."""
    rng = np.random.default_rng(5)
    n = 3
    a1 = 0.6 * rng.standard_normal((n, n))
    a2 = 0.6 * rng.standard_normal((n, n))
    cs = brute.fock_annihilators(2 * n)
    u = scipy.linalg.expm(brute.fock_quadratic(cs, a1)) @ scipy.linalg.expm(brute.fock_quadratic(cs, a2))
    z = np.trace(u)

    def ev(x):
        return np.trace(x @ u) / z
    g = np.linalg.inv(np.eye(n) + scipy.linalg.expm(a1) @ scipy.linalg.expm(a2))
    return g, ev, cs, n


def test_green_convention(gaussian):
    """<c_a c_b^+> = [(I + e^{A1} e^{A2})^{-1}]_ab for each spin."""
    g, ev, cs, n = gaussian
    for s in range(2):
        for a in range(n):
            for b in range(n):
                x = ev(cs[s * n + a] @ cs[s * n + b].T)
                assert abs(x - g[a, b]) < 1e-12


def test_pair_correlation_wick(gaussian):
    g, ev, cs, n = gaussian
    corr = measure.pair_correlation(g)
    for i in range(n):
        for j in range(n):
            di = cs[n + i] @ cs[i]          # D_i = c_{i dn} c_{i up}
            dj = cs[n + j] @ cs[j]
            x = ev(di.T @ dj + dj @ di.T)
            assert abs(x - corr[i, j]) < 1e-12, (i, j)


def test_density_correlation_wick(gaussian):
    g, ev, cs, n = gaussian
    nn = measure.density_correlation(g)
    for a in range(n):
        for b in range(n):
            na = cs[a].T @ cs[a] + cs[n + a].T @ cs[n + a]
            nb = cs[b].T @ cs[b] + cs[n + b].T @ cs[n + b]
            assert abs(ev(na @ nb) - nn[a, b]) < 1e-12, (a, b)


@pytest.mark.parametrize("L", [3, 6])
def test_geometry_bonds(L):
    """With 60-degree lattice vectors and the sublattice offsets of the reading,
    every bond of K (minimal image on the torus) has the same length 1/2 and
    no non-bond pair is that close."""
    a1 = np.array([1.0, 0.0])
    a2 = np.array([0.5, np.sqrt(3) / 2])
    x = measure.site_coords(L)
    k = lattice.kagome_K(L)
    n = 3 * L * L
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d = x[i] - x[j]
            best = min(np.linalg.norm((d[0] + p) * a1 + (d[1] + q) * a2)
                       for p in (-L, 0, L) for q in (-L, 0, L))
            if k[i, j] != 0.0:
                assert abs(best - 0.5) < 1e-12, (i, j, best)
            else:
                assert best > 0.5 + 1e-6, (i, j, best)


def _product_state(occ):
    """G of a product state with n_a in {0, 2}: G_aa = 1 - n_a / 2."""
    return np.diag(1.0 - np.asarray(occ, float) / 2.0)


@pytest.mark.parametrize("L", [3, 6])
def test_classical_limits(L):
    """Product states (n_a in {0, 2}): every on-site pair is sharp, so
    S_Pair(Q) = 1 at every Q; the CDW field is the classical one:
    A filled in every cell gives phi(Gamma) = 2 L^2 / N = 2/3 and phi(K) = 0;
    a pattern filling A only where x1 - x2 = 0 (mod 3) gives
    phi(K) = (2/N) sum over those cells of e^{iK.R}, |phi(K)| = 2/9."""
    n = 3 * L * L
    occ = np.zeros(n)
    occ[0::3] = 2.0
    g = _product_state(occ)
    for m in ((0, 0), measure.DK1, measure.k_point(L)):
        assert abs(measure.s_pair(g, L, m) - 1.0) < 1e-12
    assert abs(measure.cdw_d2(g, L, (0, 0)) - 4.0 / 9.0) < 1e-12
    assert abs(measure.cdw_d2(g, L, measure.k_point(L))) < 1e-12
    occ = np.zeros(n)
    for x1 in range(L):
        for x2 in range(L):
            if (x1 - x2) % 3 == 0:
                occ[(x1 * L + x2) * 3] = 2.0
    g = _product_state(occ)
    # K.R = 2 pi (x1 + 2 x2) / 3 = 2 pi (x1 - x2) / 3 (mod 2 pi): every filled cell has phase 1
    assert abs(measure.cdw_d2(g, L, measure.k_point(L)) - (2.0 / 9.0) ** 2) < 1e-12
    assert abs(measure.density(g) - 2.0 / 9.0) < 1e-12
