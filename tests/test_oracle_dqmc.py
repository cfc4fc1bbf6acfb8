"""Pins of the oracle's DQMC module: decoupling identity, multiprecision
brute force, free-fermion closed forms, determinant ratios, and the identity
of delayed and undelayed updates."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import brute, dqmc, lattice


@pytest.fixture(scope="module")
def c1():
    w = si.C1
    m = dqmc.Model.from_workload(w)
    f = si.ising_fields(w.L, m.L_tau, w.seed)
    return w, m, f


@pytest.mark.parametrize("U", [-3.0, -4.0, -5.0, -8.0])
def test_hs_decoupling_identity(U):
    """(1/2) e^{-dtau|U|/4} sum_s e^{alpha s (n-1)} = e^{-dtau U (nu-1/2)(nd-1/2)}."""
    dtau = 0.1
    a = dqmc.hs_alpha(U, dtau)
    for nu in (0, 1):
        for nd in (0, 1):
            lhs = 0.5 * np.exp(-dtau * abs(U) / 4) * sum(np.exp(a * s * (nu + nd - 1)) for s in (-1, 1))
            rhs = np.exp(-dtau * U * (nu - 0.5) * (nd - 0.5))
            assert abs(lhs / rhs - 1) < 1e-15


def test_green_scratch_vs_multiprecision(c1):
    w, m, f = c1
    e = brute.mp_propagator(m, dps=40)
    for l in (0, 7, 20):
        g = dqmc.green_scratch(m, f, l)
        gm = brute.mp_green(m, f, l, dps=40, e=e)
        assert np.abs(g - gm).max() < 1e-13, l


def test_green_scratch_vs_dense(c1):
    w, m, f = c1
    for l in (0, 3, 11):
        assert np.abs(dqmc.green_scratch(m, f, l) - dqmc.green_dense(m, f, l)).max() < 1e-10


def test_green_cyclic(c1):
    w, m, f = c1
    assert np.abs(dqmc.green_scratch(m, f, 0) - dqmc.green_scratch(m, f, m.L_tau)).max() < 1e-13


@pytest.mark.parametrize("L,beta", [(3, 2.0), (6, 4.0)])
def test_free_fermions(L, beta):
    """U = 0: alpha = 0, every B equals exp(-dtau(K-mu)); the stabilized chain
    must reproduce (I + e^{-beta(K-mu)})^{-1} (eigenbasis) and the Bloch form."""
    mu = lattice.dirac_mu(L)
    m = dqmc.Model(L=L, t=1.0, U=0.0, beta=beta, dtau=0.1, mu=mu)
    assert m.alpha == 0.0
    f = si.ising_fields(L, m.L_tau, 1)
    g = dqmc.green_scratch(m, f, 4)
    gfree = dqmc.green_free(m)
    assert np.abs(g - gfree).max() < 1e-13
    gb = lattice.apply_block_operator(L, lattice.free_green_blocks(L, 1.0, beta, mu), np.eye(m.N))
    assert np.abs(gb.real - gfree).max() < 1e-13
    # at U = 0 the wrap leaves G invariant
    assert np.abs(dqmc.wrap(m, gfree, f[0]) - gfree).max() < 1e-13


def test_wrap_relation(c1):
    """G(l) = B_l G(l-1) B_l^{-1} for unchanged fields."""
    w, m, f = c1
    for l in (1, 5, 20):
        g_prev = dqmc.green_scratch(m, f, l - 1)
        assert np.abs(dqmc.wrap(m, g_prev, f[l - 1]) - dqmc.green_scratch(m, f, l)).max() < 1e-12


def test_flip_ratio_vs_determinants(c1):
    """Rank-one ratio e^{2 alpha s} R^2 equals the ratio of the brute-force
    weights prod e^{-alpha s} det(I + B...B)^2 (multiprecision)."""
    w, m, f = c1
    e = brute.mp_propagator(m, dps=30)
    lw0 = brute.mp_log_weight(m, f, dps=30, e=e)
    for (l, i) in [(1, 0), (3, 5), (10, 26), (20, 13)]:
        g_prev = dqmc.green_scratch(m, f, l - 1)
        ev = np.exp(m.alpha * f[l - 1])
        gt = ev[:, None] * g_prev / ev[None, :]
        ratio, _, _ = dqmc.flip_ratio(m.alpha, int(f[l - 1, i]), gt[i, i])
        f2 = f.copy()
        f2[l - 1, i] *= -1
        rb = float(brute.mp.exp(brute.mp_log_weight(m, f2, dps=30, e=e) - lw0))
        assert abs(ratio / rb - 1) < 1e-11, (l, i, ratio, rb)


def test_rank_one_update_then_wrap_equals_scratch(c1):
    w, m, f = c1
    l = 4
    g_prev = dqmc.green_scratch(m, f, l - 1)
    ev = np.exp(m.alpha * f[l - 1])
    gt = ev[:, None] * g_prev / ev[None, :]
    forced = np.zeros(m.N, dtype=np.uint8)
    forced[[2, 9, 17]] = 1
    s = f[l - 1].copy()
    gt2, acc, _ = dqmc.update_slice(gt, s, m.alpha, forced=forced, k=1)
    f2 = f.copy()
    f2[l - 1] = s
    g_new = m.EK @ gt2 @ m.EKinv
    assert np.abs(g_new - dqmc.green_scratch(m, f2, l)).max() < 1e-12
    assert list(np.nonzero(acc)[0]) == [2, 9, 17]


@pytest.mark.parametrize("k", [2, 5, 32])
def test_delayed_equals_undelayed(c1, k):
    w, m, f = c1
    g0 = dqmc.green_scratch(m, f, 0)
    u = si.metropolis_uniforms(w.L, m.L_tau, w.seed)[0]
    r1 = dqmc.sweep(m, f, g0, uniforms=u, k=1)
    rk = dqmc.sweep(m, f, g0, uniforms=u, k=k)
    assert np.array_equal(r1["accepted"], rk["accepted"])
    assert np.array_equal(r1["fields"], rk["fields"])
    for a, b in zip(r1["G_slices"], rk["G_slices"]):
        assert np.abs(a - b).max() < 1e-11


def test_sweep_consistency(c1):
    w, m, f = c1
    g0 = dqmc.green_scratch(m, f, 0)
    u = si.metropolis_uniforms(w.L, m.L_tau, w.seed)[0]
    r = dqmc.sweep(m, f, g0, uniforms=u, k=1)
    flipped = r["fields"] != f
    assert np.array_equal(flipped, r["accepted"])
    assert np.all(r["ratios"] > 0)
    assert max(r["wrap_err"].values()) < 1e-9
    # the last slice is stabilized: G(L_tau) is the fresh G(0) of the new fields
    assert np.abs(r["G"] - dqmc.green_scratch(m, r["fields"], 0)).max() < 1e-13
    # Metropolis rule
    acc_rule = u < r["ratios"]
    assert np.array_equal(acc_rule, r["accepted"])
    # a pre-stabilization G after ten updated slices is still close to fresh
    for l, g in r["G_prestab"].items():
        f_at_l = np.concatenate([r["fields"][:l], f[l:]])   # slices > l not yet visited
        assert np.abs(g - dqmc.green_scratch(m, f_at_l, l)).max() < 1e-9


def test_down_slice_update_equals_scratch(c1):
    """Downward step: from the fresh G(l), forced flips at slice l give the
    fresh G(l-1) of the new fields."""
    w, m, f = c1
    for l, sites in ((7, [0, 4, 26]), (1, [3, 11])):
        forced = np.zeros((m.L_tau, m.N), dtype=np.uint8)
        forced[l - 1, sites] = 1
        r = dqmc.sweep_down(m, f, dqmc.green_scratch(m, f, l), forced=forced, k=1,
                            n_stab=m.L_tau + 1, l_start=l, l_stop=l)
        assert np.abs(r["G"] - dqmc.green_scratch(m, r["fields"], l - 1)).max() < 1e-12
        assert list(np.nonzero(r["accepted"][l - 1])[0]) == sites


def test_down_ratio_vs_determinants(c1):
    """The ratio read off exp(dtau K) G(l) exp(-dtau K) (the downward pass's
    matrix) equals the multiprecision weight ratio of the flip."""
    w, m, f = c1
    e = brute.mp_propagator(m, dps=30)
    lw0 = brute.mp_log_weight(m, f, dps=30, e=e)
    for (l, i) in [(20, 2), (6, 19), (1, 8)]:
        gt = m.EKinv @ dqmc.green_scratch(m, f, l) @ m.EK
        ratio, _, _ = dqmc.flip_ratio(m.alpha, int(f[l - 1, i]), gt[i, i])
        f2 = f.copy()
        f2[l - 1, i] *= -1
        rb = float(brute.mp.exp(brute.mp_log_weight(m, f2, dps=30, e=e) - lw0))
        assert abs(ratio / rb - 1) < 1e-11, (l, i, ratio, rb)


@pytest.mark.parametrize("k", [2, 5, 32])
def test_down_delayed_equals_undelayed(c1, k):
    w, m, f = c1
    gt = dqmc.green_scratch(m, f, m.L_tau)
    u = si.metropolis_uniforms(w.L, m.L_tau, w.seed)[0]
    r1 = dqmc.sweep_down(m, f, gt, uniforms=u, k=1)
    rk = dqmc.sweep_down(m, f, gt, uniforms=u, k=k)
    assert np.array_equal(r1["accepted"], rk["accepted"])
    for a, b in zip(r1["G_slices"], rk["G_slices"]):
        assert np.abs(a - b).max() < 1e-11


def test_down_sweep_consistency(c1):
    """A Metropolis downward pass: decisions follow the rule, every slice's G is
    the fresh G of the fields so far, the pass ends at the fresh G(0)."""
    w, m, f = c1
    u = si.metropolis_uniforms(w.L, m.L_tau, w.seed + 1)[0]
    r = dqmc.sweep_down(m, f, dqmc.green_scratch(m, f, m.L_tau), uniforms=u, k=4)
    assert np.array_equal(r["fields"] != f, r["accepted"])
    assert np.array_equal(u < r["ratios"], r["accepted"])
    assert sorted(r["wrap_err"]) == [0, 10]
    assert max(r["wrap_err"].values()) < 1e-9
    assert np.abs(r["G"] - dqmc.green_scratch(m, r["fields"], 0)).max() < 1e-13
    for idx, g in enumerate(r["G_slices"]):
        l = m.L_tau - idx            # slice just processed; g is G(l-1)
        f_now = np.concatenate([f[:l - 1], r["fields"][l - 1:]])
        assert np.abs(g - dqmc.green_scratch(m, f_now, l - 1)).max() < 1e-9


def test_up_then_down_returns_to_scratch(c1):
    """An upward pass followed by a downward pass from its end matrix."""
    w, m, f = c1
    u = si.metropolis_uniforms(w.L, m.L_tau, w.seed, n_sweeps=2)
    r1 = dqmc.sweep(m, f, dqmc.green_scratch(m, f, 0), uniforms=u[0], k=3)
    r2 = dqmc.sweep_down(m, r1["fields"], r1["G"], uniforms=u[1], k=3)
    assert np.abs(r2["G"] - dqmc.green_scratch(m, r2["fields"], 0)).max() < 1e-13
    assert r2["accepted"].any()


def test_golden_multiprecision_fixture():
    """G(0) and G(10) of the smallest workload, 50-digit brute force, stored
    by tests/golden/make_golden.py (which calls only the oracle)."""
    import os
    here = os.path.join(os.path.dirname(__file__), "golden", "c1_green_mp50.npz")
    data = np.load(here)
    w = si.C1
    m = dqmc.Model.from_workload(w, mu=-1.0)
    f = si.ising_fields(w.L, m.L_tau, w.seed)
    assert np.array_equal(data["fields"], f)
    for l in (0, 10):
        assert np.abs(dqmc.green_scratch(m, f, l) - data[f"G{l}"]).max() < 1e-13
