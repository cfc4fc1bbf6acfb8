"""The persistent slice launch (one resident launch per slice, tiles of G
held in registers, workgroups handing over through counters) against the
per-window launches it replaces: the same G, decisions and ratios bit for bit
over an upward and a downward Metropolis pass, at shapes with one tile
(L = 3), ragged 16- and 32-site windows (L = 6, 9), the headline lattice
(L = 12), one tile per workgroup up to L = 15 (121 tiles) and two or three
per workgroup at L = 18 and 24; and against the oracle at L = 6 with its
decisions replayed."""
import numpy as np
import pytest

import seeded_inputs as si
from gpu_helpers import dev, say, torch
from oracle import dqmc

pytestmark = pytest.mark.gpu


def _run(L, U, beta, k, persistent, seed):
    from paper_2608_03894_amd import kdqmc
    t = torch()
    p = kdqmc.make_params(L, U, beta, 0.1, mu=-1.0, n_stab=10, delay_k=k)
    ch = kdqmc.Chain(p)
    used = ch.set_slice_launch(persistent)
    Lt, N = ch.L_tau, ch.N
    ch.set_fields(dev(si.ising_fields(L, Lt, seed)))
    us = si.metropolis_uniforms(L, Lt, seed, n_sweeps=2)
    acc = t.zeros((Lt, N), dtype=t.uint8, device="cuda:0")
    rat = t.zeros((Lt, N), dtype=t.float64, device="cuda:0")
    ch.sweep(dev(us[0]), None, acc, rat, None)
    a1, r1 = acc.cpu().numpy().copy(), rat.cpu().numpy().copy()
    ch.sweep_down(dev(us[1]), None, acc, rat, None)
    a2, r2 = acc.cpu().numpy().copy(), rat.cpu().numpy().copy()
    G = ch.G().cpu().numpy()
    worst, ok = ch.health(raise_on_error=False)
    ch.close()
    return used, G, (a1, r1, a2, r2), ok


@pytest.mark.timeout(300)
@pytest.mark.parametrize("L,k", [(3, 8), (6, 16), (9, 32), (12, 32), (15, 32), (18, 32), (24, 32)])
def test_persistent_equals_per_window(gpu_lib, L, k):
    """(L = 18 and 24: 256 and 729 tiles, two and three per workgroup.)"""
    say("persistent vs per-window", L, k)
    U, beta, seed = -4.0, (2.0 if L <= 15 else 1.0), 500 + L
    used_p, Gp, dp, okp = _run(L, U, beta, k, True, seed)
    used_w, Gw, dw, okw = _run(L, U, beta, k, False, seed)
    say("  persistent used", used_p, "per-window used", used_w)
    assert used_p and not used_w
    assert okp and okw
    assert dp[0].sum() > 0
    for x, y in zip(dp, dw):
        assert np.array_equal(x, y)
    assert np.array_equal(Gp, Gw)


def test_persistent_against_oracle(gpu_lib):
    """L = 6 (2 x 2 tiles, 16-site windows in one resident launch per slice),
    the oracle's decisions replayed: every slice within the FP64 bound."""
    from paper_2608_03894_amd import kdqmc
    t = torch()
    L, U, beta = 6, -4.0, 2.0
    m = dqmc.Model(L=L, t=1.0, U=U, beta=beta, dtau=0.1, mu=-1.0)
    f = si.ising_fields(L, m.L_tau, 61)
    u = si.metropolis_uniforms(L, m.L_tau, 61)[0]
    g0 = dqmc.green_scratch(m, f, 0)
    r = dqmc.sweep(m, f, g0, uniforms=u, k=1)
    ch = kdqmc.Chain(kdqmc.make_params(L, U, beta, 0.1, mu=-1.0, delay_k=16))
    assert ch.set_slice_launch(True)
    ch.set_fields(dev(f))
    forced = dev(r["accepted"].astype(np.uint8))
    for l in range(1, m.L_tau + 1):
        ch.sweep_slice(l, None, forced[l - 1])
        if l % 10 == 0:
            ch.stabilize()
            tol = 1e-10
        else:
            tol = max(1e-10, 2.0 * r["wrap_err"][(l // 10 + 1) * 10])
        d = float(np.abs(ch.G().cpu().numpy() - r["G_slices"][l - 1]).max())
        assert d < tol, (l, d, tol)
    ch.close()
