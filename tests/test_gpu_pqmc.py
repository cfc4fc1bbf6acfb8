"""GPU parity of the projector form (Sec. II: trial wave function of the
lowest N_occ eigenstates, rho = 2 N_occ / N; projection over beta) through
the C ABI, against the oracle's projector passes on identical seeded fields
with its decisions replayed: G(0) from the stacks of orthonormal panels,
every slice of an upward and of a downward pass, the flip ratios, the
stabilizations, Metropolis decisions, graph replay and the call order."""
import numpy as np
import pytest

import seeded_inputs as si
from gpu_helpers import dev, model, say, torch
from oracle import pqmc

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def pq_chain(L, U, beta, n_occ, delay_k=16, window=0, n_stab=10, prec="fp64"):
    from paper_2608_03894_amd import kdqmc
    p = kdqmc.make_params(L, U, beta, 0.1, mu=-1.0, n_stab=n_stab, delay_k=delay_k, window=window,
                          prec=prec, n_occ=n_occ)
    ch = kdqmc.Chain(p)
    ch.set_trial(dev(kdqmc.trial_orbitals(L, n_occ)))
    return ch


def _replay_up(ch, f, r, n_stab=10):
    t = torch()
    L_tau, N = f.shape
    forced = dev(r["accepted"].astype(np.uint8))
    ratio = t.zeros((L_tau, N), dtype=t.float64, device="cuda:0")
    gs, pre, errs = [], {}, {}
    e = t.zeros(1, dtype=t.float64, device="cuda:0")
    for l in range(1, L_tau + 1):
        ch.sweep_slice(l, None, forced[l - 1], None, ratio[l - 1])
        if l % n_stab == 0:
            pre[l] = ch.G().cpu().numpy()
            ch.stabilize(e)
            errs[l] = float(e.cpu()[0])
        gs.append(ch.G().cpu().numpy())
    return gs, ratio.cpu().numpy(), pre, errs


def _replay_down(ch, f, r, n_stab=10):
    t = torch()
    L_tau, N = f.shape
    forced = dev(r["accepted"].astype(np.uint8))
    ratio = t.zeros((L_tau, N), dtype=t.float64, device="cuda:0")
    gs = []
    for l in range(L_tau, 0, -1):
        ch.sweep_slice_down(l, None, forced[l - 1], None, ratio[l - 1])
        if (l - 1) % n_stab == 0:
            ch.stabilize()
        gs.append(ch.G().cpu().numpy())
    return gs, ratio.cpu().numpy()


@pytest.mark.parametrize("L,beta,n_occ", [(3, 2.0, 9), (6, 2.0, 36), (6, 2.0, 31), (12, 1.0, 144)])
def test_pqmc_green_zero(gpu_lib, L, beta, n_occ):
    """G(0) = I - P (L(0) P)^{-1} L(0) from the left stack, against the oracle
    (which builds its own trial orbitals by dense diagonalisation)."""
    say("pqmc G0", L, beta, n_occ)
    m = model(L, -4.0, beta)
    f = si.ising_fields(L, m.L_tau, 40 + L)
    ch = pq_chain(L, -4.0, beta, n_occ)
    ch.set_fields(dev(f))
    p, _ = pqmc.trial_orbitals(L, n_occ)
    d = float(np.abs(ch.G().cpu().numpy() - pqmc.green(m, f, p, 0)).max())
    say("pqmc G0 err", d)
    assert d < TOL64
    ch.close()


@pytest.mark.parametrize("L,k,window", [(3, 1, 1), (3, 8, 4), (6, 16, 0), (6, 64, 32)])
def test_pqmc_passes_forced(gpu_lib, L, k, window):
    """An upward pass then a downward pass, slice by slice, with the oracle's
    Metropolis decisions replayed: every G, ratio and stabilization."""
    say("pqmc passes", L, k, window)
    m = model(L, -4.0, 2.0)
    n_occ = L * L
    f = si.ising_fields(L, m.L_tau, 50 + L)
    u = si.metropolis_uniforms(L, m.L_tau, 50 + L, n_sweeps=2)
    p, _ = pqmc.trial_orbitals(L, n_occ)
    r_up = pqmc.sweep(m, f, p, pqmc.green(m, f, p, 0), uniforms=u[0], k=1)
    r_dn = pqmc.sweep_down(m, r_up["fields"], p, r_up["G"], uniforms=u[1], k=1)
    ch = pq_chain(L, -4.0, 2.0, n_occ, delay_k=k, window=window)
    ch.set_fields(dev(f))
    gs, ratio, pre, errs = _replay_up(ch, f, r_up)
    worst = max(np.abs(a - b).max() for a, b in zip(gs, r_up["G_slices"]))
    say("pqmc up worst", worst, "wrap errors", errs, "oracle", r_up["wrap_err"])
    assert worst < TOL64
    assert np.abs(ratio - r_up["ratios"]).max() < 1e-9 * np.abs(r_up["ratios"]).max()
    assert ch.current_slice() == m.L_tau            # the pass ends at slice L_tau
    gs, ratio = _replay_down(ch, r_up["fields"], r_dn)
    worst = max(np.abs(a - b).max() for a, b in zip(gs, r_dn["G_slices"]))
    say("pqmc down worst", worst)
    assert worst < TOL64
    assert np.abs(ratio - r_dn["ratios"]).max() < 1e-9 * np.abs(r_dn["ratios"]).max()
    assert ch.current_slice() == 0
    fields = torch().zeros(f.shape, dtype=torch().int8, device="cuda:0")
    ch.get_fields(fields)
    assert np.array_equal(fields.cpu().numpy(), r_dn["fields"])
    ch.close()


@pytest.mark.timeout(600)
def test_pqmc_l12_u5_ten_slices(gpu_lib):
    """The lattice and coupling of the timing workload of Sec. III (U=-5,
    rho = 2/3) at L=12 (N=432, n_occ=144), beta=2: ten slices and the first
    stabilization with the oracle's decisions replayed.  Per slice within
    max(1e-10, 2 x the oracle's own drift at slice 10), after the
    stabilization within 1e-10."""
    say("pqmc L12 U-5")
    L, U, beta = 12, -5.0, 2.0
    m = model(L, U, beta)
    f = si.ising_fields(L, m.L_tau, 120)
    u = si.metropolis_uniforms(L, m.L_tau, 120)[0]
    p, _ = pqmc.trial_orbitals(L, L * L)
    g0 = pqmc.green(m, f, p, 0)
    r = pqmc.sweep(m, f, p, g0, uniforms=u, k=32, l_stop=10)
    ch = pq_chain(L, U, beta, L * L, delay_k=32)
    ch.set_fields(dev(f))
    assert np.abs(ch.G().cpu().numpy() - g0).max() < TOL64
    forced = dev(r["accepted"][:10].astype(np.uint8))
    tol = max(TOL64, 2.0 * r["wrap_err"][10])
    diffs = []
    for l in range(1, 11):
        ch.sweep_slice(l, None, forced[l - 1])
        ref = r["G_prestab"][l] if l == 10 else r["G_slices"][l - 1]
        diffs.append(float(np.abs(ch.G().cpu().numpy() - ref).max()))
    ch.stabilize()
    post = float(np.abs(ch.G().cpu().numpy() - r["G_slices"][9]).max())
    say("pqmc L12 per slice", diffs, "tol", tol, "post", post)
    assert max(diffs) < tol
    assert post < TOL64
    ch.close()


def test_pqmc_metropolis_and_graphs(gpu_lib):
    """Metropolis decisions from the same uniforms as the oracle (no replay)
    over an upward and a downward pass, through the captured-graph passes;
    and the same passes of direct launches equal them bit for bit."""
    say("pqmc metropolis + graphs")
    t = torch()
    L = 3
    m = model(L, -4.0, 2.0)
    f = si.ising_fields(L, m.L_tau, 77)
    u = si.metropolis_uniforms(L, m.L_tau, 77, n_sweeps=2)
    p, _ = pqmc.trial_orbitals(L, 9)
    r_up = pqmc.sweep(m, f, p, pqmc.green(m, f, p, 0), uniforms=u[0], k=1)
    r_dn = pqmc.sweep_down(m, r_up["fields"], p, r_up["G"], uniforms=u[1], k=1)
    near = np.abs(u[0] - r_up["ratios"]) < 1e-9
    assert not near.any()
    outs = []
    for graphs in (True, False):
        ch = pq_chain(L, -4.0, 2.0, 9, delay_k=8)
        ch.use_graphs(graphs)
        ch.set_fields(dev(f))
        a1 = t.zeros(f.shape, dtype=t.uint8, device="cuda:0")
        a2 = t.zeros(f.shape, dtype=t.uint8, device="cuda:0")
        ub = dev(u)
        ch.sweep(ub[0], None, a1, None, None)
        g_top = ch.G().cpu().numpy()
        ch.sweep_down(ub[1], None, a2, None, None)
        outs.append((g_top, ch.G().cpu().numpy(), a1.cpu().numpy(), a2.cpu().numpy()))
        ch.close()
    g_top, g_end, a1, a2 = outs[0]
    assert np.array_equal(a1.astype(bool), r_up["accepted"])
    assert np.array_equal(a2.astype(bool), r_dn["accepted"])
    assert np.abs(g_top - r_up["G"]).max() < TOL64
    assert np.abs(g_end - r_dn["G"]).max() < TOL64
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)


def test_pqmc_state_errors(gpu_lib):
    from paper_2608_03894_amd import kdqmc
    say("pqmc state errors")
    t = torch()
    p = kdqmc.make_params(3, -4.0, 2.0, 0.1, mu=-1.0, delay_k=4, n_occ=9)
    ch = kdqmc.Chain(p)
    f = dev(si.ising_fields(3, 20, 5))
    with pytest.raises(kdqmc.KdqmcError) as e:
        ch.set_fields(f)                               # no trial orbitals yet
    assert e.value.code == kdqmc.ESTATE
    ch.set_trial(dev(kdqmc.trial_orbitals(3, 9)))
    ch.set_fields(f)
    u = dev(si.metropolis_uniforms(3, 20, 5)[0])
    with pytest.raises(kdqmc.KdqmcError) as e:
        ch.sweep_down(u)                               # a projector pass starts upward
    assert e.value.code == kdqmc.ESTATE
    ch.sweep(u)
    with pytest.raises(kdqmc.KdqmcError) as e:
        ch.sweep(u)                                    # ... and they alternate
    assert e.value.code == kdqmc.ESTATE
    ch.sweep_down(u)
    assert ch.current_slice() == 0
    ch.close()
    fin = kdqmc.Chain(kdqmc.make_params(3, -4.0, 2.0, 0.1, mu=-1.0, delay_k=4))
    with pytest.raises(kdqmc.KdqmcError) as e:
        fin.set_trial(dev(kdqmc.trial_orbitals(3, 9)))
    assert e.value.code == kdqmc.EINVAL
    fin.close()
    del t
