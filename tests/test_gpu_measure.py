"""GPU parity of the equal-time estimators of Secs. IV-V (kdqmc_measure)
against the oracle's Wick-contraction estimators evaluated on the same G
(read back from the device): finite-temperature chains at L = 3, 6, 12 and
24 (every size but 24 ends in a ragged 64 x 64 tile), mixed precision,
a batch of chains, and a projector chain."""
import numpy as np
import pytest

import seeded_inputs as si
from gpu_helpers import chain, dev, say, torch
from oracle import measure

pytestmark = pytest.mark.gpu

NAMES = ("s_pair_gamma", "s_pair_dk1", "s_pair_dk2", "cdw2_gamma", "cdw2_k", "density")


def _compare(got, G, L, tol):
    want = measure.estimators(G, L)
    for k in NAMES:
        say("  ", k, got[k], want[k])
        assert abs(got[k] - want[k]) <= tol * max(1.0, abs(want[k])), (k, got[k], want[k])


@pytest.mark.timeout(300)
@pytest.mark.parametrize("L,beta,slices", [(3, 2.0, 5), (6, 2.0, 7), (12, 1.0, 3), (24, 0.4, 0)])
def test_measure_fp64(gpu_lib, L, beta, slices):
    say("measure fp64", L, beta, slices)
    Lt = int(round(beta / 0.1))
    f = si.ising_fields(L, Lt, 90 + L)
    u = dev(si.metropolis_uniforms(L, Lt, 90 + L)[0])
    ch = chain(L, -4.0, beta, delay_k=16, n_stab=Lt if Lt < 10 else 10)
    ch.set_fields(dev(f))
    for l in range(1, slices + 1):
        ch.sweep_slice(l, u[l - 1])
    G = ch.G().cpu().numpy()
    _compare(ch.observables(), G, L, 1e-12)
    ch.close()


def test_measure_mixed_and_batch(gpu_lib):
    """FP32 G (mixed precision) and a batch of three chains: each chain's
    record against the oracle on that chain's G."""
    from paper_2608_03894_amd import kdqmc
    say("measure mixed + batch")
    L, beta, Lt = 6, 2.0, 20
    ch = chain(L, -5.0, beta, delay_k=16, prec="mixed_f16", n_stab=2)
    ch.set_fields(dev(si.ising_fields(L, Lt, 4)))
    u = dev(si.metropolis_uniforms(L, Lt, 4)[0])
    for l in range(1, 5):
        ch.sweep_slice(l, u[l - 1])
        if l % 2 == 0:
            ch.stabilize()
    ch.sweep_slice(5, u[4])
    _compare(ch.observables(), ch.G().cpu().numpy(), L, 1e-10)
    ch.close()
    p = kdqmc.make_params(L, -3.0, beta, 0.1, mu=-1.0, delay_k=16)
    b = kdqmc.Chain(p, n_chains=3, U=[-3.0, -4.0, -5.0])
    b.set_fields(dev(np.stack([si.ising_fields(L, Lt, s) for s in (1, 2, 3)])))
    U = dev(np.stack([si.metropolis_uniforms(L, Lt, s)[0] for s in (1, 2, 3)]))
    for l in range(1, 4):
        b.sweep_slice(l, U[:, l - 1].contiguous())
    got = b.observables()
    G = b.G().cpu().numpy()
    for z in range(3):
        _compare(got[z], G[z], L, 1e-12)
    b.close()


def test_measure_projector(gpu_lib):
    """A projector chain (Dirac filling, n_occ = L^2): the estimators of its G;
    the density is the trial state's filling 2 n_occ / N = 2/3 at every slice
    (the projection conserves the particle number)."""
    from paper_2608_03894_amd import kdqmc
    say("measure projector")
    L, beta, Lt = 6, 2.0, 20
    p = kdqmc.make_params(L, -4.0, beta, 0.1, mu=-1.0, delay_k=16, n_occ=L * L)
    ch = kdqmc.Chain(p)
    ch.set_trial(dev(kdqmc.trial_orbitals(L, L * L)))
    ch.set_fields(dev(si.ising_fields(L, Lt, 8)))
    u = dev(si.metropolis_uniforms(L, Lt, 8)[0])
    for l in range(1, 7):
        ch.sweep_slice(l, u[l - 1])
    got = ch.observables()
    _compare(got, ch.G().cpu().numpy(), L, 1e-12)
    assert abs(got["density"] - 2.0 / 3.0) < 1e-10
    ch.close()
