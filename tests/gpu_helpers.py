"""Shared helpers of the GPU tests: seeded inputs, oracle runs (cached), and
device tensors.  Every GPU step prints the case it runs first."""
import functools
import sys

import numpy as np

import seeded_inputs as si
from oracle import dqmc, lattice


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def torch():
    import torch as t
    return t


def dev(x, dtype=None):
    t = torch()
    a = t.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        a = a.to(dtype)
    return a.to("cuda:0")


def model(L, U, beta, dtau=0.1):
    return dqmc.Model(L=L, t=1.0, U=U, beta=beta, dtau=dtau, mu=-1.0)


@functools.lru_cache(maxsize=None)
def oracle_run(L, U, beta, seed, k=1, n_stab=10, l_stop=None):
    """Oracle sweep with Metropolis uniforms; returns (model, fields, G0, result, uniforms)."""
    m = model(L, U, beta)
    f = si.ising_fields(L, m.L_tau, seed)
    u = si.metropolis_uniforms(L, m.L_tau, seed)[0]
    g0 = dqmc.green_scratch(m, f, 0)
    r = dqmc.sweep(m, f, g0, uniforms=u, k=k, n_stab=n_stab, l_stop=l_stop)
    return m, f, g0, r, u


def chain(L, U, beta, prec="fp64", delay_k=32, window=0, n_stab=10, fft_tile=0):
    from paper_2608_03894_amd import kdqmc
    p = kdqmc.make_params(L, U, beta, 0.1, mu=-1.0, n_stab=n_stab, delay_k=delay_k, window=window,
                          prec=prec, fft_tile=fft_tile)
    return kdqmc.Chain(p)
