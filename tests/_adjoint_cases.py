"""Shared inputs of the adjoint tests: single-fluid acoustic cases over a
smooth background wave (so that a finite-difference perturbation stays far
below the data's own variation everywhere, where the WENO weights respond
smoothly), smooth seeded perturbation directions, and the pressure-probe
loss J = sum_probes (p - p0)^2 / 1e6."""
import numpy as np

from paper_1905_03917_amd import workloads as WL

P0 = 1.0e5


def case(n, ndim, bc=0, seed=5, width=0.15):
    return WL.pulse_air(n=n, ndim=ndim, seed=seed, bc=bc, width=width, u0=(60.0, 35.0, 20.0), bg=3.0e3)


def direction(n, ndim, seed=7):
    """(D+2, cells) smooth random direction: three seeded low-frequency
    products of sines per component, scaled to rho ~ 1, u ~ 10, p ~ 1e3."""
    rng = np.random.default_rng(seed)
    xs = (np.arange(n) + 0.5) / n
    grids = np.meshgrid(*([xs] * ndim), indexing="ij")     # grids[-1] varies along x
    out = np.zeros((ndim + 2, n ** ndim))
    for q in range(ndim + 2):
        f = np.zeros([n] * ndim)
        for _ in range(3):
            k = rng.integers(1, 3, size=ndim)
            ph = rng.uniform(0, 2 * np.pi, size=ndim)
            term = np.ones([n] * ndim)
            for d in range(ndim):
                term = term * np.sin(2 * np.pi * k[d] * grids[ndim - 1 - d] + ph[d])
            f += rng.standard_normal() * term
        out[q] = f.reshape(-1) * (1.0 if q == 0 else (10.0 if q <= ndim else 1.0e3))
    return out


def probes(n, ndim, count=6, seed=5):
    return WL.probe_cells(n, ndim, count=count, seed=seed)
