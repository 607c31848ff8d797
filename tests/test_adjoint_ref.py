"""Pins of the oracle-side reference gradient (oracle/adjoint_ref.py): its
forward equals the C oracle on single-fluid runs, and its autograd gradient
equals central finite differences of its own forward with the step lengths
held fixed (the frozen schedule the adjoint differentiates)."""
import numpy as np
import pytest
import torch

from paper_1905_03917_amd import workloads as WL

import _adjoint_cases as AC


def _ref():
    from oracle import adjoint_ref as R
    return R


@pytest.mark.parametrize("ndim,n,bc", [(1, 48, 0), (1, 40, 1), (2, 20, 0), (2, 18, 1)])
def test_reference_forward_matches_oracle(oracle, ndim, n, bc):
    R = _ref()
    c = WL.pulse_air(n=n, ndim=ndim, seed=3, bc=bc, width=0.15)
    o = oracle.OracleSim(c)
    so = o.advance(1.0, mode=0, max_cycles=6)
    _, co, _ = o.state()
    prim0 = torch.tensor(c["prim"][0])
    U, dts = R.run(prim0, torch.tensor(c["gamma"][0], dtype=torch.float64), torch.tensor(c["pinf"][0], dtype=torch.float64),
                   c, so["t"])
    assert len(dts) == so["steps"][0]
    U = U.numpy()
    scale = np.abs(co[0]).max(axis=1, keepdims=True)
    scale[1:ndim + 1] = max(scale[0, 0] * 1.0, 1.0)
    err = (np.abs(U - co[0]) / scale).max()
    assert err < 1e-12, err


def _loss(R, U, gamma, pinf, probes):
    p = R.pressure(U, gamma, pinf)
    return ((p[probes] - AC.P0) ** 2).sum() / 1e6


@pytest.mark.parametrize("ndim,n,bc", [(1, 32, 0), (2, 12, 1)])
def test_reference_gradient_matches_finite_differences(ndim, n, bc):
    R = _ref()
    c = AC.case(n, ndim, bc=bc)
    probes = torch.tensor(AC.probes(n, ndim))
    prim0 = torch.tensor(c["prim"][0], requires_grad=True)
    gam = torch.tensor(1.4, dtype=torch.float64, requires_grad=True)
    pin = torch.tensor(2.0e4, dtype=torch.float64, requires_grad=True)
    # a fixed schedule of 5 steps from the CFL of the initial state
    U0 = R.prim2cons(prim0.detach().reshape([ndim + 2] + [n] * ndim), 1.4, 2.0e4)
    dts = [R.cfl_dt(U0, 1.4, 2.0e4, c["h"], 0.6)] * 5
    U, _ = R.run(prim0, gam, pin, c, 1e30, dts=dts)
    J = _loss(R, U, gam, pin, probes)
    J.backward()

    def J_at(x, g, p):
        with torch.no_grad():
            Ux, _ = R.run(x, torch.tensor(g, dtype=torch.float64), torch.tensor(p, dtype=torch.float64), c, 1e30,
                          dts=dts)
            return float(_loss(R, Ux, g, p, probes))

    x0 = prim0.detach()
    for q, eps in enumerate([1e-7] + [1e-6] * (ndim + 1)):
        dirn = torch.zeros_like(x0)
        dirn[q] = torch.tensor(AC.direction(n, ndim, seed=11 + q)[q])
        ad = float((prim0.grad * dirn).sum())
        fd = (J_at(x0 + eps * dirn, 1.4, 2.0e4) - J_at(x0 - eps * dirn, 1.4, 2.0e4)) / (2 * eps)
        assert abs(ad - fd) <= 1e-5 * abs(fd), (q, ad, fd)
    for par, val, hrel in ((gam, 1.4, 1e-6), (pin, 2.0e4, 1e-6)):
        e = val * hrel
        if par is gam:
            fd = (J_at(x0, val + e, 2.0e4) - J_at(x0, val - e, 2.0e4)) / (2 * e)
        else:
            fd = (J_at(x0, 1.4, val + e) - J_at(x0, 1.4, val - e)) / (2 * e)
        assert abs(float(par.grad) - fd) <= 1e-6 * abs(fd), (float(par.grad), fd)
