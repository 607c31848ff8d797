"""Reference gradients of single-fluid runs, by PyTorch autograd on the CPU.

TEST INFRASTRUCTURE ONLY: imported by the test suite.  The product path never
imports it.

A plain, vectorised FP64 restatement of the update that the adjoint covers:
one fluid fills a uniform grid (zero-gradient or periodic boundaries), the
stiffened-gas EOS (Sec. 2.1), the face flux of Sec. 2.1 with local
Lax-Friedrichs splitting (speed = max of |u_n| + c over the six-cell stencil)
and WENO5-JS per conservative component, and the Shu-Osher Runge-Kutta
stages (SSP-RK3, or the paper's TVD-RK2).  The step lengths come from the
CFL condition evaluated on the forward state and are held constant for the
derivative (the same frozen schedule the GPU adjoint differentiates).
Autograd then gives d loss / d (initial primitives, gamma, p_inf).

Its forward is pinned to the C oracle on the same inputs, and its gradient
to central finite differences of itself.
"""
from __future__ import annotations

import torch

RK3_A = (0.0, 0.75, 1.0 / 3.0)
RK2_A = (0.0, 0.5)


def prim2cons(W, gamma, pinf):
    """W: (D+2, *shape) = rho, u_1..u_D, p -> U = rho, rho u, E"""
    D = W.shape[0] - 2
    rho, p = W[0], W[D + 1]
    u = W[1:D + 1]
    E = (p + gamma * pinf) / (gamma - 1.0) + 0.5 * rho * (u * u).sum(0)
    return torch.cat([rho[None], rho[None] * u, E[None]], 0)


def cons2prim(U, gamma, pinf):
    D = U.shape[0] - 2
    rho = U[0]
    u = U[1:D + 1] / rho
    p = (gamma - 1.0) * (U[D + 1] - 0.5 * rho * (u * u).sum(0)) - gamma * pinf
    return rho, u, p


def weno5(v0, v1, v2, v3, v4, eps):
    """WENO5-JS value at the right edge of v2 from the left-biased stencil."""
    q0 = (2 * v0 - 7 * v1 + 11 * v2) / 6
    q1 = (-v1 + 5 * v2 + 2 * v3) / 6
    q2 = (2 * v2 + 5 * v3 - v4) / 6
    b0 = 13 / 12 * (v0 - 2 * v1 + v2) ** 2 + 0.25 * (v0 - 4 * v1 + 3 * v2) ** 2
    b1 = 13 / 12 * (v1 - 2 * v2 + v3) ** 2 + 0.25 * (v1 - v3) ** 2
    b2 = 13 / 12 * (v2 - 2 * v3 + v4) ** 2 + 0.25 * (3 * v2 - 4 * v3 + v4) ** 2
    a0 = 0.1 / (eps + b0) ** 2
    a1 = 0.6 / (eps + b1) ** 2
    a2 = 0.3 / (eps + b2) ** 2
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def _pad(x, axis, bc):
    """three ghost layers on both ends of `axis` (zero-gradient copies or periodic images)"""
    n = x.shape[axis]
    if bc == 1:
        idx = [(i % n) for i in range(-3, n + 3)]
    else:
        idx = [min(max(i, 0), n - 1) for i in range(-3, n + 3)]
    return torch.index_select(x, axis, torch.tensor(idx))


def rhs(U, gamma, pinf, h, bc, eps):
    """L(U) = sum_d (F_{i-1/2} - F_{i+1/2}) / h over the grid's directions.
    U: (NV, n_z?, n_y?, n_x) with x the last axis."""
    NV = U.shape[0]
    D = NV - 2
    L = torch.zeros_like(U)
    for d in range(D):
        axis = U.dim() - 1 - d              # x is the last array axis
        Up = _pad(U, axis, bc[d])
        rho, u, p = cons2prim(Up, gamma, pinf)
        c = torch.sqrt(gamma * (p + pinf) / rho)
        un = u[d]
        F = torch.empty_like(Up)
        F[0] = Up[1 + d]
        for e in range(D):
            F[1 + e] = Up[1 + e] * un + (p if e == d else 0.0)
        F[D + 1] = (Up[D + 1] + p) * un
        n = U.shape[axis]
        nf = n + 1

        def sl(x, start, ax):      # slice of length nf starting at `start` along ax
            return torch.narrow(x, ax, start, nf)

        # face f (0..n) lies between cells f-1 and f; padded index of cell j is j + 3
        # LLF speed: the largest |u_n| + c of the six stencil cells.  The
        # map is not differentiable where two of them tie; the derivative
        # taken there is that of the first maximal cell in stencil order
        # (upwind to downwind), a one-sided derivative of the max
        s = (torch.abs(un) + c)
        S6 = torch.stack([sl(s, m, axis - 1) for m in range(6)], 0)
        first = torch.argmax(S6, dim=0, keepdim=True)       # first maximal index
        amax = torch.gather(S6, 0, first).squeeze(0)
        Fh = []
        for q in range(NV):
            fp = [0.5 * (sl(F[q], m, axis - 1) + amax * sl(Up[q], m, axis - 1)) for m in range(6)]
            fm = [0.5 * (sl(F[q], m, axis - 1) - amax * sl(Up[q], m, axis - 1)) for m in range(6)]
            Fh.append(weno5(fp[0], fp[1], fp[2], fp[3], fp[4], eps) + weno5(fm[5], fm[4], fm[3], fm[2], fm[1], eps))
        Fh = torch.stack(Fh, 0)
        L = L + (torch.narrow(Fh, axis, 0, n) - torch.narrow(Fh, axis, 1, n)) / h
    return L


def cfl_dt(U, gamma, pinf, h, cfl):
    rho, u, p = cons2prim(U, gamma, pinf)
    c = torch.sqrt(gamma * (p + pinf) / rho)
    s = sum((torch.abs(u[d]) + c) / h for d in range(u.shape[0]))
    return cfl / float(s.max())


def run(prim0, gamma, pinf, case, t_end, rk=3, cfl=0.6, eps=1e-6, dts=None):
    """Advance the single-fluid state from primitives prim0 (D+2, cells) to
    t_end; returns (U_final (D+2, cells), list of step lengths).  Step
    lengths are computed from the state (detached) unless `dts` is given."""
    D = int(case["ndim"])
    shape = [int(case["n"][d]) for d in reversed(range(D))]
    bc = [int(case["bc"][d]) for d in range(D)]
    h = float(case["h"])
    W = prim0.reshape([D + 2] + shape)
    U = prim2cons(W, gamma, pinf)
    A = RK3_A if rk == 3 else RK2_A
    t = 0.0
    out_dts = []
    k = 0
    while t < t_end and (dts is None or k < len(dts)):
        if dts is None:
            dt = cfl_dt(U.detach(), float(gamma), float(pinf), h, cfl)
            if dt > t_end - t:
                dt = t_end - t
        else:
            dt = dts[k]
        U0 = U
        Us = U0
        for a in A:
            Un = Us + dt * rhs(Us, gamma, pinf, h, bc, eps)
            Us = Un if a == 0.0 else a * U0 + (1.0 - a) * Un
        U = Us
        out_dts.append(dt)
        t += dt
        k += 1
        if t_end - t <= 1e-14 * t_end:
            t = t_end
    return U.reshape(D + 2, -1), out_dts


def pressure(U, gamma, pinf):
    _, _, p = cons2prim(U, gamma, pinf)
    return p
