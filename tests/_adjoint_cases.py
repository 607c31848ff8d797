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


# ---- two fluids, a flat interface (frozen geometry) ----

def interface_case(n, ndim=2, seed=3):
    """Acoustic pulse in air (fluid 0, x < ~0.5) near a flat water interface
    (the differentiable configuration's shape), over smooth background waves
    in every primitive of both fluids (density 3%, velocity 10 m/s along x
    and 5 m/s across, pressure 5e3 Pa) and a flow of 20 m/s along x.  Every
    component then varies from cell to cell by far more than the
    perturbations of the finite-difference checks, which keeps the WENO
    weights in their linear response (a nearly uniform component, such as
    the water's density in an acoustic wave, would not)."""
    if ndim == 2:
        c = WL.smooth_2d(n=n, seed=seed, width=0.15)
    else:
        c = _flat_case(n, ndim, seed)
    h = c["h"]
    x = (np.arange(n) + 0.5) * h
    grids = np.meshgrid(*([x] * ndim), indexing="ij")       # grids[d] varies along axis ndim-1-d

    def wave(ph):
        w = np.sin(2 * np.pi * (grids[ndim - 1].reshape(-1) + ph))
        for d in range(1, ndim):
            w = w * np.cos(2 * np.pi * (grids[ndim - 1 - d].reshape(-1) - 0.2 * d + ph))
        return w

    for k in (0, 1):
        rho = c["prim"][k, 0].mean()
        c["prim"][k, 0] *= 1.0 + 0.03 * wave(0.3 + 0.1 * k)
        c["prim"][k, 1] += 20.0 + 10.0 * wave(0.05 + 0.2 * k)
        for d in range(1, ndim):
            c["prim"][k, 1 + d] += 5.0 * wave(0.15 * d + 0.1 * k)
        c["prim"][k, ndim + 1] += 5.0e3 * wave(0.1)
        assert rho > 0
    return c


def curved_case(n, ndim=2, seed=3, radius=0.3):
    """A water column (2-D) or droplet (3-D) of the given radius at the
    centre, in air (phi = |x - c| - R, fluid 0 = water inside), with the same
    background waves as interface_case: the extension then runs along both
    or all axes with weights from the normal, and the mixing has diagonal
    targets."""
    h = 1.0 / n
    c0 = 0.5 + np.random.default_rng(seed).uniform(-0.3, 0.3, size=ndim) * h
    x = (np.arange(n) + 0.5) * h
    grids = np.meshgrid(*([x] * ndim), indexing="ij")
    r2 = 0.0
    for d in range(ndim):
        r2 = r2 + (grids[ndim - 1 - d].reshape(-1) - c0[d]) ** 2
    phi = np.sqrt(r2) - radius
    nc = n ** ndim
    prim = np.zeros((2, ndim + 2, nc))
    prim[0, 0] = 1000.0
    prim[0, ndim + 1] = 1.0e5
    prim[1, 0] = 1.0
    prim[1, ndim + 1] = 1.0e5
    c = dict(ndim=ndim, n=[n if d < ndim else 1 for d in range(3)], lo=[0.0, 0.0, 0.0], h=h,
             bc=[0, 0, 0], gamma=[4.4, 1.4], pinf=[6.0e8, 0.0], phi=phi, prim=prim,
             t_end=1e30, name="column_%dd" % ndim)
    _background(c, ndim, n)
    return c


def _background(c, ndim, n):
    """smooth waves in every primitive of both fluids (see interface_case)"""
    x = (np.arange(n) + 0.5) * c["h"]
    grids = np.meshgrid(*([x] * ndim), indexing="ij")

    def wave(ph):
        w = np.sin(2 * np.pi * (grids[ndim - 1].reshape(-1) + ph))
        for d in range(1, ndim):
            w = w * np.cos(2 * np.pi * (grids[ndim - 1 - d].reshape(-1) - 0.2 * d + ph))
        return w

    for k in (0, 1):
        c["prim"][k, 0] *= 1.0 + 0.03 * wave(0.3 + 0.1 * k)
        c["prim"][k, 1] += 20.0 + 10.0 * wave(0.05 + 0.2 * k)
        for d in range(1, ndim):
            c["prim"][k, 1 + d] += 5.0 * wave(0.15 * d + 0.1 * k)
        c["prim"][k, ndim + 1] += 5.0e3 * wave(0.1)


def _flat_case(n, ndim, seed):
    """air (x < xi) / water (x > xi) with a Gaussian pulse in the air, 1-D or 3-D"""
    h = 1.0 / n
    xi = 0.5 + np.random.default_rng(seed).uniform(-0.25, 0.25) * h
    x = (np.arange(n) + 0.5) * h
    grids = np.meshgrid(*([x] * ndim), indexing="ij")
    X = grids[ndim - 1].reshape(-1)
    r2 = (X - 0.4) ** 2
    for d in range(1, ndim):
        r2 = r2 + (grids[ndim - 1 - d].reshape(-1) - 0.5) ** 2
    pp = 1.0e3 * np.exp(-r2 / 0.15 ** 2)
    nc = n ** ndim
    prim = np.zeros((2, ndim + 2, nc))
    prim[0, 0] = 1.0 + pp / 1.4e5
    prim[0, ndim + 1] = 1.0e5 + pp
    prim[1, 0] = 1000.0
    prim[1, ndim + 1] = 1.0e5
    return dict(ndim=ndim, n=[n if d < ndim else 1 for d in range(3)], lo=[0.0, 0.0, 0.0], h=h,
                bc=[0, 0, 0], gamma=[1.4, 4.4], pinf=[0.0, 6.0e8], phi=X - xi, prim=prim,
                t_end=1e30, name="flat_%dd" % ndim, x_interface=xi)


def interface_probes(alpha, count=8, seed=5):
    """probe cells inside either fluid's bulk (alpha 1 or 0), seeded"""
    rng = np.random.default_rng(seed)
    pure = np.flatnonzero((alpha == 1.0) | (alpha == 0.0))
    return np.sort(rng.choice(pure, size=min(count, pure.size), replace=False))


def interface_loss(cons, alpha, gamma, pinf, probes, ndim):
    """J = sum over probes of (p - p0)^2 / 1e6 with p from the probe's own
    fluid; returns (J, dJ/dcons [2][NV][cells], dJ/d(gamma, p_inf) (2, 2))
    of the loss itself (at fixed cons)"""
    NV = ndim + 2
    g = np.zeros_like(cons)
    ge = np.zeros((2, 2))
    J = 0.0
    for c in probes:
        k = 0 if alpha[c] == 1.0 else 1
        U = cons[k, :, c]
        gm, pi = gamma[k], pinf[k]
        m2 = float(np.sum(U[1:ndim + 1] ** 2))
        p = (gm - 1.0) * (U[NV - 1] - 0.5 * m2 / U[0]) - gm * pi
        J += (p - P0) ** 2 / 1e6
        w = 2.0 * (p - P0) / 1e6
        g[k, 0, c] += w * (gm - 1.0) * 0.5 * m2 / U[0] ** 2
        for d in range(ndim):
            g[k, 1 + d, c] += -w * (gm - 1.0) * U[1 + d] / U[0]
        g[k, NV - 1, c] += w * (gm - 1.0)
        ge[k, 0] += w * (U[NV - 1] - 0.5 * m2 / U[0] - pi)
        ge[k, 1] += w * (-gm)
    return J, g, ge


def interface_direction(case, seed=7):
    """smooth seeded perturbation of both fluids' primitives, about 1% of
    the background waves: rho ~ 3e-4 rho, u ~ 0.1, p ~ 50"""
    ndim, n = case["ndim"], case["n"][0]
    out = np.zeros_like(case["prim"])
    one = direction(n, ndim, seed=seed)
    two = direction(n, ndim, seed=seed + 1)
    for k, src in ((0, one), (1, two)):
        out[k, 0] = src[0] * 3e-4 * case["prim"][k, 0].mean()
        for d in range(ndim):
            out[k, 1 + d] = src[1 + d] * 0.01
        out[k, ndim + 1] = src[ndim + 1] * 0.05
    return out


def state_scales(cons, ndim):
    """per (fluid, component) magnitude of contents [2][NV][cells], shaped
    (2, NV, 1): max |value|, momentum against sqrt(max rho max E)"""
    sc = np.zeros((2, ndim + 2, 1))
    for k in range(2):
        rho, E = np.abs(cons[k, 0]).max(), np.abs(cons[k, ndim + 1]).max()
        for q in range(ndim + 2):
            sc[k, q, 0] = max(np.abs(cons[k, q]).max(), 1e-300)
            if 1 <= q <= ndim:
                sc[k, q, 0] = max(sc[k, q, 0], np.sqrt(rho * E))
    return sc
