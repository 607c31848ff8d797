"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the CPU oracle.

This module only builds initial fields: a level set (signed distance to the
interface) and piecewise-constant primitive states per fluid.  It holds none
of the method's arithmetic; both the oracle and the GPU library turn these
primitives into cell contents themselves.

Fluid 0 is the fluid where phi < 0, fluid 1 where phi >= 0.  Arrays are
numpy float64 with x fastest: phi has shape (nz, ny, nx) squeezed to the
active dimensions, prim has shape (2, D+2, cells) with components
(rho, u_1..u_D, p).

Workloads (sizes follow the paper's compressible test section, Sec. 4.1-4.2,
re-posed with stiffened-gas water gamma=4.4, p_inf=6e8 Pa and air gamma=1.4):
  tube_1d          gas-water shock tube, water at 1e9 Pa | air at 1e5 Pa
  shock_bubble_2d  planar water shock (1e9 Pa) hitting an air bubble
  shock_droplet_3d Mach-1.5 air shock hitting a water droplet
  smooth_2d        Gaussian acoustic pulse in air crossing a flat interface
  droplet_2d       periodic translation of a water droplet (Sec. 4.2 analogue)
  pulse_air        acoustic pulse in a grid filled by air (differentiable runs)
  static_drop      Tait liquid drop in Tait air with surface tension (Sec. 4.3)
  oscillating_drop elliptic drop oscillating under surface tension (Sec. 4.5)
  batch_cases      many tubes and bubbles of uneven sizes (batched runs)
"""
from __future__ import annotations

import numpy as np

WATER = (4.4, 6.0e8)
AIR = (1.4, 0.0)

# Post-shock states used as inputs.  They satisfy the stiffened-gas
# Rankine-Hugoniot conditions; the oracle tests check that the exact Riemann
# solver reproduces a single shock between them and the pre-shock states.
WATER_SHOCK_1E9 = dict(rho=1230.377372836252, u=432.6921608084541, p=1.0e9)
AIR_SHOCK_M15 = dict(rho=1.8620689655172413, u=259.83731852596816, p=245833.33333333334)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _grid(ndim, n):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    if ndim == 1:
        return h, (x,)
    if ndim == 2:
        Y, X = np.meshgrid(x, x, indexing="ij")
        return h, (X, Y)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return h, (X, Y, Z)


def _case(ndim, n, bc, eos0, eos1, phi, prim, t_end, name, **extra):
    h = 1.0 / n
    d = dict(
        name=name, ndim=ndim, n=[n if i < ndim else 1 for i in range(3)],
        lo=[0.0, 0.0, 0.0], h=h, bc=[bc if i < ndim else 0 for i in range(3)],
        gamma=[eos0[0], eos1[0]], pinf=[eos0[1], eos1[1]],
        phi=np.ascontiguousarray(phi, dtype=np.float64).reshape(-1),
        prim=np.ascontiguousarray(prim, dtype=np.float64),
        t_end=t_end,
    )
    d.update(extra)
    return d


def _fill(ndim, ncell, state):
    """primitive block (D+2, cells) of one constant state, or per-cell arrays"""
    out = np.empty((ndim + 2, ncell))
    out[0] = state["rho"]
    for d in range(ndim):
        out[1 + d] = state.get("u%d" % d, state.get("u", 0.0) if d == 0 else 0.0)
    out[ndim + 1] = state["p"]
    return out


def tube_1d(n=400, seed=0, t_end=2.2e-4):
    """Gas-water shock tube: water (fluid 0) left of x_I, air (fluid 1) right.

    x_I = 0.5 + delta, delta ~ U(-1, 1) * h (seeded), phi = x - x_I.
    """
    h, (x,) = _grid(1, n)
    xi = 0.5 + _rng(seed).uniform(-1.0, 1.0) * h
    phi = x - xi
    prim = np.stack([_fill(1, n, dict(rho=1000.0, u=0.0, p=1.0e9)),
                     _fill(1, n, dict(rho=50.0, u=0.0, p=1.0e5))])
    return _case(1, n, 0, WATER, AIR, phi, prim, t_end, "tube_1d", x_interface=xi)


def tube_1d_single(n=200, seed=0, t_end=2e-4, left=None, right=None, eos=AIR):
    """Shock tube of one fluid across a 'material' interface of identical EOS."""
    h, (x,) = _grid(1, n)
    xi = 0.5 + _rng(seed).uniform(-1.0, 1.0) * h
    left = left or dict(rho=1.0, u=0.0, p=1.0e5)
    right = right or dict(rho=0.125, u=0.0, p=1.0e4)
    prim = np.stack([_fill(1, n, left), _fill(1, n, right)])
    return _case(1, n, 0, eos, eos, x - xi, prim, t_end, "tube_1d_single", x_interface=xi)


def shock_bubble_2d(n=1024, seed=0, radius=0.15, t_end=1.5e-4):
    """Planar water shock (post-shock p=1e9) hitting an air bubble.

    Air bubble (fluid 0, phi < 0 inside) of the given radius near (0.5, 0.5),
    centre jittered by U(-0.5, 0.5) h per axis; water (fluid 1) outside, at
    rest (rho=1000, p=1e5) ahead of the shock and in the post-shock state for
    x < 96/1024 (face aligned).
    """
    h, (X, Y) = _grid(2, n)
    r = _rng(seed)
    cx, cy = 0.5 + r.uniform(-0.5, 0.5) * h, 0.5 + r.uniform(-0.5, 0.5) * h
    phi = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2) - radius
    nc = n * n
    air = _fill(2, nc, dict(rho=1.0, p=1.0e5))
    water = _fill(2, nc, dict(rho=1000.0, p=1.0e5))
    xs = 96.0 / 1024.0
    post = (X.reshape(-1) < xs)
    water[0, post] = WATER_SHOCK_1E9["rho"]
    water[1, post] = WATER_SHOCK_1E9["u"]
    water[3, post] = WATER_SHOCK_1E9["p"]
    return _case(2, n, 0, AIR, WATER, phi, np.stack([air, water]), t_end,
                 "shock_bubble_2d", centre=(cx, cy), radius=radius)


def shock_droplet_3d(n=256, seed=0, radius=0.2, t_end=None):
    """Mach-1.5 air shock hitting a water droplet (fluid 0 inside)."""
    h, (X, Y, Z) = _grid(3, n)
    r = _rng(seed)
    c = [0.5 + r.uniform(-0.5, 0.5) * h for _ in range(3)]
    phi = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) - radius
    nc = n ** 3
    water = _fill(3, nc, dict(rho=1000.0, p=1.0e5))
    air = _fill(3, nc, dict(rho=1.0, p=1.0e5))
    post = (X.reshape(-1) < 51.0 / 256.0)
    air[0, post] = AIR_SHOCK_M15["rho"]
    air[1, post] = AIR_SHOCK_M15["u"]
    air[4, post] = AIR_SHOCK_M15["p"]
    return _case(3, n, 0, WATER, AIR, phi, np.stack([water, air]),
                 t_end if t_end is not None else 1e30, "shock_droplet_3d", centre=c, radius=radius)


def smooth_2d(n=512, seed=0, amp=1.0e3, width=0.05, t_end=None):
    """Gaussian pressure pulse in air (x < 0.5, fluid 0) near a flat water
    interface; isentropic density perturbation rho' = p'/c0^2, c0^2 = 1.4e5."""
    h, (X, Y) = _grid(2, n)
    xi = 0.5 + _rng(seed).uniform(-0.25, 0.25) * h
    phi = X - xi
    pp = amp * np.exp(-((X - 0.4) ** 2 + (Y - 0.5) ** 2) / width ** 2)
    nc = n * n
    air = _fill(2, nc, dict(rho=1.0, p=1.0e5))
    air[0] += (pp / 1.4e5).reshape(-1)
    air[3] += pp.reshape(-1)
    water = _fill(2, nc, dict(rho=1000.0, p=1.0e5))
    return _case(2, n, 0, AIR, WATER, phi, np.stack([air, water]),
                 t_end if t_end is not None else 1e30, "smooth_2d", x_interface=xi)


def droplet_2d(n=64, seed=0, radius=0.1, u=None, ndim=2):
    """Periodic translation of a water droplet in air (Sec. 4.2 analogue):
    water (fluid 0) inside radius R, both fluids moving with the same u."""
    h, grid = _grid(ndim, n)
    r = _rng(seed)
    c = [0.5 + r.uniform(-0.5, 0.5) * h for _ in range(ndim)]
    phi = np.sqrt(sum((g - ci) ** 2 for g, ci in zip(grid, c))) - radius
    nc = n ** ndim
    uu = 10.0 if u is None else u
    water = _fill(ndim, nc, dict(rho=1000.0, u=uu, p=1.0e5))
    air = _fill(ndim, nc, dict(rho=1.2, u=uu, p=1.0e5))
    return _case(ndim, n, 1, WATER, AIR, phi, np.stack([water, air]), 1.0 / uu,
                 "droplet_%dd" % ndim, centre=c, radius=radius)


def vacuum_tube_1d(n=200, U=3000.0):
    """Air | air pulled apart at -U | +U (Mach 8 at U = 3000 m/s): the
    interface cell empties and turns non-physical after some 30 cycles, the
    input of the tests of the non-physical-state handling."""
    h, (x,) = _grid(1, n)
    prim = np.zeros((2, 3, n))
    prim[:, 0] = 1.0
    prim[:, 1] = np.where(x < 0.5, -U, U)
    prim[:, 2] = 1.0e5
    return _case(1, n, 0, AIR, AIR, x - 0.5, prim, 1e30, "vacuum_tube_1d")


# Tait water of the paper's Sec. 4.1-4.2 (B = 3310, p0 = 1, gamma 7.15,
# non-dimensional): along an isentrope p + (B - p0) = B (rho/rho0)^gamma, the
# stiffened gas with p_inf = B - p0
TAIT_WATER = (7.15, 3310.0 - 1.0)


def e1_gas_water_tube(n=200):
    """Sec. 4.1.1 gas-water shock tube (non-dimensional): gas
    (rho, u, p) = (0.01, 0, 1000), gamma 2, for x < 0.5 and Tait water
    (1, 0, 1) for x > 0.5; t_end = 0.0008."""
    h, (x,) = _grid(1, n)
    gas = _fill(1, n, dict(rho=0.01, p=1000.0))
    water = _fill(1, n, dict(rho=1.0, p=1.0))
    return _case(1, n, 0, (2.0, 0.0), TAIT_WATER, x - 0.5, np.stack([gas, water]), 8.0e-4, "e1_gas_water_tube",
                 x_interface=0.5)


def e2_shock_air_water(n=200):
    """Sec. 4.1.2 underwater shock hitting an air-water interface
    (non-dimensional): shocked Tait water (1.0376, 6.0151, 1000) for
    x < 0.7 and air (0.001, 0, 1), gamma 1.4, for x > 0.7; t_end = 0.003."""
    h, (x,) = _grid(1, n)
    water = _fill(1, n, dict(rho=1.0376, u=6.0151, p=1000.0))
    air = _fill(1, n, dict(rho=0.001, p=1.0))
    return _case(1, n, 0, TAIT_WATER, (1.4, 0.0), x - 0.7, np.stack([water, air]), 3.0e-3, "e2_shock_air_water",
                 x_interface=0.7)


def e3_droplet(n=64, ndim=2):
    """Sec. 4.2 periodic translation of a water droplet (non-dimensional):
    Tait water (rho 1000, p 1) inside radius 0.1 at the centre of the unit
    box, air (1.2, 1), gamma 1.4, outside, both moving with u = sqrt(10)/100
    along x; periodic; one period t_end = 10 sqrt(10)."""
    h, grid = _grid(ndim, n)
    r = np.sqrt(sum((g - 0.5) ** 2 for g in grid))
    nc = n ** ndim
    u = np.sqrt(10.0) / 100.0
    water = _fill(ndim, nc, dict(rho=1000.0, u=u, p=1.0))
    air = _fill(ndim, nc, dict(rho=1.2, u=u, p=1.0))
    return _case(ndim, n, 1, TAIT_WATER, (1.4, 0.0), r - 0.1, np.stack([water, air]), 10.0 * np.sqrt(10.0),
                 "e3_droplet_%dd" % ndim, radius=0.1)


# Sec. 4.3 fluids (non-dimensional), Tait's equation with p0 = 1000 as the
# stiffened gas p_inf = B - p0: liquid B = 5e5, gamma 7.15; air B = 100,
# gamma 1.4 (p_inf = -900: the air holds p > 900)
DROP_LIQUID = (7.15, 5.0e5 - 1.0e3)
DROP_AIR = (1.4, 100.0 - 1.0e3)


def static_drop(n=64, ndim=2, seed=0, radius=0.1, sigma=36.0, equilibrium=True, t_end=0.02):
    """Sec. 4.3 static drop: liquid (fluid 0, rho 1000) of radius 0.1 at the
    centre of the unit box (offset by a seeded fraction of a cell), air
    (rho 1) outside, both at rest, surface tension sigma = 36; zero-gradient
    boundaries.  The paper starts both fluids at p0 = 1000 and lets the drop
    relax to the Laplace jump sigma (D - 1) / R; with `equilibrium` the drop
    starts at that pressure, the state the relaxation ends in."""
    h, grid = _grid(ndim, n)
    r = _rng(seed)
    c = [0.5 + r.uniform(-0.5, 0.5) * h for _ in range(ndim)]
    phi = np.sqrt(sum((g - ci) ** 2 for g, ci in zip(grid, c))) - radius
    nc = n ** ndim
    jump = sigma * (ndim - 1) / radius if equilibrium else 0.0
    liquid = _fill(ndim, nc, dict(rho=1000.0, p=1.0e3 + jump))
    air = _fill(ndim, nc, dict(rho=1.0, p=1.0e3))
    return _case(ndim, n, 0, DROP_LIQUID, DROP_AIR, phi, np.stack([liquid, air]), t_end,
                 "static_drop_%dd" % ndim, centre=c, radius=radius, sigma=sigma)


def _ellipse_distance(X, Y, a, b, iters=16):
    """signed distance to the ellipse x^2/a^2 + y^2/b^2 = 1 (negative
    inside), from the foot point x = a cos t, y = b sin t found by Newton's
    method on the orthogonality condition, in the first quadrant, started
    from several angles (inside the evolute a point has several foot
    points): the nearest one found"""
    x, y = np.abs(X), np.abs(Y)
    best = np.minimum(np.hypot(a - x, y), np.hypot(x, b - y))
    starts = [np.arctan2(a * y, b * x)] + [np.full_like(x, v) for v in np.linspace(0.05, 0.5 * np.pi - 0.05, 5)]
    for t in starts:
        for _ in range(iters):
            ct, st = np.cos(t), np.sin(t)
            f = (a * a - b * b) * st * ct - a * x * st + b * y * ct
            df = (a * a - b * b) * (ct * ct - st * st) - a * x * ct - b * y * st
            t = np.clip(t - f / np.where(np.abs(df) > 1e-300, df, 1e-300), 0.0, 0.5 * np.pi)
        best = np.minimum(best, np.hypot(a * np.cos(t) - x, b * np.sin(t) - y))
    inside = (x / a) ** 2 + (y / b) ** 2 < 1.0
    return np.where(inside, -best, best)


# Sec. 4.5 fluids: gas B = 500, gamma 1.4; liquid B = 2e5, gamma 7.15; p0 = 1e4
OSC_LIQUID = (7.15, 2.0e5 - 1.0e4)
OSC_GAS = (1.4, 500.0 - 1.0e4)


def oscillating_drop(n=128, seed=0, sigma=341.642, t_end=0.1):
    """Sec. 4.5 drop oscillation: an elliptic liquid drop (fluid 0, rho 100,
    semi-axes 0.2 along x and 0.12 along y) at the centre of the unit box,
    gas (rho 1) outside, at rest at p0 = 1e4, surface tension sigma =
    341.642; the level set is the signed distance to the ellipse (the paper
    reinitialises its implicit function before the run).  Mode 2 of
    Rayleigh's formula extended to two fluids, Eq. (oscillation), with the
    paper's R = 0.15825, gives the period 0.0878."""
    h, (X, Y) = _grid(2, n)
    r = _rng(seed)
    c = [0.5 + r.uniform(-0.5, 0.5) * h for _ in range(2)]
    phi = _ellipse_distance(X - c[0], Y - c[1], 0.2, 0.12)
    nc = n * n
    liquid = _fill(2, nc, dict(rho=100.0, p=1.0e4))
    gas = _fill(2, nc, dict(rho=1.0, p=1.0e4))
    return _case(2, n, 0, OSC_LIQUID, OSC_GAS, phi, np.stack([liquid, gas]), t_end, "oscillating_drop",
                 centre=c, sigma=sigma, period=0.0878)


def wall_bubble_2d(n=64, seed=0, radius=0.2):
    """Air bubble (fluid 0) cut by the zero-gradient wall x = 0, at a higher
    pressure than the surrounding water: the interface band touches the wall,
    so extension, level set and mixing all meet the boundary."""
    h, (X, Y) = _grid(2, n)
    r = _rng(seed)
    cx, cy = r.uniform(-0.5, 0.5) * h, 0.5 + r.uniform(-0.5, 0.5) * h
    phi = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2) - radius
    nc = n * n
    air = _fill(2, nc, dict(rho=5.0, p=5.0e5))
    water = _fill(2, nc, dict(rho=1000.0, p=1.0e5))
    return _case(2, n, 0, AIR, WATER, phi, np.stack([air, water]), 1e30, "wall_bubble_2d", centre=(cx, cy))


def entropy_wave_1d(n=64, amp=0.2, u=1.0, p=1.0, t_end=0.1):
    """Single fluid (phi < 0 everywhere) smooth density wave on a periodic
    domain: rho = 1 + amp sin(2 pi x), uniform u and p.  Exact solution is a
    translation by u t."""
    h, (x,) = _grid(1, n)
    phi = -np.ones(n)
    st = np.stack([np.ones(n), np.full(n, u), np.full(n, p)])
    st[0] = 1.0 + amp * np.sin(2 * np.pi * x)
    prim = np.stack([st, np.stack([np.ones(n), np.zeros(n), np.ones(n)])])
    return _case(1, n, 1, (1.4, 0.0), (1.4, 0.0), phi, prim, t_end, "entropy_wave_1d")


def pulse_air(n=64, ndim=2, seed=0, amp=1.0e3, width=0.05, bc=0, t_end=None, u0=None, bg=0.0):
    """Single fluid (air, phi < 0 everywhere): a Gaussian pressure pulse
    p' = amp exp(-|x - x0|^2 / width^2) with rho' = p'/c0^2 (c0^2 = 1.4e5),
    centred near (0.4, 0.5, 0.5) with a seeded sub-cell offset, in air at
    rest or moving with the uniform velocity u0 (one entry per direction),
    optionally over a smooth background wave of amplitude bg (Pa),
    bg sin(2 pi (x + 0.1)) cos(2 pi (y - 0.2)) ..., with the same isentropic
    density perturbation.
    The smooth acoustic case of the differentiable configuration without its
    water half (the adjoint covers runs in which one fluid fills the grid)."""
    h, grid = _grid(ndim, n)
    r = _rng(seed)
    c0 = [0.4, 0.5, 0.5][:ndim]
    c = [ci + r.uniform(-0.5, 0.5) * h for ci in c0]
    r2 = sum((g - ci) ** 2 for g, ci in zip(grid, c))
    pp = amp * np.exp(-r2 / width ** 2)
    if bg:
        wave = np.sin(2 * np.pi * (grid[0] + 0.1))
        for d in range(1, ndim):
            wave = wave * np.cos(2 * np.pi * (grid[d] - 0.2 * d))
        pp = pp + bg * wave
    pp = pp.reshape(-1)
    nc = n ** ndim
    air = _fill(ndim, nc, dict(rho=1.0, p=1.0e5))
    air[0] += pp / 1.4e5
    air[ndim + 1] += pp
    if u0 is not None:
        for d in range(ndim):
            air[1 + d] = u0[d]
    other = _fill(ndim, nc, dict(rho=1000.0, p=1.0e5))
    phi = -np.ones(nc)
    return _case(ndim, n, bc, AIR, WATER, phi, np.stack([air, other]),
                 t_end if t_end is not None else 1e30, "pulse_air_%dd" % ndim, centre=c)


def batch_cases(seed=0, n_tubes=384, n_bubbles=128, tube_n=(200, 4000), bubble_n=(64, 512)):
    """Independent instances of uneven sizes for a batch.

    Tubes: 1-D water (fluid 0, left) | air (fluid 1, right), N ~ U{tube_n},
    interface at 0.5 + U(-1, 1) h; water at rho = 1000, p = 1e5 * Rp, air at
    rho = 1000 / Rr, p = 1e5, at rest.  Bubbles: 2-D air bubble (fluid 0) of
    radius U(0.1, 0.3) near the centre of water (fluid 1) on an n^2 grid,
    n ~ U{bubble_n}; water at rho = 1000, p = 1e5 * Rp, air at rho =
    1000 / Rr, p = 1e5 (a collapsing bubble).  The density and pressure
    ratios are drawn log-uniform: Rr in [1, 1e3], Rp in [1, 1e4].
    Expected cells at the default sizes: 384 * 2100 = 0.8M in 1-D and
    128 * 99.7k = 12.8M in 2-D.
    """
    r = _rng(seed + 7000)
    cases = []
    for i in range(n_tubes):
        n = int(r.integers(tube_n[0], tube_n[1] + 1))
        rr, rp = 10.0 ** r.uniform(0.0, 3.0), 10.0 ** r.uniform(0.0, 4.0)
        h, (x,) = _grid(1, n)
        xi = 0.5 + r.uniform(-1.0, 1.0) * h
        prim = np.stack([_fill(1, n, dict(rho=1000.0, u=0.0, p=1.0e5 * rp)),
                         _fill(1, n, dict(rho=1000.0 / rr, u=0.0, p=1.0e5))])
        cases.append(_case(1, n, 0, WATER, AIR, x - xi, prim, 1.0, "batch_tube_%d" % i, ratios=(rr, rp)))
    for i in range(n_bubbles):
        n = int(r.integers(bubble_n[0], bubble_n[1] + 1))
        rr, rp = 10.0 ** r.uniform(0.0, 3.0), 10.0 ** r.uniform(0.0, 4.0)
        rad = r.uniform(0.1, 0.3)
        h, (X, Y) = _grid(2, n)
        cx, cy = 0.5 + r.uniform(-0.5, 0.5) * h, 0.5 + r.uniform(-0.5, 0.5) * h
        phi = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2) - rad
        nc = n * n
        prim = np.stack([_fill(2, nc, dict(rho=1000.0 / rr, p=1.0e5)),
                         _fill(2, nc, dict(rho=1000.0, p=1.0e5 * rp))])
        cases.append(_case(2, n, 0, AIR, WATER, phi, prim, 1.0, "batch_bubble_%d" % i, radius=rad,
                           ratios=(rr, rp)))
    return cases


def probe_cells(n, ndim=2, count=16, seed=0):
    """Seeded distinct cell indices (x fastest) for a pressure-probe loss."""
    r = _rng(seed + 1000)
    return np.sort(r.choice(n ** ndim, size=count, replace=False))


def CONFIGS():
    """The named workloads and their sizes (used by the benchmark)."""
    return {
        "tube_1d": dict(fn=tube_1d, kw=dict(n=400)),
        "shock_bubble_2d": dict(fn=shock_bubble_2d, kw=dict(n=1024)),
        "shock_droplet_3d": dict(fn=shock_droplet_3d, kw=dict(n=256)),
        "smooth_2d": dict(fn=smooth_2d, kw=dict(n=512)),
    }
