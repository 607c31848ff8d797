"""Pins of the oracle's full scheme: conservation (Sec. 4.2 reports relative
droplet mass 1), equilibrium preservation, convergence order of the single-
fluid WENO5/RK3 core, shock tubes against the exact solution, linear acoustic
transmission at a material interface, reinitialisation to a distance function.
"""
import math

import numpy as np
import pytest

from paper_1905_03917_amd import workloads as WL


def _ledger(o, st, tot0):
    tot1 = o.totals()
    bf = st["bflux"]
    mass = (tot1[:, 0] - tot0[:, 0] - bf[:, 0]) / np.maximum(np.abs(tot0[:, 0]), 1e-300)
    scale = np.abs(tot0).sum(0) + np.abs(tot1).sum(0) + np.abs(bf).sum(0)
    D = o.D
    scale[1:D + 1] = scale[1:D + 1].sum()          # one scale for all momentum components
    tot = (tot1.sum(0) - tot0.sum(0) - bf.sum(0))
    return mass, tot, scale


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", ["tube", "bubble", "droplet3d"])
def test_conservation_to_round_off(oracle, mode, name):
    if name == "tube":
        c, t, mc = WL.tube_1d(n=200, seed=1), 1e-4, 0
    elif name == "bubble":
        c, t, mc = WL.shock_bubble_2d(n=48, seed=2), 3e-5, 6
    else:
        c, t, mc = WL.shock_droplet_3d(n=16, seed=3), 1e-3, 2
    o = oracle.OracleSim(c)
    tot0 = o.totals()
    st = o.advance(t, mode=mode, max_cycles=mc)
    mass, tot, scale = _ledger(o, st, tot0)
    steps = max(st["steps"])
    assert np.all(np.abs(mass) < 1e-13 * steps), mass
    D = c["ndim"]
    for q in range(D + 2):
        assert abs(tot[q]) <= 1e-13 * steps * scale[q] + 1e-300, (q, tot[q], scale[q])


def test_multi_dt_needs_the_correction(oracle):
    """Without the interfacial flux correction the accelerated cycle is not
    conservative (Sec. 3.1); with it the ledger closes."""
    c = WL.tube_1d(n=200, seed=4)
    res = {}
    for nc in (0, 1):
        o = oracle.OracleSim(c, no_correction=nc)
        tot0 = o.totals()
        st = o.advance(1e-4, mode=1)
        assert st["steps"][1] < st["steps"][0]          # air is the slow fluid
        _, tot, scale = _ledger(o, st, tot0)
        res[nc] = abs(tot[2]) / scale[2]
    assert res[0] < 1e-13
    assert res[1] > 1e-8


@pytest.mark.parametrize("mode", [0, 1])
def test_pressure_velocity_equilibrium(oracle, mode):
    """Uniform p and u across an interface between different fluids stay
    uniform (static air bubble in water)."""
    c = WL.shock_bubble_2d(n=32, seed=5)
    pr = c["prim"]
    pr[1, 0], pr[1, 1], pr[1, 3] = 1000.0, 0.0, 1e5
    o = oracle.OracleSim(c)
    o.advance(1.0, mode=mode, max_cycles=4)
    phi, cons, alpha = o.state()
    for k, (g, pi) in enumerate([WL.AIR, WL.WATER]):
        a = alpha if k == 0 else 1 - alpha
        m = a >= 0.5
        rho = cons[k, 0][m] / a[m]
        mx, my, E = cons[k, 1][m] / a[m], cons[k, 2][m] / a[m], cons[k, 3][m] / a[m]
        p = (g - 1) * (E - 0.5 * (mx ** 2 + my ** 2) / rho) - g * pi
        assert np.abs(p - 1e5).max() < 1e-9 * (1e5 + pi)
        assert np.abs(mx / rho).max() < 1e-5          # m/s, against sound speeds of 374 and 1625


def _entropy_error(oracle, n, cfl, t_end=0.1):
    c = WL.entropy_wave_1d(n=n, t_end=t_end)
    o = oracle.OracleSim(c, cfl=cfl)
    o.advance(t_end, mode=0)
    _, cons, _ = o.state()
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    # the initial cell values are samples of 1 + 0.2 sin(2 pi x); the exact
    # discrete solution is the same samples translated by u t (u = 1)
    exact = 1.0 + 0.2 * np.sin(2 * np.pi * (x - t_end))
    return np.abs(cons[0, 0] - exact).mean()


def test_entropy_wave_space_order(oracle):
    e = [_entropy_error(oracle, n, 0.05) for n in (32, 64)]
    assert e[0] / e[1] > 2 ** 4.3, e


def _entropy_solution(oracle, n, cfl, t_end=0.2):
    c = WL.entropy_wave_1d(n=n, t_end=t_end)
    o = oracle.OracleSim(c, cfl=cfl)
    o.advance(t_end, mode=0)
    return o.state()[1][0, 0]


def test_entropy_wave_time_order(oracle):
    """Differences to a small-CFL run remove the spatial error: SSP-RK3 gives
    a ratio near 2^3 per halving of the time step."""
    ref = _entropy_solution(oracle, 128, 0.05)
    d = [np.abs(_entropy_solution(oracle, 128, cfl) - ref).mean() for cfl in (0.8, 0.4)]
    assert d[0] / d[1] > 2 ** 2.7, d


def _tube_l1(oracle, c, mode, lo=0.0):
    o = oracle.OracleSim(c)
    o.advance(c["t_end"], mode=mode)
    _, cons, alpha = o.state()
    n = c["n"][0]
    x = (np.arange(n) + 0.5) / n
    ex = oracle.exact_tube(c, x, c["t_end"])
    a0 = np.maximum(alpha, 1e-300)
    a1 = np.maximum(1 - alpha, 1e-300)
    rho = np.where(alpha >= 0.5, cons[0, 0] / a0, cons[1, 0] / a1)
    u = np.where(alpha >= 0.5, cons[0, 1] / a0, cons[1, 1] / a1) / rho
    m = x >= lo
    return np.mean(np.abs(rho - ex[:, 0])[m]), np.mean(np.abs(u - ex[:, 1])[m]), rho, u


def test_single_gas_tube_converges(oracle):
    errs = []
    for n in (100, 200, 400):
        c = WL.tube_1d_single(n=n, seed=0, t_end=6e-4)
        errs.append(_tube_l1(oracle, c, 0)[0])
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] / errs[2] > 2.5, errs


@pytest.mark.slow
def test_gas_water_tube_converges_both_modes(oracle):
    """1-D gas-water tube vs the exact solution on x >= 0.25; the accelerated
    method's error against the original is below the original's own error."""
    res = {}
    for n in (200, 400, 800):
        c = WL.tube_1d(n=n, seed=0)
        e0, _, r0, _ = _tube_l1(oracle, c, 0, 0.25)
        e1, _, r1, _ = _tube_l1(oracle, c, 1, 0.25)
        x = (np.arange(n) + 0.5) / n
        dmulti = np.mean(np.abs(r1 - r0)[x >= 0.25])
        res[n] = (e0, e1, dmulti)
        assert dmulti < e0
    assert res[200][0] > res[400][0] > res[800][0]
    assert res[200][1] > res[400][1] > res[800][1]


def test_gas_water_interface_velocity(oracle):
    c = WL.tube_1d(n=400, seed=2)
    _, u_err, rho, u = _tube_l1(oracle, c, 1, 0.25)
    x = (np.arange(400) + 0.5) / 400
    st = oracle.riemann([1000.0, 0.0, 1e9], [50.0, 0.0, 1e5], 4.4, 6e8, 1.4, 0.0)
    xi = c["x_interface"] + st[1] * c["t_end"]
    # the star region spans the water rarefaction tail .. the air shock
    # (0.022 ahead of the interface at t_end): look at [xi - 0.03, xi + 0.008]
    near = (x > xi - 0.03) & (x < xi + 0.008)
    assert np.abs(u[near] - st[1]).max() < 0.01 * st[1]


@pytest.mark.parametrize("mode", [0, 1])
def test_acoustic_transmission(oracle, mode):
    """A weak pulse in air hitting water: transmitted pressure amplitude
    T = 2 Z2/(Z1+Z2), reflected R = (Z2-Z1)/(Z1+Z2), Z = rho c (linear acoustics)."""
    n = 400
    x = (np.arange(n) + 0.5) / n
    xi = 0.5 + 0.3 / n
    A, w, x0 = 100.0, 0.03, 0.3
    c_air = math.sqrt(1.4e5)
    c_w = math.sqrt(4.4 * (1e5 + 6e8) / 1000.0)
    pp = A * np.exp(-((x - x0) / w) ** 2)
    air = np.stack([1.0 + pp / c_air ** 2, pp / c_air, 1e5 + pp])
    water = np.stack([np.full(n, 1000.0), np.zeros(n), np.full(n, 1e5)])
    c = WL._case(1, n, 0, WL.AIR, WL.WATER, x - xi, np.stack([air, water]), 7.5e-4, "acoustic")
    o = oracle.OracleSim(c)
    st = o.advance(7.5e-4, mode=mode)
    _, cons, alpha = o.state()
    # pressure of each fluid from its cell-average state
    a1 = np.maximum(1 - alpha, 1e-300)
    rho1, m1, E1 = cons[1, 0] / a1, cons[1, 1] / a1, cons[1, 2] / a1
    with np.errstate(invalid="ignore", divide="ignore"):
        pw = (4.4 - 1) * (E1 - 0.5 * m1 ** 2 / rho1) - 4.4 * 6e8
        pa = (1.4 - 1) * (cons[0, 2] / np.maximum(alpha, 1e-300) - 0.5 * (cons[0, 1] / np.maximum(alpha, 1e-300)) ** 2 / (cons[0, 0] / np.maximum(alpha, 1e-300)))
    Z1, Z2 = 1.0 * c_air, 1000.0 * c_w
    T, R = 2 * Z2 / (Z1 + Z2), (Z2 - Z1) / (Z1 + Z2)
    trans = np.nanmax(np.where((x > 0.6) & (1 - alpha >= 0.5), pw, np.nan)) - 1e5
    refl = np.nanmax(np.where((x < 0.48) & (alpha >= 0.5), pa, np.nan)) - 1e5
    assert trans == pytest.approx(T * A, rel=0.03)
    assert refl == pytest.approx(R * A, rel=0.03)
    if mode == 1:
        assert st["steps"][1] > st["steps"][0]       # water sub-stepped


def test_reinit_restores_distance(oracle):
    """Static interface with the non-distance level set (r^2 - R^2)/(2R):
    only the reinitialisation moves phi; the band converges toward r - R and
    cells next to the interface are left untouched."""
    n, R = 64, 0.3
    x = (np.arange(n) + 0.5) / n
    Y, X = np.meshgrid(x, x, indexing="ij")
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2)
    phi0 = ((r ** 2 - R ** 2) / (2 * R)).reshape(-1)
    prim = np.zeros((2, 4, n * n))
    prim[:, 0] = 1.0
    prim[:, 3] = 1e5
    c = WL._case(2, n, 0, WL.AIR, WL.AIR, phi0, prim, 1.0, "reinit")
    o = oracle.OracleSim(c)
    _, _, a_before = o.state()
    o.advance(1.0, mode=0, max_cycles=12)
    phi, _, a_after = o.state()
    h = 1.0 / n
    sd = (r - R).reshape(-1)
    band = (np.abs(sd) > 2.5 * h) & (np.abs(sd) < 5.5 * h)
    err0 = np.abs(phi0 - sd)[band].max()
    err1 = np.abs(phi - sd)[band].max()
    # cells within two of the interface keep their values (about 0.1 h off the
    # distance here), the band beyond is rebuilt from them
    assert err1 < 0.35 * err0 and err1 < 0.3 * h, (err0 / h, err1 / h)
    P = phi.reshape(n, n)
    gx = (P[1:-1, 2:] - P[1:-1, :-2]) / (2 * h)
    gy = (P[2:, 1:-1] - P[:-2, 1:-1]) / (2 * h)
    gn = np.sqrt(gx ** 2 + gy ** 2)
    inner = band.reshape(n, n)[1:-1, 1:-1]
    g0 = np.sqrt(((phi0.reshape(n, n)[1:-1, 2:] - phi0.reshape(n, n)[1:-1, :-2]) / (2 * h)) ** 2
                 + ((phi0.reshape(n, n)[2:, 1:-1] - phi0.reshape(n, n)[:-2, 1:-1]) / (2 * h)) ** 2)
    assert np.abs(gn - 1)[inner].max() < 0.3 * np.abs(g0 - 1)[inner].max()
    assert np.abs(gn - 1)[inner].max() < 0.1
    np.testing.assert_allclose(a_before, a_after, rtol=0, atol=1e-13)


@pytest.mark.slow
def test_droplet_mass_is_constant(oracle):
    """Sec. 4.2 analogue: the droplet's mass stays at its initial value."""
    c = WL.droplet_2d(n=96, seed=1)
    o = oracle.OracleSim(c)
    m0 = o.totals()[0, 0]
    for mode in (1,):
        o.advance(1.0, mode=mode, max_cycles=10)
        assert abs(o.totals()[0, 0] / m0 - 1.0) < 1e-13


def test_droplet_translation_returns(oracle):
    """Sec. 4.2 analogue with the full scheme and the accelerated cycle: a
    water droplet (radius 0.2, 24^2 cells) carried diagonally by a uniform
    flow u = (200, 100) m/s through a periodic box for one period in both
    directions (t = 0.01 s: two in x, one in y).  The exact solution is the
    initial state.  Mass of each fluid is conserved to round-off over the
    ~1900 water sub-steps; the droplet's centroid comes back within a small
    fraction of a cell and its volume-fraction field within 15% in L1
    (measured 0.08 cells and 9%)."""
    n, R, u = 24, 0.2, (200.0, 100.0)
    h, (X, Y) = WL._grid(2, n)
    phi = (np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2) - R).reshape(-1)
    prim = np.zeros((2, 4, n * n))
    for k, rho in enumerate((1000.0, 1.2)):
        prim[k, 0], prim[k, 1], prim[k, 2], prim[k, 3] = rho, u[0], u[1], 1e5
    c = WL._case(2, n, 1, WL.WATER, WL.AIR, phi, prim, 0.01, "droplet_diagonal")
    o = oracle.OracleSim(c)
    tot0 = o.totals()
    _, _, a0 = o.state()
    st = o.advance(0.01, mode=1)
    assert st["t"] == 0.01 and st["steps"][0] > 3 * st["steps"][1]    # water sub-stepped
    tot1 = o.totals()
    _, _, a1 = o.state()
    mass = np.abs(tot1[:, 0] - tot0[:, 0]) / tot0[:, 0]
    assert np.all(mass < 1e-12), mass
    x, y = X.reshape(-1), Y.reshape(-1)
    for w in (x, y):
        shift = ((a1 * w).sum() / a1.sum() - (a0 * w).sum() / a0.sum()) * n
        assert abs(shift) < 0.15, shift
    assert np.abs(a1 - a0).sum() / a0.sum() < 0.15
