"""Pins of the oracle's surface tension: the Laplace pressure jump
p_0 - p_1 = sigma kappa of Eq. (surfacetension) across the interface, with
each fluid taking its own interface pressure in the exchange term (Sec. 3.1:
X_1 / X_2 = p_I1 / p_I2), and mutation checks (a copy of the oracle with a
plausible mistake planted, built on the CPU into a temporary directory, must
fail the pin that guards that part).

Closed forms used:
- the contact of the Riemann problem carries the jump: two sides at rest
  whose pressures differ by exactly the jump are already the solution;
- the stiffened-gas wave curves depend on p and p_inf only through
  p + p_inf (and on p - p_k), so the jumped problem is the plain one with
  the right side's (p, p_inf) shifted by (+jump, -jump); the plain solver is
  pinned against exact solutions elsewhere;
- mirror symmetry: exchanging the sides (velocities negated) with the jump
  negated gives the mirrored solution;
- the curvature of a circle (sphere) of radius R is 1/R (2/R) on every cut
  cell, approached at second order; a straight line has none; the concave
  side has the opposite sign;
- a drop at the Laplace equilibrium (paper Sec. 4.3: sigma = 36, R = 0.1,
  Tait liquid in Tait air) stays at rest with the jump sigma (D - 1) / R, in
  both the original method and the accelerated cycle, and the jump decays
  when sigma is left out of the same run;
- an elliptic drop (Sec. 4.5) oscillates with the period of mode 2 of
  Rayleigh's formula for two fluids, Eq. (oscillation), which the paper
  evaluates to 0.0878, within the discretisation error of a 48^2 grid.
"""
import os
import re
import shutil

import numpy as np
import pytest

from paper_1905_03917_amd import workloads as WL


@pytest.fixture(scope="module")
def oracle():
    from oracle import oracle as O
    O.lib()
    return O


def _rj(L, WL_, WR, gL, piL, gR, piR, jump):
    out = np.empty(5)
    L.or_riemann_jump(np.asarray(WL_, dtype=np.float64), np.asarray(WR, dtype=np.float64), gL, piL, gR, piR,
                      float(jump), out)
    return out


def _rp(L, WL_, WR, gL, piL, gR, piR):
    out = np.empty(5)
    L.or_riemann(np.asarray(WL_, dtype=np.float64), np.asarray(WR, dtype=np.float64), gL, piL, gR, piR, out)
    return out


FLUIDS = [WL.DROP_LIQUID, WL.DROP_AIR, WL.WATER, WL.AIR]


def _sides(seed, count):
    """random pairs of sides: (state L, state R, eos L, eos R)"""
    r = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        eL, eR = FLUIDS[r.integers(4)], FLUIDS[r.integers(4)]
        sL = [r.uniform(0.5, 2.0) * (1000.0 if eL[1] > 1e5 else 1.0), r.uniform(-2.0, 2.0),
              max(-eL[1], 0.0) + r.uniform(100.0, 400.0)]
        sR = [r.uniform(0.5, 2.0) * (1000.0 if eR[1] > 1e5 else 1.0), r.uniform(-2.0, 2.0),
              max(-eR[1], 0.0) + r.uniform(100.0, 400.0)]
        out.append((sL, sR, eL, eR))
    return out


# ----------------------------------------------------------- the jump ------

def check_jump_equilibrium(O, L):
    for (sL, sR, eL, eR) in _sides(1, 40):
        u = sL[1]
        for jump in (360.0, -150.0, 720.0):
            pR = sR[2]
            pL = pR + jump
            if pL + eL[1] <= 50.0:
                continue
            st = _rj(L, [sL[0], u, pL], [sR[0], u, pR], eL[0], eL[1], eR[0], eR[1], jump)
            assert abs(st[0] - pL) <= 1e-12 * (abs(pL) + abs(eL[1]) + abs(eR[1])), (st, pL)
            assert abs(st[1] - u) <= 1e-9 * (1.0 + abs(u)), (st, u)
            assert abs(st[2] - sL[0]) <= 1e-10 * sL[0] and abs(st[3] - sR[0]) <= 1e-10 * sR[0], st


def check_jump_shift_identity(O, L):
    for (sL, sR, eL, eR) in _sides(2, 60):
        for jump in (0.0, 36.0, 360.0, -80.0):
            if sR[2] + jump + eR[1] - jump <= 0.0:
                continue
            st = _rj(L, sL, sR, eL[0], eL[1], eR[0], eR[1], jump)
            ref = _rp(L, sL, [sR[0], sR[1], sR[2] + jump], eL[0], eL[1], eR[0], eR[1] - jump)
            scale = abs(ref[0]) + abs(eL[1]) + abs(eR[1])
            assert abs(st[0] - ref[0]) <= 1e-11 * scale, (jump, st, ref)
            assert abs(st[1] - ref[1]) <= 1e-8 * (1.0 + abs(ref[1])), (jump, st, ref)
            for q in (2, 3):
                assert abs(st[q] - ref[q]) <= 1e-9 * abs(ref[q]) + 1e-12, (jump, st, ref)
            if jump == 0.0:
                np.testing.assert_array_equal(st[:4], _rp(L, sL, sR, eL[0], eL[1], eR[0], eR[1])[:4])


def check_jump_mirror(O, L):
    for (sL, sR, eL, eR) in _sides(3, 40):
        jump = 200.0
        st = _rj(L, sL, sR, eL[0], eL[1], eR[0], eR[1], jump)
        mL = [sR[0], -sR[1], sR[2]]
        mR = [sL[0], -sL[1], sL[2]]
        sm = _rj(L, mL, mR, eR[0], eR[1], eL[0], eL[1], -jump)
        scale = abs(st[0]) + abs(eL[1]) + abs(eR[1])
        assert abs(sm[0] - (st[0] - jump)) <= 1e-11 * scale, (st, sm)
        assert abs(sm[1] + st[1]) <= 1e-8 * (1.0 + abs(st[1])), (st, sm)
        assert abs(sm[2] - st[3]) <= 1e-9 * st[3] and abs(sm[3] - st[2]) <= 1e-9 * st[2], (st, sm)


def test_jump_equilibrium(oracle):
    check_jump_equilibrium(oracle, oracle.lib())


def test_jump_is_the_shifted_plain_problem(oracle):
    check_jump_shift_identity(oracle, oracle.lib())


def test_jump_mirror_symmetry(oracle):
    check_jump_mirror(oracle, oracle.lib())


# ------------------------------------------------------- the curvature -----

def _ball(ndim, n, R, sign=1.0, seed=0):
    h, grid = WL._grid(ndim, n)
    r = np.random.Generator(np.random.PCG64(seed))
    c = [0.5 + r.uniform(-0.5, 0.5) * h for _ in range(ndim)]
    dist = np.sqrt(sum((g - ci) ** 2 for g, ci in zip(grid, c))).reshape(-1)
    return sign * (dist - R), h


def _curvature_error(O, L, ndim, n, R=0.2, sign=1.0):
    phi, h = _ball(ndim, n, R, sign)
    k = O.curvature_run(phi, ndim, n, L=L)
    cut = np.abs(phi) < 0.5 * h * np.sqrt(ndim)
    exact = sign * (ndim - 1) / R
    return np.abs(k[cut] - exact).max() / abs(exact)


def check_curvature(O, L, ndim):
    ns = (32, 64, 128) if ndim == 2 else (16, 32, 64)
    errs = [_curvature_error(O, L, ndim, n) for n in ns]
    print("curvature %d-D errors" % ndim, errs)
    # second order, and small at the finest grid
    for a, b in zip(errs, errs[1:]):
        assert b < a / 3.0, errs
    assert errs[-1] < (2e-3 if ndim == 2 else 5e-3), errs
    # the concave side (fluid 0 outside the ball) has the opposite sign
    assert _curvature_error(O, L, ndim, ns[1], sign=-1.0) < 3.0 * errs[1]


def test_curvature_of_circles(oracle):
    check_curvature(oracle, oracle.lib(), 2)


def test_curvature_of_spheres(oracle):
    check_curvature(oracle, oracle.lib(), 3)


def test_curvature_of_a_plane_and_in_1d(oracle):
    n = 32
    h, (X, Y) = WL._grid(2, n)
    phi = (0.3 * (X - 0.5) + 0.4 * (Y - 0.5)).reshape(-1)
    k = oracle.curvature_run(phi, 2, n).reshape(n, n)
    # cells whose 3x3 neighbourhood lies inside (the zero-gradient boundary
    # bends the level set there)
    assert np.abs(k[1:-1, 1:-1]).max() < 1e-9
    x = (np.arange(n) + 0.5) / n
    assert np.all(oracle.curvature_run(x - 0.5, 1, n) == 0.0)


# -------------------------------------------------------- the static drop --

def _pressures(case, cons, alpha):
    """pressure and speed of each fluid's cells, from alpha_k U_k (values of
    empty cells, alpha_k = 0, are not used)"""
    D = case["ndim"]
    out = []
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        for k in range(2):
            a = alpha if k == 0 else 1.0 - alpha
            U = cons[k]
            aa = np.maximum(a, 1e-300)
            ke = 0.5 * sum(U[1 + d] ** 2 for d in range(D)) / np.maximum(U[0], 1e-300) / aa
            E = U[D + 1] / aa
            g, pi = case["gamma"][k], case["pinf"][k]
            speed = np.sqrt(sum(U[1 + d] ** 2 for d in range(D))) / np.maximum(U[0], 1e-300)
            out.append(((g - 1.0) * (E - ke) - g * pi, speed))
    return out


def drop_jump(case, phi, cons, alpha):
    """mean pressure of the drop's pure cells minus that of the pure air
    cells around it, and the largest speed of either fluid's cells"""
    D, n = case["ndim"], case["n"][0]
    h, grid = WL._grid(D, n)
    r = np.sqrt(sum((g - ci) ** 2 for g, ci in zip(grid, case["centre"]))).reshape(-1)
    R = case["radius"]
    (p0, s0), (p1, s1) = _pressures(case, cons, alpha)
    inner = (alpha > 1.0 - 1e-9) & (r < R - 2.0 * h)
    outer = (alpha < 1e-9) & (r > R + 2.0 * h) & (r < 3.0 * R)
    assert inner.sum() > 0 and outer.sum() > 0
    vmax = max(s0[alpha > 0.5].max(), s1[alpha < 0.5].max())
    return p0[inner].mean() - p1[outer].mean(), vmax


def check_static_drop(O, L, ndim, mode, sigma=36.0):
    n, cycles = (64, 60 if mode == 0 else 12) if ndim == 2 else (32, 25 if mode == 0 else 6)
    c = WL.static_drop(n, ndim)
    c["sigma"] = sigma
    o = O.OracleSim(c, L=L)
    st = o.advance(1e30, mode=mode, max_cycles=cycles)
    phi, cons, alpha = o.state()
    jump, vmax = drop_jump(c, phi, cons, alpha)
    exact = 36.0 * (ndim - 1) / c["radius"]
    print("static drop %d-D mode %d: steps %s, jump %.4f (Laplace %.1f), max speed %.3e" %
          (ndim, mode, st["steps"], jump, exact, vmax))
    if mode == 1:
        assert st["steps"][0] >= 4 * st["steps"][1], st
    return jump, vmax, exact


@pytest.mark.parametrize("ndim,mode", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_static_drop_holds_the_laplace_jump(oracle, ndim, mode):
    jump, vmax, exact = check_static_drop(oracle, oracle.lib(), ndim, mode)
    assert abs(jump - exact) <= (2e-3 if ndim == 2 else 1e-2) * exact, (jump, exact)
    assert vmax < 2e-3, vmax


def test_static_drop_relaxes_without_surface_tension(oracle):
    """the same drop without sigma is out of equilibrium: its jump decays"""
    jump, vmax, exact = check_static_drop(oracle, oracle.lib(), 2, 0, sigma=0.0)
    assert jump < 0.8 * exact, jump


def drop_period(sim, case, mode, read_phi, t_max=0.055):
    """oscillation period of the Sec. 4.5 drop: twice the time at which the
    drop's extent along x (the zero crossing of phi on the grid row through
    the centre, interpolated linearly) first reaches its minimum, refined by
    a parabola through the three samples around it; sim is stepped one
    cycle (or step) at a time, read_phi() returns its level set"""
    n = case["n"][0]
    h = case["h"]
    j0 = int(round(case["centre"][1] / h - 0.5))
    ts, ext = [], []
    while True:
        st = sim.advance(1e30, mode=mode, max_cycles=1)
        row = np.asarray(read_phi()).reshape(n, n)[j0]
        i = np.where((row[:-1] >= 0) != (row[1:] >= 0))[0]
        i = i[i >= n // 2][0]
        ts.append(st["t"])
        ext.append((i + 0.5 + row[i] / (row[i] - row[i + 1])) * h - case["centre"][0])
        if st["t"] > t_max:
            break
    ts, ext = np.array(ts), np.array(ext)
    k = int(np.argmin(ext))
    assert 0 < k < len(ts) - 1, "no minimum of the extent before t_max"
    A = np.polyfit(ts[k - 1:k + 2] - ts[k], ext[k - 1:k + 2], 2)
    return 2.0 * (ts[k] - A[1] / (2.0 * A[0]))


def check_oscillation_period(O, L, n=48, mode=1):
    case = WL.oscillating_drop(n)
    o = O.OracleSim(case, L=L)
    T = drop_period(o, case, mode, lambda: o.state()[0])
    print("oscillating drop %d^2 mode %d: period %.5f (Rayleigh %.4f)" % (n, mode, T, case["period"]))
    assert abs(T - case["period"]) <= 0.04 * case["period"], T
    return T


def test_oscillating_drop_period(oracle):
    check_oscillation_period(oracle, oracle.lib())


# ------------------------------------------------------ mutation checks ----

def _function_span(src, name):
    m = re.search(r"\n(static )?(void|int|double) %s\(" % re.escape(name), src)
    assert m, name
    end = src.index("\n}\n", m.start())
    return m.start(), end


def _drop_ok(O, L, ndim, mode):
    jump, vmax, exact = check_static_drop(O, L, ndim, mode)
    assert abs(jump - exact) <= (2e-3 if ndim == 2 else 1e-2) * exact, (jump, exact)
    assert vmax < 2e-3, vmax


MUTANTS = {
    # the jump taken with the wrong sign
    "jump_sign": ("interaction", "s->P.sigma != 0.0 ? s->P.sigma * curvature(",
                  "s->P.sigma != 0.0 ? -s->P.sigma * curvature("),
    # fluid 1 takes fluid 0's interface pressure in its exchange term
    "exchange_one_pressure": ("exchange", "double p = k == 0 ? s->ps[c] : s->ps[c] - s->pj[c];",
                              "double p = s->ps[c];"),
    # the right side's wave function at fluid 0's contact pressure
    "riemann_right_unjumped": ("riemann_core", "double f = wave_f(&L, p, &dfl) + wave_f(&R, p - jump, &dfr) + du;",
                               "double f = wave_f(&L, p, &dfl) + wave_f(&R, p, &dfr) + du;"),
    # half the jump
    "jump_halved": ("interaction", "s->P.sigma != 0.0 ? s->P.sigma * curvature(",
                    "s->P.sigma != 0.0 ? 0.5 * s->P.sigma * curvature("),
    # the curvature at the cell centre instead of the interface
    "curvature_at_centre": ("curvature", "double den = 1.0 - phi[c] * kap / (double)(D - 1);",
                            "double den = 1.0;"),
    # the mixed second derivatives left out
    "curvature_no_cross_terms": ("curvature", "H[d][e] = H[e][d] = (a - b - cc + dd) / (4.0 * h * h);",
                                 "H[d][e] = H[e][d] = 0.0 * (a - b - cc + dd);"),
}

CHECKS = {
    "jump_sign": lambda O, L: _drop_ok(O, L, 2, 0),
    "exchange_one_pressure": lambda O, L: _drop_ok(O, L, 2, 0),
    "riemann_right_unjumped": lambda O, L: check_jump_equilibrium(O, L),
    "jump_halved": lambda O, L: check_oscillation_period(O, L),
    "curvature_at_centre": lambda O, L: check_curvature(O, L, 2),
    "curvature_no_cross_terms": lambda O, L: check_curvature(O, L, 3),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_catches_planted_mistake(oracle, tmp_path, name):
    func, old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    a, b = _function_span(src, func)
    body = src[a:b]
    assert body.count(old) == 1, (name, body.count(old))
    mutated = src[:a] + body.replace(old, new) + src[b:]
    d = str(tmp_path)
    shutil.copy(os.path.join(os.path.dirname(oracle.SRC), "sharp_oracle.h"), d)
    path = os.path.join(d, "sharp_oracle_mutant.c")
    with open(path, "w") as fh:
        fh.write(mutated)
    L = oracle.load(oracle.build_at(path, os.path.join(d, "libmutant.so")))
    with pytest.raises((AssertionError, RuntimeError)):
        CHECKS[name](oracle, L)
