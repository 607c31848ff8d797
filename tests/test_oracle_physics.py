"""Pins of the oracle's physics kernels against closed forms and textbook facts.

EOS: stiffened gas (Sec. 2.1 closes Eq. (EulerEquation) with an EOS; the
paper's Tait water is a stiffened-gas isentrope).  Interaction: exact Riemann
problem between two stiffened gases.  Flux: WENO5 with LLF splitting (Sec. 4).
"""
import math

import numpy as np
import pytest


def test_eos_round_trip_and_energy(oracle):
    # total energy of water at rest is the closed form (p + gamma pinf)/(gamma - 1)
    U = oracle.prim2cons(1, 4.4, 6e8, [1000.0, 0.0, 1e5])
    assert U[2] == pytest.approx((1e5 + 4.4 * 6e8) / 3.4, rel=1e-15)
    for D in (1, 2, 3):
        W = np.array([1.3] + [0.5 * (d + 1) for d in range(D)] + [2.5e5])
        U = oracle.prim2cons(D, 1.4, 0.0, W)
        W2, rc = oracle.cons2prim(D, 1.4, 0.0, U)
        assert rc == 0
        np.testing.assert_allclose(W2, W, rtol=1e-13)
    # non-physical state is reported
    _, rc = oracle.cons2prim(1, 1.4, 0.0, [1.0, 0.0, -1.0])
    assert rc != 0


def _two_rarefaction_pstar(WL, WR, g):
    z = (g - 1) / (2 * g)
    cL = math.sqrt(g * WL[2] / WL[0])
    cR = math.sqrt(g * WR[2] / WR[0])
    num = cL + cR - 0.5 * (g - 1) * (WR[1] - WL[1])
    return (num / (cL / WL[2] ** z + cR / WR[2] ** z)) ** (1 / z)


def test_riemann_two_rarefaction_closed_form(oracle):
    # both waves are rarefactions: p* has a closed form for an ideal gas
    WL, WR = [1.0, -2.0, 0.4], [1.0, 2.0, 0.4]
    st = oracle.riemann(WL, WR, 1.4, 0.0, 1.4, 0.0)
    assert st[0] == pytest.approx(_two_rarefaction_pstar(WL, WR, 1.4), rel=1e-12)
    assert abs(st[1]) < 1e-14                    # symmetric data: u* = 0
    WL, WR = [1.0, -1.0, 1.0], [0.5, 1.5, 0.3]
    st = oracle.riemann(WL, WR, 1.4, 0.0, 1.4, 0.0)
    assert st[0] < 0.3
    assert st[0] == pytest.approx(_two_rarefaction_pstar(WL, WR, 1.4), rel=1e-12)


def test_riemann_trivial_and_symmetric(oracle):
    W = [2.0, 3.0, 7.0e5]
    st = oracle.riemann(W, W, 4.4, 6e8, 4.4, 6e8)
    assert st[0] == pytest.approx(7.0e5, rel=1e-12)
    assert st[1] == pytest.approx(3.0, rel=1e-12)
    st = oracle.riemann([1000.0, 50.0, 1e5], [1000.0, -50.0, 1e5], 4.4, 6e8, 4.4, 6e8)
    assert abs(st[1]) < 1e-9 and st[0] > 1e5     # colliding streams: two shocks


def test_riemann_stiffened_equals_shifted_ideal(oracle):
    # with equal p_inf the stiffened-gas problem is the ideal-gas problem in p + p_inf
    pinf = 6e8
    WL, WR = [1000.0, 10.0, 1e9], [900.0, -5.0, 1e5]
    st = oracle.riemann(WL, WR, 4.4, pinf, 4.4, pinf)
    WLs, WRs = [1000.0, 10.0, 1e9 + pinf], [900.0, -5.0, 1e5 + pinf]
    si = oracle.riemann(WLs, WRs, 4.4, 0.0, 4.4, 0.0)
    assert st[0] + pinf == pytest.approx(si[0], rel=1e-11)
    assert st[1] == pytest.approx(si[1], rel=1e-11)


def _eos_e(rho, p, g, pi):
    return (p + g * pi) / ((g - 1) * rho)


def _jump_location(oracle, WL, WR, gL, piL, gR, piR, lo, hi, side):
    """bisection on the sampled exact solution for the discontinuity in (lo, hi)"""
    ref = oracle.riemann_sample(WL, WR, gL, piL, gR, piR, lo)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s = oracle.riemann_sample(WL, WR, gL, piL, gR, piR, mid)
        if abs(s[2] - ref[2]) < 1e-9 * abs(ref[2]) and s[3] == ref[3]:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("case", ["gas_water", "water_shock"])
def test_riemann_shock_rankine_hugoniot(oracle, case):
    """The right-going shock of the sampled solution satisfies the
    stiffened-gas Rankine-Hugoniot conditions (mass, momentum, energy)."""
    if case == "gas_water":
        # water pushed by high-pressure water into air: shock in air
        WL, WR, gL, piL, gR, piR = [1000.0, 0.0, 1e9], [50.0, 0.0, 1e5], 4.4, 6e8, 1.4, 0.0
    else:
        WL, WR, gL, piL, gR, piR = [1000.0, 300.0, 1e5], [1000.0, 0.0, 1e5], 4.4, 6e8, 4.4, 6e8
    st = oracle.riemann(WL, WR, gL, piL, gR, piR)
    assert st[0] > WR[2]                         # right wave is a shock
    S = _jump_location(oracle, WL, WR, gL, piL, gR, piR, st[1] + 1e-9, 1e5, 1)
    post = oracle.riemann_sample(WL, WR, gL, piL, gR, piR, S - 1e-6 * abs(S))
    pre = oracle.riemann_sample(WL, WR, gL, piL, gR, piR, S + 1e-6 * abs(S))
    r0, u0, p0 = pre[:3]
    r1, u1, p1 = post[:3]
    m0, m1 = r0 * (u0 - S), r1 * (u1 - S)
    assert m0 == pytest.approx(m1, rel=1e-9)
    assert m0 * (u0 - S) + p0 == pytest.approx(m1 * (u1 - S) + p1, rel=1e-9)
    h0 = _eos_e(r0, p0, gR, piR) + p0 / r0 + 0.5 * (u0 - S) ** 2
    h1 = _eos_e(r1, p1, gR, piR) + p1 / r1 + 0.5 * (u1 - S) ** 2
    assert h0 == pytest.approx(h1, rel=1e-9)


def test_workload_post_shock_states_are_single_shocks(oracle):
    """The post-shock inputs of the 2-D and 3-D workloads: the Riemann problem
    (post | pre) has p* = p_post, u* = u_post, i.e. a single right shock."""
    from paper_1905_03917_amd import workloads as WL
    s = WL.WATER_SHOCK_1E9
    st = oracle.riemann([s["rho"], s["u"], s["p"]], [1000.0, 0.0, 1e5], 4.4, 6e8, 4.4, 6e8)
    assert st[0] == pytest.approx(s["p"], rel=1e-10)
    assert st[1] == pytest.approx(s["u"], rel=1e-9)
    s = WL.AIR_SHOCK_M15
    st = oracle.riemann([s["rho"], s["u"], s["p"]], [1.0, 0.0, 1e5], 1.4, 0.0, 1.4, 0.0)
    assert st[0] == pytest.approx(s["p"], rel=1e-10)
    assert st[1] == pytest.approx(s["u"], rel=1e-9)


def test_gas_water_tube_star_state(oracle):
    """Star state of the 1-D gas-water workload (water 1e9 Pa | air 1e5 Pa)."""
    st = oracle.riemann([1000.0, 0.0, 1e9], [50.0, 0.0, 1e5], 4.4, 6e8, 1.4, 0.0)
    assert 1.40e7 < st[0] < 1.44e7
    assert 480.0 < st[1] < 485.0


def test_weno5_exact_for_linear_and_constant(oracle):
    for v in ([3.0] * 5, [1.0, 2.0, 3.0, 4.0, 5.0], [-2.0, -1.5, -1.0, -0.5, 0.0]):
        # cell averages of a linear function: the face value is exact
        face = v[2] + 0.5 * (v[3] - v[2]) if v[0] != v[1] else v[2]
        assert oracle.weno5(v) == pytest.approx(face, rel=1e-14, abs=1e-14)


def test_weno5_fifth_order(oracle):
    """Face values from exact cell averages of sin: error falls ~2^5 per halving."""
    errs = []
    for n in (20, 40, 80):
        h = 1.0 / n
        x = np.arange(n) * h                        # left edges
        avg = (np.cos(2 * np.pi * x) - np.cos(2 * np.pi * (x + h))) / (2 * np.pi * h)
        e = 0.0
        for i in range(n):
            v = [avg[(i + m) % n] for m in (-2, -1, 0, 1, 2)]
            e = max(e, abs(oracle.weno5(v, 1e-40) - math.sin(2 * np.pi * (x[i] + h))))
        errs.append(e)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert r2 > 20.0, errs


def test_weno5_non_oscillatory_at_a_jump(oracle):
    v = oracle.weno5([0.0, 0.0, 0.0, 1.0, 1.0])
    assert -1e-6 < v < 0.05                         # picks the smooth left stencil
    v = oracle.weno5([1.0, 1.0, 1.0, 0.0, 0.0])
    assert 0.95 < v < 1.0 + 1e-6


def test_face_flux_consistency(oracle):
    """Uniform state: the LLF-WENO flux equals the physical flux F(U)."""
    W = [1000.0, 10.0, 1e5]
    F = oracle.face_flux_1d([W] * 6, 4.4, 6e8)
    U = oracle.prim2cons(1, 4.4, 6e8, W)
    ex = [U[1], U[1] * W[1] + W[2], (U[2] + W[2]) * W[1]]
    np.testing.assert_allclose(F, ex, rtol=1e-13)


def test_riemann_stiffened_side_in_tension(oracle):
    """Water in tension (p < 0 but p + p_inf > 0) against air: the solution
    exists, is continuous in p and u across the contact, and keeps p* > -min p_inf."""
    WL, WR = [999.9, 6.8, -1.4e5], [1.2, 6.8, 1.0e5]
    st = oracle.riemann(WL, WR, 4.4, 6e8, 1.4, 0.0)
    assert np.all(np.isfinite(st)) and st[0] >= 0.0
    a = oracle.riemann_sample(WL, WR, 4.4, 6e8, 1.4, 0.0, st[1] - 1e-9)
    b = oracle.riemann_sample(WL, WR, 4.4, 6e8, 1.4, 0.0, st[1] + 1e-9)
    assert a[2] == pytest.approx(b[2], rel=1e-12, abs=1e-6) and a[1] == pytest.approx(b[1], rel=1e-12)


def test_riemann_cavitation_floor_at_the_vacuum_limit(oracle):
    """Two rarefactions leave a vacuum when the sides separate faster than
    2 cL/(gL - 1) + 2 cR/(gR - 1) (ideal gases; for stiffened gases the same
    in p + p_inf): beyond that limit p* is the floor -min(p_inf) and the star
    densities vanish; just below it p* stays above the floor and follows the
    two-rarefaction closed form."""
    g = 1.4
    W = [1.0, 0.0, 1.0e5]
    c = math.sqrt(g * W[2] / W[0])
    lim = 2.0 * c / (g - 1.0) * 2.0          # both sides
    for f in (1.01, 1.5, 16.0):
        u = 0.5 * f * lim
        st = oracle.riemann([1.0, -u, 1.0e5], [1.0, u, 1.0e5], g, 0.0, g, 0.0)
        assert st[0] == 0.0 and st[2] == 0.0 and st[3] == 0.0, (f, st)
    u = 0.5 * 0.99 * lim
    WL, WR = [1.0, -u, 1.0e5], [1.0, u, 1.0e5]
    st = oracle.riemann(WL, WR, g, 0.0, g, 0.0)
    assert st[0] > 0.0 and st[0] == pytest.approx(_two_rarefaction_pstar(WL, WR, g), rel=1e-10)
    # two stiffened gases with different p_inf: the floor is -min(p_inf); the
    # side with the smaller p_inf expands to p + p_inf = 0, the other to the
    # floor along its isentrope, and the floor is reached exactly when the
    # separation speed reaches the sum of both rarefactions' velocity changes
    gL, piL, gR, piR = 4.4, 6.0e8, 7.15, 3.309e8
    rho, p = 1000.0, 1.0e5
    cL, cR = math.sqrt(gL * (p + piL) / rho), math.sqrt(gR * (p + piR) / rho)
    floor = -min(piL, piR)
    duL = 2.0 * cL / (gL - 1.0) * (1.0 - ((floor + piL) / (p + piL)) ** ((gL - 1.0) / (2.0 * gL)))
    duR = 2.0 * cR / (gR - 1.0)
    for f, at_floor in ((1.02, True), (0.98, False)):
        u = 0.5 * f * (duL + duR)
        st = oracle.riemann([rho, -u, p], [rho, u, p], gL, piL, gR, piR)
        if at_floor:
            assert st[0] == floor and st[3] == 0.0 and st[2] > 0.0, st
        else:
            assert st[0] > floor and st[3] > 0.0, st
