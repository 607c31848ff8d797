"""GPU adjoint of single-dt runs with an interface, the geometry frozen at
the recorded stage level sets (Sec. 2.1 Eq. Eulerdiscrete with the exchange
term, Sec. 2.2-2.3 mixing and extension): the level-set tape and its replay,
against central finite differences of the oracle's own replayed run (the
oracle records and replays its own level sets; nothing of the GPU's enters
it), against central differences of the GPU's replayed run, and the
checkpoint interval."""
import numpy as np
import pytest

import _adjoint_cases as AC

pytestmark = pytest.mark.gpu


def _dt(c):
    """a CFL-limited step of the initial state of both fluids"""
    D = c["ndim"]
    m = 0.0
    for k in (0, 1):
        W = c["prim"][k]
        cs = np.sqrt(c["gamma"][k] * (W[D + 1] + c["pinf"][k]) / W[0])
        m = max(m, float(np.max(sum((np.abs(W[1 + d]) + cs) / c["h"] for d in range(D)))))
    return 0.6 / m


def _gpu_taped(c, steps, dt, ckpt, rk=3):
    import paper_1905_03917_amd as P
    sim = P.Sim(c, tape=1, dt_fixed=dt, ckpt_every=ckpt, rk=rk)
    sim.advance(1e30, mode=P.SIM_SINGLE_DT, max_cycles=steps)
    _, cons, alpha = sim.state(device=False)
    return sim, cons, alpha


def _gpu_J(c, prim, gamma, pinf, tape, dt, steps, probes, rk=3):
    import paper_1905_03917_amd as P
    cc = dict(c, gamma=list(gamma), pinf=list(pinf))
    cc.pop("phi")
    cc.pop("prim")
    sim = P.Sim(cc, ls_replay=tape, dt_fixed=dt, rk=rk)
    sim.set_state(c["phi"], prim)
    sim.advance(1e30, mode=P.SIM_SINGLE_DT, max_cycles=steps)
    _, cons, alpha = sim.state(device=False)
    sim.close()
    return AC.interface_loss(cons, alpha, gamma, pinf, probes, c["ndim"])[0]


def _oracle_J(c, prim, gamma, pinf, log, dt, steps, probes, rk=3):
    from oracle import oracle as O
    cc = dict(c, gamma=list(gamma), pinf=list(pinf))
    s = O.OracleSim(cc, ls_replay=log, dt_replay=[dt] * (2 * steps), rk=rk)
    s.set_state(c["phi"], prim)
    s.advance(1e30, mode=0, max_cycles=steps)
    _, cons, alpha = s.state()
    return AC.interface_loss(cons, alpha, gamma, pinf, probes, c["ndim"])[0]


def _oracle_log(c, dt, steps, rk=3):
    from oracle import oracle as O
    s = O.OracleSim(c, log_levelset=1, dt_replay=[dt] * (2 * steps), rk=rk)
    s.advance(1e30, mode=0, max_cycles=steps)
    return s.levelset_log()


def _richardson(J, e):
    """central difference quotient at e and e/2, extrapolated"""
    q1 = (J(e) - J(-e)) / (2 * e)
    q2 = (J(e / 2) - J(-e / 2)) / e
    return q2 + (q2 - q1) / 3.0


def _gradient(c, steps, ckpt, rk=3, fluid=None):
    """taped GPU run and its adjoint for the pressure-probe loss (probes in
    both fluids, or in `fluid` only)"""
    dt = _dt(c)
    sim, cons, alpha = _gpu_taped(c, steps, dt, ckpt, rk)
    if fluid is None:
        probes = AC.interface_probes(alpha, count=8)
    else:
        probes = AC.interface_probes(np.where(alpha == (1.0 if fluid == 0 else 0.0), alpha, 0.5), count=24)
    J, gc, ge_loss = AC.interface_loss(cons, alpha, c["gamma"], c["pinf"], probes, c["ndim"])
    gp, ge = sim.backward(gc)
    tape = sim.levelset_tape()
    sim.close()
    return dict(dt=dt, J=J, probes=probes, gp=gp, ge=ge + ge_loss, tape=tape)


CASES = [(1, 64, 3), (2, 24, 3), (2, 20, 2), (3, 12, 3)]


def _periodic_y(c):
    """the same flat interface with the y direction periodic (the background
    waves are periodic in y)"""
    c = dict(c)
    c["bc"] = [0, 1, 0]
    return c


@pytest.mark.parametrize("ndim,n,rk", CASES)
def test_levelset_tape_replays_the_run(ndim, n, rk):
    """the replayed run (stage level sets from the tape) reproduces the taped
    one, and matches the oracle's replay of its own level sets"""
    import paper_1905_03917_amd as P
    from oracle import oracle as O
    print("replay case ndim=%d n=%d rk=%d" % (ndim, n, rk), flush=True)
    c = AC.interface_case(n, ndim)
    steps, dt = 4, _dt(c)
    sim, cons, alpha = _gpu_taped(c, steps, dt, 2, rk)
    tape = sim.levelset_tape()
    sim.close()
    assert tape.shape == (steps * rk, c["phi"].size)
    rep = P.Sim(c, ls_replay=tape, dt_fixed=dt, rk=rk)
    rep.advance(1e30, mode=P.SIM_SINGLE_DT, max_cycles=steps)
    _, cons2, alpha2 = rep.state(device=False)
    # (the replay runs the unfused level-set path: the geometry kernels of
    # the two paths may round differently; momentum is measured against
    # sqrt(max rho max E), as in the parity tests)
    scale = AC.state_scales(cons, ndim)
    assert np.max(np.abs(cons2 - cons) / scale) <= 1e-12
    assert np.max(np.abs(alpha2 - alpha)) <= 1e-13
    # past the tape's end the replay refuses to go on
    with pytest.raises(P.SimError):
        rep.advance(1e30, mode=P.SIM_SINGLE_DT, max_cycles=1)
    rep.close()
    o = O.OracleSim(c, log_levelset=1, dt_replay=[dt] * (2 * steps), rk=rk)
    o.advance(1e30, mode=0, max_cycles=steps)
    log = o.levelset_log()
    assert np.max(np.abs(log - tape)) <= 1e-10 * max(1.0, np.abs(log).max())
    _, ocons, _ = o.state()
    # four steps (the one-step bar is 1e-10): the two libraries' interface
    # roots agree to the root's stopping tolerance only
    assert np.max(np.abs(ocons - cons) / scale) <= 1e-9


@pytest.mark.parametrize("ndim,n,rk", CASES)
def test_gradient_matches_oracle_finite_differences(ndim, n, rk):
    """directional derivatives along smooth perturbations of both fluids'
    primitives, and each fluid's EOS parameters (for the loss on that
    fluid's probes, where it is not buried under the other's), against
    Richardson-extrapolated central differences of the oracle's replayed run
    (1e-6 relative).  The steps are small because the map is piecewise
    smooth: the LLF speed is a maximum, and in the water's energy flux it
    multiplies a content of ~8e8 J/m^3, so a step that moves an argmax
    changes the quotient; the steps are far above the interface root's
    tolerance (~6e-5 Pa)."""
    print("adjoint interface case ndim=%d n=%d rk=%d" % (ndim, n, rk), flush=True)
    c = AC.interface_case(n, ndim)
    steps = 6
    e_dir = 1e-3 if ndim == 3 else 1e-2
    r = _gradient(c, steps, ckpt=4, rk=rk)
    log = _oracle_log(c, r["dt"], steps, rk)
    g0, p0 = list(c["gamma"]), list(c["pinf"])

    def Jp(e, dirn):
        return _oracle_J(c, c["prim"] + e * dirn, g0, p0, log, r["dt"], steps, r["probes"], rk)

    for seed in (7, 11):
        dirn = AC.interface_direction(c, seed=seed)
        want = _richardson(lambda e: Jp(e, dirn), e_dir)
        got = float(np.sum(r["gp"] * dirn))
        print("direction", seed, got, want, abs(got - want) / abs(want), flush=True)
        assert abs(got - want) <= 1e-6 * abs(want), (seed, got, want)
    steps_eos = {(0, 0): 1e-3 * g0[0], (0, 1): 100.0, (1, 0): 1e-6 * g0[1], (1, 1): 1e-6 * p0[1]}
    for k in (0, 1):
        rk_ = _gradient(c, steps, ckpt=4, rk=rk, fluid=k)
        for j in (0, 1):
            def Je(e, j=j):
                g, p = list(g0), list(p0)
                (g if j == 0 else p)[k] += e
                return _oracle_J(c, c["prim"], g, p, log, r["dt"], steps, rk_["probes"], rk)
            want = _richardson(Je, steps_eos[(k, j)])
            got = float(rk_["ge"][k, j])
            print("eos", k, j, got, want, abs(got - want) / abs(want), flush=True)
            assert abs(got - want) <= 1e-6 * abs(want), (k, j, got, want)


def test_gradient_with_a_periodic_direction_matches_oracle_finite_differences():
    """2-D, y periodic: the transposed extension and mixing gather across the
    periodic boundary"""
    c = _periodic_y(AC.interface_case(20, 2))
    steps = 6
    r = _gradient(c, steps, ckpt=4)
    log = _oracle_log(c, r["dt"], steps)
    for seed in (7, 11):
        dirn = AC.interface_direction(c, seed=seed)
        want = _richardson(lambda e: _oracle_J(c, c["prim"] + e * dirn, c["gamma"], c["pinf"], log, r["dt"], steps,
                                               r["probes"]), 1e-2)
        got = float(np.sum(r["gp"] * dirn))
        print("periodic direction", seed, got, want, abs(got - want) / abs(want), flush=True)
        assert abs(got - want) <= 1e-6 * abs(want), (seed, got, want)


@pytest.mark.parametrize("ndim,n", [(2, 24), (3, 12)])
def test_gradient_on_a_curved_interface_matches_oracle_finite_differences(ndim, n):
    """a water column (2-D) or droplet (3-D) in air: the extension's
    weights spread over the axes and the mixing has diagonal targets"""
    print("adjoint curved case ndim=%d n=%d" % (ndim, n), flush=True)
    c = AC.curved_case(n, ndim)
    steps = 6
    r = _gradient(c, steps, ckpt=4)
    log = _oracle_log(c, r["dt"], steps)
    for seed in (7, 11):
        dirn = AC.interface_direction(c, seed=seed)
        want = _richardson(lambda e: _oracle_J(c, c["prim"] + e * dirn, c["gamma"], c["pinf"], log, r["dt"], steps,
                                               r["probes"]), 3e-3)
        got = float(np.sum(r["gp"] * dirn))
        print("curved direction", seed, got, want, abs(got - want) / abs(want), flush=True)
        assert abs(got - want) <= 1e-6 * abs(want), (seed, got, want)


def test_gradient_matches_gpu_finite_differences_and_ignores_the_checkpoint_interval():
    """2-D: the same directional derivative from central differences of the
    GPU's own replayed run; checkpoints every 1, 3 and 10 steps give the same
    gradient, bit for bit"""
    c = AC.interface_case(24, 2)
    steps = 6
    ref = _gradient(c, steps, ckpt=3)
    # (a checkpoint holds what the step-start interaction left, the
    # extension's results and p*, so every segment replays the same stages
    # whatever the segment boundaries: the gradients are bitwise equal)
    for ck in (1, 10):
        other = _gradient(c, steps, ckpt=ck)
        np.testing.assert_array_equal(other["gp"], ref["gp"])
        np.testing.assert_array_equal(other["ge"], ref["ge"])
    dirn = AC.interface_direction(c, seed=7)
    want = _richardson(lambda e: _gpu_J(c, c["prim"] + e * dirn, c["gamma"], c["pinf"], ref["tape"], ref["dt"],
                                        steps, ref["probes"]), 1e-2)
    got = float(np.sum(ref["gp"] * dirn))
    assert abs(got - want) <= 1e-6 * abs(want), (got, want)


def test_backward_restores_the_forward_state():
    import paper_1905_03917_amd as P
    c = AC.interface_case(20, 2)
    dt = _dt(c)
    sim, cons, alpha = _gpu_taped(c, 3, dt, 2)
    J, gc, _ = AC.interface_loss(cons, alpha, c["gamma"], c["pinf"], AC.interface_probes(alpha), 2)
    sim.backward(gc)
    _, cons2, alpha2 = sim.state(device=False)
    assert np.array_equal(cons2, cons) and np.array_equal(alpha2, alpha)
    # and the simulation goes on from there as the run without a backward
    # (to the interface root's tolerance: its iteration starts from the
    # replay's last roots)
    sim.advance(1e30, mode=P.SIM_SINGLE_DT, max_cycles=1)
    _, c3, _ = sim.state(device=False)
    sim.close()
    ref, _, _ = _gpu_taped(c, 4, dt, 2)
    _, c4, _ = ref.state(device=False)
    ref.close()
    assert np.max(np.abs(c3 - c4) / AC.state_scales(c4, 2)) <= 1e-10


def test_levelset_replay_argument_errors():
    """the replay's arguments are checked at sim_create and the tape's
    read-out needs a tape with an interface"""
    import paper_1905_03917_amd as P
    c = AC.interface_case(16, 2)
    nc = c["phi"].size
    with pytest.raises(P.SimError) as e:
        P.Sim(c, ls_replay=np.zeros(nc + 1))            # not a whole number of level sets
    assert e.value.status == -1
    with pytest.raises(P.SimError) as e:
        P.Sim(c, ls_replay=np.zeros(nc), tape=1)       # a replay records no tape
    assert e.value.status == -1
    s = P.Sim(c)
    s.advance(1e30, mode=P.SIM_SINGLE_DT, max_cycles=1)
    with pytest.raises(P.SimError) as e:
        s.levelset_tape()
    assert e.value.status == -5
    s.close()
    r = P.Sim(c, ls_replay=np.tile(c["phi"], 3), dt_fixed=_dt(c))
    with pytest.raises(P.SimError) as e:
        r.advance(1e30, mode=P.SIM_MULTI_DT, max_cycles=1)   # single-dt steps only
    assert e.value.status == -1
    r.advance(1e30, mode=P.SIM_SINGLE_DT, max_cycles=1)       # three stage level sets: one step
    with pytest.raises(P.SimError):
        r.advance(1e30, mode=P.SIM_SINGLE_DT, max_cycles=1)
    r.close()


def _oracle_J_multi(c, prim, gamma, pinf, log, sched, cycles, probes, rk=3):
    from oracle import oracle as O
    cc = dict(c, gamma=list(gamma), pinf=list(pinf))
    s = O.OracleSim(cc, ls_replay=log, dt_replay=sched, rk=rk)
    s.set_state(c["phi"], prim)
    s.advance(1e30, mode=1, max_cycles=cycles)
    _, cons, alpha = s.state()
    return AC.interface_loss(cons, alpha, gamma, pinf, probes, c["ndim"])[0]


@pytest.mark.parametrize("ndim,n,rk,ckpt,curved", [(1, 64, 3, 1, False), (2, 24, 3, 2, False), (2, 20, 2, 1, False),
                                                    (2, 24, 3, 1, True), (3, 12, 3, 2, True)])
def test_accelerated_cycles_gradient_matches_oracle_finite_differences(ndim, n, rk, ckpt, curved):
    """accelerated cycles (Sec. 3.1): the slow fluid's interpolation, the
    correction and the sub-stepped fast fluid reversed, against central
    differences of the oracle's accelerated cycles replayed with its own
    level sets and CFL steps"""
    import paper_1905_03917_amd as P
    from oracle import oracle as O
    print("adjoint multi_dt case ndim=%d n=%d rk=%d ckpt=%d curved=%d" % (ndim, n, rk, ckpt, curved), flush=True)
    c = AC.curved_case(n, ndim) if curved else AC.interface_case(n, ndim)
    cycles = 2
    sim = P.Sim(c, tape=1, ckpt_every=ckpt, rk=rk)
    st = sim.advance(1e30, mode=P.SIM_MULTI_DT, max_cycles=cycles)
    assert st["steps"][0] != st["steps"][1]          # sub-stepping took place
    _, cons, alpha = sim.state(device=False)
    probes = AC.interface_probes(alpha)
    J, gc, ge_loss = AC.interface_loss(cons, alpha, c["gamma"], c["pinf"], probes, ndim)
    gp, ge = sim.backward(gc)
    sim.close()
    o = O.OracleSim(c, log_levelset=1, rk=rk)
    ost = o.advance(1e30, mode=1, max_cycles=cycles)
    assert ost["steps"] == st["steps"]
    log, sched = o.levelset_log(), o.schedule()
    for seed in (7, 11):
        dirn = AC.interface_direction(c, seed=seed)
        want = _richardson(lambda e: _oracle_J_multi(c, c["prim"] + e * dirn, c["gamma"], c["pinf"], log, sched,
                                                     cycles, probes, rk), 1e-3)
        got = float(np.sum(gp * dirn))
        print("multi direction", seed, got, want, abs(got - want) / abs(want), flush=True)
        assert abs(got - want) <= 1e-6 * abs(want), (seed, got, want)


def _with_sigma(c, sigma):
    c = dict(c)
    c["sigma"] = sigma
    c["name"] = c["name"] + "_sigma"
    return c


@pytest.mark.parametrize("ndim,n", [(2, 24), (3, 12)])
def test_gradient_with_surface_tension_matches_oracle_finite_differences(ndim, n):
    """surface tension (Laplace jump sigma kappa in the interaction, Eq.
    surfacetension; ~1e4 Pa on this column or droplet): with the geometry
    frozen the jump of each cut cell is a constant of the recorded level set;
    directions and both fluids' EOS parameters (the air's p_inf enters
    through the jump-shifted wave curve) against central differences of the
    oracle's replayed run"""
    print("adjoint surface tension case ndim=%d n=%d" % (ndim, n), flush=True)
    c = _with_sigma(AC.curved_case(n, ndim), 3.0e3)
    steps = 6
    r = _gradient(c, steps, ckpt=4)
    log = _oracle_log(c, r["dt"], steps)
    g0, p0 = list(c["gamma"]), list(c["pinf"])
    for seed in (7, 11):
        dirn = AC.interface_direction(c, seed=seed)
        want = _richardson(lambda e: _oracle_J(c, c["prim"] + e * dirn, g0, p0, log, r["dt"], steps, r["probes"]),
                           3e-3)
        got = float(np.sum(r["gp"] * dirn))
        print("sigma direction", seed, got, want, abs(got - want) / abs(want), flush=True)
        assert abs(got - want) <= 1e-6 * abs(want), (seed, got, want)
    # fluid 0 is the water (p_inf 6e8), fluid 1 the air (p_inf 0)
    steps_eos = {(0, 0): 1e-6 * g0[0], (0, 1): 1e-6 * p0[0], (1, 0): 1e-3 * g0[1], (1, 1): 100.0}
    for k in (0, 1):
        rk_ = _gradient(c, steps, ckpt=4, fluid=k)
        for j in (0, 1):
            def Je(e, j=j):
                g, p = list(g0), list(p0)
                (g if j == 0 else p)[k] += e
                return _oracle_J(c, c["prim"], g, p, log, r["dt"], steps, rk_["probes"])
            want = _richardson(Je, steps_eos[(k, j)])
            got = float(rk_["ge"][k, j])
            print("sigma eos", k, j, got, want, abs(got - want) / abs(want), flush=True)
            assert abs(got - want) <= 1e-6 * abs(want), (k, j, got, want)


@pytest.mark.parametrize("ndim,n,ckpt", [(2, 24, 1), (3, 12, 2)])
def test_accelerated_cycles_with_surface_tension_gradient(ndim, n, ckpt):
    """accelerated cycles with surface tension: the correction books the slow
    fluid's flux at its own interface pressure, reversed as such"""
    import paper_1905_03917_amd as P
    from oracle import oracle as O
    print("adjoint multi_dt surface tension case ndim=%d n=%d" % (ndim, n), flush=True)
    c = _with_sigma(AC.curved_case(n, ndim), 3.0e3)
    cycles = 2
    sim = P.Sim(c, tape=1, ckpt_every=ckpt)
    st = sim.advance(1e30, mode=P.SIM_MULTI_DT, max_cycles=cycles)
    assert st["steps"][0] != st["steps"][1]
    _, cons, alpha = sim.state(device=False)
    probes = AC.interface_probes(alpha)
    J, gc, ge_loss = AC.interface_loss(cons, alpha, c["gamma"], c["pinf"], probes, ndim)
    gp, ge = sim.backward(gc)
    sim.close()
    o = O.OracleSim(c, log_levelset=1)
    ost = o.advance(1e30, mode=1, max_cycles=cycles)
    assert ost["steps"] == st["steps"]
    log, sched = o.levelset_log(), o.schedule()
    for seed in (7, 11):
        dirn = AC.interface_direction(c, seed=seed)
        want = _richardson(lambda e: _oracle_J_multi(c, c["prim"] + e * dirn, c["gamma"], c["pinf"], log, sched,
                                                     cycles, probes), 1e-3)
        got = float(np.sum(gp * dirn))
        print("sigma multi direction", seed, got, want, abs(got - want) / abs(want), flush=True)
        assert abs(got - want) <= 1e-6 * abs(want), (seed, got, want)
