"""Captured steps (opts graph=1): single-dt steps of a fixed length replayed
from HIP graphs must give the states of the same steps issued launch by
launch, bit for bit, after every call, with the program's own device work
and synchronisations between the replays."""
import numpy as np
import pytest

from paper_1905_03917_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1905_03917_amd as P
    return torch, P


def _first_dt(P, case):
    s = P.Sim(case)
    st = s.advance(1.0, P.SIM_SINGLE_DT, max_cycles=1)
    s.close()
    return min(st["last_dt"])


CASES = [("tube_1d", lambda: WL.tube_1d(n=600, seed=4)),
         ("shock_bubble_2d", lambda: WL.shock_bubble_2d(n=80, seed=5)),
         ("shock_droplet_3d", lambda: WL.shock_droplet_3d(n=24, seed=6))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_graph_steps_match_launches_one_by_one(name, make):
    torch, P = _mods()
    case = make()
    dt = 0.5 * _first_dt(P, case)
    plain = P.Sim(case, dt_fixed=dt)
    graph = P.Sim(case, dt_fixed=dt, graph=1)
    junk = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    t = 0.0
    steps = 0
    print("case", name, "dt", dt, flush=True)
    for call, m in enumerate([1, 1, 3, 6, 1, 9, 2]):
        t += m * dt
        sa = plain.advance(t, P.SIM_SINGLE_DT)
        sb = graph.advance(t, P.SIM_SINGLE_DT)
        steps += sa["cycles"]
        for key in ("cycles", "steps", "cell_updates", "t", "last_dt", "bflux", "active_cells"):
            assert np.array_equal(np.asarray(sa[key]), np.asarray(sb[key])), (name, call, key, sa[key], sb[key])
        pa, ca, aa = plain.state()
        pb, cb, ab = graph.state()
        assert torch.equal(pa, pb) and torch.equal(ca, cb) and torch.equal(aa, ab), (name, call)
        # the inflow ledger's accumulators are written inside the graphs
        assert np.array_equal(plain.totals(), graph.totals()), (name, call)
        # the program's own device work between replays
        junk.add_(ca.sum())
        torch.cuda.synchronize()
    captures, replays, held = graph.graph_info()
    print("captures", captures, "replays", replays, "held", held, "steps", steps, flush=True)
    assert 1 <= captures <= replays and 1 <= held <= 4
    # the last step of a call may be shortened to reach t_end (rounding of
    # the summed steps): it runs launch by launch
    assert replays >= steps - 7, (replays, steps)
    assert plain.graph_info() == (0, 0, 0)
    plain.close()
    graph.close()


def test_graph_steps_between_accelerated_cycles():
    """accelerated cycles (never captured) and captured single-dt steps in
    turn on one simulation: the host state a replay leaves must be the one
    the launches would have left"""
    torch, P = _mods()
    case = WL.shock_bubble_2d(n=64, seed=7)
    dt = 0.4 * _first_dt(P, case)
    plain = P.Sim(case, dt_fixed=dt)
    graph = P.Sim(case, dt_fixed=dt, graph=1)
    for r in range(3):
        ta = plain.advance(1e9, P.SIM_MULTI_DT, max_cycles=1)["t"]
        tb = graph.advance(1e9, P.SIM_MULTI_DT, max_cycles=1)["t"]
        assert ta == tb, (r, ta, tb)
        t = ta + 5 * dt
        plain.advance(t, P.SIM_SINGLE_DT)
        graph.advance(t, P.SIM_SINGLE_DT)
        pa, ca, aa = plain.state()
        pb, cb, ab = graph.state()
        assert torch.equal(pa, pb) and torch.equal(ca, cb) and torch.equal(aa, ab), r
    assert graph.graph_info()[1] >= 10
    plain.close()
    graph.close()


def test_graph_size_gate():
    """graph=1 captures only grids of at most SIM_GRAPH_MAX_CELLS cells,
    graph=2 at any size; both give the launches' state"""
    torch, P = _mods()
    case = WL.tube_1d(n=P.SIM_GRAPH_MAX_CELLS + 1, seed=2)
    dt = 0.5 * _first_dt(P, case)
    sims = [P.Sim(case, dt_fixed=dt, graph=g) for g in (0, 1, 2)]
    for s in sims:
        s.advance(6 * dt, P.SIM_SINGLE_DT)
    assert sims[1].graph_info()[0] == 0 and sims[2].graph_info()[0] >= 1
    ref = sims[0].state()
    for s in sims[1:]:
        assert all(torch.equal(x, y) for x, y in zip(ref, s.state()))
    for s in sims:
        s.close()
    with pytest.raises(RuntimeError, match="graph must be"):
        P.Sim(WL.tube_1d(n=300, seed=1), dt_fixed=dt, graph=3)


def test_graph_needs_a_fixed_step():
    torch, P = _mods()
    with pytest.raises(RuntimeError, match="dt_fixed"):
        P.Sim(WL.tube_1d(n=300, seed=1), graph=1)


def test_graph_run_reports_a_nonphysical_state():
    """a run of captured steps reads the error flags once, after its last
    step: a non-physical state is reported by that call, as by the launches
    issued one by one; the captured run rolls back to its own start (the
    launches one by one to the start of the failing step), and the reported
    time and statistics are those of the rolled-back state"""
    torch, P = _mods()
    case = WL.vacuum_tube_1d()
    dt = 0.5 * _first_dt(P, case)
    for g in (0, 1):
        print("graph rollback case graph=%d" % g, flush=True)
        s = P.Sim(case, dt_fixed=dt, graph=g)
        s.advance(10 * dt, P.SIM_SINGLE_DT)
        assert s.last_stats["cycles"] == 10
        _, c10, _ = s.state(device=False)
        with pytest.raises(P.SimError) as e:
            s.advance(200 * dt, P.SIM_SINGLE_DT)
        assert e.value.status == -4, (g, str(e.value))
        st = s.last_stats
        _, cr, _ = s.state(device=False)
        if g:
            assert st["cycles"] == 0 and st["t"] == 10 * dt, st
            np.testing.assert_array_equal(cr, c10)
        else:
            assert 10 < 10 + st["cycles"] < 200 and st["t"] == pytest.approx((10 + st["cycles"]) * dt, rel=1e-12)
        s.close()


def _first_dts(P, case, rk):
    s = P.Sim(case, rk=rk)
    st = s.advance(1.0, P.SIM_MULTI_DT, max_cycles=1)
    s.close()
    return [float(x) for x in st["last_dt"]]


CYCLE_CASES = [("tube_1d", lambda: WL.tube_1d(n=600, seed=4), 3),
               ("shock_bubble_2d", lambda: WL.shock_bubble_2d(n=80, seed=5), 3),
               ("shock_bubble_2d_rk2", lambda: WL.shock_bubble_2d(n=64, seed=8), 2),
               ("shock_droplet_3d", lambda: WL.shock_droplet_3d(n=24, seed=6), 3),
               ("static_drop_2d", lambda: WL.static_drop(48, 2, seed=2), 3)]


@pytest.mark.parametrize("name,make,rk", CYCLE_CASES, ids=[c[0] for c in CYCLE_CASES])
def test_graph_cycles_match_launches_one_by_one(name, make, rk):
    """accelerated cycles with prescribed steps (dt_fixed_fluid): captured
    whole (graph=2) and replayed against the same cycles issued launch by
    launch, bit for bit after every call, statistics included"""
    torch, P = _mods()
    case = make()
    dts = [0.8 * x for x in _first_dts(P, case, rk)]
    plain = P.Sim(case, rk=rk, dt_fixed_fluid=dts)
    graph = P.Sim(case, rk=rk, dt_fixed_fluid=dts, graph=2)
    junk = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    print("case", name, "rk", rk, "dt", dts, flush=True)
    cycles = 0
    for call, m in enumerate([1, 2, 1, 4, 3]):
        sa = plain.advance(1e9, P.SIM_MULTI_DT, max_cycles=m)
        sb = graph.advance(1e9, P.SIM_MULTI_DT, max_cycles=m)
        cycles += sa["cycles"]
        for key in ("cycles", "steps", "cell_updates", "t", "last_dt", "last_n", "bflux", "active_cells"):
            assert np.array_equal(np.asarray(sa[key]), np.asarray(sb[key])), (name, call, key, sa[key], sb[key])
        pa, ca, aa = plain.state()
        pb, cb, ab = graph.state()
        assert torch.equal(pa, pb) and torch.equal(ca, cb) and torch.equal(aa, ab), (name, call)
        assert np.array_equal(plain.totals(), graph.totals()), (name, call)
        junk.add_(ca.sum())
        torch.cuda.synchronize()
    captures, replays, held = graph.graph_info()
    print("captures", captures, "replays", replays, "held", held, "cycles", cycles, "steps", sb["steps"], flush=True)
    assert 1 <= captures <= replays == cycles and 1 <= held <= 4
    plain.close()
    graph.close()


@pytest.mark.parametrize("mode_rk", [3, 2])
def test_prescribed_cycles_match_oracle(mode_rk):
    """the prescribed steps give the cycle the paper's plan computed from
    them (Sec. 3.1): the oracle replays that schedule (both fluids' steps at
    each cycle start, the fast fluid's at each later sub-step, from its own
    planning functions) and reaches the captured cycles' state at the parity
    bar"""
    torch, P = _mods()
    from oracle import oracle as O
    from test_gpu_parity import _worst
    case = WL.shock_bubble_2d(n=64, seed=9)
    dts = [0.8 * x for x in _first_dts(P, case, mode_rk)]
    ncyc = 3
    g = P.Sim(case, rk=mode_rk, dt_fixed_fluid=dts, graph=2)
    sg = g.advance(1e9, P.SIM_MULTI_DT, max_cycles=ncyc)
    S = 0 if dts[0] >= dts[1] else 1
    F = 1 - S
    t1, single = O.plan_cycle(dts[S], dts[F], 1e30)
    assert not single
    sched = []
    for _ in range(ncyc):
        sched += dts
        tau, half, first = 0.0, 0, True
        while True:
            if not first:
                sched.append(dts[F])
            d, hh, fin = O.substep(tau, t1, dts[F], mode_rk, half)
            tau = 0.5 * t1 if hh else (t1 if fin else tau + d)
            half = half or hh
            first = False
            if fin:
                break
    o = O.OracleSim(case, rk=mode_rk, dt_replay=sched)
    so = o.advance(1e9, mode=1, max_cycles=ncyc)
    assert sg["steps"] == so["steps"] and sg["cycles"] == so["cycles"], (sg, so)
    assert sg["t"] == pytest.approx(so["t"], rel=1e-13)
    _, cg, _ = g.state(device=False)
    _, co, _ = o.state()
    e, where = _worst(cg, co, 2)
    print("captured prescribed cycles vs oracle: steps %s, worst relative %.3e at %s" % (sg["steps"], e, where))
    assert e <= 1e-10, (e, where)
    g.close()


def test_prescribed_steps_refused_combinations():
    torch, P = _mods()
    case = WL.shock_bubble_2d(n=32, seed=1)
    for bad in (dict(dt_fixed_fluid=[1e-6, 0.0]), dict(dt_fixed_fluid=[1e-6, 1e-6], tape=1),
                dict(dt_fixed_fluid=[1e-6, 1e-6], dt_replay=[1e-6, 1e-6])):
        with pytest.raises(P.SimError) as e:
            P.Sim(case, **bad)
        assert e.value.status == -1, bad


def test_graph_cycle_size_gate():
    """graph=1 captures accelerated cycles only on grids of at most
    SIM_GRAPH_MAX_CELLS_CYCLE cells, graph=2 at any size; all give the
    launches' state"""
    torch, P = _mods()
    case = WL.tube_1d(n=P.SIM_GRAPH_MAX_CELLS_CYCLE + 1, seed=2)
    dts = [0.5 * x for x in _first_dts(P, case, 3)]
    sims = [P.Sim(case, dt_fixed_fluid=dts, graph=g) for g in (0, 1, 2)]
    for s in sims:
        s.advance(1e9, P.SIM_MULTI_DT, max_cycles=3)
    assert sims[1].graph_info()[0] == 0 and sims[2].graph_info()[0] >= 1
    ref = sims[0].state()
    for s in sims[1:]:
        assert all(torch.equal(x, y) for x, y in zip(ref, s.state()))
    for s in sims:
        s.close()
