"""The oracle's level-set log and replay (single-dt steps): replaying a run's
own stage level sets reproduces it, and the replayed run is a smooth map of
the initial state (the map the adjoint with frozen geometry differentiates,
Sec. 2.1 Eq. Eulerdiscrete with the cut-cell geometry of Sec. 2.3 held at
its recorded values)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_03917_amd import workloads as WL


def _case(n=24):
    # acoustic pulse in air crossing a flat air/water interface, with a
    # smooth background wave so that finite differences stay in the WENO
    # weights' linear response
    c = WL.smooth_2d(n=n, seed=3, width=0.15)
    h = c["h"]
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    wave = 2.0e3 * np.sin(2 * np.pi * (X.reshape(-1) + 0.1)) * np.cos(2 * np.pi * (Y.reshape(-1) - 0.2))
    for k, c2 in ((0, 1.4e5), (1, 4.4 * (1e5 + 6e8) / 1000.0)):
        c["prim"][k, 3] += wave
        c["prim"][k, 0] += wave / c2
        c["prim"][k, 1] += 20.0
    return c


def _run(case, steps, prim=None, **over):
    s = O.OracleSim(case, **over)
    if prim is not None:
        s.set_state(case["phi"], prim)
    s.advance(1e30, mode=0, max_cycles=steps)
    return s


def test_replaying_the_own_level_sets_reproduces_the_run():
    case = _case()
    a = _run(case, 4, log_levelset=1)
    log = a.levelset_log()
    assert log.shape == (4 * 3, case["phi"].size)
    b = _run(case, 4, ls_replay=log, dt_replay=a.schedule())
    pa, ca, _ = a.state()
    pb, cb, _ = b.state()
    assert np.array_equal(pa, pb) and np.array_equal(ca, cb)
    # the interface moved: the replay is not a run with a still level set
    assert np.max(np.abs(log[-1] - case["phi"])) > 1e-9


def test_replaying_accelerated_cycles_reproduces_them():
    """accelerated cycles (Sec. 3.1): the fast sub-steps' stage level sets
    and the CFL schedule replayed reproduce the run"""
    case = _case(24)
    a = O.OracleSim(case, log_levelset=1)
    st = a.advance(1e30, mode=1, max_cycles=2)
    assert st["steps"][0] != st["steps"][1]          # sub-stepping took place
    log = a.levelset_log()
    assert log.shape[0] == 3 * max(st["steps"])
    b = O.OracleSim(case, ls_replay=log, dt_replay=a.schedule())
    b.advance(1e30, mode=1, max_cycles=2)
    pa, ca, _ = a.state()
    pb, cb, _ = b.state()
    assert np.array_equal(pa, pb) and np.array_equal(ca, cb)
    # past the log's end the replay stops with an error
    with pytest.raises(RuntimeError):
        b.advance(1e30, mode=1, max_cycles=1)


def test_the_replayed_map_is_smooth():
    """central differences of a pressure-probe loss along a smooth direction
    converge at second order: halving eps divides the change of the
    difference quotient by about four.  (Below eps ~ 4e-3 the quotients
    wander by ~5e-7 relative: the interface Riemann root is exact only to
    its stopping tolerance, ~6e-10 relative, and its iteration count moves
    with the input.)"""
    case = _case()
    a = _run(case, 3, log_levelset=1)
    log, sched = a.levelset_log(), a.schedule()
    nc = case["phi"].size
    rng = np.random.default_rng(1)
    dirn = np.zeros_like(case["prim"])
    x = (np.arange(24) + 0.5) / 24
    X, Y = np.meshgrid(x, x, indexing="xy")
    dirn[:, 3] = (np.sin(2 * np.pi * X + 0.3) * np.cos(2 * np.pi * Y - 0.1)).reshape(-1) * 1e3
    probes = rng.choice(nc, 8, replace=False)

    def J(eps):
        s = _run(case, 3, prim=case["prim"] + eps * dirn, ls_replay=log, dt_replay=sched)
        _, cons, alpha = s.state()
        out = 0.0
        for k in (0, 1):
            a_k = alpha if k == 0 else 1.0 - alpha
            m = a_k[probes] > 0.5
            U = cons[k][:, probes[m]] / a_k[probes[m]]
            g, pi = case["gamma"][k], case["pinf"][k]
            p = (g - 1) * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / U[0]) - g * pi
            out += np.sum((p - 1e5) ** 2) / 1e6
        return out

    q = [(J(e) - J(-e)) / (2 * e) for e in (3.2e-2, 1.6e-2, 8e-3)]
    r = (q[0] - q[1]) / (q[1] - q[2])
    assert abs(q[2]) > 0
    assert 3.0 < r < 5.0, (q, r)
