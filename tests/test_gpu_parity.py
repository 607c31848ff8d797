"""GPU (gfx950) path vs the CPU oracle on the same seeded inputs, through the
C ABI.  Bar: relative L-infinity 1e-10 after one step/cycle, relative L1 1e-8
over longer runs, conservation drift <= 1e-12 per step."""
import sys

import numpy as np
import pytest

from paper_1905_03917_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _gpu(case, **opts):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1905_03917_amd as P
    return P.Sim(case, **opts)


def _scales(co, D):
    """per (fluid, component) magnitude: max |value|, with momentum measured
    against sqrt(max rho * max E) so that a fluid at rest is not judged on
    round-off noise"""
    sc = np.zeros(co.shape[:2])
    for k in range(2):
        rho, E = np.abs(co[k, 0]).max(), np.abs(co[k, D + 1]).max()
        for q in range(co.shape[1]):
            sc[k, q] = max(np.abs(co[k, q]).max(), 1e-300)
            if 1 <= q <= D:
                sc[k, q] = max(sc[k, q], np.sqrt(rho * E))
    return sc


def _worst(cg, co, D, l1=False):
    sc = _scales(co, D)
    worst = (0.0, None)
    for k in range(2):
        for q in range(co.shape[1]):
            d = np.abs(cg[k, q] - co[k, q])
            e = (d.mean() if l1 else d.max()) / (sc[k, q] if not l1 else max(np.abs(co[k, q]).mean(), sc[k, q] * 1e-3))
            if e > worst[0]:
                worst = (e, (k, q, int(np.argmax(d))))
    return worst


def _compare(case, mode, max_cycles, t_end=1.0, tol=1e-10, l1=False, gpu_opts=None, **opts):
    """Both libraries on the same input: step counts, time, the contents at
    relative L-infinity (or L1) tol, the level set at tol relative to its
    largest (or mean) magnitude, the volume fraction at tol absolute (or in
    the mean), the ledger totals and the boundary inflow at tol relative to
    their scales."""
    print("parity case=%s n=%s mode=%d cycles=%d %s" % (case["name"], case["n"], mode, max_cycles, gpu_opts or ""),
          flush=True)
    g = _gpu(case, **opts, **(gpu_opts or {}))
    sg = g.advance(t_end, mode=mode, max_cycles=max_cycles)
    from oracle import oracle as O
    o = O.OracleSim(case, **opts)
    so = o.advance(t_end, mode=mode, max_cycles=max_cycles)
    assert sg["steps"] == so["steps"], (sg["steps"], so["steps"])
    assert sg["cycles"] == so["cycles"] and sg["cell_updates"] == so["cell_updates"]
    assert sg["t"] == pytest.approx(so["t"], rel=1e-12)
    pg, cg, ag = g.state(device=False)
    po, co, ao = o.state()
    D = case["ndim"]
    e, where = _worst(cg, co, D, l1=l1)
    dphi = np.abs(pg - po)
    if l1:
        ephi = dphi.mean() / np.abs(po).mean()
        ealpha = np.abs(ag - ao).mean()
        m = int(np.argmax(dphi))
        print("largest level-set difference %.3e at cell %d, |phi| there %.3f cells" % (dphi[m], m, abs(po[m]) / case["h"]))
    else:
        ephi = dphi.max() / np.abs(po).max()
        ealpha = np.abs(ag - ao).max()
    # ledger: totals per (fluid, component) and time-integrated inflow, each
    # against the per-cell scale of its component times the grid's volume
    sc = _scales(co, D)
    dv = case["h"] ** D
    nc = po.size
    tg, to = g.totals(), o.totals()
    etot = max(abs(tg[k, q] - to[k, q]) / (sc[k, q] * nc * dv) for k in range(2) for q in range(D + 2))
    ebf = max(abs(sg["bflux"][k, q] - so["bflux"][k, q]) / (abs(so["bflux"][k, q]) + 1e-3 * sc[k, q] * nc * dv)
              for k in range(2) for q in range(D + 2))
    print("worst relative %s error %.3e at (fluid, component, cell) %s; phi %.3e alpha %.3e totals %.3e inflow %.3e"
          % ("L1" if l1 else "Linf", e, where, ephi, ealpha, etot, ebf))
    assert e <= tol, (e, where)
    assert ephi <= tol, ephi
    assert ealpha <= tol, ealpha
    assert etot <= tol and ebf <= tol, (etot, ebf)
    return g, o, sg, so


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n", [400, 300])
def test_tube_1d_one_cycle(n, mode):
    _compare(WL.tube_1d(n=n, seed=n), mode, 1)


@pytest.mark.parametrize("cycles", [3, 20])
@pytest.mark.parametrize("mode", [0, 1])
def test_cavitation_floor(mode, cycles):
    """Air pulled apart at Mach 8: the interface Riemann problem lies past
    the vacuum limit, so p* is the floor from the first cycle on (the GPU
    solver reaches it lazily, through its Newton iterates; the oracle tests it
    first).  Cycles before the state turns non-physical, against the oracle."""
    _compare(WL.vacuum_tube_1d(), mode, cycles)


@pytest.mark.parametrize("name,n,mode,cycles", [("shock_bubble_2d", 48, 1, 3), ("shock_bubble_2d", 48, 0, 4),
                                                ("shock_droplet_3d", 20, 1, 2), ("tube_1d", 300, 1, 4)])
def test_schedule_replay(name, n, mode, cycles):
    """dt_replay in both directions: the oracle replays the GPU's schedule,
    the GPU replays the oracle's, each reaching the other's state at the
    parity bar; and the GPU replaying its own schedule (host-planned sub-steps
    instead of device-planned ones in 1-D/2-D) gives the same bits."""
    from oracle import oracle as O
    case = getattr(WL, name)(n=n, seed=3)
    print("schedule replay case=%s n=%d mode=%d" % (name, n, mode), flush=True)
    g = _gpu(case)
    sg = g.advance(1.0, mode=mode, max_cycles=cycles)
    sch_g = g.schedule()
    o = O.OracleSim(case)
    so = o.advance(1.0, mode=mode, max_cycles=cycles)
    sch_o = o.schedule()
    assert len(sch_g) == len(sch_o) and sg["steps"] == so["steps"]
    # the CFL steps of the two libraries differ where the star-state speeds
    # of cut cells set them: the Riemann solver's root is fixed to ~1e-10
    # relative (its stopping tolerance), which is why the schedule is replayed
    np.testing.assert_allclose(sch_g, sch_o, rtol=1e-9)
    D = case["ndim"]
    # the oracle on the GPU's schedule
    o2 = O.OracleSim(case, dt_replay=sch_g)
    s2 = o2.advance(1.0, mode=mode, max_cycles=cycles)
    assert s2["steps"] == sg["steps"] and s2["t"] == sg["t"]
    e, _ = _worst(g.state(device=False)[1], o2.state()[1], D)
    assert e <= 1e-10, e
    # the GPU on the oracle's schedule
    g2 = _gpu(case, dt_replay=sch_o)
    s3 = g2.advance(1.0, mode=mode, max_cycles=cycles)
    assert s3["steps"] == so["steps"] and s3["t"] == so["t"]
    e, _ = _worst(g2.state(device=False)[1], o.state()[1], D)
    assert e <= 1e-10, e
    # the GPU on its own schedule
    g3 = _gpu(case, dt_replay=sch_g)
    s4 = g3.advance(1.0, mode=mode, max_cycles=cycles)
    assert s4["steps"] == sg["steps"] and s4["t"] == sg["t"]
    for x, y in zip(g.state(device=False), g3.state(device=False)):
        assert np.array_equal(x, y)
    assert np.array_equal(g3.schedule(), sch_g)
    # past the end of the schedule
    with pytest.raises(RuntimeError, match="dt_replay exhausted"):
        g3.advance(1.0, mode=mode, max_cycles=1)
    with pytest.raises(RuntimeError, match="not a positive step"):
        _gpu(case, dt_replay=np.array([1e-6, -1.0]))
    for s in (g, g2, g3):
        s.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_tube_1d_full_run_l1(mode):
    c = WL.tube_1d(n=400, seed=0)
    _compare(c, mode, 0, t_end=c["t_end"], tol=1e-8, l1=True)


@pytest.mark.parametrize("mode", [0, 1])
def test_tube_1d_fine_run_to_end(mode):
    """6400 cells to t_end (about 2000 accelerated cycles): the band never
    leaves the tiles classified at a cycle start, mass is conserved, and the
    density is close to the exact two-material Riemann solution (relative L1
    of the oracle at this resolution: 2.0e-4 to 2.1e-4)."""
    from oracle import oracle as O
    c = WL.tube_1d(n=6400, seed=0)
    print("fine tube case n=6400 mode=%d" % mode, flush=True)
    g = _gpu(c)
    tot0 = g.totals()
    st = g.advance(c["t_end"], mode=mode)
    assert st["t"] == pytest.approx(c["t_end"], rel=1e-14)
    tot1 = g.totals()
    steps = max(st["steps"])
    mass = np.abs(tot1[:, 0] - tot0[:, 0] - st["bflux"][:, 0]) / np.abs(tot0[:, 0])
    assert np.all(mass <= 1e-12 * steps), mass
    _, cons, alpha = g.state(device=False)
    x = (np.arange(6400) + 0.5) / 6400
    ex = O.exact_tube(c, x, c["t_end"])[:, 0]
    rho = np.where(alpha >= 0.5, cons[0, 0] / np.maximum(alpha, 1e-300),
                   cons[1, 0] / np.maximum(1 - alpha, 1e-300))
    sel = x >= 0.25
    l1 = np.abs(rho - ex)[sel].sum() / np.abs(ex)[sel].sum()
    assert l1 < 3e-4, l1


@pytest.mark.parametrize("rk", [2, 3])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n", [64, 50])
def test_shock_bubble_2d(n, mode, rk):
    _compare(WL.shock_bubble_2d(n=n, seed=n), mode, 2, rk=rk)


@pytest.mark.parametrize("mode", [0, 1])
def test_shock_bubble_2d_ten_cycles_l1(mode):
    _compare(WL.shock_bubble_2d(n=48, seed=7), mode, 10, tol=1e-8, l1=True)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n", [20, 17])
def test_shock_droplet_3d(n, mode):
    _compare(WL.shock_droplet_3d(n=n, seed=n), mode, 1)


@pytest.mark.parametrize("mode", [0, 1])
def test_droplet_periodic_2d(mode):
    _compare(WL.droplet_2d(n=40, seed=3), mode, 2)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n", [64, 100])
def test_band_at_zero_gradient_wall(n, mode):
    """the interface band crosses a zero-gradient wall: temporally blocked
    sweeps must evaluate positions beyond the wall as the wall cell"""
    _compare(WL.wall_bubble_2d(n=n, seed=2), mode, 2)


def test_smooth_2d(mode=1):
    _compare(WL.smooth_2d(n=48, seed=1), mode, 3)


def test_single_fluid_entropy_wave():
    c = WL.entropy_wave_1d(n=64)
    _compare(c, 0, 0, t_end=0.05)


@pytest.mark.parametrize("mode", [0, 1])
def test_gpu_conservation(mode):
    """Drift of each fluid's mass against its own total, per its own steps,
    and of the two fluids' summed momentum and energy (the interface
    exchanges them) per cycle, each at 1e-12 per step or cycle."""
    c = WL.shock_bubble_2d(n=96, seed=11)
    g = _gpu(c)
    tot0 = g.totals()
    st = g.advance(1.0, mode=mode, max_cycles=5)
    tot1 = g.totals()
    bf = st["bflux"]
    for k in range(2):
        mass = abs(tot1[k, 0] - tot0[k, 0] - bf[k, 0]) / abs(tot0[k, 0])
        assert mass <= 1e-12 * st["steps"][k], (k, mass, st["steps"])
    scale = np.abs(tot0).sum(0) + np.abs(tot1).sum(0) + np.abs(bf).sum(0)
    scale[1:3] = scale[1:3].sum()
    drift = np.abs(tot1.sum(0) - tot0.sum(0) - bf.sum(0))
    assert np.all(drift[1:4] <= 1e-12 * st["cycles"] * scale[1:4]), drift / scale


def test_ledger_is_the_deterministic_sum_of_the_state():
    """sim_totals (device tree reduction) against a compensated host sum of
    the same state, and bit-identical on repeated calls."""
    import math
    c = WL.shock_bubble_2d(n=200, seed=4)
    g = _gpu(c)
    g.advance(1.0, mode=1, max_cycles=2)
    tot = g.totals()
    _, cons, _ = g.state(device=False)
    dv = c["h"] ** 2
    for k in range(2):
        for q in range(4):
            ref = math.fsum(cons[k, q]) * dv
            assert abs(tot[k, q] - ref) <= 1e-13 * max(abs(ref), np.abs(cons[k, q]).sum() * dv), (k, q, tot[k, q], ref)
        assert tot[k, 4] == 0.0
    np.testing.assert_array_equal(tot, g.totals())


def test_gpu_rk2_cycle_reduces_bitwise():
    """RK2 and n truncated to 1: the accelerated cycle equals the original step."""
    c = WL.tube_1d_single(n=200, seed=3)
    a = _gpu(c, rk=2)
    a.advance(1e-3, mode=0, max_cycles=4)
    b = _gpu(c, rk=2, force_cycle=1)
    b.advance(1e-3, mode=1, max_cycles=4)
    for u, v in zip(a.state(device=False), b.state(device=False)):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("name,n,mode,cycles", [
    ("shock_bubble_2d", 256, 1, 3),
    ("shock_bubble_2d", 250, 0, 3),
    ("shock_bubble_2d", 1024, 1, 1),
    ("shock_droplet_3d", 48, 1, 2),
    ("tube_1d", 2000, 1, 3),
])
def test_overlapped_bulk_stages_equal_serial(name, n, mode, cycles):
    """Bulk-tile stages on their own streams (the default) give results
    bit-identical to every kernel on one stream: no kernel reads what a
    concurrently running one writes."""
    fn = getattr(WL, name)
    c = fn(n=n, seed=0)
    print("overlap case=%s n=%d mode=%d cycles=%d" % (name, n, mode, cycles), flush=True)
    a = _gpu(c, serial=1)
    sa = a.advance(1.0, mode=mode, max_cycles=cycles)
    b = _gpu(c)
    sb = b.advance(1.0, mode=mode, max_cycles=cycles)
    assert sa["steps"] == sb["steps"] and sa["t"] == sb["t"]
    np.testing.assert_array_equal(sa["bflux"], sb["bflux"])
    for u, v in zip(a.state(device=False), b.state(device=False)):
        np.testing.assert_array_equal(u, v)


def test_autotuned_launch_gives_identical_results():
    """The autotuner changes only the bulk stage's grid bound and the
    schedule (overlapped or serial): states, step counts and boundary ledgers
    equal those of the default configuration."""
    import paper_1905_03917_amd as P
    c = WL.shock_bubble_2d(n=512, seed=2)
    a = _gpu(c)
    sa = a.advance(1.0, mode=1, max_cycles=4)
    sa2 = a.advance(1.0, mode=1, max_cycles=4)
    b = _gpu(c, autotune=1)
    sb = b.advance(1.0, mode=1, max_cycles=4)
    assert not b.tuned()[1]
    sb2 = b.advance(1.0, mode=1, max_cycles=4)
    blocks, done, serial = b.tuned()
    print("autotuned: bound %d, serial %s" % (blocks, serial))
    assert done and blocks in (1024, 2048, 4096, 8192), (blocks, done)
    assert sa2["t"] == sb2["t"] and sa["steps"] == sb["steps"] and sa2["steps"] == sb2["steps"]
    for u, v in zip(a.state(device=False), b.state(device=False)):
        np.testing.assert_array_equal(u, v)
    assert P.Sim(c).tuned() == (2048, True, False)


def test_autotuned_schedule_1d_gives_identical_results():
    """On a launch-bound 1-D tube the tuner may pick the serial schedule; the
    results are those of the default configuration either way."""
    c = WL.tube_1d(n=400, seed=3)
    a = _gpu(c)
    b = _gpu(c, autotune=1)
    for s in (a, b):
        s.advance(1.0, mode=1, max_cycles=8)
    sa = a.advance(1.0, mode=1, max_cycles=40)
    sb = b.advance(1.0, mode=1, max_cycles=40)
    blocks, done, serial = b.tuned()
    print("autotuned 1-D: bound %d, serial %s" % (blocks, serial))
    assert done and sa["steps"] == sb["steps"] and sa["t"] == sb["t"]
    for u, v in zip(a.state(device=False), b.state(device=False)):
        np.testing.assert_array_equal(u, v)


def test_full_size_shock_bubble_cycle_vs_oracle():
    """One accelerated cycle of the 1024^2 shock-bubble (one air step, eight
    water sub-steps) in the benchmark's launch configuration, where every
    bulk-stage block loops over two tiles in the XCD-aware order, against
    the oracle (about 40 s of one CPU core) at the 1e-10 bar."""
    _compare(WL.shock_bubble_2d(n=1024, seed=0), 1, 1)


def test_full_size_shock_bubble_properties():
    """1024^2 shock-bubble, one accelerated cycle at the benchmark's launch
    configuration: conservation, and the far field untouched."""
    c = WL.shock_bubble_2d(n=1024, seed=0)
    g = _gpu(c)
    tot0 = g.totals()
    _, c0, _ = g.state(device=False)
    st = g.advance(1.0, mode=1, max_cycles=1)
    tot1 = g.totals()
    bf = st["bflux"]
    assert np.all(np.abs(tot1[:, 0] - tot0[:, 0] - bf[:, 0]) <= 1e-12 * 8 * np.abs(tot0[:, 0]))
    _, c1, _ = g.state(device=False)
    n = 1024
    X = (np.arange(n) + 0.5) / n
    far = np.zeros((n, n), bool)
    far[:, X > 0.8] = True             # ahead of the shock and right of the bubble
    far = far.reshape(-1)
    # the Shu-Osher combination a*x + (1-a)*x of an unchanged state rounds at one ulp
    np.testing.assert_allclose(c1[1][:, far], c0[1][:, far], rtol=4e-16, atol=0)


def test_full_size_shock_droplet_3d_properties():
    """256^3 shock-droplet, one accelerated cycle at the benchmark's launch
    configuration: conservation per fluid, and the air ahead of the shock
    and beyond the droplet untouched."""
    c = WL.shock_droplet_3d(n=256, seed=0)
    g = _gpu(c)
    tot0 = g.totals()
    _, c0, _ = g.state(device=False)
    st = g.advance(1.0, mode=1, max_cycles=1)
    assert st["steps"][0] > st["steps"][1]          # water sub-steps, one air step
    tot1 = g.totals()
    bf = st["bflux"]
    steps = max(st["steps"])
    assert np.all(np.abs(tot1[:, 0] - tot0[:, 0] - bf[:, 0]) <= 1e-12 * steps * np.abs(tot0[:, 0]))
    _, c1, _ = g.state(device=False)
    n = 256
    X = (np.arange(n) + 0.5) / n
    far = np.broadcast_to(X > 0.75, (n, n, n)).reshape(-1)
    np.testing.assert_allclose(c1[1][:, far], c0[1][:, far], rtol=4e-16, atol=0)


def test_error_paths():
    import paper_1905_03917_amd as P
    c = WL.tube_1d(n=64)
    with pytest.raises(P.SimError):
        P.Sim(dict(c, ndim=4))
    s = P.Sim({k: v for k, v in c.items() if k not in ("phi", "prim")})
    with pytest.raises(P.SimError):
        s.advance(1e-4)                      # no state yet
    bad = c["prim"].copy()
    bad[0, 0, 10] = -1.0                     # negative density in a water cell
    s.set_state(c["phi"], bad)
    with pytest.raises(P.SimError) as e:
        s.advance(1e-4, max_cycles=1)
    assert e.value.status == -4


# ---- multi-tile launches: every block of a tile-list kernel loops over
# several tiles (a cap that is a multiple of 8 takes the XCD-aware order,
# 12 the plain stride), as at the full sizes where the lists exceed the
# grid bounds
@pytest.mark.parametrize("cap", [8, 12])
@pytest.mark.parametrize("mode", [0, 1])
def test_capped_grids_2d(cap, mode):
    _compare(WL.shock_bubble_2d(n=64, seed=3), mode, 2, gpu_opts=dict(grid_cap=cap))


@pytest.mark.parametrize("cap", [8, 12])
def test_capped_grids_3d(cap):
    _compare(WL.shock_droplet_3d(n=20, seed=4), 1, 1, gpu_opts=dict(grid_cap=cap))


@pytest.mark.parametrize("cap", [8, 12])
def test_capped_grids_1d(cap):
    _compare(WL.tube_1d(n=3000, seed=5), 1, 3, gpu_opts=dict(grid_cap=cap))


# ---- to t_end: the 2-D shock-bubble (t_end 1.5e-4 s) at 64^2 and the 3-D
# shock-droplet at 24^3 to 3e-4 s (the time the 256^3 benchmark's 200
# cycles reach), in both modes, at relative L1 1e-8
@pytest.mark.parametrize("mode", [0, 1])
def test_shock_bubble_2d_to_t_end(mode):
    c = WL.shock_bubble_2d(n=64, seed=8)
    _compare(c, mode, 0, t_end=c["t_end"], tol=1e-8, l1=True)


@pytest.mark.parametrize("mode", [0, 1])
def test_shock_droplet_3d_to_t_end(mode):
    c = WL.shock_droplet_3d(n=24, seed=9)
    _compare(c, mode, 0, t_end=3.0e-4, tol=1e-8, l1=True)


# ---- the paper's own cases in its TVD-RK2 scheme, Tait water as the
# stiffened gas of its isentrope: the two 1-D tubes of Sec. 4.1 to their
# t_end (L1 1e-8) and one cycle (L-infinity 1e-10), the Sec. 4.2 droplet
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", ["e1_gas_water_tube", "e2_shock_air_water"])
def test_paper_tubes_rk2(name, mode):
    c = getattr(WL, name)(n=200)
    _compare(c, mode, 1, rk=2)
    _compare(c, mode, 0, t_end=c["t_end"], tol=1e-8, l1=True, rk=2)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("ndim,n", [(2, 32), (3, 24)])
def test_paper_droplet_rk2(ndim, n, mode):
    _compare(WL.e3_droplet(n=n, ndim=ndim), mode, 3, rk=2)
