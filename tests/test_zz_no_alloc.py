"""sim_totals_noalloc, the ledger for callers that cannot allocate: through
the C ABI its totals equal sim_totals' bit for bit (same kernels, grid and
summation order, with the partial sums in the library's per-device scratch
array), on two calls in a row, the second on a smaller simulation, to a
host array and to a device buffer; a call before sim_set_state is
refused."""
import ctypes as C

import numpy as np
import pytest

from paper_1905_03917_amd import workloads as WL

pytestmark = pytest.mark.gpu


def test_noalloc_totals_equal_the_allocating_ledger():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1905_03917_amd as P
    L = P.lib()
    cases = [WL.shock_bubble_2d(n=256, seed=3), WL.shock_bubble_2d(n=64, seed=4), WL.tube_1d(n=300, seed=5)]
    out_dev = torch.full((10,), float("nan"), dtype=torch.float64, device="cuda")
    for i, c in enumerate(cases):
        print("noalloc ledger case %s n=%s" % (c["name"], c["n"]), flush=True)
        s = P.Sim(c)
        s.advance(1.0, mode=1, max_cycles=2)
        ref = s.totals()
        host = np.full(10, np.nan)
        rc = L.sim_totals_noalloc(s.h, C.c_void_p(host.ctypes.data), 0)
        assert rc == 0, P.SimError(rc, "sim_totals_noalloc")
        np.testing.assert_array_equal(host.reshape(2, 5), ref)
        out_dev.fill_(float("nan"))
        rc = L.sim_totals_noalloc(s.h, C.c_void_p(out_dev.data_ptr()), 1)
        assert rc == 0
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out_dev.cpu().numpy().reshape(2, 5), ref)
        # the binding's wrapper, both ways
        np.testing.assert_array_equal(s.totals_noalloc(), ref)
        s.close()


def test_noalloc_totals_before_state_is_refused():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1905_03917_amd as P
    c = WL.tube_1d(n=64)
    s = P.Sim({k: v for k, v in c.items() if k not in ("phi", "prim")})
    host = np.zeros(10)
    assert P.lib().sim_totals_noalloc(s.h, C.c_void_p(host.ctypes.data), 0) == -5
    assert P.lib().sim_totals_noalloc(s.h, None, 0) == -1
    s.close()
