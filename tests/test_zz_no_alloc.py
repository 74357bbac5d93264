"""The no-allocation diagnostics entry point against ocn_diagnostics, through
the C ABI: two calls in a row on one GPU, the second on a smaller grid, in
both precisions; and the size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_2309_06662_amd import inputs
from tests.helpers import small_latlon

pytestmark = pytest.mark.gpu


def _both(m):
    from paper_2309_06662_amd import ocn

    L = ocn.lib()
    a, b = ocn.Diag(), ocn.Diag()
    ra = L.ocn_diagnostics(m.handle, C.byref(a))
    rb = L.ocn_diagnostics_noalloc(m.handle, C.byref(b))
    assert ra == rb == 0, (ra, rb, L.ocn_last_error())
    return ({n: getattr(a, n) for n, _ in ocn.Diag._fields_}, {n: getattr(b, n) for n, _ in ocn.Diag._fields_})


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_diagnostics_equal_the_arena_ones(precision):
    from paper_2309_06662_amd import ocn

    big = small_latlon(nx=300, ny=140, nz=7, tau0=0.3)
    small = inputs.BETA_BASIN_64.replace(name="beta_37x21x5", nx=37, ny=21, nz=5)
    for w, steps in ((big, 4), (small, 3)):
        m = ocn.Model(w, precision, inputs.make_inputs(w))
        m.step(steps)
        a, b = _both(m)
        for k in a:
            assert a[k] == b[k] or (np.isnan(a[k]) and np.isnan(b[k])), (w.name, k, a[k], b[k])
        assert a["kinetic_energy"] > 0 and a["step"] == steps
        m.close()


def test_noalloc_rejects_grids_beyond_its_scratch():
    from paper_2309_06662_amd import ocn

    w = inputs.BETA_BASIN_64.replace(name="beta_4160x2048x1", nx=4160, ny=2048, nz=1, depth=100.0)
    m = ocn.Model(w, "fp32", inputs.make_inputs(w))
    d = ocn.Diag()
    rc = ocn.lib().ocn_diagnostics_noalloc(m.handle, C.byref(d))
    assert rc == ocn.OCN_E_UNSUPPORTED
    assert b"fixed diagnostics scratch" in ocn.lib().ocn_last_error()
    m.close()
