"""The allocation-free reduction (krt_reduce_noalloc, block partials in the
library's static device scratch) against krt_reduce (partials in the
context's buffer): the same fluxes and I_max bit for bit, on two calls in a
row, the second on a smaller image, through the C ABI."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2302_02733_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def krt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_02733_amd import krt as K
    return K


def _noalloc(K, ctx, stokes, cam):
    c = K.make_camera(cam)
    flux = (ctypes.c_double * 4)()
    imax = ctypes.c_double()
    ctx._stream()
    ctx._check(K.lib().krt_reduce_noalloc(ctx.h, K._ptr(stokes), ctypes.byref(c), flux, ctypes.byref(imax)))
    return [flux[k] for k in range(4)], imax.value


def test_noalloc_reduce_equals_reduce(krt):
    with krt.Context(0) as ctx:
        ctx.set_units(W.UNITS)
        ctx.set_model(W.ADAF)
        results = []
        for n, m in ((256, 256), (37, 23)):
            cam = dict(W.adaf_camera(n), ny=m)
            out = ctx.trace(cam)
            # a reference call first, then the allocation-free one, then the
            # reference again: the shared scratch keeps no state between calls
            f0, i0 = ctx.reduce(out["stokes"], cam)
            f1, i1 = _noalloc(krt, ctx, out["stokes"], cam)
            f2, i2 = ctx.reduce(out["stokes"], cam)
            results.append((n, m, f0, f1))
            assert list(f1) == list(f0) and i1 == i0
            assert list(f2) == list(f0) and i2 == i0
            assert f0[0] > 0.0 and i0 > 0.0
        # the two images differ, so a stale scratch would show
        assert results[0][2][0] != results[1][2][0]
