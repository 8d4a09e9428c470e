"""gs_sqdiff_noalloc (the no-allocation variant of gs_sqdiff, whose partial
sums live in the library's static device array) against gs_sqdiff through the
C ABI: two calls in a row, the second with a smaller input, for every storage
type; the results must be bitwise equal (same kernel, same fold order). Also
checks the size limit and that validation happens before any device work."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def test_noalloc_matches_workspace_variant(torch):
    from paper_2309_10292_amd import gs
    L = gs.load()
    ws = torch.empty(int(L.gs_sqdiff_workspace_bytes()), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(20231)
    dtypes = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16, 3: torch.float16}
    for storage, dt in dtypes.items():
        big = 3 * (1 << 20) + 77
        a = torch.from_numpy(rng.uniform(0, 1, size=big)).to(device="cuda", dtype=dt)
        b = torch.from_numpy(rng.uniform(0, 1, size=big)).to(device="cuda", dtype=dt)
        for n in (big, 1000):  # the second call is smaller: stale partials of the first must not leak in
            ref, got = ctypes.c_double(), ctypes.c_double()
            gs.check(L.gs_sqdiff(a.data_ptr(), b.data_ptr(), n, storage, ws.data_ptr(), stream, ctypes.byref(ref)))
            gs.check(L.gs_sqdiff_noalloc(a.data_ptr(), b.data_ptr(), n, storage, stream, ctypes.byref(got)))
            exact = float(((a[:n].double() - b[:n].double()) ** 2).sum())
            assert got.value == ref.value, (storage, n, got.value, ref.value)
            assert abs(got.value - exact) <= 1e-12 * exact, (storage, n)
    assert gs.sqdiff_noalloc(a[:5], b[:5]) == gs.sqdiff(a[:5], b[:5])
    # validation before any device work
    out = ctypes.c_double()
    assert L.gs_sqdiff_noalloc(a.data_ptr(), b.data_ptr(), (1 << 40) + 1, 0, stream, ctypes.byref(out)) == \
        gs.GS_ERR_UNSUPPORTED
    assert L.gs_sqdiff_noalloc(None, b.data_ptr(), 10, 0, stream, ctypes.byref(out)) == gs.GS_ERR_INVALID_ARG
    assert L.gs_sqdiff_noalloc(a.data_ptr(), b.data_ptr(), 10, 7, stream, ctypes.byref(out)) == gs.GS_ERR_INVALID_ARG
