"""pn_batch_scan_noalloc (the batch scan on the library's static device
workspace, for callers that cannot allocate) against pn_batch_scan on the
same inputs, bit for bit, on two calls in a row, the second smaller."""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, dev

pytestmark = pytest.mark.gpu

KEYS = ("fli", "label", "status", "y_final", "dH", "dJ", "newton_max", "renorms", "steps")


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1802_00147_amd import pn as P
    P.lib()
    return P


def _inputs(pn, n, seed):
    from paper_1802_00147_amd import workloads as W
    wl = W.batch(n=n, seed=seed, tmin=50.0, tmax=800.0)
    cols = [dev(getattr(wl, k)) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")]
    b, c1, c2, t = (dev(getattr(wl, k)) for k in ("beta", "chi1", "chi2", "t_end"))
    return pn.init_state(*cols, b, c1, c2), t, b, c1, c2


def _host(out):
    return {k: out[k].cpu().numpy() for k in KEYS}


def test_noalloc_batch_scan_equals_batch_scan(pn):
    for n, seed in ((5000, 61), (1200, 62)):          # the second call smaller than the first
        y0, t, b, c1, c2 = _inputs(pn, n, seed)
        got = _host(pn.batch_scan_noalloc(y0, t, b, c1, c2))
        ref = _host(pn.batch_scan(y0, t, b, c1, c2))
        torch.cuda.synchronize()
        for k in KEYS:
            assert np.array_equal(got[k].view(np.uint8), ref[k].view(np.uint8)), (n, k)
        assert np.all(got["steps"][(got["status"] & 0xFF) == 0] == np.ceil(t.cpu().numpy())[(got["status"] & 0xFF) == 0])
