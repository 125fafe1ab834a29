"""The FP32 FMA probe that the roofline's ceiling comes from computes what it says: every
thread's 16 chains of x <- fma(x, a, b) from x0 = tid / 1000 + i, summed in chain order,
against the same recurrence on the host (each step evaluated in float64, where the product
is exact, and rounded to FP32: within a few units in the last place of a fused FMA)."""
import numpy as np
import pytest

from helpers import log, require_gpu

pytestmark = pytest.mark.gpu


def test_fma_probe_matches_its_recurrence():
    torch = require_gpu()
    from paper_2508_06672_amd import geoloc
    blocks, iters = 3, 500
    out = torch.full((blocks * 256,), float("nan"), dtype=torch.float32, device="cuda")
    per_lane = geoloc.geoloc_fma_probe(blocks, iters, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert per_lane == 16 * iters
    got = out.cpu().numpy().reshape(blocks, 256)
    a, b = np.float32(0.999), np.float32(1e-4)
    tid = np.arange(256, dtype=np.float32)
    x = np.stack([tid * np.float32(1e-3) + np.float32(i) for i in range(16)])      # [chain][thread]
    for _ in range(iters):
        x = (x.astype(np.float64) * np.float64(a) + np.float64(b)).astype(np.float32)
    s = np.zeros(256, dtype=np.float32)
    for i in range(16):
        s = (s + x[i]).astype(np.float32)
    err = np.max(np.abs(got - s[None, :]) / np.abs(s[None, :]))
    log(f"fma probe: max rel err {err:.3g} over {blocks} x 256 threads")
    assert err <= 1e-6
    with pytest.raises(geoloc.GeolocError) as ei:
        geoloc.geoloc_fma_probe(0, iters, out.data_ptr())
    assert ei.value.status == geoloc.EINVAL
