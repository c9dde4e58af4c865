"""gesr_bin_static -- the binning entry point for callers that cannot allocate
device memory, whose scratch is a static per-GPU array -- against gesr_bin
through the C ABI: bit-identical sorted lists, ranges, worklist, instance
bases and counters on calls in a row with shrinking inputs (the array keeps
the previous call's contents), and a binning whose scratch exceeds the array
rejected on the host with GESR_ERR_CAPACITY."""
import numpy as np
import pytest

import gesr_inputs as gi
import oracle
from tests.gpu_util import log, raster_settings, splats_of, u32

pytestmark = pytest.mark.gpu


def _scene(name):
    if name == "spheres-100k":
        return gi.make_workload(2), oracle.Settings(sh_degree=3)
    if name == "blobs-100k-2v":
        return gi.make_workload(5, n_override=100_000, views_override=2), oracle.Settings(sh_degree=3)
    if name == "plain-2k":
        return gi.make_workload(1), oracle.Settings()
    if name == "drt-20k-8v":
        return gi.make_workload(3, n_override=20_000), oracle.Settings()
    raise KeyError(name)


def _outputs(b):
    cnt = u32(b["counters"]).copy()
    L = int(min(cnt[3], b["m_cap"]))
    return dict(counters=cnt, inst_base=u32(b["inst_base"]).copy(), ranges=u32(b["ranges"]).copy(),
                worklist=u32(b["worklist"]).copy(), val_sorted=u32(b["val_sorted"])[:L].copy(),
                tile_sorted=u32(b["tile_sorted"])[:L].copy())


def test_bin_static_equals_bin_on_calls_in_a_row():
    import torch
    from paper_2411_09156_amd import Rasterizer
    for name in ("spheres-100k", "blobs-100k-2v", "plain-2k"):
        scene, st = _scene(name)
        rast = Rasterizer(scene.cameras, raster_settings(st))
        sp = splats_of(scene)
        proj = rast.project(sp)
        ref = rast.bin(proj, scene.n, sync=True)
        need = int(rast.sizes(scene.n, ref["m_cap"]).bin_scratch_bytes)
        log(f"[gpu] static scratch: {name}, M={ref['M']}, scratch {need / 2**20:.1f} MiB")
        got = rast.bin(proj, scene.n, m_cap=ref["m_cap"], sync=True, static_scratch=True)
        assert got["scratch"] is None and got["M"] == ref["M"]
        torch.cuda.synchronize()
        a, b = _outputs(ref), _outputs(got)
        for k in a:
            np.testing.assert_array_equal(b[k], a[k], err_msg=f"{name}: {k}")
        assert a["counters"][3] > 0


def test_bin_static_rejects_a_binning_beyond_its_scratch():
    from paper_2411_09156_amd import Rasterizer
    from paper_2411_09156_amd._lib import BIN_STATIC_SCRATCH_BYTES, GESR_ERR_CAPACITY, GesrError
    scene, st = _scene("drt-20k-8v")
    rast = Rasterizer(scene.cameras, raster_settings(st))
    proj = rast.project(splats_of(scene))
    m_cap = 10_000_000
    assert rast.sizes(scene.n, m_cap).bin_scratch_bytes > BIN_STATIC_SCRATCH_BYTES
    with pytest.raises(GesrError) as ei:
        rast.bin(proj, scene.n, m_cap=m_cap, sync=False, static_scratch=True)
    assert ei.value.status == GESR_ERR_CAPACITY and "static scratch" in str(ei.value)
