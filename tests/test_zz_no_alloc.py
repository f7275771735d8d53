"""The allocation-free binning entry point (ts_bin_sort_noalloc, on the
library's fixed scratch array) against ts_bin_sort with a caller workspace:
sorted keys, values, tile ranges and device counters bit-exact and the
raster tile order valid (tiles of equal list length may come in any order),
on two calls in a row, the second with a smaller input (the
scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_19175_amd import binding as B
from paper_2505_19175_amd import synth
from paper_2505_19175_amd.render import Rasterizer, ViewState, scene_to_device

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


class _Bins:
    """A second set of list buffers for the same view."""

    def __init__(self, st: ViewState):
        self.keys = torch.empty(st.capacity, dtype=torch.int64, device=DEV)
        self.vals = torch.empty(st.capacity, dtype=torch.int32, device=DEV)
        self.ranges = torch.empty((st.num_tiles, 2), dtype=torch.int32, device=DEV)
        self.order = torch.empty(max(st.num_tiles, 1), dtype=torch.int32, device=DEV)
        self.d_count = torch.zeros(4, dtype=torch.int32, device=DEV)
        self.blocks = torch.empty(st.capacity, dtype=torch.int16, device=DEV)
        self.c = B.ts_bins(self.keys.data_ptr(), self.vals.data_ptr(), self.ranges.data_ptr(),
                           self.d_count.data_ptr(), st.capacity, self.order.data_ptr(),
                           self.blocks.data_ptr(), st.bins.flags)


def _bin_both(scene, cam, cfg, sync):
    sct = scene_to_device(scene, DEV)
    st = ViewState(scene.n, cam.width, cam.height, max(4 * scene.n, 1 << 16), device=DEV,
                   keys=True)
    ras = Rasterizer(cfg, device=DEV)
    ccam = ras.project(st, sct, cam)
    ras.bin_sort(st, ccam, sync=True)            # sizes the lists, reference result
    other = _Bins(st)
    stream = torch.cuda.current_stream().cuda_stream
    hc = (ctypes.c_uint32 * 2)() if sync else None
    B.ts_bin_sort_noalloc(st.proj, st.N, ccam, other.c, hc, stream)
    torch.cuda.synchronize()
    M = st.M
    if sync:
        assert (hc[0], hc[1]) == (st.M, st.N_v)
    dc_ref = st.d_count.cpu().numpy()
    dc = other.d_count.cpu().numpy()
    np.testing.assert_array_equal(dc, dc_ref)
    np.testing.assert_array_equal(other.keys[:M].cpu().numpy(), st.keys[:M].cpu().numpy())
    np.testing.assert_array_equal(other.vals[:M].cpu().numpy(), st.vals[:M].cpu().numpy())
    np.testing.assert_array_equal(other.ranges.cpu().numpy(), st.ranges.cpu().numpy())
    # the raster order ranks tiles by list length; tiles of equal length may
    # come in any order: check it is a permutation by non-increasing length
    order = other.order.cpu().numpy()[: st.num_tiles].astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(st.num_tiles))
    r = st.ranges.cpu().numpy().astype(np.int64)
    lens = np.minimum(r[:, 1] - r[:, 0], 2047)
    assert np.all(np.diff(lens[order]) <= 0)
    return M


def test_noalloc_bin_sort_matches_workspace_form_twice():
    mid = synth.workload_mid()
    M1 = _bin_both(mid.scene, mid.cameras[0], mid.config, sync=False)
    small = synth.workload_small()
    M2 = _bin_both(small.scene, small.cameras[0], small.config, sync=True)
    assert M2 < M1
    print("noalloc bins", M1, M2)


def test_noalloc_rejects_oversized_lists():
    small = synth.workload_small()
    st = ViewState(small.scene.n, 128, 128, 1 << 16, device=DEV)
    big = B.ts_bins(1, 1, 1, 1, 1 << 30, 1, 1, 0)       # 1G instances: never fits
    with pytest.raises(B.TSError) as e:
        B.ts_bin_sort_noalloc(st.proj, st.N, B.make_camera(small.cameras[0]), big, None, 0)
    assert e.value.code == B.TS_EWORKSPACE
    assert "fixed scratch" in str(e.value)
