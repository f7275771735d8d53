"""The C ABI without a GPU: libts.so loads, exports every function that
include/ts.h declares, the Python binding covers them all, and the ctypes
struct layouts equal the header's (measured by compiling a C probe)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2505_19175_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ts.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ts_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_hot_path_calls():
    fns = declared_functions()
    for name in ("ts_project", "ts_bin_sort", "ts_render_forward", "ts_render_backward"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    L = B.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(B.EXPORTS) == declared_functions()


def test_host_only_queries():
    assert B.ts_proj_record_bytes() == 128
    assert B.ts_num_tiles(1280, 720) == 80 * 45
    assert B.ts_num_tiles(1600, 1040) == 100 * 65
    assert B.ts_num_tiles(17, 1) == 2
    a = B.ts_bin_sort_workspace_bytes(1000, 5000, 64)
    b = B.ts_bin_sort_workspace_bytes(1000, 50000, 64)
    assert 0 < a < b
    assert B.ts_error_string(B.TS_ECAPACITY) == "instance count exceeds capacity"


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "ts.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F))
int main(void) {
  printf("ts_camera %zu\n", sizeof(ts_camera)); P(ts_camera, t); P(ts_camera, fx); P(ts_camera, width);
  printf("ts_config %zu\n", sizeof(ts_config)); P(ts_config, sh_degree); P(ts_config, bg); P(ts_config, window);
  printf("ts_proj %zu\n", sizeof(ts_proj)); P(ts_proj, g2d); P(ts_proj, cgrad);
  printf("ts_bins %zu\n", sizeof(ts_bins)); P(ts_bins, d_count); P(ts_bins, capacity); P(ts_bins, order); P(ts_bins, blocks); P(ts_bins, flags);
  printf("ts_prune_stats %zu\n", sizeof(ts_prune_stats)); P(ts_prune_stats, pixels);
  printf("ts_view %zu\n", sizeof(ts_view)); P(ts_view, tile_offset); P(ts_view, tiles_x); P(ts_view, pixel_offset);
  return 0;
}
"""


def test_struct_layouts_match_header():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write(PROBE)
        subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                               "-I", "/opt/rocm/include", src, "-o", exe])
        lines = subprocess.check_output([exe], text=True).split("\n")
    got = dict(l.split() for l in lines if l)
    ct = {"ts_camera": B.ts_camera, "ts_config": B.ts_config, "ts_proj": B.ts_proj,
          "ts_bins": B.ts_bins, "ts_view": B.ts_view, "ts_prune_stats": B.ts_prune_stats}
    for k, v in got.items():
        if "." in k:
            s, f = k.split(".")
            assert getattr(ct[s], f).offset == int(v), k
        else:
            assert ctypes.sizeof(ct[k]) == int(v), k


def test_argument_checks_need_no_gpu():
    """Validation errors of the training-side entry points return before any
    HIP call: TS_EINVAL / TS_EWORKSPACE on the host alone."""
    # the allocation-free binning call refuses lists its fixed scratch cannot hold
    from paper_2505_19175_amd import synth as _s
    big = B.ts_bins(1, 1, 1, 1, 1 << 30, 1, 1, 0)
    with pytest.raises(B.TSError) as e:
        B.ts_bin_sort_noalloc(B.ts_proj(16, 16, 16, 16, 16, 16), 1000,
                              B.make_camera(_s.identity_camera(128, 128)), big)
    assert e.value.code == B.TS_EWORKSPACE and "fixed scratch" in str(e.value)
    assert B.ts_bin_sort_workspace_bytes(3_000_000, 2_500_000, 3600) <= B.TS_NOALLOC_SCRATCH_BYTES
    assert B.ts_densify_workspace_bytes(10) < B.ts_densify_workspace_bytes(10_000)
    assert B.ts_image_loss_workspace_bytes(0, 5) == 0
    assert B.ts_image_loss_workspace_bytes(64, 48) < B.ts_image_loss_workspace_bytes(128, 96)
    with pytest.raises(B.TSError) as e:
        B.ts_densify_select(None, None, -1, B.TS_DENSIFY_OPACITY, 1.0, None, None, None, 0)
    assert e.value.code == B.TS_EINVAL
    with pytest.raises(B.TSError) as e:
        B.ts_densify_select(None, None, 5, 7, 1.0, None, None, None, 0)
    assert e.value.code == B.TS_EINVAL
    with pytest.raises(B.TSError) as e:
        B.ts_densify_select(1, 1, 5, B.TS_DENSIFY_INV_SIGMA, float("nan"), 1, 1, 1, 1 << 20)
    assert e.value.code == B.TS_EINVAL
    with pytest.raises(B.TSError) as e:
        B.ts_densify_select(1, 1, 5000, B.TS_DENSIFY_OPACITY, 1.0, 1, 1, 1, 8)
    assert e.value.code == B.TS_EWORKSPACE
    with pytest.raises(B.TSError) as e:
        B.ts_densify_subdivide(1, 1, 1, 1, 3, 10, 5, 1, 1, 1 << 20, 1)
    assert e.value.code == B.TS_EINVAL                        # capacity below N
    with pytest.raises(B.TSError) as e:
        B.ts_image_loss(1, 1, 0, 8, 0.2, 1, None, 1, 1 << 20)
    assert e.value.code == B.TS_EINVAL
    with pytest.raises(B.TSError) as e:
        B.ts_image_loss(1, 1, 8, 8, 1.5, 1, None, 1, 1 << 20)
    assert e.value.code == B.TS_EINVAL
    with pytest.raises(B.TSError) as e:
        B.ts_image_loss(1, 1, 64, 64, 0.2, 1, None, 1, 16)
    assert e.value.code == B.TS_EWORKSPACE
    st = B.ts_adam_state(*([1] * 8))
    with pytest.raises(B.TSError) as e:
        B.ts_optimizer_step(1, 1, 1, 1, 1, 1, 3, 10, 1, 1, 1, 1, st, B.ts_optimizer(step=0))
    assert e.value.code == B.TS_EINVAL
    with pytest.raises(B.TSError) as e:
        B.ts_optimizer_step(1, 1, 1, 1, 1, 1, 4, 10, 1, 1, 1, 1, st, B.ts_optimizer(step=1))
    assert e.value.code == B.TS_EINVAL
    # the fused backward projection + optimizer: bad step, bad config, null
    # parameter, null projection state
    from paper_2505_19175_amd import synth
    cam = B.make_camera(synth.identity_camera(32, 32))
    cfg = B.make_config(synth.Config(sh_degree=1))
    proj = B.ts_proj(16, 16, 16, 16, 16)
    for kw, args in ((dict(step=0), (1, 1, 1, 1, 1, 1, 10, proj, cam, cfg)),
                     (dict(step=1), (1, 1, 1, 1, 1, 1, 10, proj, cam,
                                     B.make_config(synth.Config(sh_degree=7)))),
                     (dict(step=1), (1, None, 1, 1, 1, 1, 10, proj, cam, cfg)),
                     (dict(step=1), (1, 1, 1, 1, 1, 1, 10, B.ts_proj(), cam, cfg))):
        with pytest.raises(B.TSError) as e:
            B.ts_project_backward_adam(*args, st, B.ts_optimizer(**kw))
        assert e.value.code == B.TS_EINVAL
