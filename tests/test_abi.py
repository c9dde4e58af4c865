"""C ABI contract checks that need no GPU: the library loads, exports every
function declared in include/gesr.h, its struct layouts match the header
(compiled independently with gcc), and invalid arguments are rejected on the
host with GESR_ERR_INVALID / GESR_ERR_UNSUPPORTED before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2411_09156_amd import _lib
from paper_2411_09156_amd.rasterizer import RasterSettings, cameras_to_c

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gesr.h")


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_function(lib):
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(gesr_[a-z0-9_]+)\s*\(", text))
    assert declared == set(_lib.EXPORTS)
    nm = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\b(gesr_[a-z0-9_]+)\b", nm.stdout))
    assert declared <= exported, declared - exported


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "gesr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gesr_camera), sizeof(gesr_settings), sizeof(gesr_splats),
         sizeof(gesr_proj), sizeof(gesr_bins), sizeof(gesr_grads), sizeof(gesr_sizes), sizeof(gesr_fwd_counts));
  printf("%zu %zu %zu %zu\\n", offsetof(gesr_settings, bg), offsetof(gesr_bins, scratch_bytes),
         offsetof(gesr_camera, campos), offsetof(gesr_bins, tile_work));
  return 0;
}
""")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(x) for x in out[0].split()]
    offs = [int(x) for x in out[1].split()]
    mine = [ctypes.sizeof(t) for t in (_lib.Camera, _lib.Settings, _lib.Splats, _lib.Proj, _lib.Bins, _lib.Grads,
                                       _lib.Sizes, _lib.FwdCounts)]
    assert sizes == mine
    assert offs == [_lib.Settings.bg.offset, _lib.Bins.scratch_bytes.offset, _lib.Camera.campos.offset,
                    _lib.Bins.tile_work.offset]


def _ctx(lib):
    ctx = ctypes.c_void_p()
    assert lib.gesr_ctx_create(0, ctypes.byref(ctx)) == _lib.GESR_OK
    return ctx


class _Cam:
    def __init__(self, w=64, h=48):
        self.width, self.height, self.fx, self.fy, self.cx, self.cy = w, h, 50.0, 50.0, w / 2, h / 2
        self.viewmat = [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 4]]
        self.campos = [0, 0, -4]


def test_defaults_match_binding(lib):
    s = _lib.Settings()
    lib.gesr_default_settings(ctypes.byref(s))
    d = RasterSettings()
    assert (s.sh_degree, s.tile_w, s.tile_h, s.batch, s.radix_bits) == (d.sh_degree, d.tile_w, d.tile_h, d.batch,
                                                                         d.radix_bits)
    for k in ("kappa", "rho", "alpha_min", "alpha_max", "t_min", "blur", "znear", "clip_fac"):
        assert getattr(s, k) == pytest.approx(getattr(d, k), rel=1e-7)


def test_query_sizes_host_only(lib):
    ctx = _ctx(lib)
    cams = cameras_to_c([_Cam(64, 48), _Cam(33, 17)])
    st = RasterSettings().to_c()
    out = _lib.Sizes()
    assert lib.gesr_query_sizes(ctx, cams, 2, 100, ctypes.byref(st), 5000, ctypes.byref(out)) == _lib.GESR_OK
    assert out.total_tiles == 4 * 3 + 3 * 2
    assert out.total_pixels == 64 * 48 + 33 * 17
    assert out.bwd_workspace_bytes >= 5000 * 12 * 4 + 5000 // 8 + 200 * 12 * 4
    assert out.bin_scratch_bytes > 0
    lib.gesr_ctx_destroy(ctx)


@pytest.mark.parametrize("field,value,status", [
    ("sh_degree", 4, _lib.GESR_ERR_INVALID),
    ("sh_degree", -1, _lib.GESR_ERR_INVALID),
    ("kappa", 0.0, _lib.GESR_ERR_INVALID),
    ("alpha_min", 0.995, _lib.GESR_ERR_INVALID),
    ("t_min", 0.0, _lib.GESR_ERR_INVALID),
    ("znear", -1.0, _lib.GESR_ERR_INVALID),
    ("radix_bits", 9, _lib.GESR_ERR_INVALID),
    ("tile_w", 24, _lib.GESR_ERR_UNSUPPORTED),
])
def test_invalid_settings_rejected(lib, field, value, status):
    ctx = _ctx(lib)
    cams = cameras_to_c([_Cam()])
    st = RasterSettings().to_c()
    setattr(st, field, value)
    out = _lib.Sizes()
    assert lib.gesr_query_sizes(ctx, cams, 1, 10, ctypes.byref(st), 100, ctypes.byref(out)) == status
    assert len(lib.gesr_last_error(ctx)) > 0
    lib.gesr_ctx_destroy(ctx)


def test_invalid_views_and_sizes_rejected(lib):
    ctx = _ctx(lib)
    st = RasterSettings().to_c()
    out = _lib.Sizes()
    cams = cameras_to_c([_Cam()])
    assert lib.gesr_query_sizes(ctx, cams, 0, 10, ctypes.byref(st), 100, ctypes.byref(out)) == _lib.GESR_ERR_INVALID
    assert lib.gesr_query_sizes(ctx, cams, 1, -5, ctypes.byref(st), 100, ctypes.byref(out)) == _lib.GESR_ERR_INVALID
    assert lib.gesr_query_sizes(ctx, cams, 1, 10, ctypes.byref(st), 0, ctypes.byref(out)) == _lib.GESR_ERR_INVALID
    bad = cameras_to_c([_Cam(0, 10)])
    assert lib.gesr_query_sizes(ctx, bad, 1, 10, ctypes.byref(st), 100, ctypes.byref(out)) == _lib.GESR_ERR_INVALID
    many = cameras_to_c([_Cam()] * (_lib.MAX_VIEWS + 1))
    assert lib.gesr_query_sizes(ctx, many, _lib.MAX_VIEWS + 1, 10, ctypes.byref(st), 100,
                                ctypes.byref(out)) == _lib.GESR_ERR_INVALID
    lib.gesr_ctx_destroy(ctx)


def test_null_and_misaligned_pointers_rejected_before_launch(lib):
    ctx = _ctx(lib)
    st = RasterSettings().to_c()
    cams = cameras_to_c([_Cam()])
    sp = _lib.Splats(10, 0, 0, 0, 0, 0, 0)
    proj = _lib.Proj(0, 0, 0, 0)
    assert lib.gesr_project(ctx, ctypes.byref(sp), cams, 1, ctypes.byref(st), ctypes.byref(proj),
                            None) == _lib.GESR_ERR_INVALID
    assert "NULL" in lib.gesr_last_error(ctx).decode()
    sp = _lib.Splats(10, 16, 32, 48, 64, 80, 8)  # sh misaligned
    assert lib.gesr_project(ctx, ctypes.byref(sp), cams, 1, ctypes.byref(st), ctypes.byref(proj),
                            None) == _lib.GESR_ERR_INVALID
    assert "aligned" in lib.gesr_last_error(ctx).decode()
    # NULL context
    assert lib.gesr_project(None, ctypes.byref(sp), cams, 1, ctypes.byref(st), ctypes.byref(proj),
                            None) == _lib.GESR_ERR_INVALID
    bins = _lib.Bins()
    bins.m_cap = 0
    proj = _lib.Proj(16, 16, 16, 16)
    assert lib.gesr_bin(ctx, ctypes.byref(proj), cams, 1, 10, ctypes.byref(st), ctypes.byref(bins), 0, None,
                        None) == _lib.GESR_ERR_INVALID
    lib.gesr_ctx_destroy(ctx)


def test_status_strings(lib):
    for s in range(5):
        assert len(lib.gesr_status_string(s)) > 0


def test_autotune_candidates_are_valid_settings(lib):
    n = lib.gesr_autotune_candidate(-1, None)
    assert n >= 8
    ctx = _ctx(lib)
    cams = cameras_to_c([_Cam(64, 48), _Cam(33, 17)])
    seen = set()
    for k in range(n):
        st = RasterSettings().to_c()
        assert lib.gesr_autotune_candidate(k, ctypes.byref(st)) == 0
        out = _lib.Sizes()
        assert lib.gesr_query_sizes(ctx, cams, 2, 100, ctypes.byref(st), 5000, ctypes.byref(out)) == _lib.GESR_OK
        seen.add((st.tile_w, st.tile_h, st.variant, st.batch, st.radix_bits))
    assert len(seen) == n
    assert lib.gesr_autotune_candidate(n, ctypes.byref(_lib.Settings())) == -1
    lib.gesr_ctx_destroy(ctx)


def test_autotune_rejects_bad_arguments_on_the_host(lib):
    ctx = _ctx(lib)
    cams = cameras_to_c([_Cam()])
    st = RasterSettings().to_c()
    sp = _lib.Splats(10, 16, 32, 48, 64, 80, 96)
    times = (ctypes.c_float * 4)()
    nt = ctypes.c_int(-1)
    for reps in (0, 101):
        assert lib.gesr_autotune(ctx, ctypes.byref(sp), cams, 1, ctypes.byref(st), reps, times, 4, ctypes.byref(nt),
                                 None) == _lib.GESR_ERR_INVALID
    assert lib.gesr_autotune(ctx, ctypes.byref(sp), cams, 1, None, 3, times, 4, ctypes.byref(nt),
                             None) == _lib.GESR_ERR_INVALID
    # no splats: nothing to time, settings unchanged
    empty = _lib.Splats(0, 0, 0, 0, 0, 0, 0)
    before = (st.tile_w, st.tile_h, st.batch, st.radix_bits, st.variant)
    assert lib.gesr_autotune(ctx, ctypes.byref(empty), cams, 1, ctypes.byref(st), 3, times, 4, ctypes.byref(nt),
                             None) == _lib.GESR_OK
    assert nt.value == 0 and (st.tile_w, st.tile_h, st.batch, st.radix_bits, st.variant) == before
    lib.gesr_ctx_destroy(ctx)


@pytest.mark.parametrize("batch,status", [(16, _lib.GESR_ERR_INVALID), (96, _lib.GESR_ERR_INVALID),
                                          (32, _lib.GESR_OK), (128, _lib.GESR_OK)])
def test_batch_values(lib, batch, status):
    ctx = _ctx(lib)
    cams = cameras_to_c([_Cam()])
    st = RasterSettings().to_c()
    st.batch = batch
    out = _lib.Sizes()
    assert lib.gesr_query_sizes(ctx, cams, 1, 10, ctypes.byref(st), 100, ctypes.byref(out)) == status
    lib.gesr_ctx_destroy(ctx)


def test_adam_structs_and_defaults(lib, tmp_path):
    """gesr_params / gesr_adam_settings layouts against gcc, and the defaults
    against the binding's AdamConfig."""
    from paper_2411_09156_amd.optim import AdamConfig
    src = tmp_path / "adam.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "gesr.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(gesr_params), sizeof(gesr_adam_settings), offsetof(gesr_params, sh),
         offsetof(gesr_adam_settings, step));
  return 0;
}
""")
    exe = tmp_path / "adam"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [ctypes.sizeof(_lib.Params), ctypes.sizeof(_lib.AdamSettings), _lib.Params.sh.offset,
                   _lib.AdamSettings.step.offset]
    s = _lib.AdamSettings()
    lib.gesr_default_adam_settings(ctypes.byref(s))
    d = AdamConfig()
    for f in ("lr_mean", "lr_scale", "lr_quat", "lr_opacity", "lr_beta", "lr_sh_dc", "lr_sh_rest", "beta1", "beta2",
              "eps", "entropy_weight"):
        assert getattr(s, f) == pytest.approx(getattr(d, f), rel=1e-7), f
    assert s.step == 1


def test_adam_step_rejects_bad_arguments_on_the_host(lib):
    ctx = _ctx(lib)
    ok = _lib.Params(10, 1, 16, 32, 48, 64, 80, 96)
    g = _lib.Grads(16, 32, 48, 64, 80, 96)
    st = _lib.AdamSettings()
    lib.gesr_default_adam_settings(ctypes.byref(st))

    def call(p=ok, m=ok, v=ok, s=st, so=16, oo=32):
        return lib.gesr_adam_step(ctx, ctypes.byref(p), ctypes.byref(m), ctypes.byref(v), ctypes.byref(g),
                                  ctypes.byref(s) if s is not None else None, so, oo, None)
    assert call(s=None) == _lib.GESR_ERR_INVALID
    assert call(m=_lib.Params(11, 1, 16, 32, 48, 64, 80, 96)) == _lib.GESR_ERR_INVALID
    assert call(v=_lib.Params(10, 4, 16, 32, 48, 64, 80, 96)) == _lib.GESR_ERR_INVALID
    assert call(p=_lib.Params(10, 17, 16, 32, 48, 64, 80, 96)) == _lib.GESR_ERR_INVALID
    assert call(p=_lib.Params(10, 1, 16, 32, 48, 0, 80, 96)) == _lib.GESR_ERR_INVALID
    assert call(v=_lib.Params(10, 1, 16, 32, 48, 64, 84, 96)) == _lib.GESR_ERR_INVALID
    assert "aligned" in lib.gesr_last_error(ctx).decode()
    assert call(oo=0) == _lib.GESR_ERR_INVALID
    for field, value in (("step", 0), ("beta1", 1.0), ("beta2", -0.1), ("eps", 0.0), ("lr_beta", -1e-3),
                         ("lr_mean", float("nan")), ("entropy_weight", float("inf"))):
        bad = _lib.AdamSettings()
        lib.gesr_default_adam_settings(ctypes.byref(bad))
        setattr(bad, field, value)
        assert call(s=bad) == _lib.GESR_ERR_INVALID, field
    lib.gesr_ctx_destroy(ctx)


def test_prune_and_shape_reset_reject_bad_arguments_on_the_host(lib):
    ctx = _ctx(lib)
    ok = _lib.Params(10, 1, 16, 32, 48, 64, 80, 96)
    ps = _lib.PruneSettings(0.5, 0.5)
    need = lib.gesr_prune_workspace_size(10)
    assert need >= 4 * (32 + 2) and lib.gesr_prune_workspace_size(3_000_000) > need

    def call(p=ok, m=None, v=None, s=ps, om=None, ov=None, nk=16, ws=16, wsb=None):
        r = lambda x: ctypes.byref(x) if x is not None else None  # noqa: E731
        return lib.gesr_prune(ctx, r(p), r(m), r(v), r(s), ctypes.byref(ok), r(om), r(ov), None, None, nk, ws,
                              need if wsb is None else wsb, None)
    assert call(s=None) == _lib.GESR_ERR_INVALID
    assert call(m=ok) == _lib.GESR_ERR_INVALID  # v missing
    assert call(m=ok, v=ok) == _lib.GESR_ERR_INVALID  # moment outputs missing
    assert call(nk=0) == _lib.GESR_ERR_INVALID
    assert call(wsb=need - 1) == _lib.GESR_ERR_INVALID
    assert call(ws=8) == _lib.GESR_ERR_INVALID
    assert call(s=_lib.PruneSettings(1.0, 0.5)) == _lib.GESR_ERR_INVALID
    assert call(s=_lib.PruneSettings(0.5, float("nan"))) == _lib.GESR_ERR_INVALID
    assert call(p=_lib.Params(10, 1, 16, 32, 48, 0, 80, 96)) == _lib.GESR_ERR_INVALID
    assert lib.gesr_shape_reset(ctx, ctypes.byref(ok), None, None, 0.0, None) == _lib.GESR_ERR_INVALID
    assert lib.gesr_shape_reset(ctx, None, None, None, 2.0, None) == _lib.GESR_ERR_INVALID
    assert lib.gesr_shape_reset(ctx, ctypes.byref(_lib.Params(10, 1, 16, 32, 48, 64, 0, 96)), None, None, 2.0,
                                None) == _lib.GESR_ERR_INVALID
    lib.gesr_ctx_destroy(ctx)
