"""CPU checks of the C ABI: the library loads, exports every function that
include/hdof.h declares, its structs have the header's layout, and calls
with invalid arguments fail with HDOF_ERR_INVALID_ARG before touching a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdof.h")


@pytest.fixture(scope="module")
def hd():
    lib = os.path.join(ROOT, "paper_2210_04981_amd", "libhdof.so")
    if not os.path.exists(lib):
        from paper_2210_04981_amd import build
        build.build()
    from paper_2210_04981_amd import hdof
    return hdof


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:hdof_status|void|const char\*)\s+(hdof_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(hd):
    names = declared_functions()
    assert len(names) >= 18
    out = subprocess.run(["nm", "-D", "--defined-only", hd.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(hd.EXPORTED) == set(names)


def test_struct_layout_matches_header(hd, tmp_path):
    structs = ["hdof_camera", "hdof_lens", "hdof_light", "hdof_mask_params", "hdof_pp_params",
               "hdof_composite_params", "hdof_frame_params", "hdof_gbuffer_bufs", "hdof_rt_bufs",
               "hdof_frame_bufs", "hdof_scene_info", "hdof_view", "hdof_tuning", "hdof_autotune_report"]
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "hdof.h"\nint main(void){\n' +
                   "".join(f'printf("%zu\\n", sizeof({s}));\n' for s in structs) + "return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    sizes = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    py = [hd.Camera, hd.Lens, hd.Light, hd.MaskParams, hd.PPParams, hd.CompositeParams, hd.FrameParams,
          hd.GBufferBufs, hd.RTBufs, hd.FrameBufs, hd.SceneInfo, hd.View, hd.Tuning, hd.AutotuneReport]
    assert sizes == [C.sizeof(t) for t in py]


def test_status_strings(hd):
    L = hd._lib
    assert L.hdof_status_str(0) == b"HDOF_OK"
    assert L.hdof_status_str(1) == b"HDOF_ERR_INVALID_ARG"
    assert L.hdof_status_str(4) == b"HDOF_ERR_CAPACITY"


def test_null_arguments_rejected(hd):
    L = hd._lib
    INVALID = 1
    cam = hd.camera((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), 0.36, 64, 64)
    lns = hd.lens(0.05, 0.025, 2.0)
    lit = hd.light((0, 1, 0), (1, 1, 1), (0, 0, 0))
    mp, pp, cp = hd.mask_params(), hd.pp_params(), hd.composite_params()
    assert L.hdof_create(0, None) == INVALID
    assert L.hdof_sync(None, None) == INVALID
    assert L.hdof_gbuffer(None, None, C.byref(cam), C.byref(lns), C.byref(lit), hd.GBufferBufs(), None) == INVALID
    assert b"context" in L.hdof_last_error()
    assert L.hdof_postfilter(None, None, None, C.byref(cam), C.byref(lns), C.byref(pp), None, None) == INVALID
    assert L.hdof_composite(None, None, None, None, None, hd.RTBufs(), C.byref(cam), C.byref(lns), C.byref(cp),
                            None, None, None) == INVALID
    assert L.hdof_postfilter_specular(None, None, None, None, None, C.byref(cam), C.byref(lns), C.byref(pp),
                                      None, None, None) == INVALID
    assert L.hdof_scene_set_specular(None, None, None) == INVALID
    assert L.hdof_history_reset(None) == INVALID
    assert L.hdof_postfilter_noalloc(None, None, None, C.byref(cam), C.byref(lns), C.byref(pp), None, None) == INVALID
    fp = hd.FrameParams()
    t = hd.Tuning()
    assert L.hdof_autotune(None, None, C.byref(lit), C.byref(fp), 1, None, None, None, 0, C.byref(t), None,
                           None) == INVALID
    h = C.c_void_p()
    assert L.hdof_build_bvh(None, None, None, 1, C.byref(h), None) == INVALID
    L.hdof_destroy(None)
    L.hdof_scene_destroy(None)


def test_create_without_gpu_is_unsupported(hd):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = hd._lib.hdof_create(0, C.byref(h))
    assert st == 2 and not h.value
