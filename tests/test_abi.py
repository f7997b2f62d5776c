"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/adop.h, and its host-only queries behave."""
import ctypes as ct
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def A():
    from paper_2110_06635_amd import adop
    if not os.path.exists(adop.LIB_PATH):
        from paper_2110_06635_amd import build
        build.build()
    adop.lib()
    return adop


def declared_functions():
    src = open(os.path.join(ROOT, "include", "adop.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(adop_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported(A):
    names = declared_functions()
    assert len(names) >= 14
    L = A.lib()
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(A.EXPORTS)


def test_struct_sizes(A):
    assert ct.sizeof(A.Camera) == 100
    from oracle import oracle as O
    assert ct.sizeof(O.OracleCamera) == ct.sizeof(A.Camera)


def test_version_and_status(A):
    assert b"gfx950" in A.lib().adop_version()
    assert A.lib().adop_status_string(0) == b"ok"
    assert A.lib().adop_status_string(3) == b"workspace too small"


def _cam(w, h):
    from paper_2110_06635_amd import synth
    return synth.Camera(w, h, 100.0, 100.0, w / 2, h / 2)


def test_views_layout(A):
    cams = [_cam(1920, 1080), _cam(640, 480), _cam(33, 17)]
    total, offs = A.views_layout(cams, 4)
    p = [sum((w >> l) * (h >> l) for l in range(4)) for (w, h) in [(1920, 1080), (640, 480), (33, 17)]]
    assert total == sum(p)
    assert offs[0, 0] == 0 and offs[0, 1] == 1920 * 1080
    assert offs[1, 0] == p[0] and offs[2, 3] == p[0] + p[1] + 33 * 17 + 16 * 8 + 8 * 4
    # 5-layer 1080p pyramid: layer 4 is 120 x 67
    total5, _ = A.views_layout([_cam(1920, 1080)], 5)
    assert total5 == 2_762_040


@pytest.mark.parametrize("w,h,L", [(1, 5, 2), (8, 8, 9), (0, 4, 1), (16, 16, 0), (65537, 2, 1), (4, 65537, 1)])
def test_views_layout_rejects(A, w, h, L):
    with pytest.raises(A.AdopError):
        A.views_layout([_cam(w, h)], L)


def test_views_layout_largest_size(A):
    total, _ = A.views_layout([_cam(65536, 2)], 1)
    assert total == 131072


def test_workspace_bytes(A):
    L = A.lib()
    a = L.adop_workspace_bytes(None, 4, 1, 1000)
    b = L.adop_workspace_bytes(None, 4, 1, 2000)
    assert a > 1000 * 4 * 4 and b > a
    assert L.adop_workspace_bytes(None, 0, 1, 10) == 0
    assert L.adop_workspace_bytes(None, 17, 1, 10) == 0
    assert L.adop_feature_bytes(10, 4, A.BF16) == 80
    assert L.adop_feature_bytes(10, 4, A.F32) == 160


def test_pyramid_layout(A):
    lay = A.pyramid_layout(1920, 1080, 5, 4)
    assert lay["width"] == [1920, 960, 480, 240, 120] and lay["height"] == [1080, 540, 270, 135, 67]
    total, offs = A.views_layout([_cam(1920, 1080)], 5)
    assert lay["pixels"] == total == 2_762_040
    assert lay["pixel_offset"] == list(offs[0])
    assert lay["image_bytes"] == 4 * 4 * total and lay["key_bytes"] == 8 * total and lay["count_bytes"] == 4 * total
    for w, h, L, C in [(1, 5, 2, 4), (8, 8, 9, 1), (16, 16, 2, 0), (16, 16, 2, 17)]:
        with pytest.raises(A.AdopError):
            A.pyramid_layout(w, h, L, C)


def test_scene_bind_layout(A):
    """The single-buffer scene: parts in order x, y, z, feat, orig_index, each
    on a 256-byte boundary inside adop_scene_bytes; binding reads nothing."""
    L = A.lib()
    for n, C, dt in [(1, 1, A.F32), (1000, 4, A.F32), (1000, 3, A.BF16), (12345, 8, A.F16)]:
        nb = L.adop_scene_bytes(n, C, dt)
        base = 1 << 40                      # a 256-aligned address that is never dereferenced
        d = A.SceneDesc()
        assert L.adop_scene_bind(ct.c_void_p(base), n, C, dt, ct.byref(d)) == A.OK
        s = 4 if dt == A.F32 else 2
        ptrs = [d.x, d.y, d.z, d.feat, d.orig_index]
        sizes = [4 * n, 4 * n, 4 * n, s * C * n, 4 * n]
        assert ptrs[0] == base and all(p % 256 == 0 for p in ptrs)
        for k in range(4):
            assert ptrs[k + 1] >= ptrs[k] + sizes[k]
            assert ptrs[k + 1] - (ptrs[k] + sizes[k]) < 256
        assert ptrs[4] + sizes[4] <= base + nb
        assert (d.n, d.channels, d.dtype) == (n, C, dt)
        assert not d.nx and not d.radius and not d.beta
    d = A.SceneDesc()
    assert L.adop_scene_bind(ct.c_void_p((1 << 40) + 16), 10, 4, A.F32, ct.byref(d)) == A.E_INVALID
    assert L.adop_scene_bind(ct.c_void_p(1 << 40), 10, 0, A.F32, ct.byref(d)) == A.E_INVALID
    assert L.adop_scene_bytes(-1, 4, A.F32) == 0 and L.adop_scene_bytes(10, 4, 7) == 0
    # point counts stop at 2^31 - 1: the point kernels number chunks and
    # points in 32 bits, which needs (chunks * chunk size) below 2^32
    assert L.adop_scene_bytes((1 << 31) - 1, 4, A.F32) > 0
    assert L.adop_scene_bytes(1 << 31, 4, A.F32) == 0
    assert L.adop_scene_bind(ct.c_void_p(1 << 40), 1 << 31, 4, A.F32, ct.byref(d)) == A.E_INVALID
