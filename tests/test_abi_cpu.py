"""Host-side checks of the C ABI: the library loads, exports what include/isogs.h
declares, and rejects invalid arguments before touching a device. No GPU needed."""
import ctypes
import subprocess
import sys
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isogs.h")


def _abi():
    from paper_2403_14244_amd import _abi as A
    if not os.path.exists(A.LIB_PATH):
        pytest.skip("libisogs.so not built (run python paper_2403_14244_amd/build.py)")
    return A


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(isogs_\w+)\s*\(", text, re.M)))


def test_header_declares_the_four_pipeline_calls():
    fns = header_functions()
    for name in ("isogs_project", "isogs_bin_sort", "isogs_render_fwd", "isogs_render_bwd", "isogs_last_error"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    A = _abi()
    L = ctypes.CDLL(A.LIB_PATH)
    for name in header_functions():
        assert hasattr(L, name), name
    assert set(header_functions()) <= set(A.EXPORTED)


def test_header_constants_match_the_oracle():
    """The method constants stated in the header and in the oracle agree (they are
    written independently in both places)."""
    import oracle as O
    text = open(HEADER).read()
    val = lambda name: float(re.search(rf"#define {name} \(?([-0-9.e]+)f?\)?", text).group(1))
    assert val("ISOGS_TILE") == O.TILE
    assert 1.0 / val("ISOGS_ALPHA_MIN_INV") == O.ALPHA_MIN
    assert val("ISOGS_ALPHA_MAX") == O.ALPHA_MAX
    assert val("ISOGS_T_MIN") == O.T_MIN


def test_struct_layouts_match_header(tmp_path):
    A = _abi()
    assert ctypes.sizeof(A.Camera) == 4 * (9 + 3 + 3 + 4) + 8
    assert ctypes.sizeof(A.Scene) == 4 * 8 + 8
    assert ctypes.sizeof(A.Projected) == 3 * 8
    assert ctypes.sizeof(A.Bins) == 7 * 8
    assert A.Bins.capacity.offset == 32
    # sizes and field offsets as a C compiler lays the header's structs out
    structs = {"isogs_scene": A.Scene, "isogs_camera": A.Camera, "isogs_projected": A.Projected,
               "isogs_bins": A.Bins, "isogs_field2d": A.Field2D, "isogs_aniso_scene": A.AnisoScene,
               "isogs_aniso_projected": A.AnisoProjected, "isogs_octree_grid": A.OctreeGrid,
               "isogs_field2d_aniso": A.Field2DAniso}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, ct in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in ct._fields_:
            cf = "near_z" if fname == "near_z" else fname
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, ct in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(ct), cname
        for fname, _ in ct._fields_:
            assert got[(cname, fname)] == getattr(ct, fname).offset, (cname, fname)


def test_binding_fails_loudly_without_the_library(tmp_path):
    # the package copied without libisogs.so: importing it raises, no fallback path exists
    import shutil
    pkg = tmp_path / "paper_2403_14244_amd"
    pkg.mkdir()
    src = os.path.join(os.path.dirname(HEADER), "..", "paper_2403_14244_amd")
    for f in os.listdir(src):
        if f.endswith(".py"):
            shutil.copy(os.path.join(src, f), pkg / f)
    r = subprocess.run([sys.executable, "-c", "import paper_2403_14244_amd"], cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "libisogs.so is missing" in r.stderr


def _cam(w=64, h=48):
    import scenegen
    return scenegen.look_at_camera((0, 0, 3.0), width=w, height=h)


def test_invalid_arguments_are_rejected_without_a_device():
    A = _abi()
    L = A.lib()
    cams = A.camera_array([_cam()])
    sc = (A.Scene * 1)()
    sc[0].n = 4
    sc[0].sh_degree = 0            # NULL buffers with n > 0
    proj = A.Projected()
    assert L.isogs_project(sc, cams, 1, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID
    assert b"NULL" in L.isogs_last_error()
    assert L.isogs_project(sc, cams, 0, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID
    sc[0].sh_degree = 4
    assert L.isogs_project(sc, cams, 1, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID
    assert b"sh_degree" in L.isogs_last_error()
    sc[0].sh_degree = 0
    sc[0].n = -1
    assert L.isogs_project(sc, cams, 1, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID
    bad = _cam()
    bad.f = -1.0
    assert L.isogs_project(sc, A.camera_array([bad]), 1, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID
    bad = _cam()
    bad.near = 0.0
    assert L.isogs_project(sc, A.camera_array([bad]), 1, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID
    bad = _cam(w=0)
    assert L.isogs_project(sc, A.camera_array([bad]), 1, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID


def test_workspace_query_and_too_small_workspace():
    A = _abi()
    L = A.lib()
    cams = A.camera_array([_cam(64, 48), _cam(33, 17)])
    npv = A.int_array([100, 50])
    bins = A.Bins()
    bins.capacity = 5000
    need = ctypes.c_size_t(0)
    proj = A.Projected()
    assert L.isogs_bin_sort(ctypes.byref(proj), npv, cams, 2, ctypes.byref(bins), None, ctypes.byref(need),
                            None) == A.ISOGS_OK
    # ping-pong keys + values per entry, plus bookkeeping
    assert need.value >= 5000 * 12
    small = ctypes.c_size_t(need.value - 1)
    fake_ws = ctypes.c_void_p(1 << 20)   # never dereferenced: rejected first
    assert L.isogs_bin_sort(ctypes.byref(proj), npv, cams, 2, ctypes.byref(bins), fake_ws, ctypes.byref(small),
                            None) == A.ISOGS_ERR_WORKSPACE
    bins.capacity = 1 << 31
    assert L.isogs_bin_sort(ctypes.byref(proj), npv, cams, 2, ctypes.byref(bins), fake_ws, ctypes.byref(need),
                            None) in (A.ISOGS_ERR_INVALID, A.ISOGS_ERR_WORKSPACE)
    # render_bwd workspace: 32 bytes per entry
    bins.capacity = 1000
    sc = (A.Scene * 1)()
    gs = (A.Scene * 1)()
    assert L.isogs_render_bwd(sc, cams, 1, ctypes.byref(proj), ctypes.byref(bins), None, None, None, None, None,
                              None, gs, None, ctypes.byref(need), None) == A.ISOGS_OK
    assert need.value >= 32 * 1000


def test_negative_view_particle_counts_rejected():
    A = _abi()
    L = A.lib()
    cams = A.camera_array([_cam()])
    bins = A.Bins()
    need = ctypes.c_size_t(0)
    proj = A.Projected()
    assert L.isogs_bin_sort(ctypes.byref(proj), A.int_array([-3]), cams, 1, ctypes.byref(bins), None,
                            ctypes.byref(need), None) == A.ISOGS_ERR_INVALID


def test_ordered_forward_rejects_unknown_flags():
    """Every argument is well formed except ``flags``: the call must fail before any launch."""
    A = _abi()
    L = A.lib()
    cams = A.camera_array([_cam(64, 48)])
    npv = A.int_array([10])
    fake = 1 << 20                      # 256-byte aligned addresses that are never dereferenced
    proj = A.Projected(fake, fake, fake)
    bins = A.Bins(fake, fake, fake, fake, 100, fake, fake)
    bg = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    need = ctypes.c_size_t(0)
    assert L.isogs_render_fwd_ordered(ctypes.byref(proj), npv, ctypes.byref(bins), cams, 1, bg, None, None,
                                      None, None, 0, None, ctypes.byref(need), None) == A.ISOGS_OK
    # the stamps of ISOGS_FWD_TIMES: 80 bytes per tile more (64x48: 12 tiles)
    need_t = ctypes.c_size_t(0)
    assert L.isogs_render_fwd_ordered(ctypes.byref(proj), npv, ctypes.byref(bins), cams, 1, bg, None, None,
                                      None, None, A.ISOGS_FWD_TIMES, None, ctypes.byref(need_t), None) == A.ISOGS_OK
    assert need_t.value == need.value + 12 * 80
    out = ctypes.c_void_p(fake)
    for flags in (4, 1 << 31, A.ISOGS_FWD_WIDE | 4, A.ISOGS_FWD_TIMES | 8):
        assert L.isogs_render_fwd_ordered(ctypes.byref(proj), npv, ctypes.byref(bins), cams, 1, bg, out, out,
                                          out, None, flags, ctypes.c_void_p(fake), ctypes.byref(need),
                                          None) == A.ISOGS_ERR_INVALID
        assert b"flags" in L.isogs_last_error()


def test_field2d_invalid_arguments_and_workspace_query():
    A = _abi()
    L = A.lib()
    f = A.Field2D()
    f.K = 10
    proj = A.Projected()
    bins = A.Bins()
    bins.capacity = 1000
    need = ctypes.c_size_t(0)
    # NULL parameter arrays are only checked once a workspace is given; the query works
    assert L.isogs_field2d_bin(ctypes.byref(f), 64, 48, 5.0, ctypes.byref(proj), ctypes.byref(bins), None,
                               ctypes.byref(need), None) == A.ISOGS_OK
    assert need.value >= 1000 * 12
    for w, h, d in ((0, 48, 5.0), (64, -1, 5.0), (64, 48, 0.0), (64, 48, float("nan")), (64, 48, float("inf"))):
        assert L.isogs_field2d_bin(ctypes.byref(f), w, h, d, ctypes.byref(proj), ctypes.byref(bins), None,
                                   ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    f.K = -1
    assert L.isogs_field2d_bin(ctypes.byref(f), 64, 48, 5.0, ctypes.byref(proj), ctypes.byref(bins), None,
                               ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    f.K = 10
    fake = ctypes.c_void_p(1 << 20)
    assert L.isogs_field2d_bin(ctypes.byref(f), 64, 48, 5.0, ctypes.byref(proj), ctypes.byref(bins), fake,
                               ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    assert b"NULL" in L.isogs_last_error()
    # backward workspace: 32 bytes per entry of capacity
    g = A.Field2D()
    g.K = 10
    assert L.isogs_field2d_bwd(ctypes.byref(proj), 10, ctypes.byref(bins), 64, 48, 5.0, None, ctypes.byref(g),
                               None, ctypes.byref(need), None) == A.ISOGS_OK
    assert need.value == 32 * 1000
    assert L.isogs_field2d_fwd(ctypes.byref(proj), 10, ctypes.byref(bins), 64, 48, 5.0, None,
                               None) == A.ISOGS_ERR_INVALID


def test_ssim_invalid_arguments_and_workspace_query():
    A = _abi()
    L = A.lib()
    need = ctypes.c_size_t(0)
    assert L.isogs_ssim_fwd(None, None, 3, 48, 64, None, None, ctypes.byref(need), None) == A.ISOGS_OK
    assert need.value >= 12 * 3 * 48 * 64
    for c, h, w in ((0, 48, 64), (3, 0, 64), (3, 48, -2), (70000, 4, 4)):
        assert L.isogs_ssim_fwd(None, None, c, h, w, None, None, ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    fake = ctypes.c_void_p(1 << 20)
    small = ctypes.c_size_t(16)
    assert L.isogs_ssim_fwd(fake, fake, 3, 48, 64, fake, fake, ctypes.byref(small), None) == A.ISOGS_ERR_WORKSPACE
    assert L.isogs_ssim_bwd(fake, fake, 3, 48, 64, fake, None, 0, fake, None) == A.ISOGS_ERR_WORKSPACE


def test_tree_init_and_edits_invalid_arguments():
    A = _abi()
    L = A.lib()
    need = ctypes.c_size_t(0)
    out = A.Field2D()
    out.K = 100
    assert L.isogs_field2d_tree_init(None, 64, 64, 16, 2, 1e-3, 100, ctypes.byref(out), None, None,
                                     ctypes.byref(need), None) == A.ISOGS_OK and need.value > 0
    for root, ms, tau, K in ((24, 2, 1e-3, 100), (16, 32, 1e-3, 100), (16, 0, 1e-3, 100), (16, 2, -1.0, 100),
                             (16, 2, float("nan"), 100), (16, 2, 1e-3, 15)):
        assert L.isogs_field2d_tree_init(None, 64, 64, root, ms, tau, K, ctypes.byref(out), None, None,
                                         ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    fi = A.Field2D()
    fi.K = -1
    for fn in (L.isogs_field2d_prune, L.isogs_field2d_split):
        assert fn(ctypes.byref(fi), 0.1, ctypes.byref(out), None, None, ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    fi.K = 1000
    assert L.isogs_field2d_split(ctypes.byref(fi), 0.1, ctypes.byref(out), None, None, ctypes.byref(need),
                                 None) == A.ISOGS_OK
    assert need.value >= 4 * 4
    assert L.isogs_field2d_split(ctypes.byref(fi), float("nan"), ctypes.byref(out), None, None, ctypes.byref(need),
                                 None) == A.ISOGS_ERR_INVALID


def test_l1_invalid_arguments_and_workspace_query():
    A = _abi()
    L = A.lib()
    need = ctypes.c_size_t(0)
    assert L.isogs_l1_fwd(None, None, 10_000, None, None, ctypes.byref(need), None) == A.ISOGS_OK
    assert need.value >= 8 * 3
    assert L.isogs_l1_fwd(None, None, -1, None, None, ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    assert L.isogs_l1_bwd(None, None, 5, None, None, None) == A.ISOGS_ERR_INVALID


def test_static_bin_sort_rejects_oversize_and_bad_arguments_without_a_device():
    """isogs_bin_sort_static checks its arguments and the size of its static scratch before
    it looks up the array on a device."""
    A = _abi()
    L = A.lib()
    cams = A.camera_array([_cam(64, 48)])
    npv = A.int_array([100])
    bins = A.Bins()
    proj = A.Projected()
    # the scratch a workspace call would need for this capacity exceeds the static array
    bins.capacity = (A.ISOGS_STATIC_SCRATCH_BYTES // 20) + 1
    need = ctypes.c_size_t(0)
    assert L.isogs_bin_sort(ctypes.byref(proj), npv, cams, 1, ctypes.byref(bins), None, ctypes.byref(need),
                            None) == A.ISOGS_OK
    assert need.value > A.ISOGS_STATIC_SCRATCH_BYTES
    assert L.isogs_bin_sort_static(ctypes.byref(proj), npv, cams, 1, ctypes.byref(bins), None) == A.ISOGS_ERR_WORKSPACE
    assert b"static scratch" in L.isogs_last_error()
    assert L.isogs_bin_sort_static(ctypes.byref(proj), npv, cams, 0, ctypes.byref(bins), None) == A.ISOGS_ERR_INVALID
    assert L.isogs_bin_sort_static(ctypes.byref(proj), None, cams, 1, ctypes.byref(bins), None) == A.ISOGS_ERR_INVALID
    assert L.isogs_bin_sort_static(ctypes.byref(proj), npv, cams, 1, None, None) == A.ISOGS_ERR_INVALID
    # within the limit, NULL buffers are still rejected before any device call
    bins.capacity = 1000
    assert L.isogs_bin_sort_static(ctypes.byref(proj), npv, cams, 1, ctypes.byref(bins), None) == A.ISOGS_ERR_INVALID


def test_header_states_the_static_scratch_size():
    A = _abi()
    text = open(HEADER).read()
    m = re.search(r"#define ISOGS_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and (int(m.group(1)) << int(m.group(2))) == A.ISOGS_STATIC_SCRATCH_BYTES


def test_aniso_invalid_arguments_are_rejected_without_a_device():
    """The anisotropic calls validate like the isotropic ones, before any launch."""
    A = _abi()
    L = A.lib()
    cams = A.camera_array([_cam()])
    sc = (A.AnisoScene * 1)()
    sc[0].n = 4
    sc[0].sh_degree = 0
    proj = A.AnisoProjected()
    assert L.isogs_aniso_project(sc, cams, 1, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID
    assert b"NULL" in L.isogs_last_error()
    sc[0].sh_degree = 5
    assert L.isogs_aniso_project(sc, cams, 1, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID
    assert b"sh_degree" in L.isogs_last_error()
    # buffers given, but the conic misaligned
    sc[0].sh_degree = 0
    for f in ("pos", "rot", "scale", "opacity", "color"):
        setattr(sc[0], f, 4096)
    proj.fp.record, proj.fp.depth, proj.fp.tile_count, proj.conic = 4096, 4096, 4096, 4100
    assert L.isogs_aniso_project(sc, cams, 1, ctypes.byref(proj), None) == A.ISOGS_ERR_INVALID
    assert b"conic" in L.isogs_last_error()
    # workspace queries answer without a device; the backward's records are 48 bytes
    bins = A.Bins()
    bins.capacity = 1000
    need_iso, need_an = ctypes.c_size_t(0), ctypes.c_size_t(0)
    npv = A.int_array([4])
    bg = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    assert L.isogs_aniso_render_fwd(ctypes.byref(proj), npv, ctypes.byref(bins), cams, 1, bg, None, None, None, None,
                                    0, None, ctypes.byref(need_an), None) == A.ISOGS_OK
    assert need_an.value > 0
    iso = (A.Scene * 1)()
    iso[0].n = 4
    assert L.isogs_render_bwd(iso, cams, 1, None, ctypes.byref(bins), bg, None, None, None, None, None, iso, None,
                              ctypes.byref(need_iso), None) == A.ISOGS_OK
    assert L.isogs_aniso_render_bwd(sc, cams, 1, ctypes.byref(proj), ctypes.byref(bins), bg, None, None, None, None,
                                    None, sc, None, ctypes.byref(need_an), None) == A.ISOGS_OK
    assert need_an.value - need_iso.value >= 1000 * 16
    assert L.isogs_aniso_render_fwd(ctypes.byref(proj), npv, ctypes.byref(bins), cams, 1, bg, None, None, None, None,
                                    2, None, ctypes.byref(need_an), None) == A.ISOGS_OK   # query ignores flags


def test_tree_and_loss_calls_validate_without_a_device():
    """Octree initialisation, merge and the combined loss reject bad arguments and answer
    workspace queries before touching a device."""
    A = _abi()
    L = A.lib()
    g = A.OctreeGrid()
    g.lo[:] = [-1.0, -1.0, -1.0]
    g.root_side = 0.5
    g.roots[:] = [4, 4, 4]
    g.levels = 6
    need = ctypes.c_size_t(0)
    out = A.Scene()
    assert L.isogs_octree_init(None, None, 0, ctypes.byref(g), 1e-3, 10, 0.5, ctypes.byref(out), None, None,
                               ctypes.byref(need), None) == A.ISOGS_OK
    cells = sum((4 << l) ** 3 for l in range(6))
    assert need.value >= cells * 58
    g.levels = 13
    assert L.isogs_octree_init(None, None, 0, ctypes.byref(g), 1e-3, 10, 0.5, ctypes.byref(out), None, None,
                               ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    g.levels = 6
    g.root_side = -1.0
    assert L.isogs_octree_init(None, None, 0, ctypes.byref(g), 1e-3, 10, 0.5, ctypes.byref(out), None, None,
                               ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    g.root_side = 0.5
    ws = ctypes.create_string_buffer(need.value + 256)
    aligned = (ctypes.addressof(ws) + 255) & ~255
    have = ctypes.c_size_t(need.value)
    out.n = 5    # capacity below K
    assert L.isogs_octree_init(None, None, 0, ctypes.byref(g), 1e-3, 10, 0.5, ctypes.byref(out), None, aligned,
                               ctypes.byref(have), None) == A.ISOGS_ERR_INVALID
    assert b"K" in L.isogs_last_error()
    fi, fo = A.Field2D(), A.Field2D()
    assert L.isogs_field2d_merge(ctypes.byref(fi), 64, 64, 0.0, 1.0, ctypes.byref(fo), None, None,
                                 ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    assert L.isogs_field2d_merge(ctypes.byref(fi), 64, 64, 4.0, 1.0, ctypes.byref(fo), None, None,
                                 ctypes.byref(need), None) == A.ISOGS_OK
    assert need.value >= 16 * 16 * 56
    assert L.isogs_loss_fwd(None, None, 3, 8, 8, 1.5, None, None, ctypes.byref(need), None) == A.ISOGS_ERR_INVALID
    assert L.isogs_loss_fwd(None, None, 3, 8, 8, 0.2, None, None, ctypes.byref(need), None) == A.ISOGS_OK


def test_stream_calls_reject_null_before_touching_the_device():
    A = _abi()
    L = A.lib()
    assert L.isogs_stream_create(None) == A.ISOGS_ERR_INVALID
    assert b"stream" in L.isogs_last_error()
    assert L.isogs_stream_destroy(None) == A.ISOGS_ERR_INVALID
