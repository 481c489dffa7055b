"""The C ABI without a GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "voronoi_rt.h")
DIAG_HEADER = os.path.join(ROOT, "include", "voronoi_rt_diag.h")


def _declared(headers=(HEADER, DIAG_HEADER)):
    names = set()
    for h in headers:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(vor_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1310_1854_amd import vrt
    if not os.path.exists(vrt.LIB_PATH):
        from paper_1310_1854_amd import build_lib
        build_lib.build()
    return vrt.load()


def test_header_declares_the_boundary():
    names = _declared((HEADER,))
    assert "vor_grid_truncate_row" not in names   # the diagnostic hook lives in voronoi_rt_diag.h
    for n in ["vor_build_grid", "vor_locate", "vor_trace", "vor_grid_free", "vor_grid_neighbors",
              "vor_grid_get_info", "vor_exclusive_scan", "vor_status_str", "vor_version"]:
        assert n in names


def test_binding_constants_match_the_header():
    from paper_1310_1854_amd import vrt
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define (VOR_\w+) (\d+)", text))
    assert int(defs["VOR_SPILL_CHUNK"]) == vrt.SPILL_CHUNK
    assert int(defs["VOR_WORK_WORDS"]) == vrt.WORK_WORDS
    assert int(re.search(r"#define VOR_SERVE_GRID_DENSITY (0x[0-9a-fA-F]+)", text).group(1), 16) == vrt.SERVE_GRID_DENSITY
    import torch
    assert vrt.TraceBuffers(10, device="cpu").work.numel() == vrt.WORK_WORDS
    enum = re.search(r"enum \{ VOR_RECORDS_AUTO = (\d+), VOR_RECORDS_FP32 = (\d+), VOR_RECORDS_COMPACT = (\d+) \}", text)
    assert [int(x) for x in enum.groups()] == [vrt.RECORD_LAYOUTS[k] for k in ("auto", "fp32", "compact")]
    # the option and info structs end with the record layout, as in the header
    assert vrt.BuildOpts.record_layout.offset == 24 and ctypes.sizeof(vrt.BuildOpts) == 32
    assert vrt.GridInfo.record_layout.offset == ctypes.sizeof(vrt.GridInfo) - 8


def test_library_exports_every_declared_symbol(lib):
    from paper_1310_1854_amd import vrt
    names = _declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert sorted(vrt.EXPORTS) == names


def test_status_strings(lib):
    from paper_1310_1854_amd import vrt
    for code in range(8):
        assert len(vrt.status_str(code)) >= 2
    assert vrt.status_str(99) == "unknown status"
    assert "gfx950" in vrt.version()


def test_argument_errors_before_device_work(lib):
    from paper_1310_1854_amd import vrt
    box = (ctypes.c_double * 6)(-1, -1, -1, 1, 1, 1)
    fake = (ctypes.c_double * 30)()
    out = ctypes.c_void_p(1234)
    # no sites
    assert lib.vor_build_grid(None, 10, box, None, None, None, ctypes.byref(out)) == vrt.VOR_EINVAL
    assert out.value is None
    # no sites count
    assert lib.vor_build_grid(fake, 0, box, None, None, None, ctypes.byref(out)) == vrt.VOR_EINVAL
    assert lib.vor_build_grid(fake, -5, box, None, None, None, ctypes.byref(out)) == vrt.VOR_EINVAL
    # empty or inverted box, non-finite box
    for b in [(0, -1, -1, 0, 1, 1), (1, -1, -1, -1, 1, 1), (float("nan"), -1, -1, 1, 1, 1),
              (-1, -1, -1, float("inf"), 1, 1)]:
        bb = (ctypes.c_double * 6)(*b)
        assert lib.vor_build_grid(fake, 10, bb, None, None, None, ctypes.byref(out)) == vrt.VOR_EINVAL
    # no box, no out
    assert lib.vor_build_grid(fake, 10, None, None, None, None, ctypes.byref(out)) == vrt.VOR_EINVAL
    assert lib.vor_build_grid(fake, 10, box, None, None, None, None) == vrt.VOR_EINVAL
    # bad options of the block-list locate structure
    for bl, bo in [(2, 0.0), (-1, 0.0), (1, -1.0), (1, float("nan"))]:
        opts = vrt.BuildOpts(0.0, bl, bo)
        assert lib.vor_build_grid(fake, 10, box, ctypes.byref(opts), None, None, ctypes.byref(out)) == vrt.VOR_EINVAL
    for layout in (-1, 3):   # record layouts: auto, fp32, compact
        opts = vrt.BuildOpts(0.0, 0, 0.0, layout)
        assert lib.vor_build_grid(fake, 10, box, ctypes.byref(opts), None, None, ctypes.byref(out)) == vrt.VOR_EINVAL
    # an allocator without its functions
    bad = vrt.Allocator()
    assert lib.vor_build_grid(fake, 10, box, None, ctypes.byref(bad), None, ctypes.byref(out)) == vrt.VOR_EINVAL
    # calls on a missing grid
    cell = (ctypes.c_int32 * 10)()
    assert lib.vor_locate(None, fake, 10, cell, None) == vrt.VOR_EINVAL
    assert lib.vor_locate_blocks(None, fake, 10, cell, None) == vrt.VOR_EINVAL
    assert lib.vor_grid_bboxes(None, fake, None) == vrt.VOR_EINVAL
    assert lib.vor_grid_bind_density(None, fake, None) == vrt.VOR_EINVAL
    assert lib.vor_grid_bind_density(None, None, None) == vrt.VOR_EINVAL
    o = vrt.TraceOut()
    assert lib.vor_trace(None, fake, fake, 10, None, 1.0, None, ctypes.byref(o), None) == vrt.VOR_EINVAL
    info = vrt.GridInfo()
    assert lib.vor_grid_get_info(None, ctypes.byref(info)) == vrt.VOR_EINVAL
    assert lib.vor_grid_neighbors(None, fake, cell, None) == vrt.VOR_EINVAL
    g = lib.vor_gather_paths
    assert g(fake, 10, fake, fake, 0, None, None, None, None, fake, fake, fake, None) == vrt.VOR_EINVAL   # stride 0
    assert g(fake, -1, fake, fake, 8, None, None, None, None, fake, fake, fake, None) == vrt.VOR_EINVAL
    assert g(fake, 10, fake, fake, 8, fake, None, None, None, fake, fake, fake, None) == vrt.VOR_EINVAL   # part of a spill
    assert g(fake, 10, None, fake, 8, None, None, None, None, fake, fake, fake, None) == vrt.VOR_EINVAL
    assert g(fake, 10, fake, fake, 8, None, None, None, None, None, fake, fake, None) == vrt.VOR_EINVAL
    assert g(None, 0, None, None, 8, None, None, None, None, None, None, None, None) == vrt.VOR_OK       # nothing to do
    assert lib.vor_exclusive_scan(cell, -1, fake, None) == vrt.VOR_EINVAL
    assert lib.vor_exclusive_scan(None, 5, fake, None) == vrt.VOR_EINVAL
    lib.vor_grid_free(None)


def test_oracle_and_product_share_no_code():
    """The oracle (test infrastructure) and the HIP path neither include nor
    import each other."""
    csrc = os.path.join(ROOT, "paper_1310_1854_amd", "csrc")
    for f in os.listdir(csrc):
        if f.endswith((".hip", ".h", ".cpp")):
            text = open(os.path.join(csrc, f)).read()
            assert "oracle" not in text.lower(), f
    for f in ("vrt.py", "build_lib.py", "workloads.py", "__init__.py"):
        text = open(os.path.join(ROOT, "paper_1310_1854_amd", f)).read()
        assert "import oracle" not in text and "from oracle" not in text, f
    otext = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert "voronoi_rt" not in otext and "vrt_" not in otext
    for f in ("__init__.py", "exact.py", "dda.py"):
        text = open(os.path.join(ROOT, "oracle", f)).read()
        assert "paper_1310_1854_amd" not in text, f


def test_server_argument_errors_before_device_work(lib):
    from paper_1310_1854_amd import vrt
    out = ctypes.c_void_p(77)
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.vor_server_create(None, 1, 1 << 20, ctypes.byref(out)) == vrt.VOR_EINVAL
    assert out.value is None
    assert lib.vor_server_create(arr, 1, 1 << 20, ctypes.byref(out)) == vrt.VOR_EINVAL
    assert lib.vor_server_create(arr, 0, 1 << 20, ctypes.byref(out)) == vrt.VOR_EINVAL
    rid = ctypes.c_int64(5)
    fake = (ctypes.c_double * 30)()
    assert lib.vor_server_submit(None, 0, fake, fake, 10, None, 1.0, 0, 0, 0, None, ctypes.byref(rid)) == vrt.VOR_EINVAL
    assert rid.value == 0
    assert lib.vor_server_copy_result(None, 1, None, None, None, None, None, None, None) == vrt.VOR_EINVAL
    done = ctypes.c_int32()
    assert lib.vor_server_poll(None, 1, ctypes.byref(done)) == vrt.VOR_EINVAL
    assert lib.vor_server_wait(None, 1, 0.1) == vrt.VOR_EINVAL
    assert lib.vor_server_release(None, 1) == vrt.VOR_EINVAL
    st = vrt.ServerStats()
    assert lib.vor_server_get_stats(None, ctypes.byref(st)) == vrt.VOR_EINVAL
    lib.vor_server_destroy(None)
