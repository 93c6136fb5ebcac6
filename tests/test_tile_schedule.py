"""Host logic of the FFT tile schedule (no GPU): the shapes of the four tile
variants (workgroup shape x transform plan) at every supported length, the
process-wide table, and its text file (save, load, rejection of malformed
files)."""
import os

import pytest

import paper_1210_2258_amd as m

SIZES = [16, 32, 64, 128, 256, 512, 1024, 2048, 80, 160, 320, 640, 1280]


@pytest.fixture(autouse=True)
def _restore_defaults():
    yield
    for L in SIZES:
        m.set_tile_schedule(L, 0, 0)


def _points(L, v):
    return L * v["row_pairs"] // v["row_threads"]


@pytest.mark.parametrize("L", SIZES)
def test_variant_shapes(L):
    vs = [m.tile_info(L, k) for k in range(4)]
    for v in vs:
        # rows: 2 RP rows per workgroup inside the 8-row block of the spectrum layout
        assert v["row_pairs"] in (1, 2, 4) and v["row_threads"] % v["row_pairs"] == 0
        assert v["row_threads"] <= 1024 and v["col_threads"] <= (1024 if v["col_width"] <= 2 else 512)
        # columns: the LDS tile of C columns stays within 40 KB unless one column exceeds it
        assert v["col_width"] == 1 or v["col_width"] * L * 8 <= 40960
        assert v["col_threads"] % v["col_width"] == 0
        # whole transforms per workgroup, and a multiple of the wavefront
        assert v["row_threads"] % 64 == 0 or v["row_threads"] < 64
        assert L % _points(L, v) == 0
    for v0, v1 in ((vs[0], vs[1]), (vs[2], vs[3])):
        # one FFT's thread count is the same under both shapes of a plan
        assert v0["row_threads"] // v0["row_pairs"] == v1["row_threads"] // v1["row_pairs"]
        assert v0["col_threads"] // v0["col_width"] == v1["col_threads"] // v1["col_width"]
    # variant 1: half the row pairs, or the same shape where that would not fill a wavefront
    if v1["row_pairs"] != v0["row_pairs"]:
        assert v1["row_pairs"] * 2 == v0["row_pairs"] and v1["row_threads"] >= 64
    assert v1["col_width"] in (2 * v0["col_width"], v0["col_width"] // 2, v0["col_width"])
    if v1["col_width"] != v0["col_width"]:
        assert v1["col_threads"] >= 64


def test_variant_one_differs_where_expected():
    # 2048: 512-thread row workgroups (2 row pairs) and 2-column workgroups
    assert m.tile_info(2048, 0) == dict(row_threads=1024, row_pairs=4, col_threads=256, col_width=1)
    assert m.tile_info(2048, 1) == dict(row_threads=512, row_pairs=2, col_threads=512, col_width=2)
    # 1280: four points per thread, 320 threads per transform; one column per
    # workgroup, two in variant 1 (640 threads); two row pairs, one in variant 1
    assert m.tile_info(1280, 0) == dict(row_threads=640, row_pairs=2, col_threads=320, col_width=1)
    assert m.tile_info(1280, 1) == dict(row_threads=320, row_pairs=1, col_threads=640, col_width=2)
    # no second plan at 1280: variants 2 and 3 run plan 0
    assert m.tile_info(1280, 2) == m.tile_info(1280, 0) and m.tile_info(1280, 3) == m.tile_info(1280, 1)


@pytest.mark.parametrize("L,p0,p1", [(128, 4, 8), (256, 4, 8), (512, 4, 8), (1024, 4, 8), (2048, 8, 8),
                                     (1280, 4, 4)])
def test_transform_plans(L, p0, p1):
    """Plan 0 and plan 1 (tile variants 0/1 and 2/3) take the documented
    points per thread."""
    assert _points(L, m.tile_info(L, 0)) == _points(L, m.tile_info(L, 1)) == p0
    assert _points(L, m.tile_info(L, 2)) == _points(L, m.tile_info(L, 3)) == p1


def test_unsupported_length_and_variant():
    with pytest.raises(m.SgpError):
        m.tile_info(100, 0)
    with pytest.raises(m.SgpError):
        m.tile_info(256, 4)
    with pytest.raises(m.SgpError):
        m.tile_info(256, -1)
    with pytest.raises(m.SgpError):
        m.set_tile_schedule(96, 0, 0)
    with pytest.raises(m.SgpError):
        m.set_tile_schedule(256, 0, 4)
    assert m.get_tile_schedule(256) == (0, 0)


def test_table_and_file_round_trip(tmp_path):
    assert m.get_tile_schedule(512) == (0, 0)  # default
    m.set_tile_schedule(512, 1, 0)
    m.set_tile_schedule(1280, 0, 1)
    m.set_tile_schedule(2048, 3, 2)
    assert m.get_tile_schedule(512) == (1, 0) and m.get_tile_schedule(1280) == (0, 1)
    path = tmp_path / "tiles.txt"
    m.save_tile_schedule(str(path))
    lines = path.read_text().splitlines()
    assert lines[0].startswith("#")
    assert "512 1 0" in lines and "1280 0 1" in lines and "2048 3 2" in lines
    m.set_tile_schedule(512, 0, 0)
    m.set_tile_schedule(1280, 0, 0)
    m.set_tile_schedule(2048, 0, 0)
    m.load_tile_schedule(str(path))
    assert m.get_tile_schedule(512) == (1, 0) and m.get_tile_schedule(1280) == (0, 1)
    assert m.get_tile_schedule(2048) == (3, 2)


@pytest.mark.parametrize("bad", ["256 1\n", "256 1 4\n", "100 0 0\n", "256 0 1 7\n", "x y z\n"])
def test_malformed_file_applies_nothing(tmp_path, bad):
    path = tmp_path / "tiles.txt"
    path.write_text("# schedule\n64 1 1\n" + bad)
    with pytest.raises(m.SgpError, match=":3:"):
        m.load_tile_schedule(str(path))
    assert m.get_tile_schedule(64) == (0, 0)


def test_missing_file():
    with pytest.raises(m.SgpError):
        m.load_tile_schedule(os.path.join("/nonexistent", "tiles.txt"))


def test_autotune_argument_checks_before_any_device_work():
    """The autotuner rejects a null problem, an iteration count out of range
    and an unsupported FFT size before touching a device, and leaves the
    table as it was."""
    import ctypes

    from paper_1210_2258_amd import _lib as L
    lib = m.load()
    m.set_tile_schedule(256, 1, 0)
    dummy = ctypes.c_void_p(1)  # never dereferenced: every call below fails its checks first

    def run(ny, nx, iters, prob=True):
        pr = L._Problem(dummy.value, dummy.value, None, dummy.value, 1, ny, nx, ny, nx, 0, 0, 0)
        return lib.sgp_autotune(ctypes.byref(pr) if prob else None, dummy if prob else None, iters,
                                None, None, None, None)

    assert run(256, 256, 10, prob=False) == -1
    assert run(256, 256, 0) == -1 and run(256, 256, 100001) == -1
    assert run(96, 256, 10) == -2
    assert m.get_tile_schedule(256) == (1, 0)
