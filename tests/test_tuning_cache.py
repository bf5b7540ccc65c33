"""The autotuner's cache file (el_tuning_save / el_tuning_load /
el_tuning_reset): host-only logic, no GPU needed."""
import pytest

from paper_2308_02467_amd import el

HEADER = "# el autotuner choices v2"


@pytest.fixture(autouse=True)
def fresh():
    el.tuning_reset()
    yield
    el.tuning_reset()


def _write(path, lines):
    path.write_text("\n".join(lines) + "\n")
    return path


def test_load_save_round_trip(tmp_path):
    src = _write(tmp_path / "in.txt", [
        HEADER,
        "gfx950 gemm AB hidden M=16384 N=1024 K=1024 splits=1\t3\t256x256 direct-to-LDS",
        "gfx942 gemm AtBt f32 M=1024 N=128 K=4096 splits=8\t2\t128x64",
        "gfx950 matvec f16 m=224\t1\t2 rows x 8 chunks",
        "",
        # a tuner kind this library does not have: skipped
        "gfx950 lu f64 n=784\t0\t7 tiles",
        # a tile index this library names differently, and one it does not have: skipped
        "gfx950 gemm AB mae M=4096 N=225792 K=1024 splits=1\t1\t128x128",
        "gfx950 gemm AB f32 M=1 N=1 K=1 splits=1\t99\t64x64",
    ])
    assert el.tuning_load(src) == 3
    rep = el.tuning_report()
    assert "gfx950 gemm AB hidden M=16384 N=1024 K=1024 splits=1 -> tile 256x256 direct-to-LDS (from a cache file)" in rep
    assert "gfx942 gemm AtBt f32 M=1024 N=128 K=4096 splits=8 -> tile 128x64 (from a cache file)" in rep
    assert "gfx950 matvec f16 m=224 -> shape 2 rows x 8 chunks (from a cache file)" in rep
    assert "mae" not in rep and "M=1 N=1" not in rep and " lu " not in rep
    out = tmp_path / "out.txt"
    el.tuning_save(out)
    lines = out.read_text().splitlines()
    assert lines[0] == HEADER
    assert sorted(lines[1:]) == sorted([
        "gfx950 gemm AB hidden M=16384 N=1024 K=1024 splits=1\t3\t256x256 direct-to-LDS",
        "gfx942 gemm AtBt f32 M=1024 N=128 K=4096 splits=8\t2\t128x64",
        "gfx950 matvec f16 m=224\t1\t2 rows x 8 chunks"])
    # a second load of the saved file takes the same choices
    el.tuning_reset()
    assert el.tuning_report() == ""
    assert el.tuning_load(out) == 3
    assert el.tuning_report() == rep


@pytest.mark.parametrize("lines", [
    ["# another format", "gfx950 gemm AB f32 M=1 N=1 K=1 splits=1\t0\t128x128"],
    [HEADER, "gfx950 gemm AB f32 M=1 N=1 K=1 splits=1\t0"],
    [HEADER, "gfx950 gemm AB f32 M=1 N=1 K=1 splits=1\tx\t128x128"],
    [HEADER, "\t0\t128x128"],
    [HEADER, "gfx950 gemm AB f32 M=1 N=1 K=1 splits=1\t0\t128x128\textra"],
    [],
])
def test_malformed_file_takes_nothing(tmp_path, lines):
    good = _write(tmp_path / "good.txt", [HEADER, "gfx950 gemm AB f32 M=2 N=2 K=64 splits=1\t0\t128x128"])
    assert el.tuning_load(good) == 1
    before = el.tuning_report()
    bad = tmp_path / "bad.txt"
    bad.write_text("\n".join(lines) + ("\n" if lines else ""))
    with pytest.raises(el.ElError):
        el.tuning_load(bad)
    assert el.tuning_report() == before


def test_unreadable_and_unwritable_paths(tmp_path):
    with pytest.raises(el.ElError):
        el.tuning_load(tmp_path / "missing.txt")
    with pytest.raises(el.ElError):
        el.tuning_save(tmp_path / "no_such_dir" / "x.txt")
    L = el.lib()
    assert L.el_tuning_save(None) != 0
    assert L.el_tuning_load(None, None) != 0
