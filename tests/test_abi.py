"""The C-ABI library loads on the CPU host and exports every declared symbol;
host-only queries (no device work) agree with the oracle bit-exactly."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.quadrature import lgl_nodes_weights
from oracle.local import LocalDisc
from oracle.mesh import Mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "el.h")).read()
    return sorted(set(re.findall(r"\b(el_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2308_02467_amd import el
    L = el.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(el.exported_symbols()) == set(names)


@pytest.mark.parametrize("p", [1, 2, 3, 6, 9, 12])
def test_lgl_matches_oracle(p):
    from paper_2308_02467_amd import el
    xi, w = el.lgl(p)
    xo, wo = lgl_nodes_weights(p)
    assert np.abs(xi - xo).max() < 4e-16
    assert np.abs(w - wo).max() < 1e-15


@pytest.mark.parametrize("p,n_a", [(3, 8), (6, 16), (4, 4), (6, 32), (2, 12)])
def test_index_tables_bit_exact(p, n_a):
    from paper_2308_02467_amd import el
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    o = LocalDisc(p, n_a)
    assert (nn, n, m) == (o.nn, o.n, o.m)
    ins, outs = el.index_tables(d)
    assert np.array_equal(ins, o.in_rows)
    assert np.array_equal(outs, o.out_rows)


def test_trace_size_matches_oracle():
    from paper_2308_02467_amd import el
    for (p, n_a, nx, ny) in [(3, 8, 4, 4), (6, 16, 32, 32), (6, 16, 5, 3)]:
        ms = el.mesh(nx, ny, 1.0 / max(nx, ny))
        assert el.trace_size(el.disc(p, n_a), ms) == Mesh(nx, ny, 1.0).n_trace(LocalDisc(p, n_a))


def test_bad_disc_rejected():
    from paper_2308_02467_amd import el
    with pytest.raises(el.ElError):
        el.disc_sizes(el.disc(6, 6))
    with pytest.raises(el.ElError):
        el.disc_sizes(el.disc(0, 8))


def test_matvec_shape_pin_validates_its_argument():
    """el_matvec_shape is host-only: -1 (autotuner) and the three row shapes
    are accepted, anything else is EL_ERR_ARG."""
    from paper_2308_02467_amd import el
    L = el.lib()
    for v in (-1, 0, 1, 2, -1):
        assert L.el_matvec_shape(v) == 0, v
    for v in (-2, 3, 1 << 20):
        assert L.el_matvec_shape(v) != 0, v
    with pytest.raises(ValueError):
        el.matvec_shape(5)
    el.matvec_shape(-1)


def test_gemm_tile_pin_validates_its_argument():
    """el_gemm_tile is host-only: -1 (autotuner) and the four tiles are
    accepted, anything else is EL_ERR_ARG and leaves the setting alone."""
    from paper_2308_02467_amd import el
    L = el.lib()
    for v in (-1, 0, 1, 2, 3, -1):
        assert L.el_gemm_tile(v) == 0, v
    for v in (-2, 4, 1 << 20):
        assert L.el_gemm_tile(v) != 0, v
    with pytest.raises(ValueError):
        el.gemm_tile(7)
    el.gemm_tile(-1)


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message (one GPU only)."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_recorded_matvec_traffic_is_tied_to_the_source(tmp_path, monkeypatch):
    """The roofline's measured traffic comes from the committed counter
    summary only while the skeleton-product sources keep its hash and only
    for the row shape the autotuner chose: a summary line for that kernel with
    the current hash gives its figure; another hash, another shape or another
    operator type gives None."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert "paper_2308_02467_amd/csrc/el_internal.h" in bench.MATVEC_SOURCES   # the DiscDev layout
    text = open(os.path.join(ROOT, bench.TRAFFIC_SUMMARY["float16"])).read()
    assert re.search(r"traffic_bytes_per_launch k_matvec<_Float16, \d> = ([0-9.eE+]+) source_sha256 = ([0-9a-f]+)",
                     text)

    class FakeEl:
        @staticmethod
        def tuning_report():
            return ("gfx950 gemm M=16384 N=225792 K=1024 -> tile 256x256 lds (ms: 8.5 9.1)\n"
                    "gfx950 matvec f16 m=224 -> shape 4 rows x 4 chunks (ms: 0.317 0.320 0.345)\n")
    k4 = bench.matvec_kernel(FakeEl, "float16", 224)
    assert k4 == "k_matvec<_Float16, 4>"
    assert bench.matvec_kernel(FakeEl, "float16", 120) == "k_matvec<_Float16, ?>"
    cur = bench.matvec_source_hash()
    for sha, expect in ((cur, 1.5e9), ("0" * 64, None)):
        os.makedirs(tmp_path / "profiles", exist_ok=True)
        (tmp_path / bench.TRAFFIC_SUMMARY["float16"]).write_text(
            f"traffic_bytes_per_launch k_matvec<_Float16, 4> = 1.5e9 source_sha256 = {sha}\n")
        for f in bench.MATVEC_SOURCES:
            os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
            (tmp_path / f).write_bytes(open(os.path.join(ROOT, f), "rb").read())
        monkeypatch.setattr(bench, "ROOT", str(tmp_path))
        assert bench.recorded_traffic("float16", k4) == expect
        assert bench.recorded_traffic("float16", "k_matvec<_Float16, 2>") is None
    assert bench.recorded_traffic("float32", "k_matvec<float, 4>") is None
