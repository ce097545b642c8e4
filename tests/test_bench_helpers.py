"""bench.py's local helpers: the Kronecker product it uses to check square-free
decompositions, and its reader of the stored oracle output."""
import os
import random

import bench
from tests.golden.make_golden import load


def _schoolbook(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    while out and out[-1] == 0:
        out.pop()
    return out


def test_kronecker_product_matches_schoolbook():
    rng = random.Random(3)
    for _ in range(200):
        a = [rng.randint(-(1 << rng.randint(1, 300)), 1 << 200) for _ in range(rng.randint(1, 12))]
        b = [rng.randint(-(1 << 90), 1 << rng.randint(1, 300)) for _ in range(rng.randint(1, 12))]
        a[-1] = a[-1] or 1
        b[-1] = b[-1] or -1
        assert bench._zx_mul(a, b) == _schoolbook(a, b)
    assert bench._zx_mul([], [1, 2]) == []
    assert bench._zx_derivative([5, 3, 0, 4]) == [3, 0, 12]
    assert bench._zx_derivative([7]) == []


def test_golden_reader_matches_the_loader():
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    for name in ("deg6_res_0.txt", "deg20_res_0.txt"):
        assert bench.read_golden(os.path.join(here, name)) == load(name)[1]


def test_model_mulmods_and_peak():
    rowdeg = [20 - j for j in range(21)]
    # 231 + 231 evaluation products, 2 * 20 * 20 elimination products
    assert bench.model_mulmods(rowdeg, rowdeg) == 462 + 800
    assert abs(bench.int_peak_tops({"cus": 256, "clock_khz": 2400000}) - 39.3216) < 1e-9


def test_stored_counters_reads_only_current_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    digest = bench.kernel_source_digest()
    (prof / "valu_kx_wl.md").write_text("x\nsource_sha256: %s\nint_lane_ops_per_instance: 3557.5\n" % digest)
    (prof / "valu_ky_wl.md").write_text("source_sha256: %s\nint_lane_ops_per_instance: 1\n" % ("0" * 64))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: digest)
    assert bench.stored_counters("valu", "kx", "wl", "int_lane_ops_per_instance") == 3557.5
    assert bench.stored_counters("valu", "ky", "wl", "int_lane_ops_per_instance") is None
    assert bench.stored_counters("valu", "kz", "wl", "int_lane_ops_per_instance") is None
