"""Host logic behind the roofline figures: the per-site byte models of the
stencil launches, and the scaling of the FETCH_SIZE / WRITE_SIZE counters by
the 2 GiB calibration copy, on small synthetic rocprofv3 CSV files."""
import csv
import os

import pytest

from paper_2212_06635_amd import counters as C

STENCIL = "void tmx::dslash_kernel<0, 1, 0, 1>(tmx::DslashArgs)"  # K1 in FP64, one site per thread
COPY = "__amd_rocclr_copyBuffer"


def test_stencil_byte_models():
    """Bytes per output site, counted by hand from the operands each launch
    reads and writes once: links 8 x 12 reals, the inverse site blocks
    2 x 72 reals (K1) or the packed Hermitian clover 72 reals (K2), spinors of
    24 reals (K1 reads one, writes one; K2 reads the hop input and x, writes
    one), an FP16 spinor carrying a 4-byte scale."""
    b = {"f64": 8, "f32": 4, "f16": 2}
    for p in ("f64", "f32", "f16"):
        s = 4 if p == "f16" else 0
        assert C.kernel_bytes_per_site(f"K1_{p}") == (96 + 144) * b[p] + 2 * (24 * b[p] + s)
        assert C.kernel_bytes_per_site(f"K2_{p}") == (96 + 72) * b[p] + 3 * (24 * b[p] + s)
    assert C.kernel_bytes_per_site("K1_f64") == 2304 and C.kernel_bytes_per_site("K2_f64") == 1920
    # two flavours double the spinor part; n right-hand sides share the fixed part
    assert C.kernel_bytes_per_site("K1_f64_nd") == 2688 and C.kernel_bytes_per_site("K2_f64_nd") == 2496
    assert C.kernel_bytes_per_site("K1_f32_r4") == (96 + 144) * 4 + 4 * 2 * 24 * 4


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


@pytest.fixture
def run(tmp_path):
    """A profile directory: the stencil kernel at 400 us; the copy counters
    read half the true 2 GiB (FETCH) and exactly it (WRITE), so the scales
    are 2 and 1; the kernel's raw counters are 1 GiB fetched, 256 MiB written."""
    d = str(tmp_path)
    kib = C.COPY_BYTES / 1024
    _write(os.path.join(d, "p_k", "x", "k_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
           [[STENCIL, 10, 4.0e6, 4.0e5, 60.0], [COPY, 3, 3.0e6, 1.0e6, 40.0]])
    _write(os.path.join(d, "p_f", "x", "f_counter_collection.csv"),
           ["Kernel_Name", "Counter_Name", "Counter_Value"],
           [[STENCIL, "FETCH_SIZE", 2 ** 20]] * 10 + [[COPY, "FETCH_SIZE", kib / 2]] * 3
           + [[COPY, "FETCH_SIZE", 4.0]])  # a small copy elsewhere in the run is not the calibration
    _write(os.path.join(d, "p_w", "x", "w_counter_collection.csv"),
           ["Kernel_Name", "Counter_Name", "Counter_Value"],
           [[STENCIL, "WRITE_SIZE", 2 ** 18]] * 10 + [[COPY, "WRITE_SIZE", kib]] * 3)
    return d


def test_summary_scales_counters_by_the_copy(run, tmp_path):
    vh = 1048576
    txt = C.summarize(run, vh)
    assert "FETCH scale 2.000, WRITE scale 1.000" in txt
    row = next(ln.split() for ln in txt.splitlines() if ln.startswith("K1_f64"))
    fetch_mb, write_mb = float(row[6]), float(row[7])
    assert fetch_mb == pytest.approx(2 * 2 ** 30 / 1e6, abs=0.1)
    assert write_mb == pytest.approx(2 ** 28 / 1e6, abs=0.1)
    alg = C.kernel_bytes_per_site("K1_f64") * vh
    assert float(row[3]) == pytest.approx(alg / 1e6, abs=0.1)
    assert float(row[4]) == pytest.approx(alg / 4.0e-4 / 1e9, abs=0.1)  # GB/s at 400 us
    out = tmp_path / "summary.txt"
    out.write_text(txt)
    assert C.read_traffic(str(out), "K1_f64") == pytest.approx((fetch_mb + write_mb) * 1e6)
    assert C.read_traffic(str(out), "K2_f64") is None  # not in this profile


def test_traffic_ignored_for_other_kernel_sources(run, tmp_path):
    txt = C.summarize(run, 1048576).replace(C.source_digest(), "0" * 16)
    out = tmp_path / "stale.txt"
    out.write_text(txt)
    assert C.read_traffic(str(out), "K1_f64") is None
    assert C.read_traffic(str(tmp_path / "absent.txt"), "K1_f64") is None
