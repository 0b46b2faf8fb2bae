"""Host logic of the measurement, on the CPU: the roofline's choice of
kernel and its fraction, and the committed HBM-traffic summaries it reads."""
import glob
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _summary(path):
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def test_roofline_takes_the_byte_moving_kernel_with_most_time():
    # name -> (ms per step, algorithmic bytes per launch, ms per launch, launches per step, impl bytes)
    cands = {"k_apply_counted": (0.28, 84e6, 0.28, 1, 216e6),
             "k_bin": (0.12, 48e6, 0.12, 1, 192e6),
             "close_graph": (0.40, 0.0, 0.40, 1, None)}      # more time, no algorithmic bytes
    ro = bench.roofline(cands, "no_such_workload")
    assert ro["kernel"] == "k_apply_counted"
    assert ro["achieved"] == pytest.approx(84e6 / 0.28e-3 / 1e9, rel=1e-4)
    assert ro["frac"] == pytest.approx(ro["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    assert ro["traffic"] is None and ro["peak"] == 8000.0 and ro["bound"] == "hbm"
    assert set(ro["others"]) == {"k_bin", "close_graph"}


def test_traffic_summaries_are_consistent():
    """Every committed summary's HBM bytes are its scaled counters; those taken
    on the current kernel source are the ones the benchmark reads."""
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.txt")))
    assert files
    current = bench.kernel_source_sha()
    n_current = 0
    for path in files:
        kv = _summary(path)
        want = (float(kv["fetch_kib_per_launch"]) * float(kv["fetch_scale"]) +
                float(kv["write_kib_per_launch"]) * float(kv["write_scale"])) * 1024
        # (the scales are printed to three decimals; the bytes were computed from the measured ones)
        assert float(kv["hbm_bytes_per_launch"]) == pytest.approx(want, rel=1e-4), path
        name = os.path.basename(path)[len("traffic_"):-len(".txt")]
        assert name == f"{kv['kernel']}_{kv['workload']}", path
        got = bench.load_traffic(kv["kernel"], kv["workload"])
        if kv["kernel_source_sha"] == current:
            n_current += 1
            assert got == float(kv["hbm_bytes_per_launch"]), path
        else:
            assert got is None, path
    assert n_current > 0


def test_kernel_source_hash_ignores_comments(tmp_path, monkeypatch):
    src = tmp_path / "paper_1803_11036_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "internal.h").write_text("constexpr int A = 1;\n")
    (src / "kernels.hip").write_text("int f() { return 1; }\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_sha()
    (src / "kernels.hip").write_text("// a comment\n/* a block\n comment */\nint f() { return 1; }  // trailing\n\n")
    assert bench.kernel_source_sha() == h0
    (src / "kernels.hip").write_text("int f() { return 2; }\n")
    assert bench.kernel_source_sha() != h0
