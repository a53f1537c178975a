"""Host-side pieces of bench.py (no GPU): workload table, step accounting,
algorithmic bytes, the traffic gate and the one-GPU guard."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_workload_and_rhs_accounting():
    import bench
    c4 = bench.CONFIGS["c4"]
    assert c4["dims"] == (32, 32, 32, 64) and c4["nprobe"] == [20, 100, 400]
    # O_l and F_l per non-coarsest level (F_l solves on l and l + 1), coarsest once
    assert bench.rhs_per_step([20, 100, 400]) == 3 * 20 + 3 * 100 + 400


def test_dslash_algorithmic_bytes():
    import bench
    V = 32 * 32 * 32 * 64
    # FP32, one rhs: 768 bytes per site (links 288, clover 288, spinor in + out 192)
    assert bench.dslash_bytes("dslash_f32", V, 1) == 768 * V
    assert bench.dslash_bytes("dslash_f64", V, 1) == 1536 * V
    assert bench.dslash_bytes("dslash_f16", V, 1) == 384 * V


def test_traffic_gate_rejects_other_sources(tmp_path, monkeypatch):
    import bench
    f = tmp_path / "t.txt"
    f.write_text("kernel_sources_sha256: 0000\nfetch_scale: 2\nwrite_scale: 1\n"
                 "fetch_kib_nrhs8: 1\nwrite_kib_nrhs8: 1\nfetch_kib_nrhs4: 1\nwrite_kib_nrhs4: 1\n")
    monkeypatch.setitem(bench.TRAFFIC_FILES, "dslash_f16", str(f))
    V = 1024
    assert bench.measured_traffic("dslash_f16", V, 3, 3 * bench.dslash_bytes("dslash_f16", V, 8)) is None
    f.write_text(f.read_text().replace("0000", bench.kernel_sources_hash()))
    t = bench.measured_traffic("dslash_f16", V, 3, 2 * bench.dslash_bytes("dslash_f16", V, 8)
                               + bench.dslash_bytes("dslash_f16", V, 4))
    assert abs(t - 3 * 1024.0) < 1e-9  # (1 * 2 + 1) KiB at every rhs count


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_gate_rejects_other_launch_variants(tmp_path, monkeypatch):
    import bench
    f = tmp_path / "t.txt"
    f.write_text("kernel_sources_sha256: %s\nfetch_scale: 2\nwrite_scale: 1\nvariant_nrhs8: 2\nvariant_nrhs4: 2\n"
                 "fetch_kib_nrhs8: 1\nwrite_kib_nrhs8: 1\nfetch_kib_nrhs4: 1\nwrite_kib_nrhs4: 1\n"
                 % bench.kernel_sources_hash())
    monkeypatch.setitem(bench.TRAFFIC_FILES, "dslash_f16", str(f))
    V = 1024
    total = 3 * bench.dslash_bytes("dslash_f16", V, 8)
    assert bench.measured_traffic("dslash_f16", V, 3, total, {8: 2, 4: 2}) == 3 * 1024.0
    assert bench.measured_traffic("dslash_f16", V, 3, total, {8: 3, 4: 2}) is None
    assert bench.traffic_record("dslash_f16")["variant_nrhs8"] == "2"
    assert bench.kernel_name("dslash_f16", {8: 2, 4: 2}).startswith("k_dslash_march")
    assert bench.kernel_name("dslash_f16", {8: 0, 4: 2}).startswith("k_dslash<")


def test_traffic_gate_with_one_rhs_count(tmp_path, monkeypatch):
    """A record of one rhs count (the bench's 20-rhs batches run the step in
    4-rhs groups only): every launch must be of that count."""
    import bench
    f = tmp_path / "t.txt"
    f.write_text("kernel_sources_sha256: %s\nrhs_counts: 4\nfetch_scale: 2\nwrite_scale: 1\nvariant_nrhs4: 25\n"
                 "fetch_kib_nrhs4: 3\nwrite_kib_nrhs4: 5\n" % bench.kernel_sources_hash())
    monkeypatch.setitem(bench.TRAFFIC_FILES, "dslash_f16", str(f))
    V = 1024
    b4 = bench.dslash_bytes("dslash_f16", V, 4)
    assert bench.rhs_counts(bench.traffic_record("dslash_f16")) == (4, 4)
    assert bench.measured_traffic("dslash_f16", V, 5, 5 * b4, {4: 25}) == (3 * 2 + 5) * 1024.0
    assert bench.measured_traffic("dslash_f16", V, 5, 4 * b4 + bench.dslash_bytes("dslash_f16", V, 8),
                                  {4: 25}) is None
    assert bench.measured_traffic("dslash_f16", V, 5, 5 * b4, {4: 24}) is None


def test_auxiliary_fine_batch():
    import bench
    assert bench.aux_fine_batch(bench.CONFIGS["c4"]) == 8
    assert bench.aux_fine_batch(bench.CONFIGS["c2"]) == bench.CONFIGS["c2"]["batch"][0] // 2


def test_roofline_takes_the_tighter_roof():
    import bench
    V = 32 * 32 * 32 * 64
    b8 = bench.dslash_bytes("dslash_f16", V, 8)
    # 1896 flop per site and rhs: at 8 FP16 rhs the unpacked-FMA floor (0.40 ms)
    # is above the HBM floor of the algorithmic bytes (0.28 ms)
    assert abs(bench.dslash_flops("dslash_f16", V, 2, 2 * b8) - 2 * 8 * 1896 * V) < 1
    q = {"launches": 1, "bytes": b8}
    r = bench.roofline("dslash_f16", V, q, b8 / 1e-3 / 1e9, 1.0, b8, {}, None)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["other_roof"]["bound"] == "hbm"
    assert abs(r["frac"] - 8 * 1896 * V / 1e-3 / 1e12 / bench.VALU_PEAK_TFLOPS) < 1e-12
    # FP64 at one rhs: 1536 bytes per site for 1896 flop, HBM is the tighter roof
    b1 = bench.dslash_bytes("dslash_f64", V, 1)
    r = bench.roofline("dslash_f64", V, {"launches": 1, "bytes": b1}, 1.0, 1.0, b1, {}, None)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"


def test_traffic_split_follows_the_recorded_rhs_counts(tmp_path, monkeypatch):
    import bench
    f = tmp_path / "t.txt"
    f.write_text("kernel_sources_sha256: %s\nrhs_counts: 16 4\nfetch_scale: 2\nwrite_scale: 1\n"
                 "fetch_kib_nrhs16: 3\nwrite_kib_nrhs16: 0\nfetch_kib_nrhs4: 1\nwrite_kib_nrhs4: 0\n"
                 % bench.kernel_sources_hash())
    monkeypatch.setitem(bench.TRAFFIC_FILES, "dslash_f16", str(f))
    V = 1024
    # two launches at 16 rhs and one at 4: (2 * 6 + 2) KiB / 3
    total = 2 * bench.dslash_bytes("dslash_f16", V, 16) + bench.dslash_bytes("dslash_f16", V, 4)
    assert abs(bench.measured_traffic("dslash_f16", V, 3, total) - 14 * 1024.0 / 3) < 1e-9
    assert bench.rhs_counts(bench.traffic_record("dslash_f16")) == (16, 4)


def test_run_batches():
    import bench
    c4 = bench.CONFIGS["c4"]
    assert bench.run_batches(c4, "mixed", False) == c4["batch"] == [20, 100, 80]
    assert bench.run_batches(c4, "f64", False) == c4["batch_f64"]
    assert bench.run_batches(c4, "mixed", True) == [16, 100, 80]
    assert bench.run_batches(c4, "f64", True, [4, 8, 8]) == [4, 8, 8]
    c3 = bench.CONFIGS["c3"]
    assert bench.run_batches(c3, "f64", True) == c3["batch"]
