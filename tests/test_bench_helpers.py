"""Host-side helpers of the benchmark: the per-kernel byte models and the reader of
the committed counter summary (no GPU)."""
import os

import bench


def test_byte_models_cover_the_assembly_kernels():
    N, NT, nnz = 4198401, 8388608, 29372417
    names = ["k_l1_hist", "k_l1_scatter", "k_l1_fine", "k_l2_bucket", "k_pi", "k_rows_count",
             "k_rows_final", "k_label_rows", "k_pattern_to_label", "k_scatter_coords", "k_assemble_2d",
             "k_values_to_label"]
    for n in names:
        b = bench.kernel_bytes(n, N, NT, nnz, 2, False)
        assert b is not None and b > 0, n
    # the numeric kernel writes every row in processing order (8 bytes per stored
    # entry plus two right-hand side words a row) and reads one 8-byte word per
    # incidence at least; nodal data adds 8 bytes a vertex
    b2 = bench.kernel_bytes("k_assemble_2d", N, NT, nnz, 2, False)
    assert b2 > 8 * (nnz + 2 * N) + 8 * 3 * NT
    assert bench.kernel_bytes("k_assemble_2d", N, NT, nnz, 2, True) == b2 + 8 * N
    # the label-order copy writes val and val_bc
    assert bench.kernel_bytes("k_values_to_label", N, NT, nnz, 2, False) > 16 * nnz
    assert bench.kernel_bytes("k_fill", N, NT, nnz, 2, False) is None


def test_counter_summary_is_read_only_for_matching_sources(tmp_path, monkeypatch):
    text = ("fetch_scale: 2.0\nwrite_scale: 1.0\nsources_sha256: %s\n"
            "k_assemble_2d   100.0   50.0\n" % bench.source_hash())
    p = tmp_path / "counters_w.txt"
    p.write_text(text)
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "counters_{workload}.txt"))
    c = bench.read_counters("w")
    assert c["k_assemble_2d"] == (100.0 * 1024 * 2.0, 50.0 * 1024 * 1.0)
    p.write_text(text.replace(bench.source_hash(), "0" * 16))
    assert bench.read_counters("w") is None
    assert bench.read_counters("missing") is None


def test_source_hash_is_stable():
    assert bench.source_hash() == bench.source_hash()
    assert len(bench.source_hash()) == 16


def test_compulsory_bytes_per_element():
    """Inputs once plus outputs once: 79 B per triangle for the cold step of the
    2049^2 mesh (63 B warm, without rowptr/colind), 64.5 B per tetrahedron for the
    129^3 cube (+ 8 B per vertex of nodal f)."""
    N, NT, nnz = 4198401, 8388608, 29372417
    cold, warm = bench.step_bytes(N, NT, nnz, 2, False)
    assert abs(cold / NT - 79.0) < 0.05 and abs(warm / NT - 63.0) < 0.05
    n = 129
    N3, NT3 = n ** 3, 6 * (n - 1) ** 3
    nnz3 = N3 + 2 * (3 * n * n * (n - 1) + 3 * n * (n - 1) ** 2 + (n - 1) ** 3)
    cold3, warm3 = bench.step_bytes(N3, NT3, nnz3, 3, False)
    assert abs(cold3 / NT3 - 64.5) < 0.05
    assert bench.step_bytes(N3, NT3, nnz3, 3, True)[0] == cold3 + 8 * N3


def test_roofline_takes_the_longest_kernel_and_the_step_bytes():
    N, NT, nnz = 4198401, 8388608, 29372417
    kern = {"k_a": {"launches": 2, "total_ms": 0.2, "avg_ms": 0.1},
            "k_b": {"launches": 1, "total_ms": 0.3, "avg_ms": 0.3}}
    table = bench.kernel_table(kern, 1, N, NT, nnz, 2, False)
    cold, warm = bench.step_bytes(N, NT, nnz, 2, False)
    r = bench.roofline(table, {"k_a": (1e8, 1e8), "k_b": (3e8, 2e8)}, N, NT, nnz, 2, False, 2.0, 0.5)
    assert r["kernel"] == "k_b"
    assert abs(r["achieved"] - cold / 0.3e-3 / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    assert r["traffic"] == 5e8 and abs(r["traffic_ratio"] - 5e8 / cold) < 1e-12
    assert abs(r["warm_step"]["frac"] - warm / 0.5e-3 / 1e9 / 8000.0) < 1e-12
    assert abs(r["cold_step"]["traffic_ratio"] - (2 * 2e8 + 5e8) / cold) < 1e-12
