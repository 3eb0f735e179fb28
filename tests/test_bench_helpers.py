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
