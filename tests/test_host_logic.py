"""Host-side logic that needs no GPU."""
import json
import sys
import os

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_big_endian_lanes_order_equals_byte_order():
    """Equal-length byte strings zero-padded to whole 8-byte lanes compare like
    memcmp when the lanes are compared as big-endian unsigned integers, most
    significant lane first (the fixed-width key rows the GPU sorts)."""
    rng = np.random.default_rng(14)
    for L in (1, 3, 4, 5, 8, 9, 15, 16, 17, 24, 31, 32):
        W = -(-L // 8) * 8
        A = np.zeros((4000, W), np.uint8)
        A[:, :L] = rng.integers(0, 256, (4000, L), dtype=np.uint8)
        A[::7, :L] = A[1::7, :L][: A[::7].shape[0]]      # plenty of equal words
        lanes = A.view(">u8")
        by_bytes = sorted(range(len(A)), key=lambda i: (A[i].tobytes(), i))
        by_lanes = sorted(range(len(A)), key=lambda i: (tuple(int(x) for x in lanes[i]), i))
        assert by_bytes == by_lanes, L


def test_class_of_length_and_element_bytes():
    assert [bench.class_of_len(L) for L in (0, 4, 5, 8, 9, 16, 17, 24, 25, 32)] == [0, 0, 1, 1, 2, 2, 3, 3, 4, 4]
    assert [bench.element_bytes(c) for c in range(5)] == [8, 12, 20, 28, 36]


def test_levels_and_byte_model():
    assert bench.levels_for(1, 4096) == 0 and bench.levels_for(4096, 4096) == 0
    assert bench.levels_for(4097, 4096) == 1 and bench.levels_for(8192, 4096) == 1
    assert bench.levels_for(8193, 4096) == 2
    fam = bench.algorithmic_bytes([(3, 10000), (6, 100), (7, 3000)], [4096] * 5)
    # class 0 segment of 10000: m = 2 levels; chunk sort reads 8 and writes 8
    assert fam["sort_tiles_c0"] == 16 * 10000
    assert fam["merge_c0"] == (8 + 8) * 10000 + (8 + 4) * 10000
    # a short class 1 segment is sorted in a packed tile; a 3000-word one fits
    # one chunk-sort tile and is finished there
    assert fam["sort_packed_c1"] == (12 + 4) * 100
    assert fam["sort_tiles_c1"] == (12 + 4) * 3000 and "merge_c1" not in fam
    assert fam["hist"] == 4 * 13100
    assert fam["scatter_pack"] == (4 + 3 + 8) * 10000 + (4 + 6 + 12) * 100 + (4 + 7 + 12) * 3000


def test_alu_roofline_from_counter_summary(tmp_path, monkeypatch):
    """The chunk sort's VALU view: issued lane-operations (SQ_INSTS_VALU x 64)
    per launch over the live launch time, against 256 CUs x 64 lanes x 2.4 GHz;
    no counters for the current source, workload and tiles -> no fraction."""
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9
    tiles = {"chunk": [16] * 5, "variant": [3, 3, 1, 0, 0], "merge": [0] * 5}
    info = {"avg_launch_us": 200.0, "launches_per_step": 1}
    monkeypatch.setattr(bench, "counter_file", lambda kind, w: str(tmp_path / ("%s_%s.json" % (kind, w))))
    r = bench.alu_roofline("sort_tiles_c0", info, "c3", tiles, {"sort_tiles_c0": 1.6e8})
    assert r["bound"] == "alu" and r["achieved"] is None and r["frac"] is None and r["counters"] is None
    assert abs(r["hbm_frac"] - 1.6e8 / 200e-6 / 1e9 / 8000) < 1e-12
    row = {"SQ_INSTS_VALU_per_dispatch": 6.0e7, "SQ_ACTIVE_INST_VALU_per_dispatch": 1.2e8,
           "GRBM_GUI_ACTIVE_per_dispatch": 480000.0, "SQ_INSTS_LDS_per_dispatch": 1e6,
           "SQ_LDS_BANK_CONFLICT_per_dispatch": 5e5}
    doc = {"source_hash": bench.kernel_source_hash(), "workload": "c3: docs (bench.py --serial)", "tiles": tiles,
           "kernels": {"sort_tiles_c0": row}}
    (tmp_path / "sq_counters_c3.json").write_text(json.dumps(doc))
    r = bench.alu_roofline("sort_tiles_c0", info, "c3", tiles, {"sort_tiles_c0": 1.6e8})
    assert abs(r["achieved"] - 6.0e7 * 64 / 200e-6 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / bench.VALU_PEAK_TOPS) < 1e-12
    assert abs(r["valu_busy"] - 1.2e8 * 4 / (1024 * 480000.0 / 8)) < 1e-12
    assert abs(r["clock_GHz"] - 480000.0 / 8 / 200e-6 / 1e9) < 1e-12
    assert r["lds_conflict_cycles_per_lds_inst"] == 0.5
    # another tile configuration or workload: the summary does not apply
    assert bench.alu_roofline("sort_tiles_c0", info, "c3", dict(tiles, chunk=[32] * 5), {})["frac"] is None
    assert bench.alu_roofline("sort_tiles_c0", info, "c4", tiles, {})["frac"] is None
