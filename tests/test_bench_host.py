"""CPU tests of bench.py's host-side accounting: how rocprofv3 counter rows become measured bytes
per stage group (ingest_pmc), which stage group a kernel belongs to, and the rule that measured
traffic is reported only for the kernel source it was taken on."""
import csv
import json

import pytest

import bench

NS = "dsort::(anonymous namespace)::"
L1_TILE = f"void {NS}k_tile<unsigned int, false, 16, 16384, 0, false, false, false>({NS}TileArgs)"
L2_TILE = f"void {NS}k_tile<unsigned int, false, 16, 16384, 0, false, false, true>({NS}TileArgs)"
ONE_SORT = [
    (NS + "k_init(unsigned int*)", 1, 0),
    (L1_TILE, 1000, 1100),
    (f"void {NS}k_sort_samples<unsigned long, 16, 16384>(...)", 30, 20),
    (f"void {NS}k_merge_round<unsigned long, 8, 8192>(...)", 40, 30),
    (f"void {NS}k_rank<unsigned int, false>(...)", 500, 10),
    (NS + "k_scan_partial(unsigned int const*, unsigned int*, unsigned int, unsigned int)", 20,
     5),
    (L2_TILE, 1300, 1100),
    (f"void {NS}k_gather_bsort<unsigned int, false, 8192, false, false>(...)", 1200, 1000),
]
COPY = "__amd_rocclr_copyBuffer"


def write_counters(path, counter, rows):
    """rows: (kernel name, value in KiB), in dispatch order."""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": v})


def test_group_of_alternates_the_tile_levels():
    seen = {}
    groups = [bench._group_of(name, seen) for name, _, _ in ONE_SORT + ONE_SORT]
    assert groups[1] == "steps1-3 local sort + sampling"
    assert groups[6] == "step8 + level2 steps1-3"
    assert groups[9] == "steps1-3 local sort + sampling"  # the second sort's level 1
    assert groups[14] == "step8 + level2 steps1-3"
    assert groups[2] == groups[3] == "step4 sample sort"
    assert groups[4] == "steps5-6 rank"
    assert groups[5] == "step7 scan"
    assert groups[7] == "steps8-9 gather + bucket sort"
    assert groups[0] == "init"


def test_ingest_pmc_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    # two sorts; the copy after them reads twice its size (FETCH_SIZE) and writes its size
    copy_bytes = 1 << 20
    fetch = [(n, f) for n, f, _ in ONE_SORT] * 2 + [(COPY, 2 * copy_bytes / 1024),
                                                    (COPY, 4.0)]  # a small read-back as well
    write = [(n, w) for n, _, w in ONE_SORT] * 2 + [(COPY, copy_bytes / 1024), (COPY, 4.0)]
    fcsv, wcsv, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    write_counters(fcsv, "FETCH_SIZE", fetch)
    write_counters(wcsv, "WRITE_SIZE", write)
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0123456789abcdef")
    bench.ingest_pmc(str(fcsv), str(wcsv), copy_bytes, 2, str(out))
    t = json.load(open(out))
    assert t["fetch_scale"] == pytest.approx(0.5)
    assert t["write_scale"] == pytest.approx(1.0)
    assert t["kernel_source_sha256_16"] == "0123456789abcdef"
    per = t["bytes_per_step"]
    # per sort: FETCH KiB * 1024 * 0.5 + WRITE KiB * 1024
    assert per["steps1-3 local sort + sampling"] == pytest.approx(1000 * 512 + 1100 * 1024)
    assert per["step8 + level2 steps1-3"] == pytest.approx(1300 * 512 + 1100 * 1024)
    assert per["step4 sample sort"] == pytest.approx(70 * 512 + 50 * 1024)
    assert per["steps8-9 gather + bucket sort"] == pytest.approx(1200 * 512 + 1000 * 1024)
    assert "init" not in per and "other" not in per
    # reported only while the kernel source hash matches
    assert bench.traffic_for("steps5-6 rank", str(out)) == pytest.approx(500 * 512 + 10 * 1024)
    monkeypatch.setattr(bench, "kernel_hash", lambda: "fedcba9876543210")
    assert bench.traffic_for("steps5-6 rank", str(out)) is None
    assert bench.traffic_for("steps5-6 rank", str(tmp_path / "missing.json")) is None


def test_committed_traffic_files_match_the_kernel_source():
    # profiles/traffic.json and traffic_c3b.json carry the hash of the kernel source they were
    # measured on; a change to the kernels without new counter runs turns them off (null)
    for path in (bench.TRAFFIC_FILE, bench.TRAFFIC_C3B_FILE):
        t = json.load(open(path))
        assert set(t["bytes_per_step"]) <= set(bench.STAGE_GROUPS)
        assert all(v > 0 for v in t["bytes_per_step"].values())
        if t["kernel_source_sha256_16"] == bench.kernel_hash():
            for g in t["bytes_per_step"]:
                assert bench.traffic_for(g, path) == pytest.approx(t["bytes_per_step"][g])
