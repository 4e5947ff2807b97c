"""The conversion of rocprofv3 counter passes into the stored counter files
that bench.py reads (bench.py --ingest-profiles), on synthetic CSV files:
medians over dispatches, the calibration copy, VALU busy and HBM bytes."""
import csv
import json
import os

import bench

HDR = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
       "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
       "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
FWD = "void dmi::k_fwd_cols<9, 4, 24, true>(dmi::Work, dmi::Consts, dmi::TwiddleSet, dmi::DivTable const*)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for disp, name, counter, value, ns in rows:
            w.writerow([disp, disp, "Agent 1", 1, 1, 1, 512, 1, name, 256, 0, 0, 8, 0, 32,
                        counter, value, 1000, 1000 + ns])


def test_ingest_counters(tmp_path):
    prof = tmp_path / "prof"
    # three fwd_cols dispatches (median = the middle one) and two copies (the
    # larger one is the 256 MiB calibration copy)
    valu = []
    for disp, (insts, ns) in enumerate([(1000.0, 50_000), (2000.0, 40_000), (3000.0, 60_000)], start=1):
        for c, v in (("SQ_INSTS_VALU", insts), ("SQ_ACTIVE_INST_VALU", insts), ("SQ_WAVES", 10.0),
                     ("SQ_LDS_BANK_CONFLICT", 5.0), ("SQ_ACTIVE_INST_LDS", 10.0)):
            valu.append((disp, FWD, c, v, ns))
    _write(str(prof / "pmc_valu" / "c2_counter_collection.csv"), valu)
    _write(str(prof / "pmc_fetch" / "c2_counter_collection.csv"),
           [(1, FWD, "FETCH_SIZE", 100.0, 50_000), (2, COPY, "FETCH_SIZE", 4.0, 3_000),
            (3, COPY, "FETCH_SIZE", 131072.0, 60_000)])
    _write(str(prof / "pmc_write" / "c2_counter_collection.csv"),
           [(1, FWD, "WRITE_SIZE", 300.0, 50_000), (2, COPY, "WRITE_SIZE", 4.0, 3_000),
            (3, COPY, "WRITE_SIZE", 262144.0, 60_000)])
    out = tmp_path / "out"
    out.mkdir()
    bench.ingest_profiles(str(prof), 256, str(out))
    d = json.load(open(out / "c2_10m_counters.json"))
    assert d["source_hash"] == bench.kernel_source_hash()
    assert abs(d["fetch_scale"] - 2.0) < 1e-12 and abs(d["write_scale"] - 1.0) < 1e-12
    c = d["kernels"]["fwd_cols"]
    assert c["SQ_INSTS_VALU"] == 2000.0 and c["ns_valu"] == 50_000
    assert abs(c["valu_busy"] - 2000.0 * 4 / (1024 * 2.4e9 * 50e-6)) < 1e-12
    assert c["lds_bank_conflict_per_lds_active"] == 0.5
    assert abs(c["hbm_bytes"] - 1024.0 * (100.0 * 2.0 + 300.0 * 1.0)) < 1e-9
    h = json.load(open(out / "hbm_traffic.json"))
    assert h["kernels"]["fwd_cols"]["bytes_per_launch"] == c["hbm_bytes"]
    assert h["source_hash"] == d["source_hash"]
