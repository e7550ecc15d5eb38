"""Host logic of bench.py that needs no GPU: reading rocprofv3 counter files."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, grid, wg, counter, value) in enumerate(rows):
            w.writerow({k: 0 for k in FIELDS} | {"Dispatch_Id": i + 1, "Grid_Size": grid, "Kernel_Name": name,
                                                  "Workgroup_Size": wg, "Counter_Name": counter,
                                                  "Counter_Value": value})


def test_pmc_rows_count_workgroups_whatever_the_block_size(tmp_path):
    # a 12-wave (768-thread) launch of 8192 tiles and an 8-wave one of 3199:
    # one workgroup per 64-point tile either way
    kz = "void mala::k_zb<10>(float2 const*, long, float*, float const*, int const*, int const*, int)"
    _write(str(tmp_path / "f"), [(kz, 8192 * 768, 768, "FETCH_SIZE", 100.0),
                                 ("other", 1024, 256, "FETCH_SIZE", 5.0),
                                 (kz, 3199 * 512, 512, "FETCH_SIZE", 40.0),
                                 (kz, 8192 * 768, 768, "WRITE_SIZE", 7.0)])
    rows = bench._pmc_rows(str(tmp_path / "f"), "FETCH_SIZE", "void mala::k_zb<10>")
    assert [(nb, v) for _, nb, v in rows] == [(8192, 100.0), (3199, 40.0)]
