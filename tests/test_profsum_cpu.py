"""Host-only checks of the rocprofv3 summary tool that regenerates the
profile tables: working-dispatch filtering of a kernel trace, and the
counter traffic scaled by what each counter reads for the 1 GiB copy."""
import csv
import json

from paper_1807_08692_amd import profsum


def write_csv(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_trace_working_dispatches(tmp_path):
    p = tmp_path / "trace.csv"
    rows = []
    t = 0
    # five launches of 1000 us and two returning at once (3 us)
    for d in [1000, 1000, 3, 1000, 1000, 3, 1000]:
        rows.append({"Kernel_Name": "void hd::k_spmm<1, false, false>(long, ...)", "Start_Timestamp": t,
                     "End_Timestamp": t + d * 1000})
        t += d * 1000 + 10
    rows.append({"Kernel_Name": "hipMemsetAsync", "Start_Timestamp": t, "End_Timestamp": t + 5000})
    write_csv(p, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    out = profsum.trace(str(p)).splitlines()
    assert len(out) == 3  # header, rule, the one library kernel
    cells = [c.strip() for c in out[2].strip("|").split("|")]
    assert cells[0] == "hd::k_spmm<1, false, false>"
    assert cells[1] == "7" and cells[3] == "5"
    assert float(cells[4]) == 1000.0
    assert abs(float(cells[2]) - (5000 + 6) / 7) < 0.05


def test_traffic_scaled_by_the_copy(tmp_path):
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    fields = ["Kernel_Name", "Grid_Size", "Counter_Value"]
    # the 1 GiB copy reads 1 GiB and writes 1 GiB: FETCH_SIZE counts half
    # of it, WRITE_SIZE all of it (KiB)
    copy = "hd::k_probe_copy(float const*, float*, unsigned long)"
    spmm = "hd::k_spmm<1, false, false>(long, ...)"
    write_csv(f, fields, [{"Kernel_Name": copy, "Grid_Size": 1, "Counter_Value": 524288},
                          {"Kernel_Name": spmm, "Grid_Size": 1, "Counter_Value": 1000},
                          {"Kernel_Name": spmm, "Grid_Size": 1, "Counter_Value": 3000},
                          {"Kernel_Name": spmm, "Grid_Size": 1, "Counter_Value": 10}])
    write_csv(w, fields, [{"Kernel_Name": copy, "Grid_Size": 1, "Counter_Value": 1048576},
                          {"Kernel_Name": spmm, "Grid_Size": 1, "Counter_Value": 500},
                          {"Kernel_Name": spmm, "Grid_Size": 1, "Counter_Value": 500},
                          {"Kernel_Name": spmm, "Grid_Size": 1, "Counter_Value": 500}])
    out_json = tmp_path / "t.json"
    table = profsum.traffic(str(f), str(w), str(out_json))
    assert "FETCH_SIZE x 2.000, WRITE_SIZE x 1.000" in table
    d = json.load(open(out_json))
    k = d["kernels"]["hd::k_spmm<1, false, false>"]
    # the 10 KiB dispatch (an iteration that returned at once) is not a working one
    assert k["fetch_bytes"] == 2.0 * 2000 * 1024
    assert k["write_bytes"] == 500 * 1024
    assert k["kind"] == "spmm" and k["source"] == "k_spmm.hip" and len(k["sha256"]) == 64
