"""Host-side checks of the profile summaries that feed the benchmark's
roofline object (paper_2506_20513_amd/rocprof_summary.py): the HBM counter
calibration against a plain copy, the choice of the timed launches, the
source hash that ties a summary to the kernels it measured, and the lookup
the benchmark does.  Synthetic counter files; no GPU."""
import argparse
import csv
import json

from paper_2506_20513_amd import rocprof_summary as R

FWD = "void fwi::(anonymous namespace)::k_fwd<8, false, 0>(fwi::FwdStreamArgs)"
REFWD = "void fwi::(anonymous namespace)::k_fwd<8, false, 1>(fwi::FwdStreamArgs)"
ADJ = "void fwi::(anonymous namespace)::k_adj<8, false>(fwi::AdjStreamArgs)"
COPY = R.COPY_KERNEL


def _write_run(tmp, name, counter, rows, bench):
    d = tmp / name
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name",
                               "Counter_Value"])
        w.writeheader()
        for i, (kernel, grid, kib) in enumerate(rows, 1):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Grid_Size": grid,
                        "Counter_Name": counter, "Counter_Value": kib})
    js = tmp / f"{name}.json"
    js.write_text("log line\n" + json.dumps(bench) + "\n")
    return str(d), str(js)


def _bench():
    return {"config": {"workload": "synthetic", "grid": [40, 30], "shots": 2}, "steps": 1,
            "kernels": {"k_fwd_sweep": {"launches_per_step": 2, "bytes_per_launch": 1.0e5},
                        "k_fwd_reforward": {"launches_per_step": 1, "bytes_per_launch": 1.5e5},
                        "k_adj": {"launches_per_step": 1, "bytes_per_launch": 2.0e5}}}


def test_counter_calibration_and_timed_launches(tmp_path):
    copy_mb = 1
    copy_kib = copy_mb * 1024
    # FETCH_SIZE counts half of the copy's reads (factor 2), WRITE_SIZE all
    # of them (factor 1); a small copy elsewhere in the run is not the probe.
    fetch_rows = [(COPY, 64, 3.0), (FWD, 10, 10.0), (FWD, 10, 20.0), (ADJ, 10, 7.0),
                  (REFWD, 10, 40.0), (FWD, 10, 30.0), (REFWD, 10, 50.0), (ADJ, 10, 9.0),
                  (COPY, 4096, copy_kib / 2)]
    write_rows = [(COPY, 64, 5.0), (FWD, 10, 4.0), (FWD, 10, 6.0), (ADJ, 10, 1.0),
                  (REFWD, 10, 11.0), (FWD, 10, 8.0), (REFWD, 10, 13.0), (ADJ, 10, 3.0),
                  (COPY, 4096, copy_kib)]
    fd, fj = _write_run(tmp_path, "fetch", "FETCH_SIZE", fetch_rows, _bench())
    wd, wj = _write_run(tmp_path, "write", "WRITE_SIZE", write_rows, _bench())
    a = argparse.Namespace(fetch_dir=fd, fetch_json=fj, write_dir=wd, write_json=wj,
                           command_fetch="cmd f", command_write="cmd w", copy_mb=copy_mb)
    text = R.counters_summary(a)
    machine = json.loads(text.split("```json\n")[1].split("\n```")[0])
    assert machine["kernel_sources"] == R.kernel_source_hash()
    assert machine["grid"] == [40, 30] and machine["shots"] == 2
    # timed launches are the last launches_per_step * steps dispatches
    fwd = machine["kernels"]["k_fwd_sweep"]
    assert abs(fwd["fetch_bytes"] - 2.0 * 25.0 * 1024) < 1e-6
    assert abs(fwd["write_bytes"] - 1.0 * 7.0 * 1024) < 1e-6
    assert abs(fwd["traffic_bytes"] - (51200.0 + 7168.0)) < 1e-6
    adj = machine["kernels"]["k_adj"]
    assert abs(adj["traffic_bytes"] - (2.0 * 9.0 + 3.0) * 1024) < 1e-6
    assert adj["algorithmic_bytes"] == 2.0e5
    ref = machine["kernels"]["k_fwd_reforward"]      # its last launch only
    assert abs(ref["traffic_bytes"] - (2.0 * 50.0 + 13.0) * 1024) < 1e-6

    # the benchmark's lookup: found for this workload, not for another
    path = tmp_path / "summary.md"
    path.write_text(text)
    assert R.read_traffic(str(path), "k_fwd_sweep", [40, 30], 2) == fwd["traffic_bytes"]
    assert R.read_traffic(str(path), "k_fwd_sweep", [40, 31], 2) is None
    assert R.read_traffic(str(path), "k_fwd_sweep", [40, 30], 3) is None
    assert R.read_traffic(str(tmp_path / "missing.md"), "k_fwd_sweep", [40, 30], 2) is None
    # a summary taken on other kernel sources is ignored
    stale = text.replace(R.kernel_source_hash(), "0" * 16)
    path.write_text(stale)
    assert R.read_traffic(str(path), "k_fwd_sweep", [40, 30], 2) is None


def test_source_hash_ignores_comments_only():
    src = ("// header\nint f(int a) {\n  /* block\n comment */ return a + 1;  // tail\n}\n")
    same = "int f(int a) {\n return a + 1;\n}\n// another comment\n"
    other = "int f(int a) {\n  return a + 2;\n}\n"
    assert R._code_only(src) == R._code_only(same)
    assert R._code_only(src) != R._code_only(other)



def test_forward_kernel_variants_have_their_own_names():
    assert R.short_name(FWD) == "k_fwd_sweep"
    assert R.short_name(REFWD) == "k_fwd_reforward"
    assert R.short_name("void fwi::(anonymous namespace)::k_fwd<4, true, 1>(fwi::FwdStreamArgs)") \
        == "k_fwd_reforward"
    assert R.short_name(ADJ) == "k_adj"
    assert R.short_name("void fwi::(anonymous namespace)::k_fwd_tab<4, false>(x)") == "k_fwd_tab"
