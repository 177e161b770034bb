"""Host logic of the profile summaries (paper_1410_2153_amd.counters) on synthetic rocprofv3 CSVs."""
import csv

import pytest

from paper_1410_2153_amd import counters as C


def _pmc(path, counter, kernel_vals, copy_kib):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size"])
        w.writeheader()
        w.writerow({"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter, "Counter_Value": 1.0,
                    "Grid_Size": 64})
        w.writerow({"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter, "Counter_Value": copy_kib,
                    "Grid_Size": 1 << 20})
        for v in kernel_vals:
            w.writerow({"Kernel_Name": f"void {C.KERNEL}(int, int)", "Counter_Name": counter, "Counter_Value": v,
                        "Grid_Size": 4096})
            w.writerow({"Kernel_Name": "void asmg::k_sell<1, double>(int)", "Counter_Name": counter,
                        "Counter_Value": 1e9, "Grid_Size": 4096})


def test_traffic_record_scales_by_the_copy(tmp_path):
    # the copy moves COPY_BYTES; FETCH_SIZE reading half of it gives factor 2, WRITE_SIZE exact 1
    _pmc(tmp_path / "f.csv", "FETCH_SIZE", [100.0, 300.0], C.COPY_BYTES / 1024 / 2)
    _pmc(tmp_path / "w.csv", "WRITE_SIZE", [10.0, 30.0], C.COPY_BYTES / 1024)
    rec = C.record("graded1M", tmp_path / "f.csv", tmp_path / "w.csv")
    assert rec["dispatches"] == 2
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2)
    assert rec["write_bytes_per_launch"] == pytest.approx(20.0 * 1024)
    assert rec["traffic_bytes_per_launch"] == pytest.approx(200.0 * 2048 + 20.0 * 1024)
    assert rec["kernel_code_key"] == C.source_key()
    assert rec["kernel"] == C.WORKLOADS["graded1M"]["kernel"]


def test_batched_record_averages_both_pass_kernels(tmp_path):
    # the batched colour pass runs as two kernels (sweeps from zero and the others): the record
    # averages the dispatches of both, and ignores the other kernels
    names = C.WORKLOADS["batched256x4"]["kernel"]
    assert isinstance(names, tuple) and len(names) == 2
    for path, counter, vals, copy in ((tmp_path / "f.csv", "FETCH_SIZE", (100.0, 300.0, 500.0), C.COPY_BYTES / 2048),
                                      (tmp_path / "w.csv", "WRITE_SIZE", (10.0, 20.0, 60.0), C.COPY_BYTES / 1024)):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, ["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size"])
            w.writeheader()
            w.writerow({"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter, "Counter_Value": copy,
                        "Grid_Size": 1 << 20})
            for name, v in zip((names[0], names[1], names[1]), vals):
                w.writerow({"Kernel_Name": f"void {name}(int, int)", "Counter_Name": counter, "Counter_Value": v,
                            "Grid_Size": 4096})
            w.writerow({"Kernel_Name": "void asmg::kb_sell<1, 4, double, 0>(int)", "Counter_Name": counter,
                        "Counter_Value": 1e9, "Grid_Size": 4096})
    rec = C.record("batched256x4", tmp_path / "f.csv", tmp_path / "w.csv")
    assert rec["dispatches"] == 3
    assert rec["fetch_bytes_per_launch"] == pytest.approx(300.0 * 1024 * 2)
    assert rec["write_bytes_per_launch"] == pytest.approx(30.0 * 1024)
    assert rec["kernel"] == " and ".join(names)


def test_bco_kernel_classification():
    yes64 = ["asmg::k_sell<0, double>", "asmg::k_sell<1, double>", "asmg::k_sell<2, double, 1>",
             "asmg::k_sell_spmv<0, 1, double, 16>",
             "asmg::k_sell_spmv<1, 0, double, 32>", "asmg::k_gemv<double>", "asmg::k_gs_first<double>"]
    yes32 = [n.replace("double", "float") for n in yes64] + ["asmg::k_gs_first_cvt"]
    no = ["asmg::k_cg_spmv", "asmg::k_cg_rz<double>", "asmg::k_cg_axpy<float>", "asmg::kb_sell<0, 4, double>",
          "__amd_rocclr_copyBuffer", "asmg::k_true_res<8>"]
    assert all(C._bco_kernel(n, "double") and not C._bco_kernel(n, "float") for n in yes64)
    assert all(C._bco_kernel(n, "float") and not C._bco_kernel(n, "double") for n in yes32)
    assert not any(C._bco_kernel(n, p) for n in no for p in ("double", "float"))
    # the batched engine's kernels
    b64 = ["asmg::kb_sell<0, 4, double>", "asmg::kb_sell<1, 2, double>", "asmg::kb_sell_spmv<0, 1, 4, double>",
           "asmg::kb_sell_spmv<1, 0, 1, double>", "asmg::kb_gemv<4, double>", "asmg::kb_first<4, double>",
           "asmg::kb_sell<2, 4, double, 0>", "asmg::kb_sell<3, 4, double, 1>", "asmg::kb_sell_spmv<0, 0, 4, double, 0>"]
    b32 = [n.replace("double", "float") for n in b64] + ["asmg::kb_first_cvt<4>"]
    bno = ["asmg::kb_cg_spmv<4>", "asmg::kb_cg_rz<4, double>", "asmg::k_sell<0, double>", "asmg::kb_cg_axpy<4, float>"]
    assert all(C._bco_kernel(n, "double", "batch") and not C._bco_kernel(n, "float", "batch") for n in b64)
    assert all(C._bco_kernel(n, "float", "batch") and not C._bco_kernel(n, "double", "batch") for n in b32)
    assert not any(C._bco_kernel(n, p, "batch") for n in bno for p in ("double", "float"))
    assert C._bco_application("asmg::kb_cg_rz<4, double>", "double", "batch")
    assert not C._bco_application("asmg::kb_cg_rz<4, float>", "double", "batch")
    assert C._bco_application("asmg::k_gemv<float>", "float", "single")


def test_source_key_ignores_comments_and_whitespace(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x) { return x + 1; }\n")
    b.write_text("// note\nint f(int x)  {\n  /* block */ return x + 1;  // tail\n}\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    assert C.source_key([a]) == C.source_key([b]) != C.source_key([c])


def test_trace_phases_split_at_gaps(tmp_path):
    cols = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Workgroup_Size_X"]
    rows = []
    t = 0
    for phase, (n, dur, wg) in enumerate([(3, 4000, 256), (2, 6000, 128)]):
        for _ in range(n):
            rows.append({"Kernel_Name": f"void {C.KERNEL}(int)", "Start_Timestamp": t, "End_Timestamp": t + dur,
                         "Workgroup_Size_X": wg})
            rows.append({"Kernel_Name": "void other(int)", "Start_Timestamp": t + dur + 100,
                         "End_Timestamp": t + dur + 200, "Workgroup_Size_X": 64})
            t += dur + 1000
        t += 10 ** 6  # 1 ms idle: a new phase
    with open(tmp_path / "t.csv", "w", newline="") as f:
        w = csv.DictWriter(f, cols)
        w.writeheader()
        w.writerows(rows[::-1])  # unsorted on purpose
    ph = C.trace_phases(tmp_path / "t.csv")
    assert [p["launches"] for p in ph] == [3, 2]
    assert ph[0]["mean_us"] == pytest.approx(4.0) and ph[1]["mean_us"] == pytest.approx(6.0)
    assert ph[0]["block_sizes"] == {256: 3} and ph[1]["block_sizes"] == {128: 2}
