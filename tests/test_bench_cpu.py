"""Host logic of bench.py (no GPU): bytes per update, the step-kernel
dispatch names, counter ingestion from rocprofv3 CSV files, and the refusal
of more than one GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def test_bytes_per_update():
    assert bench.bytes_per_update("f32") == 72 and bench.bytes_per_update("f16dev") == 36
    assert bench.bytes_per_update("f64") == 144 and bench.bytes_per_update("f32", 21) == 168


def test_step_dispatch_names():
    k = bench._step_dispatch_key
    assert k("void lbmwet::k_step_tiles<float, float, 0, 8, 1>(lbmwet::LatDev<float>, void const*, void*)") == 8
    assert k("void lbmwet::k_step_tiles<lbmwet::Dev16, float, 0, 5, 0>(lbmwet::LatDev<float>, void const*, "
             "void*)") == 5
    assert k("void lbmwet::k_step_pass2<float, float, 0, 1, 24, 12, 1>(lbmwet::LatDev<float>, void const*, "
             "void*)") == "pass2v8"
    assert k("void lbmwet::k_step_pass2<float, float, 1, 2, 8, 4, 0>(lbmwet::LatDev<float>, void const*, "
             "void*)") == "pass2v2"
    # single-step batches launch one kernel per tile shape over a subset of the lattices: not keyed
    assert k("void lbmwet::k_step_tiles_batch<float, float, 0, 5>(lbmwet::LatDev<float> const*, uint4 const*, int)") \
        is None
    assert k("void lbmwet::(anonymous namespace)::k_march_q21<0, 1, 1>(lbmwet::LatDev<float>, float const*, "
             "float*, unsigned int)") == 1
    assert k("void lbmwet::(anonymous namespace)::k_tile_q21<float, float, 0, 1, 0, 1, 2>(lbmwet::LatDev<float>, "
             "void const*, void*, int, int, int)") == 0
    assert k("void lbmwet::(anonymous namespace)::k_tile_q21<float, float, 1, 1, 0, 0, 1>(lbmwet::LatDev<float>, "
             "void const*, void*, int, int, int)") == 2             # one-row tiles
    assert k("void lbmwet::(anonymous namespace)::k_tile_q21<float, float, 0, 1, 1, 1, 2>(lbmwet::LatDev<float>, "
             "void const*, void*, int, int, int)") is None          # the diagnostic pass
    assert k("void lbmwet::k_diag<float, float, 0>(...)") is None
    assert bench.traffic_key("spinodal4096", "f32", 8) == "spinodal4096:f32:shape8"
    assert bench.traffic_key("spinodal4096_q21", "f32", 1) == "spinodal4096_q21:f32:k_march_q21"
    assert bench.traffic_key("drop1024_q21", "f32", 2) == "drop1024_q21:f32:k_tile_q21_r1"
    # two steps per launch: <storage, arithmetic, wall, strips, rows, waves per strip> -> variant
    assert k("void lbmwet::k_step_pass2<float, float, 0, 1, 24, 8>(lbmwet::LatDev<float>, void const*, void*)") \
        == "pass2v7"
    assert k("void lbmwet::k_step_pass2<__half, float, 1, 2, 8, 4>(lbmwet::LatDev<float>, void const*, void*)") \
        == "pass2v2"
    assert k("void lbmwet::k_step_pass2_batch<1, 24, 12>(lbmwet::LatDev<float> const*, uint4 const*, int)") \
        == "batch_pass2v8"
    assert k("void lbmwet::k_step_pass2_batch<2, 8, 4>(lbmwet::LatDev<float> const*, uint4 const*, int)") \
        == "batch_pass2v2"
    assert bench.traffic_key("spinodal4096", "f32", "pass2v7") == "spinodal4096:f32:pass2v7"
    assert bench.PASS2_GEOMETRY == [(s, r, w // s) for s, r, w in
                                    [(1, 8, 4), (1, 8, 8), (2, 8, 8), (1, 12, 6), (1, 12, 12), (1, 16, 8),
                                     (1, 16, 16), (1, 24, 8), (1, 24, 12)]]


def _write_run(path, counter, copy_kib, steps):
    os.makedirs(path)
    with open(os.path.join(path, "1_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        rows = [("__amd_rocclr_copyBuffer", 131072, copy_kib)]
        rows += [(name, 1024, v) for name, v in steps]
        for i, (name, grid, v) in enumerate(rows):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": i, "Grid_Size": grid, "Kernel_Name": name,
                        "Counter_Name": counter, "Counter_Value": v})


def test_ingest_counters(tmp_path):
    name = "void lbmwet::k_step_tiles<float, float, 0, 8, 1>(lbmwet::LatDev<float>, void const*, void*)"
    diag = "void lbmwet::k_diag<float, float, 0>(x)"
    # FETCH_SIZE books 128-byte requests as 64 bytes: the 1 GiB copy reads as 524288 KiB
    _write_run(str(tmp_path / "f"), "FETCH_SIZE", 524288.0, [(name, 300000.0), (name, 310000.0), (diag, 9e9)])
    _write_run(str(tmp_path / "w"), "WRITE_SIZE", 1048576.0, [(name, 589824.0), (name, 589824.0), (diag, 9e9)])
    out = tmp_path / "traffic.json"
    bench.ingest_counters(str(tmp_path / "f"), str(tmp_path / "w"), "spinodal4096", "f32", str(out))
    rec = json.loads(out.read_text())["spinodal4096:f32:shape8"]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["read_bytes"] == round(305000.0 * 2.0 * 1024)
    assert rec["write_bytes"] == 589824 * 1024 == 72 // 2 * 4096 * 4096
    assert rec["bytes_per_launch"] == rec["read_bytes"] + rec["write_bytes"]
    assert rec["kernel_sources_sha256"] == bench.kernel_sources_digest(9)
    assert bench.stored_traffic(str(out), "spinodal4096:f32:shape8") == rec["bytes_per_launch"]
    assert "valu_insts" not in rec
    # with a VALU run the record carries the instructions per launch and the ALU roofline follows
    _write_run(str(tmp_path / "v"), "SQ_INSTS_VALU", 1.0, [(name, 4.0e7), (name, 5.0e7)])
    bench.ingest_counters(str(tmp_path / "f"), str(tmp_path / "w"), "spinodal4096", "f32", str(out),
                          valu_dir=str(tmp_path / "v"))
    v = bench.stored_traffic(str(out), "spinodal4096:f32:shape8", "valu_insts")
    assert v == 45000000
    a = bench.alu_roofline(v, 0.1)
    assert a["frac"] == round(4.5e7 / 1e-4 / (256 * 2.4e9 * 2), 4) and a["bound"] == "alu"
    data = json.loads(out.read_text())
    data["spinodal4096:f32:shape8"]["kernel_sources_sha256"] = "0" * 64
    out.write_text(json.dumps(data))
    assert bench.stored_traffic(str(out), "spinodal4096:f32:shape8") is None


def test_ingest_counters_ensemble(tmp_path, capsys):
    """The ensemble's two-step batch kernel is keyed by variant; compulsory
    bytes count every lattice's nodes."""
    p2 = "void lbmwet::k_step_pass2_batch<1, 24, 8>(lbmwet::LatDev<float> const*, uint4 const*, int)"
    t4 = "void lbmwet::k_step_tiles_batch<float, float, 0, 4>(lbmwet::LatDev<float> const*, uint4 const*, int)"
    nodes = bench.workload_nodes("ensemble256")
    assert nodes == 44916736
    one = "void lbmwet::k_step_pass2<float, float, 0, 1, 24, 8, 1>(lbmwet::LatDev<float>, void const*, void*)"
    _write_run(str(tmp_path / "f"), "FETCH_SIZE", 524288.0,
               [(p2, nodes * 36 / 1024 / 2 * 1.5), (t4, 1000.0), (one, 50.0)])
    _write_run(str(tmp_path / "w"), "WRITE_SIZE", 1048576.0, [(p2, nodes * 36 / 1024), (t4, 2000.0), (one, 60.0)])
    out = tmp_path / "traffic.json"
    bench.ingest_counters(str(tmp_path / "f"), str(tmp_path / "w"), "ensemble256", "f32", str(out))
    data = json.loads(out.read_text())
    rec = data["ensemble256:f32:batch_pass2v7"]
    assert rec["read_bytes"] == round(nodes * 36 * 1.5) and rec["write_bytes"] == nodes * 36
    assert "| batch_pass2v7 | 1 |" in capsys.readouterr().out
    # the sequential leg's single-lattice launches are not the ensemble's kernel
    assert sorted(data) == ["ensemble256:f32:batch_pass2v7"]


def test_counter_table(tmp_path, capsys):
    """Per-dispatch means, per-update instruction counts (a two-step pass
    performs two updates per node) and the VALU issue fraction."""
    p2 = "void lbmwet::k_step_pass2<float, float, 0, 1, 24, 12, 1>(lbmwet::LatDev<float>, void const*, void*)"
    nodes = 4096 * 4096
    _write_run(str(tmp_path / "a"), "SQ_INSTS_VALU", 1.0, [(p2, 100.0 * nodes / 64 * 2), (p2, 100.0 * nodes / 64 * 2)])
    _write_run(str(tmp_path / "b"), "GRBM_GUI_ACTIVE", 1.0, [(p2, 8 * 1000.0), (p2, 8 * 1000.0)])
    out = bench.counter_table([str(tmp_path / "a"), str(tmp_path / "b")], "spinodal4096")
    k = "k_step_pass2<float, float, 0, 1, 24, 12, 1>"
    assert out[k]["SQ_INSTS_VALU"] == 100.0 * nodes / 32
    assert out[k]["valu_issue_fraction"] == pytest.approx(100.0 * nodes / 32 / (1000.0 * 256 * 2))
    assert "| 100.0 |" in capsys.readouterr().out


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _rec(rid, arrival, solve, **kw):
    r = {"rid": rid, "kind": "angle", "nx": 32, "ny": 32, "arrival": arrival, "solve_s": solve, "steps": 100,
         "converged": True, "floor": False, "rest": False, "residual": 1e-6, "value": [], "error": ""}
    r.update(kw)
    return r


def test_fifo_schedule():
    """One server in arrival order: a request waits for the previous finish or
    its own arrival, whichever is later."""
    out = bench.fifo_schedule([_rec(1, 0.5, 2.0), _rec(0, 0.0, 1.0), _rec(2, 10.0, 1.0)])
    assert [r["rid"] for r in out] == [0, 1, 2]
    assert [r["finished"] for r in out] == [1.0, 3.0, 11.0]
    assert [r["latency"] for r in out] == [1.0, 2.5, 1.0]
    s = bench.summarize_records(out)
    assert s["completed"] == 3 and s["elapsed_s"] == 11.0 and abs(s["solves_per_s"] - 3 / 11) < 1e-15


def test_serving_combine(tmp_path):
    cont = {"continuous": {"solves_per_s": 2.0, "p99_s": 4.0}}
    a = {"sequential_records": [_rec(0, 0.0, 1.0), _rec(1, 0.1, 1.0)], "sequential_two_step": 7}
    b = {"sequential_records": [_rec(2, 0.2, 3.0, rest=True)], "sequential_two_step": 7}
    paths = []
    for k, d in enumerate((cont, a, b)):
        paths.append(str(tmp_path / f"{k}.json"))
        json.dump(d, open(paths[-1], "w"))
    out = bench.serving_combine(paths, 3, 1000, 1e-5, 1 << 20)
    q = out["sequential"]
    assert q["elapsed_s"] == 5.0 and q["p99_s"] > 4.7 and q["converged_at_rest"] == 1 and q["two_step"] == 7
    assert out["p99_speedup"] == round(q["p99_s"] / 4.0, 2)
    json.dumps(out)
    with pytest.raises(SystemExit):
        bench.serving_combine(paths[:2], 3, 1000, 1e-5, 1 << 20)


def test_trace_table(tmp_path, capsys):
    d = tmp_path / "t" / "vm"
    os.makedirs(d)
    (d / "1_kernel_stats.csv").write_text(
        '"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
        '"void lbmwet::k_step_tiles<float, float, 0, 8, 1>(lbmwet::LatDev<float>, void const*, void*)",4,'
        '900000,225000.0,60.0,224000,226000,1.0\n'
        '"__amd_rocclr_copyBuffer",2,600000,300000.0,40.0,1000,599000,1.0\n')
    out = bench.trace_table(str(tmp_path / "t"))
    assert out == {"k_step_tiles<float, float, 0, 8, 1>": 225.0, "__amd_rocclr_copyBuffer": 300.0}
    assert "| `k_step_tiles<float, float, 0, 8, 1>` | 4 | 225.0 | 224.0 | 226.0 | 60.00 |" in capsys.readouterr().out
