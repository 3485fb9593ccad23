"""The counter arithmetic behind the roofline's `traffic` field, on synthetic rocprofv3
CSVs (no GPU): each counter is scaled by what it reads for the plain copy kernel of
known size, per dispatch, and bench.py uses an entry only for the kernel source, storage,
lattice size and workload it was measured on."""
import csv
import importlib.util
import json
import os
import subprocess
import sys

from paper_2212_14153_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY = "fpd::copy_kernel(float __vector(4) const*, float __vector(4)*, unsigned long)"
STEP = "void fpd::step_kernel<1, 1, 0>(fpd::StepArgs)"
GIB = 1 << 30


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, kib) in enumerate(rows):
            w.writerow([i, name, counter, kib])


def counters(tmp_path, fetch_copy_kib, write_copy_kib, fetch_step_kib, write_step_kib):
    fetch = str(tmp_path / "fetch.csv")
    write = str(tmp_path / "write.csv")
    # the copy's median is taken, so one outlier dispatch does not move the factor
    write_counters(fetch, "FETCH_SIZE", [(COPY, fetch_copy_kib), (COPY, fetch_copy_kib),
                                         (COPY, 3 * fetch_copy_kib)] +
                   [(STEP, fetch_step_kib)] * 4)
    write_counters(write, "WRITE_SIZE", [(COPY, write_copy_kib)] * 3 +
                   [(STEP, write_step_kib)] * 4)
    return fetch, write


def test_short_names():
    assert profsum.short_name(STEP) == "step_kernel<1, 1, 0>"
    assert profsum.short_name(COPY) == "copy_kernel"


def test_traffic_is_scaled_by_the_copy_kernel(tmp_path):
    # FETCH_SIZE reads half of the copy's 1 GiB (factor 2), WRITE_SIZE all of it (factor 1)
    fetch, write = counters(tmp_path, GIB / 2 / 1024, GIB / 1024, 300_000.0, 600_000.0)
    ent = profsum.traffic_entry(fetch, write, "step_kernel", GIB)
    assert ent["fetch_factor"] == 2.0 and ent["write_factor"] == 1.0
    assert ent["read_bytes_per_launch"] == 2 * 300_000 * 1024
    assert ent["write_bytes_per_launch"] == 600_000 * 1024
    assert ent["bytes_per_launch"] == (600_000 + 600_000) * 1024
    assert ent["dispatches"] == [4, 4]


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_uses_an_entry_only_where_it_was_measured(tmp_path, monkeypatch):
    bench = load_bench()
    sha = profsum.kernel_source_hash()
    path = tmp_path / "traffic.json"
    split = "fluid_kernel+fiber_kernel"
    rec = {"kernel_sha": sha,
           "entries": {"f32": {"bytes_per_launch": 1234, "nodes": 4096, "workload": "c3",
                               "kernel": split}}}
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic("f32", 4096, "c3", split) == 1234
    assert bench.measured_traffic("f32", 4096, "c3", "step_kernel") is None  # other kernels
    assert bench.measured_traffic("f32", 4096, "suspension", split) is None  # same lattice size
    assert bench.measured_traffic("f32", 8192, "c3", split) is None
    assert bench.measured_traffic("f64", 4096, "c3", split) is None
    rec["kernel_sha"] = "0" * 16                                         # kernels changed since
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("f32", 4096, "c3", split) is None


def test_traffic_of_a_pass_adds_its_kernels(tmp_path):
    """'a+b': the per-dispatch medians of both kernels add up, each scaled by the factor
    the copy kernel of the same run gives."""
    def write(path, counter, copy_kib, a_kib, b_kib):
        lines = ["Kernel_Name,Counter_Name,Counter_Value"]
        lines += [f"copy_kernel,{counter},{copy_kib}"] * 3
        lines += [f'"void fpd::fluid_kernel<1, 1, 0>(fpd::StepArgs)",{counter},{v}' for v in a_kib]
        lines += [f'"void fpd::fiber_kernel<1, 1, 0>(fpd::StepArgs)",{counter},{v}' for v in b_kib]
        path.write_text("\n".join(lines) + "\n")
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    write(f, "FETCH_SIZE", 512.0, [100.0, 101.0, 99.0], [10.0, 12.0, 11.0])
    write(w, "WRITE_SIZE", 1024.0, [90.0, 90.0, 91.0], [8.0, 8.0, 9.0])
    ent = profsum.traffic_entry(str(f), str(w), "fluid_kernel+fiber_kernel", 1024 * 1024)
    assert ent["fetch_factor"] == 2.0 and ent["write_factor"] == 1.0
    assert ent["read_bytes_per_launch"] == round((100.0 + 11.0) * 1024 * 2.0)
    assert ent["write_bytes_per_launch"] == round((90.0 + 8.0) * 1024)
    assert ent["dispatches"] == [3, 3]


def test_committed_traffic_entries_name_their_workload():
    with open(os.path.join(ROOT, "profiles", "traffic_step_kernel.json")) as f:
        rec = json.load(f)
    for storage, ent in rec["entries"].items():
        assert ent["workload"] == "c3" and f"--storage {storage}" in ent["command"]
        assert ent["bytes_per_launch"] == ent["read_bytes_per_launch"] + ent["write_bytes_per_launch"]


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=60, cwd=ROOT)
    assert out.returncode == 2 and "one GPU only" in out.stderr and out.stdout == ""


def test_graph_chunk_covers_the_timed_steps():
    """The timed steps replay captured graphs: the chunk is even, at most 64 and divides the
    step count when an even divisor exists; odd counts leave their last step direct."""
    bench = load_bench()
    assert bench.choose_chunk(20) == 20 and bench.choose_chunk(2000) == 50
    assert bench.choose_chunk(128) == 64 and bench.choose_chunk(6) == 6
    assert bench.choose_chunk(1) is None
    assert bench.timed_path(20, 20) == {"graph_chunk": 20, "graph_replays": 1, "direct_steps": 0}
    assert bench.timed_path(2000, 50)["graph_replays"] == 40
    c = bench.choose_chunk(25)
    assert c == 24 and bench.timed_path(25, c) == {"graph_chunk": 24, "graph_replays": 1,
                                                   "direct_steps": 1}
    assert bench.timed_path(1, None) == {"graph_chunk": None, "graph_replays": 0,
                                         "direct_steps": 1}
