"""Host logic of the rocprofv3 summaries that give bench.py its measured
HBM traffic: counter scaling by the copy probe, and the choice of summary by
kernel, workload and source fingerprint (no GPU needed)."""
import csv
import os

from paper_2411_16445_amd import profiling


def _counter_csv(d, counter, kernel_kib, copy_kib):
    os.makedirs(d, exist_ok=True)
    rows = [dict(Dispatch_Id="1", Kernel_Name="void pa::k_epoch<float, 128u>(...)", Grid_Size="128000",
                 Counter_Name=counter, Counter_Value=str(kernel_kib)),
            dict(Dispatch_Id="2", Kernel_Name="__amd_rocclr_copyBuffer", Grid_Size="4096",
                 Counter_Name=counter, Counter_Value="1.0"),
            dict(Dispatch_Id="3", Kernel_Name="__amd_rocclr_copyBuffer", Grid_Size="1048576",
                 Counter_Name=counter, Counter_Value=str(copy_kib))]
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_counters_are_scaled_by_the_copy_probe(tmp_path):
    # a 256 MiB copy reads 131072 KiB of FETCH_SIZE (factor 2) and 262144
    # KiB of WRITE_SIZE (factor 1); the largest copy is the probe
    _counter_csv(tmp_path / "f", "FETCH_SIZE", 100.0, 131072.0)
    _counter_csv(tmp_path / "w", "WRITE_SIZE", 50.0, 262144.0)
    text = profiling.counters_summary(str(tmp_path / "f"), str(tmp_path / "w"), "k_epoch<float", 256,
                                      ["cmd"], 10, "ei2000x21")
    fields = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith("|"))
    assert float(fields["traffic_bytes_per_launch"]) == (100.0 * 2 + 50.0) * 1024
    assert float(fields["traffic_bytes_per_step"]) == (100.0 * 2 + 50.0) * 1024 / 10
    assert fields["workload"] == "ei2000x21"
    assert fields["source_sha256"] == profiling.source_fingerprint()


def test_bench_takes_the_summary_of_its_kernel_workload_and_sources(tmp_path):
    fp = profiling.source_fingerprint()

    def write(name, workload, per_step, sha):
        (tmp_path / name).write_text(f"traffic_bytes_per_step: {per_step}\nkernel: k_epoch<float\n"
                                     f"workload: {workload}\nsource_sha256: {sha}\n")

    write("counters_a.md", "ei2000x101", 2.0, fp)
    write("counters_b.md", "ei2000x21", 1.0, fp)
    write("counters_c.md", "trees4096", 3.0, "0" * 64)
    assert profiling.traffic_for_bench(str(tmp_path), "k_epoch<float>", "ei2000x21") == (1.0, "counters_b.md")
    assert profiling.traffic_for_bench(str(tmp_path), "k_epoch<float>", "ei2000x101") == (2.0, "counters_a.md")
    v, why = profiling.traffic_for_bench(str(tmp_path), "k_epoch<float>", "trees4096")
    assert v is None and "changed" in why
    v, why = profiling.traffic_for_bench(str(tmp_path), "k_epoch<double>", "ei2000x21")
    assert v is None



def test_only_the_last_dispatches_count_when_asked(tmp_path):
    """A bench run's timed launches are the kernel's last dispatches: trials
    and settling before them are left out."""
    def csv_with(d, counter, values, copy_kib):
        os.makedirs(d, exist_ok=True)
        rows = [dict(Dispatch_Id=str(i + 1), Kernel_Name="void pa::k_epoch<float, 128u>(...)", Grid_Size="128000",
                     Counter_Name=counter, Counter_Value=str(v)) for i, v in enumerate(values)]
        rows.append(dict(Dispatch_Id="99", Kernel_Name="__amd_rocclr_copyBuffer", Grid_Size="1048576",
                         Counter_Name=counter, Counter_Value=str(copy_kib)))
        with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=list(rows[0]))
            w.writeheader()
            w.writerows(rows)
    csv_with(tmp_path / "f", "FETCH_SIZE", [1.0, 2.0, 100.0, 300.0], 131072.0)
    csv_with(tmp_path / "w", "WRITE_SIZE", [5.0, 5.0, 50.0, 150.0], 262144.0)
    text = profiling.counters_summary(str(tmp_path / "f"), str(tmp_path / "w"), "k_epoch<float", 256,
                                      ["cmd"], 20, "ei2000x101", last=2)
    fields = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith("|"))
    per_launch = (200.0 * 2 + 100.0) * 1024
    assert float(fields["traffic_bytes_per_launch"]) == per_launch
    assert float(fields["traffic_bytes_per_step"]) == per_launch / 20


def test_trace_summary_reports_the_timed_launches(tmp_path):
    stats = tmp_path / "run_kernel_stats.csv"
    with open(stats, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                                          "MaxNs"])
        w.writeheader()
        w.writerow(dict(Name="void pa::k_epoch<float, 128u>(...)", Calls=3, TotalDurationNs=21000,
                        AverageNs=7000, Percentage=100, MinNs=1000, MaxNs=10000))
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for i, (a, b) in enumerate([(0, 1000), (5000, 15000), (20000, 30000)]):
            w.writerow(dict(Dispatch_Id=i + 1, Kernel_Name="void pa::k_epoch<float, 128u>(...)",
                            Start_Timestamp=a, End_Timestamp=b))
    text = profiling.trace_summary(str(stats), ["cmd"], "t", kernel="k_epoch<float", last=2)
    assert "timed_launch_mean_us: 10.000" in text
