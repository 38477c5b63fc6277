"""Host logic of the counter summary behind roofline.traffic: scaling by the
copy kernel's counters, kind and precision from the kernel name, the mean
over dispatches, and the most-dispatched kernel of each kind winning."""
import csv
import os

from paper_1204_5434_amd import build, traffic_summary


def write_run(base, counter, rows):
    d = os.path.join(base, f"pmc_{counter}")
    os.makedirs(d)
    with open(os.path.join(d, "lam128_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": v})


def test_summary_scales_and_classifies(tmp_path):
    base = str(tmp_path)
    y64 = "void pft::k_spass<double, 16, 8, 1, 1, 2>(pft::SArgs<double>)"
    x64 = "void pft::k_spass<double, 16, 8, 0, 1, 2>(pft::SArgs<double>)"
    x64_probe = "void pft::k_spass<double, 8, 16, 0, 1, 2>(pft::SArgs<double>)"  # a tuner variant, rarer
    dens = "void pft::k_density<float>(pft::cx<float> const*, ...)"
    other = "void (anonymous namespace)::k_field_tables<double>(...)"
    probe = "(anonymous namespace)::k_copy_probe(double4 const*, double4*, long)"
    # the copy kernel moves 512 MiB: FETCH reads half of it, WRITE all of it
    fetch = [(probe, 262144), (probe, 262144), (y64, 1000), (y64, 3000), (x64, 500), (x64, 500), (x64, 500),
             (x64_probe, 9999), (dens, 10), (other, 77)]
    write = [(probe, 524288), (probe, 524288), (y64, 100), (y64, 300), (x64, 50), (x64, 50), (x64, 50),
             (x64_probe, 1), (dens, 2), (other, 5)]
    write_run(base, "FETCH_SIZE", fetch)
    write_run(base, "WRITE_SIZE", write)
    txt, rows = traffic_summary.summarize(base)
    rec = {ln.split()[0]: ln.split()[1:] for ln in txt if not ln.startswith("#")}
    assert set(rec) == {"ypass:f64", "xpass:f64", "density:f32"}
    # mean KiB x scale x 1024: y = (2000 x 2 + 200 x 1) KiB
    assert float(rec["ypass:f64"][0]) == (2000 * 2 + 200) * 1024
    assert float(rec["xpass:f64"][0]) == (500 * 2 + 50) * 1024  # the 3-dispatch kernel, not the probe
    assert rec["xpass:f64"][1] == "pft::k_spass<double,16,8,0,1,2>"
    assert float(rec["density:f32"][0]) == (10 * 2 + 2) * 1024
    assert rec["ypass:f64"][2] == build.kernel_hash("ypass")
    assert rec["density:f32"][2] == build.kernel_hash("density")
    assert len(rows) == 4


def test_density_hash_ignores_host_runtime():
    # the density kernel's counters stay valid across edits of the host runtime
    density = build.KERNEL_FILES[build.KIND_GROUP["density"]]
    assert "context.hip" not in density and "runtime.h" not in density
    assert "density.h" in density


def test_build_compiles_every_unit_and_hashes_existing_files():
    # every HIP translation unit of csrc goes into the library, and every file
    # a kernel kind's staleness hash covers exists
    units = sorted(f for f in os.listdir(build.CSRC) if f.endswith(".hip"))
    assert sorted(build.SOURCES) == units
    for kind, files in build.KERNEL_FILES.items():
        for f in files:
            assert os.path.isfile(os.path.join(build.CSRC, f)), (kind, f)
    # the plane-pass hash covers the walled plane kernels too
    assert {"planes_walls.inc", "planes_walls_f32_z0.hip"} <= set(build.KERNEL_FILES["yzpass"])
