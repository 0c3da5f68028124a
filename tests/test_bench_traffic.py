"""bench.py's counter summary (--traffic-from): the copy calibration and the per-kernel averages,
on synthetic rocprofv3 counter files (no GPU)."""
import csv
import json
import os

import bench

FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for disp, name, grid, v in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": v})


def test_traffic_summary_scales_by_the_copy_and_averages_per_kernel(tmp_path, capsys):
    n, k = 1 << 18, 64
    grid = (n >> 3) * 512
    split = "void fio::(anonymous namespace)::k_split_fused<3, true>(fio::(anonymous namespace)::SplitArgsK)"
    f64 = "void fio::k_struct_fused<double, 9, 3, false, false, false, false>(fio::StructArgs<double, 9>)"
    leaf = "void fio::k_struct_fused<double, 9, 3, false, false, true, true>(fio::StructArgs<double, 9>)"
    gib = float(1 << 20)                      # KiB
    # the copy reads half of what it moves on this counter (scale 2), writes all of it (scale 1);
    # a fill of the same size writes without reading and must not be taken for the copy
    fetch = [(1, "fill", 1, 0.0), (2, "copy", 1, gib / 2),
             (3, split, grid, 1000.0), (4, split, grid, 3000.0), (5, split, grid // 2, 9e9),
             (6, f64, grid, 500.0), (7, leaf, grid, 100.0)]
    write = [(1, "fill", 1, gib), (2, "copy", 1, gib),
             (3, split, grid, 10.0), (4, split, grid, 30.0), (5, split, grid // 2, 9e9),
             (6, f64, grid, 50.0), (7, leaf, grid, 20.0)]
    _write(str(tmp_path / "F"), "FETCH_SIZE", fetch)
    _write(str(tmp_path / "W"), "WRITE_SIZE", write)
    out = str(tmp_path / "traffic.json")
    bench.traffic_from(str(tmp_path / "F"), str(tmp_path / "W"), n=n, k=k, q=9, out_path=out)
    d = json.load(open(out))
    assert abs(d["fetch_scale"] - 2.0) < 1e-12 and abs(d["write_scale"] - 1.0) < 1e-12
    ks = d["kernels"]
    # split: dispatches 3 and 4 only (5 has another grid): ((1000 + 3000) / 2 * 2 + (10 + 30) / 2) KiB
    assert abs(ks["bf_split16"]["hbm_bytes_per_launch"] - (4000.0 + 20.0) * 1024) < 1e-6
    assert ks["bf_split16"]["dispatches"] == 2
    assert abs(ks["bf_struct_f64"]["hbm_bytes_per_launch"] - (1000.0 + 50.0) * 1024) < 1e-6
    assert abs(ks["bf_struct_leaf_f64"]["hbm_bytes_per_launch"] - (200.0 + 20.0) * 1024) < 1e-6
    assert "bf_struct_f32" not in ks
    assert ks["bf_split16"]["algorithmic_bytes_per_launch"] == bench.kernel_model("bf_split16", n, 9, k)[0]
    assert d["source_hash"] == bench.kernel_source_hash()
    assert "| bf_split16 | 2 |" in capsys.readouterr().out


def test_roofline_prices_the_explicit_form_per_launch():
    """The roofline of the headline's passes at N = 2^18, q = 9, 64 columns, from the explicit
    factor form written out here: 12 transfer levels of (N/2) groups of 2q x 2q entries in four
    3-level passes, the middle factor's N q^2 entries on one of them, 8 bytes per entry as split
    halves (16 in FP64); 8 flops per entry and column, three split products on the matrix cores;
    the coefficient round trip 2 N q k e apart.  A measured launch time then fixes frac."""
    n, q, k = 1 << 18, 9, 64
    assert bench.pass_plan(n) == [(3, False), (3, True), (3, False), (3, False)]
    per_pass = (3 * (n // 2) * (2 * q) ** 2 * 4 + n * q * q) / 4      # entries, M averaged over 4 passes
    byts, flops, spill, peak = bench.kernel_model("bf_split16", n, q, k)
    assert byts == per_pass * 8 == 1061683200
    assert flops == 3 * 8 * per_pass * k and spill == 2 * n * q * k * 8 and peak == 2500.0
    r = bench.roofline_of("bf_split16", n, q, k, 0.7422, None)
    assert r["bound"] == "hbm" and abs(r["frac"] - 1061683200 / 0.7422e-3 / 8e12) < 1e-4
    byts, flops, spill, peak = bench.kernel_model("bf_struct_f64", n, q, k)
    assert byts == per_pass * 16 and flops == 8 * per_pass * k and spill == 2 * n * q * k * 16 and peak == 78.6
    r = bench.roofline_of("bf_struct_f64", n, q, k, 1.3278, None)
    assert r["bound"] == "alu" and abs(r["achieved"] - 8 * per_pass * k / 1.3278e-3 / 1e12) < 0.01
