"""Write a short markdown summary of a rocprofv3 --stats kernel table.

    python -m paper_2604_00250_amd.profile_summary STATS_CSV BENCH_JSON OUT_MD "COMMAND"
"""
import csv
import json
import sys


def main(stats_csv, bench_json, out_md, command):
    rows = list(csv.DictReader(open(stats_csv)))
    b = json.load(open(bench_json))
    rf = b.get("roofline", {})
    with open(out_md, "w") as f:
        f.write(f"# Kernel statistics: {b['config']['workload']} "
                f"({b['config']['voxels']:,} voxels, N={b['config']['measurements']}, K={b['config']['K']}, "
                f"{b['config']['mode'].upper()})\n\n")
        f.write("Command (repository root `$R` on the MI355X box):\n\n```\n" + command + "\n```\n\n")
        f.write("| kernel | calls | average ns | total ns | % |\n|---|---|---|---|---|\n")
        for r in rows:
            f.write(f"| {r['Name']} | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['TotalDurationNs']} | "
                    f"{float(r['Percentage']):.2f} |\n")
        kp = [r for r in rows if r["Name"].startswith("k_pass")]
        if kp and rf:
            f.write(f"\nThe benchmark's own HIP-event timing of k_pass (a separate run of the same build, "
                    f"{rf['launches']} launches): {rf['kernel_ms'] * 1e3:.0f} us; rocprofv3 average: "
                    f"{float(kp[0]['AverageNs']) / 1e3:.0f} us.\n")


if __name__ == "__main__":
    main(*sys.argv[1:5])


def kernel_source_hash(root=None) -> str:
    """SHA-1 of the kernel sources (a profile's counters describe this build only)."""
    import hashlib
    import os
    here = root or os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha1()
    for name in ("prism_kernels.hip", "prism_device.h", "prism_internal.h", "bessel_fit.h"):
        with open(os.path.join(here, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def traffic_summary(fetch_csv, write_csv, out_md, kernel, command_fetch, command_write, workload):
    """FETCH_SIZE / WRITE_SIZE per dispatch of `kernel`, scaled by what the same
    counters read for the microbenchmark's copy of a known size (2 x 1 GiB)."""
    def per_kernel(path):
        agg = {}
        for r in csv.DictReader(open(path)):
            agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in agg.items()}
    f = per_kernel(fetch_csv)
    w = per_kernel(write_csv)
    kib = 1 << 30 >> 10  # the copy reads 1 GiB and writes 1 GiB
    sf = kib / f["mb_copy_kernel"]
    sw = kib / w["mb_copy_kernel"]
    fk, wk = f[kernel], w[kernel]
    traffic = (fk * sf + wk * sw) * 1024
    with open(out_md, "w") as o:
        o.write(f"# HBM traffic of {kernel} on {workload}\n\n")
        o.write("Two rocprofv3 counter passes of the benchmark (repository root `$R`):\n\n```\n"
                + command_fetch + "\n" + command_write + "\n```\n\n")
        o.write("| counter | mb_copy_kernel (KiB/dispatch, 1 GiB read + 1 GiB written) | scale | "
                f"{kernel} (KiB/dispatch) | scaled bytes |\n|---|---|---|---|---|\n")
        o.write(f"| FETCH_SIZE | {f['mb_copy_kernel']:.1f} | {sf:.4f} | {fk:.1f} | {fk * sf * 1024:.4e} |\n")
        o.write(f"| WRITE_SIZE | {w['mb_copy_kernel']:.1f} | {sw:.4f} | {wk:.1f} | {wk * sw * 1024:.4e} |\n\n")
        o.write(f"traffic_bytes_per_dispatch: {traffic:.6e}\n")
        o.write(f"kernel_source_sha1: {kernel_source_hash()}\n")
    return traffic
