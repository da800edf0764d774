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
