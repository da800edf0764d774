"""Short markdown summaries of rocprofv3 output for the fused kernel.

    python -m paper_2604_00250_amd.profile_summary stats   STATS_CSV BENCH_JSON OUT_MD "COMMAND"
    python -m paper_2604_00250_amd.profile_summary traffic FETCH_CSV WRITE_CSV OUT_MD KERNEL WORKLOAD "CMD_F" "CMD_W"
    python -m paper_2604_00250_amd.profile_summary valu    AGENT_CSV BENCH_JSON OUT_MD KERNEL "COMMANDS" PASS_CSV...

stats: the kernel table of `rocprofv3 --kernel-trace --stats`.  traffic: HBM
bytes per dispatch from FETCH_SIZE / WRITE_SIZE, scaled by what the same
counters read for the microbenchmark's copy of a known size.  valu: issue
and utilisation figures of one kernel from SQ counter passes.
"""
import csv
import json
import sys


def stats_summary(stats_csv, bench_json, out_md, command):
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


def kernel_source_hash(root=None) -> str:
    """SHA-1 of the kernel sources (a profile's counters hold only for kernels built from them)."""
    import hashlib
    import os
    here = root or os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha1()
    names = sorted(n for n in os.listdir(here) if n.endswith((".hip", ".h")) and n != "microbench.hip")
    for name in names:
        with open(os.path.join(here, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def _per_kernel(path):
    agg = {}
    for r in csv.DictReader(open(path)):
        agg.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def traffic_summary(fetch_csv, write_csv, out_md, kernel, command_fetch, command_write, workload):
    """FETCH_SIZE / WRITE_SIZE per dispatch of `kernel`, scaled by what the same
    counters read for the microbenchmark's copy of a known size (2 x 1 GiB)."""
    f = {k[0]: v for k, v in _per_kernel(fetch_csv).items()}
    w = {k[0]: v for k, v in _per_kernel(write_csv).items()}
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


def valu_summary(agent_csv, bench_json, out_md, kernel, commands, pass_csvs):
    """Issue counts per (voxel, measurement) pair and busy fractions of `kernel`
    from SQ counter passes (averages over its dispatches).  Elapsed cycles are
    GRBM_GUI_ACTIVE / XCDs; SQ_ACTIVE_INST_VALU and SQ_WAVE_CYCLES count quad
    cycles summed over waves."""
    agent = [r for r in csv.DictReader(open(agent_csv)) if r["Agent_Type"].strip('"') == "GPU"][0]
    n_xcc = int(agent["Num_Xcc"])
    simds = int(agent["Cu_Count"]) * int(agent["Simd_Per_Cu"])
    c = {}
    for p in pass_csvs:
        for (k, name), v in _per_kernel(p).items():
            if k == kernel:
                c.setdefault(name, v)
    b = json.load(open(bench_json))
    cfg = b["config"]
    pairs = cfg["voxels"] * cfg["measurements"]
    cyc = c["GRBM_GUI_ACTIVE"] / n_xcc
    lanes = 64.0
    per_pair = lambda name: c[name] * lanes / pairs  # noqa: E731
    busy_valu = c["SQ_ACTIVE_INST_VALU"] * 4 / (simds * cyc)
    waves = c["SQ_WAVE_CYCLES"] * 4 / (simds * cyc)
    mfma = c["SQ_VALU_MFMA_BUSY_CYCLES"] / (simds * cyc) if "SQ_VALU_MFMA_BUSY_CYCLES" in c else None
    flops = None
    if "SQ_INSTS_VALU_FMA_F32" in c:
        flops = (2 * c["SQ_INSTS_VALU_FMA_F32"] + c["SQ_INSTS_VALU_ADD_F32"] + c["SQ_INSTS_VALU_MUL_F32"]
                 + c["SQ_INSTS_VALU_TRANS_F32"]) * lanes
    rows = [
        ("VALU instructions per pair", per_pair("SQ_INSTS_VALU")),
        ("  of which FP32 transcendental (exp, log, rcp)", per_pair("SQ_INSTS_VALU_TRANS_F32")),
        ("  of which FP32 FMA", per_pair("SQ_INSTS_VALU_FMA_F32") if "SQ_INSTS_VALU_FMA_F32" in c else None),
        ("  of which FP32 MUL", per_pair("SQ_INSTS_VALU_MUL_F32") if "SQ_INSTS_VALU_MUL_F32" in c else None),
        ("  of which FP32 ADD", per_pair("SQ_INSTS_VALU_ADD_F32") if "SQ_INSTS_VALU_ADD_F32" in c else None),
        ("MFMA instructions per pair", per_pair("SQ_INSTS_MFMA")),
        ("LDS instructions per pair", per_pair("SQ_INSTS_LDS")),
        ("SALU instructions per pair", per_pair("SQ_INSTS_SALU")),
        ("vector memory instructions per pair", per_pair("SQ_INSTS_VMEM")),
        ("elapsed cycles per dispatch (GRBM_GUI_ACTIVE / XCDs)", cyc),
        ("VALU busy (fraction of SIMD-cycles)", busy_valu),
        ("matrix core busy (fraction of SIMD-cycles)", mfma),
        ("mean resident waves per SIMD", waves),
        ("wave-cycles waiting for an instruction to issue (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES)",
         c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"] if "SQ_WAIT_INST_ANY" in c else None),
        ("wave-cycles waiting on a dependency or counter (SQ_WAIT_ANY / SQ_WAVE_CYCLES)",
         c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"] if "SQ_WAIT_ANY" in c else None),
    ]
    with open(out_md, "w") as o:
        o.write(f"# VALU, transcendental and matrix-core use of {kernel} on {cfg['workload']}\n\n")
        o.write(f"{cfg['voxels']:,} voxels x {cfg['measurements']} measurements = {pairs:,} pairs per "
                f"dispatch; {simds} SIMDs in {n_xcc} XCDs.  Counter passes (repository root `$R`):\n\n```\n"
                + commands + "\n```\n\n| quantity | value |\n|---|---|\n")
        for name, v in rows:
            if v is None:
                continue
            o.write(f"| {name} | {v:.4g} |\n")
        if flops is not None:
            o.write(f"| FP32 VALU FLOPs per pair (FMA = 2) | {flops / pairs:.4g} |\n")
        o.write(f"\nkernel_source_sha1: {kernel_source_hash()}\n")
    return dict(rows)


if __name__ == "__main__":
    cmd, args = sys.argv[1], sys.argv[2:]
    if cmd == "stats":
        stats_summary(*args[:4])
    elif cmd == "traffic":
        fetch, write, out, kernel, workload, cf, cw = args[:7]
        traffic_summary(fetch, write, out, kernel, cf, cw, workload)
    elif cmd == "valu":
        agent, bench, out, kernel, commands = args[:5]
        valu_summary(agent, bench, out, kernel, commands, args[5:])
    else:
        raise SystemExit(f"unknown summary {cmd}")
