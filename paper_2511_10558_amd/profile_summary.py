"""Turns rocprofv3 CSV output into the short summaries kept in profiles/.

    python -m paper_2511_10558_amd.profile_summary TRACE_DIR FETCH_DIR WRITE_DIR FETCH_LOG [TRACE_LOG]
    python -m paper_2511_10558_amd.profile_summary --markers MARKER_DIR COMMAND
    python -m paper_2511_10558_amd.profile_summary --mfma MFMA_DIR MFMA_LOG COMMAND
    python -m paper_2511_10558_amd.profile_summary --trace TRACE_DIR LOG NAME TITLE COMMAND

TRACE_DIR holds run_kernel_stats.csv of a --kernel-trace --stats run;
FETCH_DIR / WRITE_DIR hold run_counter_collection.csv of the FETCH_SIZE and
WRITE_SIZE passes of a bench run started with --calibrate-copy (one
elementwise multiply of 32 Mi doubles: 256 MiB read, 256 MiB written);
FETCH_LOG is that bench run's
output line (for the number of factorisations); TRACE_LOG, if given, the
traced run's output (its standalone right-hand-side figure).  Writes
profiles/kernel_stats_net500.md and profiles/traffic.json.  With --markers,
MARKER_DIR holds run_marker_api_trace.csv of a --marker-trace run (the
library's host ranges) and COMMAND is the command that made it; writes
profiles/markers_net500.md.  With --mfma, MFMA_DIR holds run_counter_collection.csv
of a run with the counters SQ_VALU_MFMA_BUSY_CYCLES, SQ_BUSY_CU_CYCLES,
SQ_INSTS_VALU_MFMA_MOPS_F64 and SQ_WAVE_CYCLES and MFMA_LOG that run's bench
line; writes profiles/mfma_net500.md.  With --trace, a kernel-statistics table
of another run goes to profiles/NAME.md.
"""
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_2511_10558_amd/csrc/device_lu2.hpp", "paper_2511_10558_amd/csrc/device_lu.hpp",
                  "paper_2511_10558_amd/csrc/device_chem.hpp", "paper_2511_10558_amd/csrc/kernels.hip",
                  "paper_2511_10558_amd/csrc/device_common.hpp"]
COPY_BYTES = 256 * 1024 * 1024


def source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name):
    """Kernel name without return type, namespace and argument list."""
    if "MulFunctor" in name:
        return "reference multiply"
    base = name.split("(")[0].strip()
    if base.startswith("void "):
        base = base[5:]
    base = base.replace("abdf::", "")
    return base[:48]


def counters(path):
    per = {}
    with open(os.path.join(path, "run_counter_collection.csv")) as fh:
        for row in csv.DictReader(fh):
            k = short(row["Kernel_Name"])
            v = float(row["Counter_Value"])
            n, s = per.get(k, (0, 0.0))
            per[k] = (n + 1, s + v)
    return per


def markers(mdir, command):
    """Host ranges of the library (count, total and mean duration) from a
    rocprofv3 --marker-trace run."""
    rows = list(csv.DictReader(open(os.path.join(mdir, "run_marker_api_trace.csv"))))
    agg = {}
    for r in rows:
        name = r.get("Function") or r.get("Name") or ""
        if not name.startswith("abdf"):
            continue
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        n, tot = agg.get(name, (0, 0.0))
        agg[name] = (n + 1, tot + dt)
    out = ["# Host ranges of the library (rocprofv3 --marker-trace): 500-species network, 4096 cells, FP64", "",
           "Command (repo root, on one MI355X):", "", "    " + command, "",
           "| range | count | total ms | mean us |", "|---|---|---|---|"]
    for name, (n, tot) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| {name} | {n} | {tot:.1f} | {1e3 * tot / n:.1f} |")
    open(os.path.join(PROFILES, "markers_net500.md"), "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def mfma(mdir, mlog, command):
    """Per-kernel MFMA counters: executed FP64 MFMA work (SQ_INSTS_VALU_MFMA_MOPS_F64
    counts 512 flops each) per factorisation against the algorithmic 2/3 n^3,
    and MFMA busy cycles against CU busy cycles."""
    agg, calls = {}, {}
    for r in csv.DictReader(open(os.path.join(mdir, "run_counter_collection.csv"))):
        k = short(r["Kernel_Name"])
        d = agg.setdefault(k, {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        if r["Counter_Name"] == "SQ_BUSY_CU_CYCLES":
            calls[k] = calls.get(k, 0) + 1
    line = json.loads([l for l in open(mlog) if l.startswith("{")][-1])
    n_lu = line["work"]["factorisations"]
    S = line["config"]["species"]
    out = ["# MFMA counters: 500-species / 6000-reaction network, 512 cells, FP64", "",
           "Command (repo root, on one MI355X):", "", "    " + command, "",
           "| kernel | dispatches | SQ_INSTS_VALU_MFMA_MOPS_F64 | SQ_VALU_MFMA_BUSY_CYCLES | SQ_BUSY_CU_CYCLES | "
           "SQ_WAVE_CYCLES |", "|---|---|---|---|---|---|"]
    for k, d in sorted(agg.items(), key=lambda kv: -kv[1].get("SQ_BUSY_CU_CYCLES", 0.0)):
        if d.get("SQ_BUSY_CU_CYCLES", 0.0) < 1e6:
            continue
        out.append(f"| {k} | {calls.get(k, 0)} | {d.get('SQ_INSTS_VALU_MFMA_MOPS_F64', 0):.4g} | "
                   f"{d.get('SQ_VALU_MFMA_BUSY_CYCLES', 0):.4g} | {d.get('SQ_BUSY_CU_CYCLES', 0):.4g} | "
                   f"{d.get('SQ_WAVE_CYCLES', 0):.4g} |")
    f = agg.get("k_factor<double>", {})
    executed = f.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512 / max(1, n_lu)
    out += ["", f"k_factor<double>: {n_lu} factorisations; MFMA work executed per factorisation "
                f"{executed:.4g} flop (MOPS x 512) against the algorithmic 2/3 n^3 = {2 / 3 * S ** 3:.4g} "
                f"({executed / (2 / 3 * S ** 3):.3f}x: the padding to 512 rows and the diagonal-block inverses).",
            f"MFMA busy / CU busy cycles: {f.get('SQ_VALU_MFMA_BUSY_CYCLES', 0) / max(1, f.get('SQ_BUSY_CU_CYCLES', 1)):.3f}"
            " (both summed over the device as the counters report them)."]
    open(os.path.join(PROFILES, "mfma_net500.md"), "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def trace_table(tdir, log, name, title, command):
    rows = list(csv.DictReader(open(os.path.join(tdir, "run_kernel_stats.csv"))))
    line = json.loads([l for l in open(log) if l.startswith("{")][-1])
    out = [f"# {title}", "", "Command (repo root, on one MI355X):", "", "    " + command, "",
           "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in rows:
        if float(r["Percentage"]) < 0.01:
            continue
        out.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs'])/1e6:.1f} | "
                   f"{float(r['AverageNs'])/1e3:.1f} | {float(r['Percentage']):.2f} |")
    out += ["", f"Bench line of the run: {line['value']} {line['unit']}, {line['ms_per_step']} ms per solve; "
                f"work {json.dumps(line['work'])}."]
    if "roofline_rhs" in line:
        rr = line["roofline_rhs"]
        out.append(f"Standalone right-hand side ({rr['kernel'].split()[0]}): {rr['achieved']} GB/s of algorithmic traffic "
                   f"({rr['work']}), {rr['avg_launch_ms']} ms per launch over {rr['cells']} cells.")
    open(os.path.join(PROFILES, name + ".md"), "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def main():
    if sys.argv[1] == "--markers":
        markers(sys.argv[2], sys.argv[3])
        return
    if sys.argv[1] == "--mfma":
        mfma(sys.argv[2], sys.argv[3], sys.argv[4])
        return
    if sys.argv[1] == "--trace":
        trace_table(*sys.argv[2:7])
        return
    trace, fetch, write, flog = sys.argv[1:5]
    rows = list(csv.DictReader(open(os.path.join(trace, "run_kernel_stats.csv"))))
    out = ["# rocprofv3 kernel statistics: 500-species / 6000-reaction network, 4096 cells, FP64", "",
           "Command (repo root, on one MI355X):", "",
           "    rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- "
           "python3 bench.py --cells 4096 --steps 1 --warmup 0 --no-cpu-baseline --no-compare-fp32 "
           "--no-compare-reuse --no-compare-esdirk --batch-serve-requests 0", "",
           "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in rows:
        if float(r["Percentage"]) < 0.01:
            continue
        out.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs'])/1e6:.1f} | "
                   f"{float(r['AverageNs'])/1e3:.1f} | {float(r['Percentage']):.2f} |")
    # per hardware queue: the solver's stream and the side stream of the
    # Newton iterations that run beside the factorisation
    trace_rows = list(csv.DictReader(open(os.path.join(trace, "run_kernel_trace.csv"))))
    perq = {}
    spans = []
    for r in trace_rows:
        k = short(r["Kernel_Name"])
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        spans.append((t0, t1))
        key = (k, r["Queue_Id"])
        n, tot = perq.get(key, (0, 0))
        perq[key] = (n + 1, tot + (t1 - t0))
    spans.sort()
    busy, cs, ce = 0, None, None
    for a, b in spans:
        if ce is None or a > ce:
            if ce is not None:
                busy += ce - cs
            cs, ce = a, b
        else:
            ce = max(ce, b)
    if ce is not None:
        busy += ce - cs
    out += ["", "Per hardware queue (kernel trace).  Kernels on the second queue are the Newton "
            "iterations of cells whose factorisation is current; they are launched beside k_factor "
            "and their spans include the time their workgroups wait for compute units that "
            "k_factor holds, so their totals overlap the factorisation's.", "",
            "| kernel | queue | calls | total ms | average us |", "|---|---|---|---|---|"]
    for (k, q), (n, tot) in sorted(perq.items(), key=lambda kv: -kv[1][1]):
        if tot < 1e6:
            continue
        out.append(f"| {k} | {q} | {n} | {tot / 1e6:.1f} | {tot / n / 1e3:.1f} |")
    out += ["", f"GPU busy (union of all kernel spans): {busy / 1e6:.1f} ms, of which k_factor "
                f"{sum(t for (k, q), (n, t) in perq.items() if k.startswith('k_factor')) / 1e6:.1f} ms."]
    if len(sys.argv) > 5:
        tl = json.loads([l for l in open(sys.argv[5]) if l.startswith("{")][-1])
        out += ["", f"Bench line of the traced run: {tl['value']} {tl['unit']}, {tl['ms_per_step']} ms per solve, "
                    f"work {json.dumps(tl['work'])}."]
        if "roofline_rhs" in tl:
            rr = tl["roofline_rhs"]
            name = rr["kernel"].split()[0]
            runs = [(n, t) for (k, q), (n, t) in perq.items() if k.startswith(name)]
            n_rhs, t_rhs = (sum(n for n, t in runs), sum(t for n, t in runs)) if runs else (0, 0)
            per_cell = float(rr["work"].split("=")[1].split("B")[0])
            if n_rhs:
                us = t_rhs / n_rhs / 1e3
                gbs = per_cell * rr["cells"] / (us * 1e-6) / 1e9
                out.append(f"Standalone right-hand side ({name}, the {n_rhs} launches above): {us:.1f} us per launch "
                           f"over {rr['cells']} cells by the kernel trace, {gbs:.1f} GB/s of algorithmic traffic "
                           f"({rr['work']}), {gbs / 8000.0:.4f} of 8 TB/s.  The same run's events recorded by each "
                           f"dispatch give {rr['avg_launch_ms']} ms per launch ({rr['achieved']} GB/s): under the "
                           f"profiler they include its dispatch overhead; without it they agree with the trace.")
    f = counters(fetch)
    w = counters(write)
    cf = COPY_BYTES / (f["reference multiply"][1] * 1024.0)
    cw = COPY_BYTES / (w["reference multiply"][1] * 1024.0)
    line = [l for l in open(flog) if l.startswith("{")][-1]
    work = json.loads(line)["work"]
    out += ["", "## HBM traffic (FETCH_SIZE, WRITE_SIZE; 512 cells, one solve)", "",
            "Commands: the bench command above with --cells 512 --calibrate-copy under "
            "`rocprofv3 --pmc FETCH_SIZE` and, separately, `rocprofv3 --pmc WRITE_SIZE`.", "",
            f"Calibration: an elementwise multiply reading and writing 256 MiB reads "
            f"{f['reference multiply'][1]/1024:.1f} MiB by FETCH_SIZE (scale {cf:.3f}) and writes "
            f"{w['reference multiply'][1]/1024:.1f} MiB by WRITE_SIZE (scale {cw:.3f}).", "",
            "| kernel | dispatches | fetched MiB (scaled) | written MiB (scaled) |", "|---|---|---|---|"]
    traffic = {}
    for k in sorted(set(f) | set(w)):
        fb = f.get(k, (0, 0.0))[1] * 1024 * cf
        wb = w.get(k, (0, 0.0))[1] * 1024 * cw
        out.append(f"| {k} | {f.get(k, (0, 0))[0]} | {fb/2**20:.1f} | {wb/2**20:.1f} |")
        traffic[k] = fb + wb
    per_lu = traffic.get("k_factor<double>", 0.0) / max(1, work["factorisations"])
    per_it = sum(v for k, v in traffic.items() if k.startswith("k_newton_solve<double")) / \
        max(1, work["newton_iterations"])
    out += ["", f"Per factorisation (k_factor, assembly + LU): {per_lu/2**20:.2f} MiB of HBM traffic; "
                f"per Newton solve (k_newton_solve): {per_it/2**20:.3f} MiB."]
    rec = {"source_hash": source_hash(), "network": "net500", "k_factor_bytes_per_lu": per_lu,
           "k_newton_solve_bytes_per_iteration": per_it}
    # the standalone right-hand side: its launches cover the run's whole batch
    cells = json.loads(line)["config"]["cells"]
    rhs = [(k, n) for k, (n, _) in f.items() if k.startswith("k_rhs_stream") or k.startswith("k_rhs_only")]
    if rhs:
        k, n = rhs[0]
        per_cell = traffic[k] / (n * cells)
        rec["k_rhs_bytes_per_cell"] = per_cell
        out.append(f"Standalone right-hand side ({k}): {per_cell / 1e3:.1f} kB of HBM traffic per cell-evaluation "
                   f"({n} launches over {cells} cells).")
    open(os.path.join(PROFILES, "kernel_stats_net500.md"), "w").write("\n".join(out) + "\n")
    json.dump(rec, open(os.path.join(PROFILES, "traffic.json"), "w"), indent=1)
    print("\n".join(out))


if __name__ == "__main__":
    main()
