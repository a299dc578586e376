"""Summaries of the rocprofv3 runs behind bench.py's roofline fields.

Reads the outputs of the commands below (run from the repository root on an
MI355X) and writes, under profiles/:

* sample_kernel_mixed16_trace.md: kernel statistics and the sampler
  dispatches of one bench step (kernel trace), next to bench.py's own
  event-timed duration of the dominant launch in the same run;
* terms_kernel_differentiation_trace.md: the differentiable form's kernels
  from the same trace;
* sample_kernel_mixed16_counters.md and traffic.json: hardware counters of
  every MC-step launch from two counter runs, with FETCH_SIZE / WRITE_SIZE
  scaled by what the same counters read for a plain device copy of known
  size in the same run.  traffic.json carries a SHA-256 of the library
  sources; bench.py uses it only while the sources hash the same.

    python bench_profiles.py --runs OUT [--out profiles]

OUT is the folder the runs wrote to (`<out>` in the commands).
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sqlite3

ROOT = os.path.dirname(os.path.abspath(__file__))
SIMDS, CUS, CLK = 1024, 256, 2.4e9
COPY_KIB = 262144.0          # the calibration copy: 256 MiB each way
N_BUCKET_LAUNCHES = 6        # MC-step launches of the mixed-pocket step (one per lane bucket)

CMD_INPUTS = ("python bench.py --inputs /tmp/c5.pkl --steps 1 --warmup 0 --no-plain --no-cpu-baseline "
              "--no-extras")
CMD_TRACE = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d <out>/prof_trace "
             "-o trace -- python3 <repo>/bench.py --inputs /tmp/c5.pkl --workers 1 --steps 1 --warmup 0 "
             "--no-plain --no-cpu-baseline --extras-only differentiation --out <out>/prof_trace_bench.json")
PMC_A = ("FETCH_SIZE SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_LDS SQ_INSTS_SALU "
         "SQ_INSTS_VMEM_RD SQ_WAVES")
PMC_B = ("WRITE_SIZE TCC_HIT_sum TCC_REQ_sum SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_LDS SQ_LDS_IDX_ACTIVE "
         "SQ_WAIT_INST_LDS SQ_INSTS_VALU")


def cmd_pmc(counters, d):
    return ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc %s --output-format csv -d <out>/%s -o pmc "
            "-- python3 <repo>/bench.py --inputs /tmp/c5.pkl --workers 1 --steps 1 --warmup 0 --no-plain "
            "--no-cpu-baseline --no-extras --calib-copy-mib 256" % (counters, d))


def short(name):
    return name.replace("void ", "").replace("dock::", "").split("(")[0]


def source_sha256():
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2510_24186_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def trace_summaries(runs, out):
    db = sqlite3.connect(os.path.join(runs, "prof_trace", "trace_results.db"))
    with open(os.path.join(runs, "prof_trace_bench.json")) as f:
        bench = json.load(f)
    rows = list(db.execute("select name, grid_x, workgroup_x, duration, lds_size, scratch_size, start "
                           "from kernels order by start"))
    stats = {}
    for n, g, wg, dur, lds, scr, st in rows:
        s = stats.setdefault(short(n), [0, 0.0])
        s[0] += 1
        s[1] += dur / 1e6
    lines = ["# Kernel trace: the mixed-pocket workload (one step) and the differentiation workload", "",
             "Commands (repo root = <repo>, run outputs in <out>; the first, unprofiled, draws the inputs and saves them; "
             "`python bench_profiles.py` wrote this file):", "",
             "    " + CMD_INPUTS, "    " + CMD_TRACE, "",
             "One step: 16 map rebuilds, the batched sampler over 65,536 ligands (64 trajectories x 200 MC steps x",
             "10 Adam steps, 9.23 G evaluations) as six lane-bucket launches on concurrent streams, grouped by",
             "occupancy class, best poses, and",
             "the deterministic adjoint of the summed best-pose energies to every pocket's maps and weights; then",
             "the differentiation workload (2,048 poses, Vina-form terms) forward and adjoint, twice.", "",
             "## Kernel statistics (from the run's kernel dispatch records; durations in ms)", "",
             "| Kernel | Calls | Total ms | Average ms |", "|---|---|---|---|"]
    for k, (c, t) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        if t >= 0.01:
            lines.append("| `%s` | %d | %.3f | %.3f |" % (k, c, t, t / c))
    lines += ["", "## Sampler dispatches (grid = blocks x 256 threads)", "",
              "| Kernel | Grid (threads) | LDS bytes | Scratch bytes/lane | Duration ms |", "|---|---|---|---|---|"]
    for n, g, wg, dur, lds, scr, st in rows:
        if "sample_kernel" in n:
            lines.append("| `%s` | %d | %d | %d | %.3f |" % (short(n), g, lds, scr, dur / 1e6))
    dom = bench["roofline"]
    key = "sample_kernel<%s, %s, 256" % tuple(dom["kernel"].split("<")[1].split(",")[:2])
    grid_threads = [b["grid"] for b in dom["buckets"] if abs(b["ms"] - dom["launch_ms"]) < 1e-3][0] * 256
    dom_trace = [d for n, g, wg, d, lds, scr, st in rows if key in short(n) and g == grid_threads][-1] / 1e6
    lines += ["", "The first six dispatches draw and score the initial poses; the next six are the MC-step "
              "launches of", "the six buckets, concurrent within each occupancy class (three blocks per CU, "
              "then two).  The dominant", "launch (most algorithmic work) is", "`%s, 0>` with grid %d threads: %.3f ms here;" % (key, grid_threads, dom_trace),
              "bench.py measured the same launch with HIP events on its stream as %.3f ms (`roofline.launch_ms`)."
              % dom["launch_ms"], "",
              "Same run, bench line: value %.1f M evals/s, dominant launch %.3f TFLOP/s = %.4f of 157.3." % (
                  bench["value"] / 1e6, dom["achieved"], dom["frac"]), ""]
    with open(os.path.join(out, "sample_kernel_mixed16_trace.md"), "w") as f:
        f.write("\n".join(lines))
    terms = [(short(n), g, dur / 1e6) for n, g, wg, dur, lds, scr, st in rows if "terms_kernel" in n or "adj_" in n]
    tl = ["# Kernel trace: the differentiable form (terms_kernel and the deterministic adjoint's helpers)", "",
          "From the same rocprofv3 run as sample_kernel_mixed16_trace.md:", "", "    " + CMD_TRACE, "",
          "* `terms_kernel<64, 2, 3, false>`: the adjoint over the 65,536 best poses of the mixed-pocket step "
          "(TRIDS,", "  16 pockets, deterministic: 64-bit fixed-point dL/dG).",
          "* `terms_kernel<64, 1, 5, false>`: the differentiation workload (2,048 poses, Vina-form terms, "
          "64^3 x 8 x 5", "  maps): forward, adjoint with float atomics, adjoint deterministic, twice.", "",
          "| Kernel | Grid (threads) | Duration ms |", "|---|---|---|"]
    for k, g, d in terms:
        tl.append("| `%s` | %d | %.3f |" % (k, g, d))
    tl += ["", "bench.py, same run (`extras.differentiation`, event times of the whole calls): %s" % json.dumps(
        bench["extras"]["differentiation"]), ""]
    with open(os.path.join(out, "terms_kernel_differentiation_trace.md"), "w") as f:
        f.write("\n".join(tl))
    return dom_trace, dom["launch_ms"]


def load_counters(path):
    """Counter values per dispatch of one rocprofv3 --pmc CSV (instances summed)."""
    disp = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = disp.setdefault(int(r["Dispatch_Id"]), dict(
                name=short(r["Kernel_Name"]), grid=int(r["Grid_Size"]),
                dur_ms=(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6))
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return disp


def calibration(A, B):
    """FETCH_SIZE and WRITE_SIZE factors from the calibration copy.  The
    step copies other buffers too; the calibration copy is the first copy
    dispatch of run B whose WRITE_SIZE is within 1 % of the bytes it writes,
    and the dispatch with the same id in run A (same program, same order)."""
    ids = sorted(i for i, d in B.items()
                 if "copyBuffer" in d["name"] and abs(d.get("WRITE_SIZE", 0.0) - COPY_KIB) <= 0.01 * COPY_KIB)
    if not ids or "copyBuffer" not in A.get(ids[0], {}).get("name", ""):
        raise SystemExit("no calibration copy found (run bench.py with --calib-copy-mib 256)")
    copy_a, copy_b = A[ids[0]], B[ids[0]]
    return COPY_KIB / copy_a["FETCH_SIZE"], COPY_KIB / copy_b["WRITE_SIZE"], copy_a["FETCH_SIZE"], copy_b["WRITE_SIZE"]


def launch_records(A, B, cal_f, cal_w):
    """Per MC-step launch (the longest sampler dispatches of run A, each
    matched with run B's dispatch of the same kernel and grid): derived
    figures keyed "lanes,atoms per lane,block,grid blocks"."""
    sa = sorted((d for d in A.values() if "sample_kernel" in d["name"]), key=lambda d: -d["dur_ms"])
    sb = [d for d in B.values() if "sample_kernel" in d["name"]]
    recs = []
    for da in sa[:N_BUCKET_LAUNCHES]:
        db_ = min((d for d in sb if d["name"] == da["name"] and d["grid"] == da["grid"]),
                  key=lambda d: abs(d["dur_ms"] - da["dur_ms"]))
        ms = da["dur_ms"]
        lanes, apl = [int(x) for x in da["name"].split("<")[1].split(",")[:2]]
        rec = dict(
            fetch_kib=da["FETCH_SIZE"], write_kib=db_["WRITE_SIZE"],
            hbm_bytes=da["FETCH_SIZE"] * 1024 * cal_f + db_["WRITE_SIZE"] * 1024 * cal_w,
            l2_req=db_["TCC_REQ_sum"], l2_hit=round(db_["TCC_HIT_sum"] / max(1.0, db_["TCC_REQ_sum"]), 4),
            valu_busy=round(da["SQ_INSTS_VALU"] * 4 / (ms * 1e-3 * CLK * SIMDS), 3),
            lds_busy=round(db_["SQ_LDS_IDX_ACTIVE"] / (db_["dur_ms"] * 1e-3 * CLK * CUS), 3),
            bank_conflict=round(db_["SQ_LDS_BANK_CONFLICT"] / max(1.0, db_["SQ_LDS_IDX_ACTIVE"]), 3),
            valu_instr=da["SQ_INSTS_VALU"], ms=ms)
        recs.append(("%d,%d,256,%d" % (lanes, apl, da["grid"] // 256), da, db_, rec))
    return recs


def counter_summaries(runs, out):
    A = load_counters(os.path.join(runs, "pmc_a", "pmc_counter_collection.csv"))
    B = load_counters(os.path.join(runs, "pmc_b", "pmc_counter_collection.csv"))
    cal_f, cal_w, copy_f, copy_w = calibration(A, B)
    recs = launch_records(A, B, cal_f, cal_w)
    cl = ["# sample_kernel on the mixed-pocket workload: hardware counters", "",
          "Two rocprofv3 counter runs (one MC step of the bench; counter runs serialise the launches, so the",
          "durations below are each launch alone), with a 256 MiB device copy in the same run as calibration",
          "(`python bench_profiles.py` wrote this file and traffic.json):", "",
          "    " + CMD_INPUTS, "    " + cmd_pmc(PMC_A, "pmc_a"), "    " + cmd_pmc(PMC_B, "pmc_b"), "",
          "Calibration: the copy moves 262,144 KiB each way and reads FETCH_SIZE = %.0f KiB, WRITE_SIZE = %.0f KiB:"
          % (copy_f, copy_w),
          "factors %.3f (fetch) and %.3f (write).  Values are summed over the counter instances of each dispatch."
          % (cal_f, cal_w), "",
          "Derived: VALU busy = SQ_INSTS_VALU x 4 cycles / (duration x 2.4 GHz x 1,024 SIMDs); LDS busy =",
          "SQ_LDS_IDX_ACTIVE / (duration x 2.4 GHz x 256 CUs); bank-conflict share = SQ_LDS_BANK_CONFLICT /",
          "SQ_LDS_IDX_ACTIVE; L2 hit = TCC_HIT_sum / TCC_REQ_sum; L2 GB/s = TCC_REQ_sum x 128 B / duration;",
          "fabric (HBM or Infinity Cache) bytes = FETCH_SIZE x %.3f + WRITE_SIZE x %.3f." % (cal_f, cal_w), "",
          "| MC-step launch | grid | ms alone | VALU instr | VALU busy | LDS busy | bank conflicts | L2 hit | "
          "L2 GB/s | fabric GB | fabric GB/s |",
          "|---|---|---|---|---|---|---|---|---|---|---|"]
    for key, da, db_, r in recs:
        ms = r["ms"]
        cl.append("| `%s` | %d | %.1f | %.3g | %.0f %% | %.0f %% | %.0f %% | %.1f %% | %.0f | %.1f | %.1f |" % (
            da["name"], da["grid"], ms, r["valu_instr"], 100 * r["valu_busy"], 100 * r["lds_busy"],
            100 * r["bank_conflict"], 100 * r["l2_hit"], r["l2_req"] * 128 / (db_["dur_ms"] * 1e-3) / 1e9,
            r["hbm_bytes"] / 1e9, r["hbm_bytes"] / (ms * 1e-3) / 1e9))
    cl += ["", "Raw counters of the MC-step launches:", ""]
    for key, da, db_, r in recs:
        cl.append("## %s, grid %d (%.1f ms alone)" % (da["name"], da["grid"], da["dur_ms"]))
        for k in sorted(set(da) | set(db_)):
            if k not in ("name", "grid", "dur_ms"):
                cl.append("    %-22s %.6g" % (k, da.get(k, db_.get(k))))
        cl.append("")
    with open(os.path.join(out, "sample_kernel_mixed16_counters.md"), "w") as f:
        f.write("\n".join(cl))
    traffic = dict(source_sha256=source_sha256(), fetch_calibration=cal_f, write_calibration=cal_w,
                   copy_mib=256, copy_fetch_kib=copy_f, copy_write_kib=copy_w,
                   note="per MC-step launch of each sampler bucket; key lanes,atoms per lane,block,grid blocks",
                   workloads={"C5": {key: r for key, da, db_, r in recs}})
    with open(os.path.join(out, "traffic.json"), "w") as f:
        json.dump(traffic, f, indent=1)
    return traffic


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", required=True, help="folder holding the runs' outputs (<out> in the commands)")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    args = ap.parse_args()
    tr, ev = trace_summaries(args.runs, args.out)
    print("dominant launch: %.3f ms in the trace, %.3f ms by bench.py's events" % (tr, ev))
    t = counter_summaries(args.runs, args.out)
    for k, r in t["workloads"]["C5"].items():
        print("%-16s %9.1f ms  fabric %.1f GB  VALU %.0f %%" % (k, r["ms"], r["hbm_bytes"] / 1e9, 100 * r["valu_busy"]))


if __name__ == "__main__":
    main()
