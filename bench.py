"""Benchmark: pass-efficient randomized truncated QSVD on one MI355X.

Headline workload (the largest single-GPU configuration): a dense 16384 x 16384 quaternion FP32
matrix A = U diag(sigma) V^H with sigma_i = i^-1/2 and unitaries that are products of 8 random
quaternion Householder reflectors and a unit-quaternion diagonal (synthetic, seeded, built on the
host by workloads.config4), block Krylov scheme (Alg. 4) with k = 128, p = 32 and a budget of
v = 8 views: seven views 160 columns wide, the Krylov stack of 640 columns, the last view 640
wide, CholeskyQR after every view, the final QSVD and the back-multiplication, with per-pass
error estimates.  One step = one such solve (8 passes over A); value = passes / second of the
plain FP32 path (v / end-to-end solve time).

Printed: one JSON line with
- value (FP32 A-passes/s) and the same for the reduced-precision forms (BF16 views 1..6 with FP32
  views 7 and 8, and the BF16 split form of views 7 and 8), each with its error
  ||A - U S V^H||_F / ||A||_F computed directly on the device in FP64 and its ratio to the FP64
  oracle's error on the same A and sketch (the oracle's solve of this A is stored in
  tests/golden/, written by a script that calls only the oracle), and the sampled distance of
  U diag(S) V^H from the oracle's;
- the roofline position of the dominant kernel (the FP32 view product, 16384 x 16384 by 160
  columns, timed with HIP events on its own stream) and of every other view kernel the solve
  runs (FP32 at 640 columns, BF16 at 160, BF16 split at 640);
- the FP64 CPU oracle timed on the host (single thread and all cores) on a bounded sample of
  the same workload, as a baseline;
- secondary records: the 2048 x 2048 subspace workload (budgets 2, 3, 4, 6), the serving stream
  and the matrix-completion workloads.
"""
import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12
PEAK_BF16_MFMA = 2516.6e12
PEAK_HBM = 8.0e12
SIMDS = 256 * 4
XCDS = 8

# the headline: 16384 x 16384, block Krylov, k = 128, p = 32, v = 8, sketch seed 11
LN, LK, LP, LV, LSEED = 16384, 128, 32, 8, 11
LL = LK + LP
LW = (LV // 2) * LL            # width of the Krylov stack and of the last view (even v)
GOLDEN = os.path.join(ROOT, "tests", "golden", "config4_krylov_k128_p32_v8_seed11.json")
PMC_FILE = os.path.join(ROOT, "profiles", "qgemm_f32_view_16384x16384x160_pmc.json")
PMC_FILE_LOWP = os.path.join(ROOT, "profiles", "qgemm_bf16_view_16384x16384x160_pmc.json")
TRACE_FILE = os.path.join(ROOT, "profiles", "solve_16384x16384_krylov_k128_p32_v8_trace.md")

# secondary: 2048 x 2048, sigma_i = exp(-i/20) + noise, subspace k = 50, p = 10, budgets 2, 3, 4, 6
M1 = N1 = 2048
K1, P1 = 50, 10
BUDGETS1 = (2, 3, 4, 6)
SEED_DATA1, SEED_SKETCH1 = 1, 1

# server slots: one per hardware queue HIP gives a process by default (measured with 256
# requests: 1861 req/s closed loop with 4 slots, 1508 with 8, 1444 with 16)
SERVE_SLOTS = 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=5)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-completion", action="store_true")
    ap.add_argument("--no-config1", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="only the 16384 x 16384 solves (timed steps, accuracy, view kernels); for a kernel trace")
    ap.add_argument("--only-completion", action="store_true",
                    help="run only the matrix-completion workloads (for a kernel trace) and print their record")
    ap.add_argument("--counters", action="store_true",
                    help="launch sequence for hardware-counter runs only (view products and calibration copies)")
    ap.add_argument("--trace-summary", nargs="+", metavar="FILE",
                    help="kernel trace CSV of a rocprofv3 --kernel-trace run of the default bench (then, optionally, "
                         "that run's output): writes the per-kernel summary of the headline solves under profiles/")
    ap.add_argument("--counters-lowp", action="store_true",
                    help="the same launch sequence with the BF16 view products (from the solve's copies of A)")
    ap.add_argument("--pmc-summary-lowp", nargs="+", metavar="CSV",
                    help="as --pmc-summary, for three --counters-lowp runs: writes the BF16 view's record")
    ap.add_argument("--pmc-summary", nargs="+", metavar="CSV",
                    help="FETCH_SIZE and WRITE_SIZE CSVs of two --counters runs (then optional MFMA counter "
                         "CSVs): writes the traffic record under profiles/")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_2507_13731_amd", "csrc", "qgemm.hip"), "rb").read())
    return h.hexdigest()[:16]


def host_cores():
    return len(os.sched_getaffinity(0))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def headline_matrix(torch):
    """The 16384 x 16384 matrix on the host (bitwise reproducible), checked against the hash the
    stored oracle solve was made on, then uploaded."""
    import workloads as W
    log(f"building the {LN}x{LN} matrix on the host")
    t0 = time.perf_counter()
    A32, sigma = W.config4(threads=min(16, host_cores()))
    golden = json.load(open(GOLDEN)) if os.path.exists(GOLDEN) else None
    sha = hashlib.sha256(A32.tobytes()).hexdigest()
    same = golden is not None and golden["sha256"] == sha
    log(f"  built in {time.perf_counter() - t0:.1f} s; matches the oracle's input: {same}")
    A = torch.from_numpy(A32).cuda()
    torch.cuda.synchronize()
    return A, A32, sigma, (golden if same else None)


COPY_BYTES = 256 << 20
COUNTER_REPS = 3
COUNTER_OPS = ((0, LL, "forward"), (1, LL, "adjoint"))


def counters_run(Q, torch, A, lowp=False):
    """The launch sequence the hardware counters are read on: COUNTER_REPS forward and adjoint
    view products (16384 x 16384 by 160; FP32, or BF16 from the solve's copies of A with lowp),
    then COUNTER_REPS elementwise passes over 256 MiB (read once, written once) whose counter
    readings calibrate the scale of FETCH_SIZE and WRITE_SIZE."""
    g = torch.Generator(device="cuda").manual_seed(0)
    copies = Q.qlra_lowp_copy(A, Q.QLRA_BF16) if lowp else None
    torch.cuda.synchronize()
    for op, w, _ in COUNTER_OPS:
        X = torch.randn((4, LN, w), device="cuda", generator=g)
        if lowp:
            ws = Q.qlra_qgemm_lp_workspace(op, Q.QLRA_BF16, LN, LN, w)
        else:
            ws = Q.qlra_qgemm_workspace(op, LN, LN, w)
        C = torch.empty((4, LN, w), device="cuda")
        for _ in range(COUNTER_REPS):
            if lowp:
                Q.qlra_qgemm_lp(op, Q.QLRA_BF16, copies[op], LN, LN, X, C, stream=torch.cuda.current_stream(),
                                workspace=ws)
            else:
                Q.qlra_qgemm(op, A, X, C, stream=torch.cuda.current_stream(), workspace=ws)
            torch.cuda.synchronize()
    src = torch.ones(COPY_BYTES // 4, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(COUNTER_REPS):
        torch.neg(src, out=dst)            # an elementwise kernel: reads and writes COPY_BYTES
        torch.cuda.synchronize()
    print(json.dumps({"counters_run": "done", "view_launches_per_op": COUNTER_REPS, "copy_bytes": COPY_BYTES}))


def _read_counter_csv(path):
    """{counter: [(dispatch, kernel, value, duration_ns)]} in dispatch order: a counter's rows of
    one dispatch summed (per-SE and per-channel instances), GRBM counters maximised."""
    import csv
    rows = {}
    for r in csv.DictReader(open(path)):
        key = (r["Counter_Name"], int(r["Dispatch_Id"]))
        v = float(r["Counter_Value"])
        dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        old = rows.get(key, ("", None, 0))[1]
        if old is None:
            new = v
        elif r["Counter_Name"].startswith("GRBM"):
            new = max(old, v)
        else:
            new = old + v
        rows[key] = (r["Kernel_Name"], new, dur)
    out = {}
    for (cn, d), (kn, v, dur) in sorted(rows.items(), key=lambda t: t[0][1]):
        out.setdefault(cn, []).append((d, kn, v, dur))
    return out


def pmc_summary(paths, lowp=False):
    """Per-dispatch counters from rocprofv3 --pmc runs of --counters (CSV output): FETCH_SIZE
    and WRITE_SIZE (KiB; the elementwise pass's readings give the factor that turns each into
    bytes), and any further counters (MFMA activity) per view kernel.  lowp: the runs of
    --counters-lowp (BF16 views), written to their own record."""
    import statistics
    view_kernels = ("k_lp_thin", "k_qgemm_lp", "k_splitk_reduce") if lowp else ("k_thin_t", "k_qview", "k_splitk_reduce")
    product = "k_qgemm_lp" if lowp else "k_qview"
    out = {}
    extra = {}
    for path in paths:
        for counter, seq in _read_counter_csv(path).items():
            view = [(n, v, t) for _, n, v, t in seq if any(k in n for k in view_kernels)]
            nper = len(view) // len(COUNTER_OPS)
            if counter in ("FETCH_SIZE", "WRITE_SIZE"):
                copies = [v for _, _, v, _ in seq[-COUNTER_REPS:]]  # the calibration copies end the sequence
                kib_copy = statistics.median(copies)
                scale = COPY_BYTES / (kib_copy * 1024.0)
                per_op = {}
                for i, (_, w, name) in enumerate(COUNTER_OPS):
                    part = view[i * nper:(i + 1) * nper]
                    kib = sum(v for _, v, _ in part) / COUNTER_REPS
                    per_op[name] = {"kib_per_launch": round(kib, 1), "bytes_per_launch": round(kib * 1024.0 * scale),
                                    "kernels": sorted({re.search(r"k_\w+", n).group(0) for n, _, _ in part})}
                out[counter] = {"copy_kib": round(kib_copy, 1), "scale": round(scale, 4), **per_op}
            else:
                per_op, dur_op = {}, {}
                for i, (_, w, name) in enumerate(COUNTER_OPS):
                    part = [(n, v, t) for n, v, t in view[i * nper:(i + 1) * nper] if product in n]
                    per_op[name] = round(sum(v for _, v, _ in part) / max(1, len(part)), 1)
                    dur_op[name] = round(sum(t for _, _, t in part) / max(1, len(part)))
                extra[counter] = {"per_product_kernel_launch": per_op, "duration_ns": dur_op}
    hbm = 0.5 * sum(out[c][o]["bytes_per_launch"] for c in ("FETCH_SIZE", "WRITE_SIZE") for _, _, o in COUNTER_OPS)
    # MFMA activity of the product kernel: busy cycles over (active cycles x SIMDs), and the FLOPs
    # the MFMA pipes executed (512 per MOPS unit) against the algorithmic 32 m n w.  GRBM_GUI_ACTIVE
    # reads as the sum over the XCDs (it is about XCDS x the dispatch's duration x the clock), so
    # one XCD's active cycles are a XCDS-th of it; the implied clock is recorded as the check.
    mfma = {}
    if "SQ_VALU_MFMA_BUSY_CYCLES" in extra and "GRBM_GUI_ACTIVE" in extra:
        for _, w, name in COUNTER_OPS:
            busy = extra["SQ_VALU_MFMA_BUSY_CYCLES"]["per_product_kernel_launch"][name]
            act = extra["GRBM_GUI_ACTIVE"]["per_product_kernel_launch"][name] / XCDS
            dur = extra["GRBM_GUI_ACTIVE"]["duration_ns"][name]
            rec_op = {"mfma_busy_frac": round(busy / (act * SIMDS), 4), "active_cycles_per_xcd": round(act),
                      "dispatch_ns": dur, "implied_clock_ghz": round(act / dur, 3) if dur else None}
            mops = "SQ_INSTS_VALU_MFMA_MOPS_BF16" if lowp else "SQ_INSTS_VALU_MFMA_MOPS_F32"
            if mops in extra:
                fl = 512.0 * extra[mops]["per_product_kernel_launch"][name]
                rec_op["mfma_flops"] = fl
                rec_op["mfma_flops_over_algorithmic"] = round(fl / (32.0 * LN * LN * w), 4)
            if dur:
                rec_op["tflops_at_dispatch_duration"] = round(32.0 * LN * LN * w / dur / 1e3, 1)
            mfma[name] = rec_op
    mode, tag, mops = ("--counters-lowp", "lp", "SQ_INSTS_VALU_MFMA_MOPS_BF16") if lowp else \
        ("--counters", "", "SQ_INSTS_VALU_MFMA_MOPS_F32")
    what = "BF16 view product (k_lp_thin + k_qgemm_lp)" if lowp else "FP32 view product"
    rec = {"kernel": f"{what} {LN}x{LN} by {LL} (the product kernel and any split-K reduction), "
                     "mean of A X and A^H X",
           "commands": [f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/"
                        f"pmc{tag}_fetch -o f -- python3 <repo>/bench.py {mode}",
                        f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/"
                        f"pmc{tag}_write -o w -- python3 <repo>/bench.py {mode}",
                        f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES "
                        f"{mops} GRBM_GUI_ACTIVE --output-format csv -d <out>/pmc{tag}_mfma -o m -- "
                        f"python3 <repo>/bench.py {mode}",
                        f"python bench.py --pmc-summary{'-lowp' if lowp else ''} <out>/pmc{tag}_fetch/f_counter_collection.csv "
                        f"<out>/pmc{tag}_write/w_counter_collection.csv <out>/pmc{tag}_mfma/m_counter_collection.csv"],
           "kernel_source_hash": kernel_source_hash(), "hbm_bytes_per_launch": round(hbm),
           "algorithmic_bytes_per_launch": (8 if lowp else 16) * LN * LN + 2 * 16 * LN * LL, **out, "mfma": mfma,
           "other_counters": extra}
    path = PMC_FILE_LOWP if lowp else PMC_FILE
    os.makedirs(os.path.dirname(path), exist_ok=True)
    json.dump(rec, open(path, "w"), indent=1)
    print(json.dumps(rec))


def _kshort(name):
    """k_name<template args> of a kernel symbol (library kernels), else the first 40 characters."""
    m = re.search(r"(k_\w+?)(<[^()]*>)?\(", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    m = re.search(r"(k_\w+)", name)
    return m.group(1) if m else name[:40]


def trace_summary(path, bench_out=None):
    """Summary of a rocprofv3 kernel trace (CSV) of the default bench run: the roofline kernel's
    launches at the headline shape, and per-kernel totals of one timed solve of each precision.
    The headline solves come first in the run (warmup + steps each for FP32, BF16, BF16 split);
    a solve starts at its k_solve_prologue and holds the library's kernels up to the next one."""
    import csv
    import statistics
    rows = []
    for r in csv.DictReader(open(path)):
        rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"], int(r["Grid_Size_X"]),
                     int(r["Grid_Size_Y"]), int(r["Grid_Size_Z"])))
    rows.sort()
    lib = [r for r in rows if "qlra_impl" in r[2]]
    starts = [i for i, r in enumerate(lib) if "k_solve_prologue" in r[2]]
    starts.append(len(lib))
    per = None
    out = ["# Kernel trace: 16384 x 16384 block Krylov solve (k = 128, p = 32, v = 8), default bench run", "",
           "Commands (repository root on one MI355X; `<out>` a scratch folder):", "",
           "    cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
           "-d <out>/trace -o bench -- python3 <repo>/bench.py > <out>/bench.log",
           "    grep '^{' <out>/bench.log | tail -1 > <out>/bench.json",
           "    python bench.py --trace-summary <out>/trace/bench_kernel_trace.csv <out>/bench.json", ""]
    # the roofline kernel: FP32 views at 160 columns (grid of 512 workgroups of 256 threads)
    out += ["## The roofline kernel (FP32 view product, 16384 x 16384 by 160)", "",
            "Every launch in the run at this shape (in the solves and in the bench's graph-timed view loop).", "",
            "| kernel | launches | mean us | median us | TFLOP/s (32 m n w / mean) | of 157.3 |", "|---|---|---|---|---|---|"]
    flops = 32.0 * LN * LN * LL
    means, medians = [], []
    for label, pat in (("A X", "k_qview<5, false, true, false, false>"), ("A^H X", "k_qview<5, true, false, false, false>")):
        d = [(b - a) / 1e3 for a, b, n, gx, gy, gz in rows if _kshort(n) == pat and gx == 512 * 256 and gz == 1]
        if not d:
            continue
        mu = statistics.mean(d)
        means.append(mu)
        medians.append(statistics.median(d))
        out.append(f"| `{pat}` ({label}) | {len(d)} | {mu:.1f} | {statistics.median(d):.1f} | "
                   f"{flops / mu / 1e6:.1f} | {flops / mu / 1e6 / 157.3:.3f} |")
    thin = [(b - a) / 1e3 for a, b, n, gx, gy, gz in rows if _kshort(n) == "k_thin_t" and gx == 1024 * 256 and gy == 3]
    if thin:
        out.append(f"| `k_thin_t` (the thin operand's transpose, per view) | {len(thin)} | {statistics.mean(thin):.1f} | "
                   f"{statistics.median(thin):.1f} | | |")
    if means:
        mu = statistics.mean(means) + (statistics.mean(thin) if thin else 0.0)
        md = statistics.mean(medians) + (statistics.median(thin) if thin else 0.0)
        out += ["", f"Mean of the two products plus the transpose: {mu:.1f} us per view, "
                    f"{flops / mu / 1e6:.1f} TFLOP/s, {flops / mu / 1e6 / 157.3:.3f} of the FP32 MFMA peak; "
                    f"with the medians (the launches inside solves run beside the estimates' side stream now and "
                    f"then): {md:.1f} us, {flops / md / 1e6:.1f} TFLOP/s, {flops / md / 1e6 / 157.3:.3f}.  The "
                    "bench's `roofline` times the same launch sequence in its own graph-replayed loop with HIP "
                    "events.", ""]
    if bench_out:
        lines = [ln for ln in open(bench_out) if ln.startswith("{")]
        if lines:
            rec = json.loads(lines[-1])
            rf = rec.get("roofline", {})
            out += [f"The bench line of this (traced) run: value {rec.get('value')} {rec.get('unit')}, "
                    f"{rec.get('ms_per_step')} ms per solve; roofline achieved {rf.get('achieved')} TFLOP/s, "
                    f"frac {rf.get('frac')}.", ""]
    names = ("FP32", "BF16", "BF16 split")
    # the headline solves open the run and take tens of milliseconds each; the solves of the
    # other records (2048 x 2048, serving, completion) take about one
    nsolve = 0
    while nsolve + 1 < len(starts) and lib[starts[nsolve + 1] - 1][1] - lib[starts[nsolve]][0] > 10_000_000:
        nsolve += 1
    per = nsolve // 3 if nsolve >= 3 else 0
    if per:
        out += [f"## One timed solve of each precision (the last of {per} per precision)", ""]
        for pi, pname in enumerate(names):
            i0, i1 = starts[(pi + 1) * per - 1], starts[(pi + 1) * per]
            seg = lib[i0:i1]
            # the solve ends with its phase normalisation (the view timing loop follows the last one)
            ends = [i for i, r in enumerate(seg) if "k_phase_apply" in r[2]]
            if ends:
                seg = seg[:ends[-1] + 1]
            span = (max(r[1] for r in seg) - seg[0][0]) / 1e6
            agg = {}
            for a, b, n, gx, gy, gz in seg:
                k = _kshort(n)
                c, t = agg.get(k, (0, 0.0))
                agg[k] = (c + 1, t + (b - a) / 1e6)
            busy = sum(t for _, t in agg.values())
            out += [f"### {pname}: span {span:.2f} ms, kernel time {busy:.2f} ms (the estimates overlap on a side stream), "
                    f"{len(seg)} launches", "", "| kernel | launches | total ms | mean us |", "|---|---|---|---|"]
            for k, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:22]:
                out.append(f"| `{k}` | {c} | {t:.3f} | {1e3 * t / c:.1f} |")
            out.append("")
    total = {}
    for a, b, n, *_ in rows:
        k = _kshort(n)
        c, t = total.get(k, (0, 0.0))
        total[k] = (c + 1, t + (b - a) / 1e6)
    out += ["## Whole run: kernels by total time", "", "| kernel | launches | total ms | mean us |", "|---|---|---|---|"]
    for k, (c, t) in sorted(total.items(), key=lambda kv: -kv[1][1])[:30]:
        out.append(f"| `{k}` | {c} | {t:.2f} | {1e3 * t / c:.1f} |")
    os.makedirs(os.path.dirname(TRACE_FILE), exist_ok=True)
    with open(TRACE_FILE, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


def graph_time(torch, fn, reps):
    """Average GPU time of fn() (library launches on the current stream): reps calls captured
    in one HIP graph, replayed between two events on the stream the graph runs on, so that host
    call overhead between launches is not counted."""
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        for _ in range(2):
            fn()
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    g.replay()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def view_kernel_times(Q, torch, A, m, n, shapes, reps):
    """Average duration of each view product in `shapes` ((label, op, w, precision)), HIP events
    on its stream around a graph of reps launches; the copies of A the reduced-precision forms
    read are made once, outside the timed region."""
    g = torch.Generator(device="cuda").manual_seed(0)
    copies = {}
    out = {}
    for label, op, w, prec in shapes:
        kdim = n if op == 0 else m
        X = torch.randn((4, kdim, w), device="cuda", generator=g)
        C = torch.empty((4, m if op == 0 else n, w), device="cuda")
        cur = torch.cuda.current_stream
        if prec == "fp32":
            ws = Q.qlra_qgemm_workspace(op, m, n, w)
            fn = lambda: Q.qlra_qgemm(op, A, X, C, stream=cur(), workspace=ws)   # noqa: E731
        else:
            p = Q.QLRA_BF16
            if "copy" not in copies:
                copies["copy"] = Q.qlra_lowp_copy(A, p)
            src = copies["copy"][0 if op == 0 else 1]
            if prec == "bf16":
                ws = Q.qlra_qgemm_lp_workspace(op, p, m, n, w)
                fn = lambda: Q.qlra_qgemm_lp(op, p, src, m, n, X, C, stream=cur(), workspace=ws)   # noqa: E731
            else:
                if "res" not in copies:
                    copies["res"] = Q.qlra_lowp_copy_residual(A, p)
                res = copies["res"][0 if op == 0 else 1]
                ws = Q.qlra_qgemm_split_workspace(op, p, m, n, w)
                fn = lambda: Q.qlra_qgemm_split(op, p, src, res, m, n, X, C, stream=cur(), workspace=ws)   # noqa: E731
        out[label] = graph_time(torch, fn, reps)
        del X, C, ws
    del copies
    torch.cuda.empty_cache()
    return out


def view_roofline(label, prec, m, n, w, t):
    """Roofline position of one view product: 32 m n w algorithmic flops (16 real FMAs per
    quaternion multiply-add); bytes = A once (16 m n in FP32, 8 m n for a BF16 copy, 24 m n for
    the split form's copy, residual copy and second read) plus the thin operand and the result."""
    flops = 32.0 * m * n * w
    abytes = {"fp32": 16.0, "bf16": 8.0, "bf16_split": 16.0}[prec] * m * n
    nbytes = abytes + 16.0 * (m + n) * w
    peak_f = PEAK_FP32_MFMA if prec == "fp32" else PEAK_BF16_MFMA
    mult = 3 if prec == "bf16_split" else 1          # three BF16 products
    roof = min(peak_f / mult, flops / nbytes * PEAK_HBM)
    bound = "mfma" if peak_f / mult <= flops / nbytes * PEAK_HBM else "hbm"
    ach = flops / t
    return {"view": label, "precision": prec, "us": round(t * 1e6, 2), "tflops": round(ach / 1e12, 2),
            "hbm_gbs_algorithmic": round(nbytes / t / 1e9, 1), "bound": bound,
            "roof_tflops": round(roof / 1e12, 2), "frac_of_roof": round(ach / roof, 4)}


def direct_error(torch, A, U, S, V):
    """||A - U diag(S) V^H||_F / ||A||_F in FP64 on the device, from
    ||A||^2 - 2 sum_j S_j Re(U^H A V)_jj + sum_j S_j^2 (U and V orthonormal)."""
    def pair(X):
        X = X.to(torch.float64)
        return torch.complex(X[0], X[1]), torch.complex(X[2], X[3])
    Aa, Ab = pair(A)
    nA2 = float(torch.sum(torch.abs(Aa) ** 2 + torch.abs(Ab) ** 2))
    Va, Vb = pair(V)
    Ta = Aa @ Va - Ab @ torch.conj(Vb)
    Tb = Aa @ Vb + Ab @ torch.conj(Va)
    del Aa, Ab
    Ua, Ub = pair(U)
    # diag of U^H T: (a + b j)^H (c + d j) has complex part conj(a) c + b conj(d)... entry-wise sums
    d = torch.sum(torch.conj(Ua) * Ta + Ub * torch.conj(Tb), dim=0).real
    Sd = S.to(torch.float64)
    e2 = nA2 - 2.0 * float(torch.sum(Sd * d)) + float(torch.sum(Sd * Sd))
    return (max(e2, 0.0) / nA2) ** 0.5


def sampled_ahat(torch, U, S, V, rows, cols):
    """U diag(S) V^H at the entries (rows[t], cols[t]) in FP64 on the device, (4, len(rows))."""
    import numpy as np
    ri = torch.as_tensor(np.asarray(rows), device=U.device)
    ci = torch.as_tensor(np.asarray(cols), device=U.device)

    def pair(X):
        X = X.to(torch.float64)
        return torch.complex(X[0], X[1]), torch.complex(X[2], X[3])
    Ua, Ub = pair(U[:, ri, :])
    Va, Vb = pair(V[:, ci, :])
    Sd = S.to(torch.float64)[None, :]
    Ua, Ub = Ua * Sd, Ub * Sd
    xa = torch.sum(Ua * torch.conj(Va) + Ub * torch.conj(Vb), dim=1)
    xb = torch.sum(Ub * Va - Ua * Vb, dim=1)
    return torch.stack([xa.real, xa.imag, xb.real, xb.imag]).cpu().numpy()


def headline(Q, torch, args):
    """The timed 16384 x 16384 solves (FP32, BF16, BF16 split), their accuracy against the stored
    oracle solve, and the view kernels' roofline positions."""
    import numpy as np
    A, A32, sigma, golden = headline_matrix(torch)
    precs = {"fp32": Q.QLRA_FP32, "bf16": Q.QLRA_BF16, "bf16_split": Q.QLRA_BF16_SPLIT}
    U = torch.empty((4, LN, LK), device="cuda")
    V = torch.empty((4, LN, LK), device="cuda")
    S = torch.empty(LK, dtype=torch.float64, device="cuda")
    e = torch.empty(LV, dtype=torch.float64, device="cuda")
    res = {}
    for name, prec in precs.items():
        need = Q.qlra_workspace_size(LN, LN, LK, LP, LV, "krylov", precision=prec)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")

        def solve():
            Q.qlra(A, LK, LP, LV, "krylov", LSEED, U=U, S=S, V=V, pass_err=e, workspace=ws, precision=prec)
        log(f"{name}: warmup {args.warmup}, timing {args.steps} solves")
        for _ in range(args.warmup):
            solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert Q.qlra_status(ws) == Q.QLRA_OK
        err = direct_error(torch, A, U, S, V)
        r = {"value": round(LV * args.steps / dt, 3), "unit": "A-passes/s", "ms_per_solve": round(dt * 1e3 / args.steps, 3),
             "rel_err": err, "e_v": float(e[-1].item()), "workspace_gb": round(need / 2 ** 30, 3)}
        if golden is not None:
            eo = golden["pass_err"][-1]
            r["rel_err_oracle"] = eo
            r["error_ratio_vs_oracle"] = err / eo
            got = sampled_ahat(torch, U, S, V, golden["rows"], golden["cols"])
            want = np.asarray(golden["ahat"])
            r["ahat_diff_sampled"] = float(np.sqrt(np.mean(np.sum((got - want) ** 2, axis=0)) * LN * LN / golden["nA2"]))
            r["max_rel_sv_diff"] = float(np.max(np.abs(S.cpu().numpy() - np.asarray(golden["S"])) /
                                                np.asarray(golden["S"])))
        res[name] = r
        del ws
        torch.cuda.empty_cache()
    for name in ("bf16", "bf16_split"):
        res[name]["speedup_vs_fp32"] = round(res[name]["value"] / res["fp32"]["value"], 3)
    opt = float(np.sqrt(np.sum(sigma[LK:] ** 2) / np.sum(sigma ** 2)))
    log("timing the view kernels")
    shapes = [("fp32 A X, w=160", 0, LL, "fp32"), ("fp32 A^H X, w=160", 1, LL, "fp32"),
              ("fp32 A^H X, w=640 (last view)", 1, LW, "fp32"),
              ("bf16 A X, w=160", 0, LL, "bf16"), ("bf16 A^H X, w=160", 1, LL, "bf16"),
              ("bf16 split A X, w=160", 0, LL, "bf16_split"),
              ("bf16 split A^H X, w=640 (last view)", 1, LW, "bf16_split")]
    kt = view_kernel_times(Q, torch, A, LN, LN, shapes, args.kernel_reps)
    views = [view_roofline(lab, prec, LN, LN, w, kt[lab]) for lab, _, w, prec in shapes]
    del A
    torch.cuda.empty_cache()
    return res, views, kt, opt, golden, A32


def cpu_baseline(A32):
    """The FP64 oracle on the host, as it stands, on a bounded sample of the headline workload:
    its first view A Omega (16384 x 16384 by 160) restricted to a block of rows, single thread and
    all cores (OpenMP over output rows), scaled to A-passes/s (rows sampled / 16384 of a pass).
    The full solve is dominated by its 8 views; its QR and QSVD steps are not in the sample."""
    import numpy as np
    cores = host_cores()
    out = {"unit": "A-passes/s", "kind": "oracle", "cores": cores, "cpu_model": cpu_model()}
    tmp = "/tmp/qlra_bench_rows.npy"
    for threads, rows in ((1, 192), (cores, max(192, 96 * cores))):
        np.save(tmp, np.ascontiguousarray(A32[:, :rows, :]))
        code = ("import sys, time, numpy as np; sys.path.insert(0, %r); from oracle import oracle as O; "
                "A = np.load(%r).astype(np.float64); Om = O.omega(%d, %d, %d).astype(np.float64); "
                "t = time.perf_counter(); O.qgemm(A, Om); print(time.perf_counter() - t)"
                % (ROOT, tmp, LSEED, LN, LL))
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        log(f"cpu baseline: oracle view on {rows} rows, {threads} thread(s)")
        t = float(subprocess.check_output([sys.executable, "-c", code], env=env, text=True).strip().splitlines()[-1])
        rate = (rows / LN) / t
        key = "single_thread" if threads == 1 else "all_cores"
        out[key] = {"value": round(rate, 6), "threads": threads, "rows": rows, "seconds": round(t, 2)}
    os.remove(tmp)
    out["value"] = out["all_cores"]["value"]
    out["sample"] = (f"the oracle's first view A Omega of the {LN}x{LN} workload ({LL} columns) on "
                     f"{out['all_cores']['rows']} rows with all {cores} cores ({out['all_cores']['seconds']} s) and on "
                     f"{out['single_thread']['rows']} rows with one thread ({out['single_thread']['seconds']} s), "
                     "scaled to whole passes; QR and QSVD steps not included")
    return out


def config1_record(Q, torch, W, args):
    """The 2048 x 2048 subspace workload: one step = the solves of the four budgets, each on a
    stream of its own (the longest on the current stream), graph-replayed; plus the accuracy of
    each budget against the oracle."""
    import numpy as np
    from oracle import oracle as O
    log("2048x2048 workload")
    A_np, _ = W.config1(seed=SEED_DATA1, n=M1, noise_std=0.01)
    A = torch.from_numpy(A_np).cuda()
    outs = {}
    for v in BUDGETS1:
        need = Q.qlra_workspace_size(M1, N1, K1, P1, v, "subspace")
        outs[v] = dict(U=torch.empty((4, M1, K1), device="cuda"), V=torch.empty((4, N1, K1), device="cuda"),
                       S=torch.empty(K1, dtype=torch.float64, device="cuda"),
                       e=torch.empty(v, dtype=torch.float64, device="cuda"),
                       ws=torch.empty(need, dtype=torch.uint8, device="cuda"))
    streams = {v: torch.cuda.Stream() for v in BUDGETS1[:-1]}

    def solve(v, stream=None):
        o = outs[v]
        Q.qlra(A, K1, P1, v, "subspace", SEED_SKETCH1, U=o["U"], S=o["S"], V=o["V"], pass_err=o["e"],
               workspace=o["ws"], graph=True, stream=stream)

    def step():
        cur = torch.cuda.current_stream()
        for v in BUDGETS1[:-1]:
            streams[v].wait_stream(cur)
            solve(v, streams[v])
        solve(BUDGETS1[-1], cur)
        for v in BUDGETS1[:-1]:
            cur.wait_stream(streams[v])

    steps = 20
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_v = {}
    for v in BUDGETS1:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            solve(v)
        torch.cuda.synchronize()
        per_v[f"v{v}_ms"] = round((time.perf_counter() - t1) * 1e3 / 5, 4)
    kt = view_kernel_times(Q, torch, A, M1, N1, [("fwd", 0, K1 + P1, "fp32"), ("adj", 1, K1 + P1, "fp32")], 50)
    A64 = A_np.astype(np.float64)
    nA = np.sqrt(np.sum(A64 ** 2))
    acc = []
    for v in BUDGETS1:
        Uo, So, Vo, _ = O.qlra(A64, K1, P1, v, O.SUBSPACE, SEED_SKETCH1)
        Ao = O.reconstruct(Uo, So, Vo)
        solve(v)
        torch.cuda.synchronize()
        o = outs[v]
        Ag = O.reconstruct(*(x.cpu().numpy().astype(np.float64) for x in (o["U"], o["S"], o["V"])))
        eg, eo = np.sqrt(np.sum((A64 - Ag) ** 2)) / nA, np.sqrt(np.sum((A64 - Ao) ** 2)) / nA
        acc.append({"v": v, "rel_err_gpu": float(eg), "rel_err_oracle": float(eo), "ratio": float(eg / eo),
                    "ahat_diff": float(np.sqrt(np.sum((Ag - Ao) ** 2)) / nA)})
    return {"workload": "dense quaternion 2048x2048 FP32, sigma_i=exp(-i/20)+N(0,1e-4) noise, k=50, p=10, "
                        "subspace scheme (Alg. 2), budgets v=2,3,4,6 per step (concurrent on four streams)",
            "value": round(sum(BUDGETS1) * steps / dt, 3), "unit": "A-passes/s",
            "ms_per_step": round(dt * 1e3 / steps, 4), "solve_ms": per_v,
            "view_roofline": [view_roofline(lab, "fp32", M1, N1, K1 + P1, t) for lab, t in kt.items()],
            "accuracy": acc}


def serving(Q, torch, nreq, seed=3):
    """The serving stream: nreq requests of mixed sizes, ranks, budgets and schemes through the
    library's continuous-batching server.  First all at once (closed loop) to find the FP32
    saturation rate, then Poisson arrivals at 0.7 of it, FP32 and FP16 views on the same
    arrival times.  Latency = completion - arrival on the server's clock."""
    import numpy as np
    from workloads import gpu as WG
    reqs = WG.serving_stream(seed, nreq)
    for r in reqs:
        r["U"] = torch.empty((4, r["m"], r["k"]), device="cuda")
        r["V"] = torch.empty((4, r["n"], r["k"]), device="cuda")
        r["S"] = torch.empty(r["k"], dtype=torch.float64, device="cuda")
        r["e"] = torch.empty(r["v"], dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    hbm = 24 << 30
    passes = sum(r["v"] for r in reqs)

    def run(prec, arrivals, graphs=False, subset=None, arena=hbm):
        rs = reqs if subset is None else reqs[:subset]
        srv = Q.Server(arena, max_active=SERVE_SLOTS, graphs=graphs)
        t0 = Q.server_clock() + 0.005
        tickets = []
        for i, r in enumerate(rs):
            ta = t0 + arrivals[i]
            while Q.server_clock() < ta:
                pass
            tickets.append(srv.submit(r["A"], r["k"], r["p"], r["v"], r["scheme"], r["seed"], U=r["U"], S=r["S"],
                                      V=r["V"], pass_err=r["e"], precision=prec, arrival_time=ta))
        srv.drain()
        lats, done = [], []
        for i, t in enumerate(tickets):
            st, lat, _ = srv.poll(t, wait=True)
            assert st == Q.QLRA_OK, st
            lats.append(lat)
            done.append(t0 + arrivals[i] + lat)
        stats = srv.stats()
        srv.close()
        return np.array(lats), max(done) - t0, stats

    zeros = np.zeros(nreq)
    run(Q.QLRA_FP32, zeros, subset=min(32, nreq))           # warm-up (first launches of every kernel)
    run(Q.QLRA_FP16, zeros, subset=min(32, nreq))
    _, span32, _ = run(Q.QLRA_FP32, zeros)
    _, span32g, _ = run(Q.QLRA_FP32, zeros, graphs=True)
    rate = nreq / span32
    lam = 0.7 * rate
    arrivals = np.cumsum(np.random.default_rng(seed).exponential(1.0 / lam, nreq))
    out = {"requests": nreq, "workload": "m, n in {256..2048 step 128}, sigma_i = i^-1, dense/pure 50/50, "
                                         "k in {8..64}, p = k/4, v in {2..6}, subspace/Krylov 50/50 (seeded)",
           "passes": int(passes), "slots": SERVE_SLOTS, "arena_gb": hbm / 2 ** 30,
           "closed_loop": {"fp32_req_per_s": round(rate, 2), "fp32_passes_per_s": round(passes / span32, 1),
                           "fp32_graphs_req_per_s": round(nreq / span32g, 2)},
           "poisson_rate_req_per_s": round(lam, 2)}
    def record(lat, span, stats):
        return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "mean_ms": round(float(lat.mean()) * 1e3, 3),
                "throughput_req_per_s": round(nreq / span, 2), "passes_per_s": round(passes / span, 1),
                "max_in_flight": stats["max_active_seen"],
                "max_arena_gb": round(stats["max_arena_used"] / 2 ** 30, 3)}

    for name, prec in (("fp32", Q.QLRA_FP32), ("fp16", Q.QLRA_FP16)):
        out[name] = record(*run(prec, arrivals))
    # the same arrivals through an arena that holds the largest request and little else: admission
    # is then bound by HBM, not by the slots, whenever a large request is in flight
    small = int(max(Q.qlra_workspace_size(r["m"], r["n"], r["k"], r["p"], r["v"], r["scheme"]) for r in reqs) * 1.05)
    out["fp32_hbm_bound"] = {"arena_gb": round(small / 2 ** 30, 4), **record(*run(Q.QLRA_FP32, arrivals, arena=small))}
    return out


# Quaternion matrix completion (Sec. 7) in the set-up of the inpainting experiments (70 % of the
# pixels missing, rank 30, two passes of Alg. 2, Gaussian smoothing 0.6 after each iteration) on
# a pure quaternion image stand-in, at the experiments' 256 x 256 and at 2048 x 2048:
# (name, m, n, rank, p, passes, observed fraction, sigma, iterations)
COMPLETION = [
    ("inpainting 256x256 pure quaternion image, 70% missing, rank 30, p 10, 2 passes (Alg. 2), smoothing 0.6",
     256, 256, 30, 10, 2, 0.3, 0.6, 50),
    ("inpainting 2048x2048 pure quaternion image, 70% missing, rank 30, p 10, 2 passes (Alg. 2), smoothing 0.6",
     2048, 2048, 30, 10, 2, 0.3, 0.6, 20),
]


def completion(Q, torch, W):
    """Completion iterations per second, the iteration captured once as a HIP graph and replayed
    (graph) and launched kernel by kernel (eager); the misfit on the observed entries at the first
    and last iteration and the relative error of X on all entries."""
    out = []
    for name, m, n, rank, p, v, observed, sigma, iters in COMPLETION:
        log(f"completion {m}x{n}, {iters} iterations")
        M = torch.from_numpy(W.image_like(5, m, n)).cuda()
        K = torch.from_numpy(W.random_mask(6, m, n, observed)).cuda()
        X = torch.empty_like(M)
        fit = torch.empty(iters, dtype=torch.float64, device="cuda")
        ws = None
        rec = {"workload": name, "m": m, "n": n, "rank": rank, "p": p, "passes": v, "observed": observed,
               "sigma": sigma, "iterations": iters}
        for mode, graph in (("graph", True), ("eager", False)):
            _, _, ws = Q.qlra_complete(M, K, rank, p, v, 0, 7, iters, sigma, X=X, fit=fit, workspace=ws, graph=graph)
            torch.cuda.synchronize()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                Q.qlra_complete(M, K, rank, p, v, 0, 7, iters, sigma, X=X, fit=fit, workspace=ws, graph=graph)
            torch.cuda.synchronize()
            rec[f"{mode}_ms_per_iteration"] = round((time.perf_counter() - t0) * 1e3 / (reps * iters), 4)
        assert Q.qlra_status(ws) == Q.QLRA_OK
        rec["iterations_per_s"] = round(1e3 / rec["graph_ms_per_iteration"], 2)
        f = fit.cpu().numpy()
        rec["fit_first_last"] = [round(float(f[0]), 6), round(float(f[-1]), 6)]
        rec["relative_error_all_entries"] = round(float(torch.linalg.norm(X - M) / torch.linalg.norm(M)), 6)
        out.append(rec)
    return out


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary)
        return
    if args.pmc_summary_lowp:
        pmc_summary(args.pmc_summary_lowp, lowp=True)
        return
    if args.trace_summary:
        trace_summary(*args.trace_summary[:2])
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2507_13731_amd import qlra as Q
    import workloads as W

    if args.only_completion:
        print(json.dumps({"completion": completion(Q, torch, W)}))
        return
    if args.counters or args.counters_lowp:
        A, _, _, _ = headline_matrix(torch)
        counters_run(Q, torch, A, lowp=args.counters_lowp)
        return
    res, views, kt, opt, golden, A32 = headline(Q, torch, args)
    fp = res["fp32"]
    # the dominant kernel: the FP32 view product at 160 columns (7 of the 8 views), forward and
    # adjoint averaged
    t_view = 0.5 * (kt["fp32 A X, w=160"] + kt["fp32 A^H X, w=160"])
    flops = 32.0 * LN * LN * LL
    achieved = flops / t_view
    traffic = None
    if os.path.exists(PMC_FILE):
        pmc = json.load(open(PMC_FILE))
        if pmc.get("kernel_source_hash") == kernel_source_hash():
            traffic = pmc.get("hbm_bytes_per_launch")
    roofline = {"bound": "mfma", "achieved": round(achieved / 1e12, 3), "peak": PEAK_FP32_MFMA / 1e12,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 4), "traffic": traffic,
                "kernel": f"k_qview FP32 view product, {LN}x{LN} by {LL} quaternion columns (mean of A X and A^H X)",
                "algorithmic_flops_per_launch": flops,
                "algorithmic_bytes_per_launch": 16.0 * LN * LN + 2 * 16.0 * LN * LL}
    if args.only_headline:
        print(json.dumps({"headline": res, "view_kernels": views, "roofline": roofline}))
        return
    sec = None if args.no_config1 else config1_record(Q, torch, W, args)
    serve = None
    if not args.no_serve:
        log(f"serving stream ({args.serve_requests} requests)")
        serve = serving(Q, torch, args.serve_requests)
    comp = None if args.no_completion else completion(Q, torch, W)
    cpu = None if args.no_cpu_baseline else cpu_baseline(A32)
    line = {"metric": "A-passes/s", "value": fp["value"], "unit": "A-passes/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": fp["ms_per_solve"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded; sigma_i = i^-1/2, reflector-product quaternion unitaries, built on the host)",
            "config": {"workload": f"dense quaternion {LN}x{LN} FP32, sigma_i=i^-1/2, block Krylov (Alg. 4) "
                                   f"k={LK}, p={LP}, v={LV}: one solve (8 passes over A) per step",
                       "m": LN, "n": LN, "k": LK, "p": LP, "pass_budget": LV, "scheme": "block_krylov",
                       "sketch_seed": LSEED},
            "qgemm_tflops": round(achieved / 1e12, 3), "rel_err_gpu": fp["rel_err"],
            "rel_err_oracle": fp.get("rel_err_oracle"), "error_ratio_vs_oracle": fp.get("error_ratio_vs_oracle"),
            "ahat_diff_vs_oracle_sampled": fp.get("ahat_diff_sampled"),
            "optimum_rank_k_error": opt,
            "roofline": roofline, "cpu_baseline": cpu,
            "precision_form": {"views": "BF16: views 1..6 on BF16 copies of A (FP32 accumulation), views 7 and 8 FP32; "
                                        "BF16 split: views 7 and 8 as three BF16 products of values and residuals; "
                                        "Gram/Cholesky/QSVD FP64", "fp32": fp,
                               "bf16": res["bf16"], "bf16_split": res["bf16_split"]},
            "view_kernels": views,
            "oracle_full_solve_context": (None if golden is None else
                                          {"seconds": round(golden["oracle_seconds"], 1),
                                           "a_passes_per_s": round(LV / golden["oracle_seconds"], 5),
                                           "where": "the run that wrote the stored oracle solve (another host, "
                                                    "8 cores); context only"}),
            "config_2048": sec, "serving": serve, "completion": comp}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
