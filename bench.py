"""Benchmark: pass-efficient randomized truncated QSVD on one MI355X.

Workload (the 2048 x 2048 configuration): dense quaternion FP32 matrix
A = U diag(sigma) V^H + E, sigma_i = exp(-i/20), Haar quaternion unitaries, E i.i.d. N(0, 1e-4)
per real component (synthetic, seeded).  k = 50, p = 10, subspace scheme (Alg. 2).  One step
= one solve for each pass budget v in {2, 3, 4, 6}: 15 passes over A, each a quaternion view
product A X or A^H X followed by its CholeskyQR, then the small QSVD and the
back-multiplication, with per-pass error estimates.  The four solves are independent and run
concurrently, the longest on the current stream and the others on three streams of their own
(one per hardware queue), so that the latency-bound small steps of one overlap the views of
the others; the same step with the solves one after another is reported beside it
(sequential_value), and the latency of each solve alone (solve_ms).

Printed: one JSON line with passes/s (value), the dominant kernel's roofline position (FP32
MFMA view product, timed with HIP events on its own stream), the FP64 CPU oracle timed on the
host as a baseline, and accuracy against the oracle.  The precision form (views 1 .. v-2 in
BF16 / FP16 with FP32 accumulation, the last two views FP32) is timed on the same step and
reported beside it with its error ratio to the oracle.
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M = N = 2048
K_RANK, P_OVER = 50, 10
BUDGETS = (2, 3, 4, 6)
SEED_DATA, SEED_SKETCH = 1, 1
PEAK_FP32_MFMA = 157.3e12
PEAK_HBM = 8.0e12
PMC_FILE = os.path.join(ROOT, "profiles", "qgemm_f32_view_2048x2048x60_pmc.json")
# server slots: one per hardware queue HIP gives a process by default (measured with 256
# requests: 1861 req/s closed loop with 4 slots, 1508 with 8, 1444 with 16)
SERVE_SLOTS = 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-completion", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--only-large", action="store_true",
                    help="run only the 16384 x 16384 solves and print their record")
    ap.add_argument("--only-completion", action="store_true",
                    help="run only the matrix-completion workloads (for a kernel trace) and print their record")
    ap.add_argument("--counters", action="store_true",
                    help="launch sequence for hardware-counter runs only (view products and calibration copies)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn the counter CSVs of two --counters runs into the traffic record under profiles/")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_2507_13731_amd", "csrc", "qgemm.hip"), "rb").read())
    return h.hexdigest()[:16]


COPY_BYTES = 256 << 20
COUNTER_REPS = 5


def counters_run(Q, torch, A):
    """The launch sequence the traffic counters are read on: COUNTER_REPS forward and adjoint
    FP32 view products (2048 x 2048 by 60), then COUNTER_REPS elementwise passes over 256 MiB
    (read once, written once) whose counter readings calibrate the scale of FETCH_SIZE and
    WRITE_SIZE."""
    w = K_RANK + P_OVER
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((4, N, w), device="cuda", generator=g)
    for op in (0, 1):
        ws = Q.qlra_qgemm_workspace(op, M, N, w)
        C = torch.empty((4, M if op == 0 else N, w), device="cuda")
        for _ in range(COUNTER_REPS):
            Q.qlra_qgemm(op, A, X, C, stream=torch.cuda.current_stream(), workspace=ws)
            torch.cuda.synchronize()
    src = torch.ones(COPY_BYTES // 4, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(COUNTER_REPS):
        torch.neg(src, out=dst)            # an elementwise kernel: reads and writes COPY_BYTES
        torch.cuda.synchronize()
    print(json.dumps({"counters_run": "done", "view_launches_per_op": COUNTER_REPS, "copy_bytes": COPY_BYTES}))


def pmc_summary(fetch_csv, write_csv):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) from two rocprofv3 --pmc runs of --counters
    (CSV output).  A view is the thin-block transpose, the product kernel and the ordered split-K
    reduction; the elementwise pass's readings give the factor that turns each counter into
    bytes."""
    import csv
    import statistics

    def read(path, counter):
        rows = {}
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") != counter:
                continue
            key = int(r["Dispatch_Id"])
            rows[key] = (r["Kernel_Name"], rows.get(key, ("", 0.0))[1] + float(r["Counter_Value"]))
        return [rows[k] for k in sorted(rows)]

    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        seq = read(path, counter)
        view = [(n, v) for n, v in seq if any(t in n for t in ("k_thin_t", "k_qview", "k_splitk_reduce"))]
        copies = [v for _, v in seq[-COUNTER_REPS:]]     # the calibration copies end the sequence
        kib_copy = statistics.median(copies)
        scale = COPY_BYTES / (kib_copy * 1024.0)
        per_op = {}
        for op, name in ((0, "forward"), (1, "adjoint")):
            part = view[op * len(view) // 2:(op + 1) * len(view) // 2]
            kib = sum(v for _, v in part) / COUNTER_REPS
            per_op[name] = {"kib_per_launch": round(kib, 1), "bytes_per_launch": round(kib * 1024.0 * scale),
                            "kernels": sorted({re.search(r"k_\w+", n).group(0) for n, _ in part})}
        out[counter] = {"copy_kib": round(kib_copy, 1), "scale": round(scale, 4), **per_op}
    hbm = 0.5 * sum(out[c][o]["bytes_per_launch"] for c in ("FETCH_SIZE", "WRITE_SIZE") for o in ("forward", "adjoint"))
    rec = {"kernel": "FP32 view product 2048x2048 by 60 (transpose + product kernel + split-K reduction), "
                     "mean of A X and A^H X",
           "commands": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/"
                        "pmc_fetch -o f -- python3 <repo>/bench.py --counters",
                        "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/"
                        "pmc_write -o w -- python3 <repo>/bench.py --counters",
                        "python bench.py --pmc-summary <out>/pmc_fetch/f_counter_collection.csv "
                        "<out>/pmc_write/w_counter_collection.csv"],
           "kernel_source_hash": kernel_source_hash(), "hbm_bytes_per_launch": round(hbm),
           "algorithmic_bytes_per_launch": 16 * M * N + 2 * 16 * N * (K_RANK + P_OVER), **out}
    os.makedirs(os.path.dirname(PMC_FILE), exist_ok=True)
    json.dump(rec, open(PMC_FILE, "w"), indent=1)
    print(json.dumps(rec))


def graph_time(torch, fn, reps):
    """Average GPU time of fn() (library launches on the current stream): reps calls captured
    in one HIP graph, replayed between two events on the stream the graph runs on, so that host
    call overhead between launches is not counted."""
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        for _ in range(3):
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


def time_view_kernels(Q, torch, A, reps):
    """Average duration of the FP32 view product (both orientations; the product kernel and, for
    split K, its ordered reduction) with HIP events on the stream the kernels run on."""
    w = K_RANK + P_OVER
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((4, N, w), device="cuda", generator=g)
    out = {}
    for op in (0, 1):
        ws = Q.qlra_qgemm_workspace(op, M, N, w)
        C = torch.empty((4, M if op == 0 else N, w), device="cuda")
        out[op] = graph_time(torch, lambda: Q.qlra_qgemm(op, A, X, C, stream=torch.cuda.current_stream(), workspace=ws),
                             reps)
    return out


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

    def run(prec, arrivals, graphs=False, subset=None):
        rs = reqs if subset is None else reqs[:subset]
        srv = Q.Server(hbm, max_active=SERVE_SLOTS, graphs=graphs)
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
    for name, prec in (("fp32", Q.QLRA_FP32), ("fp16", Q.QLRA_FP16)):
        lat, span, stats = run(prec, arrivals)
        out[name] = {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                     "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                     "mean_ms": round(float(lat.mean()) * 1e3, 3),
                     "throughput_req_per_s": round(nreq / span, 2), "passes_per_s": round(passes / span, 1),
                     "max_in_flight": stats["max_active_seen"],
                     "max_arena_gb": round(stats["max_arena_used"] / 2 ** 30, 3)}
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
        print(f"completion {m}x{n}, {iters} iterations", file=sys.stderr, flush=True)
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


# The large single matrix: 16384 x 16384 dense FP32, sigma_i = i^-1/2, block Krylov k = 128,
# p = 32, budget 8 (final view 640 columns wide), plain FP32 against the precision form
LARGE_N, LARGE_K, LARGE_P, LARGE_V = 16384, 128, 32, 8


def large(Q, torch):
    """End-to-end solve time of the 16384 x 16384 workload for each view precision (the mean of 3
    solves after a warm-up, synchronised around each) and the returned error estimate e_v, which
    is ||A - U S V^H||_F / ||A||_F by an exact identity (checked against the direct residual by
    the full-size tests)."""
    import numpy as np
    from workloads import gpu as WG
    print(f"large solve {LARGE_N}x{LARGE_N}: generating", file=sys.stderr, flush=True)
    sigma = np.arange(1, LARGE_N + 1, dtype=np.float64) ** -0.5
    A = WG.spectrum_matrix(4, LARGE_N, LARGE_N, sigma)
    torch.cuda.synchronize()
    rec = {"workload": f"dense {LARGE_N}x{LARGE_N} FP32, sigma_i = i^-1/2, block Krylov (Alg. 4) k={LARGE_K}, "
                       f"p={LARGE_P}, v={LARGE_V}", "solves": 3}
    U = torch.empty((4, LARGE_N, LARGE_K), device="cuda")
    V = torch.empty((4, LARGE_N, LARGE_K), device="cuda")
    S = torch.empty(LARGE_K, dtype=torch.float64, device="cuda")
    e = torch.empty(LARGE_V, dtype=torch.float64, device="cuda")
    for name, prec in (("fp32", Q.QLRA_FP32), ("bf16", Q.QLRA_BF16), ("bf16_split", Q.QLRA_BF16_SPLIT)):
        print(f"large solve {name}", file=sys.stderr, flush=True)
        ws = None
        _, _, _, _, ws = Q.qlra(A, LARGE_K, LARGE_P, LARGE_V, "krylov", 11, U=U, S=S, V=V, pass_err=e, precision=prec)
        torch.cuda.synchronize()
        t = []
        for _ in range(3):
            t0 = time.perf_counter()
            Q.qlra(A, LARGE_K, LARGE_P, LARGE_V, "krylov", 11, U=U, S=S, V=V, pass_err=e, workspace=ws, precision=prec)
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        assert Q.qlra_status(ws) == Q.QLRA_OK
        rec[f"{name}_solve_ms"] = round(1e3 * sum(t) / len(t), 3)
        rec[f"{name}_e_v"] = float(e[-1].item())
        del ws
    for name in ("bf16", "bf16_split"):
        rec[f"{name}_speedup_vs_fp32"] = round(rec["fp32_solve_ms"] / rec[f"{name}_solve_ms"], 3)
        rec[f"{name}_error_ratio"] = rec[f"{name}_e_v"] / rec["fp32_e_v"]
    rec["optimum_rank_k_error"] = float(np.sqrt(np.sum(sigma[LARGE_K:] ** 2) / np.sum(sigma ** 2)))
    del A
    torch.cuda.empty_cache()
    return rec


def cpu_baseline(A_np):
    """The FP64 oracle on the host: one full step (v = 2, 3, 4, 6) on the same matrix."""
    from oracle import oracle as O
    import numpy as np
    cores = len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(cores)
    A64 = A_np.astype(np.float64)
    t0 = time.perf_counter()
    for v in BUDGETS:
        O.qlra(A64, K_RANK, P_OVER, v, O.SUBSPACE, SEED_SKETCH)
    dt = time.perf_counter() - t0
    return {"value": round(sum(BUDGETS) / dt, 4), "unit": "A-passes/s", "cores": cores, "kind": "oracle",
            "sample": "one full step (subspace solves at v = 2, 3, 4, 6; 15 passes) on the same 2048x2048 matrix, "
                      f"{dt:.1f} s wall"}


def accuracy(Q, torch, A, A_np, precisions):
    """Error of the GPU result (each precision) and of the oracle against A for each budget
    (outside the timed region)."""
    import numpy as np
    from oracle import oracle as O
    A64 = A_np.astype(np.float64)
    nA = np.sqrt(np.sum(A64 ** 2))
    rows = {name: [] for name in precisions}
    for v in BUDGETS:
        Uo, So, Vo, eo = O.qlra(A64, K_RANK, P_OVER, v, O.SUBSPACE, SEED_SKETCH)
        Ao = O.reconstruct(Uo, So, Vo)
        eo_ = np.sqrt(np.sum((A64 - Ao) ** 2)) / nA
        for name, prec in precisions.items():
            U, S, V, e, ws = Q.qlra(A, K_RANK, P_OVER, v, "subspace", SEED_SKETCH, precision=prec)
            torch.cuda.synchronize()
            Ug, Sg, Vg = (x.cpu().numpy().astype(np.float64) for x in (U, S, V))
            Ag = O.reconstruct(Ug, Sg, Vg)
            eg_ = np.sqrt(np.sum((A64 - Ag) ** 2)) / nA
            rows[name].append({"v": v, "rel_err_gpu": float(eg_), "rel_err_oracle": float(eo_),
                               "ratio": float(eg_ / eo_), "ahat_diff": float(np.sqrt(np.sum((Ag - Ao) ** 2)) / nA),
                               "pass_err_gpu_last": float(e.cpu().numpy()[-1])})
    return rows


def time_split_view_kernels(Q, torch, A, prec, reps):
    """Average duration of the split-form view product (both orientations), as above."""
    w = K_RANK + P_OVER
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((4, N, w), device="cuda", generator=g)
    Alo, Alo_t = Q.qlra_lowp_copy(A, prec)
    Ar, Ar_t = Q.qlra_lowp_copy_residual(A, prec)
    out = {}
    for op in (0, 1):
        ws = Q.qlra_qgemm_split_workspace(op, prec, M, N, w)
        C = torch.empty((4, M if op == 0 else N, w), device="cuda")
        a, r = (Alo, Ar) if op == 0 else (Alo_t, Ar_t)
        out[op] = graph_time(torch, lambda: Q.qlra_qgemm_split(op, prec, a, r, M, N, X, C,
                                                               stream=torch.cuda.current_stream(), workspace=ws), reps)
    return out


def time_lowp_view_kernels(Q, torch, A, prec, reps):
    """Average duration of the reduced-precision view product (both orientations), HIP events on
    its stream around a graph of reps launches.  The copies of A are made once, outside the
    timed region."""
    w = K_RANK + P_OVER
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((4, N, w), device="cuda", generator=g)
    Alo, Alo_t = Q.qlra_lowp_copy(A, prec)
    out = {}
    for op in (0, 1):
        ws = Q.qlra_qgemm_lp_workspace(op, prec, M, N, w)
        C = torch.empty((4, M if op == 0 else N, w), device="cuda")
        src = Alo if op == 0 else Alo_t
        out[op] = graph_time(torch, lambda: Q.qlra_qgemm_lp(op, prec, src, M, N, X, C, stream=torch.cuda.current_stream(),
                                                            workspace=ws), reps)
    return out


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2507_13731_amd import qlra as Q
    import workloads as W

    if args.only_completion:
        print(json.dumps({"completion": completion(Q, torch, W)}))
        return
    if args.only_large:
        print(json.dumps({"large": large(Q, torch)}))
        return
    print("generating the 2048x2048 workload", file=sys.stderr, flush=True)
    A_np, _ = W.config1(seed=SEED_DATA, n=M, noise_std=0.01)
    A = torch.from_numpy(A_np).cuda()
    if args.counters:
        counters_run(Q, torch, A)
        return
    precisions = {"fp32": Q.QLRA_FP32, "bf16": Q.QLRA_BF16, "fp16": Q.QLRA_FP16, "bf16_split": Q.QLRA_BF16_SPLIT}
    outs = {}
    for name, prec in precisions.items():
        for v in BUDGETS:
            need = Q.qlra_workspace_size(M, N, K_RANK, P_OVER, v, "subspace", precision=prec)
            outs[name, v] = dict(U=torch.empty((4, M, K_RANK), device="cuda"),
                                 V=torch.empty((4, N, K_RANK), device="cuda"),
                                 S=torch.empty(K_RANK, dtype=torch.float64, device="cuda"),
                                 e=torch.empty(v, dtype=torch.float64, device="cuda"),
                                 ws=torch.empty(need, dtype=torch.uint8, device="cuda"))

    # one step = the solves of the four budgets, independent of each other: each on a stream of
    # its own (default priority), so that one solve's latency-bound small steps overlap the
    # others' views
    # the longest solve (v = 6) on the current stream, the others on three streams of their own:
    # four streams for the four hardware queues HIP gives a process by default (with a fifth,
    # two of them would share a queue and run one after the other)
    streams = {v: torch.cuda.Stream() for v in BUDGETS[:-1]}

    def solve(name, v, stream=None):
        o = outs[name, v]
        Q.qlra(A, K_RANK, P_OVER, v, "subspace", SEED_SKETCH, U=o["U"], S=o["S"], V=o["V"], pass_err=o["e"],
               workspace=o["ws"], graph=True, precision=precisions[name], stream=stream)

    def step(name):
        cur = torch.cuda.current_stream()
        for v in BUDGETS[:-1]:
            streams[v].wait_stream(cur)
            solve(name, v, streams[v])
        solve(name, BUDGETS[-1], cur)
        for v in BUDGETS[:-1]:
            cur.wait_stream(streams[v])

    def timed_steps(name, steps, warmup):
        for _ in range(warmup):
            step(name)
        torch.cuda.synchronize()
        for v in BUDGETS:
            assert Q.qlra_status(outs[name, v]["ws"]) == Q.QLRA_OK
        t0 = time.perf_counter()
        for _ in range(steps):
            step(name)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def per_budget(name):
        res = {}
        for v in BUDGETS:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(5):
                solve(name, v)
            torch.cuda.synchronize()
            res[f"v{v}_ms"] = round((time.perf_counter() - t1) * 1e3 / 5, 4)
        return res

    print(f"warmup {args.warmup} steps, timing {args.steps} steps (FP32 views)", file=sys.stderr, flush=True)
    dt = timed_steps("fp32", args.steps, args.warmup)
    ms_per_step = dt * 1e3 / args.steps
    passes = sum(BUDGETS) * args.steps
    value = passes / dt
    per_v = per_budget("fp32")
    # the same step with the four solves one after another on one stream (latency view)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        for v in BUDGETS:
            solve("fp32", v)
    torch.cuda.synchronize()
    sequential_value = passes / (time.perf_counter() - t1)

    lowp = {}
    for name in ("bf16", "fp16", "bf16_split"):
        print(f"timing {args.steps} steps ({name} views 1..v-2)", file=sys.stderr, flush=True)
        dtl = timed_steps(name, args.steps, args.warmup)
        split = name.endswith("_split")
        kt_l = time_lowp_view_kernels(Q, torch, A, precisions["bf16" if split else name], args.kernel_reps)
        t_l = 0.5 * (kt_l[0] + kt_l[1])
        lowp[name] = {"value": round(passes / dtl, 3), "unit": "A-passes/s", "ms_per_step": round(dtl * 1e3 / args.steps, 4),
                      "speedup_vs_fp32": round(dt / dtl, 4), "solve_ms": per_budget(name),
                      "view_kernel_us": {"forward": round(kt_l[0] * 1e6, 2), "adjoint": round(kt_l[1] * 1e6, 2)},
                      "view_hbm_gbs": round(8.0 * M * N / t_l / 1e9, 1),
                      "view_hbm_frac": round(8.0 * M * N / t_l / PEAK_HBM, 4)}
        if split:
            ks = time_split_view_kernels(Q, torch, A, Q.QLRA_BF16, args.kernel_reps)
            lowp[name]["split_view_kernel_us"] = {"forward": round(ks[0] * 1e6, 2), "adjoint": round(ks[1] * 1e6, 2)}

    print("timing the view kernels", file=sys.stderr, flush=True)
    kt = time_view_kernels(Q, torch, A, args.kernel_reps)
    w = K_RANK + P_OVER
    flops = 32.0 * M * N * w                      # algorithmic flops of one view (16 real FMAs per qMAC)
    t_view = 0.5 * (kt[0] + kt[1])
    achieved = flops / t_view
    traffic = None
    if os.path.exists(PMC_FILE):
        pmc = json.load(open(PMC_FILE))
        if pmc.get("kernel_source_hash") == kernel_source_hash():
            traffic = pmc.get("hbm_bytes_per_launch")
    roofline = {"bound": "mfma", "achieved": round(achieved / 1e12, 3), "peak": PEAK_FP32_MFMA / 1e12,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 4), "traffic": traffic,
                "kernel": "k_qgemm FP32 view product, 2048x2048 by 60 quaternion columns",
                "t_forward_us": round(kt[0] * 1e6, 2), "t_adjoint_us": round(kt[1] * 1e6, 2),
                "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": 16.0 * M * N + 2 * 16.0 * N * w}

    for name in lowp:
        lowp[name]["view_speedup_vs_fp32"] = round(t_view / (0.5 * (lowp[name]["view_kernel_us"]["forward"] +
                                                                   lowp[name]["view_kernel_us"]["adjoint"]) * 1e-6), 3)
    print("accuracy against the oracle", file=sys.stderr, flush=True)
    acc_all = accuracy(Q, torch, A, A_np, precisions)
    acc = acc_all["fp32"]
    for name in lowp:
        lowp[name]["accuracy"] = acc_all[name]
        lowp[name]["max_error_ratio"] = round(max(r["ratio"] for r in acc_all[name]), 8)
    serve = None
    if not args.no_serve:
        print(f"serving stream ({args.serve_requests} requests)", file=sys.stderr, flush=True)
        serve = serving(Q, torch, args.serve_requests)
    comp = None if args.no_completion else completion(Q, torch, W)
    big = None if args.no_large else large(Q, torch)
    cpu = None if args.no_cpu_baseline else cpu_baseline(A_np)
    line = {"metric": "A-passes/s", "value": round(value, 3), "unit": "A-passes/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded; Haar quaternion unitaries, exp(-i/20) spectrum + Gaussian noise)",
            "config": {"workload": "dense quaternion 2048x2048 FP32, sigma_i=exp(-i/20)+N(0,1e-4) noise, "
                                   "k=50, p=10, subspace scheme (Alg. 2), budgets v=2,3,4,6 per step",
                       "m": M, "n": N, "k": K_RANK, "p": P_OVER, "budgets": list(BUDGETS),
                       "passes_per_step": sum(BUDGETS)},
            "step": "the solves of the four budgets, concurrently (the current stream and three others)",
            "sequential_value": round(sequential_value, 3),
            "qgemm_tflops": round(achieved / 1e12, 3), "solve_ms": per_v, "accuracy": acc,
            "roofline": roofline, "cpu_baseline": cpu,
            "precision_form": {"views": "1..v-2 reduced (FP32 accumulation), v-1 and v FP32 (split: v-1 and v as three "
                                        "BF16 products of values and residuals); Gram/Cholesky/QSVD FP64",
                               **lowp},
            "serving": serve, "completion": comp, "large": big}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
