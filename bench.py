"""Benchmark: selected-basis Davidson solve on one MI355X.

One step = one whole solve of the hot path on a synthetic workload: basis
build (sort/dedupe), excitation tables, Hamiltonian set-up (diagonal and
coefficients), and the Davidson iteration to ||r|| <= 1e-6 in the chosen form
(FP32 sigma with FP64 Gram-Schmidt / Rayleigh-Ritz / residuals and FP64
refinement).  ``value`` is whole-job throughput: determinants solved per
second (N x steps / wall time).  Also reported: sigma determinants/s per
precision, the plain-FP64 solve of the same workload, time to 1e-6 Ha for
both, the dominant kernel's roofline, the CPU oracle's sigma rate, and the
serving stream (continuous batching of 256 solves, p50/p99 latency).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sel26]
"""
import argparse
import hashlib
import json
import os
import sys
import time

# One hardware queue per serving worker stream (HIP's default is 4 per process):
# with fewer, a small request's kernels wait behind a large request's kernels in
# a shared queue.  Must be set before the runtime starts.
os.environ["GPU_MAX_HW_QUEUES"] = "16"

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU = 157.3e12  # MI355X fp32 vector FLOP/s
PEAK_FP64_VALU = 78.6e12
PEAK_HBM = 8.0e12
# Davidson subspace of the timed solves (the workload allows up to 20): the
# update passes stream the whole subspace, and at sel26 a 10-vector subspace
# needs about the same number of iterations as 20 (28-30 vs 26-28).
MAX_SPACE = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sigma kernel source (the row-stream kernel and its launcher
    live in k_sigma.hip): traffic figures are valid only for it."""
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_2601_16637_amd", "csrc", "k_sigma.hip"), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/sigma_traffic.txt, lines 'kernel workload source_hash bytes'),
    or None if it is missing or was taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", "sigma_traffic.txt")
    if not os.path.exists(p):
        return None
    for line in open(p):
        f = line.split()
        if len(f) == 4 and not line.startswith("#") and f[0] == kernel and f[1] == workload:
            return float(f[3]) if f[2] == kernel_source_hash() else None
    return None


def time_to(hist_theta, hist_time, e_ref, tol=1e-6):
    for th, t in zip(hist_theta, hist_time):
        if abs(th - e_ref) <= tol:
            return t
    return None


def sigma_stages(sbd, H, N, prec, stream, reps=10):
    """Mean per-stage milliseconds of sigma over reps launches (HIP events)."""
    import torch
    dt = torch.float64 if prec == sbd.FP64 else torch.float32
    x = torch.randn(N, device="cuda", dtype=dt)
    y = torch.empty_like(x)
    for _ in range(2):
        sbd.sigma(H, x, y, prec=prec, shift=-200.0, stream=stream)
    acc = None
    for _ in range(reps):
        st = sbd.sigma_timed(H, x, y, prec=prec, shift=-200.0, stream=stream)
        acc = st if acc is None else {k: acc[k] + st[k] for k in st}
    return {k: v / reps for k, v in acc.items()}


def stream_kernel_name(tune):
    """Instantiation of the FP32 single-vector row stream that a tune selects
    (columns per lane: 2, or 4 with 16-byte loads; output rows per wavefront,
    or ket entries per load step in the ket-split form)."""
    vec = 4 if tune['stream_wide'] else 2
    if tune.get('stream_split', 1) > 1:
        return f"k_stream_ks<float,1,{vec},{tune['stream_split']}>"
    return f"k_stream<float,1,{vec},{tune['stream_rw']}>"


def kernel_only(sbd, W, stream):
    """Short run for hardware-counter passes: five FP32 sigma launches and one
    device copy of known size (2 * N * 4 bytes) used to calibrate the counters."""
    import torch
    B = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, stream=stream)
    X = sbd.Excitations(B, stream=stream)
    H = sbd.Hamiltonian(B, X, W.h, W.eri, W.e_core, stream=stream)
    H.autotune(sbd.FP32, stream=stream)
    x = torch.randn(W.ndet, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    for _ in range(5):
        sbd.sigma(H, x, y, prec=sbd.FP32, shift=-200.0, stream=stream)
    z = torch.empty_like(x)
    z.copy_(x)
    torch.cuda.synchronize()
    tune = H.get_tune(sbd.FP32)
    print(json.dumps(dict(kernel_only=True, workload=W.name, ndet=W.ndet,
                          copy_bytes_read=4 * W.ndet, copy_bytes_written=4 * W.ndet,
                          tune=tune, stream_kernel=stream_kernel_name(tune))))


def cpu_baseline(W, target_s=15.0):
    """Oracle sigma rate (determinants/s) on a bounded random sample of rows."""
    import oracle
    S = oracle.OracleSystem.from_workload(W)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(S.N)
    idx = rng.integers(0, S.N, 4000)
    t0 = time.perf_counter()
    S.sigma_at(x, idx)
    dt = time.perf_counter() - t0
    m = int(min(max(4000 * target_s / max(dt, 1e-3), 4000), 5_000_000))
    idx = rng.integers(0, S.N, m)
    t0 = time.perf_counter()
    S.sigma_at(x, idx)
    dt = time.perf_counter() - t0
    return dict(value=m / dt, unit="det/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"FP64 sigma of {m} random determinants of the same basis "
                       f"({dt:.1f} s, C oracle, OpenMP over rows)")


def serving(sbd, wl, nreq=256, budget=96 << 30, inflight=16):
    """Serving stream: Poisson arrivals at 20/s of solves with 1e4-2e7
    determinants (norb 12-32, 1-2 roots, FP32 sigma + FP64 refinement);
    each request is generated at its arrival time and submitted then."""
    descs = wl.serving_stream(nreq=nreq)
    srv = sbd.Server(budget, inflight)
    t0 = time.perf_counter()
    tickets = []
    for d in descs:
        W = wl.make_request(d)
        delay = d["arrival"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append((W, srv.submit(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, W.h, W.eri,
                                      W.e_core, W.nroots, sigma_prec=sbd.FP32, tol_residual=1e-6,
                                      max_space=20)))
        if len(tickets) % 64 == 0:
            log(f"[bench] serving: {len(tickets)} requests submitted")
    res = [(W, srv.wait(t)) for W, t in tickets]
    wall = time.perf_counter() - t0
    srv.close()
    bad = [r for _, r in res if r["status"] < 0]
    lat = np.array([r["latency_ms"] for _, r in res])
    dets = sum(r["ndet"] for _, r in res)
    apps = sum(r["ndet"] * r["report"]["sigma_calls"] for _, r in res)
    conv = sum(1 for _, r in res if r["report"]["converged"])
    return dict(requests=nreq, rate_per_s=20.0, budget_bytes=budget, max_inflight=inflight,
                hw_queues=int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                failed=len(bad), converged=conv, wall_s=wall,
                latency_p50_ms=float(np.percentile(lat, 50)),
                latency_p99_ms=float(np.percentile(lat, 99)),
                queue_p99_ms=float(np.percentile([r["queue_ms"] for _, r in res], 99)),
                determinants_per_s=dets / wall, sigma_determinants_per_s=apps / wall,
                max_request_ndet=int(max(r["ndet"] for _, r in res)))


def _csv_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _col(row, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(names)


def _short(name):
    """Kernel name without namespaces, return type and argument list."""
    n = name.replace("sbd::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    if n.startswith("void "):
        n = n[5:]
    depth = 0
    for i, ch in enumerate(n):
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            n = n[:i]
            break
    return n.replace(", ", ",").strip()


def stats_summary(csv_path, top=25):
    """Markdown table of a rocprofv3 --stats kernel summary (kernel_stats.csv)."""
    rows = _csv_rows(csv_path)
    rows.sort(key=lambda r: -float(_col(r, "TotalDurationNs")))
    out = ["| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{_short(_col(r, 'Name'))}` | {_col(r, 'Calls')} | "
                   f"{float(_col(r, 'TotalDurationNs')) / 1e6:.2f} | "
                   f"{float(_col(r, 'AverageNs')) / 1e3:.1f} | {float(_col(r, 'Percentage')):.1f} |")
    return "\n".join(out)


def _counter_values(csv_path, counter):
    """Counter value of every dispatch, per short kernel name."""
    acc = {}
    per_dispatch = {}
    for r in _csv_rows(csv_path):
        if _col(r, "Counter_Name") != counter:
            continue
        key = (_col(r, "Dispatch_Id"), _short(_col(r, "Kernel_Name")))
        per_dispatch[key] = per_dispatch.get(key, 0.0) + float(_col(r, "Counter_Value"))
    for (_, k), v in per_dispatch.items():
        acc.setdefault(k, []).append(v)
    return acc


def traffic_summary(fetch_csv, write_csv, kernel_json, workload):
    """HBM bytes per launch of `kernel` from FETCH_SIZE / WRITE_SIZE runs (KiB per
    dispatch), each scaled by what the counter reads for the calibration copy of
    known size in the same --kernel-only run."""
    info = json.loads([l for l in open(kernel_json) if l.startswith("{")][-1])
    kernel = info["stream_kernel"]
    fv = _counter_values(fetch_csv, "FETCH_SIZE")
    wv = _counter_values(write_csv, "WRITE_SIZE")
    # the calibration copy is the largest blit of the run (the others upload inputs)
    copy = next(k for k in fv if "copyBuffer" in k)
    fetch = {k: sum(v) / len(v) for k, v in fv.items()}
    write = {k: sum(v) / len(v) for k, v in wv.items()}
    fetch[copy], write[copy] = max(fv[copy]), max(wv[copy])
    f_scale = info["copy_bytes_read"] / (1024.0 * fetch[copy])
    w_scale = info["copy_bytes_written"] / (1024.0 * write[copy])
    kf, kw = fetch[kernel] * 1024.0, write[kernel] * 1024.0
    total = kf * f_scale + kw * w_scale
    lines = [f"# {kernel} on {workload}: FETCH_SIZE {fetch[kernel]:.0f} KiB/dispatch (x{f_scale:.3f}), "
             f"WRITE_SIZE {write[kernel]:.0f} KiB/dispatch (x{w_scale:.3f}); calibration copy "
             f"{copy}: read {info['copy_bytes_read']} B, FETCH_SIZE {fetch[copy]:.0f} KiB, "
             f"WRITE_SIZE {write[copy]:.0f} KiB",
             f"# mean over {len(fv[kernel])} dispatches (alpha and beta launches)",
             f"{kernel} {workload} {kernel_source_hash()} {total:.0f}"]
    return "\n".join(lines)


def block_leg(sbd, wl, stream):
    """Block workload (block20: 4 roots): chosen form = FP32 sigma with FP64
    refinement, interleaved block sigma, sigma sequences replayed from HIP
    graphs; plain = FP64 sigma one vector at a time.  Each form is solved once
    untimed (autotuning, graph capture) and once timed, from scratch."""
    W = wl.make_config("block20")

    def solve(prec, block, graph):
        B = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, stream=stream)
        X = sbd.Excitations(B, stream=stream)
        H = sbd.Hamiltonian(B, X, W.h, W.eri, W.e_core, stream=stream)
        e, rep, st = sbd.davidson(H, W.nroots, stream=stream, tol_residual=1e-6, sigma_prec=prec,
                                  max_space=20, use_autotune=1, use_graph=graph, block_sigma=block)
        return e, rep

    out = {}
    for name, prec, block, graph in (("chosen", sbd.FP32, 1, 1), ("plain_fp64", sbd.FP64, 0, 0)):
        solve(prec, block, graph)
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, rep = solve(prec, block, graph)
        torch.cuda.synchronize()
        out[name] = dict(ms_solve=1e3 * (time.perf_counter() - t0), iterations=rep["iterations"],
                         sigma_calls=rep["sigma_calls"], sigma_calls_fp64=rep["sigma_calls_fp64"],
                         energies=[float(v) for v in e[:W.nroots]])
    out["energy_max_diff"] = float(max(abs(a - b) for a, b in zip(out["chosen"]["energies"],
                                                               out["plain_fp64"]["energies"])))
    out.update(workload="block20", determinants=W.ndet, nroots=W.nroots, tol_residual=1e-6)
    return out


def sqd_leg(sbd, wl, stream, sequences=(("coarse", (6000, 8000, 10000)), ("fine", (9000, 9500, 10000)))):
    """Successive solves of an SQD run on a growing configuration set: sel26
    string sets of increasing size per spin (nested: the same seeds draw the
    larger sets as supersets), in a coarse and a fine growth sequence.  Cold:
    each solve starts from the unit vector on the lowest diagonal entry.  Warm:
    each solve after the first starts from the previous eigenvector carried
    into the new basis (sbd_map_vectors).  Chosen form (FP32 sigma, FP64
    refinement); each sequence runs once untimed (autotuning of its shapes) and
    then cold and warm, timed, basis, tables and Hamiltonian included."""
    import torch

    def run(Ws, warm):
        steps, prev = [], None
        for W in Ws:
            t0 = time.perf_counter()
            B = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, stream=stream)
            X = sbd.Excitations(B, stream=stream)
            H = sbd.Hamiltonian(B, X, W.h, W.eri, W.e_core, stream=stream)
            kw = {}
            if warm and prev is not None:
                g = torch.empty(W.ndet, device="cuda", dtype=torch.float64)
                sbd.map_vectors(prev[0], B, prev[1], g, stream=stream)
                kw = dict(guess=g.view(1, -1), n_guess=1)
            v = torch.empty(W.ndet, device="cuda", dtype=torch.float64)
            e, rep, st = sbd.davidson(H, 1, vectors=v, stream=stream, tol_residual=1e-6, sigma_prec=sbd.FP32,
                                      max_space=MAX_SPACE, use_autotune=1, **kw)
            torch.cuda.synchronize()
            steps.append(dict(strings_per_spin=int(W.alpha.size), determinants=W.ndet,
                              ms=1e3 * (time.perf_counter() - t0), solver_ms=rep["t_total_ms"],
                              iterations=rep["iterations"], sigma_calls=rep["sigma_calls"],
                              energy=float(e[0]), status=int(st)))
            prev = (B, v)
        return steps

    out = dict(workload="sel26 nested string sets", tol_residual=1e-6)
    for name, sizes in sequences:
        Ws = [wl.make_config("sel26", nstr=n) for n in sizes]
        run(Ws, False)
        cold, warm = run(Ws, False), run(Ws, True)
        out[name] = dict(strings_per_spin=list(sizes), cold=cold, warm=warm,
                         cold_ms=sum(x["ms"] for x in cold), warm_ms=sum(x["ms"] for x in warm),
                         energy_max_diff=max(abs(a["energy"] - b["energy"]) for a, b in zip(cold, warm)))
    return out


def assembled_leg(sbd, wl, stream, cases=(("sel16", 300), ("sel16", 1000), ("sel16", None))):
    """Explicit (assembled CSR) against matrix-free realization of H on sel16
    bases of 9e4, 1e6 and 4e6 determinants: assembly time and size, sigma time
    per precision with each realization, the CSR product's algorithmic HBM rate
    (stored entries x (value + 4-byte column) + row pointers + x and y once),
    and a chosen-form solve with each."""
    import torch

    out = []
    for name, nstr in cases:
        W = wl.make_config(name, nstr=nstr)
        B = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, stream=stream)
        X = sbd.Excitations(B, stream=stream)
        H = sbd.Hamiltonian(B, X, W.h, W.eri, W.e_core, stream=stream)
        N = W.ndet
        row = dict(workload=f"{name} ({W.alpha.size} strings per spin)", determinants=N)

        def sig_ms(prec):
            dt = torch.float64 if prec == sbd.FP64 else torch.float32
            x = torch.randn(N, device="cuda", dtype=dt)
            y = torch.empty_like(x)
            sbd.sigma(H, x, y, prec=prec, shift=-200.0, stream=stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(torch.cuda.current_stream())
            for _ in range(10):
                sbd.sigma(H, x, y, prec=prec, shift=-200.0, stream=stream)
            e1.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / 10

        def solve_ms():
            sbd.davidson(H, 1, stream=stream, tol_residual=1e-6, sigma_prec=sbd.FP32, use_autotune=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, rep, st = sbd.davidson(H, 1, stream=stream, tol_residual=1e-6, sigma_prec=sbd.FP32, use_autotune=1)
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - t0), float(e[0]), rep["iterations"]

        H.autotune(sbd.FP64, stream=stream)
        H.autotune(sbd.FP32, stream=stream)
        row["free_sigma_ms"] = {"f64": sig_ms(sbd.FP64), "f32": sig_ms(sbd.FP32)}
        row["free_solve_ms"], e_free, row["free_iterations"] = solve_ms()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nnz = H.assemble(3, stream=stream)
        torch.cuda.synchronize()
        row["assemble_ms"] = 1e3 * (time.perf_counter() - t0)
        row["stored_entries"] = nnz
        row["csr_bytes"] = nnz * (4 + 8 + 4) + 8 * (N + 1)
        row["csr_sigma_ms"] = {"f64": sig_ms(sbd.FP64), "f32": sig_ms(sbd.FP32)}
        for key, vb in (("f64", 8), ("f32", 4)):
            bytes_ = nnz * (vb + 4) + 8 * (N + 1) + 2 * vb * N
            row.setdefault("csr_hbm_TBps", {})[key] = bytes_ / (row["csr_sigma_ms"][key] * 1e-3) / 1e12
        row["csr_solve_ms"], e_csr, row["csr_iterations"] = solve_ms()
        row["energy_diff"] = abs(e_csr - e_free)
        H.release_assembled()
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sel26")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-block", action="store_true")
    ap.add_argument("--no-sqd", action="store_true")
    ap.add_argument("--no-assembled", action="store_true")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only a few sigma launches and a calibration copy (counter runs)")
    ap.add_argument("--stats-summary", metavar="KERNEL_STATS_CSV",
                    help="print a markdown summary of a rocprofv3 --stats run and exit")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "KERNEL_ONLY_LOG"),
                    help="print calibrated HBM bytes per launch of the dominant kernel and exit")
    args = ap.parse_args()
    if args.stats_summary:
        print(stats_summary(args.stats_summary))
        return
    if args.traffic_summary:
        print(traffic_summary(*args.traffic_summary, workload=args.workload))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU path is not built "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2601_16637_amd as sbd
    import workload as wl

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    W = wl.make_config(args.workload)
    N = W.ndet
    tol = 1e-6
    log(f"[bench] workload {W.name}: norb={W.norb} n={W.n_alpha} strings={W.alpha.size}x"
        f"{W.beta.size} N={N} roots={W.nroots}")
    if args.kernel_only:
        kernel_only(sbd, W, stream)
        return

    def solve(prec, tol_r):
        B = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, stream=stream)
        X = sbd.Excitations(B, stream=stream)
        H = sbd.Hamiltonian(B, X, W.h, W.eri, W.e_core, stream=stream)
        e, rep, st = sbd.davidson(H, W.nroots, stream=stream, tol_residual=tol_r,
                                  sigma_prec=prec, max_space=MAX_SPACE, use_autotune=1)
        return e, rep, st, (B, X, H)

    for i in range(args.warmup):
        e, rep, st, _ = solve(sbd.FP32, tol)
        log(f"[bench] warmup {i}: E={e[0]:.10f} it={rep['iterations']} "
            f"t={rep['t_total_ms']:.1f} ms")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for i in range(args.steps):
        e, rep, st, _ = solve(sbd.FP32, tol)
        reps.append((e, rep))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    applications = sum(r["sigma_calls"] for _, r in reps)
    value = N * args.steps / dt
    e_mixed = reps[-1][0]
    rep_m = reps[-1][1]
    log(f"[bench] timed: {args.steps} steps {ms_per_step:.1f} ms/step, sigma apps "
        f"{applications}, E={e_mixed[0]:.10f}")

    extra = {}
    if not args.no_plain:
        tp = time.perf_counter()
        e64, rep64, st64, keep = solve(sbd.FP64, tol)
        torch.cuda.synchronize()
        t_plain = 1e3 * (time.perf_counter() - tp)
        # tight FP64 reference energy for time-to-1e-6 Ha
        eref, repref, _ = sbd.davidson(keep[2], W.nroots, stream=stream, tol_residual=1e-8,
                                       sigma_prec=sbd.FP64, max_space=20, use_autotune=1)
        ttp = time_to(rep64["theta_history"], rep64["time_history_ms"], eref[0])
        ttm = time_to(rep_m["theta_history"], rep_m["time_history_ms"], eref[0])
        extra = dict(
            plain_fp64=dict(ms_solve=t_plain, iterations=rep64["iterations"],
                            sigma_calls=rep64["sigma_calls"], energy=float(e64[0]),
                            time_to_1e6_ms=ttp, sigma_ms=rep64["t_sigma_ms"],
                            update_ms=rep64["t_update_ms"]),
            chosen_fp32_sigma=dict(ms_solve=ms_per_step, iterations=rep_m["iterations"],
                                   sigma_calls=rep_m["sigma_calls"],
                                   sigma_calls_fp64=rep_m["sigma_calls_fp64"],
                                   energy=float(e_mixed[0]), time_to_1e6_ms=ttm,
                                   sigma_ms=rep_m["t_sigma_ms"], update_ms=rep_m["t_update_ms"]),
            reference_energy=float(eref[0]),
            energy_error_chosen_vs_fp64=float(abs(e_mixed[0] - eref[0])),
            energy_error_plain_vs_fp64=float(abs(e64[0] - eref[0])),
        )
        log(f"[bench] plain FP64: {t_plain:.1f} ms, E={e64[0]:.10f}; ref {eref[0]:.10f}")

    # dominant kernel: the FP32 same-spin row stream (two launches per sigma),
    # timed live with HIP events recorded on the launch stream
    B = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, stream=stream)
    X = sbd.Excitations(B, stream=stream)
    H = sbd.Hamiltonian(B, X, W.h, W.eri, W.e_core, stream=stream)
    H.autotune(sbd.FP32, stream=stream)
    kname = stream_kernel_name(H.get_tune(sbd.FP32))
    stages32 = sigma_stages(sbd, H, N, sbd.FP32, stream)
    H.autotune(sbd.FP64, stream=stream)
    stages64 = sigma_stages(sbd, H, N, sbd.FP64, stream)
    p1a, p2a = X.count(0, 1), X.count(0, 2)
    p1b, p2b = X.count(1, 1), X.count(1, 2)
    nnz = N + B.nb * (p1a + p2a) + B.na * (p1b + p2b) + p1a * p1b
    # algorithmic flops of the two stream launches: one multiply-add per
    # connected same-spin pair (+ the diagonal term and the spectator add of singles)
    f_alpha = 2.0 * (B.nb * (p1a + p2a) + N) + 1.0 * B.nb * p1a
    f_beta = 2.0 * B.na * (p1b + p2b) + 1.0 * B.na * p1b
    t_stream = (stages32["alpha_stream"] + stages32["beta_stream"]) * 1e-3
    achieved = (f_alpha + f_beta) / t_stream
    t_sig32 = sum(stages32.values()) * 1e-3
    t_sig64 = sum(stages64.values()) * 1e-3
    traffic = traffic_for(kname, W.name)
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_FP32_VALU / 1e12,
                    unit="TFLOP/s", frac=achieved / PEAK_FP32_VALU,
                    traffic=None if traffic is None else traffic,
                    # the measured bytes at the measured launch time, against the HBM peak
                    traffic_rate_TBps=None if traffic is None else traffic / (t_stream / 2) / 1e12,
                    traffic_frac_of_hbm_peak=None if traffic is None else traffic / (t_stream / 2) / PEAK_HBM,
                    kernel=f"{kname} (alpha and beta launches of one FP32 sigma)",
                    launch_ms=1e3 * t_stream / 2, algorithmic_flops_per_launch=(f_alpha + f_beta) / 2,
                    sigma_fp32_stage_ms=stages32, sigma_fp64_stage_ms=stages64,
                    sigma_fp32_det_per_s=N / t_sig32, sigma_fp64_det_per_s=N / t_sig64,
                    nnz_pairs=nnz, sigma_fp32_pair_flops_per_s=2.0 * nnz / t_sig32)
    log(f"[bench] sigma fp32 {1e3*t_sig32:.3f} ms ({stages32}), fp64 {1e3*t_sig64:.3f} ms; "
        f"stream {achieved/1e12:.2f} TFLOP/s")

    if not args.no_block:
        extra["block"] = block_leg(sbd, wl, stream)
        log(f"[bench] block: {extra['block']}")
    if not args.no_sqd:
        extra["sqd_loop"] = sqd_leg(sbd, wl, stream)
        for name in ("coarse", "fine"):
            q = extra["sqd_loop"][name]
            log(f"[bench] sqd loop {name} {q['strings_per_spin']}: cold {q['cold_ms']:.0f} ms "
                f"{[x['iterations'] for x in q['cold']]} it, warm {q['warm_ms']:.0f} ms "
                f"{[x['iterations'] for x in q['warm']]} it, energies {[round(x['energy'], 6) for x in q['warm']]}")
    if not args.no_assembled:
        extra["assembled"] = assembled_leg(sbd, wl, stream)
        for r in extra["assembled"]:
            log(f"[bench] assembled {r['workload']}: N={r['determinants']} entries={r['stored_entries']} "
                f"assemble {r['assemble_ms']:.1f} ms; sigma free {r['free_sigma_ms']} csr {r['csr_sigma_ms']} "
                f"({r['csr_hbm_TBps']} TB/s); solve free {r['free_solve_ms']:.1f} csr {r['csr_solve_ms']:.1f} ms")
    if not args.no_serving:
        extra["serving"] = serving(sbd, wl)
        log(f"[bench] serving: {extra['serving']}")
    cpu = None if args.no_cpu_baseline else cpu_baseline(W)
    out = dict(metric="determinants/s of whole Davidson solves to 1e-6 (chosen form: FP32 sigma "
                      "+ FP64 refinement); sigma determinants/s and time-to-1e-6 Ha, plain FP64 "
                      "vs chosen, alongside",
               value=value, unit="det/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=ms_per_step, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=W.name, norb=W.norb, n_alpha=W.n_alpha, n_beta=W.n_beta,
                           strings_per_spin=int(W.alpha.size), determinants=N,
                           nroots=W.nroots, tol_residual=tol, max_space=MAX_SPACE),
               sigma_applications_per_step=applications / args.steps,
               roofline=roofline, cpu_baseline=cpu, **extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
