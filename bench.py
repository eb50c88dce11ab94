"""Benchmark: the sigma = H c product and the Davidson solve on one MI355X.

One step = one sigma = H c in FP64 (the paper's `mult`: all five launches,
alpha-alpha, beta-beta and alpha-beta terms with the diagonal) on one vector of
the sel26 workload (N = 1e8 determinants), with the tables, Hamiltonian and
vector resident in device memory.  ``value`` = N x steps / wall time of the
timed steps (determinants/s, FP64).  Alongside, on the same workload: the FP32
sigma, per-stage times and the roofline report of each precision; the whole
Davidson solve to ||r|| <= 1e-6 in plain FP64 and in the chosen form (FP32
sigma with FP64 Gram-Schmidt / Rayleigh-Ritz / residuals and refinement),
repeated the same number of times, with per-solve phase splits and the time
to 1e-6 Ha of a tight FP64 reference energy; sigma rows of the sel16 and
block20 workloads; the block, SQD-loop (sbd_sqd_run on a sampled
configuration record), explicit-realization, full-bitstring,
device-driven-iteration and serving legs; and the CPU oracle's sigma rate.

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


def traffic_lines(workload):
    """{kernel: HBM bytes per launch} from the committed rocprofv3 counter
    summary (profiles/sigma_traffic.txt, lines 'kernel workload source_hash
    bytes') for kernels measured on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "sigma_traffic.txt")
    out = {}
    if not os.path.exists(p):
        return out
    for line in open(p):
        f = line.split()
        if len(f) == 4 and not line.startswith("#") and f[1] == workload and f[2] == kernel_source_hash():
            out[f[0]] = float(f[3])
    return out


def traffic_for(kernel, workload):
    """HBM bytes per launch of one kernel, or None if not measured on this source."""
    return traffic_lines(workload).get(kernel)


def time_to(hist_theta, hist_time, e_ref, tol=1e-6):
    for th, t in zip(hist_theta, hist_time):
        if abs(th - e_ref) <= tol:
            return t
    return None


def kernel_only(sbd, W, stream, prec):
    """Short run for hardware-counter passes: five sigma launches in precision
    `prec` in the handle's default launch configuration (no autotuning, so each
    stage runs exactly one kernel instantiation), then one device copy of known
    size (N elements of that precision read and written) that calibrates the
    counters."""
    import torch
    B = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, stream=stream)
    X = sbd.Excitations(B, stream=stream)
    H = sbd.Hamiltonian(B, X, W.h, W.eri, W.e_core, stream=stream)
    dt = torch.float64 if prec == sbd.FP64 else torch.float32
    w = 8 if prec == sbd.FP64 else 4
    x = torch.randn(W.ndet, device="cuda", dtype=dt)
    y = torch.empty_like(x)
    for _ in range(5):
        sbd.sigma(H, x, y, prec=prec, shift=-200.0, stream=stream)
    z = torch.empty_like(x)
    z.copy_(x)
    torch.cuda.synchronize()
    tune = H.get_tune(prec)
    c = table_counts(B, X)
    print(json.dumps(dict(kernel_only=True, workload=W.name, ndet=W.ndet, precision=prec,
                          copy_bytes_read=w * W.ndet, copy_bytes_written=w * W.ndet,
                          tune=tune, stream_kernel=stream_kernel(tune, prec), table_entries=c,
                          alpha_beta_fma=c["p1a"] * c["p1b"])))


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
    each request is generated at its arrival time and submitted then.
    Latency percentiles are also reported per size class, and the largest
    request is solved again alone on the idle server to split its latency
    into its own run time and the cost of sharing the device."""
    descs = wl.serving_stream(nreq=nreq)
    srv = sbd.Server(budget, inflight)
    kw = dict(sigma_prec=sbd.FP32, tol_residual=1e-6, max_space=20)
    t0 = time.perf_counter()
    tickets = []
    for d in descs:
        W = wl.make_request(d)
        delay = d["arrival"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append((W, srv.submit(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, W.h, W.eri,
                                      W.e_core, W.nroots, **kw)))
        if len(tickets) % 64 == 0:
            log(f"[bench] serving: {len(tickets)} requests submitted")
    res = [(W, srv.wait(t)) for W, t in tickets]
    wall = time.perf_counter() - t0
    bad = [r for _, r in res if r["status"] < 0]
    lat = np.array([r["latency_ms"] for _, r in res])
    dets = sum(r["ndet"] for _, r in res)
    apps = sum(r["ndet"] * r["report"]["sigma_calls"] for _, r in res)
    conv = sum(1 for _, r in res if r["report"]["converged"])
    classes = {}
    for cname, lo, hi in (("small_lt_1e5", 0, 1e5), ("medium_1e5_to_2e6", 1e5, 2e6), ("large_ge_2e6", 2e6, 1e30)):
        sel = [r for _, r in res if lo <= r["ndet"] < hi]
        if not sel:
            continue
        l = np.array([r["latency_ms"] for r in sel])
        q = np.array([r["queue_ms"] for r in sel])
        u = np.array([r["run_ms"] for r in sel])
        classes[cname] = dict(requests=len(sel), latency_p50_ms=float(np.percentile(l, 50)),
                              latency_p99_ms=float(np.percentile(l, 99)),
                              queue_p99_ms=float(np.percentile(q, 99)), run_p50_ms=float(np.percentile(u, 50)))
    # the largest request again, alone on the idle server
    Wl, rl = max(res, key=lambda p: p[1]["ndet"])
    alone = srv.wait(srv.submit(Wl.norb, Wl.n_alpha, Wl.n_beta, Wl.alpha, Wl.beta, Wl.h, Wl.eri,
                                Wl.e_core, Wl.nroots, **kw))
    srv.close()
    return dict(requests=nreq, rate_per_s=20.0, budget_bytes=budget, max_inflight=inflight,
                hw_queues=int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                failed=len(bad), converged=conv, wall_s=wall,
                latency_p50_ms=float(np.percentile(lat, 50)),
                latency_p99_ms=float(np.percentile(lat, 99)),
                queue_p99_ms=float(np.percentile([r["queue_ms"] for _, r in res], 99)),
                determinants_per_s=dets / wall, sigma_determinants_per_s=apps / wall,
                max_request_ndet=int(rl["ndet"]), classes=classes,
                largest_request=dict(ndet=int(rl["ndet"]), nroots=int(Wl.nroots), norb=int(Wl.norb),
                                     latency_in_mix_ms=rl["latency_ms"], run_in_mix_ms=rl["run_ms"],
                                     queue_in_mix_ms=rl["queue_ms"], run_alone_ms=alone["run_ms"],
                                     iterations=rl["report"]["iterations"],
                                     energies_equal=bool(np.array_equal(alone["energies"], rl["energies"]))))


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


def stats_summary(csv_path, top=25, prefix=None):
    """Markdown table of a rocprofv3 --stats kernel summary (kernel_stats.csv),
    optionally only of the kernels whose short name starts with `prefix` (or
    with one of several comma-separated prefixes)."""
    rows = _csv_rows(csv_path)
    if prefix:
        keep = tuple(p for p in prefix.split(",") if p)
        rows = [r for r in rows if _short(_col(r, "Name")).startswith(keep)]
    rows.sort(key=lambda r: -float(_col(r, "TotalDurationNs")))
    out = ["| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        name = _short(_col(r, "Name"))
        if len(name) > 80:
            name = name[:77] + "..."
        out.append(f"| `{name}` | {_col(r, 'Calls')} | "
                   f"{float(_col(r, 'TotalDurationNs')) / 1e6:.2f} | "
                   f"{float(_col(r, 'AverageNs')) / 1e3:.1f} | {float(_col(r, 'Percentage')):.1f} |")
    return "\n".join(out)


def launch_gaps(trace_csv):
    """Idle time between the five launches of each FP64 single-vector sigma
    (transpose, two row streams, alpha-beta, transpose-add) in a rocprofv3
    --kernel-trace run: per sigma, the sum over the four launch boundaries of
    (start of a launch - end of the one before it)."""
    rows = _csv_rows(trace_csv)
    rows.sort(key=lambda r: int(_col(r, "Start_Timestamp")))
    names = [_short(_col(r, "Kernel_Name")) for r in rows]
    stages = ("k_transpose<double,1,false>", "k_stream", "k_stream", "k_ab", "k_transpose<double,1,true>")
    seqs = {}
    for i in range(len(rows) - 4):
        if not all(names[i + j].startswith(stages[j]) for j in range(5)):
            continue
        g = sum(int(_col(rows[i + j + 1], "Start_Timestamp")) - int(_col(rows[i + j], "End_Timestamp"))
                for j in range(4))
        span = int(_col(rows[i + 4], "End_Timestamp")) - int(_col(rows[i], "Start_Timestamp"))
        seqs.setdefault(tuple(names[i:i + 5]), []).append((g / 1e3, span / 1e3))
    if not seqs:
        return "no FP64 single-vector sigma sequence in the trace"
    # the launch configuration the run used most (the benchmark's steps; the
    # autotuner's candidates and the per-stage timing, which records events
    # between the stages, appear less often)
    key, v = max(seqs.items(), key=lambda kv: len(kv[1]))
    gaps = [a for a, _ in v]
    spans = [b for _, b in v]
    return (f"{len(v)} sigma sequences of {' -> '.join(key)}: launch gaps per sigma median "
            f"{float(np.median(gaps)):.1f} us, max {max(gaps):.1f} us; sigma span median "
            f"{float(np.median(spans)):.1f} us")


def _counter_values_all(csv_paths, counter):
    """_counter_values over several runs, dispatch values pooled per kernel."""
    acc = {}
    for path in csv_paths:
        for k, v in _counter_values(path, counter).items():
            acc.setdefault(k, []).extend(v)
    return acc


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


SIGMA_KERNELS = ("k_transpose", "k_transpose_v", "k_stream", "k_stream_ks", "k_ab", "k_ab2")


def counters_summary(csv_paths):
    """Markdown table of the L1/L2-side counters of every sigma kernel from
    rocprofv3 --pmc runs (counter_collection.csv files), each counter averaged
    over the kernel's dispatches: L1 TLB miss rate, L1->L2 read requests, L2
    hits, misses and miss rate, mean L1->L2 read latency in cycles, and the
    wavefront-level vector and scalar instruction counts and wavefronts where
    a run collected them."""
    names = ("TCP_UTCL1_TRANSLATION_MISS_sum", "TCP_UTCL1_REQUEST_sum", "TCP_TCC_READ_REQ_sum",
             "TCP_TCC_READ_REQ_LATENCY_sum", "TCC_HIT_sum", "TCC_MISS_sum")
    vals = {n: {} for n in names}
    for path in csv_paths:
        for n in names:
            for k, v in _counter_values(path, n).items():
                vals[n].setdefault(k, []).extend(v)
    mean = {n: {k: sum(v) / len(v) for k, v in d.items()} for n, d in vals.items()}
    kernels = sorted({k for d in mean.values() for k in d if k.split("<")[0] in SIGMA_KERNELS})

    def get(n, k):
        return mean[n].get(k)

    sq = {n: {k: sum(v) / len(v) for k, v in _counter_values_all(csv_paths, n).items()}
          for n in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_WAVES")}
    out = ["| kernel | TLB miss | L1->L2 reads | L2 hit | L2 miss | miss % | latency | VALU insts | SALU insts | waves |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    for k in kernels:
        tm, tr = get(names[0], k), get(names[1], k)
        rq, lat = get(names[2], k), get(names[3], k)
        hit, miss = get(names[4], k), get(names[5], k)
        cell = lambda v, f: "-" if v is None else f.format(v)
        tlb = f"{100.0 * tm / tr:.3f} %" if tm is not None and tr else "-"
        mp = f"{100.0 * miss / (hit + miss):.1f}" if hit is not None and miss is not None and hit + miss > 0 else "-"
        lt = f"{lat / rq:.0f}" if lat is not None and rq else "-"
        out.append(f"| `{k}` | {tlb} | {cell(rq, '{:.3g}')} | {cell(hit, '{:.3g}')} | {cell(miss, '{:.3g}')} | "
                   f"{mp} | {lt} | {cell(sq['SQ_INSTS_VALU'].get(k), '{:.3g}')} | "
                   f"{cell(sq['SQ_INSTS_SALU'].get(k), '{:.3g}')} | {cell(sq['SQ_WAVES'].get(k), '{:.3g}')} |")
    return "\n".join(out)


def traffic_summary(fetch_csv, write_csv, kernel_json, workload):
    """HBM bytes per launch of every sigma kernel of a --kernel-only run from
    FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch, averaged over the kernel's
    dispatches), each scaled by what the counter reads for the calibration copy
    of known size in the same run."""
    info = json.loads([l for l in open(kernel_json) if l.startswith("{")][-1])
    fv = _counter_values(fetch_csv, "FETCH_SIZE")
    wv = _counter_values(write_csv, "WRITE_SIZE")
    # the calibration copy is the largest blit of the run (the others upload inputs)
    copy = next(k for k in fv if "copyBuffer" in k)
    fetch = {k: sum(v) / len(v) for k, v in fv.items()}
    write = {k: sum(v) / len(v) for k, v in wv.items()}
    fetch[copy], write[copy] = max(fv[copy]), max(wv[copy])
    f_scale = info["copy_bytes_read"] / (1024.0 * fetch[copy])
    w_scale = info["copy_bytes_written"] / (1024.0 * write[copy])
    lines = [f"# calibration copy {copy}: read {info['copy_bytes_read']} B, FETCH_SIZE {fetch[copy]:.0f} KiB "
             f"(x{f_scale:.3f}), written {info['copy_bytes_written']} B, WRITE_SIZE {write[copy]:.0f} KiB "
             f"(x{w_scale:.3f})"]
    data = []
    for kernel in sorted(fv):
        if not kernel.split("<")[0] in SIGMA_KERNELS or kernel not in wv:
            continue
        kf, kw = fetch[kernel] * 1024.0, write[kernel] * 1024.0
        total = kf * f_scale + kw * w_scale
        lines.append(f"# {kernel}: FETCH_SIZE {fetch[kernel]:.0f} KiB, WRITE_SIZE {write[kernel]:.0f} KiB per "
                     f"dispatch, mean over {len(fv[kernel])} dispatches")
        data.append(f"{kernel} {workload} {kernel_source_hash()} {total:.0f}")
    return "\n".join(lines + data)


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


def sqd_leg(sbd, wl, stream, steps=(2500, 5000, 7500, 10000)):
    """SQD outer loop (sbd_sqd_run, Sec. I) on a synthetic measurement record:
    norb 26 with 7 + 7 electrons (the sel26 integrals), configurations drawn
    with level weights, taken in growing prefixes; each step diagonalises over
    the product of the distinct sampled strings (up to 1e8 determinants) in
    the chosen form, cold and warm (previous eigenvector carried over); the
    same record with bit-flip noise and sample recovery; and full-bitstring
    steps over the full16 list."""
    import torch
    W = wl.make_config("sel26", nstr=10)
    smp = wl.sample_configurations(W.norb, W.n_alpha, W.n_beta, max(steps), 3101)
    out = dict(workload="sel26 integrals, sampled configurations", samples=max(steps), tol_residual=1e-6)
    kw = dict(sigma_prec=sbd.FP32, tol_residual=1e-6, max_space=MAX_SPACE, use_autotune=1)
    # untimed pass over every step first: the autotuner's measurements of each shape are cached
    sbd.sqd_run(W.norb, W.n_alpha, W.n_beta, W.h, W.eri, W.e_core, smp, steps, stream=stream, **kw)
    for name, warm in (("cold", False), ("warm", True)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, rep = sbd.sqd_run(W.norb, W.n_alpha, W.n_beta, W.h, W.eri, W.e_core, smp, steps, warm_start=warm,
                             stream=stream, **kw)
        torch.cuda.synchronize()
        out[name] = dict(ms=1e3 * (time.perf_counter() - t0), energies=[float(x) for x in e[:, 0]],
                         steps=[dict(samples=r["samples"], strings=[r["n_alpha_str"], r["n_beta_str"]],
                                     determinants=r["ndet"], iterations=r["iterations"],
                                     setup_ms=r["setup_ms"], solve_ms=r["solve_ms"], status=r["status"])
                                for r in rep])
    out["energy_max_diff"] = float(max(abs(a - b) for a, b in zip(out["cold"]["energies"], out["warm"]["energies"])))
    # the same record read out with bit-flip noise (each bit flipped with probability 0.003, so
    # about 7 % of the strings of each spin carry a wrong electron count), with recovery: wrong
    # samples dropped at the first step and corrected from the previous ground state after it
    noisy = wl.add_readout_noise(smp, W.norb, 0.003, 3103)
    rkw = dict(kw, recovery=True, recovery_seed=3104)
    sbd.sqd_run(W.norb, W.n_alpha, W.n_beta, W.h, W.eri, W.e_core, noisy, steps, stream=stream, **rkw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, rep = sbd.sqd_run(W.norb, W.n_alpha, W.n_beta, W.h, W.eri, W.e_core, noisy, steps, stream=stream, **rkw)
    torch.cuda.synchronize()
    out["recovery_warm"] = dict(workload="sel26 record with bit-flip noise 0.003, recovery",
                                ms=1e3 * (time.perf_counter() - t0), energies=[float(x) for x in e[:, 0]],
                                steps=[dict(samples=r["samples"], corrected=r["corrected"], dropped=r["dropped"],
                                            strings=[r["n_alpha_str"], r["n_beta_str"]], determinants=r["ndet"],
                                            iterations=r["iterations"], setup_ms=r["setup_ms"],
                                            solve_ms=r["solve_ms"], status=r["status"]) for r in rep])
    # full-bitstring steps: the basis of a step is the set of sampled determinants.  The record
    # is the full16 determinant list (drawn from the sel16 string product with level weights,
    # connected like a selected basis) in a random drawing order, taken in growing prefixes.
    F = wl.make_full_config("full16")
    fsmp = F.dets[np.random.default_rng(3102).permutation(F.dets.shape[0])]
    fsteps = (25000, 50000, 100000, 200000)
    sbd.sqd_run(F.norb, F.n_alpha, F.n_beta, F.h, F.eri, F.e_core, fsmp, fsteps, full_bitstring=True,
                stream=stream, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, rep = sbd.sqd_run(F.norb, F.n_alpha, F.n_beta, F.h, F.eri, F.e_core, fsmp, fsteps, full_bitstring=True,
                         stream=stream, **kw)
    torch.cuda.synchronize()
    out["full_bitstring_warm"] = dict(workload="full16 list, random drawing order",
                                      ms=1e3 * (time.perf_counter() - t0), energies=[float(x) for x in e[:, 0]],
                                      steps=[dict(samples=r["samples"], determinants=r["ndet"],
                                                  alpha_strings=r["n_alpha_str"], iterations=r["iterations"],
                                                  setup_ms=r["setup_ms"], solve_ms=r["solve_ms"],
                                                  status=r["status"]) for r in rep])
    return out


def full_leg(sbd, wl, stream):
    """Full-bitstring path (Sec. II-F, III-F) on determinant lists that are not
    Cartesian products (full16: 1e6, full26: 4e6 determinants drawn from the
    sel16 / sel26 string products): basis build (sort, groups, connections),
    Hamiltonian, sigma per precision, and plain / chosen-form solves; then the
    same with every connection's element kept (sbd_full_assemble, Sec. II-A)."""
    import torch
    out = []

    def sigma_ms(B, H, prec):
        dt = torch.float64 if prec == sbd.FP64 else torch.float32
        x = torch.randn(B.N, device="cuda", dtype=dt)
        y = torch.empty_like(x)
        sbd.full_sigma(H, x, y, prec=prec, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            sbd.full_sigma(H, x, y, prec=prec, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 10

    def solves(H):
        res = {}
        for form, prec in (("plain_fp64", sbd.FP64), ("chosen", sbd.FP32)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, rep, st = sbd.full_davidson(H, 1, stream=stream, tol_residual=1e-6, sigma_prec=prec,
                                           max_space=MAX_SPACE)
            torch.cuda.synchronize()
            res[form] = dict(ms=1e3 * (time.perf_counter() - t0), iterations=rep["iterations"],
                             sigma_calls=rep["sigma_calls"], energy=float(e[0]), status=int(st))
        return res

    for name in ("full16", "full26"):
        F = wl.make_full_config(name)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B = sbd.FullBasis(F.norb, F.n_alpha, F.n_beta, F.dets, stream=stream)
        t1 = time.perf_counter()
        H = sbd.FullHamiltonian(B, F.h, F.eri, F.e_core, stream=stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        row = dict(workload=name, determinants=B.N, connections=B.nconn, alpha_strings=B.nalpha,
                   basis_ms=1e3 * (t1 - t0), hamiltonian_ms=1e3 * (t2 - t1))
        for prec, tag in ((sbd.FP64, "f64"), (sbd.FP32, "f32")):
            ms = sigma_ms(B, H, prec)
            row[f"sigma_ms_{tag}"] = ms
            row[f"sigma_det_per_s_{tag}"] = B.N / (ms * 1e-3)
            row[f"connections_per_s_{tag}"] = (B.N + B.nconn) / (ms * 1e-3)
        row.update(solves(H))
        # explicit realization: the elements kept (12 bytes per connection for both precisions)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.assemble(3, stream=stream)
        asm = dict(assemble_ms=1e3 * (time.perf_counter() - t0), element_bytes=12 * B.nconn)
        for prec, tag in ((sbd.FP64, "f64"), (sbd.FP32, "f32")):
            ms = sigma_ms(B, H, prec)
            w = 8 if prec == sbd.FP64 else 4
            # algorithmic bytes: elements and ket indices once, x and y once, the diagonal once
            b = B.nconn * (w + 4) + 8 * (B.N + 1) + 2 * w * B.N + 8 * B.N
            asm[f"sigma_ms_{tag}"] = ms
            asm[f"hbm_TBps_{tag}"] = b / (ms * 1e-3) / 1e12
        asm.update(solves(H))
        asm["energy_diff_vs_matrix_free"] = abs(asm["plain_fp64"]["energy"] - row["plain_fp64"]["energy"])
        row["assembled"] = asm
        H.release_assembled()
        out.append(row)
        del H, B
    return out


def projection_leg(sbd, N, stream, rows=(4, 10, 20), reps=5):
    """HBM rate of the Davidson update's tall-skinny projection pass
    (sbd_gram: out = A^T x over ma rows of N doubles and one vector, the pass
    behind the Gram-Schmidt and Rayleigh-Ritz projections) at the benchmark's
    vector length: algorithmic bytes (ma + 1) 8 N per call over the median
    wall time of `reps` calls (each synchronises)."""
    import torch
    A = torch.randn(max(rows), N, device="cuda", dtype=torch.float64)
    x = torch.randn(N, device="cuda", dtype=torch.float64)
    out = []
    for ma in rows:
        sbd.gram(A, ma, x, 1, N, stream=stream)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sbd.gram(A, ma, x, 1, N, stream=stream)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        b = (ma + 1) * 8.0 * N
        out.append(dict(rows=ma, determinants=N, ms=1e3 * t, algorithmic_bytes=b, TBps=b / t / 1e12,
                        hbm_frac=b / t / PEAK_HBM))
    del A, x
    return out


def devloop_leg(sbd, wl, stream, sizes=(100, 300)):
    """Device-driven iterations (opts.device_iterations = 8, whole iterations
    replayed from one captured graph, one host synchronisation per batch)
    against host-driven ones (sigma sequences replayed from graphs) on small
    solves (sel16 subsets of 1e4 and 9e4 determinants), 1 and 2 roots, plain
    and chosen form; median of three solves each."""
    import torch
    out = []
    for nstr in sizes:
        W = wl.make_config("sel16", nstr=nstr)
        B = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, stream=stream)
        X = sbd.Excitations(B, stream=stream)
        H = sbd.Hamiltonian(B, X, W.h, W.eri, W.e_core, stream=stream)
        for prec in (sbd.FP64, sbd.FP32):
            for k in (1, 2):
                row = dict(determinants=W.ndet, roots=k, precision="f64" if prec == sbd.FP64 else "f32")
                for name, dev in (("host_driven", 0), ("device_driven", 8)):
                    kw = dict(tol_residual=1e-6, sigma_prec=prec, max_space=20, use_graph=1, device_iterations=dev,
                              use_autotune=1)
                    sbd.davidson(H, k, stream=stream, **kw)
                    ts = []
                    for _ in range(3):
                        torch.cuda.synchronize()
                        e, rep, st = sbd.davidson(H, k, stream=stream, **kw)
                        ts.append(rep["t_total_ms"])
                    t = float(np.median(ts))
                    row[name] = dict(ms=t, iterations=rep["iterations"], ms_per_iteration=t / rep["iterations"],
                                     device_iterations=rep["device_iterations"], energy=float(e[0]))
                out.append(row)
        del H, X, B
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


def stream_kernel(tune, prec):
    """Row-stream instantiation a tune selects for single-vector sigma: columns
    per lane (FP32: 2, or 4 with 16-byte loads; FP64: 1, or 2), output rows per
    wavefront, or ket entries per load step in the ket-split form."""
    t = "float" if prec == 1 else "double"
    vec = (4 if tune["stream_wide"] else 2) if prec == 1 else (2 if tune["stream_wide"] else 1)
    if tune.get("stream_split", 1) > 1:
        return f"k_stream_ks<{t},1,{vec},{tune['stream_split']}>"
    return f"k_stream<{t},1,{vec},{tune['stream_rw']}>"


def table_counts(B, X):
    p1a, p2a, p1b, p2b = X.count(0, 1), X.count(0, 2), X.count(1, 1), X.count(1, 2)
    N = B.na * B.nb
    nnz = N + B.nb * (p1a + p2a) + B.na * (p1b + p2b) + p1a * p1b
    return dict(p1a=p1a, p2a=p2a, p1b=p1b, p2b=p2b, nnz=nnz)


def sigma_report(sbd, W, B, X, H, prec, stream, nvec=1, reps=10):
    """Per-stage times and the measurement items of one sigma shape: det/s;
    fraction of the binding roof max(B/BW, F/P)/t with F = 2 k NNZ and B the
    compulsory bytes (k N (w_in + w_out) + 8 N diagonal + tables, coefficients
    and integrals); the HBM fraction (B/t)/BW beside its cap t_HBM/t_ALU; and
    the gather volume k w (NNZ - N)/t as an effective cache bandwidth."""
    import torch
    layout = 1 if nvec > 1 else 0
    H.autotune(prec, nvec=nvec, layout=layout, stream=stream)
    dt = torch.float64 if prec == sbd.FP64 else torch.float32
    N = W.ndet
    x = torch.randn(N * nvec, device="cuda", dtype=dt)
    y = torch.empty_like(x)
    for _ in range(2):
        sbd.sigma(H, x, y, nvec=nvec, prec=prec, shift=-200.0, layout=layout, stream=stream)
    acc = None
    for _ in range(reps):
        st = sbd.sigma_timed(H, x, y, nvec=nvec, prec=prec, shift=-200.0, layout=layout, stream=stream)
        acc = st if acc is None else {k: acc[k] + st[k] for k in st}
    stages = {k: v / reps for k, v in acc.items()}
    t = sum(stages.values()) * 1e-3
    c = table_counts(B, X)
    w = 8 if prec == sbd.FP64 else 4
    F = 2.0 * nvec * c["nnz"]
    tables = (c["p1a"] + c["p1b"]) * (8 + 8 + 4 + w) + (c["p2a"] + c["p2b"]) * (8 + 4 + w)
    Bytes = nvec * N * 2 * w + 8 * N + tables + W.norb ** 4 * w
    peak = PEAK_FP64_VALU if prec == sbd.FP64 else PEAK_FP32_VALU
    t_hbm, t_alu = Bytes / PEAK_HBM, F / peak
    return dict(workload=W.name, precision="f64" if prec == sbd.FP64 else "f32", vectors=nvec,
                determinants=N, stage_ms=stages, sigma_ms=1e3 * t, det_per_s=nvec * N / t,
                nnz_pairs=c["nnz"], flops=F, compulsory_bytes=Bytes,
                binding_roof="alu" if t_alu >= t_hbm else "hbm",
                binding_roof_frac=max(t_hbm, t_alu) / t, alu_frac=t_alu / t,
                hbm_frac=t_hbm / t, hbm_frac_cap=min(1.0, t_hbm / t_alu),
                gather_TBps=nvec * w * (c["nnz"] - N) / t / 1e12,
                tune=H.get_tune(prec))


def solve_runs(sbd, H, W, stream, reps, e_ref, tol):
    """Plain FP64 and chosen-form solves, alternating, `reps` of each; per
    solve: host wall time, the report's phases (workspace, autotune, sigma,
    update, the rest = host decisions and synchronisation), iterations and the
    time to |theta - e_ref| <= 1e-6 Ha."""
    import torch
    forms = (("plain_fp64", sbd.FP64), ("chosen", sbd.FP32))
    runs = {name: [] for name, _ in forms}
    for r in range(reps):
        for name, prec in forms:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, rep, st = sbd.davidson(H, W.nroots, stream=stream, tol_residual=tol, sigma_prec=prec,
                                      max_space=MAX_SPACE, use_autotune=1)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            other = rep["t_total_ms"] - rep["t_sigma_ms"] - rep["t_update_ms"] - rep["t_workspace_ms"] \
                - rep["t_autotune_ms"]
            runs[name].append(dict(ms=ms, solver_ms=rep["t_total_ms"], workspace_ms=rep["t_workspace_ms"],
                                   autotune_ms=rep["t_autotune_ms"], sigma_ms=rep["t_sigma_ms"],
                                   update_ms=rep["t_update_ms"], host_other_ms=other,
                                   iterations=rep["iterations"], sigma_calls=rep["sigma_calls"],
                                   sigma_calls_fp64=rep["sigma_calls_fp64"], energy=float(e[0]),
                                   energy_error=float(abs(e[0] - e_ref)), status=int(st),
                                   time_to_1e6_ms=time_to(rep["theta_history"], rep["time_history_ms"], e_ref)))
            log(f"[bench] solve {name} #{r}: {ms:.1f} ms, {rep['iterations']} it, "
                f"sigma {rep['t_sigma_ms']:.1f} update {rep['t_update_ms']:.1f} "
                f"workspace {rep['t_workspace_ms']:.1f} ms, E={e[0]:.10f}")
    out = {}
    for name, rs in runs.items():
        ms = np.array([x["ms"] for x in rs])
        tt = [x["time_to_1e6_ms"] for x in rs if x["time_to_1e6_ms"] is not None]
        out[name] = dict(runs=rs, median_ms=float(np.median(ms)), max_ms=float(ms.max()),
                         min_ms=float(ms.min()), max_over_median=float(ms.max() / np.median(ms)),
                         time_to_1e6_median_ms=float(np.median(tt)) if tt else None,
                         energy_error_max=float(max(x["energy_error"] for x in rs)))
    out["speedup_median"] = out["plain_fp64"]["median_ms"] / out["chosen"]["median_ms"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sel26")
    ap.add_argument("--solve-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="skip the sel16 / block20 sigma rows")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-block", action="store_true")
    ap.add_argument("--no-sqd", action="store_true")
    ap.add_argument("--no-assembled", action="store_true")
    ap.add_argument("--no-full", action="store_true", help="skip the full-bitstring leg")
    ap.add_argument("--no-devloop", action="store_true", help="skip the device-driven iteration leg")
    ap.add_argument("--no-projection", action="store_true", help="skip the projection-pass rate leg")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only a few sigma launches and a calibration copy (counter runs)")
    ap.add_argument("--prec", type=int, default=0, help="precision of --kernel-only (0 FP64, 1 FP32)")
    ap.add_argument("--stats-summary", metavar="KERNEL_STATS_CSV",
                    help="print a markdown summary of a rocprofv3 --stats run and exit")
    ap.add_argument("--stats-prefix", metavar="PREFIX",
                    help="with --stats-summary: only kernels whose name starts with PREFIX "
                         "(several prefixes separated by commas)")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "KERNEL_ONLY_LOG"),
                    help="print calibrated HBM bytes per launch of the dominant kernel and exit")
    ap.add_argument("--launch-gaps", metavar="KERNEL_TRACE_CSV",
                    help="print the idle time between the launches of each FP64 sigma in a kernel trace and exit")
    ap.add_argument("--counters-summary", nargs="+", metavar="COUNTER_CSV",
                    help="print the L1/L2-side counters of the sigma kernels from rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.launch_gaps:
        print(launch_gaps(args.launch_gaps))
        return
    if args.counters_summary:
        print(counters_summary(args.counters_summary))
        return
    if args.stats_summary:
        print(stats_summary(args.stats_summary, prefix=args.stats_prefix))
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
        kernel_only(sbd, W, stream, args.prec)
        return

    # set-up, once: basis, tables, Hamiltonian (strings and integrals uploaded from the host)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, stream=stream)
    t1 = time.perf_counter()
    X = sbd.Excitations(B, stream=stream)
    t2 = time.perf_counter()
    H = sbd.Hamiltonian(B, X, W.h, W.eri, W.e_core, stream=stream)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    setup = dict(basis_ms=1e3 * (t1 - t0), tables_ms=1e3 * (t2 - t1), hamiltonian_ms=1e3 * (t3 - t2))
    best64 = H.autotune(sbd.FP64, stream=stream)
    best32 = H.autotune(sbd.FP32, stream=stream)
    setup.update(autotune_best_ms_fp64=best64, autotune_best_ms_fp32=best32)
    log(f"[bench] set-up {setup}")

    # ---- the timed steps: FP64 sigma = H c on one resident vector
    x = torch.randn(N, device="cuda", dtype=torch.float64)
    x /= torch.linalg.vector_norm(x)
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        sbd.sigma(H, x, y, prec=sbd.FP64, stream=stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        sbd.sigma(H, x, y, prec=sbd.FP64, stream=stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    ms_per_step = 1e3 * dt / args.steps
    value = N * args.steps / dt
    log(f"[bench] timed: {args.steps} FP64 sigma steps {ms_per_step:.3f} ms/step "
        f"(events: median {np.median(step_ms):.3f}, max {step_ms.max():.3f} ms), {value:.3e} det/s")

    # ---- roofline of the dominant kernel of the FP64 sigma, and the measurement items
    rows = {}
    rows["sel26_f64"] = sigma_report(sbd, W, B, X, H, sbd.FP64, stream)
    rows["sel26_f32"] = sigma_report(sbd, W, B, X, H, sbd.FP32, stream)
    H.autotune(sbd.FP64, stream=stream)
    s64 = rows["sel26_f64"]["stage_ms"]
    c = table_counts(B, X)
    tune64 = H.get_tune(sbd.FP64)
    kname = stream_kernel(tune64, sbd.FP64)
    f_alpha = 2.0 * (B.nb * (c["p1a"] + c["p2a"]) + N) + 1.0 * B.nb * c["p1a"]
    f_beta = 2.0 * B.na * (c["p1b"] + c["p2b"]) + 1.0 * B.na * c["p1b"]
    b_alpha = 8.0 * 3 * N   # read c, read the diagonal, write sigma
    b_beta = 8.0 * 2 * N    # read c^T, write the partial sigma^T
    t_stream = (s64["alpha_stream"] + s64["beta_stream"]) * 1e-3
    flops_rate = (f_alpha + f_beta) / t_stream
    bytes_rate = (b_alpha + b_beta) / t_stream
    alu_frac, hbm_frac = flops_rate / PEAK_FP64_VALU, bytes_rate / PEAK_HBM
    traffic = traffic_for(kname, W.name)
    share = {k: v / sum(s64.values()) for k, v in s64.items()}
    if hbm_frac >= alu_frac:
        roofline = dict(bound="hbm", achieved=bytes_rate / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                        frac=hbm_frac)
    else:
        roofline = dict(bound="alu", achieved=flops_rate / 1e12, peak=PEAK_FP64_VALU / 1e12,
                        unit="TFLOP/s", frac=alu_frac)
    roofline.update(
        traffic=traffic,
        kernel=f"{kname} (alpha and beta row-stream launches of one FP64 sigma)",
        launch_ms=1e3 * t_stream / 2,
        algorithmic_bytes_per_launch=(b_alpha + b_beta) / 2,
        algorithmic_flops_per_launch=(f_alpha + f_beta) / 2,
        alu_frac_fp64=alu_frac, hbm_frac=hbm_frac,
        traffic_rate_TBps=None if traffic is None else traffic / (t_stream / 2) / 1e12,
        traffic_over_algorithmic=None if traffic is None else traffic / ((b_alpha + b_beta) / 2),
        stage_share_of_sigma=share)
    # whole-sigma HBM traffic from the counters (profiles/sigma_traffic.txt, taken in the
    # handle's default launch configuration): valid when this run's configuration matches
    tl = {k: v for k, v in traffic_lines(W.name).items() if "<double," in k}
    t_sigma = sum(s64.values()) * 1e-3
    whole = None
    if kname in tl and any(k.startswith("k_ab") for k in tl) and \
            any(k.startswith("k_transpose") and k.endswith("false>") for k in tl) and \
            any(k.startswith("k_transpose") and k.endswith("true>") for k in tl) and \
            sum(1 for k in tl if k.startswith("k_stream")) == 1:
        per = {k: v * (2 if k.startswith("k_stream") else 1) for k, v in tl.items()}
        tot = sum(per.values())
        whole = dict(bytes_per_sigma=tot, sigma_ms=1e3 * t_sigma, TBps=tot / t_sigma / 1e12,
                     frac_of_hbm_peak=tot / t_sigma / PEAK_HBM, per_kernel_bytes=per,
                     algorithmic_bytes=rows["sel26_f64"]["compulsory_bytes"],
                     traffic_over_algorithmic=tot / rows["sel26_f64"]["compulsory_bytes"])
    roofline["whole_sigma_hbm_counters"] = whole
    log(f"[bench] sigma f64 {rows['sel26_f64']['sigma_ms']:.3f} ms {s64}; "
        f"f32 {rows['sel26_f32']['sigma_ms']:.3f} ms; roofline {roofline['bound']} {roofline['frac']:.3f}")

    extra = dict(setup=setup, step_event_ms=dict(median=float(np.median(step_ms)), max=float(step_ms.max()),
                                                 min=float(step_ms.min())))
    if not args.no_solves:
        # tight FP64 reference energy for the time to 1e-6 Ha
        eref, repref, _ = sbd.davidson(H, W.nroots, stream=stream, tol_residual=1e-8,
                                       sigma_prec=sbd.FP64, max_space=20, use_autotune=1)
        extra["reference_energy"] = float(eref[0])
        extra["reference_iterations"] = repref["iterations"]
        extra["solves"] = solve_runs(sbd, H, W, stream, args.solve_reps, float(eref[0]), tol)
        sv = extra["solves"]
        log(f"[bench] solves: plain median {sv['plain_fp64']['median_ms']:.1f} (max/median "
            f"{sv['plain_fp64']['max_over_median']:.3f}), chosen median {sv['chosen']['median_ms']:.1f} "
            f"(max/median {sv['chosen']['max_over_median']:.3f}) ms; time to 1e-6 Ha "
            f"{sv['plain_fp64']['time_to_1e6_median_ms']} vs {sv['chosen']['time_to_1e6_median_ms']} ms")
    del x, y
    if not args.no_rows:
        for name, nv in (("sel16", 1), ("block20", 4)):
            Wr = wl.make_config(name)
            Br = sbd.Basis(Wr.norb, Wr.n_alpha, Wr.n_beta, Wr.alpha, Wr.beta, stream=stream)
            Xr = sbd.Excitations(Br, stream=stream)
            Hr = sbd.Hamiltonian(Br, Xr, Wr.h, Wr.eri, Wr.e_core, stream=stream)
            for prec, tag in ((sbd.FP64, "f64"), (sbd.FP32, "f32")):
                rows[f"{name}_{tag}"] = sigma_report(sbd, Wr, Br, Xr, Hr, prec, stream, nvec=nv)
                r = rows[f"{name}_{tag}"]
                log(f"[bench] sigma row {name} {tag} k={nv}: {r['sigma_ms']:.3f} ms, {r['det_per_s']:.3e} det/s, "
                    f"binding {r['binding_roof']} {r['binding_roof_frac']:.3f}")
            del Hr, Xr, Br
    extra["sigma_rows"] = rows
    del H, X, B
    torch.cuda.synchronize()
    sbd.release_cached_memory()
    if not args.no_block:
        extra["block"] = block_leg(sbd, wl, stream)
        log(f"[bench] block: {extra['block']}")
        sbd.release_cached_memory()
    if not args.no_sqd:
        extra["sqd_loop"] = sqd_leg(sbd, wl, stream)
        q = extra["sqd_loop"]
        for name in ("cold", "warm"):
            log(f"[bench] sqd loop {name}: {q[name]['ms']:.0f} ms, steps "
                f"{[(x['determinants'], x['iterations'], round(x['solve_ms'], 1)) for x in q[name]['steps']]}, "
                f"energies {[round(x, 6) for x in q[name]['energies']]}")
        rq = q["recovery_warm"]
        log(f"[bench] sqd loop with recovery: {rq['ms']:.0f} ms, steps "
            f"{[(x['corrected'], x['dropped'], x['determinants'], x['iterations'], round(x['solve_ms'], 1)) for x in rq['steps']]}, "
            f"energies {[round(x, 6) for x in rq['energies']]}")
        fq = q["full_bitstring_warm"]
        log(f"[bench] sqd loop full bitstring: {fq['ms']:.0f} ms, steps "
            f"{[(x['determinants'], x['iterations'], round(x['solve_ms'], 1)) for x in fq['steps']]}, "
            f"energies {[round(x, 6) for x in fq['energies']]}")
        sbd.release_cached_memory()
    if not args.no_full:
        extra["full_bitstring"] = full_leg(sbd, wl, stream)
        for r in extra["full_bitstring"]:
            log(f"[bench] full bitstring {r['workload']}: N={r['determinants']} connections={r['connections']} "
                f"basis {r['basis_ms']:.1f} ms; sigma f64 {r['sigma_ms_f64']:.3f} f32 {r['sigma_ms_f32']:.3f} ms; "
                f"solve plain {r['plain_fp64']['ms']:.1f} chosen {r['chosen']['ms']:.1f} ms")
            a = r["assembled"]
            log(f"[bench] full bitstring {r['workload']} assembled: {a['assemble_ms']:.1f} ms; sigma f64 "
                f"{a['sigma_ms_f64']:.3f} ({a['hbm_TBps_f64']:.2f} TB/s) f32 {a['sigma_ms_f32']:.3f} ms; solve plain "
                f"{a['plain_fp64']['ms']:.1f} chosen {a['chosen']['ms']:.1f} ms")
        sbd.release_cached_memory()
    if not args.no_projection:
        extra["projection_pass"] = projection_leg(sbd, N, stream)
        for r in extra["projection_pass"]:
            log(f"[bench] projection pass {r['rows']} rows x 1 vector, N={N}: {r['ms']:.3f} ms, "
                f"{r['TBps']:.2f} TB/s ({r['hbm_frac']:.2f} of HBM peak)")
        sbd.release_cached_memory()
    if not args.no_devloop:
        extra["device_iterations"] = devloop_leg(sbd, wl, stream)
        for r in extra["device_iterations"]:
            log(f"[bench] device-driven iterations N={r['determinants']} k={r['roots']} {r['precision']}: "
                f"host {r['host_driven']['ms_per_iteration']:.3f} device {r['device_driven']['ms_per_iteration']:.3f} "
                f"ms/iteration")
    if not args.no_assembled:
        extra["assembled"] = assembled_leg(sbd, wl, stream)
        for r in extra["assembled"]:
            log(f"[bench] assembled {r['workload']}: N={r['determinants']} entries={r['stored_entries']} "
                f"assemble {r['assemble_ms']:.1f} ms; sigma free {r['free_sigma_ms']} csr {r['csr_sigma_ms']} "
                f"({r['csr_hbm_TBps']} TB/s); solve free {r['free_solve_ms']:.1f} csr {r['csr_solve_ms']:.1f} ms")
        sbd.release_cached_memory()
    if not args.no_serving:
        extra["serving"] = serving(sbd, wl)
        log(f"[bench] serving: { {k: v for k, v in extra['serving'].items() if k != 'classes'} }")
    cpu = None if args.no_cpu_baseline else cpu_baseline(W)
    out = dict(metric="sigma=H.c determinants/s (FP64, one vector, sel26); Davidson time-to-1e-6 Ha, "
                      "plain FP64 vs chosen form, alongside",
               value=value, unit="det/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=ms_per_step, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload=W.name, norb=W.norb, n_alpha=W.n_alpha, n_beta=W.n_beta,
                           strings_per_spin=int(W.alpha.size), determinants=N, vectors_per_step=1,
                           solve_tol_residual=tol, solve_max_space=MAX_SPACE),
               roofline=roofline, cpu_baseline=cpu, **extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
