"""Benchmark: A-orthonormalised columns per second on one MI355X.

One step = one complete A-orthonormalisation Z = QR, Q^T A Q = I of the
workload, every step of the method included (block product or per-column
MV, projections, A-norms, normalisation), with the inputs resident in device
memory.  The headline line is the default workload:

  lap128_n128    7-point 3-D Laplacian on a 128^3 grid + 1e-2 I (CSR,
                 m = 2,097,152, nnz = 14,581,760), Z 2097152 x 128 with
                 kappa(Z) ~ 1e4, HA form in binary64 in the two-level panel
                 schedule (value: the fastest n-MV configuration, gated
                 against the column algorithm at this size in the GPU
                 tests), plus naive / HA / HP in binary64 and in the
                 binary32-storage form, with and without the binary64 second
                 pass, in the column schedule and both panel schedules.

Other workloads (same JSON shape, reported in the design notes):
  lap64_n64      Laplacian 64^3 + 1e-2 I, Z 262144 x 64, kappa(Z) ~ 1e6.
  dense512_n32   dense spd 512 x 512 (B B^T/m + I), Z 512 x 32.
  dense16k_n256  dense spd 16384 x 16384, Z 16384 x 256 (HP block product on
                 the matrix cores).
  batch2048      2048 independent pentadiagonal instances, m ~ U[64,4096],
                 n ~ U[4,64], one persistent launch replayed from a HIP graph.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A-orthonormalised cols/s + %HBM roofline: HA/HP n-MV vs 2n-MV, FP64 vs FP32"
HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks of MI355X (TFLOP/s) for the block product's dtype
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
# HBM byte counters of the dominant kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE,
# scaled by a plain copy's reading), per kernel and workload, with a hash of
# the kernel's sources: a record whose sources have changed is not used
TRAFFIC_FILES = {
    ("sweep", "lap64_n64"): os.path.join(ROOT, "profiles", "sweep_lap64_traffic.json"),
    ("block_sweep", "lap128_n128"): os.path.join(ROOT, "profiles", "psweep_lap128_traffic.json"),
    ("block_sweep8", "lap128_n128"): os.path.join(ROOT, "profiles", "bsweep_lap128_traffic.json"),
    ("block_sweep16", "lap128_n128"): os.path.join(ROOT, "profiles", "bsweep16_lap128_traffic.json"),
    ("mv", "lap128_n128"): os.path.join(ROOT, "profiles", "mv_lap128_traffic.json"),
}
KERNEL_SOURCES = {
    "sweep": ("amgs_single.hip", "amgs_device.h", "amgs_internal.h"),
    "block_sweep": ("amgs_panel.hip", "amgs_device.h", "amgs_internal.h"),
    "block_sweep8": ("amgs_bsweep.hip", "amgs_device.h", "amgs_internal.h"),
    "block_sweep16": ("amgs_bsweep.hip", "amgs_device.h", "amgs_internal.h"),
    "mv": ("amgs_single.hip", "amgs_device.h", "amgs_internal.h"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------- workloads
def make_problem(name, device):
    from paper_1703_10440_amd import inputs
    if name == "dense16k_n256":
        return inputs.dense16k_problem(device=device)
    return inputs.WORKLOADS[name]()


def to_device(prob, dev, torch):
    import numpy as np
    d = {"Z": torch.from_numpy(np.ascontiguousarray(prob.Z)).to(dev)}
    if prob.csr is not None:
        d["row_ptr"] = torch.from_numpy(prob.csr.row_ptr).to(dev)
        d["col_idx"] = torch.from_numpy(prob.csr.col_idx).to(dev)
        d["vals"] = torch.from_numpy(prob.csr.vals).to(dev)
    else:
        d["A"] = torch.from_numpy(np.ascontiguousarray(prob.dense)).to(dev)
    return d


class Runner:
    """Preallocated device buffers for repeated calls of one configuration."""

    def __init__(self, data, variant, precision, torch, amgs, reorth=False, panel=0, cgs=False):
        self.torch, self.amgs = torch, amgs
        dt = torch.float64 if precision == "fp64" else torch.float32
        self.variant, self.precision, self.reorth, self.panel = variant, precision, reorth, panel
        self.cgs = cgs
        self.Z = amgs.colmajor(data["Z"], dt)
        m, n = self.Z.shape
        self.m, self.n = m, n
        self.Q = amgs.empty_colmajor(m, n, dt, self.Z.device)
        self.P = amgs.empty_colmajor(m, n, dt, self.Z.device)
        self.dense = "A" in data
        if self.dense:
            self.A = amgs.colmajor(data["A"], dt)
        else:
            self.rp, self.ci = data["row_ptr"], data["col_idx"]
            self.vals = data["vals"].to(dt)
        h = amgs.handle(0)
        wb = amgs.amgs_workspace_bytes(h, m, n, int(self.dense), amgs.VARIANTS[variant],
                                       amgs.PRECISIONS[precision], 1,
                                       amgs.Opts(int(reorth), int(panel), int(cgs), 0))
        self.work = torch.empty(max(wb, 1), dtype=torch.uint8, device=self.Z.device)

    def __call__(self):
        a = self.amgs
        kw = dict(variant=self.variant, precision=self.precision, Q=self.Q, P=self.P,
                  work=self.work, reorth=self.reorth, panel=self.panel, cgs=self.cgs)
        if self.dense:
            return a.qr_dense(self.A, self.Z, **kw)
        return a.qr_csr(self.rp, self.ci, self.vals, self.Z, **kw)


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def time_graph(fn, steps, torch):
    """The same call captured once in a HIP graph (torch.cuda.graph, after a
    warm-up on the capturing stream) and replayed `steps` times: the library
    only enqueues kernels, so the replay does the same work without the
    host-side launch of each kernel."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = fn()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out, g


def accuracy(data, out, torch):
    """||Q^T A Q - I||_2 and ||Z - QR||_F / ||Z||_F in binary64 (torch used
    only to evaluate the metrics)."""
    Q = out.Q.double()
    R = out.R
    Z = data["Z"].double()
    if "A" in data:
        AQ = data["A"].double() @ Q
    else:
        m = Q.shape[0]
        S = torch.sparse_csr_tensor(data["row_ptr"].long(), data["col_idx"].long(),
                                    data["vals"].double(), size=(m, m))
        AQ = S @ Q
    G = Q.T @ AQ
    n = G.shape[0]
    orth = torch.linalg.matrix_norm(G - torch.eye(n, dtype=G.dtype, device=G.device), ord=2)
    res = torch.linalg.norm(Z - Q @ torch.triu(R)) / torch.linalg.norm(Z)
    return float(orth), float(res)


def source_sha(kind="sweep"):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1703_10440_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kind, workload, runner):
    """The measured HBM bytes per launch of a kernel, from its record, if the
    record matches the kernel's sources and the run's precision, variant and
    schedule."""
    path = TRAFFIC_FILES.get((kind, workload))
    if path and os.path.exists(path):
        rec = json.load(open(path))
        if rec.get("source_sha") == source_sha(kind) and rec.get("precision", "fp64") == \
                runner.precision and rec.get("variant", runner.variant) == runner.variant and \
                rec.get("panel", runner.panel) == runner.panel:
            return rec.get("traffic_bytes_per_launch")
    return None


def _hbm_line(kernel, nbytes_per_launch, ms, launches, traffic):
    avg_s = ms / 1e3 / max(launches, 1)
    achieved = nbytes_per_launch / avg_s / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "avg_us": round(avg_s * 1e6, 3), "launches": int(launches),
            "bytes_per_launch": nbytes_per_launch, "total_ms": round(ms, 4)}


def headline_rooflines(runner, amgs, torch, workload):
    """One profiled call of the headline configuration.  Its projection
    sweep (the block sweep after each panel's last column in the panel
    schedules, the column sweep in the column schedule) and, for HA, its
    column MV (both forms, Alg. 5): each with its average duration from HIP
    events that the library binds to each dispatch on the call's stream
    (hipExtLaunchKernel start/stop events), its total time in the call and
    its algorithmic bytes per launch from the library's counters.  The
    dominant kernel is the one with the larger total time.  Returns
    (dominant, sweep, mv); mv is None for naive (its second MV is not timed)
    and HP (no column MV)."""
    h = amgs.handle(0)
    amgs.amgs_profile_reset(h)
    amgs.amgs_profile_enable(h, 1)
    out = runner()
    torch.cuda.synchronize()
    amgs.amgs_profile_enable(h, 0)
    st = out.stats
    if runner.panel in (8, 16):
        kind = f"block_sweep{runner.panel}"
        kernel = ("k_bsweep (block sweep after each panel of "
                  + ("eight)" if runner.panel == 8 else "sixteen)"))
        ms, launches = amgs.amgs_profile_read(h, 3)
        nbytes, nl = st.block_sweep_bytes, st.block_sweep_launches
    elif runner.panel:
        kind, kernel = "block_sweep", "k_psweep (block sweep after each panel)"
        ms, launches = amgs.amgs_profile_read(h, 3)
        nbytes, nl = st.block_sweep_bytes, st.block_sweep_launches
    else:
        kind, kernel = "sweep", "k_sweep"
        ms, launches = amgs.amgs_profile_read(h, 0)
        nbytes, nl = st.sweep_bytes, st.sweep_launches
    sweep = _hbm_line(kernel, nbytes / max(nl, 1), ms, launches, _traffic(kind, workload, runner))
    mv = None
    if runner.variant == "ha":
        ms1, n1 = amgs.amgs_profile_read(h, 1)
        if n1 > 0:
            mv = _hbm_line("k_csr_mv_ell / k_dense_mv (HA column MV, both forms)",
                           st.mv_bytes / max(st.mv_calls, 1), ms1, n1,
                           _traffic("mv", workload, runner))
    dominant = mv if mv is not None and mv["total_ms"] > sweep["total_ms"] else sweep
    return dominant, sweep, mv


def gemm_roofline(runner, m, n, precision, amgs, torch):
    """The HP block product X = A Z for dense A on the matrix cores: its
    duration from HIP events recorded around the launch on the call's
    stream, and its 2 m^2 n flops."""
    h = amgs.handle(0)
    amgs.amgs_profile_reset(h)
    amgs.amgs_profile_enable(h, 1)
    runner()
    torch.cuda.synchronize()
    amgs.amgs_profile_enable(h, 0)
    ms, launches = amgs.amgs_profile_read(h, 2)
    avg_s = ms / 1e3 / max(launches, 1)
    tflops = 2.0 * m * m * n / avg_s / 1e12
    peak = MFMA_PEAK_TFLOPS[precision]
    return {"bound": "mfma", "kernel": "k_gemm_atb (HP block product)", "achieved": round(tflops, 2),
            "peak": peak, "unit": "TFLOP/s", "frac": round(tflops / peak, 4),
            "avg_us": round(avg_s * 1e6, 2), "launches": int(launches),
            "flops_per_launch": 2.0 * m * m * n}


def cpu_baseline(prob, variant, budget_s=10.0):
    """The oracle as it stands, repeated on the full workload until about
    budget_s seconds of host time have passed."""
    from oracle import ref
    runs, total = 0, 0.0
    while total < budget_s and runs < 1000:
        t0 = time.perf_counter()
        r = ref.qr_problem(prob, variant=variant)
        total += time.perf_counter() - t0
        runs += 1
        assert r.info == 0
        if total > 3 * budget_s:
            break
    return {"value": round(runs * prob.n / total, 2), "unit": "cols/s",
            "cores": ref.num_threads(), "kind": "oracle",
            "sample": f"full workload, {variant} binary64, {runs} run(s) in {total:.1f} s"}


def cpu_baseline_one_thread(workload, variant, budget_s=5.0):
    """The same oracle on one host thread (the paper timed one core), in a
    child process so that OpenMP starts with one thread; the child builds the
    workload itself and never touches the GPU."""
    import subprocess
    code = (
        "import json, sys, time\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from oracle import ref\n"
        "from paper_1703_10440_amd import inputs\n"
        f"p = inputs.WORKLOADS[{workload!r}]()\n"
        "runs, total = 0, 0.0\n"
        f"while total < {budget_s} and runs < 1000:\n"
        "    t0 = time.perf_counter()\n"
        f"    r = ref.qr_problem(p, variant={variant!r})\n"
        "    total += time.perf_counter() - t0\n"
        "    runs += 1\n"
        "    assert r.info == 0\n"
        "print(json.dumps({'runs': runs, 'total': total, 'n': p.n, 'threads': ref.num_threads()}))\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": round(d["runs"] * d["n"] / d["total"], 2), "unit": "cols/s",
            "cores": d["threads"], "kind": "oracle",
            "sample": f"full workload, {variant} binary64, {d['runs']} run(s) in {d['total']:.1f} s"}


# -------------------------------------------------------------- single problem
def bench_single(args, torch, amgs):
    dev = torch.device("cuda:0")
    log(f"[bench] building workload {args.workload}")
    prob = make_problem(args.workload, dev)
    data = to_device(prob, dev, torch)
    log(f"[bench] m={prob.m} n={prob.n}")
    big = prob.m * prob.m if prob.csr is None else prob.csr.nnz
    head_v, head_p = args.variant, args.precision
    run = Runner(data, head_v, head_p, torch, amgs, reorth=args.reorth, panel=args.panel)
    t, out = time_steps(run, args.steps, args.warmup, torch)
    info = int(out.info.item())
    log(f"[bench] {head_v}/{head_p}: {t * 1e3:.3f} ms/step info={info}")
    tg, gout, graph = time_graph(run, args.steps, torch)
    graph_line = {"ms_per_step": round(tg * 1e3, 4), "value": round(prob.n / tg, 2),
                  "info": int(gout.info.item()),
                  "same_result": bool(torch.equal(gout.R, out.R))}
    del graph, gout
    log(f"[bench] {head_v}/{head_p} graph replay: {tg * 1e3:.3f} ms/step {graph_line}")
    roof, sweeproof, mvroof = headline_rooflines(run, amgs, torch, args.workload)
    log(f"[bench] sweep roofline {sweeproof}")
    log(f"[bench] mv roofline {mvroof}")
    gemmroof = None
    if prob.csr is None and head_v == "hp":
        gemmroof = gemm_roofline(run, prob.m, prob.n, head_p, amgs, torch)
        log(f"[bench] gemm roofline {gemmroof}")
    del run

    variants = {}
    if not args.no_variants:
        combos = [(v, p, False, 0, False) for p in ("fp64", "fp32") for v in ("naive", "ha", "hp")]
        combos += [(v, p, True, pan, False) for p in ("fp32", "fp64") for pan in (0, 4, 8)
                   for v in ("ha", "hp")]
        # the blocked second pass (two-level schedule only)
        combos += [(v, p, 2, 8, False) for p in ("fp32", "fp64") for v in ("ha", "hp")]
        combos += [(v, p, False, pan, False) for pan in (4, 8) for p in ("fp64", "fp32")
                   for v in ("naive", "ha", "hp")]
        # the three-level schedule (naive and HA only)
        combos += [(v, p, False, 16, False) for p in ("fp64", "fp32") for v in ("naive", "ha")]
        combos += [("ha", p, True, 16, False) for p in ("fp32", "fp64")]
        combos += [(v, "fp64", ro, 0, True) for ro in (False, True) for v in ("naive", "ha", "hp")]
        for v, p, ro, pan, cgs in combos:
            r = Runner(data, v, p, torch, amgs, reorth=ro, panel=pan, cgs=cgs)
            heavy = v == "naive" and prob.csr is None and prob.m > 4096
            steps = 1 if heavy else (max(2, args.steps // 4) if v == "naive" else max(3, args.steps // 2))
            tv, o = time_steps(r, steps, 1, torch)
            orth, res = accuracy(data, o, torch)
            key = (("cgs_" if cgs else "") + f"{v}_{p}"
                   + ("_reorthblk" if ro == 2 else "_reorth" if ro else "")
                   + (f"_panel{pan}" if pan else ""))
            variants[key] = {"cols_per_s": round(prob.n / tv, 1), "ms": round(tv * 1e3, 4),
                             "orth_loss": orth, "residual": res, "info": int(o.info.item())}
            log(f"[bench] {key}: {tv * 1e3:.3f} ms  |QtAQ-I| {orth:.2e}  res {res:.2e}")
            del r, o
        for sfx in ("", "_panel4", "_panel8"):
            for p in ("fp64", "fp32"):
                nv = variants[f"naive_{p}{sfx}"]["ms"]
                for v in ("ha", "hp"):
                    e = variants[f"{v}_{p}{sfx}"]
                    e["speedup_vs_naive"] = round(nv / e["ms"], 3)
            for v in ("naive", "ha", "hp"):
                variants[f"{v}_fp32{sfx}"]["speedup_vs_fp64"] = round(
                    variants[f"{v}_fp64{sfx}"]["ms"] / variants[f"{v}_fp32{sfx}"]["ms"], 3)
            # the binary32 form with the binary64 second pass against plain
            # binary64 in the same schedule
            for v in ("ha", "hp"):
                for kind in ("reorth", "reorthblk"):
                    k = f"{v}_fp32_{kind}{sfx}"
                    if k in variants:
                        variants[k]["speedup_vs_fp64"] = round(
                            variants[f"{v}_fp64{sfx}"]["ms"] / variants[k]["ms"], 3)
        sfx = "_panel16"
        for p in ("fp64", "fp32"):
            variants[f"ha_{p}{sfx}"]["speedup_vs_naive"] = round(
                variants[f"naive_{p}{sfx}"]["ms"] / variants[f"ha_{p}{sfx}"]["ms"], 3)
        for k, k64 in (("naive_fp32", "naive_fp64"), ("ha_fp32", "ha_fp64"),
                       ("ha_fp32_reorth", "ha_fp64")):
            variants[k + sfx]["speedup_vs_fp64"] = round(
                variants[k64 + sfx]["ms"] / variants[k + sfx]["ms"], 3)
        # fastest modified Gram-Schmidt configuration per precision (either
        # schedule, no second pass)
        best = {}
        for p in ("fp64", "fp32"):
            keys = [k for k in variants if not k.startswith("cgs_") and "reorth" not in k
                    and k.split("_")[1] == p]
            k = max(keys, key=lambda k: variants[k]["cols_per_s"])
            best[p] = {"variant": k, "cols_per_s": variants[k]["cols_per_s"],
                       "ms": variants[k]["ms"], "orth_loss": variants[k]["orth_loss"]}
        variants["best"] = best

    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle")
        cpu = cpu_baseline(prob, head_v, args.cpu_budget)
        log(f"[bench] cpu {cpu}")
    cpu1 = None
    if not args.no_cpu and args.workload in ("lap64_n64", "dense512_n32"):
        cpu1 = cpu_baseline_one_thread(args.workload, head_v)
        log(f"[bench] cpu, one thread {cpu1}")
    cfg = {"workload": args.workload, "m": prob.m, "n": prob.n,
           "A": "csr" if prob.csr is not None else "dense", "nnz": int(big),
           "variant": head_v, "precision": head_p, "reorth": int(args.reorth),
           "schedule": f"panel{args.panel}" if args.panel else "column"}
    line = {"metric": METRIC, "value": round(prob.n / t, 2), "unit": "cols/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t * 1e3, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if head_p == "fp64" else "f32", "data": "synthetic", "config": cfg,
            "roofline": roof, "sweep_roofline": sweeproof, "mv_roofline": mvroof,
            "cpu_baseline": cpu, "variants": variants,
            "graph_replay": graph_line}
    if gemmroof is not None:
        line["gemm_roofline"] = gemmroof
    if cpu1 is not None:
        line["cpu_baseline_one_thread"] = cpu1
    return line


# --------------------------------------------------------------------- batched
def batch_size_class(m, n):
    """Size class of an instance in the batch plan (4 ranges of m, n <= 16
    or not); the plan autotunes one column-block width per class."""
    mc = 0 if m <= 512 else 1 if m <= 1024 else 2 if m <= 2048 else 3
    return mc * 2 + (1 if n > 16 else 0)


def batch_requested_bytes(problems, tiles, variant, w):
    """Bytes the persistent batched kernel requests from memory in one pass,
    each vector pass counted once (no credit for cache hits).  Per instance
    with column-block width B: Z read once, Q and P written once, every
    earlier p_i and q_i read once per block, A (row_ptr, col_idx, vals) read
    per column MV (the MV's source vector sits in LDS), R zeroed and its
    upper triangle written; HP adds X = A Z (A and one Z pass per column, X
    written) and X read once."""
    total = 0.0
    for p in problems:
        m, n, nnz = p.m, p.n, int(p.csr.nnz)
        B = max(1, tiles[batch_size_class(m, n)])
        col = m * w
        A = 4.0 * (m + 1) + nnz * (4.0 + w)
        nb = (n + B - 1) // B
        earlier = sum(b * B for b in range(nb))
        mvs = {"naive": 2, "ha": 1, "hp": 0}[variant]
        b = 8.0 * n * n + 8.0 * n * (n + 1) / 2
        b += n * col + 2.0 * n * col + 2.0 * earlier * col + mvs * n * A
        if variant == "hp":
            b += n * (A + 2.0 * col) + n * col
        total += b
    return total


def batch_model_bytes(problems, variant, w):
    """The streaming byte model of the method per pass (summed over the
    instances): B_alg = (#MV passes) S + m n (n - 1) w + I/O, with S = one
    CSR MV (A once, source and result vectors) for naive (2n passes) and HA
    (n), and one n-column block product for HP; I/O = Z read, Q written, R
    written.  Also the compulsory floor: A, Z read once, Q and R written
    once."""
    alg = floor = 0.0
    for p in problems:
        m, n, nnz = p.m, p.n, int(p.csr.nnz)
        A = 4.0 * (m + 1) + nnz * (4.0 + w)
        io = 2.0 * m * n * w + 8.0 * n * n
        if variant == "hp":
            mv = A + 2.0 * m * n * w
        else:
            mv = (2 if variant == "naive" else 1) * n * (A + 2.0 * m * w)
        alg += mv + m * n * (n - 1) * w + io
        floor += A + io
    return alg, floor


def batch_cpu_baseline(problems, variant, budget_s=10.0):
    """The oracle on a seeded sample of the batch's instances, until about
    budget_s seconds of host time have passed."""
    import numpy as np
    from oracle import ref
    order = np.random.default_rng(0).permutation(len(problems))
    cols, total, done = 0, 0.0, 0
    for k in order:
        p = problems[int(k)]
        t0 = time.perf_counter()
        ref.qr_problem(p, variant=variant)
        total += time.perf_counter() - t0
        cols += p.n
        done += 1
        if total >= budget_s:
            break
    return {"value": round(cols / total, 1), "unit": "cols/s", "cores": ref.num_threads(),
            "kind": "oracle",
            "sample": f"{done} of {len(problems)} instances (seeded order), {variant} binary64, "
                      f"{cols} columns in {total:.1f} s"}


def bench_batched(args, torch, amgs):
    import numpy as np
    from paper_1703_10440_amd import inputs
    dev = torch.device("cuda:0")
    log("[bench] building 2048 pentadiagonal instances")
    b = inputs.pentadiag_batch(batch=2048, seed=5)
    cols = sum(p.n for p in b.problems)
    results = {}
    head = None
    for prec in ("fp64", "fp32"):
        for v in ("ha", "hp"):
            dt = np.float64 if prec == "fp64" else np.float32
            insts = [(torch.from_numpy(p.csr.row_ptr).to(dev), torch.from_numpy(p.csr.col_idx).to(dev),
                      torch.from_numpy(p.csr.vals.astype(dt)).to(dev),
                      torch.from_numpy(np.ascontiguousarray(p.Z.astype(dt))).to(dev))
                     for p in b.problems]
            t0 = time.perf_counter()
            Qs, Rs, info, plan, keep = amgs.qr_batched(insts, variant=v, precision=prec,
                                                       autotune=True)
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            items, desc, work = keep

            def step():
                plan.run(desc, work, info)
            t, _ = time_steps(step, args.steps, args.warmup, torch)
            bad = int((info != 0).sum().item())
            key = f"{v}_{prec}"
            w = 8 if prec == "fp64" else 4
            req = batch_requested_bytes(b.problems, plan.tiles(), v, w)
            alg, floor = batch_model_bytes(b.problems, v, w)
            results[key] = {"cols_per_s": round(cols / t, 1), "ms": round(t * 1e3, 4),
                            "tiles": plan.tiles(), "plan_and_first_call_s": round(setup, 3),
                            "breakdowns": bad,
                            "B_alg_GB": round(alg / 1e9, 3),
                            "B_alg_frac": round(alg / t / 1e9 / HBM_PEAK_GBS, 4),
                            "floor_GB": round(floor / 1e9, 3),
                            "floor_frac": round(floor / t / 1e9 / HBM_PEAK_GBS, 4),
                            "requested_GB": round(req / 1e9, 3),
                            "requested_GB_per_s": round(req / t / 1e9, 1),
                            "requested_frac": round(req / t / 1e9 / HBM_PEAK_GBS, 4)}
            log(f"[bench] batched {key}: {t * 1e3:.3f} ms  tiles {plan.tiles()}  "
                f"B_alg {alg / 1e9:.2f} GB  floor {floor / 1e9:.3f} GB  requested {req / 1e9:.2f} GB")
            if head is None:
                head = (t, key, alg, floor, req)
            del Qs, Rs, info, plan, keep, insts
    t, key, alg, floor, req = head
    cfg = {"workload": "batch2048", "instances": 2048, "total_columns": cols,
           "m_range": [64, 4096], "n_range": [4, 64], "A": "csr pentadiagonal",
           "variant": "ha", "precision": "fp64"}
    # the whole pass is one persistent kernel, so its duration is the step's;
    # achieved = the method's streaming byte model (B_alg) over that time,
    # which the blocked in-workgroup schedule can exceed (frac > 1), so the
    # compulsory floor and the bytes the kernel requests are given beside it
    ach = alg / t / 1e9
    roof = {"bound": "hbm", "kernel": "k_batched (one persistent launch per pass)",
            "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_launch": alg,
            "floor_bytes": floor, "floor_frac": round(floor / t / 1e9 / HBM_PEAK_GBS, 4),
            "requested_bytes": req, "requested_frac": round(req / t / 1e9 / HBM_PEAK_GBS, 4),
            "note": "B_alg per pass (naive 2n / HA n CSR MV passes, HP one block product, "
                    "m n (n-1) w of projections, I/O); time of the graph replay"}
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a sample of instances")
        cpu = batch_cpu_baseline(b.problems, "ha", args.cpu_budget)
        log(f"[bench] cpu {cpu}")
    return {"metric": METRIC, "value": round(cols / t, 2), "unit": "cols/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t * 1e3, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": cfg, "roofline": roof, "cpu_baseline": cpu,
            "variants": results}


# ------------------------------------------------------ timing experiment
def bench_exp1(args, torch, amgs):
    """Experiment I (Section 4) in shape: the time of naive, HA and HP in
    binary64 against the number of columns n, on a dense spd A = B B^T/m + I
    with m = 10000 and on a sparse spd stand-in for the paper's sparse matrix
    (m = 9180, about 387 entries per row, symmetric and strictly diagonally
    dominant: only its size and density follow the paper's matrix).  Z is
    Gaussian.  Reports ms per call and the speed-up of HA and HP over naive."""
    import numpy as np
    from paper_1703_10440_amd import inputs
    dev = torch.device("cuda:0")
    ns = [5, 10, 20, 50, 100, 200, 500, 1000, 2000]
    out = {"workload": "exp1", "precision": "fp64", "ns": ns, "results": {}}
    log("[bench] exp1: building A (dense 10000, sparse 9180)")
    A = torch.from_numpy(inputs.gram_spd(inputs.rng(11), 10000, device="cuda:0")).to(dev)
    A = amgs.colmajor(A, torch.float64)
    sp = inputs.random_csr_problem(9180, 1, 387, seed=12).csr
    out["sparse_nnz"] = int(sp.nnz)
    csr = {"row_ptr": torch.from_numpy(sp.row_ptr).to(dev),
           "col_idx": torch.from_numpy(sp.col_idx).to(dev),
           "vals": torch.from_numpy(sp.vals).to(dev)}
    for name, m, dense in (("dense_m10000", 10000, True), ("sparse_m9180", 9180, False)):
        Zall = inputs.rng(13).standard_normal((m, max(ns)))
        rec = {}
        for n in ns:
            data = {"Z": torch.from_numpy(np.ascontiguousarray(Zall[:, :n])).to(dev)}
            if dense:
                data["A"] = A
            else:
                data.update(csr)
            row = {}
            for v in ("naive", "ha", "hp"):
                r = Runner(data, v, "fp64", torch, amgs)
                t, o = time_steps(r, 3, 1, torch)
                if int(o.info.item()) != 0:
                    raise RuntimeError(f"exp1 {name} n={n} {v}: breakdown")
                row[v] = round(t * 1e3, 4)
                del r, o
            row["ha_over_naive"] = round(row["naive"] / row["ha"], 2)
            row["hp_over_naive"] = round(row["naive"] / row["hp"], 2)
            rec[str(n)] = row
            log(f"[bench] exp1 {name} n={n}: {row}")
        out["results"][name] = rec
    return out


# ------------------------------------------------------- accuracy experiment
def bench_exp2(args, torch, amgs):
    """Experiments II/III (Section 4) on the GPU binary64 path: m = 100,
    n = 20, kappa(A), kappa(Z) on the 28-point grid 10^0.5 .. 10^14, cases 1
    and 2.  Reports the loss of A-orthogonality of each variant against
    delta_1 = u kappa(A) kappa(A^{1/2} Z) and delta_2 = u (kappa(A) +
    kappa(A^{1/2} Z)); kappa(A^{1/2} Z) is taken as kappa(R)."""
    import numpy as np
    from paper_1703_10440_amd import inputs
    u = 2.0 ** -53
    dev = torch.device("cuda:0")
    grid = [10.0 ** (0.5 * k) for k in range(1, 29)]
    out = {}
    t0 = time.perf_counter()
    for case in (1, 2):
        rec = {v: [] for v in ("naive", "ha", "hp", "cgs_naive")}
        for ia, ka in enumerate(grid):
            for iz, kz in enumerate(grid):
                p = inputs.exp2_problem(100, 20, ka, kz, case, seed=10000 * case + 100 * ia + iz)
                A = torch.from_numpy(np.ascontiguousarray(p.dense)).to(dev)
                Zt = torch.from_numpy(np.ascontiguousarray(p.Z)).to(dev)
                for v in rec:
                    if v == "cgs_naive":
                        o = amgs.qr_dense(A, Zt, variant="naive", cgs=True)
                    else:
                        o = amgs.qr_dense(A, Zt, variant=v)
                    Q, R = o.Q, o.R
                    G = Q.T @ (A @ Q)
                    loss = float(torch.linalg.matrix_norm(G - torch.eye(20, dtype=G.dtype, device=dev), ord=2))
                    kAZ = float(torch.linalg.cond(R))
                    rec[v].append((ka, kAZ, loss, int(o.info.item())))
        summ = {}
        for v, rows in rec.items():
            ok = [r for r in rows if r[3] == 0]
            d1 = np.array([u * r[0] * r[1] for r in ok])
            d2 = np.array([u * (r[0] + r[1]) for r in ok])
            lo = np.array([r[2] for r in ok])
            summ[v] = {"problems": len(rows), "breakdowns": len(rows) - len(ok),
                       "median_loss_over_delta1": float(np.median(lo / d1)),
                       "max_loss_over_delta1": float(np.max(lo / d1)),
                       "median_loss_over_delta2": float(np.median(lo / d2))}
            # least-squares exponents of the loss in kappa(A) and kappa(A^{1/2} Z)
            # over the problems above rounding level and below saturation
            fit = [r for r in ok if 1e-13 < r[2] < 1e-2]
            if len(fit) >= 10:
                M = np.array([[1.0, np.log10(r[0]), np.log10(r[1])] for r in fit])
                y = np.array([np.log10(r[2]) for r in fit])
                coef = np.linalg.lstsq(M, y, rcond=None)[0]
                summ[v]["fit_exponent_kappa_A"] = round(float(coef[1]), 2)
                summ[v]["fit_exponent_kappa_A12Z"] = round(float(coef[2]), 2)
                summ[v]["fit_points"] = len(fit)
        n = len(rec["ha"])
        better = sum(1 for a, b in zip(rec["ha"], rec["naive"]) if a[2] < b[2])
        summ["ha_more_accurate_than_naive"] = f"{better}/{n}"
        out[f"case{case}"] = summ
        log(f"[bench] exp2 case {case}: {summ}")
    return {"workload": "exp2", "grid": "28 x 28 kappa(A), kappa(Z) in 10^0.5..10^14",
            "m": 100, "n": 20, "seconds": round(time.perf_counter() - t0, 1), "results": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lap128_n128",
                    choices=["lap64_n64", "lap128_n128", "dense512_n32", "dense16k_n256",
                             "batch2048", "copy1g", "stream", "exp1", "exp2"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--variant", default="ha", choices=["naive", "ha", "hp"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--reorth", type=int, nargs="?", const=1, default=0, choices=[0, 1, 2],
                    help="second pass in the headline run: 1 per column, 2 blocked "
                         "(two-level schedule only)")
    ap.add_argument("--panel", type=int, default=None, choices=[0, 4, 8, 16],
                    help="schedule of the headline run: 0 column order, 4 panels of four, "
                         "8 panels of eight taken apart as panels of four, 16 panels of "
                         "sixteen taken apart as panels of eight (naive and HA; the "
                         "default for them, 8 for HP)")
    args = ap.parse_args()
    if args.panel is None:
        args.panel = 8 if args.variant == "hp" or args.reorth == 2 else 16
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported here "
              "(the design notes describe how the path would shard).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1703_10440_amd import amgs
    amgs.load()
    if args.workload == "copy1g":
        # a plain 1 GiB device-to-device copy: the reference reading for the
        # HBM byte counters (FETCH_SIZE / WRITE_SIZE) of the profiler
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0").fill_(1)
        y = torch.empty_like(x)
        t, _ = time_steps(lambda: y.copy_(x), args.steps, args.warmup, torch)
        print(json.dumps({"workload": "copy1g", "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                          "ms": round(t * 1e3, 4), "GB_per_s": round(2 * (1 << 30) / t / 1e9, 1)}),
              flush=True)
        return
    if args.workload == "stream":
        # what plain streaming kernels (torch's own) reach on this GPU: an
        # in-place read-modify-write (the access pattern of a sweep), a copy
        # and a read-only sum, at a size that fits the 256 MB last-level
        # cache and at one that does not
        out = {"workload": "stream", "kernels": "torch add_ / copy_ / sum", "rates_GB_per_s": {}}
        for mib in (128, 2048):
            x = torch.ones(mib << 17, dtype=torch.float64, device="cuda:0")
            y = torch.empty_like(x)
            nb = x.numel() * 8
            for name, fn, moved in (("rmw", lambda: x.add_(1.0), 2 * nb),
                                    ("copy", lambda: y.copy_(x), 2 * nb),
                                    ("read", lambda: x.sum(), nb)):
                t, _ = time_steps(fn, max(args.steps, 20), args.warmup, torch)
                out["rates_GB_per_s"][f"{name}_{mib}MiB"] = round(moved / t / 1e9, 1)
            del x, y
        print(json.dumps(out), flush=True)
        return
    if args.workload == "exp1":
        print(json.dumps(bench_exp1(args, torch, amgs)), flush=True)
        return
    if args.workload == "exp2":
        print(json.dumps(bench_exp2(args, torch, amgs)), flush=True)
        return
    if args.workload == "batch2048":
        line = bench_batched(args, torch, amgs)
    else:
        line = bench_single(args, torch, amgs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
