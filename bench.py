"""Benchmark: A-orthonormalised columns per second on one MI355X.

One step = one complete A-orthonormalisation Z = QR, Q^T A Q = I of the
workload (every step of the method: block product or per-column MV,
projections, A-norms, normalisation), inputs resident in device memory.

Default workload: 7-point 3-D Laplacian on a 64^3 grid plus 1e-2 I (CSR,
m = 262144, nnz = 1,810,432), Z = 262144 x 64 with kappa(Z) ~ 1e6; the
headline value is the HP form in binary64.  The same line also reports the
naive 2n-MV form, the HA form and the binary32-storage forms, the roofline of
the dominant kernel (the projection sweep), and the CPU oracle timed on the
host.

    python bench.py [--steps K] [--warmup W] [--workload lap64_n64|lap128_n128|dense512_n32|dense16k_n256]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A-orthonormalised cols/s + %HBM roofline: HA/HP n-MV vs 2n-MV, FP64 vs FP32"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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

    def __init__(self, prob, dev_data, variant, precision, torch, amgs):
        self.torch, self.amgs = torch, amgs
        self.prob = prob
        dt = torch.float64 if precision == "fp64" else torch.float32
        self.dt = dt
        self.variant, self.precision = variant, precision
        self.Z = amgs.colmajor(dev_data["Z"], dt)
        m, n = self.Z.shape
        self.m, self.n = m, n
        self.Q = amgs.empty_colmajor(m, n, dt, self.Z.device)
        self.P = amgs.empty_colmajor(m, n, dt, self.Z.device)
        self.dense = "A" in dev_data
        if self.dense:
            self.A = amgs.colmajor(dev_data["A"], dt)
        else:
            self.rp, self.ci = dev_data["row_ptr"], dev_data["col_idx"]
            self.vals = dev_data["vals"].to(dt)
        h = amgs.handle(0)
        opts = amgs.Opts(0, 0, 0, 0)
        wb = amgs.amgs_workspace_bytes(h, m, n, int(self.dense), amgs.VARIANTS[variant],
                                       amgs.PRECISIONS[precision], 1, opts)
        self.work = torch.empty(max(wb, 1), dtype=torch.uint8, device=self.Z.device)

    def __call__(self):
        a = self.amgs
        kw = dict(variant=self.variant, precision=self.precision, Q=self.Q, P=self.P,
                  work=self.work)
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
    dt = time.perf_counter() - t0
    return dt / steps, out


def sweep_roofline(runner, amgs, torch):
    """Average duration of the projection-sweep kernel, from HIP events the
    library records on the call's stream, and its algorithmic bytes."""
    h = amgs.handle(0)
    amgs.amgs_profile_reset(h)
    amgs.amgs_profile_enable(h, 1)
    out = runner()
    torch.cuda.synchronize()
    amgs.amgs_profile_enable(h, 0)
    ms, launches = amgs.amgs_profile_read(h, 0)
    st = out.stats
    avg_s = ms / 1e3 / max(launches, 1)
    bytes_per_launch = st.sweep_bytes / max(st.sweep_launches, 1)
    achieved = bytes_per_launch / avg_s / 1e9
    return {"bound": "hbm", "kernel": "k_sweep", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None, "avg_us": round(avg_s * 1e6, 3), "launches": int(launches),
            "bytes_per_launch": bytes_per_launch}


def cpu_baseline(prob, variant):
    from oracle import ref
    t0 = time.perf_counter()
    r = ref.qr_problem(prob, variant=variant)
    dt = time.perf_counter() - t0
    assert r.info == 0
    return {"value": round(prob.n / dt, 2), "unit": "cols/s", "cores": ref.num_threads(),
            "kind": "oracle",
            "sample": f"full workload, {variant} binary64, one run of {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lap64_n64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--variant", default="hp", choices=["naive", "ha", "hp"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(instances of the batched form shard across GPUs without exchange, but this "
              "build measures one GPU).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1703_10440_amd import amgs
    amgs.load()
    dev = torch.device("cuda:0")
    log(f"[bench] building workload {args.workload}")
    prob = make_problem(args.workload, dev)
    data = to_device(prob, dev, torch)
    log(f"[bench] m={prob.m} n={prob.n}")

    head_variant, head_prec = args.variant, args.precision
    run = Runner(prob, data, head_variant, head_prec, torch, amgs)
    t, out = time_steps(run, args.steps, args.warmup, torch)
    info = int(out.info.item())
    log(f"[bench] {head_variant}/{head_prec}: {t * 1e3:.3f} ms/step info={info}")
    roof = sweep_roofline(run, amgs, torch)
    log(f"[bench] sweep roofline {roof}")

    variants = {}
    if not args.no_variants:
        for prec in ("fp64", "fp32"):
            for v in ("naive", "ha", "hp"):
                r = Runner(prob, data, v, prec, torch, amgs)
                steps = max(2, args.steps // 4) if v == "naive" else max(3, args.steps // 2)
                tv, o = time_steps(r, steps, 1, torch)
                Qn = o.Q.double()
                variants[f"{v}_{prec}"] = {"cols_per_s": round(prob.n / tv, 1),
                                           "ms": round(tv * 1e3, 4),
                                           "info": int(o.info.item())}
                log(f"[bench] {v}/{prec}: {tv * 1e3:.3f} ms")
                del r
        for prec in ("fp64", "fp32"):
            nv = variants[f"naive_{prec}"]["ms"]
            for v in ("ha", "hp"):
                variants[f"{v}_{prec}"]["speedup_vs_naive"] = round(nv / variants[f"{v}_{prec}"]["ms"], 3)
        for v in ("naive", "ha", "hp"):
            variants[f"{v}_fp32"]["speedup_vs_fp64"] = round(
                variants[f"{v}_fp64"]["ms"] / variants[f"{v}_fp32"]["ms"], 3)

    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle")
        cpu = cpu_baseline(prob, head_variant)

    cfg = {"workload": args.workload, "m": prob.m, "n": prob.n,
           "A": "csr" if prob.csr is not None else "dense",
           "nnz": int(prob.csr.nnz) if prob.csr is not None else prob.m * prob.m,
           "variant": head_variant, "precision": head_prec}
    line = {"metric": METRIC, "value": round(prob.n / t, 2), "unit": "cols/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t * 1e3, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if head_prec == "fp64" else "f32", "data": "synthetic", "config": cfg, "roofline": roof,
            "cpu_baseline": cpu, "variants": variants}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
