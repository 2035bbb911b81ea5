"""Benchmark of the Hubbard exact-diagonalisation hot path on one MI355X.

Workload: the 4x4 periodic square lattice at half filling (8 up + 8 down
electrons, t = 1, U = 8; dim = 12870^2 = 165,636,900), seeded synthetic start
vector.  One step = one Lanczos iteration of Alg. 1 (fused H.v with the
three-term update, the a_j / b_{j+1} reductions, the q - a_j f_j update and
the host tridiagonal solve).

Printed JSON line (one):
  value          H.v algorithmic bandwidth in GB/s, FP64: 2 * dim * 8 bytes
                 (x read once, y written once) / mean H.v kernel time
  ms_per_step    FP64 Lanczos iteration time
  lanczos_*      Lanczos iterations/s in FP64 and in mixed precision
  roofline       the H.v kernel against the 8 TB/s HBM peak
  cpu_baseline   the sequential FP64 oracle on one host core, on a bounded sample
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·v HBM GB/s + Lanczos iters/s, 4x4 Hubbard; batched p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_apply(hb, torch, h, precision, steps, warmup):
    """Mean duration of one H.v kernel, from HIP events on the launch stream."""
    hb.hubbard_set_precision(h, precision)
    dt = torch.float64 if precision == hb.HUBBARD_FP64 else torch.float32
    x = torch.empty(h.dim, dtype=dt, device="cuda:0")
    y = torch.empty_like(x)
    f = torch.empty(h.dim, dtype=torch.float64, device="cuda:0")
    hb.hubbard_start_raw(12043425, h.dim, f)
    x.copy_(f)
    del f
    for _ in range(warmup):
        hb.hubbard_apply(h, x, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        hb.hubbard_apply(h, x, y)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps * 1e-3


def time_lanczos(hb, torch, h, precision, steps, warmup, seed):
    if warmup:
        hb.hubbard_lanczos_ex(h, tol=-1.0, max_iter=warmup, precision=precision, seed=seed, history=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = hb.hubbard_lanczos_ex(h, tol=-1.0, max_iter=steps, precision=precision, seed=seed)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, r


def cpu_baseline(p):
    """The oracle, as it stands, on one host core: one Lanczos iteration of the
    same sector (model build and start vector excluded)."""
    import numpy as np  # noqa: F401
    import oracle
    m = oracle.Model(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    f1 = oracle.start_vector(p.seed, m.dim)
    t0 = time.perf_counter()
    m.lanczos(f1, tol=-1.0, max_iter=1)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "Lanczos iters/s", "cores": 1, "kind": "oracle",
            "sample": "1 FP64 Lanczos iteration (H.v + 3 vector passes) of the 4x4 8u8d sector, "
                      "single thread, gcc -O2; %.1f s" % dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1204_3425_amd as hb
    import workload

    p = workload.square4x4()
    log("building", p.name)
    h = hb.hubbard_build(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    hb.hubbard_set_stream(h, torch.cuda.current_stream().cuda_stream)
    info = hb.hubbard_info(h)

    res = {}
    for name, prec, es in (("fp64", hb.HUBBARD_FP64, 8), ("mixed", hb.HUBBARD_MIXED, 4)):
        log("timing H.v", name)
        t_hv = time_apply(hb, torch, h, prec, max(10, args.steps // 4), 3)
        log("timing Lanczos", name, args.steps, "steps")
        t_lz, r = time_lanczos(hb, torch, h, prec, args.steps, args.warmup, p.seed)
        res[name] = {"hv_s": t_hv, "hv_gbs": 2.0 * p.dim * es / t_hv / 1e9, "lanczos_s": t_lz,
                     "iters": r["n_iter"], "E0": r["E0"]}
        log(name, "H.v %.1f us (%.0f GB/s)" % (t_hv * 1e6, res[name]["hv_gbs"]),
            "Lanczos %.3f ms/iter, E0 %.12f" % (t_lz / r["n_iter"] * 1e3, r["E0"]))

    f64 = res["fp64"]
    ms_step = f64["lanczos_s"] / f64["iters"] * 1e3
    out = {
        "metric": METRIC,
        "value": round(f64["hv_gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "4x4 periodic square lattice, 8 up + 8 down, t=1, U=8, dim 165,636,900; "
                               "seeded SplitMix64 start vector; %d Lanczos iterations" % args.steps,
                   "dim": p.dim, "precision": "fp64 (mixed reported beside)"},
        "lanczos_iters_per_s": {k: round(v["iters"] / v["lanczos_s"], 2) for k, v in res.items()},
        "hv_us": {k: round(v["hv_s"] * 1e6, 1) for k, v in res.items()},
        "hv_gbs": {k: round(v["hv_gbs"], 1) for k, v in res.items()},
        "E0": {k: v["E0"] for k, v in res.items()},
        "roofline": {"bound": "hbm", "achieved": round(f64["hv_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(f64["hv_gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "hv_kernel (FP64 H.v, store mode)",
                     "algorithmic_bytes_per_launch": 2 * p.dim * 8},
        "table_bytes": info["device_bytes"],
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one core)")
        cb = cpu_baseline(p)
        cb["gpu_fp64_vs_cpu"] = round(out["lanczos_iters_per_s"]["fp64"] / cb["value"], 1)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
