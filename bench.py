#!/usr/bin/env python
"""Benchmark of the adaptive-MG Wilson-Dirac hot path on one MI355X.

One step = one pass of the whole hot path on the two-level 16^3x32 workload
(random SU(3) links with eps = 0.3, mass for min Re lambda(D) = 0.01,
aggregates 4^4, Nv = 20, one complex Gaussian right-hand side):
mg_setup (null-vector relaxation, block orthonormalisation, Galerkin D_c)
followed by mg_solve to a 1e-10 relative residual with the FP32
preconditioner (FP64 outer FGCR).  Inputs are generated on the host and
resident in device memory before the timed region.

Prints one JSON line.  Besides the step throughput it reports the plain FP64
MG time-to-solution on the same setup, the fine-stencil (dslash) GB/s
measured live in the timed solves, the roofline of the dominant kernel, the
dslash on the 32^3x64 lattice (working set far above the last-level cache),
and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
WORKLOAD = "C1"


# bytes per real of (vectors, operators) for each precision class; "f16" keeps
# FP32 vectors and stores the operators (links, P, D_c) in binary16
WIDTH = {"f64": (8.0, 8.0), "f32": (4.0, 4.0), "f16": (4.0, 2.0)}


def dslash_bytes(prec, compressed=False):
    """Algorithmic bytes per site: spinor in (24 reals) + 4 links (18 reals, or
    12 when stored as two rows) + spinor out (24 reals)."""
    wv, wl = WIDTH[prec]
    return 48 * wv + 4 * (12 if compressed else 18) * wl


def coarse_bytes(n, prec):    # 9 n^2 operator entries + vector in/out, per coarse site
    wv, wl = WIDTH[prec]
    return 2 * (9 * n * n * wl + 2 * n * wv)


def dslash_flops(compressed=False):
    """Hop term 1320 flops + diagonal 48; + 8 x 42 to rebuild third link rows."""
    return 1320.0 + 48.0 + (8 * 42.0 if compressed else 0.0)


def coarse_flops(n):
    return 8.0 * 9 * n * n


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precond", default="f32", choices=["f64", "f32", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    return ap.parse_args()


def cpu_baseline(U_np, psi_np, mass):
    """The numpy FP64 oracle Wilson operator on the same lattice (bounded sample)."""
    from oracle import wilson as wi
    V = psi_np.size // 12
    wi.apply_D(U_np, psi_np, mass)
    n, t0 = 0, time.perf_counter()
    while n < 3 or time.perf_counter() - t0 < 10.0:
        wi.apply_D(U_np, psi_np, mass)
        n += 1
    dt = (time.perf_counter() - t0) / n
    return {"value": round(dslash_bytes("f64") * V / dt / 1e9, 3), "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n} applications of the numpy FP64 oracle Wilson operator on 16^3x32 "
                      f"({dt * 1e3:.0f} ms each; numpy elementwise work is single-threaded)"}


def random_su3(torch, shape, g):
    """Random SU(3) matrices on the device (Gram-Schmidt of Gaussian rows,
    third row = conj(row0 x row1)); used only to time the stencil."""
    a = torch.randn(shape + (3, 3), dtype=torch.complex128, device="cuda", generator=g)
    r0 = a[..., 0, :] / torch.linalg.vector_norm(a[..., 0, :], dim=-1, keepdim=True)
    r1 = a[..., 1, :] - (r0.conj() * a[..., 1, :]).sum(-1, keepdim=True) * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.linalg.cross(r0, r1).conj()
    return torch.stack([r0, r1, r2], dim=-2).contiguous()


def large_dslash(mgwd, torch):
    """Fine stencil on the 32^3x64 lattice (links and vectors 2-4x the last-level cache)."""
    L = (32, 32, 32, 64)
    g = torch.Generator(device="cuda").manual_seed(0)
    U = random_su3(torch, (4, L[3], L[2], L[1], L[0]), g)
    v = torch.randn((1, L[3], L[2], L[1], L[0], 4, 3), dtype=torch.complex128, device="cuda", generator=g)
    ctx = mgwd.MG(U, 0.1, [(4, 4, 4, 4)], [1], [v], setup_rounds=0)
    out = {}
    V = L[0] * L[1] * L[2] * L[3]
    for prec in ("f64", "f32", "f16"):
        ms = ctx.time_dslash(prec, 1, 30)
        gbs = dslash_bytes(prec) * V / (ms * 1e-3) / 1e9
        gbs_fmt = dslash_bytes(prec, compressed=True) * V / (ms * 1e-3) / 1e9
        out[prec] = {"ms": round(ms, 4), "GBps_18real_equiv": round(gbs, 1),
                     "GBps_stored_format": round(gbs_fmt, 1), "frac_hbm": round(gbs_fmt / HBM_PEAK_GBPS, 3),
                     "TFLOPs": round(dslash_flops(True) * V / (ms * 1e-3) / 1e12, 2)}
    ctx.close()
    del U, v
    torch.cuda.empty_cache()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU path is design-only.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1005_3043_amd as mgwd
    import workloads as W

    cfg = W.CONFIGS[WORKLOAD]
    L, nv, blocks = cfg["L"], cfg["nv"], cfg["blocks"]
    mass = W.mass_for(WORKLOAD)
    U_np = W.gauge_field(L, cfg["eps"], cfg["seed"])
    b_np = W.gaussian_spinor(L, cfg["seed"])
    st_np = W.setup_starts(L, nv[0], cfg["seed"])
    dev = torch.device("cuda:0")
    U = torch.from_numpy(U_np).to(dev)
    b = torch.from_numpy(b_np).to(dev)
    starts = torch.from_numpy(st_np).to(dev)
    V = L[0] * L[1] * L[2] * L[3]
    n_c = 2 * nv[0]
    Vc = V // 256

    def step(prec, timing):
        ctx = mgwd.MG(U, mass, blocks, nv, [starts])
        ctx.set_timing(timing)
        if prec != "f64":
            ctx.set_precond_prec(prec)
        x, info, rc = ctx.solve(b, 1e-10)
        ctx.close()
        if rc != 0:
            raise RuntimeError("mg_solve did not converge")
        return x, info

    for _ in range(a.warmup):
        step(a.precond, True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        x, info = step(a.precond, True)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / a.steps * 1e3

    # true residual of the last solution, FP64 on the GPU via the fine operator
    r = b - mgwd.wilson_apply(U, x, mass)
    true_res = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))

    # plain FP64 MG on the same workload (time-to-solution reference)
    _, info64 = step("f64", True)

    # kernel-class aggregates over the timed steps.  Coarse-stencil bytes
    # count only effective applications (n_coarse_apply); the time includes
    # the early-exit dispatches queued after CGNR convergence.
    agg = {}
    for inf in infos:
        for k, d in inf["kernels"].items():
            e = agg.setdefault(k, {"ms": 0.0, "launches": 0, "sites": 0.0})
            e["ms"] += d["ms"]
            e["launches"] += d["launches"]
            e["sites"] += d["sites"] if k.startswith("dslash") else inf["n_coarse_apply"] * Vc

    def achieved(k):
        e = agg[k]
        if e["launches"] == 0 or e["ms"] == 0:
            return None
        prec = k.split("_")[1]
        # the workload links are SU(3), so the stencil reads them as two rows
        per_site = dslash_bytes(prec, True) if k.startswith("dslash") else coarse_bytes(n_c, prec)
        fl = dslash_flops(True) if k.startswith("dslash") else coarse_flops(n_c)
        return {"GBps": per_site * e["sites"] / (e["ms"] * 1e-3) / 1e9,
                "TFLOPs": fl * e["sites"] / (e["ms"] * 1e-3) / 1e12,
                "avg_us": e["ms"] * 1e3 / e["launches"], "launches": e["launches"],
                "bytes_per_launch": per_site * e["sites"] / e["launches"], "total_ms": e["ms"]}

    kern = {k: achieved(k) for k in agg if achieved(k) is not None}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    kd = kern[dom]
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(kd["GBps"], 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(kd["GBps"] / HBM_PEAK_GBPS, 4), "traffic": None,
                "avg_launch_us": round(kd["avg_us"], 2), "bytes_per_launch": kd["bytes_per_launch"]}

    solve_s = sum(i["t_solve_s"] for i in infos) / len(infos)
    setup_s = sum(i["t_setup_s"] for i in infos) / len(infos)
    dsl = {k: {"GBps": round(v["GBps"], 1), "avg_us": round(v["avg_us"], 2), "launches": v["launches"]}
           for k, v in kern.items()}
    out = {
        "metric": "dslash HBM GB/s; MG time-to-solution to 1e-10 rel. residual vs plain FP64 MG",
        "value": round(1e3 / ms_step, 4),
        "unit": "solves/s (mg_setup + mg_solve to 1e-10, one RHS)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 outer / " + a.precond + " preconditioner",
        "data": "synthetic (seeded random SU(3) links, Gaussian source)",
        "config": {"workload": f"two-level MG, {L[0]}^3x{L[3]}, eps {cfg['eps']}, min Re lambda "
                               f"{cfg['targets'][0]}, aggregates 4^4, Nv {nv[0]}, 1 RHS",
                   "mass": mass, "precond": a.precond},
        "time_to_solution_s": round(solve_s, 4),
        "setup_s": round(setup_s, 4),
        "fp64_plain_time_to_solution_s": round(info64["t_solve_s"], 4),
        "speedup_vs_plain_fp64": round(info64["t_solve_s"] / solve_s, 3),
        "iters": infos[-1]["iters"][0], "iters_fp64": info64["iters"][0],
        "true_rel_resid": true_res,
        "fine_dslash_per_solve": infos[-1]["n_fine_dslash"],
        "cgnr_iters_per_solve": infos[-1]["n_cgnr_iters"],
        "kernels": dsl,
        "roofline": roofline,
    }
    if not a.no_large:
        out["dslash_32^3x64"] = large_dslash(mgwd, torch)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(U_np, b_np, mass)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
