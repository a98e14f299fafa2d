#!/usr/bin/env python
"""Benchmark of the adaptive-MG Wilson-Dirac hot path on one MI355X.

One step = one pass of the whole hot path on the two-level 16^3 x 32 workload
(random SU(3) links of generator width eps = 0.3, mass for min Re lambda(D) =
0.01 from the oracle's Arnoldi estimate, aggregates 4^4, Nv = 20, one complex
Gaussian right-hand side): mg_setup (null-vector relaxation, block
orthonormalisation, Galerkin D_c) followed by mg_solve to a 1e-10 relative
residual with the mixed-precision preconditioner (FP16-stored operators and
FP32 arithmetic by default; FP64 outer FGCR).  Inputs are generated on the
host and resident in device memory before the timed region.

Prints one JSON line: the step throughput, time-to-solution against plain
FP64 MG on the same setup, the roofline of the dominant kernel of the timed
solves (device time from HIP events on the library's stream), the fine
stencil on 32^3 x 64 (working set above the last-level cache) and the CPU
oracle on a bounded sample.

--kernel-probe runs fixed launches of the profiled kernels (a 1 GiB device
copy for counter calibration, the coarse stencil of the workload in every
precision, the 32^3 x 64 fine stencil) for rocprofv3 counter runs.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
WORKLOAD = "C1"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "coarse_c1_traffic.txt")

# bytes per real of (vectors, operators) for each precision class; "f16"
# keeps FP32 vectors and stores the operators (links, P, D_c) in binary16
WIDTH = {"f64": (8.0, 8.0), "f32": (4.0, 4.0), "f16": (4.0, 2.0)}


def dslash_bytes(prec, compressed=False):
    """Algorithmic bytes per site: spinor in (24 reals) + 4 links (18 reals, or
    12 when stored as two rows) + spinor out (24 reals)."""
    wv, wl = WIDTH[prec]
    return 48 * wv + 4 * (12 if compressed else 18) * wl


def coarse_bytes(n, prec):
    """Per coarse site: 9 n^2 operator entries + vector in and out."""
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
    ap.add_argument("--precond", default="f16", choices=["f64", "f32", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--kernel-probe", action="store_true")
    ap.add_argument("--workload", default="C1", choices=["C1", "C2", "C3"],
                    help="C1: the benchmark step; C2: 12 batched point sources on 24^3x48 against 12 plain "
                         "FP64 single-RHS solves; C3: three-level 32^3x64, 12 point sources, mass sweep")
    return ap.parse_args()


def workload(torch, W):
    cfg = W.CONFIGS[WORKLOAD]
    L = cfg["L"]
    U_np = W.gauge_field(L, cfg["eps"], cfg["seed"])
    b_np = W.gaussian_spinor(L, cfg["seed"])
    st_np = W.setup_starts(L, cfg["nv"][0], cfg["seed"])
    dev = torch.device("cuda:0")
    return cfg, U_np, b_np, torch.from_numpy(U_np).to(dev), torch.from_numpy(b_np).to(dev), \
        torch.from_numpy(st_np).to(dev)


def cpu_baseline(U_np, psi_np, mass, n_d_per_step):
    """Numpy FP64 oracle Wilson operator on the workload lattice; the oracle's
    step rate is bounded above by 1 / (fine-D applications per step x time
    per application)."""
    from oracle import wilson as wi
    wi.apply_D(U_np, psi_np, mass)
    n, t0 = 0, time.perf_counter()
    while n < 3 or time.perf_counter() - t0 < 15.0:
        wi.apply_D(U_np, psi_np, mass)
        n += 1
    dt = (time.perf_counter() - t0) / n
    return {"value": round(1.0 / (n_d_per_step * dt), 6), "unit": "solves/s (upper bound)", "cores": 1,
            "kind": "oracle",
            "sample": f"{n} applications of the numpy FP64 oracle Wilson operator on 16^3x32 "
                      f"({dt * 1e3:.0f} ms each, numpy elementwise work on one core); rate = 1 / "
                      f"({n_d_per_step} fine-D applications per step, setup + solve, as counted on the "
                      f"GPU run x time per application), ignoring the oracle's coarse-level work"}


def random_su3(torch, shape, g):
    """Random SU(3) matrices on the device (Gram-Schmidt of Gaussian rows,
    third row = conj(row0 x row1)); used only to time the stencil."""
    a = torch.randn(shape + (3, 3), dtype=torch.complex128, device="cuda", generator=g)
    r0 = a[..., 0, :] / torch.linalg.vector_norm(a[..., 0, :], dim=-1, keepdim=True)
    r1 = a[..., 1, :] - (r0.conj() * a[..., 1, :]).sum(-1, keepdim=True) * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.linalg.cross(r0, r1).conj()
    return torch.stack([r0, r1, r2], dim=-2).contiguous()


def large_ctx(mgwd, torch):
    L = (32, 32, 32, 64)
    g = torch.Generator(device="cuda").manual_seed(0)
    U = random_su3(torch, (4, L[3], L[2], L[1], L[0]), g)
    v = torch.randn((1, L[3], L[2], L[1], L[0], 4, 3), dtype=torch.complex128, device="cuda", generator=g)
    ctx = mgwd.MG(U, 0.1, [(4, 4, 4, 4)], [1], [v], setup_rounds=0)
    return L, ctx


def large_dslash(mgwd, torch):
    """Fine stencil on the 32^3x64 lattice (links and vectors 2-4x the last-level cache)."""
    L, ctx = large_ctx(mgwd, torch)
    out = {}
    V = L[0] * L[1] * L[2] * L[3]
    for prec in ("f64", "f32", "f16"):
        ms = ctx.time_dslash(prec, 1, 30)
        gbs_fmt = dslash_bytes(prec, compressed=True) * V / (ms * 1e-3) / 1e9
        out[prec] = {"ms": round(ms, 4), "GBps": round(gbs_fmt, 1), "frac_hbm": round(gbs_fmt / HBM_PEAK_GBPS, 3),
                     "TFLOPs": round(dslash_flops(True) * V / (ms * 1e-3) / 1e12, 2),
                     "bytes_per_site": dslash_bytes(prec, True)}
    ctx.close()
    torch.cuda.empty_cache()
    # What plain streaming reaches on this GPU: a device-to-device copy (a
    # PyTorch kernel, timed on its own stream) of as many bytes as the FP64
    # stencil reads and writes per launch.
    nbytes = int(dslash_bytes("f64", compressed=True)) * V
    src = torch.ones(nbytes // 16, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    copy_gbps = 2 * src.numel() * 8 / (e0.elapsed_time(e1) / 20 * 1e-3) / 1e9
    out["copy_GBps"] = round(copy_gbps, 1)
    for prec in ("f64", "f32", "f16"):
        out[prec]["frac_copy"] = round(out[prec]["GBps"] / copy_gbps, 3)
    del src, dst
    torch.cuda.empty_cache()
    return out


def stored_traffic(kernel, workload_name):
    """Per-launch HBM traffic of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on this kernel and workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                m = re.match(r"^TRAFFIC\s+(\S+)\s+(\S+)\s+bytes_per_launch=(\S+)", line)
                if m and m.group(1) == kernel and m.group(2) == workload_name:
                    return float(m.group(3))
    except OSError:
        pass
    return None


def kernel_probe(mgwd, torch, W):
    """Fixed launches for counter runs (one process, printed as they go)."""
    n = 1 << 27  # 1 GiB of float64
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "copy", "bytes_read": n * 8, "bytes_written": n * 8, "launches": 5}), flush=True)
    del a, b
    cfg, U_np, b_np, U, b, starts = workload(torch, W)
    ctx = mgwd.MG(U, W.mass_for(WORKLOAD), cfg["blocks"], cfg["nv"], [starts])
    for prec in ("f64", "f32", "f16"):
        ms = ctx.time_coarse(1, prec, 1, 20)
        print(json.dumps({"probe": f"coarse_{prec}", "launches": 22, "avg_ms": ms}), flush=True)
    ctx.close()
    Lg, lctx = large_ctx(mgwd, torch)
    for prec in ("f64", "f32", "f16"):
        ms = lctx.time_dslash(prec, 1, 20)
        print(json.dumps({"probe": f"dslash_{prec}_32^3x64", "launches": 22, "avg_ms": ms}), flush=True)
    lctx.close()
    # 24^3x48 with 12 right-hand sides: the matrix-core coarse stencil (tuned
    # K split) and the matrix-core restriction / prolongation, FP16-stored
    cfg2 = W.CONFIGS["C2"]
    L2 = cfg2["L"]
    U2 = torch.from_numpy(W.gauge_field(L2, cfg2["eps"], cfg2["seed"])).cuda()
    st2 = torch.from_numpy(W.setup_starts(L2, cfg2["nv"][0], cfg2["seed"])).cuda()
    ctx2 = mgwd.MG(U2, W.mass_for("C2"), cfg2["blocks"], cfg2["nv"], [st2], max_rhs=12, precond_prec="f16")
    ms = ctx2.time_coarse(1, "f16", 12, 20)
    var, us = ctx2.coarse_variant(1, "f16", 12)
    print(json.dumps({"probe": "coarse_f16_12rhs_24^3x48", "launches": 22, "avg_ms": ms, "variant": var}), flush=True)
    r12 = torch.from_numpy(W.point_sources(L2)).cuda()
    ec12 = ctx2.transfer(0, r12, 0, "f16")
    ctx2.set_transfer_variant(1)
    for _ in range(10):
        ctx2.transfer(0, r12, 0, "f16")
        ctx2.transfer(0, ec12, 1, "f16")
    torch.cuda.synchronize()
    print(json.dumps({"probe": "transfer_mma_f16_12rhs_24^3x48", "launches": 10}), flush=True)
    ctx2.close()


def multi_rhs_report(mgwd, torch, W):
    """12 point sources on 24^3x48 in one batched FP16-preconditioned solve
    against plain FP64 MG run once per source on the same setup."""
    cfg = W.CONFIGS["C2"]
    L, nv, blocks = cfg["L"], cfg["nv"], cfg["blocks"]
    U = torch.from_numpy(W.gauge_field(L, cfg["eps"], cfg["seed"])).cuda()
    st = torch.from_numpy(W.setup_starts(L, nv[0], cfg["seed"])).cuda()
    mass = W.mass_for("C2")
    b = torch.from_numpy(W.point_sources(L)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = mgwd.MG(U, mass, blocks, nv, [st], max_rhs=12)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log = lambda msg: print(msg, file=sys.stderr, flush=True)  # noqa: E731
    log(f"24^3x48: setup {setup_s:.3f} s")
    ctx.set_precond_prec("f16")
    ctx.solve(b[:12], 1e-10)  # warm-up: graphs, autotuning
    x, info, rc = ctx.solve(b, 1e-10)
    log(f"24^3x48: batched FP16 solve {info['t_solve_s']:.3f} s, iterations {info['iters'][:12]}")
    var, us = ctx.coarse_variant(1, "f16", 12)
    tr_r, tr_p, tr_us = ctx.transfer_variant("f16", 12)
    ctx.set_precond_prec("f64")
    t64, it64 = 0.0, []
    for i in range(12):
        _, i1, _ = ctx.solve(b[i:i + 1].contiguous(), 1e-10)
        t64 += i1["t_solve_s"]
        it64.append(i1["iters"][0])
        log(f"24^3x48: plain FP64 solve of source {i}: {i1['t_solve_s']:.3f} s, {i1['iters'][0]} iterations")
    ctx.close()
    # setup stage two (groups of 8 prototypes, 5 truncated-MG GCR steps,
    # FP16-stored V-cycles), then the same batched solve
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = mgwd.MG(U, mass, blocks, nv, [st], max_rhs=12, precond_prec="f16", refine_group=8, refine_iters=5)
    torch.cuda.synchronize()
    setup_r = time.perf_counter() - t0
    log(f"24^3x48: setup with stage two {setup_r:.3f} s")
    _, info_r, rc_r = ctx.solve(b, 1e-10)
    log(f"24^3x48: batched FP16 solve after stage two {info_r['t_solve_s']:.3f} s")
    ctx.close()
    refined = {"refine_group": 8, "refine_iters": 5, "setup_s": round(setup_r, 3),
               "batched_f16_solve_s": round(info_r["t_solve_s"], 3), "batched_iters": info_r["iters"][:12],
               "converged": rc_r == 0}
    return {"workload": "24^3x48, eps 0.3, aggregates 4^4, Nv 24, 12 point sources", "mass": mass,
            "setup_stage_two": refined,
            "setup_s": round(setup_s, 3), "batched_f16_solve_s": round(info["t_solve_s"], 3),
            "batched_iters": info["iters"][:12], "plain_f64_12_solves_s": round(t64, 3), "plain_f64_iters": it64,
            "speedup": round(t64 / info["t_solve_s"], 2), "coarse_variant_12rhs": var,
            "coarse_12rhs_us": round(us, 1),
            "transfer_12rhs": {"restrict_variant": tr_r, "prolong_variant": tr_p,
                               "us": {f"{d}_{'mfma' if v else 'vector'}": round(t, 1) for (d, v), t in tr_us.items()}},
            "converged": rc == 0}


def three_level_report(mgwd, torch, W):
    """Three-level MG on 32^3x64 with 12 point sources at the three nominal
    masses: outer iterations and time-to-solution (FP32 preconditioner), with
    a fresh setup at every mass and with one setup at the lightest mass reused
    for the heavier ones (mg_set_mass)."""
    cfg = W.CONFIGS["C3"]
    L, nv, blocks = cfg["L"], cfg["nv"], cfg["blocks"]
    U = torch.from_numpy(W.gauge_field(L, cfg["eps"], cfg["seed"])).cuda()
    st = torch.from_numpy(W.setup_starts(L, nv[0], cfg["seed"])).cuda()
    Lc = tuple(L[mu] // blocks[0][mu] for mu in range(4))
    st1 = torch.from_numpy(W.coarse_setup_starts(Lc, 2 * nv[0], nv[1], cfg["seed"])).cuda()
    b = torch.from_numpy(W.point_sources(L)).cuda()

    def setup(mass, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = mgwd.MG(U, mass, blocks, nv, [st, st1], max_rhs=12, precond_prec="f32", **kw)
        torch.cuda.synchronize()
        return ctx, time.perf_counter() - t0

    def solve(ctx):
        x, info, rc = ctx.solve(b, 1e-10)
        return {"solve_s": round(info["t_solve_s"], 3), "iters_mean": round(float(sum(info["iters"][:12])) / 12, 1),
                "iters_max": max(info["iters"][:12]), "converged": rc == 0}

    fresh, reuse = [], []
    for target in cfg["targets"]:
        mass = W.mass_for("C3", target)
        ctx, ts = setup(mass)
        fresh.append(dict(min_re_lambda_nominal=target, mass=mass, setup_s=round(ts, 3), **solve(ctx)))
        ctx.close()
        print(json.dumps(fresh[-1]), file=sys.stderr, flush=True)
    lightest = min(cfg["targets"])
    ctx, ts = setup(W.mass_for("C3", lightest))
    for target in sorted(cfg["targets"]):
        ctx.set_mass(W.mass_for("C3", target))
        reuse.append(dict(min_re_lambda_nominal=target, **solve(ctx)))
        print(json.dumps(reuse[-1]), file=sys.stderr, flush=True)
    ctx.close()
    # the paper's cycle (V(0,4) with GMRES(4) post-relaxation, W-cycle on the
    # intermediate level) and its setup stage two, against the default MR
    # 4/4 V-cycle, at the lightest mass
    mass = W.mass_for("C3", lightest)
    cycles = []
    for name, kw in (("MR 4/4 V-cycle", {}),
                     ("GMRES(4) V(0,4) W-cycle", dict(smoother="gmres", pre=0, post=4, cycles=2)),
                     ("MR 4/4 V-cycle, setup stage two (groups of 8)", dict(refine_group=8, refine_iters=5)),
                     ("GMRES(4) V(0,4) W-cycle, setup stage two (groups of 4)",
                      dict(smoother="gmres", pre=0, post=4, cycles=2, refine_group=4, refine_iters=5))):
        c2, ts2 = setup(mass, **kw)
        cycles.append(dict(cycle=name, setup_s=round(ts2, 3), **solve(c2)))
        c2.close()
        print(json.dumps(cycles[-1]), file=sys.stderr, flush=True)
    return {"workload": "32^3x64, eps 0.35, aggregates 4^4 then 2^4, Nv 24/24, 12 point sources, FP32 "
                        "preconditioner", "fresh_setup": fresh,
            "setup_at_lightest_mass_reused": {"setup_s": round(ts, 3), "solves": reuse},
            "cycles_at_lightest_mass": cycles,
            "dslash_32^3x64": large_dslash(mgwd, torch)}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); multi-GPU execution is not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1005_3043_amd as mgwd
    import workloads as W

    if a.kernel_probe:
        kernel_probe(mgwd, torch, W)
        return
    if a.workload == "C2":
        print(json.dumps(multi_rhs_report(mgwd, torch, W)), flush=True)
        return
    if a.workload == "C3":
        print(json.dumps(three_level_report(mgwd, torch, W)), flush=True)
        return

    cfg, U_np, b_np, U, b, starts = workload(torch, W)
    L, nv, blocks = cfg["L"], cfg["nv"], cfg["blocks"]
    mass = W.mass_for(WORKLOAD)
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

    # plain FP64 MG and the FP32 preconditioner on the same workload
    _, info64 = step("f64", True)
    _, info32 = step("f32", True)

    # the paper's setup stage two on the same workload (groups of 4 of the
    # N_v prototypes, 5 truncated-MG GCR steps each, V-cycles in the
    # preconditioner precision), reported beside the headline setup
    torch.cuda.synchronize()
    t0r = time.perf_counter()
    ctx_r = mgwd.MG(U, mass, blocks, nv, [starts], refine_group=4, refine_iters=5, precond_prec=a.precond)
    torch.cuda.synchronize()
    setup_r = time.perf_counter() - t0r
    _, info_r, rc_r = ctx_r.solve(b, 1e-10)
    ctx_r.close()
    refined = {"refine_group": 4, "refine_iters": 5, "setup_s": round(setup_r, 4),
               "time_to_solution_s": round(info_r["t_solve_s"], 4), "iters": info_r["iters"][0],
               "converged": rc_r == 0}

    # kernel-class aggregates over the timed steps.  Every fine-stencil
    # launch is timed; inside the captured CGNR chunks the event pairs sample
    # the first iteration's two coarse launches of every chunk.  The coarse
    # average launch time therefore comes from the sample, and its bytes per
    # launch count only the effective applications among all dispatches
    # (dispatches queued after a right-hand side converged return at once).
    # Stencil applications made inside whole-solve CGNR launches count as
    # applications, not dispatches, and are left out of the per-launch class.
    agg = {}
    for inf in infos:
        in_whole = sum(d["sites"] for k, d in inf["kernels"].items() if k.startswith("cgnr")) / Vc
        for k, d in inf["kernels"].items():
            e = agg.setdefault(k, {"ms": 0.0, "launches": 0, "sites": 0.0, "eff": 0.0})
            e["ms"] += d["ms"]
            e["launches"] += d["launches"]
            e["sites"] += d["sites"]
            if k.startswith("coarse") and d["launches"]:
                e["eff"] += (inf["n_coarse_apply"] - in_whole) / max(inf["n_coarse_dispatch"], 1) * d["launches"]

    def achieved(k):
        e = agg[k]
        if e["launches"] == 0 or e["ms"] == 0:
            return None
        prec = k.split("_")[1]
        avg_us = e["ms"] * 1e3 / e["launches"]
        if k.startswith("dslash"):
            # the workload links are SU(3), so the stencil reads them as two rows
            bpl = dslash_bytes(prec, True) * e["sites"] / e["launches"]
            fpl = dslash_flops(True) * e["sites"] / e["launches"]
        elif k.startswith("cgnr"):
            # one launch = one whole coarsest CGNR: the operator read once
            # (then held in registers), and per iteration and site the FP32
            # vectors of both phases (reads z, p_old, r_old, w, p, e; writes
            # p, w, r, z, e: 11 n complex) plus five partial sums
            apps = e["sites"] / Vc / e["launches"]  # stencil applications per launch
            wv, wl = WIDTH[prec]
            bpl = (2 * 9 * n_c * n_c * wl + (apps / 2) * (11 * n_c * 2 * wv + 5 * 8)) * Vc
            fpl = coarse_flops(n_c) * Vc * apps
        else:
            frac = e["eff"] / e["launches"]
            bpl = coarse_bytes(n_c, prec) * Vc * frac
            fpl = coarse_flops(n_c) * Vc * frac
        return {"GBps": bpl / avg_us / 1e3, "TFLOPs": fpl / avg_us / 1e6, "avg_us": avg_us,
                "launches": e["launches"], "bytes_per_launch": bpl, "total_ms": e["ms"]}

    kern = {k: achieved(k) for k in agg if achieved(k) is not None}
    # dominant kernel by estimated device time over all its dispatches
    disp = {k: (infos[-1]["n_coarse_dispatch"] * len(infos) if k.startswith("coarse") else kern[k]["launches"])
            for k in kern}
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * disp[k])
    kd = kern[dom]
    traffic = stored_traffic(dom, WORKLOAD)
    roofline = {"bound": "hbm", "achieved": round(kd["GBps"], 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(kd["GBps"] / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": dom, "avg_launch_us": round(kd["avg_us"], 2),
                "bytes_per_launch": round(kd["bytes_per_launch"])}

    solve_s = sum(i["t_solve_s"] for i in infos) / len(infos)
    setup_s = sum(i["t_setup_s"] for i in infos) / len(infos)
    dsl = {k: {"GBps": round(v["GBps"], 1), "avg_us": round(v["avg_us"], 2), "launches": v["launches"]}
           for k, v in kern.items()}
    n_d_setup = 5 * (1 + 4) * nv[0]
    out = {
        "metric": "dslash HBM GB/s; MG time-to-solution to 1e-10 rel. residual vs plain FP64 MG",
        "value": round(1e3 / ms_step, 4),
        "unit": "solves/s (mg_setup + mg_solve to 1e-10, one RHS)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 outer / " + {"f16": "f16-stored operators, f32 arithmetic", "f32": "f32",
                                   "f64": "f64"}[a.precond] + " preconditioner",
        "data": "synthetic (seeded random SU(3) links, Gaussian source)",
        "config": {"workload": f"two-level MG, {L[0]}^3x{L[3]}, eps {cfg['eps']}, min Re lambda "
                               f"{cfg['targets'][0]}, aggregates 4^4, Nv {nv[0]}, 1 RHS",
                   "mass": mass, "precond": a.precond},
        "time_to_solution_s": round(solve_s, 4),
        "setup_s": round(setup_s, 4),
        "fp64_plain_time_to_solution_s": round(info64["t_solve_s"], 4),
        "fp32_time_to_solution_s": round(info32["t_solve_s"], 4),
        "speedup_vs_plain_fp64": round(info64["t_solve_s"] / solve_s, 3),
        "iters": infos[-1]["iters"][0], "iters_fp64": info64["iters"][0], "iters_fp32": info32["iters"][0],
        "true_rel_resid": true_res,
        "fine_dslash_per_solve": infos[-1]["n_fine_dslash"],
        "cgnr_iters_per_solve": infos[-1]["n_cgnr_iters"],
        "kernels": dsl,
        "setup_stage_two": refined,
        "roofline": roofline,
    }
    if not a.no_large:
        out["dslash_32^3x64"] = large_dslash(mgwd, torch)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(U_np, b_np, mass, n_d_setup + infos[-1]["n_fine_dslash"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
