#!/usr/bin/env python
"""Benchmark of the adaptive-MG Wilson-Dirac hot path on one MI355X.

One step = one pass of the whole hot path on the three-level 32^3 x 64
workload (random SU(3) links of generator width eps = 0.35, the mass of
nominal min Re lambda(D) = 0.1, aggregates 4^4 then 2^4, Nv = 24 on both
levels, the 12 spin-colour point sources at the origin): mg_setup (null-vector
relaxation in FP32, block orthonormalisation and Galerkin D_c on both levels
in FP64) followed by one batched mg_solve of all 12 sources to a 1e-10
relative residual with the FP32 preconditioner (FP64 outer flexible GCR).  Inputs are generated on
the host and resident in device memory before the timed region.

Prints one JSON line: right-hand sides solved per second, the plain FP64
single-RHS MG on the same setup (each source on its own), the FP16-stored
preconditioner, the FP32 preconditioner with binary16-stored P in its
transfers (transfer_prec), the lightest nominal mass with the paper's setup stage two,
the roofline of the dominant kernel of the timed steps (device time from HIP
events on the library's stream), the fine stencil on 32^3 x 64 with one
right-hand side, the two-level 16^3 x 32 workload, and the CPU oracle on a
bounded sample.

--kernel-probe runs fixed launches of the profiled kernels (a 1 GiB device
copy for counter calibration, the 32^3 x 64 fine stencil with 12 and 1
right-hand sides in each precision class, and with 12 in the form of the MR
step by the q recursion in the FP32 and FP16 classes) for rocprofv3 counter
runs.
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
HEADLINE_TARGET = 0.1   # nominal min Re lambda of the headline 32^3 x 64 step
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_c3_12rhs_traffic.txt")
# kernel name in the counter summary for each precision class of the stencil
TRAFFIC_KERNEL = {"dslash_f64": "dslash_f64_12rhs", "dslash_f32": "dslash_f32_12rhs",
                  "dslash_f16": "dslash_f16_12rhs", "dslash_mrq_f32": "dslash_mrq_f32_12rhs",
                  "dslash_mrq_f16": "dslash_mrq_f16_12rhs"}

# bytes per real of (fine-level spinors, operators) for each precision class;
# "f16" stores the operators (links, P, D_c) in binary16 and the fine spinors
# of the cycle in binary16 with one FP32 scale per site (52 bytes per site
# for 24 reals); coarse vectors stay FP32 in that class
WIDTH = {"f64": (8.0, 8.0), "f32": (4.0, 4.0), "f16": (52.0 / 24.0, 2.0)}
COARSE_VEC = {"f64": 8.0, "f32": 4.0, "f16": 4.0}


def dslash_bytes(prec, compressed=False):
    """Algorithmic bytes per site: spinor in (24 reals) + 4 links (18 reals, or
    12 when stored as two rows) + spinor out (24 reals)."""
    wv, wl = WIDTH[prec]
    return 48 * wv + 4 * (12 if compressed else 18) * wl


def coarse_bytes(n, prec):
    """Per coarse site: 9 n^2 operator entries + vector in and out."""
    wl = WIDTH[prec][1]
    return 2 * (9 * n * n * wl + 2 * n * COARSE_VEC[prec])


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
    ap.add_argument("--setup-prec", default="f32", choices=["f64", "f32"],
                    help="arithmetic of the null-vector relaxation (setup stage one)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-c1", action="store_true")
    ap.add_argument("--kernel-probe", action="store_true")
    ap.add_argument("--workload", default="C3", choices=["C3", "C1", "C2", "C3sweep"],
                    help="C3: the benchmark step (three-level 32^3x64, 12 batched point sources); C1: two-level "
                         "16^3x32, one source; C2: 12 batched point sources on 24^3x48 against 12 plain FP64 "
                         "single-RHS solves; C3sweep: 32^3x64 at the three nominal masses")
    return ap.parse_args()


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
    """Fixed launches for counter runs, printed as they go: a 1 GiB device copy
    (counter calibration), then on the 32^3 x 64 workload (its links, the
    headline setup) the fine stencil with 12 right-hand sides per launch in
    each precision class, as the benchmark step launches it (the step's MR
    launches add per-tile partial sums, 24 bytes per tile and right-hand
    side), and with one right-hand side; then the coarse stencil of levels 1
    and 2 and the fine-level restriction and prolongation with 12 right-hand
    sides in the FP32 class (the kernels the autotuner picks for those shapes:
    the matrix-core GEMMs; the transfers here without the V-cycle's fused
    smoother terms)."""
    n = 1 << 27  # 1 GiB of float64
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "copy", "bytes_read": n * 8, "bytes_written": n * 8, "launches": 5}), flush=True)
    del a, b
    cfg = W.CONFIGS["C3"]
    L, nv, blocks = cfg["L"], cfg["nv"], cfg["blocks"]
    U = torch.from_numpy(W.gauge_field(L, cfg["eps"], cfg["seed"])).cuda()
    st = torch.from_numpy(W.setup_starts(L, nv[0], cfg["seed"])).cuda()
    Lc = tuple(L[mu] // blocks[0][mu] for mu in range(4))
    st1 = torch.from_numpy(W.coarse_setup_starts(Lc, 2 * nv[0], nv[1], cfg["seed"])).cuda()
    ctx = mgwd.MG(U, W.mass_for("C3", HEADLINE_TARGET), blocks, nv, [st, st1], max_rhs=12, setup_prec="f32")
    for prec in ("f64", "f32", "f16"):
        for nrhs in (12, 1):
            ms = ctx.time_dslash(prec, nrhs, 10)
            print(json.dumps({"probe": f"dslash_{prec}_{nrhs}rhs", "launches": 12, "avg_ms": ms}), flush=True)
    for prec in ("f32", "f16"):
        ms = ctx.time_dslash_mrq(prec, 12, 10)
        print(json.dumps({"probe": f"dslash_mrq_{prec}_12rhs", "launches": 12, "avg_ms": ms}), flush=True)
    for level in (1, 2):
        ms = ctx.time_coarse(level, "f32", 12, 10)
        var, _ = ctx.coarse_variant(level, "f32", 12)
        print(json.dumps({"probe": f"coarse_f32_level{level}_12rhs", "variant": var, "launches": 12, "avg_ms": ms}),
              flush=True)
    gen = torch.Generator(device="cuda").manual_seed(7)
    v = torch.randn((12, L[3], L[2], L[1], L[0], 4, 3), dtype=torch.complex128, device="cuda", generator=gen)
    for _ in range(6):
        vc = ctx.transfer(0, v, 0, "f32")
        ctx.transfer(0, vc, 1, "f32")
    torch.cuda.synchronize()
    rv, pv, _ = ctx.transfer_variant("f32", 12)
    print(json.dumps({"probe": "transfer_f32_12rhs", "restrict_variant": rv, "prolong_variant": pv, "launches": 6}),
          flush=True)
    del v, vc
    ctx.close()


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


def oracle_baseline(U3_np, mass3, n_d_step, nrhs):
    """The CPU oracle timed on this host: one full C0 setup + solve with the
    numpy oracle, and the oracle's C operator (OpenMP) on the 32^3 x 64
    lattice; the rate for the headline step is bounded above by nrhs / (fine-D
    applications of the step x time per application), which leaves out all
    coarse-level and vector work (about a tenth of the oracle's C0 time)."""
    import numpy as np

    import workloads as W
    from oracle import cref
    from oracle import solvers as so
    from oracle import wilson as wi

    cfg = W.CONFIGS["C0"]
    L = cfg["L"]
    U = W.gauge_field(L, cfg["eps"], cfg["seed"])
    m = W.mass_for("C0")
    t0 = time.perf_counter()
    h = so.mg_setup(U, m, so.MGParams(blocks=cfg["blocks"], nv=cfg["nv"]), W.setup_starts(L, cfg["nv"][0], cfg["seed"]))
    t1 = time.perf_counter()
    b = W.gaussian_spinor(L, cfg["seed"])
    _, it0, conv0, _ = so.mg_solve(h, b, 1e-10)
    t2 = time.perf_counter()
    nD0 = h.stats["fine_D"]
    tD0 = 0.0
    for _ in range(3):
        ta = time.perf_counter()
        wi.apply_D(U, b, m)
        tD0 += (time.perf_counter() - ta) / 3
    psi = np.ascontiguousarray(W.gaussian_spinor(tuple(reversed(U3_np.shape[1:5])), 3))
    cref.apply_D(U3_np, psi, mass3)
    n, ta = 0, time.perf_counter()
    while n < 3 or time.perf_counter() - ta < 5.0:
        cref.apply_D(U3_np, psi, mass3)
        n += 1
    tD3 = (time.perf_counter() - ta) / n
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(nrhs / (n_d_step * tD3), 6), "unit": "right-hand sides/s (upper bound)",
            "cores": threads, "kind": "oracle",
            "sample": f"C0 (8^4, Nv 8) oracle setup + solve timed in full: {t1 - t0:.1f} s + {t2 - t1:.1f} s, "
                      f"{it0} iterations, {nD0} fine-D applications in the solve ({nD0 * tD0 / (t2 - t1):.0%} of its "
                      f"time); the oracle's C operator on 32^3x64 timed {n} times ({tD3:.3f} s each, OpenMP on "
                      f"{threads} threads of {model or 'this host'}); rate = {nrhs} / ({n_d_step} fine-D "
                      f"applications of the step x time per application), coarse work left out",
            "cpu_model": model, "c0_setup_s": round(t1 - t0, 2), "c0_solve_s": round(t2 - t1, 2)}


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
    if a.workload == "C3sweep":
        print(json.dumps(three_level_report(mgwd, torch, W)), flush=True)
        return
    if a.workload == "C1":
        print(json.dumps(c1_report(mgwd, torch, W, a)), flush=True)
        return

    log = lambda msg: print(msg, file=sys.stderr, flush=True)  # noqa: E731
    cfg = W.CONFIGS["C3"]
    L, nv, blocks = cfg["L"], cfg["nv"], cfg["blocks"]
    target = HEADLINE_TARGET
    mass = W.mass_for("C3", target)
    V = L[0] * L[1] * L[2] * L[3]
    log("generating the 32^3x64 inputs")
    U_np = W.gauge_field(L, cfg["eps"], cfg["seed"])
    U = torch.from_numpy(U_np).cuda()
    st = torch.from_numpy(W.setup_starts(L, nv[0], cfg["seed"])).cuda()
    Lc = tuple(L[mu] // blocks[0][mu] for mu in range(4))
    st1 = torch.from_numpy(W.coarse_setup_starts(Lc, 2 * nv[0], nv[1], cfg["seed"])).cuda()
    b = torch.from_numpy(W.point_sources(L)).cuda()
    nrhs = b.shape[0]
    torch.cuda.synchronize()

    def setup(**kw):
        return mgwd.MG(U, mass, blocks, nv, [st, st1], max_rhs=nrhs, precond_prec=a.precond,
                       setup_prec=a.setup_prec, **kw)

    phase_ms = {"create": [], "solve": [], "close": []}

    def step(timing):
        t0 = time.perf_counter()
        ctx = setup()
        t1 = time.perf_counter()
        ctx.set_timing(timing)
        x, info, rc = ctx.solve(b, 1e-10)
        t2 = time.perf_counter()
        ctx.close()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for k, v in (("create", t1 - t0), ("solve", t2 - t1), ("close", t3 - t2)):
            phase_ms[k].append(round(v * 1e3, 1))
        if rc != 0:
            raise RuntimeError("mg_solve did not converge")
        return x, info

    for i in range(a.warmup):
        step(True)
        log(f"warm-up step {i + 1}/{a.warmup} done")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        x, info = step(True)
        infos.append(info)
        log(f"step {i + 1}/{a.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / a.steps * 1e3

    # true residual of every right-hand side of the last step, FP64 on the GPU
    r = b - mgwd.wilson_apply(U, x, mass)
    true_res = max(float(torch.linalg.vector_norm(r[i]) / torch.linalg.vector_norm(b[i])) for i in range(nrhs))
    del r

    # plain FP64 single-RHS MG on the same setup: every source on its own
    ctx = setup()
    ctx.set_precond_prec("f64")
    t64, it64 = 0.0, []
    for i in range(nrhs):
        _, i1, rc1 = ctx.solve(b[i:i + 1].contiguous(), 1e-10)
        if rc1 != 0:
            raise RuntimeError("plain FP64 solve did not converge")
        t64 += i1["t_solve_s"]
        it64.append(i1["iters"][0])
    log(f"plain FP64 MG, {nrhs} sources one at a time: {t64:.3f} s")
    # the same batched solve with the FP16-stored preconditioner (second solve:
    # the first also tunes that class's kernels, once per process)
    ctx.set_precond_prec("f16")
    for _ in range(2):
        _, i16, rc16 = ctx.solve(b, 1e-10)
    ctx.close()
    # the FP32 preconditioner with its transfers reading the binary16 copy of P
    # (second solve on the context: the first also tunes the transfer kernels
    # for that storage, once per process)
    ctx = setup(transfer_prec="f16")
    for _ in range(2):
        _, itp, rctp = ctx.solve(b, 1e-10)
    ctx.close()
    setup64_s = sum(i["t_setup_s"] for i in infos) / len(infos)

    # the lightest nominal mass with the paper's setup stage two
    light = min(cfg["targets"])
    torch.cuda.synchronize()
    tl0 = time.perf_counter()
    ctx = mgwd.MG(U, W.mass_for("C3", light), blocks, nv, [st, st1], max_rhs=nrhs, precond_prec=a.precond,
                  setup_prec=a.setup_prec, refine_group=8, refine_iters=5)
    torch.cuda.synchronize()
    setup_l = time.perf_counter() - tl0
    _, il, rcl = ctx.solve(b, 1e-10)
    ctx.close()
    log(f"min Re lambda {light} with setup stage two: setup {setup_l:.2f} s, solve {il['t_solve_s']:.2f} s")

    # roofline of the dominant kernel class of the timed steps (device time
    # from HIP events on the library's stream around every fine-stencil
    # launch; coarse launches inside captured CGNR chunks are sampled)
    agg = {}
    for inf in infos:
        for k, d in inf["kernels"].items():
            e = agg.setdefault(k, {"ms": 0.0, "launches": 0, "sites": 0.0})
            e["ms"] += d["ms"]
            e["launches"] += d["launches"]
            e["sites"] += d["sites"]
    fine = {k: e for k, e in agg.items() if k.startswith("dslash") and e["launches"]}
    dom = max(fine, key=lambda k: fine[k]["ms"])
    e = fine[dom]
    prec = dom.split("_")[-1]
    mrq = dom.startswith("dslash_mrq")
    avg_us = e["ms"] * 1e3 / e["launches"]
    rhs_per_launch = e["sites"] / e["launches"] / V
    wv, wl = WIDTH[prec]
    # algorithmic bytes per launch: each site's links (two rows) once, and
    # per right-hand side the input spinor once and the output spinor once;
    # the MR step by the q recursion also reads r_k and writes r_{k+1}
    spinors = 4 if mrq else 2
    bpl = V * (48 * wl + rhs_per_launch * 24 * spinors * wv)
    fpl = V * rhs_per_launch * (dslash_flops(True) + (192 if mrq else 0))
    achieved = bpl / avg_us / 1e3
    traffic = stored_traffic(TRAFFIC_KERNEL[dom], "C3")
    form = "MR step by the q recursion" if mrq else "plain / MR / residual form"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": f"fine Wilson stencil, {prec} class, {form}, {rhs_per_launch:.0f} right-hand sides "
                          "per launch",
                "avg_launch_us": round(avg_us, 2), "bytes_per_launch": round(bpl),
                "TFLOPs": round(fpl / avg_us / 1e6, 2),
                "device_ms_per_step": {k: round(v["ms"] / len(infos), 1) for k, v in agg.items() if v["launches"]}}

    solve_s = sum(i["t_solve_s"] for i in infos) / len(infos)
    n_d_step = 5 * (1 + 4) * nv[0] + infos[-1]["n_fine_dslash"]
    out = {
        "metric": "dslash HBM GB/s; MG time-to-solution to 1e-10 rel. residual vs plain FP64 MG",
        "value": round(nrhs * 1e3 / ms_step, 4),
        "unit": "right-hand sides/s (mg_setup + one batched mg_solve of the 12 point sources to 1e-10)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 outer / " + {"f16": "f16-stored operators and fine spinors, f32 arithmetic", "f32": "f32",
                                   "f64": "f64"}[a.precond] + " preconditioner",
        "data": "synthetic (seeded random SU(3) links, 12 spin-colour point sources at the origin)",
        "config": {"workload": f"three-level MG, 32^3x64, eps {cfg['eps']}, aggregates 4^4 then 2^4, Nv 24/24, "
                               f"12 point sources batched, nominal min Re lambda {target}",
                   "mass": mass, "precond": a.precond, "setup_relaxation": a.setup_prec},
        "host_ms_per_phase": phase_ms,
        "time_to_solution_s": round(solve_s, 4),
        "setup_s": round(setup64_s, 4),
        "iters": infos[-1]["iters"][:nrhs],
        "true_rel_resid_max": true_res,
        "plain_fp64_single_rhs": {"time_to_solution_s": round(t64, 3), "iters": it64,
                                  "speedup_of_batched": round(t64 / solve_s, 2)},
        "f16_batched_time_to_solution_s": round(i16["t_solve_s"], 4) if rc16 == 0 else None,
        "f32_precond_f16_transfers": {"time_to_solution_s": round(itp["t_solve_s"], 4) if rctp == 0 else None,
                                      "iters_max": max(itp["iters"][:nrhs])},
        "lightest_mass_setup_stage_two": {"min_re_lambda_nominal": light, "setup_s": round(setup_l, 3),
                                          "time_to_solution_s": round(il["t_solve_s"], 3),
                                          "iters_max": max(il["iters"][:nrhs]), "converged": rcl == 0},
        "fine_dslash_per_solve": infos[-1]["n_fine_dslash"],
        "cgnr_iters_per_solve": infos[-1]["n_cgnr_iters"],
        "roofline": roofline,
    }
    if not a.no_large:
        out["dslash_32^3x64"] = large_dslash(mgwd, torch)
    if not a.no_c1:
        out["c1_two_level"] = c1_report(mgwd, torch, W, a, steps=5, warmup=1, quiet=True)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = oracle_baseline(U_np, mass, n_d_step, nrhs)
    print(json.dumps(out), flush=True)


def c1_report(mgwd, torch, W, a, steps=None, warmup=None, quiet=False):
    """The two-level 16^3 x 32 workload (Nv 20, one Gaussian source,
    FP16-stored preconditioner): setup + solve per step, and plain FP64 MG
    on the same setup."""
    steps = a.steps if steps is None else steps
    warmup = a.warmup if warmup is None else warmup
    cfg = W.CONFIGS["C1"]
    L, nv, blocks = cfg["L"], cfg["nv"], cfg["blocks"]
    mass = W.mass_for("C1")
    U = torch.from_numpy(W.gauge_field(L, cfg["eps"], cfg["seed"])).cuda()
    b = torch.from_numpy(W.gaussian_spinor(L, cfg["seed"])).cuda()
    st = torch.from_numpy(W.setup_starts(L, nv[0], cfg["seed"])).cuda()

    def step(prec):
        ctx = mgwd.MG(U, mass, blocks, nv, [st])
        if prec != "f64":
            ctx.set_precond_prec(prec)
        x, info, rc = ctx.solve(b, 1e-10)
        ctx.close()
        if rc != 0:
            raise RuntimeError("mg_solve did not converge")
        return info

    for _ in range(warmup):
        step("f16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step("f16") for _ in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    i64 = step("f64")
    solve = sum(i["t_solve_s"] for i in infos) / len(infos)
    return {"workload": f"two-level MG, 16^3x32, eps {cfg['eps']}, min Re lambda {cfg['targets'][0]}, Nv {nv[0]}, "
                        f"1 Gaussian source, f16-stored preconditioner",
            "steps_per_s": round(1e3 / ms, 3), "ms_per_step": round(ms, 2), "time_to_solution_s": round(solve, 4),
            "fp64_plain_time_to_solution_s": round(i64["t_solve_s"], 4),
            "speedup_vs_plain_fp64": round(i64["t_solve_s"] / solve, 2), "iters": infos[-1]["iters"][0],
            "iters_fp64": i64["iters"][0]}


if __name__ == "__main__":
    main()
