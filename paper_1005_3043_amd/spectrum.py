"""Eigenvalues of the fine Wilson operator D(m) (Eq. 2) nearest to zero, by
implicitly restarted Arnoldi (ARPACK, through scipy) on D(m)^{-1}, each
application one mg_solve to a tight tolerance on the device.

The masses of the 24^3 x 48 and 32^3 x 64 workloads come from Arnoldi runs
on 16^3 x 32 proxy lattices of the same generator width (the CPU run on the
large lattices is out of reach); this measures where the leftmost
eigenvalues of the large lattices really are at those masses.  Since D(m) =
D(0) + m, one run gives Re lambda_min(D(0)) for every mass.  The result is
reported, not fed back: the workloads keep their proxy masses.

Usage: python -m paper_1005_3043_amd.spectrum --workload C3 --target 0.1
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import scipy.sparse.linalg as sla
import torch

from . import MG


def nearest_eigenvalues(U, mass, blocks, nv, starts, k=16, ncv=48, tol=1e-6, solve_tol=1e-10, **mg_kw):
    """The k eigenvalues of D(mass) nearest to zero: the largest-magnitude
    eigenvalues 1/lambda of D^{-1}, applied by the MG solver."""
    Lt, Lz, Ly, Lx = U.shape[1:5]
    shp = (Lt, Lz, Ly, Lx, 4, 3)
    n = int(np.prod(shp))
    t0 = time.perf_counter()
    ctx = MG(U, mass, blocks, nv, starts, **mg_kw)
    setup_s = time.perf_counter() - t0
    count, iters = [0], []

    def inv(v):
        b = torch.from_numpy(np.ascontiguousarray(v.reshape(shp))).cuda()
        x, info, rc = ctx.solve(b, solve_tol)
        if rc != 0:
            raise RuntimeError("mg_solve did not converge")
        count[0] += 1
        iters.append(info["iters"][0])
        if count[0] % 10 == 0:
            print(f"{count[0]} solves, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        return x.cpu().numpy().ravel()

    op = sla.LinearOperator((n, n), matvec=inv, dtype=np.complex128)
    rng = np.random.default_rng(7)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    mu = sla.eigs(op, k=k, which="LM", tol=tol, ncv=ncv, v0=v0, return_eigenvectors=False)
    ctx.close()
    lam = np.sort_complex(1.0 / mu)
    return lam, dict(solves=count[0], mean_outer_iterations=float(np.mean(iters)), setup_s=round(setup_s, 2),
                     seconds=round(time.perf_counter() - t0, 1))


def main():
    import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C3", choices=["C2", "C3"])
    ap.add_argument("--target", type=float, default=None, help="nominal min Re lambda of the mass used")
    ap.add_argument("--k", type=int, default=16)
    a = ap.parse_args()
    cfg = W.CONFIGS[a.workload]
    target = a.target if a.target is not None else cfg["targets"][0] if "targets" in cfg else None
    mass = W.mass_for(a.workload, target)
    L, nv, blocks = cfg["L"], cfg["nv"], cfg["blocks"]
    U = torch.from_numpy(W.gauge_field(L, cfg["eps"], cfg["seed"])).cuda()
    starts = [torch.from_numpy(W.setup_starts(L, nv[0], cfg["seed"])).cuda()]
    if len(blocks) > 1:
        Lc = tuple(L[mu] // blocks[0][mu] for mu in range(4))
        starts.append(torch.from_numpy(W.coarse_setup_starts(Lc, 2 * nv[0], nv[1], cfg["seed"])).cuda())
    lam, stats = nearest_eigenvalues(U, mass, blocks, nv, starts, k=a.k, precond_prec="f32", setup_prec="f32",
                                     refine_group=8, refine_iters=5)
    i = int(np.argmin(lam.real))
    proxy = W.MASS_PROXY.get(a.workload, a.workload)
    re0_proxy = W.load_masses()[proxy]["re_lambda_min_m0"]
    print(json.dumps({
        "workload": a.workload, "lattice": list(L), "mass": mass, "nominal_min_re_lambda": target,
        "eigenvalues_nearest_zero": [[round(float(z.real), 6), round(float(z.imag), 6)] for z in lam],
        "min_re_lambda": float(lam[i].real), "its_imag": float(abs(lam[i].imag)),
        "re_lambda_min_D0": float(lam[i].real) - mass, "re_lambda_min_D0_proxy": re0_proxy, "proxy": proxy,
        **stats}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
