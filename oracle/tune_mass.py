"""Arnoldi estimate of min Re lambda(D(m=0)) for the synthetic workloads.

TEST INFRASTRUCTURE ONLY: writes the stored masses used by every workload.

D(m) = D(0) + m 1 (Eq. 2), so every eigenvalue shifts by m and one Arnoldi
run per gauge field fixes the mass for any target min Re lambda:
m = target - Re lambda_min(D(0)).  k = 12 wanted eigenvalues cover the
lowest free-field cluster (momentum (0, 0, 0, +-pi/Lt), 6-fold each), which
converges far faster than asking for fewer or more; tol = 1e-5 relative gives
Re lambda to ~1e-5, well inside the mass targets (>= 1e-3).  gamma_5-Hermiticity makes the spectrum
closed under complex conjugation, so Re lambda_min is well defined.

Usage:  python -m oracle.tune_mass C0 C1 ...
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as sla

import workloads
from . import cref


def re_lambda_min(U, tol=1e-5, k=12, ncv=64, maxiter=100000):
    shp = (U.shape[1], U.shape[2], U.shape[3], U.shape[4], 4, 3)
    n = int(np.prod(shp))
    count = [0]

    def mv(v):
        count[0] += 1
        return cref.apply_D(U, v.reshape(shp), 0.0).ravel()

    op = sla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    v0 = workloads.gaussian_spinor(tuple(reversed(shp[:4])), 99).ravel()
    vals = sla.eigs(op, k=k, which="SR", tol=tol, ncv=ncv, v0=v0, maxiter=maxiter,
                    return_eigenvectors=False)
    return vals, count[0]


def main(names):
    path = os.path.join(os.path.dirname(workloads.__file__), "masses.json")
    rec = workloads.load_masses()
    for name in names:
        cfg = workloads.CONFIGS[name]
        t0 = time.time()
        U = workloads.gauge_field(cfg["L"], cfg["eps"], cfg["seed"])
        vals, nmv = re_lambda_min(U)
        lam = vals[np.argmin(vals.real)]
        rec[name] = dict(L=list(cfg["L"]), eps=cfg["eps"], seed=cfg["seed"],
                         re_lambda_min_m0=float(lam.real), im_lambda_min_m0=float(abs(lam.imag)),
                         arnoldi=dict(k=12, ncv=64, which="SR", tol=1e-5, matvecs=nmv),
                         seconds=round(time.time() - t0, 1))
        print(name, rec[name], flush=True)
        with open(path, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
