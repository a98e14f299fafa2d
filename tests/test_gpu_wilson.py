"""GPU parity of wilson_apply (fine stencil, Eq. 2) against the oracle."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import cref, wilson as wi

pytestmark = pytest.mark.gpu


def _run(L, eps, m, prec, nrhs=1, anti=True, seed=0):
    import paper_1005_3043_amd as mgwd
    U = W.gauge_field(L, eps, seed)
    psi = W.gaussian_spinor(L, seed + 1, batch=(nrhs,))
    dU = torch.from_numpy(U).cuda()
    dpsi = torch.from_numpy(psi).cuda()
    out = mgwd.wilson_apply(dU, dpsi, m, prec=prec, t_antiperiodic=anti)
    torch.cuda.synchronize()
    return U, psi, out.cpu().numpy()


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (8, 8, 8, 8), (6, 4, 2, 10), (2, 2, 2, 2), (3, 5, 7, 2), (12, 4, 8, 6)])
def test_wilson_f64_parity(cuda, L):
    U, psi, got = _run(L, 0.3, -0.25, "f64", nrhs=2)
    ref = wi.apply_D(U, psi, -0.25)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"wilson f64 L={L} rel err {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("L,nrhs", [((8, 8, 8, 8), 5), ((6, 4, 2, 10), 3), ((4, 4, 4, 4), 12)])
def test_wilson_multi_rhs_parity(cuda, L, nrhs):
    """Several right-hand sides in one launch (groups of four per workgroup,
    a ragged last group) against the oracle, every right-hand side."""
    U, psi, got = _run(L, 0.3, -0.25, "f64", nrhs=nrhs)
    ref = wi.apply_D(U, psi, -0.25)
    for k in range(nrhs):
        err = np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k])
        assert err < 1e-12, (k, err)


def test_wilson_periodic_time(cuda):
    U, psi, got = _run((4, 4, 4, 8), 0.3, 0.1, "f64", anti=False)
    ref = wi.apply_D(U, psi, 0.1, antiperiodic_t=False)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


def test_wilson_f32_error(cuda):
    U, psi, got = _run((8, 8, 8, 8), 0.3, -0.25, "f32")
    ref = wi.apply_D(U, psi, -0.25)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"wilson f32 rel err vs FP64 oracle {err:.3e}")
    assert err < 1e-6


def test_wilson_full_size_sampled(cuda):
    """16^3 x 32 (the two-level benchmark lattice): full output against the C
    oracle matvec (itself pinned to the numpy oracle)."""
    L = (16, 16, 16, 32)
    U, psi, got = _run(L, 0.3, -0.4, "f64")
    ref = cref.apply_D(U, psi[0], -0.4)
    err = np.linalg.norm(got[0] - ref) / np.linalg.norm(ref)
    print(f"wilson f64 16^3x32 rel err {err:.3e}")
    assert err < 1e-12


def test_wilson_full_size_multi_rhs_sampled(cuda):
    """32^3 x 64 (the three-level workload lattice), five right-hand sides in
    one launch (a group of four and a ragged one): every right-hand side
    against the oracle's per-site evaluation on 2048 sampled sites."""
    L = (32, 32, 32, 64)
    U, psi, got = _run(L, 0.35, -1.05, "f64", nrhs=5)
    rng = np.random.default_rng(11)
    sites = np.stack([rng.integers(0, L[mu], 2048) for mu in range(4)], 1)
    sites[:8] = [(0, 0, 0, 0), (31, 31, 31, 63), (0, 31, 0, 63), (31, 0, 31, 0), (5, 0, 9, 63),
                 (0, 7, 31, 32), (31, 31, 0, 1), (16, 16, 16, 62)]
    ref = wi.apply_D_sites(U, psi, -1.05, sites)
    g = got[:, sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]
    for k in range(5):
        err = np.linalg.norm(g[k] - ref[k]) / np.linalg.norm(ref[k])
        print(f"wilson f64 32^3x64 rhs {k} sampled rel err {err:.3e}")
        assert err < 1e-12
