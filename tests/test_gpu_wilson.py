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
