"""wilson_apply_noalloc (the entry point that allocates nothing) against
wilson_apply (same kernels: bit-identical output) and the oracle (Eq. 2,
1e-12 in FP64), on two calls in a row with the second input smaller than
the first, in FP64 and FP32; an input above the fixed scratch is refused on
the host before any work is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle import wilson as wi

pytestmark = pytest.mark.gpu


def test_noalloc_matches_allocating_entry_point(cuda):
    import paper_1005_3043_amd as mgwd
    for L, nrhs, m in (((8, 8, 8, 16), 3, -0.3), ((4, 6, 2, 8), 1, 0.1)):
        U = W.gauge_field(L, 0.3, 7)
        psi = W.gaussian_spinor(L, 8, batch=(nrhs,))
        dU, dpsi = torch.from_numpy(U).cuda(), torch.from_numpy(psi).cuda()
        for prec in ("f64", "f32"):
            ref_gpu = mgwd.wilson_apply(dU, dpsi, m, prec=prec)
            out = torch.full_like(dpsi, float("nan"))
            got = mgwd.wilson_apply_noalloc(dU, dpsi, m, out, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(got, ref_gpu), (L, nrhs, prec)
            if prec == "f64":
                ref = wi.apply_D(U, psi, m)
                err = np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref)
                print(f"noalloc L={L} nrhs={nrhs}: rel err vs oracle {err:.2e}")
                assert err < 1e-12


def test_noalloc_refuses_oversized_input(cuda):
    import paper_1005_3043_amd as mgwd
    lib = mgwd.lib()
    lat = mgwd.lattice((32, 32, 32, 64))
    dummy = torch.zeros(16, dtype=torch.complex128, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    q = ctypes.c_void_p(dummy.data_ptr() + 128)
    rc = lib.wilson_apply_noalloc(ctypes.byref(lat), p, 0.0, p, q, 1, 0, None)
    assert rc == -4  # MG_ENOMEM
    assert b"above" in lib.mg_last_error()
