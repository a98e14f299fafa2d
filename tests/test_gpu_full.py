"""Parity at the workloads' full sizes, in the configurations bench.py runs.

16^3x32 (the two-level workload, FP16-stored preconditioner): the solution's
true residual is recomputed by the oracle's operator; the exported
prolongator and Galerkin operator are checked by the oracle's own transfer,
Wilson and coarse-stencil arithmetic on sampled vectors (D_c v = P^dag D P v,
P^dag P = I per block).  24^3x48 with the twelve point sources in one batched
solve, and the three-level 32^3x64 solve with twelve point sources: every
right-hand side's true residual by the oracle's operator.  On 32^3x64 also
the FP32 null-vector relaxation, whose stencils are the smoother's in the
benchmark's launch configuration (twelve right-hand sides per launch), on
sampled vectors element by element against the oracle's relaxation."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import coarse as co
from oracle import cref
from oracle import solvers as so
from oracle import transfer as tr

pytestmark = pytest.mark.gpu


def _true_res(U_np, x, b, mass):
    x = x.cpu().numpy()
    b = b.cpu().numpy()
    return [float(np.linalg.norm(b[i] - cref.apply_D(U_np, x[i], mass)) / np.linalg.norm(b[i]))
            for i in range(x.shape[0])]


@pytest.fixture(scope="module")
def c1(cuda):
    import paper_1005_3043_amd as mgwd
    cfg = W.CONFIGS["C1"]
    L = cfg["L"]
    U_np = W.gauge_field(L, cfg["eps"], cfg["seed"])
    mass = W.mass_for("C1")
    st = torch.from_numpy(W.setup_starts(L, cfg["nv"][0], cfg["seed"])).cuda()
    ctx = mgwd.MG(torch.from_numpy(U_np).cuda(), mass, cfg["blocks"], cfg["nv"], [st])
    return cfg, U_np, mass, ctx


def test_c1_solve_fp16_preconditioner(c1):
    cfg, U_np, mass, ctx = c1
    b = torch.from_numpy(W.gaussian_spinor(cfg["L"], cfg["seed"])[None]).cuda()
    ctx.set_precond_prec("f16")
    ctx.set_timing(True)
    try:
        x, info, rc = ctx.solve(b, 1e-10)
    finally:
        ctx.set_timing(False)
        ctx.set_precond_prec("f64")
    res = _true_res(U_np, x, b, mass)
    print(f"16^3x32: FP16-preconditioned solve, {info['iters'][0]} iterations, true rel resid {res[0]:.2e}")
    assert rc == 0 and res[0] <= 1e-10 * 1.001


def test_c1_galerkin_and_P_sampled(c1):
    """The exported operators of the full-size setup, checked by oracle
    arithmetic: P^dag P = I on every block, and D_c v = P^dag (D (P v)) for a
    random coarse vector (oracle prolong, C Wilson operator, oracle restrict,
    oracle coarse stencil on the exported X, Y)."""
    cfg, U_np, mass, ctx = c1
    L, blk = cfg["L"], cfg["blocks"][0]
    geom = tr.BlockGeometry(L, blk)
    P = ctx.export_P(0)
    G = np.einsum("cxri,cxrj->cxij", np.conj(P), P)
    eye_err = float(np.max(np.abs(G - np.eye(P.shape[-1]))))
    X, Y = ctx.export_coarse_op(1)
    rng = np.random.default_rng(21)
    Lc = geom.Lc
    v = rng.standard_normal((Lc[3], Lc[2], Lc[1], Lc[0], 2 * P.shape[-1])) + \
        1j * rng.standard_normal((Lc[3], Lc[2], Lc[1], Lc[0], 2 * P.shape[-1]))
    f = tr.generic_to_fine(tr.prolong(P, geom, v))
    Df = tr.fine_to_generic(cref.apply_D(U_np, f, mass))
    lhs = tr.restrict(P, geom, Df)
    rhs = co.coarse_apply(X, Y, v)
    e = float(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs))
    print(f"16^3x32: max |P^dag P - I| {eye_err:.1e}, D_c v vs P^dag D P v rel err {e:.1e}")
    assert eye_err < 1e-12 and e < 1e-12


def test_c2_twelve_point_sources_batched(cuda):
    import paper_1005_3043_amd as mgwd
    cfg = W.CONFIGS["C2"]
    L = cfg["L"]
    U_np = W.gauge_field(L, cfg["eps"], cfg["seed"])
    mass = W.mass_for("C2")
    st = torch.from_numpy(W.setup_starts(L, cfg["nv"][0], cfg["seed"])).cuda()
    ctx = mgwd.MG(torch.from_numpy(U_np).cuda(), mass, cfg["blocks"], cfg["nv"], [st], max_rhs=12,
                  precond_prec="f16")
    b = torch.from_numpy(W.point_sources(L)).cuda()
    x, info, rc = ctx.solve(b, 1e-10)
    var, us = ctx.coarse_variant(1, "f16", 12)
    ctx.close()
    res = _true_res(U_np, x, b, mass)
    print(f"24^3x48, 12 point sources: iterations {info['iters'][:12]}, max true rel resid {max(res):.2e}, "
          f"coarse variant {var} ({us:.0f} us)")
    assert rc == 0 and max(res) <= 1e-10 * 1.001


@pytest.fixture(scope="module")
def c3(cuda):
    """The 32^3x64 links and the 24 level-0 setup starts (host arrays)."""
    cfg = W.CONFIGS["C3"]
    L = cfg["L"]
    print("generating the 32^3x64 links and setup starts", flush=True)
    return cfg, W.gauge_field(L, cfg["eps"], cfg["seed"]), W.setup_starts(L, cfg["nv"][0], cfg["seed"])


@pytest.mark.timeout(300)
def test_c3_fp32_relaxation_sampled(c3):
    """Setup stage one in FP32 on 32^3x64 with the workload's 24 null vectors,
    which the library relaxes in two batches of twelve: the FP32 stencil with
    twelve right-hand sides per launch in its plain, MR and q-recursion
    forms, the MR combine pass and the normalisation, all in the launch
    configuration of the benchmark's smoothing (the lattice-chunked order of
    the right-hand-side groups included, which small lattices do not reach).
    One round of four MR steps; vectors 0 and 23 (first of the first batch,
    last of the second) against the oracle's FP64 relaxation of the same
    starts with the oracle's C operator, element by element.  Bound as on
    the small lattices: a handful of FP32 operations per entry and step
    after a 9-term stencil sum, about 50 u per step with u = 2^-24, so
    4 x 50 x 6e-8 = 1.2e-5 < 1e-4; the lower bound shows FP32 arithmetic
    ran."""
    import paper_1005_3043_amd as mgwd
    cfg, U_np, starts = c3
    mass = W.mass_for("C3", 0.1)
    ctx = mgwd.MG(torch.from_numpy(U_np).cuda(), mass, [cfg["blocks"][0]], [cfg["nv"][0]],
                  [torch.from_numpy(starts).cuda()], setup_rounds=1, setup_mr_steps=4, setup_prec="f32",
                  max_rhs=12)
    Vg = ctx.export_nullvecs(0)
    ctx.close()
    A = lambda v: cref.apply_D(U_np, v, mass)  # noqa: E731
    for k in (0, cfg["nv"][0] - 1):
        Vo = so.relax_nullspace(A, starts[[k]], 1, 4)[0]
        err = float(np.linalg.norm(Vg[k] - Vo) / np.linalg.norm(Vo))
        print(f"32^3x64 FP32 relaxation, vector {k}: rel err {err:.2e}", flush=True)
        assert 1e-9 < err < 1e-4


def test_c3_three_level_point_sources(c3):
    import paper_1005_3043_amd as mgwd
    cfg, U_np, starts = c3
    L, blocks, nv = cfg["L"], cfg["blocks"], cfg["nv"]
    mass = W.mass_for("C3", 0.01)
    st = torch.from_numpy(starts).cuda()
    Lc = tuple(L[mu] // blocks[0][mu] for mu in range(4))
    st1 = torch.from_numpy(W.coarse_setup_starts(Lc, 2 * nv[0], nv[1], cfg["seed"])).cuda()
    ctx = mgwd.MG(torch.from_numpy(U_np).cuda(), mass, blocks, nv, [st, st1], max_rhs=12, precond_prec="f32")
    b = torch.from_numpy(W.point_sources(L)).cuda()
    x, info, rc = ctx.solve(b, 1e-10)
    ctx.close()
    res = _true_res(U_np, x, b, mass)
    print(f"32^3x64 three-level, 12 point sources: iterations {info['iters'][:12]}, "
          f"max true rel resid {max(res):.2e}")
    assert rc == 0 and max(res) <= 1e-10 * 1.001
