"""Parity of the kernel paths the full-size workloads take, isolated on the
operators the GPU setup exported (so the only difference to the oracle is
the kernel's arithmetic): the matrix-core transfers with two row tiles (Nv =
20 and 24) for 12 and 16 right-hand sides, every coarse-stencil variant at
the coarse operator widths n = 40 and 48 for 1 and 12 right-hand sides, and
the coarsest-level CGNR of the cycle at n = 40 (one right-hand side, whole-
solve launch and chunks) and n = 48 (twelve right-hand sides) on 512 coarse
sites, against the oracle's CGNR on the same stored operator.

Stored-precision kernels are compared with the oracle applied, in FP64, to
the operator and inputs rounded to the storage formats the library uses
(round to nearest even, as numpy's conversions do), so the bound is that of
FP32 accumulation: a sum of K products carries a relative error of at most
about K u with u = 2^-24, and about sqrt(K) u for random signs; the tests
take 2e-5, above sqrt(9 * 48 * 16) u = 5e-6 and below the FP16 storage
error they would otherwise show (1e-4 and more)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import coarse as co
from oracle import solvers as so
from oracle import transfer as tr

pytestmark = pytest.mark.gpu

FP32_ACC = 2e-5


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def _stored(a, prec):
    """Entries rounded to the storage format of the precision class."""
    if prec == "f64":
        return a
    if prec == "f32":
        return a.astype(np.complex64).astype(np.complex128)
    return a.real.astype(np.float16).astype(np.float64) + 1j * a.imag.astype(np.float16).astype(np.float64)


def _vec_in(a, prec):
    """Input vectors as the kernels see them (FP32 for the FP32 and FP16 classes)."""
    return a if prec == "f64" else a.astype(np.complex64).astype(np.complex128)


_CTX = {}


def _ctx(L, nv, seed=0, mass=-0.3, max_rhs=16):
    import paper_1005_3043_amd as mgwd
    key = (L, nv, seed)
    if key not in _CTX:
        U = W.gauge_field(L, 0.3, seed)
        st = torch.from_numpy(W.setup_starts(L, nv, seed)).cuda()
        _CTX[key] = mgwd.MG(torch.from_numpy(U).cuda(), mass, [(4, 4, 4, 4)], [nv], [st], setup_rounds=2,
                            max_rhs=max_rhs)
    return _CTX[key]


@pytest.fixture(scope="module", autouse=True)
def _close_contexts():
    yield
    for c in _CTX.values():
        c.close()
    _CTX.clear()


@pytest.mark.parametrize("nv", [20, 24])
@pytest.mark.parametrize("nrhs", [12, 16])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_fine_transfers_two_row_tiles(cuda, nv, nrhs, prec):
    """Restriction P^dag r and prolongation P e_c on 8^3 x 16 (32 aggregates)
    with the exported P: FP64 to 1e-12; FP32 / FP16-stored P with the vector
    kernels and with the matrix-core GEMM (Nv > 16: two row tiles of 16) to
    the FP32 accumulation bound."""
    L = (8, 8, 8, 16)
    ctx = _ctx(L, nv)
    geom = tr.BlockGeometry(L, (4, 4, 4, 4))
    P = _stored(ctx.export_P(0), prec)
    r = _vec_in(W.gaussian_spinor(L, 31, batch=(nrhs,)), prec)
    rng = np.random.default_rng(32)
    Lc = geom.Lc
    ec = _vec_in(rng.standard_normal((nrhs, Lc[3], Lc[2], Lc[1], Lc[0], 2 * nv))
                 + 1j * rng.standard_normal((nrhs, Lc[3], Lc[2], Lc[1], Lc[0], 2 * nv)), prec)
    ref_r = tr.restrict(P, geom, tr.fine_to_generic(r))
    ref_p = tr.generic_to_fine(tr.prolong(P, geom, ec))
    variants = (0,) if prec == "f64" else (0, 1)
    try:
        for var in variants:
            ctx.set_transfer_variant(var)
            got_r = ctx.transfer(0, torch.from_numpy(r).cuda(), 0, prec).cpu().numpy()
            got_p = ctx.transfer(0, torch.from_numpy(ec).cuda(), 1, prec).cpu().numpy()
            er = max(_rel(got_r[i], ref_r[i]) for i in range(nrhs))
            ep = max(_rel(got_p[i], ref_p[i]) for i in range(nrhs))
            print(f"Nv {nv}, {nrhs} RHS, {prec}, variant {var}: restrict {er:.2e}, prolong {ep:.2e}")
            tol = 1e-12 if prec == "f64" else FP32_ACC
            assert er < tol and ep < tol
    finally:
        ctx.set_transfer_variant(-1)


@pytest.mark.parametrize("nv", [20, 24])
@pytest.mark.parametrize("nrhs", [1, 12])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_coarse_variants_full_width(cuda, nv, nrhs, prec):
    """D_c at n = 2 Nv = 40 and 48 on a 4^4 coarse lattice (16^4 fine), every
    kernel variant (per-RHS FMA; matrix-core GEMM with K split 1/2/4 on the
    stencil or on its row-major copy; three M tiles at n = 48), against the
    oracle stencil on the exported, storage-rounded operator."""
    L = (16, 16, 16, 16)
    ctx = _ctx(L, nv, seed=1)
    X, Y = ctx.export_coarse_op(1)
    Xs, Ys = _stored(X, prec), _stored(Y, prec)
    rng = np.random.default_rng(40 + nrhs)
    shp = (nrhs,) + X.shape[:-1]
    v = _vec_in(rng.standard_normal(shp) + 1j * rng.standard_normal(shp), prec)
    ref = np.stack([co.coarse_apply(Xs, Ys, v[i]) for i in range(nrhs)])
    variants = (0,) if prec == "f64" else (0, 1, 2, 4, 9, 10, 12)
    try:
        for var in variants:
            ctx.set_coarse_variant(var)
            got = ctx.apply_op(1, torch.from_numpy(v).cuda(), prec).cpu().numpy()
            e = max(_rel(got[i], ref[i]) for i in range(nrhs))
            print(f"n {2 * nv}, {nrhs} RHS, {prec}, variant {var}: rel err {e:.2e}")
            assert e < (1e-12 if prec == "f64" else FP32_ACC)
    finally:
        ctx.set_coarse_variant(-1)


def _oracle_cgnr(X, Y, b, tol=1e-3, maxiter=1000):
    A = lambda u: co.coarse_apply(X, Y, u)  # noqa: E731
    Ad = lambda u: co.sigma3(co.coarse_apply(X, Y, co.sigma3(u)))  # noqa: E731
    return so.cgnr(A, Ad, b, tol, maxiter)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_coarsest_cgnr_n40_one_rhs(cuda, prec):
    """The cycle's coarsest solve at n = 40 on 4^3 x 8 coarse sites (the
    16^3 x 32 workload's coarse grid): the whole-solve launch and the chunks
    give the same iterate bit for bit with the same iteration count, and both
    match the oracle's CGNR on the stored operator (D_c^dag = sigma_3 D_c
    sigma_3) within one iteration and the FP32 bound on the iterate; a zero
    right-hand side takes no iteration on either path."""
    L = (16, 16, 16, 32)
    ctx = _ctx(L, 20, seed=2, mass=-0.8)
    X, Y = ctx.export_coarse_op(1)
    Xs, Ys = _stored(X, prec), _stored(Y, prec)
    rng = np.random.default_rng(50)
    b = rng.standard_normal((1,) + X.shape[:-1]) + 1j * rng.standard_normal((1,) + X.shape[:-1])
    db = torch.from_numpy(b).cuda()
    out = {}
    for on in (True, False):
        ctx.set_cgnr_persistent(on)
        x, it = ctx.coarse_solve(db, prec)
        out[on] = (x.cpu().numpy(), it[0])
    ctx.set_cgnr_persistent(True)
    ref, it_ref = _oracle_cgnr(Xs, Ys, _vec_in(b[0], prec))
    e = _rel(out[True][0][0], ref)
    print(f"n 40, {prec}: CGNR iterations whole {out[True][1]}, chunks {out[False][1]}, oracle {it_ref}; "
          f"iterate rel err {e:.2e}")
    assert out[True][1] == out[False][1]
    assert np.array_equal(out[True][0], out[False][0])
    assert abs(out[True][1] - it_ref) <= 1
    if prec == "f64":
        assert out[True][1] == it_ref and e < 1e-10
    else:
        # the recursion of 50-odd FP32 iterations against the FP64 one on the
        # same operator: a relative difference of order (iterations) u kappa
        # with kappa^2 of D_c^dag D_c in the thousands
        assert e < 1e-3
    z = torch.zeros_like(db)
    for on in (True, False):
        ctx.set_cgnr_persistent(on)
        x0, it0 = ctx.coarse_solve(z, prec)
        assert it0 == [0] and not x0.abs().max().item()
    ctx.set_cgnr_persistent(True)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_coarsest_cgnr_n48_twelve_rhs(cuda, prec):
    """Twelve right-hand sides of the coarsest solve at n = 48 on 4^3 x 8
    coarse sites (the shape of the three-level workload's coarsest grid),
    one of them zero: per right-hand side the iteration count within one of
    the oracle's CGNR on the stored operator and the iterate within the same
    bound as one right-hand side; the zero one takes no iteration."""
    L = (16, 16, 16, 32)
    ctx = _ctx(L, 24, seed=3, mass=-0.8)
    X, Y = ctx.export_coarse_op(1)
    Xs, Ys = _stored(X, prec), _stored(Y, prec)
    rng = np.random.default_rng(60)
    b = rng.standard_normal((12,) + X.shape[:-1]) + 1j * rng.standard_normal((12,) + X.shape[:-1])
    b[5] = 0.0
    x, its = ctx.coarse_solve(torch.from_numpy(b).cuda(), prec)
    x = x.cpu().numpy()
    assert its[5] == 0 and not np.abs(x[5]).max()
    for i in range(12):
        if i == 5:
            continue
        ref, it_ref = _oracle_cgnr(Xs, Ys, _vec_in(b[i], prec))
        e = _rel(x[i], ref)
        print(f"n 48, {prec}, rhs {i}: CGNR iterations {its[i]} (oracle {it_ref}), iterate rel err {e:.2e}")
        assert abs(its[i] - it_ref) <= 1 and e < 1e-3
