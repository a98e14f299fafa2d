"""Pins of the oracle's multigrid pieces against definitions, invariants and
brute force: aggregate maps, block QR (Eq. 4), R = P^dag with the chirality
split (P^dag gamma_5 = sigma_3 P^dag), the Galerkin stencil against dense
P^dag D P, sigma_3-Hermiticity, gauge invariance, the mass shift, the
two-grid Galerkin orthogonality (Eq. 3), square-P exactness, MR/CGNR/FGCR
against their defining properties and dense LU."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import coarse as co
from oracle import solvers as so
from oracle import transfer as tr
from oracle import wilson as wi


def _setup(L, b, nv, m=-0.2, eps=0.3, seed=0, rounds=2):
    U = W.gauge_field(L, eps, seed)
    p = so.MGParams(blocks=[b], nv=[nv], setup_rounds=rounds)
    h = so.mg_setup(U, m, p, W.setup_starts(L, nv, seed))
    return U, h


# ---------------------------------------------------------------- maps (a4)
@pytest.mark.parametrize("L,b", [((4, 4, 4, 4), (2, 2, 2, 2)), ((6, 4, 2, 8), (3, 2, 1, 4)), ((4, 4, 4, 4), (4, 4, 4, 4))])
def test_maps_brute_force(L, b):
    g = tr.BlockGeometry(L, b)
    f2c, f2l, nbr, face = g.maps()
    Lc = g.Lc
    for i, (t, z, y, x) in enumerate(itertools.product(range(L[3]), range(L[2]), range(L[1]), range(L[0]))):
        X = [x, y, z, t]
        assert i == X[0] + L[0] * (X[1] + L[1] * (X[2] + L[2] * X[3]))
        cc = [X[mu] // b[mu] for mu in range(4)]
        o = [X[mu] % b[mu] for mu in range(4)]
        assert f2c[i] == cc[0] + Lc[0] * (cc[1] + Lc[1] * (cc[2] + Lc[2] * cc[3]))
        assert f2l[i] == o[0] + b[0] * (o[1] + b[1] * (o[2] + b[2] * o[3]))
        for mu in range(4):
            assert bool(face[i] >> (2 * mu) & 1) == (o[mu] == b[mu] - 1)
            assert bool(face[i] >> (2 * mu + 1) & 1) == (o[mu] == 0)
    for ic in range(g.Vc):
        cc = [ic % Lc[0], ic // Lc[0] % Lc[1], ic // (Lc[0] * Lc[1]) % Lc[2], ic // (Lc[0] * Lc[1] * Lc[2])]
        for mu in range(4):
            for d, st in ((0, 1), (1, -1)):
                n = list(cc)
                n[mu] = (n[mu] + st) % Lc[mu]
                assert nbr[ic, 2 * mu + d] == n[0] + Lc[0] * (n[1] + Lc[1] * (n[2] + Lc[2] * n[3]))


def test_blockify_roundtrip_and_rows():
    L, b = (4, 6, 2, 4), (2, 3, 1, 2)
    g = tr.BlockGeometry(L, b)
    f = W.gaussian_spinor(L, 3)
    F = tr.fine_to_generic(f)
    B = g.blockify(F)
    assert np.array_equal(g.unblockify(B), F)
    f2c, f2l, _, _ = g.maps()
    flat = F.reshape(-1, 12)
    for i in range(g.V):
        for comp in range(12):
            chi, j = divmod(comp, 6)
            assert B[f2c[i], chi, f2l[i] * 6 + j] == flat[i, comp]


# ---------------------------------------------------------------- block QR (a6)
def test_block_qr_matches_library_qr():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((5, 2, 30, 7)) + 1j * rng.standard_normal((5, 2, 30, 7))
    Q, R = tr.block_qr(A)
    for c in range(5):
        for x in range(2):
            q, r = np.linalg.qr(A[c, x])
            ph = np.diag(r) / np.abs(np.diag(r))          # make diag(R) positive real
            q = q * ph[None, :]
            r = np.conj(ph)[:, None] * r
            assert np.abs(Q[c, x] - q).max() < 1e-13
            assert np.abs(R[c, x] - r).max() < 1e-12
            assert np.allclose(np.triu(R[c, x]), R[c, x])
            assert np.all(np.diag(R[c, x]).real > 0) and np.all(np.diag(R[c, x]).imag == 0)


def test_block_qr_rank_deficient():
    A = np.ones((1, 2, 6, 3), dtype=np.complex128)
    with pytest.raises(ValueError):
        tr.block_qr(A)


# ---------------------------------------------------------------- P, R (a7, a8)
def test_prolongator_invariants():
    L, b, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    U, h = _setup(L, b, nv)
    lv = h.levels[0]
    g = lv.geom
    P = tr.P_dense(lv.Pb, g)
    assert np.abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-14          # Eq. 4
    Vn = tr.fine_to_generic(lv.nullvecs).reshape(nv, -1).T                     # P V_c = V
    Vc = np.zeros((P.shape[1], nv), dtype=np.complex128)
    for c in range(g.Vc):
        for x in range(2):
            Vc[(c * 2 + x) * nv:(c * 2 + x + 1) * nv, :] = lv.Rc[c, x]
    assert np.abs(P @ Vc - Vn).max() < 1e-13
    g5 = np.kron(np.eye(g.V), np.kron(wi.GAMMA5, np.eye(3)))
    s3 = np.kron(np.eye(g.Vc), np.diag([1.0] * nv + [-1.0] * nv))
    assert np.abs(P.conj().T @ g5 - s3 @ P.conj().T).max() < 1e-15            # chirality kept
    r = W.gaussian_spinor(L, 5)
    rc = h.restrict(0, r)
    assert np.abs(rc.ravel() - P.conj().T @ r.ravel()).max() < 1e-13          # R = P^dag
    e = h.prolong(0, rc)
    assert np.abs(e.ravel() - P @ rc.ravel()).max() < 1e-13
    assert np.abs(h.restrict(0, e) - rc).max() < 1e-13                         # P^dag P = I


# ---------------------------------------------------------------- Galerkin (a9, a10)
@pytest.mark.parametrize("L,b,nv", [((4, 4, 4, 4), (2, 2, 2, 2), 4), ((2, 2, 2, 4), (1, 1, 1, 2), 3),
                                    ((4, 2, 4, 4), (4, 2, 2, 4), 5)])
def test_galerkin_equals_dense(L, b, nv):
    U, h = _setup(L, b, nv, m=-0.3, rounds=1)
    lv = h.levels[0]
    P = tr.P_dense(lv.Pb, lv.geom)
    D = wi.D_dense(U, -0.3)
    Dc = co.coarse_dense(lv.X, lv.Y)
    ref = P.conj().T @ D @ P
    assert np.abs(Dc - ref).max() < 1e-13 * np.abs(ref).max()
    # sigma_3 Hermiticity of the assembled operator, and blockwise per face pair
    s3 = np.kron(np.eye(lv.geom.Vc), np.diag([1.0] * nv + [-1.0] * nv))
    assert np.abs(Dc.conj().T - s3 @ Dc @ s3).max() < 1e-13
    sig = np.diag([1.0] * nv + [-1.0] * nv)
    for mu in range(4):
        Yp, Ym = lv.Y[2 * mu], lv.Y[2 * mu + 1]
        Ymsh = np.roll(Ym, -1, axis=co.SITE_AXIS[mu] - 1)    # Y_-mu(x_c + mu)
        assert np.abs(Ymsh - sig @ np.conj(np.swapaxes(Yp, -1, -2)) @ sig).max() < 1e-13


def test_coarse_dagger_is_adjoint():
    U, h = _setup((4, 4, 4, 4), (2, 2, 2, 2), 3, rounds=1)
    lv = h.levels[0]
    Dc = co.coarse_dense(lv.X, lv.Y)
    v = np.random.default_rng(2).standard_normal(Dc.shape[0]) + 0j
    got = co.coarse_apply_dag(lv.X, lv.Y, v.reshape(lv.X.shape[:-1])).ravel()
    assert np.abs(got - Dc.conj().T @ v).max() < 1e-13
    got2 = co.sigma3(co.coarse_apply(lv.X, lv.Y, co.sigma3(v.reshape(lv.X.shape[:-1])))).ravel()
    assert np.abs(got2 - Dc.conj().T @ v).max() < 1e-13


def test_coarse_gauge_invariance():
    """D_c(U^g, g V) = D_c(U, V): g is block-diagonal unitary, P -> g P."""
    L, b, nv = (4, 4, 4, 4), (2, 2, 2, 2), 3
    U = W.gauge_field(L, 0.3, 1)
    V = W.setup_starts(L, nv, 1)
    g = W.gauge_transform(L, 2)
    geom = tr.BlockGeometry(L, b)

    def build(Uu, Vv):
        Pb, _ = tr.block_qr(np.moveaxis(geom.blockify(tr.fine_to_generic(Vv)), 0, -1))
        return co.galerkin_fine(Uu, -0.2, Pb, geom)
    X1, Y1 = build(U, V)
    X2, Y2 = build(wi.gauge_transform_links(U, g), wi.gauge_transform_spinor(g, V))
    assert np.abs(X1 - X2).max() < 1e-13 and np.abs(Y1 - Y2).max() < 1e-13


def test_mass_shift():
    """X(m + d) - X(m) = d I and Y unchanged (P^dag P = I)."""
    L, b, nv = (4, 4, 4, 4), (2, 2, 2, 2), 3
    U, h = _setup(L, b, nv, rounds=1)
    lv = h.levels[0]
    X2, Y2 = co.galerkin_fine(U, -0.2 + 0.37, lv.Pb, lv.geom)
    assert np.abs(X2 - lv.X - 0.37 * np.eye(2 * nv)).max() < 1e-13
    assert np.abs(Y2 - lv.Y).max() < 1e-14


# ---------------------------------------------------------------- two-grid (Eq. 3)
def test_galerkin_orthogonality_exact_coarse_solve():
    """With an exact coarse solve, P^dag (r - D P D_c^{-1} P^dag r) = 0."""
    L, b, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    U, h = _setup(L, b, nv, rounds=1)
    lv = h.levels[0]
    P = tr.P_dense(lv.Pb, lv.geom)
    D = wi.D_dense(U, -0.2)
    Dc = co.coarse_dense(lv.X, lv.Y)
    r = W.gaussian_spinor(L, 7).ravel()
    e = P @ np.linalg.solve(Dc, P.conj().T @ r)
    assert np.abs(P.conj().T @ (r - D @ e)).max() < 1e-12 * np.abs(r).max()


def test_square_prolongator_exact():
    """Blocks of one site with Nv = 6 make P unitary: one V-cycle with an
    (exactly solved) coarse grid reproduces D^{-1} b."""
    L = (2, 2, 2, 4)
    m = -0.1
    U = W.gauge_field(L, 0.3, 0)
    p = so.MGParams(blocks=[(1, 1, 1, 1)], nv=[6], setup_rounds=1, coarse_tol=1e-14,
                    coarse_maxiter=5000, pre=0, post=0)
    h = so.mg_setup(U, m, p, W.setup_starts(L, 6, 0))
    b = W.gaussian_spinor(L, 1)
    x, it, conv, _ = so.mg_solve(h, b, 1e-12)
    xe = np.linalg.solve(wi.D_dense(U, m), b.ravel())
    assert conv and it <= 2
    assert np.linalg.norm(x.ravel() - xe) / np.linalg.norm(xe) < 1e-11


# ---------------------------------------------------------------- smoother / Krylov
def test_mr_residual_nonincreasing_and_step():
    L = (4, 4, 2, 4)
    U = W.gauge_field(L, 0.3, 0)
    A = lambda v: wi.apply_D(U, v, -0.2)  # noqa: E731
    b = W.gaussian_spinor(L, 1)
    prev = np.linalg.norm(b)
    for n in range(1, 6):
        x, r = so.mr(A, b, n, 0.9)
        rn = np.linalg.norm(b - A(x))
        assert np.abs(r - (b - A(x))).max() < 1e-12 * prev
        assert rn <= prev * (1 + 1e-14)
        prev = rn
    # one step equals the minimiser of ||b - a A b|| (closed form) times omega
    q = A(b)
    a = np.vdot(q.ravel(), b.ravel()) / np.vdot(q.ravel(), q.ravel())
    x1, _ = so.mr(A, b, 1, 0.9)
    assert np.abs(x1 - 0.9 * a * b).max() < 1e-14


def test_cgnr_matches_lu():
    U, h = _setup((4, 4, 4, 4), (2, 2, 2, 2), 3, rounds=1)
    lv = h.levels[0]
    Dc = co.coarse_dense(lv.X, lv.Y)
    rng = np.random.default_rng(3)
    r = (rng.standard_normal(Dc.shape[0]) + 1j * rng.standard_normal(Dc.shape[0])).reshape(lv.X.shape[:-1])
    A = lambda v: co.coarse_apply(lv.X, lv.Y, v)  # noqa: E731
    Ad = lambda v: co.coarse_apply_dag(lv.X, lv.Y, v)  # noqa: E731
    e, it = so.cgnr(A, Ad, r, tol=1e-3)
    assert np.linalg.norm(r - A(e)) <= 1e-3 * np.linalg.norm(r)
    e2, _ = so.cgnr(A, Ad, r, tol=1e-12, maxiter=5000)
    ex = np.linalg.solve(Dc, r.ravel())
    assert np.linalg.norm(e2.ravel() - ex) / np.linalg.norm(ex) < 1e-9


def test_fgcr_mg_matches_lu_4444():
    """Two-level FGCR(8)-MG on 4^4 against a dense LU solve."""
    L, m = (4, 4, 4, 4), -0.2
    U = W.gauge_field(L, 0.3, 0)
    p = so.MGParams(blocks=[(2, 2, 2, 2)], nv=[4])
    h = so.mg_setup(U, m, p, W.setup_starts(L, 4, 0))
    b = W.gaussian_spinor(L, 0)
    x, it, conv, hist = so.mg_solve(h, b, 1e-10)
    D = wi.D_dense(U, m)
    xe = np.linalg.solve(D, b.ravel())
    kappa = np.linalg.cond(D)
    assert conv
    assert np.linalg.norm(b.ravel() - D @ x.ravel()) <= 1e-10 * np.linalg.norm(b) * 1.0001
    assert np.linalg.norm(x.ravel() - xe) / np.linalg.norm(xe) < kappa * 1e-10
    # residual non-increasing within each restart cycle (minimal residual property)
    for j in range(1, len(hist)):
        if j % 8 != 0:
            assert hist[j] <= hist[j - 1] * (1 + 1e-12)


def test_three_level_hierarchy_galerkin():
    """Second-level Galerkin on the coarse stencil equals dense P2^dag D_c P2."""
    L, m = (4, 4, 4, 8), -0.2
    U = W.gauge_field(L, 0.3, 0)
    p = so.MGParams(blocks=[(2, 2, 2, 2), (1, 1, 1, 2)], nv=[4, 3], setup_rounds=1)
    starts = W.setup_starts(L, 4, 0)
    cst = W.coarse_setup_starts((2, 2, 2, 4), 8, 3, 0)
    h = so.mg_setup(U, m, p, starts, cst)
    l1, l2 = h.levels
    Dc1 = co.coarse_dense(l1.X, l1.Y)
    P2 = tr.P_dense(l2.Pb, l2.geom)
    assert np.abs(P2.conj().T @ P2 - np.eye(P2.shape[1])).max() < 1e-14
    ref = P2.conj().T @ Dc1 @ P2
    assert np.abs(co.coarse_dense(l2.X, l2.Y) - ref).max() < 1e-13 * np.abs(ref).max()
    b = W.gaussian_spinor(L, 2)
    x, it, conv, _ = so.mg_solve(h, b, 1e-10)
    assert conv
    assert np.linalg.norm(b - wi.apply_D(U, x, m)) <= 1.0001e-10 * np.linalg.norm(b)


# ---------------------------------------------------------------- setup stage two
def test_gcr_homogeneous_minimal_residual():
    """GCR steps on A x = 0 from v: the recurred residual is -A x, the w_j are
    orthonormal and orthogonal to the final residual, x - v lies in span(Z),
    and ||A x|| is the least-squares minimum over v + span(Z) (library lstsq),
    for a flexible (arbitrary linear) preconditioner."""
    rng = np.random.default_rng(5)
    n = 40
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    K = np.linalg.inv(A) + 0.05 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, r, Z, Wv = so.gcr_homogeneous(lambda u: A @ u, lambda u: K @ u, v, 5)
    assert np.abs(r + A @ x).max() < 1e-12 * np.abs(A @ v).max()
    Wm, Zm = np.stack(Wv, 1), np.stack(Z, 1)
    assert np.abs(Wm.conj().T @ Wm - np.eye(5)).max() < 1e-12
    assert np.abs(Wm.conj().T @ r).max() < 1e-12 * np.linalg.norm(A @ v)
    c, *_ = np.linalg.lstsq(A @ Zm, -(A @ v), rcond=None)
    assert np.abs(x - (v + Zm @ c)).max() < 1e-10 * np.linalg.norm(v)
    assert abs(np.linalg.norm(A @ x) - np.linalg.norm(A @ (v + Zm @ c))) < 1e-12 * np.linalg.norm(A @ v)
    assert np.linalg.norm(A @ x) < np.linalg.norm(A @ v)


def _refine_case():
    L, b, nv, m = (4, 4, 4, 4), (2, 2, 2, 2), 5, -0.3
    U = W.gauge_field(L, 0.3, 4)
    p = so.MGParams(blocks=[b], nv=[nv], setup_rounds=2, coarse_tol=1e-12, coarse_maxiter=5000)
    h = so.mg_setup(U, m, p, W.setup_starts(L, nv, 4))
    return U, m, p, h.levels[0].nullvecs


def test_refine_gauge_covariant_and_scale_invariant():
    """Refining g V on U^g gives g (refined V) (the truncated hierarchy, the
    V-cycle and GCR are gauge covariant), and rescaling the prototypes by
    complex factors only rephases the refined ones (block QR fixes the span,
    GCR is linear in its start, the result is normalised).  Group 2 of 5
    prototypes leaves a ragged last group of one."""
    U, m, p, V = _refine_case()
    Vr = so.refine_nullspace(U, m, p, V, 2, 3)
    g = W.gauge_transform(U.shape[1:5][::-1], 9)
    Vg = so.refine_nullspace(wi.gauge_transform_links(U, g), m, p, wi.gauge_transform_spinor(g, V), 2, 3)
    assert np.abs(Vg - wi.gauge_transform_spinor(g, Vr)).max() < 1e-9
    ph = np.exp(1j * np.arange(1, 6)) * np.arange(1, 6)
    Vs = so.refine_nullspace(U, m, p, V * ph[:, None, None, None, None, None, None], 2, 3)
    ph_n = (ph / np.abs(ph))[:, None, None, None, None, None, None]
    assert np.abs(Vs - Vr * ph_n).max() < 1e-9


def test_refine_lowers_residual_and_keeps_norm():
    """Every refined prototype has unit norm, and the group's GCR makes
    ||D v|| / ||v|| no larger than the relaxed prototype's; zero iterations
    leave V unchanged."""
    U, m, p, V = _refine_case()
    assert np.array_equal(so.refine_nullspace(U, m, p, V, 2, 0), V)
    Vr = so.refine_nullspace(U, m, p, V, 2, 3)
    A = lambda u: wi.apply_D(U, u, m)  # noqa: E731
    for k in range(V.shape[0]):
        assert abs(np.linalg.norm(Vr[k]) - 1) < 1e-12
        assert np.linalg.norm(A(Vr[k])) <= np.linalg.norm(A(V[k])) / np.linalg.norm(V[k]) * (1 + 1e-12)


def test_refine_one_step_is_projection_on_kept_span():
    """With no smoothing and an exact coarse solve the truncated method is
    K = P_k (P_k^dag D P_k)^{-1} P_k^dag, P_k spanning the kept prototypes
    restricted to each (aggregate, chirality) (K does not depend on the basis,
    so P_k is built from the raw prototypes, by coordinates).  One GCR step
    from v is x = v + a K(-D v) with a minimising ||D x|| (closed form), then
    x / ||x||.  Groups of one: the second prototype is refined with the first
    one already replaced."""
    U, m, p, V = _refine_case()
    L, (bx, by, bz, bt), nv = (4, 4, 4, 4), (2, 2, 2, 2), V.shape[0]
    p0 = so.MGParams(blocks=[(bx, by, bz, bt)], nv=[nv], pre=0, post=0, coarse_tol=1e-13,
                     coarse_maxiter=20000)
    Vr = so.refine_nullspace(U, m, p0, V, 1, 1)
    D = wi.D_dense(U, m)

    agg = np.array([(x // bx) + 2 * ((y // by) + 2 * ((z // bz) + 2 * (t // bt)))
                    for t in range(L[3]) for z in range(L[2]) for y in range(L[1]) for x in range(L[0])])
    comp_chi = np.arange(12) // 6

    def refined(Vcur, k):
        cols = []
        for j in range(nv):
            if j == k:
                continue
            f = Vcur[j].reshape(-1, 12)
            for a in range(16):
                for h in range(2):
                    mask = (agg[:, None] == a) & (comp_chi[None, :] == h)
                    cols.append(np.where(mask, f, 0).ravel())
        Pk = np.stack(cols, 1)
        v = Vcur[k].ravel()
        z = -Pk @ np.linalg.solve(Pk.conj().T @ D @ Pk, Pk.conj().T @ (D @ v))
        Dz, Dv = D @ z, D @ v
        x = v - np.vdot(Dz, Dv) / np.vdot(Dz, Dz) * z
        return (x / np.linalg.norm(x)).reshape(V[k].shape)
    e0 = refined(V, 0)
    assert np.abs(Vr[0] - e0).max() < 1e-8
    V1 = V.copy()
    V1[0] = Vr[0]
    assert np.abs(Vr[1] - refined(V1, 1)).max() < 1e-8


# ---------------------------------------------------------------- GMRES smoother, W-cycle
def test_gmres_is_krylov_minimiser():
    """GMRES(k) from 0 equals the brute-force least-squares minimiser of
    ||b - A y|| over span{b, Ab, ..., A^(k-1) b} (raw Krylov basis, library
    lstsq); k = dimension gives A^{-1} b (dense solve); b = 0 gives 0; the
    smoother returns omega y and the true residual."""
    rng = np.random.default_rng(8)
    n = 50
    A = np.eye(n) * 2 + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Af = lambda u: A @ u  # noqa: E731
    for k in (1, 2, 4):
        K = np.stack([np.linalg.matrix_power(A, j) @ b for j in range(k)], 1)
        c, *_ = np.linalg.lstsq(A @ K, b, rcond=None)
        y = so.gmres(Af, b, k)
        assert np.linalg.norm(y - K @ c) < 1e-10 * np.linalg.norm(K @ c)
    A6 = A[:6, :6]
    y6 = so.gmres(lambda u: A6 @ u, b[:6], 6)
    assert np.linalg.norm(y6 - np.linalg.solve(A6, b[:6])) < 1e-11 * np.linalg.norm(y6)
    assert not so.gmres(Af, np.zeros(n, complex), 4).any()
    x, r = so.gmres_smooth(Af, b, 4, 0.9)
    assert np.abs(x - 0.9 * so.gmres(Af, b, 4)).max() < 1e-14 and np.abs(r - (b - A @ x)).max() < 1e-13


def test_w_cycle_identity_and_effect():
    """Three levels with no smoothing and an exact coarsest solve: the
    intermediate correction K1 = P1 A2^{-1} P1^dag satisfies K1 A1 K1 = K1,
    so the W-cycle (second intermediate cycle on the updated residual)
    equals the V-cycle; with GMRES(4) post-smoothing it differs, and the
    fine-level cycle stays a good preconditioner (one FGCR solve to 1e-10)."""
    L, m = (4, 4, 4, 8), -0.2
    U = W.gauge_field(L, 0.3, 0)
    blocks, nv = [(2, 2, 2, 2), (1, 1, 1, 2)], [4, 3]
    st = W.setup_starts(L, 4, 0)
    cst = W.coarse_setup_starts((2, 2, 2, 4), 8, 3, 0)
    base = dict(blocks=blocks, nv=nv, setup_rounds=1, coarse_tol=1e-13, coarse_maxiter=20000)
    hV = so.mg_setup(U, m, so.MGParams(**base, pre=0, post=0), st, cst)
    hW = so.mg_setup(U, m, so.MGParams(**base, pre=0, post=0, cycles=2), st, cst)
    r = W.gaussian_spinor(L, 3)
    zV, zW = hV.vcycle(r, 0), hW.vcycle(r, 0)
    assert np.linalg.norm(zW - zV) < 1e-9 * np.linalg.norm(zV)
    g1 = so.mg_setup(U, m, so.MGParams(**base, pre=0, post=4, smoother="gmres"), st, cst)
    g2 = so.mg_setup(U, m, so.MGParams(**base, pre=0, post=4, smoother="gmres", cycles=2), st, cst)
    assert np.linalg.norm(g2.vcycle(r, 0) - g1.vcycle(r, 0)) > 1e-6 * np.linalg.norm(zV)
    b = W.gaussian_spinor(L, 4)
    x, it, conv, _ = so.mg_solve(g2, b, 1e-10)
    assert conv and np.linalg.norm(b - wi.apply_D(U, x, m)) <= 1e-10 * np.linalg.norm(b) * 1.0001


def test_refine_level1_one_step_is_projection_on_kept_span():
    """The same dense construction one level down (three-level hierarchy):
    the level-1 prototypes are refined with the truncated method from level
    1 (no smoothing, exact CGNR on the truncated level 2), against
    v + a K(-A_1 v) with A_1 the dense level-1 operator and K built from the
    raw kept level-1 prototypes restricted to each (aggregate, chirality)."""
    L, m = (4, 4, 4, 8), -0.2
    U = W.gauge_field(L, 0.3, 2)
    blocks, nv = [(2, 2, 2, 2), (1, 1, 1, 2)], [4, 3]
    Lc = (2, 2, 2, 4)
    base = dict(blocks=blocks, nv=nv, setup_rounds=2, coarse_tol=1e-13, coarse_maxiter=20000)
    h = so.mg_setup(U, m, so.MGParams(**base), W.setup_starts(L, 4, 2), W.coarse_setup_starts(Lc, 8, 3, 2))
    V1 = h.levels[1].nullvecs
    p0 = so.MGParams(**base, pre=0, post=0)
    Vr = so.refine_nullspace(U, m, p0, V1, 1, 1, h.levels[:1])
    A1 = co.coarse_dense(h.levels[0].X, h.levels[0].Y)
    agg = np.array([x + 2 * (y + 2 * (z + 2 * (t // 2)))
                    for t in range(Lc[3]) for z in range(Lc[2]) for y in range(Lc[1]) for x in range(Lc[0])])
    comp_chi = np.arange(8) // 4
    cols = []
    for j in (1, 2):
        f = V1[j].reshape(-1, 8)
        for a in range(16):
            for hh in range(2):
                mask = (agg[:, None] == a) & (comp_chi[None, :] == hh)
                cols.append(np.where(mask, f, 0).ravel())
    Pk = np.stack(cols, 1)
    v = V1[0].ravel()
    z = -Pk @ np.linalg.solve(Pk.conj().T @ A1 @ Pk, Pk.conj().T @ (A1 @ v))
    Az, Av = A1 @ z, A1 @ v
    x = v - np.vdot(Az, Av) / np.vdot(Az, Az) * z
    assert np.abs(Vr[0].ravel() - x / np.linalg.norm(x)).max() < 1e-8


# ---------------------------------------------------------------- setup stage one (a5)
def _dense_case(L=(4, 4, 4, 4), m=-0.2, eps=0.3, seed=5):
    U = W.gauge_field(L, eps, seed)
    return U, m, wi.D_dense(U, m)


def test_relax_one_round_one_step_is_damped_minimiser():
    """One round of one MR step moves each start v along -D v by omega times
    the scalar that minimises ||D (v - c D v)|| (library least squares on the
    dense operator), then normalises: the relaxation solves D e = -D v, it
    does not move v towards the large modes."""
    L = (4, 4, 4, 4)
    U, m, D = _dense_case(L)
    starts = W.setup_starts(L, 2, 3)
    A = lambda u: wi.apply_D(U, u, m)  # noqa: E731
    for omega in (1.0, 0.9):
        Vr = so.relax_nullspace(A, starts, 1, 1, omega)
        for k in range(2):
            v = starts[k].ravel()
            Dv = D @ v
            c, *_ = np.linalg.lstsq((D @ Dv)[:, None], Dv, rcond=None)
            x = v - omega * c[0] * Dv
            ref = x / np.linalg.norm(x)
            assert np.abs(Vr[k].ravel() - ref).max() < 1e-12
            assert abs(np.linalg.norm(Vr[k]) - 1.0) < 1e-13


def test_relax_rounds_compose_and_lower_the_rayleigh_ratio():
    """Rounds compose (two rounds = one round applied to the result of one
    round), every relaxed vector has unit norm, and five rounds of four MR
    steps lower ||D v|| / ||v|| of every start well below the start's value
    (relaxation leaves the near-null space)."""
    L = (4, 4, 4, 4)
    U, m, D = _dense_case(L)
    starts = W.setup_starts(L, 3, 4)
    A = lambda u: wi.apply_D(U, u, m)  # noqa: E731
    two = so.relax_nullspace(A, starts, 2, 3, 0.9)
    once_twice = so.relax_nullspace(A, so.relax_nullspace(A, starts, 1, 3, 0.9), 1, 3, 0.9)
    assert np.abs(two - once_twice).max() < 1e-13
    V5 = so.relax_nullspace(A, starts, 5, 4, 0.9)
    svals = np.linalg.svd(D, compute_uv=False)
    for k in range(3):
        before = np.linalg.norm(D @ starts[k].ravel()) / np.linalg.norm(starts[k])
        after = np.linalg.norm(D @ V5[k].ravel())
        assert abs(np.linalg.norm(V5[k]) - 1.0) < 1e-13
        assert svals[-1] * (1 - 1e-12) <= after < 0.5 * before


# ---------------------------------------------------------------- smoothed cycle (a12)
def _exact_coarse_projector(h, L, b):
    """K = P (P^dag D P)^{-1} P^dag with P spanning the raw null vectors
    restricted to each (aggregate, chirality) by coordinates (K does not
    depend on the basis of that span)."""
    V = h.levels[0].nullvecs
    nv = V.shape[0]
    Cx, Cy, Cz = L[0] // b[0], L[1] // b[1], L[2] // b[2]
    agg = np.array([(x // b[0]) + Cx * ((y // b[1]) + Cy * ((z // b[2]) + Cz * (t // b[3])))
                    for t in range(L[3]) for z in range(L[2]) for y in range(L[1]) for x in range(L[0])])
    nagg = agg.max() + 1
    comp_chi = np.arange(12) // 6
    cols = []
    for j in range(nv):
        f = V[j].reshape(-1, 12)
        for a in range(nagg):
            for hh in range(2):
                mask = (agg[:, None] == a) & (comp_chi[None, :] == hh)
                cols.append(np.where(mask, f, 0).ravel())
    P = np.stack(cols, 1)
    return P


@pytest.mark.parametrize("pre,post", [(0, 1), (1, 0), (1, 1)])
def test_vcycle_smoothing_around_exact_coarse_correction(pre, post):
    """Two levels with an exact coarse solve (CGNR to 1e-13): the cycle is
    x1 = omega c1 r (pre-step, c1 = argmin ||r - c D r||), rho1 = r - D x1,
    x2 = x1 + K rho1 with K the exact coarse correction of the null-vector
    span, rho2 = r - D x2, z = x2 + omega c2 rho2 (post-step, c2 =
    argmin ||rho2 - c D rho2||): each minimiser by library least squares on
    the dense operator.  The post-step never raises the residual."""
    L, b, nv, m = (4, 4, 4, 4), (2, 2, 2, 2), 4, -0.2
    U = W.gauge_field(L, 0.3, 6)
    p = so.MGParams(blocks=[b], nv=[nv], setup_rounds=2, pre=pre, post=post, coarse_tol=1e-13,
                    coarse_maxiter=20000)
    h = so.mg_setup(U, m, p, W.setup_starts(L, nv, 6))
    D = wi.D_dense(U, m)
    P = _exact_coarse_projector(h, L, b)
    K = lambda v: P @ np.linalg.solve(P.conj().T @ D @ P, P.conj().T @ v)  # noqa: E731
    r = W.gaussian_spinor(L, 7)
    rv = r.ravel()

    def mr_step(res):
        c, *_ = np.linalg.lstsq((D @ res)[:, None], res, rcond=None)
        return 0.9 * c[0] * res

    x = mr_step(rv) if pre else np.zeros_like(rv)
    x = x + K(rv - D @ x)
    xc = x.copy()
    if post:
        x = x + mr_step(rv - D @ x)
    z = h.vcycle(r, 0).ravel()
    assert np.linalg.norm(z - x) < 1e-9 * np.linalg.norm(x)
    if post:
        assert np.linalg.norm(rv - D @ z) <= np.linalg.norm(rv - D @ xc) * (1 + 1e-12)
