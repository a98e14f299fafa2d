"""Oracle: MR smoother, CGNR coarsest solve, null-vector setup, V-cycle, FGCR(8).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper sources:
  * V(m,n)-cycle: m pre- and n post-relaxations per level, recursion down to
    a solve on the coarsest grid ("Adaptive Multigrid").
  * Relaxation: a minimal-residual Krylov smoother with under-relaxation
    omega = 0.9 that reduces the residual in the D^dag D norm ("Formulating an
    algorithm").  Here each step is GMRES(1), i.e. MR, a fixed number of
    times (4 pre, 4 post).
  * Coarsest grid: CG on the normal equations to relative accuracy 1e-3
    ("Numerical Results").  D_c^dag is the plain adjoint of the stencil.
  * The paper's own cycle ("Numerical Results"): V(0,4) with GMRES(4)
    post-relaxation under-relaxed by omega, and a W-cycle in which every
    correction of the fine grid takes two cycles of the intermediate grid.
    Readings: the GMRES smoother is x = omega * GMRES(k)(A, r) from x = 0
    (one cycle, no restart); the second intermediate cycle is applied to the
    intermediate residual left by the first and its result added.
  * Outer solver: flexible GCR with restart length 8, because the
    preconditioner is non-stationary ("Formulating an algorithm").
  * Setup stage 1: relaxation applied to random vectors on A x = 0 gives
    the initial prototypes, which are then block-orthonormalised.
Readings: one setup round = one smoother application (n_s MR steps) on
D e = 0 started from the current vector, i.e. v <- v - MR(D, D v), then
v <- v / ||v||; the pre-smoother residual entering restriction is the MR
recursion's residual; FGCR restarts every 8 with the true residual b - D x
and orthogonalises by modified Gram-Schmidt.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import coarse as co
from . import transfer as tr
from . import wilson


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _nrm2(a):
    return float(np.real(np.vdot(a.ravel(), a.ravel())))


def mr(A, b, steps: int, omega: float = 0.9):
    """MR from x = 0: q = A r, alpha = <q,r>/<q,q>, x += w alpha r, r -= w alpha q.
    Returns (x, r) with r the recursively updated residual."""
    x = np.zeros_like(b)
    r = b.copy()
    for _ in range(steps):
        q = A(r)
        qq = _nrm2(q)
        if qq == 0.0:
            break
        a = omega * _dot(q, r) / qq
        x = x + a * r
        r = r - a * q
    return x, r


def gmres(A, b, k: int):
    """One GMRES(k) cycle from y = 0: the y in the Krylov space
    span{b, Ab, ..., A^(k-1) b} that minimises ||b - A y||, through Arnoldi
    with modified Gram-Schmidt and the (k+1) x k Hessenberg least-squares
    problem (library lstsq).  A zero subdiagonal entry means the space is
    invariant and ends it early; b = 0 gives y = 0."""
    y = np.zeros_like(b)
    beta = np.sqrt(_nrm2(b))
    if beta == 0.0 or k <= 0:
        return y
    V = [b / beta]
    H = np.zeros((k + 1, k), dtype=np.complex128)
    kk = k
    for j in range(k):
        w = A(V[j])
        for i in range(j + 1):
            H[i, j] = _dot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.sqrt(_nrm2(w))
        if H[j + 1, j] == 0.0:
            kk = j + 1
            break
        V.append(w / H[j + 1, j])
    g = np.zeros(kk + 1, dtype=np.complex128)
    g[0] = beta
    c, *_ = np.linalg.lstsq(H[:kk + 1, :kk], g, rcond=None)
    for j in range(kk):
        y = y + c[j] * V[j]
    return y


def gmres_smooth(A, b, steps: int, omega: float = 0.9):
    """GMRES smoother with under-relaxation ("Formulating an algorithm"):
    x = omega * GMRES(steps)(A, b) from x = 0.  Returns (x, b - A x)."""
    if steps <= 0:
        return np.zeros_like(b), b.copy()
    x = omega * gmres(A, b, steps)
    return x, b - A(x)


def mr_batch(A, b, steps: int, omega: float = 0.9):
    """MR applied independently to each b[k] of a batch (per-vector scalars)."""
    xs, rs = [], []
    for k in range(b.shape[0]):
        x, r = mr(A, b[k], steps, omega)
        xs.append(x)
        rs.append(r)
    return np.stack(xs), np.stack(rs)


def cgnr(A, Adag, b, tol: float = 1e-3, maxiter: int = 1000):
    """CG on A^dag A e = A^dag b from e = 0; stop when ||b - A e|| <= tol ||b||
    (recursive residual).  Returns (e, iterations)."""
    e = np.zeros_like(b)
    r = b.copy()
    nb = np.sqrt(_nrm2(b))
    if nb == 0.0:
        return e, 0
    z = Adag(r)
    p = z.copy()
    zz = _nrm2(z)
    it = 0
    while it < maxiter:
        w = A(p)
        ww = _nrm2(w)
        if ww == 0.0:
            break
        alpha = zz / ww
        e = e + alpha * p
        r = r - alpha * w
        it += 1
        if np.sqrt(_nrm2(r)) <= tol * nb:
            break
        z = Adag(r)
        zz_new = _nrm2(z)
        beta = zz_new / zz
        zz = zz_new
        p = z + beta * p
    return e, it


def relax_nullspace(A, starts, rounds: int, steps: int, omega: float = 0.9):
    """Setup stage 1: v <- v - MR(A, A v, steps), then v <- v/||v||, `rounds` times."""
    V = np.array(starts, dtype=np.complex128, copy=True)
    for _ in range(rounds):
        for k in range(V.shape[0]):
            x, _r = mr(A, A(V[k]), steps, omega)
            V[k] = V[k] - x
            V[k] = V[k] / np.sqrt(_nrm2(V[k]))
    return V


@dataclass
class MGParams:
    blocks: list = field(default_factory=lambda: [(4, 4, 4, 4)])
    nv: list = field(default_factory=lambda: [8])
    setup_rounds: int = 5
    setup_mr_steps: int = 4
    omega: float = 0.9
    pre: int = 4
    post: int = 4
    coarse_tol: float = 1e-3
    coarse_maxiter: int = 1000
    gcr_restart: int = 8
    max_iter: int = 10000
    antiperiodic_t: bool = True
    refine_group: int = 0      # setup stage two: group size (0 = off)
    refine_iters: int = 5
    smoother: str = "mr"       # "mr": pre/post MR steps; "gmres": GMRES(pre), GMRES(post)
    cycles: int = 1            # cycles of level l+1 per correction of level l (2 = W-cycle)


@dataclass
class Level:
    geom: tr.BlockGeometry      # aggregation of this level's lattice
    Pb: np.ndarray              # [Vc, 2, rows, Nv]
    Rc: np.ndarray              # coarse coefficients V_c (QR R factors)
    X: np.ndarray               # coarse operator of the next level
    Y: np.ndarray
    nullvecs: np.ndarray


class Hierarchy:
    """Adaptive MG hierarchy: level 0 = fine Wilson operator, level l >= 1 =
    Galerkin coarse stencil of level l-1."""

    def __init__(self, U, m, params: MGParams, levels):
        self.U, self.m, self.p, self.levels = U, m, params, levels
        self.stats = dict(fine_D=0, coarse_apply=0, cgnr_iters=[])

    # operators ------------------------------------------------------------
    def op(self, lvl: int):
        if lvl == 0:
            def A(v):
                self.stats["fine_D"] += 1
                return wilson.apply_D(self.U, v, self.m, self.p.antiperiodic_t)
            return A
        L = self.levels[lvl - 1]

        def Ac(v):
            self.stats["coarse_apply"] += 1
            return co.coarse_apply(L.X, L.Y, v)
        return Ac

    def op_dag(self, lvl: int):
        L = self.levels[lvl - 1]

        def Acd(v):
            self.stats["coarse_apply"] += 1
            return co.coarse_apply_dag(L.X, L.Y, v)
        return Acd

    def restrict(self, lvl, f):
        L = self.levels[lvl]
        g = tr.fine_to_generic(f) if lvl == 0 else f
        return tr.restrict(L.Pb, L.geom, g)

    def prolong(self, lvl, ec):
        L = self.levels[lvl]
        g = tr.prolong(L.Pb, L.geom, ec)
        return tr.generic_to_fine(g) if lvl == 0 else g

    # V-cycle (a12) --------------------------------------------------------
    def vcycle(self, r, lvl: int = 0):
        p = self.p
        nlev = len(self.levels) + 1
        if lvl == nlev - 1:
            e, it = cgnr(self.op(lvl), self.op_dag(lvl), r, p.coarse_tol, p.coarse_maxiter)
            self.stats["cgnr_iters"].append(it)
            return e
        A = self.op(lvl)
        smooth = gmres_smooth if p.smoother == "gmres" else mr
        x, rho = smooth(A, r, p.pre, p.omega)
        rc = self.restrict(lvl, rho)
        ec = self.vcycle(rc, lvl + 1)
        if lvl + 1 < nlev - 1:
            # W-cycle: further cycles of the next level on its updated residual
            Ac = self.op(lvl + 1)
            for _ in range(1, p.cycles):
                ec = ec + self.vcycle(rc - Ac(ec), lvl + 1)
        x = x + self.prolong(lvl, ec)
        rho = r - A(x)
        x2, _ = smooth(A, rho, p.post, p.omega)
        return x + x2


def mg_setup(U, m, params: MGParams, starts, coarse_starts=None):
    """Two- or three-level setup: relaxation of random starts, block QR, Galerkin."""
    levels = []
    h = Hierarchy(U, m, params, levels)
    L = tuple(reversed(U.shape[1:5]))
    geom = tr.BlockGeometry(L, params.blocks[0])
    V = relax_nullspace(h.op(0), starts, params.setup_rounds, params.setup_mr_steps, params.omega)
    if params.refine_group > 0 and params.refine_iters > 0:
        V = refine_nullspace(U, m, params, V, params.refine_group, params.refine_iters)
    Pb, Rc = tr.block_qr(np.moveaxis(geom.blockify(tr.fine_to_generic(V)), 0, -1))
    X, Y = co.galerkin_fine(U, m, Pb, geom, params.antiperiodic_t)
    levels.append(Level(geom, Pb, Rc, X, Y, V))
    for lv in range(1, len(params.blocks)):
        geom2 = tr.BlockGeometry(levels[-1].geom.Lc, params.blocks[lv])
        V2 = relax_nullspace(h.op(lv), coarse_starts, params.setup_rounds,
                             params.setup_mr_steps, params.omega)
        if params.refine_group > 0 and params.refine_iters > 0:
            V2 = refine_nullspace(U, m, params, V2, params.refine_group, params.refine_iters, levels)
        Pb2, Rc2 = tr.block_qr(np.moveaxis(geom2.blockify(V2), 0, -1))
        X2, Y2 = co.galerkin_coarse(levels[-1].X, levels[-1].Y, Pb2, geom2)
        levels.append(Level(geom2, Pb2, Rc2, X2, Y2, V2))
    h.stats = dict(fine_D=0, coarse_apply=0, cgnr_iters=[])
    return h


def refine_nullspace(U, m, params: MGParams, V, group: int, iters: int, levels=()):
    """Setup stage two ("Numerical Results"): the prototypes of level
    l = len(levels) (the levels below already built) are refined in groups of
    `group`: a group is taken out of V, a truncated two-level method from
    level l is built from the remaining prototypes (block QR and Galerkin
    operator as in stage one; the cycle of level l over a CGNR solve on the
    truncated next level), the truncated MG method is iterated `iters` times
    on A_l v = 0 from every prototype of the group, and the normalised result
    goes back into V before the next group is taken.  Reading: "the MG method"
    is the solver of the adaptive process, the MG-preconditioned flexible GCR
    applied to the homogeneous system ("Adaptive Multigrid"), so the
    iterations are GCR steps (no restart within them) started at the
    prototype."""
    V = np.array(V, dtype=np.complex128, copy=True)
    nv = V.shape[0]
    if group <= 0 or iters <= 0 or group >= nv:
        return V
    lvl = len(levels)
    if lvl == 0:
        geom = tr.BlockGeometry(tuple(reversed(U.shape[1:5])), params.blocks[0])
    else:
        geom = tr.BlockGeometry(levels[-1].geom.Lc, params.blocks[lvl])
    for g0 in range(0, nv, group):
        grp = list(range(g0, min(g0 + group, nv)))
        keep = [k for k in range(nv) if k not in grp]
        B = tr.fine_to_generic(V[keep]) if lvl == 0 else V[keep]
        Pb, Rc = tr.block_qr(np.moveaxis(geom.blockify(B), 0, -1))
        if lvl == 0:
            X, Y = co.galerkin_fine(U, m, Pb, geom, params.antiperiodic_t)
        else:
            X, Y = co.galerkin_coarse(levels[-1].X, levels[-1].Y, Pb, geom)
        pt = MGParams(**{**params.__dict__, "blocks": list(params.blocks[:lvl + 1]),
                         "nv": list(params.nv[:lvl]) + [len(keep)]})
        h = Hierarchy(U, m, pt, list(levels) + [Level(geom, Pb, Rc, X, Y, V[keep])])
        A = h.op(lvl)
        for k in grp:
            x, _, _, _ = gcr_homogeneous(A, lambda r: h.vcycle(r, lvl), V[k], iters)
            V[k] = x / np.sqrt(_nrm2(x))
    return V


def gcr_homogeneous(A, K, v, iters: int):
    """`iters` steps of flexible GCR preconditioned by K on A x = 0 from x = v
    (no restart): z_j = K(r), w_j = A z_j made orthonormal to the earlier w
    (the same combination applied to z_j), x += <w_j, r> z_j,
    r -= <w_j, r> w_j.  Returns (x, r, Z, W)."""
    x = v.copy()
    r = -A(x)
    Z, Wv = [], []
    for _ in range(iters):
        z = K(r)
        w = A(z)
        for zi, wi in zip(Z, Wv):
            beta = _dot(wi, w)
            w = w - beta * wi
            z = z - beta * zi
        nw = np.sqrt(_nrm2(w))
        w, z = w / nw, z / nw
        Z.append(z)
        Wv.append(w)
        alpha = _dot(w, r)
        x = x + alpha * z
        r = r - alpha * w
    return x, r, Z, Wv


def fgcr(A, K, b, tol: float, restart: int = 8, max_iter: int = 10000, x0=None):
    """Flexible GCR(restart): z_j = K(r), w_j = A z_j, MGS against previous w,
    normalise, alpha = <w_j, r>, x += alpha z_j, r -= alpha w_j; restart with
    the true residual.  Converged when ||b - A x|| <= tol ||b||.
    Returns (x, iterations, converged, residual history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    nb = np.sqrt(_nrm2(b))
    r = b - A(x) if x0 is not None else b.copy()
    hist = [np.sqrt(_nrm2(r)) / nb]
    it = 0
    if hist[0] <= tol:
        return x, 0, True, hist
    while it < max_iter:
        Z, W = [], []
        for j in range(restart):
            z = K(r)
            w = A(z)
            for i in range(j):
                beta = _dot(W[i], w)
                w = w - beta * W[i]
                z = z - beta * Z[i]
            nw = np.sqrt(_nrm2(w))
            w = w / nw
            z = z / nw
            W.append(w)
            Z.append(z)
            alpha = _dot(w, r)
            x = x + alpha * z
            r = r - alpha * w
            it += 1
            rn = np.sqrt(_nrm2(r)) / nb
            hist.append(rn)
            if rn <= tol or it >= max_iter:
                break
        r = b - A(x)
        rn = np.sqrt(_nrm2(r)) / nb
        hist[-1] = rn
        if rn <= tol:
            return x, it, True, hist
    return x, it, False, hist


def mg_solve(h: Hierarchy, b, tol: float = 1e-10):
    p = h.p
    A = h.op(0)
    return fgcr(A, lambda r: h.vcycle(r, 0), b, tol, p.gcr_restart, p.max_iter)
