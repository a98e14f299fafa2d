"""Oracle: Galerkin coarse operator D_c = P^dag D P as a 9-point stencil.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper, "Adaptive Multigrid": A_c = P^dag A P with R = P^dag; "Formulating an
algorithm": with uniform hypercubic aggregates and chirality kept separate the
coarse operator is nearest neighbour, with effective link matrices of size
2Nv x 2Nv, and recursing keeps that sparsity pattern on every level.

Representation on a coarse lattice Lc = (Cx, Cy, Cz, Ct) with n = 2Nv:
  X[t, z, y, x, n, n]        self coupling
  Y[d, t, z, y, x, n, n]     d = 2 mu + dir; dir 0 couples x_c to x_c + mu,
                             dir 1 couples x_c to x_c - mu (periodic wrap).
  (D_c v)(x_c) = X(x_c) v(x_c) + sum_mu [Y_{2mu}(x_c) v(x_c+mu) + Y_{2mu+1}(x_c) v(x_c-mu)].
Boundary phases of the fine level are inside Y.  Y_d collects exactly the fine
hops that leave a block through its face in slot d (even when the coarse
extent is 1 or 2 and both slots reach the same coarse site).
"""
from __future__ import annotations

import numpy as np

from . import wilson
from .transfer import BlockGeometry, fine_to_generic, generic_to_fine, prolong, restrict

SITE_AXIS = (-2, -3, -4, -5)  # axis of direction mu in a [..., t, z, y, x, n] array


def _unit_columns(geom: BlockGeometry, nv: int, j: int):
    Cx, Cy, Cz, Ct = geom.Lc
    e = np.zeros((Ct, Cz, Cy, Cx, 2 * nv), dtype=np.complex128)
    e[..., j] = 1.0
    return e


def _galerkin(diag_op, hops, Pb, geom: BlockGeometry, to_level, from_level):
    """Generic Galerkin product.  For every coarse column j, W = P e_j (the j-th
    column in every block); X[:, j] = P^dag diag(W) + P^dag (intra-block hops
    of W); Y_d[:, j] = P^dag (hops of W in slot d that cross the block face)."""
    nv = Pb.shape[-1]
    n = 2 * nv
    Cx, Cy, Cz, Ct = geom.Lc
    X = np.zeros((Ct, Cz, Cy, Cx, n, n), dtype=np.complex128)
    Y = np.zeros((8, Ct, Cz, Cy, Cx, n, n), dtype=np.complex128)
    faces = [geom.face_field(d) for d in range(8)]
    for j in range(n):
        W = from_level(prolong(Pb, geom, _unit_columns(geom, nv, j)))
        X[..., :, j] = restrict(Pb, geom, to_level(diag_op(W)))
        for d in range(8):
            h = to_level(hops(W, d))
            X[..., :, j] += restrict(Pb, geom, h * (1.0 - faces[d]))
            Y[d, ..., :, j] = restrict(Pb, geom, h * faces[d])
    return X, Y


def galerkin_fine(U, m: float, Pb, geom: BlockGeometry, antiperiodic_t: bool = True):
    """D_c = P^dag D(U) P for the fine Wilson operator of Eq. (2)."""
    def diag_op(w):
        return (4.0 + m) * w

    def hops(w, d):
        mu, dr = divmod(d, 2)
        return wilson.hop(U, w, mu, dr == 0, antiperiodic_t)

    return _galerkin(diag_op, hops, Pb, geom, fine_to_generic, generic_to_fine)


def coarse_hop(Y, v, d: int):
    """Y_d(x_c) v(x_c +/- mu) for one stencil slot."""
    mu, dr = divmod(d, 2)
    nb = np.roll(v, -1 if dr == 0 else +1, axis=SITE_AXIS[mu])
    return np.einsum("...ij,...j->...i", Y[d], nb)


def galerkin_coarse(X1, Y1, Pb, geom: BlockGeometry):
    """D_c2 = P2^dag D_c1 P2 for a coarse stencil operator (3-level hierarchy)."""
    def diag_op(w):
        return np.einsum("...ij,...j->...i", X1, w)

    def hops(w, d):
        return coarse_hop(Y1, w, d)

    ident = lambda f: f  # noqa: E731
    return _galerkin(diag_op, hops, Pb, geom, ident, ident)


def coarse_apply(X, Y, v):
    """D_c v as the 9-point stencil."""
    out = np.einsum("...ij,...j->...i", X, v)
    for d in range(8):
        out = out + coarse_hop(Y, v, d)
    return out


def coarse_apply_dag(X, Y, v):
    """D_c^dag v from the plain adjoint of the stencil:
    (D_c^dag v)(y) = X(y)^dag v(y) + sum_mu [Y_{2mu}(y-mu)^dag v(y-mu) + Y_{2mu+1}(y+mu)^dag v(y+mu)]."""
    out = np.einsum("...ji,...j->...i", np.conj(X), v)
    for d in range(8):
        mu, dr = divmod(d, 2)
        shift = +1 if dr == 0 else -1          # source site of the transposed hop
        Ys = np.roll(Y[d], shift, axis=SITE_AXIS[mu] - 1)
        vs = np.roll(v, shift, axis=SITE_AXIS[mu])
        out = out + np.einsum("...ji,...j->...i", np.conj(Ys), vs)
    return out


def sigma3(v):
    """Coarse chirality sigma_3 = diag(+1_Nv, -1_Nv) (P^dag gamma_5 = sigma_3 P^dag)."""
    n = v.shape[-1]
    s = np.ones(n)
    s[n // 2:] = -1.0
    return v * s


def coarse_dense(X, Y):
    """Dense D_c (coarse lexicographic site-major index)."""
    Ct, Cz, Cy, Cx, n, _ = X.shape
    N = Ct * Cz * Cy * Cx * n
    eye = np.eye(N, dtype=np.complex128).reshape(N, Ct, Cz, Cy, Cx, n)
    cols = coarse_apply(X, Y, eye).reshape(N, N)
    return cols.T.copy()
