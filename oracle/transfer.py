"""Oracle: aggregates, chirality-split block QR prolongator P, R = P^dag.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper, "Adaptive Multigrid": the candidate vectors V are partitioned into
disjoint local blocks (aggregates) and QR-factorised per block; Q gives the
columns of P and R the coarse coefficients V_c, so P^dag P = I_c and
P V_c = V (Eq. 4).  "Formulating an algorithm": the upper and lower spin
halves are coarsened separately (chirality kept intact), so that
P^dag gamma_5 = sigma_3 P^dag, each prototype gives two coarse degrees of
freedom, and R = P^dag (Eq. 8 with the gamma_5 factors cancelled).  The
aggregates are uniform hypercubic blocks, so the coarse operator is again a
nearest-neighbour stencil.

Generic field layout used here: f[..., t, z, y, x, n] with n = 2h components
split into two chirality halves (fine level: n = 12 spin-colour components in
order 3s + c, chirality 0 = spins {0,1} = components 0..5; coarse level:
n = 2 Nv, chirality 0 = components 0..Nv-1, i.e. sigma_3 = diag(1, -1)).

Readings: aggregate of site x is floor(x_mu / b_mu); local index
l = o_x + b_x (o_y + b_y (o_z + b_z o_t)) with o = x mod b; the row of a
(block, chirality) matrix is l*h + j for the j-th component of that
chirality half.  QR phase: R has a positive real diagonal (this makes Q
unique).  A block is rank deficient, an error, when r_kk < 1e-14 times the
norm of the column before orthogonalisation.
"""
from __future__ import annotations

import numpy as np


class BlockGeometry:
    """Hypercubic aggregation of an L = (Lx, Ly, Lz, Lt) lattice into blocks b."""

    def __init__(self, L, b):
        self.L = tuple(int(v) for v in L)
        self.b = tuple(int(v) for v in b)
        for mu in range(4):
            if self.b[mu] <= 0 or self.L[mu] % self.b[mu] != 0:
                raise ValueError(f"block {self.b} does not divide lattice {self.L}")
        self.Lc = tuple(self.L[mu] // self.b[mu] for mu in range(4))
        self.V = int(np.prod(self.L))
        self.Vc = int(np.prod(self.Lc))
        self.vol_b = int(np.prod(self.b))

    # ---- index maps (a4) -------------------------------------------------
    def coords(self):
        """Coordinates (x, y, z, t) of every fine site in lexicographic order."""
        Lx, Ly, Lz, Lt = self.L
        i = np.arange(self.V)
        x = i % Lx
        y = (i // Lx) % Ly
        z = (i // (Lx * Ly)) % Lz
        t = i // (Lx * Ly * Lz)
        return np.stack([x, y, z, t])

    def maps(self):
        """(fine->coarse, fine->local, coarse neighbour table [Vc, 8], face mask [V]).

        Neighbour slot d = 2*mu + dir, dir 0 = +mu, dir 1 = -mu (periodic).
        Face mask bit d is set when the hop of site x in slot d leaves the
        site's block (o_mu = b_mu - 1 forward, o_mu = 0 backward).
        """
        c = self.coords()
        b = np.array(self.b)[:, None]
        Lc = np.array(self.Lc)[:, None]
        xc = c // b
        o = c % b
        f2c = xc[0] + Lc[0] * (xc[1] + Lc[1] * (xc[2] + Lc[2] * xc[3]))
        f2l = o[0] + b[0] * (o[1] + b[1] * (o[2] + b[2] * o[3]))
        face = np.zeros(self.V, dtype=np.int64)
        for mu in range(4):
            face |= (o[mu] == self.b[mu] - 1).astype(np.int64) << (2 * mu)
            face |= (o[mu] == 0).astype(np.int64) << (2 * mu + 1)
        ic = np.arange(self.Vc)
        cc = np.stack([ic % self.Lc[0], (ic // self.Lc[0]) % self.Lc[1],
                       (ic // (self.Lc[0] * self.Lc[1])) % self.Lc[2],
                       ic // (self.Lc[0] * self.Lc[1] * self.Lc[2])])
        nbr = np.zeros((self.Vc, 8), dtype=np.int64)
        for mu in range(4):
            for d, step in ((0, 1), (1, -1)):
                n = cc.copy()
                n[mu] = (n[mu] + step) % self.Lc[mu]
                nbr[:, 2 * mu + d] = n[0] + self.Lc[0] * (n[1] + self.Lc[1] * (n[2] + self.Lc[2] * n[3]))
        return (f2c.astype(np.int32), f2l.astype(np.int32), nbr.astype(np.int32),
                face.astype(np.int32))

    def face_field(self, slot: int):
        """[t, z, y, x, 1] array: 1 where the hop in slot d leaves the block."""
        Lx, Ly, Lz, Lt = self.L
        mu, d = divmod(slot, 2)
        ax_len = self.L[mu]
        o = np.arange(ax_len) % self.b[mu]
        sel = (o == self.b[mu] - 1) if d == 0 else (o == 0)
        shape = [1, 1, 1, 1]
        shape[3 - mu] = ax_len
        f = np.broadcast_to(sel.reshape(shape), (Lt, Lz, Ly, Lx)).astype(np.float64)
        return f[..., None]

    # ---- blocking of fields --------------------------------------------
    def blockify(self, f):
        """f[..., t, z, y, x, n] -> B[..., Vc, 2, vol_b * n/2] (row = l*h + j)."""
        Lx, Ly, Lz, Lt = self.L
        bx, by, bz, bt = self.b
        Cx, Cy, Cz, Ct = self.Lc
        n = f.shape[-1]
        h = n // 2
        lead = f.shape[:-5]
        g = f.reshape(lead + (Ct, bt, Cz, bz, Cy, by, Cx, bx, 2, h))
        k = len(lead)
        perm = list(range(k)) + [k + 0, k + 2, k + 4, k + 6, k + 8, k + 1, k + 3, k + 5, k + 7, k + 9]
        g = np.transpose(g, perm)
        return g.reshape(lead + (self.Vc, 2, self.vol_b * h))

    def unblockify(self, B):
        """Inverse of blockify."""
        bx, by, bz, bt = self.b
        Cx, Cy, Cz, Ct = self.Lc
        lead = B.shape[:-3]
        h = B.shape[-1] // self.vol_b
        g = B.reshape(lead + (Ct, Cz, Cy, Cx, 2, bt, bz, by, bx, h))
        k = len(lead)
        perm = list(range(k)) + [k + 0, k + 5, k + 1, k + 6, k + 2, k + 7, k + 3, k + 8, k + 4, k + 9]
        g = np.transpose(g, perm)
        Lx, Ly, Lz, Lt = self.L
        return g.reshape(lead + (Lt, Lz, Ly, Lx, 2 * h))


def fine_to_generic(psi):
    """[..., t, z, y, x, 4, 3] -> [..., t, z, y, x, 12] (component 3s + c)."""
    return psi.reshape(psi.shape[:-2] + (12,))


def generic_to_fine(f):
    return f.reshape(f.shape[:-1] + (4, 3))


def block_qr(B):
    """Per-block QR of B[Vc, 2, rows, Nv] by modified Gram-Schmidt applied twice.

    Returns (Q, R) with Q[Vc, 2, rows, Nv] having orthonormal columns per
    block and R[Vc, 2, Nv, Nv] upper triangular with a positive real
    diagonal, B = Q R (Eq. 4: P^dag P = I, P V_c = V).
    Raises ValueError if a block is rank deficient.
    """
    B = np.array(B, dtype=np.complex128, copy=True)
    nb, two, rows, nv = B.shape
    Q = np.zeros_like(B)
    R = np.zeros((nb, two, nv, nv), dtype=np.complex128)
    for k in range(nv):
        v = B[..., k].copy()
        n0 = np.sqrt(np.sum(np.abs(v) ** 2, axis=-1))
        for _sweep in range(2):
            for j in range(k):
                c = np.sum(np.conj(Q[..., j]) * v, axis=-1)
                v = v - c[..., None] * Q[..., j]
                R[..., j, k] += c
        r = np.sqrt(np.sum(np.abs(v) ** 2, axis=-1))
        if np.any(r < 1e-14 * n0) or np.any(r == 0):
            raise ValueError("rank-deficient aggregate in block QR")
        Q[..., k] = v / r[..., None]
        R[..., k, k] = r
    return Q, R


def restrict(Pb, geom: BlockGeometry, f):
    """R f = P^dag f:  rc[..., x_c, chi*Nv + k] = sum_row conj(P[x_c,chi][row,k]) f_blk[x_c,chi][row]."""
    B = geom.blockify(f)
    rc = np.einsum("cxrk,...cxr->...cxk", np.conj(Pb), B)
    Cx, Cy, Cz, Ct = geom.Lc
    nv = Pb.shape[-1]
    return rc.reshape(rc.shape[:-3] + (Ct, Cz, Cy, Cx, 2 * nv))


def prolong(Pb, geom: BlockGeometry, ec):
    """P e_c:  f_blk[x_c,chi][row] = sum_k P[x_c,chi][row,k] e_c[x_c, chi*Nv + k]."""
    nv = Pb.shape[-1]
    lead = ec.shape[:-5]
    e = ec.reshape(lead + (geom.Vc, 2, nv))
    B = np.einsum("cxrk,...cxk->...cxr", Pb, e)
    return geom.unblockify(B)


def P_dense(Pb, geom: BlockGeometry):
    """Dense P (fine generic index (site, comp) x coarse index (site_c, comp_c))."""
    nv = Pb.shape[-1]
    nc = geom.Vc * 2 * nv
    Cx, Cy, Cz, Ct = geom.Lc
    eye = np.eye(nc, dtype=np.complex128).reshape(nc, Ct, Cz, Cy, Cx, 2 * nv)
    cols = prolong(Pb, geom, eye)
    return cols.reshape(nc, -1).T.copy()
