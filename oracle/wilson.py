"""Oracle: the Wilson-Dirac operator D(U) of Eq. (2) and its symmetries.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Eq. (2):  D_{x,y} = (4+m) delta_{x,y}
                    - sum_mu [ (1-gamma_mu)/2 U_mu(x) delta_{x+mu,y}
                             + (1+gamma_mu)/2 U_mu(x-mu)^dag delta_{x-mu,y} ].
gamma_5-Hermiticity D^dag = gamma_5 D gamma_5 (Introduction, after Eq. 2).

Readings where the paper is silent:
  * directions mu = 0,1,2,3 = x,y,z,t (the paper's mu = 1..4, time last);
  * chiral gamma basis gamma_k = [[0,-i s_k],[i s_k,0]] (k = 1,2,3),
    gamma_4 = [[0,1],[1,0]], so gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4
    = diag(1,1,-1,-1) and chirality 0 = spins {0,1};
  * periodic in space, antiperiodic in time: a hop that crosses the t
    boundary picks up a factor -1 (links stay SU(3)).
Array layout: psi[..., t, z, y, x, s, c], U[mu, t, z, y, x, a, b].
"""
from __future__ import annotations

import numpy as np

_S1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_S2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_S3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)


def _chiral(A):
    return np.block([[_Z2, A], [A.conj().T, _Z2]])


GAMMA = np.stack([_chiral(-1j * _S1), _chiral(-1j * _S2), _chiral(-1j * _S3), _chiral(_I2)])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)
PROJ_MINUS = np.stack([ID4 - GAMMA[mu] for mu in range(4)])  # (1 - gamma_mu)
PROJ_PLUS = np.stack([ID4 + GAMMA[mu] for mu in range(4)])   # (1 + gamma_mu)

# numpy axis of direction mu in a [..., t, z, y, x, s, c] array
SITE_AXIS = (-3, -4, -5, -6)


def dims_of(psi_or_U_shape_tail):
    """(Lx, Ly, Lz, Lt) from the trailing [t, z, y, x, s, c] shape."""
    Lt, Lz, Ly, Lx = psi_or_U_shape_tail
    return (Lx, Ly, Lz, Lt)


def _colour(U, psi):
    """out[..., s, a] = sum_b U[..., a, b] psi[..., s, b] (site-local)."""
    out = U[..., None, :, 0] * psi[..., :, 0:1]
    for b in range(1, 3):
        out = out + U[..., None, :, b] * psi[..., :, b:b + 1]
    return out


def _colour_dag(U, psi):
    """out[..., s, a] = sum_b conj(U[..., b, a]) psi[..., s, b]."""
    Uc = np.conj(U)
    out = Uc[..., None, 0, :] * psi[..., :, 0:1]
    for b in range(1, 3):
        out = out + Uc[..., None, b, :] * psi[..., :, b:b + 1]
    return out


def _spin(G, psi):
    """out[..., s, c] = sum_t G[s, t] psi[..., t, c] for a 4x4 spin matrix G."""
    out = np.zeros_like(psi)
    for s in range(4):
        for t in range(4):
            if G[s, t] != 0:
                out[..., s, :] += G[s, t] * psi[..., t, :]
    return out


def bc_phase(L, mu: int, forward: bool, antiperiodic_t: bool = True):
    """eta(x) for the hop x -> x +/- mu, as a [t, z, y, x, 1, 1] array of +-1."""
    Lx, Ly, Lz, Lt = L
    eta = np.ones((Lt, Lz, Ly, Lx, 1, 1))
    if mu == 3 and antiperiodic_t:
        if forward:
            eta[Lt - 1] = -1.0
        else:
            eta[0] = -1.0
    return eta


def hop(U, psi, mu: int, forward: bool, antiperiodic_t: bool = True):
    """One direction-split hopping term of Eq. (2), with its -1/2 factor:

      forward : -1/2 eta (1 - gamma_mu) U_mu(x) psi(x + mu)
      backward: -1/2 eta (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
    """
    L = dims_of(U.shape[1:5])
    ax = SITE_AXIS[mu]
    if forward:
        nb = np.roll(psi, -1, axis=ax)
        t = _colour(U[mu], nb)
        t = _spin(PROJ_MINUS[mu], t)
    else:
        nb = np.roll(psi, +1, axis=ax)
        Ub = np.roll(U[mu], +1, axis=ax)  # Ub[x] = U_mu(x - mu)
        t = _colour_dag(Ub, nb)
        t = _spin(PROJ_PLUS[mu], t)
    return -0.5 * bc_phase(L, mu, forward, antiperiodic_t) * t


def apply_D(U, psi, m: float, antiperiodic_t: bool = True):
    """D(U) psi of Eq. (2).  psi may carry leading batch axes."""
    out = (4.0 + m) * psi
    for mu in range(4):
        out = out + hop(U, psi, mu, True, antiperiodic_t)
        out = out + hop(U, psi, mu, False, antiperiodic_t)
    return out


def apply_D_sites(U, psi, m: float, sites, antiperiodic_t: bool = True):
    """(D psi)(x) of Eq. (2) evaluated only at the listed sites, one term at a
    time: sites is an integer array [n, 4] of (x, y, z, t); psi may carry
    leading batch axes.  Returns [..., n, 4, 3].  For checking large lattices
    on a sample of sites."""
    L = dims_of(U.shape[1:5])
    X = np.asarray(sites, dtype=np.int64)
    out = (4.0 + m) * psi[..., X[:, 3], X[:, 2], X[:, 1], X[:, 0], :, :]
    for mu in range(4):
        e = np.zeros(4, dtype=np.int64)
        e[mu] = 1
        Xf = (X + e) % np.array(L)
        Xb = (X - e) % np.array(L)
        etaf = np.ones(len(X))
        etab = np.ones(len(X))
        if mu == 3 and antiperiodic_t:
            etaf[X[:, 3] == L[3] - 1] = -1.0
            etab[X[:, 3] == 0] = -1.0
        Uf = U[mu, X[:, 3], X[:, 2], X[:, 1], X[:, 0]]        # U_mu(x)
        Ub = U[mu, Xb[:, 3], Xb[:, 2], Xb[:, 1], Xb[:, 0]]    # U_mu(x - mu)
        pf = psi[..., Xf[:, 3], Xf[:, 2], Xf[:, 1], Xf[:, 0], :, :]
        pb = psi[..., Xb[:, 3], Xb[:, 2], Xb[:, 1], Xb[:, 0], :, :]
        tf = np.einsum("nab,...nsb->...nsa", Uf, pf)
        tb = np.einsum("nba,...nsb->...nsa", np.conj(Ub), pb)
        tf = np.einsum("st,...ntc->...nsc", PROJ_MINUS[mu], tf)
        tb = np.einsum("st,...ntc->...nsc", PROJ_PLUS[mu], tb)
        out = out - 0.5 * (etaf[:, None, None] * tf + etab[:, None, None] * tb)
    return out


def apply_gamma5(psi):
    return _spin(GAMMA5, psi)


def apply_Ddag(U, psi, m: float, antiperiodic_t: bool = True):
    """D^dag psi = gamma_5 D gamma_5 psi (gamma_5-Hermiticity)."""
    return apply_gamma5(apply_D(U, apply_gamma5(psi), m, antiperiodic_t))


def D_dense(U, m: float, antiperiodic_t: bool = True):
    """Dense matrix of D on a tiny lattice, index (site, s, c) site-major."""
    Lt, Lz, Ly, Lx = U.shape[1:5]
    n = Lt * Lz * Ly * Lx * 12
    eye = np.eye(n, dtype=np.complex128).reshape(n, Lt, Lz, Ly, Lx, 4, 3)
    cols = apply_D(U, eye, m, antiperiodic_t).reshape(n, n)
    return cols.T.copy()


def dot(a, b):
    """<a, b> = sum conj(a) b."""
    return np.vdot(a.ravel(), b.ravel())


def norm(a):
    return float(np.sqrt(np.real(np.vdot(a.ravel(), a.ravel()))))


def gauge_transform_links(U, g):
    """U^g_mu(x) = g(x) U_mu(x) g(x + mu)^dag."""
    out = np.empty_like(U)
    for mu in range(4):
        gn = np.roll(g, -1, axis=SITE_AXIS[mu])  # gn[x] = g(x + mu)
        out[mu] = g @ U[mu] @ np.conj(np.swapaxes(gn, -1, -2))
    return out


def gauge_transform_spinor(g, psi):
    """(g psi)(x) = g(x) psi(x), acting on colour."""
    return _colour(g, psi)
