"""Pins of the oracle's Wilson operator (Eq. 2) against closed forms and symmetries.

Free-field spectrum and plane-wave action (closed forms), gamma_5-Hermiticity
(Introduction), gauge covariance, the SU(3) input generator, and the C matvec
used by the Arnoldi mass tuning against the numpy operator.
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import cref, wilson as wi


def test_gamma_algebra():
    G = wi.GAMMA
    for a in range(4):
        assert np.allclose(G[a], G[a].conj().T)
        for b in range(4):
            assert np.allclose(G[a] @ G[b] + G[b] @ G[a], 2 * (a == b) * np.eye(4))
    assert np.allclose(wi.GAMMA5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("L,m", [((4, 2, 2, 4), 0.1), ((2, 2, 2, 6), -0.3), ((4, 4, 2, 2), 0.0)])
def test_free_field_spectrum(L, m):
    """U = 1: eigenvalues m + sum(1 - cos p) +- i sqrt(sum sin^2 p), multiplicity 6,
    p = 2 pi n / L in space, (2n + 1) pi / Lt in time."""
    U = W.unit_gauge_field(L)
    ev = np.linalg.eigvals(wi.D_dense(U, m))
    exp = []
    for n in itertools.product(*[range(l) for l in L]):
        p = [2 * np.pi * n[mu] / L[mu] for mu in range(3)] + [(2 * n[3] + 1) * np.pi / L[3]]
        re = m + sum(1 - np.cos(q) for q in p)
        im = np.sqrt(sum(np.sin(q) ** 2 for q in p))
        exp += [re + 1j * im] * 6 + [re - 1j * im] * 6
    key = lambda z: (round(z.real, 7), round(z.imag, 7))  # noqa: E731
    a = np.array(sorted(ev, key=key))
    b = np.array(sorted(exp, key=key))
    assert np.abs(a - b).max() < 1e-10


def test_plane_wave_action():
    """D (e^{ipx} u) = (m + sum(1 - cos p) + i sum gamma_mu sin p_mu) e^{ipx} u."""
    L = (4, 6, 4, 8)
    m = 0.37
    rng = np.random.default_rng(5)
    n = [1, 5, 3, 2]
    p = [2 * np.pi * n[mu] / L[mu] for mu in range(3)] + [(2 * n[3] + 1) * np.pi / L[3]]
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    t, z, y, x = np.meshgrid(*[np.arange(L[3 - k]) for k in range(4)], indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = phase[..., None, None] * u
    M = (m + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(wi.GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
    expect = phase[..., None, None] * (M @ u)
    got = wi.apply_D(W.unit_gauge_field(L), psi, m)
    assert np.abs(got - expect).max() < 1e-12


def test_gamma5_hermiticity():
    L = (4, 4, 2, 6)
    U = W.gauge_field(L, 0.4, 3)
    phi = W.gaussian_spinor(L, 1)
    psi = W.gaussian_spinor(L, 2)
    lhs = wi.dot(phi, wi.apply_D(U, psi, -0.2))
    rhs = wi.dot(wi.apply_gamma5(wi.apply_D(U, wi.apply_gamma5(phi), -0.2)), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # dense form D^dag = gamma5 D gamma5 on a tiny lattice
    Ls = (2, 2, 2, 4)
    Us = W.gauge_field(Ls, 0.5, 4)
    D = wi.D_dense(Us, 0.1)
    g5 = np.kron(np.eye(32), np.kron(wi.GAMMA5, np.eye(3)))
    assert np.abs(D.conj().T - g5 @ D @ g5).max() < 1e-14


def test_gauge_covariance():
    """D(U^g)(g psi) = g D(U) psi with U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag."""
    L = (4, 2, 4, 4)
    U = W.gauge_field(L, 0.3, 7)
    g = W.gauge_transform(L, 8)
    psi = W.gaussian_spinor(L, 9)
    Ug = wi.gauge_transform_links(U, g)
    lhs = wi.apply_D(Ug, wi.gauge_transform_spinor(g, psi), -0.4)
    rhs = wi.gauge_transform_spinor(g, wi.apply_D(U, psi, -0.4))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_antiperiodic_sign():
    """A constant spinor on U = 1 with periodic time is an exact eigenvector
    with eigenvalue m; with antiperiodic time it is not."""
    L = (2, 2, 2, 4)
    U = W.unit_gauge_field(L)
    psi = np.ones((4, 2, 2, 2, 4, 3), dtype=np.complex128)
    assert np.abs(wi.apply_D(U, psi, 0.3, antiperiodic_t=False) - 0.3 * psi).max() < 1e-14
    out = wi.apply_D(U, psi, 0.3, antiperiodic_t=True)
    assert np.abs(out - 0.3 * psi).max() > 0.1


def test_su3_generator():
    L = (4, 4, 4, 4)
    for eps in (0.05, 0.3):
        U = W.gauge_field(L, eps, 0)
        I = np.eye(3)
        assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - I).max() < 1e-14
        assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # small eps: U = 1 + i eps H + O(eps^2) with H = sum_k a_k lambda_k
    eps = 1e-4
    a = W.rng(0, W.STREAM_GAUGE).standard_normal((4, 4, 4, 4, 4, 8))
    H = np.tensordot(a, W.GELL_MANN, axes=([5], [0]))
    U = W.gauge_field(L, eps, 0)
    assert np.abs(U - np.eye(3) - 1j * eps * H).max() < 50 * eps ** 2


def test_c_matvec_matches_numpy():
    for L, anti in (((4, 4, 2, 6), True), ((3, 2, 4, 2), False)):
        U = W.gauge_field(L, 0.3, 1)
        psi = W.gaussian_spinor(L, 2)
        a = wi.apply_D(U, psi, -0.3, anti)
        b = cref.apply_D(U, psi, -0.3, anti)
        assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


def test_sampled_sites_match_full_operator():
    """The per-site evaluation of Eq. (2) agrees with the full operator at
    every site of a small lattice (both time boundary conditions, a batch of
    two spinors)."""
    L = (4, 6, 2, 8)
    U = W.gauge_field(L, 0.3, 3)
    psi = W.gaussian_spinor(L, 4, batch=(2,))
    sites = np.array([(x, y, z, t) for t in range(L[3]) for z in range(L[2]) for y in range(L[1])
                      for x in range(L[0])])
    for anti in (True, False):
        full = wi.apply_D(U, psi, -0.3, anti)
        part = wi.apply_D_sites(U, psi, -0.3, sites, anti)
        ref = full.reshape(2, -1, 4, 3)
        assert np.abs(part - ref).max() < 1e-14
