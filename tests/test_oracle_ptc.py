"""Pins of the oracle's parallel-transport network (learned null-vector
proposal): the hop operators against the Wilson operator of Eq. 2, their
adjoints, gauge equivariance, the subspace-fit loss on constructed cases, the
gradients against central finite differences, and the Adam step."""
import numpy as np
import pytest

import workloads as W
from oracle import ptc
from oracle import transfer as tr
from oracle import wilson as wi

L = (4, 2, 2, 4)
BLK = (2, 2, 2, 2)


def _field(seed, batch=()):
    return W.gaussian_spinor(L, seed, batch=batch)


def _ip(a, b):
    return np.vdot(a.ravel(), b.ravel())


def test_transport_adjoints():
    U = W.gauge_field(L, 0.4, 1)
    phi, psi = _field(2), _field(3)
    for k in range(ptc.N_HOPS):
        lhs = _ip(phi, ptc.transport(U, psi, k))
        rhs = _ip(ptc.transport(U, phi, ptc.adjoint_hop(k)), psi)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_layer_reproduces_wilson_operator():
    """A one-channel layer with W_0 = (4+m), W_{+mu} = -(1-gamma_mu)/2 and
    W_{-mu} = -(1+gamma_mu)/2 is exactly D of Eq. 2 (ties the transport,
    its boundary signs and the hop order to the pinned Wilson operator)."""
    U = W.gauge_field(L, 0.4, 4)
    m = -0.3
    Wd = np.zeros((1, 1, ptc.N_HOPS, 4, 4), dtype=np.complex128)
    Wd[0, 0, 0] = (4.0 + m) * np.eye(4)
    for mu in range(4):
        Wd[0, 0, 1 + 2 * mu] = -0.5 * wi.PROJ_MINUS[mu]
        Wd[0, 0, 2 + 2 * mu] = -0.5 * wi.PROJ_PLUS[mu]
    psi = _field(5)
    out = ptc.layer(Wd, U, psi[None])[0]
    ref = wi.apply_D(U, psi, m)
    assert np.linalg.norm(out - ref) < 1e-13 * np.linalg.norm(ref)


def test_gauge_equivariance():
    U = W.gauge_field(L, 0.4, 6)
    g = W.gauge_transform(L, 7)
    Ug = wi.gauge_transform_links(U, g)
    W1, W2 = W.ptc_init_weights(3, 4, 0)
    eta = _field(8)
    _, Y = ptc.forward(W1, W2, U, eta)
    _, Yg = ptc.forward(W1, W2, Ug, wi.gauge_transform_spinor(g, eta))
    ref = np.stack([wi.gauge_transform_spinor(g, y) for y in Y])
    assert np.linalg.norm(Yg - ref) < 1e-12 * np.linalg.norm(ref)


def test_block_fit_cases():
    geom = tr.BlockGeometry(L, BLK)
    rng = np.random.default_rng(9)
    Y = _field(10, batch=(4,))
    YB = np.moveaxis(geom.blockify(tr.fine_to_generic(Y)), 0, -1)  # [Vc,2,rows,4]
    # targets inside the per-block span of Y: zero loss, zero gradient
    C = rng.standard_normal(YB.shape[:2] + (4, 3)) + 1j * rng.standard_normal(YB.shape[:2] + (4, 3))
    VB = np.einsum("cxri,cxij->cxrj", YB, C)
    V = tr.generic_to_fine(geom.unblockify(np.moveaxis(VB, -1, 0)))
    loss, gY = ptc.block_fit(geom, Y, V)
    assert loss < 1e-24 and np.linalg.norm(gY) < 1e-10
    # targets orthogonal to the span in every block: loss exactly 1
    R = rng.standard_normal(YB.shape[:3] + (3,)) + 1j * rng.standard_normal(YB.shape[:3] + (3,))
    Q, _ = np.linalg.qr(YB)
    R = R - np.einsum("cxri,cxsi,cxsj->cxrj", Q, np.conj(Q), R)
    V2 = tr.generic_to_fine(geom.unblockify(np.moveaxis(R, -1, 0)))
    loss2, _ = ptc.block_fit(geom, Y, V2)
    assert abs(loss2 - 1.0) < 1e-12
    # the fit depends on the span only: invariant under channel mixing
    A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    Vr = _field(11, batch=(3,))
    la, _ = ptc.block_fit(geom, Y, Vr)
    lb, _ = ptc.block_fit(geom, np.einsum("ij,j...->i...", A, Y), Vr)
    assert abs(la - lb) < 1e-12 and 0.0 < la < 1.0


@pytest.mark.parametrize("which", ["W1", "W2"])
def test_gradients_finite_differences(which):
    geom = tr.BlockGeometry(L, BLK)
    U = W.gauge_field(L, 0.4, 12)
    W1, W2 = W.ptc_init_weights(2, 4, 1)
    eta = _field(13)
    V = _field(14, batch=(3,))
    loss, g1, g2 = ptc.loss_and_grad(W1, W2, U, eta, V, geom)
    g = g1 if which == "W1" else g2
    rng = np.random.default_rng(15)
    h = 1e-6
    for _ in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in g.shape)
        for unit in (1.0, 1j):
            def f(d):
                A, B = W1.copy(), W2.copy()
                (A if which == "W1" else B)[idx] += d * unit
                return ptc.block_fit(geom, ptc.forward(A, B, U, eta)[1], V)[0]
            fd = (f(h) - f(-h)) / (2 * h)
            an = g[idx].real if unit == 1.0 else g[idx].imag
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (idx, unit, fd, an)


def test_adam_first_step():
    """The first bias-corrected Adam step is lr * sign(g) per real component."""
    p = np.array([1.0 + 2.0j, -1.0 + 0.5j])
    g = np.array([0.3 - 2.0j, -5.0 + 1e-3j])
    opt = ptc.Adam(lr=1e-3)
    (q,) = opt.step([p], [g])
    step = (p - q) / 1e-3
    ref = np.sign(g.real) + 1j * np.sign(g.imag)
    assert np.allclose(step, ref, rtol=1e-4)


@pytest.mark.parametrize("t", [2, 3])
def test_adam_bias_correction_later_steps(t):
    """Bias correction at steps after the first.  With the same gradient g at
    every step, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the corrected
    step is lr g / (|g| + eps) per real component at every t.  With alternating gradients g, -g, g the
    second moment is still (1 - b2^t) g^2 per component while
    m_2 = -(1 - b1)^2 g and m_3 = (1 - b1)(1 - b1 (1 - b1)) g, so the steps
    are -(1 - b1) / (1 + b1) = -0.0526315789... times that at t = 2 and
    0.091 / 0.271 = 0.3357933579... times it at t = 3 (b1 = 0.9)."""
    p0 = np.array([1.0 + 2.0j, -1.0 + 0.5j, 0.25 - 3.0j])
    g = np.array([0.3 - 2.0j, -5.0 + 1e-3j, 7.0 + 0.02j])
    eps = 1e-8
    sg = g.real / (np.abs(g.real) + eps) + 1j * g.imag / (np.abs(g.imag) + eps)
    lr = 1e-3
    for alternate, expect in ((False, {2: 1.0, 3: 1.0}), (True, {2: -0.05263157894736842, 3: 0.33579335793357934})):
        opt = ptc.Adam(lr=lr, eps=eps)
        p = p0
        for k in range(1, t + 1):
            gk = -g if (alternate and k % 2 == 0) else g
            (q,) = opt.step([p], [gk])
            if k == t:
                step = (p - q) / lr
            p = q
        assert np.allclose(step, expect[t] * sg, rtol=1e-9, atol=0)
