"""Oracle: learned proposal of near-null vectors by a gauge-equivariant network
of parallel-transport convolutions (PTC), an extension of the adaptive setup.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper relaxes random vectors on D x = 0 to find the near-null space
("Adaptive Multigrid", setup stage one in "Numerical Results").  The extension
replaces the random start vectors with vectors proposed by a small network
that maps a noise spinor and the links to candidate vectors; the plain
relaxation still runs after it and remains the fallback.  The paper says
nothing about such a network, so every convention here is a reading:

  * hop operators T_k, k = 0..8: T_0 = 1; for k = 1 + 2 mu + dir,
      dir 0:  (T_k psi)(x) = eta U_mu(x) psi(x + mu)
      dir 1:  (T_k psi)(x) = eta U_mu(x - mu)^dag psi(x - mu)
    with eta = -1 on hops across the antiperiodic time boundary (the same
    parallel transport as the hopping term of Eq. 2, without the spin
    projector).  T_{+mu}^dag = T_{-mu}, so every T_k^dag is another T_k';
  * a layer maps channels b to channels a:
      out_a(x) = sum_{b, k} W_{a b k} (T_k in_b)(x)
    with W_{a b k} a complex 4x4 matrix on the spin index (identity on
    colour); no nonlinearity;
  * the network: psi1 = layer(W1, eta) (1 -> 8 channels),
    Y = layer(W2, psi1) (8 -> n_out channels);
  * the training loss is the per-block subspace fit of target vectors v_i
    (the null vectors found by the plain setup), over the chirality-split
    aggregates on which the prolongator is built (Eq. 4):
      L = sum_blocks sum_i || v_ib - Y_b c_ib ||^2 / sum_i || v_i ||^2,
      c_ib = (Y_b^dag Y_b)^{-1} Y_b^dag v_ib;
  * gradients are g = dL/dRe(z) + i dL/dIm(z) = 2 dL/dconj(z).  Because c
    minimises the fit, dL/dconj(Y_b) = -E_b C_b^dag / Z (E the fit
    residuals, C the coefficients, Z = sum ||v_i||^2), and through a layer
      dL/dconj(in_b) = sum_{a,k} T_k^dag W_abk^dag dL/dconj(out_a),
      dL/dconj(W_abk)[s, t] = sum_{x, c} dL/dconj(out_a)(x)[s, c]
                              * conj((T_k in_b)(x)[t, c]);
  * Adam on the real and imaginary parts (learning rate 1e-3, betas
    0.9 / 0.999, eps 1e-8).

Array layouts: fields [channel, t, z, y, x, 4, 3]; weights
[c_out, c_in, 9, 4, 4] complex; links U[mu, t, z, y, x, 3, 3].
"""
from __future__ import annotations

import numpy as np

from . import transfer as tr
from . import wilson as wi

N_HOPS = 9


def _spin_mat(G, psi):
    """out[..., s, c] = sum_t G[s, t] psi[..., t, c] (G may be any 4x4)."""
    return np.einsum("st,...tc->...sc", G, psi)


def transport(U, psi, k: int, antiperiodic_t: bool = True):
    """(T_k psi): identity for k = 0, else the parallel transport of a hop."""
    if k == 0:
        return psi.copy()
    mu, back = (k - 1) // 2, (k - 1) % 2 == 1
    L = wi.dims_of(U.shape[1:5])
    ax = wi.SITE_AXIS[mu]
    if not back:
        t = wi._colour(U[mu], np.roll(psi, -1, axis=ax))
    else:
        Ub = np.roll(U[mu], +1, axis=ax)
        t = wi._colour_dag(Ub, np.roll(psi, +1, axis=ax))
    return wi.bc_phase(L, mu, not back, antiperiodic_t) * t


def adjoint_hop(k: int) -> int:
    """Index k' with T_k^dag = T_k'."""
    if k == 0:
        return 0
    return k + 1 if (k - 1) % 2 == 0 else k - 1


def layer(W, U, x):
    """out_a = sum_{b,k} W[a,b,k] (T_k x_b);  x [C_in, ...], out [C_out, ...]."""
    cout, cin = W.shape[:2]
    out = np.zeros((cout,) + x.shape[1:], dtype=np.complex128)
    for b in range(cin):
        for k in range(N_HOPS):
            h = transport(U, x[b], k)
            for a in range(cout):
                out[a] += _spin_mat(W[a, b, k], h)
    return out


def layer_backward(W, U, x, g_out):
    """Gradients of a layer: (g_in, g_W) from g_out = 2 dL/dconj(out)."""
    cout, cin = W.shape[:2]
    g_in = np.zeros_like(x)
    g_W = np.zeros_like(W)
    for b in range(cin):
        for k in range(N_HOPS):
            h = transport(U, x[b], k)
            acc = np.zeros_like(x[b])
            for a in range(cout):
                g_W[a, b, k] = np.einsum("xsc,xtc->st", g_out[a].reshape(-1, 4, 3), np.conj(h).reshape(-1, 4, 3))
                acc += _spin_mat(W[a, b, k].conj().T, g_out[a])
            g_in[b] += transport(U, acc, adjoint_hop(k))
    return g_in, g_W


def forward(W1, W2, U, eta):
    """(psi1, Y) for a noise field eta [..., 4, 3] (one channel)."""
    psi1 = layer(W1, U, eta[None])
    return psi1, layer(W2, U, psi1)


def block_fit(geom: tr.BlockGeometry, Y, V):
    """Subspace fit of V by Y per chirality-split aggregate.

    Returns (loss, g_Y) with g_Y = 2 dL/dconj(Y) (same layout as Y).
    """
    YB = geom.blockify(tr.fine_to_generic(Y))   # [nY, Vc, 2, rows]
    VB = geom.blockify(tr.fine_to_generic(V))   # [nV, Vc, 2, rows]
    Ym = np.moveaxis(YB, 0, -1)                 # [Vc, 2, rows, nY]
    Vm = np.moveaxis(VB, 0, -1)                 # [Vc, 2, rows, nV]
    G = np.einsum("cxri,cxrj->cxij", np.conj(Ym), Ym)
    R = np.einsum("cxri,cxrj->cxij", np.conj(Ym), Vm)
    C = np.linalg.solve(G, R)                   # [Vc, 2, nY, nV]
    E = Vm - np.einsum("cxri,cxij->cxrj", Ym, C)
    Z = float(np.sum(np.abs(V) ** 2))
    loss = float(np.sum(np.abs(E) ** 2)) / Z
    gYm = -2.0 * np.einsum("cxrj,cxij->cxri", E, np.conj(C)) / Z
    gY = tr.generic_to_fine(geom.unblockify(np.moveaxis(gYm, -1, 0)))
    return loss, gY


def loss_and_grad(W1, W2, U, eta, V, geom: tr.BlockGeometry):
    """Loss of the proposal against targets V and its weight gradients."""
    psi1, Y = forward(W1, W2, U, eta)
    loss, gY = block_fit(geom, Y, V)
    g_psi1, gW2 = layer_backward(W2, U, psi1, gY)
    _, gW1 = layer_backward(W1, U, eta[None], g_psi1)
    return loss, gW1, gW2


class Adam:
    """Adam on complex parameters, real and imaginary parts separately."""

    def __init__(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = None
        self.v = None

    def step(self, params, grads):
        if self.m is None:
            self.m = [np.zeros_like(p) for p in params]
            self.v = [np.zeros((2,) + p.shape) for p in params]
        self.t += 1
        out = []
        for i, (p, g) in enumerate(zip(params, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            gr = np.stack([g.real, g.imag])
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * gr * gr
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            step = (mh.real / (np.sqrt(vh[0]) + self.eps)) + 1j * (mh.imag / (np.sqrt(vh[1]) + self.eps))
            out.append(p - self.lr * step)
        return out
