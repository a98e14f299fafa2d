// Site-level pieces of the fine Wilson-Dirac stencil, Eq. (2), shared by the
// stencil kernels and the Galerkin construction.
//
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^dag, 0]] with A_k = -i sigma_k,
// A_4 = 1.  Each row r of A_mu has one entry i^{a_r} in column p_r, so
// (1 -/+ gamma_mu) psi has rank 2: the upper half is h_r = psi_r -/+ i^{a_r}
// psi_{2+p_r} and the lower half is -/+ A^dag h.  One hop therefore costs
// the projection to h (6 complex), two SU(3) mat-vecs on h and a
// reconstruction by multiplications with +-1, +-i.
#pragma once

#include "common.h"

namespace mg {

template <int mu> struct SpinProj;
template <> struct SpinProj<0> { static constexpr int p0 = 1, p1 = 0, a0 = 3, a1 = 3; };
template <> struct SpinProj<1> { static constexpr int p0 = 1, p1 = 0, a0 = 2, a1 = 0; };
template <> struct SpinProj<2> { static constexpr int p0 = 0, p1 = 1, a0 = 3, a1 = 1; };
template <> struct SpinProj<3> { static constexpr int p0 = 0, p1 = 1, a0 = 0, a1 = 0; };

// acc += (1 -/+ gamma_mu) [U or U^dag] psi, eta folded in (fwd: minus sign,
// link U_mu(x); bwd: plus sign, link U_mu(x-mu)^dag).
template <int mu, bool fwd, typename C>
__host__ __device__ __forceinline__ void hop_site(C (&acc)[12], const C (&psi)[12], const C (&u)[9],
                                                  decltype(C::x) eta) {
  using S = SpinProj<mu>;
  constexpr int hs0 = fwd ? (S::a0 + 2) % 4 : S::a0;
  constexpr int hs1 = fwd ? (S::a1 + 2) % 4 : S::a1;
  constexpr int ls0 = fwd ? ((4 - S::a0) % 4 + 2) % 4 : (4 - S::a0) % 4;
  constexpr int ls1 = fwd ? ((4 - S::a1) % 4 + 2) % 4 : (4 - S::a1) % 4;
  C h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h0[c] = cadd(psi[c], mul_ipow<hs0>(psi[(2 + S::p0) * 3 + c]));
    h1[c] = cadd(psi[3 + c], mul_ipow<hs1>(psi[(2 + S::p1) * 3 + c]));
  }
  C w0[3], w1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C s0 = mk<C>(0, 0), s1 = mk<C>(0, 0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if constexpr (fwd) {
        s0 = cfma(u[a * 3 + b], h0[b], s0);
        s1 = cfma(u[a * 3 + b], h1[b], s1);
      } else {
        s0 = cfmac(u[b * 3 + a], h0[b], s0);
        s1 = cfmac(u[b * 3 + a], h1[b], s1);
      }
    }
    if constexpr (mu == 3) {
      s0 = cscale(s0, eta);
      s1 = cscale(s1, eta);
    }
    w0[a] = s0;
    w1[a] = s1;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[c] = cadd(acc[c], w0[c]);
    acc[3 + c] = cadd(acc[3 + c], w1[c]);
    acc[(2 + S::p0) * 3 + c] = cadd(acc[(2 + S::p0) * 3 + c], mul_ipow<ls0>(w0[c]));
    acc[(2 + S::p1) * 3 + c] = cadd(acc[(2 + S::p1) * 3 + c], mul_ipow<ls1>(w1[c]));
  }
}

template <bool fwd, typename C>
__host__ __device__ __forceinline__ void hop_dispatch(int mu, C (&acc)[12], const C (&psi)[12], const C (&u)[9],
                                                      decltype(C::x) eta) {
  switch (mu) {
    case 0: hop_site<0, fwd>(acc, psi, u, eta); break;
    case 1: hop_site<1, fwd>(acc, psi, u, eta); break;
    case 2: hop_site<2, fwd>(acc, psi, u, eta); break;
    default: hop_site<3, fwd>(acc, psi, u, eta); break;
  }
}

}  // namespace mg
