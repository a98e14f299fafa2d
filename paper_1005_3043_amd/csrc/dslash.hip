// Fine-level Wilson-Dirac operator, Eq. (2):
//   (D psi)(x) = (4+m) psi(x) - 1/2 sum_mu [ eta (1-gamma_mu) U_mu(x) psi(x+mu)
//                                          + eta (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
// eta = -1 on hops across an antiperiodic time boundary.
//
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^dag, 0]] with A_k = -i sigma_k,
// A_4 = 1.  Each row r of A_mu has one entry i^{a_r} in column p_r, so
// (1 -/+ gamma_mu) psi has rank 2: the upper half is h_r = psi_r -/+ i^{a_r}
// psi_{2+p_r} and the lower half is -/+ A^dag h.  One hop therefore costs
// the projection to h (6 complex), two SU(3) mat-vecs on h and a
// reconstruction by multiplications with +-1, +-i (1320 flops per site for
// all eight hops).
//
// One thread per site of the site-blocked SoA layout: each wavefront reads 64
// consecutive sites of a 4D tile per component plane (coalesced), and the
// neighbour reads of adjacent tiles hit L2 / the last-level cache.
#include "kernels.h"

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

template <typename C>
__host__ __device__ __forceinline__ void load_spinor(C (&psi)[12], const C *__restrict__ in, uint32_t s,
                                                     size_t V) {
#pragma unroll
  for (int k = 0; k < 12; ++k) psi[k] = in[(size_t)k * V + s];
}

template <typename C>
__host__ __device__ __forceinline__ void load_link(C (&u)[9], const C *__restrict__ U, int mu, uint32_t s,
                                                   size_t V) {
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = U[(size_t)(mu * 9 + e) * V + s];
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

// Full stencil at one site: returns D psi at s in `res` and the centre value
// psi(s) in `ctr`.
template <typename C>
__host__ __device__ __forceinline__ void dslash_site(C (&res)[12], C (&ctr)[12], const Geom &g, uint32_t s,
                                                     const C *__restrict__ U, const C *__restrict__ in,
                                                     decltype(C::x) diag) {
  using R = decltype(C::x);
  const size_t V = g.V;
  const Coords k = decode(g, s);
  C acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = mk<C>(0, 0);
  // A rolled loop over the eight hops (wave-uniform branch on mu): the loads
  // of one hop cannot be hoisted above the previous hop's arithmetic, which
  // keeps the FP64 kernel within ~130 registers; other waves hide latency.
#pragma unroll 1
  for (int h = 0; h < 8; ++h) {
    const int mu = h >> 1;
    const bool fwd = (h & 1) == 0;
    C psi[12], u[9];
    R eta = 1;
    uint32_t sn;
    if (fwd) {
      sn = nbr_fwd(g, s, k, mu);
      if (mu == 3 && g.antiperiodic && k.o[3] == g.b[3] - 1 && k.c[3] == g.C[3] - 1) eta = -1;
    } else {
      sn = nbr_bwd(g, s, k, mu);
      if (mu == 3 && g.antiperiodic && k.o[3] == 0 && k.c[3] == 0) eta = -1;
    }
    load_spinor(psi, in, sn, V);
    load_link(u, U, mu, fwd ? s : sn, V);
    if (fwd) hop_dispatch<true>(mu, acc, psi, u, eta);
    else hop_dispatch<false>(mu, acc, psi, u, eta);
  }
  load_spinor(ctr, in, s, V);
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    res[i].x = fma(diag, ctr[i].x, (R)-0.5 * acc[i].x);
    res[i].y = fma(diag, ctr[i].y, (R)-0.5 * acc[i].y);
  }
}

template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_dslash(Geom g, const c_t<R> *__restrict__ U,
                                                const c_t<R> *__restrict__ in, c_t<R> *__restrict__ out,
                                                const c_t<R> *__restrict__ b, R diag,
                                                double *__restrict__ partials) {
  using C = c_t<R>;
  const size_t V = g.V;
  const size_t off = (size_t)blockIdx.y * 12 * V;
  in += off;
  out += off;
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t s = tile * blockDim.x + threadIdx.x;
  double red[3] = {0.0, 0.0, 0.0};
  if (s < g.V) {
    C res[12], ctr[12];
    dslash_site(res, ctr, g, s, U, in, diag);
    if constexpr (MODE == DS_RESID) {
      const C *bb = b + off;
#pragma unroll
      for (int i = 0; i < 12; ++i) res[i] = csub(bb[(size_t)i * V + s], res[i]);
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) out[(size_t)i * V + s] = res[i];
    if constexpr (MODE == DS_MR) {
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        // <q, r> = sum conj(q) r with q = D r, r = centre
        red[0] += (double)res[i].x * ctr[i].x + (double)res[i].y * ctr[i].y;
        red[1] += (double)res[i].x * ctr[i].y - (double)res[i].y * ctr[i].x;
        red[2] += (double)res[i].x * res[i].x + (double)res[i].y * res[i].y;
      }
    }
  }
  if constexpr (MODE == DS_MR) {
    __shared__ double lds[16 * 3];
    block_sum<3>(red, lds);
    if (threadIdx.x == 0) {
      double *p = partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 3;
      p[0] = red[0];
      p[1] = red[1];
      p[2] = red[2];
    }
  }
}

int dslash_blocks(const Geom &g) { return div_up(g.V, 256); }

template <typename R>
hipError_t dslash(const Geom &g, const c_t<R> *U, const c_t<R> *in, c_t<R> *out, const c_t<R> *b,
                  double diag, int nrhs, DslashMode mode, double *partials, hipStream_t st) {
  dim3 grid(dslash_blocks(g), nrhs);
  switch (mode) {
    case DS_PLAIN:
      hipLaunchKernelGGL((k_dslash<R, DS_PLAIN>), grid, dim3(256), 0, st, g, U, in, out, b, (R)diag, partials);
      break;
    case DS_RESID:
      hipLaunchKernelGGL((k_dslash<R, DS_RESID>), grid, dim3(256), 0, st, g, U, in, out, b, (R)diag, partials);
      break;
    case DS_MR:
      hipLaunchKernelGGL((k_dslash<R, DS_MR>), grid, dim3(256), 0, st, g, U, in, out, b, (R)diag, partials);
      break;
  }
  return hipGetLastError();
}

template hipError_t dslash<double>(const Geom &, const double2 *, const double2 *, double2 *, const double2 *,
                                   double, int, DslashMode, double *, hipStream_t);
template hipError_t dslash<float>(const Geom &, const float2 *, const float2 *, float2 *, const float2 *,
                                  double, int, DslashMode, double *, hipStream_t);

}  // namespace mg
