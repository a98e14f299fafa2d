// Fine-level Wilson-Dirac operator, Eq. (2):
//   (D psi)(x) = (4+m) psi(x) - 1/2 sum_mu [ eta (1-gamma_mu) U_mu(x) psi(x+mu)
//                                          + eta (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
// eta = -1 on hops across an antiperiodic time boundary.
//
// The spin projection (wilson_site.h) reduces each hop to a half spinor and
// two SU(3) mat-vecs: 1320 flops per site for all eight hops.
//
// One thread per site of the site-blocked SoA layout: each wavefront reads 64
// consecutive sites of a 4D tile per component plane (coalesced), and the
// neighbour reads of adjacent tiles hit L2 / the last-level cache.
#include "kernels.h"
#include "wilson_site.h"

namespace mg {

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
