// Restriction R = P^dag and prolongation P through the block-orthonormalised,
// chirality-split prolongator (P^dag gamma_5 = sigma_3 P^dag, so R = P^dag;
// Eq. 8 with the gamma_5 factors cancelled).
//
// Fine level: P is held as the Nv orthonormalised null-vector fields in the
// fine layout [Nv][12 * Vpad]; column (chi, k) of P on aggregate B is field k
// restricted to the spin half chi (components 6 chi .. 6 chi + 5) on the
// sites of B.  With the site-blocked order the sites of one aggregate are a
// contiguous run of tiles, so a workgroup per aggregate streams P and the
// residual with fully coalesced loads and reduces 2 Nv inner products.
// Coarse level l -> l+1: vectors are site-major [V][n]; P is [Nv][V][n] and
// chirality is the upper / lower half of the n components (sigma_3).
#include "kernels.h"

namespace mg {

// Coarse lexicographic coordinates of the aggregate holding fine site s,
// mapped to the site-blocked index of the coarse level.
__device__ __forceinline__ uint32_t coarse_index(const Geom &g, const Geom &gc, uint32_t s) {
  const Coords k = decode(g, s);
  return encode(gc, k.c);
}

// ------------------------------------------------------------------ fine
// The fine vectors are stored as TF: c_t<R>, or binary16 with a per-site
// scale (h16, R = float).
template <typename R, typename S, typename TF>
__global__ __launch_bounds__(256) void k_restrict_fine(Geom g, Geom gc, int nv, const S *__restrict__ P,
                                                       const TF *__restrict__ fine, c_t<R> *__restrict__ coarse) {
  using C = c_t<R>;
  __shared__ double2 part[4][2 * COARSE_NMAX];
  const size_t V = g.Vpad;
  const uint32_t B = blockIdx.x;
  fine += (size_t)blockIdx.y * site_slots<TF>() * V;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int k = lane; k < 2 * nv; k += 64) part[w][k] = make_double2(0.0, 0.0);
  __syncthreads();
  for (uint32_t t0 = 0; t0 < g.vb; t0 += blockDim.x) {
    const uint32_t t = t0 + tid;
    const bool act = t < g.vb;
    const uint32_t s = B * g.vb + (act ? t : 0);
    C r[12];
    load_site(r, fine, s);
    if (!act) {
#pragma unroll
      for (int c = 0; c < 12; ++c) r[c] = mk<C>(0, 0);
    }
    for (int kk = 0; kk < nv; ++kk) {
      const S *Pk = P + (size_t)kk * 12 * V;
      C d0 = mk<C>(0, 0), d1 = mk<C>(0, 0);
      if (act) {
#pragma unroll
        for (int c = 0; c < 6; ++c) d0 = cfmac(cvt<C>(Pk[fidx(s, c, 12)]), r[c], d0);
#pragma unroll
        for (int c = 6; c < 12; ++c) d1 = cfmac(cvt<C>(Pk[fidx(s, c, 12)]), r[c], d1);
      }
      double a0 = wave_sum((double)d0.x), b0 = wave_sum((double)d0.y);
      double a1 = wave_sum((double)d1.x), b1 = wave_sum((double)d1.y);
      if (lane == 0) {
        part[w][kk].x += a0;
        part[w][kk].y += b0;
        part[w][nv + kk].x += a1;
        part[w][nv + kk].y += b1;
      }
    }
  }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  uint32_t ic = 0;
  if (tid < 2 * nv) {
    const int x[4] = {(int)(B % gc.L[0]), (int)((B / gc.L[0]) % gc.L[1]),
                      (int)((B / (gc.L[0] * gc.L[1])) % gc.L[2]), (int)(B / (gc.L[0] * gc.L[1] * gc.L[2]))};
    ic = encode(gc, x);
    double2 a = part[0][tid];
    for (int q = 1; q < nw; ++q) {
      a.x += part[q][tid].x;
      a.y += part[q][tid].y;
    }
    coarse[((size_t)blockIdx.y * gc.V + ic) * (2 * nv) + tid] = mk<C>((R)a.x, (R)a.y);
  }
}

template <typename R, typename S>
__global__ __launch_bounds__(256) void k_prolong_fine(Geom g, Geom gc, int nv, const S *__restrict__ P,
                                                      const c_t<R> *__restrict__ coarse, c_t<R> *__restrict__ fine,
                                                      int accumulate) {
  using C = c_t<R>;
  const size_t V = g.Vpad;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  fine += (size_t)blockIdx.y * 12 * V;
  const uint32_t ic = coarse_index(g, gc, s);
  const C *ec = coarse + ((size_t)blockIdx.y * gc.V + ic) * (2 * nv);
  C acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = mk<C>(0, 0);
  for (int kk = 0; kk < nv; ++kk) {
    const S *Pk = P + (size_t)kk * 12 * V;
    const C e0 = ec[kk], e1 = ec[nv + kk];
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] = cfma(cvt<C>(Pk[fidx(s, c, 12)]), e0, acc[c]);
#pragma unroll
    for (int c = 6; c < 12; ++c) acc[c] = cfma(cvt<C>(Pk[fidx(s, c, 12)]), e1, acc[c]);
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    C v = acc[c];
    if (accumulate) v = cadd(fine[fidx(s, c, 12)], v);
    fine[fidx(s, c, 12)] = v;
  }
}

// Several right-hand sides per workgroup (TR_RG of them): every null-vector
// entry loaded from memory serves TR_RG vectors instead of one.
constexpr int TR_RG = 4;

template <typename R, typename S, typename TF>
__global__ __launch_bounds__(256) void k_restrict_fine_mrhs(Geom g, Geom gc, int nv, int nrhs,
                                                            const S *__restrict__ P, const TF *__restrict__ fine,
                                                            c_t<R> *__restrict__ coarse) {
  using C = c_t<R>;
  __shared__ double2 part[4][TR_RG][2 * COARSE_NMAX];
  const size_t V = g.Vpad;
  const uint32_t B = blockIdx.x;
  const int r0 = blockIdx.y * TR_RG;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int k = lane; k < 2 * nv; k += 64)
#pragma unroll
    for (int q = 0; q < TR_RG; ++q) part[w][q][k] = make_double2(0.0, 0.0);
  __syncthreads();
  for (uint32_t t0 = 0; t0 < g.vb; t0 += blockDim.x) {
    const uint32_t t = t0 + tid;
    const bool act = t < g.vb;
    const uint32_t s = B * g.vb + (act ? t : 0);
    C f[TR_RG][12];
#pragma unroll
    for (int q = 0; q < TR_RG; ++q) {
      const bool on = act && r0 + q < nrhs;
      load_site(f[q], fine + (size_t)(on ? r0 + q : 0) * site_slots<TF>() * V, s);
      if (!on) {
#pragma unroll
        for (int c = 0; c < 12; ++c) f[q][c] = mk<C>(0, 0);
      }
    }
    for (int kk = 0; kk < nv; ++kk) {
      const S *Pk = P + (size_t)kk * 12 * V;
      C pk[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) pk[c] = act ? cvt<C>(Pk[fidx(s, c, 12)]) : mk<C>(0, 0);
#pragma unroll
      for (int q = 0; q < TR_RG; ++q) {
        C d0 = mk<C>(0, 0), d1 = mk<C>(0, 0);
#pragma unroll
        for (int c = 0; c < 6; ++c) d0 = cfmac(pk[c], f[q][c], d0);
#pragma unroll
        for (int c = 6; c < 12; ++c) d1 = cfmac(pk[c], f[q][c], d1);
        const double a0 = wave_sum((double)d0.x), b0 = wave_sum((double)d0.y);
        const double a1 = wave_sum((double)d1.x), b1 = wave_sum((double)d1.y);
        if (lane == 0) {
          part[w][q][kk].x += a0;
          part[w][q][kk].y += b0;
          part[w][q][nv + kk].x += a1;
          part[w][q][nv + kk].y += b1;
        }
      }
    }
  }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  for (int o = tid; o < TR_RG * 2 * nv; o += blockDim.x) {
    const int q = o / (2 * nv), k = o % (2 * nv);
    if (r0 + q >= nrhs) continue;
    const int x[4] = {(int)(B % gc.L[0]), (int)((B / gc.L[0]) % gc.L[1]),
                      (int)((B / (gc.L[0] * gc.L[1])) % gc.L[2]), (int)(B / (gc.L[0] * gc.L[1] * gc.L[2]))};
    const uint32_t ic = encode(gc, x);
    double2 a = part[0][q][k];
    for (int qq = 1; qq < nw; ++qq) {
      a.x += part[qq][q][k].x;
      a.y += part[qq][q][k].y;
    }
    coarse[((size_t)(r0 + q) * gc.V + ic) * (2 * nv) + k] = mk<C>((R)a.x, (R)a.y);
  }
}

template <typename R, typename S>
__global__ __launch_bounds__(256) void k_prolong_fine_mrhs(Geom g, Geom gc, int nv, int nrhs,
                                                           const S *__restrict__ P, const c_t<R> *__restrict__ coarse,
                                                           c_t<R> *__restrict__ fine, int accumulate) {
  using C = c_t<R>;
  const size_t V = g.Vpad;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int r0 = blockIdx.y * TR_RG;
  const uint32_t ic = coarse_index(g, gc, s);
  C acc[TR_RG][12];
#pragma unroll
  for (int q = 0; q < TR_RG; ++q)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[q][c] = mk<C>(0, 0);
  for (int kk = 0; kk < nv; ++kk) {
    const S *Pk = P + (size_t)kk * 12 * V;
    C pk[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) pk[c] = cvt<C>(Pk[fidx(s, c, 12)]);
#pragma unroll
    for (int q = 0; q < TR_RG; ++q) {
      const int r = min(r0 + q, nrhs - 1);
      const C *ec = coarse + ((size_t)r * gc.V + ic) * (2 * nv);
      const C e0 = ec[kk], e1 = ec[nv + kk];
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[q][c] = cfma(pk[c], e0, acc[q][c]);
#pragma unroll
      for (int c = 6; c < 12; ++c) acc[q][c] = cfma(pk[c], e1, acc[q][c]);
    }
  }
#pragma unroll
  for (int q = 0; q < TR_RG; ++q) {
    if (r0 + q >= nrhs) break;
    C *fr = fine + (size_t)(r0 + q) * 12 * V;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      C v = acc[q][c];
      if (accumulate) v = cadd(fr[fidx(s, c, 12)], v);
      fr[fidx(s, c, 12)] = v;
    }
  }
}

template <typename R, typename S, typename TF>
hipError_t restrict_fine(const Geom &g, const Geom &gc, int nv, const S *P, const TF *fine, c_t<R> *coarse,
                         int nrhs, hipStream_t st) {
  const int th = g.vb >= 256 ? 256 : (int)((g.vb + 63) / 64 * 64);
  if (nrhs > 1)
    hipLaunchKernelGGL((k_restrict_fine_mrhs<R, S, TF>), dim3(g.Vc, (nrhs + TR_RG - 1) / TR_RG), dim3(th), 0, st, g,
                       gc, nv, nrhs, P, fine, coarse);
  else
    hipLaunchKernelGGL((k_restrict_fine<R, S, TF>), dim3(g.Vc, nrhs), dim3(th), 0, st, g, gc, nv, P, fine, coarse);
  return hipGetLastError();
}

template <typename R, typename S>
hipError_t prolong_fine(const Geom &g, const Geom &gc, int nv, const S *P, const c_t<R> *coarse, c_t<R> *fine,
                        int nrhs, int accumulate, hipStream_t st) {
  if (nrhs > 1)
    hipLaunchKernelGGL((k_prolong_fine_mrhs<R, S>), dim3(div_up(g.V, 256), (nrhs + TR_RG - 1) / TR_RG), dim3(256), 0,
                       st, g, gc, nv, nrhs, P, coarse, fine, accumulate);
  else
    hipLaunchKernelGGL((k_prolong_fine<R, S>), dim3(div_up(g.V, 256), nrhs), dim3(256), 0, st, g, gc, nv, P, coarse,
                       fine, accumulate);
  return hipGetLastError();
}

// ------------------------------------------------------------------ coarse
// Elements of aggregate B: e = t * n + j (site t of the block, component j),
// contiguous in the site-major layout.  Chirality of j: j >= n/2.
constexpr int RC_EMAX = 8;  // elements per thread (block volume * n <= 2048)

template <typename R, typename S>
__global__ __launch_bounds__(256) void k_restrict_coarse(Geom g, Geom gc, int n, int nv,
                                                         const S *__restrict__ P, const c_t<R> *__restrict__ fine,
                                                         c_t<R> *__restrict__ coarse) {
  using C = c_t<R>;
  __shared__ double2 part[4][2 * COARSE_NMAX];
  const uint32_t B = blockIdx.x;
  const size_t V = g.V;
  fine += (size_t)blockIdx.y * V * n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ne = (int)g.vb * n;
  const size_t base = (size_t)B * g.vb * n;
  C r[RC_EMAX];
#pragma unroll
  for (int q = 0; q < RC_EMAX; ++q) {
    const int e = tid + q * (int)blockDim.x;
    r[q] = e < ne ? fine[base + e] : mk<C>(0, 0);
  }
  const int half = n >> 1;
  for (int kk = 0; kk < nv; ++kk) {
    const S *Pk = P + (size_t)kk * V * n + base;
    C d0 = mk<C>(0, 0), d1 = mk<C>(0, 0);
#pragma unroll
    for (int q = 0; q < RC_EMAX; ++q) {
      const int e = tid + q * (int)blockDim.x;
      if (e < ne) {
        const int j = e % n;
        if (j < half) d0 = cfmac(cvt<C>(Pk[e]), r[q], d0);
        else d1 = cfmac(cvt<C>(Pk[e]), r[q], d1);
      }
    }
    double a0 = wave_sum((double)d0.x), b0 = wave_sum((double)d0.y);
    double a1 = wave_sum((double)d1.x), b1 = wave_sum((double)d1.y);
    if (lane == 0) {
      part[w][kk] = make_double2(a0, b0);
      part[w][nv + kk] = make_double2(a1, b1);
    }
  }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  if (tid < 2 * nv) {
    const int x[4] = {(int)(B % gc.L[0]), (int)((B / gc.L[0]) % gc.L[1]),
                      (int)((B / (gc.L[0] * gc.L[1])) % gc.L[2]), (int)(B / (gc.L[0] * gc.L[1] * gc.L[2]))};
    const uint32_t ic = encode(gc, x);
    double2 a = part[0][tid];
    for (int q = 1; q < nw; ++q) {
      a.x += part[q][tid].x;
      a.y += part[q][tid].y;
    }
    coarse[((size_t)blockIdx.y * gc.V + ic) * (2 * nv) + tid] = mk<C>((R)a.x, (R)a.y);
  }
}

template <typename R, typename S>
__global__ __launch_bounds__(256) void k_prolong_coarse(Geom g, Geom gc, int n, int nv, const S *__restrict__ P,
                                                        const c_t<R> *__restrict__ coarse, c_t<R> *__restrict__ fine,
                                                        int accumulate) {
  using C = c_t<R>;
  const size_t V = g.V;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= V * n) return;
  fine += (size_t)blockIdx.y * V * n;
  const uint32_t s = (uint32_t)(e / n);
  const int j = (int)(e - (size_t)s * n);
  const uint32_t ic = coarse_index(g, gc, s);
  const C *ec = coarse + ((size_t)blockIdx.y * gc.V + ic) * (2 * nv) + (j < (n >> 1) ? 0 : nv);
  C acc = mk<C>(0, 0);
  for (int kk = 0; kk < nv; ++kk) acc = cfma(cvt<C>(P[(size_t)kk * V * n + e]), ec[kk], acc);
  if (accumulate) acc = cadd(fine[e], acc);
  fine[e] = acc;
}

template <typename R, typename S>
hipError_t restrict_coarse(const Geom &g, const Geom &gc, int n, int nv, const S *P, const c_t<R> *fine,
                           c_t<R> *coarse, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_restrict_coarse<R, S>), dim3(g.Vc, nrhs), dim3(256), 0, st, g, gc, n, nv, P, fine, coarse);
  return hipGetLastError();
}

template <typename R, typename S>
hipError_t prolong_coarse(const Geom &g, const Geom &gc, int n, int nv, const S *P, const c_t<R> *coarse,
                          c_t<R> *fine, int nrhs, int accumulate, hipStream_t st) {
  hipLaunchKernelGGL((k_prolong_coarse<R, S>), dim3(div_up((long)g.V * n, 256), nrhs), dim3(256), 0, st, g, gc, n,
                     nv, P, coarse, fine, accumulate);
  return hipGetLastError();
}

#define INST(R, S)                                                                                                \
  template hipError_t restrict_fine<R, S, c_t<R>>(const Geom &, const Geom &, int, const S *, const c_t<R> *,       \
                                                  c_t<R> *, int, hipStream_t);                                      \
  template hipError_t prolong_fine<R, S>(const Geom &, const Geom &, int, const S *, const c_t<R> *, c_t<R> *, int,   \
                                         int, hipStream_t);                                                         \
  template hipError_t restrict_coarse<R, S>(const Geom &, const Geom &, int, int, const S *, const c_t<R> *,          \
                                            c_t<R> *, int, hipStream_t);                                            \
  template hipError_t prolong_coarse<R, S>(const Geom &, const Geom &, int, int, const S *, const c_t<R> *,           \
                                           c_t<R> *, int, int, hipStream_t);
INST(double, double2)
INST(float, float2)
INST(float, chalf)
#undef INST
template hipError_t restrict_fine<float, chalf, h16>(const Geom &, const Geom &, int, const chalf *, const h16 *,
                                                     float2 *, int, hipStream_t);

}  // namespace mg
