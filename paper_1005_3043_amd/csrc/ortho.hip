// Block orthonormalisation of the null-space candidates (Eq. 4): per
// (aggregate, chirality) block B = Q R with Q having orthonormal columns and
// R upper triangular with a positive real diagonal (this fixes Q uniquely).
// Modified Gram-Schmidt applied twice, in place, FP64.
//
// One workgroup per aggregate handles both chirality halves: each thread
// keeps its site's (fine) or elements' (coarse) part of the current column
// (fine: of the current block of columns) in registers; each projection coefficient is a block reduction (wavefront
// shuffles, then a fixed-order sum of the per-wave partials in LDS that every
// thread evaluates identically).
#include "kernels.h"

namespace mg {

// Sum of W doubles over the workgroup, result in every thread.
template <int W> __device__ __forceinline__ void block_allsum(double (&v)[W], double (*lds)[W]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < W; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < W; ++i) lds[w][i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < W; ++i) {
    double a = lds[0][i];
    for (int q = 1; q < nw; ++q) a += lds[q][i];
    v[i] = a;
  }
  __syncthreads();
}

constexpr double RANK_TOL = 1e-14;

// Fine level: V[k][fidx(s, c)], aggregate of vb <= 256 sites, comps 0..5 =
// chirality 0, 6..11 = chirality 1.  The columns are taken in blocks of BK: a
// block is held in registers and projected against every earlier column
// (twice), one load of that column and one reduction of 4 BK coefficients
// for the whole block, then orthonormalised within itself (Gram-Schmidt
// twice).  Each earlier column is read once per block instead of once per
// column, so the aggregate's columns, which do not stay in L2 between
// reads, move BK times fewer bytes.  The factor Q is the same.  On 32^3 x 64
// with Nv = 24: 42.9 ms with BK = 1 (column by column),
// 22.2 ms with BK = 2 (228 registers, two waves per SIMD), 32.8 ms with
// BK = 4 (one wave per SIMD).
#ifndef MG_ORTHO_BK
#define MG_ORTHO_BK 2
#endif
constexpr int OF_BK = MG_ORTHO_BK;
__global__ __launch_bounds__(256) void k_ortho_fine_blk(Geom g, int nv, double2 *__restrict__ V, int *flag) {
  constexpr int BK = OF_BK;
  __shared__ double lds[4][4 * BK];
  __shared__ double lds4[4][4];
  const size_t Vn = g.Vpad;
  const uint32_t t = threadIdx.x;
  const bool act = t < g.vb;
  const uint32_t s = blockIdx.x * g.vb + (act ? t : 0);
  for (int kb = 0; kb < nv; kb += BK) {
    const int nb = nv - kb < BK ? nv - kb : BK;
    double2 v[BK][12];
#pragma unroll
    for (int b = 0; b < BK; ++b) {
      const double2 *Vk = V + (size_t)(kb + b) * 12 * Vn;
#pragma unroll
      for (int c = 0; c < 12; ++c) v[b][c] = (act && b < nb) ? Vk[fidx(s, c, 12)] : make_double2(0, 0);
    }
    double n0[4 * BK];
#pragma unroll
    for (int b = 0; b < BK; ++b) {
      n0[4 * b] = n0[4 * b + 1] = n0[4 * b + 2] = n0[4 * b + 3] = 0.0;
#pragma unroll
      for (int c = 0; c < 12; ++c) n0[4 * b + c / 6] += v[b][c].x * v[b][c].x + v[b][c].y * v[b][c].y;
    }
    block_allsum<4 * BK>(n0, lds);
    for (int sweep = 0; sweep < 2; ++sweep) {
      for (int j = 0; j < kb; ++j) {
        const double2 *Vj = V + (size_t)j * 12 * Vn;
        double2 q[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) q[c] = act ? Vj[fidx(s, c, 12)] : make_double2(0, 0);
        double cc[4 * BK];
#pragma unroll
        for (int b = 0; b < BK; ++b) {
          double2 c0 = make_double2(0, 0), c1 = make_double2(0, 0);
#pragma unroll
          for (int c = 0; c < 6; ++c) c0 = cfmac(q[c], v[b][c], c0);
#pragma unroll
          for (int c = 6; c < 12; ++c) c1 = cfmac(q[c], v[b][c], c1);
          cc[4 * b] = c0.x;
          cc[4 * b + 1] = c0.y;
          cc[4 * b + 2] = c1.x;
          cc[4 * b + 3] = c1.y;
        }
        block_allsum<4 * BK>(cc, lds);
#pragma unroll
        for (int b = 0; b < BK; ++b) {
          const double2 a0 = make_double2(-cc[4 * b], -cc[4 * b + 1]);
          const double2 a1 = make_double2(-cc[4 * b + 2], -cc[4 * b + 3]);
#pragma unroll
          for (int c = 0; c < 6; ++c) v[b][c] = cfma(a0, q[c], v[b][c]);
#pragma unroll
          for (int c = 6; c < 12; ++c) v[b][c] = cfma(a1, q[c], v[b][c]);
        }
      }
    }
    // within the block: column b against the block's columns a < b (already
    // orthonormal), twice, then normalised
#pragma unroll
    for (int b = 0; b < BK; ++b) {
      if (b < nb) {
        for (int sweep = 0; sweep < 2; ++sweep) {
#pragma unroll
          for (int a = 0; a < BK; ++a) {
            if (a < b) {
              double2 c0 = make_double2(0, 0), c1 = make_double2(0, 0);
#pragma unroll
              for (int c = 0; c < 6; ++c) c0 = cfmac(v[a][c], v[b][c], c0);
#pragma unroll
              for (int c = 6; c < 12; ++c) c1 = cfmac(v[a][c], v[b][c], c1);
              double cc[4] = {c0.x, c0.y, c1.x, c1.y};
              block_allsum<4>(cc, lds4);
              const double2 a0 = make_double2(-cc[0], -cc[1]), a1 = make_double2(-cc[2], -cc[3]);
#pragma unroll
              for (int c = 0; c < 6; ++c) v[b][c] = cfma(a0, v[a][c], v[b][c]);
#pragma unroll
              for (int c = 6; c < 12; ++c) v[b][c] = cfma(a1, v[a][c], v[b][c]);
            }
          }
        }
        double nn[4] = {0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < 12; ++c) nn[c / 6] += v[b][c].x * v[b][c].x + v[b][c].y * v[b][c].y;
        block_allsum<4>(nn, lds4);
        const double r0 = sqrt(nn[0]), r1 = sqrt(nn[1]);
        if (t == 0 && (!(r0 > RANK_TOL * sqrt(n0[4 * b])) || !(r1 > RANK_TOL * sqrt(n0[4 * b + 1])))) *flag = 1;
        const double i0 = r0 > 0 ? 1.0 / r0 : 0.0, i1 = r1 > 0 ? 1.0 / r1 : 0.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) v[b][c] = cscale(v[b][c], c < 6 ? i0 : i1);
      }
    }
    if (act) {
#pragma unroll
      for (int b = 0; b < BK; ++b) {
        if (b < nb) {
          double2 *Vk = V + (size_t)(kb + b) * 12 * Vn;
#pragma unroll
          for (int c = 0; c < 12; ++c) Vk[fidx(s, c, 12)] = v[b][c];
        }
      }
    }
    __syncthreads();
  }
}

// Coarse level: V[k][s][j] (site-major), elements e = t * n + j of the
// aggregate (vb * n <= 2048), chirality = (j >= n / 2).
constexpr int OC_EMAX = 8;

__global__ __launch_bounds__(256) void k_ortho_coarse(Geom g, int n, int nv, double2 *__restrict__ V, int *flag) {
  __shared__ double lds[4][4];
  const size_t Vn = g.V;
  const int tid = threadIdx.x;
  const int ne = (int)g.vb * n, half = n >> 1;
  const size_t base = (size_t)blockIdx.x * g.vb * n;
  for (int kk = 0; kk < nv; ++kk) {
    double2 *Vk = V + (size_t)kk * Vn * n + base;
    double2 v[OC_EMAX];
#pragma unroll
    for (int q = 0; q < OC_EMAX; ++q) {
      const int e = tid + q * (int)blockDim.x;
      v[q] = e < ne ? Vk[e] : make_double2(0, 0);
    }
    double n0[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < OC_EMAX; ++q) {
      const int e = tid + q * (int)blockDim.x;
      n0[(e % n) < half ? 0 : 1] += v[q].x * v[q].x + v[q].y * v[q].y;
    }
    block_allsum<4>(n0, lds);
    for (int sweep = 0; sweep < 2; ++sweep) {
      for (int j = 0; j < kk; ++j) {
        const double2 *Vj = V + (size_t)j * Vn * n + base;
        double2 qv[OC_EMAX];
        double2 c0 = make_double2(0, 0), c1 = make_double2(0, 0);
#pragma unroll
        for (int q = 0; q < OC_EMAX; ++q) {
          const int e = tid + q * (int)blockDim.x;
          qv[q] = e < ne ? Vj[e] : make_double2(0, 0);
          if ((e % n) < half) c0 = cfmac(qv[q], v[q], c0);
          else c1 = cfmac(qv[q], v[q], c1);
        }
        double cc[4] = {c0.x, c0.y, c1.x, c1.y};
        block_allsum<4>(cc, lds);
        const double2 a0 = make_double2(-cc[0], -cc[1]), a1 = make_double2(-cc[2], -cc[3]);
#pragma unroll
        for (int q = 0; q < OC_EMAX; ++q) {
          const int e = tid + q * (int)blockDim.x;
          v[q] = cfma((e % n) < half ? a0 : a1, qv[q], v[q]);
        }
      }
    }
    double nn[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < OC_EMAX; ++q) {
      const int e = tid + q * (int)blockDim.x;
      nn[(e % n) < half ? 0 : 1] += v[q].x * v[q].x + v[q].y * v[q].y;
    }
    block_allsum<4>(nn, lds);
    const double r0 = sqrt(nn[0]), r1 = sqrt(nn[1]);
    if (tid == 0 && (!(r0 > RANK_TOL * sqrt(n0[0])) || !(r1 > RANK_TOL * sqrt(n0[1])))) *flag = 1;
    const double i0 = r0 > 0 ? 1.0 / r0 : 0.0, i1 = r1 > 0 ? 1.0 / r1 : 0.0;
#pragma unroll
    for (int q = 0; q < OC_EMAX; ++q) {
      const int e = tid + q * (int)blockDim.x;
      if (e < ne) Vk[e] = cscale(v[q], (e % n) < half ? i0 : i1);
    }
    __syncthreads();
  }
}

hipError_t ortho_fine(const Geom &g, int nv, double2 *V, int *flag, hipStream_t st) {
  const int th = (int)((g.vb + 63) / 64 * 64);
  hipLaunchKernelGGL(k_ortho_fine_blk, dim3(g.Vc), dim3(th), 0, st, g, nv, V, flag);
  return hipGetLastError();
}

hipError_t ortho_coarse(const Geom &g, int n, int nv, double2 *V, int *flag, hipStream_t st) {
  hipLaunchKernelGGL(k_ortho_coarse, dim3(g.Vc), dim3(256), 0, st, g, n, nv, V, flag);
  return hipGetLastError();
}

}  // namespace mg
