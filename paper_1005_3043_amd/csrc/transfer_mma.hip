// Fine-level restriction r_c = P^dag r and prolongation e (+)= P e_c for many
// right-hand sides as complex GEMMs on the FP32 matrix cores (Eq. 4, Eq. 8;
// 16x16x4 MFMA, four real products per complex one).  One workgroup per
// aggregate B serves every right-hand side, so each entry of P is read once
// per application instead of once per group of right-hand sides.  Per
// chirality h the restriction is C = P_h^dag F (M = Nv, N = nrhs,
// K = 6 |B|) and the prolongation F (+)= P_h E (M = 6 |B|, N = nrhs, K = Nv).
// The 6 |B| index runs over (component c' of the spin half, site t of the
// aggregate) with t fastest: four consecutive indices are four consecutive
// sites of one component plane of the tile-interleaved layout (|B| % 4 == 0
// is required).  MFMA lane layouts (16x16x4, FP32): A lane l = (row l % 16,
// k l / 16); B lane l = (k l / 16, column l % 16); C lane l = (rows
// 4 (l / 16) + 0..3, column l % 16).
#include "kernels.h"

namespace mg {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int TM_NR = 16;    // right-hand sides per tile (N of the MFMA)
constexpr int TM_U = 2;      // k-blocks (16 indices each) per load batch of the restriction
constexpr int TM_WAVES = 8;  // wavefronts per workgroup

// Site-blocked coarse index of aggregate B (aggregates are numbered
// lexicographically over the coarse lattice).
__device__ __forceinline__ uint32_t agg_site(const Geom &gc, uint32_t B) {
  const int x[4] = {(int)(B % gc.L[0]), (int)((B / gc.L[0]) % gc.L[1]), (int)((B / (gc.L[0] * gc.L[1])) % gc.L[2]),
                    (int)(B / (gc.L[0] * gc.L[1] * gc.L[2]))};
  return encode(gc, x);
}

// Four consecutive stored entries (16-byte aligned) as FP32 complex.
__device__ __forceinline__ void load4(const chalf *p, float2 (&o)[4]) {
  const chalf4 v = *reinterpret_cast<const chalf4 *>(p);
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q] = cvt<float2>(v.v[q]);
}
__device__ __forceinline__ void load4(const float2 *p, float2 (&o)[4]) {
  const float4 a = reinterpret_cast<const float4 *>(p)[0], b = reinterpret_cast<const float4 *>(p)[1];
  o[0] = make_float2(a.x, a.y);
  o[1] = make_float2(a.z, a.w);
  o[2] = make_float2(b.x, b.y);
  o[3] = make_float2(b.z, b.w);
}

// Component comp of the four consecutive sites s .. s + 3 (s % 4 == 0) of a
// fine vector stored as FP32 complex or as binary16 with per-site scales.
__device__ __forceinline__ void load4_site(const float2 *f, uint32_t s, int comp, float2 (&o)[4]) {
  load4(f + fidx(s, comp, 12), o);
}
__device__ __forceinline__ void load4_site(const h16 *f, uint32_t s, int comp, float2 (&o)[4]) {
  const chalf4 v = *reinterpret_cast<const chalf4 *>(f + fidx(s, comp, 13));
  const float4 m = *reinterpret_cast<const float4 *>(f + fidx(s, 12, 13));
  o[0] = make_float2((float)v.v[0].x * m.x, (float)v.v[0].y * m.x);
  o[1] = make_float2((float)v.v[1].x * m.y, (float)v.v[1].y * m.y);
  o[2] = make_float2((float)v.v[2].x * m.z, (float)v.v[2].y * m.z);
  o[3] = make_float2((float)v.v[3].x * m.w, (float)v.v[3].y * m.w);
}

// Restriction.  Wavefront w = (ks, h): both row tiles (Nv <= 32) of the
// chirality-h output over the k-blocks ks, ks + KS, ... of 16 indices, so
// each fine-vector entry is loaded once per wavefront; the KS partial tiles
// are summed in LDS in a fixed order.  In a k-block, lane (i, kk) loads the
// four consecutive sites 4 kk .. 4 kk + 3 of its row of P (per tile) and of
// its column of the fine vectors in one access each, and the four MFMAs
// u = 0..3 of the block take index 4 kk + u in k-slot kk (the sum over K
// does not depend on the order of its terms).
template <typename S, typename TF>
__global__ __launch_bounds__(64 * TM_WAVES) void k_restrict_fine_mma(Geom g, Geom gc, int nv, int nrhs,
                                                                     const S *__restrict__ P,
                                                                     const TF *__restrict__ fine,
                                                                     float2 *__restrict__ coarse,
                                                                     const TF *__restrict__ qv,
                                                                     const double2 *__restrict__ alpha) {
  constexpr int KS = TM_WAVES / 2;
  __shared__ float red[TM_WAVES - 2][64][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int MT = (nv + 15) >> 4;
  const int h = wv & 1, ks = wv >> 1;
  const uint32_t B = blockIdx.x;
  const size_t V = g.Vpad;
  const int vb = (int)g.vb, Kh = 6 * vb, KB = (Kh + 15) >> 4;
  const int kq = lane >> 4, col = lane & 15;
  const int ar0 = lane & 15, ar1 = 16 + (lane & 15);
  const bool a0_ok = ar0 < nv, a1_ok = MT > 1 && ar1 < nv, col_ok = col < nrhs;
  const S *Pa0 = P + (size_t)(a0_ok ? ar0 : 0) * 12 * V;
  const S *Pa1 = P + (size_t)(a1_ok ? ar1 : 0) * 12 * V;
  const TF *Fb = fine + (size_t)(col_ok ? col : 0) * site_slots<TF>() * V;
  const TF *Qb = qv ? qv + (size_t)(col_ok ? col : 0) * site_slots<TF>() * V : nullptr;
  float2 ma = make_float2(0.f, 0.f);
  if (Qb) {
    const double2 ad = alpha[col_ok ? col : 0];
    ma = make_float2((float)-ad.x, (float)-ad.y);
  }
  const uint32_t s0 = B * (uint32_t)vb;
  const int nb = ks < KB ? (KB - ks + KS - 1) / KS : 0;  // k-blocks of this wavefront
  floatx4 cre0 = {0.f, 0.f, 0.f, 0.f}, cim0 = {0.f, 0.f, 0.f, 0.f};
  floatx4 cre1 = {0.f, 0.f, 0.f, 0.f}, cim1 = {0.f, 0.f, 0.f, 0.f};
  for (int b0 = 0; b0 < nb; b0 += TM_U) {
    float2 av0[TM_U][4], av1[TM_U][4], bv[TM_U][4];
    bool kin[TM_U];
#pragma unroll
    for (int u = 0; u < TM_U; ++u) {
      const int K0 = 16 * (ks + min(b0 + u, nb - 1) * KS) + 4 * kq;
      kin[u] = K0 < Kh;
      const int Kc = kin[u] ? K0 : 0;
      const int cp = Kc / vb, t = Kc - cp * vb;
      const size_t o = fidx(s0 + (uint32_t)t, 6 * h + cp, 12);
      load4(Pa0 + o, av0[u]);
      if (MT > 1) load4(Pa1 + o, av1[u]);
      load4_site(Fb, s0 + (uint32_t)t, 6 * h + cp, bv[u]);
      if (Qb) {
        float2 qq[4];
        load4_site(Qb, s0 + (uint32_t)t, 6 * h + cp, qq);
#pragma unroll
        for (int e = 0; e < 4; ++e) bv[u][e] = cfma(ma, qq[e], bv[u][e]);
      }
    }
#pragma unroll
    for (int u = 0; u < TM_U; ++u) {
      if (b0 + u < nb) {
        const bool bon = col_ok && kin[u];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float2 b = bon ? bv[u][q] : make_float2(0.f, 0.f);
          // conj(P) F: re += a.x b.x + a.y b.y, im += a.x b.y - a.y b.x
          const float2 a = (a0_ok && kin[u]) ? av0[u][q] : make_float2(0.f, 0.f);
          cre0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cre0, 0, 0, 0);
          cre0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, cre0, 0, 0, 0);
          cim0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, cim0, 0, 0, 0);
          cim0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.x, cim0, 0, 0, 0);
          if (MT > 1) {
            const float2 a1 = (a1_ok && kin[u]) ? av1[u][q] : make_float2(0.f, 0.f);
            cre1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, b.x, cre1, 0, 0, 0);
            cre1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.y, b.y, cre1, 0, 0, 0);
            cim1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, b.y, cim1, 0, 0, 0);
            cim1 = __builtin_amdgcn_mfma_f32_16x16x4f32(-a1.y, b.x, cim1, 0, 0, 0);
          }
        }
      }
    }
  }
  if (ks > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      red[wv - 2][lane][v] = cre0[v];
      red[wv - 2][lane][4 + v] = cim0[v];
      red[wv - 2][lane][8 + v] = cre1[v];
      red[wv - 2][lane][12 + v] = cim1[v];
    }
  }
  __syncthreads();
  if (ks == 0) {
    for (int q = 1; q < KS; ++q) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cre0[v] += red[2 * q + h - 2][lane][v];
        cim0[v] += red[2 * q + h - 2][lane][4 + v];
        cre1[v] += red[2 * q + h - 2][lane][8 + v];
        cim1[v] += red[2 * q + h - 2][lane][12 + v];
      }
    }
    const uint32_t ic = agg_site(gc, B);
    float2 *out = coarse + ((size_t)col * gc.V + ic) * (2 * nv) + h * nv;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k0 = 4 * kq + v, k1 = 16 + 4 * kq + v;
      if (col_ok && k0 < nv) out[k0] = make_float2(cre0[v], cim0[v]);
      if (col_ok && MT > 1 && k1 < nv) out[k1] = make_float2(cre1[v], cim1[v]);
    }
  }
}

// Prolongation.  The aggregate's coarse values are staged in LDS; wavefront
// w takes the output row tiles w, w + 8, ... of both chiralities.
template <typename S, typename TR>
__global__ __launch_bounds__(64 * TM_WAVES) void k_prolong_fine_mma(Geom g, Geom gc, int nv, int nrhs,
                                                                    const S *__restrict__ P,
                                                                    const float2 *__restrict__ coarse,
                                                                    float2 *__restrict__ fine, int accumulate,
                                                                    MrqList<TR> rs, int steps,
                                                                    const double2 *__restrict__ alpha) {
  __shared__ float2 eb[COARSE_NMAX][TM_NR];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t B = blockIdx.x;
  const size_t V = g.Vpad;
  const int vb = (int)g.vb, Mh = 6 * vb, MTh = (Mh + 15) >> 4;
  const uint32_t ic = agg_site(gc, B), s0 = B * (uint32_t)vb;
  for (int idx = tid; idx < 2 * nv * TM_NR; idx += blockDim.x) {
    const int j = idx % TM_NR, hk = idx / TM_NR;
    eb[hk][j] = j < nrhs ? coarse[((size_t)j * gc.V + ic) * (2 * nv) + hk] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int kq = lane >> 4, col = lane & 15;
  const bool col_ok = col < nrhs;
  const int nks = (nv + 3) >> 2;
  float2 *Fc = fine + (size_t)(col_ok ? col : 0) * 12 * V;
  for (int tile = wv; tile < 2 * MTh; tile += TM_WAVES) {
    const int h = tile / MTh, mt = tile - h * MTh;
    const int row = mt * 16 + (lane & 15);
    const bool row_ok = row < Mh;
    const int rc = row_ok ? row : Mh - 1;
    const int cpa = rc / vb, ta = rc - cpa * vb;
    const size_t oa = fidx(s0 + (uint32_t)ta, 6 * h + cpa, 12);
    float2 av[COARSE_NMAX / 8];
#pragma unroll
    for (int u = 0; u < COARSE_NMAX / 8; ++u) {
      const int k = min(4 * u + kq, nv - 1);
      av[u] = u < nks ? cvt<float2>(P[(size_t)k * 12 * V + oa]) : make_float2(0.f, 0.f);
    }
    floatx4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < COARSE_NMAX / 8; ++u) {
      if (u < nks) {
        const int k = 4 * u + kq;
        const bool k_ok = k < nv;
        const float2 a = (row_ok && k_ok) ? av[u] : make_float2(0.f, 0.f);
        const float2 b = k_ok ? eb[h * nv + k][col] : make_float2(0.f, 0.f);
        cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cre, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, cim, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, cim, 0, 0, 0);
      }
    }
    // The lane's four rows 4 kq .. 4 kq + 3 of the tile are four consecutive
    // sites of one component (|B| % 4 == 0, tiles start at multiples of 16):
    // 32 contiguous bytes, read and written as two 16-byte accesses, so that
    // the four lanes of a column cover 128 contiguous bytes per access.
    const int r = mt * 16 + 4 * kq;
    if (r < Mh && col_ok) {
      const int cp = r / vb, t = r - cp * vb;
      float4 *o4 = reinterpret_cast<float4 *>(Fc + fidx(s0 + (uint32_t)t, 6 * h + cp, 12));
      float4 lo = make_float4(cre[0], cim[0], cre[1], cim[1]), hi = make_float4(cre[2], cim[2], cre[3], cim[3]);
      if (steps > 0) {
        // + sum_k a_k r_k of this right-hand side at the four sites
        float2 acc[4] = {make_float2(lo.x, lo.y), make_float2(lo.z, lo.w), make_float2(hi.x, hi.y),
                         make_float2(hi.z, hi.w)};
        const size_t ro = (size_t)col * site_slots<TR>() * V;
#pragma unroll
        for (int k = 0; k < MRQ_MAX; ++k) {
          if (k < steps) {
            const double2 ad = alpha[(size_t)k * MG_MAX_RHS + col];
            const float2 a = make_float2((float)ad.x, (float)ad.y);
            float2 rv[4];
            load4_site(rs.r[k] + ro, s0 + (uint32_t)t, 6 * h + cp, rv);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = cfma(a, rv[e], acc[e]);
          }
        }
        lo = make_float4(acc[0].x, acc[0].y, acc[1].x, acc[1].y);
        hi = make_float4(acc[2].x, acc[2].y, acc[3].x, acc[3].y);
      } else if (accumulate) {
        const float4 a = o4[0], b = o4[1];
        lo = make_float4(lo.x + a.x, lo.y + a.y, lo.z + a.z, lo.w + a.w);
        hi = make_float4(hi.x + b.x, hi.y + b.y, hi.z + b.z, hi.w + b.w);
      }
      o4[0] = lo;
      o4[1] = hi;
    }
  }
}

}  // namespace

bool transfer_mma_ok(const Geom &g, int nv, int nrhs) {
  return nrhs >= 1 && nrhs <= TM_NR && nv >= 1 && 2 * nv <= COARSE_NMAX && g.vb % 4 == 0 && nv <= 32;
}

template <typename S, typename TF>
hipError_t restrict_fine_mma(const Geom &g, const Geom &gc, int nv, const S *P, const TF *fine, float2 *coarse,
                             int nrhs, hipStream_t st, const TF *q, const double2 *alpha) {
  if (!transfer_mma_ok(g, nv, nrhs)) return hipErrorInvalidValue;
  if (q && !alpha) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_restrict_fine_mma<S, TF>), dim3(g.Vc), dim3(64 * TM_WAVES), 0, st, g, gc, nv, nrhs, P, fine,
                     coarse, q, alpha);
  return hipGetLastError();
}

template <typename S, typename TR>
hipError_t prolong_fine_mma(const Geom &g, const Geom &gc, int nv, const S *P, const float2 *coarse, float2 *fine,
                            int nrhs, int accumulate, hipStream_t st, const MrqList<TR> *rs, int steps,
                            const double2 *alpha) {
  if (!transfer_mma_ok(g, nv, nrhs)) return hipErrorInvalidValue;
  MrqList<TR> l{};
  if (rs) {
    if (steps < 1 || steps > MRQ_MAX || !alpha) return hipErrorInvalidValue;
    l = *rs;
  } else {
    steps = 0;
  }
  hipLaunchKernelGGL((k_prolong_fine_mma<S, TR>), dim3(g.Vc), dim3(64 * TM_WAVES), 0, st, g, gc, nv, nrhs, P, coarse,
                     fine, accumulate, l, steps, alpha);
  return hipGetLastError();
}

template hipError_t restrict_fine_mma<float2, float2>(const Geom &, const Geom &, int, const float2 *,
                                                      const float2 *, float2 *, int, hipStream_t, const float2 *,
                                                      const double2 *);
template hipError_t restrict_fine_mma<chalf, float2>(const Geom &, const Geom &, int, const chalf *, const float2 *,
                                                     float2 *, int, hipStream_t, const float2 *, const double2 *);
template hipError_t restrict_fine_mma<chalf, h16>(const Geom &, const Geom &, int, const chalf *, const h16 *,
                                                  float2 *, int, hipStream_t, const h16 *, const double2 *);
template hipError_t prolong_fine_mma<float2, float2>(const Geom &, const Geom &, int, const float2 *, const float2 *,
                                                     float2 *, int, int, hipStream_t, const MrqList<float2> *, int,
                                                     const double2 *);
template hipError_t prolong_fine_mma<chalf, float2>(const Geom &, const Geom &, int, const chalf *, const float2 *,
                                                    float2 *, int, int, hipStream_t, const MrqList<float2> *, int,
                                                    const double2 *);
template hipError_t prolong_fine_mma<chalf, h16>(const Geom &, const Geom &, int, const chalf *, const float2 *,
                                                 float2 *, int, int, hipStream_t, const MrqList<h16> *, int,
                                                 const double2 *);

}  // namespace mg
