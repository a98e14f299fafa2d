// Galerkin coarse operator D_c = P^dag D P as a nearest-neighbour stencil of
// n x n blocks, n = 2 Nv (paper: A_c = P^dag A P; uniform aggregates keep the
// coarse operator nearest neighbour with 2Nv x 2Nv link matrices).
//
// For coarse column j = (chi_j, k_j) let W = P e_j, i.e. null vector k_j
// restricted to spin half chi_j on every aggregate.  Every hop of D applied to
// W at site x reads W from one neighbour; it contributes to X(x_c) when the
// hop stays inside the aggregate and to the stencil slot of the face it
// crosses otherwise.  So
//   X(x_c)[:, j]   = P^dag [ diag W + sum of intra-aggregate hops of W ] on x_c
//   Y_d(x_c)[:, j] = P^dag [ hops of W in slot d that leave the aggregate ]
// with P^dag the block-local restriction.  One workgroup per (coarse site,
// column j), the columns of one site consecutive on one XCD; threads over the
// sites (fine) or elements (coarse) of the aggregate; the 2Nv row inner
// products of each of the 9 slots are wavefront shuffle reductions plus a
// fixed-order sum over waves.  FP64.
// Output layout L[site][slot][j][i] (column-major blocks), slot 0 = X,
// slot 1 + (2 mu + dir) = Y (dir 0: couples to x_c + mu).
#include "kernels.h"
#include "wilson_site.h"

namespace mg {

// Workgroup i -> (aggregate B, coarse column j).  Workgroups go round-robin
// to the 8 XCDs; this order hands every XCD whole aggregates and runs the
// 2Nv columns of one aggregate back to back there, so the aggregate's null
// vectors (fine) or operator blocks (coarse) come from HBM once and from that
// XCD's L2 for the other columns.  Aggregates beyond the last multiple of 8
// follow in plain aggregate-major order.
__device__ __forceinline__ void agg_col_of(uint32_t i, uint32_t nagg, uint32_t ncol, uint32_t &B, int &j) {
  const uint32_t nagg8 = nagg & ~7u;
  if (i < nagg8 * ncol) {
    const uint32_t t = i >> 3;
    B = (t / ncol) * 8u + (i & 7u);
    j = (int)(t % ncol);
  } else {
    const uint32_t r = i - nagg8 * ncol;
    B = nagg8 + r / ncol;
    j = (int)(r % ncol);
  }
}

__device__ __forceinline__ uint32_t coarse_site_of(const Geom &gc, uint32_t B, const Geom &g) {
  const int x[4] = {(int)(B % g.C[0]), (int)((B / g.C[0]) % g.C[1]), (int)((B / (g.C[0] * g.C[1])) % g.C[2]),
                    (int)(B / (g.C[0] * g.C[1] * g.C[2]))};
  return encode(gc, x);
}

// ------------------------------------------------------------------ fine
// Hop d of W at site s (W = field k masked to chirality chi), times -1/2.
__device__ __forceinline__ void fine_hop(double2 (&f)[12], const Geom &g, uint32_t s, const Coords &k, int d,
                                         const double2 *__restrict__ U, const double2 *__restrict__ Pk, int chi) {
  const int mu = d >> 1;
  const bool fwd = (d & 1) == 0;
  uint32_t sn;
  double eta = 1.0;
  if (fwd) {
    sn = nbr_fwd(g, s, k, mu);
    if (mu == 3 && g.antiperiodic && k.o[3] == g.b[3] - 1 && k.c[3] == g.C[3] - 1) eta = -1.0;
  } else {
    sn = nbr_bwd(g, s, k, mu);
    if (mu == 3 && g.antiperiodic && k.o[3] == 0 && k.c[3] == 0) eta = -1.0;
  }
  double2 psi[12], u[9], acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const bool on = (c / 6) == chi;
    psi[c] = on ? Pk[fidx(sn, c, 12)] : make_double2(0, 0);
    acc[c] = make_double2(0, 0);
  }
  const uint32_t sl = fwd ? s : sn;
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = U[fidx(sl, mu * 9 + e, 36)];
  if (fwd) hop_dispatch<true>(mu, acc, psi, u, eta);
  else hop_dispatch<false>(mu, acc, psi, u, eta);
#pragma unroll
  for (int c = 0; c < 12; ++c) f[c] = cfma(make_double2(-0.5, 0.0), acc[c], f[c]);
}

// One workgroup per (aggregate, column j); one thread per site of the
// aggregate.  Each thread forms the slot-0 vector (diagonal plus the hops
// that stay inside the aggregate) and the face hops of its site; since an
// aggregate is at least two sites wide in every direction a site lies on at
// most one face per direction, so direction mu contributes one hop vector,
// credited to slot 1 + 2 mu (upper face) or 2 + 2 mu (lower face).  The
// projections onto the nv null vectors then load P_ki once per pass for all
// slots of the pass (pass 0: slot 0 and directions x, y; pass 1: directions
// z, t) instead of once per slot.
//
// Sum over the sites: for every ki each wavefront stages the KV per-site
// terms of its 64 sites (re, im of both spin halves of each slot) in its own
// LDS region, site-major, and 8 lanes per term add the 64 sites in a fixed
// interleaved order and combine with 3 shuffle steps (8 LDS reads and 3
// shuffles per term instead of a 6-step wavefront shuffle reduction).  The
// exchange stays inside one wavefront, whose LDS operations complete in
// issue order, so it needs no workgroup barrier; the per-wave results meet in
// a fixed-order sum over the waves after the ki loop.
constexpr int GF_KV = 20;  // terms per site and ki, pass 0 (5 slots x 4)
constexpr int GF_LD = 72;  // row stride of a wave's term rows (64 sites + 8)

template <int PASS>
__device__ __forceinline__ void galerkin_pass(const Geom &g, uint32_t s, const Coords &k, bool act, int chi,
                                              double diag, const double2 *__restrict__ U,
                                              const double2 *__restrict__ Pj, const double2 *__restrict__ P,
                                              int nv, int jcol, int n, uint32_t ic, double *red,
                                              double2 (*part)[COARSE_NMAX], double2 *__restrict__ Lc) {
  constexpr int NS = PASS == 0 ? 3 : 2;  // vectors of this pass: [slot0,] mu, mu + 1
  constexpr int MU0 = PASS == 0 ? 0 : 2;
  constexpr int NSLOT = PASS == 0 ? 5 : 4;
  constexpr int KV = 4 * NSLOT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = (int)(blockDim.x >> 6);
  double *rw = red + w * GF_KV * GF_LD;
  const size_t V = g.Vpad;
  double2 f[NS][12];
  bool up[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    up[q] = false;
#pragma unroll
    for (int c = 0; c < 12; ++c) f[q][c] = make_double2(0, 0);
  }
  if (act) {
    int q0 = 0;
    if constexpr (PASS == 0) {
#pragma unroll
      for (int c = 0; c < 12; ++c)
        if ((c / 6) == chi) f[0][c] = cscale(Pj[fidx(s, c, 12)], diag);
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int mu = d >> 1;
        const bool face = (d & 1) == 0 ? (k.o[mu] == g.b[mu] - 1) : (k.o[mu] == 0);
        if (!face) fine_hop(f[0], g, s, k, d, U, Pj, chi);
      }
      q0 = 1;
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int mu = MU0 + m;
      if (k.o[mu] == g.b[mu] - 1) {
        fine_hop(f[q0 + m], g, s, k, 2 * mu, U, Pj, chi);
        up[q0 + m] = true;
      } else if (k.o[mu] == 0) {
        fine_hop(f[q0 + m], g, s, k, 2 * mu + 1, U, Pj, chi);
      }
    }
  }
  for (int ki = 0; ki < nv; ++ki) {
    const double2 *Pi = P + (size_t)ki * 12 * V;
    double2 pi[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) pi[c] = act ? Pi[fidx(s, c, 12)] : make_double2(0, 0);
    double2 dv[NS][2];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      double2 d0 = make_double2(0, 0), d1 = make_double2(0, 0);
#pragma unroll
      for (int c = 0; c < 6; ++c) d0 = cfmac(pi[c], f[q][c], d0);
#pragma unroll
      for (int c = 6; c < 12; ++c) d1 = cfmac(pi[c], f[q][c], d1);
      dv[q][0] = d0;
      dv[q][1] = d1;
    }
    // this site's term of each slot: term 4 sl + (0, 1, 2, 3) = (re, im) of
    // the upper-half row ki, then of the lower-half row nv + ki
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
      double2 v0, v1;
      if (PASS == 0 && sl == 0) {
        v0 = dv[0][0];
        v1 = dv[0][1];
      } else {
        const int qi = (PASS == 0 ? 1 : 0) + (sl - (PASS == 0 ? 1 : 0)) / 2;
        const bool want_up = ((sl - (PASS == 0 ? 1 : 0)) % 2) == 0;
        const bool mine = up[qi] == want_up;
        v0 = mine ? dv[qi][0] : make_double2(0, 0);
        v1 = mine ? dv[qi][1] : make_double2(0, 0);
      }
      rw[(4 * sl + 0) * GF_LD + lane] = v0.x;
      rw[(4 * sl + 1) * GF_LD + lane] = v0.y;
      rw[(4 * sl + 2) * GF_LD + lane] = v1.x;
      rw[(4 * sl + 3) * GF_LD + lane] = v1.y;
    }
    __builtin_amdgcn_wave_barrier();
    // 8 consecutive lanes per term (a group never straddles an iteration);
    // lane p adds sites p, p + 8, ..., p + 56 of this wave
    for (int o = lane; o < KV * 8; o += 64) {
      const int term = o >> 3, p = o & 7;
      const double *row = rw + term * GF_LD;
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < 64; j += 8) a += row[j + p];
      a += __shfl_xor(a, 4, 64);
      a += __shfl_xor(a, 2, 64);
      a += __shfl_xor(a, 1, 64);
      if (p == 0) {
        const int sl = term >> 2, e = term & 3;
        double *r = reinterpret_cast<double *>(&part[w * NSLOT + sl][(e < 2 ? 0 : nv) + ki]);
        r[e & 1] = a;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  for (int o = tid; o < NSLOT * n; o += blockDim.x) {
    const int sl = o / n, i = o % n;
    double2 a = part[sl][i];
    for (int q = 1; q < nw; ++q) {
      a.x += part[q * NSLOT + sl][i].x;
      a.y += part[q * NSLOT + sl][i].y;
    }
    const int slot = PASS == 0 ? sl : 5 + sl;
    Lc[(((size_t)ic * 9 + slot) * n + jcol) * n + i] = a;
  }
  __syncthreads();
}

// At most 256 VGPRs so that two workgroups share a CU (a handful of spills).
__global__ __launch_bounds__(256, 2) void k_galerkin_fine(Geom g, Geom gc, double diag,
                                                          const double2 *__restrict__ U, int nv,
                                                          const double2 *__restrict__ P, double2 *__restrict__ Lc) {
  __shared__ double red[4 * GF_KV * GF_LD];
  __shared__ double2 part[4 * 5][COARSE_NMAX];
  uint32_t B;
  int jcol;
  agg_col_of(blockIdx.x, g.Vc, 2 * nv, B, jcol);
  const int chi = jcol / nv, kj = jcol % nv;
  const int n = 2 * nv;
  const int tid = threadIdx.x;
  const bool act = (uint32_t)tid < g.vb;
  const uint32_t s = B * g.vb + (act ? tid : 0);
  const Coords k = decode(g, s);
  const double2 *Pj = P + (size_t)kj * 12 * g.Vpad;
  const uint32_t ic = coarse_site_of(gc, B, g);
  galerkin_pass<0>(g, s, k, act, chi, diag, U, Pj, P, nv, jcol, n, ic, red, part, Lc);
  galerkin_pass<1>(g, s, k, act, chi, diag, U, Pj, P, nv, jcol, n, ic, red, part, Lc);
}

// Any aggregate shape (also one site wide in some direction, where a site
// lies on both faces): one slot at a time.
__global__ __launch_bounds__(256) void k_galerkin_fine_generic(Geom g, Geom gc, double diag, const double2 *__restrict__ U,
                                                       int nv, const double2 *__restrict__ P,
                                                       double2 *__restrict__ Lc) {
  __shared__ double2 part[4][2 * COARSE_NMAX];
  const size_t V = g.Vpad;
  uint32_t B;
  int jcol;
  agg_col_of(blockIdx.x, g.Vc, 2 * nv, B, jcol);
  const int chi = jcol / nv, kj = jcol % nv;
  const int n = 2 * nv;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = (blockDim.x + 63) >> 6;
  const bool act = (uint32_t)tid < g.vb;
  const uint32_t s = B * g.vb + (act ? tid : 0);
  const Coords k = decode(g, s);
  const double2 *Pj = P + (size_t)kj * 12 * V;
  const uint32_t ic = coarse_site_of(gc, B, g);
  for (int slot = 0; slot < 9; ++slot) {
    double2 f[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) f[c] = make_double2(0, 0);
    if (act) {
      if (slot == 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c)
          if ((c / 6) == chi) f[c] = cscale(Pj[fidx(s, c, 12)], diag);
        for (int d = 0; d < 8; ++d) {
          const int mu = d >> 1;
          const bool face = (d & 1) == 0 ? (k.o[mu] == g.b[mu] - 1) : (k.o[mu] == 0);
          if (!face) fine_hop(f, g, s, k, d, U, Pj, chi);
        }
      } else {
        const int d = slot - 1, mu = d >> 1;
        const bool face = (d & 1) == 0 ? (k.o[mu] == g.b[mu] - 1) : (k.o[mu] == 0);
        if (face) fine_hop(f, g, s, k, d, U, Pj, chi);
      }
    }
    for (int ki = 0; ki < nv; ++ki) {
      const double2 *Pi = P + (size_t)ki * 12 * V;
      double2 d0 = make_double2(0, 0), d1 = make_double2(0, 0);
      if (act) {
#pragma unroll
        for (int c = 0; c < 6; ++c) d0 = cfmac(Pi[fidx(s, c, 12)], f[c], d0);
#pragma unroll
        for (int c = 6; c < 12; ++c) d1 = cfmac(Pi[fidx(s, c, 12)], f[c], d1);
      }
      const double a0 = wave_sum(d0.x), b0 = wave_sum(d0.y), a1 = wave_sum(d1.x), b1 = wave_sum(d1.y);
      if (lane == 0) {
        part[w][ki] = make_double2(a0, b0);
        part[w][nv + ki] = make_double2(a1, b1);
      }
    }
    __syncthreads();
    if (tid < n) {
      double2 a = part[0][tid];
      for (int q = 1; q < nw; ++q) {
        a.x += part[q][tid].x;
        a.y += part[q][tid].y;
      }
      Lc[(((size_t)ic * 9 + slot) * n + jcol) * n + tid] = a;
    }
    __syncthreads();
  }
}

hipError_t galerkin_fine(const Geom &g, const Geom &gc, double mass, const double2 *U, int nv, const double2 *P,
                         double2 *Lc, hipStream_t st) {
  const int th = (int)((g.vb + 63) / 64 * 64);
  const bool wide = g.b[0] > 1 && g.b[1] > 1 && g.b[2] > 1 && g.b[3] > 1;
  if (wide)
    hipLaunchKernelGGL(k_galerkin_fine, dim3(g.Vc * 2 * nv), dim3(th), 0, st, g, gc, 4.0 + mass, U, nv, P, Lc);
  else
    hipLaunchKernelGGL(k_galerkin_fine_generic, dim3(g.Vc * 2 * nv), dim3(th), 0, st, g, gc, 4.0 + mass, U, nv, P,
                       Lc);
  return hipGetLastError();
}

// ------------------------------------------------------------------ coarse
// EM elements per thread (256 threads): 4 when the aggregate has at most
// 1024 elements (fewer registers, two workgroups per CU), else 8.
template <int EM>
__global__ __launch_bounds__(256, EM == 4 ? 2 : 1) void k_galerkin_coarse(Geom g, Geom gc, int n, const double2 *__restrict__ L1,
                                                         int nv, const double2 *__restrict__ P,
                                                         double2 *__restrict__ Lc) {
  constexpr int KB = 4;  // null vectors per wave-local reduction round
  __shared__ double red[4 * 4 * KB * GF_LD];
  __shared__ double2 part[4][COARSE_NMAX];
  const size_t V = g.V;
  uint32_t B;
  int jcol;
  agg_col_of(blockIdx.x, g.Vc, 2 * nv, B, jcol);
  const int chi = jcol / nv, kj = jcol % nv;
  const int nc = 2 * nv, half = n >> 1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = (blockDim.x + 63) >> 6;
  const int ne = (int)g.vb * n;
  const double2 *Pj = P + (size_t)kj * V * n;
  const uint32_t ic = coarse_site_of(gc, B, g);
  for (int slot = 0; slot < 9; ++slot) {
    double2 f[EM];
#pragma unroll
    for (int q = 0; q < EM; ++q) {
      f[q] = make_double2(0, 0);
      const int e = tid + q * (int)blockDim.x;
      if (e >= ne) continue;
      const uint32_t t = (uint32_t)(e / n);
      const int ii = e - (int)t * n;
      const uint32_t s = B * g.vb + t;
      const Coords k = decode(g, s);
      // (L1[s][slot1] W(site))_ii summed over the needed slots
      for (int s1 = 0; s1 < 9; ++s1) {
        bool use;
        uint32_t src = s;
        if (s1 == 0) {
          use = (slot == 0);
        } else {
          const int d = s1 - 1, mu = d >> 1;
          const bool face = (d & 1) == 0 ? (k.o[mu] == g.b[mu] - 1) : (k.o[mu] == 0);
          use = (slot == 0) ? !face : (slot == s1 && face);
          src = (d & 1) ? nbr_bwd(g, s, k, mu) : nbr_fwd(g, s, k, mu);
        }
        if (!use) continue;
        const double2 *Lb = L1 + ((size_t)s * 9 + s1) * n * n + ii;
        const double2 *Wv = Pj + (size_t)src * n;
        double2 a = f[q];
        const int j0 = chi * half;
        for (int jj = j0; jj < j0 + half; ++jj) a = cfma(Lb[(size_t)jj * n], Wv[jj], a);
        f[q] = a;
      }
    }
    // projections onto KB null vectors at a time; the sum over this wave's
    // elements is the wave-local LDS reduction of the fine kernel (4 KB
    // terms: re, im of the upper- and lower-half rows of each null vector)
    double *rw = red + w * 4 * KB * GF_LD;
    for (int k0 = 0; k0 < nv; k0 += KB) {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int ki = k0 + u;
        double2 d0 = make_double2(0, 0), d1 = make_double2(0, 0);
        if (ki < nv) {
          const double2 *Pi = P + (size_t)ki * V * n + (size_t)B * g.vb * n;
#pragma unroll
          for (int q = 0; q < EM; ++q) {
            const int e = tid + q * (int)blockDim.x;
            if (e < ne) {
              if ((e % n) < half) d0 = cfmac(Pi[e], f[q], d0);
              else d1 = cfmac(Pi[e], f[q], d1);
            }
          }
        }
        rw[(4 * u + 0) * GF_LD + lane] = d0.x;
        rw[(4 * u + 1) * GF_LD + lane] = d0.y;
        rw[(4 * u + 2) * GF_LD + lane] = d1.x;
        rw[(4 * u + 3) * GF_LD + lane] = d1.y;
      }
      __builtin_amdgcn_wave_barrier();
      for (int o = lane; o < 4 * KB * 8; o += 64) {
        const int term = o >> 3, p = o & 7;
        const double *row = rw + term * GF_LD;
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < 64; j += 8) a += row[j + p];
        a += __shfl_xor(a, 4, 64);
        a += __shfl_xor(a, 2, 64);
        a += __shfl_xor(a, 1, 64);
        const int ki = k0 + (term >> 2), e = term & 3;
        if (p == 0 && ki < nv) reinterpret_cast<double *>(&part[w][(e < 2 ? 0 : nv) + ki])[e & 1] = a;
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (tid < nc) {
      double2 a = part[0][tid];
      for (int q = 1; q < nw; ++q) {
        a.x += part[q][tid].x;
        a.y += part[q][tid].y;
      }
      Lc[(((size_t)ic * 9 + slot) * nc + jcol) * nc + tid] = a;
    }
    __syncthreads();
  }
}

hipError_t galerkin_coarse(const Geom &g, const Geom &gc, int n, const double2 *L1, int nv, const double2 *P,
                           double2 *Lc, hipStream_t st) {
  if (g.vb * n <= 4 * 256)
    hipLaunchKernelGGL(k_galerkin_coarse<4>, dim3(g.Vc * 2 * nv), dim3(256), 0, st, g, gc, n, L1, nv, P, Lc);
  else
    hipLaunchKernelGGL(k_galerkin_coarse<8>, dim3(g.Vc * 2 * nv), dim3(256), 0, st, g, gc, n, L1, nv, P, Lc);
  return hipGetLastError();
}

}  // namespace mg
