// Learned near-null-vector proposal: a two-layer gauge-equivariant network of
// parallel-transport convolutions (an extension of the adaptive setup of
// "Adaptive Multigrid"; the paper has no such network).
//
// Hop operators T_k, k = 0..8: T_0 = 1; k = 1 + 2 mu + dir transports the
// neighbour value along the link of the hopping term of Eq. 2 (dir 0:
// eta U_mu(x) psi(x+mu); dir 1: eta U_mu(x-mu)^dag psi(x-mu)), eta = -1
// across the antiperiodic time boundary.  A layer is
//   out_a(x) = sum_{b,k} W_abk (T_k in_b)(x),   W_abk a complex 4x4 spin matrix.
// Forward and backward passes are split into a transport stage (H_bk = T_k
// in_b, stored for the weight gradient) and site-local channel mixing; the
// adjoint transport uses T_{+mu}^dag = T_{-mu}.  The training loss is the
// subspace fit of target vectors per chirality-split aggregate (the blocks
// on which P is built, Eq. 4), solved by Cholesky of the 24 x 24 Gram
// matrices in FP64.  FP32 weights and arithmetic; fields in the fine
// tile-interleaved layout [channel][12 * Vpad].
#include "ptc.h"

namespace mg {

__device__ __forceinline__ float2 cf(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ float2 cmulf(float2 a, float2 b) { return cf(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ float2 cfmaf(float2 a, float2 b, float2 c) {
  return cf(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
// conj(a) * b + c
__device__ __forceinline__ float2 cfmacf(float2 a, float2 b, float2 c) {
  return cf(fmaf(a.x, b.x, fmaf(a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(-a.y, b.x, c.y)));
}

// h = T_kk psi at site s (12 complex: spin-major 3 s + c).
__device__ __forceinline__ void transport_site(float2 (&h)[12], const Geom &g, uint32_t s, const Coords &k, int kk,
                                               const float2 *__restrict__ U, const float2 *__restrict__ psi) {
  if (kk == 0) {
#pragma unroll
    for (int c = 0; c < 12; ++c) h[c] = psi[fidx(s, c, 12)];
    return;
  }
  const int mu = (kk - 1) >> 1;
  const bool back = ((kk - 1) & 1) != 0;
  uint32_t sn;
  float eta = 1.f;
  if (!back) {
    sn = nbr_fwd(g, s, k, mu);
    if (mu == 3 && g.antiperiodic && k.o[3] == g.b[3] - 1 && k.c[3] == g.C[3] - 1) eta = -1.f;
  } else {
    sn = nbr_bwd(g, s, k, mu);
    if (mu == 3 && g.antiperiodic && k.o[3] == 0 && k.c[3] == 0) eta = -1.f;
  }
  const uint32_t sl = back ? sn : s;
  float2 u[9], p[12];
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = U[fidx(sl, mu * 9 + e, 36)];
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = psi[fidx(sn, c, 12)];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float2 acc = cf(0.f, 0.f);
#pragma unroll
      for (int b = 0; b < 3; ++b)
        acc = back ? cfmacf(u[b * 3 + a], p[sp * 3 + b], acc) : cfmaf(u[a * 3 + b], p[sp * 3 + b], acc);
      h[sp * 3 + a] = cf(eta * acc.x, eta * acc.y);
    }
}

__device__ __forceinline__ int adjoint_hop(int kk) { return kk == 0 ? 0 : (((kk - 1) & 1) ? kk - 1 : kk + 1); }

// H[b * 9 + k] = T_k in[b]
__global__ __launch_bounds__(256) void k_ptc_transport(Geom g, const float2 *__restrict__ U,
                                                       const float2 *__restrict__ in, float2 *__restrict__ H) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int b = blockIdx.y;
  const size_t F = (size_t)12 * g.Vpad;
  const Coords k = decode(g, s);
  const float2 *src = in + b * F;
#pragma unroll 1
  for (int kk = 0; kk < PTC_HOPS; ++kk) {
    float2 h[12];
    transport_site(h, g, s, k, kk, U, src);
    float2 *dst = H + ((size_t)b * PTC_HOPS + kk) * F;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[fidx(s, c, 12)] = h[c];
  }
}

// out[a] = sum_{b,k} W[a][b][k] H[b*9+k]   (4 output channels per block row)
__global__ __launch_bounds__(256) void k_ptc_mix(Geom g, int cin, int cout, const float2 *__restrict__ W,
                                                 const float2 *__restrict__ H, float2 *__restrict__ out) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int a0 = blockIdx.y * 4;
  const size_t F = (size_t)12 * g.Vpad;
  float2 acc[4][12];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[q][c] = cf(0.f, 0.f);
  for (int bk = 0; bk < cin * PTC_HOPS; ++bk) {
    float2 h[12];
    const float2 *src = H + (size_t)bk * F;
#pragma unroll
    for (int c = 0; c < 12; ++c) h[c] = src[fidx(s, c, 12)];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = a0 + q;
      if (a >= cout) break;
      const float2 *Wm = W + ((size_t)a * cin * PTC_HOPS + bk) * 16;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float2 w = Wm[sp * 4 + t];
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[q][sp * 3 + c] = cfmaf(w, h[t * 3 + c], acc[q][sp * 3 + c]);
        }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = a0 + q;
    if (a >= cout) break;
    float2 *dst = out + (size_t)a * F;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[fidx(s, c, 12)] = acc[q][c];
  }
}

// A[b*9+k] = sum_a W[a][b][k]^dag G[a]   (3 hops per block row: y = b*3 + kg)
__global__ __launch_bounds__(256) void k_ptc_mix_adj(Geom g, int cin, int cout, const float2 *__restrict__ W,
                                                     const float2 *__restrict__ G, float2 *__restrict__ A) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int b = blockIdx.y / 3, k0 = (blockIdx.y % 3) * 3;
  const size_t F = (size_t)12 * g.Vpad;
  float2 acc[3][12];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[q][c] = cf(0.f, 0.f);
  for (int a = 0; a < cout; ++a) {
    float2 gv[12];
    const float2 *src = G + (size_t)a * F;
#pragma unroll
    for (int c = 0; c < 12; ++c) gv[c] = src[fidx(s, c, 12)];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float2 *Wm = W + (((size_t)a * cin + b) * PTC_HOPS + k0 + q) * 16;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float2 w = Wm[sp * 4 + t];   // (W^dag)[t][sp] = conj(W[sp][t])
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[q][t * 3 + c] = cfmacf(w, gv[sp * 3 + c], acc[q][t * 3 + c]);
        }
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    float2 *dst = A + ((size_t)b * PTC_HOPS + k0 + q) * F;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[fidx(s, c, 12)] = acc[q][c];
  }
}

// gin[b] = sum_k T_k^dag A[b*9+k]
__global__ __launch_bounds__(256) void k_ptc_transport_adj(Geom g, const float2 *__restrict__ U,
                                                           const float2 *__restrict__ A, float2 *__restrict__ gin) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int b = blockIdx.y;
  const size_t F = (size_t)12 * g.Vpad;
  const Coords k = decode(g, s);
  float2 acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = cf(0.f, 0.f);
#pragma unroll 1
  for (int kk = 0; kk < PTC_HOPS; ++kk) {
    float2 h[12];
    transport_site(h, g, s, k, adjoint_hop(kk), U, A + ((size_t)b * PTC_HOPS + kk) * F);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cf(acc[c].x + h[c].x, acc[c].y + h[c].y);
  }
  float2 *dst = gin + (size_t)b * F;
#pragma unroll
  for (int c = 0; c < 12; ++c) dst[fidx(s, c, 12)] = acc[c];
}

// Weight-gradient partials: part[(abk * nchunk + chunk) * 16 + (s t)] =
// sum over the chunk's sites and colours of G_a[s][c] conj(H_bk[t][c]).
__global__ __launch_bounds__(256) void k_ptc_wgrad(Geom g, int cin, int nchunk, const float2 *__restrict__ G,
                                                   const float2 *__restrict__ H, double2 *__restrict__ part) {
  __shared__ double lds[4 * 32];
  const int abk = blockIdx.y, chunk = blockIdx.x;
  const int a = abk / (cin * PTC_HOPS), bk = abk % (cin * PTC_HOPS);
  const size_t F = (size_t)12 * g.Vpad;
  const float2 *ga = G + (size_t)a * F, *hb = H + (size_t)bk * F;
  const uint32_t per = (g.V + nchunk - 1) / nchunk;
  const uint32_t lo = chunk * per, hi = min(g.V, lo + per);
  float2 acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = cf(0.f, 0.f);
  for (uint32_t s = lo + threadIdx.x; s < hi; s += blockDim.x) {
    float2 gv[12], hv[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      gv[c] = ga[fidx(s, c, 12)];
      hv[c] = hb[fidx(s, c, 12)];
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[sp * 4 + t] = cfmacf(hv[t * 3 + c], gv[sp * 3 + c], acc[sp * 4 + t]);
  }
  double v[32];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    v[2 * e] = acc[e].x;
    v[2 * e + 1] = acc[e].y;
  }
  block_sum<32>(v, lds);
  if (threadIdx.x == 0) {
    double2 *p = part + ((size_t)abk * nchunk + chunk) * 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) p[e] = make_double2(v[2 * e], v[2 * e + 1]);
  }
}

__global__ void k_ptc_wgrad_final(int nabk, int nchunk, const double2 *__restrict__ part, float2 *__restrict__ gW) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nabk * 16) return;
  const int abk = i / 16, e = i % 16;
  double x = 0.0, y = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    const double2 v = part[((size_t)abk * nchunk + c) * 16 + e];
    x += v.x;
    y += v.y;
  }
  gW[i] = cf((float)x, (float)y);
}

// ------------------------------------------------------------ subspace fit
// Block (aggregate B, chirality chi): rows r = (site l of B, component
// 6 chi + j), j < 6.  Gram G = Y^dag Y (ny x ny) and R = Y^dag V (ny x nv),
// FP64, rows staged through LDS 16 sites at a time.
constexpr int FIT_SITES = 16;

__global__ __launch_bounds__(256) void k_fit_gram(Geom g, int ny, int nv, const float2 *__restrict__ Y,
                                                  const float2 *__restrict__ V, double2 *__restrict__ GR) {
  extern __shared__ float2 rows[];  // [FIT_SITES * 6][ny + nv]
  const uint32_t B = blockIdx.x;
  const int chi = blockIdx.y;
  const int nc = ny + nv, nout = ny * nc;
  const size_t F = (size_t)12 * g.Vpad;
  constexpr int MAXO = 8;
  double2 acc[MAXO];
#pragma unroll
  for (int q = 0; q < MAXO; ++q) acc[q] = make_double2(0.0, 0.0);
  for (uint32_t l0 = 0; l0 < g.vb; l0 += FIT_SITES) {
    __syncthreads();
    const int nr = FIT_SITES * 6;
    for (int idx = threadIdx.x; idx < nr * nc; idx += blockDim.x) {
      const int col = idx / nr, r = idx % nr;
      const uint32_t l = l0 + r / 6;
      float2 v = cf(0.f, 0.f);
      if (l < g.vb) {
        const uint32_t s = B * g.vb + l;
        const int comp = 6 * chi + r % 6;
        v = col < ny ? Y[col * F + fidx(s, comp, 12)] : V[(col - ny) * F + fidx(s, comp, 12)];
      }
      rows[r * nc + col] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXO; ++q) {
      const int o = threadIdx.x + q * blockDim.x;
      if (o >= nout) break;
      const int i = o / nc, j = o % nc;
      double2 a = acc[q];
      for (int r = 0; r < nr; ++r) {
        const float2 yi = rows[r * nc + i], xj = rows[r * nc + j];
        a.x += (double)yi.x * xj.x + (double)yi.y * xj.y;
        a.y += (double)yi.x * xj.y - (double)yi.y * xj.x;
      }
      acc[q] = a;
    }
  }
  double2 *out = GR + ((size_t)B * 2 + chi) * nout;
#pragma unroll
  for (int q = 0; q < MAXO; ++q) {
    const int o = threadIdx.x + q * blockDim.x;
    if (o < nout) out[o] = acc[q];
  }
}

// C = G^{-1} R per block by Cholesky (G = L L^dag), FP64 in LDS.  A
// non-positive pivot marks the block (flag = 1) and leaves C = 0.
__global__ __launch_bounds__(64) void k_fit_solve(int ny, int nv, const double2 *__restrict__ GR,
                                                  double2 *__restrict__ Cout, int *__restrict__ flag) {
  extern __shared__ double2 sm[];  // G [ny][ny], R [ny][nv]
  const int blk = blockIdx.x;
  const int nc = ny + nv;
  double2 *G = sm, *R = sm + ny * ny;
  const double2 *src = GR + (size_t)blk * ny * nc;
  for (int o = threadIdx.x; o < ny * nc; o += blockDim.x) {
    const int i = o / nc, j = o % nc;
    if (j < ny) G[i * ny + j] = src[o];
    else R[i * nv + (j - ny)] = src[o];
  }
  __syncthreads();
  __shared__ int bad;
  if (threadIdx.x == 0) {
    bad = 0;
    // in-place Cholesky: lower triangle of G holds L
    for (int j = 0; j < ny && !bad; ++j) {
      double d = G[j * ny + j].x;
      for (int p = 0; p < j; ++p) d -= G[j * ny + p].x * G[j * ny + p].x + G[j * ny + p].y * G[j * ny + p].y;
      if (!(d > 0.0)) {
        bad = 1;
        break;
      }
      const double ljj = sqrt(d);
      G[j * ny + j] = make_double2(ljj, 0.0);
      for (int i = j + 1; i < ny; ++i) {
        double2 a = G[i * ny + j];
        for (int p = 0; p < j; ++p) {  // a -= L[i][p] conj(L[j][p])
          const double2 x = G[i * ny + p], y = G[j * ny + p];
          a.x -= x.x * y.x + x.y * y.y;
          a.y -= x.y * y.x - x.x * y.y;
        }
        G[i * ny + j] = make_double2(a.x / ljj, a.y / ljj);
      }
    }
  }
  __syncthreads();
  double2 *C = Cout + (size_t)blk * ny * nv;
  if (bad) {
    if (threadIdx.x == 0) atomicOr(flag, 1);
    for (int o = threadIdx.x; o < ny * nv; o += blockDim.x) C[o] = make_double2(0.0, 0.0);
    return;
  }
  // one column of R per thread: L z = r, then L^dag c = z
  for (int j = threadIdx.x; j < nv; j += blockDim.x) {
    for (int i = 0; i < ny; ++i) {
      double2 a = R[i * nv + j];
      for (int p = 0; p < i; ++p) {
        const double2 l = G[i * ny + p], z = R[p * nv + j];
        a.x -= l.x * z.x - l.y * z.y;
        a.y -= l.x * z.y + l.y * z.x;
      }
      const double d = G[i * ny + i].x;
      R[i * nv + j] = make_double2(a.x / d, a.y / d);
    }
    for (int i = ny - 1; i >= 0; --i) {
      double2 a = R[i * nv + j];
      for (int p = i + 1; p < ny; ++p) {  // a -= conj(L[p][i]) c[p]
        const double2 l = G[p * ny + i], z = R[p * nv + j];
        a.x -= l.x * z.x + l.y * z.y;
        a.y -= l.x * z.y - l.y * z.x;
      }
      const double d = G[i * ny + i].x;
      R[i * nv + j] = make_double2(a.x / d, a.y / d);
    }
    for (int i = 0; i < ny; ++i) C[i * nv + j] = R[i * nv + j];
  }
}

// Residual E = V - Y C per row, loss partial sum |E|^2 per block and the
// gradient gY = -(2 / Z) E C^dag.  One thread per row of the block.
__global__ __launch_bounds__(256) void k_fit_resid(Geom g, int ny, int nv, const float2 *__restrict__ Y,
                                                   const float2 *__restrict__ V, const double2 *__restrict__ Cm,
                                                   const double *__restrict__ Z, float2 *__restrict__ gY,
                                                   double *__restrict__ part) {
  extern __shared__ float2 cs[];  // C [ny][nv] in FP32
  __shared__ double lds[4];
  const uint32_t B = blockIdx.x;
  const int chi = blockIdx.y;
  const size_t F = (size_t)12 * g.Vpad;
  const double2 *C = Cm + ((size_t)B * 2 + chi) * ny * nv;
  for (int o = threadIdx.x; o < ny * nv; o += blockDim.x) cs[o] = cf((float)C[o].x, (float)C[o].y);
  __syncthreads();
  const float sc = (float)(-2.0 / Z[0]);
  double t[1] = {0.0};
  for (int r = threadIdx.x; r < (int)g.vb * 6; r += blockDim.x) {
    const uint32_t s = B * g.vb + r / 6;
    const size_t off = fidx(s, 6 * chi + r % 6, 12);
    float2 y[PTC_MAX_OUT], gacc[PTC_MAX_OUT];
#pragma unroll
    for (int i = 0; i < PTC_MAX_OUT; ++i) {
      y[i] = i < ny ? Y[i * F + off] : cf(0.f, 0.f);
      gacc[i] = cf(0.f, 0.f);
    }
    for (int j = 0; j < nv; ++j) {
      float2 e = V[j * F + off];
#pragma unroll
      for (int i = 0; i < PTC_MAX_OUT; ++i) {
        if (i >= ny) break;
        const float2 c = cs[i * nv + j];
        e = cf(e.x - (y[i].x * c.x - y[i].y * c.y), e.y - (y[i].x * c.y + y[i].y * c.x));
      }
      t[0] += (double)e.x * e.x + (double)e.y * e.y;
#pragma unroll
      for (int i = 0; i < PTC_MAX_OUT; ++i) {
        if (i >= ny) break;
        gacc[i] = cfmacf(cs[i * nv + j], e, gacc[i]);  // e conj(c)
      }
    }
#pragma unroll
    for (int i = 0; i < PTC_MAX_OUT; ++i)
      if (i < ny) gY[i * F + off] = cf(sc * gacc[i].x, sc * gacc[i].y);
  }
  block_sum<1>(t, lds);
  if (threadIdx.x == 0) part[(size_t)B * 2 + chi] = t[0];
}

__global__ void k_ptc_sum(const double *__restrict__ p, int n, double *__restrict__ out) {
  __shared__ double lds[4];
  double t[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) t[0] += p[i];
  block_sum<1>(t, lds);
  if (threadIdx.x == 0) out[0] = t[0];
}

__global__ __launch_bounds__(256) void k_ptc_norm2(const float2 *__restrict__ x, size_t n, double *__restrict__ part) {
  __shared__ double lds[4];
  double t[1] = {0.0};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    t[0] += (double)x[i].x * x[i].x + (double)x[i].y * x[i].y;
  block_sum<1>(t, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t[0];
}

// Adam on the real and imaginary parts of complex parameters.
__global__ __launch_bounds__(256) void k_ptc_adam(float2 *__restrict__ W, const float2 *__restrict__ gW,
                                                  float2 *__restrict__ m, float2 *__restrict__ v, size_t n, float lr,
                                                  float b1, float b2, float eps, float c1, float c2) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 g = gW[i];
  float2 mi = m[i], vi = v[i];
  mi = cf(b1 * mi.x + (1.f - b1) * g.x, b1 * mi.y + (1.f - b1) * g.y);
  vi = cf(b2 * vi.x + (1.f - b2) * g.x * g.x, b2 * vi.y + (1.f - b2) * g.y * g.y);
  m[i] = mi;
  v[i] = vi;
  const float2 w = W[i];
  W[i] = cf(w.x - lr * (mi.x / c1) / (sqrtf(vi.x / c2) + eps), w.y - lr * (mi.y / c1) / (sqrtf(vi.y / c2) + eps));
}

// ---------------------------------------------------------------- launchers
hipError_t ptc_transport(const Geom &g, const float2 *U, const float2 *in, int cin, float2 *H, hipStream_t st) {
  hipLaunchKernelGGL(k_ptc_transport, dim3(div_up(g.V, 256), cin), dim3(256), 0, st, g, U, in, H);
  return hipGetLastError();
}
hipError_t ptc_mix(const Geom &g, int cin, int cout, const float2 *W, const float2 *H, float2 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_ptc_mix, dim3(div_up(g.V, 256), (cout + 3) / 4), dim3(256), 0, st, g, cin, cout, W, H, out);
  return hipGetLastError();
}
hipError_t ptc_mix_adj(const Geom &g, int cin, int cout, const float2 *W, const float2 *G, float2 *A,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_ptc_mix_adj, dim3(div_up(g.V, 256), cin * 3), dim3(256), 0, st, g, cin, cout, W, G, A);
  return hipGetLastError();
}
hipError_t ptc_transport_adj(const Geom &g, const float2 *U, const float2 *A, int cin, float2 *gin, hipStream_t st) {
  hipLaunchKernelGGL(k_ptc_transport_adj, dim3(div_up(g.V, 256), cin), dim3(256), 0, st, g, U, A, gin);
  return hipGetLastError();
}
hipError_t ptc_wgrad(const Geom &g, int cin, int cout, const float2 *G, const float2 *H, double2 *part, float2 *gW,
                     hipStream_t st) {
  const int nabk = cout * cin * PTC_HOPS;
  hipLaunchKernelGGL(k_ptc_wgrad, dim3(PTC_WCHUNK, nabk), dim3(256), 0, st, g, cin, PTC_WCHUNK, G, H, part);
  hipLaunchKernelGGL(k_ptc_wgrad_final, dim3(div_up(nabk * 16, 256)), dim3(256), 0, st, nabk, PTC_WCHUNK, part, gW);
  return hipGetLastError();
}
hipError_t ptc_fit(const Geom &g, int ny, int nv, const float2 *Y, const float2 *V, const double *Z, double2 *GR,
                   double2 *C, int *flag, float2 *gY, double *part, double *loss, hipStream_t st) {
  const int nc = ny + nv;
  hipLaunchKernelGGL(k_fit_gram, dim3(g.Vc, 2), dim3(256), sizeof(float2) * FIT_SITES * 6 * nc, st, g, ny, nv, Y, V,
                     GR);
  hipLaunchKernelGGL(k_fit_solve, dim3(g.Vc * 2), dim3(64), sizeof(double2) * ny * nc, st, ny, nv, GR, C, flag);
  hipLaunchKernelGGL(k_fit_resid, dim3(g.Vc, 2), dim3(256), sizeof(float2) * ny * nv, st, g, ny, nv, Y, V, C, Z, gY,
                     part);
  hipLaunchKernelGGL(k_ptc_sum, dim3(1), dim3(256), 0, st, part, (int)(g.Vc * 2), loss);
  return hipGetLastError();
}
hipError_t ptc_norm2(const float2 *x, size_t n, double *part, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_ptc_norm2, dim3(256), dim3(256), 0, st, x, n, part);
  hipLaunchKernelGGL(k_ptc_sum, dim3(1), dim3(256), 0, st, part, 256, out);
  return hipGetLastError();
}
hipError_t ptc_adam_k(float2 *W, const float2 *gW, float2 *m, float2 *v, size_t n, int step, double lr, double b1,
                      double b2, double eps, hipStream_t st) {
  const float c1 = (float)(1.0 - pow(b1, step)), c2 = (float)(1.0 - pow(b2, step));
  hipLaunchKernelGGL(k_ptc_adam, dim3(div_up((long)n, 256)), dim3(256), 0, st, W, gW, m, v, n, (float)lr, (float)b1,
                     (float)b2, (float)eps, c1, c2);
  return hipGetLastError();
}

}  // namespace mg
