// Flexible GCR ("Formulating an algorithm": GCR restarted every m steps,
// flexible because the multigrid preconditioner changes from step to step)
// with the solution update deferred to the end of each restart cycle.
//
// Step j of a cycle has the preconditioned vector z_j = K(r_j) and w_j =
// D z_j.  Classical Gram-Schmidt against the earlier directions, kept
// unnormalised, gives
//   w^_j = w_j - sum_{i<j} g_ij w^_i,   g_ij = <w^_i, w_j> / ||w^_i||^2,
// and the residual moves along w^_j:
//   r_{j+1} = r_j - a_j w^_j,           a_j = <w^_j, r_j> / ||w^_j||^2.
// With W = [w_j] and W^ = [w^_j], W = W^ T for the unit upper-triangular T
// with T_ij = g_ij (i < j), so the vectors whose images are w^_j are
// Z^ = Z T^{-1} and the cycle's solution update is
//   x += Z^ a = Z c,                    T c = a (back substitution).
// This is the same iterate as updating x and orthogonalising z_j with every
// step (GCR in its usual form) up to rounding, without the per-step passes
// over Z and x: the raw z_j are written once by the preconditioner and read
// once at the end of the cycle, in the preconditioner's storage precision.
//
// Device scalars per right-hand side (GcrScalars): gam[i * m + j] = g_ij,
// a[j], e[i] = <w^_i, r_j> and f = <w_j, r_j> of the current step (so that
// <w^_j, r_j> = f - sum_i conj(g_ij) e_i), nu2[j] = ||w^_j||^2, c[j], and the
// number of steps taken in the cycle, cnt.  Vectors are flat complex arrays
// of n entries per right-hand side (blockIdx.y = right-hand side).
#include "solver.h"

namespace mg {

static inline int ggrid(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b < RED_BLOCKS ? (b == 0 ? 1 : b) : RED_BLOCKS);
}
#define GSTRIDE(i, n) \
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

namespace {

// Per-RHS scalar block inside gs (double2) / nu2 (double) / cnt (int);
// flag->x != 0: the fused step's a_j waits for the measured ||w^_j||^2.
struct GS {
  double2 *gam, *a, *e, *f, *c, *flag;
  double *nu2;
};
__device__ __forceinline__ GS gs_of(double2 *gs, double *nu, int m, int rhs) {
  GS s;
  double2 *b = gs + (size_t)rhs * gcr_scalars_per_rhs(m);
  s.gam = b;
  s.a = b + (size_t)m * m;
  s.e = s.a + m;
  s.c = s.e + m;
  s.f = s.c + m;
  s.flag = s.f + 1;
  s.nu2 = nu + (size_t)rhs * m;
  return s;
}
__device__ __forceinline__ bool gs_flag(const double2 *gs, int m, int rhs) {
  return gs[(size_t)rhs * gcr_scalars_per_rhs(m) + (size_t)m * m + 3 * (size_t)m + 1].x != 0.0;
}

template <int W>
__device__ __forceinline__ void block_partials(double (&t)[W], double *part) {
  __shared__ double lds[4 * W];
  block_sum<W>(t, lds);
  if (threadIdx.x == 0) {
    double *p = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * W;
#pragma unroll
    for (int q = 0; q < W; ++q) p[q] = t[q];
  }
}

// Sum np partials of width W of this workgroup's right-hand side (thread 0).
template <int W> __device__ __forceinline__ void fin(const double *__restrict__ part, int np, double (&tot)[W]) {
  __shared__ double lds[4 * W];
  part += (size_t)blockIdx.y * np * W;
#pragma unroll
  for (int q = 0; q < W; ++q) tot[q] = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
#pragma unroll
    for (int q = 0; q < W; ++q) tot[q] += part[(size_t)i * W + q];
  }
  block_sum<W>(tot, lds);
}

constexpr int DW = 4 * GCR_CHUNK + 3;  // partial width of the inner-product pass

// Inner products of one chunk of earlier directions w^_{i0..i0+ni-1} with w_j
// and with r; with i0 == 0 also <w_j, r> and ||w_j||^2.
__global__ __launch_bounds__(256) void k_gcr2_dots(const double2 *__restrict__ Wh, size_t vs, int ni,
                                                   const double2 *__restrict__ wj, const double2 *__restrict__ r,
                                                   size_t n, int first, const int *skip, double *part) {
  const size_t off = (size_t)blockIdx.y * n;
  double t[DW];
#pragma unroll
  for (int q = 0; q < DW; ++q) t[q] = 0.0;
  if (!(skip && skip[blockIdx.y])) {
    GSTRIDE(idx, n) {
      const double2 w = wj[off + idx], rv = r[off + idx];
#pragma unroll
      for (int i = 0; i < GCR_CHUNK; ++i) {
        if (i < ni) {
          const double2 v = Wh[(size_t)i * vs + off + idx];
          t[4 * i] += v.x * w.x + v.y * w.y;
          t[4 * i + 1] += v.x * w.y - v.y * w.x;
          t[4 * i + 2] += v.x * rv.x + v.y * rv.y;
          t[4 * i + 3] += v.x * rv.y - v.y * rv.x;
        }
      }
      if (first) {
        t[4 * GCR_CHUNK] += w.x * rv.x + w.y * rv.y;
        t[4 * GCR_CHUNK + 1] += w.x * rv.y - w.y * rv.x;
        t[4 * GCR_CHUNK + 2] += w.x * w.x + w.y * w.y;
      }
    }
  }
  block_partials<DW>(t, part);
}

// g_ij and e_i of the chunk; with i0 == 0 f = <w_j, r>; at j == 0 (no
// earlier directions) w^_0 = w_0, so ||w^_0||^2 and a_0 are final here.
__global__ void k_gcr2_dots_fin(const double *part, int np, int i0, int ni, int j, int m, double2 *gs,
                                double *nu, int *cnt, const int *skip) {
  if (skip && skip[blockIdx.y]) return;
  double t[DW];
  fin<DW>(part, np, t);
  if (threadIdx.x != 0) return;
  GS s = gs_of(gs, nu, m, blockIdx.y);
  for (int i = 0; i < ni; ++i) {
    const double nn = s.nu2[i0 + i];
    const double inv = nn > 0.0 ? 1.0 / nn : 0.0;
    s.gam[(size_t)(i0 + i) * m + j] = make_double2(t[4 * i] * inv, t[4 * i + 1] * inv);
    s.e[i0 + i] = make_double2(t[4 * i + 2], t[4 * i + 3]);
  }
  if (i0 == 0) s.f[0] = make_double2(t[4 * GCR_CHUNK], t[4 * GCR_CHUNK + 1]);
  if (j == 0) {
    const double nn = t[4 * GCR_CHUNK + 2];
    s.nu2[0] = nn;
    const double2 g = s.f[0];
    s.a[0] = nn > 0.0 ? make_double2(g.x / nn, g.y / nn) : make_double2(0.0, 0.0);
    cnt[blockIdx.y] = 1;
  }
}

// w^_j = w_j - sum over the chunk g_ij w^_i (in place); partial ||w^_j||^2.
__global__ __launch_bounds__(256) void k_gcr2_orth(const double2 *__restrict__ Wh, size_t vs, int i0, int ni,
                                                   double2 *wj, size_t n, int j, int m, const double2 *gs,
                                                   const int *skip, double *part) {
  const size_t off = (size_t)blockIdx.y * n;
  double t[1] = {0.0};
  if (!(skip && skip[blockIdx.y])) {
    const double2 *gam = gs + (size_t)blockIdx.y * gcr_scalars_per_rhs(m);
    double2 c[GCR_CHUNK];
#pragma unroll
    for (int i = 0; i < GCR_CHUNK; ++i) {
      const double2 v = i < ni ? gam[(size_t)(i0 + i) * m + j] : make_double2(0.0, 0.0);
      c[i] = make_double2(-v.x, -v.y);
    }
    GSTRIDE(idx, n) {
      double2 w = wj[off + idx];
#pragma unroll
      for (int i = 0; i < GCR_CHUNK; ++i)
        if (i < ni) w = cfma(c[i], Wh[(size_t)i * vs + off + idx], w);
      wj[off + idx] = w;
      t[0] += w.x * w.x + w.y * w.y;
    }
  }
  block_partials<1>(t, part);
}

// ||w^_j||^2, then a_j = (f - sum_{i<j} conj(g_ij) e_i) / ||w^_j||^2.
__global__ void k_gcr2_orth_fin(const double *part, int np, int j, int m, double2 *gs, double *nu, int *cnt,
                                const int *skip) {
  if (skip && skip[blockIdx.y]) return;
  double t[1];
  fin<1>(part, np, t);
  if (threadIdx.x != 0) return;
  GS s = gs_of(gs, nu, m, blockIdx.y);
  s.nu2[j] = t[0];
  double2 g = s.f[0];
  for (int i = 0; i < j; ++i) {
    const double2 gi = s.gam[(size_t)i * m + j], ei = s.e[i];
    // conj(g_ij) e_i
    g.x -= gi.x * ei.x + gi.y * ei.y;
    g.y -= gi.x * ei.y - gi.y * ei.x;
  }
  s.a[j] = t[0] > 0.0 ? make_double2(g.x / t[0], g.y / t[0]) : make_double2(0.0, 0.0);
  cnt[blockIdx.y] = j + 1;
}

// r -= a_j w^_j; partial ||r||^2; optionally r32 = r rounded to FP32 (the
// next preconditioner input).
__global__ __launch_bounds__(256) void k_gcr2_rupd(double2 *r, const double2 *__restrict__ wj, size_t n, int j,
                                                   int m, const double2 *gs, const int *skip, double *part,
                                                   float2 *r32, int flagged_only) {
  if (flagged_only && !gs_flag(gs, m, blockIdx.y)) return;
  const size_t off = (size_t)blockIdx.y * n;
  double t[1] = {0.0};
  if (!(skip && skip[blockIdx.y])) {
    const double2 a = gs[(size_t)blockIdx.y * gcr_scalars_per_rhs(m) + (size_t)m * m + j];
    const double2 ma = make_double2(-a.x, -a.y);
    GSTRIDE(idx, n) {
      const double2 rv = cfma(ma, wj[off + idx], r[off + idx]);
      r[off + idx] = rv;
      if (r32) r32[off + idx] = make_float2((float)rv.x, (float)rv.y);
      t[0] += rv.x * rv.x + rv.y * rv.y;
    }
  }
  block_partials<1>(t, part);
}

// The same with the next preconditioner input in binary16 with a per-site
// scale (r16, 13 slots per site): one site (12 entries) per thread, over the
// Vpad sites of the fine level.
__global__ __launch_bounds__(256) void k_gcr2_rupd_h(double2 *r, const double2 *__restrict__ wj, uint32_t Vpad,
                                                     int j, int m, const double2 *gs, const int *skip, double *part,
                                                     h16 *r16, int flagged_only) {
  if (flagged_only && !gs_flag(gs, m, blockIdx.y)) return;
  const size_t off = (size_t)blockIdx.y * 12 * Vpad;
  double t[1] = {0.0};
  if (!(skip && skip[blockIdx.y])) {
    const double2 a = gs[(size_t)blockIdx.y * gcr_scalars_per_rhs(m) + (size_t)m * m + j];
    const double2 ma = make_double2(-a.x, -a.y);
    h16 *o16 = r16 + (size_t)blockIdx.y * 13 * Vpad;
    GSTRIDE(i, Vpad) {
      const uint32_t s = (uint32_t)i;
      double2 rv[12], w[12];
      load_site(rv, r + off, s);
      load_site(w, wj + off, s);
      float2 f[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        rv[c] = cfma(ma, w[c], rv[c]);
        t[0] += rv[c].x * rv[c].x + rv[c].y * rv[c].y;
        f[c] = make_float2((float)rv[c].x, (float)rv[c].y);
      }
      store_site(r + off, s, rv);
      store_site(o16, s, f);
    }
  }
  block_partials<1>(t, part);
}

// ---- fused step (1 <= j <= GCR_CHUNK, one chunk of earlier directions)
// After k_gcr2_dots over all j earlier directions: g_ij, e_i, f as
// k_gcr2_dots_fin, and a_j from the Pythagorean ||w^_j||^2 unless it has
// cancelled (then flag).
constexpr double GCR_CANCEL = 1e-4;
__global__ void k_gcr2_dots_fin_fused(const double *part, int np, int j, int m, double2 *gs, double *nu, int *cnt,
                                      const int *skip, double cancel) {
  if (skip && skip[blockIdx.y]) return;
  double t[DW];
  fin<DW>(part, np, t);
  if (threadIdx.x != 0) return;
  GS s = gs_of(gs, nu, m, blockIdx.y);
  const double ww = t[4 * GCR_CHUNK + 2];
  double proj = 0.0;
  double2 g = make_double2(t[4 * GCR_CHUNK], t[4 * GCR_CHUNK + 1]);
  s.f[0] = g;
  for (int i = 0; i < j; ++i) {
    const double nn = s.nu2[i];
    const double inv = nn > 0.0 ? 1.0 / nn : 0.0;
    const double2 gi = make_double2(t[4 * i] * inv, t[4 * i + 1] * inv), ei = make_double2(t[4 * i + 2], t[4 * i + 3]);
    s.gam[(size_t)i * m + j] = gi;
    s.e[i] = ei;
    proj += (t[4 * i] * t[4 * i] + t[4 * i + 1] * t[4 * i + 1]) * inv;
    // conj(g_ij) e_i
    g.x -= gi.x * ei.x + gi.y * ei.y;
    g.y -= gi.x * ei.y - gi.y * ei.x;
  }
  const double nw2 = ww - proj;
  if (nw2 > cancel * ww) {
    s.nu2[j] = nw2;
    s.a[j] = make_double2(g.x / nw2, g.y / nw2);
    s.flag[0] = make_double2(0.0, 0.0);
  } else {
    s.a[j] = make_double2(0.0, 0.0);
    s.flag[0] = make_double2(1.0, 0.0);
  }
  cnt[blockIdx.y] = j + 1;
}

// w^_j = w_j - sum_i g_ij w^_i (in place) and, unless flagged, r -= a_j w^_j
// (r32 = r in FP32 when given); partials ||w^_j||^2, ||r||^2.
__global__ __launch_bounds__(256) void k_gcr2_orth_rupd(const double2 *__restrict__ Wh, size_t vs, int ni,
                                                        double2 *wj, double2 *r, size_t n, int j, int m,
                                                        const double2 *gs, const int *skip, double *part,
                                                        float2 *r32) {
  const size_t off = (size_t)blockIdx.y * n;
  double t[2] = {0.0, 0.0};
  if (!(skip && skip[blockIdx.y])) {
    const double2 *b = gs + (size_t)blockIdx.y * gcr_scalars_per_rhs(m);
    const bool fl = gs_flag(gs, m, blockIdx.y);
    const double2 a = b[(size_t)m * m + j];
    const double2 ma = make_double2(-a.x, -a.y);
    double2 c[GCR_CHUNK];
#pragma unroll
    for (int i = 0; i < GCR_CHUNK; ++i) {
      const double2 v = i < ni ? b[(size_t)i * m + j] : make_double2(0.0, 0.0);
      c[i] = make_double2(-v.x, -v.y);
    }
    GSTRIDE(idx, n) {
      double2 w = wj[off + idx];
#pragma unroll
      for (int i = 0; i < GCR_CHUNK; ++i)
        if (i < ni) w = cfma(c[i], Wh[(size_t)i * vs + off + idx], w);
      wj[off + idx] = w;
      t[0] += w.x * w.x + w.y * w.y;
      if (!fl) {
        const double2 rv = cfma(ma, w, r[off + idx]);
        r[off + idx] = rv;
        if (r32) r32[off + idx] = make_float2((float)rv.x, (float)rv.y);
        t[1] += rv.x * rv.x + rv.y * rv.y;
      }
    }
  }
  block_partials<2>(t, part);
}

// The same with the next preconditioner input in binary16 with a per-site
// scale (r16): one site per thread over the Vpad sites of the fine level.
__global__ __launch_bounds__(256) void k_gcr2_orth_rupd_h(const double2 *__restrict__ Wh, size_t vs, int ni,
                                                          double2 *wj, double2 *r, uint32_t Vpad, int j, int m,
                                                          const double2 *gs, const int *skip, double *part,
                                                          h16 *r16) {
  const size_t off = (size_t)blockIdx.y * 12 * Vpad;
  double t[2] = {0.0, 0.0};
  if (!(skip && skip[blockIdx.y])) {
    const double2 *b = gs + (size_t)blockIdx.y * gcr_scalars_per_rhs(m);
    const bool fl = gs_flag(gs, m, blockIdx.y);
    const double2 a = b[(size_t)m * m + j];
    const double2 ma = make_double2(-a.x, -a.y);
    double2 c[GCR_CHUNK];
#pragma unroll
    for (int i = 0; i < GCR_CHUNK; ++i) {
      const double2 v = i < ni ? b[(size_t)i * m + j] : make_double2(0.0, 0.0);
      c[i] = make_double2(-v.x, -v.y);
    }
    h16 *o16 = r16 + (size_t)blockIdx.y * 13 * Vpad;
    GSTRIDE(i, Vpad) {
      const uint32_t s = (uint32_t)i;
      double2 w[12];
      load_site(w, wj + off, s);
#pragma unroll
      for (int q = 0; q < GCR_CHUNK; ++q) {
        if (q < ni) {
          double2 h[12];
          load_site(h, Wh + (size_t)q * vs + off, s);
#pragma unroll
          for (int e = 0; e < 12; ++e) w[e] = cfma(c[q], h[e], w[e]);
        }
      }
      store_site(wj + off, s, w);
#pragma unroll
      for (int e = 0; e < 12; ++e) t[0] += w[e].x * w[e].x + w[e].y * w[e].y;
      if (!fl) {
        double2 rv[12];
        float2 f[12];
        load_site(rv, r + off, s);
#pragma unroll
        for (int e = 0; e < 12; ++e) {
          rv[e] = cfma(ma, w[e], rv[e]);
          t[1] += rv[e].x * rv[e].x + rv[e].y * rv[e].y;
          f[e] = make_float2((float)rv[e].x, (float)rv[e].y);
        }
        store_site(r + off, s, rv);
        store_site(o16, s, f);
      }
    }
  }
  block_partials<2>(t, part);
}

// nu2[j] = measured ||w^_j||^2; unflagged: rr = ||r||^2; flagged: a_j from
// the measured ||w^_j||^2 (the residual follows in a second pass).
__global__ void k_gcr2_orth_rupd_fin(const double *part, int np, int j, int m, double2 *gs, double *nu, double *rr,
                                     const int *skip) {
  if (skip && skip[blockIdx.y]) return;
  double t[2];
  fin<2>(part, np, t);
  if (threadIdx.x != 0) return;
  GS s = gs_of(gs, nu, m, blockIdx.y);
  s.nu2[j] = t[0];
  if (s.flag[0].x == 0.0) {
    rr[blockIdx.y] = t[1];
    return;
  }
  double2 g = s.f[0];
  for (int i = 0; i < j; ++i) {
    const double2 gi = s.gam[(size_t)i * m + j], ei = s.e[i];
    g.x -= gi.x * ei.x + gi.y * ei.y;
    g.y -= gi.x * ei.y - gi.y * ei.x;
  }
  s.a[j] = t[0] > 0.0 ? make_double2(g.x / t[0], g.y / t[0]) : make_double2(0.0, 0.0);
}

// c = T^{-1} a over the cnt steps of the cycle (one thread per right-hand side).
__global__ void k_gcr2_backsub(double2 *gs, double *nu, const int *cnt, int m, int nrhs) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  GS s = gs_of(gs, nu, m, rhs);
  const int k = cnt[rhs];
  for (int q = k; q < m; ++q) s.c[q] = make_double2(0.0, 0.0);
  for (int q = k - 1; q >= 0; --q) {
    double2 v = s.a[q];
    for (int l = q + 1; l < k; ++l) {
      const double2 g = s.gam[(size_t)q * m + l], cl = s.c[l];
      v.x -= g.x * cl.x - g.y * cl.y;
      v.y -= g.x * cl.y + g.y * cl.x;
    }
    s.c[q] = v;
  }
}

// x += sum over a chunk of steps c_q z_q (z in storage type TZ).
template <typename TZ>
__global__ __launch_bounds__(256) void k_gcr2_xupd(double2 *x, const TZ *__restrict__ Z, size_t vs, int q0, int nq,
                                                   size_t n, int m, const double2 *gs, const int *cnt) {
  const size_t off = (size_t)blockIdx.y * n;
  const int k = cnt[blockIdx.y];
  if (q0 >= k) return;
  const double2 *c = gs + (size_t)blockIdx.y * gcr_scalars_per_rhs(m) + (size_t)m * m + 2 * (size_t)m;
  double2 cc[GCR_CHUNK];
#pragma unroll
  for (int i = 0; i < GCR_CHUNK; ++i) cc[i] = (i < nq && q0 + i < k) ? c[q0 + i] : make_double2(0.0, 0.0);
  GSTRIDE(idx, n) {
    double2 v = x[off + idx];
#pragma unroll
    for (int i = 0; i < GCR_CHUNK; ++i)
      if (i < nq) v = cfma(cc[i], cvt<double2>(Z[(size_t)i * vs + off + idx]), v);
    x[off + idx] = v;
  }
}

__global__ void k_gcr2_fin1(const double *part, int np, double *out, const int *skip, const double2 *gs, int m) {
  if (skip && skip[blockIdx.y]) return;
  if (gs && !gs_flag(gs, m, blockIdx.y)) return;
  double t[1];
  fin<1>(part, np, t);
  if (threadIdx.x == 0) out[blockIdx.y] = t[0];
}

}  // namespace

hipError_t gcr2_step(double2 *Wh, size_t vs, int j, int m, const double2 *r_in, size_t n, int nrhs,
                     double2 *gs, double *nu, int *cnt, const int *skip, double *part, hipStream_t st) {
  const int g = ggrid(n);
  double2 *wj = Wh + (size_t)j * vs;
  if (j == 0) {
    hipLaunchKernelGGL(k_gcr2_dots, dim3(g, nrhs), dim3(256), 0, st, Wh, vs, 0, wj, r_in, n, 1, skip, part);
    hipLaunchKernelGGL(k_gcr2_dots_fin, dim3(1, nrhs), dim3(256), 0, st, part, g, 0, 0, 0, m, gs, nu, cnt, skip);
    return hipGetLastError();
  }
  for (int i0 = 0; i0 < j; i0 += GCR_CHUNK) {
    const int ni = j - i0 < GCR_CHUNK ? j - i0 : GCR_CHUNK;
    hipLaunchKernelGGL(k_gcr2_dots, dim3(g, nrhs), dim3(256), 0, st, Wh + (size_t)i0 * vs, vs, ni, wj, r_in, n,
                       i0 == 0 ? 1 : 0, skip, part);
    hipLaunchKernelGGL(k_gcr2_dots_fin, dim3(1, nrhs), dim3(256), 0, st, part, g, i0, ni, j, m, gs, nu, cnt, skip);
  }
  for (int i0 = 0; i0 < j; i0 += GCR_CHUNK) {
    const int ni = j - i0 < GCR_CHUNK ? j - i0 : GCR_CHUNK;
    hipLaunchKernelGGL(k_gcr2_orth, dim3(g, nrhs), dim3(256), 0, st, Wh + (size_t)i0 * vs, vs, i0, ni, wj, n, j, m,
                       (const double2 *)gs, skip, part);
  }
  hipLaunchKernelGGL(k_gcr2_orth_fin, dim3(1, nrhs), dim3(256), 0, st, part, g, j, m, gs, nu, cnt, skip);
  return hipGetLastError();
}

hipError_t gcr2_residual(double2 *r, const double2 *Wh, size_t vs, int j, int m, size_t n, int nrhs,
                         const double2 *gs, const int *skip, double *part, double *rr, float2 *r32, h16 *r16,
                         hipStream_t st) {
  if (r16) {
    const uint32_t Vpad = (uint32_t)(n / 12);
    const int g = ggrid(Vpad);
    hipLaunchKernelGGL(k_gcr2_rupd_h, dim3(g, nrhs), dim3(256), 0, st, r, Wh + (size_t)j * vs, Vpad, j, m, gs, skip,
                       part, r16, 0);
    hipLaunchKernelGGL(k_gcr2_fin1, dim3(1, nrhs), dim3(256), 0, st, part, g, rr, skip, nullptr, m);
    return hipGetLastError();
  }
  const int g = ggrid(n);
  hipLaunchKernelGGL(k_gcr2_rupd, dim3(g, nrhs), dim3(256), 0, st, r, Wh + (size_t)j * vs, n, j, m, gs, skip,
                     part, r32, 0);
  hipLaunchKernelGGL(k_gcr2_fin1, dim3(1, nrhs), dim3(256), 0, st, part, g, rr, skip, nullptr, m);
  return hipGetLastError();
}

hipError_t gcr2_step_residual(double2 *Wh, size_t vs, int j, int m, double2 *r, size_t n, int nrhs, double2 *gs,
                              double *nu, int *cnt, const int *skip, double *part, double *rr, float2 *r32,
                              h16 *r16, int mode, hipStream_t st) {
  if (mode == 0 || j < 1 || j > GCR_CHUNK) {
    hipError_t e = gcr2_step(Wh, vs, j, m, r, n, nrhs, gs, nu, cnt, skip, part, st);
    if (e != hipSuccess) return e;
    return gcr2_residual(r, Wh, vs, j, m, n, nrhs, gs, skip, part, rr, r32, r16, st);
  }
  const int g = ggrid(n);
  double2 *wj = Wh + (size_t)j * vs;
  hipLaunchKernelGGL(k_gcr2_dots, dim3(g, nrhs), dim3(256), 0, st, Wh, vs, j, wj, r, n, 1, skip, part);
  // mode 2: a threshold no difference passes (every step takes the second pass)
  const double cancel = mode == 2 ? 2.0 : GCR_CANCEL;
  hipLaunchKernelGGL(k_gcr2_dots_fin_fused, dim3(1, nrhs), dim3(256), 0, st, part, g, j, m, gs, nu, cnt, skip,
                     cancel);
  if (r16) {
    const uint32_t Vpad = (uint32_t)(n / 12);
    const int gh = ggrid(Vpad);
    hipLaunchKernelGGL(k_gcr2_orth_rupd_h, dim3(gh, nrhs), dim3(256), 0, st, Wh, vs, j, wj, r, Vpad, j, m,
                       (const double2 *)gs, skip, part, r16);
    hipLaunchKernelGGL(k_gcr2_orth_rupd_fin, dim3(1, nrhs), dim3(256), 0, st, part, gh, j, m, gs, nu, rr, skip);
    hipLaunchKernelGGL(k_gcr2_rupd_h, dim3(gh, nrhs), dim3(256), 0, st, r, wj, Vpad, j, m, (const double2 *)gs, skip,
                       part, r16, 1);
    hipLaunchKernelGGL(k_gcr2_fin1, dim3(1, nrhs), dim3(256), 0, st, part, gh, rr, skip, (const double2 *)gs, m);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_gcr2_orth_rupd, dim3(g, nrhs), dim3(256), 0, st, Wh, vs, j, wj, r, n, j, m,
                     (const double2 *)gs, skip, part, r32);
  hipLaunchKernelGGL(k_gcr2_orth_rupd_fin, dim3(1, nrhs), dim3(256), 0, st, part, g, j, m, gs, nu, rr, skip);
  hipLaunchKernelGGL(k_gcr2_rupd, dim3(g, nrhs), dim3(256), 0, st, r, wj, n, j, m, (const double2 *)gs, skip, part,
                     r32, 1);
  hipLaunchKernelGGL(k_gcr2_fin1, dim3(1, nrhs), dim3(256), 0, st, part, g, rr, skip, (const double2 *)gs, m);
  return hipGetLastError();
}

template <typename TZ>
hipError_t gcr2_solution(double2 *x, const TZ *Z, size_t vs, int kmax, int m, size_t n, int nrhs, double2 *gs,
                         double *nu, const int *cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_gcr2_backsub, dim3(1), dim3(64), 0, st, gs, nu, cnt, m, nrhs);
  const int g = ggrid(n);
  for (int q0 = 0; q0 < kmax; q0 += GCR_CHUNK) {
    const int nq = kmax - q0 < GCR_CHUNK ? kmax - q0 : GCR_CHUNK;
    hipLaunchKernelGGL(k_gcr2_xupd<TZ>, dim3(g, nrhs), dim3(256), 0, st, x, Z + (size_t)q0 * vs, vs, q0, nq, n, m,
                       (const double2 *)gs, cnt);
  }
  return hipGetLastError();
}

template hipError_t gcr2_solution<double2>(double2 *, const double2 *, size_t, int, int, size_t, int, double2 *,
                                           double *, const int *, hipStream_t);
template hipError_t gcr2_solution<float2>(double2 *, const float2 *, size_t, int, int, size_t, int, double2 *,
                                          double *, const int *, hipStream_t);

}  // namespace mg
