// Streaming kernels of the Krylov / smoothing loops.  Scalars (inner
// products, step lengths, convergence flags) stay on the device: reductions
// write per-block partials, a one-workgroup finisher per right-hand side sums
// them in a fixed order and derives the coefficient, and the consuming kernel
// reads it.  The host only reads residual norms for convergence decisions.
// Vectors are flat complex arrays of N entries per right-hand side
// (blockIdx.y = right-hand side); any site layout works.
#include <algorithm>

#include "solver.h"

namespace mg {

static inline int sgrid(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b < RED_BLOCKS ? (b == 0 ? 1 : b) : RED_BLOCKS);
}
#define GSTRIDE(i, n) \
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

// --------------------------------------------------------------- finishers
// Sum np partials of width w (stride w) for the RHS blockIdx.y into tot[0..w).
// Each thread loads FU of its partials before adding them (fixed order), so
// that their round trips overlap: with np = 8192 a thread takes 32, and one
// dependent load after another made the MR step-length kernel take 16 us.
template <int W>
__device__ __forceinline__ void finish_sum(const double *__restrict__ part, int np, double (&tot)[W]) {
  constexpr int FU = 8;
  __shared__ double lds[4 * W];
  part += (size_t)blockIdx.y * np * W;
#pragma unroll
  for (int q = 0; q < W; ++q) tot[q] = 0.0;
  const int bd = (int)blockDim.x;
  int i = (int)threadIdx.x;
  for (; i + (FU - 1) * bd < np; i += FU * bd) {
    double v[FU][W];
#pragma unroll
    for (int u = 0; u < FU; ++u)
#pragma unroll
      for (int q = 0; q < W; ++q) v[u][q] = part[(size_t)(i + u * bd) * W + q];
#pragma unroll
    for (int u = 0; u < FU; ++u)
#pragma unroll
      for (int q = 0; q < W; ++q) tot[q] += v[u][q];
  }
  for (; i < np; i += bd) {
#pragma unroll
    for (int q = 0; q < W; ++q) tot[q] += part[(size_t)i * W + q];
  }
  block_sum<W>(tot, lds);
}

// MR: alpha = omega <q,r> / <q,q>  (stored as complex; 0 when q = 0)
__global__ void k_fin_mr(const double *part, int np, double omega, double2 *alpha) {
  double t[3];
  finish_sum<3>(part, np, t);
  if (threadIdx.x == 0) {
    double2 a = make_double2(0.0, 0.0);
    if (t[2] > 0.0) a = make_double2(omega * t[0] / t[2], omega * t[1] / t[2]);
    alpha[blockIdx.y] = a;
  }
}

// plain sums: out[rhs*W + q]
template <int W> __global__ void k_fin_sum(const double *part, int np, double *out) {
  double t[W];
  finish_sum<W>(part, np, t);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < W; ++q) out[(size_t)blockIdx.y * W + q] = t[q];
  }
}

// --------------------------------------------------------------- reductions
template <typename R>
__global__ __launch_bounds__(256) void k_norm2(const c_t<R> *a, size_t n, double *part) {
  __shared__ double lds[4];
  a += (size_t)blockIdx.y * n;
  double t[1] = {0.0};
  GSTRIDE(i, n) {
    const c_t<R> v = a[i];
    t[0] += (double)v.x * v.x + (double)v.y * v.y;
  }
  block_sum<1>(t, lds);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t[0];
}

// <a, b> = sum conj(a) b -> 2 doubles per block
template <typename R>
__global__ __launch_bounds__(256) void k_dot(const c_t<R> *a, const c_t<R> *b, size_t n, double *part) {
  __shared__ double lds[8];
  a += (size_t)blockIdx.y * n;
  b += (size_t)blockIdx.y * n;
  double t[2] = {0.0, 0.0};
  GSTRIDE(i, n) {
    const c_t<R> u = a[i], v = b[i];
    t[0] += (double)u.x * v.x + (double)u.y * v.y;
    t[1] += (double)u.x * v.y - (double)u.y * v.x;
  }
  block_sum<2>(t, lds);
  if (threadIdx.x == 0) {
    double *p = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
    p[0] = t[0];
    p[1] = t[1];
  }
}

// --------------------------------------------------------------- updates
// MR: x = (first ? 0 : x) + alpha r;  r -= alpha q
template <typename R>
__global__ __launch_bounds__(256) void k_mr_update(c_t<R> *x, c_t<R> *r_out, const c_t<R> *r_in, const c_t<R> *q,
                                                   size_t n, const double2 *alpha, int first, int upd_r) {
  using C = c_t<R>;
  const size_t off = (size_t)blockIdx.y * n;
  x += off; r_out += off; r_in += off; q += off;
  const double2 ad = alpha[blockIdx.y];
  const C a = mk<C>((R)ad.x, (R)ad.y), ma = mk<C>((R)-ad.x, (R)-ad.y);
  if (upd_r) {
    GSTRIDE(i, n) {
      const C rv = r_in[i];
      x[i] = first ? cmul(a, rv) : cfma(a, rv, x[i]);
      r_out[i] = cfma(ma, q[i], rv);
    }
  } else {
    GSTRIDE(i, n) x[i] = first ? cmul(a, r_in[i]) : cfma(a, r_in[i], x[i]);
  }
}

// The same on the fine level with the residual and q stored in binary16 with
// a per-site scale (x in FP32): one site per thread, so that the new
// residual's scale is formed from all 12 of its components.
__global__ __launch_bounds__(256) void k_mr_update_h(float2 *x, h16 *r_out, const h16 *r_in, const h16 *q,
                                                     uint32_t V, uint32_t Vpad, const double2 *alpha, int first,
                                                     int upd_r) {
  x += (size_t)blockIdx.y * 12 * Vpad;
  const size_t off = (size_t)blockIdx.y * 13 * Vpad;
  r_out += off; r_in += off; q += off;
  const double2 ad = alpha[blockIdx.y];
  const float2 a = make_float2((float)ad.x, (float)ad.y), ma = make_float2((float)-ad.x, (float)-ad.y);
  GSTRIDE(i, V) {
    const uint32_t s = (uint32_t)i;
    float2 rv[12], xv[12];
    load_site(rv, r_in, s);
    if (first) {
#pragma unroll
      for (int c = 0; c < 12; ++c) xv[c] = cmul(a, rv[c]);
    } else {
      load_site(xv, x, s);
#pragma unroll
      for (int c = 0; c < 12; ++c) xv[c] = cfma(a, rv[c], xv[c]);
    }
    store_site(x, s, xv);
    if (upd_r) {
      float2 qv[12];
      load_site(qv, q, s);
#pragma unroll
      for (int c = 0; c < 12; ++c) rv[c] = cfma(ma, qv[c], rv[c]);
      store_site(r_out, s, rv);
    }
  }
}

// MR by the q recursion: x = (first ? 0 : x) + xs sum_k a_k r_k, and r_out =
// r_{n-1} - a_{n-1} q when upd_r.  One site per thread (the binary16 scale of
// r_out needs the whole site); the step loop is unrolled to MRQ_MAX so that
// the list of residuals stays in kernel arguments.
template <typename TR>
__global__ __launch_bounds__(256) void k_mrq_combine(float2 *x, TR *r_out, MrqList<TR> rs, const TR *q, uint32_t V,
                                                     uint32_t Vpad, int steps, const double2 *alpha, int first,
                                                     int upd_r, float xs) {
  x += (size_t)blockIdx.y * 12 * Vpad;
  const size_t off = (size_t)blockIdx.y * site_slots<TR>() * Vpad;
  GSTRIDE(i, V) {
    const uint32_t s = (uint32_t)i;
    float2 xv[12], rv[12];
    if (first) {
#pragma unroll
      for (int c = 0; c < 12; ++c) xv[c] = make_float2(0.f, 0.f);
    } else {
      load_site(xv, x, s);
    }
    float2 a = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < MRQ_MAX; ++k) {
      if (k < steps) {
        const double2 ad = alpha[(size_t)k * MG_MAX_RHS + blockIdx.y];
        a = make_float2((float)ad.x, (float)ad.y);
        const float2 ax = make_float2(xs * a.x, xs * a.y);
        load_site(rv, rs.r[k] + off, s);
#pragma unroll
        for (int c = 0; c < 12; ++c) xv[c] = cfma(ax, rv[c], xv[c]);
      }
    }
    store_site(x, s, xv);
    if (upd_r) {
      float2 qv[12];
      load_site(qv, q + off, s);
      const float2 ma = make_float2(-a.x, -a.y);
#pragma unroll
      for (int c = 0; c < 12; ++c) rv[c] = cfma(ma, qv[c], rv[c]);
      store_site(r_out + off, s, rv);
    }
  }
}

// y -= c x and v -= c u with c = sc[rhs] (complex)  (FGCR Gram-Schmidt)
__global__ __launch_bounds__(256) void k_sub2(double2 *y, const double2 *x, double2 *v, const double2 *u, size_t n,
                                              const double2 *sc, const int *skip) {
  if (skip && skip[blockIdx.y]) return;
  const size_t off = (size_t)blockIdx.y * n;
  y += off; x += off; v += off; u += off;
  const double2 c = sc[blockIdx.y];
  const double2 mc = make_double2(-c.x, -c.y);
  GSTRIDE(i, n) {
    y[i] = cfma(mc, x[i], y[i]);
    v[i] = cfma(mc, u[i], v[i]);
  }
}

// y *= 1/sqrt(nrm2[rhs]), v *= same
__global__ __launch_bounds__(256) void k_scale2(double2 *y, double2 *v, size_t n, const double *nrm2,
                                                const int *skip) {
  if (skip && skip[blockIdx.y]) return;
  const size_t off = (size_t)blockIdx.y * n;
  y += off; v += off;
  const double nn = nrm2[blockIdx.y];
  const double s = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
  GSTRIDE(i, n) {
    y[i] = cscale(y[i], s);
    v[i] = cscale(v[i], s);
  }
}

// FGCR orthogonalisation of w_j against up to GCR_CHUNK earlier directions
// w_i0 .. w_{i0+ni-1} by classical Gram-Schmidt: all inner products <w_i,
// w_j> in one pass (GCR_CHUNK x 2 partials per block), then one pass
// w_j -= sum c_i w_i, z_j -= sum c_i z_i with the partial ||w_j||^2.
__global__ __launch_bounds__(256) void k_gcr_mdot(const double2 *__restrict__ W, size_t vs, int ni,
                                                  const double2 *__restrict__ wj, size_t n, const int *skip,
                                                  double *part) {
  __shared__ double lds[4 * 2 * GCR_CHUNK];
  const size_t off = (size_t)blockIdx.y * n;
  double t[2 * GCR_CHUNK];
#pragma unroll
  for (int q = 0; q < 2 * GCR_CHUNK; ++q) t[q] = 0.0;
  if (!(skip && skip[blockIdx.y])) {
    GSTRIDE(idx, n) {
      const double2 w = wj[off + idx];
#pragma unroll
      for (int i = 0; i < GCR_CHUNK; ++i) {
        if (i < ni) {
          const double2 v = W[(size_t)i * vs + off + idx];
          t[2 * i] += v.x * w.x + v.y * w.y;
          t[2 * i + 1] += v.x * w.y - v.y * w.x;
        }
      }
    }
  }
  block_sum<2 * GCR_CHUNK>(t, lds);
  if (threadIdx.x == 0) {
    double *p = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2 * GCR_CHUNK;
#pragma unroll
    for (int q = 0; q < 2 * GCR_CHUNK; ++q) p[q] = t[q];
  }
}
__global__ void k_gcr_mdot_fin(const double *part, int np, int ni, double2 *sc) {
  double t[2 * GCR_CHUNK];
  finish_sum<2 * GCR_CHUNK>(part, np, t);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < GCR_CHUNK; ++i)
      if (i < ni) sc[(size_t)blockIdx.y * GCR_CHUNK + i] = make_double2(t[2 * i], t[2 * i + 1]);
  }
}
__global__ __launch_bounds__(256) void k_gcr_orth(const double2 *__restrict__ W, const double2 *__restrict__ Z,
                                                  size_t vs, int ni, double2 *wj, double2 *zj, size_t n,
                                                  const double2 *sc, const int *skip, double *part) {
  __shared__ double lds[4];
  const size_t off = (size_t)blockIdx.y * n;
  double t[1] = {0.0};
  if (!(skip && skip[blockIdx.y])) {
    double2 c[GCR_CHUNK];
#pragma unroll
    for (int i = 0; i < GCR_CHUNK; ++i) {
      const double2 v = i < ni ? sc[(size_t)blockIdx.y * GCR_CHUNK + i] : make_double2(0.0, 0.0);
      c[i] = make_double2(-v.x, -v.y);
    }
    GSTRIDE(idx, n) {
      double2 w = wj[off + idx], z = zj[off + idx];
#pragma unroll
      for (int i = 0; i < GCR_CHUNK; ++i) {
        if (i < ni) {
          w = cfma(c[i], W[(size_t)i * vs + off + idx], w);
          z = cfma(c[i], Z[(size_t)i * vs + off + idx], z);
        }
      }
      wj[off + idx] = w;
      zj[off + idx] = z;
      t[0] += w.x * w.x + w.y * w.y;
    }
  }
  block_sum<1>(t, lds);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t[0];
}

// x += a z; r -= a w (a = sc[rhs]); partial ||r||^2
__global__ __launch_bounds__(256) void k_gcr_update(double2 *x, const double2 *z, double2 *r, const double2 *w,
                                                    size_t n, const double2 *sc, const int *skip, double *part) {
  __shared__ double lds[4];
  const size_t off = (size_t)blockIdx.y * n;
  double t[1] = {0.0};
  const bool sk = skip && skip[blockIdx.y];
  if (!sk) {
    x += off; z += off; r += off; w += off;
    const double2 a = sc[blockIdx.y];
    const double2 ma = make_double2(-a.x, -a.y);
    GSTRIDE(i, n) {
      x[i] = cfma(a, z[i], x[i]);
      const double2 rv = cfma(ma, w[i], r[i]);
      r[i] = rv;
      t[0] += rv.x * rv.x + rv.y * rv.y;
    }
  } else {
    r += off;
    GSTRIDE(i, n) {
      const double2 rv = r[i];
      t[0] += rv.x * rv.x + rv.y * rv.y;
    }
  }
  block_sum<1>(t, lds);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t[0];
}

template <typename R>
__global__ __launch_bounds__(256) void k_sub(c_t<R> *v, const c_t<R> *x, size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  v += off; x += off;
  GSTRIDE(i, n) v[i] = csub(v[i], x[i]);
}
template <typename R>
__global__ __launch_bounds__(256) void k_add(c_t<R> *v, const c_t<R> *x, size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  v += off; x += off;
  GSTRIDE(i, n) v[i] = cadd(v[i], x[i]);
}
template <typename R>
__global__ __launch_bounds__(256) void k_scale_rsqrt(c_t<R> *v, size_t n, const double *nrm2) {
  v += (size_t)blockIdx.y * n;
  const double nn = nrm2[blockIdx.y];
  const R s = (R)(nn > 0.0 ? 1.0 / sqrt(nn) : 0.0);
  GSTRIDE(i, n) v[i] = cscale(v[i], s);
}
template <typename R>
__global__ __launch_bounds__(256) void k_resid_from(c_t<R> *out, const c_t<R> *b, size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  out += off; b += off;
  GSTRIDE(i, n) out[i] = csub(b[i], out[i]);
}

// --------------------------------------------------------------- CGNR (fused)
// Sum of np partials of RHS blockIdx.y over the workgroup, in every thread
// (fixed order: identical in every workgroup).
__device__ __forceinline__ double allsum(const double *__restrict__ p, int np, double *lds) {
  p += (size_t)blockIdx.y * np;
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) a += p[i];
  a = wave_sum(a);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = a;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < nw; ++q) t += lds[q];
  __syncthreads();
  return t;
}

// ||b||^2, tol^2, done = (b == 0), both iteration-count slots = 0
__global__ void k_cg2_init(const double *part_b, int npb, double *cg, int *done, int *it, double tol2) {
  __shared__ double lds[4];
  const double nb2 = allsum(part_b, npb, lds);
  if (threadIdx.x == 0) {
    double *c = cg + (size_t)blockIdx.y * CG_NS;
    c[3] = nb2;
    c[4] = tol2;
    it[blockIdx.y] = 0;
    it[gridDim.y + blockIdx.y] = 0;
    done[blockIdx.y] = nb2 > 0.0 ? 0 : 1;
  }
}

// alpha = zz / ww from the partials; e += alpha p; r -= alpha w; partial ||r||^2
template <typename R>
__global__ __launch_bounds__(256) void k_cg2_update(c_t<R> *e, const c_t<R> *p, c_t<R> *r, const c_t<R> *w, size_t n,
                                                    const double *part_w, const double *part_z, int npc, int *done,
                                                    double *part_r) {
  using C = c_t<R>;
  __shared__ double lds[4];
  if (done[blockIdx.y]) return;
  const double ww = allsum(part_w, npc, lds);
  const double zz = allsum(part_z, npc, lds);
  if (!(ww > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) done[blockIdx.y] = 1;
    return;
  }
  const R a = (R)(zz / ww);
  const size_t off = (size_t)blockIdx.y * n;
  e += off; p += off; r += off; w += off;
  double t[1] = {0.0};
  GSTRIDE(i, n) {
    e[i] = cfma(mk<C>(a, 0), p[i], e[i]);
    const C rv = cfma(mk<C>(-a, 0), w[i], r[i]);
    r[i] = rv;
    t[0] += (double)rv.x * rv.x + (double)rv.y * rv.y;
  }
  block_sum<1>(t, lds);
  if (threadIdx.x == 0) part_r[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t[0];
}

// beta = zz_new / zz_old from the partials; p = z + beta p
template <typename R>
__global__ __launch_bounds__(256) void k_cg2_p(c_t<R> *p, const c_t<R> *z, size_t n, const double *part_znew,
                                               const double *part_zold, int npc, const int *done) {
  using C = c_t<R>;
  __shared__ double lds[4];
  if (done[blockIdx.y]) return;
  const double zn = allsum(part_znew, npc, lds);
  const double zo = allsum(part_zold, npc, lds);
  const R b = (R)(zo > 0.0 ? zn / zo : 0.0);
  const size_t off = (size_t)blockIdx.y * n;
  p += off; z += off;
  GSTRIDE(i, n) p[i] = cfma(mk<C>(b, 0), p[i], z[i]);
}

// ====================================================================== host
hipError_t cg2_init(const double *part_b, int npb, int nrhs, double *cg, int *done, int *it, double tol,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_cg2_init, dim3(1, nrhs), dim3(256), 0, st, part_b, npb, cg, done, it, tol * tol);
  return hipGetLastError();
}
// The CGNR update kernels re-derive alpha and beta from the stencil's
// per-workgroup partials in every workgroup, so their grids are kept small.
constexpr int CG_BLOCKS = 64;
static inline int cgrid(size_t n) { return std::min(sgrid(n), CG_BLOCKS); }

template <typename R>
int cg2_update(c_t<R> *e, const c_t<R> *p, c_t<R> *r, const c_t<R> *w, size_t n, int nrhs, const double *part_w,
               const double *part_z, int npc, int *done, double *part_r, hipStream_t st) {
  const int g = cgrid(n);
  hipLaunchKernelGGL(k_cg2_update<R>, dim3(g, nrhs), dim3(256), 0, st, e, p, r, w, n, part_w, part_z, npc, done,
                     part_r);
  return g;
}
template <typename R>
hipError_t cg2_p(c_t<R> *p, const c_t<R> *z, size_t n, int nrhs, const double *part_znew, const double *part_zold,
                 int npc, const int *done, hipStream_t st) {
  hipLaunchKernelGGL(k_cg2_p<R>, dim3(cgrid(n), nrhs), dim3(256), 0, st, p, z, n, part_znew, part_zold, npc, done);
  return hipGetLastError();
}

template <typename R> hipError_t sub_inplace(c_t<R> *v, const c_t<R> *x, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_sub<R>, dim3(sgrid(n), nrhs), dim3(256), 0, st, v, x, n);
  return hipGetLastError();
}
template <typename R> hipError_t add_inplace(c_t<R> *v, const c_t<R> *x, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_add<R>, dim3(sgrid(n), nrhs), dim3(256), 0, st, v, x, n);
  return hipGetLastError();
}
template <typename R> hipError_t scale_rsqrt(c_t<R> *v, size_t n, int nrhs, const double *nrm2, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_rsqrt<R>, dim3(sgrid(n), nrhs), dim3(256), 0, st, v, n, nrm2);
  return hipGetLastError();
}
template <typename R> hipError_t resid_from(c_t<R> *out, const c_t<R> *b, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_resid_from<R>, dim3(sgrid(n), nrhs), dim3(256), 0, st, out, b, n);
  return hipGetLastError();
}

template <typename R>
hipError_t mr_update(c_t<R> *x, c_t<R> *r_out, const c_t<R> *r_in, const c_t<R> *q, size_t n, int nrhs,
                     const double *part, int np, double omega, double2 *alpha, int first, int upd_r,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_fin_mr, dim3(1, nrhs), dim3(256), 0, st, part, np, omega, alpha);
  hipLaunchKernelGGL(k_mr_update<R>, dim3(sgrid(n), nrhs), dim3(256), 0, st, x, r_out, r_in, q, n, alpha, first,
                     upd_r);
  return hipGetLastError();
}

hipError_t mr_update_h(float2 *x, h16 *r_out, const h16 *r_in, const h16 *q, const Geom &g, int nrhs,
                       const double *part, int np, double omega, double2 *alpha, int first, int upd_r,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_fin_mr, dim3(1, nrhs), dim3(256), 0, st, part, np, omega, alpha);
  hipLaunchKernelGGL(k_mr_update_h, dim3(sgrid(g.V), nrhs), dim3(256), 0, st, x, r_out, r_in, q, g.V, g.Vpad, alpha,
                     first, upd_r);
  return hipGetLastError();
}

hipError_t fin_mr(const double *part, int np, int nrhs, double omega, double2 *alpha, hipStream_t st) {
  hipLaunchKernelGGL(k_fin_mr, dim3(1, nrhs), dim3(256), 0, st, part, np, omega, alpha);
  return hipGetLastError();
}

template <typename TR>
hipError_t mrq_combine(float2 *x, TR *r_out, const MrqList<TR> &rs, const TR *q, const Geom &g, int steps, int nrhs,
                       const double2 *alpha, int first, int upd_r, float xs, hipStream_t st) {
  if (steps < 1 || steps > MRQ_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mrq_combine<TR>, dim3(sgrid(g.V), nrhs), dim3(256), 0, st, x, r_out, rs, q, g.V, g.Vpad,
                     steps, alpha, first, upd_r, xs);
  return hipGetLastError();
}
template hipError_t mrq_combine<float2>(float2 *, float2 *, const MrqList<float2> &, const float2 *, const Geom &,
                                        int, int, const double2 *, int, int, float, hipStream_t);
template hipError_t mrq_combine<h16>(float2 *, h16 *, const MrqList<h16> &, const h16 *, const Geom &, int, int,
                                     const double2 *, int, int, float, hipStream_t);

template <typename R>
hipError_t norm2(const c_t<R> *a, size_t n, int nrhs, double *part, double *out, hipStream_t st) {
  const int g = sgrid(n);
  hipLaunchKernelGGL(k_norm2<R>, dim3(g, nrhs), dim3(256), 0, st, a, n, part);
  hipLaunchKernelGGL(k_fin_sum<1>, dim3(1, nrhs), dim3(256), 0, st, part, g, out);
  return hipGetLastError();
}

template <typename R> int norm2_partials(const c_t<R> *a, size_t n, int nrhs, double *part, hipStream_t st) {
  const int g = sgrid(n);
  hipLaunchKernelGGL(k_norm2<R>, dim3(g, nrhs), dim3(256), 0, st, a, n, part);
  return g;
}

template <typename R>
hipError_t dot(const c_t<R> *a, const c_t<R> *b, size_t n, int nrhs, double *part, double2 *out, hipStream_t st) {
  const int g = sgrid(n);
  hipLaunchKernelGGL(k_dot<R>, dim3(g, nrhs), dim3(256), 0, st, a, b, n, part);
  hipLaunchKernelGGL(k_fin_sum<2>, dim3(1, nrhs), dim3(256), 0, st, part, g, (double *)out);
  return hipGetLastError();
}

hipError_t finish_sum1(const double *part, int np, int nrhs, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_fin_sum<1>, dim3(1, nrhs), dim3(256), 0, st, part, np, out);
  return hipGetLastError();
}

hipError_t gcr_sub2(double2 *y, const double2 *x, double2 *v, const double2 *u, size_t n, int nrhs,
                    const double2 *sc, const int *skip, hipStream_t st) {
  hipLaunchKernelGGL(k_sub2, dim3(sgrid(n), nrhs), dim3(256), 0, st, y, x, v, u, n, sc, skip);
  return hipGetLastError();
}

hipError_t gcr_scale2(double2 *y, double2 *v, size_t n, int nrhs, const double *nrm2, const int *skip,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_scale2, dim3(sgrid(n), nrhs), dim3(256), 0, st, y, v, n, nrm2, skip);
  return hipGetLastError();
}

hipError_t gcr_cgs(const double2 *W, const double2 *Z, size_t vs, int ni, double2 *wj, double2 *zj, size_t n,
                   int nrhs, double2 *sc, const int *skip, double *part, double *nrm2, hipStream_t st) {
  if (ni < 1 || ni > GCR_CHUNK) return hipErrorInvalidValue;
  const int g = sgrid(n);
  hipLaunchKernelGGL(k_gcr_mdot, dim3(g, nrhs), dim3(256), 0, st, W, vs, ni, wj, n, skip, part);
  hipLaunchKernelGGL(k_gcr_mdot_fin, dim3(1, nrhs), dim3(256), 0, st, part, g, ni, sc);
  hipLaunchKernelGGL(k_gcr_orth, dim3(g, nrhs), dim3(256), 0, st, W, Z, vs, ni, wj, zj, n, sc, skip, part);
  hipLaunchKernelGGL(k_fin_sum<1>, dim3(1, nrhs), dim3(256), 0, st, part, g, nrm2);
  return hipGetLastError();
}

hipError_t gcr_update(double2 *x, const double2 *z, double2 *r, const double2 *w, size_t n, int nrhs,
                      const double2 *sc, const int *skip, double *part, double *rr, hipStream_t st) {
  const int g = sgrid(n);
  hipLaunchKernelGGL(k_gcr_update, dim3(g, nrhs), dim3(256), 0, st, x, z, r, w, n, sc, skip, part);
  hipLaunchKernelGGL(k_fin_sum<1>, dim3(1, nrhs), dim3(256), 0, st, part, g, rr);
  return hipGetLastError();
}

#define INST(R)                                                                                                     \
  template hipError_t mr_update<R>(c_t<R> *, c_t<R> *, const c_t<R> *, const c_t<R> *, size_t, int, const double *, \
                                   int, double, double2 *, int, int, hipStream_t);                                  \
  template hipError_t norm2<R>(const c_t<R> *, size_t, int, double *, double *, hipStream_t);                       \
  template int norm2_partials<R>(const c_t<R> *, size_t, int, double *, hipStream_t);                               \
  template hipError_t dot<R>(const c_t<R> *, const c_t<R> *, size_t, int, double *, double2 *, hipStream_t);        \
  template hipError_t sub_inplace<R>(c_t<R> *, const c_t<R> *, size_t, int, hipStream_t);                           \
  template hipError_t add_inplace<R>(c_t<R> *, const c_t<R> *, size_t, int, hipStream_t);                           \
  template hipError_t scale_rsqrt<R>(c_t<R> *, size_t, int, const double *, hipStream_t);                           \
  template hipError_t resid_from<R>(c_t<R> *, const c_t<R> *, size_t, int, hipStream_t);                           \
  template int cg2_update<R>(c_t<R> *, const c_t<R> *, c_t<R> *, const c_t<R> *, size_t, int, const double *,        \
                             const double *, int, int *, double *, hipStream_t);                                    \
  template hipError_t cg2_p<R>(c_t<R> *, const c_t<R> *, size_t, int, const double *, const double *, int,          \
                               const int *, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace mg
