// GMRES(k) relaxation ("Formulating an algorithm": GMRES as the smoother,
// under-relaxed by omega; "Numerical Results": GMRES(4) post-relaxation).
// One cycle from x = 0: Arnoldi with classical Gram-Schmidt (all inner
// products of a column in one pass over the vectors, then one subtraction
// pass that also sums ||w||^2), Givens least squares on the Hessenberg
// matrix, and x (+)= omega sum_j y_j v_j.  The basis v_0..v_k of a level is
// stored [i][rhs][n]; per right-hand side H (row i, column j at
// H[(rhs * (GM_KMAX + 1) + i) * GM_KMAX + j]), beta = ||b|| and y stay on
// the device.
#include "solver.h"

namespace mg {

namespace {

constexpr int GW = 2 * (GM_KMAX + 1);  // partial width of the column inner products

inline int ggrid(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b < RED_BLOCKS ? (b == 0 ? 1 : b) : RED_BLOCKS);
}

__host__ __device__ inline size_t hix(int rhs, int i, int j) {
  return ((size_t)rhs * (GM_KMAX + 1) + i) * GM_KMAX + j;
}

#define GM_STRIDE(i, n) \
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

// Sum np partials of width W (stride W) of the RHS blockIdx.y; thread 0 holds the result.
template <int W> __device__ void fin_sum(const double *__restrict__ part, int np, double (&tot)[W]) {
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

// v0 = b / ||b|| (zero when b = 0); beta = ||b||
template <typename R>
__global__ __launch_bounds__(256) void k_gm_start(c_t<R> *v0, const c_t<R> *b, size_t n, const double *nrm2,
                                                  double *beta) {
  const size_t off = (size_t)blockIdx.y * n;
  v0 += off;
  b += off;
  const double nn = nrm2[blockIdx.y];
  const R s = (R)(nn > 0.0 ? 1.0 / sqrt(nn) : 0.0);
  if (blockIdx.x == 0 && threadIdx.x == 0) beta[blockIdx.y] = nn > 0.0 ? sqrt(nn) : 0.0;
  GM_STRIDE(i, n) v0[i] = cscale(b[i], s);
}

// partial <v_i, w> = sum conj(v_i) w for i < j1
template <typename R>
__global__ __launch_bounds__(256) void k_gm_mdot(const c_t<R> *__restrict__ V, size_t vs, int j1,
                                                 const c_t<R> *__restrict__ w, size_t n, double *part) {
  __shared__ double lds[4 * GW];
  const size_t off = (size_t)blockIdx.y * n;
  double t[GW];
#pragma unroll
  for (int q = 0; q < GW; ++q) t[q] = 0.0;
  GM_STRIDE(idx, n) {
    const c_t<R> wv = w[off + idx];
#pragma unroll
    for (int i = 0; i < GM_KMAX + 1; ++i) {
      if (i < j1) {
        const c_t<R> v = V[(size_t)i * vs + off + idx];
        t[2 * i] += (double)v.x * wv.x + (double)v.y * wv.y;
        t[2 * i + 1] += (double)v.x * wv.y - (double)v.y * wv.x;
      }
    }
  }
  block_sum<GW>(t, lds);
  if (threadIdx.x == 0) {
    double *p = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * GW;
#pragma unroll
    for (int q = 0; q < GW; ++q) p[q] = t[q];
  }
}

// column j of H: H[i][j] = <v_i, w>, i < j1
__global__ void k_gm_fin_mdot(const double *part, int np, int j1, int j, double2 *H) {
  double t[GW];
  fin_sum<GW>(part, np, t);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < GM_KMAX + 1; ++i)
      if (i < j1) H[hix(blockIdx.y, i, j)] = make_double2(t[2 * i], t[2 * i + 1]);
  }
}

// w -= sum_{i < j1} H[i][j] v_i; partial ||w||^2
template <typename R>
__global__ __launch_bounds__(256) void k_gm_orth(const c_t<R> *__restrict__ V, size_t vs, int j1, c_t<R> *w,
                                                 size_t n, const double2 *H, int j, double *part) {
  using C = c_t<R>;
  __shared__ double lds[4];
  const int rhs = blockIdx.y;
  const size_t off = (size_t)rhs * n;
  C h[GM_KMAX + 1];
#pragma unroll
  for (int i = 0; i < GM_KMAX + 1; ++i) {
    const double2 v = i < j1 ? H[hix(rhs, i, j)] : make_double2(0.0, 0.0);
    h[i] = mk<C>((R)-v.x, (R)-v.y);
  }
  double t[1] = {0.0};
  GM_STRIDE(idx, n) {
    C a = w[off + idx];
#pragma unroll
    for (int i = 0; i < GM_KMAX + 1; ++i)
      if (i < j1) a = cfma(h[i], V[(size_t)i * vs + off + idx], a);
    w[off + idx] = a;
    t[0] += (double)a.x * a.x + (double)a.y * a.y;
  }
  block_sum<1>(t, lds);
  if (threadIdx.x == 0) part[(size_t)rhs * gridDim.x + blockIdx.x] = t[0];
}

// H[j+1][j] = ||w||
__global__ void k_gm_fin_norm(const double *part, int np, int j, double2 *H) {
  double t[1];
  fin_sum<1>(part, np, t);
  if (threadIdx.x == 0) H[hix(blockIdx.y, j + 1, j)] = make_double2(sqrt(t[0]), 0.0);
}

// v_{j+1} = w / H[j+1][j] (zero on breakdown)
template <typename R> __global__ __launch_bounds__(256) void k_gm_scale(c_t<R> *w, size_t n, const double2 *H, int j) {
  w += (size_t)blockIdx.y * n;
  const double h = H[hix(blockIdx.y, j + 1, j)].x;
  const R s = (R)(h > 0.0 ? 1.0 / h : 0.0);
  GM_STRIDE(i, n) w[i] = cscale(w[i], s);
}

__device__ inline double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 zsc(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// min || beta e_0 - H y || by Givens rotations and back substitution; one
// thread per right-hand side, H copied to LDS.  A zero pivot (a breakdown
// column) gives a zero coefficient.
__global__ void k_gm_lsq(const double2 *H, const double *beta, int k, int nrhs, double2 *y) {
  __shared__ double2 Rm[MG_MAX_RHS][(GM_KMAX + 1) * GM_KMAX];
  __shared__ double2 g[MG_MAX_RHS][GM_KMAX + 1];
  __shared__ double cs[MG_MAX_RHS][GM_KMAX];
  __shared__ double2 sn[MG_MAX_RHS][GM_KMAX];
  __shared__ double2 yy[MG_MAX_RHS][GM_KMAX];
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  for (int i = 0; i <= k; ++i) {
    for (int j = 0; j < k; ++j) Rm[r][i * GM_KMAX + j] = H[hix(r, i, j)];
    g[r][i] = make_double2(0.0, 0.0);
  }
  g[r][0] = make_double2(beta[r], 0.0);
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < j; ++i) {
      const double2 a = Rm[r][i * GM_KMAX + j], b = Rm[r][(i + 1) * GM_KMAX + j];
      Rm[r][i * GM_KMAX + j] = zadd(zsc(a, cs[r][i]), zmul(sn[r][i], b));
      Rm[r][(i + 1) * GM_KMAX + j] = zadd(zsc(zmul(zconj(sn[r][i]), a), -1.0), zsc(b, cs[r][i]));
    }
    const double2 a = Rm[r][j * GM_KMAX + j], b = Rm[r][(j + 1) * GM_KMAX + j];
    const double na = sqrt(a.x * a.x + a.y * a.y), nb = sqrt(b.x * b.x + b.y * b.y);
    const double nu = sqrt(na * na + nb * nb);
    double c;
    double2 s;
    if (nu == 0.0) {
      c = 1.0;
      s = make_double2(0.0, 0.0);
    } else if (na == 0.0) {
      c = 0.0;
      s = make_double2(1.0, 0.0);
    } else {
      c = na / nu;
      s = zsc(zmul(zsc(a, 1.0 / na), zconj(b)), 1.0 / nu);
    }
    cs[r][j] = c;
    sn[r][j] = s;
    Rm[r][j * GM_KMAX + j] = zadd(zsc(a, c), zmul(s, b));
    Rm[r][(j + 1) * GM_KMAX + j] = make_double2(0.0, 0.0);
    const double2 gj = g[r][j], gj1 = g[r][j + 1];
    g[r][j] = zadd(zsc(gj, c), zmul(s, gj1));
    g[r][j + 1] = zadd(zsc(zmul(zconj(s), gj), -1.0), zsc(gj1, c));
  }
  for (int j = k - 1; j >= 0; --j) {
    double2 acc = g[r][j];
    for (int i = j + 1; i < k; ++i) acc = zadd(acc, zsc(zmul(Rm[r][j * GM_KMAX + i], yy[r][i]), -1.0));
    const double2 d = Rm[r][j * GM_KMAX + j];
    const double dd = d.x * d.x + d.y * d.y;
    yy[r][j] = dd > 0.0 ? zsc(zmul(acc, zconj(d)), 1.0 / dd) : make_double2(0.0, 0.0);
  }
  for (int j = 0; j < k; ++j) y[(size_t)r * GM_KMAX + j] = yy[r][j];
}

// x = (accumulate ? x : 0) + omega sum_{j < k} y_j v_j
template <typename R>
__global__ __launch_bounds__(256) void k_gm_combine(c_t<R> *x, const c_t<R> *__restrict__ V, size_t vs, int k,
                                                    size_t n, const double2 *y, double omega, int accumulate) {
  using C = c_t<R>;
  const int rhs = blockIdx.y;
  const size_t off = (size_t)rhs * n;
  C yc[GM_KMAX];
#pragma unroll
  for (int j = 0; j < GM_KMAX; ++j) {
    const double2 v = j < k ? y[(size_t)rhs * GM_KMAX + j] : make_double2(0.0, 0.0);
    yc[j] = mk<C>((R)(omega * v.x), (R)(omega * v.y));
  }
  GM_STRIDE(idx, n) {
    C a = accumulate ? x[off + idx] : mk<C>(0, 0);
#pragma unroll
    for (int j = 0; j < GM_KMAX; ++j)
      if (j < k) a = cfma(yc[j], V[(size_t)j * vs + off + idx], a);
    x[off + idx] = a;
  }
}

}  // namespace

template <typename R>
hipError_t gm_start(c_t<R> *v0, const c_t<R> *b, size_t n, int nrhs, const double *nrm2, double *beta,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_gm_start<R>, dim3(ggrid(n), nrhs), dim3(256), 0, st, v0, b, n, nrm2, beta);
  return hipGetLastError();
}

template <typename R>
hipError_t gm_arnoldi_col(c_t<R> *V, size_t vs, int j, size_t n, int nrhs, double2 *H, double *part,
                          hipStream_t st) {
  const int g = ggrid(n);
  c_t<R> *w = V + (size_t)(j + 1) * vs;
  hipLaunchKernelGGL(k_gm_mdot<R>, dim3(g, nrhs), dim3(256), 0, st, V, vs, j + 1, w, n, part);
  hipLaunchKernelGGL(k_gm_fin_mdot, dim3(1, nrhs), dim3(256), 0, st, part, g, j + 1, j, H);
  hipLaunchKernelGGL(k_gm_orth<R>, dim3(g, nrhs), dim3(256), 0, st, V, vs, j + 1, w, n, H, j, part);
  hipLaunchKernelGGL(k_gm_fin_norm, dim3(1, nrhs), dim3(256), 0, st, part, g, j, H);
  hipLaunchKernelGGL(k_gm_scale<R>, dim3(g, nrhs), dim3(256), 0, st, w, n, H, j);
  return hipGetLastError();
}

hipError_t gm_lsq(const double2 *H, const double *beta, int k, int nrhs, double2 *y, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_lsq, dim3(1), dim3(64), 0, st, H, beta, k, nrhs, y);
  return hipGetLastError();
}

template <typename R>
hipError_t gm_combine(c_t<R> *x, const c_t<R> *V, size_t vs, int k, size_t n, int nrhs, const double2 *y,
                      double omega, int accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_combine<R>, dim3(ggrid(n), nrhs), dim3(256), 0, st, x, V, vs, k, n, y, omega, accumulate);
  return hipGetLastError();
}

#define INST(R)                                                                                                    \
  template hipError_t gm_start<R>(c_t<R> *, const c_t<R> *, size_t, int, const double *, double *, hipStream_t); \
  template hipError_t gm_arnoldi_col<R>(c_t<R> *, size_t, int, size_t, int, double2 *, double *, hipStream_t);    \
  template hipError_t gm_combine<R>(c_t<R> *, const c_t<R> *, size_t, int, size_t, int, const double2 *, double,  \
                                    int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace mg
