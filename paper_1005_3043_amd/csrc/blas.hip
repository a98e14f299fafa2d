// Streaming level-1 kernels on flat complex arrays (any layout: these are
// elementwise).  Grid-stride loops over n complex entries.
#include "kernels.h"

namespace mg {

static inline int stream_grid(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b < 16384 ? (b == 0 ? 1 : b) : 16384);
}

template <typename C> __global__ __launch_bounds__(256) void k_zero(C *x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] = mk<C>(0, 0);
}
template <typename C> __global__ __launch_bounds__(256) void k_copy(C *y, const C *x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}
template <typename Cd, typename Cs> __global__ __launch_bounds__(256) void k_convert(Cd *y, const Cs *x, size_t n) {
  using Rd = decltype(Cd::x);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    Cs v = x[i];
    y[i] = mk<Cd>((Rd)v.x, (Rd)v.y);
  }
}

template <typename R> hipError_t zero(c_t<R> *x, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero<c_t<R>>, dim3(stream_grid(n)), dim3(256), 0, st, x, n);
  return hipGetLastError();
}
template <typename R> hipError_t copy(c_t<R> *y, const c_t<R> *x, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy<c_t<R>>, dim3(stream_grid(n)), dim3(256), 0, st, y, x, n);
  return hipGetLastError();
}
template <typename Rd, typename Rs> hipError_t convert(c_t<Rd> *y, const c_t<Rs> *x, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<c_t<Rd>, c_t<Rs>>), dim3(stream_grid(n)), dim3(256), 0, st, y, x, n);
  return hipGetLastError();
}

template <typename C> __global__ __launch_bounds__(256) void k_fill(C *x, size_t n, C v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] = v;
}
template <typename R> hipError_t fill_const(c_t<R> *x, size_t n, R v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<c_t<R>>, dim3(stream_grid(n)), dim3(256), 0, st, x, n, mk<c_t<R>>(v, (R)0));
  return hipGetLastError();
}
template hipError_t fill_const<float>(float2 *, size_t, float, hipStream_t);

// X += delta * I on the diagonal block (slot 0) of every site of a coarse
// stencil L[site][slot][j][i] (n x n blocks).
__global__ __launch_bounds__(256) void k_shift_diag(double2 *L, uint32_t V, int n, double delta) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)V * n) return;
  const size_t site = i / n, j = i % n;
  double2 &x = L[(site * 9) * n * n + j * n + j];
  x.x += delta;
}
hipError_t shift_diag(double2 *L, uint32_t V, int n, double delta, hipStream_t st) {
  if (V == 0) return hipSuccess;
  hipLaunchKernelGGL(k_shift_diag, dim3(stream_grid((size_t)V * n)), dim3(256), 0, st, L, V, n, delta);
  return hipGetLastError();
}
template hipError_t fill_const<double>(double2 *, size_t, double, hipStream_t);

template <typename S> __global__ __launch_bounds__(256) void k_store_convert(S *y, const double2 *x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = cvt<S>(x[i]);
}
template <typename S> hipError_t store_convert(S *y, const double2 *x, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_store_convert<S>, dim3(stream_grid(n)), dim3(256), 0, st, y, x, n);
  return hipGetLastError();
}
// Lt[s][i][p] = L[s][p][i]: row i of a site's 9n-column block row made contiguous.
template <typename S>
__global__ __launch_bounds__(256) void k_transpose_convert(S *Lt, const double2 *L, uint32_t V, int n) {
  const size_t per = (size_t)9 * n * n, tot = per * V, K = (size_t)9 * n;
  for (size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x; o < tot; o += (size_t)gridDim.x * blockDim.x) {
    const size_t s = o / per, r = o - s * per, i = r / K, p = r - i * K;
    Lt[o] = cvt<S>(L[s * per + p * n + i]);
  }
}
template <typename S> hipError_t transpose_convert(S *Lt, const double2 *L, uint32_t V, int n, hipStream_t st) {
  const size_t tot = (size_t)9 * n * n * V;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_convert<S>, dim3(stream_grid(tot)), dim3(256), 0, st, Lt, L, V, n);
  return hipGetLastError();
}
template hipError_t transpose_convert<float2>(float2 *, const double2 *, uint32_t, int, hipStream_t);
template hipError_t transpose_convert<chalf>(chalf *, const double2 *, uint32_t, int, hipStream_t);
template hipError_t store_convert<float2>(float2 *, const double2 *, size_t, hipStream_t);
template hipError_t store_convert<chalf>(chalf *, const double2 *, size_t, hipStream_t);

// ---------------------------------------------------------------- binary16 spinor fields
// One site per thread: the site's scale needs all 12 of its components.
// Every site of the Vpad padded sites is written (padding sites are zero in
// the source, so they get scale 0 and zero entries).
template <typename Cs> __global__ __launch_bounds__(256) void k_to_h16(h16 *y, const Cs *x, uint32_t Vpad) {
  y += (size_t)blockIdx.y * 13 * Vpad;
  x += (size_t)blockIdx.y * 12 * Vpad;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < Vpad; s += gridDim.x * blockDim.x) {
    float2 v[12];
    load_site(v, x, s);
    store_site(y, s, v);
  }
}
template <typename Cd> __global__ __launch_bounds__(256) void k_from_h16(Cd *y, const h16 *x, uint32_t Vpad) {
  y += (size_t)blockIdx.y * 12 * Vpad;
  x += (size_t)blockIdx.y * 13 * Vpad;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < Vpad; s += gridDim.x * blockDim.x) {
    float2 v[12];
    load_site(v, x, s);
    Cd w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = cvt<Cd>(v[c]);
    store_site(y, s, w);
  }
}
__global__ __launch_bounds__(256) void k_copy_words(uint32_t *y, const uint32_t *x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

template <typename Cs> hipError_t to_h16(h16 *y, const Cs *x, uint32_t Vpad, int nrhs, hipStream_t st) {
  if (Vpad == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_h16<Cs>, dim3(stream_grid(Vpad), nrhs), dim3(256), 0, st, y, x, Vpad);
  return hipGetLastError();
}
template <typename Cd> hipError_t from_h16(Cd *y, const h16 *x, uint32_t Vpad, int nrhs, hipStream_t st) {
  if (Vpad == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_from_h16<Cd>, dim3(stream_grid(Vpad), nrhs), dim3(256), 0, st, y, x, Vpad);
  return hipGetLastError();
}
hipError_t copy_h16(h16 *y, const h16 *x, uint32_t Vpad, int nrhs, hipStream_t st) {
  const size_t n = (size_t)13 * Vpad * nrhs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_words, dim3(stream_grid(n)), dim3(256), 0, st, (uint32_t *)y, (const uint32_t *)x, n);
  return hipGetLastError();
}
template hipError_t to_h16<double2>(h16 *, const double2 *, uint32_t, int, hipStream_t);
template hipError_t to_h16<float2>(h16 *, const float2 *, uint32_t, int, hipStream_t);
template hipError_t from_h16<double2>(double2 *, const h16 *, uint32_t, int, hipStream_t);
template hipError_t from_h16<float2>(float2 *, const h16 *, uint32_t, int, hipStream_t);

template hipError_t zero<double>(double2 *, size_t, hipStream_t);
template hipError_t zero<float>(float2 *, size_t, hipStream_t);
template hipError_t copy<double>(double2 *, const double2 *, size_t, hipStream_t);
template hipError_t copy<float>(float2 *, const float2 *, size_t, hipStream_t);
template hipError_t convert<double, float>(double2 *, const float2 *, size_t, hipStream_t);
template hipError_t convert<float, double>(float2 *, const double2 *, size_t, hipStream_t);

}  // namespace mg
