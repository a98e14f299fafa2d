// Layout conversion between the boundary's canonical complex128 arrays
// (lexicographic sites, components innermost) and the internal site-blocked
// structure-of-arrays planes, with an optional precision change.
#include "kernels.h"

namespace mg {

template <typename T>
__global__ __launch_bounds__(256) void k_pack(Geom g, const double2 *__restrict__ canon,
                                              c_t<T> *__restrict__ internal, int ncomp) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const size_t vec = blockIdx.y;
  const Coords k = decode(g, s);
  const uint32_t i = canon_index(g, k);
  const double2 *src = canon + (vec * g.V + i) * (size_t)ncomp;
  c_t<T> *dst = internal + vec * (size_t)ncomp * g.V + s;
  for (int c = 0; c < ncomp; ++c) {
    double2 v = src[c];
    dst[(size_t)c * g.V] = mk<c_t<T>>((T)v.x, (T)v.y);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack(Geom g, const c_t<T> *__restrict__ internal,
                                                double2 *__restrict__ canon, int ncomp) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const size_t vec = blockIdx.y;
  const Coords k = decode(g, s);
  const uint32_t i = canon_index(g, k);
  double2 *dst = canon + (vec * g.V + i) * (size_t)ncomp;
  const c_t<T> *src = internal + vec * (size_t)ncomp * g.V + s;
  for (int c = 0; c < ncomp; ++c) {
    c_t<T> v = src[(size_t)c * g.V];
    dst[c] = make_double2((double)v.x, (double)v.y);
  }
}

template <typename T>
hipError_t pack_field(const Geom &g, const double2 *canon, c_t<T> *internal, int ncomp, int nvec,
                      hipStream_t st) {
  if (nvec <= 0 || g.V == 0) return hipSuccess;
  dim3 grid(div_up(g.V, 256), nvec);
  hipLaunchKernelGGL(k_pack<T>, grid, dim3(256), 0, st, g, canon, internal, ncomp);
  return hipGetLastError();
}

template <typename T>
hipError_t unpack_field(const Geom &g, const c_t<T> *internal, double2 *canon, int ncomp, int nvec,
                        hipStream_t st) {
  if (nvec <= 0 || g.V == 0) return hipSuccess;
  dim3 grid(div_up(g.V, 256), nvec);
  hipLaunchKernelGGL(k_unpack<T>, grid, dim3(256), 0, st, g, internal, canon, ncomp);
  return hipGetLastError();
}

template hipError_t pack_field<double>(const Geom &, const double2 *, double2 *, int, int, hipStream_t);
template hipError_t pack_field<float>(const Geom &, const double2 *, float2 *, int, int, hipStream_t);
template hipError_t unpack_field<double>(const Geom &, const double2 *, double2 *, int, int, hipStream_t);
template hipError_t unpack_field<float>(const Geom &, const float2 *, double2 *, int, int, hipStream_t);

}  // namespace mg
