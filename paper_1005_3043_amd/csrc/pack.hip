// Layout conversion between the boundary's canonical complex128 arrays
// (lexicographic sites, components innermost) and the internal site-blocked
// structure-of-arrays planes, with an optional precision change.
#include "solver.h"

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
  c_t<T> *dst = internal + vec * (size_t)ncomp * g.Vpad;
  for (int c = 0; c < ncomp; ++c) {
    double2 v = src[c];
    dst[fidx(s, c, ncomp)] = mk<c_t<T>>((T)v.x, (T)v.y);
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
  const c_t<T> *src = internal + vec * (size_t)ncomp * g.Vpad;
  for (int c = 0; c < ncomp; ++c) {
    c_t<T> v = src[fidx(s, c, ncomp)];
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

// Gauge field: canonical U[mu][lex site][3][3] -> internal 36-component
// fine field, component mu * 9 + (3 a + b).
template <typename T>
__global__ __launch_bounds__(256) void k_pack_gauge(Geom g, const double2 *__restrict__ canon,
                                                    c_t<T> *__restrict__ internal) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const Coords k = decode(g, s);
  const uint32_t i = canon_index(g, k);
  for (int mu = 0; mu < 4; ++mu) {
    const double2 *src = canon + ((size_t)mu * g.V + i) * 9;
    for (int e = 0; e < 9; ++e) internal[fidx(s, mu * 9 + e, 36)] = mk<c_t<T>>((T)src[e].x, (T)src[e].y);
  }
}
template <typename T> hipError_t pack_gauge(const Geom &g, const double2 *canon, c_t<T> *internal, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_gauge<T>, dim3(div_up(g.V, 256)), dim3(256), 0, st, g, canon, internal);
  return hipGetLastError();
}
template hipError_t pack_gauge<double>(const Geom &, const double2 *, double2 *, hipStream_t);
template hipError_t pack_gauge<float>(const Geom &, const double2 *, float2 *, hipStream_t);

// Site-major (coarse) vectors: canonical [vec][lex site][n] <-> internal
// [vec][site-blocked s][n].
template <typename T>
__global__ __launch_bounds__(256) void k_pack_aos(Geom g, const double2 *__restrict__ canon,
                                                  c_t<T> *__restrict__ internal, int ncomp) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)g.V * ncomp) return;
  const uint32_t s = (uint32_t)(e / ncomp);
  const int c = (int)(e - (size_t)s * ncomp);
  const Coords k = decode(g, s);
  const uint32_t i = canon_index(g, k);
  const size_t vec = (size_t)blockIdx.y * g.V * ncomp;
  const double2 v = canon[vec + (size_t)i * ncomp + c];
  internal[vec + e] = mk<c_t<T>>((T)v.x, (T)v.y);
}
template <typename T>
__global__ __launch_bounds__(256) void k_unpack_aos(Geom g, const c_t<T> *__restrict__ internal,
                                                    double2 *__restrict__ canon, int ncomp) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)g.V * ncomp) return;
  const uint32_t s = (uint32_t)(e / ncomp);
  const int c = (int)(e - (size_t)s * ncomp);
  const Coords k = decode(g, s);
  const uint32_t i = canon_index(g, k);
  const size_t vec = (size_t)blockIdx.y * g.V * ncomp;
  const c_t<T> v = internal[vec + e];
  canon[vec + (size_t)i * ncomp + c] = make_double2((double)v.x, (double)v.y);
}
template <typename T>
hipError_t pack_aos(const Geom &g, const double2 *canon, c_t<T> *internal, int ncomp, int nvec, hipStream_t st) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_aos<T>, dim3(div_up((long)g.V * ncomp, 256), nvec), dim3(256), 0, st, g, canon,
                     internal, ncomp);
  return hipGetLastError();
}
template <typename T>
hipError_t unpack_aos(const Geom &g, const c_t<T> *internal, double2 *canon, int ncomp, int nvec, hipStream_t st) {
  if (nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_aos<T>, dim3(div_up((long)g.V * ncomp, 256), nvec), dim3(256), 0, st, g, internal,
                     canon, ncomp);
  return hipGetLastError();
}
template hipError_t pack_aos<double>(const Geom &, const double2 *, double2 *, int, int, hipStream_t);
template hipError_t pack_aos<float>(const Geom &, const double2 *, float2 *, int, int, hipStream_t);
template hipError_t unpack_aos<double>(const Geom &, const double2 *, double2 *, int, int, hipStream_t);
template hipError_t unpack_aos<float>(const Geom &, const float2 *, double2 *, int, int, hipStream_t);

// Aggregate maps in canonical (lexicographic) terms, computed with the same
// site decoding and neighbour arithmetic the kernels use.
__global__ void k_maps_fine(Geom g, int32_t *f2c, int32_t *f2l, int32_t *face) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const Coords k = decode(g, s);
  const uint32_t i = canon_index(g, k);
  f2c[i] = (int32_t)k.B;
  f2l[i] = (int32_t)k.l;
  int f = 0;
  for (int mu = 0; mu < 4; ++mu) {
    if (k.o[mu] == g.b[mu] - 1) f |= 1 << (2 * mu);
    if (k.o[mu] == 0) f |= 1 << (2 * mu + 1);
  }
  face[i] = f;
}
__global__ void k_maps_coarse(Geom gc, int32_t *cnbr) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= gc.V) return;
  const Coords k = decode(gc, s);
  const uint32_t i = canon_index(gc, k);
  for (int mu = 0; mu < 4; ++mu) {
    for (int d = 0; d < 2; ++d) {
      const uint32_t t = d == 0 ? nbr_fwd(gc, s, k, mu) : nbr_bwd(gc, s, k, mu);
      cnbr[(size_t)i * 8 + 2 * mu + d] = (int32_t)canon_index(gc, decode(gc, t));
    }
  }
}
hipError_t export_maps_k(const Geom &g, const Geom &gc, int32_t *f2c, int32_t *f2l, int32_t *face, int32_t *cnbr,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_maps_fine, dim3(div_up(g.V, 256)), dim3(256), 0, st, g, f2c, f2l, face);
  hipLaunchKernelGGL(k_maps_coarse, dim3(div_up(gc.V, 256)), dim3(256), 0, st, gc, cnbr);
  return hipGetLastError();
}

template hipError_t pack_field<double>(const Geom &, const double2 *, double2 *, int, int, hipStream_t);
template hipError_t pack_field<float>(const Geom &, const double2 *, float2 *, int, int, hipStream_t);
template hipError_t unpack_field<double>(const Geom &, const double2 *, double2 *, int, int, hipStream_t);
template hipError_t unpack_field<float>(const Geom &, const float2 *, double2 *, int, int, hipStream_t);

}  // namespace mg
