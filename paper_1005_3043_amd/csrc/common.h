// Internal definitions shared by the HIP kernels and the host orchestration.
//
// Internal data layout (all levels): sites are ordered aggregate-major
// ("site-blocked"): s = B * vol_b + l, where B is the lexicographic index of
// the aggregate on the coarse lattice and l = o_x + b_x (o_y + b_y (o_z +
// b_z o_t)) the lexicographic index inside it.  Fine-level fields are stored
// in 64-site tiles (one tile per wavefront): entry (s, c) of an ncomp-component
// field sits at ((s / 64) * ncomp + c) * 64 + s % 64, so a wavefront reading
// one component of 64 consecutive sites issues one contiguous 1 KiB (FP64)
// load and all components of a tile share a few DRAM pages.  The fine stencil
// walks a 4D tile (neighbours stay in the same or the adjacent aggregate), and
// the transfer kernels see each aggregate as a contiguous run of tiles.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <string>

#include "../../include/mgwd.h"

namespace mg {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
std::string hip_error_string(hipError_t e, const char *what);

#define MG_HIP(call)                                                      \
  do {                                                                    \
    hipError_t _e = (call);                                               \
    if (_e != hipSuccess) {                                               \
      ::mg::set_error(::mg::hip_error_string(_e, #call));                 \
      return MG_EHIP;                                                     \
    }                                                                     \
  } while (0)

#define MG_TRY(call)                                                      \
  do {                                                                    \
    int _rc = (call);                                                     \
    if (_rc < 0) return _rc;                                              \
  } while (0)

// ---------------------------------------------------------------- complex
template <typename R> struct cpx;
template <> struct cpx<double> { using t = double2; };
template <> struct cpx<float> { using t = float2; };
template <typename R> using c_t = typename cpx<R>::t;

template <typename C> __host__ __device__ __forceinline__ C mk(decltype(C::x) a, decltype(C::x) b) {
  C c; c.x = a; c.y = b; return c;
}
template <typename C> __host__ __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __host__ __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __host__ __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * b accumulated: acc += a * b
template <typename C> __host__ __device__ __forceinline__ C cfma(C a, C b, C acc) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// conj(a) * b accumulated
template <typename C> __host__ __device__ __forceinline__ C cfmac(C a, C b, C acc) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
template <typename C> __host__ __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }

// Complex number stored in IEEE half precision (operator storage of the
// FP16 preconditioner; arithmetic is done after conversion to FP32).
struct __align__(4) chalf { _Float16 x, y; };
struct __align__(8) chalf2 { chalf v[2]; };
struct __align__(16) chalf4 { chalf v[4]; };
// Conversion between complex storage types (narrowing conversions round to
// nearest even in one step).
template <typename C, typename S> __host__ __device__ __forceinline__ C cvt(S v) {
  C c;
  c.x = static_cast<decltype(C::x)>(v.x);
  c.y = static_cast<decltype(C::x)>(v.y);
  return c;
}
// Fine-level spinor entry of the FP16 preconditioner.  A site's 12 complex
// components are stored in binary16 after division by the site's scale m =
// max |Re|, |Im| over them (so every stored magnitude is at most 1 and the
// relative rounding is that of binary16, 2^-11, whatever the site's size),
// and m itself sits in a 13th slot of the site as an FP32 number.  A field
// of V sites takes 13 slots of 4 bytes per site (52 bytes against 96 in
// FP32), in the tile-interleaved layout with ncomp = 13.
struct __align__(4) h16 { _Float16 x, y; };

// multiply by i^k (k = 0: 1, 1: i, 2: -1, 3: -i)
template <int k, typename C> __host__ __device__ __forceinline__ C mul_ipow(C a) {
  if constexpr (k == 0) return a;
  else if constexpr (k == 1) return mk<C>(-a.y, a.x);
  else if constexpr (k == 2) return mk<C>(-a.x, -a.y);
  else return mk<C>(a.y, -a.x);
}

// ---------------------------------------------------------------- fast div
// Division of 32-bit unsigned n by a runtime-invariant d with a multiply-high
// and shifts (Granlund & Montgomery, "Division by invariant integers using
// multiplication", 1994).
struct FastDiv {
  uint32_t d = 1, m = 0, s1 = 0, s2 = 0;
  FastDiv() = default;
  explicit FastDiv(uint32_t dd) : d(dd) {
    uint32_t l = 0;
    while ((1ull << l) < dd) ++l;
    uint64_t mm = ((1ull << 32) * ((1ull << l) - dd)) / dd + 1;
    m = (uint32_t)mm;
    s1 = l > 0 ? 1 : 0;
    s2 = l > 0 ? l - 1 : 0;
  }
  __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
#ifdef __HIP_DEVICE_COMPILE__
    uint32_t t = __umulhi(n, m);
#else
    uint32_t t = (uint32_t)(((uint64_t)n * m) >> 32);
#endif
    return (t + ((n - t) >> s1)) >> s2;
  }
};

// ---------------------------------------------------------------- geometry
// Site-blocked ordering of one lattice level.  L = lattice, b = aggregate
// (tile) shape, C = L / b = coarse lattice.
struct Geom {
  int L[4], b[4], C[4];
  uint32_t V, vb, Vc;
  uint32_t Vpad;  // V rounded up to whole 64-site tiles
  int Sl[4];   // stride of o_mu inside an aggregate
  int Sb[4];   // stride of c_mu between aggregates (in sites)
  FastDiv fvb, fb[3], fC[3];
  int antiperiodic;
};

Geom make_geom(const int L[4], const int b[4], int antiperiodic);

struct Coords { int o[4]; int c[4]; uint32_t B, l; };

// Tile-interleaved index of entry c of site s in an ncomp-component field.
constexpr int TILE = 64;
__host__ __device__ __forceinline__ size_t fidx(uint32_t s, int c, int ncomp) {
  return ((size_t)(s >> 6) * ncomp + c) * TILE + (s & (TILE - 1));
}

// Slots per site of a fine-level spinor field stored as T.
template <typename T> struct SiteSlots { static constexpr int n = 12; };
template <> struct SiteSlots<h16> { static constexpr int n = 13; };
template <typename T> constexpr int site_slots() { return SiteSlots<T>::n; }

// The 12 components of site s of one spinor field, as complex type C.
template <typename C, typename T>
__host__ __device__ __forceinline__ void load_site(C (&v)[12], const T *__restrict__ f, uint32_t s) {
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = cvt<C>(f[fidx(s, c, 12)]);
}
template <typename C>
__host__ __device__ __forceinline__ void load_site(C (&v)[12], const h16 *__restrict__ f, uint32_t s) {
  const float m = __builtin_bit_cast(float, f[fidx(s, 12, 13)]);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const h16 e = f[fidx(s, c, 13)];
    v[c] = mk<C>((float)e.x * m, (float)e.y * m);
  }
}

// The same with non-temporal loads, for input read once by the launch.
template <typename C, typename T>
__device__ __forceinline__ void load_site_nt(C (&v)[12], const T *__restrict__ f, uint32_t s) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const T *p = &f[fidx(s, c, 12)];
    T e;
    e.x = __builtin_nontemporal_load(&p->x);
    e.y = __builtin_nontemporal_load(&p->y);
    v[c] = cvt<C>(e);
  }
}
template <typename C>
__device__ __forceinline__ void load_site_nt(C (&v)[12], const h16 *__restrict__ f, uint32_t s) {
  const float m = __builtin_nontemporal_load(reinterpret_cast<const float *>(&f[fidx(s, 12, 13)]));
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const h16 e = __builtin_bit_cast(h16, __builtin_nontemporal_load(reinterpret_cast<const float *>(&f[fidx(s, c, 13)])));
    v[c] = mk<C>((float)e.x * m, (float)e.y * m);
  }
}

// Stores the 12 components of site s (NT: non-temporal stores, for output
// that the launch does not read again).  For binary16 storage the site's
// scale is computed here and v is replaced by the values as stored (decoded),
// so that sums formed from v afterwards agree with what was written.
template <bool NT = false, typename C, typename T>
__device__ __forceinline__ void store_site(T *__restrict__ f, uint32_t s, C (&v)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const T e = cvt<T>(v[c]);
    if constexpr (NT) {
      __builtin_nontemporal_store(e.x, &f[fidx(s, c, 12)].x);
      __builtin_nontemporal_store(e.y, &f[fidx(s, c, 12)].y);
    } else {
      f[fidx(s, c, 12)] = e;
    }
  }
}
template <bool NT = false, typename C>
__device__ __forceinline__ void store_site(h16 *__restrict__ f, uint32_t s, C (&v)[12]) {
  float m = 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf((float)v[c].x), fabsf((float)v[c].y)));
  const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    h16 e;
    e.x = (_Float16)((float)v[c].x * inv);
    e.y = (_Float16)((float)v[c].y * inv);
    v[c] = mk<C>((float)e.x * m, (float)e.y * m);
    if constexpr (NT) __builtin_nontemporal_store(__builtin_bit_cast(float, e), (float *)&f[fidx(s, c, 13)]);
    else f[fidx(s, c, 13)] = e;
  }
  const h16 ms = __builtin_bit_cast(h16, m);
  if constexpr (NT) __builtin_nontemporal_store(m, (float *)&f[fidx(s, 12, 13)]);
  else f[fidx(s, 12, 13)] = ms;
}

__host__ __device__ __forceinline__ Coords decode(const Geom &g, uint32_t s) {
  Coords r;
  r.B = g.fvb.div(s);
  r.l = s - r.B * g.vb;
  uint32_t q = r.l;
#pragma unroll
  for (int mu = 0; mu < 3; ++mu) {
    uint32_t q2 = g.fb[mu].div(q);
    r.o[mu] = (int)(q - q2 * (uint32_t)g.b[mu]);
    q = q2;
  }
  r.o[3] = (int)q;
  q = r.B;
#pragma unroll
  for (int mu = 0; mu < 3; ++mu) {
    uint32_t q2 = g.fC[mu].div(q);
    r.c[mu] = (int)(q - q2 * (uint32_t)g.C[mu]);
    q = q2;
  }
  r.c[3] = (int)q;
  return r;
}

// Site index of the forward (+mu) neighbour, periodic.
__host__ __device__ __forceinline__ uint32_t nbr_fwd(const Geom &g, uint32_t s, const Coords &k, int mu) {
  if (k.o[mu] + 1 < g.b[mu]) return s + g.Sl[mu];
  int64_t t = (int64_t)s - (int64_t)(g.b[mu] - 1) * g.Sl[mu];
  t += (k.c[mu] + 1 < g.C[mu]) ? (int64_t)g.Sb[mu] : -(int64_t)(g.C[mu] - 1) * g.Sb[mu];
  return (uint32_t)t;
}
// Site index of the backward (-mu) neighbour, periodic.
__host__ __device__ __forceinline__ uint32_t nbr_bwd(const Geom &g, uint32_t s, const Coords &k, int mu) {
  if (k.o[mu] > 0) return s - g.Sl[mu];
  int64_t t = (int64_t)s + (int64_t)(g.b[mu] - 1) * g.Sl[mu];
  t += (k.c[mu] > 0) ? -(int64_t)g.Sb[mu] : (int64_t)(g.C[mu] - 1) * g.Sb[mu];
  return (uint32_t)t;
}
// Lexicographic (canonical) index of an internal site.
__host__ __device__ __forceinline__ uint32_t canon_index(const Geom &g, const Coords &k) {
  uint32_t x[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) x[mu] = (uint32_t)(k.c[mu] * g.b[mu] + k.o[mu]);
  return x[0] + (uint32_t)g.L[0] * (x[1] + (uint32_t)g.L[1] * (x[2] + (uint32_t)g.L[2] * x[3]));
}

// Site-blocked index of the site with lattice coordinates x[4].
__host__ __device__ __forceinline__ uint32_t encode(const Geom &g, const int x[4]) {
  int c[4], o[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    c[mu] = x[mu] / g.b[mu];
    o[mu] = x[mu] - c[mu] * g.b[mu];
  }
  const uint32_t B = (uint32_t)(c[0] + g.C[0] * (c[1] + g.C[1] * (c[2] + g.C[2] * c[3])));
  const uint32_t l = (uint32_t)(o[0] + g.b[0] * (o[1] + g.b[1] * (o[2] + g.b[2] * o[3])));
  return B * g.vb + l;
}

// XCD-aware block remapping: the hardware hands consecutive workgroup ids
// round-robin to the 8 XCDs (each with its own L2).  Remapping so that every
// XCD walks one contiguous range of tiles keeps stencil neighbours that are
// shared between adjacent tiles inside one L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblk) {
  if ((nblk & 7u) != 0u) return bid;
  return (bid & 7u) * (nblk >> 3) + (bid >> 3);
}

// ---------------------------------------------------------------- reductions
// Wavefront (64 lanes) sum via cross-lane shuffles.
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum of NV doubles: result valid in thread 0.  blockDim.x <= 1024,
// multiple of 64.  Fixed order -> deterministic.
template <int NV> __device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[w * NV + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double a = 0.0;
      for (int j = 0; j < nw; ++j) a += lds[j * NV + i];
      v[i] = a;
    }
  }
}

inline int div_up(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace mg
