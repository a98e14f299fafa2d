// C ABI: the stateless fine operator wilson_apply (and its variant that
// allocates nothing, wilson_apply_noalloc) and mg_last_error.
#include <cstdio>
#include <mutex>

#include "kernels.h"

namespace mg {
const char *last_error_cstr();

static void pick_tile(const int L[4], int b[4]) {
  for (int mu = 0; mu < 4; ++mu) b[mu] = (L[mu] % 4 == 0) ? 4 : ((L[mu] % 2 == 0) ? 2 : 1);
}

int check_lattice(const mg_lattice_t *lat) {
  if (!lat) { set_error("lattice is NULL"); return MG_EINVAL; }
  uint64_t V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (lat->L[mu] <= 0) { set_error("lattice extent must be positive"); return MG_EINVAL; }
    V *= (uint64_t)lat->L[mu];
  }
  if (V > (1ull << 28)) { set_error("lattice volume above 2^28 sites"); return MG_EINVAL; }
  return MG_OK;
}

template <typename T>
static int wilson_apply_t(const mg_lattice_t *lat, const void *U, double mass, const void *in, void *out,
                          int nrhs, hipStream_t st) {
  int b[4];
  pick_tile(lat->L, b);
  Geom g = make_geom(lat->L, b, lat->t_antiperiodic ? 1 : 0);
  using C = c_t<T>;
  C *Ui = nullptr, *xi = nullptr, *yi = nullptr;
  const size_t Vp = g.Vpad;
  MG_HIP(hipMallocAsync((void **)&Ui, sizeof(C) * 36 * Vp, st));
  hipError_t e = hipMallocAsync((void **)&xi, sizeof(C) * 12 * Vp * nrhs, st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&yi, sizeof(C) * 12 * Vp * nrhs, st);
  if (e == hipSuccess) e = pack_gauge<T>(g, (const double2 *)U, Ui, st);
  if (e == hipSuccess) e = pack_field<T>(g, (const double2 *)in, xi, 12, nrhs, st);
  if (e == hipSuccess) e = dslash<T>(g, Ui, 9, xi, yi, nullptr, 4.0 + mass, nrhs, DS_PLAIN, nullptr, st);
  if (e == hipSuccess) e = unpack_field<T>(g, yi, (double2 *)out, 12, nrhs, st);
  if (yi) (void)hipFreeAsync(yi, st);
  if (xi) (void)hipFreeAsync(xi, st);
  (void)hipFreeAsync(Ui, st);
  if (e != hipSuccess) {
    set_error(hip_error_string(e, "wilson_apply"));
    return MG_EHIP;
  }
  return MG_OK;
}

// FP16 class: links and spinors stored in binary16 (spinors with a per-site
// scale), FP32 arithmetic; the complex128 input is rounded to FP32 and then
// to binary16, and the output widened back.
static int wilson_apply_f16(const mg_lattice_t *lat, const void *U, double mass, const void *in, void *out,
                            int nrhs, hipStream_t st) {
  int b[4];
  pick_tile(lat->L, b);
  Geom g = make_geom(lat->L, b, lat->t_antiperiodic ? 1 : 0);
  const size_t Vp = g.Vpad;
  double2 *U64 = nullptr, *f64 = nullptr;
  chalf *Uh = nullptr;
  h16 *xh = nullptr, *yh = nullptr;
  hipError_t e = hipMallocAsync((void **)&U64, sizeof(double2) * 36 * Vp, st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&f64, sizeof(double2) * 12 * Vp * nrhs, st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&Uh, sizeof(chalf) * 36 * Vp, st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&xh, sizeof(h16) * 13 * Vp * nrhs, st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&yh, sizeof(h16) * 13 * Vp * nrhs, st);
  if (e == hipSuccess) e = pack_gauge<double>(g, (const double2 *)U, U64, st);
  if (e == hipSuccess) e = store_convert<chalf>(Uh, U64, 36 * Vp, st);
  if (e == hipSuccess) e = pack_field<double>(g, (const double2 *)in, f64, 12, nrhs, st);
  if (e == hipSuccess) e = to_h16<double2>(xh, f64, (uint32_t)Vp, nrhs, st);
  if (e == hipSuccess)
    e = dslash<float, chalf, h16, h16>(g, Uh, 9, xh, yh, nullptr, 4.0 + mass, nrhs, DS_PLAIN, nullptr, st);
  if (e == hipSuccess) e = from_h16<double2>(f64, yh, (uint32_t)Vp, nrhs, st);
  if (e == hipSuccess) e = unpack_field<double>(g, f64, (double2 *)out, 12, nrhs, st);
  if (yh) (void)hipFreeAsync(yh, st);
  if (xh) (void)hipFreeAsync(xh, st);
  if (Uh) (void)hipFreeAsync(Uh, st);
  if (f64) (void)hipFreeAsync(f64, st);
  if (U64) (void)hipFreeAsync(U64, st);
  if (e != hipSuccess) {
    set_error(hip_error_string(e, "wilson_apply"));
    return MG_EHIP;
  }
  return MG_OK;
}

// ---------------------------------------------------------------- no-alloc
// Scratch of wilson_apply_noalloc: the internal link and spinor layouts of
// one call, in a file-scope device array that each GPU the library runs on
// holds until the process ends.  Host code never uses the array's name as an
// address: it takes the per-device address from hipGetSymbolAddress once per
// device (on the first call with that device current) and passes that.
static __device__ __align__(256) unsigned char scratch[MG_NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex noalloc_mu;
static void *noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

static int noalloc_scratch(unsigned char **out) {
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    set_error("wilson_apply_noalloc: device ordinal out of range");
    return MG_EINVAL;
  }
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void *p = nullptr;
    MG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    noalloc_ptr[dev] = p;
  }
  *out = static_cast<unsigned char *>(noalloc_ptr[dev]);
  return MG_OK;
}

template <typename T>
static int wilson_apply_noalloc_t(const mg_lattice_t *lat, const void *U, double mass, const void *in, void *out,
                                  int nrhs, hipStream_t st) {
  int b[4];
  pick_tile(lat->L, b);
  Geom g = make_geom(lat->L, b, lat->t_antiperiodic ? 1 : 0);
  using C = c_t<T>;
  const size_t Vp = g.Vpad;
  const size_t need = sizeof(C) * (36 + 24 * (size_t)nrhs) * Vp;  // links, in, out
  if (need > (size_t)MG_NOALLOC_BYTES) {
    char buf[256];
    std::snprintf(buf, sizeof(buf),
                  "wilson_apply_noalloc: this lattice and nrhs need %zu bytes of scratch, above the %zu-byte limit",
                  need, (size_t)MG_NOALLOC_BYTES);
    set_error(buf);
    return MG_ENOMEM;
  }
  unsigned char *base = nullptr;
  MG_TRY(noalloc_scratch(&base));
  C *Ui = reinterpret_cast<C *>(base);
  C *xi = Ui + 36 * Vp;
  C *yi = xi + 12 * Vp * (size_t)nrhs;
  hipError_t e = pack_gauge<T>(g, (const double2 *)U, Ui, st);
  if (e == hipSuccess) e = pack_field<T>(g, (const double2 *)in, xi, 12, nrhs, st);
  if (e == hipSuccess) e = dslash<T>(g, Ui, 9, xi, yi, nullptr, 4.0 + mass, nrhs, DS_PLAIN, nullptr, st);
  if (e == hipSuccess) e = unpack_field<T>(g, yi, (double2 *)out, 12, nrhs, st);
  if (e != hipSuccess) {
    set_error(hip_error_string(e, "wilson_apply_noalloc"));
    return MG_EHIP;
  }
  return MG_OK;
}

}  // namespace mg

using namespace mg;

extern "C" int wilson_apply_noalloc(const mg_lattice_t *lat, const void *U, double mass, const void *in, void *out,
                                    int nrhs, mg_prec_t prec, hipStream_t stream) {
  set_error("");
  MG_TRY(check_lattice(lat));
  if (!U || !in || !out) { set_error("wilson_apply_noalloc: NULL buffer"); return MG_EINVAL; }
  if (in == out) { set_error("wilson_apply_noalloc: in and out alias"); return MG_EINVAL; }
  if (nrhs < 1 || nrhs > 65535) { set_error("wilson_apply_noalloc: nrhs out of range"); return MG_EINVAL; }
  if (prec == MG_F64) return wilson_apply_noalloc_t<double>(lat, U, mass, in, out, nrhs, stream);
  if (prec == MG_F32) return wilson_apply_noalloc_t<float>(lat, U, mass, in, out, nrhs, stream);
  set_error("wilson_apply_noalloc: precision must be MG_F64 or MG_F32");
  return MG_ENOTSUP;
}

extern "C" int wilson_apply(const mg_lattice_t *lat, const void *U, double mass, const void *in, void *out,
                            int nrhs, mg_prec_t prec, hipStream_t stream) {
  set_error("");
  MG_TRY(check_lattice(lat));
  if (!U || !in || !out) { set_error("wilson_apply: NULL buffer"); return MG_EINVAL; }
  if (in == out) { set_error("wilson_apply: in and out alias"); return MG_EINVAL; }
  if (nrhs < 1 || nrhs > 65535) { set_error("wilson_apply: nrhs out of range"); return MG_EINVAL; }
  if (prec == MG_F64) return wilson_apply_t<double>(lat, U, mass, in, out, nrhs, stream);
  if (prec == MG_F32) return wilson_apply_t<float>(lat, U, mass, in, out, nrhs, stream);
  if (prec == MG_F16) return wilson_apply_f16(lat, U, mass, in, out, nrhs, stream);
  set_error("wilson_apply: precision must be MG_F64, MG_F32 or MG_F16");
  return MG_ENOTSUP;
}

extern "C" const char *mg_last_error(void) { return last_error_cstr(); }
