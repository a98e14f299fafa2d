// C ABI: the stateless fine operator wilson_apply and mg_last_error.
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

}  // namespace mg

using namespace mg;

extern "C" int wilson_apply(const mg_lattice_t *lat, const void *U, double mass, const void *in, void *out,
                            int nrhs, mg_prec_t prec, hipStream_t stream) {
  set_error("");
  MG_TRY(check_lattice(lat));
  if (!U || !in || !out) { set_error("wilson_apply: NULL buffer"); return MG_EINVAL; }
  if (in == out) { set_error("wilson_apply: in and out alias"); return MG_EINVAL; }
  if (nrhs < 1 || nrhs > 65535) { set_error("wilson_apply: nrhs out of range"); return MG_EINVAL; }
  if (prec == MG_F64) return wilson_apply_t<double>(lat, U, mass, in, out, nrhs, stream);
  if (prec == MG_F32) return wilson_apply_t<float>(lat, U, mass, in, out, nrhs, stream);
  set_error("wilson_apply: precision must be MG_F64 or MG_F32");
  return MG_ENOTSUP;
}

extern "C" const char *mg_last_error(void) { return last_error_cstr(); }
