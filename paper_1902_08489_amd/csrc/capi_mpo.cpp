// C ABI: errors and the Hamiltonian MPO entry points.
#include <cstdlib>
#include <cstring>

#include "engine.h"

namespace tdmps {
namespace {
thread_local std::string g_last_error;
}
void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }
}  // namespace tdmps

using namespace tdmps;

extern "C" const char* tdmps_last_error(void) { return tdmps::last_error_cstr(); }

extern "C" tdmps_status tdmps_mpo_from_integrals(tdmps_ctx ctx, int32_t L, const double* h, const double* eri,
                                                 double e0, tdmps_mpo* out) {
  return guard([&] {
    TDMPS_REQUIRE(out && h && eri, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    auto* m = new tdmps_mpo_s();
    try {
      m->ctx = ctx;
      // pair-channel routing window (the adjacent-operator rule of mpo.cpp): L/6 cuts on each
      // side of the centre (the lowest D^3-weighted pattern count of a sweep at L = 16..30);
      // TDMPS_MPO_ROUTING_WINDOW overrides it, -1 gives the plain rule everywhere
      int window = L / 6;
      if (const char* e = std::getenv("TDMPS_MPO_ROUTING_WINDOW")) window = std::atoi(e);
      m->host = build_mpo(L, h, eri, e0, true, window);
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

namespace tdmps {
std::vector<int> fiedler_order(int L, const double* h, const double* eri);
}

extern "C" tdmps_status tdmps_fiedler_order(int32_t L, const double* h, const double* eri, int32_t* perm) {
  return guard([&] {
    TDMPS_REQUIRE(h && perm, TDMPS_ERR_ARG, "NULL argument");
    const std::vector<int> p = tdmps::fiedler_order(L, h, eri);
    for (int i = 0; i < L; ++i) perm[i] = p[i];
  });
}

extern "C" tdmps_status tdmps_mpo_one_body(tdmps_ctx ctx, int32_t L, const double* t, tdmps_mpo* out) {
  return guard([&] {
    TDMPS_REQUIRE(out && t, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    auto* m = new tdmps_mpo_s();
    try {
      m->ctx = ctx;
      m->host = build_mpo(L, t, nullptr, 0.0, false);
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

extern "C" tdmps_status tdmps_mpo_set_one_body(tdmps_mpo mpo, const double* h) {
  return guard([&] {
    TDMPS_REQUIRE(mpo && h, TDMPS_ERR_ARG, "NULL argument");
    const uint64_t old = mpo->host.version;
    mpo_set_one_body(mpo->host, h);
    premix_cache_forget(old);  // no handle holds the old version any more
  });
}

extern "C" tdmps_status tdmps_mpo_bond_dims(tdmps_mpo mpo, int32_t* out) {
  return guard([&] {
    TDMPS_REQUIRE(mpo && out, TDMPS_ERR_ARG, "NULL argument");
    for (int i = 0; i <= mpo->host.L; ++i) out[i] = mpo->host.cut[i].size();
  });
}

extern "C" tdmps_status tdmps_mpo_to_dense(tdmps_mpo mpo, double* out, int64_t len) {
  return guard([&] {
    TDMPS_REQUIRE(mpo && out, TDMPS_ERR_ARG, "NULL argument");
    int64_t n = 1;
    for (int i = 0; i < mpo->host.L; ++i) n *= 4;
    TDMPS_REQUIRE(len == n * n, TDMPS_ERR_ARG, "len must be 16^L");
    mpo_to_dense(mpo->host, out);
  });
}

extern "C" tdmps_status tdmps_mpo_det_element(tdmps_mpo mpo, const uint8_t* bra, const uint8_t* ket, double* out) {
  return guard([&] {
    TDMPS_REQUIRE(mpo && bra && ket && out, TDMPS_ERR_ARG, "NULL argument");
    *out = mpo_det_element(mpo->host, bra, ket);
  });
}

extern "C" tdmps_status tdmps_mpo_destroy(tdmps_mpo mpo) {
  return guard([&] { delete mpo; });
}
