// C ABI: contexts, states, operations, time steps and the kernel-level H_eff handle.
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "drivers.h"
#include "io.h"
#include "pulse.h"
#include "engine.h"

using namespace tdmps;

struct tdmps_heff_s {
  Ctx* ctx = nullptr;
  int precision = TDMPS_FP64;
  std::unique_ptr<Env> L, R;
  std::unique_ptr<SideOps> lops, rops;
  TwoLayout kl, bl;
  Bond ket_l, ket_r, bra_l, bra_r;
  std::unique_ptr<HeffPlan> plan;
  const void* last_in = nullptr;
  void* last_out = nullptr;
  double alg_flops = 0;
  const MpoHost* H = nullptr;
  int plan_gen = -1;     // tile-rule generation the plan was made under
  void* graph = nullptr;  // captured launch sequence of the plan (launch mode 2)
  ~tdmps_heff_s() { tdmps::graph_destroy(graph); }
};

namespace {

// Parameters of the library's own contractions (no caller parameters): FP64 unless stated,
// grouped launches.  A zero-initialised tdmps_fit_params would select the per-block baseline.
tdmps_fit_params internal_params(int32_t precision = TDMPS_FP64) {
  tdmps_fit_params p{};
  p.precision = precision;
  p.batched = 1;
  return p;
}

Contractor make_contractor(Ctx* ctx, const tdmps_fit_params* prm) {
  dev_bind(ctx->device, ctx->stream);
  Contractor C;
  C.ctx = ctx;
  if (prm) {
    C.precision = prm->precision;
    C.batched = prm->batched;
  }
  return C;
}

void publish(Ctx* ctx, const Contractor& C) {
  ctx->counters[0] = C.heff_alg_flops;
  ctx->counters[1] = C.heff_flops;
  ctx->counters[2] = C.t_heff;
  ctx->counters[3] = C.t_env;
  ctx->counters[4] = C.t_svd;
  ctx->counters[5] = C.t_mix;
  ctx->counters[6] = C.t_sandwich;
  ctx->counters[7] = C.env_flops;
  ctx->counters[8] = C.mix_flops;
  ctx->counters[9] = C.svd_sweeps;
  ctx->counters[10] = C.svd_rounds;
  ctx->counters[11] = C.n_svd;
  ctx->counters[12] = C.n_heff;
  ctx->counters[13] = C.n_env;
  ctx->counters[14] = C.n_sandwich;
  ctx->counters[15] = C.t_qr;
  ctx->counters[16] = C.t_plan;
  dev_alloc_stats(&ctx->counters[17], &ctx->counters[18]);
  ctx->counters[19] = tdmps::premix_structures_built();
  ctx->counters[20] = C.fit_discarded;
}

void check_prm(const tdmps_fit_params* p) {
  TDMPS_REQUIRE(p, TDMPS_ERR_ARG, "NULL fit parameters");
  TDMPS_REQUIRE(p->Dmax >= 1 && p->n_sweeps >= 1, TDMPS_ERR_ARG, "Dmax and n_sweeps must be >= 1");
  TDMPS_REQUIRE(p->svd_cutoff >= 0 && std::isfinite(p->svd_cutoff), TDMPS_ERR_ARG, "bad svd_cutoff");
  TDMPS_REQUIRE(p->precision >= TDMPS_FP64 && p->precision <= TDMPS_BF16X6,
                TDMPS_ERR_ARG, "unknown precision");
}

void fill_info(tdmps_fit_info* info, const FitOut& f, const Mps* m) {
  if (!info) return;
  info->sweeps_used = f.sweeps;
  info->discarded_max = f.disc_max;
  info->discarded_sum = f.disc_sum;
  info->norm2 = f.norm2;
  int mb = 0;
  for (auto& b : m->bond) mb = std::max(mb, b.total());
  info->max_bond = mb;
}

cplx read_cplx(const double* p) { return cplx{p[0], p[1]}; }

}  // namespace

extern "C" tdmps_status tdmps_ctx_create(int32_t device, void* hip_stream, tdmps_ctx* out) {
  return guard([&] {
    TDMPS_REQUIRE(out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    auto* c = new tdmps_ctx_s();
    c->device = device;
    dev_set_device(device);
    if (hip_stream) {
      c->stream = hip_stream;
    } else {
      c->stream = dev_stream_create();
      c->own_stream = true;
    }
    c->phase_sync = std::getenv("TDMPS_PHASE_TIMING") != nullptr;
    if (const char* ms = std::getenv("TDMPS_MIXED_STORAGE")) c->mixed_storage = std::atoi(ms) != 0;
    dev_bind(device, c->stream);
    noalloc_init(device);
    *out = c;
  });
}

extern "C" tdmps_status tdmps_ctx_destroy(tdmps_ctx ctx) {
  return guard([&] {
    if (!ctx) return;
    dev_sync(ctx->stream);
    if (ctx->own_stream) dev_stream_destroy(ctx->stream);
    delete ctx;
  });
}

extern "C" tdmps_status tdmps_ctx_counters(tdmps_ctx ctx, double* out) {
  return guard([&] {
    TDMPS_REQUIRE(ctx && out, TDMPS_ERR_ARG, "NULL argument");
    for (int i = 0; i < TDMPS_NCOUNTERS; ++i) out[i] = ctx->counters[i];
  });
}

extern "C" tdmps_status tdmps_ctx_set_launch_mode(tdmps_ctx ctx, int32_t batched) {
  return guard([&] {
    TDMPS_REQUIRE(ctx, TDMPS_ERR_ARG, "NULL argument");
    TDMPS_REQUIRE(batched >= 0 && batched <= 2, TDMPS_ERR_ARG, "launch mode must be 0, 1 or 2");
    ctx->batched = batched;
  });
}

static_assert(TDMPS_TILE_CONFIGS == GEMM_NCFG, "tile configuration count");
static_assert(TDMPS_TILE_BUCKETS == TILE_NB * TILE_NB * TILE_NK, "tile bucket count");

extern "C" tdmps_status tdmps_ctx_set_tile_config(tdmps_ctx ctx, int32_t cfg) {
  return guard([&] {
    TDMPS_REQUIRE(ctx, TDMPS_ERR_ARG, "NULL argument");
    TDMPS_REQUIRE(cfg >= -1 && cfg < GEMM_NCFG, TDMPS_ERR_ARG, "tile configuration out of range");
    ctx->tile_cfg = cfg;
    ctx->tune_gen++;
  });
}

extern "C" tdmps_status tdmps_ctx_autotune(tdmps_ctx ctx, int32_t precision, int32_t* cfg_out, double* tflops_out) {
  return guard([&] {
    TDMPS_REQUIRE(ctx, TDMPS_ERR_ARG, "NULL argument");
    TDMPS_REQUIRE(precision >= TDMPS_FP64 && precision <= TDMPS_BF16X6, TDMPS_ERR_ARG,
                  "unknown precision");
    dev_bind(ctx->device, ctx->stream);
    TileTable t;
    autotune_tiles(ctx, precision, t);
    ctx->tune[precision] = t;
    ctx->tune_gen++;
    int q = 0;
    for (int a = 0; a < TILE_NB; ++a)
      for (int b = 0; b < TILE_NB; ++b)
        for (int c = 0; c < TILE_NK; ++c, ++q) {
          if (cfg_out) cfg_out[q] = t.cfg[a][b][c];
          if (tflops_out) tflops_out[q] = t.tflops[a][b][c];
        }
  });
}

extern "C" tdmps_status tdmps_ctx_clear_tuning(tdmps_ctx ctx) {
  return guard([&] {
    TDMPS_REQUIRE(ctx, TDMPS_ERR_ARG, "NULL argument");
    for (auto& t : ctx->tune) t.valid = false;
    ctx->tune_gen++;
  });
}

extern "C" tdmps_status tdmps_ctx_reset_counters(tdmps_ctx ctx) {
  return guard([&] {
    TDMPS_REQUIRE(ctx, TDMPS_ERR_ARG, "NULL argument");
    for (double& x : ctx->counters) x = 0;
  });
}

// ---------------------------------------------------------------- states
extern "C" tdmps_status tdmps_mps_from_determinant(tdmps_ctx ctx, int32_t L, const uint8_t* occ, tdmps_mps* out) {
  return guard([&] {
    TDMPS_REQUIRE(ctx && occ && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    TDMPS_REQUIRE(L >= 2 && L <= 64, TDMPS_ERR_ARG, "L must be in [2, 64]");
    std::vector<Bond> bonds(L + 1);
    Charge q(0, 0);
    bonds[0].q = {q};
    bonds[0].dim = {1};
    for (int i = 0; i < L; ++i) {
      TDMPS_REQUIRE(occ[i] < 4, TDMPS_ERR_ARG, "occupation codes must be 0..3");
      q = q + local_charge(occ[i]);
      bonds[i + 1].q = {q};
      bonds[i + 1].dim = {1};
    }
    Mps* m = mps_new(ctx, L, bonds);
    std::unique_ptr<Mps> g(m);
    mps_from_det(m, occ);
    *out = g.release();
  });
}

extern "C" tdmps_status tdmps_mps_from_blocks(tdmps_ctx ctx, int32_t L, const int32_t* bond_nsec,
                                              const int32_t* bond_sec, const double* data, int64_t len,
                                              tdmps_mps* out) {
  return guard([&] {
    TDMPS_REQUIRE(ctx && bond_nsec && bond_sec && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    TDMPS_REQUIRE(L >= 2 && L <= 64, TDMPS_ERR_ARG, "L must be in [2, 64]");
    std::vector<Bond> bonds(L + 1);
    int64_t k = 0;
    for (int i = 0; i <= L; ++i) {
      TDMPS_REQUIRE(bond_nsec[i] >= 1, TDMPS_ERR_ARG, "every bond needs a sector");
      for (int s = 0; s < bond_nsec[i]; ++s, ++k) {
        Charge q(bond_sec[3 * k], bond_sec[3 * k + 1]);
        int d = bond_sec[3 * k + 2];
        TDMPS_REQUIRE(d >= 1, TDMPS_ERR_ARG, "sector dimensions must be >= 1");
        TDMPS_REQUIRE(bonds[i].q.empty() || bonds[i].q.back() < q, TDMPS_ERR_ARG,
                      "sectors of a bond must be listed in ascending (n_up, n_dn) order");
        bonds[i].q.push_back(q);
        bonds[i].dim.push_back(d);
      }
    }
    std::unique_ptr<Mps> m(mps_new(ctx, L, bonds));
    int64_t need = 0;
    for (int i = 0; i < L; ++i) need += 2 * m->lay[i].size;
    TDMPS_REQUIRE(len == need, TDMPS_ERR_ARG, "data length does not match the block layout");
    TDMPS_REQUIRE(data || need == 0, TDMPS_ERR_ARG, "NULL data");
    for (int64_t x = 0; x < need; ++x) TDMPS_REQUIRE(std::isfinite(data[x]), TDMPS_ERR_NUMERIC, "non-finite data");
    int64_t off = 0;
    for (int i = 0; i < L; ++i) {
      if (m->lay[i].size) dev_h2d(m->site[i].p, data + off, m->lay[i].size * sizeof(cplx), ctx->stream);
      off += 2 * m->lay[i].size;
    }
    dev_sync(ctx->stream);
    *out = m.release();
  });
}

extern "C" tdmps_status tdmps_mps_sectors(tdmps_mps m, int32_t* bond_nsec, int32_t* bond_sec, int64_t* total) {
  return guard([&] {
    TDMPS_REQUIRE(m, TDMPS_ERR_ARG, "NULL argument");
    int64_t k = 0;
    for (int i = 0; i <= m->L; ++i) {
      if (bond_nsec) bond_nsec[i] = m->bond[i].nsec();
      for (int s = 0; s < m->bond[i].nsec(); ++s, ++k)
        if (bond_sec) {
          bond_sec[3 * k] = m->bond[i].q[s].nu;
          bond_sec[3 * k + 1] = m->bond[i].q[s].nd;
          bond_sec[3 * k + 2] = m->bond[i].dim[s];
        }
    }
    if (total) *total = k;
  });
}

extern "C" tdmps_status tdmps_mps_get_blocks(tdmps_mps m, double* data, int64_t* len) {
  return guard([&] {
    TDMPS_REQUIRE(m && len, TDMPS_ERR_ARG, "NULL argument");
    int64_t need = 0;
    for (int i = 0; i < m->L; ++i) need += 2 * m->lay[i].size;
    if (!data) {
      *len = need;
      return;
    }
    TDMPS_REQUIRE(*len >= need, TDMPS_ERR_ARG, "buffer too small");
    int64_t off = 0;
    for (int i = 0; i < m->L; ++i) {
      if (m->lay[i].size) dev_d2h(data + off, m->site[i].p, m->lay[i].size * sizeof(cplx), m->ctx->stream);
      off += 2 * m->lay[i].size;
    }
    *len = need;
  });
}

extern "C" tdmps_status tdmps_mps_to_dense(tdmps_mps m, double* out, int64_t len) {
  return guard([&] {
    TDMPS_REQUIRE(m && out, TDMPS_ERR_ARG, "NULL argument");
    TDMPS_REQUIRE(m->L <= 12, TDMPS_ERR_ARG, "to_dense supports L <= 12");
    int64_t full = 1;
    for (int i = 0; i < m->L; ++i) full *= 4;
    TDMPS_REQUIRE(len == 2 * full, TDMPS_ERR_ARG, "len must be 2*4^L");
    using zd = std::complex<double>;
    // V (configs of sites < i) x (bond i index); bond index = sector offset + inner index
    std::vector<zd> V(1, zd(1.0));
    int64_t nconf = 1;
    for (int i = 0; i < m->L; ++i) {
      const Bond& l = m->bond[i];
      const Bond& r = m->bond[i + 1];
      const SiteLayout& lay = m->lay[i];
      std::vector<zd> A(lay.size);
      if (lay.size) dev_d2h(A.data(), m->site[i].p, lay.size * sizeof(cplx), m->ctx->stream);
      std::vector<int> loff(l.nsec()), roff(r.nsec());
      int Dl = 0, Dr = 0;
      for (int s = 0; s < l.nsec(); ++s) loff[s] = Dl, Dl += l.dim[s];
      for (int s = 0; s < r.nsec(); ++s) roff[s] = Dr, Dr += r.dim[s];
      std::vector<zd> W(nconf * 4 * Dr, zd(0));
      for (int64_t x = 0; x < nconf; ++x)
        for (int s = 0; s < l.nsec(); ++s)
          for (int n = 0; n < 4; ++n) {
            int t = lay.rs[s][n];
            if (t < 0) continue;
            for (int a = 0; a < l.dim[s]; ++a) {
              zd va = V[x * Dl + loff[s] + a];
              if (va == zd(0)) continue;
              const zd* row = A.data() + lay.panel_off[s] + (int64_t)a * lay.width[s] + lay.col[s][n];
              zd* dst = W.data() + (x * 4 + n) * Dr + roff[t];
              for (int b = 0; b < r.dim[t]; ++b) dst[b] += va * row[b];
            }
          }
      V.swap(W);
      nconf *= 4;
    }
    for (int64_t x = 0; x < full; ++x) {
      out[2 * x] = V[x].real();
      out[2 * x + 1] = V[x].imag();
    }
  });
}

extern "C" tdmps_status tdmps_mps_copy(tdmps_mps m, tdmps_mps* out) {
  return guard([&] {
    TDMPS_REQUIRE(m && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    *out = mps_clone(m);
  });
}

extern "C" tdmps_status tdmps_mps_bond_dims(tdmps_mps m, int32_t* out) {
  return guard([&] {
    TDMPS_REQUIRE(m && out, TDMPS_ERR_ARG, "NULL argument");
    for (int i = 0; i <= m->L; ++i) out[i] = m->bond[i].total();
  });
}

extern "C" tdmps_status tdmps_mps_from_dense(tdmps_ctx ctx, int32_t L, int32_t N, int32_t twoSz, const double* coeffs,
                                             int64_t len, int32_t Dmax, double svd_cutoff, tdmps_mps* out) {
  return guard([&] {
    TDMPS_REQUIRE(ctx && coeffs && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    TDMPS_REQUIRE(L >= 2 && L <= 12, TDMPS_ERR_ARG, "from_dense supports 2 <= L <= 12");
    int64_t full = 1;
    for (int i = 0; i < L; ++i) full *= 4;
    TDMPS_REQUIRE(len == 2 * full, TDMPS_ERR_ARG, "len must be 2*4^L");
    TDMPS_REQUIRE(((N + twoSz) & 1) == 0 && N >= 0 && std::abs(twoSz) <= N, TDMPS_ERR_SECTOR,
                  "N and 2Sz must have equal parity with |2Sz| <= N");
    TDMPS_REQUIRE(svd_cutoff >= 0 && std::isfinite(svd_cutoff), TDMPS_ERR_ARG, "bad svd_cutoff");
    tdmps_fit_params prm = internal_params();
    Contractor C = make_contractor(ctx, &prm);
    *out = mps_from_dense(C, L, Charge((N + twoSz) / 2, (N - twoSz) / 2), coeffs, Dmax, svd_cutoff);
  });
}

extern "C" tdmps_status tdmps_mps_save(tdmps_mps m, const char* path) {
  return guard([&] {
    TDMPS_REQUIRE(m && path, TDMPS_ERR_ARG, "NULL argument");
    dev_bind(m->ctx->device, m->ctx->stream);
    mps_save(m, path);
  });
}

extern "C" tdmps_status tdmps_mps_load(tdmps_ctx ctx, const char* path, tdmps_mps* out) {
  return guard([&] {
    TDMPS_REQUIRE(ctx && path && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    dev_bind(ctx->device, ctx->stream);
    *out = mps_load(ctx, path);
  });
}

extern "C" tdmps_status tdmps_mps_destroy(tdmps_mps m) {
  return guard([&] { delete m; });
}

// ---------------------------------------------------------------- operations
extern "C" tdmps_status tdmps_mps_scale(tdmps_mps m, const double* alpha) {
  return guard([&] {
    TDMPS_REQUIRE(m && alpha, TDMPS_ERR_ARG, "NULL argument");
    TDMPS_REQUIRE(std::isfinite(alpha[0]) && std::isfinite(alpha[1]), TDMPS_ERR_NUMERIC, "non-finite scale");
    scale_mps(m->ctx, m, read_cplx(alpha));
  });
}

extern "C" tdmps_status tdmps_mps_overlap(tdmps_mps a, tdmps_mps b, double* out) {
  return guard([&] {
    TDMPS_REQUIRE(a && b && out, TDMPS_ERR_ARG, "NULL argument");
    Contractor C = make_contractor(a->ctx, nullptr);
    cplx r = overlap(C, a, b);
    out[0] = r.x;
    out[1] = r.y;
  });
}

extern "C" tdmps_status tdmps_mps_expect(tdmps_mpo op, tdmps_mps bra, tdmps_mps ket, double* out) {
  return guard([&] {
    TDMPS_REQUIRE(op && bra && ket && out, TDMPS_ERR_ARG, "NULL argument");
    Contractor C = make_contractor(bra->ctx, nullptr);
    cplx r = sandwich(C, op->host, bra, ket);
    publish(bra->ctx, C);
    out[0] = r.x;
    out[1] = r.y;
  });
}

extern "C" tdmps_status tdmps_mps_apply_H(tdmps_mpo H, const double* alpha, tdmps_mps psi, int32_t nterms,
                                          const double* beta, const tdmps_mps* phi, const tdmps_fit_params* prm,
                                          tdmps_mps* out, tdmps_fit_info* info) {
  return guard([&] {
    TDMPS_REQUIRE(H && alpha && psi && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    check_prm(prm);
    TDMPS_REQUIRE(nterms >= 0 && (nterms == 0 || (beta && phi)), TDMPS_ERR_ARG, "bad terms");
    std::vector<FitTerm> terms;
    for (int j = 0; j < nterms; ++j) {
      TDMPS_REQUIRE(phi[j], TDMPS_ERR_ARG, "NULL term state");
      terms.push_back({read_cplx(beta + 2 * j), phi[j]});
    }
    Contractor C = make_contractor(psi->ctx, prm);
    FitOut f;
    Mps* m = fit(C, &H->host, read_cplx(alpha), psi, terms, *prm, &f);
    publish(psi->ctx, C);
    fill_info(info, f, m);
    *out = m;
  });
}

extern "C" tdmps_status tdmps_mps_compress(int32_t nterms, const double* beta, const tdmps_mps* phi,
                                           const tdmps_fit_params* prm, tdmps_mps* out, tdmps_fit_info* info) {
  return guard([&] {
    TDMPS_REQUIRE(beta && phi && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    check_prm(prm);
    TDMPS_REQUIRE(nterms >= 1, TDMPS_ERR_ARG, "need at least one term");
    std::vector<FitTerm> terms;
    for (int j = 0; j < nterms; ++j) {
      TDMPS_REQUIRE(phi[j], TDMPS_ERR_ARG, "NULL term state");
      terms.push_back({read_cplx(beta + 2 * j), phi[j]});
    }
    Contractor C = make_contractor(phi[0]->ctx, prm);
    FitOut f;
    Mps* m = fit(C, nullptr, cplx{0, 0}, nullptr, terms, *prm, &f);
    publish(phi[0]->ctx, C);
    fill_info(info, f, m);
    *out = m;
  });
}

extern "C" tdmps_status tdmps_mps_annihilate(tdmps_mps psi, int32_t site, int32_t spin, tdmps_mps* out) {
  return guard([&] {
    TDMPS_REQUIRE(psi && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    dev_bind(psi->ctx->device, psi->ctx->stream);
    *out = mps_annihilate(psi->ctx, psi, site, spin);
  });
}

extern "C" tdmps_status tdmps_krylov_ground(tdmps_mpo H, tdmps_mps psi, int32_t m, int32_t restarts,
                                            const tdmps_fit_params* prm, tdmps_mps* out, double* energy) {
  return guard([&] {
    TDMPS_REQUIRE(H && psi && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    check_prm(prm);
    Contractor C = make_contractor(psi->ctx, prm);
    double E = 0;
    Mps* r = krylov_ground(C, &H->host, psi, m, restarts, *prm, &E);
    publish(psi->ctx, C);
    if (energy) *energy = E;
    *out = r;
  });
}

extern "C" tdmps_status tdmps_mps_one_rdm(tdmps_mps psi, double* gamma) {
  return guard([&] {
    TDMPS_REQUIRE(psi && gamma, TDMPS_ERR_ARG, "NULL argument");
    tdmps_fit_params prm = internal_params();
    Contractor C = make_contractor(psi->ctx, &prm);
    const std::vector<std::complex<double>> g = one_rdm(C, psi);
    publish(psi->ctx, C);
    for (size_t i = 0; i < g.size(); ++i) {
      gamma[2 * i] = g[i].real();
      gamma[2 * i + 1] = g[i].imag();
    }
  });
}

extern "C" tdmps_status tdmps_krylov_step(tdmps_mpo H, tdmps_mps psi, double dt, int32_t m, int32_t flags,
                                          const tdmps_fit_params* prm, tdmps_mps* out, double* Nmat, double* Hmat) {
  return guard([&] {
    TDMPS_REQUIRE(H && psi && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    check_prm(prm);
    TDMPS_REQUIRE(std::isfinite(dt), TDMPS_ERR_NUMERIC, "non-finite dt");
    TDMPS_REQUIRE(flags == TDMPS_KRYLOV_ORTHO || flags == TDMPS_KRYLOV_NONORTHO, TDMPS_ERR_ARG, "bad flags");
    Contractor C = make_contractor(psi->ctx, prm);
    std::vector<std::complex<double>> N, Hm;
    Mps* r = krylov_step(C, &H->host, psi, dt, m, flags == TDMPS_KRYLOV_ORTHO, *prm, &N, &Hm);
    publish(psi->ctx, C);
    for (int i = 0; i < m * m; ++i) {
      if (Nmat) Nmat[2 * i] = N[i].real(), Nmat[2 * i + 1] = N[i].imag();
      if (Hmat) Hmat[2 * i] = Hm[i].real(), Hmat[2 * i + 1] = Hm[i].imag();
    }
    *out = r;
  });
}

extern "C" tdmps_status tdmps_rk4_step(tdmps_mpo H_t, tdmps_mpo H_mid, tdmps_mpo H_t1, tdmps_mps psi, double dt,
                                       const tdmps_fit_params* prm, tdmps_mps* out, tdmps_fit_info* info) {
  return guard([&] {
    TDMPS_REQUIRE(H_t && H_mid && H_t1 && psi && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    check_prm(prm);
    TDMPS_REQUIRE(std::isfinite(dt), TDMPS_ERR_NUMERIC, "non-finite dt");
    Contractor C = make_contractor(psi->ctx, prm);
    FitOut f;
    Mps* r = rk4_step(C, &H_t->host, &H_mid->host, &H_t1->host, psi, dt, *prm, &f);
    publish(psi->ctx, C);
    fill_info(info, f, r);
    *out = r;
  });
}

// ---------------------------------------------------------------- H_eff handle
extern "C" tdmps_status tdmps_heff_create(tdmps_mpo H, tdmps_mps bra, tdmps_mps ket, int32_t site, int32_t precision,
                                          tdmps_heff* out) {
  return guard([&] {
    TDMPS_REQUIRE(H && bra && ket && out, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    const int L = bra->L;
    TDMPS_REQUIRE(ket->L == L && H->host.L == L, TDMPS_ERR_ARG, "length mismatch");
    TDMPS_REQUIRE(site >= 0 && site + 1 < L, TDMPS_ERR_ARG, "site out of range");
    TDMPS_REQUIRE(bra->total == ket->total, TDMPS_ERR_SECTOR, "bra and ket differ in total charge");
    std::unique_ptr<tdmps_heff_s> h(new tdmps_heff_s());
    h->ctx = bra->ctx;
    h->precision = precision;
    h->H = &H->host;
    tdmps_fit_params prm = internal_params(precision);
    Contractor C = make_contractor(bra->ctx, &prm);
    const MpoHost& W = H->host;
    auto E = std::make_unique<Env>(env_left_boundary(C.ctx, bra->bond[0], ket->bond[0]));
    for (int i = 0; i < site; ++i) {
      SideOps ops = premix_left(C, *E, W, i);
      auto N = std::make_unique<Env>(env_left_update(C, ops, bra, bra->site[i].c(), bra->lay[i], bra->bond[i],
                                                     bra->bond[i + 1], ket->site[i].c(), ket->lay[i], ket->bond[i],
                                                     ket->bond[i + 1], W));
      E = std::move(N);
    }
    auto R = std::make_unique<Env>(env_right_boundary(C.ctx, bra->bond[L], ket->bond[L], L));
    for (int i = L - 1; i >= site + 2; --i) {
      SideOps ops = premix_right(C, *R, W, i);
      auto N = std::make_unique<Env>(env_right_update(C, ops, bra->site[i].c(), bra->lay[i], bra->bond[i],
                                                      bra->bond[i + 1], ket->site[i].c(), ket->lay[i], ket->bond[i],
                                                      ket->bond[i + 1], W));
      R = std::move(N);
    }
    h->L = std::move(E);
    h->R = std::move(R);
    h->lops = std::make_unique<SideOps>(premix_left(C, *h->L, W, site));
    h->rops = std::make_unique<SideOps>(premix_right(C, *h->R, W, site + 1));
    h->ket_l = ket->bond[site];
    h->ket_r = ket->bond[site + 2];
    h->bra_l = bra->bond[site];
    h->bra_r = bra->bond[site + 2];
    h->kl.build(h->ket_l, h->ket_r);
    h->bl.build(h->bra_l, h->bra_r);
    *out = h.release();
  });
}

extern "C" tdmps_status tdmps_heff_layout(tdmps_heff h, int32_t which, int64_t* total, int64_t* nblocks,
                                          int32_t* blocks) {
  return guard([&] {
    TDMPS_REQUIRE(h && total && nblocks, TDMPS_ERR_ARG, "NULL argument");
    const TwoLayout& t = which ? h->bl : h->kl;
    const Bond& l = which ? h->bra_l : h->ket_l;
    const Bond& r = which ? h->bra_r : h->ket_r;
    int64_t nb = 0;
    for (int s = 0; s < l.nsec(); ++s)
      for (int n = 0; n < 16; ++n) {
        int b = t.rs[s][n];
        if (b < 0) continue;
        if (blocks) {
          int32_t* o = blocks + 9 * nb;
          int64_t off = 2 * (t.panel_off[s] + t.col[s][n]);
          o[0] = l.q[s].nu;
          o[1] = l.q[s].nd;
          o[2] = n >> 2;
          o[3] = n & 3;
          o[4] = l.dim[s];
          o[5] = r.dim[b];
          o[6] = (int32_t)(off & 0x7fffffff);
          o[7] = (int32_t)(off >> 31);
          o[8] = t.width[s];
        }
        ++nb;
      }
    *nblocks = nb;
    *total = 2 * t.size;
  });
}

extern "C" tdmps_status tdmps_heff_apply(tdmps_heff h, const void* in, void* out) {
  return guard([&] {
    TDMPS_REQUIRE(h && in && out, TDMPS_ERR_ARG, "NULL argument");
    TDMPS_REQUIRE(in != out, TDMPS_ERR_ARG, "in-place apply is not supported");
    dev_bind(h->ctx->device, h->ctx->stream);
    Ctx* c = h->ctx;
    if (!h->plan || h->last_in != in || h->last_out != out || h->plan_gen != c->tune_gen) {
      graph_destroy(h->graph);
      h->graph = nullptr;
      h->plan.reset();
      tdmps_fit_params prm = internal_params(h->precision);
      Contractor C = make_contractor(c, &prm);
      h->plan = heff_plan(C, *h->lops, *h->rops, (const cplx*)in, h->kl, h->ket_l, h->ket_r, (cplx*)out, h->bl,
                          h->bra_l, h->bra_r, cplx{1, 0}, false);
      h->last_in = in;
      h->last_out = out;
      h->plan_gen = c->tune_gen;
      h->alg_flops = h->plan->alg_flops;
      c->counters[0] = h->alg_flops;
      c->counters[1] = h->plan->p1.flops + h->plan->p1b.flops;
      c->counters[2] = h->plan->p2.flops;
      c->counters[3] = (double)h->plan->T.bytes;
      c->counters[4] = (double)(h->plan->p1.task_count() + h->plan->p1b.task_count());
      c->counters[5] = (double)h->plan->p2.task_count();
      c->counters[6] = (double)(h->plan->p1.seg_count() + h->plan->p1b.seg_count());
      c->counters[7] = (double)h->plan->p2.seg_count();
      c->counters[8] = (double)h->plan->share_host.size();
      c->counters[9] = (double)h->plan->X.bytes;
    }
    if (c->batched == 2) {
      if (!h->graph) {
        // the plan's task tables were uploaded on this stream; capture only launches
        dev_sync(c->stream);
        graph_begin(c->stream);
        try {
          h->plan->launch(c, h->precision, true);
        } catch (...) {
          graph_abort(c->stream);
          throw;
        }
        h->graph = graph_end(c->stream);
      }
      graph_launch(h->graph, c->stream);
    } else {
      h->plan->launch(c, h->precision, c->batched != 0);
    }
    dev_sync(c->stream);
  });
}

extern "C" tdmps_status tdmps_heff_apply_noalloc(tdmps_heff h, const void* in, void* out) {
  return guard([&] {
    TDMPS_REQUIRE(h && in && out, TDMPS_ERR_ARG, "NULL argument");
    TDMPS_REQUIRE(in != out, TDMPS_ERR_ARG, "in-place apply is not supported");
    Ctx* c = h->ctx;
    dev_set_device(c->device);
    size_t cap = 0;
    char* base = (char*)noalloc_scratch(c->device, &cap);
    TDMPS_REQUIRE(base != nullptr, TDMPS_ERR_HIP, "no-allocation scratch not resolved on this device");
    // the plan (intermediate, split-K parts, shared products, task tables) is laid out in the
    // scratch from its start on every call: another call on this GPU may have reused it
    Arena arena{base, cap, 0};
    Contractor C;
    C.ctx = c;
    C.precision = h->precision;
    auto plan = heff_plan(C, *h->lops, *h->rops, (const cplx*)in, h->kl, h->ket_l, h->ket_r, (cplx*)out, h->bl,
                          h->bra_l, h->bra_r, cplx{1, 0}, false, &arena);
    plan->launch(c, h->precision, true);
    dev_sync(c->stream);
  });
}

extern "C" tdmps_status tdmps_heff_set_precision(tdmps_heff h, int32_t precision) {
  return guard([&] {
    TDMPS_REQUIRE(h, TDMPS_ERR_ARG, "NULL argument");
    TDMPS_REQUIRE(precision >= TDMPS_FP64 && precision <= TDMPS_BF16X6, TDMPS_ERR_ARG,
                  "unknown precision");
    if (precision == h->precision) return;
    dev_bind(h->ctx->device, h->ctx->stream);
    dev_sync(h->ctx->stream);
    graph_destroy(h->graph);
    h->graph = nullptr;
    h->plan.reset();
    h->precision = precision;
  });
}

extern "C" tdmps_status tdmps_heff_flops(tdmps_heff h, double* flops) {
  return guard([&] {
    TDMPS_REQUIRE(h && flops, TDMPS_ERR_ARG, "NULL argument");
    if (!h->plan) {
      // plan once on scratch pointers to count
      DevBuf a(std::max<int64_t>(h->kl.size, 1) * sizeof(cplx)), b(std::max<int64_t>(h->bl.size, 1) * sizeof(cplx));
      tdmps_fit_params prm = internal_params(h->precision);
      Contractor C = make_contractor(h->ctx, &prm);
      auto p = heff_plan(C, *h->lops, *h->rops, a.c(), h->kl, h->ket_l, h->ket_r, b.c(), h->bl, h->bra_l, h->bra_r,
                         cplx{1, 0}, false);
      *flops = p->alg_flops;
      return;
    }
    *flops = h->alg_flops;
  });
}

extern "C" tdmps_status tdmps_heff_destroy(tdmps_heff h) {
  return guard([&] { delete h; });
}

// ---------------------------------------------------------------- differentiation
struct tdmps_traj_s {
  tdmps_ctx ctx = nullptr;
  tdmps::PulseRun run;
};

extern "C" tdmps_status tdmps_pulse_forward(tdmps_mpo H0, const double* h0, const double* m, tdmps_mpo mu,
                                            tdmps_mps psi0, const tdmps_pulse* pulse, double dt, int32_t nsteps,
                                            int32_t checkpoint_every, const tdmps_fit_params* prm, tdmps_traj* out,
                                            double* value) {
  using namespace tdmps;
  return guard([&] {
    TDMPS_REQUIRE(H0 && h0 && m && mu && psi0 && pulse && out && value, TDMPS_ERR_ARG, "NULL argument");
    *out = nullptr;
    check_prm(prm);
    const int L = psi0->L;
    TDMPS_REQUIRE(H0->host.L == L && mu->host.L == L, TDMPS_ERR_ARG, "length mismatch");
    TDMPS_REQUIRE(nsteps >= 1 && checkpoint_every >= 1, TDMPS_ERR_ARG, "need nsteps >= 1 and checkpoint_every >= 1");
    TDMPS_REQUIRE(std::isfinite(dt) && std::isfinite(pulse->amplitude) && std::isfinite(pulse->omega) &&
                      std::isfinite(pulse->t_center) && std::isfinite(pulse->width) && pulse->width > 0,
                  TDMPS_ERR_NUMERIC, "non-finite pulse parameters or width <= 0");
    for (int i = 0; i < L * L; ++i)
      TDMPS_REQUIRE(std::isfinite(h0[i]) && std::isfinite(m[i]), TDMPS_ERR_NUMERIC, "non-finite integrals");
    std::unique_ptr<tdmps_traj_s> t(new tdmps_traj_s());
    t->ctx = psi0->ctx;
    PulseRun& r = t->run;
    r.amplitude = pulse->amplitude;
    r.omega = pulse->omega;
    r.t_center = pulse->t_center;
    r.width = pulse->width;
    r.dt = dt;
    r.nsteps = nsteps;
    r.every = checkpoint_every;
    r.prm = *prm;
    r.h0.assign(h0, h0 + L * L);
    r.m.assign(m, m + L * L);
    for (auto& f : r.field) f = H0->host;
    r.M = build_mpo(L, m, nullptr, 0.0, false);
    r.mu = mu->host;
    Contractor C = make_contractor(psi0->ctx, prm);
    pulse_forward(C, r, psi0);
    publish(psi0->ctx, C);
    *value = r.value;
    *out = t.release();
  });
}

extern "C" tdmps_status tdmps_pulse_backward(tdmps_traj traj, double* dvalue_damplitude) {
  using namespace tdmps;
  return guard([&] {
    TDMPS_REQUIRE(traj && dvalue_damplitude, TDMPS_ERR_ARG, "NULL argument");
    Contractor C = make_contractor(traj->ctx, &traj->run.prm);
    *dvalue_damplitude = pulse_backward(C, traj->run);
    publish(traj->ctx, C);
  });
}

extern "C" tdmps_status tdmps_traj_destroy(tdmps_traj traj) {
  return tdmps::guard([&] { delete traj; });
}
