// Tile-shape autotuner of the grouped block GEMM.
//
// The symmetry blocks of the contractions come in a few hundred uneven shapes (sector sizes
// 1..~500, reductions from one sector to ~10^3 stacked channels).  Which tile shape runs a
// block product fastest depends on padding, on how many tiles the launch has and on the
// reduction length, so the choice is measured: for every bucket of (rows, columns, total
// reduction length) a grouped launch of synthetic products of the bucket's upper-edge shape,
// enough of them to fill the chip, is timed with every tile shape, and the fastest shape is
// recorded.  The plan builder then picks a task's shape from its bucket.
#include <algorithm>
#include <vector>

#include "engine.h"

namespace tdmps {

void autotune_tiles(Ctx* ctx, int precision, TileTable& tab) {
  TDMPS_REQUIRE(precision >= 0 && precision < 4, TDMPS_ERR_ARG, "unknown precision");
  const int KREP[TILE_NK] = {32, 256, 2048};  // representative total reduction per bucket
  const int KCH = 64;                         // reduction split into channels of <= 64 (as in the stacked products)
  const int64_t POOL = int64_t(1) << 23;      // complex elements per operand pool (128 MiB)
  const int64_t OUT_ELEMS = int64_t(1) << 21;  // output elements per timed launch
  DevBuf A(POOL * sizeof(cplx)), B(POOL * sizeof(cplx)), C(OUT_ELEMS * sizeof(cplx));
  dev_zero(A.p, A.bytes, ctx->stream);
  dev_zero(B.p, B.bytes, ctx->stream);
  void* e0 = dev_event_create();
  void* e1 = dev_event_create();
  try {
    for (int im = 0; im < TILE_NB; ++im)
      for (int in = 0; in < TILE_NB; ++in)
        for (int ik = 0; ik < TILE_NK; ++ik) {
          const int m = TILE_EDGES[im], n = TILE_EDGES[in], ktot = KREP[ik];
          const int k = std::min(ktot, KCH), nred = ktot / k;
          const int64_t ntask = std::max<int64_t>(1, OUT_ELEMS / ((int64_t)m * n));
          const int64_t aslots = std::max<int64_t>(1, POOL / ((int64_t)m * ktot));
          const int64_t bslots = std::max<int64_t>(1, POOL / ((int64_t)ktot * n));
          std::vector<GemmSeg> segs((size_t)ntask);
          std::vector<GemmTask> tasks((size_t)ntask);
          for (int64_t t = 0; t < ntask; ++t) {
            GemmSeg& g = segs[t];
            g.A = A.c() + ((t * 7919) % aslots) * (int64_t)m * ktot;
            g.B = B.c() + ((t * 104729) % bslots) * (int64_t)ktot * n;
            g.bsA = g.bsB = 0;
            g.rsA = (int64_t)m * k;
            g.rsB = (int64_t)k * n;
            g.nred = nred;
            g.k = k;
            g.lda = k;
            g.ldb = n;
            g.opA = OP_N;
            g.opB = OP_N;
            g.alpha = cplx{1, 0};
            GemmTask& c = tasks[t];
            c.C = C.c() + t * (int64_t)m * n;
            c.bsC = 0;
            c.ldc = n;
            c.m = m;
            c.n = n;
            c.nbatch = 1;
            c.seg0 = (int32_t)t;
            c.nseg = 1;
            c.flags = 0;
          }
          DevBuf dsegs(segs.size() * sizeof(GemmSeg));
          dev_h2d(dsegs.p, segs.data(), segs.size() * sizeof(GemmSeg), ctx->stream);
          const double flops = 8.0 * m * n * (double)ktot * ntask;
          int best = 0;
          double best_rate = -1;
          for (int cfg = 0; cfg < GEMM_NCFG; ++cfg) {
            const int bm = gemm_tile_m(cfg), bn = gemm_tile_n(cfg);
            const int tm = (m + bm - 1) / bm, tn = (n + bn - 1) / bn;
            std::vector<int32_t> tt((size_t)(ntask * tm * tn));
            for (int64_t t = 0; t < ntask; ++t) {
              tasks[t].tiles_m = tm;
              tasks[t].tiles_n = tn;
              tasks[t].tile_base = t * tm * tn;
              std::fill(tt.begin() + t * tm * tn, tt.begin() + (t + 1) * tm * tn, (int32_t)t);
            }
            DevBuf dt(tasks.size() * sizeof(GemmTask)), dtile(tt.size() * sizeof(int32_t));
            dev_h2d(dt.p, tasks.data(), tasks.size() * sizeof(GemmTask), ctx->stream);
            dev_h2d(dtile.p, tt.data(), tt.size() * sizeof(int32_t), ctx->stream);
            const int64_t tiles = (int64_t)tt.size();
            launch_gemm((const GemmTask*)dt.p, (const GemmSeg*)dsegs.p, (const int32_t*)dtile.p, tiles, cfg, precision,
                        ctx->stream, 0);
            const int reps = 3;
            dev_event_record(e0, ctx->stream);
            for (int r = 0; r < reps; ++r)
              launch_gemm((const GemmTask*)dt.p, (const GemmSeg*)dsegs.p, (const int32_t*)dtile.p, tiles, cfg,
                          precision, ctx->stream, 0);
            dev_event_record(e1, ctx->stream);
            const double ms = dev_event_elapsed_ms(e0, e1) / reps;
            const double rate = flops / (ms * 1e-3);
            if (rate > best_rate) {
              best_rate = rate;
              best = cfg;
            }
          }
          tab.cfg[im][in][ik] = (int8_t)best;
          tab.tflops[im][in][ik] = (float)(best_rate * 1e-12);
        }
  } catch (...) {
    dev_event_destroy(e0);
    dev_event_destroy(e1);
    throw;
  }
  dev_event_destroy(e0);
  dev_event_destroy(e1);
  tab.valid = true;
}

}  // namespace tdmps
