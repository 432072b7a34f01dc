// SVD truncation (Methods, "MPS" paragraph: keep the D largest singular values) with a
// QR-preconditioned batched block one-sided Jacobi SVD on the device, always in FP64.
//
// Each charge sector of a two-site tensor is a matrix M (R x C).  It is decomposed as G = M
// or G = M^H, chosen so that the side of M that becomes the canonical site tensor is the
// ell side of G: G = Q R (Householder), block Jacobi on X = R^H until every column pair is
// orthogonal to rounding (X V = W), then G = (Q [V; 0]) Sigma (W Sigma^{-1})^H.  The ell-side
// vectors Q [V; 0] are orthonormal to rounding, so the canonical tensor is exactly isometric
// even for tiny kept singular values; the other side carries sigma.  Truncation: all
// sectors' sigma sorted together (value descending, then sector in charge order, then index),
// at most Dmax kept and only those above cutoff * sigma_max (never fewer than one); no
// renormalisation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>

#include "engine.h"

namespace tdmps {
namespace {

struct SvdJob {
  int R = 0, C = 0;
  bool gm = true;         // G = M (ell side = rows of M) else G = M^H (ell side = columns of M)
  int ell = 0, k = 0, n = 0;  // G is ell x k, n = min(ell, k) singular values
  int64_t goff = 0, boff = 0, xoff = 0, voff = 0, toff = 0;
  std::vector<double> sigma;
};

struct SvdBatch {
  std::vector<SvdJob> jobs;
  DevBuf G, X, V, B, T;
  int64_t gsize = 0, bsize = 0, xsize = 0, vsize = 0, tsize = 0;
  int sweeps = 0, rounds = 0;
  double t_qr = 0;

  // row_side: the rows of M (left of the bond) become the canonical side, else its columns.
  void add(int R, int C, bool row_side) {
    SvdJob j;
    j.R = R;
    j.C = C;
    j.gm = row_side;
    j.ell = j.gm ? R : C;
    j.k = j.gm ? C : R;
    j.n = std::min(j.ell, j.k);
    j.goff = gsize;
    j.boff = bsize;
    j.xoff = xsize;
    j.voff = vsize;
    j.toff = tsize;
    gsize += (int64_t)j.ell * j.k;
    bsize += (int64_t)j.ell * j.n;
    xsize += (int64_t)j.k * j.n;
    vsize += (int64_t)j.n * j.n;
    tsize += (int64_t)((j.n + QR_PANEL - 1) / QR_PANEL) * QR_PANEL * QR_PANEL;
    jobs.push_back(j);
  }
  void alloc() {
    G = DevBuf(std::max<int64_t>(gsize, 1) * sizeof(cplx));
    B = DevBuf(std::max<int64_t>(bsize, 1) * sizeof(cplx));
    X = DevBuf(std::max<int64_t>(xsize, 1) * sizeof(cplx));
    V = DevBuf(std::max<int64_t>(vsize, 1) * sizeof(cplx));
    T = DevBuf(std::max<int64_t>(tsize, 1) * sizeof(cplx));
  }
  cplx* in(int j) const { return G.c() + jobs[j].goff; }
  // After run(): u(j) (ell x n) holds the ell-side singular vectors, w(j) (k x n) the k-side
  // ones, both unit columns, G = u Sigma w^H.
  cplx* u(int j) const { return B.c() + jobs[j].boff; }
  cplx* w(int j) const { return X.c() + jobs[j].xoff; }

  // Copy a block of M (rows r0.., cols c0..) given as a row-major source with leading dim ld.
  void gather(CopyPlan& cp, int j, const cplx* src, int ld, int rows, int cols, int r0, int c0) const {
    const SvdJob& J = jobs[j];
    if (J.gm)  // G[c][r] (column-major) = M[r][c]: dst rows = M cols
      cp.add(src, 1, ld, in(j) + (int64_t)c0 * J.ell + r0, J.ell, cols, rows, 0);
    else  // G[r][c] = conj(M[r][c]) in G's column-major (ell = C) order: dst rows = M rows
      cp.add(src, ld, 1, in(j) + (int64_t)r0 * J.ell + c0, J.ell, rows, cols, 1);
  }

  // Column norms of the matrices described by mats into host memory (maxk per matrix).
  static std::vector<double> norms(Ctx* ctx, const std::vector<SvdMat>& mats, int maxk) {
    DevBuf sig(std::max<size_t>(1, mats.size() * (size_t)maxk) * sizeof(double));
    std::vector<double> hs(mats.size() * (size_t)maxk);
    Staging st;
    const SvdMat* dm = st.put(ctx, mats);
    launch_svd_norms(dm, (int)mats.size(), maxk, (double*)sig.p, ctx->stream);
    dev_d2h(hs.data(), sig.p, hs.size() * sizeof(double), ctx->stream);
    return hs;
  }

  void run(Ctx* ctx) {
    if (jobs.empty()) return;
    const int nm = (int)jobs.size();
    int maxk = 0, maxn = 0;
    std::vector<QrMat> qm(nm);
    std::vector<SvdMat> gmats(nm), xm(nm);
    int cblocks = 0, pairs = 0, maxrounds = 0;
    for (int j = 0; j < nm; ++j) {
      const SvdJob& J = jobs[j];
      maxk = std::max(maxk, J.k);
      maxn = std::max(maxn, J.n);
      QrMat& q = qm[j];
      q.G = G.c() + J.goff;
      q.B = B.c() + J.boff;
      q.X = X.c() + J.xoff;
      q.V = V.c() + J.voff;
      q.T = T.c() + J.toff;
      q.ell = J.ell;
      q.k = J.k;
      q.nsv = J.n;
      q.cb_base = cblocks;
      cblocks += (J.k + QR_PANEL - 1) / QR_PANEL;
      gmats[j] = SvdMat{q.G, q.V, J.ell, J.k, 2, 0, 0.0};
      const int nb = (J.n + SVD_BLOCK - 1) / SVD_BLOCK;
      SvdMat& x = xm[j];
      x.G = q.X;
      x.V = q.V;
      x.ell = J.k;
      x.k = J.n;
      x.nblk = std::max(2, nb + (nb & 1));
      x.pair_base = pairs;
      pairs += x.nblk / 2;
      maxrounds = std::max(maxrounds, x.nblk - 1);
    }
    // Rounding leaves every column with an absolute error of order eps |A|, so the overlap
    // of columns p, q cannot be resolved below ~ eps |A| max(|g_p|, |g_q|): such pairs count
    // as orthogonal (accuracy eps * sigma_max, as for LAPACK).  |X|_F = |G|_F.
    {
      std::vector<double> hs = norms(ctx, gmats, maxk);
      for (int j = 0; j < nm; ++j) {
        double f = 0;
        for (int c = 0; c < jobs[j].k; ++c) f += hs[(size_t)j * maxk + c] * hs[(size_t)j * maxk + c];
        xm[j].thr = 8 * 2.220446049250313e-16 * std::sqrt(f);
      }
    }
    Staging st;
    const QrMat* dq = st.put(ctx, qm);
    const double tq = wall_seconds();
    for (int j0 = 0; j0 < maxn; j0 += QR_PANEL) {
      int rows = 0;
      for (int j = 0; j < nm; ++j)
        if (j0 < jobs[j].n) rows = std::max(rows, jobs[j].ell - j0);
      launch_qr_panel(dq, nm, j0, rows, ctx->stream);
      launch_qr_apply(dq, nm, cblocks, j0, 0, ctx->stream);
    }
    launch_qr_rt(dq, nm, ctx->stream);
    if (ctx->phase_sync) dev_sync(ctx->stream);
    t_qr = wall_seconds() - tq;
    const SvdMat* dm = st.put(ctx, xm);
    launch_svd_init(dm, nm, ctx->stream);
    // Sweeps are queued in batches with one rotation counter each; a sweep whose predecessor
    // rotated nothing skips on the device, so the host reads the counters once per batch.
    const double tol = 1e-15;
    const int max_sweeps = 60;
    // four waves per block pair while every column is short (256 rows or fewer), eight beyond
    int max_len = 0;
    for (const SvdMat& x : xm) max_len = std::max(max_len, std::max(x.ell, x.k));
    const int waves = max_len <= 256 ? 4 : 8;
    DevBuf counter(max_sweeps * sizeof(int32_t));
    int32_t* dc = (int32_t*)counter.p;
    dev_zero(counter.p, counter.bytes, ctx->stream);
    bool converged = maxn <= 1;
    int sweeps_done = 0, queued = 0;
    std::vector<int32_t> rot(max_sweeps);
    while (!converged && queued < max_sweeps) {
      const int batch = std::min(max_sweeps - queued, queued == 0 ? 6 : 3);
      for (int sw = queued; sw < queued + batch; ++sw)
        for (int r = -1; r < maxrounds; ++r)
          launch_svd_round(dm, nm, pairs, r, tol, dc + sw, sw > 0 ? dc + sw - 1 : nullptr, waves, ctx->stream);
      dev_d2h(rot.data() + queued, dc + queued, batch * sizeof(int32_t), ctx->stream);
      for (int sw = queued; sw < queued + batch && !converged; ++sw) {
        sweeps_done = sw + 1;
        converged = rot[sw] == 0;
      }
      queued += batch;
    }
    TDMPS_REQUIRE(converged, TDMPS_ERR_NUMERIC, "Jacobi SVD did not converge");
    sweeps = sweeps_done;
    rounds = sweeps_done * (maxrounds + 1);
    if (std::getenv("TDMPS_SVD_STATS"))
      std::fprintf(stderr, "svd: %d matrices, max n %d, %d rounds per sweep, %d sweeps\n", nm, maxn, maxrounds,
                   sweeps_done);
    std::vector<double> hs = norms(ctx, xm, maxn);
    for (int j = 0; j < nm; ++j)
      jobs[j].sigma.assign(hs.begin() + (size_t)j * maxn, hs.begin() + (size_t)j * maxn + jobs[j].n);
    const double* dsig = st.put(ctx, hs);
    launch_qr_finish(dq, nm, dsig, maxn, ctx->stream);
    for (int j0 = (maxn - 1) / QR_PANEL * QR_PANEL; j0 >= 0; j0 -= QR_PANEL)
      launch_qr_apply(dq, nm, cblocks, j0, 1, ctx->stream);
  }
};

struct Kept {
  int job;
  std::vector<int> cols;  // kept vector indices, sigma descending
};

// global selection; returns per job the kept columns
std::vector<Kept> select(const SvdBatch& b, int Dmax, double cutoff, double* disc, double* norm2) {
  struct C {
    double s;
    int job, idx;
  };
  std::vector<C> all;
  for (size_t j = 0; j < b.jobs.size(); ++j)
    for (int i = 0; i < b.jobs[j].n; ++i) all.push_back({b.jobs[j].sigma[i], (int)j, i});
  std::sort(all.begin(), all.end(), [](const C& x, const C& y) {
    if (x.s != y.s) return x.s > y.s;
    if (x.job != y.job) return x.job < y.job;
    return x.idx < y.idx;
  });
  double smax = all.empty() ? 0.0 : all[0].s;
  size_t keep = 0;
  while (keep < all.size() && (int)keep < Dmax && all[keep].s > cutoff * smax) ++keep;
  if (keep == 0 && !all.empty()) keep = 1;
  double d = 0, n = 0;
  for (size_t i = 0; i < all.size(); ++i) (i < keep ? n : d) += all[i].s * all[i].s;
  *disc = d;
  *norm2 = n;
  std::vector<Kept> out(b.jobs.size());
  for (size_t j = 0; j < out.size(); ++j) out[j].job = (int)j;
  for (size_t i = 0; i < keep; ++i) out[all[i].job].cols.push_back(all[i].idx);  // already sigma-descending
  return out;
}

}  // namespace

TruncResult split_theta(Contractor& C, const cplx* theta, const TwoLayout& tl, Mps* m, int i, int Dmax, double cutoff,
                        bool move_right) {
  const double t0 = wall_seconds();
  struct Acc {
    Contractor& C;
    double t0;
    ~Acc() { C.t_svd += wall_seconds() - t0; }
  } acc_{C, t0};
  const Bond& l = m->bond[i];
  const Bond& r = m->bond[i + 2];
  // middle charges and their row / column groups
  std::vector<Charge> mids;
  for (int s = 0; s < l.nsec(); ++s)
    for (int s1 = 0; s1 < 4; ++s1) mids.push_back(l.q[s] + local_charge(s1));
  std::sort(mids.begin(), mids.end());
  mids.erase(std::unique(mids.begin(), mids.end()), mids.end());
  std::vector<Charge> sec;
  std::vector<std::vector<std::pair<int, int>>> rowg, colg;  // (s, s1) and (s2, t)
  std::vector<std::vector<int>> rowoff, coloff;
  for (Charge qm : mids) {
    std::vector<std::pair<int, int>> rg, cg;
    std::vector<int> ro, co;
    int R = 0, Cc = 0;
    for (int s = 0; s < l.nsec(); ++s)
      for (int s1 = 0; s1 < 4; ++s1)
        if (l.q[s] + local_charge(s1) == qm) {
          rg.push_back({s, s1});
          ro.push_back(R);
          R += l.dim[s];
        }
    for (int s2 = 0; s2 < 4; ++s2) {
      int t = r.find(qm + local_charge(s2));
      if (t < 0) continue;
      cg.push_back({s2, t});
      co.push_back(Cc);
      Cc += r.dim[t];
    }
    if (R == 0 || Cc == 0) continue;
    sec.push_back(qm);
    rowg.push_back(rg);
    colg.push_back(cg);
    rowoff.push_back(ro);
    coloff.push_back(co);
  }
  SvdBatch b;
  for (size_t k = 0; k < sec.size(); ++k) {
    int R = 0, Cc = 0;
    for (auto& x : rowg[k]) R += l.dim[x.first];
    for (auto& x : colg[k]) Cc += r.dim[x.second];
    b.add(R, Cc, move_right);
  }
  b.alloc();
  {
    CopyPlan cp;
    for (size_t k = 0; k < sec.size(); ++k)
      for (size_t a = 0; a < rowg[k].size(); ++a)
        for (size_t c = 0; c < colg[k].size(); ++c) {
          int s = rowg[k][a].first, s1 = rowg[k][a].second, s2 = colg[k][c].first, t = colg[k][c].second;
          int sig = s1 * 4 + s2;
          if (tl.rs[s][sig] != t) continue;
          b.gather(cp, (int)k, theta + tl.panel_off[s] + tl.col[s][sig], tl.width[s], l.dim[s], r.dim[t], rowoff[k][a],
                   coloff[k][c]);
        }
    cp.run(C.ctx);
  }
  b.run(C.ctx);
  C.n_svd += 1;
  C.svd_sweeps += b.sweeps;
  C.svd_rounds += b.rounds;
  C.t_qr += b.t_qr;
  TruncResult res;
  auto kept = select(b, Dmax, cutoff, &res.discarded, &res.norm2);
  // new middle bond
  Bond mid;
  std::vector<int> job_of_sec;
  for (size_t k = 0; k < sec.size(); ++k)
    if (!kept[k].cols.empty()) {
      mid.q.push_back(sec[k]);
      mid.dim.push_back((int)kept[k].cols.size());
      job_of_sec.push_back((int)k);
      res.kept += (int)kept[k].cols.size();
    }
  SiteLayout la, lb;
  la.build(l, mid);
  lb.build(mid, r);
  DevBuf A(la.size * sizeof(cplx)), B(lb.size * sizeof(cplx));
  // per kept sector: index and scale arrays
  std::vector<int32_t> idx;
  std::vector<double> one_s, sig_s;
  std::vector<int64_t> base(mid.nsec());
  for (int ms = 0; ms < mid.nsec(); ++ms) {
    const auto& kc = kept[job_of_sec[ms]].cols;
    base[ms] = (int64_t)idx.size();
    const auto& sv = b.jobs[job_of_sec[ms]].sigma;
    for (int c : kc) {
      idx.push_back(c);
      one_s.push_back(1.0);
      sig_s.push_back(sv[c]);
    }
  }
  Staging st;
  const int32_t* didx = st.put(C.ctx, idx);
  const double* d1 = st.put(C.ctx, one_s);
  const double* ds = st.put(C.ctx, sig_s);
  CopyPlan cp;
  for (int ms = 0; ms < mid.nsec(); ++ms) {
    int k = job_of_sec[ms];
    const SvdJob& J = b.jobs[k];
    int nk = mid.dim[ms];
    const int32_t* ix = didx + base[ms];
    // left site blocks (s, s1) -> ms: ul (times sigma when moving left)
    const double* lsc = move_right ? d1 + base[ms] : ds + base[ms];
    for (size_t a = 0; a < rowg[k].size(); ++a) {
      int s = rowg[k][a].first, s1 = rowg[k][a].second;
      cplx* dst = A.c() + la.panel_off[s] + la.col[s][s1];
      if (J.gm)  // ul = u
        cp.add(b.u(k) + rowoff[k][a], 1, J.ell, dst, la.width[s], l.dim[s], nk, 0, nullptr, ix, nullptr, lsc);
      else  // ul = w
        cp.add(b.w(k) + rowoff[k][a], 1, J.k, dst, la.width[s], l.dim[s], nk, 0, nullptr, ix, nullptr, lsc);
    }
    // right site blocks ms -> (s2, t): (sigma when moving right) vr^H
    const double* rsc = move_right ? ds + base[ms] : d1 + base[ms];
    for (size_t c = 0; c < colg[k].size(); ++c) {
      int s2 = colg[k][c].first, t = colg[k][c].second;
      cplx* dst = B.c() + lb.panel_off[ms] + lb.col[ms][s2];
      if (J.gm)  // vr = w
        cp.add(b.w(k) + coloff[k][c], J.k, 1, dst, lb.width[ms], nk, r.dim[t], 1, ix, nullptr, rsc, nullptr);
      else  // vr = u
        cp.add(b.u(k) + coloff[k][c], J.ell, 1, dst, lb.width[ms], nk, r.dim[t], 1, ix, nullptr, rsc, nullptr);
    }
  }
  cp.run(C.ctx);
  m->bond[i + 1] = mid;
  m->lay[i] = la;
  m->lay[i + 1] = lb;
  m->site[i] = std::move(A);
  m->site[i + 1] = std::move(B);
  res.mid = mid;
  return res;
}

void right_canonicalize(Contractor& C, Mps* m, double cutoff) {
  for (int i = m->L - 1; i >= 1; --i) {
    const Bond& l = m->bond[i];
    const SiteLayout& lay = m->lay[i];
    SvdBatch b;
    std::vector<int> job_of(l.nsec(), -1);
    for (int s = 0; s < l.nsec(); ++s)
      if (lay.width[s] > 0) {
        job_of[s] = (int)b.jobs.size();
        b.add(l.dim[s], lay.width[s], false);
      }
    b.alloc();
    {
      CopyPlan cp;
      for (int s = 0; s < l.nsec(); ++s)
        if (job_of[s] >= 0) b.gather(cp, job_of[s], m->site[i].c() + lay.panel_off[s], lay.width[s], l.dim[s], lay.width[s], 0, 0);
      cp.run(C.ctx);
    }
    b.run(C.ctx);
    C.n_svd += 1;
    C.svd_sweeps += b.sweeps;
    C.svd_rounds += b.rounds;
    C.t_qr += b.t_qr;
    double disc, n2;
    auto kept = select(b, 1 << 30, cutoff, &disc, &n2);
    Bond nb;
    std::vector<int> sec_of;
    for (int s = 0; s < l.nsec(); ++s)
      if (job_of[s] >= 0 && !kept[job_of[s]].cols.empty()) {
        nb.q.push_back(l.q[s]);
        nb.dim.push_back((int)kept[job_of[s]].cols.size());
        sec_of.push_back(s);
      }
    SiteLayout nl, pl;
    nl.build(nb, m->bond[i + 1]);
    pl.build(m->bond[i - 1], nb);
    DevBuf A(nl.size * sizeof(cplx)), P(pl.size * sizeof(cplx));
    std::vector<int32_t> idx;
    std::vector<double> ones, sig;
    std::vector<int64_t> base;
    for (size_t ns = 0; ns < sec_of.size(); ++ns) {
      int j = job_of[sec_of[ns]];
      base.push_back((int64_t)idx.size());
      for (int c : kept[j].cols) {
        idx.push_back(c);
        ones.push_back(1.0);
        double sv = b.jobs[j].sigma[c];
        sig.push_back(sv);
      }
    }
    Staging st;
    const int32_t* didx = st.put(C.ctx, idx);
    const double* d1 = st.put(C.ctx, ones);
    const double* ds = st.put(C.ctx, sig);
    // new site i = vr^H (rows = kept), and US = ul * sigma per sector (D_s x k)
    int64_t us_size = 0;
    std::vector<int64_t> us_off;
    for (size_t ns = 0; ns < sec_of.size(); ++ns) {
      us_off.push_back(us_size);
      us_size += (int64_t)l.dim[sec_of[ns]] * nb.dim[ns];
    }
    DevBuf US(std::max<int64_t>(us_size, 1) * sizeof(cplx));
    CopyPlan cp;
    for (size_t ns = 0; ns < sec_of.size(); ++ns) {
      int s = sec_of[ns];
      int j = job_of[s];
      const SvdJob& J = b.jobs[j];
      int nk = nb.dim[ns];
      const int32_t* ix = didx + base[ns];
      // vr^H into the new panel (width identical to the old one: same right bond); G = M^H so
      // vr = u (isometric) and ul = w
      cplx* dst = A.c() + nl.panel_off[ns];
      cp.add(b.u(j), J.ell, 1, dst, nl.width[ns], nk, lay.width[s], 1, ix, nullptr, d1 + base[ns], nullptr);
      cp.add(b.w(j), 1, J.k, US.c() + us_off[ns], nk, l.dim[s], nk, 0, nullptr, ix, nullptr, ds + base[ns]);
    }
    cp.run(C.ctx);
    // site i-1: A_{i-1}[a, n, s] (US)_s
    const Bond& pbl = m->bond[i - 1];
    const SiteLayout& ol = m->lay[i - 1];
    if (pl.size) dev_zero(P.p, P.bytes, C.ctx->stream);
    GemmPlan gp;
    for (int a = 0; a < pbl.nsec(); ++a)
      for (int n = 0; n < 4; ++n) {
        int so = ol.rs[a][n];
        int sn = pl.rs[a][n];
        if (so < 0 || sn < 0) continue;
        TDMPS_REQUIRE(sec_of[sn] == so, TDMPS_ERR_NUMERIC, "internal: canonicalisation sector map");
        gp.begin_task(P.c() + pl.panel_off[a] + pl.col[a][n], 0, pl.width[a], pbl.dim[a], nb.dim[sn], 1, false);
        gp.add_seg(m->site[i - 1].c() + ol.panel_off[a] + ol.col[a][n], 0, 0, ol.width[a], OP_N, US.c() + us_off[sn],
                   0, 0, nb.dim[sn], OP_N, l.dim[so], 1, cplx{1, 0});
      }
    gp.run(C.ctx, TDMPS_FP64, C.batched);
    m->bond[i] = nb;
    m->lay[i] = nl;
    m->lay[i - 1] = pl;
    m->site[i] = std::move(A);
    m->site[i - 1] = std::move(P);
  }
}

}  // namespace tdmps
