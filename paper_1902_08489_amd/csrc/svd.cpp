// SVD truncation (Methods, "MPS" paragraph: keep the D largest singular values) with a
// batched one-sided Jacobi SVD on the device, always in FP64.
//
// Each charge sector of a two-site tensor is a matrix M (R x C).  The smaller dimension is
// orthogonalised: G = M (R >= C) or G = M^H (R < C), rotating column pairs of G and
// accumulating the rotations in V until every pair is orthogonal to rounding; then
// sigma_j = |g_j| and M = sum_j sigma_j ul_j vr_j^H with (ul, vr) = (g/sigma, v) or
// (v, g/sigma).  Truncation: all sectors' sigma sorted together (value descending, then
// sector in charge order, then index), at most Dmax kept and only those above
// cutoff * sigma_max (never fewer than one); no renormalisation.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "engine.h"

namespace tdmps {
namespace {

struct SvdJob {
  int R = 0, C = 0;
  bool tall = true;  // G = M (R >= C) else G = M^H
  int ell = 0, k = 0;
  int64_t goff = 0, voff = 0;
  std::vector<double> sigma;
};

struct SvdBatch {
  std::vector<SvdJob> jobs;
  DevBuf G, V;
  int64_t gsize = 0, vsize = 0;

  void add(int R, int C) {
    SvdJob j;
    j.R = R;
    j.C = C;
    j.tall = R >= C;
    j.ell = j.tall ? R : C;
    j.k = j.tall ? C : R;
    j.goff = gsize;
    j.voff = vsize;
    gsize += (int64_t)j.ell * j.k;
    vsize += (int64_t)j.k * j.k;
    jobs.push_back(j);
  }
  void alloc() {
    G = DevBuf(std::max<int64_t>(gsize, 1) * sizeof(cplx));
    V = DevBuf(std::max<int64_t>(vsize, 1) * sizeof(cplx));
  }
  cplx* g(int j) const { return G.c() + jobs[j].goff; }
  cplx* v(int j) const { return V.c() + jobs[j].voff; }

  // Copy a block of M (rows r0.., cols c0..) given as a row-major source with leading dim ld.
  void gather(CopyPlan& cp, int j, const cplx* src, int ld, int rows, int cols, int r0, int c0) const {
    const SvdJob& J = jobs[j];
    if (J.tall)  // G[c][r] (column-major) = M[r][c]: dst rows = M cols
      cp.add(src, 1, ld, g(j) + (int64_t)c0 * J.ell + r0, J.ell, cols, rows, 0);
    else  // G[r][c] = conj(M[r][c]) in G's column-major (ell = C) order: dst rows = M rows
      cp.add(src, ld, 1, g(j) + (int64_t)r0 * J.ell + c0, J.ell, rows, cols, 1);
  }

  void run(Ctx* ctx) {
    if (jobs.empty()) return;
    std::vector<SvdMat> mats;
    int64_t pairs = 0;
    int maxk = 0, maxrounds = 0;
    for (size_t j = 0; j < jobs.size(); ++j) {
      SvdMat m;
      m.G = g((int)j);
      m.V = v((int)j);
      m.ell = jobs[j].ell;
      m.k = jobs[j].k;
      m.kpad = m.k + (m.k & 1);
      m.pair_base = (int32_t)pairs;
      pairs += m.kpad / 2;
      maxk = std::max(maxk, m.k);
      maxrounds = std::max(maxrounds, m.kpad - 1);
      mats.push_back(m);
    }
    // Rounding leaves every column with an absolute error of order eps |A|, so the
    // overlap of columns p, q cannot be resolved below ~ eps |A| max(|g_p|, |g_q|):
    // such pairs count as orthogonal (accuracy eps * sigma_max, as for LAPACK).
    DevBuf sig(std::max<size_t>(1, mats.size() * (size_t)maxk) * sizeof(double));
    std::vector<double> hs(mats.size() * (size_t)maxk);
    {
      Staging st0;
      const SvdMat* dm0 = st0.put(ctx, mats);
      launch_svd_norms(dm0, (int)mats.size(), maxk, (double*)sig.p, ctx->stream);
      dev_d2h(hs.data(), sig.p, hs.size() * sizeof(double), ctx->stream);
    }
    for (size_t j = 0; j < mats.size(); ++j) {
      double f = 0;
      for (int c = 0; c < mats[j].k; ++c) f += hs[j * maxk + c] * hs[j * maxk + c];
      mats[j].thr = 8 * 2.220446049250313e-16 * std::sqrt(f);
    }
    Staging st;
    const SvdMat* dm = st.put(ctx, mats);
    launch_svd_init(dm, (int)mats.size(), ctx->stream);
    DevBuf counter(sizeof(int32_t));
    const double tol = 1e-15;
    const int max_sweeps = 60;
    bool converged = maxk <= 1;
    for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
      dev_zero(counter.p, sizeof(int32_t), ctx->stream);
      for (int r = 0; r < maxrounds; ++r)
        launch_svd_round(dm, (int)mats.size(), pairs, r, tol, (int32_t*)counter.p, ctx->stream);
      int32_t rot = 0;
      dev_d2h(&rot, counter.p, sizeof(int32_t), ctx->stream);
      converged = rot == 0;
    }
    TDMPS_REQUIRE(converged, TDMPS_ERR_NUMERIC, "Jacobi SVD did not converge");
    launch_svd_norms(dm, (int)mats.size(), maxk, (double*)sig.p, ctx->stream);
    dev_d2h(hs.data(), sig.p, hs.size() * sizeof(double), ctx->stream);
    for (size_t j = 0; j < jobs.size(); ++j)
      jobs[j].sigma.assign(hs.begin() + j * maxk, hs.begin() + j * maxk + jobs[j].k);
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
    for (int i = 0; i < b.jobs[j].k; ++i) all.push_back({b.jobs[j].sigma[i], (int)j, i});
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
    b.add(R, Cc);
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
  std::vector<double> one_s, sig_s, inv_s;
  std::vector<int64_t> base(mid.nsec());
  for (int ms = 0; ms < mid.nsec(); ++ms) {
    const auto& kc = kept[job_of_sec[ms]].cols;
    base[ms] = (int64_t)idx.size();
    const auto& sv = b.jobs[job_of_sec[ms]].sigma;
    for (int c : kc) {
      idx.push_back(c);
      one_s.push_back(1.0);
      sig_s.push_back(sv[c]);
      inv_s.push_back(sv[c] > 0 ? 1.0 / sv[c] : 0.0);
    }
  }
  Staging st;
  const int32_t* didx = st.put(C.ctx, idx);
  const double* d1 = st.put(C.ctx, one_s);
  const double* ds = st.put(C.ctx, sig_s);
  const double* di = st.put(C.ctx, inv_s);
  CopyPlan cp;
  for (int ms = 0; ms < mid.nsec(); ++ms) {
    int k = job_of_sec[ms];
    const SvdJob& J = b.jobs[k];
    int nk = mid.dim[ms];
    const int32_t* ix = didx + base[ms];
    // left site blocks (s, s1) -> ms: ul * (sigma if !move_right)
    for (size_t a = 0; a < rowg[k].size(); ++a) {
      int s = rowg[k][a].first, s1 = rowg[k][a].second;
      cplx* dst = A.c() + la.panel_off[s] + la.col[s][s1];
      if (J.tall) {  // ul = g / sigma
        const double* sc = move_right ? di + base[ms] : d1 + base[ms];
        cp.add(b.g(k) + rowoff[k][a], 1, J.ell, dst, la.width[s], l.dim[s], nk, 0, nullptr, ix, nullptr, sc);
      } else {  // ul = v
        const double* sc = move_right ? d1 + base[ms] : ds + base[ms];
        cp.add(b.v(k) + rowoff[k][a], 1, J.k, dst, la.width[s], l.dim[s], nk, 0, nullptr, ix, nullptr, sc);
      }
    }
    // right site blocks ms -> (s2, t): (sigma if move_right) * vr^H
    for (size_t c = 0; c < colg[k].size(); ++c) {
      int s2 = colg[k][c].first, t = colg[k][c].second;
      cplx* dst = B.c() + lb.panel_off[ms] + lb.col[ms][s2];
      if (J.tall) {  // vr = v
        const double* sc = move_right ? ds + base[ms] : d1 + base[ms];
        cp.add(b.v(k) + coloff[k][c], J.k, 1, dst, lb.width[ms], nk, r.dim[t], 1, ix, nullptr, sc, nullptr);
      } else {  // vr = g / sigma
        const double* sc = move_right ? d1 + base[ms] : di + base[ms];
        cp.add(b.g(k) + coloff[k][c], J.ell, 1, dst, lb.width[ms], nk, r.dim[t], 1, ix, nullptr, sc, nullptr);
      }
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
        b.add(l.dim[s], lay.width[s]);
      }
    b.alloc();
    {
      CopyPlan cp;
      for (int s = 0; s < l.nsec(); ++s)
        if (job_of[s] >= 0) b.gather(cp, job_of[s], m->site[i].c() + lay.panel_off[s], lay.width[s], l.dim[s], lay.width[s], 0, 0);
      cp.run(C.ctx);
    }
    b.run(C.ctx);
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
    std::vector<double> ones, sig, inv;
    std::vector<int64_t> base;
    for (size_t ns = 0; ns < sec_of.size(); ++ns) {
      int j = job_of[sec_of[ns]];
      base.push_back((int64_t)idx.size());
      for (int c : kept[j].cols) {
        idx.push_back(c);
        ones.push_back(1.0);
        double sv = b.jobs[j].sigma[c];
        sig.push_back(sv);
        inv.push_back(sv > 0 ? 1.0 / sv : 0.0);
      }
    }
    Staging st;
    const int32_t* didx = st.put(C.ctx, idx);
    const double* d1 = st.put(C.ctx, ones);
    const double* ds = st.put(C.ctx, sig);
    const double* di = st.put(C.ctx, inv);
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
      // vr^H into the new panel (width identical to the old one: same right bond)
      cplx* dst = A.c() + nl.panel_off[ns];
      if (J.tall)
        cp.add(b.v(j), J.k, 1, dst, nl.width[ns], nk, lay.width[s], 1, ix, nullptr, d1 + base[ns], nullptr);
      else
        cp.add(b.g(j), J.ell, 1, dst, nl.width[ns], nk, lay.width[s], 1, ix, nullptr, di + base[ns], nullptr);
      if (J.tall)
        cp.add(b.g(j), 1, J.ell, US.c() + us_off[ns], nk, l.dim[s], nk, 0, nullptr, ix, nullptr, d1 + base[ns]);
      else
        cp.add(b.v(j), 1, J.k, US.c() + us_off[ns], nk, l.dim[s], nk, 0, nullptr, ix, nullptr, ds + base[ns]);
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
    gp.run(C.ctx, TDMPS_FP64);
    m->bond[i] = nb;
    m->lay[i] = nl;
    m->lay[i - 1] = pl;
    m->site[i] = std::move(A);
    m->site[i - 1] = std::move(P);
  }
}

}  // namespace tdmps
