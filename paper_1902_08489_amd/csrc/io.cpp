// States from dense vectors (Methods, Eq. (mps)) and the checkpoint file format.
//
// Dense -> MPS: the paper obtains an MPS from a state vector by reshaping it and splitting
// off one site after another with SVDs, keeping the D largest singular values at every
// step.  Here the vector is first written exactly as a block-sparse MPS whose left bonds
// (cuts 1..c) enumerate the configurations of the sites left of the cut and whose right
// bonds (cuts c+1..L-1) those right of it (0/1 selection tensors), with the coefficients on
// site c.  Right canonicalisation (exact up to the cut-off) and one left-to-right pass of
// two-site SVD splits truncated to Dmax then give the sequential-SVD truncation: with the
// sites right of a bond right-orthonormal, the SVD of the two-site tensor at that bond has
// the singular values and left vectors of the remainder matrix of the sequential scheme.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>

#include "io.h"

namespace tdmps {
namespace {

bool feasible(int L, int i, Charge Q, Charge q) {
  return q.nu >= 0 && q.nd >= 0 && q.nu <= i && q.nd <= i && Q.nu - q.nu >= 0 && Q.nd - q.nd >= 0 &&
         Q.nu - q.nu <= L - i && Q.nd - q.nd <= L - i;
}

Bond bond_of(const std::map<Charge, std::vector<int64_t>>& cfg) {
  Bond b;
  for (auto& kv : cfg) {
    b.q.push_back(kv.first);
    b.dim.push_back((int)kv.second.size());
  }
  return b;
}

}  // namespace

Mps* mps_from_dense(Contractor& C, int L, Charge Q, const double* coeffs, int Dmax, double cutoff) {
  TDMPS_REQUIRE(L >= 2 && L <= 12, TDMPS_ERR_ARG, "from_dense supports 2 <= L <= 12");
  TDMPS_REQUIRE(Dmax >= 1, TDMPS_ERR_ARG, "Dmax must be >= 1");
  TDMPS_REQUIRE(Q.nu >= 0 && Q.nd >= 0 && Q.nu <= L && Q.nd <= L, TDMPS_ERR_SECTOR, "total charge out of range");
  int64_t full = 1;
  for (int i = 0; i < L; ++i) full *= 4;
  // every entry finite, and zero outside the (Nu, Nd) sector
  for (int64_t x = 0; x < full; ++x) {
    TDMPS_REQUIRE(std::isfinite(coeffs[2 * x]) && std::isfinite(coeffs[2 * x + 1]), TDMPS_ERR_NUMERIC,
                  "non-finite coefficient");
    int nu = 0, nd = 0;
    for (int64_t y = x; y; y >>= 2) nu += (int)(y & 1), nd += (int)((y >> 1) & 1);
    if (nu != Q.nu || nd != Q.nd)
      TDMPS_REQUIRE(coeffs[2 * x] == 0.0 && coeffs[2 * x + 1] == 0.0, TDMPS_ERR_SECTOR,
                    "the vector has weight outside the (N_up, N_dn) sector");
  }
  const int c = L / 2;
  // left configurations of sites 0..i-1 (base-4 numbers, site 0 most significant) per charge
  std::vector<std::map<Charge, std::vector<int64_t>>> S(c + 1), T(L + 1);
  S[0][Charge(0, 0)] = {0};
  for (int i = 0; i < c; ++i)
    for (auto& kv : S[i])
      for (int64_t x : kv.second)
        for (int n = 0; n < 4; ++n) {
          Charge q = kv.first + local_charge(n);
          if (feasible(L, i + 1, Q, q)) S[i + 1][q].push_back(x * 4 + n);
        }
  // right configurations of sites i..L-1 per left charge Q - charge(config)
  T[L][Q] = {0};
  int64_t w = 1;  // 4^(L-i-1)
  for (int i = L - 1; i > c; --i, w *= 4)
    for (auto& kv : T[i + 1])
      for (int64_t y : kv.second)
        for (int n = 0; n < 4; ++n) {
          Charge q = kv.first - local_charge(n);
          if (feasible(L, i, Q, q)) T[i][q].push_back(n * w + y);
        }
  for (auto& m : S)
    for (auto& kv : m) std::sort(kv.second.begin(), kv.second.end());
  for (int i = c + 1; i <= L; ++i)
    for (auto& kv : T[i]) std::sort(kv.second.begin(), kv.second.end());
  std::vector<Bond> bonds(L + 1);
  for (int i = 0; i <= c; ++i) bonds[i] = bond_of(S[i]);
  for (int i = c + 1; i <= L; ++i) bonds[i] = bond_of(T[i]);
  std::unique_ptr<Mps> m(mps_new(C.ctx, L, bonds));
  std::vector<cplx> host;
  for (int i = 0; i < L; ++i) {
    const SiteLayout& lay = m->lay[i];
    host.assign(lay.size, cplx{0, 0});
    const Bond& l = bonds[i];
    const Bond& r = bonds[i + 1];
    for (int s = 0; s < l.nsec(); ++s)
      for (int n = 0; n < 4; ++n) {
        const int t = lay.rs[s][n];
        if (t < 0) continue;
        cplx* panel = host.data() + lay.panel_off[s] + lay.col[s][n];
        if (i < c) {  // left selection: S_{i+1}[b] = S_i[a] * 4 + n
          const auto& A = S[i].at(l.q[s]);
          const auto& B = S[i + 1].at(r.q[t]);
          for (size_t a = 0; a < A.size(); ++a) {
            auto it = std::lower_bound(B.begin(), B.end(), A[a] * 4 + n);
            if (it != B.end() && *it == A[a] * 4 + n) panel[(int64_t)a * lay.width[s] + (it - B.begin())] = cplx{1, 0};
          }
        } else if (i > c) {  // right selection: T_i[a] = n 4^(L-i-1) + T_{i+1}[b]
          int64_t wi = 1;
          for (int k = i + 1; k < L; ++k) wi *= 4;
          const auto& A = T[i].at(l.q[s]);
          const auto& B = T[i + 1].at(r.q[t]);
          for (size_t b = 0; b < B.size(); ++b) {
            auto it = std::lower_bound(A.begin(), A.end(), n * wi + B[b]);
            if (it != A.end() && *it == n * wi + B[b])
              panel[(int64_t)(it - A.begin()) * lay.width[s] + b] = cplx{1, 0};
          }
        } else {  // coefficients: x = S_c[a] 4^(L-c) + n 4^(L-c-1) + T_{c+1}[b]
          int64_t wr = 1;
          for (int k = c + 1; k < L; ++k) wr *= 4;
          const auto& A = S[c].at(l.q[s]);
          const auto& B = T[c + 1].at(r.q[t]);
          for (size_t a = 0; a < A.size(); ++a)
            for (size_t b = 0; b < B.size(); ++b) {
              const int64_t x = A[a] * 4 * wr + n * wr + B[b];
              panel[(int64_t)a * lay.width[s] + b] = cplx{coeffs[2 * x], coeffs[2 * x + 1]};
            }
        }
      }
    if (lay.size) dev_h2d(m->site[i].p, host.data(), lay.size * sizeof(cplx), C.ctx->stream);
  }
  right_canonicalize(C, m.get(), cutoff);
  for (int i = 0; i + 1 < L; ++i) {
    TwoLayout tl;
    tl.build(m->bond[i], m->bond[i + 2]);
    DevBuf theta(std::max<int64_t>(tl.size, 1) * sizeof(cplx));
    form_theta(C, m.get(), i, theta.c(), tl);
    split_theta(C, theta.c(), tl, m.get(), i, Dmax, cutoff, true);
  }
  dev_sync(C.ctx->stream);
  return m.release();
}

// ---------------------------------------------------------------- checkpoint files
namespace {

constexpr char MAGIC[8] = {'T', 'D', 'M', 'P', 'S', 'v', '1', '\0'};

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  }
};

struct File {
  FILE* f = nullptr;
  explicit File(const char* path, const char* mode) : f(std::fopen(path, mode)) {}
  ~File() {
    if (f) std::fclose(f);
  }
};

void put(FILE* f, Fnv& h, const void* p, size_t n) {
  TDMPS_REQUIRE(std::fwrite(p, 1, n, f) == n, TDMPS_ERR_ARG, "checkpoint write failed");
  h.add(p, n);
}

void get(FILE* f, Fnv& h, void* p, size_t n) {
  TDMPS_REQUIRE(std::fread(p, 1, n, f) == n, TDMPS_ERR_ARG, "checkpoint file is truncated");
  h.add(p, n);
}

}  // namespace

void mps_save(const Mps* m, const char* path) {
  // read the site tensors first: a failed readback leaves no partial file behind
  std::vector<std::vector<cplx>> sites(m->L);
  for (int i = 0; i < m->L; ++i) {
    sites[i].resize(m->lay[i].size);
    if (m->lay[i].size) dev_d2h(sites[i].data(), m->site[i].p, m->lay[i].size * sizeof(cplx), m->ctx->stream);
  }
  File fh(path, "wb");
  TDMPS_REQUIRE(fh.f, TDMPS_ERR_ARG, std::string("cannot open checkpoint for writing: ") + path);
  Fnv h;
  put(fh.f, h, MAGIC, sizeof MAGIC);
  const int32_t head[4] = {m->L, m->total.nu, m->total.nd, 0};
  put(fh.f, h, head, sizeof head);
  for (int i = 0; i <= m->L; ++i) {
    const int32_t n = m->bond[i].nsec();
    put(fh.f, h, &n, sizeof n);
    for (int s = 0; s < n; ++s) {
      const int32_t sec[3] = {m->bond[i].q[s].nu, m->bond[i].q[s].nd, m->bond[i].dim[s]};
      put(fh.f, h, sec, sizeof sec);
    }
  }
  for (int i = 0; i < m->L; ++i) {
    const int64_t n = m->lay[i].size;
    put(fh.f, h, &n, sizeof n);
    if (n) put(fh.f, h, sites[i].data(), n * sizeof(cplx));
  }
  const uint64_t sum = h.h;
  TDMPS_REQUIRE(std::fwrite(&sum, 1, sizeof sum, fh.f) == sizeof sum, TDMPS_ERR_ARG, "checkpoint write failed");
  TDMPS_REQUIRE(std::fflush(fh.f) == 0, TDMPS_ERR_ARG, "checkpoint write failed");
}

Mps* mps_load(Ctx* ctx, const char* path) {
  File fh(path, "rb");
  TDMPS_REQUIRE(fh.f, TDMPS_ERR_ARG, std::string("cannot open checkpoint: ") + path);
  Fnv h;
  char magic[8];
  get(fh.f, h, magic, sizeof magic);
  TDMPS_REQUIRE(std::memcmp(magic, MAGIC, sizeof MAGIC) == 0, TDMPS_ERR_ARG, "not a tdmps checkpoint");
  int32_t head[4];
  get(fh.f, h, head, sizeof head);
  const int L = head[0];
  TDMPS_REQUIRE(L >= 2 && L <= 64, TDMPS_ERR_ARG, "checkpoint: bad chain length");
  std::vector<Bond> bonds(L + 1);
  for (int i = 0; i <= L; ++i) {
    int32_t n = 0;
    get(fh.f, h, &n, sizeof n);
    TDMPS_REQUIRE(n >= 1 && n <= (i + 1) * (i + 1), TDMPS_ERR_ARG, "checkpoint: bad sector count");
    for (int s = 0; s < n; ++s) {
      int32_t sec[3];
      get(fh.f, h, sec, sizeof sec);
      const Charge q(sec[0], sec[1]);
      TDMPS_REQUIRE(sec[2] >= 1 && (bonds[i].q.empty() || bonds[i].q.back() < q), TDMPS_ERR_ARG,
                    "checkpoint: bad sector table");
      bonds[i].q.push_back(q);
      bonds[i].dim.push_back(sec[2]);
    }
  }
  TDMPS_REQUIRE(bonds[L].nsec() == 1 && bonds[L].q[0] == Charge(head[1], head[2]), TDMPS_ERR_ARG,
                "checkpoint: total charge does not match the last bond");
  std::unique_ptr<Mps> m(mps_new(ctx, L, bonds));
  std::vector<cplx> buf;
  for (int i = 0; i < L; ++i) {
    int64_t n = 0;
    get(fh.f, h, &n, sizeof n);
    TDMPS_REQUIRE(n == m->lay[i].size, TDMPS_ERR_ARG, "checkpoint: site size does not match its bonds");
    buf.resize(n);
    if (n) get(fh.f, h, buf.data(), n * sizeof(cplx));
    for (const cplx& z : buf) TDMPS_REQUIRE(std::isfinite(z.x) && std::isfinite(z.y), TDMPS_ERR_NUMERIC, "checkpoint: non-finite data");
    if (n) dev_h2d(m->site[i].p, buf.data(), n * sizeof(cplx), ctx->stream);
  }
  const uint64_t want = h.h;
  uint64_t sum = 0;
  TDMPS_REQUIRE(std::fread(&sum, 1, sizeof sum, fh.f) == sizeof sum, TDMPS_ERR_ARG, "checkpoint file is truncated");
  TDMPS_REQUIRE(sum == want, TDMPS_ERR_ARG, "checkpoint checksum mismatch (corrupt file)");
  char extra;
  TDMPS_REQUIRE(std::fread(&extra, 1, 1, fh.f) == 0, TDMPS_ERR_ARG, "checkpoint: trailing data");
  dev_sync(ctx->stream);
  return m.release();
}

}  // namespace tdmps
