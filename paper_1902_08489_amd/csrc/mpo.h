// Host-side matrix product operator of the electronic Hamiltonian (Eq. (hamil)).
#pragma once

#include <array>
#include <utility>

#include "common.h"

namespace tdmps {

// One non-zero of a site tensor: W[w -> v] contains coefficient c on the matrix unit
// |s><sp| of the local 4-dimensional space.
struct MpoEntry {
  int32_t w, v;
  int8_t s, sp;
  double c;
};

// Channels (MPO bond indices) at one cut, ordered class-major: channels with equal
// left-part charge form a contiguous "class".
struct MpoCut {
  std::vector<uint64_t> key;
  std::vector<Charge> q;
  std::vector<int8_t> parity;
  std::vector<Charge> cls_q;
  std::vector<int32_t> cls_start, cls_count, cls_of;
  int size() const { return (int)key.size(); }
  int find_class(Charge c) const {
    for (size_t k = 0; k < cls_q.size(); ++k)
      if (cls_q[k] == c) return (int)k;
    return -1;
  }
};

struct OneBodyRef {
  int32_t site, entry;
  int16_t p, q;
  double factor;
};

uint64_t next_mpo_version();

struct MpoHost {
  int L = 0;
  std::vector<MpoCut> cut;                   // L+1 cuts (cut i is left of site i)
  std::vector<std::vector<MpoEntry>> W;      // L sites, entries sorted by (v, w, s, sp)
  std::vector<std::vector<double>> c_fixed;  // part of each coefficient not from h
  std::vector<OneBodyRef> onebody;           // linear dependence of coefficients on h
  std::vector<double> h;
  // (charge, channel count) classes per cut of the plain rule: the operator whose bond
  // dimension is 2L^2 + 3L + 2 at the centre, the reference of the algorithmic flop count
  std::vector<std::vector<std::pair<Charge, int>>> plain_cls;
  // Identifies the coefficients: a process-wide counter gives every new operator and every
  // set_one_body a fresh value, and copies keep it while their coefficients are equal.
  uint64_t version = next_mpo_version();
};

// adjacent_window: at the cuts within this distance of the chain centre, pair channels next to
// an operator site are named by the other side (see mpo.cpp); -1 gives the plain rule (left
// pairs left of the centre, right pairs right of it) everywhere.
MpoHost build_mpo(int L, const double* h, const double* eri, double e0, bool two_body, int adjacent_window = -1);
// Kind of a channel (from MpoCut::key): 0 = identity so far, 1 = complete (H), 2 = one open
// operator left of the cut (*so = spin orbital 2p + spin, *op = 0 creator / 1 annihilator),
// 3 = anything else.
int mpo_channel_kind(uint64_t key, int* so, int* op);
void mpo_set_one_body(MpoHost& m, const double* h);
void mpo_to_dense(const MpoHost& m, double* out);
double mpo_det_element(const MpoHost& m, const uint8_t* bra, const uint8_t* ket);

}  // namespace tdmps
