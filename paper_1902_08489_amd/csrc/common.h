// Shared host-side definitions of the tdmps library (error state, charges, checks).
#pragma once

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "tdmps.h"

namespace tdmps {

// Error carried out of the library as a status code plus a thread-local message.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define TDMPS_REQUIRE(cond, code, msg)                                     \
  do {                                                                     \
    if (!(cond)) throw ::tdmps::Error((code), std::string(msg));           \
  } while (0)

// (n_up, n_dn) carried by the sites left of a bond, or by an operator's left part.
struct Charge {
  int16_t nu = 0, nd = 0;
  Charge() = default;
  Charge(int a, int b) : nu((int16_t)a), nd((int16_t)b) {}
  bool operator==(const Charge& o) const { return nu == o.nu && nd == o.nd; }
  bool operator!=(const Charge& o) const { return !(*this == o); }
  bool operator<(const Charge& o) const { return nu < o.nu || (nu == o.nu && nd < o.nd); }
  Charge operator+(const Charge& o) const { return Charge(nu + o.nu, nd + o.nd); }
  Charge operator-(const Charge& o) const { return Charge(nu - o.nu, nd - o.nd); }
  uint32_t packed() const { return (uint32_t)(uint16_t)nu << 16 | (uint16_t)nd; }
};

// Local basis of one spatial orbital: n = n_up + 2 n_dn -> |0>, |up>, |dn>, |up dn>.
inline Charge local_charge(int n) { return Charge(n & 1, (n >> 1) & 1); }
inline int local_parity(int n) { return ((n & 1) + ((n >> 1) & 1)) & 1; }

}  // namespace tdmps
