// Shared host-side helpers: status codes, error reporting, small utilities.
#pragma once
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cutcell.h"

namespace cc {

// An error carrying one of the CC_* status codes; converted at the C ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

void set_last_error(const std::string& msg);

// Monomials xi^a with |a| <= deg, ordered by degree, then a0 descending, then a1
// descending.  N4 = 35, N3 = 20.
constexpr int N4 = 35;
constexpr int N3 = 20;
struct MonoTable {
  int e4[N4][3];
  int e3[N3][3];
  int idx4[5][5][5];  // exponent -> index (or -1)
  int idx3[4][4][4];
  MonoTable();
};
const MonoTable& mono();

}  // namespace cc
