/*
 * Op-counting build of the oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * opcount.cpp compiles oracle.c as C++ with every `double` replaced by
 * `cd`, a type holding one double whose arithmetic operators and math
 * functions perform exactly the same IEEE double operation and count it.
 * The oracle's source and its arithmetic are unchanged; the counts give the
 * floating-point work of one evaluation as the oracle states it.
 *
 * Counting rule: add, subtract, multiply, divide = 1 each (compound
 * assignments included); sqrt, exp, log, sin, cos = 1 each (a transcendental
 * counts as one operation); negation, comparisons, fabs, floor and
 * conversions = 0.  `cd` is trivially copyable with the size and alignment
 * of double, so the library keeps the oracle's C ABI.
 */
#ifndef ORACLE_OPCOUNT_HPP
#define ORACLE_OPCOUNT_HPP
#include <math.h>
#include <stdint.h>

struct OpCounts {
  uint64_t add, mul, div, func;
};
extern thread_local OpCounts orc_ops;

struct cd {
  double v;
  cd() = default;
  constexpr cd(double x) : v(x) {}
  explicit operator double() const { return v; }
  explicit operator float() const { return (float)v; }
  explicit operator int() const { return (int)v; }
  cd &operator+=(cd o) { ++orc_ops.add; v += o.v; return *this; }
  cd &operator-=(cd o) { ++orc_ops.add; v -= o.v; return *this; }
  cd &operator*=(cd o) { ++orc_ops.mul; v *= o.v; return *this; }
  cd &operator/=(cd o) { ++orc_ops.div; v /= o.v; return *this; }
};

inline cd operator+(cd a, cd b) { ++orc_ops.add; return cd(a.v + b.v); }
inline cd operator-(cd a, cd b) { ++orc_ops.add; return cd(a.v - b.v); }
inline cd operator*(cd a, cd b) { ++orc_ops.mul; return cd(a.v * b.v); }
inline cd operator/(cd a, cd b) { ++orc_ops.div; return cd(a.v / b.v); }
inline cd operator-(cd a) { return cd(-a.v); }
inline cd operator+(cd a) { return a; }
inline bool operator<(cd a, cd b) { return a.v < b.v; }
inline bool operator>(cd a, cd b) { return a.v > b.v; }
inline bool operator<=(cd a, cd b) { return a.v <= b.v; }
inline bool operator>=(cd a, cd b) { return a.v >= b.v; }
inline bool operator==(cd a, cd b) { return a.v == b.v; }
inline bool operator!=(cd a, cd b) { return a.v != b.v; }

inline cd sqrt(cd a) { ++orc_ops.func; return cd(::sqrt(a.v)); }
inline cd exp(cd a) { ++orc_ops.func; return cd(::exp(a.v)); }
inline cd log(cd a) { ++orc_ops.func; return cd(::log(a.v)); }
inline cd sin(cd a) { ++orc_ops.func; return cd(::sin(a.v)); }
inline cd cos(cd a) { ++orc_ops.func; return cd(::cos(a.v)); }
inline cd fabs(cd a) { return cd(::fabs(a.v)); }
inline cd floor(cd a) { return cd(::floor(a.v)); }
inline bool isfinite(cd a) { return std::isfinite(a.v); }
inline bool isnan(cd a) { return std::isnan(a.v); }
#endif
