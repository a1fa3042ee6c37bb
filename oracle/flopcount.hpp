// flopcount.hpp -- operation-counting stand-in for double, force-included
// (g++ -include) when oracle/mhd_oracle.c is compiled as C++ by
// oracle/flopcount.py.  Test infrastructure only.
//
// Every +, -, *, / and square root of two floating-point values counts one
// flop (there is no fused multiply-add in the oracle); negation, absolute
// value, min/max and comparisons count none.  The values themselves are
// computed in double exactly as in the plain build.
#pragma once
#include <cmath>
#include <cstdlib>
#include <cstring>

extern "C" {
unsigned long long orc_flops_total = 0;
unsigned long long orc_flops(void) { return orc_flops_total; }
void orc_flops_reset(void) { orc_flops_total = 0; }
}

struct fd {
  double v;
  fd() = default;
  constexpr fd(double x) : v(x) {}
  fd(int x) : v(x) {}
  fd(long x) : v((double)x) {}
  fd(unsigned long x) : v((double)x) {}
  fd(long long x) : v((double)x) {}
  fd(unsigned long long x) : v((double)x) {}
  explicit operator int() const { return (int)v; }
  fd& operator+=(fd o) { v += o.v; orc_flops_total++; return *this; }
  fd& operator-=(fd o) { v -= o.v; orc_flops_total++; return *this; }
  fd& operator*=(fd o) { v *= o.v; orc_flops_total++; return *this; }
  fd& operator/=(fd o) { v /= o.v; orc_flops_total++; return *this; }
};
inline fd operator+(fd a, fd b) { orc_flops_total++; return fd(a.v + b.v); }
inline fd operator-(fd a, fd b) { orc_flops_total++; return fd(a.v - b.v); }
inline fd operator*(fd a, fd b) { orc_flops_total++; return fd(a.v * b.v); }
inline fd operator/(fd a, fd b) { orc_flops_total++; return fd(a.v / b.v); }
inline fd operator-(fd a) { return fd(-a.v); }
inline bool operator<(fd a, fd b) { return a.v < b.v; }
inline bool operator>(fd a, fd b) { return a.v > b.v; }
inline bool operator<=(fd a, fd b) { return a.v <= b.v; }
inline bool operator>=(fd a, fd b) { return a.v >= b.v; }
inline bool operator==(fd a, fd b) { return a.v == b.v; }
inline bool operator!=(fd a, fd b) { return a.v != b.v; }
inline fd sqrt(fd a) { orc_flops_total++; return fd(std::sqrt(a.v)); }
inline fd fabs(fd a) { return fd(std::fabs(a.v)); }
inline fd fmax(fd a, fd b) { return fd(std::fmax(a.v, b.v)); }
inline fd fmin(fd a, fd b) { return fd(std::fmin(a.v, b.v)); }
inline bool isfinite(fd a) { return std::isfinite(a.v); }
inline bool isnan(fd a) { return std::isnan(a.v); }
#define double fd
