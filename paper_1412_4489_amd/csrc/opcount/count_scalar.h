// count_scalar.h -- scalar types that count the floating-point operations
// applied to them, for the algorithmic operation count of the device
// arithmetic (opcount.cpp).  D stands in for double, F for the compute type
// float; every +, -, *, / counts one operation of its type, fma two, and
// sqrt / exp / erfc one transcendental.  Comparisons, negation, fabs,
// fmin / fmax and conversions are not counted.
#pragma once

#include <cmath>
#include <cstdint>

namespace gks_opcount {

struct Counts {
  int64_t d = 0, f = 0, dtrans = 0;
};
inline Counts& counts() {
  static Counts c;
  return c;
}

template <typename R, int kKind>  // kind 0: double, 1: float
struct Num {
  R v;
  constexpr Num() : v(0) {}
  constexpr Num(double x) : v((R)x) {}
  constexpr Num(float x) : v((R)x) {}
  constexpr Num(int x) : v((R)x) {}
  constexpr Num(long x) : v((R)x) {}
  constexpr Num(unsigned x) : v((R)x) {}
  template <typename R2, int k2>
  constexpr explicit Num(const Num<R2, k2>& o) : v((R)o.v) {}
  explicit operator double() const { return (double)v; }
  explicit operator float() const { return (float)v; }
  explicit operator int() const { return (int)v; }
  static void tick(int n = 1) { (kKind == 0 ? counts().d : counts().f) += n; }
  Num operator-() const { return Num(-v); }
  Num& operator+=(const Num& o) { tick(); v += o.v; return *this; }
  Num& operator-=(const Num& o) { tick(); v -= o.v; return *this; }
  Num& operator*=(const Num& o) { tick(); v *= o.v; return *this; }
  Num& operator/=(const Num& o) { tick(); v /= o.v; return *this; }
  friend Num operator+(Num a, const Num& b) { tick(); a.v += b.v; return a; }
  friend Num operator-(Num a, const Num& b) { tick(); a.v -= b.v; return a; }
  friend Num operator*(Num a, const Num& b) { tick(); a.v *= b.v; return a; }
  friend Num operator/(Num a, const Num& b) { tick(); a.v /= b.v; return a; }
  friend bool operator<(const Num& a, const Num& b) { return a.v < b.v; }
  friend bool operator>(const Num& a, const Num& b) { return a.v > b.v; }
  friend bool operator<=(const Num& a, const Num& b) { return a.v <= b.v; }
  friend bool operator>=(const Num& a, const Num& b) { return a.v >= b.v; }
  friend bool operator==(const Num& a, const Num& b) { return a.v == b.v; }
  friend bool operator!=(const Num& a, const Num& b) { return a.v != b.v; }
};

using D = Num<double, 0>;
using F = Num<float, 1>;

// mixed operands (a literal or an int with a counted value)
#define GKS_OPC_MIX(T)                                                      \
  inline T operator+(double a, const T& b) { return T(a) + b; }             \
  inline T operator-(double a, const T& b) { return T(a) - b; }             \
  inline T operator*(double a, const T& b) { return T(a) * b; }             \
  inline T operator/(double a, const T& b) { return T(a) / b; }             \
  inline T operator+(const T& a, double b) { return a + T(b); }             \
  inline T operator-(const T& a, double b) { return a - T(b); }             \
  inline T operator*(const T& a, double b) { return a * T(b); }             \
  inline T operator/(const T& a, double b) { return a / T(b); }             \
  inline T operator*(int a, const T& b) { return T(a) * b; }                \
  inline T operator*(const T& a, int b) { return a * T(b); }                \
  inline bool operator<(const T& a, double b) { return a.v < b; }           \
  inline bool operator>(const T& a, double b) { return a.v > b; }           \
  inline bool operator<=(const T& a, double b) { return a.v <= b; }         \
  inline bool operator>=(const T& a, double b) { return a.v >= b; }         \
  inline bool operator<(double a, const T& b) { return a < b.v; }           \
  inline bool operator>(double a, const T& b) { return a > b.v; }           \
  inline T fabs(const T& a) { return T(std::fabs(a.v)); }                   \
  inline T fmin(const T& a, const T& b) { return T(std::fmin(a.v, b.v)); }  \
  inline T fmax(const T& a, const T& b) { return T(std::fmax(a.v, b.v)); }  \
  inline T fma(const T& a, const T& b, const T& c) {                        \
    T::tick(2);                                                             \
    return T(std::fma(a.v, b.v, c.v));                                      \
  }                                                                         \
  inline bool isfinite(const T& a) { return std::isfinite(a.v); }
GKS_OPC_MIX(D)
GKS_OPC_MIX(F)
#undef GKS_OPC_MIX

inline D sqrt(const D& a) { ++counts().dtrans; return D(std::sqrt(a.v)); }
inline D exp(const D& a) { ++counts().dtrans; return D(std::exp(a.v)); }
inline D erfc(const D& a) { ++counts().dtrans; return D(std::erfc(a.v)); }

}  // namespace gks_opcount
