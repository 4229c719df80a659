// Counting scalar for the algorithmic FLOP count of one solver iteration.
//
// The device math is instantiated on the host with this type.  An operation
// counts only when none of its operands is an exact zero: products with the
// structural zeros of the code (no curvature on planes, padded rows of a
// diffraction, accumulators starting at zero) are not work the method needs.
#pragma once
#include <math.h>
#include <stdint.h>

namespace mpt {

struct FlopTally {
    int64_t add = 0, mul = 0, div = 0, sqrt = 0;
    int64_t flops() const { return add + mul + div + sqrt; }
};

inline FlopTally &tally()
{
    static thread_local FlopTally t;
    return t;
}

struct Cnt {
    double v;
    Cnt() : v(0) {}
    Cnt(double x) : v(x) {}
};

inline bool nz(const Cnt &a) { return a.v != 0.0; }
inline Cnt operator+(Cnt a, Cnt b) { if (nz(a) && nz(b)) tally().add++; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { if (nz(a) && nz(b)) tally().add++; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { if (nz(a) && nz(b)) tally().mul++; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { if (nz(a)) tally().div++; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt &operator+=(Cnt &a, Cnt b) { a = a + b; return a; }
inline Cnt &operator-=(Cnt &a, Cnt b) { a = a - b; return a; }
inline Cnt &operator*=(Cnt &a, Cnt b) { a = a * b; return a; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>=(Cnt a, Cnt b) { return a.v >= b.v; }
inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
inline Cnt fmax(Cnt a, Cnt b) { return Cnt(a.v > b.v ? a.v : b.v); }
inline Cnt fabs(Cnt a) { return Cnt(a.v < 0 ? -a.v : a.v); }
inline Cnt dsqrt(Cnt a) { if (nz(a)) tally().sqrt++; return Cnt(::sqrt(a.v)); }
// 1/x and 1/sqrt(x) count as what they are algorithmically: a division and a
// square root plus a division
inline Cnt drcp(Cnt a) { if (nz(a)) tally().div++; return Cnt(1.0 / a.v); }
inline Cnt drsqrt(Cnt a) { if (nz(a)) tally().sqrt++, tally().div++; return Cnt(1.0 / ::sqrt(a.v)); }
// the sine and cosine of the circle's parametrisation count as one
// operation each (counted with the square roots and divisions)
inline Cnt sin(Cnt a) { tally().sqrt++; return Cnt(::sin(a.v)); }
inline Cnt cos(Cnt a) { tally().sqrt++; return Cnt(::cos(a.v)); }

}  // namespace mpt
