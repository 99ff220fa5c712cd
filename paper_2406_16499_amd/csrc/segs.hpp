// Mixed-precision vector glue of the classical correction solves: several
// independent segments, each dst[i] = c (a src[s1(i)] + b src2[s2(i)]) with
// s(i) = n - 1 - i when that source is reversed, in one launch.  Sources and
// destination are FP32 or FP64 (element size 4 or 8); the expression is
// evaluated in FP64 and rounded once to the destination, as the one-step
// conversions and axpys it replaces do.  A null source contributes 0 (both
// null: a zero fill); the src2 term applies for s2(i) >= lo.  A segment may
// update its own destination in place only without reversal.
#pragma once
#include <initializer_list>

#include "engine.hpp"

namespace lsq {

struct VecSegT {
  void* dst;
  const void* src;
  const void* src2;
  int n, rev, rev2, lo;
  double a, b, c;
  int td, ts, ts2;   // element sizes
};
constexpr int kVecSegsT = 6;
struct VecSegsT {
  VecSegT s[kVecSegsT];
  int count;
};
void vec_segs_t(Ctx& ctx, std::initializer_list<VecSegT> segs);

// dst (td) = src (ts), reversed if rev, times c
inline VecSegT tcopy(void* dst, int td, const void* src, int ts, int n, bool rev = false, double c = 1.0) {
  return VecSegT{dst, src, nullptr, n, rev ? 1 : 0, 0, 0, 1.0, 0.0, c, td, ts, 4};
}
inline VecSegT tzero(void* dst, int td, int n) {
  return VecSegT{dst, nullptr, nullptr, n, 0, 0, 0, 0.0, 0.0, 1.0, td, 4, 4};
}
// dst = src + b src2 (each reversed or not)
inline VecSegT tadd(void* dst, int td, const void* src, int ts, bool rev, const void* src2, int ts2, bool rev2,
                    int n, double b) {
  return VecSegT{dst, src, src2, n, rev ? 1 : 0, rev2 ? 1 : 0, 0, 1.0, b, 1.0, td, ts, ts2};
}
// y += b x (y in place; x reversed if rev)
inline VecSegT taxpy(void* y, int ty, double b, const void* x, int tx, int n, bool rev = false) {
  return VecSegT{y, y, x, n, 0, rev ? 1 : 0, 0, 1.0, b, 1.0, ty, ty, tx};
}

}  // namespace lsq
