// Exhaustive host check of the transform geometry used by the kernels: for every
// supported (log2 n, residues per thread), pass, thread and element,
//  - the global index splits into a per-thread base and a per-element offset on
//    disjoint bits, and the padded exchange position splits the same way;
//  - each pass maps (thread, element) one to one onto the n indices;
//  - the butterfly block index taken from the sub-problem number (twiddle
//    lookup) is the index's block;
//  - with the wave-local last boundary (WLAST), every wave owns the same
//    contiguous block of 64 E indices in the last two passes, so crossing
//    that boundary never reads another wave's writes.
// Exit status 0 = all hold.
#include <cstdio>
#include <vector>

#include "lrhe_math.h"

using namespace lrhe;

template <int LN, int LE, bool WL>
static int check1() {
  using G = Geom<LN, LE, WL>;
  int bad = 0;
  for (int p = 0; p < G::NPASS; ++p) {
    std::vector<int> hit(G::N, 0);
    const int rr = G::r(p), ls = LN - G::s0(p) - rr;
    for (int t = 0; t < G::T; ++t)
      for (int e = 0; e < G::E; ++e) {
        const uint32_t i = G::idx(p, t, e), b = G::tbase(p, t), o = G::eoff(p, e);
        if (i != b + o || (b & o) != 0 || G::pad(i) != G::pad(b) + G::padoff(o)) ++bad;
        if (i < (uint32_t)G::N) ++hit[i];
        else ++bad;
        const uint32_t u = (uint32_t)e >> rr;
        if ((G::sp(p, t, u) >> ls) != (i >> (LN - G::s0(p)))) ++bad;
      }
    for (int v : hit)
      if (v != 1) ++bad;
  }
  if (G::WLAST) {
    const int P1 = G::NPASS - 2, P2 = G::NPASS - 1;
    const uint32_t blk = 64u * G::E;
    for (int t = 0; t < G::T; ++t)
      for (int e = 0; e < G::E; ++e) {
        const uint32_t w = (uint32_t)t / 64;
        if (G::idx(P1, t, e) / blk != w || G::idx(P2, t, e) / blk != w) ++bad;
      }
  }
  if (bad) std::printf("log2 n %d, log2 E %d, wave-local last pass %d: %d mismatches\n", LN, LE, (int)WL, bad);
  return bad;
}

// both numberings of the last pass
template <int LN, int LE>
static int check() {
  return check1<LN, LE, true>() + check1<LN, LE, false>();
}

int main() {
  int bad = check<10, 4>() + check<10, 5>() + check<11, 4>() + check<11, 5>() + check<12, 4>() + check<12, 5>() +
            check<12, 6>() + check<13, 4>() + check<13, 5>() + check<13, 6>() + check<14, 4>() + check<14, 5>() +
            check<14, 6>() + check<15, 5>() + check<15, 6>();
  std::printf(bad ? "geometry split: FAILED\n" : "geometry split: ok\n");
  return bad != 0;
}
