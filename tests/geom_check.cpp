// Exhaustive host check of the transform geometry used by the kernels: for every
// supported (log2 n, residues per thread), pass, thread and element, the global
// index splits into a per-thread base and a per-element offset on disjoint bits,
// and the padded exchange position splits the same way.  Exit status 0 = holds.
#include <cstdio>

#include "lrhe_math.h"

using namespace lrhe;

template <int LN, int LE>
static int check() {
  using G = Geom<LN, LE>;
  int bad = 0;
  for (int p = 0; p < G::NPASS; ++p)
    for (int t = 0; t < G::T; ++t)
      for (int e = 0; e < G::E; ++e) {
        const uint32_t i = G::idx(p, t, e), b = G::tbase(p, t), o = G::eoff(p, e);
        if (i != b + o || (b & o) != 0 || G::pad(i) != G::pad(b) + G::padoff(o)) ++bad;
      }
  if (bad) std::printf("log2 n %d, log2 E %d: %d mismatches\n", LN, LE, bad);
  return bad;
}

int main() {
  int bad = check<10, 4>() + check<10, 5>() + check<11, 4>() + check<11, 5>() + check<12, 4>() + check<12, 5>() +
            check<12, 6>() + check<13, 4>() + check<13, 5>() + check<13, 6>() + check<14, 4>() + check<14, 5>() +
            check<14, 6>() + check<15, 5>() + check<15, 6>();
  std::printf(bad ? "geometry split: FAILED\n" : "geometry split: ok\n");
  return bad != 0;
}
