// ks_step.hip -- launchers of the rotate-and-accumulate steps (key switching)
// and of the mask for one ring dimension.  Compiled once per log2 n with
// -DLRHE_KS_LOGN=<10..15>, so the many instantiations of the transform kernels
// build in parallel.
#include "kernels_dev.h"

#ifndef LRHE_KS_LOGN
#error "compile once per ring dimension with -DLRHE_KS_LOGN=<log2 n>"
#endif

namespace lrhe {

// residues-per-thread choices available at ring dimension 2^LN (at most 1024
// threads per workgroup; 16 residues up to n = 16384, 64 from n = 4096)
template <int LN, int LE>
constexpr bool le_ok = LN - LE <= 10 && !(LE == 4 && LN > 14) && !(LE == 6 && LN < 12);

#define LRHE_LE_SWITCH(LEVAR, ...)                                         \
  switch (LEVAR) {                                                         \
    case 4: { constexpr int LE = 4; if constexpr (le_ok<LN, 4>) { __VA_ARGS__; } else { return hipErrorInvalidValue; } } break; \
    case 5: { constexpr int LE = 5; if constexpr (le_ok<LN, 5>) { __VA_ARGS__; } else { return hipErrorInvalidValue; } } break; \
    case 6: { constexpr int LE = 6; if constexpr (le_ok<LN, 6>) { __VA_ARGS__; } else { return hipErrorInvalidValue; } } break; \
    default: return hipErrorInvalidValue;                                  \
  }

// k_ks_mac variants selectable through the "mac_mode" tuning key (index -> MODE bits)
#ifndef LRHE_MAC_MODES
#define LRHE_MAC_MODE_CASE(IDX, LN, LE, MODE) \
  case IDX: k_ks_mac<LN, LE, MODE><<<grid, Geom<LN, LE>::T, 0, s>>>(c->dc, cur, D, tp, gk_d, gi, g, ACC, ACC2, nxt); break;
#define LRHE_MAC_MODES(LN, LE)                                                           \
  LRHE_MAC_MODE_CASE(0, LN, LE, 104) /* one buffer, 2 workgroups/CU, pair per XCD, rotated */ \
  LRHE_MAC_MODE_CASE(1, LN, LE, 108) /* as 0, with twiddle prefetch */                       \
  LRHE_MAC_MODE_CASE(2, LN, LE, 225) /* double buffer, pair per XCD, rotated, 64-bit MAC */   \
  LRHE_MAC_MODE_CASE(3, LN, LE, 3)   /* double buffer, digit prefetch */                           \
  LRHE_MAC_MODE_CASE(4, LN, LE, 385) /* double buffer, 64-bit MAC, two workgroups per item (digit halves) */ \
  LRHE_MAC_MODE_CASE(5, LN, LE, 524) /* one buffer, 2 workgroups/CU, twiddle prefetch, moduli by XCD */
/* mac_modes 6 and 7 (LRHE_MAC_MODE_SPLIT, LRHE_MAC_MODE_SPLIT64) are launched on their own
   below: MODE 5132 = the special-prime items with the digits, then the data-modulus items with
   part 3: MODE 2060 (one buffer, 2 workgroups/CU) or 2181 (double buffer, unreduced 64-bit
   inner products) */
#endif

template <int LN>
hipError_t launch_ks_step(const lrhe_ctx* c, const Knobs& kn, const PairDesc* tp, const uint32_t* gk_d, uint32_t Bt,
                          uint32_t gi, const uint32_t* cur, uint32_t* D, uint32_t* ACC, uint64_t acc_slots,
                          uint32_t* nxt, bool d_ready, bool d_next, hipStream_t s) {
  const uint32_t L = c->L, g = c->gal[gi];
  // the digit-halves variant keeps a second accumulator per item, ACC2, in the
  // slots after the tile's own
  const bool half = kn.mac_mode == LRHE_MAC_MODE_HALF;
  uint32_t* ACC2 = nullptr;
  if (half) {
    if (2ull * Bt > acc_slots) return hipErrorInvalidValue;
    ACC2 = ACC + (uint64_t)Bt * (L + 1) * 2 * c->n;
  }
  // the digits of this step: from k_ks_intt, or already written by the
  // previous step's k_ks_moddown (d_ready), or (split variant) made by its
  // special-prime launch
  const bool split = kn.mac_mode == LRHE_MAC_MODE_SPLIT || kn.mac_mode == LRHE_MAC_MODE_SPLIT64;
  if (!d_ready && !split) {
    ProfScope ps(s, "k_ks_intt");
    LRHE_LE_SWITCH(kn.le_intt, {
      k_ks_intt<LN, LE><<<(unsigned)(Bt * L), Geom<LN, LE>::T, 0, s>>>(c->dc, cur, g, D);
    });
  }
  if (split) {
    // the special-prime items, which also make the step's digits (D) and rho
    // (ACC), then the L data-modulus items, each ending with the rounded
    // division by P and the rotate-and-accumulate of its limb
    if (d_next || d_ready) return hipErrorInvalidValue;
    {
      ProfScope ps(s, "k_ks_mac_p");
      LRHE_LE_SWITCH(kn.le_mac_p, {
        k_ks_mac<LN, LE, 5132><<<(unsigned)Bt, Geom<LN, LE>::T, 0, s>>>(c->dc, cur, D, tp, gk_d, gi, g, ACC, nullptr,
                                                                       nxt);
      });
    }
    ProfScope ps(s, "k_ks_mac_md");
    LRHE_LE_SWITCH(kn.le_mac, {
      if (kn.mac_mode == LRHE_MAC_MODE_SPLIT64)
        k_ks_mac<LN, LE, 2181><<<(unsigned)(Bt * L), Geom<LN, LE>::T, 0, s>>>(c->dc, cur, D, tp, gk_d, gi, g, ACC,
                                                                             nullptr, nxt);
      else
        k_ks_mac<LN, LE, 2060><<<(unsigned)(Bt * L), Geom<LN, LE>::T, 0, s>>>(c->dc, cur, D, tp, gk_d, gi, g, ACC,
                                                                             nullptr, nxt);
    });
    return hipGetLastError();
  }
  {
    ProfScope ps(s, "k_ks_mac");
    LRHE_LE_SWITCH(kn.le_mac, {
      const unsigned grid = (unsigned)(Bt * (L + 1) * (half ? 2 : 1));
      switch (kn.mac_mode) {
        LRHE_MAC_MODES(LN, LE)
        default: return hipErrorInvalidValue;
      }
    });
  }
  if (half) {
    {
      ProfScope ps(s, "k_ks_rho");
      LRHE_LE_SWITCH(kn.le_moddown, {
        k_ks_rho<LN, LE><<<(unsigned)(Bt * 2), Geom<LN, LE>::T, 0, s>>>(c->dc, ACC, ACC2);
      });
    }
    ProfScope ps(s, "k_ks_moddown");
    LRHE_LE_SWITCH(kn.le_moddown, {
      k_ks_moddown_part<LN, LE><<<(unsigned)(Bt * L * 2), Geom<LN, LE>::T, 0, s>>>(c->dc, cur, ACC, ACC2, g, nxt);
    });
  } else {
    // d_next: the digits of step gi + 1 come out of this k_ks_moddown
    if (d_next && gi + 1 >= c->ngal) return hipErrorInvalidValue;
    const uint32_t gn = d_next ? c->gal[gi + 1] : 0;
    ProfScope ps(s, "k_ks_moddown");
    LRHE_LE_SWITCH(kn.le_moddown, {
      k_ks_moddown<LN, LE><<<(unsigned)(Bt * L), Geom<LN, LE>::T, 0, s>>>(c->dc, cur, ACC, g, nxt, gn, D);
    });
  }
  return hipGetLastError();
}

template <int LN>
hipError_t launch_mask_step(const lrhe_ctx* c, const Knobs& kn, const uint32_t* cur, const PairDesc* tp,
                            const GroupDesc* tg, uint32_t ngt, int mode, uint32_t* dst, hipStream_t s) {
  const uint32_t L = c->L;
  LRHE_LE_SWITCH(kn.le_mask, {
    k_mask<LN, LE><<<(unsigned)(ngt * L), Geom<LN, LE>::T, 0, s>>>(c->dc, cur, tp, tg, mode, dst);
  });
  return hipGetLastError();
}

template hipError_t launch_ks_step<LRHE_KS_LOGN>(const lrhe_ctx*, const Knobs&, const PairDesc*, const uint32_t*,
                                                 uint32_t, uint32_t, const uint32_t*, uint32_t*, uint32_t*, uint64_t,
                                                 uint32_t*, bool, bool, hipStream_t);
template hipError_t launch_mask_step<LRHE_KS_LOGN>(const lrhe_ctx*, const Knobs&, const uint32_t*, const PairDesc*,
                                                   const GroupDesc*, uint32_t, int, uint32_t*, hipStream_t);

}  // namespace lrhe
