// lrhe_math.h -- modular arithmetic and negacyclic NTT pass structure shared by
// the gfx950 kernels and the host runtime (keygen, decryption) of the encrypted
// logistic-regression library.  Everything here is __host__ __device__ so the
// host executes the very same index and twiddle arithmetic as the kernels.
//
// Residues are uint32 modulo primes q < 2^30 (4q < 2^32 leaves room for lazy
// reduction).  Products use Montgomery reduction with R = 2^32: for x < q 2^32,
// redc(x) = x R^-1 mod q in [0, 2q).  Operands that are fixed per model or per
// key (twiddles, keys, public key, weights, masks) are stored premultiplied by
// R so that redc(a * bR) = a b mod q with one 64-bit multiply-add pair.
//
// Transform: negacyclic NTT over Z_q[X]/(X^n + 1).  The forward transform maps
// natural-order coefficients to evaluations at psi^(2 brv(k) + 1) stored at
// index k (bit-reversed order); it is the merged-twist Cooley-Tukey form whose
// stage with m blocks uses psi^brv(m + i) for block i.  The inverse is the
// matching Gentleman-Sande form with psi^-brv(m + i) and a final n^-1.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define LRHE_HD __host__ __device__ __forceinline__
#else
#define LRHE_HD inline
#endif

// Scheduling fence between butterfly stages in device code: one stage holds
// E/2 independent butterflies, enough ILP, and the fence stops the scheduler
// from hoisting later stages' twiddle loads (which costs registers).
#if defined(__HIP_DEVICE_COMPILE__)
#define LRHE_STAGE_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define LRHE_STAGE_FENCE() ((void)0)
#endif

namespace lrhe {

struct Mod {
  uint32_t q;       // prime modulus, q < 2^30
  uint32_t qinv;    // -q^-1 mod 2^32
  uint32_t r2;      // R^2 mod q (to enter Montgomery form)
  uint32_t ninv_m;  // n^-1 R mod q
};

LRHE_HD uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// x < q 2^32 (or any x with x + (2^32-1) q < 2^64): returns x R^-1 mod q, in [0, 2q)
// when x < q 2^32, and in [0, x/2^32 + q) otherwise.
LRHE_HD uint32_t redc(uint64_t x, uint32_t q, uint32_t qinv) {
  const uint32_t m = (uint32_t)x * qinv;
  uint64_t y = x + (uint64_t)m * q;
  return (uint32_t)(y >> 32);
}
// a < 2^32, bm = b R mod q: returns a b mod q in [0, 2q)
LRHE_HD uint32_t mulm(uint32_t a, uint32_t bm, uint32_t q, uint32_t qinv) { return redc((uint64_t)a * bm, q, qinv); }
// [0, 2q) -> [0, q)
LRHE_HD uint32_t red1(uint32_t a, uint32_t q) { return umin(a, a - q); }
// [0, 4q) -> [0, q)
LRHE_HD uint32_t red2(uint32_t a, uint32_t q) { return red1(umin(a, a - 2 * q), q); }
LRHE_HD uint32_t addm(uint32_t a, uint32_t b, uint32_t q) { return red1(a + b, q); }   // a, b < q
LRHE_HD uint32_t subm(uint32_t a, uint32_t b, uint32_t q) { return red1(a + q - b, q); }
// to Montgomery form: a R mod q, a < 2^32
LRHE_HD uint32_t to_mont(uint32_t a, const Mod& m) { return red1(mulm(a, m.r2, m.q, m.qinv), m.q); }

LRHE_HD uint32_t brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// ---------------------------------------------------------------------------
// NTT geometry: n = 2^LOGN coefficients spread over T = n / 2^LOGE threads,
// E = 2^LOGE per thread.  The LOGN stages are cut into passes of LOGE stages
// (the last pass may be shorter).  In pass p (stages s0 .. s0 + r - 1) the
// array splits into independent sub-problems of 2^r elements with stride
// n >> (s0 + r); thread t owns the sub-problems sp(p, t, u), u < E >> r:
// sp = u T + t, except in the last pass of a multi-wave transform of three or
// more passes when WL is set (WLAST).  There the lane (t mod 64) takes the low
// bits of sp, u the next ones and the wave (t / 64) the top ones, so each wave
// owns one contiguous block of 64 E residues, the same block it owns in the
// pass before: that boundary is crossed without a workgroup barrier.  The
// numbering only changes which thread holds which residue in registers; global
// data keeps its natural order, so kernels may choose WL independently.
// ---------------------------------------------------------------------------
template <int LOGN_, int LOGE_, bool WL = true>
struct Geom {
  static constexpr int LOGN = LOGN_, LOGE = LOGE_;
  static constexpr int N = 1 << LOGN, E = 1 << LOGE, T = N >> LOGE;
  static constexpr int NPASS = (LOGN + LOGE - 1) / LOGE;
  static constexpr int LOGT = LOGN - LOGE;
  static constexpr bool WLAST = WL && NPASS >= 3 && LOGT > 6;
  static constexpr int LOGNU_LAST = LOGE - (LOGN - (NPASS - 1) * LOGE);   // log2 (E >> r) in the last pass
  // padded exchange buffer: one pad word per 2^PADSH words keeps every wave's
  // exchange accesses free of LDS bank conflicts (64 banks, 32 lanes per cycle)
  static constexpr int PADSH = LOGE == 4 ? 3 : LOGE;
  static constexpr int LDS_WORDS = N + (N >> PADSH);
  LRHE_HD static constexpr int s0(int p) { return p * LOGE; }
  LRHE_HD static constexpr int r(int p) { return (LOGN - p * LOGE) < LOGE ? (LOGN - p * LOGE) : LOGE; }
  // sub-problem u of thread t in pass p
  LRHE_HD static uint32_t sp(int p, int t, uint32_t u) {
    const uint32_t ut = (uint32_t)t;
    if (WLAST && p == NPASS - 1) return (ut & 63u) | (u << 6) | ((ut >> 6) << (6 + LOGNU_LAST));
    return u * T + ut;
  }
  // global index of element e (= u 2^r + c) of thread t in pass p
  LRHE_HD static uint32_t idx(int p, int t, int e) {
    const int rr = r(p), sh = s0(p);
    const uint32_t c = (uint32_t)e & ((1u << rr) - 1), u = (uint32_t)e >> rr;
    const uint32_t sp = Geom::sp(p, t, u);
    const int lstride = LOGN - sh - rr;   // log2 of the stride
    const uint32_t h = sp >> lstride, l = sp & ((1u << lstride) - 1);
    return (h << (LOGN - sh)) + (c << lstride) + l;
  }
  // padded position in the exchange buffer
  LRHE_HD static uint32_t pad(uint32_t j) { return j + (j >> PADSH); }
  // idx(p, t, e) = tbase(p, t) + eoff(p, e), the two parts on disjoint bits
  // (h field, stride field, low field; T is a multiple of the stride), so also
  // pad(idx) = pad(tbase) + padoff(eoff): one per-thread base and a
  // compile-time offset per element.
  // (the last pass has stride 1: index = sp 2^r + c; under WLAST its lane and
  // wave fields are per thread, u and c per element)
  LRHE_HD static uint32_t tbase(int p, int t) {
    const int ls = LOGN - s0(p) - r(p);
    const uint32_t ut = (uint32_t)t;
    if (WLAST && p == NPASS - 1) return ((ut & 63u) | ((ut >> 6) << (6 + LOGNU_LAST))) << r(p);
    return ((ut >> ls) << (LOGN - s0(p))) + (ut & ((1u << ls) - 1));
  }
  LRHE_HD static constexpr uint32_t eoff(int p, int e) {
    if (WLAST && p == NPASS - 1) return (((uint32_t)(e >> r(p)) << 6) << r(p)) + ((uint32_t)e & ((1u << r(p)) - 1));
    return ((((uint32_t)(e >> r(p)) * (uint32_t)T) >> (LOGN - s0(p) - r(p))) << (LOGN - s0(p))) +
           (((uint32_t)e & ((1u << r(p)) - 1)) << (LOGN - s0(p) - r(p)));
  }
  LRHE_HD static constexpr uint32_t padoff(uint32_t o) { return o + (o >> PADSH); }
};

// Twiddle access: on the host a plain pointer; in the kernels a view with a
// per-lane path and a wave-uniform (scalar-load) path.  In the pass that
// starts at stage 0 the block index h equals u, so its twiddles are uniform.
LRHE_HD uint32_t tw_get(const uint32_t* tw, uint32_t i, bool) { return tw[i]; }
// b w_i mod q in [0, 2q) for a twiddle table of Montgomery words w_i R
LRHE_HD uint32_t tw_mul(const uint32_t* tw, uint32_t i, bool, uint32_t b, uint32_t q, uint32_t qinv) {
  return mulm(b, tw[i], q, qinv);
}

// Twiddles of one (unit u, stage tau) step of a pass: the 2^tau distinct values
// w[j] = tw[2^(s0 + tau) + h 2^tau + j], h the unit's block index.
template <class G, class TW>
LRHE_HD void stage_tw(int p, int t, int u, int tau, const TW& tw, uint32_t* w) {
  const int rr = G::r(p), sh = G::s0(p);
  const int lstride = G::LOGN - sh - rr;
  const int h = sh == 0 ? u : (int)(G::sp(p, t, (uint32_t)u) >> lstride);
  // a fixed trip count, so the loop unrolls before tau is known; the guards
  // fold once the callers' stage loops are unrolled
#pragma unroll
  for (int j = 0; j < (G::E > 1 ? G::E / 2 : 1); ++j)
    if (j < (1 << tau)) w[j] = tw_get(tw, (uint32_t)((1 << (sh + tau)) + (h << tau) + j), sh == 0);
}

// One pass of the forward (Cooley-Tukey) transform on the E registers of
// thread t.  x holds the elements of pass p in Geom::idx order, values in
// [0, 4q); output in [0, 4q).  tw: psi^brv(k) R mod q, k < n.  Each (unit,
// stage) step reads its twiddles as its butterflies need them; with PF the
// 2^tau twiddles of the next step are loaded while the current step computes.
// STRICT keeps every value canonical in [0, q) instead (input and output), for
// moduli from 2^30 up to 2^31 where 4q no longer fits in 32 bits.
template <class G, bool PF = false, bool STRICT = false, class TW>
LRHE_HD void fwd_pass(int p, int t, uint32_t* x, const TW& tw, uint32_t q, uint32_t qinv) {
  const int rr = G::r(p);
  const int nu = G::E >> rr;
  const uint32_t q2 = 2 * q;
  uint32_t wc[PF ? G::E / 2 : 1], wn[PF ? G::E / 2 : 1];
  if constexpr (PF) stage_tw<G>(p, t, 0, 0, tw, wc);
#pragma unroll
  for (int u = 0; u < nu; ++u) {
#pragma unroll
    for (int tau = 0; tau < rr; ++tau) {
      const bool more = tau + 1 < rr || u + 1 < nu;
      if constexpr (PF) {
        if (more) stage_tw<G>(p, t, tau + 1 < rr ? u : u + 1, tau + 1 < rr ? tau + 1 : 0, tw, wn);
      }
      const int half = 1 << (rr - 1 - tau);
      const int h = G::s0(p) == 0 ? u : (int)(G::sp(p, t, (uint32_t)u) >> (G::LOGN - G::s0(p) - rr));
#pragma unroll
      for (int c = 0; c < (1 << rr); ++c) {
        if (c & half) continue;
        uint32_t* a = &x[(u << rr) + c];
        uint32_t* b = &x[(u << rr) + c + half];
        const uint32_t Tm =
            PF ? mulm(*b, wc[c >> (rr - tau)], q, qinv)
               : tw_mul(tw, (uint32_t)((1 << (G::s0(p) + tau)) + (h << tau) + (c >> (rr - tau))), G::s0(p) == 0, *b,
                        q, qinv);
        if constexpr (STRICT) {
          const uint32_t X = *a, Tc = red1(Tm, q);
          *a = addm(X, Tc, q);
          *b = subm(X, Tc, q);
        } else {
          const uint32_t X = umin(*a, *a - q2);
          *a = X + Tm;
          *b = X + q2 - Tm;
        }
      }
      LRHE_STAGE_FENCE();
      if constexpr (PF) {
        if (more) {
#pragma unroll
          for (int j = 0; j < G::E / 2; ++j) wc[j] = wn[j];
        }
      }
    }
  }
}

// One pass of the inverse (Gentleman-Sande) transform; passes run in the order
// NPASS-1 .. 0 and stages inside a pass from the last to the first.  Values in
// and out in [0, 2q).  itw: psi^-brv(k) R mod q.  PF and STRICT as in fwd_pass.
// SCALE (pass 0 only): the final stage also multiplies by n^-1 (ninv_m = n^-1 R
// mod q): its one twiddle w becomes w n^-1, and the sums are scaled, which
// saves the n^-1 product of the other half of the residues.
template <class G, bool PF = false, bool STRICT = false, class TW, bool SCALE = false>
LRHE_HD void inv_pass(int p, int t, uint32_t* x, const TW& itw, uint32_t q, uint32_t qinv, uint32_t ninv_m = 0) {
  const int rr = G::r(p);
  const int nu = G::E >> rr;
  const uint32_t q2 = 2 * q;
  uint32_t wc[PF ? G::E / 2 : 1], wn[PF ? G::E / 2 : 1];
  if constexpr (PF) stage_tw<G>(p, t, 0, rr - 1, itw, wc);
#pragma unroll
  for (int u = 0; u < nu; ++u) {
#pragma unroll
    for (int tau = rr - 1; tau >= 0; --tau) {
      const bool more = tau > 0 || u + 1 < nu;
      if constexpr (PF) {
        if (more) stage_tw<G>(p, t, tau > 0 ? u : u + 1, tau > 0 ? tau - 1 : rr - 1, itw, wn);
      }
      const int half = 1 << (rr - 1 - tau);
      const int h = G::s0(p) == 0 ? u : (int)(G::sp(p, t, (uint32_t)u) >> (G::LOGN - G::s0(p) - rr));
#pragma unroll
      for (int c = 0; c < (1 << rr); ++c) {
        if (c & half) continue;
        uint32_t* a = &x[(u << rr) + c];
        uint32_t* b = &x[(u << rr) + c + half];
        uint32_t U, V;
        if constexpr (STRICT) {
          U = addm(*a, *b, q);
          V = subm(*a, *b, q);
        } else {
          U = *a + *b;
          U = umin(U, U - q2);
          V = *a + q2 - *b;
        }
        if (SCALE && tau == 0) {
          // the transform's last stage (block index 0, twiddle index 1):
          // U n^-1 and V w n^-1, w n^-1 canonical so that the products of V < 4q
          // stay below 2q
          const uint32_t w = PF ? wc[c >> (rr - tau)] : tw_get(itw, 1u, true);
          const uint32_t wn = red1(mulm(w, ninv_m, q, qinv), q);
          *a = mulm(U, ninv_m, q, qinv);
          *b = mulm(V, wn, q, qinv);
        } else {
          *a = U;
          *b = PF ? mulm(V, wc[c >> (rr - tau)], q, qinv)
                  : tw_mul(itw, (uint32_t)((1 << (G::s0(p) + tau)) + (h << tau) + (c >> (rr - tau))), G::s0(p) == 0,
                           V, q, qinv);
        }
        if constexpr (STRICT) *b = red1(*b, q);
      }
      LRHE_STAGE_FENCE();
      if constexpr (PF) {
        if (more) {
#pragma unroll
          for (int j = 0; j < G::E / 2; ++j) wc[j] = wn[j];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// ChaCha20 block function (RFC 8439, section 2.3).  Stream convention of the
// library: key = (seed low, seed high, 0, 0, 0, 0, 0, 0), nonce = (kind,
// id low, id high), block counter = word index / 16.
// ---------------------------------------------------------------------------
#define LRHE_ROTL(v, c) (((v) << (c)) | ((v) >> (32 - (c))))
#define LRHE_QR(a, b, c, d)                      \
  a += b; d ^= a; d = LRHE_ROTL(d, 16);          \
  c += d; b ^= c; b = LRHE_ROTL(b, 12);          \
  a += b; d ^= a; d = LRHE_ROTL(d, 8);           \
  c += d; b ^= c; b = LRHE_ROTL(b, 7);

LRHE_HD void chacha20(uint64_t seed, uint32_t kind, uint64_t id, uint32_t counter, uint32_t out[16]) {
  const uint32_t s0 = 0x61707865u, s1 = 0x3320646eu, s2 = 0x79622d32u, s3 = 0x6b206574u;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint32_t n0 = kind, n1 = (uint32_t)id, n2 = (uint32_t)(id >> 32);
  uint32_t x0 = s0, x1 = s1, x2 = s2, x3 = s3, x4 = k0, x5 = k1, x6 = 0, x7 = 0;
  uint32_t x8 = 0, x9 = 0, x10 = 0, x11 = 0, x12 = counter, x13 = n0, x14 = n1, x15 = n2;
  for (int i = 0; i < 10; ++i) {
    LRHE_QR(x0, x4, x8, x12) LRHE_QR(x1, x5, x9, x13) LRHE_QR(x2, x6, x10, x14) LRHE_QR(x3, x7, x11, x15)
    LRHE_QR(x0, x5, x10, x15) LRHE_QR(x1, x6, x11, x12) LRHE_QR(x2, x7, x8, x13) LRHE_QR(x3, x4, x9, x14)
  }
  out[0] = x0 + s0; out[1] = x1 + s1; out[2] = x2 + s2; out[3] = x3 + s3;
  out[4] = x4 + k0; out[5] = x5 + k1; out[6] = x6; out[7] = x7;
  out[8] = x8; out[9] = x9; out[10] = x10; out[11] = x11;
  out[12] = x12 + counter; out[13] = x13 + n0; out[14] = x14 + n1; out[15] = x15 + n2;
}

// random-stream kinds (one per sampled polynomial family)
enum StreamKind : uint32_t {
  KIND_SECRET = 1, KIND_PK_A = 2, KIND_PK_E = 3, KIND_GK_A = 4, KIND_GK_E = 5,
  KIND_ENC_U = 6, KIND_ENC_E0 = 7, KIND_ENC_E1 = 8
};

// ternary from one stream word: w mod 3 -> {0, +1, -1}
LRHE_HD int ternary_of(uint32_t w) {
  uint32_t r = w % 3u;
  return r == 0 ? 0 : (r == 1 ? 1 : -1);
}
// centred binomial (eta = 21) from two words: popcount(bits 0..20) - popcount(bits 21..41)
LRHE_HD int popc32(uint32_t v) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __popc(v);
#else
  return __builtin_popcount(v);
#endif
}
LRHE_HD int cbd21_of(uint32_t lo, uint32_t hi) {
  const uint32_t a = lo & 0x1FFFFFu;
  const uint32_t b = ((lo >> 21) | (hi << 11)) & 0x1FFFFFu;
  return popc32(a) - popc32(b);
}
// uniform mod m from two words: ((hi << 32) | lo) mod m
LRHE_HD uint32_t uniform_of(uint32_t lo, uint32_t hi, uint32_t m) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) % m);
}

}  // namespace lrhe
