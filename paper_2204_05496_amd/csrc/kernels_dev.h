// kernels_dev.h -- gfx950 kernels of the encrypted logistic-regression path
// (device code; included by kernels.hip and by the per-ring-dimension
// key-switch launchers in ks_step.hip).
//
// Every polynomial transform runs inside one workgroup: T = n / 2^LE threads
// hold 2^LE residues each in VGPRs (LE = 4, 5 or 6; 5 by default), do LE
// butterfly stages per pass in registers and exchange through a padded LDS
// buffer between passes (3 passes at n = 16384, LE = 5).  Elementwise steps
// are fused into the transform kernels' load and store phases so that each
// residue makes one HBM round trip per step.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "lrhe_internal.h"

namespace lrhe {

// geometry of the one-transform-per-workgroup kernels outside the key switch
// (encoding, encryption, model lift): 16 residues per thread up to n = 16384
// (1024 threads), 32 above; the forward transforms measured fastest there
template <int LOGN>
using Gm = Geom<LOGN, (LOGN <= 14 ? 4 : 5)>;

// ------------------------------------------------------------------ helpers
// Read/write view of a device array through a buffer resource held in SGPRs:
// every access is a scalar base plus a 32-bit per-lane offset (no 64-bit
// address per lane), and the hardware returns 0 / drops writes outside
// [0, words).  Word 3 of the resource is the gfx9-family raw-buffer format.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
struct DBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ DBuf(const uint32_t* p, uint32_t words)
      : r(__builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(words * 4u), 0x00020000)) {}
  __device__ __forceinline__ uint32_t operator[](uint32_t i) const {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)(i * 4u), 0, 0);
  }
  __device__ __forceinline__ u32x4 ld4(uint32_t i) const {
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)(i * 4u), 0, 0);
  }
  __device__ __forceinline__ void st(uint32_t i, uint32_t v) const {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)(i * 4u), 0, 0);
  }
  __device__ __forceinline__ void st4(uint32_t i, u32x4 v) const {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)(i * 4u), 0, 0);
  }
  // word vi + si: vi per lane (a VGPR), si wave-uniform (the SGPR offset of the
  // instruction), so per-element constants cost no vector instruction.  The
  // hardware range check covers the per-lane part only: callers keep vi + si
  // inside the buffer.
  __device__ __forceinline__ uint32_t at(uint32_t vi, uint32_t si) const {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)(vi * 4u), (int)(si * 4u), 0);
  }
  __device__ __forceinline__ u32x4 at4(uint32_t vi, uint32_t si) const {
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)(vi * 4u), (int)(si * 4u), 0);
  }
  __device__ __forceinline__ void put(uint32_t vi, uint32_t si, uint32_t v) const {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)(vi * 4u), (int)(si * 4u), 0);
  }
  __device__ __forceinline__ void put4(uint32_t vi, uint32_t si, u32x4 v) const {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)(vi * 4u), (int)(si * 4u), 0);
  }
};

// twiddle table of modulus mi (forward or inverse): per-lane reads through the
// buffer view, wave-uniform reads as scalar loads through the plain pointer
struct TwView {
  DBuf b;
  const uint32_t* p;
  __device__ __forceinline__ TwView(const uint32_t* base, int mi, uint32_t n)
      : b(base + (size_t)mi * n, n), p(base + (size_t)mi * n) {}
};
__device__ __forceinline__ uint32_t tw_get(const TwView& tw, uint32_t i, bool uniform) {
  return uniform ? tw.p[i] : tw.b[i];
}
__device__ __forceinline__ TwView twv(const uint32_t* base, int mi, uint32_t n) { return TwView(base, mi, n); }
__device__ __forceinline__ uint32_t tw_mul(const TwView& tw, uint32_t i, bool uniform, uint32_t b, uint32_t q,
                                           uint32_t qinv) {
  return mulm(b, tw_get(tw, i, uniform), q, qinv);
}


__device__ __forceinline__ uint32_t dbrv(uint32_t x, int logn) { return __brev(x) >> (32 - logn); }

// Thread id hidden from loop-invariant code motion: inside the digit and pair
// loops every LDS address, twiddle offset and operand offset derived from it
// is recomputed (a few ALU ops) instead of being hoisted and kept live in
// ~100 VGPRs for the whole loop.  An empty register-only asm, no memory access.
__device__ __forceinline__ int tid_fresh() {
  uint32_t v = threadIdx.x;
  asm volatile("" : "+v"(v));
  return (int)v;
}

// NTT-domain automorphism: output index k holds the input at auto_perm(k), for
// sigma_g: a(X) -> a(X^g) with evaluations stored at psi^(2 brv(k) + 1).
__device__ __forceinline__ uint32_t auto_perm(uint32_t k, uint32_t g, int logn) {
  const uint32_t e = 2 * dbrv(k, logn) + 1;
  const uint32_t ge = (g * e) & ((2u << logn) - 1);
  return dbrv((ge - 1) >> 1, logn);
}

// Exchange between passes.  Single-buffered (DB = false): a barrier before the
// writes (earlier reads of the buffer must be done) and one after.  Double-
// buffered (DB = true, two LDS buffers, `par` selects one and flips): the
// write-after-read barrier is not needed, because consecutive exchanges use
// different buffers and the barrier of the exchange in between orders them.
// Addresses: one padded per-thread base per side, constant element offsets.
//
// The boundary next to the last pass of a WLAST geometry stays inside each
// wave: the wave reads back only the block it wrote, so a wave-scope fence
// replaces the barrier after the writes (one wave's LDS operations execute in
// program order).  Forward direction (pto = last pass): the block was last read,
// since the previous barrier, by its own wave only (the exchange into pass
// NPASS - 2 is block-local on its read side), so the barrier before the writes
// goes too.  Inverse direction (pfrom = last pass): this is the transform's first
// exchange and may follow reads of the whole buffer by every wave (a gather, an
// earlier transform), so that barrier stays.  Single-buffered only: the
// double-buffered order relies on every exchange having its barrier.
template <class G, bool DB = false>
__device__ __forceinline__ void xchg(uint32_t* lds, int pfrom, int pto, uint32_t* x, int t, int* par = nullptr) {
  const bool wave_local = !DB && G::WLAST && (pfrom == G::NPASS - 1 || pto == G::NPASS - 1);
  if constexpr (DB) {
    lds += (*par) * G::LDS_WORDS;
    *par ^= 1;
  } else {
    if (!(wave_local && pto == G::NPASS - 1)) __syncthreads();
  }
  uint32_t* wr = lds + G::pad(G::tbase(pfrom, t));
#pragma unroll
  for (int e = 0; e < G::E; ++e) wr[G::padoff(G::eoff(pfrom, e))] = x[e];
  if (wave_local) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
  const uint32_t* rd = lds + G::pad(G::tbase(pto, t));
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = rd[G::padoff(G::eoff(pto, e))];
}

// forward transform: x in pass-0 layout with values < 4q; returns the
// evaluations in last-pass layout, canonical [0, q) (LAZY: left in [0, 4q))
template <class G, bool DB = false, bool PF = false, class TW = TwView, bool LAZY = false>
__device__ __forceinline__ void ntt_fwd(uint32_t* x, uint32_t* lds, const TW& tw, const Mod& m, int t,
                                        int* par = nullptr) {
#pragma unroll
  for (int p = 0; p < G::NPASS; ++p) {
    if (p > 0) xchg<G, DB>(lds, p - 1, p, x, t, par);
    fwd_pass<G, PF>(p, t, x, tw, m.q, m.qinv);
  }
  if constexpr (!LAZY) {
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = red2(x[e], m.q);
  }
}

// inverse transform: x in last-pass layout with values < 2q (canonical with
// STRICT, for moduli of 2^30 and above); returns canonical coefficients in
// pass-0 layout
template <class G, bool DB = false, bool PF = false, class TW = TwView, bool STRICT = false>
__device__ __forceinline__ void ntt_inv(uint32_t* x, uint32_t* lds, const TW& itw, const Mod& m, int t,
                                        int* par = nullptr) {
#pragma unroll
  for (int p = G::NPASS - 1; p >= 0; --p) {
    if (p < G::NPASS - 1) xchg<G, DB>(lds, p + 1, p, x, t, par);
    // pass 0 ends with the transform's last stage, which also scales by n^-1
    if (p == 0) inv_pass<G, PF, STRICT, TW, true>(p, t, x, itw, m.q, m.qinv, m.ninv_m);
    else inv_pass<G, PF, STRICT>(p, t, x, itw, m.q, m.qinv);
  }
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = red1(x[e], m.q);
}

// pass-0 layout: element e of thread t is index e T + t (coalesced).  Offsets
// are 32-bit unsigned and bases wave-uniform, so loads use a scalar base plus a
// 32-bit vector offset instead of a 64-bit address per lane.
template <class G>
__device__ __forceinline__ uint32_t idx0(int e, int t) { return (uint32_t)e * G::T + (uint32_t)t; }
// last-pass layout index
template <class G>
__device__ __forceinline__ uint32_t idxL(int e, int t) { return (uint32_t)G::idx(G::NPASS - 1, t, e); }
// the same with a fresh thread id per call, for loop bodies (see tid_fresh)
template <class G>
__device__ __forceinline__ uint32_t idx0f(int e) { return idx0<G>(e, tid_fresh()); }
template <class G>
__device__ __forceinline__ uint32_t idxLf(int e) { return idxL<G>(e, tid_fresh()); }



template <class G>
__device__ __forceinline__ void load0(const DBuf& g, uint32_t* x, int t, uint32_t s = 0) {
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = g.at((uint32_t)t, s + G::eoff(0, e));
}
template <class G>
__device__ __forceinline__ void store0(const DBuf& g, const uint32_t* x, int t) {
#pragma unroll
  for (int e = 0; e < G::E; ++e) g.put((uint32_t)t, G::eoff(0, e), x[e]);
}
// last-pass layout: contiguous chunks of 2^r_last residues; vector access when possible
template <class G>
__device__ __forceinline__ void loadL(const DBuf& g, uint32_t* x, int t) {
  constexpr int C = 1 << G::r(G::NPASS - 1);
  const uint32_t b = G::tbase(G::NPASS - 1, t);
  if constexpr (C % 4 == 0) {
#pragma unroll
    for (int e = 0; e < G::E; e += 4) {
      const u32x4 v = g.at4(b, G::eoff(G::NPASS - 1, e));
      x[e] = v.x; x[e + 1] = v.y; x[e + 2] = v.z; x[e + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = g.at(b, G::eoff(G::NPASS - 1, e));
  }
}
template <class G>
__device__ __forceinline__ void storeL(const DBuf& g, const uint32_t* x, int t) {
  constexpr int C = 1 << G::r(G::NPASS - 1);
  const uint32_t b = G::tbase(G::NPASS - 1, t);
  if constexpr (C % 4 == 0) {
#pragma unroll
    for (int e = 0; e < G::E; e += 4) {
      u32x4 v;
      v.x = x[e]; v.y = x[e + 1]; v.z = x[e + 2]; v.w = x[e + 3];
      g.put4(b, G::eoff(G::NPASS - 1, e), v);
    }
  } else {
#pragma unroll
    for (int e = 0; e < G::E; ++e) g.put(b, G::eoff(G::NPASS - 1, e), x[e]);
  }
}

// lazy accumulate: a, v in [0, 2q) -> [0, 2q)
__device__ __forceinline__ uint32_t acc2(uint32_t a, uint32_t v, uint32_t q) {
  const uint32_t s = a + v;
  return umin(s, s - 2 * q);
}

// four residues e .. e + 3 (e a multiple of 4) of the last-pass layout at
// sbase + index (b: the thread's last-pass base): one vector load when the last
// pass keeps chunks of at least 4 contiguous residues, else four loads (a last
// pass of 1 stage keeps pairs)
template <class G>
__device__ __forceinline__ u32x4 ld4L(const DBuf& g, uint32_t b, uint32_t sbase, int e) {
  constexpr int C = 1 << G::r(G::NPASS - 1);
  constexpr int PL = G::NPASS - 1;
  if constexpr (C % 4 == 0) {
    return g.at4(b, sbase + G::eoff(PL, e));
  } else {
    u32x4 v;
    v.x = g.at(b, sbase + G::eoff(PL, e));
    v.y = g.at(b, sbase + G::eoff(PL, e + 1));
    v.z = g.at(b, sbase + G::eoff(PL, e + 2));
    v.w = g.at(b, sbase + G::eoff(PL, e + 3));
    return v;
  }
}

// x = hi 2^32 + lo is congruent to hi (2^32 mod q) + lo (r1 = 2^32 mod q), which
// is below 2^61 + 2^32 for q < 2^30
__device__ __forceinline__ uint64_t fold32(uint64_t x, uint32_t r1) {
  return (uint64_t)(uint32_t)(x >> 32) * r1 + (uint32_t)x;
}


// ------------------------------------------------------------------ batched transform
// One limb per workgroup, at LE_ residues per thread (the forward transform
// measured fastest at 16, the inverse at 32), the next stage's twiddles loaded
// during the current one.
template <int LOGN, int LE_, bool INV>
__global__ __launch_bounds__((Geom<LOGN, LE_>::T)) void k_ntt(DevCtx c, uint32_t* data, uint32_t nmod, uint32_t mod0) {
  using G = Geom<LOGN, LE_>;
  const int t = threadIdx.x;
  __shared__ uint32_t lds[G::LDS_WORDS];
  const size_t p = blockIdx.x;
  const int mi = mod0 + (int)(p % nmod);
  const DBuf g(data + p * G::N, G::N);
  uint32_t x[G::E];
  if (!INV) {
    load0<G>(g, x, t);
    ntt_fwd<G, false, true>(x, lds, twv(c.tw, mi, G::N), c.mod[mi], t);
    storeL<G>(g, x, t);
  } else {
    loadL<G>(g, x, t);
    ntt_inv<G, false, true>(x, lds, twv(c.itw, mi, G::N), c.mod[mi], t);
    store0<G>(g, x, t);
  }
}

// ------------------------------------------------------------------ encoding mod t
// Source of slot values for the batch encoder.
enum EncSrc { SRC_ROWS = 0, SRC_COLS = 1, SRC_WT = 2 };

__device__ __forceinline__ uint32_t mod_t_i64(int64_t v, uint32_t t) {
  int64_t r = v % (int64_t)t;
  return (uint32_t)(r < 0 ? r + t : r);
}

// plaintext poly ci (coefficients mod t, canonical, natural order) from slot
// values; rows: ci = i K + k -> X[i][k n + s]; cols: ci = k -> X[s][k] (s < rows);
// wt: ci = j K + k -> W[k n + s][j] (W is f x classes).  Also writes
// rnd[ci][k] = round((Q mod t) m_k / t) for the encryption's Delta(m).
template <int LOGN>
__global__ __launch_bounds__(Gm<LOGN>::T) void k_encode(DevCtx c, const int64_t* __restrict__ src, int mode,
                                                        uint32_t rows, uint32_t f, uint32_t K, uint32_t classes,
                                                        uint32_t* __restrict__ m_out, uint32_t* __restrict__ rnd) {
  using G = Gm<LOGN>;
  const int t = threadIdx.x;
  __shared__ uint32_t lds[G::LDS_WORDS];
  const size_t ci = blockIdx.x;
  const uint32_t tm = c.t;
  const DBuf pos(c.pos_slot, G::N);
  uint32_t x[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) {
    const uint32_t s = pos[idxL<G>(e, t)];
    int64_t v = 0;
    if (mode == SRC_ROWS) {
      const uint64_t i = ci / K, k = ci % K, col = k * G::N + s;
      if (col < f) v = src[i * f + col];
    } else if (mode == SRC_COLS) {
      if (s < rows) v = src[(size_t)s * f + ci];
    } else {
      const uint64_t j = ci / K, k = ci % K, row = k * G::N + s;
      if (row < f) v = src[row * classes + j];
    }
    x[e] = mod_t_i64(v, tm);
  }
  // the mod-t transform: lazy reduction where 4t fits in 32 bits, canonical
  // residues throughout for t of 2^30 and above (the paper's plaintext modulus
  // t0 = 1073872897)
  const int mt = c.L + 1;
  if (tm < (1u << 30)) ntt_inv<G>(x, lds, twv(c.itw, mt, G::N), c.mod[mt], t);
  else ntt_inv<G, false, false, TwView, true>(x, lds, twv(c.itw, mt, G::N), c.mod[mt], t);
  store0<G>(DBuf(m_out + ci * G::N, G::N), x, t);
  if (rnd) {
    const DBuf r(rnd + ci * G::N, G::N);
#pragma unroll
    for (int e = 0; e < G::E; ++e) {
      const uint64_t y = (uint64_t)c.qmodt * x[e] + (tm - 1) / 2;
      uint64_t qd = (uint64_t)((double)y / (double)tm);
      if (qd * tm > y) --qd;
      else if ((qd + 1) * tm <= y) ++qd;
      r.st(idx0<G>(e, t), (uint32_t)qd);
    }
  }
}

// ------------------------------------------------------------------ encryption
// u (ternary), e0, e1 (CBD eta = 21) of ciphertext ci, 16 coefficients per thread.
static __global__ __launch_bounds__(256) void k_sample(uint64_t seed, uint64_t id0, uint32_t n, uint64_t nct,
                                                int8_t* __restrict__ small) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t per = n / 16;
  const uint64_t ci = gid / per;
  const uint32_t grp = (uint32_t)(gid % per);
  if (ci >= nct) return;
  const uint64_t id = id0 + ci;
  int8_t* u = small + ci * 3 * n;
  int8_t* e0 = u + n;
  int8_t* e1 = e0 + n;
  uint32_t w[16];
  chacha20(seed, KIND_ENC_U, id, grp, w);
#pragma unroll
  for (int k = 0; k < 16; ++k) u[16 * grp + k] = (int8_t)ternary_of(w[k]);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    chacha20(seed, KIND_ENC_E0, id, 2 * grp + half, w);
#pragma unroll
    for (int k = 0; k < 8; ++k) e0[16 * grp + 8 * half + k] = (int8_t)cbd21_of(w[2 * k], w[2 * k + 1]);
    chacha20(seed, KIND_ENC_E1, id, 2 * grp + half, w);
#pragma unroll
    for (int k = 0; k < 8; ++k) e1[16 * grp + 8 * half + k] = (int8_t)cbd21_of(w[2 * k], w[2 * k + 1]);
  }
}

__device__ __forceinline__ uint32_t small_mod(int v, uint32_t q) { return v < 0 ? q + v : (uint32_t)v; }

// ct = (pk0 U + NTT(e0 + Delta(m)), pk1 U + NTT(e1)) for ciphertext ci, limb j
template <int LOGN>
__global__ __launch_bounds__(Gm<LOGN>::T) void k_encrypt(DevCtx c, const uint32_t* __restrict__ pk,
                                                         const int8_t* __restrict__ small,
                                                         const uint32_t* __restrict__ m,
                                                         const uint32_t* __restrict__ rnd,
                                                         uint32_t* __restrict__ ct) {
  using G = Gm<LOGN>;
  const int t = threadIdx.x;
  __shared__ uint32_t lds[G::LDS_WORDS];
  const size_t ci = blockIdx.x / c.L;
  const int j = blockIdx.x % c.L;
  const Mod md = c.mod[j];
  const TwView tw = twv(c.tw, j, G::N);
  const int8_t* su = small + ci * 3 * G::N;
  const DBuf mv(m + ci * G::N, G::N), rv(rnd + ci * G::N, G::N);
  uint32_t U[G::E], x[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) U[e] = small_mod(su[idx0<G>(e, t)], md.q);
  ntt_fwd<G, false, true>(U, lds, tw, md, t);
#pragma unroll
  for (int e = 0; e < G::E; ++e) {
    const uint32_t k = idx0<G>(e, t);
    // rnd < t < 2 q_j: one conditional subtraction makes it a residue mod q_j
    const uint32_t delta = addm(red1(mulm(mv[k], c.qdivt_m[j], md.q, md.qinv), md.q), red1(rv[k], md.q), md.q);
    x[e] = addm(small_mod(su[G::N + k], md.q), delta, md.q);
  }
  ntt_fwd<G, false, true>(x, lds, tw, md, t);
  uint32_t* out = ct + ci * 2 * c.L * G::N;
  const DBuf pk0(pk + (size_t)j * G::N, G::N), pk1(pk + (size_t)(c.L + j) * G::N, G::N);
  uint32_t v[G::E];
  loadL<G>(pk0, v, t);
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = addm(red1(mulm(U[e], v[e], md.q, md.qinv), md.q), x[e], md.q);
  storeL<G>(DBuf(out + (size_t)j * G::N, G::N), x, t);
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = small_mod(su[2 * G::N + idx0<G>(e, t)], md.q);
  ntt_fwd<G, false, true>(x, lds, tw, md, t);
  loadL<G>(pk1, v, t);
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = addm(red1(mulm(U[e], v[e], md.q, md.qinv), md.q), x[e], md.q);
  storeL<G>(DBuf(out + (size_t)(c.L + j) * G::N, G::N), x, t);
}

// ------------------------------------------------------------------ model encoding
// centred lift of a residue v < t into q, Montgomery form: v itself up to
// (t-1)/2, v - t + q above (both in [0, q) because t < 2q)
__device__ __forceinline__ uint32_t lift_mont(uint32_t v, uint32_t t, const Mod& md) {
  const uint32_t l = v > (t - 1) / 2 ? v + md.q - t : v;
  return to_mont(l, md);
}

// weight plaintext (class j, chunk k) in limb i: lift, Montgomery form, transform
template <int LOGN>
__global__ __launch_bounds__(Gm<LOGN>::T) void k_lift_ntt(DevCtx c, const uint32_t* __restrict__ mt,
                                                          uint32_t* __restrict__ out) {
  using G = Gm<LOGN>;
  const int t = threadIdx.x;
  __shared__ uint32_t lds[G::LDS_WORDS];
  const size_t pi = blockIdx.x / c.L;
  const int i = blockIdx.x % c.L;
  const Mod md = c.mod[i];
  const DBuf src(mt + pi * G::N, G::N);
  uint32_t x[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = lift_mont(src[idx0<G>(e, t)], c.t, md);
  ntt_fwd<G, false, true>(x, lds, twv(c.tw, i, G::N), md, t);
  storeL<G>(DBuf(out + (pi * c.L + i) * G::N, G::N), x, t);
}

// scalar weights for the standard baseline: wsc[k][i][j] = lift(W[k][j] mod t) R mod q_i,
// classes padded with zeros to a multiple of 16 (cpad)
static __global__ void k_scalars(DevCtx c, const int64_t* __restrict__ W, uint32_t f, uint32_t classes, uint32_t cpad,
                          uint32_t* __restrict__ wsc) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (uint64_t)f * c.L * cpad) return;
  const uint32_t j = (uint32_t)(g % cpad);
  const uint32_t i = (uint32_t)((g / cpad) % c.L);
  const uint64_t k = g / ((uint64_t)cpad * c.L);
  wsc[g] = j < classes ? lift_mont(mod_t_i64(W[k * classes + j], c.t), c.t, c.mod[i]) : 0u;
}

// ------------------------------------------------------------------ Algorithm 1
// chunk products and add_many of the tile's pairs:
// out[lp][x][j] = sum_k xrow[k][x][j] * wcls[k][j]  (evaluation form, Montgomery weights)
static __global__ __launch_bounds__(256) void k_mac(DevCtx c, const PairDesc* __restrict__ pairs, uint32_t B,
                                             uint32_t* __restrict__ out) {
  const uint32_t n = c.n, L = c.L;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;   // one uint4 each
  const uint64_t per_pair = (uint64_t)2 * L * n / 4;
  const uint64_t lp = gid / per_pair;
  if (lp >= B) return;
  const uint64_t word = (gid % per_pair) * 4;
  const uint32_t xpoly = (uint32_t)(word / ((uint64_t)L * n));
  const uint32_t j = (uint32_t)((word / n) % L);
  const uint32_t k0 = (uint32_t)(word % n);
  const PairDesc d = pairs[lp];
  const Mod md = c.mod[j];
  uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (uint32_t k = 0; k < d.K; ++k) {
    const uint4 xv = *reinterpret_cast<const uint4*>(d.xrow + (((uint64_t)k * 2 + xpoly) * L + j) * n + k0);
    const uint4 wv = *reinterpret_cast<const uint4*>(d.wcls + ((uint64_t)k * L + j) * n + k0);
    a0 += (uint64_t)xv.x * wv.x; a1 += (uint64_t)xv.y * wv.y;
    a2 += (uint64_t)xv.z * wv.z; a3 += (uint64_t)xv.w * wv.w;
    if ((k % 8) == 7 || k + 1 == d.K) {   // at most 8 products: redc input < 8 q^2 + 2^32 q
      s0 = addm(s0, red2(redc(a0, md.q, md.qinv), md.q), md.q);
      s1 = addm(s1, red2(redc(a1, md.q, md.qinv), md.q), md.q);
      s2 = addm(s2, red2(redc(a2, md.q, md.qinv), md.q), md.q);
      s3 = addm(s3, red2(redc(a3, md.q, md.qinv), md.q), md.q);
      a0 = a1 = a2 = a3 = 0;
    }
  }
  *reinterpret_cast<uint4*>(out + lp * 2 * L * n + word) = make_uint4(s0, s1, s2, s3);
}

// key switch, part 1: d_i = INTT(sigma_g(c1))_i, digits in coefficient form
template <int LOGN, int LE>
__global__ __launch_bounds__((Geom<LOGN, LE>::T)) void k_ks_intt(DevCtx c, const uint32_t* __restrict__ cin,
                                                                uint32_t g, uint32_t* __restrict__ D) {
  using G = Geom<LOGN, LE>;
  const int t = threadIdx.x;
  __shared__ uint32_t lds[G::LDS_WORDS];
  const size_t lp = blockIdx.x / c.L;
  const int i = blockIdx.x % c.L;
  const DBuf src(cin + (lp * 2 * c.L + c.L + i) * G::N, G::N);
  uint32_t* wr = lds + G::pad((uint32_t)t);
#pragma unroll
  for (int e = 0; e < G::E; ++e) wr[G::padoff(G::eoff(0, e))] = src.at((uint32_t)t, G::eoff(0, e));
  __syncthreads();
  uint32_t x[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = lds[G::pad(auto_perm(idxL<G>(e, t), g, LOGN))];
  ntt_inv<G, false, true>(x, lds, twv(c.itw, i, G::N), c.mod[i], t);
  store0<G>(DBuf(D + (lp * c.L + i) * G::N, G::N), x, t);
}

// Part 3 of the key switch for one limb r and one ciphertext part (PART 0 =
// b, 1 = a) from the part's inner-product sum acc (registers, last-pass layout,
// [0, 2 q_r)): out = (acc - NTT_r(rho_PART - h)) P^-1 mod q_r, then the
// rotate-and-accumulate, c0 + sigma_g(c0) + out for b, c1 + out for a, stored
// to dst.  The values of k_ks_moddown: out is the canonical residue of a
// product, so it does not depend on which representatives enter it; here acc
// stays in [0, 2q) and the transform's output is only brought to [0, 2q), and
// acc + 2q - x < 4q.  A template on the part, so that acc is always a register
// array under constant indices.
template <class G, bool DB, bool PF, int PART>
__device__ __forceinline__ void ks_part3_limb(const uint32_t* acc, uint32_t* x, uint32_t* lds, int* par,
                                              const TwView& tw, const Mod& mr, uint32_t hq, uint32_t pinv,
                                              const DBuf& rho, const DBuf& c0, const DBuf& cp, uint32_t g,
                                              const DBuf& dst) {
  __builtin_amdgcn_sched_barrier(0);
  {
    const uint32_t t0 = (uint32_t)tid_fresh();
    // rho - h + q_r < P + q_r < 4 q_r is a valid lazy input
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = rho.at(t0, (uint32_t)PART * G::N + G::eoff(0, e)) + mr.q - hq;
  }
  ntt_fwd<G, DB, PF, TwView, true>(x, lds, tw, mr, tid_fresh(), par);   // [0, 4q)
  __builtin_amdgcn_sched_barrier(0);
  const int t1 = tid_fresh();
  const uint32_t bL = G::tbase(G::NPASS - 1, t1);
  const uint32_t q2 = 2 * mr.q;
#pragma unroll
  for (int e = 0; e < G::E; e += 4) {
    const u32x4 v = ld4L<G>(cp, bL, 0, e);
    const uint32_t cv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
      const int ee = e + k4;
      const uint32_t o = red1(mulm(acc[ee] + q2 - umin(x[ee], x[ee] - q2), pinv, mr.q, mr.qinv), mr.q);
      uint32_t v2 = cv[k4];
      if constexpr (PART == 0) v2 = addm(v2, c0[auto_perm(bL + G::eoff(G::NPASS - 1, ee), g, G::LOGN)], mr.q);
      x[ee] = addm(v2, o, mr.q);
    }
  }
  storeL<G>(dst, x, t1);
}

// key switch, part 2: for target modulus r, acc_x = sum_i NTT_r(d_i) ksk_{g,i,x,r}
// (for i = r the transform is skipped: NTT_r(d_r) is limb r of sigma_g(c1));
// r = P additionally returns rho_x = [INTT(acc_x) + (P-1)/2]_P in coefficient form
// Variants (MODE bits; none changes a result bit): 1 = double-buffered LDS
// exchange (one barrier per exchange) where two buffers fit in the 160 KB of
// LDS; 2 = the next digit is loaded during the current transform; 4 = the
// twiddles of the next butterfly stage are loaded during the current one;
// 8 = a register cap that lets two workgroups share a CU (only useful
// single-buffered); 32 and 64 = workgroup order (below); 128 = the inner
// products accumulate unreduced 64-bit products (one multiply-add each, folded
// every 4 digits) instead of reducing every product; 256 = two workgroups per
// item, one for each half of the digits, writing their sums to ACC and ACC2
// (canonical, no inverse transform for r = P; k_ks_rho finishes that item);
// 512 = target moduli by XCD (below).  1024 and 2048 split a step's items
// over two launches: 1024 runs the special-prime items only (one workgroup per
// pair, rho to ACC as above); 2048 then runs the L data-modulus items, and each
// finishes part 3 for its own limb r from the sums in its registers: the
// rounded division by P (rho from ACC, transformed mod q_r) and the
// rotate-and-accumulate, written to cout, so no sum goes through ACC and no
// k_ks_moddown launch follows.  The arithmetic is that of k_ks_moddown.
// 4096 (with 1024): the special-prime workgroup of a pair also makes the
// pair's digits, k_ks_intt's steps for each limb i (sigma_g of limb i of c1
// through LDS, inverse transform mod q_i), stores them to D for the
// data-modulus launch and transforms the same registers mod P; no k_ks_intt
// launch precedes.
template <int LOGN, int LE, int MODE>
__global__ __launch_bounds__((Geom<LOGN, LE>::T), ((MODE & 8) ? Geom<LOGN, LE>::T / 128 : 1)) void k_ks_mac(
    DevCtx c, const uint32_t* __restrict__ cin, uint32_t* __restrict__ D, const PairDesc* __restrict__ pairs,
    const uint32_t* __restrict__ gk_default, uint32_t gi, uint32_t g, uint32_t* __restrict__ ACC,
    uint32_t* __restrict__ ACC2, uint32_t* __restrict__ cout) {
  constexpr bool DB = (MODE & 1) && 2 * Geom<LOGN, LE>::LDS_WORDS * 4 <= 160 * 1024;
  // the wave-local last-pass blocks only pay where they remove barriers
  // (single buffer); double-buffered, the plain numbering measured faster
  using G = Geom<LOGN, LE, !DB>;
  constexpr bool DP = (MODE & 2) != 0;   // digit prefetch
  constexpr bool PF = (MODE & 4) != 0;   // twiddle prefetch
  constexpr bool A64 = (MODE & 128) != 0;
  __shared__ uint32_t lds[(DB ? 2 : 1) * G::LDS_WORDS];
  int par = 0;
  const int L = c.L;
  // consecutive workgroups go to the 8 XCDs in turn.  MODE 64: the workgroups
  // of a pair run on one XCD, one after the other, so the pair's digits are
  // fetched into that XCD's L2 once.
  uint32_t li = blockIdx.x;
  if constexpr ((MODE & 64) != 0) {
    if (gridDim.x % 8 == 0) li = (li % 8) * (gridDim.x / 8) + li / 8;
  }
  constexpr bool HALF = (MODE & 256) != 0;
  const int per_pair = HALF ? 2 * (L + 1) : L + 1;   // workgroups per pair
  size_t lp = li / per_pair;
  const int wi = (int)(li % per_pair);
  // the special-prime item (r = L) carries more work than the others; MODE 32
  // rotates its place among the pair's workgroups from pair to pair, so the
  // heavy items spread over the launch order
  int r = HALF ? wi >> 1 : wi;
  if constexpr ((MODE & 32) != 0) r = (r + (int)(lp % (L + 1))) % (L + 1);
  if constexpr ((MODE & 512) != 0) {
    static_assert((MODE & (64 | 256)) == 0, "MODE 512 replaces the pair-per-XCD order and has one item per workgroup");
    // Eight target moduli (L = 7) on eight XCDs.  XCD x runs the workgroups
    // x, x + 8, ...; its s-th one is slot s.  The slots of each XCD are cut into
    // windows of KW pairs; in window w, XCD x takes the moduli 2m and 2m + 1,
    // m = (x + w) mod 4, for one half of the window's pairs (the half x / 4),
    // a pair's two workgroups in adjacent slots.  An XCD's L2 then holds two
    // key slices of the step instead of all eight, and the special prime
    // moves to other XCDs from window to window.  Every (pair, modulus) is
    // taken once: per window the four values of m meet both halves.
    constexpr uint32_t KW = 256;
    const uint32_t npairs = gridDim.x / 8;
    if (L == 7 && (npairs & 1) == 0) {
      const uint32_t x = blockIdx.x % 8, s = blockIdx.x / 8;
      const uint32_t w = s / KW, k = s % KW, p0 = w * KW;
      const uint32_t wl = min(KW, npairs - p0);   // pairs in this window, even
      lp = p0 + (x / 4) * (wl / 2) + k / 2;
      r = (int)(2 * ((x + w) % 4) + (k & 1));
    }
  }
  constexpr bool PONLY = (MODE & 1024) != 0, MD = (MODE & 2048) != 0, DIG = (MODE & 4096) != 0;
  static_assert(!DIG || (PONLY && !DP && !DB), "digits are made by the single-buffered special-prime launch");
  static_assert(!((PONLY || MD) && (MODE & (32 | 64 | 256 | 512))), "the split launches have their own item maps");
  if constexpr (PONLY) {
    lp = blockIdx.x;
    r = L;
  }
  if constexpr (MD) {
    // L workgroups per pair, the pair's workgroups on one XCD (as MODE 64)
    uint32_t lj = blockIdx.x;
    if (gridDim.x % 8 == 0) lj = (lj % 8) * (gridDim.x / 8) + lj / 8;
    lp = lj / L;
    r = (int)(lj % L);
  }
  // digits of this workgroup: all of them, or one half
  const int half = HALF ? wi & 1 : 0;
  const int i_lo = half ? (L + 1) / 2 : 0;
  const int i_hi = HALF && !half ? (L + 1) / 2 : L;
  const Mod mr = c.mod[r];
  const TwView tw = twv(c.tw, r, G::N);
  // the pair's Galois key for element gi, target modulus r: [L digits][2][n]
  const uint32_t* gk = pairs[lp].gk;
  const uint32_t* key = (gk ? gk : gk_default) + (size_t)gi * (L + 1) * L * 2 * G::N;
  const DBuf kr(key + (size_t)r * L * 2 * G::N, (uint32_t)(L * 2 * G::N));
  const DBuf dp(D + lp * L * G::N, (uint32_t)(L * G::N));
  uint32_t ab[G::E], aa[G::E], x[G::E];
  [[maybe_unused]] uint64_t ab64[A64 ? G::E : 1], aa64[A64 ? G::E : 1];
  [[maybe_unused]] const uint32_t r1 = red1(redc(mr.r2, mr.q, mr.qinv), mr.q);   // 2^32 mod r
#pragma unroll
  for (int e = 0; e < G::E; ++e) {
    if constexpr (A64) ab64[e] = aa64[e] = 0;
    else ab[e] = aa[e] = 0;
  }
  // digits are transformed in order i = 0..L-1 (i != r); the next one is
  // prefetched into xn while the current transform runs
  [[maybe_unused]] uint32_t xn[DP ? G::E : 1];
  if constexpr (DP) {
    const int first = r == i_lo ? i_lo + 1 : i_lo;
    if (first < i_hi) {
      const uint32_t tb = (uint32_t)tid_fresh();
#pragma unroll
      for (int e = 0; e < G::E; ++e) xn[e] = dp.at(tb, (uint32_t)first * G::N + G::eoff(0, e));
    }
  }
  for (int i = i_lo; i < i_hi; ++i) {
    const uint32_t kb = (uint32_t)(2 * i) * G::N, ka = kb + G::N;
    if (i == r) {
      // [d_r]_{q_r} in evaluation form is limb r of sigma_g(c1): a permutation of the input
      const DBuf c1r(cin + (lp * 2 * L + L + r) * G::N, G::N);
#pragma unroll
      for (int e = 0; e < G::E; ++e) x[e] = c1r[auto_perm(idxLf<G>(e), g, LOGN)];
    } else {
      // d_i < q_i < 4 q_r: a valid lazy input
      if constexpr (DIG) {
        // d_i = INTT_i(sigma_g(limb i of c1)), as k_ks_intt: the limb to LDS at its
        // natural positions (after every wave has read the last exchange), the
        // permutation gathered into the last-pass layout, the inverse transform
        const DBuf src(cin + (lp * 2 * L + L + i) * G::N, G::N);
        __syncthreads();
        {
          const int tt = tid_fresh();
          uint32_t* wr = lds + G::pad((uint32_t)tt);
#pragma unroll
          for (int e = 0; e < G::E; ++e) wr[G::padoff(G::eoff(0, e))] = src.at((uint32_t)tt, G::eoff(0, e));
        }
        __syncthreads();
        {
          const int tt = tid_fresh();
#pragma unroll
          for (int e = 0; e < G::E; ++e) x[e] = lds[G::pad(auto_perm(idxL<G>(e, tt), g, LOGN))];
        }
        ntt_inv<G, false, true>(x, lds, twv(c.itw, i, G::N), c.mod[i], tid_fresh());
        store0<G>(DBuf(D + (lp * L + i) * G::N, G::N), x, tid_fresh());
        __builtin_amdgcn_sched_barrier(0);
      } else if constexpr (DP) {
#pragma unroll
        for (int e = 0; e < G::E; ++e) x[e] = xn[e];
        int nx = i + 1;
        if (nx == r) ++nx;
        if (nx < i_hi) {
          const uint32_t tb = (uint32_t)tid_fresh();
#pragma unroll
          for (int e = 0; e < G::E; ++e) xn[e] = dp.at(tb, (uint32_t)nx * G::N + G::eoff(0, e));
        }
      } else {
        const uint32_t tb = (uint32_t)tid_fresh();
#pragma unroll
        for (int e = 0; e < G::E; ++e) x[e] = dp.at(tb, (uint32_t)i * G::N + G::eoff(0, e));
      }
      // the products reduce any input below 2^32, so the digit stays lazy in
      // [0, 4 q_r) unless it feeds the unreduced 64-bit sums
      ntt_fwd<G, DB, PF, TwView, !A64>(x, lds, tw, mr, tid_fresh(), &par);
    }
    // keep the key loads below the transform: hoisting them into it costs 64 VGPRs
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t bL = G::tbase(G::NPASS - 1, tid_fresh());
#pragma unroll
    for (int e = 0; e < G::E; e += 4) {
      const u32x4 vb = ld4L<G>(kr, bL, kb, e), va = ld4L<G>(kr, bL, ka, e);
      if constexpr (A64) {
        // x < q_r and key words < q_r: each product < 2^60
        ab64[e] += (uint64_t)x[e] * vb.x;
        ab64[e + 1] += (uint64_t)x[e + 1] * vb.y;
        ab64[e + 2] += (uint64_t)x[e + 2] * vb.z;
        ab64[e + 3] += (uint64_t)x[e + 3] * vb.w;
        aa64[e] += (uint64_t)x[e] * va.x;
        aa64[e + 1] += (uint64_t)x[e + 1] * va.y;
        aa64[e + 2] += (uint64_t)x[e + 2] * va.z;
        aa64[e + 3] += (uint64_t)x[e + 3] * va.w;
      } else {
        ab[e] = acc2(ab[e], mulm(x[e], vb.x, mr.q, mr.qinv), mr.q);
        ab[e + 1] = acc2(ab[e + 1], mulm(x[e + 1], vb.y, mr.q, mr.qinv), mr.q);
        ab[e + 2] = acc2(ab[e + 2], mulm(x[e + 2], vb.z, mr.q, mr.qinv), mr.q);
        ab[e + 3] = acc2(ab[e + 3], mulm(x[e + 3], vb.w, mr.q, mr.qinv), mr.q);
        aa[e] = acc2(aa[e], mulm(x[e], va.x, mr.q, mr.qinv), mr.q);
        aa[e + 1] = acc2(aa[e + 1], mulm(x[e + 1], va.y, mr.q, mr.qinv), mr.q);
        aa[e + 2] = acc2(aa[e + 2], mulm(x[e + 2], va.z, mr.q, mr.qinv), mr.q);
        aa[e + 3] = acc2(aa[e + 3], mulm(x[e + 3], va.w, mr.q, mr.qinv), mr.q);
      }
    }
    if constexpr (A64) {
      // every 4 digits: below 2^61 + 2^32 + 4 2^60 < 2^64 before the fold
      if ((i & 3) == 3) {
#pragma unroll
        for (int e = 0; e < G::E; ++e) {
          ab64[e] = fold32(ab64[e], r1);
          aa64[e] = fold32(aa64[e], r1);
        }
      }
    }
  }
  if constexpr (A64) {
    // fold: < 2^61 + 2^32, so redc lands below 2^29 + q < 4q; keys carry R
#pragma unroll
    for (int e = 0; e < G::E; ++e) {
      ab[e] = red2(redc(fold32(ab64[e], r1), mr.q, mr.qinv), mr.q);
      aa[e] = red2(redc(fold32(aa64[e], r1), mr.q, mr.qinv), mr.q);
    }
  }
  if constexpr (MD) {
    // part 3 for limb r: out_x = (acc_x - NTT_r(rho_x - h)) P^-1 mod q_r, then
    // c0' = c0 + sigma_g(c0) + out_b and c1' = c1 + out_a
    const DBuf rho(ACC + (lp * (L + 1) + L) * 2 * G::N, 2 * G::N);
    const DBuf c0(cin + (lp * 2 * L + r) * G::N, G::N);
    const DBuf c1(cin + (lp * 2 * L + L + r) * G::N, G::N);
    uint32_t* co = cout + lp * 2 * L * G::N;
    ks_part3_limb<G, DB, PF, 0>(ab, x, lds, &par, tw, mr, c.hmod[r], c.pinv_m[r], rho, c0, c0, g,
                                DBuf(co + (size_t)r * G::N, G::N));
    ks_part3_limb<G, DB, PF, 1>(aa, x, lds, &par, tw, mr, c.hmod[r], c.pinv_m[r], rho, c0, c1, g,
                                DBuf(co + (size_t)(L + r) * G::N, G::N));
    return;
  }
  const int t = tid_fresh();
  uint32_t* out = (half ? ACC2 : ACC) + (lp * (L + 1) + r) * 2 * G::N;
  const DBuf ob(out, G::N), oa(out + G::N, G::N);
  if (HALF || r < L) {
#pragma unroll
    for (int e = 0; e < G::E; ++e) { ab[e] = red1(ab[e], mr.q); aa[e] = red1(aa[e], mr.q); }
    storeL<G>(ob, ab, t);
    storeL<G>(oa, aa, t);
  } else {
    const uint32_t h = (mr.q - 1) / 2;
    const TwView itw = twv(c.itw, r, G::N);
    ntt_inv<G, DB, PF>(ab, lds, itw, mr, t, &par);
#pragma unroll
    for (int e = 0; e < G::E; ++e) ab[e] = addm(ab[e], h, mr.q);
    store0<G>(ob, ab, t);
    ntt_inv<G, DB, PF>(aa, lds, itw, mr, t, &par);
#pragma unroll
    for (int e = 0; e < G::E; ++e) aa[e] = addm(aa[e], h, mr.q);
    store0<G>(oa, aa, t);
  }
}

// key switch, small-tile variant, between parts 2 and 3: the special-prime
// sums of the two digit halves, acc_x = ACC + ACC2, become rho_x =
// [INTT(acc_x) + (P-1)/2]_P, written over ACC.  One workgroup per (pair, x).
template <int LOGN, int LE>
__global__ __launch_bounds__((Geom<LOGN, LE>::T)) void k_ks_rho(DevCtx c, uint32_t* __restrict__ ACC,
                                                               const uint32_t* __restrict__ ACC2) {
  using G = Geom<LOGN, LE>;
  const int t = threadIdx.x;
  __shared__ uint32_t lds[G::LDS_WORDS];
  const int L = c.L;
  const size_t lp = blockIdx.x >> 1;
  const size_t off = (lp * (L + 1) + L) * 2 * G::N + (blockIdx.x & 1) * G::N;
  const Mod mp = c.mod[L];
  uint32_t x[G::E], y[G::E];
  loadL<G>(DBuf(ACC + off, G::N), x, t);
  loadL<G>(DBuf(ACC2 + off, G::N), y, t);
  // both below P: the sum is below 2P, a valid inverse-transform input.  Every
  // load is consumed before the first exchange barrier, so the in-place store
  // below cannot overtake another thread's load.
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] += y[e];
  ntt_inv<G, false, true>(x, lds, twv(c.itw, L, G::N), mp, t);
  const uint32_t h = (mp.q - 1) / 2;
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = addm(x[e], h, mp.q);
  store0<G>(DBuf(ACC + off, G::N), x, t);
}

// key switch, part 3 of the small-tile variant: k_ks_moddown for one output
// limb and one part x (b or a) per workgroup, the accumulator being ACC + ACC2
template <int LOGN, int LE>
__global__ __launch_bounds__((Geom<LOGN, LE>::T)) void k_ks_moddown_part(DevCtx c, const uint32_t* __restrict__ cin,
                                                                        const uint32_t* __restrict__ ACC,
                                                                        const uint32_t* __restrict__ ACC2, uint32_t g,
                                                                        uint32_t* __restrict__ cout) {
  using G = Geom<LOGN, LE>;
  const int t = threadIdx.x;
  __shared__ uint32_t lds[G::LDS_WORDS];
  const int L = c.L;
  const size_t lp = blockIdx.x / (2 * L);
  const int j = (int)(blockIdx.x % (2 * L)) >> 1;
  const uint32_t part = blockIdx.x & 1;
  const Mod md = c.mod[j];
  const uint32_t hq = c.hmod[j], pinv = c.pinv_m[j];
  const size_t slot = (lp * (L + 1) + j) * 2 * G::N + part * G::N;
  const DBuf rho(ACC + (lp * (L + 1) + L) * 2 * G::N + part * G::N, G::N);
  uint32_t x[G::E];
  // rho - h + q_j < P + q_j < 4 q_j is a valid lazy input
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = rho.at((uint32_t)t, G::eoff(0, e)) + md.q - hq;
  ntt_fwd<G, false, true>(x, lds, twv(c.tw, j, G::N), md, t);
  uint32_t a[G::E], a2[G::E];
  loadL<G>(DBuf(ACC + slot, G::N), a, t);
  loadL<G>(DBuf(ACC2 + slot, G::N), a2, t);
  const DBuf cj(cin + (lp * 2 * L + part * L + j) * G::N, G::N);
  uint32_t cz[G::E];
  loadL<G>(cj, cz, t);
  const uint32_t bL = G::tbase(G::NPASS - 1, t);
#pragma unroll
  for (int e = 0; e < G::E; ++e) {
    const uint32_t acc = addm(a[e], a2[e], md.q);
    const uint32_t o = red1(mulm(acc + md.q - x[e], pinv, md.q, md.qinv), md.q);
    // b part: c0 + sigma_g(c0) + out_b; a part: c1 + out_a
    uint32_t v = cz[e];
    if (part == 0) v = addm(v, cj[auto_perm(bL + G::eoff(G::NPASS - 1, e), g, LOGN)], md.q);
    x[e] = addm(v, o, md.q);
  }
  storeL<G>(DBuf(cout + (lp * 2 * L + part * L + j) * G::N, G::N), x, t);
}

// key switch, part 3: rounded division by P, coefficient-wise
// round(acc / P) = (acc - [acc]_P) / P with [acc]_P the centred residue
// rho_x - h, so out_x = (acc_x - NTT(rho_x - h)) P^-1 mod q_j; then the
// rotate-and-accumulate c0' = c0 + sigma_g(c0) + out_b, c1' = c1 + out_a.
// With gnext != 0 the workgroup also does part 1 of the next step for its
// limb: Dn_j = INTT(sigma_gnext(c1'_j)), from the c1' limb it holds (the
// permutation through LDS, as in k_ks_intt), which saves reading c1' again.
template <int LOGN, int LE>
__global__ __launch_bounds__((Geom<LOGN, LE>::T)) void k_ks_moddown(DevCtx c, const uint32_t* __restrict__ cin,
                                                                   const uint32_t* __restrict__ ACC, uint32_t g,
                                                                   uint32_t* __restrict__ cout, uint32_t gnext,
                                                                   uint32_t* __restrict__ Dn) {
  using G = Geom<LOGN, LE>;
  const int t = threadIdx.x;
  __shared__ uint32_t lds[G::LDS_WORDS];
  const int L = c.L;
  // the L workgroups of a pair run on one XCD one after the other (consecutive
  // workgroups go to the 8 XCDs in turn), so rho is fetched into its L2 once
  uint32_t li = blockIdx.x;
  if (gridDim.x % 8 == 0) li = (li % 8) * (gridDim.x / 8) + li / 8;
  const size_t lp = li / L;
  const int j = (int)(li % L);
  const Mod md = c.mod[j];
  const TwView tw = twv(c.tw, j, G::N);
  const DBuf acc(ACC + (lp * (L + 1) + j) * 2 * G::N, 2 * G::N);
  const DBuf rho(ACC + (lp * (L + 1) + L) * 2 * G::N, 2 * G::N);
  const DBuf c0(cin + (lp * 2 * L + j) * G::N, G::N);
  const DBuf c1(cin + (lp * 2 * L + L + j) * G::N, G::N);
  uint32_t x[G::E];
  const uint32_t hq = c.hmod[j], pinv = c.pinv_m[j];
  // b part: rho - h + q_j < P + q_j < 4 q_j is a valid lazy input
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = rho.at((uint32_t)t, G::eoff(0, e)) + md.q - hq;
  ntt_fwd<G, false, true>(x, lds, tw, md, t);
  uint32_t a[G::E];
  loadL<G>(acc, a, t);
  uint32_t cz[G::E];
  loadL<G>(c0, cz, t);
  const uint32_t bL = G::tbase(G::NPASS - 1, t);
#pragma unroll
  for (int e = 0; e < G::E; ++e) {
    const uint32_t k = bL + G::eoff(G::NPASS - 1, e);
    const uint32_t ob = red1(mulm(a[e] + md.q - x[e], pinv, md.q, md.qinv), md.q);
    x[e] = addm(addm(cz[e], c0[auto_perm(k, g, LOGN)], md.q), ob, md.q);
  }
  storeL<G>(DBuf(cout + (lp * 2 * L + j) * G::N, G::N), x, t);
  // a part
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = rho.at((uint32_t)t, G::N + G::eoff(0, e)) + md.q - hq;
  ntt_fwd<G, false, true>(x, lds, tw, md, t);
  const DBuf acca(ACC + (lp * (L + 1) + j) * 2 * G::N + G::N, G::N);
  loadL<G>(acca, a, t);
  uint32_t cc[G::E];
  loadL<G>(c1, cc, t);
#pragma unroll
  for (int e = 0; e < G::E; ++e) {
    const uint32_t oa = red1(mulm(a[e] + md.q - x[e], pinv, md.q, md.qinv), md.q);
    x[e] = addm(cc[e], oa, md.q);
  }
  storeL<G>(DBuf(cout + (lp * 2 * L + L + j) * G::N, G::N), x, t);
  if (gnext) {
    // c1'_j to LDS at its natural positions (the transform's last exchange
    // has been read by every thread once all pass the barrier), then gathered
    // through the next automorphism into the last-pass layout
    // (addresses from a fresh thread id, so that none is computed early and
    // kept live through the two transforms above)
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    const uint32_t bw = G::tbase(G::NPASS - 1, tid_fresh());
#pragma unroll
    for (int e = 0; e < G::E; ++e) lds[G::pad(bw + G::eoff(G::NPASS - 1, e))] = x[e];
    __syncthreads();
    const uint32_t br = G::tbase(G::NPASS - 1, tid_fresh());
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = lds[G::pad(auto_perm(br + G::eoff(G::NPASS - 1, e), gnext, LOGN))];
    const int tf = tid_fresh();
    ntt_inv<G, false, true>(x, lds, twv(c.itw, j, G::N), md, tf);
    store0<G>(DBuf(Dn + (lp * L + j) * G::N, G::N), x, tf);
  }
}

// bias + one-hot mask of each pair of a group, the group's masked ciphertexts
// summed into one partial (the compression of Algorithm 1 is a modular sum, so
// any grouping gives the same output).  mode 0: partial part[group.part]
// (out = partial base); mode 1: each masked pair to out[lp]; mode 2: each pair
// with the bias only (no mask) to out[lp].
template <int LOGN, int LE>
__global__ __launch_bounds__((Geom<LOGN, LE>::T)) void k_mask(DevCtx c, const uint32_t* __restrict__ cin,
                                                             const PairDesc* __restrict__ pairs,
                                                             const GroupDesc* __restrict__ groups, int mode,
                                                             uint32_t* __restrict__ out) {
  // the sub-problem numbering of the last pass without the wave-local blocks:
  // this kernel's last-pass loads and stores measured faster with it
  using Gg = Geom<LOGN, LE, false>;
  __shared__ uint32_t lds[Gg::LDS_WORDS];
  const int L = c.L;
  const GroupDesc grp = groups[blockIdx.x / L];
  const int j = blockIdx.x % L;
  const Mod md = c.mod[j];
  const TwView tw = twv(c.tw, j, Gg::N);
  const DBuf mtab(c.mask_tab, 2 * Gg::N);
  const uint32_t twon_mask = 2 * Gg::N - 1;
  uint32_t a0[Gg::E], a1[Gg::E], x[Gg::E];
#pragma unroll
  for (int e = 0; e < Gg::E; ++e) a0[e] = a1[e] = 0;
  for (uint32_t lp = grp.lp0; lp < grp.lp0 + grp.cnt; ++lp) {
    const PairDesc d = pairs[lp];
    const uint32_t bj = d.dbias[j];
    const DBuf c0(cin + ((size_t)lp * 2 * L + j) * Gg::N, Gg::N);
    const DBuf c1(cin + ((size_t)lp * 2 * L + L + j) * Gg::N, Gg::N);
    if (mode == 2) {
      uint32_t* o = out + (size_t)lp * 2 * L * Gg::N;
      const DBuf o0(o + (size_t)j * Gg::N, Gg::N), o1(o + (size_t)(L + j) * Gg::N, Gg::N);
#pragma unroll
      for (int e = 0; e < Gg::E; ++e) {
        const uint32_t k = idx0f<Gg>(e);
        o0.st(k, addm(c0[k], bj, md.q));
        o1.st(k, c1[k]);
      }
      continue;
    }
    const uint32_t el = c.slot_exp[d.slot];
#pragma unroll
    for (int e = 0; e < Gg::E; ++e) x[e] = lift_mont(mtab[(el * idx0f<Gg>(e)) & twon_mask], c.t, md);
    ntt_fwd<Gg, false, true>(x, lds, tw, md, tid_fresh());
    __builtin_amdgcn_sched_barrier(0);
    uint32_t w0[Gg::E], w1[Gg::E];
    loadL<Gg>(c0, w0, tid_fresh());
    loadL<Gg>(c1, w1, tid_fresh());
#pragma unroll
    for (int e = 0; e < Gg::E; ++e) {
      const uint32_t v0 = mulm(addm(w0[e], bj, md.q), x[e], md.q, md.qinv);
      const uint32_t v1 = mulm(w1[e], x[e], md.q, md.qinv);
      if (mode == 1) {
        a0[e] = red1(v0, md.q);
        a1[e] = red1(v1, md.q);
      } else {
        a0[e] = acc2(a0[e], v0, md.q);
        a1[e] = acc2(a1[e], v1, md.q);
      }
    }
    if (mode == 1) {
      uint32_t* o = out + (size_t)lp * 2 * L * Gg::N;
      storeL<Gg>(DBuf(o + (size_t)j * Gg::N, Gg::N), a0, tid_fresh());
      storeL<Gg>(DBuf(o + (size_t)(L + j) * Gg::N, Gg::N), a1, tid_fresh());
    }
  }
  const int t = tid_fresh();
  if (mode == 0) {
    uint32_t* o = out + (size_t)grp.part * 2 * L * Gg::N;
#pragma unroll
    for (int e = 0; e < Gg::E; ++e) { a0[e] = red1(a0[e], md.q); a1[e] = red1(a1[e], md.q); }
    storeL<Gg>(DBuf(o + (size_t)j * Gg::N, Gg::N), a0, t);
    storeL<Gg>(DBuf(o + (size_t)(L + j) * Gg::N, Gg::N), a1, t);
  }
}

// compression: each output ciphertext is the modular sum of its partials
static __global__ __launch_bounds__(256) void k_compress(DevCtx c, const uint32_t* __restrict__ part,
                                                  const OutDesc* __restrict__ outs, uint32_t nout) {
  const uint32_t n = c.n, L = c.L;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t ctw = (uint64_t)2 * L * n;
  if (gid >= nout * ctw / 4) return;
  const uint64_t word = gid * 4;
  const OutDesc od = outs[word / ctw];
  const uint64_t w = word % ctw;
  const uint32_t q = c.mod[(w / n) % L].q;
  uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (uint32_t g = od.g0; g < od.g1; ++g) {
    const uint4 v = *reinterpret_cast<const uint4*>(part + g * ctw + w);
    s0 = addm(s0, v.x, q); s1 = addm(s1, v.y, q); s2 = addm(s2, v.z, q); s3 = addm(s3, v.w, q);
  }
  *reinterpret_cast<uint4*>(od.y + w) = make_uint4(s0, s1, s2, s3);
}

// descriptors of one request (pairs pair0 .. pair0 + npairs - 1, pair r = i classes + j):
// tiles of B pairs, groups of G consecutive pairs (G | n and G | B, so a group
// never straddles a tile or an output ciphertext), output m = r / n
static __global__ __launch_bounds__(256) void k_plan_single(DevCtx c, const uint32_t* xct, const uint32_t* wpt,
                                                     const uint32_t* dbias, uint32_t K, uint32_t classes,
                                                     uint32_t pair0, uint32_t npairs, uint32_t B, uint32_t G,
                                                     uint32_t* y, PairDesc* pairs, GroupDesc* groups,
                                                     uint32_t ngroups, OutDesc* outs, uint32_t nouts) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t n = c.n, L = c.L, ctw = 2 * L * n;
  if (idx < npairs) {
    const uint64_t r = (uint64_t)pair0 + idx, i = r / classes, jc = r % classes;
    PairDesc d;
    d.xrow = xct + i * K * ctw;
    d.wcls = wpt + jc * K * L * n;
    d.dbias = dbias + jc * L;
    d.gk = nullptr;
    d.K = K;
    d.slot = (uint32_t)(r % n);
    pairs[idx] = d;
  }
  if (idx < ngroups) {
    const uint32_t a = idx * G, t = a / B;
    GroupDesc g;
    g.lp0 = a - t * B;
    g.cnt = min(G, npairs - a);
    g.part = idx;
    g.pad = 0;
    groups[idx] = g;
  }
  if (idx < nouts) {
    const uint32_t gpo = (uint32_t)(n / G);
    OutDesc o;
    o.y = y + (uint64_t)idx * ctw;
    o.g0 = idx * gpo;
    o.g1 = min(o.g0 + gpo, ngroups);
    outs[idx] = o;
  }
}

// ------------------------------------------------------------------ standard baseline
// Standard baseline (one ciphertext per feature, individuals in the slots):
// y[j] = sum_k fct[k] * w[k][j] + Delta(b_j), coefficient-wise over every word
// of the ciphertexts (a scalar product commutes with the transform).
// Block: 64 consecutive words x STD_WAVES waves; wave v sums its slice of the
// features for all 16 classes of a class chunk with 64-bit multiply-adds, the
// slices meet in LDS.  Every fct word is read once; the weights of one feature
// and limb are 16 consecutive words, wave-uniform (scalar loads).
// Accumulator bound: products < q^2 < 2^60; STD_UNROLL = 8 of them on top of a
// folded value < 2^61 + 2^32 stay below 2^64.  fold(x) = hi(x) (2^32 mod q) +
// lo(x) is congruent to x and below 2^61 + 2^32.
constexpr int STD_WAVES = 8, STD_UNROLL = 8, STD_CJ = 16;
static_assert(STD_CJ == 16, "std_class_pad pads to 16 classes");
static __global__ __launch_bounds__(64 * STD_WAVES) void k_std(DevCtx c, const uint32_t* __restrict__ fct,
                                                        const uint32_t* __restrict__ wst,
                                                        const uint32_t* __restrict__ dbias, uint32_t f,
                                                        uint32_t classes, uint32_t* __restrict__ y) {
  __shared__ uint32_t part[STD_WAVES][STD_CJ][64];
  const uint32_t n = c.n, L = c.L;
  const uint32_t cpad = (classes + STD_CJ - 1) / STD_CJ * STD_CJ;
  const uint64_t ctw = (uint64_t)2 * L * n;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t w0 = (uint64_t)blockIdx.x * 64;            // 64 | n: one limb, one polynomial per block
  const uint64_t w = w0 + lane;
  const uint32_t i = (uint32_t)((w0 / n) % L);
  const uint32_t xpoly = (uint32_t)(w0 / ((uint64_t)L * n));
  const Mod md = c.mod[i];
  const uint32_t r1 = red1(redc(md.r2, md.q, md.qinv), md.q);   // 2^32 mod q
  const uint32_t k0 = (uint32_t)((uint64_t)f * wave / STD_WAVES);
  const uint32_t k1 = (uint32_t)((uint64_t)f * (wave + 1) / STD_WAVES);
  for (uint32_t j0 = 0; j0 < cpad; j0 += STD_CJ) {
    uint64_t acc[STD_CJ];
#pragma unroll
    for (int j = 0; j < STD_CJ; ++j) acc[j] = 0;
    uint32_t k = k0;
    for (; k + STD_UNROLL <= k1; k += STD_UNROLL) {
      uint32_t v[STD_UNROLL];
      const uint32_t* src = fct + (uint64_t)k * ctw + w;
#pragma unroll
      for (int u = 0; u < STD_UNROLL; ++u) v[u] = __builtin_nontemporal_load(src + (uint64_t)u * ctw);
#pragma unroll
      for (int u = 0; u < STD_UNROLL; ++u) {
        const uint32_t* wk = wst + ((uint64_t)(k + u) * L + i) * cpad + j0;
#pragma unroll
        for (int j = 0; j < STD_CJ; ++j) acc[j] += (uint64_t)v[u] * wk[j];
      }
#pragma unroll
      for (int j = 0; j < STD_CJ; ++j) acc[j] = fold32(acc[j], r1);
    }
    for (; k < k1; ++k) {
      const uint32_t v = __builtin_nontemporal_load(fct + (uint64_t)k * ctw + w);
      const uint32_t* wk = wst + ((uint64_t)k * L + i) * cpad + j0;
#pragma unroll
      for (int j = 0; j < STD_CJ; ++j) acc[j] = fold32(acc[j] + (uint64_t)v * wk[j], r1);
    }
#pragma unroll
    for (int j = 0; j < STD_CJ; ++j) {
      // two folds: < 2^59.2 < q 2^32, so redc lands in [0, 2q); weights carry R
      part[wave][j][lane] = red1(redc(fold32(fold32(acc[j], r1), r1), md.q, md.qinv), md.q);
    }
    __syncthreads();
    for (uint32_t o = threadIdx.x; o < STD_CJ * 64; o += 64 * STD_WAVES) {
      const uint32_t j = o >> 6, l = o & 63;
      uint32_t sum = 0;
#pragma unroll
      for (int v = 0; v < STD_WAVES; ++v) sum = addm(sum, part[v][j][l], md.q);
      const uint32_t cls = j0 + j;
      if (cls < classes) {
        if (xpoly == 0) sum = addm(sum, dbias[(uint64_t)cls * L + i], md.q);
        y[(uint64_t)cls * ctw + w0 + l] = sum;
      }
    }
    __syncthreads();
  }
}

}  // namespace lrhe
