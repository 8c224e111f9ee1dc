// lrhe_internal.h -- context layout shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lrhe.h"
#include "lrhe_math.h"

#define LRHE_MAXL 15
#define LRHE_MINLOGN 10
#define LRHE_MAXLOGN 15
// the fixed workspace of lrhe_matmul_fast_noalloc (bytes, per device): one
// individual x 16 classes at n = 16384 with 7 data primes needs 81 MiB
#define LRHE_SCRATCH_BYTES (96ull << 20)
#define LRHE_MAX_DEVICES 64

namespace lrhe {

// Plain-old-data view of the context passed by value to every kernel.
// Modulus index convention: 0..L-1 data primes, L = special prime P, L+1 = t.
struct DevCtx {
  uint32_t n, logn, L;
  Mod mod[LRHE_MAXL + 2];
  const uint32_t* tw;        // [(L+2)][n] psi^brv(k) R mod m
  const uint32_t* itw;       // [(L+2)][n] psi^-brv(k) R mod m
  const uint32_t* pos_slot;  // [n] transform index k -> slot j (mod-t transform)
  const uint32_t* slot_exp;  // [n] e_j
  const uint32_t* mask_tab;  // [2n] n^-1 psi_t^-x mod t
  uint32_t t, qmodt;         // t, Q mod t
  uint32_t qdivt_m[LRHE_MAXL];  // floor(Q/t) R mod q_i
  uint32_t pinv_m[LRHE_MAXL];   // P^-1 R mod q_j
  uint32_t hmod[LRHE_MAXL];     // (P-1)/2 mod q_j
};

// Offsets into the fast-matmul workspace for a tile of B pairs.
// classes of the standard baseline's scalar-weight table, padded to its class chunk
inline uint32_t std_class_pad(uint32_t classes) { return (classes + 15) / 16 * 16; }

struct FastWs {
  uint32_t B;                 // pairs per tile
  uint64_t acc_slots;         // pair slots of ACC (see acc_slots)
  uint32_t G;                 // pairs per compression group
  size_t cA, cB, D, ACC, part, desc, total;   // byte offsets, total size
  size_t npart, ndesc_pairs, ndesc_groups, ndesc_outs;
};

// One (input row, class) pair of Algorithm 1, as the kernels see it.
struct PairDesc {
  const uint32_t* xrow;   // the K ciphertexts of the row, [K][2][L][n]
  const uint32_t* wcls;   // the K plaintexts of the class, [K][L][n] (Montgomery)
  const uint32_t* dbias;  // Delta(b_class) mod q_i, [L]
  const uint32_t* gk;     // Galois keys of the pair's client, or null for the launch's default keys
  uint32_t K;             // chunks
  uint32_t slot;          // one-hot slot l = r mod n of the pair
};
// A run of consecutive pairs of one tile that land in one output ciphertext;
// their masked ciphertexts are summed into partial `part`.
struct GroupDesc {
  uint32_t lp0, cnt, part, pad;
};
// An output ciphertext: the modular sum of partials [g0, g1).
struct OutDesc {
  uint32_t* y;
  uint32_t g0, g1;
};

}  // namespace lrhe

namespace lrhe {
// Launch choices of the fast-matmul kernels (set by lrhe_tune_set / lrhe_autotune_fast):
// log2 of the residues per thread of each transform kernel, pairs per tile.
#ifndef LRHE_MAC_NMODES
#define LRHE_MAC_NMODES 8   // k_ks_mac variants behind the "mac_mode" tuning key
#endif
// the variant that splits each key-switch item's digits over two workgroups
// (latency of small tiles); it needs two accumulator slots per tile pair, so
// it is a choice of the small-tile class only
#define LRHE_MAC_MODE_HALF 4
#define LRHE_MAC_MODE_SPLIT 6   // special-prime items, then data-modulus items with part 3
#define LRHE_MAC_MODE_SPLIT64 7   // as 6, the data-modulus items double-buffered with 64-bit inner products
// Launch choices of the transform kernels (none changes a result bit).
struct Knobs {
  int le_intt = 5, le_mac = 5, le_moddown = 5, le_mask = 5;
  int mac_mode = 0;   // variant of k_ks_mac, 0 .. LRHE_MAC_NMODES - 1
  // residues per thread of the special-prime launch of the split variant
  // (le_mac sets its data-modulus launch)
  int le_mac_p = 5;
  // k_ks_moddown also writes the next step's digits (no k_ks_intt after the
  // first step); not with the digit-halves variant, whose division by P is
  // split.  Off by default: at 512 x 40,000 the extra inverse transform costs
  // k_ks_moddown more (3.51 -> 4.89 ms) than k_ks_intt takes (1.2 ms)
  int fuse_intt = 0;
};
// Tiles below small_below pairs (latency-bound: fewer workgroups than the chip
// holds) and larger tiles (throughput-bound) keep separate choices.
struct Tune {
  Knobs large;
  Knobs small{5, 5, 5, 5, 3, 5};
  uint32_t tile = 4096;
  uint32_t small_below = 64;
  const Knobs& knobs(uint64_t tile_pairs) const { return tile_pairs < small_below ? small : large; }
  Knobs& knobs(uint64_t tile_pairs) { return tile_pairs < small_below ? small : large; }
};
}  // namespace lrhe

struct lrhe_ctx {
  int device = 0;
  lrhe::Tune tune;
  uint32_t n = 0, logn = 0, L = 0, ngal = 0, t = 0, P = 0;
  std::vector<uint32_t> q;        // L data primes followed by P
  std::vector<uint32_t> gal;      // Galois elements of the rotate-and-sum
  std::vector<lrhe::Mod> mods;    // L + 2 entries
  std::vector<uint32_t> h_tw, h_itw;   // host copies of the tables, [(L+2)][n]
  std::vector<uint32_t> slot_pos, pos_slot, slot_exp, mask_tab;
  // device tables
  uint32_t* d_tw = nullptr;
  uint32_t* d_itw = nullptr;
  uint32_t* d_pos_slot = nullptr;
  uint32_t* d_slot_exp = nullptr;
  uint32_t* d_mask_tab = nullptr;
  lrhe::DevCtx dc{};
  // big-integer constants for decryption, computed at creation
  std::vector<uint32_t> dec_I;       // floor(t y_j / q_j) mod t
  std::vector<uint32_t> dec_R;       // t y_j mod q_j, y_j = (Q/q_j)^-1 mod q_j
  std::vector<double> dec_Rf;        // dec_R / q_j
  std::vector<std::vector<uint32_t>> Qhat;  // Q / q_j as little-endian 32-bit limbs
  std::vector<uint32_t> Qbig;        // Q
  double log2Q = 0;
};

struct lrhe_sk {
  uint32_t n = 0, L = 0;
  std::vector<int8_t> s;        // ternary coefficients
  std::vector<uint32_t> S;      // [L][n] evaluation form, canonical
  std::vector<uint32_t> Sm;     // the same in Montgomery form (S R mod q_j), for decryption
};

struct lrhe_pk {
  uint32_t* d = nullptr;        // [2][L][n] evaluation form, Montgomery (x R mod q)
  std::vector<uint32_t> h;      // host copy, canonical evaluation form
};

struct lrhe_gk {
  uint32_t* d = nullptr;        // [ngal][L+1 moduli r][L digits i][2][n] evaluation form, Montgomery
  size_t words = 0;
  std::vector<uint32_t> h;      // host copy, canonical evaluation form, same layout
};

struct lrhe_model {
  uint32_t f = 0, classes = 0, K = 0;
  uint32_t* wpt = nullptr;      // [classes][K][L][n] evaluation form, Montgomery
  uint32_t* wsc = nullptr;      // [f][L][std_class_pad(classes)] centred scalar weights, Montgomery
  uint32_t* dbias = nullptr;    // [classes][L] Delta(b_j) mod q_i
};

namespace lrhe {
// Sets the thread-local message returned by lrhe_last_error; returns code.
int fail(int code, const char* fmt, ...);

// Every device allocation of the library goes through these two, so that an
// armed allocation fault (environment variable LRHE_FAULT_ALLOC, or
// lrhe_fault_inject) fails the chosen one with hipErrorOutOfMemory.
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t dev_malloc_async(void** p, size_t bytes, hipStream_t s);

// Records HIP events around a kernel launch on its stream while timing is
// enabled (lrhe_prof_enable); a no-op otherwise.
struct ProfScope {
  ProfScope(hipStream_t s, const char* name);
  ~ProfScope();
  hipStream_t s_;
  const char* name_;
  void* a_ = nullptr;
  void* b_ = nullptr;
};

// kernel launchers (kernels.hip); all return a hipError_t
hipError_t launch_ntt(const lrhe_ctx* c, uint32_t* data, uint64_t npolys, uint32_t nmod, uint32_t mod0, bool inverse,
                      hipStream_t s);
hipError_t launch_encrypt(const lrhe_ctx* c, const uint32_t* pk_d, const int64_t* X, uint32_t rows, uint32_t f,
                          bool cols, uint64_t seed, uint64_t id0, uint32_t* ct_out, void* ws, hipStream_t s);
size_t encrypt_ws_bytes(const lrhe_ctx* c, uint64_t nct);
hipError_t launch_model_encode(const lrhe_ctx* c, const int64_t* W, uint32_t f, uint32_t classes, uint32_t* wpt,
                               uint32_t* wsc, hipStream_t s);
// Pair slots of the key-switch accumulator buffer for tiles of at most B pairs:
// one per pair, two for the tiles of the small class (the digit-halves variant
// needs ACC and ACC2); a large job's last tile, if small, fits its two slots per
// pair in the B slots whenever it has at most B/2 pairs, otherwise the buffer
// grows.
inline uint64_t acc_slots(const lrhe_ctx* c, uint64_t B) {
  const uint64_t small_max = c->tune.small_below > 0 ? c->tune.small_below - 1 : 0;
  return std::max<uint64_t>(B, 2 * std::min<uint64_t>(B, small_max));
}
FastWs fast_ws_layout(const lrhe_ctx* c, uint32_t npairs, uint32_t classes);
hipError_t launch_fast(const lrhe_ctx* c, const uint32_t* gk_d, const lrhe_model* m, const uint32_t* xct,
                       uint32_t rows, uint32_t pair0, uint32_t npairs, int stage, uint32_t* out, void* ws,
                       const FastWs& lay, hipStream_t s);
// Descriptor-driven Algorithm 1 over pairs[0, npairs) (device arrays): tiles of B
// pairs; groups[tile_g0[t] .. tile_g0[t+1]) belong to tile t; stage as in
// lrhe_matmul_fast_pairs (-1 = full: mask into partials, then compress outs).
// per-ring-dimension launchers (ks_step.hip, one object per log2 n): one
// rotate-and-accumulate step (k_ks_intt, k_ks_mac, k_ks_moddown) on a tile,
// and the bias + mask + group sums of a tile
template <int LN>
hipError_t launch_ks_step(const lrhe_ctx* c, const Knobs& kn, const PairDesc* tp, const uint32_t* gk_d, uint32_t Bt,
                          uint32_t gi, const uint32_t* cur, uint32_t* D, uint32_t* ACC, uint64_t acc_slots,
                          uint32_t* nxt, bool d_ready, bool d_next, hipStream_t s);
template <int LN>
hipError_t launch_mask_step(const lrhe_ctx* c, const Knobs& kn, const uint32_t* cur, const PairDesc* tp,
                            const GroupDesc* tg, uint32_t ngt, int mode, uint32_t* dst, hipStream_t s);
hipError_t launch_plan(const lrhe_ctx* c, const uint32_t* gk_d, const PairDesc* pairs, uint32_t npairs,
                       const GroupDesc* groups, const uint32_t* tile_g0, uint32_t B, const OutDesc* outs,
                       uint32_t nouts, int stage, uint32_t* out, uint32_t* cA, uint32_t* cB, uint32_t* D,
                       uint32_t* ACC, uint64_t acc_slots, uint32_t* part, hipStream_t s);
hipError_t launch_standard(const lrhe_ctx* c, const lrhe_model* m, const uint32_t* fct, uint32_t* y_out,
                           hipStream_t s);
// host-side key and transform helpers shared by keygen and the wire format
// (host.cpp): a limb's host transform (inverse: evaluation -> coefficients),
// a secret key from its ternary coefficients, and the device copies of keys
// whose host evaluation form is filled in
void host_transform_limb(const lrhe_ctx* c, int mi, uint32_t* a, bool inverse);
lrhe_sk* make_sk(const lrhe_ctx* c, const int32_t* s);
hipError_t upload_pk(const lrhe_ctx* c, lrhe_pk* pk);
hipError_t upload_gk(const lrhe_ctx* c, lrhe_gk* gk);
int fail(int code, const char* fmt, ...);

// device address of the fixed scratch array on a device: resolved once per
// device (with that device current) by scratch_resolve, nullptr before
hipError_t scratch_resolve(int device);
void* scratch_ptr(int device);
}  // namespace lrhe
