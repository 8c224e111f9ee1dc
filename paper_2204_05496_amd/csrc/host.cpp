// host.cpp -- host runtime of the encrypted logistic-regression library:
// parameter validation, root/twiddle/RNS tables, key generation (client),
// exact decryption (client) and the C ABI entry points of include/lrhe.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lrhe_internal.h"

using namespace lrhe;

extern "C" void lrhe_prof_enable(int on);
extern "C" void lrhe_prof_reset(void);
extern "C" int lrhe_prof_get(const char* kernel, uint64_t* launches, double* total_ms);

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;
namespace lrhe {
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace lrhe
#define NEED_DEVICE(c) \
  do { if ((c)->device < 0) return fail(LRHE_EDEVICE, "host-only context (device < 0) has no GPU"); } while (0)
#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(LRHE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char* lrhe_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ allocation fault injection
// Countdown to a failing device allocation: k > 0 means the k-th allocation
// from now fails (then the countdown is spent); 0 means disarmed.  The initial
// value comes from the environment variable LRHE_FAULT_ALLOC (read once).
static std::atomic<int64_t> g_fault{0};
static std::once_flag g_fault_env;
static void fault_env_init() {
  std::call_once(g_fault_env, [] {
    if (const char* v = std::getenv("LRHE_FAULT_ALLOC")) {
      const long long k = std::atoll(v);
      if (k > 0) g_fault.store(k);
    }
  });
}
static bool fault_fires() {
  fault_env_init();
  int64_t k = g_fault.load();
  while (k > 0) {
    if (g_fault.compare_exchange_weak(k, k - 1)) return k == 1;
  }
  return false;
}
namespace lrhe {
hipError_t dev_malloc(void** p, size_t bytes) {
  *p = nullptr;
  if (fault_fires()) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}
hipError_t dev_malloc_async(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (fault_fires()) return hipErrorOutOfMemory;
  return hipMallocAsync(p, bytes, s);
}
}  // namespace lrhe
extern "C" int64_t lrhe_fault_inject(int64_t k) {
  fault_env_init();
  return k >= 0 ? g_fault.exchange(k) : g_fault.load();
}

// ------------------------------------------------------------------ number theory (host)
static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }
static uint64_t powmod64(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, b, m);
    b = mulmod64(b, b, m);
    e >>= 1;
  }
  return r;
}
static bool is_prime(uint64_t p) {
  if (p < 2) return false;
  for (uint64_t d : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull}) {
    if (p % d == 0) return p == d;
  }
  // deterministic Miller-Rabin for 64-bit inputs
  uint64_t d = p - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
    uint64_t x = powmod64(a, d, p);
    if (x == 1 || x == p - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod64(x, x, p);
      if (x == p - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}
static uint64_t min_generator(uint64_t p) {
  std::vector<uint64_t> fac;
  uint64_t m = p - 1;
  for (uint64_t d = 2; d * d <= m; ++d)
    if (m % d == 0) {
      fac.push_back(d);
      while (m % d == 0) m /= d;
    }
  if (m > 1) fac.push_back(m);
  for (uint64_t g = 2; g < p; ++g) {
    bool ok = true;
    for (uint64_t f : fac)
      if (powmod64(g, (p - 1) / f, p) == 1) { ok = false; break; }
    if (ok) return g;
  }
  return 0;
}
static uint32_t inv_mod(uint64_t a, uint64_t p) { return (uint32_t)powmod64(a % p, p - 2, p); }

static Mod make_mod(uint32_t q, uint32_t n) {
  Mod m;
  m.q = q;
  uint32_t inv = 1;   // q^-1 mod 2^32 by Newton iteration
  for (int i = 0; i < 5; ++i) inv *= 2 - q * inv;
  m.qinv = (uint32_t)(0u - inv);
  const uint64_t R = (1ull << 32) % q;
  m.r2 = (uint32_t)mulmod64(R, R, q);
  m.ninv_m = (uint32_t)mulmod64(inv_mod(n, q), R, q);
  return m;
}

// maximum log2(Q P) for 128-bit security with a ternary secret (HE standard tables)
static double security_bound_bits(uint32_t n) {
  switch (n) {
    case 1024: return 27; case 2048: return 54; case 4096: return 109;
    case 8192: return 218; case 16384: return 438; case 32768: return 881;
  }
  return 0;
}

// ------------------------------------------------------------------ host transforms
// The host runs the very same pass functions as the kernels, one emulated
// thread at a time, with the exchange done through a plain array.
template <int LOGN, bool STRICT = false>
static void host_ntt_t(uint32_t* a, const uint32_t* tw, const Mod& m, bool inverse) {
  using G = Geom<LOGN, 5>;
  std::vector<uint32_t> X((size_t)G::N), tmp((size_t)G::N);
  auto load = [&](int p) {
    for (int t = 0; t < G::T; ++t)
      for (int e = 0; e < G::E; ++e) X[(size_t)t * G::E + e] = tmp[G::idx(p, t, e)];
  };
  auto store = [&](int p) {
    for (int t = 0; t < G::T; ++t)
      for (int e = 0; e < G::E; ++e) tmp[G::idx(p, t, e)] = X[(size_t)t * G::E + e];
  };
  std::copy(a, a + G::N, tmp.begin());
  if (STRICT)   // canonical input
    for (int i = 0; i < G::N; ++i) tmp[i] %= m.q;
  if (!inverse) {
    for (int p = 0; p < G::NPASS; ++p) {
      load(p);
      for (int t = 0; t < G::T; ++t) fwd_pass<G, false, STRICT>(p, t, &X[(size_t)t * G::E], tw, m.q, m.qinv);
      store(p);
    }
    for (int i = 0; i < G::N; ++i) a[i] = STRICT ? tmp[i] : red2(tmp[i], m.q);
  } else {
    for (int p = G::NPASS - 1; p >= 0; --p) {
      load(p);
      for (int t = 0; t < G::T; ++t) inv_pass<G, false, STRICT>(p, t, &X[(size_t)t * G::E], tw, m.q, m.qinv);
      store(p);
    }
    for (int i = 0; i < G::N; ++i) a[i] = red1(mulm(tmp[i], m.ninv_m, m.q, m.qinv), m.q);
  }
}
// The same transforms as plain in-place loops (forward: Cooley-Tukey with
// psi^brv(m + i) for block i of a stage with m blocks; inverse: Gentleman-Sande
// with psi^-brv(m + i), then n^-1).  Both produce the canonical result, so they
// agree with the pass-structured version bit for bit; this one is several times
// faster on the host and serves keygen and decryption.
static void host_ntt_plain(const lrhe_ctx* c, int mi, uint32_t* a, bool inverse) {
  const uint32_t n = c->n;
  const Mod& md = c->mods[mi];
  const uint32_t q = md.q;
  const uint32_t* tb = (inverse ? c->h_itw.data() : c->h_tw.data()) + (size_t)mi * n;
  if (!inverse) {
    for (uint32_t i = 0; i < n; ++i) a[i] = red2(a[i], q);
    for (uint32_t m = 1, h = n / 2; m < n; m <<= 1, h >>= 1)
      for (uint32_t i = 0; i < m; ++i) {
        const uint32_t w = tb[m + i];
        uint32_t* x = a + (size_t)2 * i * h;
        for (uint32_t j = 0; j < h; ++j) {
          const uint32_t u = x[j], v = red1(mulm(x[j + h], w, q, md.qinv), q);
          x[j] = addm(u, v, q);
          x[j + h] = subm(u, v, q);
        }
      }
  } else {
    for (uint32_t i = 0; i < n; ++i) a[i] = red2(a[i], q);
    for (uint32_t m = n / 2, h = 1; m >= 1; m >>= 1, h <<= 1)
      for (uint32_t i = 0; i < m; ++i) {
        const uint32_t w = tb[m + i];
        uint32_t* x = a + (size_t)2 * i * h;
        for (uint32_t j = 0; j < h; ++j) {
          const uint32_t u = x[j], v = x[j + h];
          x[j] = addm(u, v, q);
          x[j + h] = red1(mulm(subm(u, v, q), w, q, md.qinv), q);
        }
      }
    for (uint32_t i = 0; i < n; ++i) a[i] = red1(mulm(a[i], md.ninv_m, q, md.qinv), q);
  }
}

// forward: natural coefficients (< 4q) -> evaluations, bit-reversed order; inverse: back
static void host_ntt(const lrhe_ctx* c, int mi, uint32_t* a, bool inverse) {
  host_ntt_plain(c, mi, a, inverse);
}
// the forward transform of host_ntt_plain with the butterflies of each stage
// shared among the OpenMP threads (one parallel region, a barrier per stage)
static void host_ntt_fwd_threads(const lrhe_ctx* c, int mi, uint32_t* a) {
  const uint32_t n = c->n;
  const Mod& md = c->mods[mi];
  const uint32_t q = md.q;
  const uint32_t* tb = c->h_tw.data() + (size_t)mi * n;
#pragma omp parallel
  {
#pragma omp for schedule(static)
    for (int i = 0; i < (int)n; ++i) a[i] = red2(a[i], q);
    for (uint32_t m = 1, lh = c->logn - 1; m < n; m <<= 1, --lh) {
      const uint32_t h = 1u << lh;
      // butterfly b of the stage: block i = b / h, offset j = b % h
#pragma omp for schedule(static)
      for (int b = 0; b < (int)(n / 2); ++b) {
        const uint32_t i = (uint32_t)b >> lh, j = (uint32_t)b & (h - 1);
        uint32_t* x = a + (size_t)2 * i * h;
        const uint32_t u = x[j], v = red1(mulm(x[j + h], tb[m + i], q, md.qinv), q);
        x[j] = addm(u, v, q);
        x[j + h] = subm(u, v, q);
      }
    }
  }
}
// the pass-structured version: the kernels' own pass arithmetic, emulated
static void host_ntt_passes(const lrhe_ctx* c, int mi, uint32_t* a, bool inverse) {
  const uint32_t* tb = (inverse ? c->h_itw.data() : c->h_tw.data()) + (size_t)mi * c->n;
  const Mod& m = c->mods[mi];
  // moduli of 2^30 and above (only t can be one) run the canonical-residue passes
  const bool strict = m.q >= (1u << 30);
#define LRHE_HOST_NTT_CASE(LN) \
  case LN: strict ? host_ntt_t<LN, true>(a, tb, m, inverse) : host_ntt_t<LN>(a, tb, m, inverse); break;
  switch (c->logn) {
    LRHE_HOST_NTT_CASE(10) LRHE_HOST_NTT_CASE(11) LRHE_HOST_NTT_CASE(12)
    LRHE_HOST_NTT_CASE(13) LRHE_HOST_NTT_CASE(14) LRHE_HOST_NTT_CASE(15)
  }
#undef LRHE_HOST_NTT_CASE
}

// ------------------------------------------------------------------ context
static bool le_valid(uint32_t logn, int le);

extern "C" int lrhe_ctx_create(const lrhe_params* p, int device, lrhe_ctx** out) {
  if (!p || !out) return fail(LRHE_EINVAL, "null argument");
  *out = nullptr;
  const uint32_t n = p->n;
  if (n < (1u << LRHE_MINLOGN) || n > (1u << LRHE_MAXLOGN) || (n & (n - 1)))
    return fail(LRHE_EPARAM, "n = %u: must be a power of two in [%u, %u]", n, 1u << LRHE_MINLOGN, 1u << LRHE_MAXLOGN);
  if (p->L < 1 || p->L > LRHE_MAXL) return fail(LRHE_EPARAM, "L = %u: must be in [1, %d]", p->L, LRHE_MAXL);
  if (!p->q) return fail(LRHE_EINVAL, "q is null");
  std::vector<uint32_t> qs(p->q, p->q + p->L);
  qs.push_back(p->P);
  double logqp = 0;
  for (size_t i = 0; i < qs.size(); ++i) {
    const uint32_t q = qs[i];
    if (q <= (1u << 28) || q >= (1u << 30))
      return fail(LRHE_EPARAM, "modulus %u outside (2^28, 2^30)", q);
    if (!is_prime(q)) return fail(LRHE_EPARAM, "modulus %u is not prime", q);
    if ((q - 1) % (2 * n)) return fail(LRHE_EPARAM, "modulus %u is not 1 mod 2n", q);
    for (size_t k = 0; k < i; ++k)
      if (qs[k] == q) return fail(LRHE_EPARAM, "modulus %u repeated", q);
    logqp += std::log2((double)q);
  }
  if (p->t < 3 || p->t >= (1u << 31) || !is_prime(p->t) || (p->t - 1) % (2 * n))
    return fail(LRHE_EPARAM, "t = %u: must be a prime < 2^31 that is 1 mod 2n", p->t);
  for (uint32_t q : qs) {
    if (q == p->t) return fail(LRHE_EPARAM, "t equals a ciphertext modulus");
    // the centred lift of a residue mod t into q, (t-1)/2 or v - t + q, must be a residue mod q
    if ((uint64_t)p->t >= 2ull * q) return fail(LRHE_EPARAM, "t = %u is not below 2 q for modulus %u", p->t, q);
  }
  if (!p->allow_insecure && logqp > security_bound_bits(n))
    return fail(LRHE_EPARAM, "log2(Q P) = %.1f exceeds the 128-bit bound %.0f for n = %u (set allow_insecure)",
                logqp, security_bound_bits(n), n);

  auto* c = new lrhe_ctx();
  c->device = device;
  c->n = n;
  while ((1u << c->logn) < n) c->logn++;
  c->L = p->L;
  c->q = qs;
  c->P = p->P;
  c->t = p->t;
  const uint32_t L = c->L;
  // Galois elements: rotations by n/4, ..., 1 within the rows, then the row swap
  for (uint32_t s = n / 4; s >= 1; s /= 2) c->gal.push_back((uint32_t)powmod64(3, s, 2 * n));
  c->gal.push_back(2 * n - 1);
  c->ngal = (uint32_t)c->gal.size();
  // default launch choices for large tiles, as measured on 512 x 40,000 at
  // n = 16384 (64 residues per thread for the inner-product and mod-down
  // kernels, 16 for the mask, where the ring dimension allows them)
  c->tune.large.le_intt = 5;
  c->tune.large.le_mac = le_valid(c->logn, 6) ? 6 : 5;
  c->tune.large.le_moddown = le_valid(c->logn, 6) ? 6 : 5;
  c->tune.large.le_mask = le_valid(c->logn, 4) ? 4 : 5;
  // the split variant: special-prime items at 32 residues per thread, then the
  // data-modulus items (with the division by P) at 64
  c->tune.large.mac_mode = LRHE_MAC_MODE_SPLIT;
  c->tune.large.le_mac_p = 5;
  // and for small tiles, as measured on a single inference (16 pairs): the
  // digit-halves variant at 16 residues per thread
  c->tune.small.le_intt = 5;
  c->tune.small.le_mac = le_valid(c->logn, 4) ? 4 : 5;
  c->tune.small.le_moddown = le_valid(c->logn, 4) ? 4 : 5;
  c->tune.small.le_mask = le_valid(c->logn, 4) ? 4 : 5;
  c->tune.small.mac_mode = LRHE_MAC_MODE_HALF;
  c->tune.small.le_mac_p = 5;
  // moduli and twiddle tables (data primes, P, t)
  std::vector<uint32_t> all = qs;
  all.push_back(p->t);
  c->h_tw.assign((size_t)(L + 2) * n, 0);
  c->h_itw.assign((size_t)(L + 2) * n, 0);
  for (uint32_t mi = 0; mi < L + 2; ++mi) {
    const uint32_t q = all[mi];
    c->mods.push_back(make_mod(q, n));
    const uint64_t g = min_generator(q);
    const uint64_t psi = powmod64(g, (q - 1) / (2 * n), q);
    const uint64_t ipsi = inv_mod(psi, q);
    const uint64_t R = (1ull << 32) % q;
    for (uint32_t k = 0; k < n; ++k) {
      const uint32_t e = brv(k, (int)c->logn);
      c->h_tw[(size_t)mi * n + k] = (uint32_t)mulmod64(powmod64(psi, e, q), R, q);
      c->h_itw[(size_t)mi * n + k] = (uint32_t)mulmod64(powmod64(ipsi, e, q), R, q);
    }
  }
  // slot layout mod t: slot j <-> psi_t^(e_j); in the bit-reversed transform the
  // evaluation at psi_t^(2m+1) sits at index brv(m)
  const uint32_t t = p->t;
  const uint64_t psit = powmod64(min_generator(t), (t - 1) / (2 * n), t);
  c->slot_exp.resize(n);
  c->slot_pos.resize(n);
  c->pos_slot.resize(n);
  uint64_t e = 1;
  for (uint32_t j = 0; j < n / 2; ++j) {
    c->slot_exp[j] = (uint32_t)e;
    c->slot_exp[n / 2 + j] = (uint32_t)(2 * n - e);
    e = e * 3 % (2 * n);
  }
  for (uint32_t j = 0; j < n; ++j) {
    const uint32_t k = brv((c->slot_exp[j] - 1) / 2, (int)c->logn);
    c->slot_pos[j] = k;
    c->pos_slot[k] = j;
  }
  // one-hot mask coefficients: mu_{l,k} = n^-1 psi_t^-(e_l k); table over x = e_l k mod 2n
  c->mask_tab.resize(2 * n);
  const uint64_t ninv_t = inv_mod(n, t), ipsit = inv_mod(psit, t);
  for (uint32_t x = 0; x < 2 * n; ++x) c->mask_tab[x] = (uint32_t)mulmod64(ninv_t, powmod64(ipsit, x, t), t);
  // BFV constants
  DevCtx& d = c->dc;
  d.n = n;
  d.logn = c->logn;
  d.L = L;
  for (uint32_t mi = 0; mi < L + 2; ++mi) d.mod[mi] = c->mods[mi];
  d.t = t;
  uint64_t qmt = 1;
  for (uint32_t i = 0; i < L; ++i) qmt = qmt * (qs[i] % t) % t;
  d.qmodt = (uint32_t)qmt;
  for (uint32_t i = 0; i < L; ++i) {
    const uint64_t q = qs[i], R = (1ull << 32) % q;
    // floor(Q/t) mod q_i = -(Q mod t) t^-1 mod q_i (Q = 0 mod q_i)
    const uint64_t qd = mulmod64((q - qmt % q) % q, inv_mod(t, q), q);
    d.qdivt_m[i] = (uint32_t)mulmod64(qd, R, q);
    d.pinv_m[i] = (uint32_t)mulmod64(inv_mod(p->P, q), R, q);
    d.hmod[i] = (uint32_t)(((uint64_t)(p->P - 1) / 2) % q);
  }
  // decryption constants: y_j = (Q/q_j)^-1 mod q_j, t y_j = I_j q_j + R_j
  {
    std::vector<uint32_t> Q = {1};
    auto mul_small = [](std::vector<uint32_t>& a, uint32_t m) {
      uint64_t carry = 0;
      for (auto& w : a) {
        uint64_t v = (uint64_t)w * m + carry;
        w = (uint32_t)v;
        carry = v >> 32;
      }
      if (carry) a.push_back((uint32_t)carry);
    };
    for (uint32_t i = 0; i < L; ++i) mul_small(Q, qs[i]);
    c->Qbig = Q;
    c->log2Q = 0;
    for (uint32_t i = 0; i < L; ++i) c->log2Q += std::log2((double)qs[i]);
    for (uint32_t j = 0; j < L; ++j) {
      std::vector<uint32_t> Qh = {1};
      uint64_t qh_mod = 1;
      for (uint32_t i = 0; i < L; ++i)
        if (i != j) {
          mul_small(Qh, qs[i]);
          qh_mod = qh_mod * qs[i] % qs[j];
        }
      c->Qhat.push_back(Qh);
      const uint64_t y = inv_mod(qh_mod, qs[j]);
      const uint64_t ty = (uint64_t)t * y;
      c->dec_I.push_back((uint32_t)((ty / qs[j]) % t));
      c->dec_R.push_back((uint32_t)(ty % qs[j]));
      c->dec_Rf.push_back((double)(ty % qs[j]) / (double)qs[j]);
    }
  }
  *out = c;
  if (device < 0) return LRHE_OK;   // host-only context: client-side host code, no device tables
  *out = nullptr;
  // upload
  hipError_t err = hipSetDevice(device);
  if (err != hipSuccess) { delete c; return fail(LRHE_EDEVICE, "hipSetDevice(%d): %s", device, hipGetErrorString(err)); }
  // the device address of the non-allocating path's fixed scratch, once per device
  err = scratch_resolve(device);
  if (err != hipSuccess) { delete c; return fail(LRHE_EDEVICE, "scratch on device %d: %s", device, hipGetErrorString(err)); }
  auto up = [&](uint32_t** dst, const std::vector<uint32_t>& src) -> hipError_t {
    hipError_t e2 = dev_malloc((void**)dst, src.size() * 4);
    if (e2 != hipSuccess) return e2;
    return hipMemcpy(*dst, src.data(), src.size() * 4, hipMemcpyHostToDevice);
  };
  if ((err = up(&c->d_tw, c->h_tw)) != hipSuccess || (err = up(&c->d_itw, c->h_itw)) != hipSuccess ||
      (err = up(&c->d_pos_slot, c->pos_slot)) != hipSuccess || (err = up(&c->d_slot_exp, c->slot_exp)) != hipSuccess ||
      (err = up(&c->d_mask_tab, c->mask_tab)) != hipSuccess) {
    lrhe_ctx_destroy(c);
    return fail(LRHE_EDEVICE, "context upload: %s", hipGetErrorString(err));
  }
  d.tw = c->d_tw;
  d.itw = c->d_itw;
  d.pos_slot = c->d_pos_slot;
  d.slot_exp = c->d_slot_exp;
  d.mask_tab = c->d_mask_tab;
  *out = c;
  return LRHE_OK;
}

extern "C" void lrhe_ctx_destroy(lrhe_ctx* c) {
  if (!c) return;
  if (c->device < 0) {
    delete c;
    return;
  }
  (void)hipSetDevice(c->device);
  (void)hipFree(c->d_tw);
  (void)hipFree(c->d_itw);
  (void)hipFree(c->d_pos_slot);
  (void)hipFree(c->d_slot_exp);
  (void)hipFree(c->d_mask_tab);
  delete c;
}

extern "C" int lrhe_ctx_info(const lrhe_ctx* c, uint32_t* n, uint32_t* L, uint32_t* ngal, uint64_t* ct_words) {
  if (!c) return fail(LRHE_EINVAL, "null context");
  if (n) *n = c->n;
  if (L) *L = c->L;
  if (ngal) *ngal = c->ngal;
  if (ct_words) *ct_words = (uint64_t)2 * c->L * c->n;
  return LRHE_OK;
}

extern "C" int lrhe_galois_element(const lrhe_ctx* c, uint32_t i, uint32_t* g) {
  if (!c || !g || i >= c->ngal) return fail(LRHE_EINVAL, "bad Galois index");
  *g = c->gal[i];
  return LRHE_OK;
}

// ------------------------------------------------------------------ keys (client)
struct Stream {
  uint64_t seed;
  uint32_t kind;
  uint64_t id;
  uint32_t cur = 0xffffffffu, blk[16];
  uint32_t word(uint64_t w) {
    const uint32_t b = (uint32_t)(w >> 4);
    if (b != cur) {
      chacha20(seed, kind, id, b, blk);
      cur = b;
    }
    return blk[w & 15];
  }
};
static void sample_ternary(uint64_t seed, uint32_t kind, uint64_t id, uint32_t n, std::vector<int32_t>& out) {
  Stream S{seed, kind, id};
  out.resize(n);
  for (uint32_t k = 0; k < n; ++k) out[k] = ternary_of(S.word(k));
}
static void sample_cbd(uint64_t seed, uint32_t kind, uint64_t id, uint32_t n, std::vector<int32_t>& out) {
  Stream S{seed, kind, id};
  out.resize(n);
  for (uint32_t k = 0; k < n; ++k) out[k] = cbd21_of(S.word(2ull * k), S.word(2ull * k + 1));
}
static void sample_uniform(uint64_t seed, uint32_t kind, uint64_t id, uint32_t m, uint32_t n, uint32_t* out) {
  Stream S{seed, kind, id};
  for (uint32_t k = 0; k < n; ++k) out[k] = uniform_of(S.word(2ull * k), S.word(2ull * k + 1), m);
}
static uint32_t smod(int64_t v, uint32_t q) {
  int64_t r = v % (int64_t)q;
  return (uint32_t)(r < 0 ? r + q : r);
}

// sigma_g on integer coefficients: a(X) -> a(X^g) mod X^n + 1
static void automorph_int(const std::vector<int32_t>& a, uint32_t g, uint32_t n, std::vector<int32_t>& out) {
  out.assign(n, 0);
  for (uint32_t k = 0; k < n; ++k) {
    const uint64_t idx = (uint64_t)g * k % (2 * n);
    if (idx < n) out[idx] = a[k];
    else out[idx - n] = -a[k];
  }
}

namespace lrhe {
void host_transform_limb(const lrhe_ctx* c, int mi, uint32_t* a, bool inverse) { host_ntt(c, mi, a, inverse); }

// s in evaluation form for every modulus (data primes and P), [L+1][n]
static std::vector<uint32_t> secret_eval(const lrhe_ctx* c, const int32_t* s) {
  const uint32_t n = c->n, L = c->L;
  std::vector<uint32_t> S((size_t)(L + 1) * n);
  for (uint32_t r = 0; r <= L; ++r) {
    uint32_t* Sr = &S[(size_t)r * n];
    for (uint32_t k = 0; k < n; ++k) Sr[k] = smod(s[k], c->q[r]);
    host_ntt(c, (int)r, Sr, false);
  }
  return S;
}

lrhe_sk* make_sk(const lrhe_ctx* c, const int32_t* s) {
  const uint32_t n = c->n, L = c->L;
  const std::vector<uint32_t> S = secret_eval(c, s);
  auto* sk = new lrhe_sk();
  sk->n = n;
  sk->L = L;
  sk->s.assign(s, s + n);
  sk->S.assign(S.begin(), S.begin() + (size_t)L * n);
  sk->Sm.resize((size_t)L * n);
  for (uint32_t j = 0; j < L; ++j)
    for (uint32_t k = 0; k < n; ++k) sk->Sm[(size_t)j * n + k] = to_mont(sk->S[(size_t)j * n + k], c->mods[j]);
  return sk;
}

// device copy of a public key from its host evaluation form (Montgomery words)
hipError_t upload_pk(const lrhe_ctx* c, lrhe_pk* pk) {
  if (c->device < 0) return hipSuccess;
  const uint32_t n = c->n, L = c->L;
  hipError_t err = hipSetDevice(c->device);
  if (err == hipSuccess) err = dev_malloc((void**)&pk->d, pk->h.size() * 4);
  if (err != hipSuccess) return err;
  std::vector<uint32_t> mont(pk->h.size());
  for (size_t x = 0; x < mont.size(); ++x) mont[x] = to_mont(pk->h[x], c->mods[(x / n) % L]);
  return hipMemcpy(pk->d, mont.data(), mont.size() * 4, hipMemcpyHostToDevice);
}

// device copy of the Galois keys from their host evaluation form (layout [g][r][i][x][n])
hipError_t upload_gk(const lrhe_ctx* c, lrhe_gk* gk) {
  if (c->device < 0) return hipSuccess;
  const uint32_t n = c->n, L = c->L;
  std::vector<uint32_t> mont(gk->words);
  for (size_t x = 0; x < mont.size(); ++x) {
    const uint32_t r = (uint32_t)((x / ((size_t)L * 2 * n)) % (L + 1));
    mont[x] = to_mont(gk->h[x], c->mods[r]);
  }
  hipError_t err = hipSetDevice(c->device);
  if (err == hipSuccess) err = dev_malloc((void**)&gk->d, gk->words * 4);
  if (err == hipSuccess) err = hipMemcpy(gk->d, mont.data(), gk->words * 4, hipMemcpyHostToDevice);
  return err;
}
}  // namespace lrhe

extern "C" int lrhe_keygen(lrhe_ctx* c, uint64_t seed, int with_galois, lrhe_sk** sk_out, lrhe_pk** pk_out,
                           lrhe_gk** gk_out) {
  if (!c) return fail(LRHE_EINVAL, "null context");
  const uint32_t n = c->n, L = c->L;
  std::vector<int32_t> s, e;
  sample_ternary(seed, KIND_SECRET, 0, n, s);
  const std::vector<uint32_t> S = secret_eval(c, s.data());
  lrhe_sk* sk = make_sk(c, s.data());
  // public key: pk = (-(a s + e), a) mod Q, evaluation form
  auto* pk = new lrhe_pk();
  pk->h.assign((size_t)2 * L * n, 0);
  sample_cbd(seed, KIND_PK_E, 0, n, e);
  std::vector<uint32_t> A(n), Ev(n);
  for (uint32_t j = 0; j < L; ++j) {
    const uint32_t q = c->q[j];
    sample_uniform(seed, KIND_PK_A, j, q, n, A.data());
    host_ntt(c, (int)j, A.data(), false);
    for (uint32_t k = 0; k < n; ++k) Ev[k] = smod(e[k], q);
    host_ntt(c, (int)j, Ev.data(), false);
    const uint32_t* Sj = &S[(size_t)j * n];
    for (uint32_t k = 0; k < n; ++k) {
      const uint64_t as = (uint64_t)A[k] * Sj[k] % q;
      pk->h[(size_t)j * n + k] = (uint32_t)((2ull * q - as - Ev[k]) % q);
      pk->h[(size_t)(L + j) * n + k] = A[k];
    }
  }
  hipError_t err = upload_pk(c, pk);
  if (err != hipSuccess) {
    delete sk;
    lrhe_pk_destroy(pk);
    return fail(LRHE_EDEVICE, "pk upload: %s", hipGetErrorString(err));
  }
  lrhe_gk* gk = nullptr;
  if (err == hipSuccess && with_galois) {
    gk = new lrhe_gk();
    gk->words = (size_t)c->ngal * (L + 1) * L * 2 * n;
    gk->h.assign(gk->words, 0);
    // ksk_{g,i} mod r = (-(a s + e) + [P]_r [i = r] sigma_g(s), a), layout [g][r][i][x][n]
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int gi = 0; gi < (int)c->ngal; ++gi)
      for (int i = 0; i < (int)L; ++i) {
        std::vector<int32_t> ee, sg;
        sample_cbd(seed, KIND_GK_E, (uint64_t)gi * L + i, n, ee);
        automorph_int(s, c->gal[gi], n, sg);
        std::vector<uint32_t> a(n), ev(n), sgv(n);
        for (uint32_t r = 0; r <= L; ++r) {
          const uint32_t m = c->q[r];
          sample_uniform(seed, KIND_GK_A, ((uint64_t)gi * L + i) * (L + 1) + r, m, n, a.data());
          host_ntt(c, (int)r, a.data(), false);
          for (uint32_t k = 0; k < n; ++k) ev[k] = smod(ee[k], m);
          host_ntt(c, (int)r, ev.data(), false);
          const bool diag = (r == (uint32_t)i);
          if (diag) {
            for (uint32_t k = 0; k < n; ++k) sgv[k] = smod(sg[k], m);
            host_ntt(c, (int)r, sgv.data(), false);
          }
          const uint64_t Pm = c->P % m;
          const uint32_t* Sr = &S[(size_t)r * n];
          uint32_t* kb = &gk->h[((((size_t)gi * (L + 1) + r) * L + i) * 2 + 0) * n];
          uint32_t* ka = kb + n;
          for (uint32_t k = 0; k < n; ++k) {
            uint64_t b = (2ull * m - (uint64_t)a[k] * Sr[k] % m - ev[k]) % m;
            if (diag) b = (b + Pm * sgv[k]) % m;
            kb[k] = (uint32_t)b;
            ka[k] = a[k];
          }
        }
      }
    err = upload_gk(c, gk);
  }
  if (err != hipSuccess) {
    delete sk;
    lrhe_pk_destroy(pk);
    lrhe_gk_destroy(gk);
    return fail(LRHE_EDEVICE, "key upload: %s", hipGetErrorString(err));
  }
  if (sk_out) *sk_out = sk; else delete sk;
  if (pk_out) *pk_out = pk; else lrhe_pk_destroy(pk);
  if (gk_out) *gk_out = gk; else lrhe_gk_destroy(gk);
  return LRHE_OK;
}

extern "C" void lrhe_sk_destroy(lrhe_sk* sk) { delete sk; }
extern "C" void lrhe_pk_destroy(lrhe_pk* pk) {
  if (!pk) return;
  if (pk->d) (void)hipFree(pk->d);
  delete pk;
}
extern "C" void lrhe_gk_destroy(lrhe_gk* gk) {
  if (!gk) return;
  if (gk->d) (void)hipFree(gk->d);
  delete gk;
}

extern "C" int lrhe_sk_export(lrhe_ctx* c, const lrhe_sk* sk, int8_t* out) {
  if (!c || !sk || !out) return fail(LRHE_EINVAL, "null argument");
  std::copy(sk->s.begin(), sk->s.end(), out);
  return LRHE_OK;
}
extern "C" int lrhe_pk_export(lrhe_ctx* c, const lrhe_pk* pk, uint32_t* out) {
  if (!c || !pk || !out) return fail(LRHE_EINVAL, "null argument");
  const uint32_t n = c->n, L = c->L;
  for (uint32_t x = 0; x < 2 * L; ++x) {
    std::copy(pk->h.begin() + (size_t)x * n, pk->h.begin() + (size_t)(x + 1) * n, out + (size_t)x * n);
    host_ntt(c, (int)(x % L), out + (size_t)x * n, true);
  }
  return LRHE_OK;
}
extern "C" int lrhe_gk_export(lrhe_ctx* c, const lrhe_gk* gk, uint32_t* out) {
  if (!c || !gk || !out) return fail(LRHE_EINVAL, "null argument");
  const uint32_t n = c->n, L = c->L;
  // device/host layout [g][r][i][x][n] -> export layout [g][i][x][r][n]
#pragma omp parallel for collapse(2)
  for (int gi = 0; gi < (int)c->ngal; ++gi)
    for (int r = 0; r <= (int)L; ++r)
      for (uint32_t i = 0; i < L; ++i)
        for (uint32_t x = 0; x < 2; ++x) {
          const uint32_t* src = &gk->h[((((size_t)gi * (L + 1) + r) * L + i) * 2 + x) * n];
          uint32_t* dst = out + ((((size_t)gi * L + i) * 2 + x) * (L + 1) + r) * n;
          std::copy(src, src + n, dst);
          host_ntt(c, r, dst, true);
        }
  return LRHE_OK;
}

// ------------------------------------------------------------------ decryption (client)
// Little-endian 32-bit limb arithmetic, enough for t x / Q with the exact noise.
using Big = std::vector<uint32_t>;
static void big_add_mul(Big& acc, const Big& a, uint64_t m) {   // acc += a m
  if (acc.size() < a.size() + 3) acc.resize(a.size() + 3, 0);
  unsigned __int128 carry = 0;
  size_t i = 0;
  for (; i < a.size(); ++i) {
    unsigned __int128 v = (unsigned __int128)a[i] * m + acc[i] + carry;
    acc[i] = (uint32_t)v;
    carry = v >> 32;
  }
  for (; carry && i < acc.size(); ++i) {
    unsigned __int128 v = (unsigned __int128)acc[i] + carry;
    acc[i] = (uint32_t)v;
    carry = v >> 32;
  }
}
static int big_cmp(const Big& a, const Big& b) {
  const size_t n = std::max(a.size(), b.size());
  for (size_t i = n; i-- > 0;) {
    const uint32_t x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}
static void big_sub(Big& a, const Big& b) {   // a -= b, a >= b
  int64_t borrow = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    int64_t v = (int64_t)a[i] - (i < b.size() ? b[i] : 0) - borrow;
    borrow = v < 0;
    a[i] = (uint32_t)(v + (borrow << 32));
  }
}
static double big_log2(const Big& a) {
  for (size_t i = a.size(); i-- > 0;)
    if (a[i]) {
      double hi = a[i], lo = i > 0 ? a[i - 1] : 0;
      return std::log2(hi + lo / 4294967296.0) + 32.0 * i;
    }
  return -INFINITY;
}

// Fixed-width unsigned integers for the exact rounding of decryption: Q has at
// most LRHE_MAXL 30-bit primes (450 bits); sums of L terms x_j R_j (Q / q_j)
// stay below 2^64 Q.  No allocation in the per-coefficient loop.
namespace {
constexpr int FW = (LRHE_MAXL * 30 + 64) / 32 + 2;
struct Fixed {
  uint32_t w[FW];
};
inline void fx_from(Fixed& a, const Big& b) {
  for (int i = 0; i < FW; ++i) a.w[i] = i < (int)b.size() ? b[i] : 0;
}
inline void fx_add_mul32(Fixed& acc, const Fixed& a, uint32_t m, int nw) {   // acc += a m (nw words)
  uint64_t carry = 0;
  for (int i = 0; i < nw; ++i) {   // below (2^32 - 1)^2 + 2 (2^32 - 1) = 2^64 - 1
    const uint64_t v = (uint64_t)a.w[i] * m + acc.w[i] + carry;
    acc.w[i] = (uint32_t)v;
    carry = v >> 32;
  }
}
inline void fx_add_mul(Fixed& acc, const Fixed& a, uint64_t m, int nw) {   // acc += a m (nw words)
  unsigned __int128 carry = 0;
  for (int i = 0; i < nw; ++i) {
    const unsigned __int128 v = (unsigned __int128)a.w[i] * m + acc.w[i] + carry;
    acc.w[i] = (uint32_t)v;
    carry = v >> 32;
  }
}
inline int fx_cmp(const Fixed& a, const Fixed& b, int nw) {
  for (int i = nw; i-- > 0;)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
  return 0;
}
inline void fx_sub(Fixed& a, const Fixed& b, int nw) {   // a -= b, a >= b
  int64_t borrow = 0;
  for (int i = 0; i < nw; ++i) {
    const int64_t v = (int64_t)a.w[i] - b.w[i] - borrow;
    borrow = v < 0;
    a.w[i] = (uint32_t)(v + (borrow << 32));
  }
}
inline double fx_log2(const Fixed& a, int nw) {
  for (int i = nw; i-- > 0;)
    if (a.w[i]) {
      const double hi = a.w[i], lo = i > 0 ? a.w[i - 1] : 0;
      return std::log2(hi + lo / 4294967296.0) + 32.0 * i;
    }
  return -INFINITY;
}
}  // namespace

static int decrypt_host(lrhe_ctx* c, const lrhe_sk* sk, const uint32_t* h, uint32_t count, int64_t* slots,
                        double* budgets) {
  const uint32_t n = c->n, L = c->L, t = c->t;
  const size_t ctw = (size_t)2 * L * n;
  Fixed Q, Qhalf, Qhat[LRHE_MAXL];
  fx_from(Q, c->Qbig);
  Qhalf = Q;   // floor(Q / 2)
  {
    uint32_t carry = 0;
    for (int i = FW; i-- > 0;) {
      const uint64_t v = ((uint64_t)carry << 32) | Qhalf.w[i];
      Qhalf.w[i] = (uint32_t)(v >> 1);
      carry = (uint32_t)(v & 1);
    }
  }
  for (uint32_t j = 0; j < L; ++j) fx_from(Qhat[j], c->Qhat[j]);
  // words that hold 2^64 Q: sums of L terms below 2^64 Q, and k0 Q
  const int nw = std::min(FW, (int)((c->log2Q + 66) / 32) + 2);
  // RQ_j = R_j (Q / q_j), below q_j Q: the terms of N are x_j RQ_j with 32-bit x_j
  Fixed RQ[LRHE_MAXL];
  for (uint32_t j = 0; j < L; ++j) {
    RQ[j] = Fixed{};
    fx_add_mul32(RQ[j], Qhat[j], c->dec_R[j], nw);
  }
  int bad = 0;
  // one ciphertext: x_j = [c0 + c1 s]_{q_j} in coefficient form, then
  // m = sum_j x_j I_j + round(sum_j x_j R_j / q_j) mod t with the rounding done
  // exactly: N = sum_j x_j R_j (Q/q_j), k0 = round(N / Q), noise w = N - k0 Q
  auto one = [&](uint32_t ci, uint32_t* X, uint32_t* mcoef, bool inner_parallel) -> int {
    const uint32_t* C = &h[(size_t)ci * ctw];
#pragma omp parallel for schedule(static) if (inner_parallel)
    for (int j = 0; j < (int)L; ++j) {
      const uint64_t q = c->q[j];
      const uint32_t* Sj = &sk->Sm[(size_t)j * n];
      const Mod& md = c->mods[j];
      uint32_t* xj = &X[(size_t)j * n];
      for (uint32_t k = 0; k < n; ++k) {
        // c0 + c1 s: the Montgomery product is below 2q, any c0 below 2^32 is
        // reduced first (a canonical c0 skips the division)
        const uint32_t c0 = C[(size_t)j * n + k];
        const uint64_t v = (uint64_t)(c0 < q ? c0 : c0 % q) + mulm(C[(size_t)(L + j) * n + k], Sj[k], (uint32_t)q, md.qinv);
        xj[k] = (uint32_t)(v >= 2 * q ? v - 2 * q : v >= q ? v - q : v);
      }
      host_ntt(c, j, xj, true);
    }
    double worst = -INFINITY;
    int err = 0;
#pragma omp parallel for schedule(static) reduction(max : worst) reduction(| : err) if (inner_parallel)
    for (int k = 0; k < (int)n; ++k) {
      // sum of x_j I_j mod t: each term below 2^60 (x_j < q_j < 2^30, I_j < t <
      // 2^30), reduced after every 8 terms so the sum stays below 2^64
      uint64_t mi = 0;
      double approx = 0;
      Fixed N{};
      for (uint32_t j = 0; j < L; ++j) {
        const uint64_t xj = X[(size_t)j * n + k];
        mi += xj * c->dec_I[j];
        if ((j & 7) == 7) mi %= t;
        approx += (double)xj * c->dec_Rf[j];
        fx_add_mul32(N, RQ[j], (uint32_t)xj, nw);
      }
      int64_t k0 = (int64_t)std::floor(approx) - 1;
      if (k0 < 0) k0 = 0;
      Fixed K0Q{};
      fx_add_mul(K0Q, Q, (uint64_t)k0, nw);
      if (fx_cmp(N, K0Q, nw) < 0) {
        err = 1;
        continue;
      }
      fx_sub(N, K0Q, nw);   // N - k0 Q >= 0
      int guard = 0;
      while (fx_cmp(N, Qhalf, nw) > 0 && guard++ < 8) {   // keep |w| <= Q/2
        if (fx_cmp(N, Q, nw) >= 0) {
          fx_sub(N, Q, nw);
          ++k0;
        } else {   // Q/2 < N < Q: w = N - Q is negative
          Fixed tmp = Q;
          fx_sub(tmp, N, nw);
          N = tmp;
          ++k0;
          break;
        }
      }
      worst = std::max(worst, fx_log2(N, nw));
      mcoef[k] = (uint32_t)((mi % t + (uint64_t)(k0 % t)) % t);
    }
    if (err) return 1;
    // decode: slot j = evaluation at psi_t^(e_j)
    if (inner_parallel)
      host_ntt_fwd_threads(c, (int)L + 1, mcoef);
    else
      host_ntt(c, (int)L + 1, mcoef, false);
    for (uint32_t j = 0; j < n; ++j) {
      const uint32_t v = mcoef[c->slot_pos[j]];
      slots[(size_t)ci * n + j] = v > (t - 1) / 2 ? (int64_t)v - t : (int64_t)v;
    }
    if (budgets) budgets[ci] = (c->log2Q - 1.0) - worst;
    return 0;
  };
  if (count == 1) {
    std::vector<uint32_t> X((size_t)L * n), mcoef(n);
    bad = one(0, X.data(), mcoef.data(), true);
  } else {
    // several ciphertexts: one per thread
#pragma omp parallel reduction(| : bad)
    {
      std::vector<uint32_t> X((size_t)L * n), mcoef(n);
#pragma omp for schedule(dynamic, 1)
      for (int ci = 0; ci < (int)count; ++ci) bad |= one((uint32_t)ci, X.data(), mcoef.data(), false);
    }
  }
  if (bad) return fail(LRHE_EINVAL, "decrypt: rounding estimate out of range");
  return LRHE_OK;
}

extern "C" int lrhe_decrypt_slots(lrhe_ctx* c, const lrhe_sk* sk, const uint32_t* ct, uint32_t count, int64_t* slots,
                                  double* budgets, void* stream) {
  if (!c || !sk || !ct || !slots) return fail(LRHE_EINVAL, "null argument");
  NEED_DEVICE(c);
  std::vector<uint32_t> h((size_t)count * 2 * c->L * c->n);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMemcpyAsync(h.data(), ct, h.size() * 4, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return decrypt_host(c, sk, h.data(), count, slots, budgets);
}

extern "C" int lrhe_decrypt_slots_host(lrhe_ctx* c, const lrhe_sk* sk, const uint32_t* ct, uint32_t count,
                                       int64_t* slots, double* budgets) {
  if (!c || !sk || !ct || !slots) return fail(LRHE_EINVAL, "null argument");
  return decrypt_host(c, sk, ct, count, slots, budgets);
}

// ciphertexts at ct: device memory copied over on `stream`, or host memory
// (flags & LRHE_CT_HOST); decrypted and decoded into slots [count][n]
static int decrypt_any(lrhe_ctx* c, const lrhe_sk* sk, const uint32_t* ct, uint32_t count, uint32_t flags,
                       void* stream, std::vector<int64_t>& slots, std::vector<double>& bud) {
  if (flags & ~(uint32_t)LRHE_CT_HOST) return fail(LRHE_EINVAL, "unknown flags 0x%x", flags);
  slots.assign((size_t)count * c->n, 0);
  bud.assign(count, 0.0);
  if (flags & LRHE_CT_HOST) return decrypt_host(c, sk, ct, count, slots.data(), bud.data());
  NEED_DEVICE(c);
  std::vector<uint32_t> h((size_t)count * 2 * c->L * c->n);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMemcpyAsync(h.data(), ct, h.size() * 4, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return decrypt_host(c, sk, h.data(), count, slots.data(), bud.data());
}

extern "C" int lrhe_decrypt_scores(lrhe_ctx* c, const lrhe_sk* sk, const uint32_t* y, uint32_t rows, uint32_t classes,
                                   uint32_t flags, int64_t* scores, double* min_budget_bits, void* stream) {
  if (!c || !sk || !y || !scores) return fail(LRHE_EINVAL, "null argument");
  if (rows == 0 || classes == 0) return fail(LRHE_EINVAL, "empty score matrix");
  const uint64_t npairs = (uint64_t)rows * classes;
  const uint64_t nout = (npairs + c->n - 1) / c->n;
  if (nout > 0xffffffffull) return fail(LRHE_EINVAL, "too many results");
  std::vector<int64_t> slots;
  std::vector<double> bud;
  const int rc = decrypt_any(c, sk, y, (uint32_t)nout, flags, stream, slots, bud);
  if (rc != LRHE_OK) return rc;
  // result r = i classes + j of Algorithm 1: output ciphertext r / n, slot r mod n;
  // slots [count][n] are contiguous, so that is slots[r]
  std::copy(slots.begin(), slots.begin() + npairs, scores);
  if (min_budget_bits) *min_budget_bits = *std::min_element(bud.begin(), bud.end());
  return LRHE_OK;
}

extern "C" int lrhe_decrypt_scores_standard(lrhe_ctx* c, const lrhe_sk* sk, const uint32_t* y, uint32_t rows,
                                            uint32_t classes, uint32_t flags, int64_t* scores,
                                            double* min_budget_bits, void* stream) {
  if (!c || !sk || !y || !scores) return fail(LRHE_EINVAL, "null argument");
  if (rows == 0 || classes == 0) return fail(LRHE_EINVAL, "empty score matrix");
  if (rows > c->n) return fail(LRHE_EINVAL, "standard layout: rows %u > n %u", rows, c->n);
  std::vector<int64_t> slots;
  std::vector<double> bud;
  const int rc = decrypt_any(c, sk, y, classes, flags, stream, slots, bud);
  if (rc != LRHE_OK) return rc;
  // score (i, j) is slot i of output ciphertext j
  for (uint32_t i = 0; i < rows; ++i)
    for (uint32_t j = 0; j < classes; ++j) scores[(size_t)i * classes + j] = slots[(size_t)j * c->n + i];
  if (min_budget_bits) *min_budget_bits = *std::min_element(bud.begin(), bud.end());
  return LRHE_OK;
}

extern "C" int lrhe_decrypt_check(lrhe_ctx* c, const lrhe_sk* sk, const uint32_t* ct, uint32_t count,
                                  const int64_t* expected, uint32_t flags, double* budgets, uint64_t* mismatches,
                                  void* stream) {
  if (!c || !sk || !ct || !expected) return fail(LRHE_EINVAL, "null argument");
  if (count == 0) return fail(LRHE_EINVAL, "no ciphertexts");
  std::vector<int64_t> slots;
  std::vector<double> bud;
  const int rc = decrypt_any(c, sk, ct, count, flags, stream, slots, bud);
  if (rc != LRHE_OK) return rc;
  if (budgets) std::copy(bud.begin(), bud.end(), budgets);
  // expected slot values are compared as residues mod t
  const int64_t t = c->t;
  uint64_t bad = 0;
  size_t first = 0;
  for (size_t k = 0; k < slots.size(); ++k) {
    const int64_t d = ((slots[k] - expected[k]) % t + t) % t;
    if (d != 0 && bad++ == 0) first = k;
  }
  if (mismatches) *mismatches = bad;
  if (bad)
    return fail(LRHE_ENOISE, "decryption differs from the expected plaintext in %llu slots (first: ciphertext %zu, "
                "slot %zu): the noise exceeded the budget", (unsigned long long)bad, first / c->n, first % c->n);
  return LRHE_OK;
}

extern "C" int lrhe_fixed_point(const double* in, uint64_t count, int bits, int64_t* out) {
  if ((!in || !out) && count) return fail(LRHE_EINVAL, "null argument");
  if (bits < 0 || bits > 62) return fail(LRHE_EINVAL, "bits = %d outside [0, 62]", bits);
  const double lim = std::ldexp(1.0, 62);
  for (uint64_t i = 0; i < count; ++i) {
    const double v = std::nearbyint(std::ldexp(in[i], bits));   // default rounding: nearest, ties to even
    if (!std::isfinite(v) || std::fabs(v) >= lim)
      return fail(LRHE_EINVAL, "value %llu (%g) does not fit after scaling by 2^%d", (unsigned long long)i, in[i], bits);
    out[i] = (int64_t)v;
  }
  return LRHE_OK;
}

extern "C" int lrhe_crt_combine(const int64_t* r0, const int64_t* r1, uint64_t count, uint64_t t0, uint64_t t1,
                                int64_t* out) {
  if ((!r0 || !r1 || !out) && count) return fail(LRHE_EINVAL, "null argument");
  if (t0 < 2 || t1 < 2) return fail(LRHE_EINVAL, "moduli must be at least 2");
  const unsigned __int128 M = (unsigned __int128)t0 * t1;
  if (M >> 63) return fail(LRHE_EINVAL, "t0 t1 must stay below 2^63");
  // t0^-1 mod t1 by the extended Euclidean algorithm
  int64_t a = (int64_t)(t0 % t1), b = (int64_t)t1, x0 = 1, x1 = 0;
  while (b) {
    const int64_t qd = a / b, r = a - qd * b, xr = x0 - qd * x1;
    a = b; b = r; x0 = x1; x1 = xr;
  }
  if (a != 1) return fail(LRHE_EINVAL, "t0 and t1 are not coprime");
  const uint64_t inv = (uint64_t)((x0 % (int64_t)t1 + (int64_t)t1) % (int64_t)t1);
  const uint64_t m = (uint64_t)M, half = m / 2;
  for (uint64_t i = 0; i < count; ++i) {
    const uint64_t u = (uint64_t)(((r0[i] % (int64_t)t0) + (int64_t)t0) % (int64_t)t0);
    const uint64_t v = (uint64_t)(((r1[i] % (int64_t)t1) + (int64_t)t1) % (int64_t)t1);
    // z = u + t0 k with k = (v - u) t0^-1 mod t1, so z = u mod t0 and z = v mod t1
    const uint64_t d = (v + t1 - u % t1) % t1;
    const uint64_t k = (uint64_t)(((unsigned __int128)d * inv) % t1);
    const uint64_t z = u + t0 * k;   // < t0 t1 < 2^63
    out[i] = z > half ? (int64_t)z - (int64_t)m : (int64_t)z;
  }
  return LRHE_OK;
}

extern "C" int lrhe_host_transform(lrhe_ctx* c, uint32_t mod_index, uint32_t* a, int inverse) {
  if (!c || !a || mod_index > c->L + 1) return fail(LRHE_EINVAL, "bad argument");
  host_ntt_passes(c, (int)mod_index, a, inverse != 0);
  return LRHE_OK;
}

// ------------------------------------------------------------------ device calls
extern "C" int lrhe_workspace_bytes(const lrhe_ctx* c, int op, uint32_t rows, uint32_t f, uint32_t classes,
                                    uint64_t* bytes) {
  if (!c || !bytes) return fail(LRHE_EINVAL, "null argument");
  const uint64_t K = (f + c->n - 1) / c->n;
  switch (op) {
    case LRHE_WS_ENCRYPT_ROWS: *bytes = encrypt_ws_bytes(c, (uint64_t)rows * K); break;
    case LRHE_WS_ENCRYPT_COLS: *bytes = encrypt_ws_bytes(c, f); break;
    case LRHE_WS_MATMUL_FAST: *bytes = fast_ws_layout(c, rows * classes, classes).total; break;
    case LRHE_WS_MATMUL_STANDARD: *bytes = 0; break;
    default: return fail(LRHE_EINVAL, "unknown workspace op %d", op);
  }
  return LRHE_OK;
}

static int encrypt_common(lrhe_ctx* c, const lrhe_pk* pk, const int64_t* X, uint32_t rows, uint32_t f, bool cols,
                          uint64_t seed, uint64_t id0, uint32_t* ct_out, void* ws, size_t ws_bytes, void* stream) {
  if (!c || !pk || !X || !ct_out) return fail(LRHE_EINVAL, "null argument");
  if (rows == 0 || f == 0) return fail(LRHE_EINVAL, "empty feature matrix");
  if (cols && rows > c->n) return fail(LRHE_EINVAL, "standard layout: rows %u > n %u", rows, c->n);
  const uint64_t K = (f + c->n - 1) / c->n;
  const uint64_t need = encrypt_ws_bytes(c, cols ? (uint64_t)f : (uint64_t)rows * K);
  if (!ws || ws_bytes < need) return fail(LRHE_ENOMEM, "workspace %zu < %llu bytes", ws_bytes, (unsigned long long)need);
  NEED_DEVICE(c);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_encrypt(c, pk->d, X, rows, f, cols, seed, id0, ct_out, ws, (hipStream_t)stream));
  return LRHE_OK;
}
extern "C" int lrhe_encrypt_rows(lrhe_ctx* c, const lrhe_pk* pk, const int64_t* X, uint32_t rows, uint32_t f,
                                 uint64_t seed, uint64_t id0, uint32_t* ct_out, void* ws, size_t ws_bytes,
                                 void* stream) {
  return encrypt_common(c, pk, X, rows, f, false, seed, id0, ct_out, ws, ws_bytes, stream);
}
extern "C" int lrhe_encrypt_cols(lrhe_ctx* c, const lrhe_pk* pk, const int64_t* X, uint32_t rows, uint32_t f,
                                 uint64_t seed, uint64_t id0, uint32_t* ct_out, void* ws, size_t ws_bytes,
                                 void* stream) {
  return encrypt_common(c, pk, X, rows, f, true, seed, id0, ct_out, ws, ws_bytes, stream);
}

extern "C" int lrhe_model_create(lrhe_ctx* c, const int64_t* W, const int64_t* bias, uint32_t f, uint32_t classes,
                                 void* stream, lrhe_model** out) {
  if (!c || !W || !out) return fail(LRHE_EINVAL, "null argument");
  if (f == 0 || classes == 0) return fail(LRHE_EINVAL, "empty model");
  *out = nullptr;
  NEED_DEVICE(c);
  HIPCHK(hipSetDevice(c->device));
  auto* m = new lrhe_model();
  m->f = f;
  m->classes = classes;
  m->K = (f + c->n - 1) / c->n;
  const uint32_t L = c->L, n = c->n;
  std::vector<uint32_t> db((size_t)classes * L);
  for (uint32_t j = 0; j < classes; ++j) {
    const uint32_t b = bias ? smod(bias[j], c->t) : 0;
    // Delta(b) = floor(Q/t) b + round((Q mod t) b / t)
    const uint64_t rnd = ((uint64_t)c->dc.qmodt * b + (c->t - 1) / 2) / c->t;
    for (uint32_t i = 0; i < L; ++i) {
      const Mod& md = c->mods[i];
      const uint32_t a = red1(mulm(b, c->dc.qdivt_m[i], md.q, md.qinv), md.q);
      db[(size_t)j * L + i] = (uint32_t)((a + rnd % md.q) % md.q);
    }
  }
  hipError_t err = dev_malloc((void**)&m->wpt, (size_t)classes * m->K * L * n * 4);
  if (err == hipSuccess) err = dev_malloc((void**)&m->wsc, (size_t)f * std_class_pad(classes) * L * 4);
  if (err == hipSuccess) err = dev_malloc((void**)&m->dbias, db.size() * 4);
  if (err == hipSuccess) err = hipMemcpy(m->dbias, db.data(), db.size() * 4, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = launch_model_encode(c, W, f, classes, m->wpt, m->wsc, (hipStream_t)stream);
  if (err == hipSuccess) err = hipStreamSynchronize((hipStream_t)stream);
  if (err != hipSuccess) {
    lrhe_model_destroy(m);
    return fail(LRHE_EDEVICE, "model encode: %s", hipGetErrorString(err));
  }
  *out = m;
  return LRHE_OK;
}
extern "C" void lrhe_model_destroy(lrhe_model* m) {
  if (!m) return;
  (void)hipFree(m->wpt);
  (void)hipFree(m->wsc);
  (void)hipFree(m->dbias);
  delete m;
}

extern "C" int lrhe_matmul_fast(lrhe_ctx* c, const lrhe_gk* gk, const lrhe_model* m, const uint32_t* xct,
                                uint32_t rows, uint32_t* y_out, void* ws, size_t ws_bytes, void* stream) {
  if (!c || !gk || !m || !xct || !y_out) return fail(LRHE_EINVAL, "null argument");
  if (rows == 0) return fail(LRHE_EINVAL, "no rows");
  const uint64_t npairs = (uint64_t)rows * m->classes;
  if (npairs > 0xffffffffull) return fail(LRHE_EINVAL, "too many pairs");
  const FastWs lay = fast_ws_layout(c, (uint32_t)npairs, m->classes);
  if (!ws || ws_bytes < lay.total) return fail(LRHE_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, lay.total);
  NEED_DEVICE(c);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_fast(c, gk->d, m, xct, rows, 0, (uint32_t)npairs, -1, y_out, ws, lay, (hipStream_t)stream));
  return LRHE_OK;
}

extern "C" int lrhe_matmul_fast_noalloc(lrhe_ctx* c, const lrhe_gk* gk, const lrhe_model* m, const uint32_t* xct,
                                        uint32_t rows, uint32_t* y_out, void* stream) {
  if (!c || !gk || !m || !xct || !y_out) return fail(LRHE_EINVAL, "null argument");
  if (rows == 0) return fail(LRHE_EINVAL, "no rows");
  const uint64_t npairs = (uint64_t)rows * m->classes;
  if (npairs > 0xffffffffull) return fail(LRHE_EINVAL, "too many pairs");
  NEED_DEVICE(c);
  const FastWs lay = fast_ws_layout(c, (uint32_t)npairs, m->classes);
  if (lay.total > LRHE_SCRATCH_BYTES)
    return fail(LRHE_EINVAL, "%llu rows x %u classes need a workspace of %zu bytes, above the fixed scratch of %llu bytes "
                "of the non-allocating path (use lrhe_matmul_fast with a caller workspace)",
                (unsigned long long)rows, m->classes, lay.total, (unsigned long long)LRHE_SCRATCH_BYTES);
  void* ws = scratch_ptr(c->device);
  if (!ws) return fail(LRHE_EDEVICE, "fixed scratch of device %d not resolved", c->device);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_fast(c, gk->d, m, xct, rows, 0, (uint32_t)npairs, -1, y_out, ws, lay, (hipStream_t)stream));
  return LRHE_OK;
}

extern "C" int lrhe_matmul_fast_pairs(lrhe_ctx* c, const lrhe_gk* gk, const lrhe_model* m, const uint32_t* xct,
                                      uint32_t rows, uint32_t pair0, uint32_t npairs, int stage, uint32_t* out,
                                      void* ws, size_t ws_bytes, void* stream) {
  if (!c || !gk || !m || !xct || !out) return fail(LRHE_EINVAL, "null argument");
  if (npairs == 0 || (uint64_t)pair0 + npairs > (uint64_t)rows * m->classes) return fail(LRHE_EINVAL, "pair range");
  if (!(stage == 0 || stage == 1 || stage == 100 || (stage >= 2 && stage <= (int)c->ngal + 2)))
    return fail(LRHE_EINVAL, "stage %d", stage);
  const FastWs lay = fast_ws_layout(c, npairs, m->classes);
  if (!ws || ws_bytes < lay.total) return fail(LRHE_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, lay.total);
  NEED_DEVICE(c);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_fast(c, gk->d, m, xct, rows, pair0, npairs, stage, out, ws, lay, (hipStream_t)stream));
  return LRHE_OK;
}

extern "C" int lrhe_matmul_standard(lrhe_ctx* c, const lrhe_model* m, const uint32_t* fct, uint32_t* y_out, void* ws,
                                    size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  if (!c || !m || !fct || !y_out) return fail(LRHE_EINVAL, "null argument");
  NEED_DEVICE(c);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_standard(c, m, fct, y_out, (hipStream_t)stream));
  return LRHE_OK;
}

extern "C" int lrhe_to_coeff(lrhe_ctx* c, const uint32_t* in, uint64_t polys, uint32_t* out, void* stream) {
  if (!c || !in || !out) return fail(LRHE_EINVAL, "null argument");
  NEED_DEVICE(c);
  HIPCHK(hipSetDevice(c->device));
  const uint64_t words = polys * c->L * c->n;
  if (in != out) HIPCHK(hipMemcpyAsync(out, in, words * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  HIPCHK(launch_ntt(c, out, polys * c->L, c->L, 0, true, (hipStream_t)stream));
  return LRHE_OK;
}

extern "C" int lrhe_ntt(lrhe_ctx* c, uint32_t* data, uint64_t polys, int inverse, void* stream) {
  if (!c || !data) return fail(LRHE_EINVAL, "null argument");
  NEED_DEVICE(c);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_ntt(c, data, polys * c->L, c->L, 0, inverse != 0, (hipStream_t)stream));
  return LRHE_OK;
}

// ------------------------------------------------------------------ tuning
static bool le_valid(uint32_t logn, int le) {
  if (le < 4 || le > 6) return false;
  if ((int)logn - le > 10) return false;   // at most 1024 threads per workgroup
  if (le == 4 && logn > 14) return false;
  if (le == 6 && logn < 12) return false;
  return true;
}

// key = [small. | large.] name; without a prefix, set applies to both classes
// and get reads the large-tile class
static lrhe::Knobs* knob_class(lrhe_ctx* c, std::string& k, bool* both) {
  *both = false;
  if (k.rfind("small.", 0) == 0) { k = k.substr(6); return &c->tune.small; }
  if (k.rfind("large.", 0) == 0) { k = k.substr(6); return &c->tune.large; }
  *both = true;
  return &c->tune.large;
}
static int* knob_field(lrhe::Knobs* kn, const std::string& k) {
  if (k == "le_intt") return &kn->le_intt;
  if (k == "le_mac") return &kn->le_mac;
  if (k == "le_moddown") return &kn->le_moddown;
  if (k == "le_mask") return &kn->le_mask;
  if (k == "mac_mode") return &kn->mac_mode;
  if (k == "le_mac_p") return &kn->le_mac_p;
  if (k == "fuse_intt") return &kn->fuse_intt;
  return nullptr;
}

extern "C" int lrhe_tune_set(lrhe_ctx* c, const char* key, int value) {
  if (!c || !key) return fail(LRHE_EINVAL, "null argument");
  std::string k = key;
  if (k == "tile" || k == "small_below") {
    if (value < 1) return fail(LRHE_EINVAL, "%s must be >= 1", key);
    (k == "tile" ? c->tune.tile : c->tune.small_below) = (uint32_t)value;
    return LRHE_OK;
  }
  bool both = false;
  lrhe::Knobs* kn = knob_class(c, k, &both);
  int* f = knob_field(kn, k);
  if (!f) return fail(LRHE_EINVAL, "unknown tuning key '%s'", key);
  if (k == "mac_mode") {
    if (value < 0 || value >= LRHE_MAC_NMODES) return fail(LRHE_EINVAL, "mac_mode must be in [0, %d)", LRHE_MAC_NMODES);
    if (value == LRHE_MAC_MODE_HALF && kn != &c->tune.small)
      return fail(LRHE_EINVAL, "mac_mode %d is a choice of the small-tile class only (small.mac_mode)",
                  LRHE_MAC_MODE_HALF);
  } else if (k == "fuse_intt") {
    if (value != 0 && value != 1) return fail(LRHE_EINVAL, "fuse_intt must be 0 or 1");
  } else if (!le_valid(c->logn, value)) {
    return fail(LRHE_EINVAL, "%s = %d not available at n = %u", key, value, c->n);
  }
  *f = value;
  if (both) *knob_field(&c->tune.small, k) = value;
  return LRHE_OK;
}

extern "C" int lrhe_tune_get(const lrhe_ctx* c, const char* key, int* value) {
  if (!c || !key || !value) return fail(LRHE_EINVAL, "null argument");
  std::string k = key;
  if (k == "tile") { *value = (int)c->tune.tile; return LRHE_OK; }
  if (k == "small_below") { *value = (int)c->tune.small_below; return LRHE_OK; }
  bool both = false;
  lrhe::Knobs* kn = knob_class(const_cast<lrhe_ctx*>(c), k, &both);
  const int* f = knob_field(kn, k);
  if (!f) return fail(LRHE_EINVAL, "unknown tuning key '%s'", key);
  *value = *f;
  return LRHE_OK;
}

// ------------------------------------------------------------------ tuning cache
// One line per key: "<key>\t<name>=<value> <name>=<value> ..." with the names of
// lrhe_tune_get (both classes, tile, small_below).
static const char* const k_tune_names[] = {"le_intt", "le_mac", "le_moddown", "le_mask", "mac_mode", "fuse_intt", "le_mac_p"};

extern "C" int lrhe_tune_save(const lrhe_ctx* c, const char* path, const char* key) {
  if (!c || !path || !key) return fail(LRHE_EINVAL, "null argument");
  if (!*key || std::strpbrk(key, "\t\n")) return fail(LRHE_EINVAL, "tuning key must be non-empty, no tab or newline");
  std::string line = std::string(key) + "\t";
  for (const char* cls : {"small.", "large."})
    for (const char* nm : k_tune_names) {
      std::string k = std::string(cls) + nm;
      int v = 0;
      lrhe_tune_get(c, k.c_str(), &v);
      line += k + "=" + std::to_string(v) + " ";
    }
  line += "tile=" + std::to_string(c->tune.tile) + " small_below=" + std::to_string(c->tune.small_below);
  // keep the other keys' lines, replace this key's
  std::vector<std::string> keep;
  if (FILE* f = std::fopen(path, "r")) {
    char buf[4096];
    while (std::fgets(buf, sizeof(buf), f)) {
      std::string l(buf);
      while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
      if (l.empty() || l.compare(0, std::strlen(key) + 1, std::string(key) + "\t") == 0) continue;
      keep.push_back(l);
    }
    std::fclose(f);
  }
  keep.push_back(line);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(LRHE_EINVAL, "cannot write %s", tmp.c_str());
  for (const auto& l : keep) std::fprintf(f, "%s\n", l.c_str());
  const bool ok = std::fclose(f) == 0 && std::rename(tmp.c_str(), path) == 0;
  return ok ? LRHE_OK : fail(LRHE_EINVAL, "cannot write %s", path);
}

extern "C" int lrhe_tune_load(lrhe_ctx* c, const char* path, const char* key) {
  if (!c || !path || !key) return fail(LRHE_EINVAL, "null argument");
  FILE* f = std::fopen(path, "r");
  if (!f) return LRHE_EAGAIN;
  std::string found;
  char buf[4096];
  const std::string pre = std::string(key) + "\t";
  while (std::fgets(buf, sizeof(buf), f)) {
    std::string l(buf);
    if (l.compare(0, pre.size(), pre) == 0) found = l.substr(pre.size());
  }
  std::fclose(f);
  if (found.empty()) return LRHE_EAGAIN;
  // apply to a copy, so that a bad entry leaves the context as it was
  const lrhe::Tune before = c->tune;
  size_t pos = 0;
  int rc = LRHE_OK;
  while (rc == LRHE_OK && pos < found.size()) {
    const size_t end = found.find_first_of(" \n\r", pos);
    const std::string tok = found.substr(pos, end == std::string::npos ? std::string::npos : end - pos);
    pos = end == std::string::npos ? found.size() : end + 1;
    if (tok.empty()) continue;
    const size_t eq = tok.find('=');
    if (eq == std::string::npos) { rc = fail(LRHE_EINVAL, "tuning cache: bad entry '%s'", tok.c_str()); break; }
    rc = lrhe_tune_set(c, tok.substr(0, eq).c_str(), std::atoi(tok.c_str() + eq + 1));
  }
  if (rc != LRHE_OK) c->tune = before;
  return rc;
}

extern "C" int lrhe_autotune_fast(lrhe_ctx* c, const lrhe_gk* gk, const lrhe_model* m, const uint32_t* xct,
                                  uint32_t rows, uint32_t* y_out, void* ws, size_t ws_bytes, void* stream, int reps) {
  if (!c || !gk || !m || !xct || !y_out) return fail(LRHE_EINVAL, "null argument");
  NEED_DEVICE(c);
  if (reps < 1) reps = 1;
  // the class of this job's tiles is the one tuned
  const uint64_t npairs = (uint64_t)rows * m->classes;
  lrhe::Knobs& K = c->tune.knobs(std::min<uint64_t>(npairs, c->tune.tile));
  const char* names[7] = {"k_ks_intt", "k_ks_moddown", "k_mask", "k_ks_mac", "k_ks_rho", "k_ks_mac_p", "k_ks_mac_md"};
  int* knobs[3] = {&K.le_intt, &K.le_moddown, &K.le_mask};
  double best_ms[3] = {1e300, 1e300, 1e300};
  int best_le[3] = {K.le_intt, K.le_moddown, K.le_mask};
  // per (residues per thread, variant): k_ks_mac time, and for the digit-halves
  // variant the whole of its step after k_ks_intt (k_ks_mac + k_ks_rho + its
  // k_ks_moddown), which the others are compared against with their best k_ks_moddown
  const bool small_class = &K == &c->tune.small;
  double mac_ms[3][LRHE_MAC_NMODES], half_ms[3];
  // the split variant's special-prime launch keeps its own fastest residues per thread
  double best_p_ms = 1e300;
  int best_p_le = K.le_mac_p;
  for (auto& row : mac_ms)
    for (double& v : row) v = 1e300;
  for (double& v : half_ms) v = 1e300;
  auto timed = [&](double* ms_out, int nk) -> int {
    int rc = lrhe_matmul_fast(c, gk, m, xct, rows, y_out, ws, ws_bytes, stream);   // warm-up
    if (rc != LRHE_OK) return rc;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return fail(LRHE_EDEVICE, "autotune: stream");
    lrhe_prof_reset();
    lrhe_prof_enable(1);
    for (int r = 0; r < reps && rc == LRHE_OK; ++r) rc = lrhe_matmul_fast(c, gk, m, xct, rows, y_out, ws, ws_bytes, stream);
    lrhe_prof_enable(0);
    for (int k = 0; k < nk; ++k) {
      uint64_t cnt = 0;
      ms_out[k] = 1e300;
      double ms = 0;
      lrhe_prof_get(names[k], &cnt, &ms);
      if (cnt) ms_out[k] = ms;
    }
    lrhe_prof_reset();
    return rc;
  };
  // every kernel is timed separately with events on its stream; each keeps its
  // own fastest residues-per-thread choice; k_ks_mac is searched jointly over
  // residues per thread and variant
  for (int le = 4; le <= 6; ++le) {
    if (!le_valid(c->logn, le)) continue;
    K.le_intt = K.le_moddown = K.le_mask = K.le_mac = K.le_mac_p = le;
    for (int mode = 0; mode < LRHE_MAC_NMODES; ++mode) {
      if (mode == LRHE_MAC_MODE_HALF && !small_class) continue;
      K.mac_mode = mode;
      double ms[7];
      const int rc = timed(ms, 7);
      if (rc != LRHE_OK) return rc;
      if (mode == 0) {
        for (int k = 0; k < 3; ++k)
          if (ms[k] < best_ms[k]) {
            best_ms[k] = ms[k];
            best_le[k] = le;
          }
      }
      // the split variant: its data-modulus launch, which includes part 3 (no
      // k_ks_moddown); its special-prime launch, which also makes the digits (no
      // k_ks_intt), is chosen on its own
      const bool split = mode == LRHE_MAC_MODE_SPLIT || mode == LRHE_MAC_MODE_SPLIT64;
      mac_ms[le - 4][mode] = split ? ms[6] : ms[3];
      if (split && ms[5] < best_p_ms) {
        best_p_ms = ms[5];
        best_p_le = le;
      }
      // the digit-halves variant runs k_ks_intt on every step (the others on
      // the first only, when k_ks_moddown writes the next step's digits)
      if (mode == LRHE_MAC_MODE_HALF) half_ms[le - 4] = ms[3] + ms[4] + ms[1] + ms[0];
    }
  }
  for (int k = 0; k < 3; ++k) *knobs[k] = best_le[k];
  double best = 1e300;
  int best_mac_le = K.le_mac, best_mode = 0;
  for (int le = 4; le <= 6; ++le)
    for (int mode = 0; mode < LRHE_MAC_NMODES; ++mode) {
      const double cost = mode == LRHE_MAC_MODE_HALF    ? half_ms[le - 4]
                          : (mode == LRHE_MAC_MODE_SPLIT || mode == LRHE_MAC_MODE_SPLIT64)
                              ? mac_ms[le - 4][mode] + best_p_ms   // makes its own digits
                                                        : mac_ms[le - 4][mode] + best_ms[1] + best_ms[0];
      if (cost < best) {
        best = cost;
        best_mac_le = le;
        best_mode = mode;
      }
    }
  // the digit-halves variant runs its own k_ks_rho and k_ks_moddown at the
  // residues per thread it was timed with
  if (best_mode == LRHE_MAC_MODE_HALF) K.le_moddown = best_mac_le;
  K.le_mac = best_mac_le;
  K.mac_mode = best_mode;
  K.le_mac_p = best_p_le;
  return LRHE_OK;
}
