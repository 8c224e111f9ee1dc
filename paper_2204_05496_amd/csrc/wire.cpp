// wire.cpp -- byte format of what crosses between client and server in the
// private inference protocol: the client sends its encrypted inputs (and,
// once, the Galois keys the rotations need), the server returns the encrypted
// results; each side can keep its keys across restarts.
//
// A message is a 64-byte header followed by a payload, little-endian:
//   magic "LRHEWIR1", u32 version (1), u32 kind (1 ciphertexts, 2 Galois
//   keys, 3 public key, 4 secret key), u32 n, u32 L, u64 t, u64 parameter
//   digest (FNV-1a 64 over n, L, the L data primes, P and t as u64 words),
//   u64 count, u64 payload bytes, u64 payload checksum (FNV-1a 64).
// Polynomials travel in canonical coefficient form (residues in [0, q) as u32),
// independent of the device's evaluation order and Montgomery factors:
//   ciphertexts [count][2][L][n]; Galois keys [ngal][L digits][2][L+1 moduli][n]
//   (count = ngal); public key [2][L][n]; secret key int8 [n] in {-1, 0, 1}.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "lrhe_internal.h"

using namespace lrhe;

namespace {

constexpr char MAGIC[8] = {'L', 'R', 'H', 'E', 'W', 'I', 'R', '1'};
constexpr uint32_t VERSION = 1;
enum Kind : uint32_t { K_CT = 1, K_GK = 2, K_PK = 3, K_SK = 4 };

struct Header {
  char magic[8];
  uint32_t version, kind, n, L;
  uint64_t t, params, count, payload, checksum;
};
static_assert(sizeof(Header) == 64, "wire header is 64 bytes");

uint64_t fnv1a(const uint8_t* p, uint64_t len, uint64_t h = 1469598103934665603ull) {
  for (uint64_t i = 0; i < len; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t param_digest(const lrhe_ctx* c) {
  std::vector<uint64_t> w = {c->n, c->L};
  for (uint32_t r = 0; r <= c->L; ++r) w.push_back(c->q[r]);
  w.push_back(c->t);
  return fnv1a(reinterpret_cast<const uint8_t*>(w.data()), w.size() * 8);
}

uint64_t payload_bytes(const lrhe_ctx* c, uint32_t kind, uint64_t count) {
  const uint64_t n = c->n, L = c->L;
  switch (kind) {
    case K_CT: return count * 2 * L * n * 4;
    case K_GK: return (uint64_t)c->ngal * L * 2 * (L + 1) * n * 4;
    case K_PK: return 2 * L * n * 4;
    case K_SK: return n;
  }
  return 0;
}

int write_header(const lrhe_ctx* c, uint32_t kind, uint64_t count, const uint8_t* payload, uint64_t plen,
                 uint8_t* out) {
  Header h;
  std::memcpy(h.magic, MAGIC, 8);
  h.version = VERSION;
  h.kind = kind;
  h.n = c->n;
  h.L = c->L;
  h.t = c->t;
  h.params = param_digest(c);
  h.count = count;
  h.payload = plen;
  h.checksum = fnv1a(payload, plen);
  std::memcpy(out, &h, sizeof(h));
  return LRHE_OK;
}

// checks a message of the given kind against the context; returns its count
int read_header(const lrhe_ctx* c, const uint8_t* in, uint64_t bytes, uint32_t kind, uint64_t* count) {
  if (bytes < sizeof(Header)) return fail(LRHE_EINVAL, "wire: %llu bytes, shorter than the header",
                                          (unsigned long long)bytes);
  Header h;
  std::memcpy(&h, in, sizeof(h));
  if (std::memcmp(h.magic, MAGIC, 8) != 0) return fail(LRHE_EINVAL, "wire: not an LRHE message");
  if (h.version != VERSION) return fail(LRHE_EINVAL, "wire: version %u, expected %u", h.version, VERSION);
  if (h.kind != kind) return fail(LRHE_EINVAL, "wire: message of kind %u, expected %u", h.kind, kind);
  if (h.n != c->n || h.L != c->L || h.t != c->t || h.params != param_digest(c))
    return fail(LRHE_EINVAL, "wire: parameters (n %u, L %u, t %llu) differ from the context's", h.n, h.L,
                (unsigned long long)h.t);
  const uint64_t want = payload_bytes(c, kind, h.count);
  if (h.payload != want || bytes != sizeof(Header) + want)
    return fail(LRHE_EINVAL, "wire: payload of %llu bytes, expected %llu", (unsigned long long)h.payload,
                (unsigned long long)want);
  if (fnv1a(in + sizeof(Header), h.payload) != h.checksum) return fail(LRHE_EINVAL, "wire: checksum mismatch");
  *count = h.count;
  return LRHE_OK;
}

// the residues of a limb must be canonical for its modulus
bool limb_ok(const uint32_t* a, uint32_t n, uint32_t q) {
  for (uint32_t k = 0; k < n; ++k)
    if (a[k] >= q) return false;
  return true;
}

}  // namespace

extern "C" int lrhe_wire_bytes(lrhe_ctx* c, int kind, uint64_t count, uint64_t* bytes) {
  if (!c || !bytes) return fail(LRHE_EINVAL, "null argument");
  if (kind < K_CT || kind > K_SK) return fail(LRHE_EINVAL, "wire: unknown kind %d", kind);
  *bytes = sizeof(Header) + payload_bytes(c, (uint32_t)kind, kind == K_CT ? count : 1);
  return LRHE_OK;
}

extern "C" int lrhe_ct_serialize(lrhe_ctx* c, const uint32_t* ct, uint32_t count, uint32_t flags, uint8_t* out,
                                 uint64_t cap, void* stream) {
  if (!c || !ct || !out) return fail(LRHE_EINVAL, "null argument");
  if (flags & ~(uint32_t)LRHE_CT_HOST) return fail(LRHE_EINVAL, "unknown flags 0x%x", flags);
  const uint64_t plen = payload_bytes(c, K_CT, count);
  if (cap < sizeof(Header) + plen) return fail(LRHE_EINVAL, "wire: buffer of %llu bytes, %llu needed",
                                               (unsigned long long)cap, (unsigned long long)(sizeof(Header) + plen));
  uint32_t* P = reinterpret_cast<uint32_t*>(out + sizeof(Header));   // 64-byte offset: aligned for u32
  if (flags & LRHE_CT_HOST) {
    std::memcpy(P, ct, plen);
  } else {
    if (c->device < 0) return fail(LRHE_EDEVICE, "host-only context: pass LRHE_CT_HOST");
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = hipMemcpyAsync(P, ct, plen, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return fail(LRHE_EDEVICE, "wire: copy: %s", hipGetErrorString(e));
  }
  // evaluation form -> coefficients, limb by limb
  const uint64_t n = c->n, L = c->L, limbs = (uint64_t)count * 2 * L;
#pragma omp parallel for schedule(dynamic)
  for (int64_t x = 0; x < (int64_t)limbs; ++x) host_transform_limb(c, (int)(x % L), P + (uint64_t)x * n, true);
  return write_header(c, K_CT, count, out + sizeof(Header), plen, out);
}

extern "C" int lrhe_ct_deserialize(lrhe_ctx* c, const uint8_t* in, uint64_t bytes, uint32_t flags, uint32_t* ct_out,
                                   uint32_t max_count, uint32_t* count_out, void* stream) {
  if (!c || !in || !ct_out) return fail(LRHE_EINVAL, "null argument");
  if (flags & ~(uint32_t)LRHE_CT_HOST) return fail(LRHE_EINVAL, "unknown flags 0x%x", flags);
  uint64_t count = 0;
  int rc = read_header(c, in, bytes, K_CT, &count);
  if (rc != LRHE_OK) return rc;
  if (count > max_count) return fail(LRHE_EINVAL, "wire: %llu ciphertexts, room for %u", (unsigned long long)count,
                                     max_count);
  const uint64_t n = c->n, L = c->L, limbs = count * 2 * L;
  std::vector<uint32_t> h(limbs * n);
  std::memcpy(h.data(), in + sizeof(Header), h.size() * 4);
  int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : bad)
  for (int64_t x = 0; x < (int64_t)limbs; ++x) {
    uint32_t* a = h.data() + (uint64_t)x * n;
    if (!limb_ok(a, (uint32_t)n, c->q[x % L])) {
      ++bad;
      continue;
    }
    host_transform_limb(c, (int)(x % L), a, false);
  }
  if (bad) return fail(LRHE_EINVAL, "wire: %d limbs hold residues outside their modulus", bad);
  if (flags & LRHE_CT_HOST) {
    std::memcpy(ct_out, h.data(), h.size() * 4);
  } else {
    if (c->device < 0) return fail(LRHE_EDEVICE, "host-only context: pass LRHE_CT_HOST");
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = hipMemcpyAsync(ct_out, h.data(), h.size() * 4, hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return fail(LRHE_EDEVICE, "wire: copy: %s", hipGetErrorString(e));
  }
  if (count_out) *count_out = (uint32_t)count;
  return LRHE_OK;
}

extern "C" int lrhe_key_serialize(lrhe_ctx* c, int kind, const void* key, uint8_t* out, uint64_t cap) {
  if (!c || !key || !out) return fail(LRHE_EINVAL, "null argument");
  if (kind < K_GK || kind > K_SK) return fail(LRHE_EINVAL, "wire: kind %d is not a key", kind);
  const uint64_t plen = payload_bytes(c, (uint32_t)kind, 1);
  if (cap < sizeof(Header) + plen) return fail(LRHE_EINVAL, "wire: buffer of %llu bytes, %llu needed",
                                               (unsigned long long)cap, (unsigned long long)(sizeof(Header) + plen));
  uint8_t* P = out + sizeof(Header);
  int rc = LRHE_OK;
  uint64_t count = 1;
  if (kind == K_GK) {
    rc = lrhe_gk_export(c, static_cast<const lrhe_gk*>(key), reinterpret_cast<uint32_t*>(P));
    count = c->ngal;
  } else if (kind == K_PK) {
    rc = lrhe_pk_export(c, static_cast<const lrhe_pk*>(key), reinterpret_cast<uint32_t*>(P));
  } else {
    rc = lrhe_sk_export(c, static_cast<const lrhe_sk*>(key), reinterpret_cast<int8_t*>(P));
  }
  if (rc != LRHE_OK) return rc;
  return write_header(c, (uint32_t)kind, count, P, plen, out);
}

extern "C" int lrhe_gk_deserialize(lrhe_ctx* c, const uint8_t* in, uint64_t bytes, lrhe_gk** out) {
  if (!c || !in || !out) return fail(LRHE_EINVAL, "null argument");
  *out = nullptr;
  uint64_t count = 0;
  int rc = read_header(c, in, bytes, K_GK, &count);
  if (rc != LRHE_OK) return rc;
  if (count != c->ngal) return fail(LRHE_EINVAL, "wire: %llu Galois keys, expected %u", (unsigned long long)count,
                                    c->ngal);
  const uint32_t n = c->n, L = c->L;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(in + sizeof(Header));
  auto* gk = new lrhe_gk();
  gk->words = (size_t)c->ngal * (L + 1) * L * 2 * n;
  gk->h.assign(gk->words, 0);
  int bad = 0;
  // wire layout [g][i][x][r][n] (coefficients) -> [g][r][i][x][n] (evaluation form)
#pragma omp parallel for collapse(2) reduction(+ : bad)
  for (int gi = 0; gi < (int)c->ngal; ++gi)
    for (int r = 0; r <= (int)L; ++r)
      for (uint32_t i = 0; i < L; ++i)
        for (uint32_t x = 0; x < 2; ++x) {
          const uint32_t* s = src + ((((size_t)gi * L + i) * 2 + x) * (L + 1) + r) * n;
          uint32_t* d = &gk->h[((((size_t)gi * (L + 1) + r) * L + i) * 2 + x) * n];
          if (!limb_ok(s, n, c->q[r])) {
            ++bad;
            continue;
          }
          std::memcpy(d, s, (size_t)n * 4);
          host_transform_limb(c, r, d, false);
        }
  if (bad) {
    lrhe_gk_destroy(gk);
    return fail(LRHE_EINVAL, "wire: %d key limbs hold residues outside their modulus", bad);
  }
  const hipError_t e = upload_gk(c, gk);
  if (e != hipSuccess) {
    lrhe_gk_destroy(gk);
    return fail(LRHE_EDEVICE, "wire: Galois key upload: %s", hipGetErrorString(e));
  }
  *out = gk;
  return LRHE_OK;
}

extern "C" int lrhe_pk_deserialize(lrhe_ctx* c, const uint8_t* in, uint64_t bytes, lrhe_pk** out) {
  if (!c || !in || !out) return fail(LRHE_EINVAL, "null argument");
  *out = nullptr;
  uint64_t count = 0;
  int rc = read_header(c, in, bytes, K_PK, &count);
  if (rc != LRHE_OK) return rc;
  const uint32_t n = c->n, L = c->L;
  auto* pk = new lrhe_pk();
  pk->h.assign((size_t)2 * L * n, 0);
  std::memcpy(pk->h.data(), in + sizeof(Header), pk->h.size() * 4);
  for (uint32_t x = 0; x < 2 * L; ++x) {
    uint32_t* a = &pk->h[(size_t)x * n];
    if (!limb_ok(a, n, c->q[x % L])) {
      lrhe_pk_destroy(pk);
      return fail(LRHE_EINVAL, "wire: public key limb %u holds residues outside its modulus", x);
    }
    host_transform_limb(c, (int)(x % L), a, false);
  }
  const hipError_t e = upload_pk(c, pk);
  if (e != hipSuccess) {
    lrhe_pk_destroy(pk);
    return fail(LRHE_EDEVICE, "wire: public key upload: %s", hipGetErrorString(e));
  }
  *out = pk;
  return LRHE_OK;
}

extern "C" int lrhe_sk_deserialize(lrhe_ctx* c, const uint8_t* in, uint64_t bytes, lrhe_sk** out) {
  if (!c || !in || !out) return fail(LRHE_EINVAL, "null argument");
  *out = nullptr;
  uint64_t count = 0;
  int rc = read_header(c, in, bytes, K_SK, &count);
  if (rc != LRHE_OK) return rc;
  const int8_t* s8 = reinterpret_cast<const int8_t*>(in + sizeof(Header));
  std::vector<int32_t> s(c->n);
  for (uint32_t k = 0; k < c->n; ++k) {
    if (s8[k] < -1 || s8[k] > 1) return fail(LRHE_EINVAL, "wire: secret key coefficient %u is not ternary", k);
    s[k] = s8[k];
  }
  *out = make_sk(c, s.data());
  return LRHE_OK;
}
