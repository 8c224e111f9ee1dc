/*
 * bfv_oracle.c -- plain, slow CPU reference of the encrypted logistic-regression
 * matrix multiplication (BFV), used ONLY as test infrastructure.
 *
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
 * load this library.  It shares no code, header, table or constant generator
 * with the HIP path in paper_2204_05496_amd/: every constant here (primitive
 * roots, twiddle powers, RNS constants, slot map) is derived in this file from
 * its mathematical definition.
 *
 * Paper: "Scalable privacy-preserving cancer type prediction with homomorphic
 * encryption" (arXiv 2204.05496).
 *   - Private inference protocol: section "Private inference protocol"
 *     (client scales/encodes/encrypts X, server computes X^ x W- + B-, client
 *     decrypts and decodes).
 *   - Fast matrix multiplication: Algorithm 1 ("Proposed matrix multiplication
 *     algorithm") and section "Matrix multiplication algorithm": per (input,
 *     output) pair, chunk-wise ciphertext x plaintext products, add_many,
 *     log2(n) rotate-and-accumulate steps, one-hot masking, compression.
 *   - Standard encrypted matrix multiplication: section "Comparison to
 *     standard LR" (baseline; the paper does not specify it further).
 *   - argmax of the scores: section "Approximation of non-linear function in
 *     private inference".
 * The paper runs on SEAL and leaves the BFV conventions (slot layout, key
 * switching, sampling) implicit; the conventions used here are stated next to
 * each function and in the design notes of the repository.
 *
 * Arithmetic: every residue is a uint64_t in [0, m) with m < 2^31, so a product
 * of two residues fits in 62 bits and is reduced with the C '%' operator.
 * Polynomials are in coefficient form, layout [limb][n].
 *
 * Parity status: every function below is pinned by the -m "not gpu" tests
 * (schoolbook products, definitional encode/decode, brute-force automorphisms,
 * big-integer rounding of the key-switch mod-down, Dec(Enc(m)) = m, the trace
 * invariant and the plain integer matmul).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

#define ORA_MAXL 16

/* ------------------------------------------------------------------ */
/* modular arithmetic (plain)                                          */
/* ------------------------------------------------------------------ */
static u64 mulmod(u64 a, u64 b, u64 m) { return (a * b) % m; }
static u64 addmod(u64 a, u64 b, u64 m) { return (a + b) % m; }
static u64 submod(u64 a, u64 b, u64 m) { return (a + m - b) % m; }
static u64 powmod(u64 b, u64 e, u64 m) {
  u64 r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod(r, b, m);
    b = mulmod(b, b, m);
    e >>= 1;
  }
  return r;
}
static u64 invmod(u64 a, u64 p) { return powmod(a, p - 2, p); } /* p prime */
static u64 reduce_signed(i64 v, u64 m) {
  i64 r = v % (i64)m;
  return (u64)(r < 0 ? r + (i64)m : r);
}

/* smallest generator of (Z/p)^*, p prime: g such that g^((p-1)/r) != 1 for
 * every prime r dividing p-1 */
static u64 smallest_generator(u64 p) {
  u64 f[64];
  int nf = 0;
  u64 m = p - 1;
  for (u64 d = 2; d * d <= m; ++d) {
    if (m % d == 0) {
      f[nf++] = d;
      while (m % d == 0) m /= d;
    }
  }
  if (m > 1) f[nf++] = m;
  for (u64 g = 2; g < p; ++g) {
    int ok = 1;
    for (int i = 0; i < nf && ok; ++i)
      if (powmod(g, (p - 1) / f[i], p) == 1) ok = 0;
    if (ok) return g;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* textbook negacyclic NTT: A[k] = sum_i a_i psi^((2k+1) i)            */
/* ------------------------------------------------------------------ */
typedef struct {
  u64 m;           /* modulus */
  int n, logn;
  u64 psi, n_inv;  /* psi: primitive 2n-th root of unity mod m */
  u64* psi_pow;    /* psi^i, i < n */
  u64* psi_ipow;   /* psi^-i, i < n */
  u64* w_pow;      /* omega^i = psi^(2i), i < n */
  u64* w_ipow;     /* omega^-i, i < n */
} ora_ntt;

static int ntt_init(ora_ntt* T, u64 m, int n) {
  memset(T, 0, sizeof(*T));
  T->m = m;
  T->n = n;
  while ((1 << T->logn) < n) T->logn++;
  if ((m - 1) % (2 * (u64)n) != 0) return -1;
  u64 g = smallest_generator(m);
  T->psi = powmod(g, (m - 1) / (2 * (u64)n), m);
  T->n_inv = invmod((u64)n, m);
  T->psi_pow = (u64*)malloc(sizeof(u64) * n);
  T->psi_ipow = (u64*)malloc(sizeof(u64) * n);
  T->w_pow = (u64*)malloc(sizeof(u64) * n);
  T->w_ipow = (u64*)malloc(sizeof(u64) * n);
  u64 psi_inv = invmod(T->psi, m);
  u64 a = 1, b = 1;
  for (int i = 0; i < n; ++i) {
    T->psi_pow[i] = a;
    T->psi_ipow[i] = b;
    a = mulmod(a, T->psi, m);
    b = mulmod(b, psi_inv, m);
  }
  for (int i = 0; i < n; ++i) {
    T->w_pow[i] = powmod(T->psi, 2 * (u64)i, m);
    T->w_ipow[i] = powmod(psi_inv, 2 * (u64)i, m);
  }
  return 0;
}
static void ntt_free(ora_ntt* T) {
  free(T->psi_pow);
  free(T->psi_ipow);
  free(T->w_pow);
  free(T->w_ipow);
}

/* cyclic DFT of length n with root table wtab (omega^i or omega^-i):
 * bit-reversal permutation followed by iterative radix-2 Cooley-Tukey */
static void dft_cyclic(const ora_ntt* T, u64* a, const u64* wtab) {
  const int n = T->n;
  const u64 m = T->m;
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      u64 tmp = a[i];
      a[i] = a[j];
      a[j] = tmp;
    }
  }
  for (int len = 2; len <= n; len <<= 1) {
    const int step = n / len;
    for (int s = 0; s < n; s += len) {
      for (int j = 0; j < len / 2; ++j) {
        u64 w = wtab[step * j];
        u64 u = a[s + j];
        u64 v = mulmod(a[s + j + len / 2], w, m);
        a[s + j] = addmod(u, v, m);
        a[s + j + len / 2] = submod(u, v, m);
      }
    }
  }
}

/* out[k] = a(psi^(2k+1)) for k < n (natural order) */
static void ntt_eval(const ora_ntt* T, const u64* a, u64* out) {
  for (int i = 0; i < T->n; ++i) out[i] = mulmod(a[i] % T->m, T->psi_pow[i], T->m);
  dft_cyclic(T, out, T->w_pow);
}
/* inverse of ntt_eval */
static void ntt_interp(const ora_ntt* T, const u64* A, u64* out) {
  if (out != A) memcpy(out, A, sizeof(u64) * T->n);
  dft_cyclic(T, out, T->w_ipow);
  for (int i = 0; i < T->n; ++i) out[i] = mulmod(mulmod(out[i], T->n_inv, T->m), T->psi_ipow[i], T->m);
}

/* ------------------------------------------------------------------ */
/* ChaCha20 block function, RFC 8439 section 2.3                        */
/* ------------------------------------------------------------------ */
#define ORA_ROTL(x, r) (((x) << (r)) | ((x) >> (32 - (r))))
static void quarter_round(u32* x, int a, int b, int c, int d) {
  x[a] += x[b]; x[d] ^= x[a]; x[d] = ORA_ROTL(x[d], 16);
  x[c] += x[d]; x[b] ^= x[c]; x[b] = ORA_ROTL(x[b], 12);
  x[a] += x[b]; x[d] ^= x[a]; x[d] = ORA_ROTL(x[d], 8);
  x[c] += x[d]; x[b] ^= x[c]; x[b] = ORA_ROTL(x[b], 7);
}
void ora_chacha20_block(const u32 key[8], u32 counter, const u32 nonce[3], u32 out[16]) {
  u32 s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u};
  for (int i = 0; i < 8; ++i) s[4 + i] = key[i];
  s[12] = counter;
  s[13] = nonce[0];
  s[14] = nonce[1];
  s[15] = nonce[2];
  u32 x[16];
  memcpy(x, s, sizeof(x));
  for (int r = 0; r < 10; ++r) {
    quarter_round(x, 0, 4, 8, 12);
    quarter_round(x, 1, 5, 9, 13);
    quarter_round(x, 2, 6, 10, 14);
    quarter_round(x, 3, 7, 11, 15);
    quarter_round(x, 0, 5, 10, 15);
    quarter_round(x, 1, 6, 11, 12);
    quarter_round(x, 2, 7, 8, 13);
    quarter_round(x, 3, 4, 9, 14);
  }
  for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

/* Word w of the stream for (seed, kind, id): key = seed as two little-endian
 * words followed by six zero words; nonce = (kind, id low, id high);
 * block counter = w / 16. */
typedef struct {
  u32 key[8], nonce[3];
  u32 block[16];
  u32 cur;   /* index of the cached block, or 0xffffffff */
} ora_stream;
static void stream_init(ora_stream* S, u64 seed, u32 kind, u64 id) {
  memset(S, 0, sizeof(*S));
  S->key[0] = (u32)seed;
  S->key[1] = (u32)(seed >> 32);
  S->nonce[0] = kind;
  S->nonce[1] = (u32)id;
  S->nonce[2] = (u32)(id >> 32);
  S->cur = 0xffffffffu;
}
static u32 stream_word(ora_stream* S, u64 w) {
  u32 b = (u32)(w >> 4);
  if (b != S->cur) {
    ora_chacha20_block(S->key, b, S->nonce, S->block);
    S->cur = b;
  }
  return S->block[w & 15];
}

/* uniform residue mod m: 2 words per coefficient, ((hi << 32) | lo) mod m */
void ora_sample_uniform(u64 seed, u32 kind, u64 id, u64 m, int n, u64* out) {
  ora_stream S;
  stream_init(&S, seed, kind, id);
  for (int k = 0; k < n; ++k) {
    u64 lo = stream_word(&S, 2 * (u64)k), hi = stream_word(&S, 2 * (u64)k + 1);
    out[k] = ((hi << 32) | lo) % m;
  }
}
/* ternary: 1 word per coefficient, w mod 3 -> {0, +1, -1} */
void ora_sample_ternary(u64 seed, u32 kind, u64 id, int n, i64* out) {
  ora_stream S;
  stream_init(&S, seed, kind, id);
  for (int k = 0; k < n; ++k) {
    u32 r = stream_word(&S, (u64)k) % 3u;
    out[k] = r == 0 ? 0 : (r == 1 ? 1 : -1);
  }
}
/* centred binomial, eta = 21: 2 words per coefficient; with v = (hi << 32) | lo,
 * value = popcount(v bits 0..20) - popcount(v bits 21..41) */
static int popcnt64(u64 v) {
  int c = 0;
  while (v) {
    c += (int)(v & 1);
    v >>= 1;
  }
  return c;
}
void ora_sample_cbd(u64 seed, u32 kind, u64 id, int n, i64* out) {
  ora_stream S;
  stream_init(&S, seed, kind, id);
  const u64 mask21 = (1ull << 21) - 1;
  for (int k = 0; k < n; ++k) {
    u64 lo = stream_word(&S, 2 * (u64)k), hi = stream_word(&S, 2 * (u64)k + 1);
    u64 v = (hi << 32) | lo;
    out[k] = (i64)popcnt64(v & mask21) - (i64)popcnt64((v >> 21) & mask21);
  }
}

/* object kinds of the random streams */
enum { K_SECRET = 1, K_PK_A = 2, K_PK_E = 3, K_GK_A = 4, K_GK_E = 5, K_ENC_U = 6, K_ENC_E0 = 7, K_ENC_E1 = 8 };

/* ------------------------------------------------------------------ */
/* context                                                             */
/* ------------------------------------------------------------------ */
typedef struct {
  int n, logn, L;         /* L data primes q_0..q_{L-1}; modulus index L is the special prime P */
  u64 q[ORA_MAXL + 1];
  u64 t;
  ora_ntt T[ORA_MAXL + 1];
  ora_ntt Tt;             /* mod t, for batch encoding */
  u64 psi_t;              /* smallest generator of Z_t^* raised to (t-1)/2n */
  u32* slot_pos;          /* slot j -> k with psi_t^(2k+1) = psi_t^(e_j) */
  int ngal;
  u32 gal[64];            /* Galois elements of the rotate-and-sum, in order */
  u64 qmod_t;             /* Q mod t */
  u64 qdivt_mod[ORA_MAXL];/* floor(Q/t) mod q_i */
} ora_ctx;

ora_ctx* ora_ctx_new(int n, int L, const u64* q_and_p, u64 t) {
  if (L < 1 || L > ORA_MAXL || n < 4 || (n & (n - 1))) return NULL;
  ora_ctx* c = (ora_ctx*)calloc(1, sizeof(ora_ctx));
  c->n = n;
  c->L = L;
  while ((1 << c->logn) < n) c->logn++;
  for (int i = 0; i <= L; ++i) {
    c->q[i] = q_and_p[i];
    if (ntt_init(&c->T[i], c->q[i], n)) { free(c); return NULL; }
  }
  c->t = t;
  if (ntt_init(&c->Tt, t, n)) { free(c); return NULL; }
  c->psi_t = c->Tt.psi;
  /* slot j < n/2 <-> exponent 3^j mod 2n; slot n/2 + j <-> -3^j mod 2n */
  c->slot_pos = (u32*)malloc(sizeof(u32) * n);
  u64 e = 1;
  for (int j = 0; j < n / 2; ++j) {
    c->slot_pos[j] = (u32)((e - 1) / 2);
    c->slot_pos[n / 2 + j] = (u32)((2 * (u64)n - e - 1) / 2);
    e = (e * 3) % (2 * (u64)n);
  }
  /* Galois elements: rotations by n/4, n/8, ..., 1 within the rows, then the row swap */
  c->ngal = 0;
  for (u64 s = (u64)n / 4; s >= 1; s /= 2) c->gal[c->ngal++] = (u32)powmod(3, s, 2 * (u64)n);
  c->gal[c->ngal++] = (u32)(2 * n - 1);
  /* Q mod t and floor(Q/t) mod q_i = -(Q mod t) * t^-1 mod q_i */
  u64 qt = 1;
  for (int i = 0; i < L; ++i) qt = mulmod(qt, c->q[i] % t, t);
  c->qmod_t = qt;
  for (int i = 0; i < L; ++i)
    c->qdivt_mod[i] = mulmod(submod(0, qt % c->q[i], c->q[i]), invmod(t % c->q[i], c->q[i]), c->q[i]);
  return c;
}
void ora_ctx_free(ora_ctx* c) {
  if (!c) return;
  for (int i = 0; i <= c->L; ++i) ntt_free(&c->T[i]);
  ntt_free(&c->Tt);
  free(c->slot_pos);
  free(c);
}
int ora_ngal(const ora_ctx* c) { return c->ngal; }
u32 ora_gal(const ora_ctx* c, int i) { return c->gal[i]; }
u64 ora_psi_t(const ora_ctx* c) { return c->psi_t; }
u64 ora_qmod_t(const ora_ctx* c) { return c->qmod_t; }
u64 ora_qdivt_mod(const ora_ctx* c, int i) { return c->qdivt_mod[i]; }
u32 ora_slot_pos(const ora_ctx* c, int j) { return c->slot_pos[j]; }

/* ------------------------------------------------------------------ */
/* ring operations in Z_m[X]/(X^n + 1)                                 */
/* ------------------------------------------------------------------ */
/* schoolbook negacyclic product (the definition) */
void ora_ring_mul_schoolbook(u64 m, int n, const u64* a, const u64* b, u64* out) {
  for (int k = 0; k < n; ++k) out[k] = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      u64 p = mulmod(a[i] % m, b[j] % m, m);
      int k = i + j;
      if (k < n) out[k] = addmod(out[k], p, m);
      else out[k - n] = submod(out[k - n], p, m);
    }
}
/* negacyclic product through the transform; modulus index mi (L = special prime, -1 = t) */
static const ora_ntt* tr(const ora_ctx* c, int mi) { return mi < 0 ? &c->Tt : &c->T[mi]; }
void ora_ring_mul(const ora_ctx* c, int mi, const u64* a, const u64* b, u64* out) {
  const ora_ntt* T = tr(c, mi);
  u64* A = (u64*)malloc(sizeof(u64) * c->n);
  u64* B = (u64*)malloc(sizeof(u64) * c->n);
  ntt_eval(T, a, A);
  ntt_eval(T, b, B);
  for (int k = 0; k < c->n; ++k) A[k] = mulmod(A[k], B[k], T->m);
  ntt_interp(T, A, out);
  free(A);
  free(B);
}
void ora_ntt_eval(const ora_ctx* c, int mi, const u64* a, u64* out) { ntt_eval(tr(c, mi), a, out); }
void ora_ntt_interp(const ora_ctx* c, int mi, const u64* A, u64* out) { ntt_interp(tr(c, mi), A, out); }

/* automorphism sigma_g: a(X) -> a(X^g) mod (X^n + 1), g odd */
static void automorph(int n, u64 m, u32 g, const u64* a, u64* out) {
  const u64 twon = 2 * (u64)n;
  for (int k = 0; k < n; ++k) {
    u64 idx = ((u64)g * (u64)k) % twon;
    if (idx < (u64)n) out[idx] = a[k];
    else out[idx - n] = submod(0, a[k], m);
  }
}
void ora_automorph(const ora_ctx* c, int mi, u32 g, const u64* a, u64* out) {
  automorph(c->n, tr(c, mi)->m, g, a, out);
}

/* ------------------------------------------------------------------ */
/* batch encoding (slots <-> plaintext polynomial mod t)               */
/* slot j is the evaluation at psi_t^(e_j), e_j = 3^j (j < n/2) and    */
/* -3^(j-n/2) (j >= n/2) modulo 2n                                     */
/* ------------------------------------------------------------------ */
void ora_encode(const ora_ctx* c, const u64* slots, u64* m) {
  u64* v = (u64*)malloc(sizeof(u64) * c->n);
  for (int j = 0; j < c->n; ++j) v[c->slot_pos[j]] = slots[j] % c->t;
  ntt_interp(&c->Tt, v, m);
  free(v);
}
void ora_decode(const ora_ctx* c, const u64* m, u64* slots) {
  u64* v = (u64*)malloc(sizeof(u64) * c->n);
  ntt_eval(&c->Tt, m, v);
  for (int j = 0; j < c->n; ++j) slots[j] = v[c->slot_pos[j]];
  free(v);
}
/* centred lift of a residue mod t into modulus m: v in (-t/2, t/2] */
static u64 lift_centred(u64 v, u64 t, u64 m) {
  i64 s = v > (t - 1) / 2 ? (i64)v - (i64)t : (i64)v;
  return reduce_signed(s, m);
}
/* Delta(v) = round(Q v / t) mod q_i = floor(Q/t) v + round((Q mod t) v / t) */
static u64 delta_mod(const ora_ctx* c, int i, u64 v) {
  u64 r = (c->qmod_t * v + (c->t - 1) / 2) / c->t;
  return addmod(mulmod(c->qdivt_mod[i], v, c->q[i]), r % c->q[i], c->q[i]);
}
u64 ora_delta_mod(const ora_ctx* c, int i, u64 v) { return delta_mod(c, i, v); }

/* ------------------------------------------------------------------ */
/* keys                                                                */
/* layouts: pk [2][L][n]; gk [ngal][L digits][2 (b, a)][L+1][n]         */
/* ------------------------------------------------------------------ */
size_t ora_gk_words(const ora_ctx* c) { return (size_t)c->ngal * c->L * 2 * (c->L + 1) * c->n; }

void ora_keygen(const ora_ctx* c, u64 seed, i64* s, u64* pk, u64* gk) {
  const int n = c->n, L = c->L;
  ora_sample_ternary(seed, K_SECRET, 0, n, s);
  u64* sr = (u64*)malloc(sizeof(u64) * n);
  u64* a = (u64*)malloc(sizeof(u64) * n);
  u64* as = (u64*)malloc(sizeof(u64) * n);
  i64* e = (i64*)malloc(sizeof(i64) * n);
  /* public key: pk = (-(a s + e), a) mod Q */
  ora_sample_cbd(seed, K_PK_E, 0, n, e);
  for (int j = 0; j < L; ++j) {
    const u64 m = c->q[j];
    for (int k = 0; k < n; ++k) sr[k] = reduce_signed(s[k], m);
    ora_sample_uniform(seed, K_PK_A, (u64)j, m, n, a);
    ora_ring_mul(c, j, a, sr, as);
    for (int k = 0; k < n; ++k) {
      pk[(size_t)j * n + k] = submod(0, addmod(as[k], reduce_signed(e[k], m), m), m);
      pk[(size_t)(L + j) * n + k] = a[k];
    }
  }
  /* Galois keys: ksk_{g,i} mod r = (-(a s + e) + [P]_r delta_{i r} sigma_g(s), a) over r in Q u {P} */
  if (gk) {
    u64* sg = (u64*)malloc(sizeof(u64) * n);
    for (int gi = 0; gi < c->ngal; ++gi) {
      for (int i = 0; i < L; ++i) {
        ora_sample_cbd(seed, K_GK_E, (u64)gi * L + i, n, e);
        for (int r = 0; r <= L; ++r) {
          const u64 m = c->q[r];
          for (int k = 0; k < n; ++k) sr[k] = reduce_signed(s[k], m);
          ora_sample_uniform(seed, K_GK_A, ((u64)gi * L + i) * (L + 1) + r, m, n, a);
          ora_ring_mul(c, r, a, sr, as);
          u64* kb = gk + ((((size_t)gi * L + i) * 2 + 0) * (L + 1) + r) * n;
          u64* ka = gk + ((((size_t)gi * L + i) * 2 + 1) * (L + 1) + r) * n;
          if (r == i) automorph(n, m, c->gal[gi], sr, sg);
          const u64 Pm = c->q[L] % m;
          for (int k = 0; k < n; ++k) {
            u64 b = submod(0, addmod(as[k], reduce_signed(e[k], m), m), m);
            if (r == i) b = addmod(b, mulmod(Pm, sg[k], m), m);
            kb[k] = b;
            ka[k] = a[k];
          }
        }
      }
    }
    free(sg);
  }
  free(sr);
  free(a);
  free(as);
  free(e);
}

/* ------------------------------------------------------------------ */
/* encryption: ct = ([pk0 u + e0 + Delta(m)]_Q, [pk1 u + e1]_Q)         */
/* m: plaintext coefficients in [0, t); ct layout [2][L][n]             */
/* ------------------------------------------------------------------ */
void ora_encrypt(const ora_ctx* c, const u64* pk, const u64* m, u64 seed, u64 ct_id, u64* ct) {
  const int n = c->n, L = c->L;
  i64* u = (i64*)malloc(sizeof(i64) * n);
  i64* e0 = (i64*)malloc(sizeof(i64) * n);
  i64* e1 = (i64*)malloc(sizeof(i64) * n);
  u64* ur = (u64*)malloc(sizeof(u64) * n);
  u64* p0 = (u64*)malloc(sizeof(u64) * n);
  u64* p1 = (u64*)malloc(sizeof(u64) * n);
  ora_sample_ternary(seed, K_ENC_U, ct_id, n, u);
  ora_sample_cbd(seed, K_ENC_E0, ct_id, n, e0);
  ora_sample_cbd(seed, K_ENC_E1, ct_id, n, e1);
  for (int j = 0; j < L; ++j) {
    const u64 q = c->q[j];
    for (int k = 0; k < n; ++k) ur[k] = reduce_signed(u[k], q);
    ora_ring_mul(c, j, pk + (size_t)j * n, ur, p0);
    ora_ring_mul(c, j, pk + (size_t)(L + j) * n, ur, p1);
    for (int k = 0; k < n; ++k) {
      ct[(size_t)j * n + k] = addmod(addmod(p0[k], reduce_signed(e0[k], q), q), delta_mod(c, j, m[k] % c->t), q);
      ct[(size_t)(L + j) * n + k] = addmod(p1[k], reduce_signed(e1[k], q), q);
    }
  }
  free(u); free(e0); free(e1); free(ur); free(p0); free(p1);
}

/* ------------------------------------------------------------------ */
/* homomorphic steps on one ciphertext ([2][L][n])                      */
/* ------------------------------------------------------------------ */
/* ct x pt: (c0 w, c1 w), w = centred lift of the plaintext w_t (values mod t) */
void ora_mul_plain(const ora_ctx* c, const u64* ct, const u64* w_t, u64* out) {
  const int n = c->n, L = c->L;
  u64* w = (u64*)malloc(sizeof(u64) * n);
  for (int j = 0; j < L; ++j) {
    for (int k = 0; k < n; ++k) w[k] = lift_centred(w_t[k] % c->t, c->t, c->q[j]);
    ora_ring_mul(c, j, ct + (size_t)j * n, w, out + (size_t)j * n);
    ora_ring_mul(c, j, ct + (size_t)(L + j) * n, w, out + (size_t)(L + j) * n);
  }
  free(w);
}
void ora_add(const ora_ctx* c, const u64* a, const u64* b, u64* out) {
  const size_t N = (size_t)2 * c->L * c->n;
  for (size_t k = 0; k < N; ++k) {
    const u64 q = c->q[(k / c->n) % c->L];
    out[k] = addmod(a[k], b[k], q);
  }
}
/* add_plain of the all-slot plaintext v (the constant polynomial v): c0 += Delta(v) X^0 */
void ora_add_const(const ora_ctx* c, u64 v_t, u64* ct) {
  for (int j = 0; j < c->L; ++j)
    ct[(size_t)j * c->n] = addmod(ct[(size_t)j * c->n], delta_mod(c, j, v_t % c->t), c->q[j]);
}

/* Key switch of d = sigma_g(c1) with ksk_g ([L][2][L+1][n], coefficient form), the
 * RNS digits of d being its limbs [d]_{q_i} read as integers in [0, q_i):
 *   acc_{x,r} = sum_i [d_i]_r * ksk_{g,i}.x  mod (X^n+1, r), r over q_0..q_{L-1}, P
 *   rounded division by P with h = (P-1)/2:
 *   rho_x = [acc_{x,P} + h]_P, out_{x,j} = (acc_{x,j} + h - rho_x) P^-1 mod q_j
 * kev (optional): the same key in transform form per modulus (ntt_eval), used to
 * avoid re-transforming the key on every call. */
void ora_key_switch(const ora_ctx* c, const u64* d, const u64* ksk, const u64* kev, u64* out_b, u64* out_a) {
  const int n = c->n, L = c->L;
  const u64 P = c->q[L], h = (P - 1) / 2;
  u64* acc = (u64*)malloc(sizeof(u64) * 2 * (L + 1) * n);   /* [x][r][n] coefficient form */
  u64* dr = (u64*)malloc(sizeof(u64) * n);
  u64* D = (u64*)malloc(sizeof(u64) * n);
  u64* K = (u64*)malloc(sizeof(u64) * n);
  u64* A = (u64*)malloc(sizeof(u64) * 2 * n);
  for (int r = 0; r <= L; ++r) {
    const u64 m = c->q[r];
    memset(A, 0, sizeof(u64) * 2 * n);
    for (int i = 0; i < L; ++i) {
      for (int k = 0; k < n; ++k) dr[k] = d[(size_t)i * n + k] % m;
      ntt_eval(&c->T[r], dr, D);
      for (int x = 0; x < 2; ++x) {
        const size_t off = (((size_t)i * 2 + x) * (L + 1) + r) * n;
        const u64* Kx;
        if (kev) Kx = kev + off;
        else { ntt_eval(&c->T[r], ksk + off, K); Kx = K; }
        for (int k = 0; k < n; ++k) A[(size_t)x * n + k] = addmod(A[(size_t)x * n + k], mulmod(D[k], Kx[k], m), m);
      }
    }
    ntt_interp(&c->T[r], A, acc + ((size_t)0 * (L + 1) + r) * n);
    ntt_interp(&c->T[r], A + n, acc + ((size_t)1 * (L + 1) + r) * n);
  }
  for (int x = 0; x < 2; ++x) {
    u64* o = x == 0 ? out_b : out_a;
    const u64* aP = acc + ((size_t)x * (L + 1) + L) * n;
    for (int j = 0; j < L; ++j) {
      const u64 q = c->q[j];
      const u64 pinv = invmod(P % q, q);
      const u64* aj = acc + ((size_t)x * (L + 1) + j) * n;
      for (int k = 0; k < n; ++k) {
        u64 rho = addmod(aP[k], h, P);
        u64 v = submod(addmod(aj[k], h % q, q), rho % q, q);
        o[(size_t)j * n + k] = mulmod(v, pinv, q);
      }
    }
  }
  free(acc); free(dr); free(D); free(K); free(A);
}

/* key in transform form, same layout as the key */
void ora_gk_transform(const ora_ctx* c, const u64* gk, u64* gk_ev) {
  const int n = c->n, L = c->L;
  const size_t polys = (size_t)c->ngal * L * 2 * (L + 1);
#pragma omp parallel for schedule(dynamic)
  for (size_t p = 0; p < polys; ++p) ntt_eval(&c->T[p % (L + 1)], gk + p * n, gk_ev + p * n);
}

/* one rotate-and-accumulate step: ct <- ct + KS_g(sigma_g(ct)), g = gal[gi] */
void ora_rotate_add(const ora_ctx* c, const u64* gk, const u64* gk_ev, int gi, u64* ct) {
  const int n = c->n, L = c->L;
  const size_t keysz = (size_t)L * 2 * (L + 1) * n;
  const u32 g = c->gal[gi];
  u64* s0 = (u64*)malloc(sizeof(u64) * L * n);
  u64* s1 = (u64*)malloc(sizeof(u64) * L * n);
  u64* ob = (u64*)malloc(sizeof(u64) * L * n);
  u64* oa = (u64*)malloc(sizeof(u64) * L * n);
  for (int j = 0; j < L; ++j) {
    automorph(n, c->q[j], g, ct + (size_t)j * n, s0 + (size_t)j * n);
    automorph(n, c->q[j], g, ct + (size_t)(L + j) * n, s1 + (size_t)j * n);
  }
  ora_key_switch(c, s1, gk + gi * keysz, gk_ev ? gk_ev + gi * keysz : NULL, ob, oa);
  for (int j = 0; j < L; ++j) {
    const u64 q = c->q[j];
    for (int k = 0; k < n; ++k) {
      size_t x = (size_t)j * n + k;
      ct[x] = addmod(ct[x], addmod(s0[x], ob[x], q), q);
      ct[(size_t)L * n + x] = addmod(ct[(size_t)L * n + x], oa[x], q);
    }
  }
  free(s0); free(s1); free(ob); free(oa);
}

/* plaintext of the one-hot slot l (the "encodeAt" of Algorithm 1), values mod t */
void ora_onehot_plain(const ora_ctx* c, int l, u64* m) {
  u64* z = (u64*)calloc(c->n, sizeof(u64));
  z[l] = 1;
  ora_encode(c, z, m);
  free(z);
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 for one (input i, output j) pair up to the masked ciphertext.
 * xct: the K ciphertexts of row i; wpt: the K plaintexts (values mod t) of
 * class j; bias_t: b_j mod t; slot: l = (i |W| + j) mod n.
 * stage (debug): 0 = full; 1 = stop after add_many; 2 + s = stop after s rotation steps
 * (s <= log2 n); 100 = stop after the bias. */
void ora_pair(const ora_ctx* c, const u64* gk, const u64* gk_ev, const u64* xct, const u64* wpt, int K,
              u64 bias_t, int slot, int stage, u64* out) {
  const int n = c->n, L = c->L;
  const size_t C = (size_t)2 * L * n;
  u64* tmp = (u64*)malloc(sizeof(u64) * C);
  memset(out, 0, sizeof(u64) * C);
  for (int k = 0; k < K; ++k) {          /* multiplication and add_many */
    ora_mul_plain(c, xct + k * C, wpt + (size_t)k * n, tmp);
    ora_add(c, out, tmp, out);
  }
  if (stage == 1) { free(tmp); return; }
  for (int gi = 0; gi < c->ngal; ++gi) {  /* rotate and accumulate */
    if (stage >= 2 && stage < 100 && gi == stage - 2) { free(tmp); return; }
    ora_rotate_add(c, gk, gk_ev, gi, out);
  }
  if (stage == 2 + c->ngal) { free(tmp); return; }   /* after every rotation step */
  ora_add_const(c, bias_t, out);          /* all-slot bias b_j */
  if (stage == 100) { free(tmp); return; }
  u64* mu = (u64*)malloc(sizeof(u64) * n); /* masking */
  ora_onehot_plain(c, slot, mu);
  ora_mul_plain(c, out, mu, tmp);
  memcpy(out, tmp, sizeof(u64) * C);
  free(mu);
  free(tmp);
}

/* Full Algorithm 1 over rows x classes pairs: result r = i*classes + j is written
 * to output ciphertext r / n (compression = modular sum of the masked ciphertexts).
 * Each thread keeps one masked ciphertext at a time and adds it into its output
 * under a lock, so memory stays bounded at any number of pairs; a sum mod q does
 * not depend on the order of its terms. */
void ora_fast_matmul(const ora_ctx* c, const u64* gk, const u64* gk_ev, const u64* xct, const u64* wpt,
                     const u64* bias_t, int rows, int classes, int K, u64* out) {
  const int n = c->n, L = c->L;
  const size_t C = (size_t)2 * L * n;
  const long npairs = (long)rows * classes;
  const long nout = (npairs + n - 1) / n;
  memset(out, 0, sizeof(u64) * C * nout);
#pragma omp parallel
  {
    u64* masked = (u64*)malloc(sizeof(u64) * C);
#pragma omp for schedule(dynamic)
    for (long r = 0; r < npairs; ++r) {
      const int i = (int)(r / classes), j = (int)(r % classes);
      ora_pair(c, gk, gk_ev, xct + (size_t)i * K * C, wpt + (size_t)j * K * n, K, bias_t[j], (int)(r % n), 0,
               masked);
#pragma omp critical(ora_compress)
      ora_add(c, out + (r / n) * C, masked, out + (r / n) * C);
    }
    free(masked);
  }
}

/* Standard encrypted matmul (baseline): fct = f feature ciphertexts (individuals in
 * slots); Y_j = sum_k fct_k * w_kj + Delta(b_j), w_kj the centred scalar lift. */
void ora_standard_matmul(const ora_ctx* c, const u64* fct, const u64* W_t /* f x classes, mod t */,
                         const u64* bias_t, int f, int classes, u64* out) {
  const int n = c->n, L = c->L;
  const size_t C = (size_t)2 * L * n;
#pragma omp parallel for
  for (int j = 0; j < classes; ++j) {
    u64* y = out + (size_t)j * C;
    memset(y, 0, sizeof(u64) * C);
    for (int k = 0; k < f; ++k) {
      const u64* x = fct + (size_t)k * C;
      for (int p = 0; p < 2; ++p)
        for (int l = 0; l < L; ++l) {
          const u64 q = c->q[l];
          const u64 w = lift_centred(W_t[(size_t)k * classes + j] % c->t, c->t, q);
          const size_t o = ((size_t)p * L + l) * n;
          for (int e = 0; e < n; ++e) y[o + e] = addmod(y[o + e], mulmod(x[o + e], w, q), q);
        }
    }
    ora_add_const(c, bias_t[j], y);
  }
}
