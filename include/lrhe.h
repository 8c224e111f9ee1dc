/*
 * lrhe.h -- C ABI of the MI355X (gfx950) library for privacy-preserving
 * logistic-regression inference under BFV, after "Scalable privacy-preserving
 * cancer type prediction with homomorphic encryption" (arXiv 2204.05496).
 *
 * Parties and calls follow the paper's private inference protocol (section
 * "Private inference protocol"): the client generates keys, encodes and
 * encrypts its |X| x f feature matrix (n features per polynomial), the server
 * encodes W^T (|Y| x ceil(f/n) plaintexts) and the all-slot biases, computes
 * Y^ = X^ x W- + B- with the fast matrix multiplication of Algorithm 1
 * (section "Matrix multiplication algorithm"), and the client decrypts and
 * decodes the class scores, whose argmax is the predicted class (section
 * "Approximation of non-linear function in private inference").  The standard
 * encrypted matrix multiplication the paper compares against (section
 * "Comparison to standard LR") is provided as the baseline.
 *
 * Conventions (the paper runs on SEAL and leaves them implicit):
 *   - ring R = Z[X]/(X^n + 1); data primes q_0..q_{L-1} and one special prime
 *     P, each < 2^30 and = 1 mod 2n; plaintext modulus t prime, = 1 mod 2n.
 *   - slot j of a plaintext is its evaluation at psi_t^(e_j), e_j = 3^j for
 *     j < n/2 and -3^(j-n/2) otherwise (mod 2n); psi_t = g^((t-1)/2n) with g
 *     the smallest generator of Z_t^*.  Plaintext polynomials are lifted to
 *     the ciphertext moduli by their centred representative.
 *   - encryption ct = ([pk0 u + e0 + round(Q m / t)]_Q, [pk1 u + e1]_Q), u
 *     ternary, e0, e1 centred binomial (eta = 21), all drawn from ChaCha20
 *     (RFC 8439) streams: key = (seed low, seed high, 0, ..., 0), nonce =
 *     (kind, id low, id high), block counter = word index / 16.
 *   - the rotate-and-accumulate loop of Algorithm 1 uses the Galois elements
 *     3^(n/4), 3^(n/8), ..., 3, then 2n-1 (row swap): log2 n rotations.
 *   - key switching: RNS digits [d]_{q_i}, one special prime P, rounded
 *     division by P.
 *   - bias: the all-slot plaintext b_j is added after the rotate-and-sum and
 *     before the one-hot mask; result r = i |Y| + j of Algorithm 1 lands in
 *     output ciphertext r / n, slot r mod n.
 *
 * Memory: keys and models are allocated by the library on the context's
 * device and freed by their destroy call.  Ciphertext matrices, feature and
 * weight inputs and workspaces are caller-owned device buffers (for example
 * torch tensors); their sizes come from lrhe_ctx_info / lrhe_workspace_bytes.
 * Ciphertexts on the device are uint32 [2][L][n] per ciphertext, evaluation
 * (NTT) form, residues in [0, q_i).  The secret key never leaves the host.
 * Streams are hipStream_t passed as void* (NULL = the default stream); every
 * call is asynchronous on its stream unless it returns host data.
 *
 * Errors: every int-returning call returns LRHE_OK (0) or a negative code;
 * lrhe_last_error() returns a thread-local message for the last failure.
 */
#ifndef LRHE_H
#define LRHE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LRHE_OK = 0,
  LRHE_EINVAL = -1,   /* bad argument, shape or handle */
  LRHE_EPARAM = -2,   /* parameters rejected (primality, congruence, size, security bound) */
  LRHE_ENOMEM = -3,   /* device allocation failed or workspace too small */
  LRHE_EAGAIN = -4,   /* server admission refused: over the memory budget */
  LRHE_EDEVICE = -5,  /* HIP runtime error */
  LRHE_ENOISE = -6    /* decryption differs from the expected plaintext (lrhe_decrypt_check only) */
};

/* flags of the decryption calls */
enum { LRHE_CT_HOST = 1 /* the ciphertexts are in host memory (else device memory, copied on `stream`) */ };

typedef struct lrhe_ctx lrhe_ctx;
typedef struct lrhe_sk lrhe_sk;       /* secret key: host memory only */
typedef struct lrhe_pk lrhe_pk;       /* public key: device */
typedef struct lrhe_gk lrhe_gk;       /* Galois (rotation) keys: device */
typedef struct lrhe_model lrhe_model; /* encoded W^T and biases: device */
typedef struct lrhe_server lrhe_server;

typedef struct {
  uint32_t n;               /* ring degree, power of two in [1024, 32768] */
  uint32_t L;               /* number of data primes, 1..15 */
  const uint32_t* q;        /* L data primes (host array, copied) */
  uint32_t P;               /* special key-switching prime */
  uint32_t t;               /* plaintext modulus, prime, = 1 mod 2n, < 2^31 and < 2 q_i for every q_i and P */
  uint32_t allow_insecure;  /* nonzero: accept log2(Q P) above the 128-bit bound */
} lrhe_params;

/* Thread-local message describing the last error. */
const char* lrhe_last_error(void);

/* Create a context on HIP device `device` (the public values {n, T} of the
 * protocol, section "Private inference protocol"; the ring and moduli follow
 * the BFV scheme the paper runs, section "Privacy-preserving model
 * evaluation"): validates the parameters (EPARAM), derives roots, twiddle and
 * RNS tables and uploads them.  t must also stay below 2^31 and below twice
 * every ciphertext prime (plaintext values are lifted into each q_i by their
 * centred representative).
 * device < 0 creates a host-only (client) context: key generation, key
 * export, host decryption and host transforms work; device calls return
 * LRHE_EDEVICE. */
int lrhe_ctx_create(const lrhe_params* params, int device, lrhe_ctx** out);
void lrhe_ctx_destroy(lrhe_ctx* ctx);
/* n, L, number of rotation steps (log2 n) and uint32 words per ciphertext (2 L n). */
int lrhe_ctx_info(const lrhe_ctx* ctx, uint32_t* n, uint32_t* L, uint32_t* ngal, uint64_t* ct_words);
/* Galois element of rotation step i (0 <= i < ngal), in the order of the rotate-and-sum. */
int lrhe_galois_element(const lrhe_ctx* ctx, uint32_t i, uint32_t* g);

/* Key generation (client, protocol step "encrypted with the client's public
 * key").  s ternary; pk = (-(a s + e), a); with_galois: the log2 n rotation
 * keys ksk_{g,i} = (-(a s + e) + P [i = j] sigma_g(s), a) over q_0..q_{L-1}, P.
 * Any of the output pointers may be NULL. */
int lrhe_keygen(lrhe_ctx* ctx, uint64_t seed, int with_galois, lrhe_sk** sk, lrhe_pk** pk, lrhe_gk** gk);
void lrhe_sk_destroy(lrhe_sk* sk);
void lrhe_pk_destroy(lrhe_pk* pk);
void lrhe_gk_destroy(lrhe_gk* gk);

/* Workspace sizes (bytes) of the device calls below (caller-allocated device
 * memory; a call given less returns LRHE_ENOMEM). */
enum { LRHE_WS_ENCRYPT_ROWS = 1, LRHE_WS_ENCRYPT_COLS = 2, LRHE_WS_MATMUL_FAST = 3, LRHE_WS_MATMUL_STANDARD = 4 };
int lrhe_workspace_bytes(const lrhe_ctx* ctx, int op, uint32_t rows, uint32_t f, uint32_t classes, uint64_t* bytes);

/* Client: encode and encrypt the scaled feature matrix (section "Private
 * inference protocol": n features per polynomial, |X| x ceil(f/n) plaintexts,
 * each encrypted with the client's public key).  X: device int64, rows x f,
 * row-major, values taken mod t.  Fast layout: row i, chunk k holds
 * X[i][k n .. k n + n) in its slots (zero past f) and is ciphertext i K + k of
 * ct_out (device, rows K ciphertexts, caller-owned), K = ceil(f/n).
 * Randomness: stream seed `seed`, ciphertext id id0 + i K + k.
 * Errors: EINVAL (null, rows or f = 0), ENOMEM (workspace too small),
 * EDEVICE (host-only context or HIP error). */
int lrhe_encrypt_rows(lrhe_ctx* ctx, const lrhe_pk* pk, const int64_t* X, uint32_t rows, uint32_t f,
                      uint64_t seed, uint64_t id0, uint32_t* ct_out, void* ws, size_t ws_bytes, void* stream);
/* Standard layout: ciphertext k (k < f) holds column X[.][k] in slots 0..rows-1
 * (rows <= n); randomness id id0 + k. */
int lrhe_encrypt_cols(lrhe_ctx* ctx, const lrhe_pk* pk, const int64_t* X, uint32_t rows, uint32_t f,
                      uint64_t seed, uint64_t id0, uint32_t* ct_out, void* ws, size_t ws_bytes, void* stream);

/* Server: encode the model (section "Private inference protocol": the server
 * transposes W, packs it into |Y| x ceil(f/n) plaintexts, and turns each bias
 * into an all-slot plaintext).  W: device int64, f x classes, row-major (the
 * paper's f x |Y| weight matrix), values taken mod t; bias: host
 * int64[classes] or NULL (zero).  Also keeps the scalar weights the standard
 * baseline needs.  The model lives in library-owned device memory until
 * lrhe_model_destroy.  Errors: EINVAL, EDEVICE (allocation or HIP error). */
int lrhe_model_create(lrhe_ctx* ctx, const int64_t* W, const int64_t* bias, uint32_t f, uint32_t classes,
                      void* stream, lrhe_model** out);
void lrhe_model_destroy(lrhe_model* m);

/* Server: Algorithm 1 (section "Matrix multiplication algorithm"),
 * Y^ = X^ x W- + B-.  xct: rows x K ciphertexts from
 * lrhe_encrypt_rows with the model's f.  y_out: ceil(rows classes / n)
 * ciphertexts; result (i, j) in ciphertext (i classes + j) / n, slot
 * (i classes + j) mod n.  ws: lrhe_workspace_bytes(LRHE_WS_MATMUL_FAST). */
int lrhe_matmul_fast(lrhe_ctx* ctx, const lrhe_gk* gk, const lrhe_model* model, const uint32_t* xct,
                     uint32_t rows, uint32_t* y_out, void* ws, size_t ws_bytes, void* stream);

/* lrhe_matmul_fast for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same output bits, with the workspace taken from a
 * fixed device array of 96 MiB (LRHE_SCRATCH_BYTES in the library) that every
 * GPU the library runs on holds from the loading of the library until the
 * process ends; its address is looked up once per device by
 * lrhe_ctx_create.  The call allocates nothing (no hipMalloc, no library
 * allocation).  The caller still passes the inputs and y_out.  Jobs whose
 * workspace (lrhe_workspace_bytes(LRHE_WS_MATMUL_FAST)) exceeds the scratch
 * are refused with EINVAL: one individual x 16 classes at n = 16384 with 7
 * data primes needs 81 MiB.  All calls on one GPU share that GPU's array and
 * nothing is cleared between them (the path writes every scratch word before
 * reading it), so calls that overlap on one GPU (other streams, other
 * threads, other contexts) race: order them.  Errors: EINVAL, EDEVICE. */
int lrhe_matmul_fast_noalloc(lrhe_ctx* ctx, const lrhe_gk* gk, const lrhe_model* model, const uint32_t* xct,
                             uint32_t rows, uint32_t* y_out, void* stream);

/* Debug/parity variant of lrhe_matmul_fast: runs pairs [pair0, pair0 + npairs)
 * (pair r = i classes + j) through the same kernels and writes each pair's
 * ciphertext after `stage` to pairs_out (npairs ciphertexts):
 * 0 = after the mask (before compression), 1 = after the chunk products and
 * add_many, 2 + s = after s rotate-and-accumulate steps, 100 = after the bias. */
int lrhe_matmul_fast_pairs(lrhe_ctx* ctx, const lrhe_gk* gk, const lrhe_model* model, const uint32_t* xct,
                           uint32_t rows, uint32_t pair0, uint32_t npairs, int stage, uint32_t* pairs_out,
                           void* ws, size_t ws_bytes, void* stream);

/* ---- Many requests (batched and served execution of Algorithm 1) ----
 * A request is one client's encrypted rows (rows x K ciphertexts from
 * lrhe_encrypt_rows, K of its model) against one model; its outputs follow the
 * layout of lrhe_matmul_fast.  Pairs of different requests share tiles; since
 * every pair is computed independently and the compression is a modular sum,
 * each request's output ciphertexts are bit-identical to lrhe_matmul_fast on
 * that request alone. */
typedef struct {
  const uint32_t* xct;        /* device, rows x K ciphertexts */
  uint32_t rows;
  const lrhe_model* model;
  uint32_t* y;                /* device, ceil(rows classes / n) ciphertexts */
  const lrhe_gk* gk;          /* the client's Galois keys; NULL = the keys given to run/capture */
} lrhe_request;

typedef struct lrhe_batch lrhe_batch;
/* Plan a fixed set of requests (descriptors uploaded to the device once). */
int lrhe_batch_create(lrhe_ctx* ctx, const lrhe_request* reqs, uint32_t nreq, lrhe_batch** out);
/* Workspace bytes, total pairs, pairs per tile and partial-sum groups of a plan. */
int lrhe_batch_info(const lrhe_batch* b, uint64_t* ws_bytes, uint32_t* npairs, uint32_t* tile, uint32_t* ngroups);
/* Run the plan on `stream`; replays the captured graph when one exists for the same ws and keys. */
int lrhe_batch_run(lrhe_ctx* ctx, const lrhe_gk* gk, lrhe_batch* b, void* ws, size_t ws_bytes, void* stream);
/* Capture the plan's launch sequence on `stream` (non-default) into a hipGraph for replay. */
int lrhe_batch_capture(lrhe_ctx* ctx, const lrhe_gk* gk, lrhe_batch* b, void* ws, size_t ws_bytes, void* stream);
void lrhe_batch_destroy(lrhe_batch* b);

/* Continuous-batching server (section "Privacy-preserving model evaluation":
 * many individuals' predictions at once; Algorithm 1's pairs are independent,
 * section "Matrix multiplication algorithm"): the Galois keys stay resident; a worker thread
 * packs the next `tile` pending pairs of the admitted requests (arrival order)
 * into each tile, so requests that arrive while others run join the next tile.
 * hbm_budget bounds the server's partial-sum arena; a request is admitted only
 * if its partial sums fit (else LRHE_EAGAIN: resubmit later).  Inputs and
 * outputs are caller-owned device buffers that must stay valid until done. */
int lrhe_server_create(lrhe_ctx* ctx, const lrhe_gk* gk, size_t hbm_budget, lrhe_server** out);
/* `stream`: the stream on which the caller wrote xct (NULL = the default
 * stream); the server's first tile with this request waits for the work queued
 * there at the time of the call, so the caller need not synchronise first. */
int lrhe_server_submit(lrhe_server* s, const lrhe_model* model, const uint32_t* xct, uint32_t rows, uint32_t* y,
                       void* stream, uint64_t* req_id);
/* The same for a request under another client's keys (gk of the same context,
 * resident until the request is done); requests of different clients share tiles. */
int lrhe_server_submit_keys(lrhe_server* s, const lrhe_gk* gk, const lrhe_model* model, const uint32_t* xct,
                            uint32_t rows, uint32_t* y, void* stream, uint64_t* req_id);
/* done = 1 once the request's outputs are written (and visible to any stream);
 * latency_s = submit -> completion. */
int lrhe_server_poll(lrhe_server* s, uint64_t req_id, int* done, double* latency_s);
/* Forget a finished request (EINVAL while it is not done): the server keeps a
 * record of every request until it is released or the server is destroyed. */
int lrhe_server_release(lrhe_server* s, uint64_t req_id);
/* Block until every admitted request is done. */
int lrhe_server_drain(lrhe_server* s);
/* ticks run, pairs computed, free partial-sum slots, pairs per tile, request records held. */
int lrhe_server_stats(lrhe_server* s, uint64_t* ticks, uint64_t* pairs, uint32_t* free_slots, uint32_t* tile,
                      uint32_t* held);
void lrhe_server_destroy(lrhe_server* s);

/* Server: the standard encrypted matrix multiplication the paper compares
 * against (section "Comparison to standard LR"; the paper does not spell it
 * out: individuals in the slots, one ciphertext per feature, scalar weights,
 * no rotations).  fct: f device ciphertexts from lrhe_encrypt_cols; y_out:
 * device, classes ciphertexts, y_out[j] = sum_k fct[k] w_kj + B_j; score
 * (i, j) is slot i of y_out[j].  ws is unused (may be NULL).
 * Errors: EINVAL (null), EDEVICE. */
int lrhe_matmul_standard(lrhe_ctx* ctx, const lrhe_model* model, const uint32_t* fct, uint32_t* y_out,
                         void* ws, size_t ws_bytes, void* stream);

/* Client decryption (section "Private inference protocol": the client decrypts
 * and decodes the result ciphertexts): copies `count` ciphertexts from the
 * device, decrypts them on the host with the secret key and decodes the slots,
 * centred into (-t/2, t/2] (slots: host int64[count][n]).  budgets
 * (optional, host double[count]): remaining noise budget
 * log2(Q/2) - log2 max|[t x]_Q| in bits.  The secret key never leaves the host. */
int lrhe_decrypt_slots(lrhe_ctx* ctx, const lrhe_sk* sk, const uint32_t* ct, uint32_t count, int64_t* slots,
                       double* budgets, void* stream);

/* Same as lrhe_decrypt_slots for ciphertexts already in host memory (same layout;
 * for example ciphertexts read back from the wire format). */
int lrhe_decrypt_slots_host(lrhe_ctx* ctx, const lrhe_sk* sk, const uint32_t* ct, uint32_t count, int64_t* slots,
                            double* budgets);
/* Client: decrypt the class scores of Algorithm 1 (section "Private inference
 * protocol"; result r = i classes + j sits in output ciphertext r / n, slot
 * r mod n, as Algorithm 1 fills its outputs).  y: the ceil(rows classes / n)
 * output ciphertexts of lrhe_matmul_fast (device memory, or host memory with
 * LRHE_CT_HOST in flags).  scores: host int64[rows][classes], centred into
 * (-t/2, t/2]; the predicted class of row i is the argmax of its row (section
 * "Approximation of non-linear function in private inference").
 * min_budget_bits (optional): the smallest remaining noise budget over the
 * ciphertexts, in bits.  Errors: EINVAL (null, empty, unknown flags), EDEVICE. */
int lrhe_decrypt_scores(lrhe_ctx* ctx, const lrhe_sk* sk, const uint32_t* y, uint32_t rows, uint32_t classes,
                        uint32_t flags, int64_t* scores, double* min_budget_bits, void* stream);
/* The same for the standard baseline's outputs (section "Comparison to
 * standard LR"): y holds `classes` ciphertexts, score (i, j) is slot i of
 * ciphertext j (rows <= n). */
int lrhe_decrypt_scores_standard(lrhe_ctx* ctx, const lrhe_sk* sk, const uint32_t* y, uint32_t rows,
                                 uint32_t classes, uint32_t flags, int64_t* scores, double* min_budget_bits,
                                 void* stream);
/* Client, the paper's precision point (section "Private inference protocol"):
 * real inputs, weights and biases become integers by scaling with 2^s_x,
 * 2^s_w and 2^(s_x + s_w) (s_x = 6, s_w = 14 there) and taking the nearest
 * integer.  out[i] = nearest integer to in[i] 2^bits, ties to even (host
 * double[count] -> host int64[count]).  EINVAL: null arguments, bits outside
 * [0, 62], or a value that is not finite or whose scaled magnitude reaches
 * 2^62. */
int lrhe_fixed_point(const double* in, uint64_t count, int bits, int64_t* out);
/* Client: recombination over the paper's CRT pair of plaintext moduli
 * T = {t0, t1} (section "Private inference protocol": each plaintext is split
 * into one polynomial mod t0 and one mod t1, each encrypted and computed on
 * separately).  r0, r1: host int64[count] residues of the same scores mod t0
 * and mod t1 (any representatives, e.g. the centred ones of
 * lrhe_decrypt_scores); out: host int64[count], the unique integer in
 * (-t0 t1 / 2, t0 t1 / 2] congruent to both.  Dividing it by 2^(s_x + s_w)
 * gives the real-valued score.  EINVAL: null arguments, t0 or t1 below 2,
 * t0 and t1 not coprime, or t0 t1 >= 2^63. */
int lrhe_crt_combine(const int64_t* r0, const int64_t* r1, uint64_t count, uint64_t t0, uint64_t t1, int64_t* out);

/* Debug decryption given the expected plaintext: decrypts `count` ciphertexts
 * (flags as above) and compares every slot with expected (host
 * int64[count][n], compared mod t).  Returns LRHE_ENOISE when any slot
 * differs, which in BFV means the noise grew past the budget; mismatches
 * (optional) receives the number of differing slots, budgets (optional, host
 * double[count]) the remaining budgets. */
int lrhe_decrypt_check(lrhe_ctx* ctx, const lrhe_sk* sk, const uint32_t* ct, uint32_t count, const int64_t* expected,
                       uint32_t flags, double* budgets, uint64_t* mismatches, void* stream);

/* Host (client-side) transform of one polynomial in place, modulus index
 * mod_index (0..L-1 data primes, L = P, L+1 = t): forward maps canonical
 * coefficients to evaluations at psi^(2 brv(k)+1) stored at index k (the
 * device's evaluation layout); inverse maps back.  Runs the same pass
 * arithmetic as the kernels. */
int lrhe_host_transform(lrhe_ctx* ctx, uint32_t mod_index, uint32_t* a, int inverse);

/* Canonical coefficient form of `polys` device polynomials of L limbs each
 * (ciphertexts are 2 such polys): inverse transform per limb, output in
 * [0, q_i) to out (device, same shape).  Used for parity checks. */
int lrhe_to_coeff(lrhe_ctx* ctx, const uint32_t* in, uint64_t polys, uint32_t* out, void* stream);
/* Batched negacyclic transform in place on `polys` device polynomials of L
 * limbs each (limb i modulo q_i): forward maps canonical coefficients to the
 * evaluation form the kernels use, inverse maps back (canonical output). */
int lrhe_ntt(lrhe_ctx* ctx, uint32_t* data, uint64_t polys, int inverse, void* stream);

/* Launch tuning of the fast matmul.  Keys: "le_intt", "le_mac", "le_moddown",
 * "le_mask" = log2 of the residues each thread holds in that transform kernel
 * (4, 5 or 6 where the workgroup stays within 1024 threads; defaults below),
 * "mac_mode" = variant of the key-switch inner-product kernel: 0:
 * one LDS exchange buffer and two workgroups per CU, the workgroups of a pair
 * on one XCD; 1: as 0 with the twiddles of the next butterfly stage loaded
 * ahead; 2: double-buffered exchange, pair per XCD, unreduced 64-bit inner
 * products; 3: double-buffered exchange with the next digit loaded ahead;
 * 4: double-buffered exchange and unreduced 64-bit inner products, with the
 * digits of each (pair, modulus) item split over two workgroups (in launch
 * order), the special-prime inverse transforms in a kernel of their own
 * and the division by P split by ciphertext part (more workgroups for tiles
 * too small to fill the GPU; small class only, EINVAL for the large class or
 * a bare key); 5: one exchange buffer, two workgroups per CU and the next
 * stage's twiddles loaded ahead, with the target moduli spread by XCD: in each
 * window of 256 pairs an XCD takes two of the eight moduli for half of the
 * pairs, so its L2 holds a quarter of the step's Galois key (needs L = 7 and
 * an even tile; otherwise the plain launch order); 6: two launches per
 * rotation step, the special-prime items first (at "le_mac_p" residues per
 * thread; they also make the step's digits, so no digit kernel runs), then the
 * data-modulus items, each of which also does the rounded
 * division by P and the rotate-and-accumulate of its limb from the sums in its
 * registers, so no k_ks_moddown runs and no sum of a data modulus goes through
 * memory; 7: as 6 with the data-modulus launch double-buffered and its inner
 * products summed unreduced in 64 bits (one workgroup per CU); "le_mac_p" =
 * residues per thread of the special-prime launch of variants 6 and 7;
 * "fuse_intt" = 1 lets the rounded division by P of each
 * rotation step also compute the next step's digits (inverse transform of the
 * automorphism of c1), so the digit kernel runs on the first step only; 0
 * (default) runs it on every step; ignored by variants 4, 6 and 7.  These seven keys exist
 * in two classes, for tiles of fewer than
 * "small_below" pairs (default 64; such launches are latency-bound) and for
 * larger tiles: "small.<key>" and "large.<key>" address one class, a bare key
 * sets both and reads the large class.  Defaults: large tiles le_intt 5,
 * le_mac 6, le_moddown 6, le_mask 4 (each 5 where the ring dimension does not
 * allow it), mac_mode 6 and le_mac_p 5; small tiles le_intt 5, le_mac, le_moddown and
 * le_mask 4 (5 where not available) and mac_mode 4.
 * "tile" = pairs per tile (default 4096), "small_below" as above; the
 * workspace size depends on both (small tiles hold two accumulators per pair).
 * No choice changes any result bit.  EINVAL for unknown keys or unavailable
 * values. */
int lrhe_tune_set(lrhe_ctx* ctx, const char* key, int value);
int lrhe_tune_get(const lrhe_ctx* ctx, const char* key, int* value);
/* Autotuner: runs lrhe_matmul_fast on the given workload (reps timed runs per
 * candidate, each kernel timed with HIP events on its stream) and keeps, in
 * the tuning class of this job's tiles, every transform kernel's fastest
 * residues-per-thread choice, searched jointly with "mac_mode" for k_ks_mac
 * ("le_mac_p", the split variant's special-prime launch, on its own).
 * Uses the kernel timer (lrhe_prof_*), whose totals it resets. */
int lrhe_autotune_fast(lrhe_ctx* ctx, const lrhe_gk* gk, const lrhe_model* model, const uint32_t* xct, uint32_t rows,
                       uint32_t* y_out, void* ws, size_t ws_bytes, void* stream, int reps);

/* Tuning cache: lrhe_tune_save writes the context's launch choices (both tile
 * classes, "tile", "small_below") to the text file `path` under `key`, one
 * line per key, replacing that key's line and keeping the others.  The key is
 * the caller's (for example GPU architecture, ring dimension, number of primes
 * and a digest of the kernel sources).  lrhe_tune_load applies the key's
 * choices: LRHE_OK when found, LRHE_EAGAIN (not an error) when the file or
 * the key is absent, EINVAL for a malformed entry or a choice unavailable at
 * this ring dimension (the context keeps its choices then). */
int lrhe_tune_save(const lrhe_ctx* ctx, const char* path, const char* key);
int lrhe_tune_load(lrhe_ctx* ctx, const char* path, const char* key);

/* Opt-in kernel timing: while enabled, every kernel launch of the library is
 * bracketed by HIP events on its own stream.  lrhe_prof_get returns the number
 * of launches and their summed duration (ms) for a kernel name (for example
 * "k_ks_mac", "k_ntt_fwd") since the last reset; it waits for pending events. */
void lrhe_prof_enable(int on);
void lrhe_prof_reset(void);
int lrhe_prof_get(const char* kernel, uint64_t* launches, double* total_ms);
/* Issue rate of the vector instructions the transforms are built from, on the
 * current device: op 0 v_add_u32, 1 v_mul_lo_u32, 2 v_mul_hi_u32,
 * 3 v_mad_u64_u32 (lane instructions per second, from dependent inline-asm
 * chains the compiler cannot fold), 4 the Montgomery forward butterfly of the
 * transforms (butterflies per second).  iters loop iterations of 128
 * operations per lane on 64 workgroups of 256 lanes per compute unit; the best
 * of reps timed launches after a warm-up.  best_ms may be NULL.  EINVAL for
 * other ops or non-positive counts, EDEVICE on a HIP error.  Measurement
 * only: it backs the ALU peak that kernel throughput is compared against. */
int lrhe_prof_valu_rate(int op, int iters, int reps, double* per_s, double* best_ms);

/* Allocation fault injection (failure handling tests): the k-th device
 * allocation of the library from now on fails as if out of memory, so the call
 * that makes it returns LRHE_EDEVICE (LRHE_ENOMEM for the server) and leaves no
 * partial object; k = 0 disarms.  The environment variable LRHE_FAULT_ALLOC
 * gives the initial k.  Returns the previous k; k < 0 only reads it. */
int64_t lrhe_fault_inject(int64_t k);

/* Wire format of the private inference protocol (section "Private inference
 * protocol": the client sends the encrypted inputs, and once its evaluation
 * keys, to the server, which returns the encrypted results; keys are kept
 * across restarts).  A message is a 64-byte header (magic "LRHEWIR1",
 * version 1, kind, n, L, t, a digest of the moduli, count, payload size and
 * an FNV-1a 64 checksum of the payload) and a payload of canonical
 * coefficient-form residues, little-endian u32: kind LRHE_WIRE_CT
 * ciphertexts [count][2][L][n]; LRHE_WIRE_GK Galois keys
 * [ngal][L digits][2][L+1 moduli][n]; LRHE_WIRE_PK public key [2][L][n];
 * LRHE_WIRE_SK secret key int8 [n].  The caller owns every buffer. */
enum { LRHE_WIRE_CT = 1, LRHE_WIRE_GK = 2, LRHE_WIRE_PK = 3, LRHE_WIRE_SK = 4 };
/* Message size in bytes for `count` ciphertexts (kind LRHE_WIRE_CT) or one key. */
int lrhe_wire_bytes(lrhe_ctx* ctx, int kind, uint64_t count, uint64_t* bytes);
/* ct: `count` ciphertexts in the library's layout (device memory, or host
 * memory with LRHE_CT_HOST; the copy runs on `stream`, which is synchronized);
 * out: host buffer of cap >= lrhe_wire_bytes bytes.  EINVAL: null, short
 * buffer, unknown flags; EDEVICE: copy error or device memory on a host-only
 * context. */
int lrhe_ct_serialize(lrhe_ctx* ctx, const uint32_t* ct, uint32_t count, uint32_t flags, uint8_t* out, uint64_t cap,
                      void* stream);
/* Reads a ciphertext message into ct_out (room for max_count ciphertexts,
 * device memory or host memory with LRHE_CT_HOST); count (optional) receives
 * the number read.  EINVAL when the message is malformed, of another kind,
 * made under other parameters, fails its checksum, holds non-canonical
 * residues or more than max_count ciphertexts; nothing is written then. */
int lrhe_ct_deserialize(lrhe_ctx* ctx, const uint8_t* in, uint64_t bytes, uint32_t flags, uint32_t* ct_out,
                        uint32_t max_count, uint32_t* count, void* stream);
/* kind LRHE_WIRE_GK (key: const lrhe_gk*), LRHE_WIRE_PK (const lrhe_pk*) or
 * LRHE_WIRE_SK (const lrhe_sk*; the secret key stays with the client). */
int lrhe_key_serialize(lrhe_ctx* ctx, int kind, const void* key, uint8_t* out, uint64_t cap);
/* New key objects from messages, checked as in lrhe_ct_deserialize (the secret
 * key's coefficients must be ternary); owned by the caller (*_destroy). */
int lrhe_gk_deserialize(lrhe_ctx* ctx, const uint8_t* in, uint64_t bytes, lrhe_gk** out);
int lrhe_pk_deserialize(lrhe_ctx* ctx, const uint8_t* in, uint64_t bytes, lrhe_pk** out);
int lrhe_sk_deserialize(lrhe_ctx* ctx, const uint8_t* in, uint64_t bytes, lrhe_sk** out);

/* Keys in canonical coefficient form on the host: pk as uint32 [2][L][n];
 * gk as uint32 [ngal][L digits][2][L+1 moduli][n] (last modulus = P). */
int lrhe_pk_export(lrhe_ctx* ctx, const lrhe_pk* pk, uint32_t* host_out);
int lrhe_gk_export(lrhe_ctx* ctx, const lrhe_gk* gk, uint32_t* host_out);
/* Secret key coefficients (ternary, host int8[n]); client-side only. */
int lrhe_sk_export(lrhe_ctx* ctx, const lrhe_sk* sk, int8_t* host_out);

#ifdef __cplusplus
}
#endif
#endif /* LRHE_H */
