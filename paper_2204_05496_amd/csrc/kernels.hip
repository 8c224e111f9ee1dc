// kernels.hip -- host-side launchers of the gfx950 kernels (transforms,
// encoding, encryption, model encoding, Algorithm 1 tiles, standard baseline).
// The key-switch steps and the mask are launched through launch_ks_step /
// launch_mask_step, instantiated per ring dimension in ks_step.hip.
#include <mutex>

#include "kernels_dev.h"

namespace lrhe {

// ------------------------------------------------------------------ launchers
#define LRHE_DISPATCH(LOGNVAR, ...)                          \
  switch (LOGNVAR) {                                         \
    case 10: { constexpr int LN = 10; __VA_ARGS__; } break; \
    case 11: { constexpr int LN = 11; __VA_ARGS__; } break; \
    case 12: { constexpr int LN = 12; __VA_ARGS__; } break; \
    case 13: { constexpr int LN = 13; __VA_ARGS__; } break; \
    case 14: { constexpr int LN = 14; __VA_ARGS__; } break; \
    case 15: { constexpr int LN = 15; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                    \
  }

static inline unsigned blocks_for(uint64_t threads, unsigned bs) { return (unsigned)((threads + bs - 1) / bs); }

hipError_t launch_ntt(const lrhe_ctx* c, uint32_t* data, uint64_t npolys, uint32_t nmod, uint32_t mod0, bool inverse,
                      hipStream_t s) {
  if (npolys == 0) return hipSuccess;
  LRHE_DISPATCH(c->logn, {
    ProfScope ps(s, inverse ? "k_ntt_inv" : "k_ntt_fwd");
    // forward at 16 residues per thread up to n = 16384 (1024 threads), inverse at
    // 32 (64 for the forward transform was faster on some MI355X GPUs and slower on
    // others, by about 3 %; the inverse at 64 is several times slower)
    constexpr int LEF = LN <= 14 ? 4 : 5;
    if (inverse) k_ntt<LN, 5, true><<<(unsigned)npolys, Geom<LN, 5>::T, 0, s>>>(c->dc, data, nmod, mod0);
    else k_ntt<LN, LEF, false><<<(unsigned)npolys, Geom<LN, LEF>::T, 0, s>>>(c->dc, data, nmod, mod0);
  });
  return hipGetLastError();
}

size_t encrypt_ws_bytes(const lrhe_ctx* c, uint64_t nct) {
  // small (3 n int8) + m (n u32) + rnd (n u32), 256-byte aligned pieces
  const uint64_t n = c->n;
  auto al = [](uint64_t b) { return (b + 255) / 256 * 256; };
  return al(nct * 3 * n) + al(nct * n * 4) * 2;
}

hipError_t launch_encrypt(const lrhe_ctx* c, const uint32_t* pk_d, const int64_t* X, uint32_t rows, uint32_t f,
                          bool cols, uint64_t seed, uint64_t id0, uint32_t* ct_out, void* ws, hipStream_t s) {
  const uint64_t n = c->n;
  const uint32_t K = (uint32_t)((f + n - 1) / n);
  const uint64_t nct = cols ? f : (uint64_t)rows * K;
  if (nct == 0) return hipSuccess;
  auto al = [](uint64_t b) { return (b + 255) / 256 * 256; };
  int8_t* small = (int8_t*)ws;
  uint32_t* m = (uint32_t*)((char*)ws + al(nct * 3 * n));
  uint32_t* rnd = (uint32_t*)((char*)m + al(nct * n * 4));
  {
    ProfScope ps(s, "k_sample");
    k_sample<<<blocks_for(nct * (n / 16), 256), 256, 0, s>>>(seed, id0, (uint32_t)n, nct, small);
  }
  LRHE_DISPATCH(c->logn, {
    { ProfScope ps(s, "k_encode");
      k_encode<LN><<<(unsigned)nct, Gm<LN>::T, 0, s>>>(c->dc, X, cols ? SRC_COLS : SRC_ROWS, rows, f, K, 0, m, rnd); }
    { ProfScope ps(s, "k_encrypt");
      k_encrypt<LN><<<(unsigned)(nct * c->L), Gm<LN>::T, 0, s>>>(c->dc, pk_d, small, m, rnd, ct_out); }
  });
  return hipGetLastError();
}

hipError_t launch_model_encode(const lrhe_ctx* c, const int64_t* W, uint32_t f, uint32_t classes, uint32_t* wpt,
                               uint32_t* wsc, hipStream_t s) {
  const uint64_t n = c->n;
  const uint32_t K = (uint32_t)((f + n - 1) / n);
  const uint64_t npt = (uint64_t)classes * K;
  uint32_t* mt = nullptr;
  hipError_t err = dev_malloc_async((void**)&mt, npt * n * 4, s);
  if (err != hipSuccess) return err;
  LRHE_DISPATCH(c->logn, {
    k_encode<LN><<<(unsigned)npt, Gm<LN>::T, 0, s>>>(c->dc, W, SRC_WT, 0, f, K, classes, mt, nullptr);
    k_lift_ntt<LN><<<(unsigned)(npt * c->L), Gm<LN>::T, 0, s>>>(c->dc, mt, wpt);
  });
  const uint32_t cpad = std_class_pad(classes);
  k_scalars<<<blocks_for((uint64_t)f * c->L * cpad, 256), 256, 0, s>>>(c->dc, W, f, classes, cpad, wsc);
  err = hipGetLastError();
  (void)hipFreeAsync(mt, s);
  return err;
}

FastWs fast_ws_layout(const lrhe_ctx* c, uint32_t npairs, uint32_t classes) {
  (void)classes;
  FastWs w{};
  const uint64_t n = c->n, L = c->L;
  const uint64_t ctb = 2 * L * n * 4;
  // pairs per compression group: a power of two dividing n, smaller for small jobs
  uint32_t G = 32;
  while (G > 1 && (uint64_t)G * 64 > npairs) G >>= 1;
  w.G = G;
  uint32_t B = npairs < c->tune.tile ? npairs : c->tune.tile;
  B = (B + G - 1) / G * G;
  if (B == 0) B = G;
  w.B = B;
  auto al = [](uint64_t b) { return (b + 255) / 256 * 256; };
  const uint64_t ngroups = (npairs + G - 1) / G;
  const uint64_t nouts = (npairs + n - 1) / n;
  w.npart = ngroups;
  w.ndesc_pairs = npairs;
  w.ndesc_groups = ngroups;
  w.ndesc_outs = nouts;
  size_t off = 0;
  w.cA = off; off += al(B * ctb);
  w.cB = off; off += al(B * ctb);
  w.D = off; off += al(B * L * n * 4);
  w.acc_slots = acc_slots(c, B);
  w.ACC = off; off += al(w.acc_slots * (L + 1) * 2 * n * 4);
  w.part = off; off += al(ngroups * ctb);
  w.desc = off; off += al(npairs * sizeof(PairDesc)) + al(ngroups * sizeof(GroupDesc)) + al(nouts * sizeof(OutDesc));
  w.total = off;
  return w;
}

hipError_t launch_plan(const lrhe_ctx* c, const uint32_t* gk_d, const PairDesc* pairs, uint32_t npairs,
                       const GroupDesc* groups, const uint32_t* tile_g0, uint32_t B, const OutDesc* outs,
                       uint32_t nouts, int stage, uint32_t* out, uint32_t* cA, uint32_t* cB, uint32_t* D,
                       uint32_t* ACC, uint64_t acc_slots, uint32_t* part, hipStream_t s) {
  const uint64_t n = c->n, L = c->L;
  const uint64_t ctw = 2 * L * n;
  for (uint32_t t = 0, pb = 0; pb < npairs; ++t, pb += B) {
    const uint32_t Bt = min(B, npairs - pb);
    const Knobs& kn = c->tune.knobs(Bt);
    const PairDesc* tp = pairs + pb;
    const GroupDesc* tg = groups + tile_g0[t];
    const uint32_t ngt = tile_g0[t + 1] - tile_g0[t];
    uint32_t* cur = cA;
    uint32_t* nxt = cB;
    {
      ProfScope ps(s, "k_mac");
      k_mac<<<blocks_for((uint64_t)Bt * ctw / 4, 256), 256, 0, s>>>(c->dc, tp, Bt, cur);
    }
    if (stage == 1) {
      (void)hipMemcpyAsync(out + (uint64_t)pb * ctw, cur, (uint64_t)Bt * ctw * 4, hipMemcpyDeviceToDevice, s);
      continue;
    }
    const int steps = (stage >= 2 && stage < 100) ? stage - 2 : (int)c->ngal;
    // digits of step gi + 1 from step gi's division by P where the variant allows
    const bool fuse = kn.fuse_intt && kn.mac_mode != LRHE_MAC_MODE_HALF && kn.mac_mode != LRHE_MAC_MODE_SPLIT &&
                      kn.mac_mode != LRHE_MAC_MODE_SPLIT64;
    for (int gi = 0; gi < steps; ++gi) {
      hipError_t e = hipErrorInvalidValue;
      const bool d_ready = fuse && gi > 0, d_next = fuse && gi + 1 < steps;
      LRHE_DISPATCH(c->logn, e = launch_ks_step<LN>(c, kn, tp, gk_d, Bt, (uint32_t)gi, cur, D, ACC, acc_slots, nxt,
                                                    d_ready, d_next, s));
      if (e != hipSuccess) return e;
      uint32_t* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    if (stage >= 2 && stage < 100) {
      (void)hipMemcpyAsync(out + (uint64_t)pb * ctw, cur, (uint64_t)Bt * ctw * 4, hipMemcpyDeviceToDevice, s);
      continue;
    }
    ProfScope ps(s, "k_mask");
    const int mode = stage == 0 ? 1 : (stage == 100 ? 2 : 0);
    uint32_t* dst = mode == 0 ? part : out + (uint64_t)pb * ctw;
    hipError_t e = hipErrorInvalidValue;
    LRHE_DISPATCH(c->logn, e = launch_mask_step<LN>(c, kn, cur, tp, tg, ngt, mode, dst, s));
    if (e != hipSuccess) return e;
  }
  if (stage < 0 && nouts) {
    ProfScope ps(s, "k_compress");
    k_compress<<<blocks_for((uint64_t)nouts * ctw / 4, 256), 256, 0, s>>>(c->dc, part, outs, nouts);
  }
  return hipGetLastError();
}

hipError_t launch_fast(const lrhe_ctx* c, const uint32_t* gk_d, const lrhe_model* m, const uint32_t* xct,
                       uint32_t rows, uint32_t pair0, uint32_t npairs, int stage, uint32_t* out, void* ws,
                       const FastWs& lay, hipStream_t s) {
  (void)rows;
  char* base = (char*)ws;
  auto al = [](uint64_t b) { return (b + 255) / 256 * 256; };
  PairDesc* pairs = (PairDesc*)(base + lay.desc);
  GroupDesc* groups = (GroupDesc*)((char*)pairs + al(lay.ndesc_pairs * sizeof(PairDesc)));
  OutDesc* outs = (OutDesc*)((char*)groups + al(lay.ndesc_groups * sizeof(GroupDesc)));
  const uint32_t ngroups = (uint32_t)lay.ndesc_groups;
  const uint32_t nouts = stage < 0 ? (uint32_t)lay.ndesc_outs : 0;
  const uint32_t most = max(npairs, max(ngroups, nouts));
  k_plan_single<<<blocks_for(most, 256), 256, 0, s>>>(c->dc, xct, m->wpt, m->dbias, m->K, m->classes, pair0, npairs,
                                                      lay.B, lay.G, out, pairs, groups, ngroups, outs, nouts);
  // first group of every tile; jobs of up to 64 tiles keep the list on the stack
  const uint32_t ntiles = (npairs + lay.B - 1) / lay.B;
  uint32_t few[65];
  std::vector<uint32_t> many;
  uint32_t* tile_g0 = few;
  if (ntiles + 1 > 65) {
    many.resize(ntiles + 1);
    tile_g0 = many.data();
  }
  for (uint32_t t = 0; t < ntiles; ++t) tile_g0[t] = t * lay.B / lay.G;
  tile_g0[ntiles] = ngroups;
  return launch_plan(c, gk_d, pairs, npairs, groups, tile_g0, lay.B, outs, nouts, stage, out,
                     (uint32_t*)(base + lay.cA), (uint32_t*)(base + lay.cB), (uint32_t*)(base + lay.D),
                     (uint32_t*)(base + lay.ACC), lay.acc_slots, (uint32_t*)(base + lay.part), s);
}

// ------------------------------------------------------------------ fixed scratch
// Workspace of lrhe_matmul_fast_noalloc: a file-scope device array that every
// GPU the library runs on holds from the loading of the code object until the
// process ends.  In host code its name is only a stand-in; the device address
// is looked up once per device (at context creation, with the device current)
// and every host-side use goes through that address.
static __device__ __align__(256) unsigned char scratch[LRHE_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch[LRHE_MAX_DEVICES];

hipError_t scratch_resolve(int device) {
  if (device < 0 || device >= LRHE_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch[device] = ptr;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= LRHE_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

hipError_t launch_standard(const lrhe_ctx* c, const lrhe_model* m, const uint32_t* fct, uint32_t* y_out,
                           hipStream_t s) {
  const uint64_t ctw = (uint64_t)2 * c->L * c->n;
  ProfScope ps(s, "k_std");
  k_std<<<(unsigned)(ctw / 64), 64 * STD_WAVES, 0, s>>>(c->dc, fct, m->wsc, m->dbias, m->f, m->classes, y_out);
  return hipGetLastError();
}

}  // namespace lrhe
