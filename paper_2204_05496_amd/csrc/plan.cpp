// plan.cpp -- batched and served execution of Algorithm 1 (the paper's fast
// matrix multiplication) over many requests on one GPU.
//
// A request is one client's encrypted feature matrix (rows x K ciphertexts)
// against one encoded model.  Its pairs (row i, class j) are independent until
// the compression, and the compression is a modular sum, so pairs of different
// requests can share tiles and the grouping of partial sums does not change
// any output bit: each request's ciphertexts are the same alone and in a mix.
//
//  * lrhe_batch_*: a fixed set of requests planned once (descriptors in HBM),
//    run eagerly or captured into a hipGraph and replayed.
//  * lrhe_server_*: continuous batching.  A worker thread packs the next B
//    pending pairs of the admitted requests (in arrival order) into each tile;
//    requests arriving while tiles run join the next tile.  Admission is by a
//    memory budget for the requests' partial sums (LRHE_EAGAIN when full).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lrhe_internal.h"

using namespace lrhe;

extern "C" void lrhe_prof_enable(int on);

namespace {
#define perr lrhe::fail
size_t al256(size_t b) { return (b + 255) / 256 * 256; }

uint32_t pick_group(uint64_t npairs) {
  uint32_t G = 32;
  while (G > 1 && (uint64_t)G * 64 > npairs) G >>= 1;
  return G;
}

struct TileWs {   // per-tile buffers of the key-switch pipeline
  size_t cA, cB, D, ACC, total;
  uint64_t acc_slots;   // pair slots of ACC (see acc_slots)
};
TileWs tile_ws(const lrhe_ctx* c, uint32_t B) {
  const uint64_t n = c->n, L = c->L, ctb = 2 * L * n * 4;
  TileWs w{};
  size_t off = 0;
  w.cA = off; off += al256(B * ctb);
  w.cB = off; off += al256(B * ctb);
  w.D = off; off += al256((uint64_t)B * L * n * 4);
  w.acc_slots = acc_slots(c, B);
  w.ACC = off; off += al256(w.acc_slots * (L + 1) * 2 * n * 4);
  w.total = off;
  return w;
}
}  // namespace

// ============================================================================ batches
struct lrhe_batch {
  lrhe_ctx* c = nullptr;
  uint32_t B = 0, G = 0, npairs = 0, ngroups = 0, nouts = 0;
  std::vector<uint32_t> tile_g0;
  void* d_desc = nullptr;          // pairs | groups | outs
  PairDesc* d_pairs = nullptr;
  GroupDesc* d_groups = nullptr;
  OutDesc* d_outs = nullptr;
  TileWs tw{};
  size_t part_off = 0, ws_bytes = 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const void* graph_ws = nullptr;
  const uint32_t* graph_gk = nullptr;
};

extern "C" int lrhe_batch_create(lrhe_ctx* c, const lrhe_request* reqs, uint32_t nreq, lrhe_batch** out) {
  if (!c || !reqs || !out || nreq == 0) return perr(LRHE_EINVAL, "null or empty argument");
  if (c->device < 0) return perr(LRHE_EDEVICE, "host-only context");
  *out = nullptr;
  const uint64_t n = c->n, L = c->L, ctw = 2 * L * n;
  uint64_t total = 0;
  for (uint32_t r = 0; r < nreq; ++r) {
    if (!reqs[r].xct || !reqs[r].model || !reqs[r].y || reqs[r].rows == 0)
      return perr(LRHE_EINVAL, "request %u: null buffer or no rows", r);
    if (reqs[r].gk && !reqs[r].gk->d) return perr(LRHE_EINVAL, "request %u: Galois keys without device copy", r);
    total += (uint64_t)reqs[r].rows * reqs[r].model->classes;
  }
  if (total > 0x7fffffffull) return perr(LRHE_EINVAL, "too many pairs");
  auto* b = new lrhe_batch();
  b->c = c;
  b->G = pick_group(total);
  b->B = (uint32_t)std::min<uint64_t>(total, c->tune.tile);
  b->B = (b->B + b->G - 1) / b->G * b->G;
  b->npairs = (uint32_t)total;
  std::vector<PairDesc> pairs;
  std::vector<GroupDesc> groups;
  std::vector<OutDesc> outs;
  pairs.reserve(total);
  uint64_t gp = 0;   // global pair index
  for (uint32_t r = 0; r < nreq; ++r) {
    const lrhe_model* m = reqs[r].model;
    const uint64_t np = (uint64_t)reqs[r].rows * m->classes;
    const uint64_t nout = (np + n - 1) / n;
    for (uint64_t o = 0; o < nout; ++o) {
      OutDesc od;
      od.y = reqs[r].y + o * ctw;
      od.g0 = (uint32_t)groups.size();
      const uint64_t p_end = std::min(np, (o + 1) * n);
      for (uint64_t p = o * n; p < p_end; ++p, ++gp) {
        const uint64_t i = p / m->classes, jc = p % m->classes;
        PairDesc d;
        d.xrow = reqs[r].xct + i * m->K * ctw;
        d.gk = reqs[r].gk ? reqs[r].gk->d : nullptr;
        d.wcls = m->wpt + jc * m->K * L * n;
        d.dbias = m->dbias + jc * L;
        d.K = m->K;
        d.slot = (uint32_t)(p % n);
        pairs.push_back(d);
        // open a new group at the output's first pair, at a tile start, or when full
        const uint32_t lp = (uint32_t)(gp % b->B);
        if (p == o * n || lp == 0 || groups.back().cnt == b->G) {
          GroupDesc g;
          g.lp0 = lp;
          g.cnt = 0;
          g.part = (uint32_t)groups.size();
          g.pad = (uint32_t)(gp / b->B);   // tile of the group (host bookkeeping)
          groups.push_back(g);
        }
        groups.back().cnt++;
      }
      od.g1 = (uint32_t)groups.size();
      outs.push_back(od);
    }
  }
  b->ngroups = (uint32_t)groups.size();
  b->nouts = (uint32_t)outs.size();
  const uint32_t ntiles = (b->npairs + b->B - 1) / b->B;
  b->tile_g0.assign(ntiles + 1, b->ngroups);
  for (uint32_t gi = (uint32_t)groups.size(); gi-- > 0;) b->tile_g0[groups[gi].pad] = gi;
  for (uint32_t t = ntiles; t-- > 0;) b->tile_g0[t] = std::min(b->tile_g0[t], b->tile_g0[t + 1]);
  const size_t sp = al256(pairs.size() * sizeof(PairDesc)), sg = al256(groups.size() * sizeof(GroupDesc)),
               so = al256(outs.size() * sizeof(OutDesc));
  hipError_t err = hipSetDevice(c->device);
  if (err == hipSuccess) err = dev_malloc(&b->d_desc, sp + sg + so);
  if (err == hipSuccess) {
    b->d_pairs = (PairDesc*)b->d_desc;
    b->d_groups = (GroupDesc*)((char*)b->d_desc + sp);
    b->d_outs = (OutDesc*)((char*)b->d_desc + sp + sg);
    err = hipMemcpy(b->d_pairs, pairs.data(), pairs.size() * sizeof(PairDesc), hipMemcpyHostToDevice);
  }
  if (err == hipSuccess) err = hipMemcpy(b->d_groups, groups.data(), groups.size() * sizeof(GroupDesc), hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(b->d_outs, outs.data(), outs.size() * sizeof(OutDesc), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(b->d_desc);
    delete b;
    return perr(LRHE_EDEVICE, "batch upload: %s", hipGetErrorString(err));
  }
  b->tw = tile_ws(c, b->B);
  b->part_off = b->tw.total;
  b->ws_bytes = b->part_off + al256((size_t)b->ngroups * ctw * 4);
  *out = b;
  return LRHE_OK;
}

extern "C" int lrhe_batch_info(const lrhe_batch* b, uint64_t* ws_bytes, uint32_t* npairs, uint32_t* tile,
                               uint32_t* ngroups) {
  if (!b) return perr(LRHE_EINVAL, "null batch");
  if (ws_bytes) *ws_bytes = b->ws_bytes;
  if (npairs) *npairs = b->npairs;
  if (tile) *tile = b->B;
  if (ngroups) *ngroups = b->ngroups;
  return LRHE_OK;
}

static hipError_t batch_launch(lrhe_batch* b, const lrhe_gk* gk, void* ws, hipStream_t s) {
  char* base = (char*)ws;
  return launch_plan(b->c, gk->d, b->d_pairs, b->npairs, b->d_groups, b->tile_g0.data(), b->B, b->d_outs, b->nouts,
                     -1, nullptr, (uint32_t*)(base + b->tw.cA), (uint32_t*)(base + b->tw.cB),
                     (uint32_t*)(base + b->tw.D), (uint32_t*)(base + b->tw.ACC), b->tw.acc_slots, (uint32_t*)(base + b->part_off), s);
}

extern "C" int lrhe_batch_run(lrhe_ctx* c, const lrhe_gk* gk, lrhe_batch* b, void* ws, size_t ws_bytes, void* stream) {
  if (!c || !gk || !b || b->c != c) return perr(LRHE_EINVAL, "bad argument");
  if (!ws || ws_bytes < b->ws_bytes) return perr(LRHE_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, b->ws_bytes);
  hipError_t err = hipSetDevice(c->device);
  if (err == hipSuccess) {
    if (b->exec && b->graph_ws == ws && b->graph_gk == gk->d) err = hipGraphLaunch(b->exec, (hipStream_t)stream);
    else err = batch_launch(b, gk, ws, (hipStream_t)stream);
  }
  if (err != hipSuccess) return perr(LRHE_EDEVICE, "batch run: %s", hipGetErrorString(err));
  return LRHE_OK;
}

extern "C" int lrhe_batch_capture(lrhe_ctx* c, const lrhe_gk* gk, lrhe_batch* b, void* ws, size_t ws_bytes,
                                  void* stream) {
  if (!c || !gk || !b || b->c != c || !stream) return perr(LRHE_EINVAL, "bad argument (a non-default stream is needed)");
  if (!ws || ws_bytes < b->ws_bytes) return perr(LRHE_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, b->ws_bytes);
  hipError_t err = hipSetDevice(c->device);
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
  }
  lrhe_prof_enable(0);   // no timing events inside the captured graph
  hipStream_t s = (hipStream_t)stream;
  if (err == hipSuccess) err = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (err == hipSuccess) {
    hipError_t e1 = batch_launch(b, gk, ws, s);
    err = hipStreamEndCapture(s, &b->graph);
    if (e1 != hipSuccess) err = e1;
  }
  if (err == hipSuccess) err = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (err != hipSuccess) {
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
    b->exec = nullptr;
    return perr(LRHE_EDEVICE, "graph capture: %s", hipGetErrorString(err));
  }
  b->graph_ws = ws;
  b->graph_gk = gk->d;
  return LRHE_OK;
}

extern "C" void lrhe_batch_destroy(lrhe_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  (void)hipFree(b->d_desc);
  delete b;
}

// ============================================================================ server
namespace {
using Clock = std::chrono::steady_clock;

struct SReq {
  uint64_t id = 0;
  const uint32_t* xct = nullptr;
  const lrhe_model* m = nullptr;
  const lrhe_gk* gk = nullptr;      // the client's Galois keys (null: the server's)
  uint32_t* y = nullptr;
  uint64_t npairs = 0, next = 0, nout = 0;
  uint32_t part0 = 0, nparts = 0;   // partial slots [part0, part0 + nparts) of the arena
  uint32_t used_parts = 0;          // groups opened so far
  std::vector<uint32_t> out_g0, out_g1;
  Clock::time_point t_submit, t_done;
  hipEvent_t ev = nullptr;          // recorded after the request's last compression
  hipEvent_t ready = nullptr;       // recorded on the submitter's stream: inputs written
  int state = 0;                    // 0 queued, 1 scheduled fully, 2 done
};
}  // namespace

struct lrhe_server {
  lrhe_ctx* c = nullptr;
  const lrhe_gk* gk = nullptr;
  hipStream_t s = nullptr;
  uint32_t B = 0, G = 32;
  TileWs tw{};
  void* d_tile = nullptr;            // key-switch buffers of one tile
  uint32_t* d_part = nullptr;        // partial-sum arena
  uint32_t arena_slots = 0;
  std::vector<std::pair<uint32_t, uint32_t>> free_ranges;   // (start, length)
  // two descriptor slots (device + pinned host) so planning overlaps the GPU
  void* d_desc[2] = {nullptr, nullptr};
  void* h_desc[2] = {nullptr, nullptr};
  hipEvent_t slot_ev[2] = {nullptr, nullptr};
  size_t desc_bytes = 0;
  uint64_t out_cap = 0;              // output descriptors per tick
  std::mutex mu;
  std::condition_variable cv;
  std::deque<SReq*> queue;           // admitted, not fully scheduled (arrival order)
  std::vector<SReq*> inflight;       // fully scheduled, waiting for completion
  std::map<uint64_t, SReq*> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  std::atomic<uint64_t> ticks{0}, pairs_done{0};
  int error = 0;
  std::string error_msg;
};

namespace {
bool arena_alloc(lrhe_server* sv, uint32_t need, uint32_t* start) {
  for (auto it = sv->free_ranges.begin(); it != sv->free_ranges.end(); ++it) {
    if (it->second >= need) {
      *start = it->first;
      it->first += need;
      it->second -= need;
      if (it->second == 0) sv->free_ranges.erase(it);
      return true;
    }
  }
  return false;
}
void arena_free(lrhe_server* sv, uint32_t start, uint32_t len) {
  sv->free_ranges.push_back({start, len});
  std::sort(sv->free_ranges.begin(), sv->free_ranges.end());
  std::vector<std::pair<uint32_t, uint32_t>> merged;
  for (auto& r : sv->free_ranges) {
    if (!merged.empty() && merged.back().first + merged.back().second == r.first) merged.back().second += r.second;
    else merged.push_back(r);
  }
  sv->free_ranges.swap(merged);
}
// partial slots a request may need: one per G pairs, plus a split at every
// tile boundary it crosses and at every output-ciphertext boundary
uint32_t parts_needed(const lrhe_server* sv, uint64_t npairs, uint64_t nout) {
  return (uint32_t)((npairs + sv->G - 1) / sv->G + (npairs + sv->B - 1) / sv->B + 1 + nout);
}

void complete_ready(lrhe_server* sv) {   // called with mu held
  for (size_t k = 0; k < sv->inflight.size();) {
    SReq* r = sv->inflight[k];
    if (!r->ev && !sv->error) {   // scheduled, event not recorded yet
      ++k;
      continue;
    }
    const hipError_t q = r->ev ? hipEventQuery(r->ev) : hipErrorNotReady;
    if (q != hipSuccess && q != hipErrorNotReady && !sv->error) {
      sv->error = LRHE_EDEVICE;
      sv->error_msg = hipGetErrorString(q);
    }
    if (q == hipSuccess || sv->error) {
      r->t_done = Clock::now();
      r->state = 2;
      arena_free(sv, r->part0, r->nparts);
      if (r->ev) (void)hipEventDestroy(r->ev);
      r->ev = nullptr;
      if (r->ready) (void)hipEventDestroy(r->ready);
      r->ready = nullptr;
      sv->inflight.erase(sv->inflight.begin() + k);
      sv->cv.notify_all();
    } else {
      ++k;
    }
  }
}

// one tile: the next B pairs of the queue, in arrival order
void run_tick(lrhe_server* sv, int slot) {
  lrhe_ctx* c = sv->c;
  const uint64_t n = c->n, L = c->L, ctw = 2 * L * n;
  std::vector<PairDesc> pairs;
  std::vector<GroupDesc> groups;
  std::vector<OutDesc> outs;
  std::vector<SReq*> finishing;
  std::vector<hipEvent_t> waits;    // inputs of requests that start in this tile
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    uint32_t lp = 0;
    size_t qi = 0;
    uint64_t nouts = 0;
    while (lp < sv->B && qi < sv->queue.size()) {
      SReq* r = sv->queue[qi];
      const lrhe_model* m = r->m;
      // a request that would finish here needs room for its output descriptors
      if (r->npairs - r->next <= sv->B - lp && nouts + r->nout > sv->out_cap) break;
      bool open = false;
      if (r->next == 0 && r->ready) waits.push_back(r->ready);
      while (lp < sv->B && r->next < r->npairs) {
        const uint64_t p = r->next;
        const uint64_t i = p / m->classes, jc = p % m->classes, o = p / n;
        PairDesc d;
        d.xrow = r->xct + i * m->K * ctw;
        d.gk = r->gk ? r->gk->d : nullptr;
        d.wcls = m->wpt + jc * m->K * L * n;
        d.dbias = m->dbias + jc * L;
        d.K = m->K;
        d.slot = (uint32_t)(p % n);
        pairs.push_back(d);
        if (!open || p % n == 0 || groups.back().cnt == sv->G) {
          if (r->used_parts == r->nparts) {   // cannot happen with parts_needed's bound
            if (!sv->error) {
              sv->error = LRHE_EINVAL;
              sv->error_msg = "partial-slot bound exceeded";
            }
            return;
          }
          GroupDesc g;
          g.lp0 = lp;
          g.cnt = 0;
          g.part = r->part0 + r->used_parts++;
          g.pad = 0;
          groups.push_back(g);
          if (r->out_g0[o] == UINT32_MAX) r->out_g0[o] = g.part;
          open = true;
        }
        groups.back().cnt++;
        r->out_g1[o] = groups.back().part + 1;
        ++r->next;
        ++lp;
      }
      if (r->next == r->npairs) {
        nouts += r->nout;
        finishing.push_back(r);
        // in flight from now on (its event is recorded after the launch), so
        // drain never sees it in neither list
        sv->inflight.push_back(r);
        sv->queue.erase(sv->queue.begin() + qi);
      } else {
        ++qi;
      }
    }
    for (SReq* r : finishing)
      for (uint64_t o = 0; o < r->nout; ++o) {
        OutDesc od;
        od.y = r->y + o * ctw;
        od.g0 = r->out_g0[o];
        od.g1 = r->out_g1[o];
        outs.push_back(od);
      }
  }
  if (pairs.empty()) return;
  // stage the descriptors through the slot's pinned buffer
  (void)hipEventSynchronize(sv->slot_ev[slot]);
  const size_t sp = al256(sv->B * sizeof(PairDesc)), sg = al256(sv->B * sizeof(GroupDesc));
  char* h = (char*)sv->h_desc[slot];
  char* d = (char*)sv->d_desc[slot];
  memcpy(h, pairs.data(), pairs.size() * sizeof(PairDesc));
  memcpy(h + sp, groups.data(), groups.size() * sizeof(GroupDesc));
  memcpy(h + sp + sg, outs.data(), outs.size() * sizeof(OutDesc));
  hipError_t err = hipSuccess;
  for (hipEvent_t w : waits)
    if (err == hipSuccess) err = hipStreamWaitEvent(sv->s, w, 0);
  if (err == hipSuccess) err = hipMemcpyAsync(d, h, sv->desc_bytes, hipMemcpyHostToDevice, sv->s);
  const uint32_t tg[2] = {0, (uint32_t)groups.size()};
  char* tb = (char*)sv->d_tile;
  if (err == hipSuccess)
    err = launch_plan(c, sv->gk->d, (PairDesc*)d, (uint32_t)pairs.size(), (GroupDesc*)(d + sp), tg, sv->B,
                      (OutDesc*)(d + sp + sg), (uint32_t)outs.size(), -1, nullptr, (uint32_t*)(tb + sv->tw.cA),
                      (uint32_t*)(tb + sv->tw.cB), (uint32_t*)(tb + sv->tw.D), (uint32_t*)(tb + sv->tw.ACC),
                      sv->tw.acc_slots, sv->d_part, sv->s);
  if (err == hipSuccess) err = hipEventRecord(sv->slot_ev[slot], sv->s);
  std::lock_guard<std::mutex> lk(sv->mu);
  for (SReq* r : finishing) {
    hipEvent_t ev = nullptr;
    if (err == hipSuccess) err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventRecord(ev, sv->s);
    r->ev = ev;
    r->state = 1;
  }
  if (err != hipSuccess && !sv->error) {
    sv->error = LRHE_EDEVICE;
    sv->error_msg = hipGetErrorString(err);
  }
  sv->ticks++;
  sv->pairs_done += pairs.size();
}

void worker_main(lrhe_server* sv) {
  (void)hipSetDevice(sv->c->device);
  int slot = 0;
  while (true) {
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      complete_ready(sv);
      if (sv->stop && ((sv->queue.empty() && sv->inflight.empty()) || sv->error)) break;
      if (sv->queue.empty() || sv->error) {
        // nothing to schedule: wait for arrivals or poll completions
        sv->cv.wait_for(lk, std::chrono::microseconds(200));
        continue;
      }
    }
    run_tick(sv, slot);
    slot ^= 1;
  }
}
}  // namespace

extern "C" int lrhe_server_create(lrhe_ctx* c, const lrhe_gk* gk, size_t hbm_budget, lrhe_server** out) {
  if (!c || !gk || !out) return perr(LRHE_EINVAL, "null argument");
  if (c->device < 0) return perr(LRHE_EDEVICE, "host-only context");
  *out = nullptr;
  auto* sv = new lrhe_server();
  sv->c = c;
  sv->gk = gk;
  sv->B = c->tune.tile;
  sv->G = 32;
  sv->B = (sv->B + sv->G - 1) / sv->G * sv->G;
  sv->tw = tile_ws(c, sv->B);
  const size_t ctb = (size_t)2 * c->L * c->n * 4;
  sv->arena_slots = (uint32_t)(hbm_budget / ctb);
  if (sv->arena_slots < 4) {
    delete sv;
    return perr(LRHE_EINVAL, "budget %zu bytes holds fewer than 4 partial ciphertexts", hbm_budget);
  }
  sv->free_ranges.push_back({0, sv->arena_slots});
  sv->out_cap = (uint64_t)sv->B + 64;
  sv->desc_bytes = al256(sv->B * sizeof(PairDesc)) + al256(sv->B * sizeof(GroupDesc)) +
                   al256((size_t)sv->out_cap * sizeof(OutDesc));
  hipError_t err = hipSetDevice(c->device);
  if (err == hipSuccess) err = hipStreamCreateWithFlags(&sv->s, hipStreamNonBlocking);
  if (err == hipSuccess) err = dev_malloc(&sv->d_tile, sv->tw.total);
  if (err == hipSuccess) err = dev_malloc((void**)&sv->d_part, (size_t)sv->arena_slots * ctb);
  for (int k = 0; k < 2 && err == hipSuccess; ++k) {
    err = dev_malloc(&sv->d_desc[k], sv->desc_bytes);
    if (err == hipSuccess) err = hipHostMalloc(&sv->h_desc[k], sv->desc_bytes, hipHostMallocDefault);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&sv->slot_ev[k], hipEventDisableTiming);
  }
  if (err != hipSuccess) {
    lrhe_server_destroy(sv);
    return perr(LRHE_ENOMEM, "server allocation: %s", hipGetErrorString(err));
  }
  sv->worker = std::thread(worker_main, sv);
  *out = sv;
  return LRHE_OK;
}

extern "C" int lrhe_server_submit(lrhe_server* sv, const lrhe_model* m, const uint32_t* xct, uint32_t rows,
                                  uint32_t* y_out, void* stream, uint64_t* req_id) {
  return lrhe_server_submit_keys(sv, nullptr, m, xct, rows, y_out, stream, req_id);
}

extern "C" int lrhe_server_submit_keys(lrhe_server* sv, const lrhe_gk* gk, const lrhe_model* m, const uint32_t* xct,
                                       uint32_t rows, uint32_t* y_out, void* stream, uint64_t* req_id) {
  if (!sv || !m || !xct || !y_out || !req_id || rows == 0) return perr(LRHE_EINVAL, "bad argument");
  if (gk && (!gk->d || gk->words != sv->gk->words)) return perr(LRHE_EINVAL, "Galois keys of another context");
  const uint64_t n = sv->c->n;
  auto* r = new SReq();
  r->xct = xct;
  r->m = m;
  r->gk = gk;
  r->y = y_out;
  r->npairs = (uint64_t)rows * m->classes;
  r->nout = (r->npairs + n - 1) / n;
  r->out_g0.assign(r->nout, UINT32_MAX);
  r->out_g1.assign(r->nout, 0);
  r->nparts = parts_needed(sv, r->npairs, r->nout);
  r->t_submit = Clock::now();
  // the worker's first tile with this request waits for what the caller queued
  // on `stream` so far (the encryption that wrote xct, typically)
  hipError_t herr = hipSetDevice(sv->c->device);
  if (herr == hipSuccess) herr = hipEventCreateWithFlags(&r->ready, hipEventDisableTiming);
  if (herr == hipSuccess) herr = hipEventRecord(r->ready, (hipStream_t)stream);
  auto drop = [&]() {
    if (r->ready) (void)hipEventDestroy(r->ready);
    delete r;
  };
  if (herr != hipSuccess) {
    drop();
    return perr(LRHE_EDEVICE, "submit: %s", hipGetErrorString(herr));
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->error) {
    drop();
    return perr(sv->error, "server stopped: %s", sv->error_msg.c_str());
  }
  if (r->nparts > sv->arena_slots) {
    drop();
    return perr(LRHE_EINVAL, "request needs %u partial slots, the budget holds %u", r->nparts, sv->arena_slots);
  }
  if (!arena_alloc(sv, r->nparts, &r->part0)) {
    drop();
    return perr(LRHE_EAGAIN, "admission refused: partial-sum budget in use");
  }
  r->id = sv->next_id++;
  sv->reqs[r->id] = r;
  sv->queue.push_back(r);
  *req_id = r->id;
  sv->cv.notify_all();
  return LRHE_OK;
}

extern "C" int lrhe_server_poll(lrhe_server* sv, uint64_t req_id, int* done, double* latency_s) {
  if (!sv || !done) return perr(LRHE_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->error) return perr(sv->error, "server stopped: %s", sv->error_msg.c_str());
  auto it = sv->reqs.find(req_id);
  if (it == sv->reqs.end()) return perr(LRHE_EINVAL, "unknown request %llu", (unsigned long long)req_id);
  *done = it->second->state == 2;
  if (latency_s)
    *latency_s = *done ? std::chrono::duration<double>(it->second->t_done - it->second->t_submit).count() : -1.0;
  return LRHE_OK;
}

extern "C" int lrhe_server_release(lrhe_server* sv, uint64_t req_id) {
  if (!sv) return perr(LRHE_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(req_id);
  if (it == sv->reqs.end()) return perr(LRHE_EINVAL, "unknown request %llu", (unsigned long long)req_id);
  if (it->second->state != 2) return perr(LRHE_EINVAL, "request %llu is not done", (unsigned long long)req_id);
  delete it->second;
  sv->reqs.erase(it);
  return LRHE_OK;
}

extern "C" int lrhe_server_drain(lrhe_server* sv) {
  if (!sv) return perr(LRHE_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv.wait(lk, [&] { return (sv->queue.empty() && sv->inflight.empty()) || sv->error; });
  if (sv->error) return perr(sv->error, "server stopped: %s", sv->error_msg.c_str());
  return LRHE_OK;
}

extern "C" int lrhe_server_stats(lrhe_server* sv, uint64_t* ticks, uint64_t* pairs, uint32_t* free_slots,
                                 uint32_t* tile, uint32_t* held) {
  if (!sv) return perr(LRHE_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticks) *ticks = sv->ticks;
  if (pairs) *pairs = sv->pairs_done;
  if (free_slots) {
    uint32_t f = 0;
    for (auto& r : sv->free_ranges) f += r.second;
    *free_slots = f;
  }
  if (tile) *tile = sv->B;
  if (held) *held = (uint32_t)sv->reqs.size();
  return LRHE_OK;
}

extern "C" void lrhe_server_destroy(lrhe_server* sv) {
  if (!sv) return;
  if (sv->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
    }
    sv->cv.notify_all();
    sv->worker.join();
  }
  if (sv->s) (void)hipStreamSynchronize(sv->s);
  for (auto& kv : sv->reqs) {
    if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete kv.second;
  }
  for (int k = 0; k < 2; ++k) {
    if (sv->d_desc[k]) (void)hipFree(sv->d_desc[k]);
    if (sv->h_desc[k]) (void)hipHostFree(sv->h_desc[k]);
    if (sv->slot_ev[k]) (void)hipEventDestroy(sv->slot_ev[k]);
  }
  if (sv->d_tile) (void)hipFree(sv->d_tile);
  if (sv->d_part) (void)hipFree(sv->d_part);
  if (sv->s) (void)hipStreamDestroy(sv->s);
  delete sv;
}
