// valu_rate.hip -- issue-rate measurement of the vector instructions the
// transforms are built from, on the GPU the library runs on.  It backs the
// ALU roofline of the key-switch kernels: a Montgomery product issues two
// v_mad_u64_u32 and one v_mul_lo_u32, and the peak follows from how many
// lanes per cycle each of them retires.
//
// Every single-instruction probe is a chain of inline-asm instructions, each
// reading the previous result of its chain, so the compiler can neither fold
// nor reassociate the chain (a chain of plain C multiplications by one value
// may be rewritten as one multiplication by a power).  Eight independent
// chains per lane and many waves per SIMD hide the dependency latency.  The
// butterfly probes are compiled C, the same arithmetic as the transforms.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lrhe.h"
#include "lrhe_internal.h"
#include "lrhe_math.h"

namespace lrhe {
namespace {

constexpr int CH = 8;        // independent chains per lane
constexpr int UNR = 16;      // instructions per chain per loop iteration
constexpr int BLOCK = 256;

template <int OP>
__global__ __launch_bounds__(BLOCK) void k_valu_rate(uint32_t y, uint32_t q, uint32_t qinv, int iters,
                                                     uint32_t* __restrict__ out) {
  const uint32_t gid = blockIdx.x * BLOCK + threadIdx.x;
  uint32_t v[CH];
  uint64_t w[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    v[c] = gid * 2654435761u + (uint32_t)c * 40503u + 1u;
    w[c] = ((uint64_t)v[c] << 32) | (v[c] ^ 0x9e3779b9u);
  }
  const uint32_t yv = y ^ (gid & 1u);   // a per-lane operand (held in a VGPR)
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        if constexpr (OP == 0) {
          asm volatile("v_add_u32 %0, %0, %1" : "+v"(v[c]) : "v"(yv));
        } else if constexpr (OP == 1) {
          asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(v[c]) : "v"(yv));
        } else if constexpr (OP == 2) {
          asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(v[c]) : "v"(yv));
        } else if constexpr (OP == 3) {
          // all chains in one asm block: the compiler puts a wait state after
          // every asm block that writes a 64-bit register pair
          if (c == 0) {
            uint64_t cy[CH];
            asm volatile(
                "v_mad_u64_u32 %0, %8, %16, %24, %0\n\t"
                "v_mad_u64_u32 %1, %9, %17, %24, %1\n\t"
                "v_mad_u64_u32 %2, %10, %18, %24, %2\n\t"
                "v_mad_u64_u32 %3, %11, %19, %24, %3\n\t"
                "v_mad_u64_u32 %4, %12, %20, %24, %4\n\t"
                "v_mad_u64_u32 %5, %13, %21, %24, %5\n\t"
                "v_mad_u64_u32 %6, %14, %22, %24, %6\n\t"
                "v_mad_u64_u32 %7, %15, %23, %24, %7"
                : "+v"(w[0]), "+v"(w[1]), "+v"(w[2]), "+v"(w[3]), "+v"(w[4]), "+v"(w[5]), "+v"(w[6]), "+v"(w[7]),
                  "=s"(cy[0]), "=s"(cy[1]), "=s"(cy[2]), "=s"(cy[3]), "=s"(cy[4]), "=s"(cy[5]), "=s"(cy[6]),
                  "=s"(cy[7])
                : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]), "v"(yv));
            // the multiplicand of each chain follows its high word
#pragma unroll
            for (int k = 0; k < CH; ++k) v[k] = (uint32_t)(w[k] >> 32);
          }
        } else if constexpr (OP == 4) {
          // Montgomery forward butterfly of the transforms (lazy, values < 4q)
          uint32_t& a = v[c];
          uint32_t b = (uint32_t)w[c];
          const uint32_t q2 = 2 * q;
          const uint32_t X = umin(a, a - q2);
          const uint32_t T = mulm(b, yv, q, qinv);
          a = X + T;
          w[c] = (w[c] & 0xffffffff00000000ull) | (uint32_t)(X + q2 - T);
        }
      }
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += v[c] + (uint32_t)w[c] + (uint32_t)(w[c] >> 32);
  out[gid] = s;
}

template <int OP>
hipError_t launch(uint32_t blocks, int iters, hipStream_t s, uint32_t* out) {
  // q: a 30-bit prime of the n = 16384 parameter set; qinv = -q^-1 mod 2^32
  const uint32_t q = 1073643521u;
  uint32_t inv = 1;
  for (int i = 0; i < 5; ++i) inv *= 2u - q * inv;
  k_valu_rate<OP><<<blocks, BLOCK, 0, s>>>(0x3bd1e995u, q, 0u - inv, iters, out);
  return hipGetLastError();
}

}  // namespace
}  // namespace lrhe

// op: 0 v_add_u32, 1 v_mul_lo_u32, 2 v_mul_hi_u32, 3 v_mad_u64_u32 (lane
// instructions per second), 4 the transforms' Montgomery forward butterfly
// (butterflies per second).  The kernel runs `iters` loop iterations of
// 8 x 16 operations per lane on 64 workgroups of 256 lanes per compute unit;
// the best of `reps` timed launches (after one warm-up) is reported.
extern "C" int lrhe_prof_valu_rate(int op, int iters, int reps, double* per_s, double* best_ms) {
  using namespace lrhe;
  if (op < 0 || op > 4 || iters <= 0 || reps <= 0 || !per_s) return LRHE_EINVAL;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return LRHE_EDEVICE;
  const uint32_t blocks = (uint32_t)cus * 64u;
  uint32_t* out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipMalloc((void**)&out, (size_t)blocks * BLOCK * 4) != hipSuccess) return LRHE_EDEVICE;
  int rc = LRHE_OK;
  double best = 1e30;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&a) != hipSuccess ||
      hipEventCreate(&b) != hipSuccess) {
    rc = LRHE_EDEVICE;
  } else {
    for (int r = 0; r <= reps && rc == LRHE_OK; ++r) {
      hipError_t e = hipEventRecord(a, s);
      if (e == hipSuccess) {
        switch (op) {
          case 0: e = launch<0>(blocks, iters, s, out); break;
          case 1: e = launch<1>(blocks, iters, s, out); break;
          case 2: e = launch<2>(blocks, iters, s, out); break;
          case 3: e = launch<3>(blocks, iters, s, out); break;
          default: e = launch<4>(blocks, iters, s, out); break;
        }
      }
      if (e == hipSuccess) e = hipEventRecord(b, s);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e != hipSuccess) rc = LRHE_EDEVICE;
      else if (r > 0 && ms < best) best = ms;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(out);
  if (rc != LRHE_OK) return rc;
  const double ops = (double)blocks * BLOCK * (double)iters * UNR * CH;
  *per_s = ops / (best * 1e-3);
  if (best_ms) *best_ms = best;
  return LRHE_OK;
}
