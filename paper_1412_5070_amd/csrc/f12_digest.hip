// Output digest for streamed runs.  The integral blocks of a long run do not
// all fit in memory, so each chunk written to the output ring is reduced to a
// 64-bit checksum that can be logged beside the chunk's quartet range and
// compared between runs (or used to restart at a chunk).
//
// Definition: for the doubles x_e of a range whose first element has the
// global index e0 (the offset of the first quartet's block in the list),
//   D = sum_e  mix(bits(x_e) + G (e0 + e + 1))   (mod 2^64),
// with G = 0x9E3779B97F4A7C15 and mix the SplitMix64 output function
// (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014):  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
// z *= 0x94D049BB133111EB; z ^= z >> 31.  For x_e = 0 the terms are the
// outputs of SplitMix64 seeded with G e0.  The sum is commutative, so the
// result does not depend on the reduction order, and the digest of a range is
// the sum (mod 2^64) of the digests of any split of it into sub-ranges.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/f12int.h"
#include "f12_handles.h"

namespace f12 {

constexpr uint64_t DIGEST_GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t digest_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Grid-stride over the range with eight loads in flight per lane (consecutive
// lanes read consecutive doubles); the position term G (e0 + e + 1) advances by
// additions.  Lanes sum their partial digests across the wave by shuffles, the
// waves through LDS, and each work-group adds its total with one 64-bit
// atomic; the grid is capped at 1024 work-groups so that the atomics, which
// all meet at one address, stay few.
constexpr int DIGEST_THREADS = 256;
constexpr int DIGEST_UNROLL = 8;
constexpr int DIGEST_MAX_GROUPS = 1024;

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)v, o, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
    v += ((uint64_t)hi << 32) | lo;
  }
  return v;
}

__global__ void __launch_bounds__(DIGEST_THREADS) digest_kernel(const double *__restrict__ x, int64_t n,
                                                                int64_t e0, unsigned long long *out) {
  const int64_t stride = (int64_t)gridDim.x * DIGEST_THREADS;
  int64_t e = (int64_t)blockIdx.x * DIGEST_THREADS + threadIdx.x;
  const uint64_t gstep = DIGEST_GAMMA * (uint64_t)stride;
  uint64_t pos = DIGEST_GAMMA * (uint64_t)(e0 + e + 1);
  uint64_t s = 0;
  for (; e + (DIGEST_UNROLL - 1) * stride < n; e += DIGEST_UNROLL * stride) {
    uint64_t b[DIGEST_UNROLL];
#pragma unroll
    for (int u = 0; u < DIGEST_UNROLL; ++u) b[u] = (uint64_t)__double_as_longlong(x[e + u * stride]);
#pragma unroll
    for (int u = 0; u < DIGEST_UNROLL; ++u) {
      s += digest_mix(b[u] + pos);
      pos += gstep;
    }
  }
  for (; e < n; e += stride) {
    s += digest_mix((uint64_t)__double_as_longlong(x[e]) + pos);
    pos += gstep;
  }
  s = wave_sum_u64(s);
  __shared__ uint64_t part[DIGEST_THREADS / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
#pragma unroll
    for (int w = 0; w < DIGEST_THREADS / 64; ++w) t += part[w];
    atomicAdd(out, (unsigned long long)t);
  }
}

}  // namespace f12

using namespace f12;

extern "C" int f12_digest(const f12_quartets *q, int64_t q_begin, int64_t q_end, const double *d_out,
                          uint64_t *d_digest, void *stream) {
  if (!q || !d_digest || q_begin < 0 || q_end > q->nq || q_begin > q_end) return F12_EINVAL;
  const int64_t e0 = q->qoff[q_begin];
  const int64_t n = q->qoff[q_end] - e0;
  if (n == 0) return F12_OK;
  if (!d_out) return F12_EINVAL;
  const int64_t per_group = (int64_t)DIGEST_THREADS * DIGEST_UNROLL;
  const unsigned grid = (unsigned)std::min<int64_t>((n + per_group - 1) / per_group, DIGEST_MAX_GROUPS);
  hipLaunchKernelGGL(digest_kernel, dim3(grid), dim3(DIGEST_THREADS), 0, (hipStream_t)stream, d_out, n, e0,
                     (unsigned long long *)d_digest);
  return hipGetLastError() == hipSuccess ? F12_OK : F12_EDEVICE;
}
