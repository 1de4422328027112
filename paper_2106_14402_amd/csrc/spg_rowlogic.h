// Per-slice index logic written for one lane of a group of `nlanes` lanes
// that run it together.  The kernels run it on the lanes of a wave or a
// workgroup, with the ordering noted at each step; the host tests run the
// same functions lane by lane on the CPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spg {

__host__ __device__ inline int imin_rl(int a, int b) { return a < b ? a : b; }

// Panel index of one slice of `len` ids: out[p] (p = 0..P) = position of the
// first id >= p * 2^wlog2 when the ids are sorted ascending, i.e. the number
// of ids below that column.  Step 1 sets every slot to len.
__host__ __device__ inline void panel_index_fill(int32_t* out, int P, int32_t len, int lane, int nlanes) {
  for (int p = lane; p <= P; p += nlanes) out[p] = len;
}

// Step 2, once step 1's writes are complete: each id opens the panels from
// the one after its predecessor's panel up to its own.  For sorted ids every
// slot up to the last id's panel is written exactly once; for any order every
// value written lies in [0, len).
// Ids are read in groups of kOpenUnroll per lane, all loads of a group
// before any use.
constexpr int kOpenUnroll = 8;

__host__ __device__ inline void panel_index_open(const int32_t* ids, int64_t len, int wlog2, int P, int32_t* out,
                                                 int lane, int nlanes) {
  for (int64_t b0 = 0; b0 < len; b0 += static_cast<int64_t>(kOpenUnroll) * nlanes) {
    int32_t cur[kOpenUnroll], prev[kOpenUnroll];
    for (int u = 0; u < kOpenUnroll; ++u) {
      const int64_t q = b0 + static_cast<int64_t>(u) * nlanes + lane;
      cur[u] = q < len ? ids[q] : 0;
      prev[u] = (q > 0 && q < len) ? ids[q - 1] : 0;
    }
    for (int u = 0; u < kOpenUnroll; ++u) {
      const int64_t q = b0 + static_cast<int64_t>(u) * nlanes + lane;
      if (q >= len) continue;
      const int cp = imin_rl(cur[u] >> wlog2, P);
      const int pp = q == 0 ? -1 : imin_rl(prev[u] >> wlog2, P);
      for (int p = pp + 1; p <= cp; ++p) out[p] = static_cast<int32_t>(q);
    }
  }
}

// One step of the bitonic sorting network over L keys (with a position
// payload) in which every comparator puts the smaller key first: merge k
// (k = 2, 4, ..., N, N the power of two >= L) starts with the mirrored step
// j = k/2 and continues with the half-cleaners j = k/4, ..., 1.  Positions at
// or past L are virtual +infinity keys: a comparator that reaches them would
// keep them in place, so it is skipped, and no padding is stored.
// Comparators c = lane, lane + nlanes, ... < N/2 of the step; the steps run in
// order with all of a step's writes complete before the next step reads.
template <class K>
__host__ __device__ inline void sort_network_step(K* key, int32_t* pos, int L, int N, int k, int j, int lane,
                                                  int nlanes) {
  const int half = N >> 1;
  for (int c = lane; c < half; c += nlanes) {
    int lo, hi;
    if (j == (k >> 1)) {
      const int base = (c / j) * k, o = c % j;
      lo = base + o;
      hi = base + k - 1 - o;
    } else {
      lo = 2 * c - (c & (j - 1));
      hi = lo + j;
    }
    if (hi < L) {
      const K a = key[lo], b = key[hi];
      if (b < a) {
        key[lo] = b;
        key[hi] = a;
        const int32_t t = pos[lo];
        pos[lo] = pos[hi];
        pos[hi] = t;
      }
    }
  }
}

__host__ __device__ inline int network_size(int L) {
  int N = 1;
  while (N < L) N <<= 1;
  return N;
}

}  // namespace spg
