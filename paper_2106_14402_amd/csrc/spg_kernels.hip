// gfx950 kernels of the semiring sparse product C = A (x).(+) B.
//
// Pipeline (paper Sec. 4.1: flop estimate and work split, symbolic phase,
// numeric phase; Sec. 4.1 hybrid accumulator chosen per output slice):
//   k_flops_bin     products per row of C and its symbolic bin
//   k_scatter       row lists per bin (heaviest dense rows first)
//   k_panel_index   per B row, offsets of its column panels
//   k_hash_sym      row pattern size with an LDS hash set (light rows)
//   k_dense_sym     row pattern size with an LDS bitmap per column panel
//   k_scan_*        int64 exclusive scan of row sizes into C's offsets
//   k_hash_num      LDS hash accumulator, compaction and bitonic sort
//   k_dense_num     dense LDS panel (presence bits + values), emitted in
//                   column order with coalesced stores
//   k_prune_*       keep entries >= threshold (Markov-clustering step)
// The work is sparse gathers, LDS atomics and streaming stores; no matrix
// cores are involved.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "spg_launch.h"
#include "spg_rowlogic.h"

namespace spg {

// ---------------------------------------------------------------------------
// Small utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = (n + nt - 1) / nt;
  hipLaunchKernelGGL(k_fill_u64, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, p, n, v);
  return hipGetLastError();
}

// Workgroups for the row-striding preparation kernels: 8 of 256 threads per
// compute unit (one workgroup per row would spend the time in dispatch).
static int64_t prep_blocks() {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                hipSuccess && v > 0)
      ncu = v;
    else
      ncu = 256;
  }
  return static_cast<int64_t>(ncu) * 8;
}

// Workgroups for the prune and inflation kernels, one wave per slice: one
// workgroup per group of slices, up to 2^22 (the kernels stride beyond).  The
// dispatcher balances their uneven slices better than a grid of a few
// workgroups per CU striding over them (prune placement 7.9 -> 6.8 ms, count
// 2.0 -> 1.7, inflation 1.9 -> 1.5 on the MCL matrix).  The operand checks
// measured slower that way, and the flop count reduces into global counters
// per workgroup: both keep the small grid of prep_blocks().
static int64_t wave_grid(int64_t slices, int nt) {
  return std::min<int64_t>((slices + nt / kWave - 1) / (nt / kWave), int64_t(1) << 22);
}

// Operand check: ptr[0] == 0, ptr non-decreasing within [0, nnz],
// ptr[nmajor] == nnz, ids in [0, nminor), and the order of the ids of each
// slice.  Error bits (kCheck*): bad endpoints, bad offsets, an id out of
// range, a descending pair of adjacent ids (the slice is not sorted), an equal
// pair of adjacent ids (a duplicate, or a possible one in an unsorted slice).
// One wave per slice; never reads outside [0, nnz).
constexpr int kValidateUnroll = 8;

__global__ void k_validate(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                           int64_t nmajor, int64_t nnz, int32_t nminor, int* err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
  int e = 0;
  for (int64_t s = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6); s < nmajor;
       s += waves) {
    if (lane == 0) {
      if (s == 0 && ptr[0] != 0) e |= kCheckEnds;
      if (s == nmajor - 1 && ptr[nmajor] != nnz) e |= kCheckEnds;
    }
    const int64_t lo = ptr[s], hi = ptr[s + 1];
    if (lo < 0 || hi > nnz || hi < lo) {
      e |= kCheckOffsets;
    } else {
      // kValidateUnroll groups of 64 ids loaded at once; an id's predecessor
      // comes from the lane below (lane 0: one more load)
      constexpr int U = kValidateUnroll;
      for (int64_t b0 = lo; b0 < hi; b0 += U * kWave) {
        int32_t c[U], pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t q = b0 + u * kWave + lane;
          c[u] = q < hi ? idx[q] : 0;
          pv[u] = (lane == 0 && q > lo && q < hi) ? idx[q - 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t q = b0 + u * kWave + lane;
          const int32_t below = __shfl_up(c[u], 1, kWave);
          const int32_t b = lane == 0 ? pv[u] : below;
          if (q < hi) {
            if (c[u] < 0 || c[u] >= nminor) e |= kCheckRange;
            if (q > lo) {
              if (b > c[u]) e |= kCheckUnsorted;
              if (b == c[u]) e |= kCheckDuplicate;
            }
          }
        }
      }
    }
  }
  e = wave_or(e);
  if (lane == 0 && e) atomicOr(err, e);
}

hipError_t launch_validate(const int64_t* ptr, const int32_t* idx, int64_t nmajor, int64_t nnz,
                           int32_t nminor, int* err, hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = std::min<int64_t>((nmajor + nt / kWave - 1) / (nt / kWave), prep_blocks());
  hipLaunchKernelGGL(k_validate, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, ptr, idx, nmajor,
                     nnz, nminor, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sorted copy of a CSR operand whose slices are not all sorted: the ids of
// every slice in ascending order, with their values, into out_idx / out_val
// (same offsets).  One workgroup per slice.  A slice that is already sorted
// is copied as it is.  Otherwise its (id, position) pairs go through a
// bitonic sorting network: in LDS up to kSortLds ids, else in global memory
// (out_idx and the position scratch `pos`, both indexed like idx).  The
// network is the variant in which each merge starts with a mirrored
// compare-exchange step, so every comparator puts the smaller id first; the
// padding up to a power of two is then never touched (it would hold +inf and
// stay in place).  Values follow their ids through the positions.  Equal ids
// keep an arbitrary order: the caller checks the copy for duplicates.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortLds = 2048;

template <class K>
__device__ __forceinline__ void sort_network(K* key, int32_t* pos, int L) {
  const int N = network_size(L);
  for (int k = 2; k <= N; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      sort_network_step(key, pos, L, N, k, j, static_cast<int>(threadIdx.x), static_cast<int>(blockDim.x));
      __syncthreads();
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_slices(const int64_t* __restrict__ ptr,
                                                              const int32_t* __restrict__ idx,
                                                              const unsigned char* __restrict__ val, int es,
                                                              int64_t nmajor, int32_t* __restrict__ out_idx,
                                                              unsigned char* __restrict__ out_val,
                                                              int32_t* __restrict__ pos) {
  __shared__ int32_t skey[kSortLds];
  __shared__ int32_t spos[kSortLds];
  __shared__ int unsorted;
  for (int64_t s = blockIdx.x; s < nmajor; s += gridDim.x) {
    const int64_t lo = ptr[s], hi = ptr[s + 1];
    const int L = static_cast<int>(hi - lo);
    if (threadIdx.x == 0) unsorted = 0;
    __syncthreads();
    int u = 0;
    for (int t = threadIdx.x + 1; t < L; t += blockDim.x) u |= idx[lo + t - 1] > idx[lo + t];
    if (u) unsorted = 1;
    __syncthreads();
    if (!unsorted) {
      for (int t = threadIdx.x; t < L; t += blockDim.x) out_idx[lo + t] = idx[lo + t];
      for (int64_t b = threadIdx.x; b < static_cast<int64_t>(L) * es; b += blockDim.x)
        out_val[lo * es + b] = val[lo * es + b];
      __syncthreads();
      continue;
    }
    int32_t* key;
    int32_t* ps;
    if (L <= kSortLds) {
      key = skey;
      ps = spos;
    } else {
      key = out_idx + lo;
      ps = pos + lo;
    }
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
      key[t] = idx[lo + t];
      ps[t] = t;
    }
    __syncthreads();
    sort_network(key, ps, L);
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
      const int src = ps[t];
      if (L <= kSortLds) out_idx[lo + t] = key[t];
      if (es == 8)
        reinterpret_cast<uint64_t*>(out_val)[lo + t] = reinterpret_cast<const uint64_t*>(val)[lo + src];
      else if (es == 4)
        reinterpret_cast<uint32_t*>(out_val)[lo + t] = reinterpret_cast<const uint32_t*>(val)[lo + src];
      else if (es == 1)
        out_val[lo + t] = val[lo + src];
    }
    __syncthreads();
  }
}

hipError_t launch_sort_slices(const int64_t* ptr, const int32_t* idx, const void* val, int es, int64_t nmajor,
                              int32_t* out_idx, void* out_val, int32_t* pos, hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const unsigned nb = static_cast<unsigned>(std::min<int64_t>(nmajor, 65536));
  hipLaunchKernelGGL(k_sort_slices, dim3(nb), dim3(kSortThreads), 0, s, ptr, idx,
                     static_cast<const unsigned char*>(val), val ? es : 0, nmajor, out_idx,
                     static_cast<unsigned char*>(out_val), pos);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Flop count and binning (paper Sec. 4.1 phase 1: estimate the flops of every
// output slice before splitting the work).  flops_i = sum over A(i,k) of
// nnz(B(k,:)).  One wave per row.
// ---------------------------------------------------------------------------
__global__ void k_flops_bin(Operands op, int64_t a_nnz, BinParams bp, int64_t* __restrict__ flops,
                            int64_t* __restrict__ c_ptr, unsigned long long* counts,
                            unsigned long long* total, int* err) {
  // Also checks A as k_validate does (same error bits into *err), and reads
  // nothing outside A's arrays or B's offsets whatever A holds.
  __shared__ unsigned int lc[kNumBins];
  __shared__ unsigned long long ltot;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  if (tid < kNumBins) lc[tid] = 0;
  if (tid == 0) ltot = 0;
  __syncthreads();
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (tid >> 6); i < op.m; i += waves) {
    int e = 0;
    int64_t f = 0;
    const int64_t lo = op.a_ptr[i], hi = op.a_ptr[i + 1];
    if (lane == 0) {
      if (i == 0 && lo != 0) e |= kCheckEnds;
      if (i == op.m - 1 && hi != a_nnz) e |= kCheckEnds;
    }
    if (lo < 0 || hi > a_nnz || hi < lo) {
      e |= kCheckOffsets;
    } else {
      for (int64_t p = lo + lane; p < hi; p += kWave) {
        const int32_t k = op.a_idx[p];
        if (k < 0 || k >= op.n) {
          e |= kCheckRange;
          continue;
        }
        if (p > lo) {
          const int32_t b = op.a_idx[p - 1];
          if (b > k) e |= kCheckUnsorted;
          if (b == k) e |= kCheckDuplicate;
        }
        f += op.b_ptr[k + 1] - op.b_ptr[k];
      }
    }
    f = wave_sum(f);
    e = wave_or(e);
    if (lane == 0) {
      flops[i] = f;
      if (f == 0) c_ptr[i + 1] = 0;
      atomicAdd(&lc[sym_bin(f, bp)], 1u);
      atomicAdd(&ltot, static_cast<unsigned long long>(f));
      if (e) atomicOr(err, e);
    }
  }
  __syncthreads();
  if (tid < kNumBins && lc[tid]) atomicAdd(&counts[tid], static_cast<unsigned long long>(lc[tid]));
  if (tid == 0 && ltot) atomicAdd(total, ltot);
}

hipError_t launch_flops_bin(const Operands& op, int64_t a_nnz, BinParams bp, int64_t* flops, int64_t* c_ptr,
                            unsigned long long* counts, unsigned long long* total, int* err, hipStream_t s) {
  if (op.m <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = std::min<int64_t>((static_cast<int64_t>(op.m) + nt / kWave - 1) / (nt / kWave), prep_blocks());
  hipLaunchKernelGGL(k_flops_bin, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, op, a_nnz, bp, flops,
                     c_ptr, counts, total, err);
  return hipGetLastError();
}

// Numeric bin counts of rows [r0, m).  Before the scan c_ptr[i+1] holds the
// nnz of row i (scanned = 0); after it, c_ptr holds offsets (scanned = 1).
__global__ void k_count_num_bins(int32_t m, int32_t r0, int scanned, const int64_t* __restrict__ flops,
                                 const int64_t* __restrict__ c_ptr, BinParams bp,
                                 unsigned long long* counts) {
  __shared__ unsigned int lc[kNumBins];
  const int tid = threadIdx.x;
  if (tid < kNumBins) lc[tid] = 0;
  __syncthreads();
  const int64_t i = r0 + static_cast<int64_t>(blockIdx.x) * blockDim.x + tid;
  if (i < m) {
    const int64_t nz = scanned ? c_ptr[i + 1] - c_ptr[i] : c_ptr[i + 1];
    const bool split = bp.split_heavy && flops[i] > bp.hash_max_flops;
    const bool ranked = bp.rank_heavy && flops[i] > bp.hash_max_flops && nz > bp.hash_max_nnz &&
                        !esc_row(nz, flops[i], bp.esc_max_flops, bp.esc_ratio_x16);
    const bool kept = bp.row_slot && flops[i] > bp.hash_max_flops && bp.row_slot[i] >= 0;
    atomicAdd(&lc[kept ? kExpandBin : ((split || ranked) ? 0 : num_bin(nz, flops[i], bp))], 1u);
  }
  __syncthreads();
  if (tid < kNumBins && lc[tid]) atomicAdd(&counts[tid], static_cast<unsigned long long>(lc[tid]));
}

hipError_t launch_count_num_bins(int32_t m, int32_t r0, int scanned, const int64_t* flops, const int64_t* c_ptr,
                                 BinParams bp, unsigned long long* counts, hipStream_t s) {
  if (m - r0 <= 0) return hipSuccess;
  const int nt = 256;
  hipLaunchKernelGGL(k_count_num_bins, dim3((m - r0 + nt - 1) / nt), dim3(nt), 0, s, m, r0, scanned, flops,
                     c_ptr, bp, counts);
  return hipGetLastError();
}

// Row lists per bin.  Each block reserves one range per bin with a single
// global atomic; row order inside a bin is unspecified.
__global__ void k_scatter(int mode, int32_t m, int32_t r0, const int64_t* __restrict__ flops,
                          const int64_t* __restrict__ c_ptr, BinParams bp, BinOffsets offs,
                          unsigned long long* cursors, int32_t* __restrict__ rows_out) {
  __shared__ unsigned int lc[kNumBins];
  __shared__ unsigned long long lbase[kNumBins];
  const int tid = threadIdx.x;
  if (tid < kNumBins) lc[tid] = 0;
  __syncthreads();
  const int64_t i = r0 + static_cast<int64_t>(blockIdx.x) * blockDim.x + tid;
  int bin = 0;
  unsigned int local = 0;
  if (i < m) {
    if (mode == 0)
      bin = sym_bin(flops[i], bp);
    else if (bp.row_slot && flops[i] > bp.hash_max_flops && bp.row_slot[i] >= 0)
      bin = kExpandBin;
    else {
      const int64_t nz = c_ptr[i + 1] - c_ptr[i];
      const bool ranked = bp.rank_heavy && flops[i] > bp.hash_max_flops && nz > bp.hash_max_nnz &&
                          !esc_row(nz, flops[i], bp.esc_max_flops, bp.esc_ratio_x16);
      bin = ((bp.split_heavy && flops[i] > bp.hash_max_flops) || ranked) ? 0 : num_bin(nz, flops[i], bp);
    }
    if (bin > 0) local = atomicAdd(&lc[bin], 1u);
  }
  __syncthreads();
  if (tid < kNumBins && lc[tid])
    lbase[tid] = atomicAdd(&cursors[tid], static_cast<unsigned long long>(lc[tid]));
  __syncthreads();
  if (bin > 0) rows_out[offs.v[bin] + static_cast<int64_t>(lbase[bin]) + local] = static_cast<int32_t>(i);
}

hipError_t launch_scatter(int mode, int32_t m, int32_t r0, const int64_t* flops, const int64_t* c_ptr,
                          BinParams bp, const BinOffsets& offs, unsigned long long* cursors,
                          int32_t* rows_out, hipStream_t s) {
  if (m - r0 <= 0) return hipSuccess;
  const int nt = 256;
  hipLaunchKernelGGL(k_scatter, dim3((m - r0 + nt - 1) / nt), dim3(nt), 0, s, mode, m, r0, flops, c_ptr, bp,
                     offs, cursors, rows_out);
  return hipGetLastError();
}

// Selector of a semiring sum of k stacked parts (m slices each): slice i
// has k entries, at t*m + i for t = 0..k-1, each the (x)-identity of the
// semiring's input type (es bytes, given as raw bits in `one`).
__global__ void k_selector(int32_t m, int k, int64_t* __restrict__ ptr, int32_t* __restrict__ idx,
                           unsigned char* __restrict__ val, int es, uint64_t one) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t first = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t i = first; i <= m; i += stride) ptr[i] = i * k;
  const int64_t total = static_cast<int64_t>(m) * k;
  for (int64_t e = first; e < total; e += stride) {
    const int64_t i = e / k;
    const int64_t t = e - i * k;
    idx[e] = static_cast<int32_t>(t * m + i);
    if (val) {
      if (es == 8)
        reinterpret_cast<uint64_t*>(val)[e] = one;
      else if (es == 4)
        reinterpret_cast<uint32_t*>(val)[e] = static_cast<uint32_t>(one);
      else
        val[e] = static_cast<unsigned char>(one);
    }
  }
}

hipError_t launch_selector(int32_t m, int k, int64_t* ptr, int32_t* idx, void* val, int sr, hipStream_t s) {
  // the (x)-identity: 1 for (+,x), (max,x) and (OR,AND); 0 for (min,+)
  uint64_t one = 0;
  int es = 0;
  switch (sr) {
    case 0: case 5: { const double v = 1.0; std::memcpy(&one, &v, 8); es = 8; break; }
    case 1: case 6: { const float v = 1.0f; uint32_t b; std::memcpy(&b, &v, 4); one = b; es = 4; break; }
    case 2: case 3: one = 0; es = 4; break;  // int32 0 and float +0.0f
    case 4: one = 1; es = 1; break;
    default: es = 0; break;                  // pattern only: no values
  }
  const int64_t work = static_cast<int64_t>(m) * k + m + 1;
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 65536));
  hipLaunchKernelGGL(k_selector, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, m, k, ptr, idx,
                     static_cast<unsigned char*>(es ? val : nullptr), es, one);
  return hipGetLastError();
}

// B's column ids and 4-byte values side by side (see Operands::b_pair).
__global__ void k_interleave_b(const int32_t* __restrict__ idx, const uint32_t* __restrict__ val, int64_t n,
                               int2* __restrict__ out) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = make_int2(idx[i], static_cast<int32_t>(val[i]));
}

hipError_t launch_interleave_b(const Operands& op, int64_t nnz, int2* out, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((nnz + 255) / 256, 65536);
  hipLaunchKernelGGL(k_interleave_b, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, op.b_idx,
                     static_cast<const uint32_t*>(op.b_val), nnz, out);
  return hipGetLastError();
}

// Smallest and largest of n int32 values into mm[0], mm[1] (initialised by
// the caller to INT32_MAX and INT32_MIN).
__global__ void k_value_range(const int32_t* __restrict__ v, int64_t n, int32_t* mm) {
  int32_t lo = INT32_MAX, hi = INT32_MIN;
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t x = v[q];
    lo = min(lo, x);
    hi = max(hi, x);
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    lo = min(lo, __shfl_xor(lo, d, kWave));
    hi = max(hi, __shfl_xor(hi, d, kWave));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMin(&mm[0], lo);
    atomicMax(&mm[1], hi);
  }
}

__global__ void k_mm_init(int32_t* mm) {
  mm[0] = INT32_MAX;
  mm[1] = INT32_MIN;
}

hipError_t launch_value_range(const int32_t* v, int64_t n, int32_t* mm, hipStream_t s) {
  hipLaunchKernelGGL(k_mm_init, dim3(1), dim3(1), 0, s, mm);
  if (n > 0) {
    const unsigned nb = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_value_range, dim3(nb), dim3(256), 0, s, v, n, mm);
  }
  return hipGetLastError();
}

// One word per entry of B: value << bits | column id (values checked to fit).
__global__ void k_pack_b(const int32_t* __restrict__ idx, const int32_t* __restrict__ val, int64_t n, int bits,
                         uint32_t* __restrict__ out) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < n) out[q] = (static_cast<uint32_t>(val[q]) << bits) | static_cast<uint32_t>(idx[q]);
}

hipError_t launch_pack_b(const Operands& op, int64_t nnz, int bits, uint32_t* out, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_b, dim3(static_cast<unsigned>((nnz + 255) / 256)), dim3(256), 0, s, op.b_idx,
                     static_cast<const int32_t*>(op.b_val), nnz, bits, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Panel index: for B row k and panel p (columns [p*W, (p+1)*W)),
// pidx[k*(P+1) + p] = number of entries of B(k,:) with column < p*W, for a
// row sorted ascending.  One wave per row.  Every slot is first set to the
// row length, so the index holds values in [0, len] for any order of ids;
// then, for a sorted row, each slot up to the last entry's panel is written
// by the entry that opens it.  (The library builds indexes only over
// operands it has checked to be sorted.)
// ---------------------------------------------------------------------------
__global__ void k_panel_index(const int64_t* __restrict__ b_ptr, const int32_t* __restrict__ b_idx,
                              int32_t nrows, int wlog2, int P, int32_t* __restrict__ pidx) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t k = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (k >= nrows) return;
  const int64_t lo = b_ptr[k], hi = b_ptr[k + 1];
  int32_t* out = pidx + k * (P + 1);
  panel_index_fill(out, P, static_cast<int32_t>(hi - lo), lane, kWave);
  // the fills reach memory before the writes below (same addresses)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0);
  panel_index_open(b_idx + lo, hi - lo, wlog2, P, out, lane, kWave);
}

hipError_t launch_panel_index(const int64_t* b_ptr, const int32_t* b_idx, int32_t nrows, int wlog2,
                              int P, int32_t* pidx, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = (static_cast<int64_t>(nrows) + nt / kWave - 1) / (nt / kWave);
  hipLaunchKernelGGL(k_panel_index, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, b_ptr, b_idx,
                     nrows, wlog2, P, pidx);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// int64 scan: tile sums, one-block scan of the tile sums, tile scans.
// ---------------------------------------------------------------------------
constexpr int kScanNT = 1024;
constexpr int kScanIPT = kScanTile / kScanNT;

__global__ __launch_bounds__(kScanNT) void k_scan_reduce(const int64_t* __restrict__ x, int64_t len,
                                                         int64_t* __restrict__ partials) {
  __shared__ int64_t tmp[16];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  int64_t v = 0;
#pragma unroll
  for (int r = 0; r < kScanIPT; ++r) {
    const int64_t i = base + r * kScanNT + threadIdx.x;
    if (i < len) v += x[i];
  }
  const int64_t t = block_sum(v, tmp);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kScanNT) void k_scan_partials(int64_t* partials, int64_t nb) {
  __shared__ int64_t tmp[16];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanNT) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nb ? partials[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(v, tmp, &tot);
    if (i < nb) partials[i] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanNT) void k_scan_apply(int64_t* __restrict__ x, int64_t len,
                                                        const int64_t* __restrict__ partials) {
  __shared__ int64_t tmp[16];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanIPT;
  int64_t v[kScanIPT];
  int64_t run = 0;
#pragma unroll
  for (int r = 0; r < kScanIPT; ++r) {
    const int64_t i = base + r;
    v[r] = i < len ? x[i] : 0;
    run += v[r];
    v[r] = run;
  }
  int64_t tot;
  const int64_t ex = block_exclusive_scan(run, tmp, &tot) + partials[blockIdx.x];
#pragma unroll
  for (int r = 0; r < kScanIPT; ++r) {
    const int64_t i = base + r;
    if (i < len) x[i] = ex + v[r];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) x[-1] = 0;
}

hipError_t launch_scan_inplace(int64_t* x, int64_t len, int64_t* partials, hipStream_t s) {
  if (len <= 0) return launch_fill_u64(reinterpret_cast<uint64_t*>(x - 1), 1, 0, s);
  const int64_t nb = (len + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reduce, dim3(static_cast<unsigned>(nb)), dim3(kScanNT), 0, s, x, len,
                     partials);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanNT), 0, s, partials, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nb)), dim3(kScanNT), 0, s, x, len,
                     partials);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Accumulator sinks
// ---------------------------------------------------------------------------
struct HashSetSink {
  int32_t* keys;
  uint32_t mask;
  int count;
  __device__ void add(int32_t col, uint32_t) {
    uint32_t h = hash_slot(col, mask);
    for (;;) {
      const int32_t cur = *reinterpret_cast<volatile int32_t*>(&keys[h]);
      if (cur == col) return;
      if (cur == kEmpty) {
        const int32_t old = atomicCAS(&keys[h], kEmpty, col);
        if (old == kEmpty) {
          ++count;
          return;
        }
        if (old == col) return;
      }
      h = (h + 1) & mask;
    }
  }
};

template <class SR>
struct HashMapSink {
  using S = typename SR::S;
  int32_t* keys;
  S* vals;
  uint32_t mask;
  __device__ void add(int32_t col, S v) {
    uint32_t h = hash_slot(col, mask);
    for (;;) {
      const int32_t cur = *reinterpret_cast<volatile int32_t*>(&keys[h]);
      if (cur == col) break;
      if (cur == kEmpty) {
        const int32_t old = atomicCAS(&keys[h], kEmpty, col);
        if (old == kEmpty || old == col) break;
      }
      h = (h + 1) & mask;
    }
    if constexpr (!SR::kPattern) SR::combine(&vals[h], v);
  }
};

struct BitmapSink {
  uint32_t* bits;
  __device__ void add(int32_t c, uint32_t) { atomicOr(&bits[c >> 5], 1u << (c & 31)); }
};

template <class SR>
struct DenseSink {
  using S = typename SR::S;
  uint32_t* bits;
  S* vals;
  __device__ void add(int32_t c, S v) {
    atomicOr(&bits[c >> 5], 1u << (c & 31));
    if constexpr (!SR::kPattern) SR::combine(&vals[c], v);
  }
};

// ---------------------------------------------------------------------------
// Symbolic phase (paper Sec. 4.1 phase 2): size of every output row.
//
// Each accumulator is a per-row device function that uses the block's
// dynamic LDS; a single-product kernel and a batched kernel (rows of many
// products in one grid-stride launch, operands read from a descriptor table)
// wrap the same function.
// ---------------------------------------------------------------------------
using PatQueue = RowQueue<SrPattern::In>;

size_t hash_sym_lds(int T, int nt) { return PatQueue::bytes(nt) + static_cast<size_t>(T) * 4; }
size_t dense_sym_lds(int wlog2, int nt) {
  return PatQueue::bytes(nt) + (static_cast<size_t>(1) << wlog2) / 8;
}

template <bool kFlat>
__device__ int64_t hash_sym_row(const Operands& op, int32_t row, int T, int short_seg,
                                unsigned char* smem) {
  const int nt = blockDim.x;
  auto q = PatQueue::carve(smem, nt);
  int32_t* keys = reinterpret_cast<int32_t*>(smem + PatQueue::bytes(nt));
  for (int t = threadIdx.x; t < T; t += nt) keys[t] = kEmpty;
  __syncthreads();
  HashSetSink sink{keys, static_cast<uint32_t>(T - 1), 0};
  enumerate_row<SrPattern, 1, kFlat>(op, op.a_ptr[row], op.a_ptr[row + 1], false, nullptr, 1, 0, 0, short_seg,
                           q, sink);
  return block_sum(sink.count, q.ctr + 2);
}

// Dense symbolic row.  With sub_cnt, also records the pattern size of every
// numeric column panel (2^sub_wlog2 columns, no wider than a bitmap panel),
// so a heavy row can later be split into (row, panel) pieces.
__device__ int64_t dense_sym_row(const Operands& op, int32_t row, int wlog2, int P,
                                 const int32_t* __restrict__ pidx, int short_seg, unsigned char* smem,
                                 int sub_wlog2 = 0, int32_t* __restrict__ sub_cnt = nullptr,
                                 uint32_t* __restrict__ keep = nullptr) {
  const int nt = blockDim.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x >> 6;
  const int nw = nt >> 6;
  auto q = PatQueue::carve(smem, nt);
  uint32_t* bits = reinterpret_cast<uint32_t*>(smem + PatQueue::bytes(nt));
  const int64_t a_lo = op.a_ptr[row], a_hi = op.a_ptr[row + 1];
  int64_t total = 0;
  for (int p = 0; p < P; ++p) {
    const int32_t c0 = p << wlog2;
    const int32_t wcols = min(1 << wlog2, op.k - c0);
    const int nwords = (wcols + 31) >> 5;
    for (int t = threadIdx.x; t < nwords; t += nt) bits[t] = 0u;
    __syncthreads();
    BitmapSink sink{bits};
    enumerate_row<SrPattern>(op, a_lo, a_hi, P > 1, pidx, P, p, c0, short_seg, q, sink);
    if (sub_cnt) {
      const int wps = 1 << (sub_wlog2 - 5);  // words per numeric panel
      const int s0 = c0 >> sub_wlog2;
      const int nsub = (wcols + (1 << sub_wlog2) - 1) >> sub_wlog2;
      for (int j = wid; j < nsub; j += nw) {
        int c = 0;
        for (int t = j * wps + lane; t < min((j + 1) * wps, nwords); t += kWave) c += __popc(bits[t]);
        c = wave_sum(c);
        if (lane == 0) sub_cnt[s0 + j] = c;
      }
    }
    int cnt = 0;
    for (int t = threadIdx.x; t < nwords; t += nt) {
      const uint32_t x = bits[t];
      cnt += __popc(x);
      if (keep) keep[t] = x;
    }
    total += block_sum(cnt, q.ctr + 2);
  }
  return total;
}

__global__ __launch_bounds__(1024) void k_hash_sym(Operands op, const int32_t* __restrict__ rows,
                                                   int64_t nrows, int T, int short_seg,
                                                   int64_t* __restrict__ c_ptr) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = uniform(rows[it]);
    const int64_t nz = hash_sym_row<true>(op, row, T, short_seg, smem);
    if (threadIdx.x == 0) c_ptr[row + 1] = nz;
  }
}

__global__ __launch_bounds__(1024) void k_dense_sym(Operands op, const int32_t* __restrict__ rows,
                                                    int64_t nrows, int wlog2, int P,
                                                    const int32_t* __restrict__ pidx, int short_seg,
                                                    int64_t* __restrict__ c_ptr, int sub_wlog2, int subP,
                                                    int32_t* __restrict__ sub_cnt, KeepBitmaps kb) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int slot_s;
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = uniform(rows[it]);
    uint32_t* keep = nullptr;
    if (kb.store) {
      // The heaviest rows come first; each takes a bitmap slot while any is left.
      if (threadIdx.x == 0) {
        int sl = -1;
        if (kb.flops[row] >= kb.min_flops) {
          const unsigned int v = atomicAdd(kb.counter, 1u);
          if (v < kb.capacity) sl = static_cast<int>(v);
        }
        slot_s = sl;
        kb.row_slot[row] = sl;
      }
      __syncthreads();
      if (slot_s >= 0) keep = kb.store + static_cast<int64_t>(slot_s) * kb.nwords;
    }
    const int64_t nz = dense_sym_row(op, row, wlog2, P, pidx, short_seg, smem, sub_wlog2,
                                     sub_cnt ? sub_cnt + it * subP : nullptr, keep);
    if (threadIdx.x == 0) c_ptr[row + 1] = nz;
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_hash_sym_b(const BatchDesc* __restrict__ descs,
                                                     const int64_t* __restrict__ row_off,
    const int32_t* __restrict__ prod_of, int nprod,
                                                     const int32_t* __restrict__ items, int64_t nitems,
                                                     int T, int short_seg) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t r = uniform(items[it]);
    const int b = uniform(prod_of[r]);
    const BatchDesc d = descs[b];  // uniform: held in scalar registers
    const int32_t row = uniform(static_cast<int32_t>(r - row_off[b]));
    const int64_t nz = hash_sym_row<false>(d.op, row, T, short_seg, smem);
    if (threadIdx.x == 0) d.c_ptr[row + 1] = nz;
  }
}

__global__ __launch_bounds__(1024) void k_dense_sym_b(const BatchDesc* __restrict__ descs,
                                                      const int64_t* __restrict__ row_off,
    const int32_t* __restrict__ prod_of, int nprod,
                                                      const int32_t* __restrict__ items, int64_t nitems,
                                                      int short_seg) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t r = uniform(items[it]);
    const int b = uniform(prod_of[r]);
    const BatchDesc d = descs[b];  // uniform: held in scalar registers
    const int32_t row = uniform(static_cast<int32_t>(r - row_off[b]));
    const int64_t nz = dense_sym_row(d.op, row, d.sym_wlog2, d.sym_P, d.psym, short_seg, smem);
    if (threadIdx.x == 0) d.c_ptr[row + 1] = nz;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Windowed dense symbolic rows.  The columns are cut into P windows and the
// work items are (row, window) pairs, taken from one queue per window.  A
// workgroup starts on the queue of the XCD it runs on: the workgroups of one
// XCD then gather from one column window of B, so the segments of the most
// shared rows of B in that window stay in that XCD's L2 instead of every L2
// holding all of them; a workgroup whose queue is empty takes items from the
// other queues, so every item is done whatever the placement.  Per item: the
// window's bitmap in LDS, its count, the counts of its rank chunks and its
// words of the kept bitmap.
// ---------------------------------------------------------------------------
// XCD of the running wave (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcc_id() {
  return static_cast<int>(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u);
}

// Next (list index, window) item for a workgroup, or it = -1 when every
// queue is exhausted.  Thread 0 only; w and tried carry over between calls.
__device__ __forceinline__ int64_t take_item(unsigned int* __restrict__ queue, int64_t nitems, int P, int& w,
                                             int& tried) {
  while (tried < P) {
    const unsigned int v = atomicAdd(&queue[w], 1u);
    if (static_cast<int64_t>(v) < nitems) return static_cast<int64_t>(v);
    w = w + 1 == P ? 0 : w + 1;
    ++tried;
  }
  return -1;
}

__global__ __launch_bounds__(1024) void k_dense_sym_win(Operands op, const int32_t* __restrict__ rows,
                                                        int64_t nrows, int wlog2, int P,
                                                        const int32_t* __restrict__ pidx, int short_seg,
                                                        int32_t* __restrict__ item_cnt,
                                                        unsigned int* __restrict__ queue, int sub_wlog2,
                                                        int subP, int32_t* __restrict__ sub_cnt,
                                                        const int32_t* __restrict__ keep_slot,
                                                        uint32_t* __restrict__ keep_store, int64_t keep_nwords) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int64_t item_s;
  __shared__ int win_s;
  const int nt = blockDim.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x >> 6;
  const int nw = nt >> 6;
  auto q = PatQueue::carve(smem, nt);
  uint32_t* bits = reinterpret_cast<uint32_t*>(smem + PatQueue::bytes(nt));
  int w = xcc_id() % P, tried = 0;  // thread 0's queue cursor
  for (;;) {
    if (threadIdx.x == 0) {
      item_s = take_item(queue, nrows, P, w, tried);
      win_s = w;
    }
    __syncthreads();
    const int64_t it = item_s;
    const int p = win_s;
    __syncthreads();  // item_s is rewritten by the next take
    if (it < 0) break;
    const int32_t row = uniform(rows[it]);
    const int64_t a_lo = op.a_ptr[row], a_hi = op.a_ptr[row + 1];
    const int32_t c0 = p << wlog2;
    const int32_t wcols = min(1 << wlog2, op.k - c0);
    const int nwords = (wcols + 31) >> 5;
    for (int t = threadIdx.x; t < nwords; t += nt) bits[t] = 0u;
    __syncthreads();
    BitmapSink sink{bits};
    enumerate_row<SrPattern>(op, a_lo, a_hi, P > 1, pidx, P, p, c0, short_seg, q, sink);
    if (sub_cnt) {
      // counts of the rank chunks (2^sub_wlog2 columns, nested in the window)
      const int wps = 1 << (sub_wlog2 - 5);
      const int s0 = c0 >> sub_wlog2;
      const int nsub = (wcols + (1 << sub_wlog2) - 1) >> sub_wlog2;
      for (int j = wid; j < nsub; j += nw) {
        int c = 0;
        for (int t = j * wps + lane; t < min((j + 1) * wps, nwords); t += kWave) c += __popc(bits[t]);
        c = wave_sum(c);
        if (lane == 0) sub_cnt[it * subP + s0 + j] = c;
      }
    }
    uint32_t* keep = nullptr;
    if (keep_slot) {
      const int32_t sl = uniform(keep_slot[row]);
      if (sl >= 0) keep = keep_store + static_cast<int64_t>(sl) * keep_nwords + (c0 >> 5);
    }
    int cnt = 0;
    for (int t = threadIdx.x; t < nwords; t += nt) {
      const uint32_t x = bits[t];
      cnt += __popc(x);
      if (keep) keep[t] = x;
    }
    const int total = block_sum(cnt, q.ctr + 2);
    if (threadIdx.x == 0) item_cnt[it * P + p] = total;
    __syncthreads();
  }
}

// c_ptr[row + 1] = sum of the row's window counts.
__global__ void k_sum_items(const int32_t* __restrict__ rows, int64_t nrows, int P,
                            const int32_t* __restrict__ item_cnt, int64_t* __restrict__ c_ptr) {
  const int64_t it = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (it >= nrows) return;
  int64_t t = 0;
  for (int p = 0; p < P; ++p) t += item_cnt[it * P + p];
  c_ptr[rows[it] + 1] = t;
}

// Kept-bitmap slots in list order (the heaviest rows first): flag[it + 1] =
// 1 for rows with at least min_flops products, then after an exclusive scan
// of the flags (flag[it] = eligible rows before it) a row takes slot flag[it]
// while slots are left.
__global__ void k_slot_flags(const int32_t* __restrict__ rows, int64_t nrows, const int64_t* __restrict__ flops,
                             int64_t min_flops, int64_t* __restrict__ flag) {
  const int64_t it = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (it < nrows) flag[it + 1] = flops[rows[it]] >= min_flops ? 1 : 0;
}
__global__ void k_slot_assign(const int32_t* __restrict__ rows, int64_t nrows, const int64_t* __restrict__ flops,
                              int64_t min_flops, const int64_t* __restrict__ pfx, int64_t capacity,
                              int32_t* __restrict__ row_slot) {
  const int64_t it = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (it >= nrows) return;
  const int32_t row = rows[it];
  const int64_t sl = pfx[it];
  row_slot[row] = (flops[row] >= min_flops && sl < capacity) ? static_cast<int32_t>(sl) : -1;
}

static unsigned grid_for(int64_t items, int64_t cap) {
  return static_cast<unsigned>(cap > 0 && items > cap ? cap : items);
}

hipError_t launch_hash_sym(const Operands& op, const int32_t* rows, int64_t nrows, int T, int nt,
                           int short_seg, int64_t* c_ptr, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_sym, dim3(grid_for(nrows, 0)), dim3(nt), hash_sym_lds(T, nt), s, op, rows,
                     nrows, T, short_seg, c_ptr);
  return hipGetLastError();
}

hipError_t launch_dense_sym(const Operands& op, const int32_t* rows, int64_t nrows, int wlog2, int P,
                            const int32_t* pidx, int nt, int short_seg, int64_t* c_ptr,
                            hipStream_t s, int sub_wlog2, int subP, int32_t* sub_cnt, KeepBitmaps kb) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_sym, dim3(grid_for(nrows, 0)), dim3(nt), dense_sym_lds(wlog2, nt), s, op,
                     rows, nrows, wlog2, P, pidx, short_seg, c_ptr, sub_wlog2, subP, sub_cnt, kb);
  return hipGetLastError();
}

hipError_t launch_keep_slots(const int32_t* rows, int64_t nrows, const int64_t* flops, int64_t min_flops,
                             int64_t capacity, int64_t* flag, int64_t* partials, int32_t* row_slot, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const unsigned nb = static_cast<unsigned>((nrows + 255) / 256);
  hipLaunchKernelGGL(k_slot_flags, dim3(nb), dim3(256), 0, s, rows, nrows, flops, min_flops, flag);
  hipError_t e = launch_scan_inplace(flag + 1, nrows, partials, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_slot_assign, dim3(nb), dim3(256), 0, s, rows, nrows, flops, min_flops, flag, capacity,
                     row_slot);
  return hipGetLastError();
}

hipError_t launch_dense_sym_win(const Operands& op, const int32_t* rows, int64_t nrows, int wlog2, int P,
                                const int32_t* pidx, int nt, int short_seg, int32_t* item_cnt,
                                unsigned int* queue, int64_t* c_ptr, int sub_wlog2, int subP, int32_t* sub_cnt,
                                const int32_t* keep_slot, uint32_t* keep_store, int64_t keep_nwords,
                                int wg_per_cu, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipError_t e = launch_fill_u64(reinterpret_cast<uint64_t*>(queue), (P + 1) / 2, 0, s);
  if (e != hipSuccess) return e;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t items = nrows * P;
  const int64_t grid = std::min<int64_t>(items, static_cast<int64_t>(ncu) * std::max(1, wg_per_cu));
  hipLaunchKernelGGL(k_dense_sym_win, dim3(static_cast<unsigned>(grid)), dim3(nt), dense_sym_lds(wlog2, nt), s,
                     op, rows, nrows, wlog2, P, pidx, short_seg, item_cnt, queue, sub_wlog2, subP, sub_cnt,
                     keep_slot, keep_store, keep_nwords);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_items, dim3(static_cast<unsigned>((nrows + 255) / 256)), dim3(256), 0, s, rows, nrows,
                     P, item_cnt, c_ptr);
  return hipGetLastError();
}

// n words from global memory (16-byte aligned) into LDS, with up to U
// 16-byte loads in flight per thread before any of them is stored.
template <int U>
__device__ __forceinline__ void load_words_lds(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                               int n) {
  const int nt = blockDim.x, tid = threadIdx.x;
  const int n4 = n >> 2;
  const uint4* s4 = reinterpret_cast<const uint4*>(src);
  uint4* d4 = reinterpret_cast<uint4*>(dst);
  for (int base = 0; base < n4; base += U * nt) {
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * nt + tid;
      if (i < n4) v[u] = s4[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * nt + tid;
      if (i < n4) d4[i] = v[u];
    }
  }
  for (int i = (n4 << 2) + tid; i < n; i += nt) dst[i] = src[i];
}

// The same copy without registers: each lane of a wave moves 16 bytes from
// global memory straight into LDS (global_load_lds_dwordx4: the LDS address
// is the wave's base, here dst + 16 bytes * the wave's first group, plus 16
// bytes per lane), so every load of the copy is in flight at once.  src and
// dst 16-byte aligned; returns after the copy has landed (the caller still
// synchronises the workgroup before other waves read dst).
__device__ __forceinline__ void load_words_lds_direct(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                                      int n) {
  const int nt = blockDim.x, tid = threadIdx.x, lane = tid & (kWave - 1);
  const int n4 = n >> 2;
  const uint4* s4 = reinterpret_cast<const uint4*>(src);
  uint4* d4 = reinterpret_cast<uint4*>(dst);
  for (int g = tid - lane; g < n4; g += nt) {  // g: the wave's first group, a multiple of 64
    const int i = g + lane;
    if (i < n4) __builtin_amdgcn_global_load_lds(s4 + i, d4 + g, 16, 0, 0);
  }
  for (int i = (n4 << 2) + tid; i < n; i += nt) dst[i] = src[i];
  __builtin_amdgcn_s_waitcnt(0);  // every counter at zero: the copies are in LDS
}

// Output entries are written once and not read again by the product:
// streaming stores keep them from displacing the operands in the caches.
// Used where a workgroup writes long contiguous runs (whole cache lines);
// short or scattered runs keep ordinary stores, which the L2 merges.
template <class T>
__device__ __forceinline__ void st_stream(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Orders the LDS accesses of one wave: writes by some lanes before the
// barrier are seen by reads of other lanes after it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Numeric phase of a pattern-only row whose bitmap the symbolic phase kept.
// The row is taken in slabs of nw * 64 * kExpandWords words.  In a slab each
// wave owns a contiguous range of at most 64 * kExpandWords words, read into
// registers (lane l has words l, l+64, ...) while the previous slab is being
// expanded; one block scan of the wave totals places the ranges.  Then, 64
// words at a time, the lanes put the column ids of their words in order into
// the wave's LDS staging area, at the same offset modulo 4 as their place in
// c_idx, and the wave writes the staged ids out with consecutive lanes on
// consecutive 16-byte groups (single ids at the unaligned ends).  Two-wave
// workgroups (17 KiB of LDS) keep many rows in flight on a CU, so that the
// load, scan and store steps of different rows overlap.
constexpr int kExpandWords = 16;
constexpr int kExpandThreads = 128;
constexpr int kExpandStage = kWave * 32 + 4;  // ids of 64 words, plus the alignment offset

__global__ __launch_bounds__(kExpandThreads) void k_expand_rows(const int32_t* __restrict__ rows, int64_t nrows,
                                                                int nwords, int64_t stride,
                                                                const uint32_t* __restrict__ store,
                                                                const int32_t* __restrict__ row_slot,
                                                                const int64_t* __restrict__ c_ptr,
                                                                int32_t* __restrict__ c_idx) {
  extern __shared__ __align__(16) unsigned char smem[];
  int* tmp = reinterpret_cast<int*>(smem);
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  int32_t* stage = reinterpret_cast<int32_t*>(smem + 256) + wid * kExpandStage;
  const int slab = nw * kWave * kExpandWords;
  // words of this wave in the slab starting at s0: [w_begin, w_end)
  auto range = [&](int s0, int& w_begin, int& w_end) {
    const int s1 = min(nwords, s0 + slab);
    const int wpw = (((s1 - s0 + nw - 1) / nw) + kWave - 1) & ~(kWave - 1);
    w_begin = min(s1, s0 + wid * wpw);
    w_end = min(s1, w_begin + wpw);
  };
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = uniform(rows[it]);
    const uint32_t* src = store + static_cast<int64_t>(row_slot[row]) * stride;
    const int64_t out_end = c_ptr[row + 1];
    int64_t o_slab = c_ptr[row];
    uint32_t wr[kExpandWords];
    {
      int wb, we;
      range(0, wb, we);
#pragma unroll
      for (int j = 0; j < kExpandWords; ++j) {
        const int w = wb + j * kWave + lane;
        wr[j] = w < we ? src[w] : 0u;
      }
    }
    for (int s0 = 0; s0 < nwords; s0 += slab) {
      int w_begin, w_end;
      range(s0, w_begin, w_end);
      int cnt = 0;
#pragma unroll
      for (int j = 0; j < kExpandWords; ++j) cnt += __popc(wr[j]);
      cnt = wave_sum(cnt);
      int ptotal;
      const int woff = __shfl(block_exclusive_scan(lane == 0 ? cnt : 0, tmp, &ptotal), 0, kWave);
      // the next slab's words, in flight while this one is expanded
      uint32_t wn[kExpandWords];
      {
        int wb = 0, we = 0;
        if (s0 + slab < nwords) range(s0 + slab, wb, we);
#pragma unroll
        for (int j = 0; j < kExpandWords; ++j) {
          const int w = wb + j * kWave + lane;
          wn[j] = w < we ? src[w] : 0u;
        }
      }
      int64_t o = o_slab + woff;
#pragma unroll
      for (int j = 0; j < kExpandWords; ++j) {
        if (w_begin + j * kWave < w_end) {  // wave-uniform
          const uint32_t word = wr[j];
          const int c = __popc(word);
          const int incl = wave_inclusive_scan(c);
          const int T = __shfl(incl, kWave - 1, kWave);
          // stage index a + t holds the id bound for c_idx[o + t]
          const int a = static_cast<int>((reinterpret_cast<uintptr_t>(c_idx + o) >> 2) & 3);
          int q = a + incl - c;
          uint32_t x = word;
          const int col0 = (w_begin + j * kWave + lane) << 5;
          while (x) {  // two ids per step
            const uint32_t y = x & (x - 1);
            stage[q] = col0 + __ffs(x) - 1;
            if (y) stage[q + 1] = col0 + __ffs(y) - 1;
            x = y & (y - 1);
            q += 2;
          }
          wave_sync();
          const int L = a + static_cast<int>(max<int64_t>(0, min<int64_t>(T, out_end - o)));
          const int vb = (a + 3) >> 2;                // first whole group of 4
          const int ve = max(vb, L >> 2);             // past the last whole group
          int32_t* dst = c_idx + o - a;               // 16-byte aligned
          if (lane < 4) {
            const int h = a + lane;                   // head: stage [a, min(4 vb, L))
            if (h < min(4 * vb, L)) dst[h] = stage[h];
            const int t = 4 * ve + lane;              // tail: stage [4 ve, L)
            if (t < L) dst[t] = stage[t];
          }
          for (int v = vb + lane; v < ve; v += kWave)
            reinterpret_cast<int4*>(dst)[v] = reinterpret_cast<const int4*>(stage)[v];
          wave_sync();
          o += T;
        }
      }
#pragma unroll
      for (int j = 0; j < kExpandWords; ++j) wr[j] = wn[j];
      o_slab += ptotal;
      __syncthreads();  // tmp is reused by the next scan
    }
  }
}

hipError_t launch_expand_rows(const int32_t* rows, int64_t nrows, int nwords, int64_t stride, const uint32_t* store,
                              const int32_t* row_slot, const int64_t* c_ptr, int32_t* c_idx, int nt,
                              hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  (void)nt;
  const size_t lds = 256 + static_cast<size_t>(kExpandThreads / kWave) * kExpandStage * sizeof(int32_t);
  hipLaunchKernelGGL(k_expand_rows, dim3(grid_for(nrows, 0)), dim3(kExpandThreads), lds, s, rows, nrows, nwords,
                     stride, store, row_slot, c_ptr, c_idx);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// (row, panel) pieces of heavy rows for the numeric phase.  Piece g of slot
// `slot` (the row's position in the dense symbolic list) and panel p is
// g = slot * subP + p; its entries go to c_ptr[row] + sub_off[g].
// ---------------------------------------------------------------------------
__host__ __device__ inline int sub_bin(int64_t cnt, const BinParams& bp) {
  if (cnt <= 0) return 0;
  if (cnt <= bp.hash_max_nnz) return hash_class(cnt);
  return dense_bin(cnt);
}

__global__ void k_sub_offsets(int64_t nslots, int subP, const int32_t* __restrict__ cnt,
                              int32_t* __restrict__ off) {
  const int64_t slot = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  int32_t run = 0;
  for (int p = 0; p < subP; ++p) {
    off[slot * subP + p] = run;
    run += cnt[slot * subP + p];
  }
}

// Group the column panels of each heavy row into windows: consecutive panels
// are merged while the window holds at most `cap` entries; a panel above cap
// is a window by itself (dense accumulator).  cnt becomes the window size at
// each window's first panel and 0 elsewhere; wend[g] is the window's end
// panel at its first panel.  The entry offsets (sub_off) do not change.
__global__ void k_sub_windows(int64_t nslots, int subP, int32_t cap, int32_t* __restrict__ cnt,
                              int32_t* __restrict__ wend) {
  const int64_t slot = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  int32_t* c = cnt + slot * subP;
  int32_t* e = wend + slot * subP;
  int p = 0;
  while (p < subP) {
    int32_t sum = c[p];
    int q = p + 1;
    if (sum <= cap) {
      while (q < subP && sum + c[q] <= cap) {
        sum += c[q];
        c[q] = 0;
        e[q] = q + 1;
        ++q;
      }
    }
    c[p] = sum;
    e[p] = q;
    p = q;
  }
}

__global__ void k_sub_count(int64_t nitems, const int32_t* __restrict__ cnt, BinParams bp,
                            unsigned long long* counts) {
  __shared__ unsigned int lc[kNumBins];
  const int tid = threadIdx.x;
  if (tid < kNumBins) lc[tid] = 0;
  __syncthreads();
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + tid;
  if (g < nitems) atomicAdd(&lc[sub_bin(cnt[g], bp)], 1u);
  __syncthreads();
  if (tid < kNumBins && lc[tid]) atomicAdd(&counts[tid], static_cast<unsigned long long>(lc[tid]));
}

__global__ void k_sub_scatter(int64_t nitems, const int32_t* __restrict__ cnt, BinParams bp,
                              BinOffsets offs, unsigned long long* cursors, int32_t* __restrict__ items) {
  __shared__ unsigned int lc[kNumBins];
  __shared__ unsigned long long lbase[kNumBins];
  const int tid = threadIdx.x;
  if (tid < kNumBins) lc[tid] = 0;
  __syncthreads();
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + tid;
  int bin = 0;
  unsigned int local = 0;
  if (g < nitems) {
    bin = sub_bin(cnt[g], bp);
    if (bin > 0) local = atomicAdd(&lc[bin], 1u);
  }
  __syncthreads();
  if (tid < kNumBins && lc[tid])
    lbase[tid] = atomicAdd(&cursors[tid], static_cast<unsigned long long>(lc[tid]));
  __syncthreads();
  if (bin > 0) items[offs.v[bin] + static_cast<int64_t>(lbase[bin]) + local] = static_cast<int32_t>(g);
}

hipError_t launch_sub_prepare(int64_t nslots, int subP, int32_t* cnt, int32_t* off, int32_t* wend,
                              BinParams bp, unsigned long long* counts, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  const int64_t nitems = nslots * subP;
  hipLaunchKernelGGL(k_sub_offsets, dim3(static_cast<unsigned>((nslots + 255) / 256)), dim3(256), 0, s,
                     nslots, subP, cnt, off);
  hipLaunchKernelGGL(k_sub_windows, dim3(static_cast<unsigned>((nslots + 255) / 256)), dim3(256), 0, s,
                     nslots, subP, static_cast<int32_t>(bp.hash_max_nnz), cnt, wend);
  hipLaunchKernelGGL(k_sub_count, dim3(static_cast<unsigned>((nitems + 255) / 256)), dim3(256), 0, s,
                     nitems, cnt, bp, counts);
  return hipGetLastError();
}

hipError_t launch_sub_scatter(int64_t nslots, int subP, const int32_t* cnt, BinParams bp,
                              const BinOffsets& offs, unsigned long long* cursors, int32_t* items,
                              hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  const int64_t nitems = nslots * subP;
  hipLaunchKernelGGL(k_sub_scatter, dim3(static_cast<unsigned>((nitems + 255) / 256)), dim3(256), 0, s,
                     nitems, cnt, bp, offs, cursors, items);
  return hipGetLastError();
}

hipError_t launch_hash_sym_b(const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                             const int32_t* items, int64_t nitems, int T, int nt, int short_seg,
                             hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_sym_b, dim3(grid_for(nitems, 0)), dim3(nt), hash_sym_lds(T, nt), s,
                     descs, row_off, prod_of, nprod, items, nitems, T, short_seg);
  return hipGetLastError();
}

hipError_t launch_dense_sym_b(const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                              const int32_t* items, int64_t nitems, int wlog2_max, int nt,
                              int short_seg, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_sym_b, dim3(grid_for(nitems, 0)), dim3(nt),
                     dense_sym_lds(wlog2_max, nt), s, descs, row_off, prod_of, nprod, items, nitems, short_seg);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Numeric phase (paper Sec. 4.1 phase 3).
// ---------------------------------------------------------------------------
template <class S>
__device__ void bitonic_sort(int32_t* keys, S* vals, int N, bool with_vals) {
  // Wave w takes the M pairs [w*M, (w+1)*M) of every stage (M a power of two,
  // at least a wave's width).  A stage with distance j <= M then pairs
  // elements inside the wave's own 2M elements, so only stages with j > M,
  // and the stages next to them, need a workgroup barrier; the others are
  // ordered within the wave.
  const int lane = threadIdx.x & (kWave - 1);
  const int nw = blockDim.x >> 6;
  const int half = N >> 1;
  int M = kWave;
  while (M * nw < half) M <<= 1;
  const int p0 = (threadIdx.x >> 6) * M;
  const int p1 = min(p0 + M, half);
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int p = p0 + lane; p < p1; p += kWave) {
        const int i = 2 * p - (p & (j - 1));
        const int l = i + j;
        const bool up = (i & k) == 0;
        const int32_t ki = keys[i], kl = keys[l];
        if ((ki > kl) == up) {
          keys[i] = kl;
          keys[l] = ki;
          if (with_vals) {
            const S vi = vals[i];
            vals[i] = vals[l];
            vals[l] = vi;
          }
        }
      }
      const int next_j = j > 1 ? j >> 1 : k;  // first distance of the next stage
      if (j > M || (next_j > M && k < N))
        __syncthreads();
      else
        wave_sync();
    }
  }
  __syncthreads();
}

constexpr int kMaxSlotsPerThread = 16;

// LDS hash accumulator for one row, then compaction, bitonic sort and
// coalesced stores of the row's entries into [out, out_end).
template <class SR, bool kFlat = false, class Src>
__device__ void hash_num_src(const Operands& op, const Src& src, int32_t c0, int T, int short_seg,
                             int64_t out, int64_t out_end, int32_t* __restrict__ c_idx,
                             typename SR::Out* __restrict__ c_val, unsigned char* smem) {
  using S = typename SR::S;
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  auto q = RowQueue<typename SR::In>::carve(smem, nt);
  int32_t* keys = reinterpret_cast<int32_t*>(smem + RowQueue<typename SR::In>::bytes(nt));
  S* vals = reinterpret_cast<S*>(keys + T);
  for (int t = tid; t < T; t += nt) {
    keys[t] = kEmpty;
    if constexpr (!SR::kPattern) vals[t] = SR::identity();
  }
  __syncthreads();
  HashMapSink<SR> sink{keys, vals, static_cast<uint32_t>(T - 1)};
  enumerate_src<SR, 1, kFlat>(op, src, c0, short_seg, q, sink);
  // Compact occupied slots to the front: every thread takes T/nt slots
  // (strided by nt, so reads are free of bank conflicts) into registers, then
  // writes them at its scanned offset.  The order does not matter: a sort
  // follows.
  constexpr int kMaxSlots = sizeof(S) > 4 ? kMaxSlotsPerThread / 2 : kMaxSlotsPerThread;
  const int per = T / nt;
  int32_t kr[kMaxSlots];
  S vr[kMaxSlots];
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < kMaxSlots; ++r) {
    kr[r] = kEmpty;
    if (r < per) {
      const int slot = r * nt + tid;
      kr[r] = keys[slot];
      if constexpr (!SR::kPattern) vr[r] = vals[slot];
      cnt += kr[r] != kEmpty;
    }
  }
  int nnz;
  int o = block_exclusive_scan(cnt, q.ctr + 2, &nnz);
#pragma unroll
  for (int r = 0; r < kMaxSlots; ++r) {
    if (r < per && kr[r] != kEmpty) {
      keys[o] = kr[r];
      if constexpr (!SR::kPattern) vals[o] = vr[r];
      ++o;
    }
  }
  int N = 1;
  while (N < nnz) N <<= 1;
  for (int t = nnz + tid; t < N; t += nt) keys[t] = INT32_MAX;
  __syncthreads();
  bitonic_sort<S>(keys, vals, N, !SR::kPattern);
  // The symbolic count and this one agree; the clamp keeps writes inside the
  // row's range of C regardless.
  const int lim = static_cast<int>(min(static_cast<int64_t>(nnz), out_end - out));
  for (int e = tid; e < lim; e += nt) {
    c_idx[out + e] = keys[e] + c0;
    if constexpr (!SR::kPattern) c_val[out + e] = SR::out(vals[e]);
  }
  __syncthreads();
}

template <class SR, bool kFlat = false>
__device__ void hash_num_row(const Operands& op, int32_t row, int T, int short_seg, int64_t out,
                             int64_t out_end, int32_t* __restrict__ c_idx,
                             typename SR::Out* __restrict__ c_val, unsigned char* smem,
                             bool paneled = false, const int32_t* __restrict__ pidx = nullptr, int P = 1,
                             int p = 0, int32_t c0 = 0, int p_hi = 0) {
  RowSource<SR> src{&op, op.a_ptr[row], op.a_ptr[row + 1], paneled, pidx, P, p, p_hi};
  hash_num_src<SR, kFlat>(op, src, c0, T, short_seg, out, out_end, c_idx, c_val, smem);
}

// Dense LDS panel accumulator for one row: presence bits plus one value per
// column of the panel, emitted in column order into [out, out_end).
template <class SR, int kBufs = 1, class MakeSrc>
__device__ void dense_num_gen(const Operands& op, int wlog2, int p_begin, int p_end, int short_seg,
                              int64_t out, int64_t out_end, int32_t* __restrict__ c_idx,
                              typename SR::Out* __restrict__ c_val, unsigned char* smem,
                              const MakeSrc& make) {
  using S = typename SR::S;
  using Q = RowQueue<typename SR::In>;
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid >> 6;
  const int nw = nt >> 6;
  const int W = 1 << wlog2;
  auto q = Q::carve(smem, nt);
  unsigned char* p0 = smem + Q::bytes(nt);
  uint32_t* bits = reinterpret_cast<uint32_t*>(p0);
  S* vals = reinterpret_cast<S*>(p0 + static_cast<size_t>(W) / 8);
  const int32_t wcols_max = min(W, op.k);
  for (int t = tid; t < (wcols_max + 31) >> 5; t += nt) bits[t] = 0u;
  if constexpr (!SR::kPattern) {
    for (int t = tid; t < wcols_max; t += nt) vals[t] = SR::identity();
  }
  __syncthreads();
  for (int p = p_begin; p < p_end; ++p) {
    const int32_t c0 = p << wlog2;
    const int32_t wcols = min(W, op.k - c0);
    const int nwords = (wcols + 31) >> 5;
    DenseSink<SR> sink{bits, vals};
    enumerate_src<SR, kBufs>(op, make(p), c0, short_seg, q, sink);
    // Emit the panel in column order.  Wave w owns a contiguous range of
    // words; one block scan of the wave totals places the ranges, then each
    // wave walks its range 64 words at a time with no further barriers.
    // Lane l writes the entries of its own word at consecutive slots, and
    // resets what it read for the next panel.
    const int wpw = (((nwords + nw - 1) / nw) + kWave - 1) & ~(kWave - 1);
    const int w_begin = min(nwords, wid * wpw);
    const int w_end = min(nwords, w_begin + wpw);
    int cnt = 0;
    for (int w = w_begin + lane; w < w_end; w += kWave) cnt += __popc(bits[w]);
    cnt = wave_sum(cnt);
    int ptotal;
    const int woff = __shfl(block_exclusive_scan(lane == 0 ? cnt : 0, q.ctr + 2, &ptotal), 0, kWave);
    int64_t o_base = out + woff;
    for (int w0 = w_begin; w0 < w_end; w0 += kWave) {
      const int w = w0 + lane;
      const uint32_t word = w < w_end ? bits[w] : 0u;
      const int c = __popc(word);
      const int incl = wave_inclusive_scan(c);
      int64_t o = o_base + (incl - c);
      uint32_t x = word;
      while (x) {
        const int b = __ffs(x) - 1;
        const int col = (w << 5) + b;
        if (o < out_end) {
          c_idx[o] = c0 + col;
          if constexpr (!SR::kPattern) c_val[o] = SR::out(vals[col]);
        }
        if constexpr (!SR::kPattern) vals[col] = SR::identity();
        x &= x - 1;
        ++o;
      }
      if (word) bits[w] = 0u;
      o_base += __shfl(incl, kWave - 1, kWave);
    }
    out += ptotal;
    __syncthreads();
  }
}

template <class SR, int kBufs = 1>
__device__ void dense_num_row(const Operands& op, int32_t row, int wlog2, int P,
                              const int32_t* __restrict__ pidx, int short_seg, int64_t out,
                              int64_t out_end, int32_t* __restrict__ c_idx,
                              typename SR::Out* __restrict__ c_val, unsigned char* smem,
                              int p_begin = 0, int p_end = -1) {
  const int64_t a_lo = op.a_ptr[row], a_hi = op.a_ptr[row + 1];
  if (p_end < 0) p_end = P;
  if (P > 1 && a_hi - a_lo <= blockDim.x && p_end - p_begin > 1) {
    CachedRowSource<SR> cs{a_hi - a_lo, 0, typename SR::In(1), 0, 0, 0};
    const int32_t* sp = nullptr;
    const int tid = threadIdx.x;
    if (tid < a_hi - a_lo) {
      const int32_t kk = op.a_idx[a_lo + tid];
      cs.a = load_val<SR>(op.a_val, a_lo + tid);
      cs.bs = op.b_ptr[kk];
      sp = pidx + static_cast<int64_t>(kk) * (P + 1);
      cs.s_cur = sp[p_begin];
      cs.s_nxt = sp[p_begin + 1];
      cs.s_nxt2 = sp[min(p_begin + 2, P)];
    }
    auto make = [&](int p) {
      if (p > p_begin) {
        cs.s_cur = cs.s_nxt;
        cs.s_nxt = cs.s_nxt2;
        if (sp) cs.s_nxt2 = sp[min(p + 2, P)];  // consumed at the next panel
      }
      return cs;
    };
    dense_num_gen<SR, kBufs>(op, wlog2, p_begin, p_end, short_seg, out, out_end, c_idx, c_val, smem, make);
    return;
  }
  auto make = [&](int p) { return RowSource<SR>{&op, a_lo, a_hi, P > 1, pidx, P, p, p + 1}; };
  dense_num_gen<SR, kBufs>(op, wlog2, p_begin, p_end, short_seg, out, out_end, c_idx, c_val, smem, make);
}

template <class SR>
__global__ __launch_bounds__(1024) void k_hash_num(Operands op, const int32_t* __restrict__ rows,
                                                   int64_t nrows, int T, int short_seg,
                                                   const int64_t* __restrict__ c_ptr,
                                                   int32_t* __restrict__ c_idx,
                                                   typename SR::Out* __restrict__ c_val) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = uniform(rows[it]);
    hash_num_row<SR, true>(op, row, T, short_seg, c_ptr[row], c_ptr[row + 1], c_idx, c_val, smem);
  }
}

// Sort of n <= R * blockDim.x (key, value) pairs in LDS by key
// (keys >= 0), by buckets of the row's own key range: every pair goes to one
// of blockDim.x buckets by a monotone function of its key (so the buckets
// are in key order), the buckets are laid out by a scan of their counts, and
// every pair then finds its place inside its bucket by counting the smaller
// keys there (equal keys by bucket position).  Buckets hold a few pairs each
// when the keys are spread over their range; the cost per pair is that
// bucket's size.  cnt: blockDim.x + 1 ints of LDS; red: 32 ints of LDS (scan
// scratch).  keys/vals hold the pairs on entry (after a barrier) and, sorted,
// on exit (after a barrier).
template <class S, bool kVals, int R>
__device__ void bucket_sort(int32_t* keys, S* vals, int n, int* cnt, int* red) {
  const int nt = blockDim.x, tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid >> 6;
  const int e0 = R * tid;
  int32_t k[R];
  S v[R];
  int kmin = INT32_MAX, kmax = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    k[r] = 0;
    if (e0 + r < n) {
      k[r] = keys[e0 + r];
      if constexpr (kVals) v[r] = vals[e0 + r];
      kmin = min(kmin, k[r]);
      kmax = max(kmax, k[r]);
    }
  }
  // the key range of the pairs
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    kmin = min(kmin, __shfl_xor(kmin, d, kWave));
    kmax = max(kmax, __shfl_xor(kmax, d, kWave));
  }
  if (lane == 0) {
    red[wid] = kmin;
    red[16 + wid] = kmax;
  }
  cnt[tid] = 0;
  __syncthreads();
  const int nw = nt >> 6;
  for (int w = 0; w < nw; ++w) {
    kmin = min(kmin, red[w]);
    kmax = max(kmax, red[16 + w]);
  }
  // bucket and position in it: (key - kmin) * scale is non-decreasing in the key
  const float scale = static_cast<float>(nt) / (static_cast<float>(kmax - kmin) + 1.0f);
  int g[R], p[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    g[r] = 0;
    p[r] = 0;
    if (e0 + r < n) {
      g[r] = min(nt - 1, static_cast<int>(static_cast<float>(k[r] - kmin) * scale));
      p[r] = atomicAdd(&cnt[g[r]], 1);
    }
  }
  __syncthreads();
  int total;
  const int start = block_exclusive_scan(cnt[tid], red, &total);  // ends with a barrier
  cnt[tid] = start;
  if (tid == 0) cnt[nt] = n;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (e0 + r < n) {
      const int d = cnt[g[r]] + p[r];
      keys[d] = k[r];
      if constexpr (kVals) vals[d] = v[r];
    }
  __syncthreads();
  int dst[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    dst[r] = 0;
    if (e0 + r < n) {
      const int b0 = cnt[g[r]], b1 = cnt[g[r] + 1], me = b0 + p[r];
      int rank = 0;
      for (int i = b0; i < b1; ++i) {
        const int32_t ki = keys[i];
        rank += (ki < k[r] || (ki == k[r] && i < me)) ? 1 : 0;
      }
      dst[r] = b0 + rank;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (e0 + r < n) {
      keys[dst[r]] = k[r];
      if constexpr (kVals) vals[dst[r]] = v[r];
    }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Expand-sort-compress (ESC) numeric rows: for a row whose products are
// almost all distinct entries (flops close to nnz, the low compression ratio
// for which the paper's hybrid picks a heap over a hash table, Sec. 4.1),
// every product is written to its own LDS position (product j to position j,
// consecutive products to consecutive positions: no hashing, no atomics),
// the (column, value) pairs are sorted by column (bucket_sort), and runs of
// one column are combined.  Products are dealt flat: product j
// of a block of A entries goes to thread j mod blockDim, its B row found by a
// binary search over the block's prefix of B-row lengths.
// ---------------------------------------------------------------------------
constexpr int kEscUnroll = 4;      // products per thread per batch of loads



template <class SR>
__host__ __device__ inline size_t esc_lds_bytes(int N, int nt) {
  return RowQueue<typename SR::In>::bytes(nt) + static_cast<size_t>(N) * (4 + sizeof(typename SR::S));
}

// R: products per thread (4 or 8); with 4 the kernel keeps its registers
// within what two 1024-thread workgroups per compute unit allow (4-byte
// values); the 8192-product class takes most of the LDS anyway.
// One row of at most N products into C's entries [out, out_end).
template <class SR, int R>
__device__ void esc_num_row(const Operands& op, int32_t row, int N, int64_t out, int64_t out_end,
                            int32_t* __restrict__ c_idx, typename SR::Out* __restrict__ c_val,
                            unsigned char* smem) {
  using S = typename SR::S;
  using In = typename SR::In;
  const int nt = blockDim.x, tid = threadIdx.x;
  auto q = RowQueue<In>::carve(smem, nt);
  int32_t* keys = reinterpret_cast<int32_t*>(smem + RowQueue<In>::bytes(nt));
  S* vals = reinterpret_cast<S*>(keys + N);
  const int64_t a_lo = op.a_ptr[row], a_hi = op.a_ptr[row + 1];
  // 1. expand
  int base = 0;
  for (int64_t r0 = a_lo; r0 < a_hi; r0 += nt) {
    int64_t lo = 0;
    int32_t len = 0;
    In a = In(1);
    if (r0 + tid < a_hi) {
      const int32_t kk = op.a_idx[r0 + tid];
      a = load_val<SR>(op.a_val, r0 + tid);
      lo = op.b_ptr[kk];
      len = static_cast<int32_t>(op.b_ptr[kk + 1] - lo);
    }
    int E;
    const int off = block_exclusive_scan(len, q.ctr + 2, &E);
    q.lo[tid] = lo;
    q.a[tid] = a;
    q.pfx[tid] = off;  // threads past the row's entries have len 0
    if (tid == 0) q.pfx[nt] = E;
    __syncthreads();
    E = min(E, N - base);  // the class bound holds the row's products; never write past it
    // entries past the block's last one have pfx == E: the search stops there
    const int nents = static_cast<int>(min(static_cast<int64_t>(nt), a_hi - r0));
    for (int j0 = 0; j0 < E; j0 += kEscUnroll * nt) {
      int es[kEscUnroll];
#pragma unroll
      for (int u = 0; u < kEscUnroll; ++u) {
        const int j = j0 + u * nt + tid;
        int e_lo = -1;
        if (j < E) {
          e_lo = 0;
          int e_hi = nents;
          while (e_hi - e_lo > 1) {
            const int mid = (e_lo + e_hi) >> 1;
            if (q.pfx[mid] <= j)
              e_lo = mid;
            else
              e_hi = mid;
          }
        }
        es[u] = e_lo;
      }
      int32_t cols[kEscUnroll];
      In bv[kEscUnroll];
#pragma unroll
      for (int u = 0; u < kEscUnroll; ++u)
        if (es[u] >= 0) load_b<SR>(op, q.lo[es[u]] + (j0 + u * nt + tid - q.pfx[es[u]]), cols[u], bv[u]);
#pragma unroll
      for (int u = 0; u < kEscUnroll; ++u)
        if (es[u] >= 0) {
          const int j = base + j0 + u * nt + tid;
          keys[j] = cols[u];
          if constexpr (!SR::kPattern) vals[j] = SR::mul(q.a[es[u]], bv[u]);
        }
    }
    base += E;
    __syncthreads();  // the queue arrays are rewritten by the next block of entries
  }
  __syncthreads();
  // 2. sort by column (the class bound N is at most R * nt)
  bucket_sort<S, !SR::kPattern, R>(keys, vals, base, q.pfx, q.ctr + 2);
  // 3. compress: each thread a contiguous run of positions; the first
  //    entry of every column keeps its place in the output, the others are
  //    combined into it (few: the rows here have almost no repeats)
  const int ch = (base + nt - 1) / nt;
  const int e0 = min(base, tid * ch), e1 = min(base, e0 + ch);
  int32_t kr[R];
  S vr[R];
  bool head[R];
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = e0 + r;
    head[r] = false;
    if (e < e1) {
      kr[r] = keys[e];
      if constexpr (!SR::kPattern) vr[r] = vals[e];
      head[r] = e == 0 || keys[e - 1] != kr[r];
      cnt += head[r] ? 1 : 0;
    }
  }
  int nnz;
  int pos = block_exclusive_scan(cnt, q.ctr + 2, &nnz);  // ends with a barrier: keys may be rewritten
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (e0 + r < e1 && head[r]) {
      keys[pos] = kr[r];
      if constexpr (!SR::kPattern) vals[pos] = vr[r];
      ++pos;
    }
  }
  __syncthreads();
  if constexpr (!SR::kPattern) {
    pos = block_exclusive_scan(cnt, q.ctr + 2, &nnz);  // first head position of this thread's run
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (e0 + r < e1) {
        if (head[r])
          ++pos;
        else
          SR::combine(&vals[pos - 1], vr[r]);  // the column's first entry is at pos - 1
      }
    }
    __syncthreads();
  }
  // the symbolic count and this one agree; the clamp keeps writes inside the row
  const int lim = static_cast<int>(min(static_cast<int64_t>(nnz), out_end - out));
  for (int e = tid; e < lim; e += nt) {
    c_idx[out + e] = keys[e];
    if constexpr (!SR::kPattern) c_val[out + e] = SR::out(vals[e]);
  }
  __syncthreads();
}

template <class SR, int R>
__global__ __launch_bounds__(1024, R > 4 ? 4 : (sizeof(typename SR::S) > 4 ? 6 : 8)) void k_esc_num(
    Operands op, const int32_t* __restrict__ rows, int64_t nrows, int N, const int64_t* __restrict__ c_ptr,
    int32_t* __restrict__ c_idx, typename SR::Out* __restrict__ c_val) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = uniform(rows[it]);
    esc_num_row<SR, R>(op, row, N, c_ptr[row], c_ptr[row + 1], c_idx, c_val, smem);
  }
}

// The same over the rows of many products (global row ids in items).
template <class SR, int R>
__global__ __launch_bounds__(1024, R > 4 ? 4 : (sizeof(typename SR::S) > 4 ? 6 : 8)) void k_esc_num_b(
    const BatchDesc* __restrict__ descs, const int64_t* __restrict__ row_off,
    const int32_t* __restrict__ prod_of, int nprod,
    const int32_t* __restrict__ items, int64_t nitems, int N) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t r = uniform(items[it]);
    const int b = uniform(prod_of[r]);
    const BatchDesc d = descs[b];  // uniform: held in scalar registers
    const int32_t row = uniform(static_cast<int32_t>(r - row_off[b]));
    esc_num_row<SR, R>(d.op, row, N, d.c_ptr[row], d.c_ptr[row + 1], d.c_idx,
                       static_cast<typename SR::Out*>(d.c_val), smem);
  }
}

template <class SR>
__global__ __launch_bounds__(1024) void k_dense_num(Operands op, const int32_t* __restrict__ rows,
                                                    int64_t nrows, int wlog2, int P,
                                                    const int32_t* __restrict__ pidx, int short_seg,
                                                    const int64_t* __restrict__ c_ptr,
                                                    int32_t* __restrict__ c_idx,
                                                    typename SR::Out* __restrict__ c_val) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = uniform(rows[it]);
    dense_num_row<SR, 2>(op, row, wlog2, P, pidx, short_seg, c_ptr[row], c_ptr[row + 1], c_idx, c_val,
                      smem);
  }
}

// ---------------------------------------------------------------------------
// Rank-compressed panels for heavy valued rows.
//
// A fixed-width value panel spends one LDS slot per column, so a row whose
// entries are spread thinly over many columns needs a pass per panel even
// when each panel holds few entries.  Here the symbolic phase has counted the
// row's entries per chunk of 2^cw columns.  A pass takes the longest run of
// chunks whose entries fit the 2^cw value slots (and whose columns fit the LDS
// bitmap), marks the pattern of that column range in a bitmap, takes a prefix
// count per bitmap word, and then combines every product into the slot given
// by its column's rank in the range.  The slots are then in column order: the
// values are written out as they stand, the column ids from the bitmap.
// Rows dense enough that fixed panels need fewer passes use fixed panels over
// the same chunk index.
// ---------------------------------------------------------------------------
// The bitmap is read in 64-bit words, each with the rank of its first bit.
template <class SR>
struct RankSink {
  using S = typename SR::S;
  const uint64_t* bits;
  const uint16_t* pre;
  S* vals;
  __device__ void add(int32_t c, S v) {
    const int w = c >> 6;
    const uint64_t below = bits[w] & ((1ull << (c & 63)) - 1ull);
    SR::combine(&vals[pre[w] + __popcll(below)], v);
  }
};

template <class SR>
__host__ __device__ inline size_t rank_queue_bytes(int nt) {
  const size_t a = RowQueue<typename SR::In>::bytes(nt);
  const size_t b = RowQueue<SrPattern::In>::bytes(nt);
  return a > b ? a : b;
}

template <class SR>
__host__ __device__ inline size_t rank_num_lds_bytes(int cw, int slots, int max_chunks, int nt) {
  const size_t cols = static_cast<size_t>(max_chunks) << cw;  // a multiple of 64 (cw >= 6)
  return rank_queue_bytes<SR>(nt) + sizeof(typename SR::S) * static_cast<size_t>(slots) + cols / 8 + (cols / 64) * 2;
}

// cv: when NC <= 64, lane c of every wave holds the row's chunk count c
// (with one-word B entries the passes are planned from these registers);
// every chunk holds at most `slots` entries (the caller picks only such
// shapes).
template <class SR>
__device__ void rank_num_row(const Operands& op, int64_t a_lo, int64_t a_hi, int cw, int slots, int NC,
                             int max_chunks, const int32_t* __restrict__ pchunk,
                             const int32_t* __restrict__ cnt, int cv, const uint32_t* __restrict__ keep,
                             int short_seg, int64_t out, int64_t out_end,
                             int32_t* __restrict__ c_idx, typename SR::Out* __restrict__ c_val,
                             unsigned char* smem, int* info) {
  using S = typename SR::S;
  using In = typename SR::In;
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  auto q = RowQueue<In>::carve(smem, nt);
  auto pq = RowQueue<SrPattern::In>::carve(smem, nt);  // same LDS, used by the pattern walk
  unsigned char* p0 = smem + rank_queue_bytes<SR>(nt);
  S* vals = reinterpret_cast<S*>(p0);
  uint32_t* bits = reinterpret_cast<uint32_t*>(p0 + sizeof(S) * static_cast<size_t>(slots));
  uint16_t* pre = reinterpret_cast<uint16_t*>(bits + (static_cast<size_t>(max_chunks) << (cw - 5)));
  // This thread's entry of the row's first round, kept across the passes:
  // each pass then loads only its two chunk offsets, issued with the
  // bitmap loads.  Only one-word B entries leave the registers for it; the
  // other forms load the round in each pass.
  constexpr bool kCache = IsPackedB<SR>::value;
  const bool mine = kCache && tid < a_hi - a_lo;
  int32_t kk0 = 0;
  In a0 = In(1);
  int64_t bs0 = 0;
  if (mine) {
    kk0 = op.a_idx[a_lo + tid];
    a0 = load_val<SR>(op.a_val, a_lo + tid);
    bs0 = op.b_ptr[kk0];
  }
  for (int c_lo = 0; c_lo < NC;) {
    if (tid < kWave) {
      // The pass: the longest run of at most max_chunks chunks from c_lo whose
      // entries fit the slots (at least one: no chunk holds more).
      const int c = c_lo + lane;
      const bool in = lane < max_chunks && c < NC;
      int v = 0;
      if constexpr (kCache) {
        const int vr = __shfl(cv, c & (kWave - 1), kWave);
        v = in ? (NC <= kWave ? vr : cnt[c]) : 0;
      } else {
        v = in ? cnt[c] : 0;
      }
      const int incl = wave_inclusive_scan(v);
      const unsigned long long fit = __ballot(in && incl <= slots);
      const int n = __popcll(fit);
      const int tot = __shfl(incl, n - 1, kWave);
      if (lane == 0) {
        info[0] = n;
        info[1] = tot;
      }
    }
    __syncthreads();
    const int n = info[0];
    const int total = info[1];
    __syncthreads();  // info is rewritten by the next pass
    const int c_hi = c_lo + n;
    if (total > 0) {
      const int32_t C0 = c_lo << cw;
      const int32_t wcols = min(n << cw, op.k - C0);
      const int nwords = (wcols + 31) >> 5;
      const int nw64 = (nwords + 1) >> 1;
      const uint64_t* bits64 = reinterpret_cast<const uint64_t*>(bits);
      // this thread's first-round segment in the range, loaded with the bitmap
      int32_t s0 = 0, s1 = 0;
      if (mine) {
        const int32_t* prow = pchunk + static_cast<int64_t>(kk0) * (NC + 1);
        s0 = prow[c_lo];
        s1 = prow[c_hi];
      }
      for (int t = tid; t < total; t += nt) vals[t] = SR::identity();
      // 1. pattern of the column range: from the kept bitmap, or by a walk
      //    over B's column ids; an odd word count gets a zero word after it
      if (keep) {
        if constexpr (kCache)
          load_words_lds_direct(bits, keep + (C0 >> 5), nwords);
        else
          load_words_lds<1>(bits, keep + (C0 >> 5), nwords);
        if ((nwords & 1) && tid == 0) bits[nwords] = 0u;
        __syncthreads();
      } else {
        for (int t = tid; t < 2 * nw64; t += nt) bits[t] = 0u;
        __syncthreads();
        BitmapSink bs{bits};
        const RowSource<SrPattern> rp{&op, a_lo, a_hi, true, pchunk, NC, c_lo, c_hi};
        if constexpr (kCache) {
          const PassSource<SrPattern> ps{rp, bs0 + s0, s1 - s0, SrPattern::In(1)};
          enumerate_src<SrPattern, 2>(op, ps, C0, short_seg, pq, bs);
        } else {
          enumerate_src<SrPattern, 2>(op, rp, C0, short_seg, pq, bs);
        }
      }
      // 2. rank of the first entry of every 64-bit word (contiguous words per thread)
      const int wpt = (nw64 + nt - 1) / nt;
      const int w0 = min(nw64, tid * wpt), w1 = min(nw64, w0 + wpt);
      int local = 0;
      for (int w = w0; w < w1; ++w) local += __popcll(bits64[w]);
      int ptotal;
      int run = block_exclusive_scan(local, q.ctr + 2, &ptotal);
      for (int w = w0; w < w1; ++w) {
        pre[w] = static_cast<uint16_t>(run);
        run += __popcll(bits64[w]);
      }
      __syncthreads();
      // 3. values, combined at their ranks
      RankSink<SR> rs{bits64, pre, vals};
      const RowSource<SR> rv{&op, a_lo, a_hi, true, pchunk, NC, c_lo, c_hi};
      if constexpr (kCache) {
        const PassSource<SR> vs{rv, bs0 + s0, s1 - s0, a0};
        enumerate_src<SR, 2>(op, vs, C0, short_seg, q, rs);
      } else {
        enumerate_src<SR, 2>(op, rv, C0, short_seg, q, rs);
      }
      // 4. write the range out: the values in slot order; then the column
      //    ids, placed at their ranks in LDS (over the value slots, 4 bytes
      //    each at most as wide as a slot) and written in order
      static_assert(sizeof(S) >= sizeof(int32_t), "ids are staged over the value slots");
      const int lim = static_cast<int>(min(static_cast<int64_t>(total), out_end - out));
      for (int r = tid; r < lim; r += nt) st_stream(&c_val[out + r], SR::out(vals[r]));
      __syncthreads();
      int32_t* ids = reinterpret_cast<int32_t*>(vals);
      for (int w = tid; w < nw64; w += nt) {
        uint64_t x = bits64[w];
        int q = pre[w];
        const int32_t col0 = C0 + (w << 6);
        while (x) {
          ids[q++] = col0 + __ffsll(static_cast<unsigned long long>(x)) - 1;
          x &= x - 1;
        }
      }
      __syncthreads();
      for (int r = tid; r < lim; r += nt) st_stream(&c_idx[out + r], ids[r]);
      out += total;
      __syncthreads();
    }
    c_lo = c_hi;
  }
}

// Heavy valued rows of the dense symbolic list (slot order), those with more
// than hash_max_nnz entries; the others went to the hash numeric bins.
template <class SR, bool kFixed>
__global__ __launch_bounds__(1024) void k_rank_num(Operands op, const int32_t* __restrict__ rows,
                                                   int64_t nrows, int32_t rb, int32_t re, int cw, int NC,
                                                   RankShapes sh,
                                                   const int32_t* __restrict__ pchunk,
                                                   const int32_t* __restrict__ rcnt, int64_t nnz_lo,
                                                   int64_t nnz_hi, int wlog2, int P, int short_seg,
                                                   const uint32_t* __restrict__ keep_store,
                                                   const int32_t* __restrict__ keep_slot, int64_t keep_nwords,
                                                   const int64_t* __restrict__ c_ptr,
                                                   int32_t* __restrict__ c_idx,
                                                   typename SR::Out* __restrict__ c_val) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int info[2];
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = uniform(rows[it]);
    if (row < rb || row >= re) continue;  // another range of rows
    const int64_t out = uniform64(c_ptr[row]), out_end = uniform64(c_ptr[row + 1]);
    const int64_t nnz = out_end - out;
    if (nnz < nnz_lo || nnz >= nnz_hi) continue;  // another launch takes this row
    if (sh.esc_max_flops > 0 && esc_row(nnz, sh.flops[row], sh.esc_max_flops, sh.esc_ratio_x16))
      continue;  // expanded, sorted and compressed instead
    const int64_t a_lo = op.a_ptr[row], a_hi = op.a_ptr[row + 1];
    if constexpr (kFixed) {
      // fixed panels of 2^wlog2 columns = 2^(wlog2-cw) chunks
      const int r = 1 << (wlog2 - cw);
      auto make = [&](int p) {
        return RowSource<SR>{&op, a_lo, a_hi, true, pchunk, NC, p * r, min((p + 1) * r, NC)};
      };
      dense_num_gen<SR, 2>(op, wlog2, 0, P, short_seg, out, out_end, c_idx, c_val, smem, make);
    } else {
      const int32_t slot = keep_slot ? uniform(keep_slot[row]) : -1;
      const uint32_t* keep = slot >= 0 ? keep_store + static_cast<int64_t>(slot) * keep_nwords : nullptr;
      // the row's chunk counts (with one-word B entries: in registers when
      // NC <= 64, and their largest; the other forms bound a chunk by the
      // row's entries, which keeps their registers free)
      const int32_t* rc = rcnt + it * NC;
      int cv = 0;
      int64_t cmax = nnz;
      if constexpr (IsPackedB<SR>::value) {
        const int lane = threadIdx.x & (kWave - 1);
        int m = 0;
        if (NC <= kWave) {
          cv = lane < NC ? rc[lane] : 0;
          m = cv;
        } else {
          for (int c = lane; c < NC; c += kWave) m = max(m, rc[c]);
        }
        cmax = wave_max(m);
      }
      // the pass shape with the fewest passes for a row spread over all
      // chunks, max(chunks / chunks per pass, entries / slots), among those
      // whose slots hold any chunk of the row (shape 0 holds any chunk)
      int k = 0;
      int64_t best = INT64_MAX;
      for (int j = 0; j < sh.n; ++j) {
        if (sh.slots[j] < (1 << cw) && sh.slots[j] < cmax) continue;
        const int64_t pj = max(static_cast<int64_t>((NC + sh.maxc[j] - 1) / sh.maxc[j]),
                               (nnz + sh.slots[j] - 1) / sh.slots[j]);
        if (pj < best) {
          best = pj;
          k = j;
        }
      }
      rank_num_row<SR>(op, a_lo, a_hi, cw, sh.slots[k], NC, sh.maxc[k], pchunk, rc, cv, keep, short_seg,
                       out, out_end, c_idx, c_val, smem, info);
    }
  }
}

// (row, panel) pieces of heavy rows: one panel of one row per work item.
template <class SR>
__global__ __launch_bounds__(1024) void k_hash_num_sub(Operands op, const int32_t* __restrict__ rows,
                                                       const int32_t* __restrict__ items, int64_t nitems,
                                                       int T, int short_seg, int subP, int sub_wlog2,
                                                       const int32_t* __restrict__ pidx,
                                                       const int32_t* __restrict__ sub_cnt,
                                                       const int32_t* __restrict__ sub_off,
                                                       const int32_t* __restrict__ wend,
                                                       const int64_t* __restrict__ c_ptr,
                                                       int32_t* __restrict__ c_idx,
                                                       typename SR::Out* __restrict__ c_val) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int32_t g = items[it];
    const int32_t slot = g / subP;
    const int p = g - slot * subP;
    const int32_t row = rows[slot];
    const int64_t out = c_ptr[row] + sub_off[g];
    hash_num_row<SR>(op, row, T, short_seg, out, out + sub_cnt[g], c_idx, c_val, smem, true, pidx, subP,
                     p, p << sub_wlog2, wend[g]);
  }
}

template <class SR>
__global__ __launch_bounds__(1024) void k_dense_num_sub(Operands op, const int32_t* __restrict__ rows,
                                                        const int32_t* __restrict__ items, int64_t nitems,
                                                        int short_seg, int subP, int sub_wlog2,
                                                        const int32_t* __restrict__ pidx,
                                                        const int32_t* __restrict__ sub_cnt,
                                                        const int32_t* __restrict__ sub_off,
                                                        const int64_t* __restrict__ c_ptr,
                                                        int32_t* __restrict__ c_idx,
                                                        typename SR::Out* __restrict__ c_val) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int32_t g = items[it];
    const int32_t slot = g / subP;
    const int p = g - slot * subP;
    const int32_t row = rows[slot];
    const int64_t out = c_ptr[row] + sub_off[g];
    dense_num_row<SR>(op, row, sub_wlog2, subP, pidx, short_seg, out, out + sub_cnt[g], c_idx, c_val, smem,
                      p, p + 1);
  }
}

// ---------------------------------------------------------------------------
// Segment lists of (row, panel) pieces: every non-empty segment of a heavy
// row, bucketed by column panel, so a piece walks only its own segments.
// Slot s is the row's position in the dense symbolic list; piece g = s*P + p.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_seg_count(Operands op, const int32_t* __restrict__ rows,
                                                   int64_t nslots, int P, const int32_t* __restrict__ pidx,
                                                   const int32_t* __restrict__ wend,
                                                   int64_t* __restrict__ cnt_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned int* lc = reinterpret_cast<unsigned int*>(smem);
  int32_t* we = reinterpret_cast<int32_t*>(smem + static_cast<size_t>(P) * 4);
  for (int64_t slot = blockIdx.x; slot < nslots; slot += gridDim.x) {
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
      lc[t] = 0u;
      we[t] = wend[slot * P + t];
    }
    __syncthreads();
    const int32_t row = rows[slot];
    for (int64_t e = op.a_ptr[row] + threadIdx.x; e < op.a_ptr[row + 1]; e += blockDim.x) {
      const int32_t* sp = pidx + static_cast<int64_t>(op.a_idx[e]) * (P + 1);
      for (int p = 0; p < P;) {
        const int q = we[p];
        if (sp[q] > sp[p]) atomicAdd(&lc[p], 1u);
        p = q;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < P; t += blockDim.x) cnt_out[slot * P + t] = lc[t];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_seg_write(Operands op, const int32_t* __restrict__ rows,
                                                   int64_t nslots, int P, const int32_t* __restrict__ pidx,
                                                   const int32_t* __restrict__ wend,
                                                   const int64_t* __restrict__ segoff,
                                                   SegDesc* __restrict__ segs) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned long long* cur = reinterpret_cast<unsigned long long*>(smem);
  int32_t* we = reinterpret_cast<int32_t*>(smem + static_cast<size_t>(P) * 8);
  for (int64_t slot = blockIdx.x; slot < nslots; slot += gridDim.x) {
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
      cur[t] = static_cast<unsigned long long>(segoff[slot * P + t]);
      we[t] = wend[slot * P + t];
    }
    __syncthreads();
    const int32_t row = rows[slot];
    const int64_t a_lo = op.a_ptr[row];
    for (int64_t e = a_lo + threadIdx.x; e < op.a_ptr[row + 1]; e += blockDim.x) {
      const int32_t k = op.a_idx[e];
      const int64_t bs = op.b_ptr[k];
      const int32_t* sp = pidx + static_cast<int64_t>(k) * (P + 1);
      for (int p = 0; p < P;) {
        const int q = we[p];
        const int32_t s0 = sp[p], s1 = sp[q];
        if (s1 > s0) {
          const unsigned long long pos = atomicAdd(&cur[p], 1ull);
          segs[pos] = SegDesc{bs + s0, s1 - s0, static_cast<int32_t>(e - a_lo)};
        }
        p = q;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_seg_count(const Operands& op, const int32_t* rows, int64_t nslots, int P,
                            const int32_t* pidx, const int32_t* wend, int64_t* cnt_out, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_count, dim3(grid_for(nslots, 0)), dim3(256), static_cast<size_t>(P) * 8, s, op, rows,
                     nslots, P, pidx, wend, cnt_out);
  return hipGetLastError();
}

hipError_t launch_seg_write(const Operands& op, const int32_t* rows, int64_t nslots, int P,
                            const int32_t* pidx, const int32_t* wend, const int64_t* segoff, void* segs,
                            hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_write, dim3(grid_for(nslots, 0)), dim3(256), static_cast<size_t>(P) * 12, s, op, rows,
                     nslots, P, pidx, wend, segoff, static_cast<SegDesc*>(segs));
  return hipGetLastError();
}

template <class SR>
__global__ __launch_bounds__(1024) void k_hash_num_seg(Operands op, const int32_t* __restrict__ rows,
                                                       const int32_t* __restrict__ items, int64_t nitems,
                                                       int T, int short_seg, int subP, int sub_wlog2,
                                                       const int64_t* __restrict__ segoff,
                                                       const SegDesc* __restrict__ segs,
                                                       const int32_t* __restrict__ sub_cnt,
                                                       const int32_t* __restrict__ sub_off,
                                                       const int64_t* __restrict__ c_ptr,
                                                       int32_t* __restrict__ c_idx,
                                                       typename SR::Out* __restrict__ c_val) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int32_t g = items[it];
    const int32_t slot = g / subP;
    const int p = g - slot * subP;
    const int32_t row = rows[slot];
    SegSource<SR> src{&op, op.a_ptr[row], segs + segoff[g], segoff[g + 1] - segoff[g]};
    const int64_t out = c_ptr[row] + sub_off[g];
    hash_num_src<SR>(op, src, p << sub_wlog2, T, short_seg, out, out + sub_cnt[g], c_idx, c_val, smem);
  }
}

template <class SR>
__global__ __launch_bounds__(1024) void k_dense_num_seg(Operands op, const int32_t* __restrict__ rows,
                                                        const int32_t* __restrict__ items, int64_t nitems,
                                                        int short_seg, int subP, int sub_wlog2,
                                                        const int64_t* __restrict__ segoff,
                                                        const SegDesc* __restrict__ segs,
                                                        const int32_t* __restrict__ sub_cnt,
                                                        const int32_t* __restrict__ sub_off,
                                                        const int64_t* __restrict__ c_ptr,
                                                        int32_t* __restrict__ c_idx,
                                                        typename SR::Out* __restrict__ c_val) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int32_t g = items[it];
    const int32_t slot = g / subP;
    const int p = g - slot * subP;
    const int32_t row = rows[slot];
    const int64_t a_lo = op.a_ptr[row];
    const SegDesc* sg = segs + segoff[g];
    const int64_t ns = segoff[g + 1] - segoff[g];
    auto make = [&](int) { return SegSource<SR>{&op, a_lo, sg, ns}; };
    const int64_t out = c_ptr[row] + sub_off[g];
    dense_num_gen<SR>(op, sub_wlog2, p, p + 1, short_seg, out, out + sub_cnt[g], c_idx, c_val, smem, make);
  }
}

template <class SR>
__global__ __launch_bounds__(1024) void k_hash_num_b(const BatchDesc* __restrict__ descs,
                                                     const int64_t* __restrict__ row_off,
    const int32_t* __restrict__ prod_of, int nprod,
                                                     const int32_t* __restrict__ items, int64_t nitems,
                                                     int T, int short_seg) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t r = uniform(items[it]);
    const int b = uniform(prod_of[r]);
    const BatchDesc d = descs[b];  // uniform: held in scalar registers
    const int32_t row = uniform(static_cast<int32_t>(r - row_off[b]));
    hash_num_row<SR>(d.op, row, T, short_seg, d.c_ptr[row], d.c_ptr[row + 1], d.c_idx,
                     static_cast<typename SR::Out*>(d.c_val), smem);
  }
}

// Rank passes over all k columns of a row (k small enough for the whole
// bitmap in LDS): the pattern by a walk over B's column ids and a prefix
// count per 64-bit word, once; then passes over runs of words whose entries
// fit the value slots (one pass when the row's entries do), each combining
// the values of its columns at their ranks and writing them in column order.
// A pass reads only the B panels that overlap its columns (the numeric panel
// index, when the product has more than one panel).  The batched heavy rows
// of small products take it instead of one fixed panel after another.
template <class SR>
struct RankRangeSink {
  using S = typename SR::S;
  const uint64_t* bits;
  const uint16_t* pre;
  S* vals;
  int w_lo, w_hi, r_lo;
  __device__ void add(int32_t c, S v) {
    const int w = c >> 6;
    if (w < w_lo || w >= w_hi) return;  // a column of a boundary panel outside the pass
    const uint64_t below = bits[w] & ((1ull << (c & 63)) - 1ull);
    SR::combine(&vals[pre[w] + __popcll(below) - r_lo], v);
  }
};

template <class SR>
__device__ void rank_row_whole(const Operands& op, int64_t a_lo, int64_t a_hi, int slots, int short_seg,
                               int wlog2, int P, const int32_t* __restrict__ pidx, int64_t out, int64_t out_end,
                               int32_t* __restrict__ c_idx, typename SR::Out* __restrict__ c_val,
                               unsigned char* smem) {
  using S = typename SR::S;
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  auto q = RowQueue<typename SR::In>::carve(smem, nt);
  auto pq = RowQueue<SrPattern::In>::carve(smem, nt);
  unsigned char* p0 = smem + rank_queue_bytes<SR>(nt);
  S* vals = reinterpret_cast<S*>(p0);
  uint32_t* bits = reinterpret_cast<uint32_t*>(p0 + sizeof(S) * static_cast<size_t>(slots));
  const int nwords = (op.k + 31) >> 5;
  const int nw64 = (nwords + 1) >> 1;
  uint16_t* pre = reinterpret_cast<uint16_t*>(bits + 2 * nw64);
  const uint64_t* bits64 = reinterpret_cast<const uint64_t*>(bits);
  for (int t = tid; t < 2 * nw64; t += nt) bits[t] = 0u;
  __syncthreads();
  BitmapSink bs{bits};
  RowSource<SrPattern> ps{&op, a_lo, a_hi, false, nullptr, 1, 0, 1};
  enumerate_src<SrPattern, 2>(op, ps, 0, short_seg, pq, bs);
  const int wpt = (nw64 + nt - 1) / nt;
  const int w0 = min(nw64, tid * wpt), w1 = min(nw64, w0 + wpt);
  int local = 0;
  for (int w = w0; w < w1; ++w) local += __popcll(bits64[w]);
  int ptotal;
  int run = block_exclusive_scan(local, q.ctr + 2, &ptotal);
  for (int w = w0; w < w1; ++w) {
    pre[w] = static_cast<uint16_t>(run);
    run += __popcll(bits64[w]);
  }
  __syncthreads();
  const int total = static_cast<int>(min(static_cast<int64_t>(ptotal), out_end - out));
  for (int w_lo = 0; w_lo < nw64;) {
    // the pass: words [w_lo, w_hi), the most whose entries fit the slots
    // (a word holds at most 64 <= slots); every thread finds the same bound
    const int r_lo = pre[w_lo];
    // all the rest, or w_hi in [w_lo + 1, nw64 - 1] (more than one word's
    // entries remain, so at least two words)
    int lo = w_lo + 1, hi = nw64 - 1;
    if (ptotal - r_lo <= slots) {
      lo = nw64;
    } else {
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] - r_lo <= slots)
          lo = mid;
        else
          hi = mid - 1;
      }
    }
    const int w_hi = lo;
    const int r_hi = w_hi < nw64 ? static_cast<int>(pre[w_hi]) : ptotal;
    const int cnt = r_hi - r_lo;
    for (int t = tid; t < cnt; t += nt) vals[t] = SR::identity();
    __syncthreads();
    RankRangeSink<SR> rs{bits64, pre, vals, w_lo, w_hi, r_lo};
    if (P > 1) {
      const int p_lo = (w_lo << 6) >> wlog2, p_hi = (((w_hi << 6) - 1) >> wlog2) + 1;
      RowSource<SR> vs{&op, a_lo, a_hi, true, pidx, P, p_lo, min(p_hi, P)};
      enumerate_src<SR, 2>(op, vs, 0, short_seg, q, rs);
    } else {
      RowSource<SR> vs{&op, a_lo, a_hi, false, nullptr, 1, 0, 1};
      enumerate_src<SR, 2>(op, vs, 0, short_seg, q, rs);
    }
    const int lim = max(0, min(cnt, total - r_lo));
    for (int r = tid; r < lim; r += nt) c_val[out + r_lo + r] = SR::out(vals[r]);
    __syncthreads();
    int32_t* ids = reinterpret_cast<int32_t*>(vals);
    static_assert(sizeof(S) >= sizeof(int32_t), "ids are staged over the value slots");
    for (int w = w_lo + tid; w < w_hi; w += nt) {
      uint64_t x = bits64[w];
      int qi = pre[w] - r_lo;
      while (x) {
        ids[qi++] = (w << 6) + __ffsll(static_cast<unsigned long long>(x)) - 1;
        x &= x - 1;
      }
    }
    __syncthreads();
    for (int r = tid; r < lim; r += nt) c_idx[out + r_lo + r] = ids[r];
    __syncthreads();
    w_lo = w_hi;
  }
}

// Heavy rows of a batch: rank passes over the whole row's bitmap when the
// product has at most kcap columns, else fixed panels.
template <class SR>
__global__ __launch_bounds__(1024) void k_dense_num_b(const BatchDesc* __restrict__ descs,
                                                      const int64_t* __restrict__ row_off,
    const int32_t* __restrict__ prod_of, int nprod,
                                                      const int32_t* __restrict__ items, int64_t nitems,
                                                      int short_seg, int kcap, int slots) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t r = uniform(items[it]);
    const int b = uniform(prod_of[r]);
    const BatchDesc d = descs[b];  // uniform: held in scalar registers
    const int32_t row = uniform(static_cast<int32_t>(r - row_off[b]));
    const int64_t out = uniform64(d.c_ptr[row]), out_end = uniform64(d.c_ptr[row + 1]);
    if constexpr (!SR::kPattern) {
      if (d.op.k <= kcap) {
        rank_row_whole<SR>(d.op, d.op.a_ptr[row], d.op.a_ptr[row + 1], slots, short_seg, d.num_wlog2, d.num_P,
                           d.pnum, out, out_end, d.c_idx, static_cast<typename SR::Out*>(d.c_val), smem);
        continue;
      }
    }
    dense_num_row<SR>(d.op, row, d.num_wlog2, d.num_P, d.pnum, short_seg, out, out_end, d.c_idx,
                      static_cast<typename SR::Out*>(d.c_val), smem);
  }
}

template <class SR>
static size_t hash_num_lds_t(int T, int nt) {
  return RowQueue<typename SR::In>::bytes(nt) +
         static_cast<size_t>(T) * (4 + (SR::kPattern ? 0 : sizeof(typename SR::S)));
}
template <class SR>
static size_t dense_num_lds_t(int wlog2, int nt) {
  const size_t W = static_cast<size_t>(1) << wlog2;
  return RowQueue<typename SR::In>::bytes(nt) + W / 8 + (SR::kPattern ? 0 : W * sizeof(typename SR::S));
}

template <class SR>
static hipError_t hash_num_t(const Operands& op, const int32_t* rows, int64_t nrows, int T, int nt,
                             int short_seg, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                             hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_num<SR>, dim3(grid_for(nrows, 0)), dim3(nt), hash_num_lds_t<SR>(T, nt), s,
                     op, rows, nrows, T, short_seg, c_ptr, c_idx, static_cast<typename SR::Out*>(c_val));
  return hipGetLastError();
}

template <class SR>
static hipError_t esc_num_t(const Operands& op, const int32_t* rows, int64_t nrows, int N, const int64_t* c_ptr,
                            int32_t* c_idx, void* c_val, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const int nt = esc_threads(N);
  const int R = esc_per_thread(N);
  const size_t lds = esc_lds_bytes<SR>(N, nt);
  if (N > R * nt || N > kEscMaxFlops || lds > static_cast<size_t>(max_lds_bytes())) return hipErrorInvalidValue;
  auto* cv = static_cast<typename SR::Out*>(c_val);
  if (R == 4)
    hipLaunchKernelGGL((k_esc_num<SR, 4>), dim3(grid_for(nrows, 0)), dim3(nt), lds, s, op, rows, nrows, N, c_ptr,
                       c_idx, cv);
  else if (R == 8)
    hipLaunchKernelGGL((k_esc_num<SR, 8>), dim3(grid_for(nrows, 0)), dim3(nt), lds, s, op, rows, nrows, N, c_ptr,
                       c_idx, cv);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// The largest expand-sort-compress class whose LDS fits the device.
template <class SR>
static int esc_class_limit_t() {
  int N = kEscMaxFlops;
  while (N > 32 && esc_lds_bytes<SR>(N, esc_threads(N)) > static_cast<size_t>(max_lds_bytes())) N >>= 1;
  return N;
}

template <class SR>
static hipError_t dense_num_t(const Operands& op, const int32_t* rows, int64_t nrows, int wlog2,
                              int P, const int32_t* pidx, int nt, int short_seg,
                              const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_num<SR>, dim3(grid_for(nrows, 0)), dim3(nt), dense_num_lds_t<SR>(wlog2, nt),
                     s, op, rows, nrows, wlog2, P, pidx, short_seg, c_ptr, c_idx,
                     static_cast<typename SR::Out*>(c_val));
  return hipGetLastError();
}

template <class SR>
static size_t rank_num_lds_t(int cw, int slots, int max_chunks, int wlog2, int nt) {
  const size_t a = rank_num_lds_bytes<SR>(cw, slots, max_chunks, nt);
  const size_t b = dense_num_lds_t<SR>(wlog2, nt);
  return a > b ? a : b;
}

// LDS of a rank launch: the largest of its pass shapes.
template <class SR>
static size_t rank_launch_lds(int cw, const RankShapes& sh, int nt) {
  size_t b = 0;
  for (int j = 0; j < sh.n; ++j) {
    const size_t a = rank_num_lds_bytes<SR>(cw, sh.slots[j], sh.maxc[j], nt);
    b = a > b ? a : b;
  }
  return b;
}

template <class SR>
static hipError_t rank_num_launch(bool fixed, const Operands& op, const int32_t* rows, int64_t nrows, int32_t rb,
                                  int32_t re, int cw, int NC, const RankShapes& sh,
                                  const int32_t* pchunk, const int32_t* rcnt,
                                  int64_t nnz_lo, int64_t nnz_hi, int wlog2, int P, int nt, int short_seg,
                                  const uint32_t* keep_store, const int32_t* keep_slot, int64_t keep_nwords,
                                  const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s) {
  if (fixed)
    hipLaunchKernelGGL((k_rank_num<SR, true>), dim3(grid_for(nrows, 0)), dim3(nt), dense_num_lds_t<SR>(wlog2, nt),
                       s, op, rows, nrows, rb, re, cw, NC, sh, pchunk, rcnt, nnz_lo,
                       nnz_hi, wlog2,
                       P, short_seg, keep_store, keep_slot, keep_nwords, c_ptr, c_idx,
                       static_cast<typename SR::Out*>(c_val));
  else
    hipLaunchKernelGGL((k_rank_num<SR, false>), dim3(grid_for(nrows, 0)), dim3(nt),
                       rank_launch_lds<SR>(cw, sh, nt), s, op, rows, nrows, rb, re, cw, NC,
                       sh, pchunk, rcnt, nnz_lo, nnz_hi, wlog2, P, short_seg, keep_store, keep_slot, keep_nwords, c_ptr,
                       c_idx, static_cast<typename SR::Out*>(c_val));
  return hipGetLastError();
}

template <class SR>
static hipError_t rank_num_t(bool fixed, const Operands& op, const int32_t* rows, int64_t nrows, int32_t rb,
                             int32_t re, int cw, int NC, const RankShapes& sh,
                             const int32_t* pchunk, const int32_t* rcnt, int64_t nnz_lo,
                             int64_t nnz_hi, int wlog2, int P, int nt, int short_seg, const uint32_t* keep_store,
                             const int32_t* keep_slot, int64_t keep_nwords, const int64_t* c_ptr,
                             int32_t* c_idx, void* c_val, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  if constexpr (SR::kPattern) {
    return hipErrorInvalidValue;  // pattern-only rows use the bitmap paths
  } else if constexpr (std::is_same<SR, SrMinPlusI32>::value) {
    if (op.b_packed)  // B is read through one word per entry (small values)
      return rank_num_t<PackedB<SR>>(fixed, op, rows, nrows, rb, re, cw, NC, sh, pchunk, rcnt, nnz_lo,
                                     nnz_hi, wlog2, P, nt, short_seg, keep_store, keep_slot, keep_nwords,
                                     c_ptr, c_idx, c_val, s);
    if (op.b_pair)
      return rank_num_t<PairedB<SR>>(fixed, op, rows, nrows, rb, re, cw, NC, sh, pchunk, rcnt, nnz_lo,
                                     nnz_hi, wlog2, P, nt, short_seg, keep_store, keep_slot, keep_nwords,
                                     c_ptr, c_idx, c_val, s);
    return rank_num_launch<SR>(fixed, op, rows, nrows, rb, re, cw, NC, sh, pchunk, rcnt, nnz_lo,
                               nnz_hi, wlog2, P, nt, short_seg, keep_store, keep_slot, keep_nwords, c_ptr,
                               c_idx, c_val, s);
  } else if constexpr (sizeof(typename SR::In) == 4 && !IsPairedB<SR>::value && !IsPackedB<SR>::value) {
    if (op.b_pair)  // B is read through its (column id, value) pairs
      return rank_num_t<PairedB<SR>>(fixed, op, rows, nrows, rb, re, cw, NC, sh, pchunk, rcnt, nnz_lo,
                                     nnz_hi, wlog2, P, nt, short_seg, keep_store, keep_slot, keep_nwords,
                                     c_ptr, c_idx, c_val, s);
    return rank_num_launch<SR>(fixed, op, rows, nrows, rb, re, cw, NC, sh, pchunk, rcnt, nnz_lo,
                               nnz_hi, wlog2, P, nt, short_seg, keep_store, keep_slot, keep_nwords, c_ptr,
                               c_idx, c_val, s);
  } else {
    return rank_num_launch<SR>(fixed, op, rows, nrows, rb, re, cw, NC, sh, pchunk, rcnt, nnz_lo,
                               nnz_hi, wlog2, P, nt, short_seg, keep_store, keep_slot, keep_nwords, c_ptr,
                               c_idx, c_val, s);
  }
}

template <class SR>
static hipError_t hash_num_b_t(const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                               const int32_t* items, int64_t nitems, int T, int nt, int short_seg,
                               hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_num_b<SR>, dim3(grid_for(nitems, 0)), dim3(nt),
                     hash_num_lds_t<SR>(T, nt), s, descs, row_off, prod_of, nprod, items, nitems, T, short_seg);
  return hipGetLastError();
}

template <class SR>
static hipError_t esc_num_b_t(const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod, const int32_t* items,
                              int64_t nitems, int N, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const int nt = esc_threads(N);
  const int R = esc_per_thread(N);
  const size_t lds = esc_lds_bytes<SR>(N, nt);
  if (N > R * nt || N > kEscMaxFlops || lds > static_cast<size_t>(max_lds_bytes())) return hipErrorInvalidValue;
  const dim3 grid(grid_for(nitems, 0));
  if (R == 4)
    hipLaunchKernelGGL((k_esc_num_b<SR, 4>), grid, dim3(nt), lds, s, descs, row_off, prod_of, nprod, items, nitems, N);
  else if (R == 8)
    hipLaunchKernelGGL((k_esc_num_b<SR, 8>), grid, dim3(nt), lds, s, descs, row_off, prod_of, nprod, items, nitems, N);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class SR>
static hipError_t dense_num_b_t(const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                                const int32_t* items, int64_t nitems, int wlog2_max, int nt,
                                int short_seg, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  // whole-row rank passes in the same LDS: up to 2^16 columns (bitmap and
  // word ranks), the rest of it value slots
  const size_t lds = dense_num_lds_t<SR>(wlog2_max, nt);
  int kcap = 0, slots = 0;
  if constexpr (!SR::kPattern) {
    const int kc = 1 << 16;
    const size_t fixed = rank_queue_bytes<SR>(nt) + kc / 8 + (kc / 64) * 2;
    if (lds > fixed) {
      const size_t sl = std::min<size_t>((lds - fixed) / sizeof(typename SR::S), 65535) & ~size_t(63);
      if (sl >= 1024) {
        kcap = kc;
        slots = static_cast<int>(sl);
      }
    }
  }
  hipLaunchKernelGGL(k_dense_num_b<SR>, dim3(grid_for(nitems, 0)), dim3(nt), lds, s, descs, row_off, prod_of, nprod,
                     items, nitems, short_seg, kcap, slots);
  return hipGetLastError();
}

template <class SR>
static hipError_t hash_num_sub_t(const Operands& op, const int32_t* rows, const int32_t* items,
                                 int64_t nitems, int T, int nt, int short_seg, int subP, int sub_wlog2,
                                 const int32_t* pidx, const int32_t* cnt, const int32_t* off,
                                 const int32_t* wend, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                                 hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_num_sub<SR>, dim3(grid_for(nitems, 0)), dim3(nt), hash_num_lds_t<SR>(T, nt), s,
                     op, rows, items, nitems, T, short_seg, subP, sub_wlog2, pidx, cnt, off, wend, c_ptr, c_idx,
                     static_cast<typename SR::Out*>(c_val));
  return hipGetLastError();
}

template <class SR>
static hipError_t dense_num_sub_t(const Operands& op, const int32_t* rows, const int32_t* items,
                                  int64_t nitems, int nt, int short_seg, int subP, int sub_wlog2,
                                  const int32_t* pidx, const int32_t* cnt, const int32_t* off,
                                  const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_num_sub<SR>, dim3(grid_for(nitems, 0)), dim3(nt),
                     dense_num_lds_t<SR>(sub_wlog2, nt), s, op, rows, items, nitems, short_seg, subP,
                     sub_wlog2, pidx, cnt, off, c_ptr, c_idx, static_cast<typename SR::Out*>(c_val));
  return hipGetLastError();
}

template <class SR>
static hipError_t hash_num_seg_t(const Operands& op, const int32_t* rows, const int32_t* items,
                                 int64_t nitems, int T, int nt, int short_seg, int subP, int sub_wlog2,
                                 const int64_t* segoff, const void* segs, const int32_t* cnt,
                                 const int32_t* off, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                                 hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_num_seg<SR>, dim3(grid_for(nitems, 0)), dim3(nt), hash_num_lds_t<SR>(T, nt), s,
                     op, rows, items, nitems, T, short_seg, subP, sub_wlog2, segoff,
                     static_cast<const SegDesc*>(segs), cnt, off, c_ptr, c_idx,
                     static_cast<typename SR::Out*>(c_val));
  return hipGetLastError();
}

template <class SR>
static hipError_t dense_num_seg_t(const Operands& op, const int32_t* rows, const int32_t* items,
                                  int64_t nitems, int nt, int short_seg, int subP, int sub_wlog2,
                                  const int64_t* segoff, const void* segs, const int32_t* cnt,
                                  const int32_t* off, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                                  hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_num_seg<SR>, dim3(grid_for(nitems, 0)), dim3(nt),
                     dense_num_lds_t<SR>(sub_wlog2, nt), s, op, rows, items, nitems, short_seg, subP,
                     sub_wlog2, segoff, static_cast<const SegDesc*>(segs), cnt, off, c_ptr, c_idx,
                     static_cast<typename SR::Out*>(c_val));
  return hipGetLastError();
}

#define SPG_DISPATCH(sr, FN, ...)                           \
  switch (sr) {                                            \
    case 0: return FN<SrPlusTimesF64>(__VA_ARGS__);        \
    case 1: return FN<SrPlusTimesF32>(__VA_ARGS__);        \
    case 2: return FN<SrMinPlusI32>(__VA_ARGS__);          \
    case 3: return FN<SrMinPlusF32>(__VA_ARGS__);          \
    case 4: return FN<SrOrAndBool>(__VA_ARGS__);           \
    case 5: return FN<SrMaxTimesF64>(__VA_ARGS__);         \
    case 6: return FN<SrMaxTimesF32>(__VA_ARGS__);         \
    default: return FN<SrPattern>(__VA_ARGS__);            \
  }

hipError_t launch_hash_num(int sr, const Operands& op, const int32_t* rows, int64_t nrows, int T,
                           int nt, int short_seg, const int64_t* c_ptr, int32_t* c_idx,
                           void* c_val, hipStream_t s) {
  SPG_DISPATCH(sr, hash_num_t, op, rows, nrows, T, nt, short_seg, c_ptr, c_idx, c_val, s)
}

hipError_t launch_esc_num(int sr, const Operands& op, const int32_t* rows, int64_t nrows, int N,
                          const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s) {
  SPG_DISPATCH(sr, esc_num_t, op, rows, nrows, N, c_ptr, c_idx, c_val, s)
}
int esc_class_limit(int sr) { SPG_DISPATCH(sr, esc_class_limit_t) }

hipError_t launch_dense_num(int sr, const Operands& op, const int32_t* rows, int64_t nrows,
                            int wlog2, int P, const int32_t* pidx, int nt, int short_seg,
                            const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s) {
  SPG_DISPATCH(sr, dense_num_t, op, rows, nrows, wlog2, P, pidx, nt, short_seg, c_ptr, c_idx, c_val,
               s)
}

hipError_t launch_rank_num(int sr, bool fixed, const Operands& op, const int32_t* rows, int64_t nrows, int32_t rb,
                           int32_t re, int cw, int NC, const RankShapes& sh,
                           const int32_t* pchunk, const int32_t* rcnt, int64_t nnz_lo,
                           int64_t nnz_hi, int wlog2, int P, int nt, int short_seg, const uint32_t* keep_store,
                           const int32_t* keep_slot, int64_t keep_nwords, const int64_t* c_ptr,
                           int32_t* c_idx, void* c_val, hipStream_t s) {
  SPG_DISPATCH(sr, rank_num_t, fixed, op, rows, nrows, rb, re, cw, NC, sh, pchunk, rcnt, nnz_lo, nnz_hi,
               wlog2, P, nt, short_seg, keep_store, keep_slot, keep_nwords, c_ptr, c_idx, c_val, s)
}

hipError_t launch_esc_num_b(int sr, const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod, const int32_t* items,
                            int64_t nitems, int N, hipStream_t s) {
  SPG_DISPATCH(sr, esc_num_b_t, descs, row_off, prod_of, nprod, items, nitems, N, s)
}
hipError_t launch_hash_num_b(int sr, const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                             const int32_t* items, int64_t nitems, int T, int nt, int short_seg,
                             hipStream_t s) {
  SPG_DISPATCH(sr, hash_num_b_t, descs, row_off, prod_of, nprod, items, nitems, T, nt, short_seg, s)
}

hipError_t launch_dense_num_b(int sr, const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                              const int32_t* items, int64_t nitems, int wlog2_max, int nt,
                              int short_seg, hipStream_t s) {
  SPG_DISPATCH(sr, dense_num_b_t, descs, row_off, prod_of, nprod, items, nitems, wlog2_max, nt, short_seg,
               s)
}

hipError_t launch_hash_num_sub(int sr, const Operands& op, const int32_t* rows, const int32_t* items,
                               int64_t nitems, int T, int nt, int short_seg, int subP, int sub_wlog2,
                               const int32_t* pidx, const int32_t* cnt, const int32_t* off,
                               const int32_t* wend, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                               hipStream_t s) {
  SPG_DISPATCH(sr, hash_num_sub_t, op, rows, items, nitems, T, nt, short_seg, subP, sub_wlog2, pidx, cnt,
               off, wend, c_ptr, c_idx, c_val, s)
}

hipError_t launch_dense_num_sub(int sr, const Operands& op, const int32_t* rows, const int32_t* items,
                                int64_t nitems, int nt, int short_seg, int subP, int sub_wlog2,
                                const int32_t* pidx, const int32_t* cnt, const int32_t* off,
                                const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s) {
  SPG_DISPATCH(sr, dense_num_sub_t, op, rows, items, nitems, nt, short_seg, subP, sub_wlog2, pidx, cnt,
               off, c_ptr, c_idx, c_val, s)
}

hipError_t launch_hash_num_seg(int sr, const Operands& op, const int32_t* rows, const int32_t* items,
                               int64_t nitems, int T, int nt, int short_seg, int subP, int sub_wlog2,
                               const int64_t* segoff, const void* segs, const int32_t* cnt,
                               const int32_t* off, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                               hipStream_t s) {
  SPG_DISPATCH(sr, hash_num_seg_t, op, rows, items, nitems, T, nt, short_seg, subP, sub_wlog2, segoff, segs,
               cnt, off, c_ptr, c_idx, c_val, s)
}

hipError_t launch_dense_num_seg(int sr, const Operands& op, const int32_t* rows, const int32_t* items,
                                int64_t nitems, int nt, int short_seg, int subP, int sub_wlog2,
                                const int64_t* segoff, const void* segs, const int32_t* cnt,
                                const int32_t* off, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                                hipStream_t s) {
  SPG_DISPATCH(sr, dense_num_seg_t, op, rows, items, nitems, nt, short_seg, subP, sub_wlog2, segoff, segs,
               cnt, off, c_ptr, c_idx, c_val, s)
}

size_t seg_desc_bytes() { return sizeof(SegDesc); }

size_t hash_num_lds(int sr, int T, int nt) { SPG_DISPATCH(sr, hash_num_lds_t, T, nt) }
size_t dense_num_lds(int sr, int wlog2, int nt) { SPG_DISPATCH(sr, dense_num_lds_t, wlog2, nt) }
template <class SR>
static size_t rank_pass_lds_t(int cw, int slots, int max_chunks, int nt) {
  return rank_num_lds_bytes<SR>(cw, slots, max_chunks, nt);
}
size_t rank_pass_lds(int sr, int cw, int slots, int max_chunks, int nt) {
  SPG_DISPATCH(sr, rank_pass_lds_t, cw, slots, max_chunks, nt)
}
size_t rank_num_lds(int sr, int cw, int slots, int max_chunks, int wlog2, int nt) {
  SPG_DISPATCH(sr, rank_num_lds_t, cw, slots, max_chunks, wlog2, nt)
}

template <class SR>
static size_t storage_bytes_t() {
  return SR::kPattern ? 0 : sizeof(typename SR::S);
}
size_t storage_bytes(int sr) { SPG_DISPATCH(sr, storage_bytes_t) }

int hash_threads_num(int c, int sr) {
  // the numeric compaction keeps 16 slots per thread (8 for 8-byte values)
  int t = hash_table_size(c) / (storage_bytes(sr) > 4 ? 8 : 16);
  return t < 64 ? 64 : (t > 1024 ? 1024 : t);
}

int max_lds_bytes() { return 160 * 1024; }

// ---------------------------------------------------------------------------
// Prune (Markov-clustering step after expansion): keep value >= thresh.
// ---------------------------------------------------------------------------
// One wave per slice, kPruneUnroll loads per lane in flight.
constexpr int kPruneUnroll = 8;

__global__ void k_prune_count(const int64_t* __restrict__ ptr, const float* __restrict__ val,
                              int64_t nmajor, float thresh, int64_t* __restrict__ cnt) {
  constexpr int U = kPruneUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
  for (int64_t s = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6); s < nmajor;
       s += waves) {
    const int64_t hi = ptr[s + 1];
    int c = 0;
    for (int64_t b = ptr[s] + lane; b < hi; b += U * kWave) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (b + u * kWave < hi) v[u] = val[b + u * kWave];
#pragma unroll
      for (int u = 0; u < U; ++u) c += (b + u * kWave < hi && v[u] >= thresh) ? 1 : 0;
    }
    const int64_t t = wave_sum(static_cast<int64_t>(c));
    if (lane == 0) cnt[s] = t;
  }
}

// Kept entries of a slice in order: kPruneUnroll groups of 64 entries are
// loaded before their keep masks place them.
__global__ void k_prune_apply(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                              const float* __restrict__ val, int64_t nmajor, float thresh,
                              const int64_t* __restrict__ new_ptr, int32_t* __restrict__ new_idx,
                              float* __restrict__ new_val) {
  constexpr int U = kPruneUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
  for (int64_t s = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6); s < nmajor;
       s += waves) {
    int64_t o = new_ptr[s];
    const int64_t hi = ptr[s + 1];
    for (int64_t b = ptr[s]; b < hi; b += U * kWave) {
      float v[U];
      int32_t c[U];
      bool keep[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t p = b + u * kWave + lane;
        keep[u] = false;
        if (p < hi) {
          v[u] = val[p];
          c[u] = idx[p];
          keep[u] = v[u] >= thresh;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const unsigned long long m = __ballot(keep[u]);
        if (keep[u]) {
          const int before = __popcll(m & ((1ull << lane) - 1ull));
          new_idx[o + before] = c[u];
          new_val[o + before] = v[u];
        }
        o += __popcll(m);
      }
    }
  }
}

// Inflation and renormalisation (the Markov-clustering step after pruning):
// every slice's values raised to the power r, then divided by their sum
// (taken in float64).  One wave per slice; val_out may be val.
// v^r.  The customary r = 2 is the single product v * v (one rounding, no
// less accurate than powf and a fraction of its instructions).
__device__ __forceinline__ float inflate_pow(float v, float r) { return r == 2.0f ? v * v : powf(v, r); }

__global__ void k_inflate(const int64_t* __restrict__ ptr, const float* val, int64_t nmajor, float r,
                          float* val_out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
  for (int64_t s = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6); s < nmajor;
       s += waves) {
    constexpr int U = kPruneUnroll;
    const int64_t lo = ptr[s], hi = ptr[s + 1];
    if (hi - lo <= 2 * U * kWave) {
      // the slice in registers: one load and one power per entry
      float w[2 * U];
#pragma unroll
      for (int u = 0; u < 2 * U; ++u)
        if (lo + lane + u * kWave < hi) w[u] = val[lo + lane + u * kWave];
      double t = 0.0;
#pragma unroll
      for (int u = 0; u < 2 * U; ++u)
        if (lo + lane + u * kWave < hi) {
          w[u] = inflate_pow(w[u], r);
          t += static_cast<double>(w[u]);
        }
      t = wave_sum(t);
      if (t == 0.0) {  // a slice whose powers sum to 0 is left as it is
        for (int64_t q = lo + lane; q < hi; q += kWave) val_out[q] = val[q];
        continue;
      }
      const double inv = 1.0 / t;
#pragma unroll
      for (int u = 0; u < 2 * U; ++u)
        if (lo + lane + u * kWave < hi) val_out[lo + lane + u * kWave] = static_cast<float>(static_cast<double>(w[u]) * inv);
      continue;
    }
    double sum = 0.0;
    for (int64_t b = lo + lane; b < hi; b += U * kWave) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (b + u * kWave < hi) v[u] = val[b + u * kWave];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (b + u * kWave < hi) sum += static_cast<double>(inflate_pow(v[u], r));
    }
    sum = wave_sum(sum);
    const double inv = sum == 0.0 ? 1.0 : 1.0 / sum;
    for (int64_t b = lo + lane; b < hi; b += U * kWave) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (b + u * kWave < hi) v[u] = val[b + u * kWave];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (b + u * kWave < hi)  // a slice whose powers sum to 0 is left as it is
          val_out[b + u * kWave] = sum == 0.0 ? v[u] : static_cast<float>(static_cast<double>(inflate_pow(v[u], r)) * inv);
    }
  }
}

hipError_t launch_inflate(const int64_t* ptr, const float* val, int64_t nmajor, float r, float* val_out,
                          hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = wave_grid(nmajor, nt);
  hipLaunchKernelGGL(k_inflate, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, ptr, val, nmajor, r, val_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Selection (the Markov-clustering step that bounds the entries kept per
// column, paper Sec. 7.5): a slice longer than S keeps the S entries with the
// largest values, ties going to the smaller id, in id order.  The order is
// that of the 64-bit key (total-order key of the float32 value, -0 < +0) << 32
// | (2^32 - 1 - id), unique within a slice.  A radix select (at most eight
// passes of 8 bits from the top over the slice, a histogram in LDS, one
// workgroup per slice) finds a threshold that exactly S keys reach: the S-th
// largest key, or its leading digits alone once every key sharing them is
// kept; those S entries are placed in order by a block scan of keep flags.
// ---------------------------------------------------------------------------
__global__ void k_select_count(const int64_t* __restrict__ ptr, int64_t nmajor, int64_t S,
                               int64_t* __restrict__ cnt) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s < nmajor) cnt[s] = min(ptr[s + 1] - ptr[s], S);
}

__device__ __forceinline__ uint64_t select_key(float v, int32_t id) {
  return (static_cast<uint64_t>(f32_key(v)) << 32) | static_cast<uint64_t>(~static_cast<uint32_t>(id));
}

constexpr int kSelectThreads = 256;

__global__ __launch_bounds__(kSelectThreads) void k_select_apply(const int64_t* __restrict__ ptr,
                                                                 const int32_t* __restrict__ idx,
                                                                 const float* __restrict__ val, int64_t nmajor,
                                                                 int64_t S, const int64_t* __restrict__ new_ptr,
                                                                 int32_t* __restrict__ new_idx,
                                                                 float* __restrict__ new_val) {
  __shared__ unsigned int hist[256];
  __shared__ uint64_t prefix_s;
  __shared__ int64_t need_s;
  __shared__ int done_s;
  __shared__ int64_t tmp[16];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (kWave - 1);
  for (int64_t s = blockIdx.x; s < nmajor; s += gridDim.x) {
    const int64_t lo = ptr[s], hi = ptr[s + 1];
    const int64_t out = new_ptr[s];
    if (hi - lo <= S) {  // kept whole
      for (int64_t p = lo + tid; p < hi; p += nt) {
        new_idx[out + p - lo] = idx[p];
        new_val[out + p - lo] = val[p];
      }
      continue;
    }
    if (S <= 0) continue;
    // radix select of the S-th largest key, 8 bits per pass from the top
    uint64_t prefix = 0;
    int64_t need = S;  // rank, from the top, among the keys that match prefix
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int t = tid; t < 256; t += nt) hist[t] = 0u;
      __syncthreads();
      const uint64_t hmask = shift == 56 ? 0ull : (~0ull << (shift + 8));
      for (int64_t p = lo + tid; p < hi; p += nt) {
        const uint64_t k = select_key(val[p], idx[p]);
        if ((k & hmask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (tid < kWave) {
        // lane l holds digits 4l..4l+3; the digit of the need-th largest key
        // lies in the lane whose digits' keys, with all keys of higher
        // digits, first reach need
        int64_t c = 0;
        for (int j = 0; j < 4; ++j) c += hist[4 * lane + j];
        const int64_t incl = wave_inclusive_scan(c);
        const int64_t total = __shfl(incl, kWave - 1, kWave);
        const int64_t above = total - incl;  // keys in higher lanes' digits
        const bool here = above < need && need <= above + c;
        const unsigned long long b = __ballot(here);
        const int L = __ffsll(b) - 1;
        if (lane == L) {
          int64_t acc = above;
          int d = 4 * lane + 3;
          for (; d > 4 * lane; --d) {
            if (acc + hist[d] >= need) break;
            acc += hist[d];
          }
          prefix_s = prefix | (static_cast<uint64_t>(d) << shift);
          need_s = need - acc;
          // every key of digit d is kept: the keys >= prefix_s (lower bits
          // zero) are then exactly the S largest, and the search ends
          done_s = hist[d] == need - acc ? 1 : 0;
        }
      }
      __syncthreads();
      prefix = prefix_s;
      need = need_s;
      const bool done = done_s != 0;
      __syncthreads();  // prefix_s, done_s and hist are rewritten by the next pass
      if (done) break;
    }
    // the S keys >= prefix, in slice order
    int64_t base = out;
    for (int64_t p0 = lo; p0 < hi; p0 += nt) {
      const int64_t p = p0 + tid;
      int64_t keep = 0;
      int32_t id = 0;
      float v = 0.0f;
      if (p < hi) {
        id = idx[p];
        v = val[p];
        keep = select_key(v, id) >= prefix ? 1 : 0;
      }
      int64_t tot;
      const int64_t off = block_exclusive_scan(keep, tmp, &tot);
      if (keep) {
        new_idx[base + off] = id;
        new_val[base + off] = v;
      }
      base += tot;
    }
  }
}

hipError_t launch_select_count(const int64_t* ptr, int64_t nmajor, int64_t S, int64_t* new_ptr, hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const int nt = 256;
  hipLaunchKernelGGL(k_select_count, dim3(static_cast<unsigned>((nmajor + nt - 1) / nt)), dim3(nt), 0, s, ptr,
                     nmajor, S, new_ptr + 1);
  return hipGetLastError();
}

hipError_t launch_select_apply(const int64_t* ptr, const int32_t* idx, const float* val, int64_t nmajor, int64_t S,
                               const int64_t* new_ptr, int32_t* new_idx, float* new_val, hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const unsigned nb = static_cast<unsigned>(std::min<int64_t>(nmajor, 65536));
  hipLaunchKernelGGL(k_select_apply, dim3(nb), dim3(kSelectThreads), 0, s, ptr, idx, val, nmajor, S, new_ptr,
                     new_idx, new_val);
  return hipGetLastError();
}

hipError_t launch_prune_count(const int64_t* ptr, const float* val, int64_t nmajor, float thresh,
                              int64_t* new_ptr, hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = wave_grid(nmajor, nt);
  hipLaunchKernelGGL(k_prune_count, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, ptr, val,
                     nmajor, thresh, new_ptr + 1);
  return hipGetLastError();
}

hipError_t launch_prune_apply(const int64_t* ptr, const int32_t* idx, const float* val,
                              int64_t nmajor, float thresh, const int64_t* new_ptr,
                              int32_t* new_idx, float* new_val, hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = wave_grid(nmajor, nt);
  hipLaunchKernelGGL(k_prune_apply, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, ptr, idx, val,
                     nmajor, thresh, new_ptr, new_idx, new_val);
  return hipGetLastError();
}

}  // namespace spg
