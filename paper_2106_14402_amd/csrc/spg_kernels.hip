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

#include "spg_launch.h"

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

// Operand check: ptr[0] == 0, ptr non-decreasing within [0, nnz],
// ptr[nmajor] == nnz, ids in [0, nminor) and strictly ascending per slice.
// Error bits: 1 bad endpoints, 2 bad offsets, 4 id out of range, 8 unsorted
// or duplicate ids.  One wave per slice; never reads outside [0, nnz).
__global__ void k_validate(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                           int64_t nmajor, int64_t nnz, int32_t nminor, int* err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t s = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (s >= nmajor) return;
  int e = 0;
  if (lane == 0) {
    if (s == 0 && ptr[0] != 0) e |= 1;
    if (s == nmajor - 1 && ptr[nmajor] != nnz) e |= 1;
  }
  const int64_t lo = ptr[s], hi = ptr[s + 1];
  if (lo < 0 || hi > nnz || hi < lo) {
    e |= 2;
  } else {
    for (int64_t q = lo + lane; q < hi; q += kWave) {
      const int32_t c = idx[q];
      if (c < 0 || c >= nminor) e |= 4;
      if (q > lo && idx[q - 1] >= c) e |= 8;
    }
  }
  if (e) atomicOr(err, e);
}

hipError_t launch_validate(const int64_t* ptr, const int32_t* idx, int64_t nmajor, int64_t nnz,
                           int32_t nminor, int* err, hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = (nmajor + nt / kWave - 1) / (nt / kWave);
  hipLaunchKernelGGL(k_validate, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, ptr, idx, nmajor,
                     nnz, nminor, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Flop count and binning (paper Sec. 4.1 phase 1: estimate the flops of every
// output slice before splitting the work).  flops_i = sum over A(i,k) of
// nnz(B(k,:)).  One wave per row.
// ---------------------------------------------------------------------------
__global__ void k_flops_bin(Operands op, BinParams bp, int64_t* __restrict__ flops,
                            int64_t* __restrict__ c_ptr, unsigned long long* counts,
                            unsigned long long* total) {
  __shared__ unsigned int lc[kNumBins];
  __shared__ unsigned long long ltot;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  if (tid < kNumBins) lc[tid] = 0;
  if (tid == 0) ltot = 0;
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (tid >> 6);
  if (i < op.m) {
    int64_t f = 0;
    for (int64_t p = op.a_ptr[i] + lane; p < op.a_ptr[i + 1]; p += kWave) {
      const int32_t k = op.a_idx[p];
      f += op.b_ptr[k + 1] - op.b_ptr[k];
    }
    f = wave_sum(f);
    if (lane == 0) {
      flops[i] = f;
      if (f == 0) c_ptr[i + 1] = 0;
      atomicAdd(&lc[sym_bin(f, bp)], 1u);
      atomicAdd(&ltot, static_cast<unsigned long long>(f));
    }
  }
  __syncthreads();
  if (tid < kNumBins && lc[tid]) atomicAdd(&counts[tid], static_cast<unsigned long long>(lc[tid]));
  if (tid == 0 && ltot) atomicAdd(total, ltot);
}

hipError_t launch_flops_bin(const Operands& op, BinParams bp, int64_t* flops, int64_t* c_ptr,
                            unsigned long long* counts, unsigned long long* total, hipStream_t s) {
  if (op.m <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = (static_cast<int64_t>(op.m) + nt / kWave - 1) / (nt / kWave);
  hipLaunchKernelGGL(k_flops_bin, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, op, bp, flops,
                     c_ptr, counts, total);
  return hipGetLastError();
}

// Numeric bin counts; c_ptr[i+1] still holds nnz of row i (before the scan).
__global__ void k_count_num_bins(int32_t m, const int64_t* __restrict__ flops,
                                 const int64_t* __restrict__ c_ptr, BinParams bp,
                                 unsigned long long* counts) {
  __shared__ unsigned int lc[kNumBins];
  const int tid = threadIdx.x;
  if (tid < kNumBins) lc[tid] = 0;
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + tid;
  if (i < m) atomicAdd(&lc[num_bin(c_ptr[i + 1], flops[i], bp)], 1u);
  __syncthreads();
  if (tid < kNumBins && lc[tid]) atomicAdd(&counts[tid], static_cast<unsigned long long>(lc[tid]));
}

hipError_t launch_count_num_bins(int32_t m, const int64_t* flops, const int64_t* c_ptr, BinParams bp,
                                 unsigned long long* counts, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int nt = 256;
  hipLaunchKernelGGL(k_count_num_bins, dim3((m + nt - 1) / nt), dim3(nt), 0, s, m, flops, c_ptr, bp,
                     counts);
  return hipGetLastError();
}

// Row lists per bin.  Each block reserves one range per bin with a single
// global atomic; row order inside a bin is unspecified.
__global__ void k_scatter(int mode, int32_t m, const int64_t* __restrict__ flops,
                          const int64_t* __restrict__ c_ptr, BinParams bp, BinOffsets offs,
                          unsigned long long* cursors, int32_t* __restrict__ rows_out) {
  __shared__ unsigned int lc[kNumBins];
  __shared__ unsigned long long lbase[kNumBins];
  const int tid = threadIdx.x;
  if (tid < kNumBins) lc[tid] = 0;
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + tid;
  int bin = 0;
  unsigned int local = 0;
  if (i < m) {
    bin = mode == 0 ? sym_bin(flops[i], bp) : num_bin(c_ptr[i + 1] - c_ptr[i], flops[i], bp);
    if (bin > 0) local = atomicAdd(&lc[bin], 1u);
  }
  __syncthreads();
  if (tid < kNumBins && lc[tid])
    lbase[tid] = atomicAdd(&cursors[tid], static_cast<unsigned long long>(lc[tid]));
  __syncthreads();
  if (bin > 0) rows_out[offs.v[bin] + static_cast<int64_t>(lbase[bin]) + local] = static_cast<int32_t>(i);
}

hipError_t launch_scatter(int mode, int32_t m, const int64_t* flops, const int64_t* c_ptr,
                          BinParams bp, const BinOffsets& offs, unsigned long long* cursors,
                          int32_t* rows_out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int nt = 256;
  hipLaunchKernelGGL(k_scatter, dim3((m + nt - 1) / nt), dim3(nt), 0, s, mode, m, flops, c_ptr, bp,
                     offs, cursors, rows_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Panel index: for B row k and panel p (columns [p*W, (p+1)*W)),
// pidx[k*(P+1) + p] = number of entries of B(k,:) with column < p*W.  Rows
// must be sorted.  One wave per row; every slot is written exactly once.
// ---------------------------------------------------------------------------
__global__ void k_panel_index(const int64_t* __restrict__ b_ptr, const int32_t* __restrict__ b_idx,
                              int32_t nrows, int wlog2, int P, int32_t* __restrict__ pidx) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t k = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (k >= nrows) return;
  const int64_t lo = b_ptr[k], hi = b_ptr[k + 1];
  int32_t* out = pidx + k * (P + 1);
  for (int64_t q = lo + lane; q < hi; q += kWave) {
    const int cp = b_idx[q] >> wlog2;
    const int pp = q == lo ? -1 : (b_idx[q - 1] >> wlog2);
    for (int p = pp + 1; p <= cp; ++p) out[p] = static_cast<int32_t>(q - lo);
  }
  if (lane == 0) {
    const int lp = hi > lo ? (b_idx[hi - 1] >> wlog2) : -1;
    for (int p = lp + 1; p <= P; ++p) out[p] = static_cast<int32_t>(hi - lo);
  }
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

__device__ int64_t hash_sym_row(const Operands& op, int32_t row, int T, int short_seg,
                                unsigned char* smem) {
  const int nt = blockDim.x;
  auto q = PatQueue::carve(smem, nt);
  int32_t* keys = reinterpret_cast<int32_t*>(smem + PatQueue::bytes(nt));
  for (int t = threadIdx.x; t < T; t += nt) keys[t] = kEmpty;
  __syncthreads();
  HashSetSink sink{keys, static_cast<uint32_t>(T - 1), 0};
  enumerate_row<SrPattern>(op, op.a_ptr[row], op.a_ptr[row + 1], false, nullptr, 1, 0, 0, short_seg,
                           q, sink);
  return block_sum(sink.count, q.ctr + 2);
}

__device__ int64_t dense_sym_row(const Operands& op, int32_t row, int wlog2, int P,
                                 const int32_t* __restrict__ pidx, int short_seg, unsigned char* smem) {
  const int nt = blockDim.x;
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
    int cnt = 0;
    for (int t = threadIdx.x; t < nwords; t += nt) cnt += __popc(bits[t]);
    total += block_sum(cnt, q.ctr + 2);
  }
  return total;
}

// Product of global row r in a batch: the last b with row_off[b] <= r.
__device__ __forceinline__ int batch_product(const int64_t* __restrict__ row_off, int nprod, int64_t r) {
  int lo = 0, hi = nprod;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (row_off[mid] <= r)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(1024) void k_hash_sym(Operands op, const int32_t* __restrict__ rows,
                                                   int64_t nrows, int T, int short_seg,
                                                   int64_t* __restrict__ c_ptr) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = rows[it];
    const int64_t nz = hash_sym_row(op, row, T, short_seg, smem);
    if (threadIdx.x == 0) c_ptr[row + 1] = nz;
  }
}

__global__ __launch_bounds__(1024) void k_dense_sym(Operands op, const int32_t* __restrict__ rows,
                                                    int64_t nrows, int wlog2, int P,
                                                    const int32_t* __restrict__ pidx, int short_seg,
                                                    int64_t* __restrict__ c_ptr) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = rows[it];
    const int64_t nz = dense_sym_row(op, row, wlog2, P, pidx, short_seg, smem);
    if (threadIdx.x == 0) c_ptr[row + 1] = nz;
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_hash_sym_b(const BatchDesc* __restrict__ descs,
                                                     const int64_t* __restrict__ row_off, int nprod,
                                                     const int32_t* __restrict__ items, int64_t nitems,
                                                     int T, int short_seg) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t r = items[it];
    const int b = batch_product(row_off, nprod, r);
    const BatchDesc& d = descs[b];
    const int32_t row = static_cast<int32_t>(r - row_off[b]);
    const int64_t nz = hash_sym_row(d.op, row, T, short_seg, smem);
    if (threadIdx.x == 0) d.c_ptr[row + 1] = nz;
  }
}

__global__ __launch_bounds__(1024) void k_dense_sym_b(const BatchDesc* __restrict__ descs,
                                                      const int64_t* __restrict__ row_off, int nprod,
                                                      const int32_t* __restrict__ items, int64_t nitems,
                                                      int short_seg) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t r = items[it];
    const int b = batch_product(row_off, nprod, r);
    const BatchDesc& d = descs[b];
    const int32_t row = static_cast<int32_t>(r - row_off[b]);
    const int64_t nz = dense_sym_row(d.op, row, d.sym_wlog2, d.sym_P, d.psym, short_seg, smem);
    if (threadIdx.x == 0) d.c_ptr[row + 1] = nz;
    __syncthreads();
  }
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
                            hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_sym, dim3(grid_for(nrows, 0)), dim3(nt), dense_sym_lds(wlog2, nt), s, op,
                     rows, nrows, wlog2, P, pidx, short_seg, c_ptr);
  return hipGetLastError();
}

hipError_t launch_hash_sym_b(const BatchDesc* descs, const int64_t* row_off, int nprod,
                             const int32_t* items, int64_t nitems, int T, int nt, int short_seg,
                             int64_t grid_cap, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_sym_b, dim3(grid_for(nitems, grid_cap)), dim3(nt), hash_sym_lds(T, nt), s,
                     descs, row_off, nprod, items, nitems, T, short_seg);
  return hipGetLastError();
}

hipError_t launch_dense_sym_b(const BatchDesc* descs, const int64_t* row_off, int nprod,
                              const int32_t* items, int64_t nitems, int wlog2_max, int nt,
                              int short_seg, int64_t grid_cap, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_sym_b, dim3(grid_for(nitems, grid_cap)), dim3(nt),
                     dense_sym_lds(wlog2_max, nt), s, descs, row_off, nprod, items, nitems, short_seg);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Numeric phase (paper Sec. 4.1 phase 3).
// ---------------------------------------------------------------------------
template <class S>
__device__ void bitonic_sort(int32_t* keys, S* vals, int N, bool with_vals) {
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < (N >> 1); t += blockDim.x) {
        const int i = 2 * t - (t & (j - 1));
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
      __syncthreads();
    }
  }
}

constexpr int kMaxSlotsPerThread = 16;

// LDS hash accumulator for one row, then compaction, bitonic sort and
// coalesced stores of the row's entries into [out, out_end).
template <class SR>
__device__ void hash_num_row(const Operands& op, int32_t row, int T, int short_seg, int64_t out,
                             int64_t out_end, int32_t* __restrict__ c_idx,
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
  enumerate_row<SR>(op, op.a_ptr[row], op.a_ptr[row + 1], false, nullptr, 1, 0, 0, short_seg, q,
                    sink);
  // Compact occupied slots to the front: every thread takes a contiguous
  // block of T/nt slots into registers, then writes them at its scanned offset.
  const int per = T / nt;
  int32_t kr[kMaxSlotsPerThread];
  S vr[kMaxSlotsPerThread];
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < kMaxSlotsPerThread; ++r) {
    kr[r] = kEmpty;
    if (r < per) {
      const int slot = tid * per + r;
      kr[r] = keys[slot];
      if constexpr (!SR::kPattern) vr[r] = vals[slot];
      cnt += kr[r] != kEmpty;
    }
  }
  int nnz;
  int o = block_exclusive_scan(cnt, q.ctr + 2, &nnz);
#pragma unroll
  for (int r = 0; r < kMaxSlotsPerThread; ++r) {
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
    c_idx[out + e] = keys[e];
    if constexpr (!SR::kPattern) c_val[out + e] = SR::out(vals[e]);
  }
  __syncthreads();
}

// Dense LDS panel accumulator for one row: presence bits plus one value per
// column of the panel, emitted in column order into [out, out_end).
template <class SR>
__device__ void dense_num_row(const Operands& op, int32_t row, int wlog2, int P,
                              const int32_t* __restrict__ pidx, int short_seg, int64_t out,
                              int64_t out_end, int32_t* __restrict__ c_idx,
                              typename SR::Out* __restrict__ c_val, unsigned char* smem) {
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
  const int64_t a_lo = op.a_ptr[row], a_hi = op.a_ptr[row + 1];
  const int32_t wcols_max = min(W, op.k);
  for (int t = tid; t < (wcols_max + 31) >> 5; t += nt) bits[t] = 0u;
  if constexpr (!SR::kPattern) {
    for (int t = tid; t < wcols_max; t += nt) vals[t] = SR::identity();
  }
  __syncthreads();
  for (int p = 0; p < P; ++p) {
    const int32_t c0 = p << wlog2;
    const int32_t wcols = min(W, op.k - c0);
    const int nwords = (wcols + 31) >> 5;
    DenseSink<SR> sink{bits, vals};
    enumerate_row<SR>(op, a_lo, a_hi, P > 1, pidx, P, p, c0, short_seg, q, sink);
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

template <class SR>
__global__ __launch_bounds__(1024) void k_hash_num(Operands op, const int32_t* __restrict__ rows,
                                                   int64_t nrows, int T, int short_seg,
                                                   const int64_t* __restrict__ c_ptr,
                                                   int32_t* __restrict__ c_idx,
                                                   typename SR::Out* __restrict__ c_val) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nrows; it += gridDim.x) {
    const int32_t row = rows[it];
    hash_num_row<SR>(op, row, T, short_seg, c_ptr[row], c_ptr[row + 1], c_idx, c_val, smem);
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
    const int32_t row = rows[it];
    dense_num_row<SR>(op, row, wlog2, P, pidx, short_seg, c_ptr[row], c_ptr[row + 1], c_idx, c_val,
                      smem);
  }
}

template <class SR>
__global__ __launch_bounds__(1024) void k_hash_num_b(const BatchDesc* __restrict__ descs,
                                                     const int64_t* __restrict__ row_off, int nprod,
                                                     const int32_t* __restrict__ items, int64_t nitems,
                                                     int T, int short_seg) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t r = items[it];
    const int b = batch_product(row_off, nprod, r);
    const BatchDesc& d = descs[b];
    const int32_t row = static_cast<int32_t>(r - row_off[b]);
    hash_num_row<SR>(d.op, row, T, short_seg, d.c_ptr[row], d.c_ptr[row + 1], d.c_idx,
                     static_cast<typename SR::Out*>(d.c_val), smem);
  }
}

template <class SR>
__global__ __launch_bounds__(1024) void k_dense_num_b(const BatchDesc* __restrict__ descs,
                                                      const int64_t* __restrict__ row_off, int nprod,
                                                      const int32_t* __restrict__ items, int64_t nitems,
                                                      int short_seg) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t r = items[it];
    const int b = batch_product(row_off, nprod, r);
    const BatchDesc& d = descs[b];
    const int32_t row = static_cast<int32_t>(r - row_off[b]);
    dense_num_row<SR>(d.op, row, d.num_wlog2, d.num_P, d.pnum, short_seg, d.c_ptr[row],
                      d.c_ptr[row + 1], d.c_idx, static_cast<typename SR::Out*>(d.c_val), smem);
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
static hipError_t hash_num_b_t(const BatchDesc* descs, const int64_t* row_off, int nprod,
                               const int32_t* items, int64_t nitems, int T, int nt, int short_seg,
                               int64_t grid_cap, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_num_b<SR>, dim3(grid_for(nitems, grid_cap)), dim3(nt),
                     hash_num_lds_t<SR>(T, nt), s, descs, row_off, nprod, items, nitems, T, short_seg);
  return hipGetLastError();
}

template <class SR>
static hipError_t dense_num_b_t(const BatchDesc* descs, const int64_t* row_off, int nprod,
                                const int32_t* items, int64_t nitems, int wlog2_max, int nt,
                                int short_seg, int64_t grid_cap, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_num_b<SR>, dim3(grid_for(nitems, grid_cap)), dim3(nt),
                     dense_num_lds_t<SR>(wlog2_max, nt), s, descs, row_off, nprod, items, nitems,
                     short_seg);
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

hipError_t launch_dense_num(int sr, const Operands& op, const int32_t* rows, int64_t nrows,
                            int wlog2, int P, const int32_t* pidx, int nt, int short_seg,
                            const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s) {
  SPG_DISPATCH(sr, dense_num_t, op, rows, nrows, wlog2, P, pidx, nt, short_seg, c_ptr, c_idx, c_val,
               s)
}

hipError_t launch_hash_num_b(int sr, const BatchDesc* descs, const int64_t* row_off, int nprod,
                             const int32_t* items, int64_t nitems, int T, int nt, int short_seg,
                             int64_t grid_cap, hipStream_t s) {
  SPG_DISPATCH(sr, hash_num_b_t, descs, row_off, nprod, items, nitems, T, nt, short_seg, grid_cap, s)
}

hipError_t launch_dense_num_b(int sr, const BatchDesc* descs, const int64_t* row_off, int nprod,
                              const int32_t* items, int64_t nitems, int wlog2_max, int nt,
                              int short_seg, int64_t grid_cap, hipStream_t s) {
  SPG_DISPATCH(sr, dense_num_b_t, descs, row_off, nprod, items, nitems, wlog2_max, nt, short_seg,
               grid_cap, s)
}

size_t hash_num_lds(int sr, int T, int nt) { SPG_DISPATCH(sr, hash_num_lds_t, T, nt) }
size_t dense_num_lds(int sr, int wlog2, int nt) { SPG_DISPATCH(sr, dense_num_lds_t, wlog2, nt) }

template <class SR>
static size_t storage_bytes_t() {
  return SR::kPattern ? 0 : sizeof(typename SR::S);
}
size_t storage_bytes(int sr) { SPG_DISPATCH(sr, storage_bytes_t) }

int max_lds_bytes() { return 160 * 1024; }

// ---------------------------------------------------------------------------
// Prune (Markov-clustering step after expansion): keep value >= thresh.
// ---------------------------------------------------------------------------
__global__ void k_prune_count(const int64_t* __restrict__ ptr, const float* __restrict__ val,
                              int64_t nmajor, float thresh, int64_t* __restrict__ cnt) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t s = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (s >= nmajor) return;
  int64_t c = 0;
  for (int64_t p = ptr[s] + lane; p < ptr[s + 1]; p += kWave) c += val[p] >= thresh;
  c = wave_sum(c);
  if (lane == 0) cnt[s] = c;
}

__global__ void k_prune_apply(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                              const float* __restrict__ val, int64_t nmajor, float thresh,
                              const int64_t* __restrict__ new_ptr, int32_t* __restrict__ new_idx,
                              float* __restrict__ new_val) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t s = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (s >= nmajor) return;
  int64_t o = new_ptr[s];
  const int64_t hi = ptr[s + 1];
  for (int64_t b = ptr[s]; b < hi; b += kWave) {
    const int64_t p = b + lane;
    const bool keep = p < hi && val[p] >= thresh;
    const unsigned long long m = __ballot(keep);
    if (keep) {
      const int before = __popcll(m & ((1ull << lane) - 1ull));
      new_idx[o + before] = idx[p];
      new_val[o + before] = val[p];
    }
    o += __popcll(m);
  }
}

hipError_t launch_prune_count(const int64_t* ptr, const float* val, int64_t nmajor, float thresh,
                              int64_t* new_ptr, hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = (nmajor + nt / kWave - 1) / (nt / kWave);
  hipLaunchKernelGGL(k_prune_count, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, ptr, val,
                     nmajor, thresh, new_ptr + 1);
  return hipGetLastError();
}

hipError_t launch_prune_apply(const int64_t* ptr, const int32_t* idx, const float* val,
                              int64_t nmajor, float thresh, const int64_t* new_ptr,
                              int32_t* new_idx, float* new_val, hipStream_t s) {
  if (nmajor <= 0) return hipSuccess;
  const int nt = 256;
  const int64_t nb = (nmajor + nt / kWave - 1) / (nt / kWave);
  hipLaunchKernelGGL(k_prune_apply, dim3(static_cast<unsigned>(nb)), dim3(nt), 0, s, ptr, idx, val,
                     nmajor, thresh, new_ptr, new_idx, new_val);
  return hipGetLastError();
}

}  // namespace spg
