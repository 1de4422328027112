// Host-side launchers of the gfx950 kernels (internal to libspg).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spg_device.h"

namespace spg {

constexpr int kNumBins = 64;
constexpr int kDenseBinBase = 16;  // bins >= this use a dense accumulator
constexpr int kScanTile = 8192;    // elements per scan block

// Operand check error bits (k_validate, k_flops_bin).
constexpr int kCheckEnds = 1;       // ptr[0] != 0 or ptr[last] != nnz
constexpr int kCheckOffsets = 2;    // a slice's offsets outside [0, nnz] or decreasing
constexpr int kCheckRange = 4;      // an id outside [0, minor dimension)
constexpr int kCheckUnsorted = 8;   // a descending pair of adjacent ids
constexpr int kCheckDuplicate = 16; // an equal pair of adjacent ids
constexpr int kCheckMalformed = kCheckEnds | kCheckOffsets | kCheckRange;

struct BinParams {
  int64_t hash_max_flops;  // symbolic: hash when flops <= this
  int64_t hash_max_nnz;    // numeric: hash when nnz <= this
  int64_t split_heavy;     // numeric: rows past hash_max_flops go as (row, panel) pieces
  const int32_t* row_slot; // numeric: rows with a kept bitmap (slot >= 0) are expanded
  int64_t rank_heavy;      // numeric: rows past hash_max_flops with more than
                           // hash_max_nnz entries go to the rank-panel kernel
  int64_t esc_max_flops;   // numeric: expand-sort-compress for rows with at most
  int64_t esc_ratio_x16;   // this many products and 16 * flops <= esc_ratio_x16 * nnz
};
constexpr int kExpandBin = 15;  // numeric bin of rows whose bitmap was kept
// Numeric bins kEscBinBase.. hold the expand-sort-compress classes of
// 32 << (bin - kEscBinBase) products (up to 8192); dense bins stay below.
constexpr int kEscBinBase = 55;
constexpr int kEscMaxFlops = 32 << (kNumBins - 1 - kEscBinBase);
static_assert(kDenseBinBase + 47 - 9 < kEscBinBase, "dense_bin stays below the expand-sort-compress bins");

// Pass shapes of the rank kernel: value slots and chunks per pass.
constexpr int kRankShapes = 6;
struct RankShapes {
  int n;
  int slots[kRankShapes];
  int maxc[kRankShapes];
  // rows the expand-sort-compress kernel takes (esc_max_flops > 0: flops per
  // row and the bounds of num_bin) are left out of the rank launches
  const int64_t* flops;
  int64_t esc_max_flops, esc_ratio_x16;
};
// A row the expand-sort-compress kernel takes.
__host__ __device__ inline bool esc_row(int64_t nnz, int64_t flops, int64_t esc_max_flops, int64_t esc_ratio_x16) {
  return esc_max_flops > 0 && nnz > 0 && flops <= esc_max_flops && 16 * flops <= esc_ratio_x16 * nnz;
}

// Symbolic bitmaps kept for the numeric phase of pattern-only products.
struct KeepBitmaps {
  uint32_t* store;           // capacity slots of nwords words; NULL: keep none
  int32_t* row_slot;         // per row: slot, or -1
  unsigned int* counter;     // next free slot (zeroed before the launch)
  const int64_t* flops;      // per row products
  int64_t min_flops;         // rows with fewer products are recomputed instead
  int64_t nwords;            // slot stride in words (a multiple of 4)
  unsigned int capacity;
};

struct BinOffsets {
  int64_t v[kNumBins];
};

__host__ __device__ inline int floor_log2_u64(uint64_t x) {
  int r = -1;
  while (x) {
    x >>= 1;
    ++r;
  }
  return r;
}
__host__ __device__ inline int ceil_log2_u64(uint64_t x) {
  return x <= 1 ? 0 : floor_log2_u64(x - 1) + 1;
}

// Hash classes 1..15 cover bound 32 << (c-1); dense classes 16..63 are
// ordered by decreasing flops so the heaviest rows are dispatched first.
__host__ __device__ inline int dense_bin(int64_t flops) {
  int fl = floor_log2_u64(static_cast<uint64_t>(flops));
  fl = fl > 47 ? 47 : fl;
  fl = fl < 9 ? 9 : fl;  // below the expand-sort-compress bins
  return kDenseBinBase + (47 - fl);
}
__host__ __device__ inline int esc_bin(int64_t flops) {
  const int c = ceil_log2_u64(static_cast<uint64_t>(flops));
  return kEscBinBase + (c < 5 ? 0 : c - 5);
}
__host__ __device__ inline int hash_class(int64_t bound) {
  const int c = ceil_log2_u64(static_cast<uint64_t>(bound));
  return (c < 5 ? 5 : c) - 4;
}
__host__ __device__ inline int sym_bin(int64_t flops, const BinParams& bp) {
  if (flops <= 0) return 0;
  if (flops <= bp.hash_max_flops) return hash_class(flops);
  return dense_bin(flops);
}
__host__ __device__ inline int num_bin(int64_t nnz, int64_t flops, const BinParams& bp) {
  if (nnz <= 0) return 0;
  if (esc_row(nnz, flops, bp.esc_max_flops, bp.esc_ratio_x16)) return esc_bin(flops);
  if (nnz <= bp.hash_max_nnz) return hash_class(nnz);
  return dense_bin(flops);
}
// One product of a batch, as the batched kernels see it.
struct BatchDesc {
  Operands op;             // oriented CSR problem
  int64_t* c_ptr;          // the product's row offsets inside the pooled array
  int32_t* c_idx;          // start of the product's ids in the pooled array
  void* c_val;             // start of the product's values in the pooled array
  const int32_t* psym;     // panel index for the symbolic bitmap (sym_P > 1)
  const int32_t* pnum;     // panel index for the numeric panels (num_P > 1)
  int32_t sym_wlog2, sym_P, num_wlog2, num_P;
  int32_t sr;              // kernel semiring code
  int32_t pad;
  int64_t a_nnz, b_nnz;    // entries of the oriented operands
};

// Hash table size and workgroup size of hash class c.
inline int hash_table_size(int c) { return 64 << (c - 1); }
inline int hash_threads(int c) {
  int t = hash_table_size(c) / 16;  // at most 16 slots per thread in the numeric compaction
  return t < 64 ? 64 : (t > 1024 ? 1024 : t);
}

// ---- launchers (all enqueue on `s`; return hipGetLastError()) ------------
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_validate(const int64_t* ptr, const int32_t* idx, int64_t nmajor, int64_t nnz,
                           int32_t nminor, int* err, hipStream_t s);
// Also checks A (error bits into *err); a_nnz = entries of A.
hipError_t launch_flops_bin(const Operands& op, int64_t a_nnz, BinParams bp, int64_t* flops, int64_t* c_ptr,
                            unsigned long long* counts, unsigned long long* total, int* err, hipStream_t s);
// Sorted copy of a CSR operand (ids ascending in every slice, values along;
// es = bytes per value, 0 or val NULL for none).  pos: int32 scratch indexed
// like idx.
hipError_t launch_sort_slices(const int64_t* ptr, const int32_t* idx, const void* val, int es, int64_t nmajor,
                              int32_t* out_idx, void* out_val, int32_t* pos, hipStream_t s);
// Rows [r0, m); scanned: c_ptr holds offsets (else c_ptr[i+1] is row i's nnz).
hipError_t launch_count_num_bins(int32_t m, int32_t r0, int scanned, const int64_t* flops, const int64_t* c_ptr,
                                 BinParams bp, unsigned long long* counts, hipStream_t s);
// Rows [r0, m).  mode 0: bins by flops; mode 1: bins by nnz = c_ptr[i+1]-c_ptr[i] (scanned)
hipError_t launch_scatter(int mode, int32_t m, int32_t r0, const int64_t* flops, const int64_t* c_ptr,
                          BinParams bp, const BinOffsets& offs, unsigned long long* cursors,
                          int32_t* rows_out, hipStream_t s);
hipError_t launch_panel_index(const int64_t* b_ptr, const int32_t* b_idx, int32_t nrows, int wlog2,
                              int P, int32_t* pidx, hipStream_t s);
// Inflation + renormalisation of every slice of a float32 matrix.
hipError_t launch_inflate(const int64_t* ptr, const float* val, int64_t nmajor, float r, float* val_out,
                          hipStream_t s);
// Selector of a semiring sum (see k_selector); sr is the kernel semiring code.
hipError_t launch_selector(int32_t m, int k, int64_t* ptr, int32_t* idx, void* val, int sr, hipStream_t s);
// (column id, value bits) pairs of B's entries, for 4-byte values.
hipError_t launch_interleave_b(const Operands& op, int64_t nnz, int2* out, hipStream_t s);
// Smallest and largest of n int32 values into mm[0..1] (device).
hipError_t launch_value_range(const int32_t* v, int64_t n, int32_t* mm, hipStream_t s);
// One word per entry of B (int32 values): value << bits | column id.
hipError_t launch_pack_b(const Operands& op, int64_t nnz, int bits, uint32_t* out, hipStream_t s);
// In-place inclusive scan of x[0..len); then x[-1] = 0 (x points one past a
// leading slot).  partials: ceil(len / kScanTile) + 1 int64.
hipError_t launch_scan_inplace(int64_t* x, int64_t len, int64_t* partials, hipStream_t s);

hipError_t launch_hash_sym(const Operands& op, const int32_t* rows, int64_t nrows, int T, int nt,
                           int short_seg, int64_t* c_ptr, hipStream_t s);
hipError_t launch_dense_sym(const Operands& op, const int32_t* rows, int64_t nrows, int wlog2, int P,
                            const int32_t* pidx, int nt, int short_seg, int64_t* c_ptr,
                            hipStream_t s, int sub_wlog2 = 0, int subP = 0, int32_t* sub_cnt = nullptr,
                            KeepBitmaps kb = KeepBitmaps{});
// Windowed dense symbolic rows: (row, window) items over P windows of
// 2^wlog2 columns, one queue per window (queue: P uint32, zeroed here), a
// workgroup starting on its XCD's window; item_cnt[it * P + w] per item,
// then c_ptr[row + 1] = the row's total.  sub_cnt (optional): counts of the
// rank chunks of 2^sub_wlog2 columns, subP per row.  keep_slot (optional):
// per row a kept-bitmap slot or -1, slots of keep_nwords words.  The grid is
// wg_per_cu workgroups per compute unit.
hipError_t launch_dense_sym_win(const Operands& op, const int32_t* rows, int64_t nrows, int wlog2, int P,
                                const int32_t* pidx, int nt, int short_seg, int32_t* item_cnt,
                                unsigned int* queue, int64_t* c_ptr, int sub_wlog2, int subP, int32_t* sub_cnt,
                                const int32_t* keep_slot, uint32_t* keep_store, int64_t keep_nwords,
                                int wg_per_cu, hipStream_t s);
// Kept-bitmap slots for the rows of a list in list order: rows with at least
// min_flops products take slots 0, 1, ... while capacity lasts, the others
// -1.  flag: int64[nrows + 1] scratch; partials: scan partials.
hipError_t launch_keep_slots(const int32_t* rows, int64_t nrows, const int64_t* flops, int64_t min_flops,
                             int64_t capacity, int64_t* flag, int64_t* partials, int32_t* row_slot, hipStream_t s);
hipError_t launch_expand_rows(const int32_t* rows, int64_t nrows, int nwords, int64_t stride, const uint32_t* store,
                              const int32_t* row_slot, const int64_t* c_ptr, int32_t* c_idx, int nt,
                              hipStream_t s);
// (row, panel) pieces: offsets within rows + bin counts, then the item lists.
hipError_t launch_sub_prepare(int64_t nslots, int subP, int32_t* cnt, int32_t* off, int32_t* wend,
                              BinParams bp, unsigned long long* counts, hipStream_t s);
hipError_t launch_sub_scatter(int64_t nslots, int subP, const int32_t* cnt, BinParams bp,
                              const BinOffsets& offs, unsigned long long* cursors, int32_t* items,
                              hipStream_t s);
hipError_t launch_hash_num_sub(int sr, const Operands& op, const int32_t* rows, const int32_t* items,
                               int64_t nitems, int T, int nt, int short_seg, int subP, int sub_wlog2,
                               const int32_t* pidx, const int32_t* cnt, const int32_t* off,
                               const int32_t* wend, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                               hipStream_t s);
hipError_t launch_dense_num_sub(int sr, const Operands& op, const int32_t* rows, const int32_t* items,
                                int64_t nitems, int nt, int short_seg, int subP, int sub_wlog2,
                                const int32_t* pidx, const int32_t* cnt, const int32_t* off,
                                const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s);
// Expand-sort-compress rows of one class (N = 32 << class products at most):
// every product at its own LDS position, a bitonic sort by column, equal
// columns combined.  sr as for launch_hash_num.
// Threads of an expand-sort-compress class of N products: N / 4 (at most
// 1024), so each thread holds R = N / threads of them, 4 or 8.
inline int esc_threads(int N) { return N / 4 < 64 ? 64 : (N / 4 > 1024 ? 1024 : N / 4); }
inline int esc_per_thread(int N) { return N / esc_threads(N) > 4 ? N / esc_threads(N) : 4; }
// The largest class (products per row) the expand-sort-compress kernel holds
// in LDS for semiring code sr.
int esc_class_limit(int sr);
hipError_t launch_esc_num(int sr, const Operands& op, const int32_t* rows, int64_t nrows, int N,
                          const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s);
// sr: semiring code 0..6, or 7 for the pattern-only boolean product.
hipError_t launch_hash_num(int sr, const Operands& op, const int32_t* rows, int64_t nrows, int T,
                           int nt, int short_seg, const int64_t* c_ptr, int32_t* c_idx,
                           void* c_val, hipStream_t s);
hipError_t launch_dense_num(int sr, const Operands& op, const int32_t* rows, int64_t nrows,
                            int wlog2, int P, const int32_t* pidx, int nt, int short_seg,
                            const int64_t* c_ptr, int32_t* c_idx, void* c_val, hipStream_t s);
// Heavy valued rows (the dense symbolic list, slot order) through rank-compressed
// panels: chunks of 2^cw columns, rcnt[slot*NC + c] entries per chunk, pchunk
// the chunk index of B; only rows in [rb, re) with nnz in [nnz_lo, nnz_hi).
// fixed: by fixed panels of 2^wlog2 columns (P of them) over the same index;
// otherwise by passes of one of sh.n shapes (at most sh.maxc[j] chunks and
// sh.slots[j] >= 2^cw value slots), each row taking the shape that needs the
// fewest passes.  Rows with a kept symbolic bitmap (keep_slot[row] >= 0,
// slots of keep_nwords words in keep_store) read their pattern from it.
hipError_t launch_rank_num(int sr, bool fixed, const Operands& op, const int32_t* rows, int64_t nrows, int32_t rb,
                           int32_t re, int cw, int NC, const RankShapes& sh,
                           const int32_t* pchunk, const int32_t* rcnt, int64_t nnz_lo,
                           int64_t nnz_hi, int wlog2, int P, int nt, int short_seg, const uint32_t* keep_store,
                           const int32_t* keep_slot, int64_t keep_nwords, const int64_t* c_ptr,
                           int32_t* c_idx, void* c_val, hipStream_t s);
size_t rank_num_lds(int sr, int cw, int slots, int max_chunks, int wlog2, int nt);
size_t rank_pass_lds(int sr, int cw, int slots, int max_chunks, int nt);  // the rank passes alone
hipError_t launch_hash_sym_b(const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                             const int32_t* items, int64_t nitems, int T, int nt, int short_seg,
                             hipStream_t s);
hipError_t launch_dense_sym_b(const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                              const int32_t* items, int64_t nitems, int wlog2_max, int nt,
                              int short_seg, hipStream_t s);
// Expand-sort-compress over the batch's rows of one class of N products.
hipError_t launch_esc_num_b(int sr, const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod, const int32_t* items,
                            int64_t nitems, int N, hipStream_t s);
hipError_t launch_hash_num_b(int sr, const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                             const int32_t* items, int64_t nitems, int T, int nt, int short_seg,
                             hipStream_t s);
hipError_t launch_dense_num_b(int sr, const BatchDesc* descs, const int64_t* row_off, const int32_t* prod_of, int nprod,
                              const int32_t* items, int64_t nitems, int wlog2_max, int nt,
                              int short_seg, hipStream_t s);
// Segment lists of (row, panel) pieces.
hipError_t launch_seg_count(const Operands& op, const int32_t* rows, int64_t nslots, int P,
                            const int32_t* pidx, const int32_t* wend, int64_t* cnt_out, hipStream_t s);
hipError_t launch_seg_write(const Operands& op, const int32_t* rows, int64_t nslots, int P,
                            const int32_t* pidx, const int32_t* wend, const int64_t* segoff, void* segs,
                            hipStream_t s);
hipError_t launch_hash_num_seg(int sr, const Operands& op, const int32_t* rows, const int32_t* items,
                               int64_t nitems, int T, int nt, int short_seg, int subP, int sub_wlog2,
                               const int64_t* segoff, const void* segs, const int32_t* cnt,
                               const int32_t* off, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                               hipStream_t s);
hipError_t launch_dense_num_seg(int sr, const Operands& op, const int32_t* rows, const int32_t* items,
                                int64_t nitems, int nt, int short_seg, int subP, int sub_wlog2,
                                const int64_t* segoff, const void* segs, const int32_t* cnt,
                                const int32_t* off, const int64_t* c_ptr, int32_t* c_idx, void* c_val,
                                hipStream_t s);
size_t seg_desc_bytes();
size_t storage_bytes(int sr);  // bytes per LDS accumulator value (0 for pattern)
int hash_threads_num(int c, int sr);  // workgroup size of numeric hash class c
size_t hash_num_lds(int sr, int T, int nt);
size_t dense_num_lds(int sr, int wlog2, int nt);
size_t dense_sym_lds(int wlog2, int nt);
size_t hash_sym_lds(int T, int nt);
int max_lds_bytes();

// Selection: new_ptr[s + 1] = min(nnz of slice s, S) (count), then the kept
// entries of every slice (apply; new_ptr scanned).
hipError_t launch_select_count(const int64_t* ptr, int64_t nmajor, int64_t S, int64_t* new_ptr, hipStream_t s);
hipError_t launch_select_apply(const int64_t* ptr, const int32_t* idx, const float* val, int64_t nmajor, int64_t S,
                               const int64_t* new_ptr, int32_t* new_idx, float* new_val, hipStream_t s);
hipError_t launch_prune_count(const int64_t* ptr, const float* val, int64_t nmajor, float thresh,
                              int64_t* new_ptr, hipStream_t s);
hipError_t launch_prune_apply(const int64_t* ptr, const int32_t* idx, const float* val,
                              int64_t nmajor, float thresh, const int64_t* new_ptr,
                              int32_t* new_idx, float* new_val, hipStream_t s);

}  // namespace spg
