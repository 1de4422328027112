// Batched products: many independent C_b = A_b (x).(+) B_b in one pass.
//
// Stand-in for the block products of one 3D Sparse SUMMA stage or a set of
// per-graph squares (paper Sec. 3: local multiplies inside 2D/3D SUMMA;
// Sec. 5: GPU offload of the per-stage local products).  Rows of all
// products form one global row space; binning, the symbolic phase and the
// numeric phase each run one grid-stride launch per accumulator class (and
// semiring) over the rows of every product, and the numeric phase can be
// captured once into a hipGraph and replayed.  Semiring arithmetic is the
// same device code as the single-product path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/spg.h"
#include "spg_launch.h"
#include "spg_rowlogic.h"

using namespace spg;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
constexpr int kMaxSlots = 8;                    // distinct kernel semirings in a batch
constexpr int kBatchBins = kNumBins * kMaxSlots;

// ---------------------------------------------------------------------------
// Batched preparation kernels over the global row space.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_segment(const int64_t* __restrict__ off, int n, int64_t r) {
  int lo = 0, hi = n;  // last b with off[b] <= r
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= r)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Product of every global row: block b writes b over its product's rows
// [off[b], off[b + 1]) (the row kernels' lookup, instead of a search per row).
__global__ void kb_fill_prod(const int64_t* __restrict__ off, int32_t* __restrict__ prod) {
  const int b = blockIdx.x;
  for (int64_t r = off[b] + threadIdx.x; r < off[b + 1]; r += blockDim.x) prod[r] = b;
}

// Operand check of every product (the checks of k_validate, error bits into
// *err): global slices [0, mtot) are the A slices, [mtot, mtot + ntot) the
// B slices; each wave takes slices g = its index, + all waves, ... (a grid
// of a few workgroups per compute unit, not one per slice).
__global__ void kb_validate(const BatchDesc* __restrict__ d, const int64_t* __restrict__ row_off,
                            const int64_t* __restrict__ brow_off, const int32_t* __restrict__ prod_of,
                            const int32_t* __restrict__ bprod_of, int64_t mtot, int64_t ntot, int* err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
  int e = 0;
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6);
       g < mtot + ntot; g += waves) {
    const bool is_a = g < mtot;
    const int b = is_a ? prod_of[g] : bprod_of[g - mtot];
    const Operands& op = d[b].op;
    const int64_t s = is_a ? g - row_off[b] : g - mtot - brow_off[b];
    const int64_t nmajor = is_a ? op.m : op.n;
    const int64_t nnz = is_a ? d[b].a_nnz : d[b].b_nnz;
    const int32_t nminor = is_a ? op.n : op.k;
    const int64_t* ptr = is_a ? op.a_ptr : op.b_ptr;
    const int32_t* idx = is_a ? op.a_idx : op.b_idx;
    if (lane == 0) {
      if (s == 0 && ptr[0] != 0) e |= kCheckEnds;
      if (s == nmajor - 1 && ptr[nmajor] != nnz) e |= kCheckEnds;
    }
    const int64_t lo = ptr[s], hi = ptr[s + 1];
    if (lo < 0 || hi > nnz || hi < lo) {
      e |= kCheckOffsets;
    } else {
      // eight groups of 64 ids loaded at once; an id's predecessor comes from
      // the lane below (lane 0: one more load)
      constexpr int U = 8;
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
            if (q > lo && b >= c[u]) e |= b > c[u] ? kCheckUnsorted : kCheckDuplicate;
          }
        }
      }
    }
  }
  e = wave_or(e);
  if (lane == 0 && e) atomicOr(err, e);
}

// flops per global row, symbolic bin counts, zero nnz for empty rows; a
// wave per row, rows strided over a grid of a few workgroups per compute unit.
__global__ void kb_flops_bin(const BatchDesc* __restrict__ d, const int64_t* __restrict__ row_off,
                             int nprod, int64_t mtot, BinParams bp, int64_t* __restrict__ flops,
                             const int32_t* __restrict__ prod_of, unsigned long long* counts,
                             unsigned long long* total) {
  __shared__ unsigned int lc[kNumBins];
  __shared__ unsigned long long ltot;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  if (tid < kNumBins) lc[tid] = 0;
  if (tid == 0) ltot = 0;
  __syncthreads();
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (tid >> 6); r < mtot; r += waves) {
    const int b = prod_of[r];
    const Operands& op = d[b].op;
    const int64_t i = r - row_off[b];
    int64_t f = 0;
    for (int64_t p = op.a_ptr[i] + lane; p < op.a_ptr[i + 1]; p += kWave) {
      const int32_t k = op.a_idx[p];
      f += op.b_ptr[k + 1] - op.b_ptr[k];
    }
    f = wave_sum(f);
    if (lane == 0) {
      flops[r] = f;
      if (f == 0) d[b].c_ptr[i + 1] = 0;
      atomicAdd(&lc[sym_bin(f, bp)], 1u);
      atomicAdd(&ltot, static_cast<unsigned long long>(f));
    }
  }
  __syncthreads();
  if (tid < kNumBins && lc[tid]) atomicAdd(&counts[tid], static_cast<unsigned long long>(lc[tid]));
  if (tid == 0 && ltot) atomicAdd(total, ltot);
}

// Bin of global row r: mode 0 symbolic (by flops), mode 1 numeric (by nnz,
// per semiring slot; nnz read from the scanned product offsets).
__device__ __forceinline__ int batch_bin(int mode, const BatchDesc* __restrict__ d,
                                         const int64_t* __restrict__ row_off, const int32_t* __restrict__ prod_of,
                                         const int32_t* __restrict__ slot_of, int64_t r,
                                         const int64_t* __restrict__ flops, BinParams bp) {
  if (mode == 0) return sym_bin(flops[r], bp);
  const int b = prod_of[r];
  const int64_t i = r - row_off[b];
  const int64_t nz = d[b].c_ptr[i + 1] - d[b].c_ptr[i];
  const int c = num_bin(nz, flops[r], bp);
  return c == 0 ? 0 : c + kNumBins * slot_of[b];
}

__global__ void kb_count(int mode, const BatchDesc* __restrict__ d, const int64_t* __restrict__ row_off,
                         const int32_t* __restrict__ prod_of, const int32_t* __restrict__ slot_of, int64_t mtot,
                         const int64_t* __restrict__ flops, BinParams bp, unsigned long long* counts) {
  __shared__ unsigned int lc[kBatchBins];
  for (int t = threadIdx.x; t < kBatchBins; t += blockDim.x) lc[t] = 0;
  __syncthreads();
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < mtot) atomicAdd(&lc[batch_bin(mode, d, row_off, prod_of, slot_of, r, flops, bp)], 1u);
  __syncthreads();
  for (int t = threadIdx.x; t < kBatchBins; t += blockDim.x)
    if (lc[t]) atomicAdd(&counts[t], static_cast<unsigned long long>(lc[t]));
}

__global__ void kb_scatter(int mode, const BatchDesc* __restrict__ d, const int64_t* __restrict__ row_off,
                           const int32_t* __restrict__ prod_of, const int32_t* __restrict__ slot_of, int64_t mtot,
                           const int64_t* __restrict__ flops, BinParams bp,
                           const int64_t* __restrict__ offs, unsigned long long* cursors,
                           int32_t* __restrict__ items) {
  __shared__ unsigned int lc[kBatchBins];
  __shared__ unsigned long long lbase[kBatchBins];
  for (int t = threadIdx.x; t < kBatchBins; t += blockDim.x) lc[t] = 0;
  __syncthreads();
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  int bin = 0;
  unsigned int local = 0;
  if (r < mtot) {
    bin = batch_bin(mode, d, row_off, prod_of, slot_of, r, flops, bp);
    if (bin > 0) local = atomicAdd(&lc[bin], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kBatchBins; t += blockDim.x)
    if (lc[t]) lbase[t] = atomicAdd(&cursors[t], static_cast<unsigned long long>(lc[t]));
  __syncthreads();
  if (bin > 0) items[offs[bin] + static_cast<int64_t>(lbase[bin]) + local] = static_cast<int32_t>(r);
}

// Panel index for every product that needs one (which: 0 symbolic, 1 numeric),
// one wave per global B row.
__global__ void kb_panel_index(const BatchDesc* __restrict__ d, const int64_t* __restrict__ brow_off,
                               const int32_t* __restrict__ bprod_of, int64_t ntot, int which) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t g = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (g >= ntot) return;
  const int b = bprod_of[g];
  const BatchDesc& db = d[b];
  const int P = which == 0 ? db.sym_P : db.num_P;
  if (P <= 1) return;
  const int wlog2 = which == 0 ? db.sym_wlog2 : db.num_wlog2;
  int32_t* pidx = const_cast<int32_t*>(which == 0 ? db.psym : db.pnum);
  const int64_t k = g - brow_off[b];
  const int64_t lo = db.op.b_ptr[k], hi = db.op.b_ptr[k + 1];
  int32_t* out = pidx + k * (P + 1);
  // as k_panel_index: every slot first holds the row length, then a sorted
  // row's entries open their panels
  panel_index_fill(out, P, static_cast<int32_t>(hi - lo), lane, kWave);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0);
  panel_index_open(db.op.b_idx + lo, hi - lo, wlog2, P, out, lane, kWave);
}

// pool[po_b] = 0 for every product (the leading slot of each offsets array).
__global__ void kb_zero_heads(const int64_t* __restrict__ pool_off, int nprod, int64_t* pool) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nprod) pool[pool_off[b]] = 0;
}
__global__ void kb_bases(const int64_t* __restrict__ pool_off, int nprod, int64_t pool_len,
                         const int64_t* __restrict__ pool, int64_t* __restrict__ bases) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nprod) bases[b] = pool[pool_off[b]];
  if (b == nprod) bases[nprod] = pool_len > 0 ? pool[pool_len - 1] : 0;
}
__global__ void kb_rebase(const int64_t* __restrict__ pool_off, int nprod, int64_t pool_len,
                          const int64_t* __restrict__ bases, int64_t* __restrict__ pool) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= pool_len) return;
  const int b = find_segment(pool_off, nprod, x);
  pool[x] -= bases[b];
}

#define SPG_TRY_HIP(expr)                      \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return SPG_E_DEVICE; \
  } while (0)

unsigned blocks(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

}  // namespace

struct spg_batch_plan {
  int nprod;
  hipStream_t stream;
  spg_options opt;
  BinParams bp;
  std::vector<BatchDesc> desc;   // host copy of the descriptor table
  std::vector<int> slot_of;      // product -> semiring slot
  std::vector<int> slot_sr;      // slot -> kernel semiring code
  std::vector<int64_t> row_off, brow_off, pool_off, psym_off, pnum_off;
  std::vector<int64_t> a_nnz, b_nnz;
  int64_t mtot, ntot, pool_len;
  int sym_wlog2_max, num_wlog2_max[kMaxSlots];
  int64_t grid_cap_per_thread;  // resident threads of the device
  size_t off_desc, off_rowoff, off_browoff, off_pooloff, off_slot, off_ctr, off_flops, off_prod, off_bprod, off_items_sym,
      off_items_num, off_scan, off_bases, off_offs, off_psym, off_pnum, ws_bytes;
  int state;
  int64_t flops_total;
  unsigned long long sym_counts[kNumBins];
  unsigned long long num_counts[kBatchBins];
  std::vector<int64_t> bases;
  std::vector<int64_t> h_offs_sym, h_offs_num;  // host sources of async uploads
  std::vector<int32_t> h_slots;
  int64_t* c_ptr_pool;
  hipGraph_t graph;
  hipGraphExec_t graph_exec;
  bool has_graph;
  // phase timing (options.timing): an event pair per batch phase, recorded
  // by eager calls only (never inside a capture)
  hipEvent_t ev[2 * SPG_BATCH_NUM_PHASES];
  bool ev_made, capturing;
  bool ran[SPG_BATCH_NUM_PHASES];
};

namespace {

constexpr int kCtrSym = 0;
constexpr int kCtrNum = kNumBins;
constexpr int kCtrCursor = kNumBins + kBatchBins;
constexpr int kCtrMisc = kNumBins + 2 * kBatchBins;
constexpr int kCtrWords = kCtrMisc + 8;

struct BatchPhaseTimer {
  spg_batch_plan* p;
  int phase;
  bool on;
  BatchPhaseTimer(spg_batch_plan* plan, int ph)
      : p(plan), phase(ph), on(plan->ev_made && !plan->capturing) {
    if (on) {
      (void)hipEventRecord(p->ev[2 * phase], p->stream);
      p->ran[phase] = true;
    }
  }
  ~BatchPhaseTimer() {
    if (on) (void)hipEventRecord(p->ev[2 * phase + 1], p->stream);
  }
};

spg_status check_one(const spg_matrix& M) {
  if (M.nrows < 0 || M.ncols < 0 || M.nnz < 0) return SPG_E_SHAPE;
  if (M.layout != SPG_CSR && M.layout != SPG_CSC) return SPG_E_LAYOUT;
  if (!M.ptr) return SPG_E_INVALID;
  if (M.nnz > 0 && !M.idx) return SPG_E_INVALID;
  return SPG_OK;
}

int ilog2c(int64_t x) { return ceil_log2_u64(static_cast<uint64_t>(x < 1 ? 1 : x)); }

std::vector<int64_t> offsets_of(const unsigned long long* counts, int n) {
  std::vector<int64_t> o(n, 0);
  int64_t run = 0;
  for (int b = 1; b < n; ++b) {
    o[b] = run;
    run += static_cast<int64_t>(counts[b]);
  }
  return o;
}

// Grid of the preparation kernels: 8 workgroups of 256 threads per compute
// unit, each wave striding over rows.
int64_t prep_grid(const spg_batch_plan* p) { return std::max<int64_t>(1, p->grid_cap_per_thread / 256); }

spg_status enqueue_numeric(spg_batch_plan* p, unsigned char* w) {
  hipStream_t s = p->stream;
  auto* d = reinterpret_cast<const BatchDesc*>(w + p->off_desc);
  auto* row_off = reinterpret_cast<const int64_t*>(w + p->off_rowoff);
  auto* brow_off = reinterpret_cast<const int64_t*>(w + p->off_browoff);
  auto* items = reinterpret_cast<const int32_t*>(w + p->off_items_num);
  auto* prod_of = reinterpret_cast<const int32_t*>(w + p->off_prod);
  auto* bprod_of = reinterpret_cast<const int32_t*>(w + p->off_bprod);  // filled by the symbolic call
  bool any_panels = false;
  for (const auto& x : p->desc) any_panels = any_panels || x.num_P > 1;
  if (any_panels && p->ntot > 0)
    hipLaunchKernelGGL(kb_panel_index, dim3(blocks(p->ntot, 4)), dim3(256), 0, s, d, brow_off, bprod_of,
                       p->ntot, 1);
  const std::vector<int64_t> no = offsets_of(p->num_counts, kBatchBins);
  const int nslots = static_cast<int>(p->slot_sr.size());
  {
    // every slot's hash classes, then every slot's dense rows (independent
    // rows: the order only groups the launches for timing)
    BatchPhaseTimer t(p, SPG_BATCH_PHASE_NUM_HASH);
    for (int sl = 0; sl < nslots; ++sl) {
      const int sr = p->slot_sr[sl];
      for (int c = 1; c < kDenseBinBase; ++c) {
        const int bin = c + kNumBins * sl;
        if (!p->num_counts[bin]) continue;
        const int nt = hash_threads_num(c, sr);
        SPG_TRY_HIP(launch_hash_num_b(sr, d, row_off, prod_of, p->nprod, items + no[bin],
                                      static_cast<int64_t>(p->num_counts[bin]), hash_table_size(c), nt,
                                      p->opt.short_seg, s));
      }
    }
  }
  {
    BatchPhaseTimer t(p, SPG_BATCH_PHASE_NUM_ESC);
    for (int sl = 0; sl < nslots; ++sl) {
      const int sr = p->slot_sr[sl];
      for (int c = kEscBinBase; c < kNumBins; ++c) {
        const int bin = c + kNumBins * sl;
        if (!p->num_counts[bin]) continue;
        const int N = 32 << (c - kEscBinBase);
        SPG_TRY_HIP(launch_esc_num_b(sr, d, row_off, prod_of, p->nprod, items + no[bin],
                                     static_cast<int64_t>(p->num_counts[bin]), N, s));
      }
    }
  }
  {
    BatchPhaseTimer t(p, SPG_BATCH_PHASE_NUM_DENSE);
    for (int sl = 0; sl < nslots; ++sl) {
      const int sr = p->slot_sr[sl];
      int64_t nd = 0;
      for (int c = kDenseBinBase; c < kEscBinBase; ++c) nd += static_cast<int64_t>(p->num_counts[c + kNumBins * sl]);
      if (nd > 0) {
        const int nt = p->opt.dense_threads;
        SPG_TRY_HIP(launch_dense_num_b(sr, d, row_off, prod_of, p->nprod, items + no[kDenseBinBase + kNumBins * sl], nd,
                                       p->num_wlog2_max[sl], nt, p->opt.short_seg, s));
      }
    }
  }
  SPG_TRY_HIP(hipGetLastError());
  return SPG_OK;
}

}  // namespace

extern "C" {

spg_status spg_batch_plan_create(int nprod, const spg_matrix* A, const spg_matrix* B,
                                 const int* semirings, const spg_options* opt_in, void* stream,
                                 spg_batch_plan** out) {
  if (!out || nprod < 0 || (nprod > 0 && (!A || !B || !semirings))) return SPG_E_INVALID;
  *out = nullptr;
  auto* p = new (std::nothrow) spg_batch_plan();
  if (!p) return SPG_E_NOMEM;
  p->nprod = nprod;
  p->stream = static_cast<hipStream_t>(stream);
  std::memset(&p->opt, 0, sizeof(p->opt));
  if (opt_in) p->opt = *opt_in;
  if (p->opt.hash_max_flops <= 0) p->opt.hash_max_flops = 8192;
  if (p->opt.hash_max_nnz <= 0) p->opt.hash_max_nnz = 2048;
  if (p->opt.short_seg <= 0) p->opt.short_seg = 16;
  if (p->opt.dense_threads <= 0) p->opt.dense_threads = 512;
  if (p->opt.sym_panel_log2 <= 0) p->opt.sym_panel_log2 = 20;
  if (p->opt.lds_budget <= 0) p->opt.lds_budget = 65536;
  if (p->opt.esc_max_flops == 0) p->opt.esc_max_flops = kEscMaxFlops;
  if (p->opt.esc_ratio_x16 <= 0) p->opt.esc_ratio_x16 = 20;  // measured: 2 is slower in batches
  if (p->opt.hash_max_flops > 16384 || p->opt.hash_max_flops < 32 || p->opt.hash_max_nnz < 32 ||
      p->opt.hash_max_nnz > 4096 || p->opt.esc_max_flops > kEscMaxFlops ||
      p->opt.dense_threads % kWave || p->opt.dense_threads > 1024 || p->opt.sym_panel_log2 < 7 ||
      p->opt.sym_panel_log2 > 20) {
    delete p;
    return SPG_E_INVALID;
  }
  p->bp.hash_max_flops = p->opt.hash_max_flops;
  p->bp.hash_max_nnz = p->opt.hash_max_nnz;
  p->bp.split_heavy = 0;
  // expand-sort-compress classes: set once the batch's semirings are known
  p->bp.esc_max_flops = 0;
  p->bp.esc_ratio_x16 = p->opt.esc_ratio_x16;
  p->desc.resize(nprod);
  p->slot_of.resize(nprod);
  p->row_off.assign(nprod + 1, 0);
  p->brow_off.assign(nprod + 1, 0);
  p->pool_off.assign(nprod + 1, 0);
  p->psym_off.assign(nprod + 1, 0);
  p->pnum_off.assign(nprod + 1, 0);
  p->a_nnz.resize(nprod);
  p->b_nnz.resize(nprod);
  p->sym_wlog2_max = 7;
  for (int i = 0; i < kMaxSlots; ++i) p->num_wlog2_max[i] = 7;
  const int nt = p->opt.dense_threads;
  for (int b = 0; b < nprod; ++b) {
    spg_status st;
    if ((st = check_one(A[b])) != SPG_OK || (st = check_one(B[b])) != SPG_OK) {
      delete p;
      return st;
    }
    const int sr = semirings[b];
    if (sr < 0 || sr > 6) {
      delete p;
      return SPG_E_SEMIRING;
    }
    if (A[b].layout != B[b].layout) {
      delete p;
      return SPG_E_LAYOUT;
    }
    if (A[b].ncols != B[b].nrows) {
      delete p;
      return SPG_E_SHAPE;
    }
    const bool bool_sr = sr == SPG_OR_AND_BOOL;
    if (!bool_sr && ((A[b].nnz > 0 && !A[b].val) || (B[b].nnz > 0 && !B[b].val))) {
      delete p;
      return SPG_E_SEMIRING;
    }
    const bool csc = A[b].layout == SPG_CSC;
    const spg_matrix& L = csc ? B[b] : A[b];
    const spg_matrix& R = csc ? A[b] : B[b];
    BatchDesc& d = p->desc[b];
    std::memset(&d, 0, sizeof(d));
    d.op.a_ptr = L.ptr;
    d.op.a_idx = L.idx;
    d.op.a_val = L.val;
    d.op.b_ptr = R.ptr;
    d.op.b_idx = R.idx;
    d.op.b_val = R.val;
    d.op.m = csc ? B[b].ncols : A[b].nrows;
    d.op.n = A[b].ncols;
    d.op.k = csc ? A[b].nrows : B[b].ncols;
    d.sr = (bool_sr && !A[b].val && !B[b].val) ? 7 : sr;
    p->a_nnz[b] = L.nnz;
    p->b_nnz[b] = R.nnz;
    d.a_nnz = L.nnz;
    d.b_nnz = R.nnz;
    int slot = -1;
    for (size_t s2 = 0; s2 < p->slot_sr.size(); ++s2)
      if (p->slot_sr[s2] == d.sr) slot = static_cast<int>(s2);
    if (slot < 0) {
      if (static_cast<int>(p->slot_sr.size()) == kMaxSlots) {
        delete p;
        return SPG_E_SEMIRING;
      }
      slot = static_cast<int>(p->slot_sr.size());
      p->slot_sr.push_back(d.sr);
    }
    p->slot_of[b] = slot;
    // panels, as in the single-product plan
    const int kbits = std::max(7, ilog2c(d.op.k));
    d.sym_wlog2 = std::min(p->opt.sym_panel_log2, kbits);
    while (d.sym_wlog2 > 7 && dense_sym_lds(d.sym_wlog2, nt) > static_cast<size_t>(max_lds_bytes()))
      --d.sym_wlog2;
    const size_t sb = storage_bytes(d.sr);
    int wl = p->opt.sym_panel_log2;
    if (sb > 0) {
      wl = 7;
      while (wl < 24 && (static_cast<size_t>(1) << (wl + 1)) * sb <= static_cast<size_t>(p->opt.lds_budget))
        ++wl;
    }
    d.num_wlog2 = std::min(wl, kbits);
    while (d.num_wlog2 > 7 && dense_num_lds(d.sr, d.num_wlog2, nt) > static_cast<size_t>(max_lds_bytes()))
      --d.num_wlog2;
    const int64_t kk = std::max<int64_t>(1, d.op.k);
    d.sym_P = static_cast<int>((kk + (int64_t(1) << d.sym_wlog2) - 1) >> d.sym_wlog2);
    d.num_P = static_cast<int>((kk + (int64_t(1) << d.num_wlog2) - 1) >> d.num_wlog2);
    p->sym_wlog2_max = std::max(p->sym_wlog2_max, d.sym_wlog2);
    p->num_wlog2_max[slot] = std::max(p->num_wlog2_max[slot], d.num_wlog2);
    p->row_off[b + 1] = p->row_off[b] + d.op.m;
    p->brow_off[b + 1] = p->brow_off[b] + d.op.n;
    p->pool_off[b + 1] = p->pool_off[b] + d.op.m + 1;
    p->psym_off[b + 1] = p->psym_off[b] + (d.sym_P > 1 ? static_cast<int64_t>(d.op.n) * (d.sym_P + 1) : 0);
    p->pnum_off[b + 1] = p->pnum_off[b] + (d.num_P > 1 ? static_cast<int64_t>(d.op.n) * (d.num_P + 1) : 0);
  }
  // rows of low compression ratio (as in the single-product plan) up to the
  // largest class every semiring of the batch holds in LDS
  if (p->opt.esc_max_flops > 0) {
    int64_t lim = p->opt.esc_max_flops;
    for (int sr : p->slot_sr) lim = std::min<int64_t>(lim, esc_class_limit(sr));
    p->bp.esc_max_flops = lim;
  }
  p->mtot = p->row_off[nprod];
  p->ntot = p->brow_off[nprod];
  p->pool_len = p->pool_off[nprod];
  if (p->mtot >= (int64_t(1) << 31)) {
    delete p;
    return SPG_E_OVERFLOW;
  }
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  p->grid_cap_per_thread = static_cast<int64_t>(ncu) * 2048;
  size_t off = 0;
  auto take = [&off](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  p->off_desc = take(sizeof(BatchDesc) * std::max(1, nprod));
  p->off_rowoff = take(sizeof(int64_t) * (nprod + 1));
  p->off_browoff = take(sizeof(int64_t) * (nprod + 1));
  p->off_pooloff = take(sizeof(int64_t) * (nprod + 1));
  p->off_slot = take(sizeof(int32_t) * std::max(1, nprod));
  p->off_ctr = take(sizeof(uint64_t) * kCtrWords);
  p->off_flops = take(sizeof(int64_t) * p->mtot);
  p->off_prod = take(sizeof(int32_t) * p->mtot);
  p->off_bprod = take(sizeof(int32_t) * p->ntot);
  p->off_items_sym = take(sizeof(int32_t) * p->mtot);
  p->off_items_num = take(sizeof(int32_t) * p->mtot);
  p->off_scan = take(sizeof(int64_t) * ((p->pool_len + kScanTile - 1) / kScanTile + 1));
  p->off_bases = take(sizeof(int64_t) * (nprod + 1));
  p->off_offs = take(sizeof(int64_t) * kBatchBins);
  p->off_psym = take(sizeof(int32_t) * p->psym_off[nprod]);
  p->off_pnum = take(sizeof(int32_t) * p->pnum_off[nprod]);
  p->ws_bytes = off;
  p->state = 0;
  p->c_ptr_pool = nullptr;
  p->has_graph = false;
  p->ev_made = false;
  p->capturing = false;
  for (int i = 0; i < SPG_BATCH_NUM_PHASES; ++i) p->ran[i] = false;
  if (p->opt.timing) {
    int made = 0;
    while (made < 2 * SPG_BATCH_NUM_PHASES && hipEventCreate(&p->ev[made]) == hipSuccess) ++made;
    if (made < 2 * SPG_BATCH_NUM_PHASES) {
      for (int i = 0; i < made; ++i) (void)hipEventDestroy(p->ev[i]);
      delete p;
      return SPG_E_DEVICE;
    }
    p->ev_made = true;
  }
  *out = p;
  return SPG_OK;
}

spg_status spg_batch_workspace_size(const spg_batch_plan* p, size_t* bytes) {
  if (!p || !bytes) return SPG_E_INVALID;
  *bytes = p->ws_bytes;
  return SPG_OK;
}

spg_status spg_batch_symbolic(spg_batch_plan* p, void* ws, int64_t* c_ptr_pool, int64_t* c_nnz,
                              int64_t* idx_off, int64_t* val_off) {
  if (!p || !c_ptr_pool || (p->nprod > 0 && (!c_nnz || !idx_off || !val_off))) return SPG_E_INVALID;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign) return SPG_E_INVALID;
  hipStream_t s = p->stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  auto* d = reinterpret_cast<BatchDesc*>(w + p->off_desc);
  auto* row_off = reinterpret_cast<int64_t*>(w + p->off_rowoff);
  auto* brow_off = reinterpret_cast<int64_t*>(w + p->off_browoff);
  auto* pool_off = reinterpret_cast<int64_t*>(w + p->off_pooloff);
  auto* slot_of = reinterpret_cast<int32_t*>(w + p->off_slot);
  auto* ctr = reinterpret_cast<unsigned long long*>(w + p->off_ctr);
  auto* flops = reinterpret_cast<int64_t*>(w + p->off_flops);
  auto* prod_of = reinterpret_cast<int32_t*>(w + p->off_prod);
  auto* items_sym = reinterpret_cast<int32_t*>(w + p->off_items_sym);
  auto* items_num = reinterpret_cast<int32_t*>(w + p->off_items_num);
  auto* scan = reinterpret_cast<int64_t*>(w + p->off_scan);
  auto* bases = reinterpret_cast<int64_t*>(w + p->off_bases);
  auto* offs = reinterpret_cast<int64_t*>(w + p->off_offs);
  const int nprod = p->nprod;
  if (p->has_graph) {
    // a new symbolic pass may change the launch shapes: the capture is dropped
    (void)hipGraphExecDestroy(p->graph_exec);
    (void)hipGraphDestroy(p->graph);
    p->has_graph = false;
  }
  for (int b = 0; b < nprod; ++b) {
    p->desc[b].c_ptr = c_ptr_pool + p->pool_off[b];
    p->desc[b].c_idx = nullptr;
    p->desc[b].c_val = nullptr;
    p->desc[b].psym = reinterpret_cast<const int32_t*>(w + p->off_psym) + p->psym_off[b];
    p->desc[b].pnum = reinterpret_cast<const int32_t*>(w + p->off_pnum) + p->pnum_off[b];
  }
  p->h_slots.assign(p->slot_of.begin(), p->slot_of.end());
  if (nprod > 0) {
    SPG_TRY_HIP(hipMemcpyAsync(d, p->desc.data(), sizeof(BatchDesc) * nprod, hipMemcpyHostToDevice, s));
    SPG_TRY_HIP(hipMemcpyAsync(row_off, p->row_off.data(), sizeof(int64_t) * (nprod + 1), hipMemcpyHostToDevice, s));
    SPG_TRY_HIP(hipMemcpyAsync(brow_off, p->brow_off.data(), sizeof(int64_t) * (nprod + 1), hipMemcpyHostToDevice, s));
    SPG_TRY_HIP(hipMemcpyAsync(pool_off, p->pool_off.data(), sizeof(int64_t) * (nprod + 1), hipMemcpyHostToDevice, s));
    SPG_TRY_HIP(hipMemcpyAsync(slot_of, p->h_slots.data(), sizeof(int32_t) * nprod, hipMemcpyHostToDevice, s));
  }
  SPG_TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(ctr), kCtrWords, 0, s));
  auto* bprod_of = reinterpret_cast<int32_t*>(w + p->off_bprod);
  if (nprod > 0) {
    hipLaunchKernelGGL(kb_fill_prod, dim3(nprod), dim3(256), 0, s, row_off, prod_of);
    hipLaunchKernelGGL(kb_fill_prod, dim3(nprod), dim3(256), 0, s, brow_off, bprod_of);
  }
  // Operand check of every product before any kernel indexes with their ids.
  if (p->mtot + p->ntot > 0) {
    int* err = reinterpret_cast<int*>(ctr + kCtrMisc + 1);
    hipLaunchKernelGGL(kb_validate, dim3(std::min<int64_t>(blocks(p->mtot + p->ntot, 4), prep_grid(p))), dim3(256),
                       0, s, d, row_off, brow_off, prod_of, bprod_of, p->mtot, p->ntot, err);
    int herr = 0;
    SPG_TRY_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    SPG_TRY_HIP(hipStreamSynchronize(s));
    if (herr) return SPG_E_INVALID;
  }
  if (p->mtot > 0)
    hipLaunchKernelGGL(kb_flops_bin, dim3(std::min<int64_t>(blocks(p->mtot, 4), prep_grid(p))), dim3(256), 0, s,
                       d, row_off, nprod, p->mtot, p->bp, flops, prod_of, ctr + kCtrSym, ctr + kCtrMisc);
  unsigned long long h[kNumBins + 1];
  SPG_TRY_HIP(hipMemcpyAsync(h, ctr + kCtrSym, sizeof(uint64_t) * kNumBins, hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipMemcpyAsync(&h[kNumBins], ctr + kCtrMisc, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipStreamSynchronize(s));
  std::memcpy(p->sym_counts, h, sizeof(p->sym_counts));
  p->flops_total = static_cast<int64_t>(h[kNumBins]);
  {
    const std::vector<int64_t> so = offsets_of(p->sym_counts, kNumBins);
    p->h_offs_sym.assign(kBatchBins, 0);
    std::copy(so.begin(), so.end(), p->h_offs_sym.begin());
    SPG_TRY_HIP(hipMemcpyAsync(offs, p->h_offs_sym.data(), sizeof(int64_t) * kBatchBins, hipMemcpyHostToDevice, s));
    if (p->mtot > 0)
      hipLaunchKernelGGL(kb_scatter, dim3(blocks(p->mtot, 256)), dim3(256), 0, s, 0, d, row_off, prod_of,
                         slot_of, p->mtot, flops, p->bp, offs, ctr + kCtrCursor, items_sym);
    bool any_panels = false;
    for (const auto& x : p->desc) any_panels = any_panels || x.sym_P > 1;
    if (any_panels && p->ntot > 0)
      hipLaunchKernelGGL(kb_panel_index, dim3(blocks(p->ntot, 4)), dim3(256), 0, s, d, brow_off, bprod_of,
                         p->ntot, 0);
    {
      BatchPhaseTimer t(p, SPG_BATCH_PHASE_SYM_HASH);
      for (int c = 1; c < kDenseBinBase; ++c) {
        if (!p->sym_counts[c]) continue;
        const int nt = hash_threads(c);
        SPG_TRY_HIP(launch_hash_sym_b(d, row_off, prod_of, nprod, items_sym + so[c],
                                      static_cast<int64_t>(p->sym_counts[c]), hash_table_size(c), nt,
                                      p->opt.short_seg, s));
      }
    }
    int64_t nd = 0;
    for (int c = kDenseBinBase; c < kNumBins; ++c) nd += static_cast<int64_t>(p->sym_counts[c]);
    if (nd > 0) {
      BatchPhaseTimer t(p, SPG_BATCH_PHASE_SYM_DENSE);
      const int nt = p->opt.dense_threads;
      SPG_TRY_HIP(launch_dense_sym_b(d, row_off, prod_of, nprod, items_sym + so[kDenseBinBase], nd, p->sym_wlog2_max,
                                     nt, p->opt.short_seg, s));
    }
  }
  // offsets: zero each product's leading slot, scan the whole pool, rebase
  if (nprod > 0) {
    hipLaunchKernelGGL(kb_zero_heads, dim3(blocks(nprod, 256)), dim3(256), 0, s, pool_off, nprod, c_ptr_pool);
    SPG_TRY_HIP(launch_scan_inplace(c_ptr_pool + 1, p->pool_len - 1, scan, s));
    hipLaunchKernelGGL(kb_bases, dim3(blocks(nprod + 1, 256)), dim3(256), 0, s, pool_off, nprod, p->pool_len,
                       c_ptr_pool, bases);
    hipLaunchKernelGGL(kb_rebase, dim3(blocks(p->pool_len, 256)), dim3(256), 0, s, pool_off, nprod,
                       p->pool_len, bases, c_ptr_pool);
  }
  if (p->mtot > 0)
    hipLaunchKernelGGL(kb_count, dim3(blocks(p->mtot, 256)), dim3(256), 0, s, 1, d, row_off, prod_of, slot_of,
                       p->mtot, flops, p->bp, ctr + kCtrNum);
  p->bases.assign(nprod + 1, 0);
  if (nprod > 0)
    SPG_TRY_HIP(hipMemcpyAsync(p->bases.data(), bases, sizeof(int64_t) * (nprod + 1), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipMemcpyAsync(p->num_counts, ctr + kCtrNum, sizeof(uint64_t) * kBatchBins, hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipStreamSynchronize(s));
  {
    p->h_offs_num = offsets_of(p->num_counts, kBatchBins);
    SPG_TRY_HIP(hipMemcpyAsync(offs, p->h_offs_num.data(), sizeof(int64_t) * kBatchBins, hipMemcpyHostToDevice, s));
    SPG_TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(ctr + kCtrCursor), kBatchBins, 0, s));
    if (p->mtot > 0)
      hipLaunchKernelGGL(kb_scatter, dim3(blocks(p->mtot, 256)), dim3(256), 0, s, 1, d, row_off, prod_of,
                         slot_of, p->mtot, flops, p->bp, offs, ctr + kCtrCursor, items_num);
    SPG_TRY_HIP(hipStreamSynchronize(s));
  }
  SPG_TRY_HIP(hipGetLastError());
  int64_t voff = 0;
  for (int b = 0; b < nprod; ++b) {
    c_nnz[b] = p->bases[b + 1] - p->bases[b];
    idx_off[b] = p->bases[b];
    val_off[b] = voff;
    const size_t sb = p->desc[b].sr == 7 ? 0 : (p->desc[b].sr == 0 || p->desc[b].sr == 5 ? 8 :
                                                 (p->desc[b].sr == 4 ? 1 : 4));
    voff += static_cast<int64_t>((c_nnz[b] * sb + 7) & ~int64_t(7));
  }
  if (nprod > 0) {
    idx_off[nprod] = p->bases[nprod];
    val_off[nprod] = voff;
  }
  p->c_ptr_pool = c_ptr_pool;
  p->state = 1;
  return SPG_OK;
}

static spg_status set_outputs(spg_batch_plan* p, void* ws, int32_t* c_idx, void* c_val,
                              const int64_t* val_off) {
  unsigned char* w = static_cast<unsigned char*>(ws);
  auto* d = reinterpret_cast<BatchDesc*>(w + p->off_desc);
  for (int b = 0; b < p->nprod; ++b) {
    p->desc[b].c_idx = c_idx ? c_idx + p->bases[b] : nullptr;
    p->desc[b].c_val = c_val ? static_cast<unsigned char*>(c_val) + val_off[b] : nullptr;
  }
  if (p->nprod > 0) {
    SPG_TRY_HIP(hipMemcpyAsync(d, p->desc.data(), sizeof(BatchDesc) * p->nprod, hipMemcpyHostToDevice,
                               p->stream));
    SPG_TRY_HIP(hipStreamSynchronize(p->stream));
  }
  return SPG_OK;
}

spg_status spg_batch_numeric(spg_batch_plan* p, void* ws, int32_t* c_idx, void* c_val,
                             const int64_t* val_off) {
  if (!p || !ws) return SPG_E_INVALID;
  if (p->state != 1) return SPG_E_STATE;
  spg_status st = set_outputs(p, ws, c_idx, c_val, val_off);
  if (st != SPG_OK) return st;
  return enqueue_numeric(p, static_cast<unsigned char*>(ws));
}

spg_status spg_batch_graph_capture(spg_batch_plan* p, void* ws, int32_t* c_idx, void* c_val,
                                   const int64_t* val_off) {
  if (!p || !ws) return SPG_E_INVALID;
  if (p->state != 1) return SPG_E_STATE;
  spg_status st = set_outputs(p, ws, c_idx, c_val, val_off);
  if (st != SPG_OK) return st;
  if (p->has_graph) {
    (void)hipGraphExecDestroy(p->graph_exec);
    (void)hipGraphDestroy(p->graph);
    p->has_graph = false;
  }
  // Capture on a private non-blocking stream (the null stream cannot be
  // captured); the graph is launched later on the plan's stream.
  hipStream_t cap = nullptr;
  SPG_TRY_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipStream_t saved = p->stream;
  p->stream = cap;
  p->capturing = true;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) st = enqueue_numeric(p, static_cast<unsigned char*>(ws));
  hipGraph_t g = nullptr;
  if (e == hipSuccess) e = hipStreamEndCapture(cap, &g);
  p->capturing = false;
  p->stream = saved;
  (void)hipStreamDestroy(cap);
  if (st != SPG_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return st != SPG_OK ? st : SPG_E_DEVICE;
  }
  if (hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return SPG_E_DEVICE;
  }
  p->graph = g;
  p->has_graph = true;
  return SPG_OK;
}

spg_status spg_batch_graph_launch(spg_batch_plan* p) {
  if (!p) return SPG_E_INVALID;
  if (!p->has_graph) return SPG_E_STATE;
  SPG_TRY_HIP(hipGraphLaunch(p->graph_exec, p->stream));
  return SPG_OK;
}

spg_status spg_batch_stats(const spg_batch_plan* p, int64_t* flops, int64_t* rows) {
  if (!p) return SPG_E_INVALID;
  if (p->state < 1) return SPG_E_STATE;
  if (flops) *flops = p->flops_total;
  if (rows) *rows = p->mtot;
  return SPG_OK;
}

spg_status spg_batch_timings(spg_batch_plan* p, float* ms) {
  if (!p || !ms) return SPG_E_INVALID;
  if (!p->ev_made) return SPG_E_STATE;
  SPG_TRY_HIP(hipStreamSynchronize(p->stream));
  for (int i = 0; i < SPG_BATCH_NUM_PHASES; ++i) {
    ms[i] = 0.0f;
    if (p->ran[i]) SPG_TRY_HIP(hipEventElapsedTime(&ms[i], p->ev[2 * i], p->ev[2 * i + 1]));
  }
  return SPG_OK;
}

spg_status spg_batch_plan_destroy(spg_batch_plan* p) {
  if (!p) return SPG_OK;
  if (p->has_graph) {
    (void)hipGraphExecDestroy(p->graph_exec);
    (void)hipGraphDestroy(p->graph);
  }
  if (p->ev_made)
    for (int i = 0; i < 2 * SPG_BATCH_NUM_PHASES; ++i) (void)hipEventDestroy(p->ev[i]);
  delete p;
  return SPG_OK;
}

}  // extern "C"
