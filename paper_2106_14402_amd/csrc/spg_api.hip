// Host side of the C ABI in include/spg.h: descriptor checks, plan state,
// workspace layout, and the launch sequence of the symbolic and numeric
// phases (paper Sec. 4.1: flop estimate, symbolic, numeric).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/spg.h"
#include "spg_launch.h"

using namespace spg;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

enum PlanState { kCreated = 0, kSymbolicDone = 1 };

}  // namespace

struct spg_plan {
  Operands op;       // oriented CSR problem
  int sr;            // kernel semiring code (0..6, 7 = pattern-only boolean)
  int user_sr;
  bool csc;
  hipStream_t stream;
  spg_options opt;
  BinParams bp;
  int sym_wlog2, sym_P, num_wlog2, num_P;
  bool sym_win;                  // dense symbolic rows as (row, window) items
  size_t off_itemcnt, off_slotflag;
  // workspace layout (byte offsets)
  size_t off_ctr, off_flops, off_rows_sym, off_rows_num, off_scan, off_psym, off_pnum, ws_bytes;
  bool split;                    // heavy rows go to the numeric phase as (row, panel) pieces
  size_t off_subcnt, off_suboff, off_subitems, off_wend;
  int64_t n_dense_sym;
  bool keep;                     // keep heavy rows' symbolic bitmaps for the numeric phase
  size_t off_rowslot, off_store;
  int64_t keep_nwords, keep_stride, keep_min_flops;  // words per bitmap; slot stride (multiple of 4)
  unsigned int keep_cap;
  size_t off_segoff, off_segs;   // (row, panel) segment lists
  bool rank;                     // heavy valued rows through rank-compressed panels
  int rank_cw, rank_NC;
  RankShapes rank_shapes;  // pass shapes of the rank kernel
  size_t off_rcnt, off_pchunk;
  bool pair;                     // rank passes read B through (column, value) pairs
  size_t off_bpair;
  int32_t lists_rb, lists_re;    // rows [lists_rb, lists_re) fill the numeric row lists
  int sum_k;                     // > 0: a semiring sum of sum_k stacked parts; A is the selector
  size_t off_sel, off_sel_idx, off_sel_val;  // built in the workspace by spg_symbolic
  int64_t seg_cap, seg_total;
  bool pnum_ready;
  unsigned long long sub_counts[kNumBins];
  int64_t a_nnz, b_nnz;  // entries of the oriented operands
  // the caller's id and value arrays of the oriented operands (op points at
  // sorted copies in the workspace after a symbolic phase that sorted them)
  const int32_t* src_a_idx;
  const void* src_a_val;
  const int32_t* src_b_idx;
  const void* src_b_val;
  int a_es, b_es;                // bytes per input value (0: none)
  bool room_a, room_b;           // workspace holds room to sort A / B
  bool check_b;                  // B is checked by the symbolic phase
  bool b_resorted;               // this symbolic phase sorted B: external panels do not apply
  size_t off_sa_idx, off_sa_val, off_sb_idx, off_sb_val, off_spos;
  const int32_t* ext_psym;  // caller-built panel indexes (NULL: build in workspace)
  const int32_t* ext_pnum;
  int state;
  int64_t flops_total;
  int64_t c_nnz;
  int64_t* c_ptr;
  unsigned long long sym_counts[kNumBins];
  unsigned long long num_counts[kNumBins];
  // phase timing (options.timing)
  hipEvent_t ev[2 * SPG_NUM_PHASES];
  bool ev_made;
  bool ran[SPG_NUM_PHASES];
};

namespace {

// Phase timing: an event pair per phase on the plan's stream.
struct PhaseTimer {
  spg_plan* p;
  int phase;
  PhaseTimer(spg_plan* plan, int ph) : p(plan), phase(ph) {
    if (p->opt.timing && p->ev_made) {
      (void)hipEventRecord(p->ev[2 * phase], p->stream);
      p->ran[phase] = true;
    }
  }
  ~PhaseTimer() {
    if (p->opt.timing && p->ev_made) (void)hipEventRecord(p->ev[2 * phase + 1], p->stream);
  }
};

// Counter block inside the workspace (uint64 words).
constexpr int kCtrSym = 0;                 // [64] symbolic bin counts
constexpr int kCtrNum = kNumBins;          // [64] numeric bin counts
constexpr int kCtrCursor = 2 * kNumBins;   // [64] scatter cursors
constexpr int kCtrMisc = 3 * kNumBins;     // [0] total flops, [1] validation error bits
constexpr int kCtrSub = 4 * kNumBins;      // [64] (row, panel) piece bin counts
constexpr int kCtrWin = 5 * kNumBins;      // [64] window queues (uint32 each) of the windowed symbolic
constexpr int kCtrRange = 6 * kNumBins;    // [0] smallest and largest int32 value of B (numeric)
constexpr int kCtrWords = 7 * kNumBins;
constexpr int kMaxWindows = 2 * kNumBins;

spg_status from_hip(hipError_t e) { return e == hipSuccess ? SPG_OK : SPG_E_DEVICE; }

#define SPG_TRY_HIP(expr)                      \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return SPG_E_DEVICE; \
  } while (0)

bool valid_semiring(int sr) { return sr >= 0 && sr <= 6; }

// Bytes of one input value of a user semiring code.
int in_bytes(int user_sr) {
  switch (user_sr) {
    case SPG_PLUS_TIMES_F64: case SPG_MAX_TIMES_F64: return 8;
    case SPG_OR_AND_BOOL: return 1;
    default: return 4;
  }
}

spg_status check_matrix(const spg_matrix* M) {
  if (!M) return SPG_E_INVALID;
  if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0) return SPG_E_SHAPE;
  if (M->layout != SPG_CSR && M->layout != SPG_CSC) return SPG_E_LAYOUT;
  if (!M->ptr) return SPG_E_INVALID;
  if (M->nnz > 0 && !M->idx) return SPG_E_INVALID;
  return SPG_OK;
}

int ilog2_ceil(int64_t x) { return ceil_log2_u64(static_cast<uint64_t>(x < 1 ? 1 : x)); }

void resolve_options(const spg_options* in, spg_options* o, int sr) {
  std::memset(o, 0, sizeof(*o));
  if (in) *o = *in;
  // Rows past 4096 products (symbolic) or 4096 entries (numeric) leave the
  // LDS hash tables for the bitmap and rank paths: measured on the R-MAT
  // and Markov-clustering products, the larger tables' sort cost more than
  // the bitmap passes they replace.
  (void)sr;
  if (o->hash_max_flops <= 0) o->hash_max_flops = 4096;
  if (o->hash_max_nnz <= 0) o->hash_max_nnz = 4096;
  if (o->short_seg <= 0) o->short_seg = 32;
  if (o->dense_threads <= 0) o->dense_threads = 1024;
  if (o->sym_panel_log2 <= 0) o->sym_panel_log2 = 20;
  if (o->lds_budget <= 0) o->lds_budget = 131072;
  if (o->seg_mib <= 0) o->seg_mib = 16384;
  if (o->rank_dense_div <= 0) o->rank_dense_div = 1;
  if (o->rank_shapes <= 0 || o->rank_shapes > kRankShapes) o->rank_shapes = kRankShapes;
  if (o->win_threads <= 0) o->win_threads = 256;
  if (o->win_wgs <= 0) o->win_wgs = 8;
  if (o->esc_max_flops == 0) o->esc_max_flops = kEscMaxFlops;
  if (o->esc_ratio_x16 <= 0) o->esc_ratio_x16 = 32;
}

spg_status check_options(const spg_options& o, int sr) {
  if (o.hash_max_flops > 16384 || o.hash_max_flops < 32) return SPG_E_INVALID;
  if (o.hash_max_nnz < 32 || o.hash_max_nnz > 8192) return SPG_E_INVALID;
  if (o.dense_threads % kWave != 0 || o.dense_threads > 1024) return SPG_E_INVALID;
  if (o.sym_panel_log2 < 7 || o.sym_panel_log2 > 20) return SPG_E_INVALID;
  if (o.sym_windows < 0 || o.sym_windows > kMaxWindows) return SPG_E_INVALID;
  if (o.win_threads % kWave != 0 || o.win_threads > 1024 || o.win_wgs > 32) return SPG_E_INVALID;
  if (o.esc_max_flops > kEscMaxFlops) return SPG_E_INVALID;
  // hash tables must fit in LDS
  const int csym = hash_class(o.hash_max_flops);
  if (hash_sym_lds(hash_table_size(csym), hash_threads(csym)) > static_cast<size_t>(max_lds_bytes()))
    return SPG_E_INVALID;
  const int cnum = hash_class(o.hash_max_nnz);
  if (hash_num_lds(sr, hash_table_size(cnum), hash_threads_num(cnum, sr)) > static_cast<size_t>(max_lds_bytes()))
    return SPG_E_INVALID;
  return SPG_OK;
}

// Offsets of bins in the row lists: bins 1..63 in ascending order.
BinOffsets offsets_of(const unsigned long long* counts) {
  BinOffsets o;
  int64_t run = 0;
  o.v[0] = 0;
  for (int b = 1; b < kNumBins; ++b) {
    o.v[b] = run;
    run += static_cast<int64_t>(counts[b]);
  }
  return o;
}

}  // namespace

// Options, panel widths, workspace layout and timing events of a plan whose
// oriented operands (p->op, a_nnz, b_nnz, sr, csc, stream) are set.
static spg_status plan_init(spg_plan* p, const spg_options* opt_in) {
  spg_status st;
  resolve_options(opt_in, &p->opt, p->sr);
  if ((st = check_options(p->opt, p->sr)) != SPG_OK) return st;
  p->bp.hash_max_flops = p->opt.hash_max_flops;
  p->bp.hash_max_nnz = p->opt.hash_max_nnz;
  p->bp.split_heavy = 0;

  // Dense panels.  Symbolic: a bitmap of 2^sym_panel_log2 columns.  Numeric:
  // presence bits plus one accumulator value per column, as wide as the LDS
  // budget allows (bits only for the pattern-only product).
  const int kbits = std::max(7, ilog2_ceil(p->op.k));
  p->sym_wlog2 = std::min(p->opt.sym_panel_log2, kbits);
  const size_t sb = storage_bytes(p->sr);
  int wl = p->opt.sym_panel_log2;
  if (sb > 0) {
    wl = 7;
    while (wl < 24 && (static_cast<size_t>(1) << (wl + 1)) * sb <= static_cast<size_t>(p->opt.lds_budget))
      ++wl;
  }
  p->num_wlog2 = std::min(wl, kbits);
  const int nt = p->opt.dense_threads;
  while (p->num_wlog2 > 7 && dense_num_lds(p->sr, p->num_wlog2, nt) > static_cast<size_t>(max_lds_bytes()))
    --p->num_wlog2;
  while (p->sym_wlog2 > 7 && dense_sym_lds(p->sym_wlog2, nt) > static_cast<size_t>(max_lds_bytes()))
    --p->sym_wlog2;
  const int64_t kk = std::max<int64_t>(1, p->op.k);
  // Column windows of the dense symbolic rows (off unless asked for: the
  // per-item work of eight windows costs more than their L2 reuse saves).
  {
    const int nwin = p->opt.sym_windows > 0 ? p->opt.sym_windows : 1;
    p->sym_win = false;
    if (nwin > 1 && p->opt.split_panels <= 0) {
      const int wl = std::max(7, ilog2_ceil((kk + nwin - 1) / nwin));
      if (wl < kbits && dense_sym_lds(wl, p->opt.win_threads) <= static_cast<size_t>(max_lds_bytes())) {
        p->sym_win = true;
        p->sym_wlog2 = wl;
      }
    }
  }
  p->sym_P = static_cast<int>((kk + (int64_t(1) << p->sym_wlog2) - 1) >> p->sym_wlog2);
  if (p->sym_P <= 1 || p->sym_P > kMaxWindows) p->sym_win = false;
  p->num_P = static_cast<int>((kk + (int64_t(1) << p->num_wlog2) - 1) >> p->num_wlog2);
  p->split = p->opt.split_panels > 0 && p->sr != 7 && p->num_P > 1 && p->sym_wlog2 >= p->num_wlog2 &&
             static_cast<int64_t>(p->op.m) * p->num_P < (int64_t(1) << 31);
  p->bp.split_heavy = p->split ? 1 : 0;
  // Expand-sort-compress for rows of at most esc_max_flops products whose
  // compression ratio flops/nnz is at most esc_ratio_x16 / 16.
  p->bp.esc_max_flops = (p->split || p->opt.esc_max_flops < 0) ? 0 : std::min(p->opt.esc_max_flops, esc_class_limit(p->sr));
  p->bp.esc_ratio_x16 = p->opt.esc_ratio_x16;

  // Rank-compressed panels: chunks of 2^cw columns, with 2^cw value slots
  // (half the LDS budget, at most 64 KiB) and a bitmap of as many chunks as
  // the rest of the LDS holds; further shapes trade bitmap for 1.25x to 2x the
  // slots, for rows whose entries rather than columns bound their passes, and
  // slots for bitmap (0.75x), for rows whose columns bound them.
  p->rank = false;
  p->rank_cw = 0;
  p->rank_NC = 0;
  p->rank_shapes = RankShapes{};
  if (p->opt.rank_panels >= 0 && sb > 0 && !p->split && p->num_P > 1) {
    const size_t vbytes = std::max<size_t>(1024, std::min<size_t>(65536, p->opt.lds_budget / 2));
    int cw = 5;
    while ((static_cast<size_t>(1) << (cw + 1)) * sb <= vbytes) ++cw;
    cw = std::min(cw, p->num_wlog2);
    // chunks per pass for a slot count: up to 64, leaving 1 KiB for the
    // kernel's own shared variables
    auto chunks_for = [&](int slots) {
      int c = 64;
      while (c > 0 && rank_pass_lds(p->sr, cw, slots, c, nt) + 1024 > static_cast<size_t>(max_lds_bytes())) --c;
      return c;
    };
    const int base = 1 << cw;
    const int maxc = chunks_for(base);
    const int64_t NC = (kk + (int64_t(1) << cw) - 1) >> cw;
    if (cw >= 6 && cw <= p->sym_wlog2 && maxc >= 1 &&
        rank_num_lds(p->sr, cw, base, maxc, p->num_wlog2, nt) <= static_cast<size_t>(max_lds_bytes()) &&
        static_cast<int64_t>(p->op.m) * NC < (int64_t(1) << 31) && NC < (int64_t(1) << 24)) {
      p->rank = true;
      p->rank_cw = cw;
      p->rank_NC = static_cast<int>(NC);
      RankShapes& sh = p->rank_shapes;
      sh.n = 1;
      sh.slots[0] = base;
      sh.maxc[0] = maxc;
      const int more[kRankShapes - 2] = {base + base / 4, base + base / 2, base + 3 * base / 4, 2 * base};
      const int want = std::min(p->opt.rank_shapes, kRankShapes);
      for (int j = 0; j < kRankShapes - 2 && sh.n < want; ++j) {
        const int c = chunks_for(more[j]);
        if (c < 2 || more[j] > 65536) break;  // ranks are 16-bit
        sh.slots[sh.n] = more[j];
        sh.maxc[sh.n] = c;
        ++sh.n;
      }
      // and 0.75x the slots over more chunks: rows of few entries spread over
      // all columns, whose passes the bitmap width bounds
      const int narrow = base - base / 4;
      const int cn = chunks_for(narrow);
      if (want == kRankShapes && sh.n == kRankShapes - 1 && cn > maxc) {
        sh.slots[sh.n] = narrow;
        sh.maxc[sh.n] = cn;
        ++sh.n;
      }
    }
  }
  p->bp.rank_heavy = p->rank ? 1 : 0;

  // Workspace layout.
  const int64_t m = p->op.m;
  const int64_t nB = p->op.n;
  size_t off = 0;
  p->off_ctr = off;
  off = align_up(off + kCtrWords * sizeof(uint64_t));
  p->off_flops = off;
  off = align_up(off + static_cast<size_t>(m) * sizeof(int64_t));
  p->off_rows_sym = off;
  off = align_up(off + static_cast<size_t>(m) * sizeof(int32_t));
  p->off_rows_num = off;
  off = align_up(off + static_cast<size_t>(m) * sizeof(int32_t));
  p->off_scan = off;
  {
    // scan partials for the row offsets and for the piece segment offsets
    const int64_t slen = std::max<int64_t>(m, 1) * std::max(1, p->num_P) + 1;
    off = align_up(off + static_cast<size_t>((slen + kScanTile - 1) / kScanTile + 1) * sizeof(int64_t));
  }
  p->off_psym = off;
  if (p->sym_P > 1) off = align_up(off + static_cast<size_t>(nB) * (p->sym_P + 1) * sizeof(int32_t));
  p->off_pnum = off;
  if (p->num_P > 1) off = align_up(off + static_cast<size_t>(nB) * (p->num_P + 1) * sizeof(int32_t));
  // Kept bitmaps: pattern-only rows are expanded from them, rank-panel rows
  // read their pattern from them, instead of walking B's column ids once
  // more; worth it for rows with at least one product per bitmap word.
  p->keep = (p->sr == 7 || p->rank) && (p->sym_P == 1 || p->sym_win) && p->opt.bitmap_mib > 0 && p->op.k > 0;
  p->keep_nwords = (static_cast<int64_t>(p->op.k) + 31) / 32;
  p->keep_stride = (p->keep_nwords + 3) & ~int64_t(3);
  p->keep_min_flops = p->keep_nwords;
  p->keep_cap = 0;
  if (p->keep) {
    const int64_t cap = (static_cast<int64_t>(p->opt.bitmap_mib) << 20) / (p->keep_stride * 4);
    p->keep_cap = static_cast<unsigned int>(std::min<int64_t>(cap, std::max<int64_t>(m, 1)));
    if (p->keep_cap == 0) p->keep = false;
  }
  p->off_rowslot = off;
  if (p->keep) off = align_up(off + static_cast<size_t>(m) * sizeof(int32_t));
  p->off_store = off;
  if (p->keep) off = align_up(off + static_cast<size_t>(p->keep_cap) * p->keep_stride * 4);
  const size_t nsub = p->split ? static_cast<size_t>(m) * p->num_P : 0;
  p->off_subcnt = off;
  off = align_up(off + nsub * sizeof(int32_t));
  p->off_suboff = off;
  off = align_up(off + nsub * sizeof(int32_t));
  p->off_subitems = off;
  off = align_up(off + nsub * sizeof(int32_t));
  p->off_wend = off;
  off = align_up(off + nsub * sizeof(int32_t));
  p->off_segoff = off;
  if (p->split) off = align_up(off + (nsub + 1) * sizeof(int64_t));
  p->off_segs = off;
  p->seg_cap = 0;
  if (p->split) {
    const int64_t bound = p->a_nnz * static_cast<int64_t>(p->num_P);
    const int64_t budget = (static_cast<int64_t>(p->opt.seg_mib) << 20) / static_cast<int64_t>(seg_desc_bytes());
    p->seg_cap = std::min(bound, budget);
    off = align_up(off + static_cast<size_t>(p->seg_cap) * seg_desc_bytes());
  }
  // windowed symbolic: a count per (row, window) item and the slot flags
  p->off_itemcnt = p->off_slotflag = off;
  if (p->sym_win) {
    off = align_up(off + static_cast<size_t>(m) * p->sym_P * sizeof(int32_t));
    p->off_slotflag = off;
    if (p->keep) off = align_up(off + static_cast<size_t>(m + 1) * sizeof(int64_t));
  }
  p->off_rcnt = off;
  if (p->rank) off = align_up(off + static_cast<size_t>(m) * p->rank_NC * sizeof(int32_t));
  p->off_pchunk = off;
  if (p->rank) off = align_up(off + static_cast<size_t>(nB) * (p->rank_NC + 1) * sizeof(int32_t));
  // 4-byte input values (float32, int32): the rank passes load each product's
  // column id and value with one 8-byte load from a paired copy of B
  p->pair = p->rank && (p->sr == SPG_PLUS_TIMES_F32 || p->sr == SPG_MIN_PLUS_I32 || p->sr == SPG_MIN_PLUS_F32 ||
                        p->sr == SPG_MAX_TIMES_F32);
  p->off_bpair = off;
  if (p->pair) off = align_up(off + static_cast<size_t>(p->b_nnz) * sizeof(int2));
  // selector of a semiring sum: ptr (m+1), ids and values (k per row)
  p->off_sel = p->off_sel_idx = p->off_sel_val = off;
  if (p->sum_k > 0) {
    const size_t sel = static_cast<size_t>(m) * p->sum_k;
    off = align_up(off + static_cast<size_t>(m + 1) * sizeof(int64_t));
    p->off_sel_idx = off;
    off = align_up(off + sel * sizeof(int32_t));
    p->off_sel_val = off;
    off = align_up(off + sel * 8);
  }
  // sorted copies of operands found unsorted (ids, values) and the position
  // scratch of the sort
  p->check_b = p->opt.b_checked != 1;
  p->room_a = p->opt.unsorted != -1 && p->sum_k == 0;
  p->room_b = p->opt.unsorted != -1 && p->check_b;
  p->off_sa_idx = p->off_sa_val = p->off_sb_idx = p->off_sb_val = p->off_spos = off;
  if (p->room_a) {
    p->off_sa_idx = off;
    off = align_up(off + static_cast<size_t>(p->a_nnz) * sizeof(int32_t));
    p->off_sa_val = off;
    off = align_up(off + static_cast<size_t>(p->a_nnz) * p->a_es);
  }
  if (p->room_b) {
    p->off_sb_idx = off;
    off = align_up(off + static_cast<size_t>(p->b_nnz) * sizeof(int32_t));
    p->off_sb_val = off;
    off = align_up(off + static_cast<size_t>(p->b_nnz) * p->b_es);
  }
  if (p->room_a || p->room_b) {
    p->off_spos = off;
    off = align_up(off + static_cast<size_t>(std::max(p->room_a ? p->a_nnz : 0, p->room_b ? p->b_nnz : 0)) *
                             sizeof(int32_t));
  }
  p->seg_total = 0;
  p->pnum_ready = false;
  p->ws_bytes = off;
  p->state = kCreated;
  p->c_ptr = nullptr;
  p->ext_psym = nullptr;
  p->ext_pnum = nullptr;
  p->b_resorted = false;
  p->ev_made = false;
  for (int i = 0; i < SPG_NUM_PHASES; ++i) p->ran[i] = false;
  if (p->opt.timing) {
    bool ok = true;
    for (int i = 0; i < 2 * SPG_NUM_PHASES; ++i) ok = ok && hipEventCreate(&p->ev[i]) == hipSuccess;
    if (!ok) return SPG_E_DEVICE;
    p->ev_made = true;
  }
  return SPG_OK;
}

extern "C" {

const char* spg_status_str(spg_status s) {
  switch (s) {
    case SPG_OK: return "ok";
    case SPG_E_INVALID: return "invalid argument or malformed matrix";
    case SPG_E_SHAPE: return "shape mismatch";
    case SPG_E_LAYOUT: return "bad or mixed layout";
    case SPG_E_SEMIRING: return "unknown semiring or missing values";
    case SPG_E_NOMEM: return "workspace too small or over budget";
    case SPG_E_OVERFLOW: return "integer overflow";
    case SPG_E_DEVICE: return "HIP device error";
    case SPG_E_STATE: return "call out of order";
  }
  return "unknown status";
}

spg_status spg_plan_create(const spg_matrix* A, const spg_matrix* B, spg_semiring sr_in,
                           const spg_options* opt_in, void* stream, spg_plan** out) {
  if (!out) return SPG_E_INVALID;
  *out = nullptr;
  spg_status st;
  if ((st = check_matrix(A)) != SPG_OK) return st;
  if ((st = check_matrix(B)) != SPG_OK) return st;
  const int sr = static_cast<int>(sr_in);
  if (!valid_semiring(sr)) return SPG_E_SEMIRING;
  if (A->layout != B->layout) return SPG_E_LAYOUT;
  if (A->ncols != B->nrows) return SPG_E_SHAPE;
  const bool bool_sr = sr == SPG_OR_AND_BOOL;
  if (!bool_sr && ((A->nnz > 0 && !A->val) || (B->nnz > 0 && !B->val))) return SPG_E_SEMIRING;

  auto* p = new (std::nothrow) spg_plan();
  if (!p) return SPG_E_NOMEM;
  p->user_sr = sr;
  p->csc = A->layout == SPG_CSC;
  p->stream = static_cast<hipStream_t>(stream);
  // Orientation.  CSR: C = A B row by row.  CSC: the arrays of a CSC matrix
  // are the CSR arrays of its transpose, and C^T = B^T A^T, so the CSR kernel
  // runs on (B^T, A^T).  Every listed multiplication is commutative, so the
  // operand swap needs no change to (x).
  const spg_matrix* L = p->csc ? B : A;
  const spg_matrix* R = p->csc ? A : B;
  p->op.a_ptr = L->ptr;
  p->op.a_idx = L->idx;
  p->op.a_val = L->val;
  p->op.b_ptr = R->ptr;
  p->op.b_idx = R->idx;
  p->op.b_val = R->val;
  p->a_nnz = L->nnz;
  p->b_nnz = R->nnz;
  p->src_a_idx = L->idx;
  p->src_a_val = L->val;
  p->src_b_idx = R->idx;
  p->src_b_val = R->val;
  p->a_es = L->val ? in_bytes(sr) : 0;
  p->b_es = R->val ? in_bytes(sr) : 0;
  p->op.m = p->csc ? B->ncols : A->nrows;
  p->op.n = A->ncols;
  p->op.k = p->csc ? A->nrows : B->ncols;
  p->sr = (bool_sr && !A->val && !B->val) ? 7 : sr;

  spg_status sti = plan_init(p, opt_in);
  if (sti != SPG_OK) {
    delete p;
    return sti;
  }
  *out = p;
  return SPG_OK;
}

spg_status spg_sum_plan_create(int k, const spg_matrix* P, spg_semiring sr_in, const spg_options* opt_in,
                               void* stream, spg_plan** out) {
  if (!out) return SPG_E_INVALID;
  *out = nullptr;
  spg_status st;
  if ((st = check_matrix(P)) != SPG_OK) return st;
  const int sr = static_cast<int>(sr_in);
  if (!valid_semiring(sr)) return SPG_E_SEMIRING;
  if (k < 1) return SPG_E_INVALID;
  const bool csc = P->layout == SPG_CSC;
  const int64_t major = csc ? P->ncols : P->nrows;
  const int64_t minor = csc ? P->nrows : P->ncols;
  if (major % k != 0) return SPG_E_SHAPE;
  const int64_t m = major / k;
  const bool bool_sr = sr == SPG_OR_AND_BOOL;
  if (!bool_sr && P->nnz > 0 && !P->val) return SPG_E_SEMIRING;
  auto* p = new (std::nothrow) spg_plan();
  if (!p) return SPG_E_NOMEM;
  p->user_sr = sr;
  p->csc = csc;
  p->stream = static_cast<hipStream_t>(stream);
  // Oriented: C = S P with S the m x (k m) selector (built at symbolic time),
  // P's slices as the rows of the right operand.
  p->op.b_ptr = P->ptr;
  p->op.b_idx = P->idx;
  p->op.b_val = P->val;
  p->b_nnz = P->nnz;
  p->src_a_idx = nullptr;
  p->src_a_val = nullptr;
  p->src_b_idx = P->idx;
  p->src_b_val = P->val;
  p->a_es = 0;
  p->b_es = P->val ? in_bytes(sr) : 0;
  p->a_nnz = m * k;
  p->op.m = static_cast<int32_t>(m);
  p->op.n = static_cast<int32_t>(major);
  p->op.k = static_cast<int32_t>(minor);
  p->sr = (bool_sr && !P->val) ? 7 : sr;
  p->sum_k = k;
  if ((st = plan_init(p, opt_in)) != SPG_OK) {
    delete p;
    return st;
  }
  *out = p;
  return SPG_OK;
}

spg_status spg_workspace_size(const spg_plan* p, size_t* bytes) {
  if (!p || !bytes) return SPG_E_INVALID;
  *bytes = p->ws_bytes;
  return SPG_OK;
}

spg_status spg_plan_stats(const spg_plan* p, int64_t* flops, int64_t* nslices) {
  if (!p) return SPG_E_INVALID;
  if (p->state < kSymbolicDone) return SPG_E_STATE;
  if (flops) *flops = p->flops_total;
  if (nslices) *nslices = p->op.m;
  return SPG_OK;
}

spg_status spg_plan_timings(spg_plan* p, float* ms) {
  if (!p || !ms) return SPG_E_INVALID;
  if (!p->ev_made) return SPG_E_STATE;
  SPG_TRY_HIP(hipStreamSynchronize(p->stream));
  for (int i = 0; i < SPG_NUM_PHASES; ++i) {
    ms[i] = 0.0f;
    if (p->ran[i]) SPG_TRY_HIP(hipEventElapsedTime(&ms[i], p->ev[2 * i], p->ev[2 * i + 1]));
  }
  return SPG_OK;
}

spg_status spg_plan_bins(const spg_plan* p, int64_t* sym, int64_t* num) {
  if (!p) return SPG_E_INVALID;
  if (p->state < kSymbolicDone) return SPG_E_STATE;
  for (int b = 0; b < kNumBins; ++b) {
    if (sym) sym[b] = static_cast<int64_t>(p->sym_counts[b]);
    if (num) num[b] = static_cast<int64_t>(p->num_counts[b]);
  }
  return SPG_OK;
}

spg_status spg_plan_options(const spg_plan* p, spg_options* out) {
  if (!p || !out) return SPG_E_INVALID;
  *out = p->opt;
  return SPG_OK;
}

spg_status spg_plan_panels(const spg_plan* p, int* sym_wlog2, int* sym_P, int* num_wlog2, int* num_P) {
  if (!p) return SPG_E_INVALID;
  if (sym_wlog2) *sym_wlog2 = p->sym_wlog2;
  if (sym_P) *sym_P = p->sym_P;
  if (num_wlog2) *num_wlog2 = p->num_wlog2;
  if (num_P) *num_P = p->num_P;
  return SPG_OK;
}

spg_status spg_panel_index_size(const spg_matrix* R, int wlog2, size_t* bytes) {
  spg_status st = check_matrix(R);
  if (st != SPG_OK) return st;
  if (!bytes || wlog2 < 1 || wlog2 > 30 || R->layout != SPG_CSR) return SPG_E_INVALID;
  const int64_t W = int64_t(1) << wlog2;
  const int64_t P = (std::max<int64_t>(1, R->ncols) + W - 1) / W;
  *bytes = static_cast<size_t>(R->nrows) * static_cast<size_t>(P + 1) * sizeof(int32_t);
  return SPG_OK;
}

spg_status spg_panel_index_build(const spg_matrix* R, int wlog2, void* out, void* stream) {
  size_t bytes = 0;
  spg_status st = spg_panel_index_size(R, wlog2, &bytes);
  if (st != SPG_OK) return st;
  if (!out && bytes > 0) return SPG_E_INVALID;
  const int64_t W = int64_t(1) << wlog2;
  const int P = static_cast<int>((std::max<int64_t>(1, R->ncols) + W - 1) / W);
  SPG_TRY_HIP(launch_panel_index(R->ptr, R->idx, R->nrows, wlog2, P, static_cast<int32_t*>(out),
                                 static_cast<hipStream_t>(stream)));
  return SPG_OK;
}

spg_status spg_plan_set_panels(spg_plan* p, int which, const void* pidx, int wlog2) {
  if (!p || (which != 0 && which != 1)) return SPG_E_INVALID;
  if (which == 0) {
    if (pidx && wlog2 != p->sym_wlog2) return SPG_E_INVALID;
    p->ext_psym = static_cast<const int32_t*>(pidx);
  } else {
    if (pidx && wlog2 != p->num_wlog2) return SPG_E_INVALID;
    p->ext_pnum = static_cast<const int32_t*>(pidx);
  }
  return SPG_OK;
}

spg_status spg_plan_destroy(spg_plan* p) {
  if (!p) return SPG_OK;
  if (p->ev_made)
    for (int i = 0; i < 2 * SPG_NUM_PHASES; ++i) (void)hipEventDestroy(p->ev[i]);
  delete p;
  return SPG_OK;
}

spg_status spg_symbolic(spg_plan* p, void* ws, int64_t* c_ptr, int64_t* c_nnz) {
  if (!p || !c_ptr || !c_nnz) return SPG_E_INVALID;
  if (!ws && p->ws_bytes > 0) return SPG_E_NOMEM;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return SPG_E_INVALID;
  hipStream_t s = p->stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  auto* ctr = reinterpret_cast<unsigned long long*>(w + p->off_ctr);
  auto* flops = reinterpret_cast<int64_t*>(w + p->off_flops);
  auto* rows_sym = reinterpret_cast<int32_t*>(w + p->off_rows_sym);
  auto* rows_num = reinterpret_cast<int32_t*>(w + p->off_rows_num);
  auto* scan = reinterpret_cast<int64_t*>(w + p->off_scan);
  auto* psym = reinterpret_cast<int32_t*>(w + p->off_psym);
  if (p->sum_k > 0) {
    // the selector: row i takes the parts' rows t*m + i with the (x)-identity
    p->op.a_ptr = reinterpret_cast<int64_t*>(w + p->off_sel);
    p->op.a_idx = reinterpret_cast<int32_t*>(w + p->off_sel_idx);
    p->op.a_val = p->sr == 7 ? nullptr : w + p->off_sel_val;
    SPG_TRY_HIP(launch_selector(p->op.m, p->sum_k, reinterpret_cast<int64_t*>(w + p->off_sel),
                                reinterpret_cast<int32_t*>(w + p->off_sel_idx),
                                p->sr == 7 ? nullptr : w + p->off_sel_val, p->sr, s));
  }
  const Operands& op = p->op;
  const int32_t m = op.m;

  for (int i = 0; i < SPG_NUM_PHASES; ++i) p->ran[i] = false;
  if (p->sum_k == 0) {
    p->op.a_idx = p->src_a_idx;
    p->op.a_val = p->src_a_val;
  }
  p->op.b_idx = p->src_b_idx;
  p->op.b_val = p->src_b_val;
  p->b_resorted = false;
  if ((op.m == 0 && p->a_nnz != 0) || (op.n == 0 && p->b_nnz != 0)) return SPG_E_INVALID;
  SPG_TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(ctr), kCtrWords, 0, s));
  // The operand check rides along: B's slices by k_validate, A's inside the
  // flop count, which never indexes with an id it has not range-checked.  The
  // bin counts and both error words come back in one copy.
  int* err_a = reinterpret_cast<int*>(ctr + kCtrMisc + 1);
  int* err_b = reinterpret_cast<int*>(ctr + kCtrMisc + 3);
  unsigned long long hcounts[kNumBins + 4];
  {
    PhaseTimer t(p, SPG_PHASE_FLOPS_BIN);
    if (p->check_b) SPG_TRY_HIP(launch_validate(op.b_ptr, op.b_idx, op.n, p->b_nnz, op.k, err_b, s));
    SPG_TRY_HIP(launch_flops_bin(op, p->a_nnz, p->bp, flops, c_ptr, ctr + kCtrSym, ctr + kCtrMisc, err_a, s));
  }
  SPG_TRY_HIP(hipMemcpyAsync(hcounts, ctr + kCtrSym, kNumBins * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipMemcpyAsync(&hcounts[kNumBins], ctr + kCtrMisc, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipStreamSynchronize(s));
  std::memcpy(p->sym_counts, hcounts, sizeof(p->sym_counts));
  p->flops_total = static_cast<int64_t>(hcounts[kNumBins]);
  {
    const int ea = static_cast<int>(hcounts[kNumBins + 1] & 0xffffffffu);
    const int eb = static_cast<int>(hcounts[kNumBins + 3] & 0xffffffffu);
    if ((ea | eb) & kCheckMalformed) return SPG_E_INVALID;
    // an equal adjacent pair in a sorted slice is a duplicate; in an
    // unsorted one it is decided on the sorted copy
    if ((ea & kCheckDuplicate) && !(ea & kCheckUnsorted)) return SPG_E_INVALID;
    if ((eb & kCheckDuplicate) && !(eb & kCheckUnsorted)) return SPG_E_INVALID;
    const bool sort_a = (ea & kCheckUnsorted) != 0, sort_b = (eb & kCheckUnsorted) != 0;
    if ((sort_a && !p->room_a) || (sort_b && !p->room_b)) return SPG_E_INVALID;
    if (sort_a || sort_b) {
      PhaseTimer t(p, SPG_PHASE_VALIDATE);
      auto* pos = reinterpret_cast<int32_t*>(w + p->off_spos);
      int herr = 0;
      SPG_TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(ctr + kCtrMisc + 1), 1, 0, s));
      if (sort_a) {
        auto* si = reinterpret_cast<int32_t*>(w + p->off_sa_idx);
        void* sv = p->a_es ? w + p->off_sa_val : nullptr;
        SPG_TRY_HIP(launch_sort_slices(op.a_ptr, op.a_idx, op.a_val, p->a_es, op.m, si, sv, pos, s));
        p->op.a_idx = si;
        p->op.a_val = sv;
        SPG_TRY_HIP(launch_validate(op.a_ptr, op.a_idx, op.m, p->a_nnz, op.n, err_a, s));
      }
      if (sort_b) {
        auto* si = reinterpret_cast<int32_t*>(w + p->off_sb_idx);
        void* sv = p->b_es ? w + p->off_sb_val : nullptr;
        SPG_TRY_HIP(launch_sort_slices(op.b_ptr, op.b_idx, op.b_val, p->b_es, op.n, si, sv, pos, s));
        p->op.b_idx = si;
        p->op.b_val = sv;
        SPG_TRY_HIP(launch_validate(op.b_ptr, op.b_idx, op.n, p->b_nnz, op.k, err_a, s));
      }
      SPG_TRY_HIP(hipMemcpyAsync(&herr, err_a, sizeof(int), hipMemcpyDeviceToHost, s));
      SPG_TRY_HIP(hipStreamSynchronize(s));
      if (herr) return SPG_E_INVALID;  // duplicates
      // external panel indexes were built over the caller's order
      p->b_resorted = sort_b;
    }
  }

  const BinOffsets so = offsets_of(p->sym_counts);
  int64_t ndense = 0;
  for (int b = kDenseBinBase; b < kNumBins; ++b) ndense += static_cast<int64_t>(p->sym_counts[b]);
  {
    PhaseTimer t(p, SPG_PHASE_SYM_HASH);
    SPG_TRY_HIP(launch_scatter(0, m, 0, flops, c_ptr, p->bp, so, ctr + kCtrCursor, rows_sym, s));
    for (int c = 1; c < kDenseBinBase; ++c) {
      if (!p->sym_counts[c]) continue;
      SPG_TRY_HIP(launch_hash_sym(op, rows_sym + so.v[c], static_cast<int64_t>(p->sym_counts[c]),
                                  hash_table_size(c), hash_threads(c), p->opt.short_seg, c_ptr, s));
    }
  }
  if (ndense > 0) {
    if (p->sym_P > 1 && p->ext_psym && !p->b_resorted) {
      psym = const_cast<int32_t*>(p->ext_psym);
    } else if (p->sym_P > 1) {
      PhaseTimer tp(p, SPG_PHASE_SYM_PANELS);
      SPG_TRY_HIP(launch_panel_index(op.b_ptr, op.b_idx, op.n, p->sym_wlog2, p->sym_P, psym, s));
    }
    PhaseTimer t(p, SPG_PHASE_SYM_DENSE);
    if (p->sym_win) {
      const int32_t* dense_rows = rows_sym + so.v[kDenseBinBase];
      auto* row_slot = reinterpret_cast<int32_t*>(w + p->off_rowslot);
      if (p->keep)
        SPG_TRY_HIP(launch_keep_slots(dense_rows, ndense, flops, p->keep_min_flops, p->keep_cap,
                                      reinterpret_cast<int64_t*>(w + p->off_slotflag), scan, row_slot, s));
      SPG_TRY_HIP(launch_dense_sym_win(
          op, dense_rows, ndense, p->sym_wlog2, p->sym_P, psym, p->opt.win_threads, p->opt.short_seg,
          reinterpret_cast<int32_t*>(w + p->off_itemcnt), reinterpret_cast<unsigned int*>(ctr + kCtrWin), c_ptr,
          p->rank ? p->rank_cw : 0, p->rank ? p->rank_NC : 0,
          p->rank ? reinterpret_cast<int32_t*>(w + p->off_rcnt) : nullptr, p->keep ? row_slot : nullptr,
          p->keep ? reinterpret_cast<uint32_t*>(w + p->off_store) : nullptr, p->keep_stride, p->opt.win_wgs, s));
    }
  }
  if (ndense > 0 && !p->sym_win) {
    PhaseTimer t(p, SPG_PHASE_SYM_DENSE);
    KeepBitmaps kb{};
    if (p->keep) {
      kb.store = reinterpret_cast<uint32_t*>(w + p->off_store);
      kb.row_slot = reinterpret_cast<int32_t*>(w + p->off_rowslot);
      kb.counter = reinterpret_cast<unsigned int*>(ctr + kCtrMisc + 2);
      kb.flops = flops;
      kb.min_flops = p->keep_min_flops;
      kb.nwords = p->keep_stride;
      kb.capacity = p->keep_cap;
    }
    SPG_TRY_HIP(launch_dense_sym(op, rows_sym + so.v[kDenseBinBase], ndense, p->sym_wlog2, p->sym_P,
                                 psym, p->opt.dense_threads, p->opt.short_seg, c_ptr, s,
                                 p->split ? p->num_wlog2 : (p->rank ? p->rank_cw : 0),
                                 p->split ? p->num_P : (p->rank ? p->rank_NC : 0),
                                 p->split  ? reinterpret_cast<int32_t*>(w + p->off_subcnt)
                                 : p->rank ? reinterpret_cast<int32_t*>(w + p->off_rcnt)
                                           : nullptr,
                                 kb));
  }
  int64_t total = 0;
  p->n_dense_sym = ndense;
  p->bp.row_slot =
      (p->keep && p->sr == 7 && ndense > 0) ? reinterpret_cast<const int32_t*>(w + p->off_rowslot) : nullptr;
  {
    PhaseTimer t(p, SPG_PHASE_SCAN);
    SPG_TRY_HIP(launch_count_num_bins(m, 0, 0, flops, c_ptr, p->bp, ctr + kCtrNum, s));
    SPG_TRY_HIP(launch_scan_inplace(c_ptr + 1, m, scan, s));
    if (p->split && ndense > 0)
      SPG_TRY_HIP(launch_sub_prepare(ndense, p->num_P, reinterpret_cast<int32_t*>(w + p->off_subcnt),
                                     reinterpret_cast<int32_t*>(w + p->off_suboff),
                                     reinterpret_cast<int32_t*>(w + p->off_wend), p->bp, ctr + kCtrSub, s));
  }
  p->pnum_ready = false;
  p->seg_total = 0;
  if (p->split && ndense > 0) {
    auto* pnum = reinterpret_cast<int32_t*>(w + p->off_pnum);
    if (!p->ext_pnum || p->b_resorted) {
      PhaseTimer tp(p, SPG_PHASE_NUM_PANELS);
      SPG_TRY_HIP(launch_panel_index(op.b_ptr, op.b_idx, op.n, p->num_wlog2, p->num_P, pnum, s));
    }
    p->pnum_ready = true;
    PhaseTimer tc(p, SPG_PHASE_SEG_COUNT);
    auto* segoff = reinterpret_cast<int64_t*>(w + p->off_segoff);
    SPG_TRY_HIP(launch_seg_count(op, rows_sym + so.v[kDenseBinBase], ndense, p->num_P,
                                 (p->ext_pnum && !p->b_resorted) ? p->ext_pnum : pnum,
                                 reinterpret_cast<const int32_t*>(w + p->off_wend), segoff + 1, s));
    SPG_TRY_HIP(launch_scan_inplace(segoff + 1, ndense * p->num_P, scan, s));
    SPG_TRY_HIP(hipMemcpyAsync(&p->seg_total, segoff + ndense * p->num_P, sizeof(int64_t),
                               hipMemcpyDeviceToHost, s));
  }
  SPG_TRY_HIP(hipMemcpyAsync(p->sub_counts, ctr + kCtrSub, kNumBins * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipMemcpyAsync(p->num_counts, ctr + kCtrNum, kNumBins * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipMemcpyAsync(&total, c_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipStreamSynchronize(s));
  const BinOffsets no = offsets_of(p->num_counts);
  SPG_TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(ctr + kCtrCursor), kNumBins, 0, s));
  SPG_TRY_HIP(launch_scatter(1, m, 0, flops, c_ptr, p->bp, no, ctr + kCtrCursor, rows_num, s));
  p->lists_rb = 0;
  p->lists_re = m;
  if (p->split && ndense > 0) {
    const BinOffsets sbo = offsets_of(p->sub_counts);
    SPG_TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(ctr + kCtrSym), kNumBins, 0, s));
    SPG_TRY_HIP(launch_sub_scatter(ndense, p->num_P, reinterpret_cast<const int32_t*>(w + p->off_subcnt), p->bp,
                                   sbo, ctr + kCtrSym, reinterpret_cast<int32_t*>(w + p->off_subitems), s));
  }
  SPG_TRY_HIP(hipGetLastError());
  p->c_nnz = total;
  p->c_ptr = c_ptr;
  p->state = kSymbolicDone;
  *c_nnz = total;
  return SPG_OK;
}

// Bytes of one output value (0: pattern only).
static int out_bytes(int sr) {
  switch (sr) {
    case 0: case 5: return 8;
    case 4: return 1;
    case 7: return 0;
    default: return 4;
  }
}

// Numeric row lists for rows [rb, re) only (after the offsets scan).
static spg_status rebin_rows(spg_plan* p, unsigned char* w, int32_t rb, int32_t re) {
  hipStream_t s = p->stream;
  auto* ctr = reinterpret_cast<unsigned long long*>(w + p->off_ctr);
  auto* flops = reinterpret_cast<int64_t*>(w + p->off_flops);
  auto* rows_num = reinterpret_cast<int32_t*>(w + p->off_rows_num);
  SPG_TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(ctr + kCtrNum), kNumBins, 0, s));
  SPG_TRY_HIP(launch_count_num_bins(re, rb, 1, flops, p->c_ptr, p->bp, ctr + kCtrNum, s));
  SPG_TRY_HIP(hipMemcpyAsync(p->num_counts, ctr + kCtrNum, kNumBins * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipStreamSynchronize(s));
  const BinOffsets no = offsets_of(p->num_counts);
  SPG_TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(ctr + kCtrCursor), kNumBins, 0, s));
  SPG_TRY_HIP(launch_scatter(1, re, rb, flops, p->c_ptr, p->bp, no, ctr + kCtrCursor, rows_num, s));
  p->lists_rb = rb;
  p->lists_re = re;
  return SPG_OK;
}

// Numeric phase of rows [rb, re); their entries go to c_idx/c_val from
// position 0 (C entry c_ptr[rb] + e is written at e).
static spg_status numeric_range(spg_plan* p, void* ws, int32_t rb, int32_t re, int32_t* c_idx_in, void* c_val_in) {
  if (p->state != kSymbolicDone) return SPG_E_STATE;
  hipStream_t s = p->stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  int64_t base = 0, range_nnz = p->c_nnz;
  if (rb != 0 || re != p->op.m) {
    if (p->split) return SPG_E_STATE;  // (row, window) items cover the whole product
    int64_t ends[2] = {0, 0};
    SPG_TRY_HIP(hipMemcpyAsync(&ends[0], p->c_ptr + rb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPG_TRY_HIP(hipMemcpyAsync(&ends[1], p->c_ptr + re, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPG_TRY_HIP(hipStreamSynchronize(s));
    base = ends[0];
    range_nnz = ends[1] - ends[0];
  }
  if (range_nnz > 0 && !c_idx_in) return SPG_E_INVALID;
  if (range_nnz > 0 && !c_val_in && p->sr != 7) return SPG_E_INVALID;
  if (rb != p->lists_rb || re != p->lists_re) {
    spg_status st = rebin_rows(p, w, rb, re);
    if (st != SPG_OK) return st;
  }
  // The kernels write entry c_ptr[row] + e; shift the outputs so that entry
  // c_ptr[rb] lands at position 0 of the caller's buffers.
  int32_t* c_idx = reinterpret_cast<int32_t*>(reinterpret_cast<uintptr_t>(c_idx_in) - base * sizeof(int32_t));
  void* c_val = c_val_in ? reinterpret_cast<void*>(reinterpret_cast<uintptr_t>(c_val_in) - base * out_bytes(p->sr))
                         : nullptr;
  auto* rows_num = reinterpret_cast<int32_t*>(w + p->off_rows_num);
  auto* pnum = reinterpret_cast<int32_t*>(w + p->off_pnum);
  const Operands& op = p->op;
  const BinOffsets no = offsets_of(p->num_counts);
  int64_t ndense = 0;
  for (int b = kDenseBinBase; b < kEscBinBase; ++b) ndense += static_cast<int64_t>(p->num_counts[b]);
  p->ran[SPG_PHASE_NUM_HASH] = p->ran[SPG_PHASE_NUM_DENSE] = p->ran[SPG_PHASE_NUM_PANELS] = false;
  p->ran[SPG_PHASE_NUM_EXPAND] = p->ran[SPG_PHASE_NUM_RANK] = p->ran[SPG_PHASE_NUM_ESC] = false;
  const bool sub = p->split && p->n_dense_sym > 0;
  const BinOffsets sbo = offsets_of(p->sub_counts);
  int64_t nsub_dense = 0;
  for (int b = kDenseBinBase; b < kNumBins; ++b) nsub_dense += static_cast<int64_t>(p->sub_counts[b]);
  const int32_t* rows_dense_sym =
      reinterpret_cast<const int32_t*>(w + p->off_rows_sym) + offsets_of(p->sym_counts).v[kDenseBinBase];
  const int32_t* subitems = reinterpret_cast<const int32_t*>(w + p->off_subitems);
  const int32_t* subcnt = reinterpret_cast<const int32_t*>(w + p->off_subcnt);
  const int32_t* suboff = reinterpret_cast<const int32_t*>(w + p->off_suboff);
  const int32_t* wend = reinterpret_cast<const int32_t*>(w + p->off_wend);
  p->ran[SPG_PHASE_SEG_WRITE] = false;
  if ((ndense > 0 || sub) && p->num_P > 1) {
    if (p->ext_pnum && !p->b_resorted) {
      pnum = const_cast<int32_t*>(p->ext_pnum);
    } else if (!p->pnum_ready) {
      PhaseTimer tp(p, SPG_PHASE_NUM_PANELS);
      SPG_TRY_HIP(launch_panel_index(op.b_ptr, op.b_idx, op.n, p->num_wlog2, p->num_P, pnum, s));
    }
  }
  const bool use_segs = sub && p->seg_total <= p->seg_cap;
  const auto* segoff = reinterpret_cast<const int64_t*>(w + p->off_segoff);
  void* segs = w + p->off_segs;
  if (use_segs) {
    PhaseTimer tw(p, SPG_PHASE_SEG_WRITE);
    SPG_TRY_HIP(launch_seg_write(op, rows_dense_sym, p->n_dense_sym, p->num_P, pnum, wend, segoff, segs, s));
  }
  {
    PhaseTimer t(p, SPG_PHASE_NUM_HASH);
    for (int c = 1; c < kExpandBin; ++c) {
      if (!p->num_counts[c]) continue;
      SPG_TRY_HIP(launch_hash_num(p->sr, op, rows_num + no.v[c], static_cast<int64_t>(p->num_counts[c]),
                                  hash_table_size(c), hash_threads_num(c, p->sr), p->opt.short_seg, p->c_ptr,
                                  c_idx, c_val, s));
    }
    if (sub) {
      for (int c = 1; c < kDenseBinBase; ++c) {
        if (!p->sub_counts[c]) continue;
        if (use_segs)
          SPG_TRY_HIP(launch_hash_num_seg(p->sr, op, rows_dense_sym, subitems + sbo.v[c],
                                          static_cast<int64_t>(p->sub_counts[c]), hash_table_size(c),
                                          hash_threads_num(c, p->sr), p->opt.short_seg, p->num_P, p->num_wlog2, segoff,
                                          segs, subcnt, suboff, p->c_ptr, c_idx, c_val, s));
        else
          SPG_TRY_HIP(launch_hash_num_sub(p->sr, op, rows_dense_sym, subitems + sbo.v[c],
                                          static_cast<int64_t>(p->sub_counts[c]), hash_table_size(c),
                                          hash_threads_num(c, p->sr), p->opt.short_seg, p->num_P, p->num_wlog2, pnum,
                                          subcnt, suboff, wend, p->c_ptr, c_idx, c_val, s));
      }
    }
  }
  if (p->bp.esc_max_flops > 0) {
    PhaseTimer t(p, SPG_PHASE_NUM_ESC);
    for (int b = kEscBinBase; b < kNumBins; ++b) {
      if (!p->num_counts[b]) continue;
      SPG_TRY_HIP(launch_esc_num(p->sr, op, rows_num + no.v[b], static_cast<int64_t>(p->num_counts[b]),
                                 32 << (b - kEscBinBase), p->c_ptr, c_idx, c_val, s));
    }
  }
  if (p->num_counts[kExpandBin]) {
    PhaseTimer t(p, SPG_PHASE_NUM_EXPAND);
    SPG_TRY_HIP(launch_expand_rows(rows_num + no.v[kExpandBin], static_cast<int64_t>(p->num_counts[kExpandBin]),
                                   static_cast<int>(p->keep_nwords), p->keep_stride,
                                   reinterpret_cast<const uint32_t*>(w + p->off_store),
                                   reinterpret_cast<const int32_t*>(w + p->off_rowslot), p->c_ptr, c_idx,
                                   1024, s));
  }
  const bool ranked = p->rank && p->n_dense_sym > 0;
  auto* pchunk = reinterpret_cast<int32_t*>(w + p->off_pchunk);
  Operands opr = op;  // the rank passes' view of the operands
  if (ranked) {
    PhaseTimer tp(p, SPG_PHASE_NUM_PANELS);
    SPG_TRY_HIP(launch_panel_index(op.b_ptr, op.b_idx, op.n, p->rank_cw, p->rank_NC, pchunk, s));
    bool packed = false;
    if (p->pair && p->sr == SPG_MIN_PLUS_I32 && p->opt.pack_b >= 0 && p->b_nnz > 0) {
      // int32 values that fit beside the column id in one word: half the
      // bytes per product (the pair area holds the words)
      const int bits = std::max(1, ilog2_ceil(op.k));
      if (bits < 31) {
        auto* mm = reinterpret_cast<int32_t*>(w + p->off_ctr) + 2 * kCtrRange;
        int32_t hmm[2] = {0, 0};
        SPG_TRY_HIP(launch_value_range(static_cast<const int32_t*>(op.b_val), p->b_nnz, mm, s));
        SPG_TRY_HIP(hipMemcpyAsync(hmm, mm, sizeof(hmm), hipMemcpyDeviceToHost, s));
        SPG_TRY_HIP(hipStreamSynchronize(s));
        if (hmm[0] >= 0 && static_cast<int64_t>(hmm[1]) < (int64_t(1) << (32 - bits))) {
          auto* bw = reinterpret_cast<uint32_t*>(w + p->off_bpair);
          SPG_TRY_HIP(launch_pack_b(op, p->b_nnz, bits, bw, s));
          opr.b_packed = bw;
          opr.pack_bits = bits;
          packed = true;
        }
      }
    }
    if (p->pair && !packed) {
      auto* bp = reinterpret_cast<int2*>(w + p->off_bpair);
      SPG_TRY_HIP(launch_interleave_b(op, p->b_nnz, bp, s));
      opr.b_pair = bp;
    }
  }
  const uint32_t* kstore = p->keep ? reinterpret_cast<const uint32_t*>(w + p->off_store) : nullptr;
  const int32_t* kslot = p->keep ? reinterpret_cast<const int32_t*>(w + p->off_rowslot) : nullptr;
  const int32_t* rcnt = reinterpret_cast<const int32_t*>(w + p->off_rcnt);
  // Heavy rows by size: rank passes, then fixed panels from fixed_lo entries
  // (nnz * rank_dense_div >= k).
  const int64_t kcols = op.k;
  const int64_t fixed_lo = std::max<int64_t>(p->bp.hash_max_nnz + 1,
                                             (kcols + p->opt.rank_dense_div - 1) / p->opt.rank_dense_div);
  RankShapes shapes = p->rank_shapes;
  shapes.flops = reinterpret_cast<const int64_t*>(w + p->off_flops);
  shapes.esc_max_flops = p->bp.esc_max_flops;
  shapes.esc_ratio_x16 = p->bp.esc_ratio_x16;
  auto rank_launch = [&](bool fixed) {
    return launch_rank_num(p->sr, fixed, opr, rows_dense_sym, p->n_dense_sym, p->lists_rb, p->lists_re,
                           p->rank_cw, p->rank_NC, shapes, pchunk, rcnt,
                           fixed ? fixed_lo : p->bp.hash_max_nnz + 1, fixed ? INT64_MAX : fixed_lo, p->num_wlog2,
                           p->num_P, p->opt.dense_threads, p->opt.short_seg, kstore, kslot, p->keep_stride,
                           p->c_ptr, c_idx, c_val, s);
  };
  if (ndense > 0 || nsub_dense > 0 || ranked) {
    PhaseTimer t(p, SPG_PHASE_NUM_DENSE);
    if (ndense > 0)
      SPG_TRY_HIP(launch_dense_num(p->sr, op, rows_num + no.v[kDenseBinBase], ndense, p->num_wlog2,
                                   p->num_P, pnum, p->opt.dense_threads, p->opt.short_seg, p->c_ptr,
                                   c_idx, c_val, s));
    if (sub && nsub_dense > 0 && use_segs)
      SPG_TRY_HIP(launch_dense_num_seg(p->sr, op, rows_dense_sym, subitems + sbo.v[kDenseBinBase], nsub_dense,
                                       p->opt.dense_threads, p->opt.short_seg, p->num_P, p->num_wlog2, segoff,
                                       segs, subcnt, suboff, p->c_ptr, c_idx, c_val, s));
    else if (sub && nsub_dense > 0)
      SPG_TRY_HIP(launch_dense_num_sub(p->sr, op, rows_dense_sym, subitems + sbo.v[kDenseBinBase], nsub_dense,
                                       p->opt.dense_threads, p->opt.short_seg, p->num_P, p->num_wlog2, pnum,
                                       subcnt, suboff, p->c_ptr, c_idx, c_val, s));
    // heavy rows dense enough for fixed panels
    if (ranked) SPG_TRY_HIP(rank_launch(true));
  }
  if (ranked) {
    PhaseTimer t(p, SPG_PHASE_NUM_RANK);
    SPG_TRY_HIP(rank_launch(false));
  }
  return SPG_OK;
}

spg_status spg_numeric(spg_plan* p, void* ws, int32_t* c_idx, void* c_val) {
  if (!p) return SPG_E_INVALID;
  return numeric_range(p, ws, 0, p->op.m, c_idx, c_val);
}

spg_status spg_numeric_rows(spg_plan* p, void* ws, int64_t row_begin, int64_t row_end, int32_t* c_idx,
                            void* c_val) {
  if (!p) return SPG_E_INVALID;
  if (row_begin < 0 || row_end < row_begin || row_end > p->op.m) return SPG_E_INVALID;
  return numeric_range(p, ws, static_cast<int32_t>(row_begin), static_cast<int32_t>(row_end), c_idx, c_val);
}

spg_status spg_matrix_check(const spg_matrix* M, void* ws, void* stream, int* flags) {
  spg_status st = check_matrix(M);
  if (st != SPG_OK) return st;
  if (!ws) return SPG_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t nmajor = M->layout == SPG_CSR ? M->nrows : M->ncols;
  const int32_t nminor = M->layout == SPG_CSR ? M->ncols : M->nrows;
  int* err = static_cast<int*>(ws);
  int h = 0;
  if (nmajor == 0) {
    h = M->nnz != 0 ? kCheckEnds : 0;
  } else {
    SPG_TRY_HIP(launch_fill_u64(static_cast<uint64_t*>(ws), 1, 0, s));
    SPG_TRY_HIP(launch_validate(M->ptr, M->idx, nmajor, M->nnz, nminor, err, s));
    SPG_TRY_HIP(hipMemcpyAsync(&h, err, sizeof(int), hipMemcpyDeviceToHost, s));
    SPG_TRY_HIP(hipStreamSynchronize(s));
  }
  if (flags) *flags = h;
  return h ? SPG_E_INVALID : SPG_OK;
}

spg_status spg_prune_workspace_size(const spg_matrix* C, size_t* bytes) {
  spg_status st = check_matrix(C);
  if (st != SPG_OK) return st;
  if (!bytes) return SPG_E_INVALID;
  const int64_t nmajor = C->layout == SPG_CSR ? C->nrows : C->ncols;
  *bytes = align_up(static_cast<size_t>((nmajor + kScanTile - 1) / kScanTile + 1) * sizeof(int64_t));
  return SPG_OK;
}

}  // extern "C"

// Count phase of the prune with the scan's tile partials in `partials`
// (at least (nslices + kScanTile - 1) / kScanTile words; every word the scan
// reads it writes first, so nothing needs clearing).
static spg_status prune_count(const spg_matrix* C, float thresh, int64_t* partials, hipStream_t s,
                              int64_t* new_ptr, int64_t* new_nnz) {
  const int64_t nmajor = C->layout == SPG_CSR ? C->nrows : C->ncols;
  SPG_TRY_HIP(launch_prune_count(C->ptr, static_cast<const float*>(C->val), nmajor, thresh, new_ptr, s));
  SPG_TRY_HIP(launch_scan_inplace(new_ptr + 1, nmajor, partials, s));
  int64_t total = 0;
  SPG_TRY_HIP(hipMemcpyAsync(&total, new_ptr + nmajor, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipStreamSynchronize(s));
  *new_nnz = total;
  return SPG_OK;
}

// Scratch of spg_prune_count_f32_noalloc: the scan's tile partials.  Every
// GPU the library runs on holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for
// that device (the array's name is not a device address on the host).
static __device__ __align__(256) int64_t scratch[SPG_NOALLOC_SCRATCH_WORDS];
static_assert(SPG_NOALLOC_MAX_SLICES <= static_cast<int64_t>(SPG_NOALLOC_SCRATCH_WORDS - 1) * kScanTile,
              "the scan of SPG_NOALLOC_MAX_SLICES slices needs more tile partials than the scratch holds");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int64_t* g_scratch_addr[kMaxDevices];  // device address of `scratch`, per device

// Address of `scratch` on the current device, looked up on the first call
// for that device.
spg_status scratch_address(int64_t** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SPG_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* a = nullptr;
    if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) return SPG_E_DEVICE;
    g_scratch_addr[dev] = static_cast<int64_t*>(a);
  }
  *out = g_scratch_addr[dev];
  return SPG_OK;
}
}  // namespace

extern "C" {

spg_status spg_prune_count_f32(const spg_matrix* C, float thresh, void* ws, void* stream,
                               int64_t* new_ptr, int64_t* new_nnz) {
  spg_status st = check_matrix(C);
  if (st != SPG_OK) return st;
  if (!new_ptr || !new_nnz || !ws) return SPG_E_INVALID;
  if (C->nnz > 0 && !C->val) return SPG_E_SEMIRING;
  return prune_count(C, thresh, static_cast<int64_t*>(ws), static_cast<hipStream_t>(stream), new_ptr, new_nnz);
}

spg_status spg_prune_count_f32_noalloc(const spg_matrix* C, float thresh, void* stream, int64_t* new_ptr,
                                       int64_t* new_nnz) {
  spg_status st = check_matrix(C);
  if (st != SPG_OK) return st;
  if (!new_ptr || !new_nnz) return SPG_E_INVALID;
  if (C->nnz > 0 && !C->val) return SPG_E_SEMIRING;
  const int64_t nmajor = C->layout == SPG_CSR ? C->nrows : C->ncols;
  if (nmajor > SPG_NOALLOC_MAX_SLICES) return SPG_E_NOMEM;
  int64_t* partials = nullptr;
  if ((st = scratch_address(&partials)) != SPG_OK) return st;
  return prune_count(C, thresh, partials, static_cast<hipStream_t>(stream), new_ptr, new_nnz);
}

spg_status spg_select_count_f32(const spg_matrix* C, int64_t S, void* ws, void* stream, int64_t* new_ptr,
                                int64_t* new_nnz) {
  spg_status st = check_matrix(C);
  if (st != SPG_OK) return st;
  if (!new_ptr || !new_nnz || !ws || S < 0) return SPG_E_INVALID;
  if (C->nnz > 0 && !C->val) return SPG_E_SEMIRING;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t nmajor = C->layout == SPG_CSR ? C->nrows : C->ncols;
  SPG_TRY_HIP(launch_select_count(C->ptr, nmajor, S, new_ptr, s));
  SPG_TRY_HIP(launch_scan_inplace(new_ptr + 1, nmajor, static_cast<int64_t*>(ws), s));
  int64_t total = 0;
  SPG_TRY_HIP(hipMemcpyAsync(&total, new_ptr + nmajor, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPG_TRY_HIP(hipStreamSynchronize(s));
  *new_nnz = total;
  return SPG_OK;
}

spg_status spg_select_apply_f32(const spg_matrix* C, int64_t S, void* ws, void* stream, const int64_t* new_ptr,
                                int32_t* new_idx, float* new_val) {
  spg_status st = check_matrix(C);
  if (st != SPG_OK) return st;
  (void)ws;
  if (!new_ptr || S < 0) return SPG_E_INVALID;
  if (C->nnz > 0 && !C->val) return SPG_E_SEMIRING;
  const int64_t nmajor = C->layout == SPG_CSR ? C->nrows : C->ncols;
  SPG_TRY_HIP(launch_select_apply(C->ptr, C->idx, static_cast<const float*>(C->val), nmajor, S, new_ptr, new_idx,
                                  new_val, static_cast<hipStream_t>(stream)));
  return SPG_OK;
}

spg_status spg_inflate_f32(const spg_matrix* C, float r, float* val_out, void* stream) {
  spg_status st = check_matrix(C);
  if (st != SPG_OK) return st;
  if (C->nnz > 0 && (!C->val || !val_out)) return SPG_E_INVALID;
  if (!(r > 0.0f)) return SPG_E_INVALID;
  const int64_t nmajor = C->layout == SPG_CSR ? C->nrows : C->ncols;
  SPG_TRY_HIP(launch_inflate(C->ptr, static_cast<const float*>(C->val), nmajor, r, val_out,
                             static_cast<hipStream_t>(stream)));
  return SPG_OK;
}

spg_status spg_prune_apply_f32(const spg_matrix* C, float thresh, void* ws, void* stream,
                               const int64_t* new_ptr, int32_t* new_idx, float* new_val) {
  spg_status st = check_matrix(C);
  if (st != SPG_OK) return st;
  (void)ws;
  if (!new_ptr) return SPG_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t nmajor = C->layout == SPG_CSR ? C->nrows : C->ncols;
  SPG_TRY_HIP(launch_prune_apply(C->ptr, C->idx, static_cast<const float*>(C->val), nmajor, thresh,
                                 new_ptr, new_idx, new_val, s));
  return SPG_OK;
}

}  // extern "C"
