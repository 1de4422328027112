/* spg.h -- local semiring sparse-times-sparse product C = A (x).(+) B on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (paper Sec. 3.1): C = AB with A in S^{m x n}, B in S^{n x k}
 * over a semiring S (Sec. 1: user-defined semirings over several value types;
 * Sec. 2: compressed column / row storage with compact local indices):
 *
 *     C(i,j) = (+)_{k : A(i,k) and B(k,j) stored}  A(i,k) (x) B(k,j)
 *
 * The pattern of C is structural: an entry is stored whenever at least one
 * product contributes to it, even if its value equals the additive identity.
 * Output slices (rows for CSR, columns for CSC) are sorted ascending.
 *
 * Like the paper's node-level product (Sec. 4.1: flop estimation, a symbolic
 * phase that sizes C, then a numeric phase), a product is two calls:
 * spg_symbolic() computes the offsets of C and its entry count, the caller
 * allocates C, and spg_numeric() fills it.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Device pointers are HIP device addresses (e.g. torch tensor data
 *   pointers); host pointers are ordinary memory.  Every device buffer is
 *   owned by the caller; the library never allocates or frees device memory.
 *   Temporary device memory comes from the caller's workspace.  The only
 *   library-owned objects are the small host-side plans.
 * - All device work is enqueued on the stream given at plan creation (a
 *   hipStream_t passed as void*; NULL is the default stream).  A call that
 *   returns a value on the host synchronises that stream before returning.
 * - Errors are reported as spg_status codes; nothing aborts or throws across
 *   this interface.  Asynchronous device faults surface as SPG_E_DEVICE at
 *   the next synchronising call.
 * - Plans are not thread-safe; use one plan per thread and stream.
 */
#ifndef SPG_H_
#define SPG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spg_status {
  SPG_OK = 0,
  SPG_E_INVALID = 1,   /* bad argument: NULL pointer, malformed matrix */
  SPG_E_SHAPE = 2,     /* inner dimensions differ, or a dimension < 0 */
  SPG_E_LAYOUT = 3,    /* unknown layout, or A and B in different layouts */
  SPG_E_SEMIRING = 4,  /* unknown semiring code, or values missing */
  SPG_E_NOMEM = 5,     /* workspace too small, or a request over budget */
  SPG_E_OVERFLOW = 6,  /* a count or index exceeds its integer type */
  SPG_E_DEVICE = 7,    /* a HIP runtime call or kernel failed */
  SPG_E_STATE = 8      /* calls out of order (create -> symbolic -> numeric) */
} spg_status;

/* Semiring codes: ((+), (x), value type).  The (+)-identity is never stored.
 *  SPG_PLUS_TIMES_F64  (+, x) float64
 *  SPG_PLUS_TIMES_F32  (+, x) float32 with float32 accumulation
 *  SPG_MIN_PLUS_I32    (min, +) int32; + is saturating (int64 sum clamped to
 *                      the int32 range), so INT32_MAX acts as +infinity
 *  SPG_MIN_PLUS_F32    (min, +) float32
 *  SPG_OR_AND_BOOL     (OR, AND) uint8 values in {0,1}; values may be NULL,
 *                      meaning every stored entry is true (pattern only)
 *  SPG_MAX_TIMES_F64   (max, x) float64
 *  SPG_MAX_TIMES_F32   (max, x) float32
 * min and max on floating point use the total order in which -0 < +0, so
 * those results do not depend on summation order.  (+, x) results do, in the
 * last bits: the accumulation order on the device is unspecified. */
typedef enum spg_semiring {
  SPG_PLUS_TIMES_F64 = 0,
  SPG_PLUS_TIMES_F32 = 1,
  SPG_MIN_PLUS_I32 = 2,
  SPG_MIN_PLUS_F32 = 3,
  SPG_OR_AND_BOOL = 4,
  SPG_MAX_TIMES_F64 = 5,
  SPG_MAX_TIMES_F32 = 6
} spg_semiring;

typedef enum spg_layout { SPG_CSR = 0, SPG_CSC = 1 } spg_layout;

/* A compressed sparse matrix held in device memory.
 *  CSR: ptr has nrows+1 entries, idx holds column ids of each row.
 *  CSC: ptr has ncols+1 entries, idx holds row ids of each column.
 * ptr[0] == 0, ptr is non-decreasing and ptr[last] == nnz.  Ids lie in
 * [0, minor dimension) with no duplicate within a slice; they need not be
 * sorted (the paper's local matrices promise no order, Sec. 2.1): every
 * symbolic phase checks the operands on the device and sorts the slices of
 * an unsorted operand into the plan's workspace first (options.unsorted).
 * val holds nnz values of the semiring's value type (double, float, int32_t
 * or uint8_t), or NULL for SPG_OR_AND_BOOL (all true).  The library only
 * reads them. */
typedef struct spg_matrix {
  int32_t nrows;
  int32_t ncols;
  int64_t nnz;
  spg_layout layout;
  const int64_t* ptr;
  const int32_t* idx;
  const void* val;
} spg_matrix;

/* Tuning knobs; a zero field takes its default.  Bins follow the paper's
 * per-slice choice of accumulator by expected output size (Sec. 4.1, hybrid
 * hash/heap by compression ratio). */
typedef struct spg_options {
  int32_t validate;        /* ignored: every symbolic phase checks both
                              operands on the device (offsets, id range,
                              order); a malformed operand gives SPG_E_INVALID */
  int32_t hash_max_flops;  /* symbolic: rows with more products than this use
                              the dense bitmap accumulator (default 4096) */
  int32_t hash_max_nnz;    /* numeric: rows with more output entries than this
                              use the rank or dense panel accumulators (at
                              most 8192, and only where a table of twice that
                              fits in LDS; default 4096) */
  int32_t short_seg;       /* B-row segments up to this length are walked by
                              one lane; longer ones are split across the
                              waves of a workgroup (default 32) */
  int32_t dense_threads;   /* workgroup size of the dense kernels (default 1024) */
  int32_t sym_panel_log2;  /* log2 of the dense symbolic bitmap width in
                              columns (default 20, i.e. 128 KiB) */
  int32_t lds_budget;      /* bytes of LDS a dense numeric workgroup may use for
                              its panel (default 131072) */
  int32_t timing;          /* 1: record HIP events around every phase on the
                              plan's stream (read with spg_plan_timings) */
  int32_t split_panels;    /* numeric phase of rows that took the dense
                              symbolic path, when the value panels are
                              narrower than C: 1 splits each such row into
                              column windows of at most hash_max_nnz entries
                              (one work item each, LDS hash or one dense
                              panel); 0 (default) or -1 processes the panels
                              of a row in sequence in one workgroup */
  int32_t bitmap_mib;      /* MiB of workspace in which the symbolic phase
                              keeps the column bitmaps of its heaviest rows
                              (C no wider than the symbolic bitmap): a
                              pattern-only (OR,AND) product expands them in
                              its numeric phase instead of recomputing; rank
                              passes read their pattern from them (default 0:
                              off) */
  int32_t seg_mib;         /* MiB of workspace for the segment lists of
                              (row, panel) pieces (default 16384); a product
                              that needs more falls back to re-walking each
                              row per piece */
  int32_t rank_panels;     /* numeric phase of heavy valued rows (more than
                              hash_max_nnz entries, dense symbolic path) when
                              the value panels are narrower than C: 0
                              (default) or 1 = passes over runs of column
                              chunks whose entries fit the LDS value slots,
                              each entry stored at its column's rank; -1 =
                              fixed-width panels in sequence */
  int32_t rank_dense_div;  /* rows with nnz * rank_dense_div >= columns of C
                              keep fixed-width panels (default 1: only full
                              rows) */
  int32_t rank_shapes;     /* pass shapes of the rank passes: 1 = the value
                              slots of one chunk width (2^cw) with the widest
                              bitmap; 2 to 5 add 1.25x, 1.5x, 1.75x and 2x the
                              slots over fewer chunks; 6 adds 0.75x the slots
                              over more chunks; each row takes the shape that
                              needs the fewest passes (default 6) */
  int32_t unsorted;        /* operands whose slices are not sorted ascending:
                              0 (default) they are sorted into the workspace,
                              which holds room for sorted copies of both
                              operands' ids and values; -1 no room is held and
                              they give SPG_E_INVALID */
  int32_t b_checked;       /* 1: the right-hand operand (B; A for CSC
                              products, the operand whose slices are
                              gathered) passed spg_matrix_check and has not
                              changed since: its device check is skipped and
                              no room is held to sort it.  For a resident
                              operand shared by many plans. */
  int32_t sym_windows;     /* symbolic phase of the rows past hash_max_flops:
                              0 or 1 (default) = one bitmap per row
                              (sym_panel_log2 wide, panel after panel); N > 1
                              = N column windows, each (row, window) a work
                              item of its own, the workgroups of one XCD taking
                              the items of one window first (more L2 reuse of
                              B, more work per item) */
  int32_t win_threads;     /* workgroup size of the windowed kernels
                              (default 256) */
  int32_t win_wgs;         /* workgroups per compute unit of the windowed
                              kernels (default 8) */
  int32_t pack_b;          /* (min,+) int32 rank passes: 0 (default) read B
                              through one 32-bit word per entry (value <<
                              bits | column) when every value of B lies in
                              [0, 2^(32 - bits)) with bits = ceil(log2
                              columns), else through 8-byte (column, value)
                              pairs; -1 always through pairs */
  int32_t esc_max_flops;   /* numeric phase: rows of at most this many
                              products (up to 8192; 0 = 8192, -1 = never)
                              whose compression ratio
                              flops / nnz is at most esc_ratio_x16 / 16 are
                              expanded, sorted and compressed in LDS instead
                              of hashed or ranked */
  int32_t esc_ratio_x16;   /* 16 x that compression ratio (default 32: 2;
                              20: 1.25 in batched plans) */
} spg_options;

/* Phases reported by spg_plan_timings, in milliseconds. */
enum {
  SPG_PHASE_VALIDATE = 0,    /* operand check kernels */
  SPG_PHASE_FLOPS_BIN = 1,   /* per-row flop count, binning, row lists */
  SPG_PHASE_SYM_HASH = 2,    /* symbolic, LDS hash rows */
  SPG_PHASE_SYM_DENSE = 3,   /* symbolic, dense bitmap rows */
  SPG_PHASE_SCAN = 4,        /* offsets scan and numeric binning */
  SPG_PHASE_NUM_HASH = 5,    /* numeric, LDS hash rows (with in-row sort) */
  SPG_PHASE_NUM_DENSE = 6,   /* numeric, dense panel rows */
  SPG_PHASE_SYM_PANELS = 7,  /* panel index of B for the symbolic bitmap */
  SPG_PHASE_NUM_PANELS = 8,  /* panel index of B for the numeric panels */
  SPG_PHASE_NUM_EXPAND = 9,  /* numeric, rows expanded from kept bitmaps */
  SPG_PHASE_SEG_COUNT = 10,  /* symbolic, segment counts of (row, panel) pieces */
  SPG_PHASE_SEG_WRITE = 11,  /* numeric, segment lists of (row, panel) pieces */
  SPG_PHASE_NUM_RANK = 12,   /* numeric, heavy valued rows by rank-compressed panels */
  SPG_PHASE_NUM_ESC = 13,    /* numeric, expand-sort-compress rows */
  SPG_NUM_PHASES = 14
};

typedef struct spg_plan spg_plan;

/* Creates a plan for C = A (x).(+) B.  Host-only: checks the descriptors
 * (non-NULL arrays, matching inner dimension, one shared layout, semiring
 * code, values present unless SPG_OR_AND_BOOL) and records the stream; it
 * launches nothing.  A and B must stay valid until the plan is destroyed.
 * CSC operands give a CSC result, computed through (AB)^T = B^T A^T on the
 * same arrays.  opt may be NULL.  *out receives the plan. */
spg_status spg_plan_create(const spg_matrix* A, const spg_matrix* B, spg_semiring sr,
                           const spg_options* opt, void* stream, spg_plan** out);

/* Semiring sum of k matrices of one shape, C(i,j) = (+)_t P_t(i,j) over the
 * parts that hold (i,j): the merge of the partial products that the stages
 * of Sparse SUMMA produce (paper Sec. 3.2: each process accumulates the
 * local products of every stage), and elementwise semiring addition (k = 2).
 * The parts come stacked in one matrix P in either layout: with m slices
 * per part, slice i of part t is slice t*m + i of P (so P has k*m rows in
 * CSR, k*m columns in CSC), each sorted strictly ascending.  C has m slices
 * in P's layout.  The plan is used like a product plan: spg_workspace_size,
 * spg_symbolic, spg_numeric, spg_plan_destroy.  It runs as C = S P with S
 * the m x (k m) selector whose slice i holds the (x)-identity at t*m + i,
 * built in the workspace by spg_symbolic, so a sum entry is combined with
 * the semiring's own (+) and no value changes on the way (x (x) one = x).
 * P must stay valid until the plan is destroyed.
 * Errors: SPG_E_INVALID (k < 1, bad descriptor), SPG_E_SHAPE (slices not a
 * multiple of k), SPG_E_SEMIRING (bad code or missing values). */
spg_status spg_sum_plan_create(int k, const spg_matrix* P, spg_semiring sr, const spg_options* opt,
                               void* stream, spg_plan** out);

/* Bytes of device workspace the plan needs (256-byte aligned base).  The same
 * workspace must be passed, untouched, to spg_symbolic and spg_numeric. */
spg_status spg_workspace_size(const spg_plan* plan, size_t* bytes);

/* Symbolic phase (paper Sec. 4.1 phases 1-2): the operand check, per-slice
 * flop count and binning, the pattern size of every output slice, and the
 * exclusive scan into c_ptr.  The check covers offsets, id range and order:
 * a malformed operand or a duplicate id gives SPG_E_INVALID before any
 * kernel uses it to index; an operand with unsorted slices is sorted into
 * the workspace and the product runs on the sorted copy (its values moved
 * with their ids), unless options.unsorted = -1 (SPG_E_INVALID).
 *   ws     device workspace of spg_workspace_size() bytes
 *   c_ptr  device, int64[nslices+1] (nslices = rows of C for CSR, columns of
 *          C for CSC), written
 *   c_nnz  host, receives nnz(C)
 * Synchronises the stream. */
spg_status spg_symbolic(spg_plan* plan, void* ws, int64_t* c_ptr, int64_t* c_nnz);

/* Numeric phase (paper Sec. 4.1 phase 3): fills C's ids (sorted within each
 * slice) and values.  Call after spg_symbolic with the same workspace and
 * c_ptr.
 *   c_idx  device, int32[nnz(C)]
 *   c_val  device, nnz(C) values of the output type (double, float, int32_t,
 *          uint8_t per semiring); may be NULL only for SPG_OR_AND_BOOL with
 *          pattern-only operands.
 * Asynchronous: returns once the work is enqueued. */
spg_status spg_numeric(spg_plan* plan, void* ws, int32_t* c_idx, void* c_val);

/* Numeric phase of output slices [row_begin, row_end) only: forming C in
 * batches when the whole output does not fit in memory (paper Sec. 7.2 and
 * 7.3: the product is formed in b batches, b computed from a symbolic step).
 * After one spg_symbolic, the caller picks slice ranges from c_ptr (each
 * range's entries are c_ptr[row_end] - c_ptr[row_begin]) and calls this once
 * per range, into buffers that need only hold that range:
 *   c_idx  device, int32[c_ptr[row_end] - c_ptr[row_begin]]; entry e of
 *          slice r (e from 0) is written at c_ptr[r] - c_ptr[row_begin] + e
 *   c_val  device, values of the same count and position (rules of
 *          spg_numeric)
 * The ids and values written are those spg_numeric writes for these slices.
 * Each call re-bins the numeric row lists of its range (one device pass over
 * the range and one device-to-host copy, which synchronise the stream); the
 * kernels then run asynchronously.  A plan and its workspace run one range
 * at a time; calls on one stream are ordered.  spg_numeric afterwards
 * re-bins the whole product by itself; in between, spg_plan_bins reports the
 * numeric classes of the last range.
 * Errors: SPG_E_INVALID (range outside [0, nslices], row_end < row_begin,
 * NULL outputs for a non-empty range), SPG_E_STATE (no symbolic phase yet,
 * or a plan with options.split_panels = 1 and a range that is not the whole
 * product: its (slice, window) work items span every slice). */
spg_status spg_numeric_rows(spg_plan* plan, void* ws, int64_t row_begin, int64_t row_end, int32_t* c_idx,
                            void* c_val);

/* Statistics of the last symbolic phase (host): total products (flops, the
 * paper's count of nonzero multiplications) and number of output slices. */
spg_status spg_plan_stats(const spg_plan* plan, int64_t* flops, int64_t* nslices);

/* Elapsed time of each phase of the last symbolic + numeric calls (ms[i]
 * for phase i < SPG_NUM_PHASES; 0 for a phase that did not run), measured
 * with HIP events on the plan's stream.  Needs options.timing = 1;
 * synchronises the stream. */
spg_status spg_plan_timings(spg_plan* plan, float* ms);

/* Number of output slices per accumulator class after the symbolic phase:
 * counts[0] empty, counts[1..15] LDS hash classes (class c holds slices of at
 * most 32 << (c-1) products in symbolic / entries in numeric), counts[16..63]
 * dense classes.  sym and num each receive 64 entries; either may be NULL. */
spg_status spg_plan_bins(const spg_plan* plan, int64_t* sym, int64_t* num);

spg_status spg_plan_destroy(spg_plan* plan);

/* The options the plan runs with, defaults filled in (host, after plan
 * creation).  Errors: SPG_E_INVALID for a NULL argument. */
spg_status spg_plan_options(const spg_plan* plan, spg_options* out);

const char* spg_status_str(spg_status s);

/* Device check of one matrix (the check every symbolic phase runs on its
 * operands): ptr[0] == 0, non-decreasing offsets within [0, nnz],
 * ptr[last] == nnz, ids in [0, minor dimension), no duplicate id in a slice,
 * slices sorted ascending.
 *   ws      device scratch of at least 256 bytes (written)
 * Synchronises `stream`.  Returns SPG_OK for a well-formed matrix with sorted
 * slices, SPG_E_INVALID otherwise; *flags (may be NULL) receives the error
 * bits: 1 bad first/last offset, 2 bad offsets, 4 id out of range,
 * 8 unsorted slice, 16 duplicate id. */
spg_status spg_matrix_check(const spg_matrix* M, void* ws, void* stream, int* flags);

/* Column panels.  A dense row accumulator covers 2^wlog2 columns of C at a
 * time; when C is wider, the plan uses P = ceil(ncols(C) / 2^wlog2) panels
 * and a panel index of the right-hand CSR operand: for every row k of it,
 * P+1 int32 offsets (relative to the row start) of the first entry with
 * column >= p * 2^wlog2.  A caller that multiplies many left operands by one
 * resident right operand (a served adjacency matrix) can build the index
 * once and hand it to every plan.
 *   spg_plan_panels:        the plan's widths and panel counts (host), after
 *                           plan creation
 *   spg_panel_index_size:   bytes of the index for operand R (CSR, the
 *                           right-hand operand as the kernels see it)
 *   spg_panel_index_build:  builds it into `out` (device) on `stream`; R's
 *                           slices must be sorted (spg_matrix_check): for
 *                           an unsorted slice every entry of the index is
 *                           still written, with a value in [0, slice length],
 *                           but it does not locate the panels
 *   spg_plan_set_panels:    which = 0 symbolic, 1 numeric; `pidx` (device,
 *                           caller-owned, built with the plan's wlog2) is used
 *                           instead of building one in the workspace.
 * Errors: SPG_E_INVALID for a wlog2 that does not match the plan. */
spg_status spg_plan_panels(const spg_plan* plan, int* sym_wlog2, int* sym_P, int* num_wlog2,
                           int* num_P);
spg_status spg_panel_index_size(const spg_matrix* R, int wlog2, size_t* bytes);
spg_status spg_panel_index_build(const spg_matrix* R, int wlog2, void* out, void* stream);
spg_status spg_plan_set_panels(spg_plan* plan, int which, const void* pidx, int wlog2);

/* Pruning of a float32 matrix (the Markov-clustering step after expansion;
 * paper Sec. 7.5: HipMCL runs each expansion's SpGEMM inside an iteration of
 * expansion, pruning and inflation, and Sec. 7.3 squares protein-similarity
 * matrices for it): keep entries with value >= thresh, drop the rest, order
 * unchanged.  Two phases like the product: the count phase sizes the result,
 * the caller allocates it, the apply phase fills it.  thresh is compared in
 * float32 with the stored values as they are.
 *   C          float32 matrix in device memory (either layout)
 *   ws         device workspace of at least spg_prune_workspace_size() bytes
 *   new_ptr    device int64[nslices+1], written by the count phase
 *   new_nnz    host, receives the kept count (synchronises the stream)
 *   new_idx/new_val  device outputs of new_nnz entries
 * Errors: SPG_E_INVALID (NULL outputs or workspace, bad descriptor),
 * SPG_E_SEMIRING (no values), SPG_E_DEVICE (a launch or the copy failed).
 * C must be well formed (the product's outputs are); it is not checked. */
spg_status spg_prune_workspace_size(const spg_matrix* C, size_t* bytes);
spg_status spg_prune_count_f32(const spg_matrix* C, float thresh, void* ws, void* stream,
                               int64_t* new_ptr, int64_t* new_nnz);
spg_status spg_prune_apply_f32(const spg_matrix* C, float thresh, void* ws, void* stream,
                               const int64_t* new_ptr, int32_t* new_idx, float* new_val);

/* Count phase of the prune for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): spg_prune_count_f32 with the workspace replaced by a 64 KiB
 * array of the library's own (SPG_NOALLOC_SCRATCH_WORDS int64 words of
 * device memory per GPU, held until the process ends).  It calls no
 * allocating routine.  Same arguments, results and errors as
 * spg_prune_count_f32, for C with at most SPG_NOALLOC_MAX_SLICES slices;
 * larger C gives SPG_E_NOMEM before any device work.  The stream must belong
 * to the current device.  Every call on one GPU uses the same array: calls
 * that overlap on one GPU (other streams, other host threads) race and must
 * be serialised by the caller.  The apply phase is spg_prune_apply_f32 (it
 * uses no workspace; pass ws = NULL). */
#define SPG_NOALLOC_SCRATCH_WORDS 8192
#define SPG_NOALLOC_MAX_SLICES ((int64_t)(SPG_NOALLOC_SCRATCH_WORDS - 1) * 8192)
spg_status spg_prune_count_f32_noalloc(const spg_matrix* C, float thresh, void* stream, int64_t* new_ptr,
                                       int64_t* new_nnz);

/* Selection (the Markov-clustering step that, with the prune, bounds the
 * entries kept per column; paper Sec. 7.5: HipMCL iterates expansion,
 * pruning and inflation, and keeps the output sparse around each
 * expansion): every slice with more than S entries keeps the S with the
 * largest values, ties going to the smaller id, values compared in float32
 * with -0 < +0; shorter slices are kept whole; the kept entries stay in id
 * order.  Two phases like the prune, with the same workspace
 * (spg_prune_workspace_size).
 *   C          float32 matrix in device memory (either layout), slices sorted
 *              by id with no duplicates (the product's outputs are)
 *   S          entries kept per slice, >= 0
 *   new_ptr    device int64[nslices+1], written by the count phase
 *   new_nnz    host, receives the kept count (synchronises the stream)
 *   new_idx/new_val  device outputs of new_nnz entries
 * Errors: SPG_E_INVALID (NULL outputs or workspace, S < 0, bad
 * descriptor), SPG_E_SEMIRING (no values), SPG_E_DEVICE (a launch or the
 * copy failed).  NaN values are undefined. */
spg_status spg_select_count_f32(const spg_matrix* C, int64_t S, void* ws, void* stream, int64_t* new_ptr,
                                int64_t* new_nnz);
spg_status spg_select_apply_f32(const spg_matrix* C, int64_t S, void* ws, void* stream, const int64_t* new_ptr,
                                int32_t* new_idx, float* new_val);

/* Inflation (the Markov-clustering step after pruning, paper Sec. 7.5: the
 * HipMCL iteration is expansion, pruning, inflation): every slice's values
 * raised to the power r and divided by their sum, so each slice sums to 1
 * again (slices are columns for the usual column-stochastic CSC matrix).
 *   C        float32 matrix in device memory (either layout), values >= 0
 *   r        inflation exponent, > 0
 *   val_out  device float[nnz]: the new values in C's entry order; may be
 *            C->val itself (in place).  Slices whose powers sum to 0 are left
 *            as they are (copied to val_out).  Powers in float32 (for
 *            r = 2 the single product v * v), their sum in float64.
 * Enqueues one kernel on `stream` and returns.
 * Errors: SPG_E_INVALID for r <= 0 or missing values. */
spg_status spg_inflate_f32(const spg_matrix* C, float r, float* val_out, void* stream);

/* ------------------------------------------------------------------------
 * Batched products: nprod independent products C_b = A_b (x).(+) B_b, such
 * as the block products of one 3D Sparse SUMMA stage (paper Sec. 3) or a set
 * of per-graph squares.  All rows of all products share one binning and one
 * launch per accumulator class and semiring; the numeric phase can be
 * captured into a hipGraph and replayed.  Each product follows the rules of
 * spg_plan_create (its own layout and semiring; at most 8 distinct kernel
 * semirings per batch).  Outputs are pooled:
 *   c_ptr_pool  device int64, sum over b of (nslices_b + 1) entries; product
 *               b's offsets (starting at 0) begin at sum_{b'<b} (nslices_b' + 1)
 *   c_idx pool  device int32; product b's ids begin at idx_off[b]
 *   c_val pool  device bytes; product b's values begin at byte val_off[b]
 *               (8-byte aligned), in its semiring's output type
 * ------------------------------------------------------------------------ */
typedef struct spg_batch_plan spg_batch_plan;

/* Host-only checks of all descriptors; semirings[b] is an spg_semiring code. */
spg_status spg_batch_plan_create(int nprod, const spg_matrix* A, const spg_matrix* B,
                                 const int* semirings, const spg_options* opt, void* stream,
                                 spg_batch_plan** out);
spg_status spg_batch_workspace_size(const spg_batch_plan* plan, size_t* bytes);

/* Symbolic phase of all products.  Host outputs (nprod+1 entries for
 * idx_off and val_off, the last holding the pool totals; nprod for c_nnz).
 * Synchronises the stream. */
spg_status spg_batch_symbolic(spg_batch_plan* plan, void* ws, int64_t* c_ptr_pool, int64_t* c_nnz,
                              int64_t* idx_off, int64_t* val_off);

/* Numeric phase of all products into the pools (val_off from the symbolic
 * call).  Enqueues the kernels and returns. */
spg_status spg_batch_numeric(spg_batch_plan* plan, void* ws, int32_t* c_idx, void* c_val,
                             const int64_t* val_off);

/* Captures the numeric phase (same arguments) into a hipGraph held by the
 * plan, without running it; spg_batch_graph_launch replays it on the plan's
 * stream.  The capture stays valid while the inputs, workspace and pools do,
 * until the next spg_batch_symbolic call, which drops it. */
spg_status spg_batch_graph_capture(spg_batch_plan* plan, void* ws, int32_t* c_idx, void* c_val,
                                   const int64_t* val_off);
spg_status spg_batch_graph_launch(spg_batch_plan* plan);

/* Total products and rows of the batch after the symbolic phase. */
spg_status spg_batch_stats(const spg_batch_plan* plan, int64_t* flops, int64_t* rows);

/* Phases reported by spg_batch_timings, in milliseconds: the launches of
 * every product's rows in one accumulator family (paper Sec. 4.1 phases (2)
 * and (3); per-stage timing of Sec. 7). */
#define SPG_BATCH_PHASE_SYM_HASH 0
#define SPG_BATCH_PHASE_SYM_DENSE 1
#define SPG_BATCH_PHASE_NUM_HASH 2
#define SPG_BATCH_PHASE_NUM_DENSE 3
#define SPG_BATCH_PHASE_NUM_ESC 4  /* expand-sort-compress rows */
#define SPG_BATCH_NUM_PHASES 5

/* Device time of each phase of the last eager spg_batch_symbolic /
 * spg_batch_numeric call (graph replays are not timed) into
 * ms[SPG_BATCH_NUM_PHASES]; 0 for a phase that launched nothing.  Needs
 * options.timing = 1 at plan creation (else SPG_E_STATE); synchronises the
 * plan's stream. */
spg_status spg_batch_timings(spg_batch_plan* plan, float* ms);
spg_status spg_batch_plan_destroy(spg_batch_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* SPG_H_ */
