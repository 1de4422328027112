// Device-side building blocks of the semiring sparse product on gfx950:
// semiring traits, block-wide scans, and the row enumerator that feeds every
// accumulator (LDS hash table or dense LDS panel).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spg {

constexpr int kWave = 64;
constexpr int kEmpty = -1;  // empty hash slot (column ids are >= 0)
constexpr int kPieceUnroll = 16;
constexpr int kPiece = kWave * kPieceUnroll;  // products per wave work unit

// ---------------------------------------------------------------------------
// Semirings.  Each trait gives the input value type In, the LDS storage type
// S (which may be an order-preserving integer encoding), the output type Out,
// the storage value of an untouched slot, the product a (x) b as storage, an
// atomic (+) into LDS, and the decoding to Out.  (Paper Sec. 1: semirings over
// user value types; the set here is fixed.)
// ---------------------------------------------------------------------------

// Float total order with -0 < +0 mapped onto unsigned integer order.
__device__ __forceinline__ uint32_t f32_key(float x) {
  uint32_t b = __float_as_uint(x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float f32_unkey(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k ^ 0x80000000u) : ~k);
}
__device__ __forceinline__ unsigned long long f64_key(double x) {
  unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double f64_unkey(unsigned long long k) {
  unsigned long long b = (k >> 63) ? (k ^ 0x8000000000000000ull) : ~k;
  return __longlong_as_double(static_cast<long long>(b));
}

struct SrPlusTimesF64 {
  static constexpr bool kNullable = false;
  using In = double;
  using S = double;
  using Out = double;
  static constexpr bool kPattern = false;
  __device__ static S identity() { return 0.0; }
  __device__ static S mul(In a, In b) { return a * b; }
  __device__ static void combine(S* p, S v) { atomicAdd(p, v); }
  __device__ static Out out(S s) { return s; }
};
struct SrPlusTimesF32 {
  static constexpr bool kNullable = false;
  using In = float;
  using S = float;
  using Out = float;
  static constexpr bool kPattern = false;
  __device__ static S identity() { return 0.0f; }
  __device__ static S mul(In a, In b) { return a * b; }
  __device__ static void combine(S* p, S v) { atomicAdd(p, v); }
  __device__ static Out out(S s) { return s; }
};
struct SrMinPlusI32 {
  static constexpr bool kNullable = false;
  using In = int32_t;
  using S = int32_t;
  using Out = int32_t;
  static constexpr bool kPattern = false;
  __device__ static S identity() { return INT32_MAX; }
  __device__ static S mul(In a, In b) {
    long long s = static_cast<long long>(a) + static_cast<long long>(b);
    s = s > INT32_MAX ? INT32_MAX : s;
    s = s < INT32_MIN ? INT32_MIN : s;
    return static_cast<S>(s);
  }
  __device__ static void combine(S* p, S v) { atomicMin(p, v); }
  __device__ static Out out(S s) { return s; }
};
struct SrMinPlusF32 {
  static constexpr bool kNullable = false;
  using In = float;
  using S = uint32_t;
  using Out = float;
  static constexpr bool kPattern = false;
  __device__ static S identity() { return 0xFFFFFFFFu; }
  __device__ static S mul(In a, In b) { return f32_key(a + b); }
  __device__ static void combine(S* p, S v) { atomicMin(p, v); }
  __device__ static Out out(S s) { return f32_unkey(s); }
};
struct SrOrAndBool {  // a NULL value array on either operand reads as all true
  using In = uint8_t;
  using S = uint32_t;
  using Out = uint8_t;
  static constexpr bool kPattern = false;
  static constexpr bool kNullable = true;
  __device__ static S identity() { return 0u; }
  __device__ static S mul(In a, In b) { return (a != 0 && b != 0) ? 1u : 0u; }
  __device__ static void combine(S* p, S v) {
    if (v) atomicOr(p, v);
  }
  __device__ static Out out(S s) { return static_cast<Out>(s != 0); }
};
// (OR,AND) with NULL values on both operands: only the pattern is computed.
struct SrPattern {
  static constexpr bool kNullable = false;
  using In = uint8_t;
  using S = uint32_t;
  using Out = uint8_t;
  static constexpr bool kPattern = true;
  __device__ static S identity() { return 0u; }
  __device__ static S mul(In, In) { return 1u; }
  __device__ static void combine(S*, S) {}
  __device__ static Out out(S) { return 1; }
};
struct SrMaxTimesF64 {
  static constexpr bool kNullable = false;
  using In = double;
  using S = unsigned long long;
  using Out = double;
  static constexpr bool kPattern = false;
  __device__ static S identity() { return 0ull; }
  __device__ static S mul(In a, In b) { return f64_key(a * b); }
  __device__ static void combine(S* p, S v) { atomicMax(p, v); }
  __device__ static Out out(S s) { return f64_unkey(s); }
};
struct SrMaxTimesF32 {
  static constexpr bool kNullable = false;
  using In = float;
  using S = uint32_t;
  using Out = float;
  static constexpr bool kPattern = false;
  __device__ static S identity() { return 0u; }
  __device__ static S mul(In a, In b) { return f32_key(a * b); }
  __device__ static void combine(S* p, S v) { atomicMax(p, v); }
  __device__ static Out out(S s) { return f32_unkey(s); }
};

// ---------------------------------------------------------------------------
// Operands of one CSR product C = A * B (A: m x n, B: n x k).
// ---------------------------------------------------------------------------
struct Operands {
  const int64_t* a_ptr;
  const int32_t* a_idx;
  const void* a_val;
  const int64_t* b_ptr;
  const int32_t* b_idx;
  const void* b_val;
  int32_t m, n, k;
  // Optional copy of B with (column id, value bits) side by side, for
  // 4-byte values: one load per product instead of two.  NULL: unused.
  const int2* b_pair;
  // Optional copy of B with each int32 value and column id in one 32-bit
  // word, value << pack_bits | column, for values in [0, 2^(32 - pack_bits))
  // and fewer than 2^pack_bits columns: half the bytes of b_pair per
  // product.  NULL: unused.
  const uint32_t* b_packed;
  int32_t pack_bits;
};

// ---------------------------------------------------------------------------
// Block-wide scans (blockDim.x a multiple of 64, at most 1024).  tmp needs 16
// elements of LDS.  Every thread of the block must call them.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  return x;
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

__device__ __forceinline__ int wave_or(int x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x |= __shfl_xor(x, d, kWave);
  return x;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x = max(x, __shfl_xor(x, d, kWave));
  return x;
}

template <class T>
__device__ T block_exclusive_scan(T v, T* tmp, T* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  T x = wave_inclusive_scan(v);
  if (lane == kWave - 1) tmp[wid] = x;
  __syncthreads();
  if (wid == 0) {
    T w = lane < nw ? tmp[lane] : T(0);
    w = wave_inclusive_scan(w);
    if (lane < nw) tmp[lane] = w;
  }
  __syncthreads();
  T off = wid > 0 ? tmp[wid - 1] : T(0);
  *total = tmp[nw - 1];
  __syncthreads();
  return off + x - v;
}

template <class T>
__device__ T block_sum(T v, T* tmp) {
  T t;
  block_exclusive_scan(v, tmp, &t);
  return t;
}

// ---------------------------------------------------------------------------
// Row enumerator.
//
// Feeds every product A(i,k) (x) B(k,j) of one row i of C to a sink, as
// Gustavson's row formulation does (paper Sec. 4.1).  The row's A entries are
// taken NT at a time (one per thread).  For each, the segment of B(k,:) that
// falls in the current column panel is looked up.  Short segments are walked
// by their own lane.  Long ones are queued in LDS and cut into pieces of
// kPiece products that the waves of the block take dynamically, so one
// heavy B row is shared by all waves and every load in a piece is coalesced.
//
// Panels: when `paneled`, only columns [c0, c0 + W) are enumerated and the
// segment bounds come from the panel index pidx (P+1 offsets per B row,
// relative to the row start); otherwise the whole B row is the segment.
// Columns are passed to the sink relative to c0.
// ---------------------------------------------------------------------------
template <class In>
struct RowQueue {
  int* ctr;       // [0] queued entries, [1] next piece, [2..33] scan scratch (16 ints or 16 int64)
  int64_t* lo;    // segment start in B
  In* a;          // A value of the entry
  int32_t* len;   // segment length
  int32_t* pfx;   // exclusive prefix of piece counts (nq + 1 entries)

  __host__ __device__ static size_t a_bytes(int nt) {
    return (static_cast<size_t>(nt) * sizeof(In) + 7) & ~static_cast<size_t>(7);
  }
  // LDS bytes for nt threads, rounded up to 16.
  __host__ __device__ static size_t bytes(int nt) {
    size_t b = 48 * sizeof(int) + static_cast<size_t>(nt) * sizeof(int64_t) + a_bytes(nt) +
               static_cast<size_t>(nt) * sizeof(int32_t) + static_cast<size_t>(nt + 1) * sizeof(int32_t);
    return (b + 15) & ~static_cast<size_t>(15);
  }
  __device__ static RowQueue carve(unsigned char* base, int nt) {
    RowQueue q;
    q.ctr = reinterpret_cast<int*>(base);
    unsigned char* p = base + 48 * sizeof(int);
    q.lo = reinterpret_cast<int64_t*>(p);
    p += static_cast<size_t>(nt) * sizeof(int64_t);
    q.a = reinterpret_cast<In*>(p);
    p += a_bytes(nt);
    q.len = reinterpret_cast<int32_t*>(p);
    p += static_cast<size_t>(nt) * sizeof(int32_t);
    q.pfx = reinterpret_cast<int32_t*>(p);
    return q;
  }
};

template <class SR>
__device__ __forceinline__ typename SR::In load_val(const void* v, int64_t p) {
  if constexpr (SR::kPattern) {
    return typename SR::In(1);
  } else {
    if constexpr (SR::kNullable) {
      if (v == nullptr) return typename SR::In(1);
    }
    return static_cast<const typename SR::In*>(v)[p];
  }
}

constexpr int kShortUnroll = 8;  // loads in flight per lane on a short segment

// Where the segments of a row come from.  RowSource walks the A entries of
// row i and looks the B segment up (whole row, or the part of it in one
// column panel through the panel index).  SegSource walks a precomputed list
// of non-empty segments of one (row, panel) piece.
template <class SR>
struct RowSource {
  const Operands* op;
  int64_t a_lo, a_hi;
  bool paneled;
  const int32_t* __restrict__ pidx;
  int P, p;
  int p_hi;  // panels [p, p_hi) form the column window (p_hi <= p means p + 1)
  __device__ int64_t count() const { return a_hi - a_lo; }
  __device__ void load(int64_t t, int64_t& lo, int32_t& len, typename SR::In& a) const {
    const int64_t pa = a_lo + t;
    const int32_t kk = op->a_idx[pa];
    a = load_val<SR>(op->a_val, pa);
    const int64_t bs = op->b_ptr[kk];
    if (paneled) {
      const int32_t* s = pidx + static_cast<int64_t>(kk) * (P + 1);
      const int32_t s0 = s[p];
      lo = bs + s0;
      len = s[p_hi > p ? p_hi : p + 1] - s0;
    } else {
      lo = bs;
      len = static_cast<int32_t>(op->b_ptr[kk + 1] - bs);
    }
  }
};

// A row's segments in one column window whose first round (entries
// [0, blockDim.x), one per thread) the caller has already loaded into
// registers; later rounds are loaded as by RowSource.
template <class SR>
struct PassSource {
  RowSource<SR> rest;
  int64_t lo0;
  int32_t len0;
  typename SR::In a0;
  __device__ int64_t count() const { return rest.count(); }
  __device__ void load(int64_t t, int64_t& lo, int32_t& len, typename SR::In& a) const {
    if (t < static_cast<int64_t>(blockDim.x)) {  // the first round: t is this thread's index
      lo = lo0;
      len = len0;
      a = a0;
    } else {
      rest.load(t, lo, len, a);
    }
  }
};

// A row of at most one entry per thread, walked panel after panel: every
// thread keeps its A entry (value, B row start, panel-index row) in registers
// and has the next panel's offset loaded one panel ahead.
template <class SR>
struct CachedRowSource {
  int64_t deg;
  int64_t bs;
  typename SR::In a;
  int32_t s_cur, s_nxt, s_nxt2;
  __device__ int64_t count() const { return deg; }
  __device__ void load(int64_t, int64_t& lo, int32_t& len, typename SR::In& av) const {
    lo = bs + s_cur;
    len = s_nxt - s_cur;
    av = a;
  }
};

// One non-empty segment of a (row, panel) piece: entries [bpos, bpos+len) of
// B, multiplied by A entry a_lo + apos.
struct SegDesc {
  int64_t bpos;
  int32_t len;
  int32_t apos;
};

template <class SR>
struct SegSource {
  const Operands* op;
  int64_t a_lo;
  const SegDesc* __restrict__ segs;
  int64_t nseg;
  __device__ int64_t count() const { return nseg; }
  __device__ void load(int64_t t, int64_t& lo, int32_t& len, typename SR::In& a) const {
    const SegDesc d = segs[t];
    lo = d.bpos;
    len = d.len;
    a = load_val<SR>(op->a_val, a_lo + d.apos);
  }
};

// A semiring whose kernels read B through Operands::b_pair (4-byte values).
template <class SR>
struct PairedB : SR {
  static_assert(!SR::kPattern && sizeof(typename SR::In) == 4, "pairs hold 4-byte values");
  static constexpr bool kPairedB = true;
};
template <class SR, class = void>
struct IsPairedB {
  static constexpr bool value = false;
};
template <class SR>
struct IsPairedB<SR, decltype(void(SR::kPairedB))> {
  static constexpr bool value = SR::kPairedB;
};

// A semiring whose kernels read B through Operands::b_packed (int32 values
// that fit beside the column id in one word).
template <class SR>
struct PackedB : SR {
  static_assert(!SR::kPattern && sizeof(typename SR::In) == 4, "packed words hold small int32 values");
  static constexpr bool kPackedB = true;
};
template <class SR, class = void>
struct IsPackedB {
  static constexpr bool value = false;
};
template <class SR>
struct IsPackedB<SR, decltype(void(SR::kPackedB))> {
  static constexpr bool value = SR::kPackedB;
};

// Column id and value of B entry q.
template <class SR>
__device__ __forceinline__ void load_b(const Operands& op, int64_t q, int32_t& col, typename SR::In& v) {
  if constexpr (IsPackedB<SR>::value) {
    // the raw word; decode_b splits it where the product is combined, so
    // the load is not waited for where it is issued
    col = static_cast<int32_t>(op.b_packed[q]);
    v = 0;
  } else if constexpr (IsPairedB<SR>::value) {
    const int2 pr = op.b_pair[q];
    col = pr.x;
    v = __builtin_bit_cast(typename SR::In, pr.y);
  } else {
    col = op.b_idx[q];
    v = load_val<SR>(op.b_val, q);
  }
}

// Column id and value of a loaded B entry (load_b's registers), at the
// point of use: splits a packed word, nothing for the other forms.
template <class SR>
__device__ __forceinline__ void decode_b(const Operands& op, int32_t& col, typename SR::In& v) {
  if constexpr (IsPackedB<SR>::value) {
    const uint32_t x = static_cast<uint32_t>(col);
    col = static_cast<int32_t>(x & ((1u << op.pack_bits) - 1u));
    v = static_cast<typename SR::In>(x >> op.pack_bits);
  }
}

// One piece of a queued segment held in registers: products [s0, s1) of B
// (this lane's share), their column ids and values, and the A value.
template <class In, int U>
struct PieceBuf {
  int64_t s0, s1;
  In ae;
  int32_t cols[U];
  In bv[U];
};

// kBufs = 1: a wave loads a whole piece, then combines it.  kBufs = 2: pieces
// are half as long and a wave keeps two in flight, issuing the next piece's
// loads before combining the current one (more registers).
// kFlat: when a round of A entries has at most a few products per thread,
// the products of all its segments are dealt to the threads directly
// (product j to thread j mod blockDim.x, its segment found by a binary
// search over the segments' prefix), so every product of the round is
// loaded in one or a few waves of independent loads.
template <class SR, int kBufs = 1, bool kFlat = false, class Src, class Sink>
__device__ void enumerate_src(const Operands& op, const Src& src, int32_t c0, int short_seg,
                              RowQueue<typename SR::In> q, Sink& sink) {
  using In = typename SR::In;
  static_assert(kBufs == 1 || kBufs == 2, "one or two piece buffers");
  // Loads per lane per piece buffer: 16 in flight per lane (8 for 8-byte
  // values, to stay in registers).
  // (half as many with kFlat, whose products mostly take the flat path).
  constexpr int kPU = (sizeof(In) > 4 ? kPieceUnroll / 2 : kPieceUnroll) / kBufs / (kFlat ? 2 : 1);
  constexpr int kPc = kWave * kPU;
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int lane = tid & (kWave - 1);
  if (tid == 0) {
    q.ctr[0] = 0;
    q.ctr[1] = 0;
  }
  __syncthreads();
  const int64_t total = src.count();
  for (int64_t base = 0; base < total; base += nt) {
    int64_t lo = 0;
    int32_t len = 0;
    In a = In(1);
    if (base + tid < total) src.load(base + tid, lo, len, a);
    if constexpr (kFlat) {
      constexpr int kFU = sizeof(In) > 4 ? 2 : 4;  // products per thread per batch
      // one scan gives each entry's product offset and, in the high bits,
      // the number of segments longer than short_seg
      long long tot;
      const long long packed = block_exclusive_scan(
          static_cast<long long>(len) + (static_cast<long long>(len > short_seg) << 40),
          reinterpret_cast<long long*>(q.ctr + 2), &tot);
      const int off = static_cast<int>(packed & ((1ll << 40) - 1));
      const int E = static_cast<int>(tot & ((1ll << 40) - 1));
      const int nlong = static_cast<int>(tot >> 40);
      // Flat when the long segments would otherwise take several piece
      // rounds per wave and the products fit a few batches.
      if (nlong > (nt >> 6) && E <= 8 * kFU * nt) {  // uniform
        q.lo[tid] = lo;
        q.a[tid] = a;
        q.pfx[tid] = off;  // threads past the row's entries have len 0: off == E
        if (tid == 0) q.pfx[nt] = E;
        __syncthreads();
        // entries past the round's last one have pfx == E: the search stops there
        const int nents = static_cast<int>(min(static_cast<int64_t>(nt), total - base));
        for (int j0 = 0; j0 < E; j0 += kFU * nt) {
          int es[kFU];  // segment of each product of this batch, or -1
#pragma unroll
          for (int u = 0; u < kFU; ++u) {
            const int j = j0 + u * nt + tid;
            int e_lo = -1;
            if (j < E) {
              e_lo = 0;
              int e_hi = nents;  // the last entry with pfx <= j has len > 0
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
          int32_t cols[kFU];
          In bv[kFU];
#pragma unroll
          for (int u = 0; u < kFU; ++u)
            if (es[u] >= 0) load_b<SR>(op, q.lo[es[u]] + (j0 + u * nt + tid - q.pfx[es[u]]), cols[u], bv[u]);
#pragma unroll
          for (int u = 0; u < kFU; ++u)
            if (es[u] >= 0) {
              decode_b<SR>(op, cols[u], bv[u]);
              sink.add(cols[u] - c0, SR::mul(q.a[es[u]], bv[u]));
            }
        }
        __syncthreads();  // the queue arrays are rewritten by the next round
        continue;
      }
    }
    if (len > short_seg) {
      const int slot = atomicAdd(&q.ctr[0], 1);
      q.lo[slot] = lo;
      q.len[slot] = len;
      q.a[slot] = a;
    } else {
      // Walked by this lane alone, kShortUnroll independent loads at a time.
      for (int32_t t = 0; t < len; t += kShortUnroll) {
        int32_t cols[kShortUnroll];
        In bv[kShortUnroll];
#pragma unroll
        for (int u = 0; u < kShortUnroll; ++u) {
          if (t + u < len) {
            load_b<SR>(op, lo + t + u, cols[u], bv[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < kShortUnroll; ++u)
          if (t + u < len) {
            decode_b<SR>(op, cols[u], bv[u]);
            sink.add(cols[u] - c0, SR::mul(a, bv[u]));
          }
      }
    }
    __syncthreads();
    const int nq = q.ctr[0];
    if (nq > 0) {
      int pieces = tid < nq ? (q.len[tid] + kPc - 1) / kPc : 0;
      int ptotal;
      const int off = block_exclusive_scan(pieces, q.ctr + 2, &ptotal);
      if (tid < nq) q.pfx[tid] = off;
      if (tid == 0) q.pfx[nq] = ptotal;
      __syncthreads();
      // Each wave takes pieces in increasing order and keeps two in flight:
      // the loads of the next piece are issued before the products of the
      // current one are combined.
      int e_lo = 0;
      auto take = [&]() {
        int u = 0;
        if (lane == 0) u = atomicAdd(&q.ctr[1], 1);
        return __shfl(u, 0, kWave);
      };
      auto fetch = [&](int u, PieceBuf<In, kPU>& b) {
        int lo_e = e_lo, hi_e = nq;  // pfx[lo_e] <= u < pfx[hi_e]
        while (hi_e - lo_e > 1) {
          const int mid = (lo_e + hi_e) >> 1;
          if (q.pfx[mid] <= u)
            lo_e = mid;
          else
            hi_e = mid;
        }
        e_lo = lo_e;
        b.s0 = q.lo[lo_e] + static_cast<int64_t>(u - q.pfx[lo_e]) * kPc;
        b.s1 = q.lo[lo_e] + q.len[lo_e];
        b.ae = q.a[lo_e];
#pragma unroll
        for (int r = 0; r < kPU; ++r) {
          const int64_t qq = b.s0 + r * kWave + lane;
          if (qq < b.s1) {
            load_b<SR>(op, qq, b.cols[r], b.bv[r]);
          }
        }
      };
      auto consume = [&](const PieceBuf<In, kPU>& b) {
#pragma unroll
        for (int r = 0; r < kPU; ++r) {
          const int64_t qq = b.s0 + r * kWave + lane;
          if (qq < b.s1) {
            int32_t c = b.cols[r];
            In v = b.bv[r];
            decode_b<SR>(op, c, v);
            sink.add(c - c0, SR::mul(b.ae, v));
          }
        }
      };
      if constexpr (kBufs == 1) {
        for (;;) {
          const int u = take();
          if (u >= ptotal) break;
          int lo_e = e_lo, hi_e = nq;  // pfx[lo_e] <= u < pfx[hi_e]
          while (hi_e - lo_e > 1) {
            const int mid = (lo_e + hi_e) >> 1;
            if (q.pfx[mid] <= u)
              lo_e = mid;
            else
              hi_e = mid;
          }
          const int e = lo_e;
          e_lo = e;
          const int64_t s0 = q.lo[e] + static_cast<int64_t>(u - q.pfx[e]) * kPc;
          const int64_t s1 = q.lo[e] + q.len[e];
          const In ae = q.a[e];
          int32_t cols[kPU];
          In bv[kPU];
#pragma unroll
          for (int r = 0; r < kPU; ++r) {
            const int64_t qq = s0 + r * kWave + lane;
            if (qq < s1) {
              load_b<SR>(op, qq, cols[r], bv[r]);
            }
          }
#pragma unroll
          for (int r = 0; r < kPU; ++r) {
            const int64_t qq = s0 + r * kWave + lane;
            if (qq < s1) {
              decode_b<SR>(op, cols[r], bv[r]);
              sink.add(cols[r] - c0, SR::mul(ae, bv[r]));
            }
          }
        }
      } else if (const int u0 = take(); u0 < ptotal) {
        PieceBuf<In, kPU> b0, b1;
        fetch(u0, b0);
        for (;;) {
          const int u1 = take();
          if (u1 < ptotal) fetch(u1, b1);
          consume(b0);
          if (u1 >= ptotal) break;
          const int u2 = take();
          if (u2 < ptotal) fetch(u2, b0);
          consume(b1);
          if (u2 >= ptotal) break;
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      q.ctr[0] = 0;
      q.ctr[1] = 0;
    }
    __syncthreads();
  }
}

template <class SR, int kBufs = 1, bool kFlat = false, class Sink>
__device__ void enumerate_row(const Operands& op, int64_t a_lo, int64_t a_hi, bool paneled,
                              const int32_t* __restrict__ pidx, int P, int p, int32_t c0,
                              int short_seg, RowQueue<typename SR::In> q, Sink& sink) {
  RowSource<SR> src{&op, a_lo, a_hi, paneled, pidx, P, p, p + 1};
  enumerate_src<SR, kBufs, kFlat>(op, src, c0, short_seg, q, sink);
}

// Wave-uniform values kept in scalar registers.
__device__ __forceinline__ int32_t uniform(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(static_cast<uint64_t>(x) >> 32));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ __forceinline__ uint32_t hash_slot(int32_t key, uint32_t mask) {
  return (static_cast<uint32_t>(key) * 2654435761u) & mask;
}

// Position (0..31) of the r-th set bit (r counted from 0) of w.
__device__ __forceinline__ int select_bit(uint32_t w, int r) {
  int pos = 0;
  int c = __popc(w & 0xFFFFu);
  if (r >= c) { r -= c; w >>= 16; pos += 16; }
  c = __popc(w & 0xFFu);
  if (r >= c) { r -= c; w >>= 8; pos += 8; }
  c = __popc(w & 0xFu);
  if (r >= c) { r -= c; w >>= 4; pos += 4; }
  c = __popc(w & 0x3u);
  if (r >= c) { r -= c; w >>= 2; pos += 2; }
  c = static_cast<int>(w & 0x1u);
  if (r >= c) { pos += 1; }
  return pos;
}

}  // namespace spg
