// Oracle for the local semiring sparse product C = A (x).(+) B.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow CPU reference that
// the GPU library is checked against.  Only the tests, the smoke check and
// the CPU-baseline leg of the benchmark load it; the product path never does,
// and the two share no code.
//
// What it computes (paper Sec. 3.1, problem statement C = AB with
// A in S^{m x n}, B in S^{n x k}; Sec. 1, semirings over user value types):
//
//     C(i,j) = (+)_{k : A(i,k) stored and B(k,j) stored}  A(i,k) (x) B(k,j)
//
// and pattern(C) = every (i,j) for which such a k exists.  The pattern is
// structural: an entry whose value equals the additive identity is still
// stored, since the paper counts flops as the nonzero multiplications
// (Sec. 3.1, Table "complexity").
//
// How (Sec. 4.1, Gustavson's algorithm): a column of C is formed by merging
// the columns of A picked out by the nonzeros of the matching column of B.
// The CSC entry point does exactly that, column by column.  The CSR entry
// point is the same algorithm applied to rows (a row of C merges the rows of
// B picked out by the nonzeros of the matching row of A).  The accumulator is
// an ordered map, so every output row/column comes out sorted ascending.
//
// Semirings (codes are an interface convention shared with the GPU library):
//   0 (+,x)   float64          3 (min,+) float32 (one IEEE rounding per +)
//   1 (+,x)   float32 inputs,  4 (OR,AND) uint8 {0,1}; NULL values = all true
//             computed in      5 (max,x) float64
//             float64          6 (max,x) float32
//   2 (min,+) int32, + is computed in int64 and clamped to the int32 range.
// min/max on floating point use the total order in which -0 < +0.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fPIC -shared
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

namespace {

// Floating-point total order used by min / max: plain comparison, except
// that -0 is taken to be smaller than +0.
template <class F>
bool fless(F x, F y) {
  if (x < y) return true;
  if (y < x) return false;
  return std::signbit(x) && !std::signbit(y);
}

struct PlusTimesF64 {
  using In = double;
  using T = double;
  static T mul(In a, In b) { return a * b; }
  static T add(T x, T y) { return x + y; }
};
struct PlusTimesF32in64 {  // float32 operands, float64 arithmetic
  using In = float;
  using T = double;
  static T mul(In a, In b) { return static_cast<double>(a) * static_cast<double>(b); }
  static T add(T x, T y) { return x + y; }
};
struct MinPlusI32 {
  using In = int32_t;
  using T = int32_t;
  static T mul(In a, In b) {
    int64_t s = static_cast<int64_t>(a) + static_cast<int64_t>(b);
    if (s > INT32_MAX) s = INT32_MAX;
    if (s < INT32_MIN) s = INT32_MIN;
    return static_cast<T>(s);
  }
  static T add(T x, T y) { return y < x ? y : x; }
};
struct MinPlusF32 {
  using In = float;
  using T = float;
  static T mul(In a, In b) { return a + b; }
  static T add(T x, T y) { return fless(y, x) ? y : x; }
};
struct OrAndBool {
  using In = uint8_t;
  using T = uint8_t;
  static T mul(In a, In b) { return (a != 0 && b != 0) ? 1 : 0; }
  static T add(T x, T y) { return (x != 0 || y != 0) ? 1 : 0; }
};
struct MaxTimesF64 {
  using In = double;
  using T = double;
  static T mul(In a, In b) { return a * b; }
  static T add(T x, T y) { return fless(x, y) ? y : x; }
};
struct MaxTimesF32 {
  using In = float;
  using T = float;
  static T mul(In a, In b) { return a * b; }
  static T add(T x, T y) { return fless(x, y) ? y : x; }
};

template <class S>
typename S::In value_at(const void* val, int64_t p) {
  if (val == nullptr) return static_cast<typename S::In>(1);  // pattern-only boolean
  return static_cast<const typename S::In*>(val)[p];
}

struct ResultBase {
  virtual ~ResultBase() = default;
  std::vector<int64_t> counts;  // entries per selected slice
  int64_t nnz = 0;
  int elem = 0;                 // bytes per output value
  virtual void copy(int64_t* ptr, int32_t* idx, void* val) const = 0;
};

template <class S>
struct Result : ResultBase {
  std::vector<std::vector<int32_t>> keys;
  std::vector<std::vector<typename S::T>> vals;
  void copy(int64_t* ptr, int32_t* idx, void* val) const override {
    int64_t off = 0;
    auto* v = static_cast<typename S::T*>(val);
    for (size_t r = 0; r < keys.size(); ++r) {
      if (ptr) ptr[r] = off;
      if (keys[r].empty()) continue;  // memcpy takes no null pointer, even for 0 bytes
      if (idx) std::memcpy(idx + off, keys[r].data(), keys[r].size() * sizeof(int32_t));
      if (v) std::memcpy(v + off, vals[r].data(), vals[r].size() * sizeof(typename S::T));
      off += static_cast<int64_t>(keys[r].size());
    }
    if (ptr) ptr[keys.size()] = off;
  }
};

// One slice (row of C for CSR, column of C for CSC) by Gustavson's merge.
//   CSR: slice i of C = (+) over stored A(i,k) of  A(i,k) (x) B(k,:)
//   CSC: slice j of C = (+) over stored B(k,j) of  A(:,k) (x) B(k,j)
// In both cases the product keeps the operand order A (x) B.
template <class S>
void one_slice(bool csc, int64_t s, const int64_t* Ap, const int32_t* Ai, const void* Av,
               const int64_t* Bp, const int32_t* Bi, const void* Bv,
               std::vector<int32_t>& keys, std::vector<typename S::T>& vals) {
  std::map<int32_t, typename S::T> acc;
  auto accumulate = [&acc](int32_t key, typename S::T prod) {
    auto it = acc.find(key);
    if (it == acc.end())
      acc.emplace(key, prod);
    else
      it->second = S::add(it->second, prod);
  };
  if (!csc) {
    for (int64_t p = Ap[s]; p < Ap[s + 1]; ++p) {
      const int32_t k = Ai[p];
      const typename S::In a = value_at<S>(Av, p);
      for (int64_t q = Bp[k]; q < Bp[k + 1]; ++q)
        accumulate(Bi[q], S::mul(a, value_at<S>(Bv, q)));
    }
  } else {
    for (int64_t q = Bp[s]; q < Bp[s + 1]; ++q) {
      const int32_t k = Bi[q];
      const typename S::In b = value_at<S>(Bv, q);
      for (int64_t p = Ap[k]; p < Ap[k + 1]; ++p)
        accumulate(Ai[p], S::mul(value_at<S>(Av, p), b));
    }
  }
  keys.clear();
  vals.clear();
  keys.reserve(acc.size());
  vals.reserve(acc.size());
  for (const auto& kv : acc) {
    keys.push_back(kv.first);
    vals.push_back(kv.second);
  }
}

template <class S>
ResultBase* run(bool csc, int64_t nsel, const int64_t* sel, const int64_t* Ap, const int32_t* Ai,
                const void* Av, const int64_t* Bp, const int32_t* Bi, const void* Bv, int nthreads) {
  auto* r = new Result<S>();
  r->elem = sizeof(typename S::T);
  r->keys.resize(nsel);
  r->vals.resize(nsel);
  r->counts.resize(nsel);
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
  for (int64_t t = 0; t < nsel; ++t) {
    const int64_t s = sel ? sel[t] : t;
    one_slice<S>(csc, s, Ap, Ai, Av, Bp, Bi, Bv, r->keys[t], r->vals[t]);
    r->counts[t] = static_cast<int64_t>(r->keys[t].size());
  }
  int64_t nnz = 0;
  for (auto c : r->counts) nnz += c;
  r->nnz = nnz;
  return r;
}

// One slice of a semiring sum of k parts stacked slice-wise (slice s of
// part t is slice t*m + s): every stored entry of the k slices, merged by
// key with (+).
template <class S>
void sum_slice(int64_t s, int64_t m, int k, const int64_t* Pp, const int32_t* Pi, const void* Pv,
               std::vector<int32_t>& keys, std::vector<typename S::T>& vals) {
  std::map<int32_t, typename S::T> acc;
  for (int t = 0; t < k; ++t) {
    const int64_t r = t * m + s;
    for (int64_t q = Pp[r]; q < Pp[r + 1]; ++q) {
      const auto v = static_cast<typename S::T>(value_at<S>(Pv, q));
      auto it = acc.find(Pi[q]);
      if (it == acc.end())
        acc.emplace(Pi[q], v);
      else
        it->second = S::add(it->second, v);
    }
  }
  keys.clear();
  vals.clear();
  for (const auto& kv : acc) {
    keys.push_back(kv.first);
    vals.push_back(kv.second);
  }
}

template <class S>
ResultBase* run_sum(int64_t m, int k, const int64_t* Pp, const int32_t* Pi, const void* Pv, int nthreads) {
  auto* r = new Result<S>();
  r->elem = sizeof(typename S::T);
  r->keys.resize(m);
  r->vals.resize(m);
  r->counts.resize(m);
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
  for (int64_t s = 0; s < m; ++s) {
    sum_slice<S>(s, m, k, Pp, Pi, Pv, r->keys[s], r->vals[s]);
    r->counts[s] = static_cast<int64_t>(r->keys[s].size());
  }
  int64_t nnz = 0;
  for (auto c : r->counts) nnz += c;
  r->nnz = nnz;
  return r;
}

// ---------------------------------------------------------------------------
// Per-slice digests of a product too large to hold (the definition of C above,
// checked over every slice without materialising C).
//
// mix64 is the output function of SplitMix64 (Steele, Lea and Flood, "Fast
// splittable pseudorandom number generators", OOPSLA 2014), with the shift
// and multiplier constants of its published reference implementation.
// Entry t (0-based, in ascending id order) of a slice, with id j and value
// bits v (the value's bytes zero-extended to 64 bits; the boolean 0/1 byte),
// contributes mix64(mix64((t << 32) | j) ^ v); the slice digest is the sum
// of its entries' contributions modulo 2^64.  Position, id and value all
// enter, so any change of pattern, order or value changes the digest.
// ---------------------------------------------------------------------------
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <class T>
uint64_t value_bits(T v) {
  uint64_t b = 0;
  std::memcpy(&b, &v, sizeof(T));  // little-endian: the value's bytes, zero-extended
  return b;
}

template <class S>
void run_digest(bool csc, int64_t nsel, const int64_t* sel, const int64_t* Ap, const int32_t* Ai, const void* Av,
                const int64_t* Bp, const int32_t* Bi, const void* Bv, int nthreads, int64_t* nnz_out,
                uint64_t* hash_out) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<int32_t> keys;
    std::vector<typename S::T> vals;
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < nsel; ++t) {
      const int64_t s = sel ? sel[t] : t;
      one_slice<S>(csc, s, Ap, Ai, Av, Bp, Bi, Bv, keys, vals);
      uint64_t h = 0;
      for (size_t e = 0; e < keys.size(); ++e) {
        const uint64_t pos_id = (static_cast<uint64_t>(e) << 32) | static_cast<uint32_t>(keys[e]);
        h += mix64(mix64(pos_id) ^ value_bits(vals[e]));
      }
      nnz_out[t] = static_cast<int64_t>(keys.size());
      hash_out[t] = h;
    }
  }
}

// Selection (the Markov-clustering step that bounds the entries kept per
// column): a slice longer than S keeps its S largest values, ties going to
// the smaller id; the kept entries stay in ascending id order.  Values are
// compared in float32 with the total order in which -0 < +0.
void select_slice(int64_t lo, int64_t hi, const int32_t* idx, const float* val, int64_t S,
                  std::vector<int64_t>& keep) {
  keep.clear();
  for (int64_t p = lo; p < hi; ++p) keep.push_back(p);
  if (hi - lo <= S) return;
  std::sort(keep.begin(), keep.end(), [&](int64_t x, int64_t y) {
    if (fless(val[y], val[x])) return true;  // larger value first
    if (fless(val[x], val[y])) return false;
    return idx[x] < idx[y];                  // equal values: smaller id first
  });
  keep.resize(static_cast<size_t>(S));
  std::sort(keep.begin(), keep.end(), [&](int64_t x, int64_t y) { return idx[x] < idx[y]; });
}

}  // namespace

extern "C" {

// Semiring sum of k parts of m slices each, stacked slice-wise in (Pp, Pi,
// Pv): slice s of the result is the (+) of slices s, m+s, ..., (k-1)m+s,
// entry by entry (the layout does not matter: slices are rows or columns
// alike).  Same result handle as orc_spgemm.
void* orc_sum(int semiring, int64_t m, int k, const int64_t* Pp, const int32_t* Pi, const void* Pv,
              int nthreads) {
  switch (semiring) {
    case 0: return run_sum<PlusTimesF64>(m, k, Pp, Pi, Pv, nthreads);
    case 1: return run_sum<PlusTimesF32in64>(m, k, Pp, Pi, Pv, nthreads);
    case 2: return run_sum<MinPlusI32>(m, k, Pp, Pi, Pv, nthreads);
    case 3: return run_sum<MinPlusF32>(m, k, Pp, Pi, Pv, nthreads);
    case 4: return run_sum<OrAndBool>(m, k, Pp, Pi, Pv, nthreads);
    case 5: return run_sum<MaxTimesF64>(m, k, Pp, Pi, Pv, nthreads);
    case 6: return run_sum<MaxTimesF32>(m, k, Pp, Pi, Pv, nthreads);
    default: return nullptr;
  }
}

// Computes the selected output slices of C = A (x).(+) B.
//   layout 0: CSR.  A is m x n with row pointers Ap (m+1) and column ids Ai;
//             B is n x k likewise; slice s = row s of C.
//   layout 1: CSC.  A is m x n with column pointers Ap (n+1) and row ids Ai;
//             B is n x k likewise; slice s = column s of C.
// sel: nsel slice ids, or NULL for all slices 0..nsel-1.
// Values: the semiring's input type, or NULL (semiring 4 only) for all true.
// Returns an opaque result; NULL on an unknown semiring.
void* orc_spgemm(int semiring, int layout, int64_t nsel, const int64_t* sel, const int64_t* Ap,
                 const int32_t* Ai, const void* Av, const int64_t* Bp, const int32_t* Bi,
                 const void* Bv, int nthreads) {
  const bool csc = layout == 1;
  switch (semiring) {
    case 0: return run<PlusTimesF64>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads);
    case 1: return run<PlusTimesF32in64>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads);
    case 2: return run<MinPlusI32>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads);
    case 3: return run<MinPlusF32>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads);
    case 4: return run<OrAndBool>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads);
    case 5: return run<MaxTimesF64>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads);
    case 6: return run<MaxTimesF32>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads);
    default: return nullptr;
  }
}

int64_t orc_nnz(void* h) { return static_cast<ResultBase*>(h)->nnz; }
int orc_elem_bytes(void* h) { return static_cast<ResultBase*>(h)->elem; }

// ptr: nsel+1 offsets (may be NULL), idx: nnz ids, val: nnz values of the
// semiring's output type (float64 for code 1).
void orc_copy(void* h, int64_t* ptr, int32_t* idx, void* val) {
  static_cast<ResultBase*>(h)->copy(ptr, idx, val);
}

void orc_free(void* h) { delete static_cast<ResultBase*>(h); }

// flops per selected slice: the number of (x) operations Gustavson performs
// for it, i.e. for CSR row i the sum over stored A(i,k) of nnz(B(k,:)).
void orc_flops(int layout, int64_t nsel, const int64_t* sel, const int64_t* Ap, const int32_t* Ai,
               const int64_t* Bp, const int32_t* Bi, int64_t* out) {
  (void)Bi;
  for (int64_t t = 0; t < nsel; ++t) {
    const int64_t s = sel ? sel[t] : t;
    int64_t f = 0;
    if (layout == 0) {
      for (int64_t p = Ap[s]; p < Ap[s + 1]; ++p) f += Bp[Ai[p] + 1] - Bp[Ai[p]];
    } else {
      for (int64_t q = Bp[s]; q < Bp[s + 1]; ++q) f += Ap[Bi[q] + 1] - Ap[Bi[q]];
    }
    out[t] = f;
  }
}

// Prune of a float32 compressed matrix (the Markov-clustering step after
// expansion): keep an entry when its value is >= thresh, drop it otherwise,
// order unchanged.  Returns the kept count; with outputs non-NULL also fills
// new_ptr (nmajor+1), new_idx and new_val.
int64_t orc_prune_f32(int64_t nmajor, const int64_t* ptr, const int32_t* idx, const float* val,
                      float thresh, int64_t* new_ptr, int32_t* new_idx, float* new_val) {
  int64_t out = 0;
  for (int64_t s = 0; s < nmajor; ++s) {
    if (new_ptr) new_ptr[s] = out;
    for (int64_t p = ptr[s]; p < ptr[s + 1]; ++p) {
      if (val[p] >= thresh) {
        if (new_idx) new_idx[out] = idx[p];
        if (new_val) new_val[out] = val[p];
        ++out;
      }
    }
  }
  if (new_ptr) new_ptr[nmajor] = out;
  return out;
}

// Digest of every selected output slice of C = A (x).(+) B (arguments as in
// orc_spgemm): nnz_out[t] entries and hash_out[t] the slice digest defined
// above.  Each slice is formed, hashed and dropped, so C is never held.
// Exact semirings only (codes 2..6); returns -1 for (+,x), 0 otherwise.
int orc_digest(int semiring, int layout, int64_t nsel, const int64_t* sel, const int64_t* Ap, const int32_t* Ai,
               const void* Av, const int64_t* Bp, const int32_t* Bi, const void* Bv, int nthreads,
               int64_t* nnz_out, uint64_t* hash_out) {
  const bool csc = layout == 1;
  switch (semiring) {
    case 2: run_digest<MinPlusI32>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads, nnz_out, hash_out); return 0;
    case 3: run_digest<MinPlusF32>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads, nnz_out, hash_out); return 0;
    case 4: run_digest<OrAndBool>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads, nnz_out, hash_out); return 0;
    case 5: run_digest<MaxTimesF64>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads, nnz_out, hash_out); return 0;
    case 6: run_digest<MaxTimesF32>(csc, nsel, sel, Ap, Ai, Av, Bp, Bi, Bv, nthreads, nnz_out, hash_out); return 0;
    default: return -1;
  }
}

// mix64 of every element of x (n values), for the block digests built on top
// of the slice digests.
void orc_mix64(int64_t n, const uint64_t* x, uint64_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = mix64(x[i]);
}

// Selection of a float32 compressed matrix: every slice keeps at most S
// entries, its S largest values (ties to the smaller id), in id order.
// Returns the kept count; with outputs non-NULL also fills new_ptr
// (nmajor+1), new_idx and new_val.
int64_t orc_select_f32(int64_t nmajor, const int64_t* ptr, const int32_t* idx, const float* val, int64_t S,
                       int64_t* new_ptr, int32_t* new_idx, float* new_val) {
  std::vector<int64_t> keep;
  int64_t out = 0;
  for (int64_t s = 0; s < nmajor; ++s) {
    if (new_ptr) new_ptr[s] = out;
    select_slice(ptr[s], ptr[s + 1], idx, val, S, keep);
    for (int64_t p : keep) {
      if (new_idx) new_idx[out] = idx[p];
      if (new_val) new_val[out] = val[p];
      ++out;
    }
  }
  if (new_ptr) new_ptr[nmajor] = out;
  return out;
}

}  // extern "C"
