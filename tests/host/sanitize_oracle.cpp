// Host driver for a sanitizer build of the oracle (AddressSanitizer and
// UndefinedBehaviorSanitizer): every entry point of oracle.cpp on small
// random operands, including empty slices, empty operands, CSC layout,
// slice selections and every semiring.  Prints "oracle sanitize ok".
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

extern "C" {
void* orc_spgemm(int semiring, int layout, int64_t nsel, const int64_t* sel, const int64_t* Ap, const int32_t* Ai,
                 const void* Av, const int64_t* Bp, const int32_t* Bi, const void* Bv, int nthreads);
void* orc_sum(int semiring, int64_t m, int k, const int64_t* Pp, const int32_t* Pi, const void* Pv, int nthreads);
int64_t orc_nnz(void* h);
int orc_elem_bytes(void* h);
void orc_copy(void* h, int64_t* ptr, int32_t* idx, void* val);
void orc_free(void* h);
void orc_flops(int layout, int64_t nsel, const int64_t* sel, const int64_t* Ap, const int32_t* Ai,
               const int64_t* Bp, const int32_t* Bi, int64_t* out);
int64_t orc_prune_f32(int64_t nmajor, const int64_t* ptr, const int32_t* idx, const float* val, float thresh,
                      int64_t* new_ptr, int32_t* new_idx, float* new_val);
int orc_digest(int semiring, int layout, int64_t nsel, const int64_t* sel, const int64_t* Ap, const int32_t* Ai,
               const void* Av, const int64_t* Bp, const int32_t* Bi, const void* Bv, int nthreads,
               int64_t* nnz_out, uint64_t* hash_out);
void orc_mix64(int64_t n, const uint64_t* x, uint64_t* out);
int64_t orc_select_f32(int64_t nmajor, const int64_t* ptr, const int32_t* idx, const float* val, int64_t S,
                       int64_t* new_ptr, int32_t* new_idx, float* new_val);
}

namespace {

struct Csr {
  int64_t nmajor, nminor;
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  std::vector<unsigned char> val;  // 8 bytes per entry, read as the semiring's type
};

Csr random_csr(std::mt19937_64& g, int64_t nmajor, int64_t nminor, int maxdeg) {
  Csr m{nmajor, nminor, {0}, {}, {}};
  std::vector<int32_t> row;
  for (int64_t i = 0; i < nmajor; ++i) {
    row.clear();
    const int d = nminor ? static_cast<int>(g() % (maxdeg + 1)) : 0;
    for (int t = 0; t < d; ++t) row.push_back(static_cast<int32_t>(g() % nminor));
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    m.idx.insert(m.idx.end(), row.begin(), row.end());
    m.ptr.push_back(static_cast<int64_t>(m.idx.size()));
  }
  m.val.resize(m.idx.size() * 8);
  for (size_t e = 0; e < m.idx.size(); ++e) {
    const double dv = static_cast<double>(g() % 1000) / 500.0 - 0.5;
    std::memcpy(&m.val[e * 8], &dv, 8);
  }
  return m;
}

// Values of the semiring's input type, in a separate array.
std::vector<unsigned char> typed(const Csr& m, int sr) {
  const size_t n = m.idx.size();
  const int es = (sr == 0 || sr == 5) ? 8 : (sr == 4 ? 1 : 4);
  std::vector<unsigned char> out(n * es + 8);
  for (size_t e = 0; e < n; ++e) {
    double d;
    std::memcpy(&d, &m.val[e * 8], 8);
    if (es == 8) std::memcpy(&out[e * 8], &d, 8);
    if (es == 1) out[e] = d > 0 ? 1 : 0;
    if (es == 4) {
      if (sr == 2) {
        const int32_t iv = static_cast<int32_t>(d * 100);
        std::memcpy(&out[e * 4], &iv, 4);
      } else {
        const float fv = static_cast<float>(d);
        std::memcpy(&out[e * 4], &fv, 4);
      }
    }
  }
  return out;
}

int check_product(const Csr& A, const Csr& B, int sr, int layout, const std::vector<int64_t>* sel) {
  const auto av = typed(A, sr), bv = typed(B, sr);
  const int64_t nsl = layout == 0 ? A.nmajor : B.nmajor;
  const int64_t nsel = sel ? static_cast<int64_t>(sel->size()) : nsl;
  void* h = orc_spgemm(sr, layout, nsel, sel ? sel->data() : nullptr, A.ptr.data(), A.idx.data(), av.data(),
                       B.ptr.data(), B.idx.data(), bv.data(), 2);
  if (!h) return 1;
  const int64_t nnz = orc_nnz(h);
  std::vector<int64_t> ptr(nsel + 1);
  std::vector<int32_t> idx(nnz + 1);
  std::vector<unsigned char> val((nnz + 1) * orc_elem_bytes(h));
  orc_copy(h, ptr.data(), idx.data(), val.data());
  orc_free(h);
  if (ptr[nsel] != nnz) return 2;
  std::vector<int64_t> fl(nsel);
  orc_flops(layout, nsel, sel ? sel->data() : nullptr, A.ptr.data(), A.idx.data(), B.ptr.data(), B.idx.data(),
            fl.data());
  if (sr >= 2) {
    std::vector<int64_t> dn(nsel);
    std::vector<uint64_t> dh(nsel);
    if (orc_digest(sr, layout, nsel, sel ? sel->data() : nullptr, A.ptr.data(), A.idx.data(), av.data(),
                   B.ptr.data(), B.idx.data(), bv.data(), 2, dn.data(), dh.data()) != 0)
      return 3;
    for (int64_t t = 0; t < nsel; ++t)
      if (dn[t] != ptr[t + 1] - ptr[t]) return 4;
  }
  return 0;
}

}  // namespace

int main() {
  std::mt19937_64 g(2106);
  int bad = 0;
  const int64_t shapes[][3] = {{0, 0, 0}, {1, 1, 1}, {7, 0, 5}, {40, 33, 50}, {100, 80, 120}, {300, 257, 64}};
  for (const auto& sh : shapes) {
    const Csr A = random_csr(g, sh[0], sh[1], 9);
    const Csr B = random_csr(g, sh[1], sh[2], 9);
    for (int sr = 0; sr <= 6; ++sr) {
      bad |= check_product(A, B, sr, 0, nullptr);
      std::vector<int64_t> sel;
      for (int64_t i = 0; i < A.nmajor; i += 3) sel.push_back(i);
      bad |= check_product(A, B, sr, 0, &sel);
      // CSC: slices are columns of C, the operands' arrays are read as CSC
      const Csr Ac = random_csr(g, sh[1], sh[0], 9);  // n x m stored by columns: ncols = sh[1]
      const Csr Bc = random_csr(g, sh[2], sh[1], 9);
      bad |= check_product(Ac, Bc, sr, 1, nullptr) << 4;
    }
    // sum of parts, prune, selection
    const Csr P = random_csr(g, 3 * sh[0], sh[2], 9);
    for (int sr = 0; sr <= 6; ++sr) {
      const auto pv = typed(P, sr);
      void* h = orc_sum(sr, sh[0], 3, P.ptr.data(), P.idx.data(), pv.data(), 2);
      if (!h) bad |= 64; else orc_free(h);
    }
    const auto fv = typed(P, 1);
    const float* f = reinterpret_cast<const float*>(fv.data());
    const int64_t kept = orc_prune_f32(P.nmajor, P.ptr.data(), P.idx.data(), f, 0.25f, nullptr, nullptr, nullptr);
    std::vector<int64_t> np(P.nmajor + 1);
    std::vector<int32_t> ni(kept + 1);
    std::vector<float> nv(kept + 1);
    if (orc_prune_f32(P.nmajor, P.ptr.data(), P.idx.data(), f, 0.25f, np.data(), ni.data(), nv.data()) != kept)
      bad |= 128;
    for (int64_t S : {0, 1, 3, 1000}) {
      const int64_t ks = orc_select_f32(P.nmajor, P.ptr.data(), P.idx.data(), f, S, nullptr, nullptr, nullptr);
      std::vector<int64_t> sp(P.nmajor + 1);
      std::vector<int32_t> si(ks + 1);
      std::vector<float> sv(ks + 1);
      if (orc_select_f32(P.nmajor, P.ptr.data(), P.idx.data(), f, S, sp.data(), si.data(), sv.data()) != ks)
        bad |= 256;
    }
  }
  std::vector<uint64_t> x(257), y(257);
  for (auto& v : x) v = g();
  orc_mix64(static_cast<int64_t>(x.size()), x.data(), y.data());
  if (bad) {
    std::printf("oracle sanitize FAILED (%d)\n", bad);
    return 1;
  }
  std::printf("oracle sanitize ok\n");
  return 0;
}
