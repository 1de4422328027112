// Host run of the per-slice index logic the kernels use (spg_rowlogic.h):
// the panel index on sorted and unsorted slices, and the sorting network.
// Lanes are run one after another, in forward and in reverse order, which
// covers every outcome of the unordered writes of step 2 on one slot that a
// wave can produce (the last writer wins).  Prints one line per failure;
// exit status 0 when all checks pass.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "spg_rowlogic.h"

using namespace spg;

static int failures = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      std::printf("FAIL %s: ", #cond);        \
      std::printf(__VA_ARGS__);               \
      std::printf("\n");                      \
      ++failures;                             \
    }                                         \
  } while (0)

constexpr int32_t kSentinel = -12345;

// The index as the kernel computes it with nlanes lanes, lanes run in the
// given order in each step.
static std::vector<int32_t> index_of(const std::vector<int32_t>& ids, int wlog2, int P, int nlanes, bool reverse) {
  std::vector<int32_t> out(P + 1, kSentinel);
  const int32_t len = static_cast<int32_t>(ids.size());
  for (int t = 0; t < nlanes; ++t) panel_index_fill(out.data(), P, len, reverse ? nlanes - 1 - t : t, nlanes);
  for (int t = 0; t < nlanes; ++t)
    panel_index_open(ids.data(), len, wlog2, P, out.data(), reverse ? nlanes - 1 - t : t, nlanes);
  return out;
}

// Whether every panel segment [out[p], out[p+1]) of the slice holds only ids
// of panel p, as the accumulators assume.
static bool segments_hold_their_panels(const std::vector<int32_t>& ids, const std::vector<int32_t>& out, int wlog2,
                                       int P) {
  for (int p = 0; p < P; ++p) {
    if (out[p + 1] < out[p]) return false;
    for (int32_t q = out[p]; q < out[p + 1]; ++q)
      if ((ids[q] >> wlog2) != p) return false;
  }
  return true;
}

static void panel_index_checks() {
  const int wlog2 = 8, P = 4;  // 1024 columns in 4 panels of 256
  // a descending slice: every slot is written and in range, but the panel
  // segments do not hold their panels' ids, so the index is only usable on
  // sorted slices; sorted first (as the library does for an unsorted
  // operand), the same ids give the right segments
  const std::vector<int32_t> desc = {900, 700, 300, 10};
  for (int nl : {1, 4, 64})
    for (bool rev : {false, true}) {
      const auto idx = index_of(desc, wlog2, P, nl, rev);
      for (int p = 0; p <= P; ++p)
        CHECK(idx[p] >= 0 && idx[p] <= 4, "descending slice, lanes %d rev %d: slot %d = %d", nl, rev, p, idx[p]);
      CHECK(!segments_hold_their_panels(desc, idx, wlog2, P), "descending slice: segments should not fit");
    }
  {
    std::vector<int32_t> key = desc, pos = {0, 1, 2, 3};
    const int N = network_size(4);
    for (int k = 2; k <= N; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) sort_network_step(key.data(), pos.data(), 4, N, k, j, 0, 1);
    const auto idx = index_of(key, wlog2, P, 64, false);
    CHECK(segments_hold_their_panels(key, idx, wlog2, P), "sorted copy: segments must hold their panels");
    CHECK(idx[0] == 0 && idx[1] == 1 && idx[2] == 2 && idx[3] == 3 && idx[4] == 4, "sorted copy index");
  }
  // sorted slices: the definition (ids below each panel start), any lane count
  std::mt19937 rng(7);
  for (int trial = 0; trial < 200; ++trial) {
    const int len = trial % 40;
    std::vector<int32_t> ids;
    std::uniform_int_distribution<int32_t> col(0, (P << wlog2) - 1);
    while (static_cast<int>(ids.size()) < len) {
      const int32_t c = col(rng);
      if (std::find(ids.begin(), ids.end(), c) == ids.end()) ids.push_back(c);
    }
    std::sort(ids.begin(), ids.end());
    for (int nl : {1, 3, 64})
      for (bool rev : {false, true}) {
        const auto idx = index_of(ids, wlog2, P, nl, rev);
        for (int p = 0; p <= P; ++p) {
          const int32_t below = static_cast<int32_t>(
              std::count_if(ids.begin(), ids.end(), [&](int32_t c) { return c < (p << wlog2); }));
          CHECK(idx[p] == below, "sorted slice len %d lanes %d: slot %d = %d, want %d", len, nl, p, idx[p], below);
        }
        CHECK(segments_hold_their_panels(ids, idx, wlog2, P), "sorted slice len %d: segments", len);
      }
    // the same ids shuffled: every slot defined and within [0, len]
    std::shuffle(ids.begin(), ids.end(), rng);
    const auto idx = index_of(ids, wlog2, P, 64, trial & 1);
    for (int p = 0; p <= P; ++p)
      CHECK(idx[p] >= 0 && idx[p] <= len, "shuffled slice: slot %d = %d (len %d)", p, idx[p], len);
  }
}

static void sort_network_checks() {
  std::mt19937 rng(11);
  for (int L : {0, 1, 2, 3, 5, 8, 13, 64, 100, 255, 256, 257, 1000, 2048, 2049, 5000}) {
    for (int dup = 0; dup < 2; ++dup) {
      std::vector<int32_t> key(L), pos(L);
      std::uniform_int_distribution<int32_t> d(0, dup ? 20 : 1 << 30);
      for (int i = 0; i < L; ++i) {
        key[i] = d(rng);
        pos[i] = i;
      }
      const std::vector<int32_t> orig = key;
      const int N = network_size(L);
      for (int nl : {1, 7}) {
        std::vector<int32_t> k2 = orig, p2 = pos;
        for (int k = 2; k <= N; k <<= 1)
          for (int j = k >> 1; j > 0; j >>= 1)
            for (int t = 0; t < nl; ++t) sort_network_step(k2.data(), p2.data(), L, N, k, j, nl - 1 - t, nl);
        CHECK(std::is_sorted(k2.begin(), k2.end()), "L %d dup %d lanes %d: not sorted", L, dup, nl);
        std::vector<int> seen(L, 0);
        for (int i = 0; i < L; ++i) {
          CHECK(p2[i] >= 0 && p2[i] < L, "L %d: position %d out of range", L, p2[i]);
          if (p2[i] >= 0 && p2[i] < L) {
            ++seen[p2[i]];
            CHECK(orig[p2[i]] == k2[i], "L %d: key %d at %d does not come from position %d", L, k2[i], i, p2[i]);
          }
        }
        for (int i = 0; i < L; ++i) CHECK(seen[i] == 1, "L %d: position %d seen %d times", L, i, seen[i]);
      }
    }
  }
}

int main() {
  panel_index_checks();
  sort_network_checks();
  if (failures == 0) std::printf("rowlogic ok\n");
  return failures == 0 ? 0 : 1;
}
