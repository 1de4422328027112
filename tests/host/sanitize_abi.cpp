// Host driver for a sanitizer build of the C ABI's host code
// (AddressSanitizer and UndefinedBehaviorSanitizer on the host side only):
// plan creation for every semiring, both layouts, empty and rectangular
// shapes and option sets, workspace sizes and layouts, panel queries, the
// sum plan, and every rejected descriptor, with no device work (descriptor
// pointers are never dereferenced by these calls).  Prints "abi sanitize ok".
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "spg.h"

int main() {
  int bad = 0;
  static int64_t dummy_ptr[4];
  void* d = dummy_ptr;
  const int32_t shapes[][3] = {{0, 0, 0}, {1, 1, 1}, {4096, 4096, 4096}, {1 << 20, 1 << 20, 1 << 20},
                               {1000, 70000, 3}, {5, 3, 200000}};
  for (const auto& sh : shapes) {
    for (int layout = 0; layout <= 1; ++layout) {
      for (int sr = 0; sr <= 6; ++sr) {
        for (int ov = 0; ov < 4; ++ov) {
          spg_options o;
          std::memset(&o, 0, sizeof(o));
          if (ov == 1) {
            o.hash_max_flops = 32;
            o.hash_max_nnz = 32;
            o.lds_budget = 1024;
            o.dense_threads = 256;
            o.bitmap_mib = 1;
          } else if (ov == 2) {
            o.sym_windows = 8;
            o.bitmap_mib = 64;
            o.sym_panel_log2 = 8;
          } else if (ov == 3) {
            o.split_panels = 1;
            o.sym_panel_log2 = 8;
            o.lds_budget = 4096;
            o.unsorted = -1;
            o.b_checked = 1;
          }
          spg_matrix A{layout ? sh[1] : sh[0], layout ? sh[0] : sh[1], 10, static_cast<spg_layout>(layout),
                       dummy_ptr, static_cast<const int32_t*>(d), d};
          spg_matrix B{layout ? sh[2] : sh[1], layout ? sh[1] : sh[2], 10, static_cast<spg_layout>(layout),
                       dummy_ptr, static_cast<const int32_t*>(d), d};
          if (layout) {  // CSC: A is m x n stored by columns; shapes as for CSR
            A.nrows = sh[0];
            A.ncols = sh[1];
            B.nrows = sh[1];
            B.ncols = sh[2];
          }
          spg_plan* p = nullptr;
          const spg_status st = spg_plan_create(&A, &B, static_cast<spg_semiring>(sr), &o, nullptr, &p);
          if (st != SPG_OK) {
            if (p) bad |= 1;
            continue;
          }
          size_t ws = 0;
          bad |= spg_workspace_size(p, &ws) != SPG_OK ? 2 : 0;
          int a, b, c, e;
          bad |= spg_plan_panels(p, &a, &b, &c, &e) != SPG_OK ? 4 : 0;
          spg_options back;
          bad |= spg_plan_options(p, &back) != SPG_OK ? 8 : 0;
          bad |= spg_numeric(p, nullptr, nullptr, nullptr) != SPG_E_STATE ? 16 : 0;
          int64_t f;
          bad |= spg_plan_stats(p, &f, nullptr) != SPG_E_STATE ? 32 : 0;
          spg_plan_destroy(p);
        }
      }
    }
  }
  // rejected descriptors and options
  spg_matrix A{4, 5, 3, SPG_CSR, dummy_ptr, static_cast<const int32_t*>(d), d};
  spg_matrix B{6, 4, 3, SPG_CSR, dummy_ptr, static_cast<const int32_t*>(d), d};
  spg_plan* p = nullptr;
  bad |= spg_plan_create(&A, &B, SPG_PLUS_TIMES_F64, nullptr, nullptr, &p) != SPG_E_SHAPE ? 64 : 0;
  B.nrows = 5;
  B.layout = SPG_CSC;
  bad |= spg_plan_create(&A, &B, SPG_PLUS_TIMES_F64, nullptr, nullptr, &p) != SPG_E_LAYOUT ? 128 : 0;
  B.layout = SPG_CSR;
  B.val = nullptr;
  bad |= spg_plan_create(&A, &B, SPG_PLUS_TIMES_F64, nullptr, nullptr, &p) != SPG_E_SEMIRING ? 256 : 0;
  spg_options o;
  std::memset(&o, 0, sizeof(o));
  o.hash_max_flops = 1 << 20;
  bad |= spg_plan_create(&A, &B, SPG_OR_AND_BOOL, &o, nullptr, &p) != SPG_E_INVALID ? 512 : 0;
  // semiring sum plan and panel index sizes
  spg_matrix P{12, 7, 5, SPG_CSR, dummy_ptr, static_cast<const int32_t*>(d), d};
  for (int sr = 0; sr <= 6; ++sr) {
    if (spg_sum_plan_create(3, &P, static_cast<spg_semiring>(sr), nullptr, nullptr, &p) != SPG_OK) {
      bad |= 1024;
      continue;
    }
    size_t ws = 0;
    spg_workspace_size(p, &ws);
    spg_plan_destroy(p);
  }
  bad |= spg_sum_plan_create(5, &P, SPG_MIN_PLUS_I32, nullptr, nullptr, &p) != SPG_E_SHAPE ? 2048 : 0;
  size_t bytes = 0;
  bad |= spg_panel_index_size(&P, 3, &bytes) != SPG_OK ? 4096 : 0;
  spg_matrix big{1, SPG_NOALLOC_MAX_SLICES + 1, 0, SPG_CSC, dummy_ptr, static_cast<const int32_t*>(d), d};
  int64_t nn = -1;
  bad |= spg_prune_count_f32_noalloc(&big, 1e-4f, nullptr, dummy_ptr, &nn) != SPG_E_NOMEM ? 8192 : 0;
  for (int s = 0; s <= 8; ++s) bad |= spg_status_str(static_cast<spg_status>(s)) ? 0 : 16384;
  if (bad) {
    std::printf("abi sanitize FAILED (%d)\n", bad);
    return 1;
  }
  std::printf("abi sanitize ok\n");
  return 0;
}
