// Per-plan table of pass launchers and plan constants, filled by
// kern_inst.hip for every compiled (length, variant) pair.
#pragma once

#include <hip/hip_runtime.h>

#include "cssar_plan.hpp"

namespace cssar {

struct RowArgs;
struct ColArgs;
struct GroupArgs;

// Column kernels (the same order as ColMode): the first CK_GROUPED also
// exist as grouped (batched) kernels, and so does CK_AS (col_group_as).
// CK_D .. CK_T: the adaptive step and threshold passes; CK_AS: the update
// pass of the sparse iterate.
enum ColKernel { CK_FWD = 0, CK_INV, CK_A, CK_R, CK_VB, CK_U, CK_XB, CK_D, CK_N, CK_V, CK_T, CK_AS, CK_COUNT };
constexpr int CK_GROUPED = 4;

struct KernelTable {
  int n, variant, E, T, C, CT, RT, LR, passes;
  int radices[8];
  hipError_t (*row)(const RowArgs&, int, hipStream_t);
  hipError_t (*col[CK_COUNT])(const ColArgs&, int, hipStream_t);
  hipError_t (*row_group)(const GroupArgs&, int, hipStream_t);
  hipError_t (*col_group[CK_GROUPED])(const GroupArgs&, int, hipStream_t);
  hipError_t (*col_group_as)(const GroupArgs&, int, hipStream_t);
  hipError_t (*row_adj[2])(const RowArgs&, int, hipStream_t);  // forward chain M (0) or G (1)
  hipError_t (*row_rda[2])(const RowArgs&, int, hipStream_t);  // range-Doppler chain M (0), G (1)
  const void* row_fn;
  const void* col_fn[CK_COUNT];
  const void* row_group_fn;
  const void* col_group_fn[CK_GROUPED];
  const void* col_group_as_fn;
  const void* row_adj_fn[2];
  const void* row_rda_fn[2];
};

#define CSSAR_DECL_TABLE(NN, VV) const KernelTable* kernel_table_##NN##_##VV();
CSSAR_FOR_EACH_PLAN(CSSAR_DECL_TABLE)
#undef CSSAR_DECL_TABLE

}  // namespace cssar
