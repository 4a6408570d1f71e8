// Per-length table of pass launchers and plan constants, filled by
// kern_inst.hip for every supported length.
#pragma once

#include <hip/hip_runtime.h>

namespace cssar {

struct RowArgs;
struct ColArgs;

enum ColKernel { CK_FWD = 0, CK_INV, CK_A, CK_R, CK_COUNT };

struct KernelTable {
  int n, E, T, C, CT, RT, LR, passes;
  int radices[8];
  hipError_t (*row)(const RowArgs&, int, hipStream_t);
  hipError_t (*col[CK_COUNT])(const ColArgs&, int, hipStream_t);
  const void* row_fn;
  const void* col_fn[CK_COUNT];
};

#define CSSAR_DECL_TABLE(NN) const KernelTable* kernel_table_##NN();
CSSAR_DECL_TABLE(64)
CSSAR_DECL_TABLE(128)
CSSAR_DECL_TABLE(256)
CSSAR_DECL_TABLE(512)
CSSAR_DECL_TABLE(768)
CSSAR_DECL_TABLE(1024)
CSSAR_DECL_TABLE(1536)
CSSAR_DECL_TABLE(2048)
CSSAR_DECL_TABLE(3072)
CSSAR_DECL_TABLE(4096)
CSSAR_DECL_TABLE(8192)
#undef CSSAR_DECL_TABLE

}  // namespace cssar
