// Instantiates the pass kernels of one plan (length CSSAR_N, variant
// CSSAR_V, set by the build) and exposes them through a KernelTable.
// Compiled once per plan so the heavily unrolled kernels build in parallel.
#include "cssar_kernels.hpp"
#include "cssar_table.hpp"

#if !defined(CSSAR_N) || !defined(CSSAR_V)
#error "CSSAR_N and CSSAR_V must be defined"
#endif

namespace cssar {

#define CSSAR_CAT4(a, b, c, d) a##b##c##d
#define CSSAR_TABLE_NAME(n, v) CSSAR_CAT4(kernel_table_, n, _, v)

const KernelTable* CSSAR_TABLE_NAME(CSSAR_N, CSSAR_V)() {
  using P = Plan<CSSAR_N, CSSAR_V>;
  using K = Kernels<P>;
  static const KernelTable t = {
      CSSAR_N, CSSAR_V, P::E, P::T, P::C, P::CT, P::RT, P::LR, P::P,
      {P::P > 0 ? P::R[0] : 0, P::P > 1 ? P::R[1] : 0, P::P > 2 ? P::R[2] : 0,
       P::P > 3 ? P::R[3] : 0, P::P > 4 ? P::R[4] : 0, 0, 0, 0},
      &K::row,
      {&K::template col<COL_FWD>, &K::template col<COL_INV>, &K::template col<COL_A>,
       &K::template col<COL_R>, &K::template col<COL_VB>, &K::template col<COL_U>,
       &K::template col<COL_XB>, &K::template col<COL_D>, &K::template col<COL_N>,
       &K::template col<COL_V>, &K::template col<COL_T>, &K::template col<COL_AS>},
      &K::row_group,
      {&K::template col_group<COL_FWD>, &K::template col_group<COL_INV>,
       &K::template col_group<COL_A>, &K::template col_group<COL_R>},
      &K::template col_group<COL_AS>,
      {&K::template row_adj<0>, &K::template row_adj<1>},
      {&K::template row_rda<0>, &K::template row_rda<1>},
      reinterpret_cast<const void*>(&row_pass_kernel<P, 0>),
      {reinterpret_cast<const void*>(&col_pass_kernel<P, COL_FWD>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_INV>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_A>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_R>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_VB>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_U>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_XB>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_D>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_N>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_V>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_T>),
       reinterpret_cast<const void*>(&col_pass_kernel<P, COL_AS>)},
      reinterpret_cast<const void*>(&row_group_kernel<P, 0>),
      {reinterpret_cast<const void*>(&col_group_kernel<P, COL_FWD>),
       reinterpret_cast<const void*>(&col_group_kernel<P, COL_INV>),
       reinterpret_cast<const void*>(&col_group_kernel<P, COL_A>),
       reinterpret_cast<const void*>(&col_group_kernel<P, COL_R>)},
      reinterpret_cast<const void*>(&col_group_kernel<P, COL_AS>),
      {reinterpret_cast<const void*>(&row_adj_kernel<P, 0>),
       reinterpret_cast<const void*>(&row_adj_kernel<P, 1>)},
      {reinterpret_cast<const void*>(&row_rda_kernel<P, 0, 8>),
       reinterpret_cast<const void*>(&row_rda_kernel<P, 1, 8>)},
  };
  return &t;
}

}  // namespace cssar
