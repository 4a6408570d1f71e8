// Instantiates the pass kernels of one line length (CSSAR_N, set by the build)
// and exposes them through a KernelTable.  Compiled once per length so the
// heavily unrolled kernels build in parallel.
#include "cssar_kernels.hpp"
#include "cssar_table.hpp"

#ifndef CSSAR_N
#error "CSSAR_N must be defined"
#endif

namespace cssar {

#define CSSAR_CAT2(a, b) a##b
#define CSSAR_CAT(a, b) CSSAR_CAT2(a, b)

const KernelTable* CSSAR_CAT(kernel_table_, CSSAR_N)() {
  using K = Kernels<CSSAR_N>;
  using P = Plan<CSSAR_N>;
  static const KernelTable t = {
      CSSAR_N, P::E, P::T, P::C, P::CT, P::RT, P::LR, P::P,
      {P::P > 0 ? P::R[0] : 0, P::P > 1 ? P::R[1] : 0, P::P > 2 ? P::R[2] : 0,
       P::P > 3 ? P::R[3] : 0, P::P > 4 ? P::R[4] : 0, 0, 0, 0},
      &K::row,
      {&K::template col<COL_FWD>, &K::template col<COL_INV>, &K::template col<COL_A>,
       &K::template col<COL_R>},
      reinterpret_cast<const void*>(&row_pass_kernel<CSSAR_N>),
      {reinterpret_cast<const void*>(&col_pass_kernel<CSSAR_N, COL_FWD>),
       reinterpret_cast<const void*>(&col_pass_kernel<CSSAR_N, COL_INV>),
       reinterpret_cast<const void*>(&col_pass_kernel<CSSAR_N, COL_A>),
       reinterpret_cast<const void*>(&col_pass_kernel<CSSAR_N, COL_R>)},
  };
  return &t;
}

}  // namespace cssar
