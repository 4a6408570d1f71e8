// Compile-time FFT plans: for each supported line length N, the number of
// elements each thread holds (E, so T = N / E threads per line) and the radix
// sequence of the Stockham passes (every radix divides E).  Column passes
// process tiles of C adjacent columns (C lines interleaved in LDS); row
// passes process LR rows per workgroup.
#pragma once

namespace cssar {

template <int N> struct Plan;

// Row passes: RT threads per workgroup handle LR rows (T = N / E threads
// each).  With LR a multiple of 4 the lanes of a wave cover whole 128-byte
// blocks of the blocked layout; with LR = 2 two workgroups share each block
// (64 bytes each), which halves the LDS per workgroup so that two fit on a
// compute unit; LR = 1 is the fallback for the longest lines.
#define CSSAR_PLAN(NN, EE, CC, RTT, ...)                                              \
  template <> struct Plan<NN> {                                                       \
    static constexpr int N = NN;                                                      \
    static constexpr int E = EE;                                                      \
    static constexpr int T = NN / EE;                                                 \
    static constexpr int C = CC; /* column tile width */                              \
    static constexpr int R[] = {__VA_ARGS__};                                         \
    static constexpr int P = sizeof(R) / sizeof(int);                                 \
    static constexpr int radix(int s) { return R[s]; }                                \
    static constexpr int sub(int s) { return s == 0 ? 1 : sub(s - 1) * R[s - 1]; }    \
    static constexpr int prod() { return sub(P); }                                    \
    static constexpr int RT = RTT;    /* row-pass workgroup threads */                \
    static constexpr int LR = RT / T; /* rows per row-pass workgroup */               \
    static constexpr int CT = C * T;  /* column-pass workgroup threads */             \
  };

#ifndef CSSAR_E4096
#define CSSAR_E4096 16
#endif
#ifndef CSSAR_LR4096
#define CSSAR_LR4096 2
#endif
#define CSSAR_RT4096 (CSSAR_LR4096 * 4096 / CSSAR_E4096)

//         N     E   C    RT   radices
CSSAR_PLAN(64, 16, 16, 256, 16, 4)
CSSAR_PLAN(128, 16, 16, 256, 16, 8)
CSSAR_PLAN(256, 16, 16, 256, 16, 16)
CSSAR_PLAN(512, 16, 16, 256, 16, 16, 2)
CSSAR_PLAN(768, 24, 16, 256, 3, 8, 8, 4)
CSSAR_PLAN(1024, 32, 16, 256, 16, 16, 4)
CSSAR_PLAN(1536, 24, 8, 256, 3, 8, 8, 8)
CSSAR_PLAN(2048, 32, 8, 256, 16, 16, 8)
CSSAR_PLAN(3072, 24, 4, 512, 3, 8, 8, 8, 2)
CSSAR_PLAN(4096, CSSAR_E4096, 4, CSSAR_RT4096, 16, 16, 16)
CSSAR_PLAN(8192, 32, 2, 256, 16, 16, 16, 2)

#undef CSSAR_PLAN

// Sanity checks evaluated at compile time for every plan.
template <int N>
constexpr bool plan_ok() {
  using P = Plan<N>;
  if (P::prod() != N) return false;
  for (int s = 0; s < P::P; ++s)
    if (P::E % P::R[s] != 0) return false;
  if (P::CT > 1024 || P::RT > 1024) return false;
  if (P::RT % P::T != 0 || P::T % 4 != 0) return false;
  if (!(P::LR == 1 || P::LR == 2 || P::LR % 4 == 0)) return false;
  return true;
}
static_assert(plan_ok<64>() && plan_ok<128>() && plan_ok<256>() && plan_ok<512>(), "plan");
static_assert(plan_ok<768>() && plan_ok<1024>() && plan_ok<1536>() && plan_ok<2048>(), "plan");
static_assert(plan_ok<3072>() && plan_ok<4096>() && plan_ok<8192>(), "plan");

#define CSSAR_FOR_EACH_LENGTH(X) \
  X(64) X(128) X(256) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096) X(8192)

}  // namespace cssar
