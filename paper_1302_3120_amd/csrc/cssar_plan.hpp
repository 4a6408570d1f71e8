// Compile-time FFT plans: for each supported line length N and plan variant
// V, the number of elements each thread holds (E, so T = N / E threads per
// line) and the radix sequence of the Stockham passes (every radix divides
// E).  Column passes process tiles of C adjacent columns (C lines interleaved
// in LDS); row passes process LR rows per workgroup.  Variant 0 is the
// default of every length; variants 1 and 2, where they exist, are
// alternative schedules (other E, radices, tile width or rows per
// workgroup) that the batched solver's autotuner may pick after measuring
// them, and that the single-array passes use where they measured faster.
// A split plan (SPLIT)
// exchanges through half the LDS, in two rounds, for rows and columns.
#pragma once

namespace cssar {

template <int N, int V> struct Plan;

// Row passes: RT threads per workgroup handle LR rows (T = N / E threads
// each).  With LR a multiple of 4 the lanes of a wave cover whole 128-byte
// blocks of the blocked layout; with LR = 2 two workgroups share each block
// (64 bytes each), which halves the LDS per workgroup so that two fit on a
// compute unit; LR = 1 is the fallback for the longest lines.
#define CSSAR_PLAN_S(NN, VV, EE, CC, RTT, SPL, ...)                                          \
  template <> struct Plan<NN, VV> {                                                   \
    static constexpr int N = NN;                                                      \
    static constexpr int V = VV;                                                      \
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
    /* column passes exchange through half the LDS (two workgroups per CU) */         \
    static constexpr bool SPLIT = SPL;                                                \
  };
#define CSSAR_PLAN(NN, VV, EE, CC, RTT, ...) CSSAR_PLAN_S(NN, VV, EE, CC, RTT, false, __VA_ARGS__)

//         N    V   E   C    RT   radices
CSSAR_PLAN(64, 0, 16, 16, 256, 16, 4)
CSSAR_PLAN(128, 0, 16, 16, 256, 16, 8)
CSSAR_PLAN(256, 0, 16, 16, 256, 16, 16)
CSSAR_PLAN(512, 0, 8, 16, 256, 8, 8, 8)
CSSAR_PLAN(512, 1, 16, 16, 256, 16, 16, 2)
CSSAR_PLAN(768, 0, 24, 16, 256, 24, 8, 4)
CSSAR_PLAN(1024, 0, 16, 8, 256, 16, 16, 4)
CSSAR_PLAN(1024, 1, 32, 16, 256, 16, 16, 4)
CSSAR_PLAN(1536, 0, 24, 4, 128, 24, 8, 8)
CSSAR_PLAN(1536, 1, 24, 8, 256, 24, 8, 8)
CSSAR_PLAN(2048, 0, 16, 8, 256, 16, 16, 8)
CSSAR_PLAN(2048, 1, 16, 4, 256, 16, 16, 8)
CSSAR_PLAN(3072, 0, 24, 4, 512, 24, 8, 8, 2)
CSSAR_PLAN(4096, 0, 16, 4, 512, 16, 16, 16)
CSSAR_PLAN(4096, 1, 32, 4, 256, 16, 16, 16)
// two-column tiles (half the LDS of a four-column tile: two workgroups per CU)
CSSAR_PLAN(4096, 2, 16, 2, 512, 16, 16, 16)
CSSAR_PLAN(8192, 0, 16, 2, 512, 16, 16, 16, 2)
// 8192-point lines through half the LDS: four-column tiles, and two rows per
// row-pass workgroup (two workgroups per CU)
CSSAR_PLAN_S(8192, 1, 32, 4, 512, true, 16, 16, 32)

#undef CSSAR_PLAN
#undef CSSAR_PLAN_S

// Sanity checks evaluated at compile time for every plan.
template <class P>
constexpr bool plan_ok() {
  if (P::prod() != P::N) return false;
  for (int s = 0; s < P::P; ++s)
    if (P::E % P::R[s] != 0) return false;
  if (P::CT > 1024 || P::RT > 1024) return false;
  if (P::RT % P::T != 0 || P::T % 4 != 0) return false;
  if (!(P::LR == 1 || P::LR == 2 || P::LR % 4 == 0)) return false;
  return true;
}

// Every (length, variant) pair that is compiled.
#define CSSAR_FOR_EACH_PLAN(X)                                                    \
  X(64, 0) X(128, 0) X(256, 0) X(512, 0) X(512, 1) X(768, 0) X(1024, 0) X(1024, 1) \
  X(1536, 0) X(1536, 1) X(2048, 0) X(2048, 1) X(3072, 0) X(4096, 0) X(4096, 1) X(4096, 2) \
  X(8192, 0) X(8192, 1)

#define CSSAR_CHECK_PLAN(NN, VV) static_assert(plan_ok<Plan<NN, VV>>(), "plan");
CSSAR_FOR_EACH_PLAN(CSSAR_CHECK_PLAN)
#undef CSSAR_CHECK_PLAN

#define CSSAR_FOR_EACH_LENGTH(X) \
  X(64) X(128) X(256) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096) X(8192)

constexpr int kMaxVariants = 3;

}  // namespace cssar
