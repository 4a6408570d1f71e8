// Declarations shared by the C-ABI sources (operator state, argument
// builders, launch helpers).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <vector>

#include "../../include/cssar.h"
#include "cssar_kernels.hpp"
#include "cssar_table.hpp"

namespace cssar {
namespace detail {

constexpr double kC = 299792458.0;
constexpr int kMaxPartials = 8192;

// Records a thread-local message (cssar_last_error) and returns code.
int fail(int code, const char* fmt, ...);

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::cssar::detail::fail(CSSAR_EHIP, "%s: %s (%s:%d)", #expr,                \
                                   hipGetErrorString(e_), __FILE__, __LINE__);         \
  } while (0)

const KernelTable* table_for(int n, int v = 0);
size_t align256(size_t n);
int occupancy(const void* fn, int block);
int grid_for(int work, int cus, int per_cu);
// Plan variant the single-array column pass of kind which uses at length n,
// and the one of the chirp-scaling row passes.
int column_variant(int n, int which);
int row_variant(int n);

}  // namespace detail
}  // namespace cssar

// Operator state: parameters, plans and the O(N_a + N_r) device tables.
struct cssar_op {
  int na = 0, nr = 0;
  cssar_params p{};
  int chain = 0;                    // CSSAR_CHAIN_CSA or CSSAR_CHAIN_RDA
  int taps = 0;                     // truncated sinc length (range-Doppler chain)
  int device = 0;
  int cus = 0;
  const cssar::KernelTable* ka = nullptr;  // azimuth length N_a (column passes)
  const cssar::KernelTable* kr = nullptr;  // range length N_r, variant 0 (adjoint, range-Doppler rows)
  const cssar::KernelTable* krow = nullptr;  // range length N_r (chirp-scaling row passes)
  const cssar::KernelTable* kcol[cssar::CK_COUNT] = {};  // per column-pass kind (N_a)
  double2* rowc1 = nullptr;         // per Doppler bin: Phi1 (a1, d1); range-Doppler: migration (a, b)
  double2* rowc2 = nullptr;         //                  Phi2 (a2, b2)
  double2* rowc3 = nullptr;         //                  Phi3 (D, b3); range-Doppler: azimuth filter (A, B)
  float2* tw_a = nullptr;           // w_{N_a}^k
  float2* tw_r = nullptr;           // w_{N_r}^k
  float* partials = nullptr;        // per-block partial sums
  unsigned* counter = nullptr;      // [1]: status bits (non-finite norms); [0] unused
  float* rowd = nullptr;            // per Doppler bin: 18 screen-derivative coefficients
  int grid_row = 0;
  int grid_rda = 0;
  int grid_col[cssar::CK_COUNT] = {};
  int grid_adj[2] = {};
  // optional per-launch HIP event timing (cssar_profile_enable)
  bool profiling = false;
  struct Rec {
    int kind;
    hipEvent_t start, stop;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
};

namespace cssar {
namespace detail {

ColArgs col_args(const cssar_op* op);
RowArgs row_args(const cssar_op* op, const void* in, void* out, int conj);
int check_op(const cssar_op* op);

// A named host range for tracers (rocprofv3 --marker-trace): each entry
// point's call, and inside it each pass launch by kind.  Without a tracer
// attached the calls do nothing.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};
// Names of the pass kinds of cssar_profile_read (the same order).
extern const char* const kPassKindName[CSSAR_PROFILE_KINDS];

// An event from the operator's pool (created when the pool is empty).
hipEvent_t take_event(cssar_op* op);
// Runs launch(), bracketed by two events on s when profiling is on.  Kind ids
// of cssar_profile_read: 0/1 row pass (M / G chain), 2 + column kernel id,
// 13/14 adjoint row pass (M / G forward), 15 selection of the adaptive threshold.
template <typename F>
inline int timed(cssar_op* op, int kind, hipStream_t s, F&& launch) {
  const TraceRange tr(kind >= 0 && kind < CSSAR_PROFILE_KINDS ? kPassKindName[kind] : "cssar_pass");
  hipEvent_t a = nullptr, b = nullptr;
  if (op->profiling) {
    a = take_event(op);
    b = take_event(op);
    if (!a || !b) return fail(CSSAR_EHIP, "hipEventCreate failed");
    HIP_TRY(hipEventRecord(a, s));
  }
  HIP_TRY(launch());
  if (op->profiling) {
    HIP_TRY(hipEventRecord(b, s));
    op->recs.push_back({kind, a, b});
  }
  return CSSAR_OK;
}

// Launch a pass kernel of the operator (timed when profiling is on).
int launch_row(cssar_op* op, const RowArgs& a, hipStream_t s);
int launch_col(cssar_op* op, int which, const ColArgs& a, hipStream_t s);
// After a residual pass (ck = CK_R) or the first, masked forward pass
// (CK_FWD): ||R||^2 into a.hist_out (if not NULL) and the non-finite check
// (if check or a.hist_out).
int residual_total(cssar_op* op, int ck, const ColArgs& a, bool check, hipStream_t s);
int launch_row_adj(cssar_op* op, int conj, const RowArgs& a, hipStream_t s);

// Workspace of the sparse iterate after the solver's three blocked arrays:
// the thread records (from byte 0), the byte offset of the wave masks, and
// the total.
struct SparseLayout {
  size_t wmask, bytes;
};
// The layout for the update plan kt (NULL: the operator's own).
SparseLayout sparse_layout(const cssar_op* op, const KernelTable* kt = nullptr);
// The largest layout over the plan variants of length N_a (batched solver).
size_t sparse_bytes_max(const cssar_op* op);
// Points a's sparse-iterate fields at base (laid out by sparse_layout for
// kt) and dense (a blocked array for the dense tiles).
void set_sparse(const cssar_op* op, ColArgs& a, void* dense, void* base, const KernelTable* kt = nullptr);

// Bytes of the support bits of the adaptive solver's column passes.
size_t support_bytes(const cssar_op* op);
// Selection candidates of the adaptive solvers' value pass: the keys in all
// (candidate_cap), the workgroups of that pass (0 if more than kMaxCandSeg:
// no candidates), the keys per workgroup, and the bytes of the selection
// state with its counts and keys.
unsigned candidate_cap(const cssar_op* op);
unsigned candidate_segments(const cssar_op* op);
unsigned candidate_segment_keys(const cssar_op* op);
size_t adapt_state_bytes(const cssar_op* op);

// Per Doppler bin, the derivatives of the three phase arguments (radians)
// with respect to K_a and K_r as polynomials of the centred column offset
// (Phi1, Phi3) or the signed range bin (Phi2): 18 floats per bin.
void build_derivatives(const cssar_params& p, int na, int nr, std::vector<float>& out);

}  // namespace detail
}  // namespace cssar
