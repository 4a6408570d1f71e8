// Batched iterative thresholding: many scenes advanced together by grouped
// persistent pass kernels (one launch per pass kind and line length), with
// optional HIP-graph replay of the middle iterations and a measuring
// autotuner for the plan variant and workgroups per compute unit.  The
// arithmetic per scene is that of cssar_ita_solve (eq. (th2d), Algorithm 1).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "cssar_internal.hpp"

using namespace cssar;
using namespace cssar::detail;

namespace {

// Pass kinds with their own plan choice.  The forward column pass of the
// first iteration keeps the default plan.
enum TuneKind { TK_ROW = 0, TK_R, TK_A, TK_COUNT };
const char* const kTuneName[TK_COUNT] = {"row", "col_residual", "col_update"};

// Launch slots of a group: which arguments and which kernel.
enum SlotKind { SL_ROW_M = 0, SL_ROW_G, SL_FWD, SL_R, SL_A_FIRST, SL_A_MID, SL_A_LAST, SL_A_ONLY, SL_COUNT };

struct Choice {
  int variant = 0;
  int per_cu = 0;  // resident workgroups per CU in the persistent grid; 0 = occupancy limit
};

struct Slot {
  size_t args = 0, start = 0;  // byte offsets in the argument table block
  int total = 0, grid = 0;
  const KernelTable* kt = nullptr;
};

struct Group {
  bool row;                 // row passes over length n = N_r, else column passes over n = N_a
  int n;
  std::vector<int> scenes;  // indices into the batch
  Choice ch[TK_COUNT];
  Slot slot[SL_COUNT];
  int def_variant[TK_COUNT] = {};  // the single-array solver's plan (the autotuner's reference)
  // autotuner parity gate: relative L2 distance of each plan variant's output
  // from the reference plan's on a seeded input (-1: not measured)
  double gate[TK_COUNT][kMaxVariants];
  Group() {
    for (auto& r : gate)
      for (double& e : r) e = -1.0;
  }
};

// A plan variant is accepted by the autotuner only within this distance of
// the reference plan's output (relative L2 over the group's scenes).
constexpr double kGateTol = 1e-5;

bool slot_used(const Group& g, int k) {
  return g.row ? (k == SL_ROW_M || k == SL_ROW_G) : (k >= SL_FWD);
}

int tune_kind(int slot) {
  switch (slot) {
    case SL_ROW_M:
    case SL_ROW_G:
      return TK_ROW;
    case SL_R:
      return TK_R;
    case SL_FWD:
      return -1;
    default:
      return TK_A;
  }
}

int col_mode(int slot) {
  switch (slot) {
    case SL_FWD:
      return CK_FWD;
    case SL_R:
      return CK_R;
    default:
      return CK_AS;
  }
}

// Grouped column kernel of a kind and its launcher (the sparse-iterate
// update has its own slot in the table).
const void* col_group_fn(const KernelTable* kt, int ck) {
  return ck == CK_AS ? kt->col_group_as_fn : kt->col_group_fn[ck];
}
hipError_t launch_col_group(const KernelTable* kt, int ck, const GroupArgs& g, int grid, hipStream_t s) {
  return ck == CK_AS ? kt->col_group_as(g, grid, s) : kt->col_group[ck](g, grid, s);
}

// ------------------------------------------------ seeded fill and distance --
// 32-bit integer hash (the "lowbias32" mix of shifts and odd multipliers
// published by C. Wellons' hash-prospector project).
__device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// n complex values, each part uniform in [-1, 1), from the hash of (seed,
// index): the autotuner's test input.
__global__ __launch_bounds__(256) void gate_fill_kernel(float2* __restrict__ p, size_t n, uint32_t seed) {
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    const uint32_t h = mix32(seed * 0x9e3779b9u ^ (uint32_t)(i >> 32) * 0x85ebca6bu);
    const uint32_t a = mix32(h ^ (uint32_t)(2 * i)), b = mix32(h ^ (uint32_t)(2 * i + 1));
    p[i] = make_float2((float)(a >> 8) * (1.0f / 8388608.0f) - 1.0f, (float)(b >> 8) * (1.0f / 8388608.0f) - 1.0f);
  }
}

constexpr int kGateBlocks = 256;

// Per block: sum |a - r|^2 and sum |r|^2 (FP64) into part[2 blk], part[2 blk + 1].
__global__ __launch_bounds__(256) void gate_diff_kernel(const float2* __restrict__ a, const float2* __restrict__ r,
                                                        size_t n, double* __restrict__ part) {
  __shared__ double sd[256], sr[256];
  double d = 0.0, q = 0.0;
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    const float2 x = a[i], y = r[i];
    const double dx = (double)x.x - y.x, dy = (double)x.y - y.y;
    d += dx * dx + dy * dy;
    q += (double)y.x * y.x + (double)y.y * y.y;
  }
  sd[threadIdx.x] = d;
  sr[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sd[threadIdx.x] += sd[threadIdx.x + w];
      sr[threadIdx.x] += sr[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sd[0];
    part[2 * blockIdx.x + 1] = sr[0];
  }
}

// ---------------------------------------------------------- finite check --
struct CheckArg {
  const float4* x;  // X of the scene (two complex values per float4)
  long long n4;     // float4 count
};

// Bit 0 of status[scene] when X of the scene (blockIdx.y) holds a NaN or an
// infinity.
__global__ __launch_bounds__(256) void finite_check_kernel(const CheckArg* __restrict__ args,
                                                           unsigned* __restrict__ status) {
  const CheckArg a = args[blockIdx.y];
  bool bad = false;
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.n4; i += step) {
    const float4 v = a.x[i];
    bad |= !(isfinite(v.x) && isfinite(v.y) && isfinite(v.z) && isfinite(v.w));
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(status + blockIdx.y, 1u);
}

}  // namespace

struct cssar_batch {
  std::vector<cssar_op*> ops;
  int device = 0, cus = 0;
  std::string arch;
  std::vector<size_t> ws_off;  // per scene: X, P, Y blocked arrays from here
  std::vector<size_t> blk;     // per scene: bytes of one blocked array (aligned)
  size_t ws_bytes = 0;
  std::vector<Group> groups;
  size_t table_bytes = 0;
  char* dev_table = nullptr;   // device copy of the argument tables
  size_t check_off = 0;        // byte offset of the finite-check arguments in the table block
  unsigned* status = nullptr;  // per scene: bit 0 non-finite X (finite_check_kernel)
  double* gate_part = nullptr; // per-block sums of gate_diff_kernel
  char* staging = nullptr;     // pinned host staging of the same
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  bool use_graph = false;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
};

namespace {

void drop_graph(cssar_batch* b) {
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->graph_exec = nullptr;
  b->graph = nullptr;
}

// Recompute the plan, unit counts and grid of every slot from the choices.
void plan_slots(cssar_batch* b) {
  for (auto& g : b->groups) {
    for (int k = 0; k < SL_COUNT; ++k) {
      if (!slot_used(g, k)) continue;
      Slot& sl = g.slot[k];
      const int tk = tune_kind(k);
      const Choice c = tk >= 0 ? g.ch[tk] : Choice{};
      sl.kt = table_for(g.n, c.variant);
      int total = 0;
      for (int s : g.scenes) {
        const cssar_op* op = b->ops[s];
        total += g.row ? op->na / sl.kt->LR : op->nr / sl.kt->C;
      }
      sl.total = total;
      const void* fn = g.row ? sl.kt->row_group_fn : col_group_fn(sl.kt, col_mode(k));
      const int occ = occupancy(fn, g.row ? sl.kt->RT : sl.kt->CT);
      const int per_cu = c.per_cu > 0 ? std::min(c.per_cu, occ) : occ;
      sl.grid = grid_for(total, b->cus, per_cu);
    }
  }
}

// A plan variant is usable for a group if every scene's other dimension
// fits its unit shape.
bool variant_fits(const cssar_batch* b, const Group& g, const KernelTable* kt) {
  for (int s : g.scenes) {
    const cssar_op* op = b->ops[s];
    if (g.row ? (op->na % kt->LR != 0) : (op->nr % kt->C != 0)) return false;
  }
  return true;
}

struct CallArgs {
  const void* const* ys = nullptr;
  const void* const* masks = nullptr;
  const float* lambdas = nullptr;
  void* const* x_outs = nullptr;
  char* ws = nullptr;
};

// Fill the staging copy of every slot's per-scene arguments and unit prefix
// sums, then copy it to the device table on the stream.
int upload_tables(cssar_batch* b, const CallArgs& c, hipStream_t s) {
  if (b->upload_pending) {
    HIP_TRY(hipEventSynchronize(b->upload_done));  // staging still being read
    b->upload_pending = false;
  }
  char* h = b->staging;
  for (auto& g : b->groups) {
    for (int k = 0; k < SL_COUNT; ++k) {
      if (!slot_used(g, k)) continue;
      const Slot& sl = g.slot[k];
      int* start = (int*)(h + sl.start);
      int acc = 0;
      for (size_t q = 0; q < g.scenes.size(); ++q) {
        const int si = g.scenes[q];
        const cssar_op* op = b->ops[si];
        start[q] = acc;
        acc += g.row ? op->na / sl.kt->LR : op->nr / sl.kt->C;
        float2* Xd = (float2*)(c.ws + b->ws_off[si]);
        float2* P = (float2*)(c.ws + b->ws_off[si] + b->blk[si]);
        float2* Y = (float2*)(c.ws + b->ws_off[si] + 2 * b->blk[si]);
        if (g.row) {
          RowArgs a = row_args(op, P, P, k == SL_ROW_M ? 0 : 1);
          std::memcpy(h + sl.args + q * sizeof(RowArgs), &a, sizeof a);
          continue;
        }
        ColArgs a = col_args(op);
        a.partials = nullptr;
        a.status = nullptr;
        a.hist_out = nullptr;
        a.y = Y;
        a.mask = c.masks ? (const uint32_t*)c.masks[si] : nullptr;
        a.sigma = (c.lambdas ? c.lambdas[si] : 0.0f) * a.mu;
        float2* xo = c.x_outs ? (float2*)c.x_outs[si] : nullptr;
        switch (k) {
          case SL_FWD:  // R(0) = m o y: P = F_eta R, Y = marked copy of m o y
            a.in0 = c.ys ? (const float2*)c.ys[si] : nullptr;
            a.out = P;
            a.out2 = Y;
            a.flags = 1 | 4;
            break;
          case SL_R:
            a.in0 = P;
            a.out = P;
            break;
          case SL_A_FIRST:
          case SL_A_MID:
          case SL_A_LAST:
          case SL_A_ONLY:
            // the sparse iterate (laid out for this slot's plan) and F_eta X+ into P
            a.in1 = P;
            a.flags = (k == SL_A_FIRST || k == SL_A_ONLY ? 1 : 0) | (k == SL_A_LAST || k == SL_A_ONLY ? 2 : 0);
            a.out = (k == SL_A_LAST || k == SL_A_ONLY) ? xo : P;
            set_sparse(op, a, Xd, c.ws + b->ws_off[si] + 3 * b->blk[si], sl.kt);
            break;
        }
        std::memcpy(h + sl.args + q * sizeof(ColArgs), &a, sizeof a);
      }
      start[g.scenes.size()] = acc;
    }
  }
  CheckArg* ck = (CheckArg*)(h + b->check_off);
  for (size_t si = 0; si < b->ops.size(); ++si) {
    const cssar_op* op = b->ops[si];
    ck[si].x = c.x_outs ? (const float4*)c.x_outs[si] : nullptr;
    ck[si].n4 = c.x_outs ? (long long)op->na * op->nr / 2 : 0;
  }
  HIP_TRY(hipMemcpyAsync(b->dev_table, b->staging, b->table_bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(b->upload_done, s));
  b->upload_pending = true;
  return CSSAR_OK;
}

int launch_slot(cssar_batch* b, const Group& g, int k, hipStream_t s) {
  const Slot& sl = g.slot[k];
  GroupArgs ga;
  ga.args = b->dev_table + sl.args;
  ga.start = (const int*)(b->dev_table + sl.start);
  ga.count = (int)g.scenes.size();
  ga.total = sl.total;
  ga.conj = k == SL_ROW_G ? 1 : 0;  // (the row arguments of the slot carry the same)
  hipError_t e = g.row ? sl.kt->row_group(ga, sl.grid, s) : launch_col_group(sl.kt, col_mode(k), ga, sl.grid, s);
  if (e != hipSuccess) return fail(CSSAR_EHIP, "grouped launch: %s", hipGetErrorString(e));
  return CSSAR_OK;
}

// One phase of an iteration: slot k of every group of the given direction.
int launch_phase(cssar_batch* b, bool row, int k, hipStream_t s) {
  for (auto& g : b->groups)
    if (g.row == row) {
      int rc = launch_slot(b, g, k, s);
      if (rc) return rc;
    }
  return CSSAR_OK;
}

int launch_mid(cssar_batch* b, hipStream_t s, int last_slot) {
  int rc;
  if ((rc = launch_phase(b, true, SL_ROW_G, s))) return rc;   // P = F_eta G X
  if ((rc = launch_phase(b, false, SL_R, s))) return rc;      // P = F_eta (m o y - m o G X)
  if ((rc = launch_phase(b, true, SL_ROW_M, s))) return rc;   // P = F_eta M R
  return launch_phase(b, false, last_slot, s);                // X = S(X + mu M R)
}

int capture_graph(cssar_batch* b) {
  if (b->graph_exec) return CSSAR_OK;
  if (!b->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
  int rc = launch_mid(b, b->capture_stream, SL_A_MID);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->capture_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(CSSAR_EHIP, "graph capture: %s", hipGetErrorString(e));
  b->graph = g;
  e = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return fail(CSSAR_EHIP, "graph instantiation: %s", hipGetErrorString(e));
  }
  return CSSAR_OK;
}

int run_iterations(cssar_batch* b, int iters, hipStream_t s) {
  int rc;
  if ((rc = launch_phase(b, false, SL_FWD, s))) return rc;
  if ((rc = launch_phase(b, true, SL_ROW_M, s))) return rc;
  if ((rc = launch_phase(b, false, iters == 1 ? SL_A_ONLY : SL_A_FIRST, s))) return rc;
  if (iters == 1) return CSSAR_OK;
  const int mids = iters - 2;
  if (mids > 0 && b->use_graph) {
    if ((rc = capture_graph(b))) return rc;
    for (int t = 0; t < mids; ++t) HIP_TRY(hipGraphLaunch(b->graph_exec, s));
  } else {
    for (int t = 0; t < mids; ++t)
      if ((rc = launch_mid(b, s, SL_A_MID))) return rc;
  }
  return launch_mid(b, s, SL_A_LAST);
}

// --------------------------------------------------------- autotuner cache --
std::string tune_key(const cssar_batch* b, const Group& g, int tk) {
  long long px = 0;
  for (int s : g.scenes) px += (long long)b->ops[s]->na * b->ops[s]->nr;
  std::ostringstream o;
  o << "cssar-tune " << b->arch << ' ' << kTuneName[tk] << ' ' << g.n << ' ' << px << ' ' << g.scenes.size();
  return o.str();
}

std::string graph_key(const cssar_batch* b) {
  std::ostringstream o;
  o << "cssar-graph " << b->arch << ' ' << b->ops.size();
  for (auto* op : b->ops) o << ' ' << op->na << 'x' << op->nr;
  return o.str();
}

// --------------------------------------------------------- parity gate --
// Runs the pass of tune kind tk of group g with its current choice on a
// seeded input, leaving the output in every scene's P.  The update pass runs
// twice (first, then middle iteration, on two inputs), so the second reads
// the sparse iterate the first wrote; its threshold keeps about 5 % of the
// values (the inverse FFT of values uniform in [-1, 1) per part, scaled by
// 1/N_a, has per-part variance 1/(3 N_a); sigma^2 = 2/N_a keeps exp(-3)).
int gate_run(cssar_batch* b, Group& g, int tk, const CallArgs& c, hipStream_t s) {
  plan_slots(b);
  int rc = upload_tables(b, c, s);
  if (rc) return rc;
  auto fill = [&](char* p, size_t bytes, uint32_t seed) {
    hipLaunchKernelGGL(gate_fill_kernel, dim3(512), dim3(256), 0, s, (float2*)p, bytes / sizeof(float2), seed);
    return hipGetLastError();
  };
  for (int si : g.scenes) {
    char* base = c.ws + b->ws_off[si];
    const size_t blk = b->blk[si];
    HIP_TRY(fill(base + blk, blk, 1u));
    if (tk == TK_R) HIP_TRY(fill(base + 2 * blk, blk, 2u));
    if (tk == TK_A) {
      HIP_TRY(hipMemsetAsync(base, 0, blk, s));
      HIP_TRY(hipMemsetAsync(base + 3 * blk, 0, sparse_bytes_max(b->ops[si]), s));
    }
  }
  if (tk == TK_ROW) return launch_slot(b, g, SL_ROW_M, s);
  if (tk == TK_R) return launch_slot(b, g, SL_R, s);
  if ((rc = launch_slot(b, g, SL_A_FIRST, s))) return rc;
  for (int si : g.scenes) HIP_TRY(fill(c.ws + b->ws_off[si] + b->blk[si], b->blk[si], 3u));
  return launch_slot(b, g, SL_A_MID, s);
}

// The gate of every plan variant of (g, tk) that fits: relative L2 distance
// of its output from the reference plan's (g.def_variant) over the group's
// scenes, into g.gate[tk].  The reference output is kept in a blocked array
// of each scene that the pass does not use (Y; X's dense tiles for the
// residual pass, which reads Y).  Leaves the workspace clobbered.
int gate_variants(cssar_batch* b, Group& g, int tk, char* ws, hipStream_t s) {
  const Choice keep = g.ch[tk];
  std::vector<float> lam(b->ops.size());
  for (size_t i = 0; i < lam.size(); ++i) lam[i] = std::sqrt(2.0f / (float)b->ops[i]->na);
  CallArgs c;
  c.ws = ws;
  c.lambdas = lam.data();
  const size_t ref_at = tk == TK_R ? 0 : 2;  // in blocked arrays from the scene's base
  auto restore = [&](int rc) {
    g.ch[tk] = keep;
    plan_slots(b);
    return rc;
  };
  g.ch[tk] = Choice{g.def_variant[tk], 0};
  int rc = gate_run(b, g, tk, c, s);
  if (rc) return restore(rc);
  for (int si : g.scenes) {
    char* base = ws + b->ws_off[si];
    if (hipMemcpyAsync(base + ref_at * b->blk[si], base + b->blk[si], b->blk[si], hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return restore(fail(CSSAR_EHIP, "hipMemcpyAsync failed"));
  }
  g.gate[tk][g.def_variant[tk]] = 0.0;
  std::vector<double> part(2 * kGateBlocks);
  for (int v = 0; v < kMaxVariants; ++v) {
    const KernelTable* kt = table_for(g.n, v);
    if (v == g.def_variant[tk] || !kt || !variant_fits(b, g, kt)) continue;
    g.ch[tk] = Choice{v, 0};
    if ((rc = gate_run(b, g, tk, c, s))) return restore(rc);
    double d = 0.0, r = 0.0;
    for (int si : g.scenes) {
      const char* base = ws + b->ws_off[si];
      hipLaunchKernelGGL(gate_diff_kernel, dim3(kGateBlocks), dim3(256), 0, s,
                         (const float2*)(base + b->blk[si]), (const float2*)(base + ref_at * b->blk[si]),
                         b->blk[si] / sizeof(float2), b->gate_part);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(part.data(), b->gate_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return restore(fail(CSSAR_EHIP, "parity gate: distance kernel failed"));
      for (int k = 0; k < kGateBlocks; ++k) {
        d += part[2 * k];
        r += part[2 * k + 1];
      }
    }
    // a non-finite distance fails the gate (stored as +inf)
    const double e = r > 0.0 ? std::sqrt(d / r) : (d > 0.0 ? HUGE_VAL : 0.0);
    g.gate[tk][v] = std::isfinite(e) ? e : HUGE_VAL;
  }
  return restore(CSSAR_OK);
}

// Time `reps` launches of fn (after one warm-up), in microseconds each.
template <typename F>
int time_launches(hipStream_t s, int reps, F&& fn, double* us) {
  int rc = fn();
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(CSSAR_EHIP, "hipEventCreate failed");
  }
  rc = CSSAR_OK;
  float ms = 0.f;
  if (hipEventRecord(e0, s) != hipSuccess) rc = fail(CSSAR_EHIP, "hipEventRecord failed");
  for (int r = 0; r < reps && !rc; ++r) rc = fn();
  if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = fail(CSSAR_EHIP, "hipEventRecord failed");
  if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(CSSAR_EHIP, "hipEventSynchronize failed");
  if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(CSSAR_EHIP, "hipEventElapsedTime failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *us = 1e3 * ms / reps;
  return rc;
}

}  // namespace

extern "C" {

int cssar_make_batch(cssar_op* const* ops, int count, cssar_batch** out) {
  if (!out) return fail(CSSAR_EINVAL, "out is NULL");
  if (!ops || count < 1) return fail(CSSAR_EINVAL, "need count >= 1 operators");
  for (int s = 0; s < count; ++s)
    if (!ops[s]) return fail(CSSAR_EINVAL, "operator %d is NULL", s);
  for (int s = 0; s < count; ++s)
    if (ops[s]->chain != CSSAR_CHAIN_CSA)
      return fail(CSSAR_EUNSUPPORTED, "operator %d: batching is built for the chirp-scaling chain only", s);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  for (int s = 0; s < count; ++s)
    if (ops[s]->device != dev) return fail(CSSAR_EINVAL, "operator %d was made on another device", s);
  cssar_batch* b = new cssar_batch();
  auto cleanup = [&](int code) {
    cssar_destroy_batch(b);
    return code;
  };
  b->ops.assign(ops, ops + count);
  b->device = dev;
  b->cus = ops[0]->cus;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return cleanup(fail(CSSAR_EHIP, "hipGetDeviceProperties failed"));
  b->arch = prop.gcnArchName;
  for (auto& ch : b->arch)
    if (ch == ' ') ch = '_';
  // workspace per scene: the dense tiles of the sparse iterate, P and Y
  // (blocked arrays), then the sparse iterate (sized for the largest layout
  // of the update plans the autotuner may pick)
  size_t off = 0;
  for (auto* op : b->ops) {
    const size_t blk = align256(b4_bytes(op->na, op->nr));
    b->ws_off.push_back(off);
    b->blk.push_back(blk);
    off += 3 * blk + sparse_bytes_max(op);
  }
  b->ws_bytes = off;
  // groups by line length, scenes in batch order
  std::map<int, int> rowg, colg;
  for (int s = 0; s < count; ++s) {
    for (int dir = 0; dir < 2; ++dir) {
      const bool row = dir == 0;
      const int n = row ? ops[s]->nr : ops[s]->na;
      auto& m = row ? rowg : colg;
      auto it = m.find(n);
      if (it == m.end()) {
        Group g;
        g.row = row;
        g.n = n;
        b->groups.push_back(g);
        it = m.emplace(n, (int)b->groups.size() - 1).first;
      }
      b->groups[it->second].scenes.push_back(s);
    }
  }
  // default plans: those of the single-array solver (same per-line arithmetic)
  for (auto& g : b->groups) {
    if (g.row) {
      const KernelTable* kt = table_for(g.n, row_variant(g.n));
      if (kt && variant_fits(b, g, kt)) g.ch[TK_ROW].variant = row_variant(g.n);
    } else {
      for (int tk : {(int)TK_R, (int)TK_A}) {
        const int v = column_variant(g.n, tk == TK_R ? CK_R : CK_AS);
        const KernelTable* kt = table_for(g.n, v);
        if (kt && variant_fits(b, g, kt)) g.ch[tk].variant = v;
      }
    }
    for (int tk = 0; tk < TK_COUNT; ++tk) {
      g.def_variant[tk] = g.ch[tk].variant;
      g.gate[tk][g.ch[tk].variant] = 0.0;
    }
  }
  // table block layout: per used slot, the argument array and the prefix sums
  size_t tb = 0;
  for (auto& g : b->groups) {
    const size_t asz = g.row ? sizeof(RowArgs) : sizeof(ColArgs);
    for (int k = 0; k < SL_COUNT; ++k) {
      if (!slot_used(g, k)) continue;
      g.slot[k].args = tb;
      tb = align256(tb + asz * g.scenes.size());
      g.slot[k].start = tb;
      tb = align256(tb + sizeof(int) * (g.scenes.size() + 1));
    }
  }
  b->check_off = tb;
  tb = align256(tb + sizeof(CheckArg) * count);
  b->table_bytes = tb;
  if (hipMalloc(&b->dev_table, tb) != hipSuccess) return cleanup(fail(CSSAR_ENOMEM, "hipMalloc of %zu bytes failed", tb));
  if (hipMalloc(&b->status, sizeof(unsigned) * count) != hipSuccess ||
      hipMalloc(&b->gate_part, sizeof(double) * 2 * kGateBlocks) != hipSuccess)
    return cleanup(fail(CSSAR_ENOMEM, "hipMalloc of the status words failed"));
  if (hipMemset(b->status, 0, sizeof(unsigned) * count) != hipSuccess)
    return cleanup(fail(CSSAR_EHIP, "hipMemset failed"));
  if (hipHostMalloc(&b->staging, tb, hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(CSSAR_ENOMEM, "hipHostMalloc of %zu bytes failed", tb));
  std::memset(b->staging, 0, tb);
  if (hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(CSSAR_EHIP, "hipEventCreate failed"));
  plan_slots(b);
  *out = b;
  return CSSAR_OK;
}

int cssar_destroy_batch(cssar_batch* b) {
  if (!b) return CSSAR_OK;
  if (b->upload_pending) (void)hipEventSynchronize(b->upload_done);
  drop_graph(b);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  if (b->upload_done) (void)hipEventDestroy(b->upload_done);
  if (b->dev_table) (void)hipFree(b->dev_table);
  if (b->status) (void)hipFree(b->status);
  if (b->gate_part) (void)hipFree(b->gate_part);
  if (b->staging) (void)hipHostFree(b->staging);
  delete b;
  return CSSAR_OK;
}

size_t cssar_batch_workspace_size(const cssar_batch* b) { return b ? b->ws_bytes : 0; }

int cssar_batch_set_graph(cssar_batch* b, int on) {
  if (!b) return fail(CSSAR_EINVAL, "batch is NULL");
  b->use_graph = on != 0;
  return CSSAR_OK;
}

int cssar_batch_describe(const cssar_batch* b, char* buf, int len) {
  if (!b) return fail(CSSAR_EINVAL, "batch is NULL");
  std::ostringstream o;
  for (const auto& g : b->groups) {
    for (int tk = 0; tk < TK_COUNT; ++tk) {
      if (g.row != (tk == TK_ROW)) continue;
      const Slot& sl = g.slot[tk == TK_ROW ? SL_ROW_M : (tk == TK_R ? SL_R : SL_A_MID)];
      o << kTuneName[tk] << " n=" << g.n << " scenes=" << g.scenes.size() << " variant=" << g.ch[tk].variant
        << " E=" << sl.kt->E << " " << (g.row ? "rows/wg=" : "cols/wg=") << (g.row ? sl.kt->LR : sl.kt->C)
        << " per_cu=" << g.ch[tk].per_cu << " grid=" << sl.grid << " units=" << sl.total << " gate=";
      // per plan variant: relative L2 distance from the reference plan's
      // output ("-": not measured; the reference itself is 0)
      for (int v = 0; v < kMaxVariants; ++v) {
        if (!table_for(g.n, v)) continue;
        char e[32];
        if (g.gate[tk][v] < 0.0) std::snprintf(e, sizeof e, "%s%d:-", v ? "," : "", v);
        else std::snprintf(e, sizeof e, "%s%d:%.2e", v ? "," : "", v, g.gate[tk][v]);
        o << e;
      }
      o << "\n";
    }
  }
  o << "graph=" << (b->use_graph ? 1 : 0) << "\n";
  const std::string t = o.str();
  if (buf && len > 0) {
    const size_t n = std::min((size_t)(len - 1), t.size());
    std::memcpy(buf, t.data(), n);
    buf[n] = '\0';
  }
  return (int)t.size();
}

int cssar_ita_solve_batched(cssar_batch* b, const void* const* ys, const void* const* mask_bits,
                            const float* lambdas, int iters, void* const* x_outs, void* ws, void* stream) {
  const TraceRange tr("cssar_ita_solve_batched");
  if (!b) return fail(CSSAR_EINVAL, "batch is NULL");
  if (!ys || !mask_bits || !lambdas || !x_outs || !ws) return fail(CSSAR_EINVAL, "NULL argument");
  if (iters < 1) return fail(CSSAR_EINVAL, "iters must be >= 1");
  const char* w0 = (const char*)ws;
  const char* w1 = w0 + b->ws_bytes;
  auto in_ws = [&](const void* p) { return (const char*)p >= w0 && (const char*)p < w1; };
  for (size_t s = 0; s < b->ops.size(); ++s) {
    if (!ys[s] || !mask_bits[s] || !x_outs[s]) return fail(CSSAR_EINVAL, "NULL array for scene %zu", s);
    if (!(lambdas[s] >= 0.0f) || !std::isfinite(lambdas[s]))
      return fail(CSSAR_EINVAL, "lambda of scene %zu must be finite and >= 0", s);
    if (x_outs[s] == ys[s] || in_ws(x_outs[s]) || in_ws(ys[s]))
      return fail(CSSAR_EINVAL, "scene %zu: x_out, y and ws must not alias", s);
  }
  hipStream_t s = (hipStream_t)stream;
  CallArgs c;
  c.ys = ys;
  c.masks = mask_bits;
  c.lambdas = lambdas;
  c.x_outs = x_outs;
  c.ws = (char*)ws;
  int rc = upload_tables(b, c, s);
  if (rc) return rc;
  if ((rc = run_iterations(b, iters, s))) return rc;
  // the non-finite check of every X^(iters) (read once per call)
  hipLaunchKernelGGL(finite_check_kernel, dim3(64, (unsigned)b->ops.size()), dim3(256), 0, s,
                     (const CheckArg*)(b->dev_table + b->check_off), b->status);
  HIP_TRY(hipGetLastError());
  return CSSAR_OK;
}

int cssar_batch_sync_status(cssar_batch* b, void* stream, int* scene) {
  if (scene) *scene = -1;
  if (!b) return fail(CSSAR_EINVAL, "batch is NULL");
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  std::vector<unsigned> st(b->ops.size());
  HIP_TRY(hipMemcpy(st.data(), b->status, sizeof(unsigned) * st.size(), hipMemcpyDeviceToHost));
  int first = -1, bad = 0;
  for (size_t i = 0; i < st.size(); ++i)
    if (st[i]) {
      if (first < 0) first = (int)i;
      ++bad;
    }
  if (first < 0) return CSSAR_OK;
  HIP_TRY(hipMemset(b->status, 0, sizeof(unsigned) * st.size()));
  if (scene) *scene = first;
  return fail(CSSAR_ENONFINITE, "non-finite image in %d scene(s), the first is scene %d", bad, first);
}

int cssar_batch_autotune(cssar_batch* b, void* ws, const char* cache_path, void* stream) {
  const TraceRange tr("cssar_batch_autotune");
  if (!b) return fail(CSSAR_EINVAL, "batch is NULL");
  if (!ws) return fail(CSSAR_EINVAL, "workspace is NULL");
  hipStream_t s = (hipStream_t)stream;
  std::map<std::string, std::string> cache;  // key -> value
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t bar = line.find(" = ");
      if (bar != std::string::npos) cache[line.substr(0, bar)] = line.substr(bar + 3);
    }
  }
  std::vector<std::string> fresh;
  drop_graph(b);
  CallArgs c;
  c.ws = (char*)ws;
  const int reps = 3;
  for (auto& g : b->groups) {
    for (int tk = 0; tk < TK_COUNT; ++tk) {
      if (g.row != (tk == TK_ROW)) continue;
      const int slot = tk == TK_ROW ? SL_ROW_M : (tk == TK_R ? SL_R : SL_A_MID);
      // every variant is checked against the reference plan first (also
      // when the choice comes from the cache); one outside the gate is
      // never taken
      int rc = gate_variants(b, g, tk, (char*)ws, s);
      if (rc) return rc;
      auto gated = [&](int v) { return g.gate[tk][v] >= 0.0 && g.gate[tk][v] <= kGateTol; };
      // timing runs on a zeroed workspace (an empty iterate)
      HIP_TRY(hipMemsetAsync(ws, 0, b->ws_bytes, s));
      const std::string key = tune_key(b, g, tk);
      auto it = cache.find(key);
      if (it != cache.end()) {
        int v = 0, pc = 0;
        if (std::sscanf(it->second.c_str(), "%d %d", &v, &pc) == 2 && v >= 0 && v < kMaxVariants &&
            table_for(g.n, v) && variant_fits(b, g, table_for(g.n, v)) && gated(v)) {
          g.ch[tk].variant = v;
          g.ch[tk].per_cu = pc;
          continue;
        }
      }
      double best = 1e30;
      Choice bestc;
      bestc.variant = g.def_variant[tk];
      for (int v = 0; v < kMaxVariants; ++v) {
        const KernelTable* kt = table_for(g.n, v);
        if (!kt || !variant_fits(b, g, kt) || !gated(v)) continue;
        const void* fn = g.row ? kt->row_group_fn : col_group_fn(kt, col_mode(slot));
        const int occ = occupancy(fn, g.row ? kt->RT : kt->CT);
        for (int pc = 1; pc <= occ; ++pc) {
          g.ch[tk].variant = v;
          g.ch[tk].per_cu = pc;
          plan_slots(b);
          rc = upload_tables(b, c, s);
          if (rc) return rc;
          double us = 0;
          rc = time_launches(s, reps, [&] { return launch_slot(b, g, slot, s); }, &us);
          if (rc) return rc;
          if (us < best) {
            best = us;
            bestc = g.ch[tk];
          }
        }
      }
      g.ch[tk] = bestc;
      char val[64];
      std::snprintf(val, sizeof val, "%d %d %.1f", bestc.variant, bestc.per_cu, best);
      fresh.push_back(key + " = " + val);
    }
  }
  plan_slots(b);
  int rc = upload_tables(b, c, s);
  if (rc) return rc;
  // graph replay versus direct launches of the middle iteration
  const std::string gk = graph_key(b);
  auto it = cache.find(gk);
  if (it != cache.end() && (it->second[0] == '0' || it->second[0] == '1')) {
    b->use_graph = it->second[0] == '1';
  } else {
    double direct = 0, graphed = 0;
    rc = time_launches(s, 5, [&] { return launch_mid(b, s, SL_A_MID); }, &direct);
    if (rc) return rc;
    rc = capture_graph(b);
    if (rc) return rc;
    rc = time_launches(s, 5, [&]() -> int {
      HIP_TRY(hipGraphLaunch(b->graph_exec, s));
      return CSSAR_OK;
    }, &graphed);
    if (rc) return rc;
    b->use_graph = graphed < direct;
    char val[96];
    std::snprintf(val, sizeof val, "%d %.1f %.1f", b->use_graph ? 1 : 0, graphed, direct);
    fresh.push_back(gk + " = " + val);
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (cache_path && !fresh.empty()) {
    std::ofstream o(cache_path, std::ios::app);
    for (auto& l : fresh) o << l << "\n";
  }
  return CSSAR_OK;
}

}  // extern "C"
