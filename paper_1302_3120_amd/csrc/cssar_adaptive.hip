// The iteration of eq. (th2d) with both parameters set per iteration as
// Section IV.B suggests:
//
//   mu_i     = ||dX_G||^2 / ||m o G(dX_G)||^2   (the normalized step of the
//              cited iterative hard thresholding; the printed ratio is
//              inverted), dX_G = dX on the support of the iterate,
//              mu_i = 1 when the support is empty;
//   lambda_i = |X + mu_i dX|_{k+1} / mu_i       (so the threshold lambda_i mu_i
//              is the (k+1)-th largest magnitude of V = X + mu_i dX).
//
// Per iteration (after the first) the passes are: the row pass of G on F X,
// the residual column pass, the row pass of M (as in the fixed-parameter
// solver), then
//   D: dX on the support -> ||dX_G||^2 and F dX_G;  row pass of G on it;
//   N: ||m o G dX_G||^2 -> mu_i (device memory);
//   V: V = X + mu_i dX (spatial);
//   the selection of the (k+1)-th largest |V|^2: three histogram levels over
//   V (11, 11 and 10 bits of the FP32 bit pattern, which orders non-negative
//   floats as their values; the first counted by the V pass itself, the
//   others by passes over V), each followed by a one-workgroup pass that
//   finds the bucket holding the rank;
//   T: X+ = S_sigma(V), the support bits of X+, F X+.
// Nothing returns to the host between iterations.
#include <algorithm>
#include <cmath>

#include "cssar_internal.hpp"

using namespace cssar;
using namespace cssar::detail;

namespace cssar {
namespace detail {

constexpr int kSelectThreads = 256;
constexpr int kFindThreads = 1024;  // two histogram bins per thread

// Bits of |V|^2 resolved by selection level 0, 1, 2 (most significant first).
__device__ __forceinline__ unsigned level_bin(unsigned key, int level) {
  return level == 0 ? key >> 21 : level == 1 ? (key >> 10) & 2047u : key & 1023u;
}
__device__ __forceinline__ unsigned level_prefix(unsigned key, int level) {
  return level == 1 ? key >> 21 : key >> 10;  // bits fixed by the earlier levels
}

// Histogram of the keys |V|^2 (FP32 bits; V in the blocked layout, pads
// skipped) at one level, over the keys that match the prefix found so far.
__global__ __launch_bounds__(kSelectThreads) void select_hist_kernel(const float4* __restrict__ v, int na,
                                                                     int nr, AdaptState* st, int level,
                                                                     const unsigned* gate) {
  if (gate && *gate == 0u) return;  // (uniform over the grid)
  __shared__ unsigned h[2048];
  for (int i = threadIdx.x; i < 2048; i += kSelectThreads) h[i] = 0u;
  __syncthreads();
  if (st->done) return;  // fewer than k + 1 keys: nothing to select
  const unsigned prefix = st->prefix;
  if (level > 0 && st->use_cand) {
    // every key of the selected first-level bin is among the candidates
    const unsigned nseg = st->nseg, seg = st->seg;
    const unsigned* cnt = adapt_cand_counts(st);
    const unsigned* cand = adapt_candidates(st);
    for (unsigned g = blockIdx.x; g < nseg; g += gridDim.x) {
      const unsigned n = cnt[g];  // (at most seg: use_cand)
      for (unsigned q = threadIdx.x; q < n; q += kSelectThreads) {
        const unsigned k0 = cand[(size_t)g * seg + q];
        if (level_prefix(k0, level) == prefix) atomicAdd(&h[level_bin(k0, level)], 1u);
      }
    }
  } else {
    const unsigned per_row = 2u * (unsigned)nr;    // float4 (two elements) per block row
    const unsigned stride = b4_stride(nr) / 16u;   // block-row stride in float4
    const unsigned total = (unsigned)(na / 4) * per_row;
    for (unsigned q = blockIdx.x * kSelectThreads + threadIdx.x; q < total; q += gridDim.x * kSelectThreads) {
      const unsigned row = q / per_row;
      const float4 p = v[row * stride + (q - row * per_row)];
      const unsigned k0 = __float_as_uint(fmaf(p.x, p.x, p.y * p.y));
      const unsigned k1 = __float_as_uint(fmaf(p.z, p.z, p.w * p.w));
      if (level == 0 || level_prefix(k0, level) == prefix) atomicAdd(&h[level_bin(k0, level)], 1u);
      if (level == 0 || level_prefix(k1, level) == prefix) atomicAdd(&h[level_bin(k1, level)], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2048; i += kSelectThreads)
    if (h[i]) atomicAdd(&st->hist[i], h[i]);
}

// One workgroup: the bucket of this level that holds the rank-th largest
// key (counting from the top bucket down), the rank left inside it, and the
// histogram cleared for the next level.  After the last level the key is
// sigma^2; sigma, lambda = sigma / mu (into lambda_out if not NULL) and the
// selection state for the next iteration follow.
__global__ __launch_bounds__(kFindThreads) void select_find_kernel(AdaptState* st, int level,
                                                                   float* lambda_out, const unsigned* gate) {
  if (gate && *gate == 0u) return;
  __shared__ unsigned suf[kFindThreads];
  const int t = threadIdx.x;
  const unsigned h0 = st->hist[2 * t], h1 = st->hist[2 * t + 1];
  st->hist[2 * t] = 0u;
  st->hist[2 * t + 1] = 0u;
  const bool done = st->done != 0u;
  const unsigned rank = st->rank;
  // suffix sums over the threads: suf[t] = keys in bins >= 2 t
  suf[t] = h0 + h1;
  __syncthreads();
  for (int off = 1; off < kFindThreads; off <<= 1) {
    const unsigned add = t + off < kFindThreads ? suf[t + off] : 0u;
    __syncthreads();
    suf[t] += add;
    __syncthreads();
  }
  const unsigned above = suf[t] - h0 - h1;  // keys in bins > 2 t + 1
  unsigned bin = 0xFFFFFFFFu, left = 0u;
  if (!done) {
    if (above < rank && above + h1 >= rank) {
      bin = 2u * t + 1u;
      left = rank - above;
    } else if (above + h1 < rank && above + h1 + h0 >= rank) {
      bin = 2u * t;
      left = rank - above - h1;
    }
  }
  const bool too_few = level == 0 && suf[0] < rank;  // (uniform)
  // level 0: whether some workgroup of the value pass had more candidates
  // than its segment holds
  bool over = false;
  if (level == 0) {
    const unsigned nseg = st->nseg, seg = st->seg;
    const unsigned* cnt = adapt_cand_counts(st);
    bool mine = nseg == 0u;
    for (unsigned g = t; g < nseg; g += kFindThreads) mine = mine || cnt[g] > seg;
    over = __syncthreads_or(mine) != 0;
  }
  if (t == 0 && too_few && !done) {
    st->done = 1u;
    st->sigma2 = 0.0f;
    st->sigma = 0.0f;
  }
  if (bin != 0xFFFFFFFFu) {
    if (level == 0) {
      // the candidates hold the selected bin's keys when it lies in the
      // window they were taken from and none was dropped; the next value
      // pass takes the bins next to this one
      st->use_cand = (bin >= st->wlo && bin <= st->whi && !over) ? 1u : 0u;
      st->wlo = bin > 0u ? bin - 1u : 0u;
      st->whi = bin < 2047u ? bin + 1u : 2047u;
    }
    if (level < 2) {
      st->prefix = level == 0 ? bin : (st->prefix << 11) | bin;
      st->rank = left;
    } else {
      const float s2 = __uint_as_float((st->prefix << 10) | bin);
      const float sg = sqrtf(s2);
      st->sigma2 = s2;
      st->sigma = sg;
      if (lambda_out) lambda_out[0] = sg / st->mu;
    }
  }
  if (level == 2) {
    __syncthreads();  // (the thread that found the bin has read the prefix)
    if (t == 0) {
      if (done && lambda_out) lambda_out[0] = 0.0f;  // threshold 0
      st->prefix = 0u;
      st->rank = st->k1;
      st->done = 0u;
      st->use_cand = 0u;
    }
  }
}

// Selection state at the start of a solve: mu_0 = 1 (the support of X(0) = 0
// is empty), histogram cleared, rank k + 1; the safeguard's constants.
__global__ void adapt_init_kernel(AdaptState* st, unsigned k1, float* mu0, double c, double shrink,
                                  unsigned nseg, unsigned seg) {
  for (int i = threadIdx.x; i < 2048; i += blockDim.x) st->hist[i] = 0u;
  if (threadIdx.x == 0) {
    st->prefix = 0u;
    st->rank = k1;
    st->k1 = k1;
    st->done = 0u;
    st->mu = 1.0f;
    st->sigma = 0.0f;
    st->sigma2 = 0.0f;
    st->num = 0.0;
    st->dnum = 0.0;
    st->c = c;
    st->shrink = shrink;
    st->active = 0u;
    st->changed = 0u;
    st->shrinks = 0u;
    st->wlo = 1u;  // an empty window: the first selection reads V
    st->whi = 0u;
    st->nseg = nseg;
    st->seg = seg;
    st->use_cand = 0u;
    if (mu0) mu0[0] = 1.0f;
  }
}

// What the one-block kernel after a pass does with the pass's total.
enum AdaptTotal { AT_NUM = 0, AT_CHANGE, AT_STEP, AT_BOUND, AT_DNUM };

// Totals of the passes of the adaptive iteration from their per-block
// partials (summed in the order of the last-block reductions; bit 0 of
// status if not finite), and what follows from them:
//   AT_NUM    (pass D): ||dX_G||^2 into num;
//   AT_CHANGE (pass T, safeguard, no partials): the shrink loop goes on
//             after a support change;
//   AT_DNUM   (the difference pass, safeguard): ||F_eta (X+ - X)||^2 into dnum;
//   AT_STEP   (pass N): the step of Section IV.B (eq. (mure) read as the
//             normalized step) mu = ||dX_G||^2 / ||m o G dX_G||^2, and mu = 1
//             when either is 0 (empty support: the same ratio over the whole
//             image is 1 because G M = I and M is unitary);
//   AT_BOUND  (pass N, safeguard): omega = (1 - c) ||X+ - X||^2 /
//             ||m o G(X+ - X)||^2 (no bound when the denominator is 0); a
//             step above it shrinks by 1 / (kappa (1 - c)) and the loop goes on.
__global__ __launch_bounds__(256) void adapt_total_kernel(const float* __restrict__ part, int nblocks,
                                                          AdaptState* st, int which, unsigned* status,
                                                          const unsigned* gate, double inv_na,
                                                          float* mu_out, int* count_out) {
  if (gate && *gate == 0u) return;
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += 256) acc += (double)part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double t = sh[0];
    if (!isfinite(t)) atomicOr(status, 1u);
    if (which == AT_NUM) {
      st->num = t;
    } else if (which == AT_CHANGE) {
      st->active = st->changed ? 1u : 0u;
      st->changed = 0u;
    } else if (which == AT_DNUM) {
      st->dnum = t;
    } else if (which == AT_STEP) {
      const double num = st->num;
      const double mu = (num == 0.0 || !(t > 0.0)) ? 1.0 : num / t;
      st->mu = (float)mu;
      st->shrinks = 0u;
      if (mu_out) mu_out[0] = (float)mu;
    } else {
      const double mu = (double)st->mu;
      const double dn = st->dnum * inv_na;  // ||X+ - X||^2 (Parseval)
      const bool shrink = t > 0.0 && mu > (1.0 - st->c) * dn / t;
      if (shrink) {
        const float m2 = (float)(mu * st->shrink);
        st->mu = m2;
        st->shrinks += 1u;
        if (mu_out) mu_out[0] = m2;
        if (count_out) count_out[0] = (int)st->shrinks;
      }
      st->active = shrink ? 1u : 0u;
    }
  }
}

// The total of nblocks partials (the pass ck's grid when nblocks < 0).
int adapt_total(cssar_op* op, int ck, int which, AdaptState* st, const unsigned* gate, float* mu_out,
                int* count_out, hipStream_t s, int nblocks = -1) {
  hipLaunchKernelGGL(adapt_total_kernel, dim3(1), dim3(256), 0, s, (const float*)op->partials,
                     nblocks < 0 ? op->grid_col[ck] : nblocks, st, which, op->counter + 1, gate, 1.0 / op->na,
                     mu_out, count_out);
  HIP_TRY(hipGetLastError());
  return CSSAR_OK;
}

// Safeguard, after a support change: D = F_eta X+ - F_eta X (blocked
// layout, pads skipped; X = 0 with zero_x) and per-block partials of
// ||D||^2 (one plain store per block, totalled by the one-block kernel).
constexpr int kDiffThreads = 256;
__global__ __launch_bounds__(kDiffThreads) void diff_norm_kernel(const float4* __restrict__ xn,
                                                                 const float4* __restrict__ x, float4* d,
                                                                 int na, int nr, int zero_x, float* partials,
                                                                 const unsigned* gate) {
  if (gate && *gate == 0u) return;  // (uniform over the grid)
  __shared__ float red[kDiffThreads / 64];
  const unsigned per_row = 2u * (unsigned)nr;    // float4 (two elements) per block row
  const unsigned stride = b4_stride(nr) / 16u;   // block-row stride in float4
  const unsigned total = (unsigned)(na / 4) * per_row;
  float acc = 0.f;
  for (unsigned q = blockIdx.x * kDiffThreads + threadIdx.x; q < total; q += gridDim.x * kDiffThreads) {
    const unsigned row = q / per_row;
    const size_t i = (size_t)row * stride + (q - row * per_row);
    float4 v = xn[i];
    if (!zero_x) {
      const float4 u = x[i];
      v = make_float4(v.x - u.x, v.y - u.y, v.z - u.z, v.w - u.w);
    }
    d[i] = v;
    acc = fmaf(v.x, v.x, fmaf(v.y, v.y, fmaf(v.z, v.z, fmaf(v.w, v.w, acc))));
  }
  const float part = block_sum<kDiffThreads>(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = part;
}

// Zero n 32-bit words (a kernel rather than a memset node, so the solve can
// be captured in a graph).
__global__ void zero_words_kernel(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Bytes of the support bits of the adaptive column passes (one word per
// thread and column tile).
size_t support_bytes(const cssar_op* op) {
  const KernelTable* kt = op->kcol[CK_T];
  return (size_t)(op->nr / kt->C) * kt->CT * sizeof(uint32_t);
}

int select_threshold(cssar_op* op, const float2* V, AdaptState* st, float* lambda_out, hipStream_t s,
                     const unsigned* gate = nullptr) {
  const int grid = std::max(1, std::min(op->cus * 4, (op->na / 4) * op->nr / 2 / kSelectThreads + 1));
  return timed(op, 15, s, [&] {
    for (int level = 0; level < 3; ++level) {
      // (the value pass that wrote V has counted level 0)
      if (level > 0)
        hipLaunchKernelGGL(select_hist_kernel, dim3(grid), dim3(kSelectThreads), 0, s, (const float4*)V,
                           op->na, op->nr, st, level, gate);
      hipLaunchKernelGGL(select_find_kernel, dim3(1), dim3(kFindThreads), 0, s, st, level,
                         level == 2 ? lambda_out : nullptr, gate);
    }
    return hipGetLastError();
  });
}

}  // namespace detail
}  // namespace cssar

extern "C" {

int cssar_ita_solve_adaptive(cssar_op* op, const void* y, const void* mask_bits, long k, int iters,
                             void* x_out, float* mu_hist, float* lambda_hist, float* resid_hist, void* ws,
                             void* stream) {
  const TraceRange tr("cssar_ita_solve_adaptive");
  int rc = check_op(op);
  if (rc) return rc;
  if (!y || !mask_bits || !x_out || !ws) return fail(CSSAR_EINVAL, "NULL array");
  if (iters < 1) return fail(CSSAR_EINVAL, "iters must be >= 1");
  if (k < 0) return fail(CSSAR_EINVAL, "k must be >= 0");
  if (x_out == y || x_out == ws || ws == y) return fail(CSSAR_EINVAL, "x_out, y and ws must not alias");
  const long n = (long)op->na * op->nr;
  const unsigned k1 = (unsigned)std::min(k, n) + 1u;  // ranks beyond n select nothing
  hipStream_t s = (hipStream_t)stream;
  const size_t blk = align256(b4_bytes(op->na, op->nr));
  char* w = (char*)ws;
  float2* X = (float2*)w;             // F_eta X (blocked layout)
  float2* P = (float2*)(w + blk);     // pass buffer; V in place of F_eta dX
  float2* Y = (float2*)(w + 2 * blk); // m o y (blocked layout, unsampled marked)
  float2* Q = (float2*)(w + 3 * blk); // F_eta dX_G, then F_eta G dX_G
  uint32_t* supp = (uint32_t*)(w + 4 * blk);
  AdaptState* st = (AdaptState*)(w + 4 * blk + align256(support_bytes(op)));
  hipLaunchKernelGGL(adapt_init_kernel, dim3(1), dim3(256), 0, s, st, k1, mu_hist, 0.0, 1.0,
                     candidate_segments(op), candidate_segment_keys(op));
  HIP_TRY(hipGetLastError());
  ColArgs a = col_args(op);
  a.y = Y;
  a.mask = (const uint32_t*)mask_bits;
  a.ad = st;
  a.supp = supp;
  for (int t = 0; t < iters; ++t) {
    const bool last = t == iters - 1;
    a.hist_out = resid_hist ? resid_hist + t : nullptr;
    if (t == 0) {
      ColArgs f = a;  // R(0) = m o y: P = F_eta R, keep m o y
      f.in0 = (const float2*)y;
      f.out = P;
      f.out2 = Y;
      f.flags = 1 | 4;
      if ((rc = launch_col(op, CK_FWD, f, s))) return rc;
      if ((rc = residual_total(op, CK_FWD, f, true, s))) return rc;
    } else {
      if ((rc = launch_row(op, row_args(op, X, P, 1), s))) return rc;
      ColArgs r = a;
      r.in0 = P;
      r.out = P;
      if ((rc = launch_col(op, CK_R, r, s))) return rc;
      if ((rc = residual_total(op, CK_R, r, t == iters - 1, s))) return rc;  // ||R||^2, non-finite check
    }
    if ((rc = launch_row(op, row_args(op, P, P, 0), s))) return rc;  // P = F_eta dX
    if (t > 0) {
      ColArgs d = a;  // Q = F_eta dX_G, ||dX_G||^2
      d.in0 = P;
      d.out = Q;
      d.hist_out = nullptr;
      if ((rc = launch_col(op, CK_D, d, s))) return rc;
      if ((rc = adapt_total(op, CK_D, AT_NUM, st, nullptr, nullptr, nullptr, s))) return rc;
      if ((rc = launch_row(op, row_args(op, Q, Q, 1), s))) return rc;
      ColArgs m = a;  // mu = ||dX_G||^2 / ||m o G dX_G||^2
      m.in0 = Q;
      m.hist_out = nullptr;
      if ((rc = launch_col(op, CK_N, m, s))) return rc;
      if ((rc = adapt_total(op, CK_N, AT_STEP, st, nullptr, mu_hist ? mu_hist + t : nullptr, nullptr, s)))
        return rc;
    }
    ColArgs v = a;  // V = X + mu dX (spatial, into P)
    v.in0 = X;
    v.in1 = P;
    v.out = P;
    v.flags = t == 0 ? 1 : 0;
    v.hist_out = nullptr;
    if ((rc = launch_col(op, CK_V, v, s))) return rc;
    if ((rc = select_threshold(op, P, st, lambda_hist ? lambda_hist + t : nullptr, s))) return rc;
    ColArgs x = a;  // X+ = S_sigma(V), support bits, F_eta X+ (or X+ at the end)
    x.in0 = P;
    x.out = last ? (float2*)x_out : X;
    x.flags = last ? 2 : 0;
    x.hist_out = nullptr;
    if ((rc = launch_col(op, CK_T, x, s))) return rc;
  }
  return CSSAR_OK;
}

int cssar_ita_solve_safeguarded(cssar_op* op, const void* y, const void* mask_bits, long k, int iters,
                                double c, double kappa, int max_shrinks, void* x_out, float* mu_hist,
                                float* lambda_hist, float* resid_hist, int* shrink_hist, void* ws,
                                void* stream) {
  const TraceRange tr("cssar_ita_solve_safeguarded");
  int rc = check_op(op);
  if (rc) return rc;
  if (!y || !mask_bits || !x_out || !ws) return fail(CSSAR_EINVAL, "NULL array");
  if (iters < 1) return fail(CSSAR_EINVAL, "iters must be >= 1");
  if (k < 0) return fail(CSSAR_EINVAL, "k must be >= 0");
  if (!(c > 0.0 && c < 1.0)) return fail(CSSAR_EINVAL, "c must lie in (0, 1)");
  if (!(kappa * (1.0 - c) > 1.0) || !std::isfinite(kappa))
    return fail(CSSAR_EINVAL, "kappa (1 - c) must exceed 1");
  if (max_shrinks < 0 || max_shrinks > CSSAR_MAX_SHRINKS)
    return fail(CSSAR_EINVAL, "max_shrinks must lie in 0..%d", CSSAR_MAX_SHRINKS);
  if (x_out == y || x_out == ws || ws == y) return fail(CSSAR_EINVAL, "x_out, y and ws must not alias");
  const long n = (long)op->na * op->nr;
  const unsigned k1 = (unsigned)std::min(k, n) + 1u;
  hipStream_t s = (hipStream_t)stream;
  const size_t blk = align256(b4_bytes(op->na, op->nr)), sb = align256(support_bytes(op));
  char* w = (char*)ws;
  float2* X = (float2*)w;              // F_eta X (blocked layout)
  float2* P = (float2*)(w + blk);      // pass buffer, then F_eta dX
  float2* Y = (float2*)(w + 2 * blk);  // m o y (blocked layout, unsampled marked)
  float2* Q = (float2*)(w + 3 * blk);  // F_eta dX_G, F_eta G dX_G, then V
  float2* Xn = (float2*)(w + 4 * blk); // F_eta X+
  float2* Df = (float2*)(w + 5 * blk); // F_eta (X+ - X), then F_eta G(X+ - X)
  uint32_t* so = (uint32_t*)(w + 6 * blk);       // support bits of X
  uint32_t* sn = (uint32_t*)(w + 6 * blk + sb);  // support bits of X+
  AdaptState* st = (AdaptState*)(w + 6 * blk + 2 * sb);
  const unsigned* active = &st->active;
  hipLaunchKernelGGL(adapt_init_kernel, dim3(1), dim3(256), 0, s, st, k1, mu_hist, c,
                     1.0 / (kappa * (1.0 - c)), candidate_segments(op), candidate_segment_keys(op));
  hipLaunchKernelGGL(zero_words_kernel, dim3(std::max<size_t>(1, std::min<size_t>(1024, sb / 1024))),
                     dim3(256), 0, s, so, sb / 4);
  if (shrink_hist)
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(256), 0, s, (uint32_t*)shrink_hist, (size_t)iters);
  HIP_TRY(hipGetLastError());
  ColArgs a = col_args(op);
  a.y = Y;
  a.mask = (const uint32_t*)mask_bits;
  a.ad = st;
  const int diff_grid =
      std::max(1, std::min(std::min(op->cus * 4, kMaxPartials), (op->na / 4) * op->nr / 2 / kDiffThreads + 1));
  for (int t = 0; t < iters; ++t) {
    a.hist_out = resid_hist ? resid_hist + t : nullptr;
    a.supp = so;  // the support of X (read by D)
    if (t == 0) {
      ColArgs f = a;  // R(0) = m o y: P = F_eta R, keep m o y
      f.in0 = (const float2*)y;
      f.out = P;
      f.out2 = Y;
      f.flags = 1 | 4;
      if ((rc = launch_col(op, CK_FWD, f, s))) return rc;
      if ((rc = residual_total(op, CK_FWD, f, true, s))) return rc;
    } else {
      if ((rc = launch_row(op, row_args(op, X, P, 1), s))) return rc;
      ColArgs r = a;
      r.in0 = P;
      r.out = P;
      if ((rc = launch_col(op, CK_R, r, s))) return rc;
      if ((rc = residual_total(op, CK_R, r, t == iters - 1, s))) return rc;  // ||R||^2, non-finite check
    }
    if ((rc = launch_row(op, row_args(op, P, P, 0), s))) return rc;  // P = F_eta dX
    if (t > 0) {
      ColArgs d = a;  // Q = F_eta dX_G, ||dX_G||^2
      d.in0 = P;
      d.out = Q;
      d.hist_out = nullptr;
      if ((rc = launch_col(op, CK_D, d, s))) return rc;
      if ((rc = adapt_total(op, CK_D, AT_NUM, st, nullptr, nullptr, nullptr, s))) return rc;
      if ((rc = launch_row(op, row_args(op, Q, Q, 1), s))) return rc;
      ColArgs m = a;  // mu = ||dX_G||^2 / ||m o G dX_G||^2; no shrinks yet
      m.in0 = Q;
      m.hist_out = nullptr;
      if ((rc = launch_col(op, CK_N, m, s))) return rc;
      if ((rc = adapt_total(op, CK_N, AT_STEP, st, nullptr, mu_hist ? mu_hist + t : nullptr, nullptr, s)))
        return rc;
    }
    // The step, then up to max_shrinks rounds that run only while the
    // previous round moved the support and its step exceeded the bound.
    for (int round = 0; round <= max_shrinks; ++round) {
      const unsigned* gate = round ? active : nullptr;
      ColArgs v = a;  // V = X + mu dX (spatial, into Q)
      v.in0 = X;
      v.in1 = P;
      v.out = Q;
      v.flags = t == 0 ? 1 : 0;
      v.hist_out = nullptr;
      v.gate = gate;
      if ((rc = launch_col(op, CK_V, v, s))) return rc;
      if ((rc = select_threshold(op, Q, st, lambda_hist ? lambda_hist + t : nullptr, s, gate))) return rc;
      ColArgs x = a;  // X+ = S_sigma(V) -> F_eta X+; support change
      x.in0 = Q;
      x.out = Xn;
      x.supp = sn;
      x.supp_old = so;
      x.out3 = (float2*)x_out;  // the last iteration's X+ (each round overwrites it)
      x.flags = 4 | (t == iters - 1 ? 16 : 0);
      x.hist_out = nullptr;
      x.gate = gate;
      if ((rc = launch_col(op, CK_T, x, s))) return rc;
      if ((rc = adapt_total(op, CK_T, AT_CHANGE, st, gate, nullptr, nullptr, s, 0))) return rc;
      if (round == max_shrinks) break;
      // after a support change: F_eta (X+ - X) and ||X+ - X||^2 (Parseval)
      hipLaunchKernelGGL(diff_norm_kernel, dim3(diff_grid), dim3(kDiffThreads), 0, s, (const float4*)Xn,
                         (const float4*)X, (float4*)Df, op->na, op->nr, t == 0 ? 1 : 0, op->partials, active);
      HIP_TRY(hipGetLastError());
      if ((rc = adapt_total(op, CK_T, AT_DNUM, st, active, nullptr, nullptr, s, diff_grid))) return rc;
      RowArgs g = row_args(op, Df, Df, 1);  // F_eta G(X+ - X)
      g.gate = active;
      if ((rc = launch_row(op, g, s))) return rc;
      ColArgs b = a;  // the bound; shrink mu or end the loop
      b.in0 = Df;
      b.hist_out = nullptr;
      b.gate = active;
      if ((rc = launch_col(op, CK_N, b, s))) return rc;
      if ((rc = adapt_total(op, CK_N, AT_BOUND, st, active, mu_hist ? mu_hist + t : nullptr,
                            shrink_hist ? shrink_hist + t : nullptr, s)))
        return rc;
    }
    std::swap(X, Xn);
    std::swap(so, sn);
  }
  return CSSAR_OK;
}

}  // extern "C"
