// Gradient of a loss of the unrolled iterative thresholding with respect to
// the raw data y, the threshold lambda and the radar parameters K_a, K_r:
// a forward solve that keeps checkpoints of the iterate, and the reverse
// pass through the iterations (recomputing each checkpoint segment).  The
// derivative of the method's map is plain calculus on eq. (th2d) /
// Algorithm 1 with G = M^H (Theorem 1); the paper does not differentiate it.
#include <algorithm>
#include <cmath>
#include <vector>

#include "cssar_internal.hpp"

using namespace cssar;
using namespace cssar::detail;

namespace cssar {
namespace detail {

// Derivatives of the screen arguments (radians) per Doppler bin, as
// polynomials in the centred column offset o = j - N_r/2 (tau' = o / fs) for
// Phi1 and Phi3 and in the signed range bin nu for Phi2.  With
// w = lambda_w f / (2 v), D = sqrt(1 - w^2), Km = Kr / (1 - Kr z),
// z = c r_ref f^2 / (2 v^2 fc^3 D^3), e = 1/D - 1, d1 = 2 r_ref e / c:
//   arg1 = pi Km e (tau' - d1)^2
//   arg2 = pi (D / Km) (nu df)^2 + 4 pi r_ref e (nu df) / c
//   arg3 = 4 pi fc r_ref D / c + 2 pi fc D tau' - pi Km h tau'^2,  h = (1 - D) / D^2
// differentiated in v (then times dv/dK_a = lambda_w r_ref / (4 v), since
// K_a = 2 v^2 / (lambda_w r_ref)) and in K_r.
void build_derivatives(const cssar_params& p, int na, int nr, std::vector<float>& out) {
  const double lam = kC / p.fc;
  const double fs = p.fs, df = p.fs / nr, pi = M_PI;
  const double dv_dka = lam * p.r_ref / (4.0 * p.v);
  out.assign((size_t)na * 18, 0.0f);
  for (int k = 0; k < na; ++k) {
    const int nu = k < (na + 1) / 2 ? k : k - na;
    const double f = p.prf * nu / na;
    const double w = lam * f / (2.0 * p.v);
    const double D = std::sqrt(1.0 - w * w);
    const double dD_dv = w * w / (p.v * D);
    double Km = p.Kr, dKm_dv = 0.0, dKm_dKr = 1.0;
    if (p.src) {
      const double z = kC * p.r_ref * f * f / (2.0 * p.v * p.v * p.fc * p.fc * p.fc * D * D * D);
      const double den = 1.0 - p.Kr * z;
      Km = p.Kr / den;
      const double dz_dv = z * (-2.0 / p.v - 3.0 * dD_dv / D);
      dKm_dv = Km * Km * dz_dv;
      dKm_dKr = 1.0 / (den * den);
    }
    const double e = 1.0 / D - 1.0;
    const double d1 = 2.0 * p.r_ref * e / kC;
    const double h = (1.0 - D) / (D * D);
    for (int th = 0; th < 2; ++th) {
      // th 0: d/dv (scaled to K_a below); th 1: d/dK_r
      const double dD = th == 0 ? dD_dv : 0.0;
      const double dKm = th == 0 ? dKm_dv : dKm_dKr;
      const double de = -dD / (D * D);
      const double dd1 = 2.0 * p.r_ref * de / kC;
      const double dKe = dKm * e + Km * de;
      const double dDK = (dD * Km - D * dKm) / (Km * Km);
      const double dh = (D - 2.0) / (D * D * D) * dD;
      const double dKh = dKm * h + Km * dh;
      double c[9];
      c[0] = pi * (dKe * d1 * d1 + 2.0 * Km * e * d1 * dd1);
      c[1] = pi * (-2.0 * dKe * d1 - 2.0 * Km * e * dd1) / fs;
      c[2] = pi * dKe / (fs * fs);
      c[3] = 0.0;
      c[4] = 4.0 * pi * p.r_ref * df * de / kC;
      c[5] = pi * dDK * df * df;
      c[6] = 4.0 * pi * p.fc * p.r_ref * dD / kC;
      c[7] = 2.0 * pi * p.fc * dD / fs;
      c[8] = -pi * dKh / (fs * fs);
      const double sc = th == 0 ? dv_dka : 1.0;
      for (int i = 0; i < 9; ++i) out[(size_t)k * 18 + th * 9 + i] = (float)(c[i] * sc);
    }
  }
}

}  // namespace detail
}  // namespace cssar

namespace {

// out[c] += scale_c * sum over blocks of part[b * comps + c], summed in FP64
// in a fixed order (one workgroup), so the result is deterministic.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const float* __restrict__ part, int nblocks,
                                                              int comps, double* __restrict__ out, double s0,
                                                              double s1) {
  __shared__ double sh[256];
  for (int c = 0; c < comps; ++c) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += 256) acc += (double)part[i * comps + c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] += sh[0] * (c == 0 ? s0 : s1);
    __syncthreads();
  }
}

// Row-major <-> blocked layout (element (i, j) of the blocked array at
// float2 index (i/4)(4 N_r + 16) + (j/4) 16 + (i%4) 4 + j%4).
template <bool TO_B4>
__global__ void relayout_kernel(const float2* __restrict__ in, float2* __restrict__ out, int na, int nr) {
  const size_t n = (size_t)na * nr;
  const size_t sb = 4 * (size_t)nr + 16;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / nr, j = e % nr;
    const size_t q = (i >> 2) * sb + (j >> 2) * 16 + (i & 3) * 4 + (j & 3);
    if (TO_B4) out[q] = in[e];
    else out[e] = in[q];
  }
}

int reduce(const cssar_op* op, int nblocks, int comps, double* out, double s0, double s1, hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, (const float*)op->partials, nblocks, comps,
                     out, s0, s1);
  HIP_TRY(hipGetLastError());
  return CSSAR_OK;
}

template <bool TO_B4>
int relayout(const cssar_op* op, const void* in, void* out, hipStream_t s) {
  const int grid = std::max(1, std::min(op->cus * 8, (op->na * op->nr + 255) / 256));
  hipLaunchKernelGGL(relayout_kernel<TO_B4>, dim3(grid), dim3(256), 0, s, (const float2*)in, (float2*)out,
                     op->na, op->nr);
  HIP_TRY(hipGetLastError());
  return CSSAR_OK;
}

// One forward iteration t of the solver on blocked arrays: Xt (NULL at
// t = 0) -> Xn (blocked), or the row-major x_out when rm_out.  P is the pass
// buffer and Y the marked copy of m o y (written at t = 0).
int forward_iteration(cssar_op* op, int t, const float2* Xt, float2* P, float2* Y, const void* y,
                      const void* mask, float sigma, void* Xn, bool rm_out, hipStream_t s) {
  int rc;
  ColArgs a = col_args(op);
  a.y = Y;
  a.mask = (const uint32_t*)mask;
  a.sigma = sigma;
  if (t == 0) {
    ColArgs f = a;
    f.in0 = (const float2*)y;
    f.out = P;
    f.out2 = Y;
    f.flags = 1 | 4;
    if ((rc = launch_col(op, CK_FWD, f, s))) return rc;
    if ((rc = residual_total(op, CK_FWD, f, true, s))) return rc;  // (non-finite check)
  } else {
    if ((rc = launch_row(op, row_args(op, Xt, P, 1), s))) return rc;
    ColArgs r = a;
    r.in0 = P;
    r.out = P;
    if ((rc = launch_col(op, CK_R, r, s))) return rc;
    if ((rc = residual_total(op, CK_R, r, rm_out, s))) return rc;  // (last iteration: non-finite check)
  }
  if ((rc = launch_row(op, row_args(op, P, P, 0), s))) return rc;
  ColArgs u = a;
  u.in0 = Xt;
  u.in1 = P;
  u.out = (float2*)Xn;
  u.flags = (t == 0 ? 1 : 0) | (rm_out ? 2 : 0);
  return launch_col(op, CK_A, u, s);
}

int check_solve_args(const cssar_op* op, const void* y, const void* mask, float lambda, int iters, int every) {
  int rc = check_op(op);
  if (rc) return rc;
  if (op->chain != CSSAR_CHAIN_CSA)
    return fail(CSSAR_EUNSUPPORTED, "the gradient is built for the chirp-scaling chain only");
  if (!y || !mask) return fail(CSSAR_EINVAL, "NULL array");
  if (iters < 1) return fail(CSSAR_EINVAL, "iters must be >= 1");
  if (every < 1) return fail(CSSAR_EINVAL, "checkpoint interval must be >= 1");
  if (!(lambda >= 0.0f) || !std::isfinite(lambda)) return fail(CSSAR_EINVAL, "lambda must be finite and >= 0");
  return CSSAR_OK;
}

}  // namespace

extern "C" {

size_t cssar_checkpoint_size(const cssar_op* op, int iters, int every) {
  if (!op || iters < 1 || every < 1) return 0;
  return (size_t)((iters - 1) / every) * align256(b4_bytes(op->na, op->nr));
}

size_t cssar_grad_workspace_size(const cssar_op* op, int every) {
  if (!op || every < 1) return 0;
  return (size_t)(every + 4) * align256(b4_bytes(op->na, op->nr));
}

int cssar_ita_forward(cssar_op* op, const void* y, const void* mask_bits, float lambda, int iters, int every,
                      void* x_out, void* ckpt, void* ws, void* stream) {
  const TraceRange tr("cssar_ita_forward");
  int rc = check_solve_args(op, y, mask_bits, lambda, iters, every);
  if (rc) return rc;
  if (!x_out || !ws || (iters - 1 >= every && !ckpt)) return fail(CSSAR_EINVAL, "NULL array");
  if (x_out == y || x_out == ws || ws == y) return fail(CSSAR_EINVAL, "x_out, y and ws must not alias");
  hipStream_t s = (hipStream_t)stream;
  const size_t blk = align256(b4_bytes(op->na, op->nr));
  float2* X = (float2*)ws;
  float2* P = (float2*)((char*)ws + blk);
  float2* Y = (float2*)((char*)ws + 2 * blk);
  const float2* cur = nullptr;
  for (int t = 0; t < iters; ++t) {
    const int nx = t + 1;  // index of the iterate this iteration produces
    const bool last = nx == iters;
    void* dst;
    if (last) dst = x_out;
    else if (nx % every == 0) dst = (char*)ckpt + (size_t)(nx / every - 1) * blk;  // checkpoint X~(nx)
    else dst = X;
    if ((rc = forward_iteration(op, t, cur, P, Y, y, mask_bits, lambda, dst, last, s))) return rc;
    cur = (const float2*)dst;
  }
  return CSSAR_OK;
}

int cssar_ita_backward(cssar_op* op, const void* y, const void* mask_bits, float lambda, int iters, int every,
                       const void* ckpt, const void* grad_x, void* grad_y, double* grad_scalars, void* ws,
                       void* stream) {
  const TraceRange tr("cssar_ita_backward");
  int rc = check_solve_args(op, y, mask_bits, lambda, iters, every);
  if (rc) return rc;
  if (!grad_x || !grad_y || !grad_scalars || !ws || (iters - 1 >= every && !ckpt))
    return fail(CSSAR_EINVAL, "NULL array");
  if (grad_y == y || grad_y == grad_x || grad_y == ws) return fail(CSSAR_EINVAL, "grad_y must not alias");
  hipStream_t s = (hipStream_t)stream;
  const size_t blk = align256(b4_bytes(op->na, op->nr));
  char* w = (char*)ws;
  float2* P = (float2*)w;
  float2* Q = (float2*)(w + blk);
  float2* Xb = (float2*)(w + 2 * blk);   // adjoint of the iterate, then of V (spatial, blocked)
  float2* Yb = (float2*)(w + 3 * blk);   // gradient in y (spatial, blocked)
  float2* Y = (float2*)(w + 4 * blk);    // marked copy of m o y
  auto seg_x = [&](int i) { return (float2*)(w + (size_t)(4 + i) * blk); };  // i = 1 .. every-1
  const float mu = 1.0f, sigma = lambda * mu;
  const double inv_na = 1.0 / op->na;

  HIP_TRY(hipMemsetAsync(grad_scalars, 0, 3 * sizeof(double), s));
  HIP_TRY(hipMemsetAsync(Yb, 0, blk, s));
  if ((rc = relayout<true>(op, grad_x, Xb, s))) return rc;
  // marked copy of m o y (the first column pass of the solver)
  {
    ColArgs f = col_args(op);
    f.in0 = (const float2*)y;
    f.mask = (const uint32_t*)mask_bits;
    f.out = P;
    f.out2 = Y;
    f.flags = 1 | 4;
    if ((rc = launch_col(op, CK_FWD, f, s))) return rc;
  }
  const int nseg = (iters + every - 1) / every;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int s0 = seg * every, s1 = std::min(s0 + every, iters);
    const float2* xs = s0 == 0 ? nullptr : (const float2*)((const char*)ckpt + (size_t)(seg - 1) * blk);
    auto x_at = [&](int t) -> const float2* { return t == s0 ? xs : seg_x(t - s0); };
    // recompute the iterates of the segment
    for (int t = s0; t + 1 < s1; ++t)
      if ((rc = forward_iteration(op, t, x_at(t), P, Y, y, mask_bits, sigma, seg_x(t + 1 - s0), false, s)))
        return rc;
    for (int t = s1 - 1; t >= s0; --t) {
      const float2* Xt = x_at(t);
      ColArgs a = col_args(op);
      a.y = Y;
      a.mask = (const uint32_t*)mask_bits;
      a.sigma = sigma;
      a.mu = mu;
      // P = F R(t)
      if (t == 0) {
        ColArgs f = a;
        f.in0 = (const float2*)y;
        f.out = P;
        f.out2 = Y;
        f.flags = 1 | 4;
        if ((rc = launch_col(op, CK_FWD, f, s))) return rc;
      } else {
        if ((rc = launch_row(op, row_args(op, Xt, P, 1), s))) return rc;
        ColArgs r = a;
        r.in0 = P;
        r.out = P;
        if ((rc = launch_col(op, CK_R, r, s))) return rc;
      }
      // Q = F M R(t)
      if ((rc = launch_row(op, row_args(op, P, Q, 0), s))) return rc;
      // Vbar = J_S(V)^T Xbar (into Xb), Q = F (mu Vbar), lambda partials
      {
        ColArgs v = a;
        v.in0 = Xt;
        v.in1 = Q;
        v.y = Xb;
        v.out = Q;
        v.out2 = Xb;
        v.flags = t == 0 ? 1 : 0;
        if ((rc = launch_col(op, CK_VB, v, s))) return rc;
        if ((rc = reduce(op, op->grid_col[CK_VB], 1, grad_scalars, mu, 0.0, s))) return rc;
      }
      // P = F G (mu Vbar), with the M-stage parameter derivatives paired
      {
        RowArgs r = row_args(op, P, P, 0);
        r.in2 = Q;
        r.rowd = op->rowd;
        r.partials = op->partials;
        if ((rc = launch_row_adj(op, 0, r, s))) return rc;
        if ((rc = reduce(op, op->grid_adj[0], 2, grad_scalars + 1, inv_na, inv_na, s))) return rc;
      }
      // ybar += m o G(mu Vbar); P = F ubar, ubar = -m o G(mu Vbar)
      {
        ColArgs u = a;
        u.in0 = P;
        u.in1 = Yb;
        u.out2 = Yb;
        u.out = P;
        if ((rc = launch_col(op, CK_U, u, s))) return rc;
      }
      if (t > 0) {
        // P = F M ubar, with the G-stage parameter derivatives paired on X(t)
        RowArgs r = row_args(op, Xt, P, 1);
        r.in2 = P;
        r.rowd = op->rowd;
        r.partials = op->partials;
        if ((rc = launch_row_adj(op, 1, r, s))) return rc;
        if ((rc = reduce(op, op->grid_adj[1], 2, grad_scalars + 1, inv_na, inv_na, s))) return rc;
        // Xbar(t) = Vbar + M ubar
        ColArgs x = a;
        x.in0 = P;
        x.in1 = Xb;
        x.out = Xb;
        if ((rc = launch_col(op, CK_XB, x, s))) return rc;
      }
    }
  }
  return relayout<false>(op, Yb, grad_y, s);
}

}  // extern "C"
