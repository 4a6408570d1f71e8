// Fused pass kernels.  A pass reads whole lines of the N_a x N_r array,
// transforms them in registers/LDS and writes them back (in place allowed):
//
//   row pass  (line = one range line, contiguous):  F_tau -> x Phi2 (or
//             Phi2*) / N_r -> F_tau^-1.  The middle of M (resp. G).
//   col pass  (tile = C adjacent azimuth columns, stride N_r):
//     FWD<ph>: [m o y, ||.||^2]  -> F_eta -> x Phi_ph (or conj)
//     INV<ph>: x Phi_ph (or conj) / N_a -> F_eta^-1
//     A:       V = F_eta^-1[Phi3 (Xt + mu W)] / N_a -> X+ = S_sigma(V)
//              -> either X+ (last iteration) or Xt+ = Phi3* F_eta X+
//     R:       GX = F_eta^-1[Phi1* Wg] / N_a -> R = m o (y - GX), ||R||^2
//              -> Phi1 F_eta R
//
// The ITA keeps the iterate as Xt = Phi3* o F_eta X (azimuth spectrum with the
// azimuth-compression phase removed) so that every pass evaluates exactly one
// phase screen per element; see the operator schedule in cssar_api.hip.
#pragma once

#include "cssar_device.hpp"

namespace cssar {

struct RowArgs {
  const float2* in;
  float2* out;
  const double2* rowc2;  // Phi2 coefficients per Doppler bin (row)
  const float2* tw;      // w_N^k, N = N_r
  int na;
  int conj;              // 1: Phi2* (operator G)
  float scale;           // 1 / N_r
};

enum ColMode { COL_FWD = 0, COL_INV = 1, COL_A = 2, COL_R = 3 };

struct ColArgs {
  const float2* in0;     // FWD/INV: input; A: Xt (NULL on the first iteration); R: Wg
  const float2* in1;     // A: W
  const float2* y;       // R and masked FWD: raw data
  const uint32_t* mask;  // R and masked FWD: packed sampling mask
  float2* out;
  const double2* rowc;   // Phi1 or Phi3 coefficients per Doppler bin
  const double2* colc;   // (P_j, dtau_j) per range column
  const float2* tw;      // w_N^k, N = N_a
  int na, nr;
  int conj;              // FWD/INV: multiply by the conjugate screen
  int flags;             // FWD: 1 = mask the input and sum |.|^2; A: 1 = no Xt input, 2 = store X
  float scale;           // 1 / N_a (inverse transforms)
  float mu, sigma;       // A: step and threshold lambda*mu
  float* partials;       // per-block partial sums of ||R||^2
  unsigned* counter;     // last-block detection
  float* hist_out;       // where the total ||R||^2 goes (may be NULL)
  unsigned* status;      // bit 0: non-finite residual
};

// Phase of element (i, j), i = b + T k: coefficients read at byte offset
// b*16 (lane) + T*k*16 (uniform).
template <int PH>
__device__ __forceinline__ Turns col_turns(const Buf& rowc, uint32_t boff, uint32_t koff, double2 cc) {
  const double2 rc = rowc.d2(boff, koff);
  if constexpr (PH == 1)
    return reduce_turns(phi1_turns(rc, cc.y));
  else
    return reduce_turns(phi3_turns(rc, cc));
}

// Elementwise work on the E register elements in chunks of CH, with
// scheduling barriers between chunks so the compiler does not hoist every
// coefficient load and FP64 phase evaluation at once (register pressure).
template <int E, int CH, typename F>
__device__ __forceinline__ void chunked(F&& f) {
#pragma unroll
  for (int k0 = 0; k0 < E; k0 += CH) {
#pragma unroll
    for (int k = k0; k < k0 + CH; ++k) f(k);
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int N>
__global__ __launch_bounds__(Plan<N>::RT, (Plan<N>::E <= 16 ? 4 : 2)) void row_pass_kernel(RowArgs a) {
  using P = Plan<N>;
  constexpr int E = P::E, T = P::T, LR = P::LR;
  constexpr int LS = LdsSize<1, N>::value;
  __shared__ float2 lds[LR * LS];
  const int line = threadIdx.x / T;
  const int b = threadIdx.x % T;
  const uint32_t bytes = clamp_bytes((size_t)a.na * N * 8);
  const Buf in(a.in, bytes), out(a.out, bytes);
  const int groups = (a.na + LR - 1) / LR;
  for (int g = blockIdx.x; g < groups; g += gridDim.x) {
    const int row = g * LR + line;
    const bool active = row < a.na;
    const uint32_t voff = ((uint32_t)(active ? row : 0) * N + b) * 8u;
    int lb = b;
    asm volatile("" : "+v"(lb));  // recompute LDS addresses per row (register pressure)
    float2* lmy = lds + line * LS;
    asm volatile("" : "+v"(lmy));
    const float2* tw0 = a.tw;
    asm volatile("" : "+s"(tw0));
    float2 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = in.f2(voff, T * k * 8);
    if (!active) {
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = make_float2(0.f, 0.f);
    }
    fft_line<N, false, 1, 0>(v, lb, 0, lmy, tw0);
    const double2 rc = a.rowc2[active ? row : 0];
    const float sy = a.conj ? -a.scale : a.scale;
    chunked<E, 4>([&](int k) {
      const int l = b + T * k;
      const int nu = l < N / 2 ? l : l - N;
      float2 p = cis_turns(phi2_turns(rc, (double)nu));
      p = make_float2(p.x * a.scale, p.y * sy);
      v[k] = cmul(v[k], p);
    });
    const float2* tw = a.tw;
    asm volatile("" : "+s"(tw));
    asm volatile("" : "+v"(lb), "+v"(lmy));
    fft_line<N, true, 1, 0>(v, lb, 0, lmy, tw);
    if (active) {
#pragma unroll
      for (int k = 0; k < E; ++k) out.st(v[k], voff, T * k * 8);
    }
  }
}

__device__ __forceinline__ int xcd_logical_block() {
  // Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
  // that consecutive logical ids (adjacent column tiles sharing cache lines)
  // run on the same XCD and share its L2.
  const int g = gridDim.x, w = blockIdx.x;
  if (g % 8 != 0) return w;
  return (w % 8) * (g / 8) + w / 8;
}

template <int N, int MODE, int PH>
__global__ __launch_bounds__(Plan<N>::CT) void col_pass_kernel(ColArgs a) {
  using P = Plan<N>;
  constexpr int E = P::E, T = P::T, C = P::C, CT = P::CT;
  constexpr int LS = LdsSize<C, N>::value;
  __shared__ float2 lds[LS];
  __shared__ float red[CT / 64];
  const int c = threadIdx.x % C;
  const int b = threadIdx.x / C;
  const int ntiles = (a.nr + C - 1) / C;
  const uint32_t nr = (uint32_t)a.nr;
  const uint32_t bytes = clamp_bytes((size_t)N * a.nr * 8);
  const Buf in0(a.in0, bytes), in1(a.in1, bytes), yb(a.y, bytes), out(a.out, bytes);
  const Buf mask(a.mask, clamp_bytes(((size_t)N * a.nr + 31) / 32 * 4));
  const Buf rowc(a.rowc, N * 16);
  const uint32_t kbytes = T * nr * 8;       // byte stride between v[k] and v[k+1]
  const uint32_t kmask = T * nr / 32 * 4;   // same, in the packed mask (nr % 32 == 0)
  const uint32_t boff = (uint32_t)b * 16u;  // coefficient offset of row b
  float acc = 0.f;
  for (int tile = xcd_logical_block(); tile < ntiles; tile += gridDim.x) {
    const int j = tile * C + c;
    const bool active = j < a.nr;
    const int jj = active ? j : 0;
    const uint32_t lane = (uint32_t)b * nr + jj;  // element index of v[0]
    const uint32_t voff = lane * 8u;
    const double2 cc = a.colc[jj];
    // Opaque per-tile copy of the twiddle pointer: keeps the compiler from
    // hoisting every pass's twiddles out of the tile loop (register pressure).
    const float2* tw = a.tw;
    asm volatile("" : "+s"(tw));
    // Likewise for the lane's LDS coordinates: the exchange addresses are
    // recomputed per tile instead of being held across the whole loop.
    int lb = b, lc = c;
    asm volatile("" : "+v"(lb), "+v"(lc));
    float2 v[E];
    if constexpr (MODE == COL_FWD) {
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = in0.f2(voff, k * kbytes);
      if (!active) {
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = make_float2(0.f, 0.f);
      }
      if (a.flags & 1) {
        const uint32_t moff = (lane >> 5) * 4u, bit = lane & 31u;
#pragma unroll
        for (int k = 0; k < E; ++k) {
          const uint32_t w = mask.u32(moff, k * kmask);
          if (!((w >> bit) & 1u)) v[k] = make_float2(0.f, 0.f);
          acc = fmaf(v[k].x, v[k].x, fmaf(v[k].y, v[k].y, acc));
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      fft_line<N, false, C, 1>(v, lb, lc, lds, tw);
      chunked<E, 4>([&](int k) {
        Turns u = col_turns<PH>(rowc, boff, T * k * 16, cc);
        float2 p = cis_quadrant(u.r, u.q);
        v[k] = a.conj ? cmulc(v[k], p) : cmul(v[k], p);
      });
    } else if constexpr (MODE == COL_INV) {
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = in0.f2(voff, k * kbytes);
      if (!active) {
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = make_float2(0.f, 0.f);
      }
      const float sy = a.conj ? -a.scale : a.scale;
      chunked<E, 4>([&](int k) {
        Turns u = col_turns<PH>(rowc, boff, T * k * 16, cc);
        float2 p = cis_quadrant(u.r, u.q);
        v[k] = cmul(v[k], make_float2(p.x * a.scale, p.y * sy));
      });
      fft_line<N, true, C, 1>(v, lb, lc, lds, tw);
    } else if constexpr (MODE == COL_A) {
      // V = F^-1[Phi3 (Xt + mu W)] / N_a; X+ = S_sigma(V); Xt+ = Phi3* F X+
      // (the screen is evaluated again on the way back: cheaper than keeping
      // it in registers across two transforms)
      const bool first = a.flags & 1;
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = in1.f2(voff, k * kbytes);
      if (!first) {
#pragma unroll
        for (int k = 0; k < E; ++k) {
          const float2 x = in0.f2(voff, k * kbytes);
          v[k] = make_float2(fmaf(a.mu, v[k].x, x.x), fmaf(a.mu, v[k].y, x.y));
        }
      } else {
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = cscale(v[k], a.mu);
      }
      if (!active) {
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = make_float2(0.f, 0.f);
      }
      chunked<E, 4>([&](int k) {
        Turns u = col_turns<3>(rowc, boff, T * k * 16, cc);
        float2 p = cis_quadrant(u.r, u.q);
        v[k] = cscale(cmul(v[k], p), a.scale);
      });
      fft_line<N, true, C, 1>(v, lb, lc, lds, tw);
      const float s2 = a.sigma * a.sigma;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const float m2 = fmaf(v[k].x, v[k].x, v[k].y * v[k].y);
        const float f = m2 > s2 ? fmaf(-a.sigma, rsqrtf(m2), 1.0f) : 0.0f;
        v[k] = cscale(v[k], f);
      }
      if (!(a.flags & 2)) {
        asm volatile("" : "+s"(tw));
        fft_line<N, false, C, 1>(v, lb, lc, lds, tw);
        chunked<E, 4>([&](int k) {
          Turns u = col_turns<3>(rowc, boff, T * k * 16, cc);
          v[k] = cmulc(v[k], cis_quadrant(u.r, u.q));
        });
      }
    } else {  // COL_R
      // GX = F^-1[Phi1* Wg] / N_a; R = m o (y - GX); out = Phi1 F R
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = in0.f2(voff, k * kbytes);
      if (!active) {
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = make_float2(0.f, 0.f);
      }
      chunked<E, 4>([&](int k) {
        Turns u = col_turns<1>(rowc, boff, T * k * 16, cc);
        float2 p = cis_quadrant(u.r, u.q);
        v[k] = cscale(cmulc(v[k], p), a.scale);
      });
      fft_line<N, true, C, 1>(v, lb, lc, lds, tw);
      const uint32_t moff = (lane >> 5) * 4u, bit = lane & 31u;
      const uint32_t act = active ? 1u : 0u;
      chunked<E, 4>([&](int k) {
        const uint32_t w = mask.u32(moff, k * kmask);
        const float keep = (float)((w >> bit) & act);
        const float2 yy = yb.f2(voff, k * kbytes);
        float2 r = cscale(csub(yy, v[k]), keep);
        acc = fmaf(r.x, r.x, fmaf(r.y, r.y, acc));
        asm volatile("" : "+v"(acc));  // accumulate here, not after the next transform
        v[k] = r;
      });
      asm volatile("" : "+s"(tw));
      fft_line<N, false, C, 1>(v, lb, lc, lds, tw);
      chunked<E, 4>([&](int k) {
        Turns u = col_turns<1>(rowc, boff, T * k * 16, cc);
        v[k] = cmul(v[k], cis_quadrant(u.r, u.q));
      });
    }
    if (active) {
#pragma unroll
      for (int k = 0; k < E; ++k) out.st(v[k], voff, k * kbytes);
    }
  }
  const bool want_norm = (MODE == COL_R) || (MODE == COL_FWD && (a.flags & 1));
  if (want_norm) {
    const float part = block_sum<CT>(acc, red);
    finish_partials(part, a.partials, a.counter, a.hist_out, a.status, gridDim.x);
  }
}

// Host-side launch helpers (one set per length, instantiated in kern_<N>.hip).
struct LaunchCfg {
  int grid;
  int block;
};

template <int N>
struct Kernels {
  static hipError_t row(const RowArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(row_pass_kernel<N>, dim3(grid), dim3(Plan<N>::RT), 0, s, a);
    return hipGetLastError();
  }
  template <int MODE, int PH>
  static hipError_t col(const ColArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((col_pass_kernel<N, MODE, PH>), dim3(grid), dim3(Plan<N>::CT), 0, s, a);
    return hipGetLastError();
  }
};

}  // namespace cssar
