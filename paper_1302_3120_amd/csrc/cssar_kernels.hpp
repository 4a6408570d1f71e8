// Fused pass kernels.  A pass reads whole lines of an N_a x N_r array,
// transforms them in registers/LDS and writes them back (in place allowed):
//
//   row pass M (line = one range line at Doppler bin i):
//       x Phi1 -> F_tau -> x Phi2 / N_r -> F_tau^-1 -> x Phi3
//   row pass G:  x Phi3* -> F_tau -> x Phi2* / N_r -> F_tau^-1 -> x Phi1*
//   col passes (tile = C adjacent azimuth columns):
//     FWD:  [m o y, ||.||^2, copy of m o y] -> F_eta
//     INV:  / N_a -> F_eta^-1
//     A:    V = F_eta^-1[Xt + mu Z] / N_a -> X+ = S_sigma(V) -> F_eta X+ (or X+)
//     R:    GX = F_eta^-1[W] / N_a -> R = m o y - m o GX, ||R||^2 -> F_eta R
//
// All three phase screens are evaluated in the row passes, where each is a
// quadratic polynomial in the element's offset along the line.
//
// Every kernel is persistent: a workgroup walks over units (row groups or
// column tiles) with a stride of the grid size, and the loads of its next
// unit are issued into a second register set before the current unit is
// transformed, so HBM traffic overlaps the FFT work.  Nothing inside the
// transform reads global memory (twiddles come from a small LDS table), so
// waiting for the current unit never waits for the prefetch.
//
// Memory layouts.  Arrays handed over by the caller are row-major ("RM":
// element (i, j) at byte 8 (i N_r + j)).  Arrays that stay inside a solve or
// an operator application use the blocked layout "B4": 4 x 4 blocks of 128
// bytes, element (i, j) at byte (i/4) S + (j/4) 128 + (i%4) 32 + (j%4) 8, with
// a block-row stride S = 32 N_r + 128.  A row pass that handles four rows and
// a column pass that handles four columns both move whole 128-byte blocks,
// and the 128-byte pad per block row spreads a column's blocks over the HBM
// channels (without it a column walks a power-of-two stride).
#pragma once

#include "cssar_device.hpp"

namespace cssar {

enum Layout { RM = 0, B4 = 1 };

#ifndef CSSAR_PREFETCH
#define CSSAR_PREFETCH 0
#endif
// 1: the next unit's loads are issued before the current unit is transformed
constexpr bool kPrefetch = CSSAR_PREFETCH != 0;

__host__ __device__ constexpr uint32_t b4_stride(int nr) { return 32u * (uint32_t)nr + 128u; }
__host__ __device__ constexpr size_t b4_bytes(int na, int nr) { return (size_t)(na / 4) * b4_stride(nr); }

// Byte offset of element (i, j), i = b + T k, as a per-lane part (k = 0) and
// a wave-uniform step per k (T a multiple of 4).
struct Addr {
  uint32_t voff, kstep;
};
__device__ __forceinline__ Addr col_addr(int layout, int b, int j, int T, int nr) {
  Addr a;
  if (layout == B4) {
    const uint32_t S = b4_stride(nr);
    a.voff = (uint32_t)(b >> 2) * S + (uint32_t)(j >> 2) * 128u + (uint32_t)(b & 3) * 32u + (uint32_t)(j & 3) * 8u;
    a.kstep = (uint32_t)(T / 4) * S;
  } else {
    a.voff = ((uint32_t)b * nr + j) * 8u;
    a.kstep = (uint32_t)T * nr * 8u;
  }
  return a;
}

struct RowArgs {
  const float2* in;      // B4
  float2* out;           // B4
  const double2* rowc1;  // per Doppler bin: Phi1 (a1, d1)
  const double2* rowc2;  //                  Phi2 (a2, b2)
  const double2* rowc3;  //                  Phi3 (D, b3)
  const float2* tw;      // w_N^k, N = N_r
  int na;
  int conj;              // 0: M (Phi1, Phi2, Phi3); 1: G (Phi3*, Phi2*, Phi1*)
  float scale;           // 1 / N_r
  double inv_fs;         // 1 / fs
  double fc_fs;          // fc / fs
  double p_c;            // fc * 2 r_ref / c (Phi3 turns per unit D at the reference range)
};

enum ColMode { COL_FWD = 0, COL_INV = 1, COL_A = 2, COL_R = 3 };

// Marks an unsampled entry of the stored copy of m o y (real part; a NaN
// with a payload that arithmetic does not produce).
constexpr uint32_t kUnsampled = 0x7FA5A5A5u;

struct ColArgs {
  const float2* in0;     // FWD: input (RM); INV: input (B4); A: Xt (B4, NULL on the first iteration); R: W (B4)
  const float2* in1;     // A: Z (B4)
  const float2* y;       // R: m o y (B4), unsampled entries marked with kUnsampled
  const uint32_t* mask;  // FWD: packed sampling mask, bit = blocked element index
  float2* out;           // FWD, R: B4; INV: RM; A: B4, or RM with flag 2
  float2* out2;          // FWD with flag 4: copy of m o y (B4, marked)
  const float2* tw;      // w_N^k, N = N_a
  int na, nr;
  int flags;             // FWD: 1 = mask the input and sum |.|^2, 4 = write out2;
                         // A: 1 = no Xt input, 2 = store X (RM) instead of F_eta X (B4)
  float scale;           // 1 / N_a (inverse transforms)
  float mu, sigma;       // A: step and threshold lambda*mu
  float* partials;       // per-block partial sums of ||R||^2
  unsigned* counter;     // last-block detection
  float* hist_out;       // where the total ||R||^2 goes (may be NULL)
  unsigned* status;      // bit 0: non-finite residual
};

// Elementwise work on the E register elements in chunks of CH, with
// scheduling barriers between chunks so the compiler does not hoist every
// FP64 phase evaluation at once (register pressure).
template <int E, int CH, typename F>
__device__ __forceinline__ void chunked(F&& f) {
#pragma unroll
  for (int k0 = 0; k0 < E; k0 += CH) {
#pragma unroll
    for (int k = k0; k < k0 + CH; ++k) f(k);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Range-Doppler screens as polynomials of the centred column offset
// o = j - N_r/2 (dtau = o / fs):
//   Phi1 turns = a1 (o/fs - d1)^2 = a1 d1^2 - 2 a1 d1 o/fs + a1 o^2/fs^2
//   Phi3 turns = D (p_c + o fc/fs) + b3 o^2/fs^2
// and the 2-D frequency screen of the signed range bin nu:
//   Phi2 turns = b2 nu + a2 nu^2
__device__ __forceinline__ Quad phi1_quad(double2 c, const RowArgs& a, int b, int T) {
  const double f = a.inv_fs;
  return quad_in_slot(c.x * c.y * c.y, -2.0 * c.x * c.y * f, c.x * f * f, b, T);
}
__device__ __forceinline__ Quad phi3_quad(double2 c, const RowArgs& a, int b, int T) {
  const double f = a.inv_fs;
  return quad_in_slot(c.x * a.p_c, c.x * a.fc_fs, c.y * f * f, b, T);
}
__device__ __forceinline__ Quad phi2_quad(double2 c, int b, int T) {
  return quad_in_slot(0.0, c.y, c.x, b, T);
}

// v[k] *= exp(+-2 pi i phase(k')) * s, with k' = k - E/2 (column offset
// screens) or the signed bin slot (frequency screen: k' = k or k - E).
template <int E, bool FREQ>
__device__ __forceinline__ void apply_quad(float2 (&v)[E], const Quad& q, bool conj, float s) {
  chunked<E, 4>([&](int k) {
    const int kk = FREQ ? (k < E / 2 ? k : k - E) : k - E / 2;
    float2 p = cis_quad(q, kk);
    p = make_float2(p.x * s, (conj ? -p.y : p.y) * s);
    v[k] = cmul(v[k], p);
  });
}

__device__ __forceinline__ int xcd_logical_block() {
  // Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
  // that consecutive logical ids (adjacent column tiles) run on the same XCD.
  const int g = gridDim.x, w = blockIdx.x;
  if (g % 8 != 0) return w;
  return (w % 8) * (g / 8) + w / 8;
}

// Row pass (B4 in and out).  Thread t of a workgroup with LR = 4 G rows:
// g = t / 4T picks the block row, and within it lane bits 0-1 give j % 4,
// bits 2-3 the row in the block, the rest the block along the row, so the
// 64 lanes of a wave read 4 consecutive 128-byte blocks.
template <int N>
__global__ __launch_bounds__(Plan<N>::RT) void row_pass_kernel(RowArgs a) {
  using P = Plan<N>;
  constexpr int E = P::E, T = P::T, LR = P::LR;
  // the rows handled together share one LDS buffer, interleaved element by
  // element like the columns of a column tile (conflict-free exchanges)
  constexpr int LI = LR >= 4 ? 4 : LR;
  constexpr int LS = LdsSize<LI, N>::value;
  __shared__ float2 lds[(LR / LI) * LS];
  __shared__ float2 twl[64 + N / 64];
  load_twiddle_table<N>(twl, a.tw);
  __syncthreads();
  // lane bits 0-1: j % 4; then log2(LI) bits: the row inside the block (or
  // half block); the rest: the block along the row
  int line, b;
  if constexpr (LR == 1) {
    line = 0;
    b = threadIdx.x;
  } else if constexpr (LR == 2) {
    line = (threadIdx.x >> 2) & 1;
    b = (threadIdx.x & 3) | ((threadIdx.x >> 3) << 2);
  } else {
    const int g = threadIdx.x / (4 * T), t = threadIdx.x % (4 * T);
    line = 4 * g + ((t >> 2) & 3);
    b = (t & 3) | ((t >> 4) << 2);
  }
  const int lsub = line % LI;  // position inside the interleaved buffer
  const uint32_t S = b4_stride(N);
  const uint32_t bytes = clamp_bytes(b4_bytes(a.na, N));
  const Buf in(a.in, bytes), out(a.out, bytes);
  const bool conj = a.conj != 0;
  const int groups = a.na / LR;  // N_a is a multiple of LR
  auto voff_of = [&](int row) {
    return (uint32_t)(row >> 2) * S + (uint32_t)(b >> 2) * 128u + (uint32_t)(row & 3) * 32u + (uint32_t)(b & 3) * 8u;
  };
  // prefetch registers: the next unit's data and its three coefficient pairs
  float2 vn[E];
  double2 c1n, c2n, c3n;
  auto fetch = [&](int gi) {
    const int row = gi * LR + line;
    const uint32_t vo = voff_of(row);
#pragma unroll
    for (int k = 0; k < E; ++k) vn[k] = in.f2(vo, T * k * 32);
    c1n = a.rowc1[row];
    c2n = a.rowc2[row];
    c3n = a.rowc3[row];
  };
  int gi = LR == 2 ? xcd_logical_block() : (int)blockIdx.x;
  if (kPrefetch && gi < groups) fetch(gi);
  for (; gi < groups; gi += gridDim.x) {
    const int row = gi * LR + line;
    if (!kPrefetch) fetch(gi);
    float2 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = vn[k];
    const double2 c1 = c1n, c2 = c2n, c3 = c3n;
    if (kPrefetch && gi + (int)gridDim.x < groups) fetch(gi + gridDim.x);
    int lb = b, lc = lsub;
    asm volatile("" : "+v"(lb), "+v"(lc));  // recompute LDS addresses per unit (register pressure)
    float2* lmy = lds + (line / LI) * LS;
    asm volatile("" : "+v"(lmy));
    const TwLds tws{twl, twl + 64};
    // first range-Doppler screen: Phi1 (M) or Phi3* (G)
    apply_quad<E, false>(v, conj ? phi3_quad(c3, a, b, T) : phi1_quad(c1, a, b, T), conj, 1.0f);
    fft_line<N, false, LI>(v, lb, lc, lmy, tws);
    apply_quad<E, true>(v, phi2_quad(c2, b, T), conj, a.scale);
    asm volatile("" : "+v"(lb), "+v"(lc), "+v"(lmy));
    fft_line<N, true, LI>(v, lb, lc, lmy, tws);
    // second range-Doppler screen: Phi3 (M) or Phi1* (G)
    apply_quad<E, false>(v, conj ? phi1_quad(c1, a, b, T) : phi3_quad(c3, a, b, T), conj, 1.0f);
    const uint32_t vo = voff_of(row);
#pragma unroll
    for (int k = 0; k < E; ++k) out.st(v[k], vo, T * k * 32);
  }
}

template <int N, int MODE>
__global__ __launch_bounds__(Plan<N>::CT) void col_pass_kernel(ColArgs a) {
  using P = Plan<N>;
  constexpr int E = P::E, T = P::T, C = P::C, CT = P::CT;
  constexpr int LS = LdsSize<C, N>::value;
  __shared__ float2 lds[LS];
  __shared__ float2 twl[64 + N / 64];
  __shared__ float red[CT / 64];
  load_twiddle_table<N>(twl, a.tw);
  __syncthreads();
  const int c = threadIdx.x % C;
  const int b = threadIdx.x / C;
  const int ntiles = a.nr / C;  // N_r is a multiple of C
  const uint32_t rmb = clamp_bytes((size_t)N * a.nr * 8), b4b = clamp_bytes(b4_bytes(N, a.nr));
  constexpr int in_layout = MODE == COL_FWD ? RM : B4;
  const int out_layout = (MODE == COL_INV || (MODE == COL_A && (a.flags & 2))) ? RM : B4;
  const Buf in0(a.in0, in_layout == RM ? rmb : b4b), in1(a.in1, b4b), yb(a.y, b4b);
  const Buf out(a.out, out_layout == RM ? rmb : b4b), out2(a.out2, b4b);
  const Buf mask(a.mask, clamp_bytes(((size_t)N * a.nr + 31) / 32 * 4));
  const uint32_t kmask = T * (uint32_t)a.nr / 32 * 4;  // mask byte step per k (T N_r % 32 == 0)
  const bool first = (MODE == COL_A) && (a.flags & 1);
  // prefetch registers of the next tile: x (main input) and, for the update
  // pass, z (second input Z)
  float2 xn[E], zn[E];
  auto fetch = [&](int tile) {
    const int j = tile * C + c;
    const Addr ai = col_addr(in_layout, b, j, T, a.nr);
    if constexpr (MODE == COL_A) {
#pragma unroll
      for (int k = 0; k < E; ++k) zn[k] = in1.f2(ai.voff, k * ai.kstep);
      if (!first) {
#pragma unroll
        for (int k = 0; k < E; ++k) xn[k] = in0.f2(ai.voff, k * ai.kstep);
      }
    } else {
#pragma unroll
      for (int k = 0; k < E; ++k) xn[k] = in0.f2(ai.voff, k * ai.kstep);
    }
  };
  float acc = 0.f;
  int tile = xcd_logical_block();
  if (kPrefetch && tile < ntiles) fetch(tile);
  for (; tile < ntiles; tile += gridDim.x) {
    const int j = tile * C + c;
    if (!kPrefetch) fetch(tile);
    const Addr ab = col_addr(B4, b, j, T, a.nr);
    float2 v[E], y2[E];
    if constexpr (MODE == COL_A) {
      // V = F^-1[Xt + mu Z] / N_a
      const float ms = a.mu * a.scale;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        v[k] = cscale(zn[k], ms);
        if (!first) v[k] = make_float2(fmaf(a.scale, xn[k].x, v[k].x), fmaf(a.scale, xn[k].y, v[k].y));
      }
    } else if constexpr (MODE == COL_FWD) {
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = xn[k];
    } else {
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = cscale(xn[k], a.scale);
      if constexpr (MODE == COL_R) {
        // m o y of this tile (issued before any prefetch of the next tile)
#pragma unroll
        for (int k = 0; k < E; ++k) y2[k] = yb.f2(ab.voff, k * ab.kstep);
      }
    }
    const int next = tile + gridDim.x;
    if (kPrefetch && next < ntiles) fetch(next);
    const TwLds tws{twl, twl + 64};
    int lb = b, lc = c;
    asm volatile("" : "+v"(lb), "+v"(lc));  // recompute LDS addresses per tile
    if constexpr (MODE == COL_FWD) {
      if (a.flags & 1) {
        // blocked element index of (b, j) addresses the packed mask
        const uint32_t e0 = (((uint32_t)(b >> 2) * (a.nr / 4) + (j >> 2)) << 4) + ((b & 3) << 2) + (j & 3);
        const uint32_t moff = (e0 >> 5) * 4u, bit = e0 & 31u;
#pragma unroll
        for (int k = 0; k < E; ++k) {
          const uint32_t w = mask.u32(moff, k * kmask);
          const bool keep = (w >> bit) & 1u;
          if (!keep) v[k] = make_float2(0.f, 0.f);
          acc = fmaf(v[k].x, v[k].x, fmaf(v[k].y, v[k].y, acc));
          if (a.flags & 4)
            out2.st(keep ? v[k] : make_float2(__uint_as_float(kUnsampled), 0.f), ab.voff, k * ab.kstep);
        }
      }
      fft_line<N, false, C>(v, lb, lc, lds, tws);
    } else if constexpr (MODE == COL_INV) {
      fft_line<N, true, C>(v, lb, lc, lds, tws);
    } else if constexpr (MODE == COL_A) {
      fft_line<N, true, C>(v, lb, lc, lds, tws);
      // X+ = S_sigma(V)
      const float s2 = a.sigma * a.sigma;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const float m2 = fmaf(v[k].x, v[k].x, v[k].y * v[k].y);
        const float f = m2 > s2 ? fmaf(-a.sigma, rsqrtf(m2), 1.0f) : 0.0f;
        v[k] = cscale(v[k], f);
      }
      if (!(a.flags & 2)) {
        asm volatile("" : "+v"(lb), "+v"(lc));
        fft_line<N, false, C>(v, lb, lc, lds, tws);  // Xt+ = F X+
      }
    } else {  // COL_R: GX = F^-1[W] / N_a; R = m o y - m o GX; out = F R
      fft_line<N, true, C>(v, lb, lc, lds, tws);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const bool keep = __float_as_uint(y2[k].x) != kUnsampled;
        const float2 r = keep ? csub(y2[k], v[k]) : make_float2(0.f, 0.f);
        acc = fmaf(r.x, r.x, fmaf(r.y, r.y, acc));
        v[k] = r;
      }
      asm volatile("" : "+v"(lb), "+v"(lc));
      fft_line<N, false, C>(v, lb, lc, lds, tws);
    }
    const Addr ao = out_layout == RM ? col_addr(RM, b, j, T, a.nr) : ab;
#pragma unroll
    for (int k = 0; k < E; ++k) out.st(v[k], ao.voff, k * ao.kstep);
  }
  const bool want_norm = (MODE == COL_R) || (MODE == COL_FWD && (a.flags & 1));
  if (want_norm) {
    const float part = block_sum<CT>(acc, red);
    finish_partials(part, a.partials, a.counter, a.hist_out, a.status, gridDim.x);
  }
}

// Host-side launch helpers (one set per length, instantiated in kern_inst.hip).
template <int N>
struct Kernels {
  static hipError_t row(const RowArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(row_pass_kernel<N>, dim3(grid), dim3(Plan<N>::RT), 0, s, a);
    return hipGetLastError();
  }
  template <int MODE>
  static hipError_t col(const ColArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((col_pass_kernel<N, MODE>), dim3(grid), dim3(Plan<N>::CT), 0, s, a);
    return hipGetLastError();
  }
};

}  // namespace cssar
