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
//   adaptive parameters (Section IV.B):
//     D:    dX = F_eta^-1[Z] / N_a -> dX on the support, ||.||^2 -> F_eta of it
//     N:    F_eta^-1[W] / N_a -> ||m o .||^2 -> the step mu = ||dX_G||^2 / that
//     V:    V = F_eta^-1[Xt + mu Z] / N_a (mu from device memory)
//     T:    X+ = S_sigma(V) (sigma from device memory), support bits -> F_eta X+
//
// All three phase screens are evaluated in the row passes, where each is a
// quadratic polynomial in the element's offset along the line.
//
// Every kernel is persistent: a workgroup walks over units (row groups or
// column tiles) with a stride of the grid size; several workgroups share a
// compute unit so that one's loads overlap another's FFT work.  Nothing
// inside the transform reads global memory (twiddles come from a small LDS
// table).  The grouped variants walk over the units of many arrays of one
// line length (the batched solver): a table of per-array arguments and the
// prefix sums of their unit counts map a global unit index to (array, unit).
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

#include <type_traits>

#include "cssar_device.hpp"

namespace cssar {

enum Layout { RM = 0, B4 = 1 };

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
  // adjoint row pass only
  const float2* in2;     // input of the adjoint chain (B4)
  const float* rowd;     // per Doppler bin: 18 floats, d arg_k / d theta as
                         // polynomials c0 + c1 o + c2 o^2 (radians), ordered
                         // [theta = K_a, K_r][stage 1, 2, 3][c0, c1, c2]
  float* partials;       // per-block partial sums (2 per block)
  // range-Doppler chain (rowc1: migration (a, b) per Doppler bin, in range
  // samples delta_j = a + b j; rowc3: azimuth filter turns (A, B), A + B j)
  double c_tau;          // range filter turns per squared range bin, df^2 / (2 K_r)
  int taps;              // truncated sinc length K (even)
  const unsigned* gate;  // if not NULL, the pass does nothing while *gate == 0
};

// Column modes.  FWD, INV, A, R: the forward passes.  VB, U, XB: the
// adjoint passes of the gradient (threshold adjoint, data adjoint, update
// of the iterate's adjoint).
// D, N, V, T: the passes of the adaptive step and threshold.  AS: the
// update pass of the sparse iterate (col_update_sparse).
enum ColMode {
  COL_FWD = 0, COL_INV = 1, COL_A = 2, COL_R = 3, COL_VB = 4, COL_U = 5, COL_XB = 6,
  COL_D = 7, COL_N = 8, COL_V = 9, COL_T = 10, COL_AS = 11
};

// Device-resident state of the adaptive solver (one per solve, in its
// workspace): the selection of the (k+1)-th largest |V|^2 by its FP32 bit
// pattern (11 + 11 + 10 bits, most significant first), and the step and
// threshold of the current iteration.
struct AdaptState {
  unsigned hist[2048];  // histogram of the current selection level (cleared after use)
  unsigned prefix;      // key bits selected so far
  unsigned rank;        // rank still to find among the keys under prefix (1 = largest)
  unsigned k1;          // k + 1
  unsigned done;        // fewer than k + 1 keys: the threshold is 0
  float mu;             // step of the current iteration
  float sigma;          // threshold lambda mu of the current iteration
  float sigma2;         // sigma^2, the selected key
  float pad;
  double num;           // ||dX_G||^2 of the current iteration
  // support-change safeguard of the step
  double dnum;          // ||F_eta (X+ - X)||^2 = N_a ||X+ - X||^2 of the last threshold pass
  double c;             // bound constant: omega = (1 - c) ||X+ - X||^2 / ||m o G(X+ - X)||^2
  double shrink;        // step factor of a shrink, 1 / (kappa (1 - c))
  unsigned active;      // 1 while this iteration's shrink loop goes on (gates its passes)
  unsigned changed;     // the threshold pass found supp X+ != supp X
  unsigned shrinks;     // shrinks taken in this iteration
  // selection candidates: each workgroup of the value pass (nseg of them)
  // stores the keys whose first-level bin lies in [wlo, whi] (around the
  // previous selection's bin) in its own segment of seg keys, and their
  // count; when the selected bin lies in that window and no segment
  // overflowed, the later levels read only the candidates (use_cand)
  unsigned wlo, whi;
  unsigned nseg, seg;
  unsigned use_cand;
  unsigned pad2;
};
// After an AdaptState: the candidate counts (kMaxCandSeg), then the keys.
constexpr int kMaxCandSeg = 4096;
__device__ __forceinline__ unsigned* adapt_cand_counts(AdaptState* st) { return (unsigned*)(st + 1); }
__device__ __forceinline__ unsigned* adapt_candidates(AdaptState* st) {
  return (unsigned*)(st + 1) + kMaxCandSeg;
}

// Marks an unsampled entry of the stored copy of m o y (real part; a NaN
// with a payload that arithmetic does not produce).
constexpr uint32_t kUnsampled = 0x7FA5A5A5u;

struct ColArgs {
  const float2* in0;     // FWD: input (RM); INV: input (B4); A, VB: Xt (B4, NULL on the first
                         // iteration); R: W (B4); U: F G Vbar; XB: F M ubar
  const float2* in1;     // A, VB: Z (B4); U: ybar accumulator (spatial); XB: Vbar (spatial)
  const float2* y;       // R, U: m o y (B4), unsampled entries marked with kUnsampled;
                         // VB: adjoint of the next iterate (spatial)
  const uint32_t* mask;  // FWD: packed sampling mask, bit = blocked element index
  float2* out;           // FWD, R: B4; INV: RM; A: B4, or RM with flag 2
  float2* out2;          // FWD with flag 4: copy of m o y (B4, marked); VB: Vbar (spatial);
                         // U: ybar accumulator (spatial, may alias in1)
  const float2* tw;      // w_N^k, N = N_a
  int na, nr;
  int flags;             // FWD: 1 = mask the input and sum |.|^2, 4 = write out2;
                         // A: 1 = no Xt input, 2 = store X (RM) instead of F_eta X (B4);
                         // T: 4 = safeguard (support change against supp_old),
                         //    16 = also store X+ (spatial, row-major) to out3
  float scale;           // 1 / N_a (inverse transforms)
  float mu, sigma;       // A: step and threshold lambda*mu
  float* partials;       // per-block partial sums (R, masked FWD, D, N)
  float* hist_out;       // R, masked FWD: where the total ||R||^2 goes (may be NULL; the
                         // passes write per-block partials, a one-block kernel the total)
  unsigned* status;      // bit 0: non-finite norm (set by the one-block total kernels)
  // adaptive passes
  AdaptState* ad;        // step, threshold, ||dX_G||^2
  uint32_t* supp;        // D (read), T (written): support bits, word tile * CT + thread,
                         // bit k = element (b + T k, tile C + c) of the column tile
  // support-change safeguard (T with flag 4)
  const uint32_t* supp_old;  // T: support bits of the iterate X (compared with X+'s)
  float2* out3;          // T with flag 16: X+ (spatial, row-major)
  const unsigned* gate;  // if not NULL, the pass does nothing while *gate == 0
  // sparse iterate (AS, col_update_sparse): per column tile, an area of 64
  // 32-byte records per wave (index tile * CT + 64 wave + slot) holding the
  // records of the wave's threads with nonzeros, packed; the 64-bit lane
  // mask of every wave (index tile * CT/64 + wave); and the dense store of
  // the threads with more than two nonzeros
  float4* xrec;
  uint64_t* xwmask;
  float2* xdense;        // B4
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
// screens) or the signed bin slot (frequency screen: k' = k or k - E); one
// FP64 evaluation per element.
template <int E, bool FREQ>
__device__ __forceinline__ void apply_quad(float2 (&v)[E], const Quad& q, bool conj, float s) {
  chunked<E, 4>([&](int k) {
    const int kk = FREQ ? (k < E / 2 ? k : k - E) : k - E / 2;
    float2 p = cis_quad(q, kk);
    p = make_float2(p.x * s, (conj ? -p.y : p.y) * s);
    v[k] = cmul(v[k], p);
  });
}

// The same screen from a per-line table: the slot phase A + B k' + C k'^2
// (A, B per thread, C per line) is applied as exp(2 pi i A) exp(2 pi i B)^k'
// tab[|k'|], with tab[m] = exp(2 pi i C m^2) computed once per line and
// shared through LDS, and the powers of exp(2 pi i B) by products from
// k' = 0 (at most E/2 of them).  Two evaluations per thread and screen
// instead of one per element.
template <int E, bool FREQ, bool TAB = true>
__device__ __forceinline__ void apply_quad_tab(float2 (&v)[E], const Quad& q, const float2* tab, bool conj,
                                               float s) {
  auto slot = [](int kk) { return FREQ ? (kk >= 0 ? kk : kk + E) : kk + E / 2; };
  auto cj = [&](float2 z) { return conj ? make_float2(z.x, -z.y) : z; };
  const float2 z0 = cscale(cj(cis_turns(q.A)), s);
  const float2 u = cj(cis_turns(q.B));
  const float2 ub = make_float2(u.x, -u.y);  // u^-1 (|u| = 1)
  // (TAB false: C = 0, every factor of the table is 1)
  auto fac = [&](float2 w, int m) { return TAB ? cmul(w, cj(tab[m])) : w; };
  float2 w = z0;
#pragma unroll
  for (int kk = 0; kk < E / 2; ++kk) {
    v[slot(kk)] = cmul(v[slot(kk)], fac(w, kk));
    if (kk + 1 < E / 2) w = cmul(w, u);
  }
  w = cmul(z0, ub);
#pragma unroll
  for (int kk = -1; kk >= -E / 2; --kk) {
    v[slot(kk)] = cmul(v[slot(kk)], fac(w, -kk));
    if (kk - 1 >= -E / 2) w = cmul(w, ub);
  }
}

__device__ __forceinline__ int xcd_logical_block() {
  // Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
  // that consecutive logical ids (adjacent units) run on the same XCD.
  const int g = gridDim.x, w = blockIdx.x;
  if (g % 8 != 0) return w;
  return (w % 8) * (g / 8) + w / 8;
}

// Units of many arrays in one launch: array s owns global units
// start[s] .. start[s+1]-1; args points at count RowArgs or ColArgs.
struct GroupArgs {
  const void* args;
  const int* start;  // count + 1 prefix sums
  int count;
  int total;         // start[count]
  int conj;          // row groups: 0 (M) or 1 (G), the same for every array of the launch
};

// Largest s with start[s] <= u (u is uniform across the workgroup, so the
// search runs on scalar loads).
__device__ __forceinline__ int group_find(const int* __restrict__ start, int count, int u) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------- row pass --
// Row pass (B4 in and out).  Thread t of a workgroup with LR = 4 G rows:
// g = t / 4T picks the block row, and within it lane bits 0-1 give j % 4,
// bits 2-3 the row in the block, the rest the block along the row, so the
// 64 lanes of a wave read 4 consecutive 128-byte blocks.  With LR = 2, lane
// bit 2 picks the row and a wave reads the halves of 8 blocks.
template <class P>
struct RowLane {
  int line, b;
  __device__ __forceinline__ RowLane() {
    constexpr int T = P::T, LR = P::LR;
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
  }
};

// The rows handled together share one LDS buffer, interleaved element by
// element like the columns of a column tile (conflict-free exchanges).
template <class P>
struct RowLds {
  static constexpr int LI = P::LR >= 4 ? 4 : P::LR;
  static constexpr int LS = LdsSize<LI, P::SPLIT ? P::N / 2 : P::N>::value;  // split: half lines
  static constexpr int size = (P::LR / LI) * LS;
  // split plans whose LDS lets two workgroups share a CU ask for the
  // registers that allow it (waves per SIMD)
  static constexpr int waves_per_eu = (P::SPLIT && size * 8 <= 78 * 1024) ? 2 * (P::RT / 64) / 4 : 1;
  // the range-Doppler row pass: two 512-thread workgroups per CU where the
  // LDS allows (128 VGPRs)
  static constexpr int rda_waves_per_eu = (!P::SPLIT && P::RT == 512 && size * 8 <= 78 * 1024) ? 4 : 1;
};

// One unit (LR rows) of the row pass of array a:
//   M: x Phi1 -> F_tau -> x Phi2 / N_r -> F_tau^-1 -> x Phi3
//   G: x Phi3* -> F_tau -> x Phi2* / N_r -> F_tau^-1 -> x Phi1*
// CJ: 0 (M) or 1 (G) fixed at compile time, -1 read from a.conj.
// Per-line tables of the screens' quadratic factors (apply_quad_tab): for
// each of the LR lines of a unit and each screen, exp(2 pi i C m^2), m <= E/2.
template <class P>
struct RowQTab {
  static constexpr int NQ = P::E / 2 + 1;
  static constexpr int PER = 3 * NQ;          // per line
  static constexpr int size = P::LR * PER;    // per unit
};

// Fill the tables of unit gi (threads 0 .. LR*PER-1, then a barrier).
template <class P>
__device__ __forceinline__ void row_qtab_fill(const RowArgs& a, int gi, float2* qt) {
  constexpr int NQ = RowQTab<P>::NQ, PER = RowQTab<P>::PER;
  for (int t = threadIdx.x; t < RowQTab<P>::size; t += P::RT) {
    const int l = t / PER, sc = (t % PER) / NQ, m = t % NQ;
    const int r = gi * P::LR + l;
    const double f2 = a.inv_fs * a.inv_fs;
    const double p2 = sc == 0 ? a.rowc1[r].x * f2 : (sc == 1 ? a.rowc2[r].x : a.rowc3[r].y * f2);
    const double C = frac1(p2 * (double)P::T * (double)P::T);  // quad_in_slot's C
    qt[t] = cis_turns(C * (double)(m * m));
  }
  __syncthreads();
}

template <class P, int CJ = -1>
__device__ __forceinline__ void row_unit(const RowArgs& a, int gi, const RowLane<P>& ln, float2* lds,
                                         const float2* twl, const TwPowers& hp, const float2* qt) {
  constexpr int HS = hoisted_pass<P>();
  constexpr int N = P::N, E = P::E, T = P::T, LR = P::LR;
  constexpr int LI = RowLds<P>::LI, LS = RowLds<P>::LS;
  const uint32_t S = b4_stride(N);
  const uint32_t bytes = clamp_bytes(b4_bytes(a.na, N));
  const Buf in(a.in, bytes), out(a.out, bytes);
  const bool conj = CJ >= 0 ? CJ != 0 : a.conj != 0;
  const int b = ln.b, line = ln.line;
  const int row = gi * LR + line;
  const uint32_t vo = (uint32_t)(row >> 2) * S + (uint32_t)(b >> 2) * 128u + (uint32_t)(row & 3) * 32u +
                      (uint32_t)(b & 3) * 8u;
  float2 v[E];
#pragma unroll
  for (int k = 0; k < E; ++k) v[k] = in.f2(vo, T * k * 32);
  const double2 c1 = a.rowc1[row], c2 = a.rowc2[row], c3 = a.rowc3[row];
  int lb = b, lc = line % LI;
  asm volatile("" : "+v"(lb), "+v"(lc));  // recompute LDS addresses per unit (register pressure)
  // the LDS line offset is kept opaque (register pressure) as an integer, so
  // the compiler still knows lds + loff is in LDS (DS, not FLAT, accesses)
  int loff = (line / LI) * LS;
  asm volatile("" : "+v"(loff));
  const TwLds tws{twl, twl + 64};
  // the screens from the per-line tables of their quadratic factors
  constexpr int NQ = RowQTab<P>::NQ;
  const float2* qline = qt + line * RowQTab<P>::PER;  // [Phi1, Phi2, Phi3] x NQ
  // first range-Doppler screen: Phi1 (M) or Phi3* (G)
  if (conj) apply_quad_tab<E, false>(v, phi3_quad(c3, a, b, T), qline + 2 * NQ, true, 1.0f);
  else apply_quad_tab<E, false>(v, phi1_quad(c1, a, b, T), qline, false, 1.0f);
  fft_line<P, false, LI, TwLds, 0, HS, P::SPLIT>(v, lb, lc, lds + loff, tws, hp);
  apply_quad_tab<E, true>(v, phi2_quad(c2, b, T), qline + NQ, conj, a.scale);
  asm volatile("" : "+v"(lb), "+v"(lc), "+v"(loff));
  fft_line<P, true, LI, TwLds, 0, HS, P::SPLIT>(v, lb, lc, lds + loff, tws, hp);
  // second range-Doppler screen: Phi3 (M) or Phi1* (G)
  if (conj) apply_quad_tab<E, false>(v, phi1_quad(c1, a, b, T), qline, true, 1.0f);
  else apply_quad_tab<E, false>(v, phi3_quad(c3, a, b, T), qline + 2 * NQ, false, 1.0f);
#pragma unroll
  for (int k = 0; k < E; ++k) out.st(v[k], vo, T * k * 32);
}

template <class P, int CJ>
__global__ __launch_bounds__(P::RT, RowLds<P>::waves_per_eu) void row_pass_kernel(RowArgs a) {
  if (a.gate && *a.gate == 0u) return;  // (uniform over the grid)
  __shared__ float2 lds[RowLds<P>::size];
  __shared__ float2 twl[64 + P::N / 64];
  __shared__ float2 qtab[2 * RowQTab<P>::size];  // double-buffered per unit
  __shared__ float2 ptab[pass_table_size<P>()];
  load_twiddle_table<P::N>(twl, a.tw);
  load_pass_table<P>(ptab, a.tw);
  __syncthreads();
  const RowLane<P> ln;
  TwPowers hp;
  if constexpr (hoisted_pass<P>() >= 0)
    hp = hoist_powers<P>(ln.b, TwLds{twl, twl + 64}, ptab);
  const int units = a.na / P::LR;  // N_a is a multiple of LR
  int par = 0;
  // units of one or two rows read part of each 128-byte block: the units of a
  // block row run on one XCD, whose L2 serves the block to all of them
  for (int gi = P::LR <= 2 ? xcd_logical_block() : (int)blockIdx.x; gi < units; gi += gridDim.x) {
    // the barrier of the fill also orders this unit's table against the
    // previous reader of the same buffer (two units ago)
    float2* qt = qtab + par * RowQTab<P>::size;
    row_qtab_fill<P>(a, gi, qt);
    row_unit<P, CJ>(a, gi, ln, lds, twl, hp, qt);
    par ^= 1;
  }
}

template <class P, int CJ>
__global__ __launch_bounds__(P::RT) void row_group_kernel(GroupArgs g) {
  __shared__ float2 lds[RowLds<P>::size];
  __shared__ float2 twl[64 + P::N / 64];
  __shared__ float2 qtab[2 * RowQTab<P>::size];
  const RowArgs* __restrict__ args = (const RowArgs*)g.args;
  __shared__ float2 ptab[pass_table_size<P>()];
  load_twiddle_table<P::N>(twl, args[0].tw);  // w_N depends on N only
  load_pass_table<P>(ptab, args[0].tw);
  __syncthreads();
  const RowLane<P> ln;
  TwPowers hp;
  if constexpr (hoisted_pass<P>() >= 0)
    hp = hoist_powers<P>(ln.b, TwLds{twl, twl + 64}, ptab);
  int par = 0;
  for (int u = xcd_logical_block(); u < g.total; u += gridDim.x) {
    const int s = group_find(g.start, g.count, u);
    float2* qt = qtab + par * RowQTab<P>::size;
    row_qtab_fill<P>(args[s], u - g.start[s], qt);
    row_unit<P, CJ>(args[s], u - g.start[s], ln, lds, twl, hp, qt);
    par ^= 1;
  }
}

// ------------------------------------------------- range-Doppler row pass --
// The row (range) part of the range-Doppler chain of eq. (RDA), one Doppler
// bin per line, the azimuth transforms being the column passes':
//   M:  F_tau -> x P_tau / N_r -> F_tau^-1 -> C (migration) -> x P_eta
//   G:  x P_eta* -> D = C^T -> F_tau -> x P_tau* / N_r -> F_tau^-1
// C (eq. (RCMCs)): U[j] = sum_t V[(p + t) mod N] sinc(t - fr), t = -K/2+1 ..
// K/2, p + fr = j + delta_j (p integer, 0 <= fr < 1), delta_j = a + b j.
// D (eq. (CD)) gathers the same pairs from the output side: V[l] = sum over
// the j whose window holds l (l = p_j + t modulo N) of U[j] sinc(x),
// x = L - j - delta_j in (-K/2, K/2] for the unwrapped L = l + m N.  The
// line goes through LDS for the gather.

// sinc(x) = sin(pi x) / (pi x) for |x| <= 1/2: Taylor polynomial in (pi x)^2
// (error < 4e-8).
__device__ __forceinline__ float sinc_small(float x) {
  const float z = 9.8696044f * x * x;  // (pi x)^2
  return fmaf(z, fmaf(z, fmaf(z, fmaf(z, fmaf(z, -2.5052108e-8f, 2.7557319e-6f), -1.9841270e-4f),
                                8.3333333e-3f), -1.6666667e-1f), 1.0f);
}

// The weights sinc(t - fr) of the taps t = -3 .. 4 of an 8-tap window
// (0 <= fr < 1, sp = sin(pi fr) / pi), except that of the tap nearest the
// position (0 or 1, the caller's polynomial): sinc(t - fr) = (-1)^(t+1) sp /
// x_t with x_t = t - fr.  The six taps away from the position share one
// reciprocal: with the pair products P_m = x_{-m} x_{1+m} (m = 1, 2, 3),
// sp / x_{-m} = x_{1+m} sp / P_m and sp / x_{1+m} = x_{-m} sp / P_m, and
// sp / P_m is the product of the other two pairs times sp / (P_1 P_2 P_3).
// (|x_t| >= 1 for these taps, so no product vanishes.)
__device__ __forceinline__ void sinc_weights8(float fr, float sp, float (&w)[8]) {
  const float xm1 = -1.0f - fr, xm2 = -2.0f - fr, xm3 = -3.0f - fr;
  const float x2 = 2.0f - fr, x3 = 3.0f - fr, x4 = 4.0f - fr;
  const float p1 = xm1 * x2, p2 = xm2 * x3, p3 = xm3 * x4;
  const float p12 = p1 * p2;
  const float r = sp * __builtin_amdgcn_rcpf(p12 * p3);  // sp / (P_1 P_2 P_3)
  const float q3 = p12 * r, q12 = p3 * r;                 // sp / P_3, sp / (P_1 P_2)
  const float q1 = p2 * q12, q2 = p1 * q12;               // sp / P_1, sp / P_2
  w[0] = x4 * q3;    // t = -3
  w[1] = -x3 * q2;   // t = -2
  w[2] = x2 * q1;    // t = -1
  w[3] = sp * __builtin_amdgcn_rcpf(fr);         // t = 0: -sp / (0 - fr)
  w[4] = sp * __builtin_amdgcn_rcpf(1.0f - fr);  // t = 1
  w[5] = -xm1 * q1;  // t = 2
  w[6] = xm2 * q2;   // t = 3
  w[7] = -xm3 * q3;  // t = 4
}

// KT: the tap count at compile time (its loops unrolled, the line staged in
// LDS without padding so every tap is an immediate offset, plus a copy of
// the line's first KT - 1 elements after its end where it fits, so a window
// never wraps), or 0 for any even count read from a.taps.
// The two screens come from their quadratic factors: the range-frequency
// screen's table rtab (exp(2 pi i C m^2), m <= E/2, the same for every
// line), and the azimuth filter, linear in the range offset, needs none.
// The twiddle powers of the hoisted pass are formed per unit just before the
// transforms, so that their registers are free during the interpolation
// (two workgroups per compute unit).
template <class P, int CONJ, int KT>
__device__ __forceinline__ void row_rda_unit(const RowArgs& a, int gi, const RowLane<P>& ln, float2* lds,
                                             const float2* twl, const float2* ptab, const float2* rtab) {
  constexpr int HS = hoisted_pass<P>();
  constexpr int N = P::N, E = P::E, T = P::T, LR = P::LR;
  constexpr int LI = RowLds<P>::LI, LS = RowLds<P>::LS;
  constexpr bool FIX = KT > 0;
  constexpr bool HALO = FIX && LS >= LI * (N + KT);  // room for the wrap copy and over-reads
  const uint32_t S = b4_stride(N);
  const uint32_t bytes = clamp_bytes(b4_bytes(a.na, N));
  const Buf in(a.in, bytes), out(a.out, bytes);
  constexpr bool cj = CONJ != 0;
  const int b = ln.b, line = ln.line;
  const int row = gi * LR + line;
  const uint32_t vo = (uint32_t)(row >> 2) * S + (uint32_t)(b >> 2) * 128u + (uint32_t)(row & 3) * 32u +
                      (uint32_t)(b & 3) * 8u;
  float2 v[E];
#pragma unroll
  for (int k = 0; k < E; ++k) v[k] = in.f2(vo, T * k * 32);
  int lb = b, lc = line % LI;
  asm volatile("" : "+v"(lb), "+v"(lc));
  int loff = (line / LI) * LS;
  asm volatile("" : "+v"(loff));
  float2* ll = lds + loff;  // this line's LDS (interleaved with the unit's other lines)
  const TwLds tws{twl, twl + 64};
  // the hoisted pass's twiddle powers (the index kept opaque so that they
  // are formed here, per unit, and not kept across units)
  auto powers = [&]() {
    TwPowers hp;
    if constexpr (HS >= 0) {
      int hb = b;
      asm volatile("" : "+v"(hb));
      hp = hoist_powers<P>(hb, tws, ptab);
    }
    return hp;
  };
  // azimuth filter turns A + B j = (A + B N/2) + B o, o = j - N/2
  auto eta_screen = [&](bool conj) {
    const double2 az = a.rowc3[row];
    apply_quad_tab<E, false, false>(v, quad_in_slot(fma(az.y, 0.5 * N, az.x), az.y, 0.0, b, T), nullptr, conj,
                                    1.0f);
  };
  // range-frequency screen between the transforms (with 1/N_r; the index
  // opaque, so that its factors are formed per unit and not held across units)
  auto tau_screen = [&](bool conj) {
    int sb = b;
    asm volatile("" : "+v"(sb));
    apply_quad_tab<E, true>(v, quad_in_slot(0.0, 0.0, a.c_tau, sb, T), rtab, conj, a.scale);
  };
  const int K = FIX ? KT : a.taps;
  // element j of this line in LDS: unpadded with a fixed tap count (reads of
  // consecutive j by the lanes of a wave are still conflict-free), else the
  // exchanges' padded order lds_pad<LI>(j LI + lc) = LI (j + j / 16) + lc
  auto idx = [&](int j) { return FIX ? LI * j + lc : LI * (j + (j >> 4)) + lc; };
  auto at = [&](int j) { return ll[idx(j)]; };
  // line through LDS (the exchanges of fft_line leave the LDS free)
  auto stage = [&](bool halo) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int j = b + T * k;
      ll[idx(j)] = v[k];
      if (halo && j < K - 1) ll[idx(N + j)] = v[k];
    }
    __syncthreads();
  };
  if constexpr (cj) {
    eta_screen(true);
    // D = C^T as a scatter: input j adds U[j] sinc(t - fr_j) to output
    // (p_j + t) mod N for each tap t, with p_j + fr_j = j + delta_j and the
    // weights of C.  The migration slope b = 1/D - 1 lies in [0, 1/2), so
    // p_j increases with j by 1 or 2 and the positions of one tap are
    // distinct within each half of the line (their span is under N): one
    // round per half and tap (the halves in turn, so that only one half's
    // positions are held), the sums formed in LDS in a fixed order.
    const double2 mig = a.rowc1[row];
    // with HALO the taps of a window that passes the line's end go to K - 1
    // slots after it, added to the line's first elements at the end, so
    // that every tap is an immediate offset from the window start
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int j = b + T * k;
      ll[idx(j)] = make_float2(0.f, 0.f);
      if (HALO && j < K - 1) ll[idx(N + j)] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    int jb = b;  // (opaque: the positions are formed per unit, not kept across units)
    asm volatile("" : "+v"(jb));
    constexpr int H = E / 2;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int pf[H];
      float fr[H], sp[H];
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const int j = jb + T * (h * H + i);
        const double pos = fma(mig.y, (double)j, mig.x) + (double)j;
        const double pfd = floor(pos);
        fr[i] = (float)(pos - pfd);
        sp[i] = __builtin_amdgcn_sinf(0.5f * fr[i]) * 0.31830989f;  // sin(pi fr) / pi
        // |delta| < N/2 (checked on the host): p_j + t stays within (-N, 2N);
        // with HALO, the window start modulo N
        if constexpr (HALO) {
          const unsigned qs = (unsigned)((int)pfd - K / 2 + 1 + 2 * N);  // (positive)
          pf[i] = (int)((N & (N - 1)) == 0 ? (qs & (unsigned)(N - 1)) : qs % (unsigned)N);
        } else {
          pf[i] = (int)pfd;
        }
      }
      auto tap_round = [&](int t) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
          const bool near = t == (fr[i] < 0.5f ? 0 : 1);
          const float w = near ? sinc_small(fr[i] < 0.5f ? fr[i] : 1.0f - fr[i])
                               : ((t & 1) ? sp[i] : -sp[i]) * __builtin_amdgcn_rcpf((float)t - fr[i]);
          const float2 u = v[h * H + i];
          float2* d;
          if constexpr (HALO) {
            d = ll + idx(pf[i]) + (t + K / 2 - 1) * LI;  // slot start + tap index
          } else {
            int q = pf[i] + t;
            q = q < 0 ? q + N : (q >= N ? q - N : q);
            d = ll + idx(q);
          }
          *d = make_float2(fmaf(w, u.x, d->x), fmaf(w, u.y, d->y));
        }
        __syncthreads();
      };
      if constexpr (FIX) {
#pragma unroll
        for (int t = -KT / 2 + 1; t <= KT / 2; ++t) tap_round(t);
      } else {
        for (int t = -K / 2 + 1; t <= K / 2; ++t) tap_round(t);
      }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int j = b + T * k;
      v[k] = ll[idx(j)];
      if (HALO && j < K - 1) v[k] = cadd(v[k], ll[idx(N + j)]);  // the wrapped taps
    }
    __syncthreads();
    const TwPowers hp = powers();
    fft_line<P, false, LI, TwLds, 0, HS>(v, lb, lc, ll, tws, hp);
    tau_screen(true);
    asm volatile("" : "+v"(lb), "+v"(lc), "+v"(loff));
    fft_line<P, true, LI, TwLds, 0, HS>(v, lb, lc, lds + loff, tws, hp);
  } else {
    {
      const TwPowers hp = powers();
      fft_line<P, false, LI, TwLds, 0, HS>(v, lb, lc, ll, tws, hp);
      tau_screen(false);
      asm volatile("" : "+v"(lb), "+v"(lc), "+v"(loff));
      fft_line<P, true, LI, TwLds, 0, HS>(v, lb, lc, lds + loff, tws, hp);
    }
    // C: the K taps of each output's window; sin(pi (t - fr)) =
    // (-1)^(t+1) sin(pi fr), and the tap nearest the position takes the
    // polynomial
    stage(HALO);
    const double2 mig = a.rowc1[row];
    int jb = b;  // (opaque: the positions are formed per unit, not kept across units)
    asm volatile("" : "+v"(jb));
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int j = jb + T * k;
      const double pos = fma(mig.y, (double)j, mig.x) + (double)j;
      const double pf = floor(pos);
      const float fr = (float)(pos - pf);
      const float sp = __builtin_amdgcn_sinf(0.5f * fr) * 0.31830989f;  // sin(pi fr) / pi
      const int tn = fr < 0.5f ? 0 : 1;
      const float wnear = sinc_small(fr < 0.5f ? fr : 1.0f - fr);
      // |delta| < N/2 (checked on the host), so the window start is > -2N and
      // the sum below is positive
      const unsigned qs = (unsigned)((int)pf - K / 2 + 1 + 2 * N);
      int q = (int)((N & (N - 1)) == 0 ? (qs & (unsigned)(N - 1)) : qs % (unsigned)N);
      float2 acc = make_float2(0.f, 0.f);
      auto tap = [&](int t, float2 u) {
        float w = ((t & 1) ? sp : -sp) * __builtin_amdgcn_rcpf((float)t - fr);
        if (t == tn) w = wnear;
        acc = make_float2(fmaf(w, u.x, acc.x), fmaf(w, u.y, acc.y));
      };
      if constexpr (HALO && KT == 8) {
        const float2* base = ll + idx(q);  // q + KT - 1 < N + KT - 1: inside the copy
        float2 u[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) u[i] = base[i * LI];
        __builtin_amdgcn_sched_barrier(0);  // the reads in flight during the weights
        float w[8];
        sinc_weights8(fr, sp, w);
        w[3] = tn == 0 ? wnear : w[3];
        w[4] = tn == 1 ? wnear : w[4];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc = make_float2(fmaf(w[i], u[i].x, acc.x), fmaf(w[i], u[i].y, acc.y));
      } else if constexpr (HALO) {
        const float2* base = ll + idx(q);  // q + KT - 1 < N + KT - 1: inside the copy
#pragma unroll
        for (int i = 0; i < KT; ++i) tap(i - KT / 2 + 1, base[i * LI]);
      } else {
#pragma unroll 2
        for (int t = -K / 2 + 1; t <= K / 2; ++t) {
          tap(t, at(q));
          if (++q == N) q = 0;
        }
      }
      v[k] = acc;
      __builtin_amdgcn_sched_barrier(0);  // one output at a time (register pressure)
    }
    __syncthreads();
    eta_screen(false);
  }
#pragma unroll
  for (int k = 0; k < E; ++k) out.st(v[k], vo, T * k * 32);
}

template <class P, int CONJ, int KT>
__global__ __launch_bounds__(P::RT, RowLds<P>::rda_waves_per_eu) void row_rda_kernel(RowArgs a) {
  if (a.gate && *a.gate == 0u) return;  // (uniform over the grid)
  __shared__ float2 lds[RowLds<P>::size];
  __shared__ float2 twl[64 + P::N / 64];
  __shared__ float2 ptab[pass_table_size<P>()];
  __shared__ float2 rtab[P::E / 2 + 1];
  load_twiddle_table<P::N>(twl, a.tw);
  load_pass_table<P>(ptab, a.tw);
  if (threadIdx.x <= P::E / 2) {  // the range screen's quadratic factors (as quad_in_slot's C)
    const double C = frac1(a.c_tau * (double)P::T * (double)P::T);
    rtab[threadIdx.x] = cis_turns(C * (double)(threadIdx.x * threadIdx.x));
  }
  __syncthreads();
  const RowLane<P> ln;
  const int units = a.na / P::LR;
  // (it stages whole lines in LDS: the host uses it with unsplit plans only;
  // the units of a block row on one XCD, as in the row pass)
  if constexpr (!P::SPLIT) {
    for (int gi = P::LR <= 2 ? xcd_logical_block() : (int)blockIdx.x; gi < units; gi += gridDim.x)
      row_rda_unit<P, CONJ, KT>(a, gi, ln, lds, twl, ptab, rtab);
  }
}

// ------------------------------------------------------ adjoint row pass --
// One unit of the adjoint row pass.  The forward chain (M for CONJ = 0, G
// for CONJ = 1) runs on the line of a.in; the opposite chain, which is its
// adjoint (Theorem 1: G = M^H, stage by stage), runs on the line of a.in2
// and is written to a.out.  At each phase stage k the derivative of the
// screen, +-i (d arg_k/d theta) exp(+-i arg_k), pairs the forward value
// a_k with the adjoint value w_k at that point:
//   d/d theta contributes  s Re(conj(w_k) i arg_k' a_k) = s arg_k' (w.y a.x - w.x a.y),
// s = +1 for M's screens, -1 for G's conjugate screens.  Because the
// screens are unimodular the product may be taken on either side of the
// screen: stage 1 pairs the forward input with the adjoint output, stage 3
// the forward value before its last screen with the adjoint value after its
// first, and stage 2 the two values in the 2-D frequency domain.  Products
// carry the factor N_a of the unnormalised azimuth spectra, removed when the
// partial sums are reduced.
__device__ __forceinline__ float dpoly(const float* c, float o) { return fmaf(fmaf(c[2], o, c[1]), o, c[0]); }

template <int E, int T, bool FREQ>
__device__ __forceinline__ void pair_stage(const float2 (&f)[E], const float2 (&w)[E], const float* dka,
                                           const float* dkr, int b, float sgn, float& acc_ka, float& acc_kr) {
  float cka[3], ckr[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cka[i] = dka[i];
    ckr[i] = dkr[i];
  }
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int kk = FREQ ? (k < E / 2 ? k : k - E) : k - E / 2;
    const float o = (float)(b + T * kk);
    const float cr = sgn * (w[k].y * f[k].x - w[k].x * f[k].y);
    acc_ka = fmaf(dpoly(cka, o), cr, acc_ka);
    acc_kr = fmaf(dpoly(ckr, o), cr, acc_kr);
  }
}

template <class P, int CONJ>
__device__ __forceinline__ void row_adj_unit(const RowArgs& a, int gi, const RowLane<P>& ln, float2* lds,
                                             const float2* twl, float& acc_ka, float& acc_kr) {
  constexpr int N = P::N, E = P::E, T = P::T, LR = P::LR;
  constexpr int LI = RowLds<P>::LI, LS = RowLds<P>::LS;
  const uint32_t S = b4_stride(N);
  const uint32_t bytes = clamp_bytes(b4_bytes(a.na, N));
  const Buf in(a.in, bytes), in2(a.in2, bytes), out(a.out, bytes);
  constexpr bool cj = CONJ != 0;
  constexpr float sgn = cj ? -1.0f : 1.0f;
  const int b = ln.b, line = ln.line;
  const int row = gi * LR + line;
  const uint32_t vo = (uint32_t)(row >> 2) * S + (uint32_t)(b >> 2) * 128u + (uint32_t)(row & 3) * 32u +
                      (uint32_t)(b & 3) * 8u;
  const double2 c1 = a.rowc1[row], c2 = a.rowc2[row], c3 = a.rowc3[row];
  const float* d = a.rowd + (size_t)row * 18;  // [theta][stage][coefficient]
  // stage index (0: arg1, 1: arg2, 2: arg3) of the forward chain's first and last screens
  constexpr int s_first = cj ? 2 : 0, s_last = cj ? 0 : 2;
  int lb = b, lc = line % LI;
  asm volatile("" : "+v"(lb), "+v"(lc));
  // the LDS line offset is kept opaque (register pressure) as an integer, so
  // the compiler still knows lds + loff is in LDS (DS, not FLAT, accesses)
  int loff = (line / LI) * LS;
  asm volatile("" : "+v"(loff));
  const TwLds tws{twl, twl + 64};
  float2 x0[E], f[E], fm[E], w[E];
#pragma unroll
  for (int k = 0; k < E; ++k) x0[k] = in.f2(vo, T * k * 32);
  // forward chain up to its last screen
#pragma unroll
  for (int k = 0; k < E; ++k) f[k] = x0[k];
  apply_quad<E, false>(f, cj ? phi3_quad(c3, a, b, T) : phi1_quad(c1, a, b, T), cj, 1.0f);
  fft_line<P, false, LI, TwLds, P::SPLIT>(f, lb, lc, lds + loff, tws);
  apply_quad<E, true>(f, phi2_quad(c2, b, T), cj, a.scale);
#pragma unroll
  for (int k = 0; k < E; ++k) fm[k] = f[k];
  asm volatile("" : "+v"(lb), "+v"(lc), "+v"(loff));
  fft_line<P, true, LI, TwLds, P::SPLIT>(f, lb, lc, lds + loff, tws);
  // adjoint chain: its first screen is the conjugate of the forward's last
#pragma unroll
  for (int k = 0; k < E; ++k) w[k] = in2.f2(vo, T * k * 32);
  apply_quad<E, false>(w, cj ? phi1_quad(c1, a, b, T) : phi3_quad(c3, a, b, T), !cj, 1.0f);
  pair_stage<E, T, false>(f, w, d + s_last * 3, d + 9 + s_last * 3, b, sgn, acc_ka, acc_kr);
  asm volatile("" : "+v"(lb), "+v"(lc), "+v"(loff));
  fft_line<P, false, LI, TwLds, P::SPLIT>(w, lb, lc, lds + loff, tws);
  pair_stage<E, T, true>(fm, w, d + 3, d + 12, b, sgn, acc_ka, acc_kr);
  apply_quad<E, true>(w, phi2_quad(c2, b, T), !cj, a.scale);
  asm volatile("" : "+v"(lb), "+v"(lc), "+v"(loff));
  fft_line<P, true, LI, TwLds, P::SPLIT>(w, lb, lc, lds + loff, tws);
  apply_quad<E, false>(w, cj ? phi3_quad(c3, a, b, T) : phi1_quad(c1, a, b, T), !cj, 1.0f);
  pair_stage<E, T, false>(x0, w, d + s_first * 3, d + 9 + s_first * 3, b, sgn, acc_ka, acc_kr);
#pragma unroll
  for (int k = 0; k < E; ++k) out.st(w[k], vo, T * k * 32);
}

template <class P, int CONJ>
__global__ __launch_bounds__(P::RT) void row_adj_kernel(RowArgs a) {
  __shared__ float2 lds[RowLds<P>::size];
  __shared__ float2 twl[64 + P::N / 64];
  __shared__ float red[P::RT / 64];
  load_twiddle_table<P::N>(twl, a.tw);
  __syncthreads();
  const RowLane<P> ln;
  const int units = a.na / P::LR;
  float acc_ka = 0.f, acc_kr = 0.f;
  for (int gi = xcd_logical_block(); gi < units; gi += gridDim.x)
    row_adj_unit<P, CONJ>(a, gi, ln, lds, twl, acc_ka, acc_kr);
  const float s0 = block_sum<P::RT>(acc_ka, red);
  if (threadIdx.x == 0) a.partials[2 * blockIdx.x] = s0;
  const float s1 = block_sum<P::RT>(acc_kr, red);
  if (threadIdx.x == 0) a.partials[2 * blockIdx.x + 1] = s1;
}

// ---------------------------------------------------------- column pass --
// One tile (C adjacent columns) of a column pass of array a.  Returns the
// thread's share of the tile's squared norm (FWD with the mask, R).
// Software pipelining: the next tile's first input (Xt for the update pass,
// W for the residual pass) is loaded while this tile is transformed, into
// registers that are free at that point, so one workgroup per compute unit
// keeps HBM busy during its FFTs.  The residual pass has room for it only
// with 32 elements per thread and at least 4 columns per tile (256 VGPRs
// per lane at two waves per SIMD); split plans get the overlap from a second
// workgroup instead.
template <class P, int MODE>
constexpr bool col_pipelined() {
  return (MODE == COL_A || ((MODE == COL_R || MODE == COL_AS) && P::E >= 32 && P::C >= 4) || MODE == COL_D ||
          MODE == COL_N) &&
         !P::SPLIT;
}

// Column passes whose twiddles come precomputed per thread (hoisted_pass,
// table_pass): the update and residual passes of unsplit plans.
template <class P, int MODE>
constexpr bool col_hoisted() {
  return (MODE == COL_A || MODE == COL_AS || MODE == COL_R) && hoisted_pass<P>() >= 0 && !P::SPLIT;
}

template <class P, int MODE>
__device__ __forceinline__ void col_preload(const ColArgs& a, int tile, int b, int c, float2 (&pre)[P::E]) {
  constexpr int E = P::E, T = P::T, C = P::C;
  const uint32_t b4b = clamp_bytes(b4_bytes(P::N, a.nr));
  const Addr ab = col_addr(B4, b, tile * C + c, T, a.nr);
  if constexpr (MODE == COL_A) {
    if (a.flags & 1) return;  // first iteration: no Xt
    const Buf in0(a.in0, b4b);
#pragma unroll
    for (int k = 0; k < E; ++k) pre[k] = in0.f2(ab.voff, k * ab.kstep);
  } else if constexpr (MODE == COL_R || MODE == COL_D || MODE == COL_N) {
    const Buf in0(a.in0, b4b);
#pragma unroll
    for (int k = 0; k < E; ++k) pre[k] = in0.f2(ab.voff, k * ab.kstep);
  } else if constexpr (MODE == COL_AS) {
    const Buf in1(a.in1, b4b);
#pragma unroll
    for (int k = 0; k < E; ++k) pre[k] = in1.f2(ab.voff, k * ab.kstep);
  }
}

// Packed sampling mask: bit e % 32 of word e / 32, e = blocked element index
// of (i, j).  Byte offset and bit of element (b, j), and the byte step per k
// (element b + T k; T N_r is a multiple of 32).
struct MaskAddr {
  uint32_t moff, bit, kstep;
};
__device__ __forceinline__ MaskAddr mask_addr(int b, int j, int T, int nr) {
  const uint32_t e0 = (((uint32_t)(b >> 2) * (nr / 4) + (j >> 2)) << 4) + ((b & 3) << 2) + (j & 3);
  return {(e0 >> 5) * 4u, e0 & 31u, (uint32_t)T * (uint32_t)nr / 32u * 4u};
}

// ------------------------------------------------ sparse-iterate update --
// The update pass with the iterate X kept spatially and sparsely (the
// thresholded iterate of a sparse scene has few nonzeros).  Each thread of a
// column tile owns E elements of X (b + T k, k < E, of its column).  A
// thread with nonzeros keeps a 32-byte record (its support word, bit k:
// element k is nonzero, and its first two nonzero values in rank order); a
// thread with more than two stores its E values densely in xdense (B4) and
// the word kDenseWord in its record; a thread without nonzeros stores
// nothing.  Per wave, a 64-bit mask of the lanes that hold a record (one
// 8-byte word, stored by lane 0).  A wave's records are packed at the start
// of its 64-record area, in lane order (a lane's slot is the number of
// flagged lanes below it), so the few records of a wave share one or two
// cache lines instead of one line each.  The pass reads the wave mask
// first, then Z, then the records of the flagged lanes only: buffer
// accesses past the end of the buffer are dropped without a memory access,
// so the lanes without a record take an address past the end, and no branch
// is needed.  No wave reads another's records, so the pass needs no
// workgroup-wide step.
//   V = F_eta^-1[Z] mu / N_a + X  ->  X+ = S_sigma(V)  ->  X+ (sparse) and
//   F_eta X+ into out (B4, in place over Z: the next row pass of G reads
//   it), or X+ row-major (flag 2: the last iteration; flag 1: X = 0).
// Bytes per pixel: Z read and F_eta X+ written (16), 8 bytes per wave each
// way, and 32 bytes per thread with nonzeros each way.
constexpr uint32_t kDenseWord = 0xFFFFFFFFu;  // (a sparse record has at most two bits)
// A buffer offset past the end of the record and mask buffers (at most
// 2 bytes per pixel: 134 MB at 8192 x 8192), with room for the 16-byte
// offsets added to it.
constexpr uint32_t kPastEnd = 0xF0000000u;

// The end of the sparse-iterate update (defined below).
template <class P, int HSC>
__device__ __forceinline__ void sparse_store(const ColArgs& a, int tile, int b, int c, float2* lds,
                                             const TwLds& tws, const TwPowers& hp, float2 (&v)[P::E],
                                             uint32_t m_new, int lb, int lc);

// PIPE: Z of this tile was loaded into pre during the previous tile, and Z
// of the next tile (next >= 0) is loaded into pre during this one.
template <class P, bool HT, bool PIPE>
__device__ __forceinline__ void col_update_sparse(const ColArgs& a, int tile, int b, int c, float2* lds,
                                                  const float2* twl, const TwPowers& hp,
                                                  float2 (&pre)[P::E], int next) {
  constexpr int HSC = HT ? hoisted_pass<P>() : -1;
  constexpr int N = P::N, E = P::E, T = P::T, C = P::C, CT = P::CT, W = CT / 64;
  static_assert(E <= 32, "support word holds E bits");
  const uint32_t b4b = clamp_bytes(b4_bytes(N, a.nr));
  const bool first = a.flags & 1;
  const int j = tile * C + c;
  const Addr ab = col_addr(B4, b, j, T, a.nr);
  const Buf zin(a.in1, b4b), xd(a.xdense, b4b);
  const uint32_t ntiles = (uint32_t)(a.nr / C);
  const Buf recs(a.xrec, clamp_bytes((size_t)ntiles * CT * 32));
  const Buf wmasks(a.xwmask, clamp_bytes((size_t)ntiles * W * 8));
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t wave_rec = ((uint32_t)tile * CT + (threadIdx.x & ~63u)) * 32u;  // the wave's area
  const uint32_t wm_off = ((uint32_t)tile * W + wid) * 8u;
  // the wave's mask, then Z, then the records of the flagged lanes
  uint32_t wm_lo = 0, wm_hi = 0;
  if (!first) {
    const auto w2 = __builtin_amdgcn_raw_buffer_load_b64(wmasks.r, wm_off, 0, 0);
    wm_lo = w2[0];
    wm_hi = w2[1];
  }
  const float ms = a.mu * a.scale;
  float2 v[E];
#pragma unroll
  for (int k = 0; k < E; ++k) v[k] = PIPE ? pre[k] : zin.f2(ab.voff, k * ab.kstep);
  if constexpr (PIPE) {
    if (next >= 0) col_preload<P, COL_AS>(a, next, b, c, pre);
  }
  __builtin_amdgcn_sched_barrier(0);
  const bool has = ((lane < 32 ? wm_lo >> lane : wm_hi >> (lane - 32)) & 1u) != 0u;
  const uint32_t ro = has ? wave_rec + 32u * __builtin_amdgcn_mbcnt_hi(wm_hi, __builtin_amdgcn_mbcnt_lo(wm_lo, 0u))
                          : kPastEnd;
  const float4 r0 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(recs.r, ro, 0, 0));
  const float4 r1 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(recs.r, ro + 16u, 0, 0));
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < E; ++k) v[k] = cscale(v[k], ms);
  const TwLds tws{twl, twl + 64};
  int lb = b, lc = c;
  asm volatile("" : "+v"(lb), "+v"(lc));  // recompute LDS addresses per tile
  fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
  // V = ... + X.  Nonzeros are rare, so each element's addition and capture
  // below run only where some lane of the wave needs them (a wave-uniform
  // branch on the ballot), not as selects in every lane.
  const uint32_t m_old = __float_as_uint(r0.x);  // (0 for a lane without a record)
  if (m_old == kDenseWord) {
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = cadd(v[k], xd.f2(ab.voff, k * ab.kstep));
  } else {
    const uint32_t k0 = m_old & (0u - m_old);  // lowest set bit: the first value
    if (__ballot(m_old != 0u)) {
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const bool bit = (m_old >> k) & 1u;
        const float2 x = (k0 >> k) & 1u ? make_float2(r0.y, r0.z) : make_float2(r1.x, r1.y);
        v[k] = cadd(v[k], bit ? x : make_float2(0.f, 0.f));
      }
    }
  }
  // X+ = S_sigma(V) (the arithmetic of the azimuth-spectrum update pass);
  // the support and the first two nonzeros as they come
  // (the threshold in one branch-free block, so the reciprocal square roots
  // of all elements are in flight together; the capture after it)
  const float s2 = a.sigma * a.sigma;
  uint32_t m_new = 0;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const float m2 = fmaf(v[k].x, v[k].x, v[k].y * v[k].y);
    const bool keep = m2 > s2;
    const float f = keep ? fmaf(-a.sigma, rsqrtf(m2), 1.0f) : 0.0f;
    v[k] = cscale(v[k], f);
    m_new |= keep ? 1u << k : 0u;
  }
  sparse_store<P, HSC>(a, tile, b, c, lds, tws, hp, v, m_new, lb, lc);
}

// The end of the sparse-iterate update for X+ in v (support bits m_new):
// the record or the dense store and the wave's mask, then F_eta X+ into out
// (B4); or, with flag 2, X+ row-major into out.
template <class P, int HSC>
__device__ __forceinline__ void sparse_store(const ColArgs& a, int tile, int b, int c, float2* lds,
                                             const TwLds& tws, const TwPowers& hp, float2 (&v)[P::E],
                                             uint32_t m_new, int lb, int lc) {
  constexpr int N = P::N, E = P::E, T = P::T, C = P::C, CT = P::CT, W = CT / 64;
  const uint32_t b4b = clamp_bytes(b4_bytes(N, a.nr));
  const int j = tile * C + c;
  const Addr ab = col_addr(B4, b, j, T, a.nr);
  const Buf xd(a.xdense, b4b);
  const uint32_t ntiles = (uint32_t)(a.nr / C);
  const Buf recs(a.xrec, clamp_bytes((size_t)ntiles * CT * 32));
  const Buf wmasks(a.xwmask, clamp_bytes((size_t)ntiles * W * 8));
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t wave_rec = ((uint32_t)tile * CT + (threadIdx.x & ~63u)) * 32u;  // the wave's area
  const uint32_t wm_off = ((uint32_t)tile * W + wid) * 8u;
  float2 x0 = make_float2(0.f, 0.f), x1 = x0;
  const uint32_t n0 = m_new & (0u - m_new);  // lowest set bit: the first value
  const uint32_t n1 = (m_new ^ n0) & (0u - (m_new ^ n0));  // the second
  if (__ballot(m_new != 0u)) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      x0 = (n0 >> k) & 1u ? v[k] : x0;
      x1 = (n1 >> k) & 1u ? v[k] : x1;
    }
  }
  if (a.flags & 2) {  // the last iteration: X+ row-major
    const Buf out(a.out, clamp_bytes((size_t)N * a.nr * 8));
    const Addr ar = col_addr(RM, b, j, T, a.nr);
#pragma unroll
    for (int k = 0; k < E; ++k) out.st(v[k], ar.voff, k * ar.kstep);
    return;
  }
  // the record (or the dense store) and the wave's mask
  const bool dense = __builtin_popcount(m_new) > 2;
  const uint32_t word = dense ? kDenseWord : m_new;
  const unsigned long long nz = __ballot(m_new != 0u);
  const uint32_t wo = m_new ? wave_rec + 32u * __builtin_amdgcn_mbcnt_hi((uint32_t)(nz >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)nz, 0u))
                            : kPastEnd;
  using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(recs.r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b128(
      __builtin_bit_cast(V4, make_float4(__uint_as_float(word), x0.x, x0.y, 0.f)), recs.r, wo, 0, 0);
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, make_float4(x1.x, x1.y, 0.f, 0.f)), recs.r,
                                         wo + 16u, 0, 0);
  if (__ballot(dense)) {
    if (dense) {
#pragma unroll
      for (int k = 0; k < E; ++k) xd.st(v[k], ab.voff, k * ab.kstep);
    }
  }
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(wmasks.r, 0u, 0u, 0));
  V2 wv;
  wv[0] = (uint32_t)nz;
  wv[1] = (uint32_t)(nz >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(wv, wmasks.r, lane == 0 ? wm_off : kPastEnd, 0, 0);
  asm volatile("" : "+v"(lb), "+v"(lc));
  fft_line<P, false, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);  // F_eta X+
  const Buf out(a.out, b4b);
#pragma unroll
  for (int k = 0; k < E; ++k) out.st(v[k], ab.voff, k * ab.kstep);
}

// Warm start of the sparse iterate: X+ given row-major in in0 (its
// support = its nonzero elements) is stored as the update pass stores its
// result, and F_eta X+ goes to out, so that a solve goes on from X+ exactly
// as after an update pass that produced it.
template <class P, bool HT>
__device__ __forceinline__ void col_warm_sparse(const ColArgs& a, int tile, int b, int c, float2* lds,
                                                const float2* twl, const TwPowers& hp) {
  constexpr int HSC = HT ? hoisted_pass<P>() : -1;
  constexpr int N = P::N, E = P::E, T = P::T, C = P::C;
  const Buf xin(a.in0, clamp_bytes((size_t)N * a.nr * 8));
  const Addr ar = col_addr(RM, b, tile * C + c, T, a.nr);
  float2 v[E];
  uint32_t m_new = 0;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    v[k] = xin.f2(ar.voff, k * ar.kstep);
    m_new |= (v[k].x != 0.0f || v[k].y != 0.0f) ? 1u << k : 0u;
  }
  const TwLds tws{twl, twl + 64};
  sparse_store<P, HSC>(a, tile, b, c, lds, tws, hp, v, m_new, b, c);
}

// HT: the twiddles of the passes a thread can precompute come from hp
// (hoisted_pass, table_pass).
template <class P, int MODE, bool PIPE = false, bool HT = false>
__device__ __forceinline__ float col_unit(const ColArgs& a, int tile, int b, int c, float2* lds,
                                          const float2* twl, float2 (&pre)[P::E], int next,
                                          const TwPowers& hp, unsigned* hist0 = nullptr,
                                          unsigned* chg = nullptr) {
  constexpr int HSC = HT ? hoisted_pass<P>() : -1;
  constexpr int N = P::N, E = P::E, T = P::T, C = P::C;
  const uint32_t rmb = clamp_bytes((size_t)N * a.nr * 8), b4b = clamp_bytes(b4_bytes(N, a.nr));
  constexpr int in_layout = MODE == COL_FWD ? RM : B4;
  const int out_layout =
      (MODE == COL_INV || ((MODE == COL_A || MODE == COL_T) && (a.flags & 2))) ? RM : B4;
  const Buf in0(a.in0, in_layout == RM ? rmb : b4b), in1(a.in1, b4b), yb(a.y, b4b);
  const Buf out(a.out, out_layout == RM ? rmb : b4b), out2(a.out2, b4b);
  const bool first = (MODE == COL_A || MODE == COL_VB || MODE == COL_V) && (a.flags & 1);
  const int j = tile * C + c;
  const Addr ai = col_addr(in_layout, b, j, T, a.nr);
  const Addr ab = col_addr(B4, b, j, T, a.nr);
  float acc = 0.f;
  float2 v[E], y2[E];
  float2 y3[(MODE == COL_VB || MODE == COL_U || MODE == COL_XB) ? E : 1];
  if constexpr (MODE == COL_A || MODE == COL_VB || MODE == COL_V) {
    // V = F^-1[Xt + mu Z] / N_a
    const float ms = (MODE == COL_V ? a.ad->mu : a.mu) * a.scale;
    if constexpr (!PIPE) {
      // both inputs in flight together (all of Z, then all of Xt), combined
      // once both arrived; on the first iteration Xt is read through an
      // empty range (every load returns 0, no access).  (Loading Xt only
      // after Z had arrived cost the batched solver 12 % of its iteration
      // time.)
      const Buf x0(a.in0, first ? 0u : b4b);
      float2 z[E];
#pragma unroll
      for (int k = 0; k < E; ++k) z[k] = in1.f2(ai.voff, k * ai.kstep);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = x0.f2(ai.voff, k * ai.kstep);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const float2 zs = cscale(z[k], ms);
        v[k] = first ? zs : make_float2(fmaf(a.scale, v[k].x, zs.x), fmaf(a.scale, v[k].y, zs.y));
      }
    } else {
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = cscale(in1.f2(ai.voff, k * ai.kstep), ms);
    if (!first) {
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const float2 x = PIPE ? pre[k] : in0.f2(ai.voff, k * ai.kstep);
        v[k] = make_float2(fmaf(a.scale, x.x, v[k].x), fmaf(a.scale, x.y, v[k].y));
      }
    }
    }
    if constexpr (PIPE && MODE == COL_A) {
      if (next >= 0) col_preload<P, MODE>(a, next, b, c, pre);
    }
    if constexpr (MODE == COL_VB) {
#pragma unroll
      for (int k = 0; k < E; ++k) y3[k] = yb.f2(ab.voff, k * ab.kstep);  // Xbar of X+
    }
  } else if constexpr (MODE == COL_FWD || MODE == COL_T) {
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = in0.f2(ai.voff, k * ai.kstep);
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = cscale(PIPE ? pre[k] : in0.f2(ai.voff, k * ai.kstep), a.scale);
    // the single-input adaptive passes load the next tile's input at once
    // (in flight during both transforms of this one)
    if constexpr (PIPE && (MODE == COL_D || MODE == COL_N)) {
      if (next >= 0) col_preload<P, MODE>(a, next, b, c, pre);
    }
    // (split plans and screened passes load m o y after the inverse
    // transform: registers)
    if constexpr ((MODE == COL_R && !P::SPLIT && !HT) || MODE == COL_U) {
#pragma unroll
      for (int k = 0; k < E; ++k) y2[k] = yb.f2(ab.voff, k * ab.kstep);
    }
    if constexpr (MODE == COL_U || MODE == COL_XB) {
#pragma unroll
      for (int k = 0; k < E; ++k) y3[k] = in1.f2(ab.voff, k * ab.kstep);
    }
  }
  const TwLds tws{twl, twl + 64};
  int lb = b, lc = c;
  asm volatile("" : "+v"(lb), "+v"(lc));  // recompute LDS addresses per tile
  if constexpr (MODE == COL_FWD) {
    if (a.flags & 1) {
      const Buf mask(a.mask, clamp_bytes(((size_t)N * a.nr + 31) / 32 * 4));
      const MaskAddr ma = mask_addr(b, j, T, a.nr);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const uint32_t w = mask.u32(ma.moff, k * ma.kstep);
        const bool keep = (w >> ma.bit) & 1u;
        if (!keep) v[k] = make_float2(0.f, 0.f);
        acc = fmaf(v[k].x, v[k].x, fmaf(v[k].y, v[k].y, acc));
        if (a.flags & 4)
          out2.st(keep ? v[k] : make_float2(__uint_as_float(kUnsampled), 0.f), ab.voff, k * ab.kstep);
      }
    }
    fft_line<P, false, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
  } else if constexpr (MODE == COL_INV) {
    fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
  } else if constexpr (MODE == COL_A) {
    fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
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
      fft_line<P, false, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);  // Xt+ = F X+
    }
  } else if constexpr (MODE == COL_VB) {
    // Vbar = J_S(V)^T Xbar (the threshold's real Jacobian, symmetric):
    // on |V| > sigma, (1 - sigma/|V|) Xbar + sigma Re(conj(V) Xbar) V / |V|^3;
    // d X+ / d sigma = -V/|V| gives the partial -Re(conj(V) Xbar)/|V|.
    // The support test is the update pass's, on the same V.
    fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
    const float s2 = a.sigma * a.sigma;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const float m2 = fmaf(v[k].x, v[k].x, v[k].y * v[k].y);
      const float2 xb = y3[k];
      float2 vb = make_float2(0.f, 0.f);
      if (m2 > s2) {
        const float inv = rsqrtf(m2);
        const float dot = fmaf(v[k].x, xb.x, v[k].y * xb.y);
        const float f = fmaf(-a.sigma, inv, 1.0f);
        const float g = a.sigma * dot * inv * inv * inv;
        vb = make_float2(fmaf(f, xb.x, g * v[k].x), fmaf(f, xb.y, g * v[k].y));
        acc = fmaf(-dot, inv, acc);
      }
      out2.st(vb, ab.voff, k * ab.kstep);
      v[k] = cscale(vb, a.mu);
    }
    asm volatile("" : "+v"(lb), "+v"(lc));
    fft_line<P, false, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);  // F (mu Vbar)
  } else if constexpr (MODE == COL_U) {
    // g = F^-1[F G mu Vbar] / N_a; ybar += m o g; ubar = -m o g; out = F ubar
    fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const bool keep = __float_as_uint(y2[k].x) != kUnsampled;
      const float2 g = keep ? v[k] : make_float2(0.f, 0.f);
      out2.st(cadd(y3[k], g), ab.voff, k * ab.kstep);
      v[k] = make_float2(-g.x, -g.y);
    }
    asm volatile("" : "+v"(lb), "+v"(lc));
    fft_line<P, false, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
  } else if constexpr (MODE == COL_XB) {
    // Xbar = Vbar + F^-1[F M ubar] / N_a (spatial)
    fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = cadd(y3[k], v[k]);
  } else if constexpr (MODE == COL_D) {
    // dX = F^-1[Z] / N_a; dX_G = dX on the support of the iterate; out = F dX_G
    static_assert(E <= 32, "support word holds E bits");
    fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
    const uint32_t w = a.supp[(uint32_t)tile * P::CT + threadIdx.x];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      if (!((w >> k) & 1u)) v[k] = make_float2(0.f, 0.f);
      acc = fmaf(v[k].x, v[k].x, fmaf(v[k].y, v[k].y, acc));
    }
    asm volatile("" : "+v"(lb), "+v"(lc));
    fft_line<P, false, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
  } else if constexpr (MODE == COL_N) {
    // g = F^-1[W] / N_a (= G dX_G); ||m o g||^2 (no output)
    fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
    const Buf mask(a.mask, clamp_bytes(((size_t)N * a.nr + 31) / 32 * 4));
    const MaskAddr ma = mask_addr(b, j, T, a.nr);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const bool keep = (mask.u32(ma.moff, k * ma.kstep) >> ma.bit) & 1u;
      const float e2 = fmaf(v[k].x, v[k].x, v[k].y * v[k].y);
      acc += keep ? e2 : 0.f;
    }
  } else if constexpr (MODE == COL_V) {
    fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);  // V (spatial)
    // first level of the selection of the threshold: histogram of the top
    // 11 bits of |V|^2 (computed as the selection and threshold passes do)
    auto key = [&](int k) { return __float_as_uint(fmaf(v[k].x, v[k].x, v[k].y * v[k].y)); };
#pragma unroll
    for (int k = 0; k < E; ++k) atomicAdd(&hist0[key(k) >> 21], 1u);
    // the keys in the candidate window, into this workgroup's segment,
    // packed per wave (an LDS atomic per wave for the wave's slots, the
    // workgroup's count after the histogram; keys past the segment are
    // counted, not stored)
    AdaptState* st = a.ad;
    const unsigned wlo = st->wlo, whi = st->whi;
    auto in_win = [&](int k) {
      const unsigned bin = key(k) >> 21;
      return bin >= wlo && bin <= whi;
    };
    unsigned tot = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) tot += (unsigned)__popcll(__ballot(in_win(k)));
    if (tot) {  // (uniform over the wave)
      const uint64_t act = __ballot(1);
      const unsigned lane_rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
      unsigned base = 0;
      if (lane_rank == 0) base = atomicAdd(&hist0[2048], tot);
      base = __builtin_amdgcn_readfirstlane(base);
      const unsigned seg = st->seg;
      unsigned* cand = adapt_candidates(st) + (size_t)blockIdx.x * seg;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const bool in = in_win(k);
        const uint64_t bal = __ballot(in);
        const unsigned idx = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (in && idx < seg) cand[idx] = key(k);
        base += (unsigned)__popcll(bal);
      }
    }
  } else if constexpr (MODE == COL_T) {
    // X+ = S_sigma(V): kept where |V|^2 > sigma^2 (sigma^2 the selected
    // (k+1)-th largest |V|^2, computed the same way); support bit = X+ != 0
    static_assert(E <= 32, "support word holds E bits");
    const float sg = a.ad->sigma, s2 = a.ad->sigma2;
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const float m2 = fmaf(v[k].x, v[k].x, v[k].y * v[k].y);
      const float f = m2 > s2 ? fmaxf(fmaf(-sg, rsqrtf(m2), 1.0f), 0.0f) : 0.0f;
      v[k] = cscale(v[k], f);
      w |= (f > 0.0f ? 1u : 0u) << k;
    }
    const uint32_t widx = (uint32_t)tile * P::CT + threadIdx.x;
    a.supp[widx] = w;
    if (a.flags & 4) {
      if (w != a.supp_old[widx]) *chg = 1u;
    }
    if (a.flags & 16) {
      const Buf o3(a.out3, rmb);
      const Addr ar = col_addr(RM, b, j, T, a.nr);
#pragma unroll
      for (int k = 0; k < E; ++k) o3.st(v[k], ar.voff, k * ar.kstep);
    }
    if (!(a.flags & 2)) fft_line<P, false, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
  } else {  // COL_R: GX = F^-1[W] / N_a; R = m o y - m o GX; out = F R
    fft_line<P, true, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
    // split plans, screened passes: m o y in chunks of 8 after the transform
    constexpr bool late = P::SPLIT || HT;
    constexpr int YC = late ? 8 : E;
#pragma unroll
    for (int k0 = 0; k0 < E; k0 += YC) {
      if constexpr (late) {
#pragma unroll
        for (int k = k0; k < k0 + YC; ++k) y2[k] = yb.f2(ab.voff, k * ab.kstep);
      }
#pragma unroll
      for (int k = k0; k < k0 + YC; ++k) {
        const float2 yk = y2[k];
        const bool keep = __float_as_uint(yk.x) != kUnsampled;
        const float2 r = keep ? csub(yk, v[k]) : make_float2(0.f, 0.f);
        acc = fmaf(r.x, r.x, fmaf(r.y, r.y, acc));
        v[k] = r;
      }
      if constexpr (late) __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (PIPE) {
      if (next >= 0) col_preload<P, MODE>(a, next, b, c, pre);
    }
    asm volatile("" : "+v"(lb), "+v"(lc));
    fft_line<P, false, C, TwLds, 0, HSC, P::SPLIT>(v, lb, lc, lds, tws, hp);
  }
  if constexpr (MODE != COL_N) {
    const Addr ao = out_layout == RM ? col_addr(RM, b, j, T, a.nr) : ab;
#pragma unroll
    for (int k = 0; k < E; ++k) out.st(v[k], ao.voff, k * ao.kstep);
  }
  return acc;
}

// Column passes keep a whole tile in LDS (one workgroup per CU), or half of
// it with the split exchange (two workgroups per CU: 4 waves per SIMD).
template <class P>
struct ColLds {
  static constexpr int size = LdsSize<P::C, P::SPLIT ? P::N / 2 : P::N>::value;
  // workgroups per CU the LDS allows (160 KB, some for twiddles and sums)
  static constexpr int wgs = size * 8 <= 78 * 1024 ? 2 : 1;
  static constexpr int waves_per_eu = P::SPLIT ? wgs * P::CT / 256 : 1;
};

template <class P, int MODE>
__global__ __launch_bounds__(P::CT, ColLds<P>::waves_per_eu) void col_pass_kernel(ColArgs a) {
  constexpr int C = P::C, CT = P::CT;
  if (a.gate && *a.gate == 0u) return;  // (uniform over the grid)
  __shared__ float2 lds[ColLds<P>::size];
  __shared__ float2 twl[64 + P::N / 64];
  __shared__ float red[CT / 64];
  __shared__ float2 ptab[pass_table_size<P>()];
  load_twiddle_table<P::N>(twl, a.tw);
  load_pass_table<P>(ptab, a.tw);
  __syncthreads();
  const int c = threadIdx.x % C;
  const int b = threadIdx.x / C;
  const int ntiles = a.nr / C;  // N_r is a multiple of C
  // the update and residual passes take the twiddles a thread can
  // precompute from registers and a small LDS table (set up once here)
  // instead of the prefetch
  constexpr bool HT = col_hoisted<P, MODE>();
  constexpr bool PIPE = col_pipelined<P, MODE>() && !HT;
  TwPowers hp;
  if constexpr (HT) hp = hoist_powers<P>(b, TwLds{twl, twl + 64}, ptab);
  float acc = 0.f;
  unsigned chg = 0u;
  float2 pre[P::E];
  // the value pass (adaptive threshold) also counts the first selection level
  // (and, after the 2048 bins, its count of selection candidates)
  __shared__ unsigned hist0[MODE == COL_V ? 2049 : 1];
  if constexpr (MODE == COL_V) {
    for (int i = threadIdx.x; i < 2049; i += CT) hist0[i] = 0u;
    __syncthreads();
  }
  int tile = xcd_logical_block();
  if constexpr (MODE == COL_AS) {
    if (a.flags & 8) {  // warm start of the sparse iterate (its own loop)
      for (; tile < ntiles; tile += gridDim.x) col_warm_sparse<P, HT>(a, tile, b, c, lds, twl, hp);
      return;
    }
  }
  if constexpr (PIPE) {
    if (tile < ntiles) col_preload<P, MODE>(a, tile, b, c, pre);
  }
  for (; tile < ntiles; tile += gridDim.x) {
    const int next = tile + (int)gridDim.x < ntiles ? tile + (int)gridDim.x : -1;
    if constexpr (MODE == COL_AS) col_update_sparse<P, HT, PIPE>(a, tile, b, c, lds, twl, hp, pre, next);
    else acc += col_unit<P, MODE, PIPE, HT>(a, tile, b, c, lds, twl, pre, next, hp, hist0, &chg);
  }
  if constexpr (MODE == COL_V) {
    __syncthreads();
    for (int i = threadIdx.x; i < 2048; i += CT)
      if (hist0[i]) atomicAdd(&a.ad->hist[i], hist0[i]);
    if (threadIdx.x == 0 && blockIdx.x < (unsigned)kMaxCandSeg) adapt_cand_counts(a.ad)[blockIdx.x] = hist0[2048];
  }
  if constexpr (MODE == COL_R) {
    // ||R||^2: one partial per block, summed by a one-block kernel launched
    // after this pass (a last-block reduction here would need a device-scope
    // fence per block, which writes back the L2 and waits for this block's
    // stores: 13 us of a 102 us pass at 4096 x 4096)
    const float part = block_sum<CT>(acc, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = part;
  }
  if (MODE == COL_FWD && (a.flags & 1)) {  // ||m o y||^2 (the first residual), as for R
    const float part = block_sum<CT>(acc, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = part;
  }
  if constexpr (MODE == COL_VB) {
    const float part = block_sum<CT>(acc, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = part;  // reduced by reduce_partials_kernel
  }
  if constexpr (MODE == COL_T) {
    // safeguard: whether the support moved (any block); the shrink loop goes
    // on only after a support change (a one-block kernel after this pass
    // sets the loop's flag)
    if (a.flags & 4) {
      if (__syncthreads_or((int)chg) && threadIdx.x == 0) atomicOr(&a.ad->changed, 1u);
    }
  }
  if constexpr (MODE == COL_D) {
    // ||dX_G||^2: per-block partials, totalled by a one-block kernel after
    // this pass (as for the residual pass: this pass writes a whole array)
    const float part = block_sum<CT>(acc, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = part;
  }
  if constexpr (MODE == COL_N) {
    // ||m o G dX_G||^2 (or ||m o G(X+ - X)||^2 for the safeguard's bound):
    // per-block partials; the step or the bound test follow in a one-block
    // kernel after this pass
    const float part = block_sum<CT>(acc, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = part;
  }
}

// Grouped column pass (batched solver): no norms are formed.
template <class P, int MODE>
__global__ __launch_bounds__(P::CT, ColLds<P>::waves_per_eu) void col_group_kernel(GroupArgs g) {
  constexpr int C = P::C;
  __shared__ float2 lds[ColLds<P>::size];
  __shared__ float2 twl[64 + P::N / 64];
  const ColArgs* __restrict__ args = (const ColArgs*)g.args;
  __shared__ float2 ptab[pass_table_size<P>()];
  load_twiddle_table<P::N>(twl, args[0].tw);
  load_pass_table<P>(ptab, args[0].tw);
  __syncthreads();
  const int c = threadIdx.x % C;
  const int b = threadIdx.x / C;
  float2 pre[P::E];
  // same per-line arithmetic as the single-array kernel (bit-identical results)
  constexpr bool HT = col_hoisted<P, MODE>();
  TwPowers hp;
  if constexpr (HT) hp = hoist_powers<P>(b, TwLds{twl, twl + 64}, ptab);
  for (int u = xcd_logical_block(); u < g.total; u += gridDim.x) {
    const int s = group_find(g.start, g.count, u);
    if constexpr (MODE == COL_AS)
      col_update_sparse<P, HT, false>(args[s], u - g.start[s], b, c, lds, twl, hp, pre, -1);
    else (void)col_unit<P, MODE, false, HT>(args[s], u - g.start[s], b, c, lds, twl, pre, -1, hp);
  }
}

// Host-side launch helpers (one set per plan, instantiated in kern_inst.hip).
template <class P>
struct Kernels {
  static hipError_t row(const RowArgs& a, int grid, hipStream_t s) {
    if (a.conj)
      hipLaunchKernelGGL((row_pass_kernel<P, 1>), dim3(grid), dim3(P::RT), 0, s, a);
    else
      hipLaunchKernelGGL((row_pass_kernel<P, 0>), dim3(grid), dim3(P::RT), 0, s, a);
    return hipGetLastError();
  }
  template <int MODE>
  static hipError_t col(const ColArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((col_pass_kernel<P, MODE>), dim3(grid), dim3(P::CT), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t row_group(const GroupArgs& g, int grid, hipStream_t s) {
    if (g.conj)
      hipLaunchKernelGGL((row_group_kernel<P, 1>), dim3(grid), dim3(P::RT), 0, s, g);
    else
      hipLaunchKernelGGL((row_group_kernel<P, 0>), dim3(grid), dim3(P::RT), 0, s, g);
    return hipGetLastError();
  }
  // range-Doppler row pass: 8 taps (the default) unrolled, other counts generic
  template <int CONJ>
  static hipError_t row_rda(const RowArgs& a, int grid, hipStream_t s) {
    if (a.taps == 8)
      hipLaunchKernelGGL((row_rda_kernel<P, CONJ, 8>), dim3(grid), dim3(P::RT), 0, s, a);
    else
      hipLaunchKernelGGL((row_rda_kernel<P, CONJ, 0>), dim3(grid), dim3(P::RT), 0, s, a);
    return hipGetLastError();
  }
  template <int CONJ>
  static hipError_t row_adj(const RowArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((row_adj_kernel<P, CONJ>), dim3(grid), dim3(P::RT), 0, s, a);
    return hipGetLastError();
  }
  template <int MODE>
  static hipError_t col_group(const GroupArgs& g, int grid, hipStream_t s) {
    hipLaunchKernelGGL((col_group_kernel<P, MODE>), dim3(grid), dim3(P::CT), 0, s, g);
    return hipGetLastError();
  }
};

}  // namespace cssar
