// Device-side building blocks for gfx950 (CDNA4, wave64): complex helpers,
// register radix kernels, LDS-staged Stockham FFT passes, FP64-argument
// phase generation and the fused row/column pass kernels of one
// approximated-observation operator application or ITA iteration.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cssar_plan.hpp"

namespace cssar {

// ---------------------------------------------------------------- complex --
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV> __device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// --------------------------------------------------------- radix kernels --
// In-place DFT of R values held in registers: out[k] = sum_n in[n] w^(n k),
// w = exp(-2 pi i / R) (forward) or its conjugate (INV).
template <bool INV> __device__ __forceinline__ void dft2(float2& a0, float2& a1) {
  float2 t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2& a0, float2& a1, float2& a2) {
  const float h = 0.86602540378443864676f;  // sqrt(3)/2
  float2 t = cadd(a1, a2), d = csub(a1, a2);
  float2 m = make_float2(fmaf(-0.5f, t.x, a0.x), fmaf(-0.5f, t.y, a0.y));
  // -i h d (forward) / +i h d (inverse)
  float2 r = mul_mi<INV>(cscale(d, h));
  a0 = cadd(a0, t);
  a1 = cadd(m, r);
  a2 = csub(m, r);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* a) {
  // even/odd split: E = DFT4(a0,a2,a4,a6), O = DFT4(a1,a3,a5,a7),
  // X[k] = E[k] + w8^k O[k], X[k+4] = E[k] - w8^k O[k]
  dft4<INV>(a[0], a[2], a[4], a[6]);
  dft4<INV>(a[1], a[3], a[5], a[7]);
  const float r = 0.70710678118654752440f;
  float2 o1 = a[3], o2 = a[5], o3 = a[7];
  // w8^1 = (1 - i)/sqrt2 (fwd), (1 + i)/sqrt2 (inv)
  o1 = INV ? make_float2((o1.x - o1.y) * r, (o1.x + o1.y) * r)
           : make_float2((o1.x + o1.y) * r, (o1.y - o1.x) * r);
  o2 = mul_mi<INV>(o2);
  // w8^3 = (-1 - i)/sqrt2 (fwd), (-1 + i)/sqrt2 (inv)
  o3 = INV ? make_float2((-o3.x - o3.y) * r, (o3.x - o3.y) * r)
           : make_float2((o3.y - o3.x) * r, (-o3.x - o3.y) * r);
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1);
  a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2);
  a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3);
  a[7] = csub(e3, o3);
}

// Product by a twiddle given in the forward convention (conjugated for the
// inverse transform).
template <bool INV> __device__ __forceinline__ float2 tw_mul(float2 x, float2 w) {
  return INV ? cmulc(x, w) : cmul(x, w);
}

// s = a + w b and d = a - w b (w conjugated for the inverse): the product
// enters through FMAs and d = 2 a - s, six instructions instead of the eight
// of a separate product, sum and difference.
template <bool INV>
__device__ __forceinline__ void fma_pair(float2 a, float2 w, float2 b, float2& s, float2& d) {
  const float wy = INV ? -w.y : w.y;
  s = make_float2(fmaf(w.x, b.x, fmaf(-wy, b.y, a.x)), fmaf(w.x, b.y, fmaf(wy, b.x, a.y)));
  d = make_float2(fmaf(2.0f, a.x, -s.x), fmaf(2.0f, a.y, -s.y));
}

// 4-point DFT of (a0, u1 a1, u2 a2, u3 a3): dft4 with its inputs 1..3
// multiplied by twiddles (forward convention), the products of inputs 2 and 3
// taken inside fma_pair.  MI2: u2 = w4 = -i (+i inverse), a free product.
template <bool INV, bool MI2 = false>
__device__ __forceinline__ void dft4_tw(float2& a0, float2& a1, float2& a2, float2& a3, float2 u1, float2 u2,
                                        float2 u3) {
  float2 t0, t1, t2, d;
  if constexpr (MI2) {
    const float2 m2 = mul_mi<INV>(a2);
    t0 = cadd(a0, m2);
    t1 = csub(a0, m2);
  } else {
    fma_pair<INV>(a0, u2, a2, t0, t1);
  }
  fma_pair<INV>(tw_mul<INV>(a1, u1), u3, a3, t2, d);
  const float2 t3 = mul_mi<INV>(d);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// 16-point DFT as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
// Y_{n2}[k1] = DFT4_{n1}(a[4 n1 + n2]); Z = Y w16^(n2 k1); X[k1 + 4 k2] = DFT4_{n2}(Z[n2][k1]).
// TW: input m is first multiplied by W[m] (forward convention; W[0] only
// with TW0), the products taken inside the first stage's butterflies.
template <bool INV, bool TW = false, bool TW0 = false>
__device__ __forceinline__ void dft16(float2* a, const float2* W = nullptr) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    if constexpr (TW) {
      if (TW0 || n2 > 0) a[n2] = tw_mul<INV>(a[n2], W[n2]);
      dft4_tw<INV>(a[n2], a[4 + n2], a[8 + n2], a[12 + n2], W[4 + n2], W[8 + n2], W[12 + n2]);
    } else {
      dft4<INV>(a[n2], a[4 + n2], a[8 + n2], a[12 + n2]);
    }
  }
  // a[4 k1 + n2] holds Y_{n2}[k1]; the second stage over n2 for each k1 with
  // the twiddles w16^(n2 k1), w16^e = exp(-2 pi i e / 16)
  const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
  const float r = 0.70710678118654752440f;
  const float2 e1 = make_float2(c1, -s1), e2 = make_float2(r, -r), e3 = make_float2(s1, -c1);
  const float2 e6 = make_float2(-r, -r), e9 = make_float2(-c1, s1);
  dft4<INV>(a[0], a[1], a[2], a[3]);
  dft4_tw<INV>(a[4], a[5], a[6], a[7], e1, e2, e3);
  dft4_tw<INV, true>(a[8], a[9], a[10], a[11], e2, e2, e6);
  dft4_tw<INV>(a[12], a[13], a[14], a[15], e3, e6, e9);
  // a[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 index
  float2 t[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) t[i] = a[i];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[4 * k1 + k2];
}

// 24-point DFT as 3 x 8 with coprime factors (Good-Thomas): input n = (8 n1
// + 3 n2) mod 24 and output k = (16 k1 + 9 k2) mod 24 make the exponent
// n k = 8 n1 k1 + 3 n2 k2 (mod 24), so X[k] is a 3-point DFT over n1 of
// 8-point DFTs over n2, with no twiddles between them.
template <bool INV>
__device__ __forceinline__ void dft24(float2* a) {
  float2 t[3][8];
#pragma unroll
  for (int n1 = 0; n1 < 3; ++n1)
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) t[n1][n2] = a[(8 * n1 + 3 * n2) % 24];
#pragma unroll
  for (int n1 = 0; n1 < 3; ++n1) dft8<INV>(t[n1]);
#pragma unroll
  for (int k2 = 0; k2 < 8; ++k2) {
    dft3<INV>(t[0][k2], t[1][k2], t[2][k2]);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) a[(16 * k1 + 9 * k2) % 24] = t[k1][k2];
  }
}

// 32-point DFT from the 16-point DFTs E, O of the even and odd inputs:
// X[k] = E[k] + w32^k O[k], X[k + 16] = E[k] - w32^k O[k], w32^k =
// (cos(k pi/16), -sin(k pi/16)), both from cos(j pi/16), j <= 8.
template <bool INV>
__device__ __forceinline__ void dft32(float2* a) {
  constexpr float C[9] = {1.0f,
                          0.98078528040323043f,
                          0.92387953251128674f,
                          0.83146961230254524f,
                          0.70710678118654752f,
                          0.55557023301960222f,
                          0.38268343236508977f,
                          0.19509032201612826f,
                          0.0f};
  float2 e[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    e[i] = a[2 * i];
    o[i] = a[2 * i + 1];
  }
  dft16<INV>(e);
  dft16<INV>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float c = k <= 8 ? C[k] : -C[16 - k];
    const float sn = k <= 8 ? C[8 - k] : C[k - 8];
    fma_pair<INV>(e[k], make_float2(c, -sn), o[k], a[k], a[k + 16]);
  }
}

template <int R, bool INV>
__device__ __forceinline__ void dft_reg(float2* a) {
  if constexpr (R == 2) {
    dft2<INV>(a[0], a[1]);
  } else if constexpr (R == 3) {
    dft3<INV>(a[0], a[1], a[2]);
  } else if constexpr (R == 4) {
    dft4<INV>(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 8) {
    dft8<INV>(a);
  } else if constexpr (R == 24) {
    dft24<INV>(a);
  } else if constexpr (R == 32) {
    dft32<INV>(a);
  } else {
    static_assert(R == 16, "radix");
    dft16<INV>(a);
  }
}

// ------------------------------------------------------------ LDS layout --
// Element a of a line-interleaved LDS buffer (C lines interleaved, element
// stride C) is stored at a + C * (a / (16 C)): one pad slot group every 16
// elements per line keeps strided butterfly writes on distinct banks.
template <int C>
__device__ __forceinline__ unsigned lds_pad(unsigned a) {
  return a + C * (a / (16u * C));
}
template <int C, int N>
struct LdsSize {
  static constexpr int value = C * N + C * ((C * N) / (16 * C)) + C;
};

// ------------------------------------------------- Stockham FFT of a line --
// A line of N = T * E points is spread over T threads; thread b holds
// x[b + T k] in v[k], k < E, before and after the transform.  Pass s has
// radix R and sub-length L (product of the earlier radices); thread b runs
// the E/R butterflies beta = b + T q, q < E/R, reading x[beta + (N/R) m]
// (= v[q + (E/R) m]), applying w_{LR}^(j m) with j = beta mod L, and writing
// y[(beta - j) R + j + L m].  After the last pass every output lands back in
// its own thread's slot, so only the passes before it go through LDS.
// Twiddle sources: w_N^e = exp(-2 pi i e / N) for 0 <= e < N.
struct TwGlobal {  // FP32 table in global memory
  const float2* p;
  __device__ __forceinline__ float2 operator()(int e) const { return p[e]; }
};
struct TwLds {  // two-level table in LDS: w^e = lo[e % 64] hi[e / 64]
  const float2* lo;
  const float2* hi;
  __device__ __forceinline__ float2 operator()(int e) const { return cmul(lo[e & 63], hi[e >> 6]); }
};

// Twiddle powers w^(j m step), m < 16, of one Stockham pass for the
// butterfly index j of a thread.  With one butterfly per thread (E = R),
// j = b mod L is the same for every line the thread transforms, so a
// persistent kernel computes them once.
struct TwPowers {
  float2 w[16];
  // the pass whose twiddles come from an LDS table (table_pass): row j of
  // the table, tab[j (R + 1) + m] = w^(j m step)
  const float2* tab;
};

template <int N, int E, int R, int L, typename TW>
__device__ __forceinline__ TwPowers tw_powers(int b, const TW& tws) {
  constexpr int step = N / (L * R);
  TwPowers h;
  h.w[0] = make_float2(1.f, 0.f);
  h.w[1] = tws((b % L) * step);
#pragma unroll
  for (int m = 2; m < R; ++m) {
    const int hi = 1 << (31 - __builtin_clz(m));
    h.w[m] = (m == hi) ? cmul(h.w[m / 2], h.w[m / 2]) : cmul(h.w[hi], h.w[m - hi]);
  }
  h.tab = nullptr;
  return h;
}

// Radix-R butterflies of one Stockham pass on the thread's registers.  The
// twiddles w^(j m), m < R, come from one lookup of w^j and products of at
// most four factors for the rest (TM = 0), from precomputed powers (TM = 1),
// or from the pass's LDS table (TM = 2).  With given twiddles a radix-16
// butterfly takes their products inside its first stage.
template <int N, int E, int R, int L, bool INV, typename TW, int TM = 0>
__device__ __forceinline__ void stockham_compute(float2 (&v)[E], int b, const TW& tws, const TwPowers& hp) {
  constexpr int Q = E / R;
  constexpr int T = N / E;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float2 a[R];
#pragma unroll
    for (int m = 0; m < R; ++m) a[m] = v[q + Q * m];
    if constexpr (TM != 0) {
      static_assert(Q == 1 && L > 1, "precomputed twiddles need one butterfly per thread");
      float2 W[R];
      if constexpr (TM == 1) {
#pragma unroll
        for (int m = 1; m < R; ++m) W[m] = hp.w[m];
      } else {
        const float2* row = hp.tab + (b % L) * (R + 1);
#pragma unroll
        for (int m = 1; m < R; ++m) W[m] = row[m];
      }
      if constexpr (R == 16) {
        dft16<INV, true>(a, W);
      } else {
#pragma unroll
        for (int m = 1; m < R; ++m) a[m] = tw_mul<INV>(a[m], W[m]);
        dft_reg<R, INV>(a);
      }
    } else {
      if constexpr (L > 1) {
        const int beta = b + T * q;
        const int j = beta % L;
        constexpr int step = N / (L * R);
        // w^m = w^hi * w^(m - hi) with hi the highest power of two <= m; each
        // product is applied as soon as it exists
        float2 w[R];
        w[1] = tws(j * step);
        if (INV) w[1].y = -w[1].y;
        a[1] = cmul(a[1], w[1]);
#pragma unroll
        for (int m = 2; m < R; ++m) {
          const int hi = 1 << (31 - __builtin_clz(m));
          w[m] = (m == hi) ? cmul(w[m / 2], w[m / 2]) : cmul(w[hi], w[m - hi]);
          a[m] = cmul(a[m], w[m]);
        }
      }
      dft_reg<R, INV>(a);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) v[q + Q * m] = a[m];
    if constexpr (Q > 1) __builtin_amdgcn_sched_barrier(0);
  }
}

template <int N, int E, int R, int L, int C>
__device__ __forceinline__ void stockham_exchange(float2 (&v)[E], int b, int c, float2* lds) {
  constexpr int Q = E / R;
  constexpr int T = N / E;
  // Writes.  When R divides 16 (first pass) or L is a multiple of 16, the
  // padded addresses of one butterfly's R outputs differ by compile-time
  // constants, which the LDS instructions take as immediate offsets.
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int beta = b + T * q;
    if constexpr (L == 1 && 16 % R == 0) {
      const unsigned off = lds_pad<C>((unsigned)(beta * R * C + c));
      __builtin_assume(off < 32768u);
      float2* p = lds + off;
#pragma unroll
      for (int m = 0; m < R; ++m) p[m * C] = v[q + Q * m];
    } else if constexpr (L % 16 == 0) {
      const int j = beta % L;
      const unsigned off = lds_pad<C>((unsigned)(((beta - j) * R + j) * C + c));
      __builtin_assume(off < 32768u);
      float2* p = lds + off;
      constexpr int step = L * C + L * C / 16;
#pragma unroll
      for (int m = 0; m < R; ++m) p[m * step] = v[q + Q * m];
    } else {
      const int j = beta % L;
      const int base = (beta - j) * R + j;
#pragma unroll
      for (int m = 0; m < R; ++m) lds[lds_pad<C>((base + L * m) * C + c)] = v[q + Q * m];
    }
  }
  __syncthreads();
  // Reads of x[b + T k]: constant stride when T is a multiple of 16.
  if constexpr (T % 16 == 0) {
    const unsigned off = lds_pad<C>((unsigned)(b * C + c));
    __builtin_assume(off < 32768u);
    const float2* p = lds + off;
    constexpr int step = T * C + T * C / 16;
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = p[k * step];
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = lds[lds_pad<C>((b + T * k) * C + c)];
  }
  __syncthreads();
}

// The same exchange through half the LDS, in two rounds: with two
// butterflies per thread (E = 2R) and T R = N/2, butterfly q of every thread
// writes only into half q of the line, and the reads x[b + T k] of half q
// are k in [q E/2, (q+1) E/2); round q writes butterfly q, then every
// thread reads its half-q elements.  Lets two column workgroups share a
// compute unit's LDS.
template <int N, int E, int R, int L, int C>
__device__ __forceinline__ void stockham_exchange_split(float2 (&v)[E], int b, int c, float2* lds) {
  constexpr int Q = E / R;
  constexpr int T = N / E;
  constexpr int H = N / 2;
  static_assert(Q == 2 && T * R == H && T % L == 0 && T % 16 == 0, "split exchange");
  float2 t[E];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int beta = b + T * h;
    const int j = beta % L;
    const int base = (beta - j) * R + j - h * H;  // position in half h
    if constexpr (L % 16 == 0 || (L == 1 && 16 % R == 0)) {
      const unsigned off = lds_pad<C>((unsigned)(base * C + c));
      __builtin_assume(off < 32768u);
      float2* p = lds + off;
      constexpr int step = L == 1 ? C : L * C + L * C / 16;
#pragma unroll
      for (int m = 0; m < R; ++m) p[m * step] = v[h + Q * m];
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m) lds[lds_pad<C>((base + L * m) * C + c)] = v[h + Q * m];
    }
    __syncthreads();
    const unsigned off = lds_pad<C>((unsigned)(b * C + c));
    __builtin_assume(off < 32768u);
    const float2* p = lds + off;
    constexpr int step = T * C + T * C / 16;
#pragma unroll
    for (int k = 0; k < E / 2; ++k) t[h * (E / 2) + k] = p[k * step];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < E; ++k) v[k] = t[k];
}

// Passes whose twiddles a thread can precompute for every line: a pass
// s >= 1 in which each thread holds exactly one butterfly (R = E), so that
// its butterfly index j = b mod L does not change between lines.  The last
// such pass (the most distinct twiddles) keeps its powers in registers
// (hoisted_pass); an earlier one with at most 512 table entries reads them
// from a small LDS table filled once per workgroup (table_pass).  -1: none.
template <class P>
constexpr int hoisted_pass() {
  int h = -1;
  for (int s = 1; s < P::P; ++s)
    if (P::radix(s) == P::E && P::radix(s) <= 16) h = s;
  return h;
}
template <class P>
constexpr int table_pass() {
  int t = -1;
  for (int s = 1; s < hoisted_pass<P>(); ++s)
    if (P::radix(s) == P::E && P::sub(s) * (P::radix(s) + 1) <= 512) t = s;
  return t;
}
// Entries of the table pass's LDS table (one row of R + 1 per butterfly
// index j, padded against bank conflicts); 1 when there is none.
template <class P>
constexpr int pass_table_size() {
  return table_pass<P>() < 0 ? 1 : P::sub(table_pass<P>()) * (P::radix(table_pass<P>()) + 1);
}

// Fill the table pass's twiddles tab[j (R + 1) + m] = w_N^(j m step) from the
// global table (all threads of the workgroup; a barrier must follow).
template <class P>
__device__ __forceinline__ void load_pass_table(float2* t, const float2* __restrict__ tw) {
  constexpr int s = table_pass<P>();
  if constexpr (s >= 0) {
    constexpr int R = P::radix(s), L = P::sub(s), step = P::N / (L * R);
    for (int i = threadIdx.x; i < L * (R + 1); i += blockDim.x) {
      const int j = i / (R + 1), m = i % (R + 1);
      t[i] = m < R ? tw[j * m * step] : make_float2(0.f, 0.f);
    }
  }
}

// The hoisted pass's twiddle powers of thread b (computed once per kernel),
// with the table pass's LDS table.
template <class P, typename TW>
__device__ __forceinline__ TwPowers hoist_powers(int b, const TW& tws, const float2* tab) {
  constexpr int s = hoisted_pass<P>();
  TwPowers h = tw_powers<P::N, P::E, P::radix(s), P::sub(s)>(b, tws);
  h.tab = tab;
  return h;
}

// One length-N transform (plan P) of the line held by the thread's
// registers (x[b + T k] in v[k]), lines interleaved C-wide in LDS (of N or,
// with SPL, N/2 points per line).
template <class P, bool INV, int C, typename TW, int S = 0, int HS = -1, bool SPL = false>
__device__ __forceinline__ void fft_line(float2 (&v)[P::E], int b, int c, float2* lds, const TW& tws,
                                         const TwPowers& hp) {
  constexpr int N = P::N;
  if constexpr (S < P::P) {
    constexpr int R = P::radix(S);
    constexpr int L = P::sub(S);
    __builtin_amdgcn_sched_barrier(0);
    constexpr int TS = HS >= 0 ? table_pass<P>() : -1;
    stockham_compute<N, P::E, R, L, INV, TW, S == HS ? 1 : (S == TS ? 2 : 0)>(v, b, tws, hp);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (S + 1 < P::P) {
      if constexpr (SPL) stockham_exchange_split<N, P::E, R, L, C>(v, b, c, lds);
      else stockham_exchange<N, P::E, R, L, C>(v, b, c, lds);
    }
    fft_line<P, INV, C, TW, S + 1, HS, SPL>(v, b, c, lds, tws, hp);
  }
}

// Transform without precomputed twiddles.
template <class P, bool INV, int C, typename TW, bool SPL = false>
__device__ __forceinline__ void fft_line(float2 (&v)[P::E], int b, int c, float2* lds, const TW& tws) {
  TwPowers none;
  fft_line<P, INV, C, TW, 0, -1, SPL>(v, b, c, lds, tws, none);
}

// Fill a two-level twiddle table (64 + N/64 entries) from the global table.
template <int N>
__device__ __forceinline__ void load_twiddle_table(float2* t, const float2* __restrict__ tw) {
  for (int i = threadIdx.x; i < 64 + N / 64; i += blockDim.x) t[i] = tw[i < 64 ? i : 64 * (i - 64)];
}

// --------------------------------------------------------- phase screens --
// Within one range line (fixed Doppler bin) each phase screen is a quadratic
// polynomial in the element's offset, in turns.  Thread b holds offsets
// o = b + T k' (k' a compile-time integer per register slot), so the phase of
// slot k' is A + B k' + C k'^2 with A, B (per thread) and C (per line)
// reduced modulo 1 in FP64 once; per element only two FP64 FMAs and the
// quarter-turn reduction remain, and the remainder is rounded to FP32.
struct Quad {
  double A, B, C;
};

__device__ __forceinline__ double frac1(double x) { return x - floor(x); }

// Polynomial p0 + p1 o + p2 o^2 over o = b + T k': coefficients in k'.
__device__ __forceinline__ Quad quad_in_slot(double p0, double p1, double p2, int b, int T) {
  const double bb = (double)b, tt = (double)T;
  Quad q;
  q.A = frac1(fma(fma(p2, bb, p1), bb, p0));
  q.B = frac1(fma(2.0 * p2 * bb, tt, p1 * tt));
  q.C = frac1(p2 * tt * tt);
  return q;
}

// exp(2 pi i (A + B k + C k^2)) for a small integer k: the argument in FP64
// turns, reduced to [-1/2, 1/2] in FP64, then the hardware FP32 sine and
// cosine of the remainder (argument in turns; |error| <= 1.3e-7 on
// [-1/2, 1/2], measured on gfx950).
__device__ __forceinline__ float2 cis_quad(const Quad& q, int k) {
  const double dk = (double)k;
  const double t = fma(fma(q.C, dk, q.B), dk, q.A);
  const float r = (float)(t - rint(t));  // |r| <= 1/2 turn
  return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
}

// exp(2 pi i t) for an FP64 argument in turns: FP64 reduction to
// [-1/2, 1/2], then the hardware FP32 sine and cosine.
__device__ __forceinline__ float2 cis_turns(double t) {
  const float r = (float)(t - rint(t));
  return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
}

// ------------------------------------------------------- buffer access --
// Global arrays are read and written through buffer resources: the
// per-lane byte offset sits in one VGPR and the wave-uniform part (row
// stride times element slot) in an SGPR, so no 64-bit per-lane addresses are
// kept live, and accesses past num_records read 0 / are dropped.
struct Buf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Buf(const void* p, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000)) {}
  __device__ __forceinline__ float2 f2(uint32_t voff, uint32_t soff) const {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  __device__ __forceinline__ double2 d2(uint32_t voff, uint32_t soff) const {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
  __device__ __forceinline__ uint32_t u32(uint32_t voff, uint32_t soff) const {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
  }
  __device__ __forceinline__ void st(float2 v, uint32_t voff, uint32_t soff) const {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 0);
  }
};

__device__ __forceinline__ uint32_t clamp_bytes(size_t n) {
  return n > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)n;
}

// ----------------------------------------------------------- reductions --
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Block-wide sum of one float per thread (result valid in thread 0).
template <int NT>
__device__ __forceinline__ float block_sum(float x, float* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = x;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w];
  }
  return s;
}

}  // namespace cssar
