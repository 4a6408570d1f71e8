// C ABI of the library: operator construction (FP64 coefficient vectors,
// twiddle tables, launch plan), operator application G / G^H and the
// iterative thresholding solver.  See include/cssar.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "cssar_internal.hpp"

using namespace cssar;
using namespace cssar::detail;

namespace cssar {
namespace detail {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

// Kernel table of a (length, plan variant) pair, or NULL if not compiled.
const KernelTable* table_for(int n, int v) {
#define CSSAR_CASE(NN, VV) \
  if (n == NN && v == VV) return kernel_table_##NN##_##VV();
  CSSAR_FOR_EACH_PLAN(CSSAR_CASE)
#undef CSSAR_CASE
  return nullptr;
}

int signed_bin(int k, int n) { return k < (n + 1) / 2 ? k : k - n; }

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// One key per 16 pixels: the keys within a factor 2^(3/4) of the selected
// |V|^2 (three first-level bins), about 3 % of the pixels when the top 1 %
// lies in a Rayleigh background.
unsigned candidate_cap(const cssar_op* op) {
  return (unsigned)std::max<size_t>(4096, (size_t)op->na * op->nr / 16);
}
unsigned candidate_segments(const cssar_op* op) {
  const int g = op->grid_col[CK_V];
  return g <= kMaxCandSeg ? (unsigned)g : 0u;
}
unsigned candidate_segment_keys(const cssar_op* op) {
  const unsigned n = candidate_segments(op);
  return n ? candidate_cap(op) / n : 0u;
}
size_t adapt_state_bytes(const cssar_op* op) {
  return align256(sizeof(AdaptState) + ((size_t)kMaxCandSeg + candidate_cap(op)) * sizeof(unsigned));
}


// FP64 coefficient vectors of the three phase screens (turns = radians/2pi).
//   D(f) = sqrt(1 - (lambda f / (2 v))^2), D_ref = 1 (zero Doppler centroid)
//   Km(f) = Kr / (1 - Kr c r_ref f^2 / (2 v^2 fc^3 D^3))   (Km = Kr if !src)
//   Phi1 = a1 (dtau - d1)^2, a1 = Km (1/D - 1) / 2, d1 = 2 r_ref (1/D - 1) / c
//   Phi2 = (a2 nu + b2) nu,  a2 = D / (2 Km) (fs/N_r)^2, b2 = 2 r_ref (1/D - 1) / c (fs/N_r)
//   Phi3 = D P_j + b3 dtau^2, b3 = -Km (1 - D) / (2 D^2), P_j = fc tau_j
// with dtau = (j - N_r/2) / fs and tau_j = 2 r_ref / c + dtau (the kernels
// expand Phi1 and Phi3 as polynomials in j - N_r/2).
void build_coefficients(const cssar_params& p, int na, int nr, std::vector<double2>& r1,
                        std::vector<double2>& r2, std::vector<double2>& r3) {
  const double lam = kC / p.fc;
  const double df = p.fs / nr;
  r1.resize(na);
  r2.resize(na);
  r3.resize(na);
  for (int k = 0; k < na; ++k) {
    const double f = p.prf * signed_bin(k, na) / na;
    const double u = lam * f / (2.0 * p.v);
    const double D = std::sqrt(1.0 - u * u);
    double Km = p.Kr;
    if (p.src) Km = p.Kr / (1.0 - p.Kr * kC * p.r_ref * f * f / (2.0 * p.v * p.v * p.fc * p.fc * p.fc * D * D * D));
    const double invD1 = 1.0 / D - 1.0;
    r1[k] = make_double2(0.5 * Km * invD1, 2.0 * p.r_ref * invD1 / kC);
    r2[k] = make_double2(0.5 * D / Km * df * df, 2.0 * p.r_ref * invD1 / kC * df);
    r3[k] = make_double2(D, -0.5 * Km * (1.0 - D) / (D * D));
  }
}

// Range-Doppler chain (eq. (RDA)) per Doppler bin: the migration in range
// samples delta_j = a + b j (b = 1/D - 1, a = tau_0 b fs, tau_0 the range
// time of column 0) and the azimuth filter exp(-i pi f^2 / K_a(tau_j)),
// K_a = 2 V^2 / (lambda R0), as turns A + B j.
void build_rda_coefficients(const cssar_params& p, int na, int nr, std::vector<double2>& mig,
                            std::vector<double2>& az) {
  const double lam = kC / p.fc;
  const double tau0 = 2.0 * p.r_ref / kC - 0.5 * nr / p.fs;
  mig.resize(na);
  az.resize(na);
  for (int k = 0; k < na; ++k) {
    const double f = p.prf * signed_bin(k, na) / na;
    const double u = lam * f / (2.0 * p.v);
    const double b = 1.0 / std::sqrt(1.0 - u * u) - 1.0;
    mig[k] = make_double2(tau0 * b * p.fs, b);
    const double c = -f * f * lam * kC / (8.0 * p.v * p.v);
    az[k] = make_double2(c * tau0, c / p.fs);
  }
}

void build_twiddles(int n, std::vector<float2>& t) {
  t.resize(n);
  for (int k = 0; k < n; ++k) {
    // exp(-2 pi i k / n), evaluated in FP64 and rounded to FP32
    const double a = 2.0 * M_PI * (double)k / (double)n;
    t[k] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
  }
}

int check_params(const cssar_params* p) {
  if (!p) return fail(CSSAR_EINVAL, "params is NULL");
  const double vals[] = {p->fc, p->Kr, p->fs, p->prf, p->v, p->r_ref};
  const char* names[] = {"fc", "Kr", "fs", "prf", "v", "r_ref"};
  for (int i = 0; i < 6; ++i)
    if (!(vals[i] > 0.0) || !std::isfinite(vals[i]))
      return fail(CSSAR_EINVAL, "parameter %s must be positive and finite", names[i]);
  if (p->f_dc != 0.0) return fail(CSSAR_EUNSUPPORTED, "non-zero Doppler centroid is not supported");
  // every Doppler bin must stay below the migration singularity
  const double umax = (kC / p->fc) * (p->prf / 2.0) / (2.0 * p->v);
  if (!(umax < 1.0)) return fail(CSSAR_EINVAL, "PRF too high for the velocity and wavelength");
  return CSSAR_OK;
}

int check_op(const cssar_op* op) {
  if (!op) return fail(CSSAR_EINVAL, "operator is NULL");
  return CSSAR_OK;
}

int occupancy(const void* fn, int block) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, block, 0) != hipSuccess || n < 1) n = 1;
  return n;
}

// Plan variant of the single-array column pass of each kind (also the
// batched solver's default), and of the chirp-scaling row passes, as
// measured on MI355X:
// - 4096: the residual pass runs variant 1 (32 elements per thread, 512
//   threads, the next tile's input loaded during the transforms: 100 us
//   against 107 with variant 0, measured with the fenced reduction of the
//   time); variant 1 is slower for the update pass (102 against 96 us) and
//   the first forward pass.  The update pass runs variant 2 (two-column
//   tiles, two workgroups per compute unit: 90 against 96 us).
// - 2048: the update pass runs variant 1 (4-column tiles, two workgroups
//   per compute unit): 23.8 against 26.9 us at 2048 x 2048.
// - 8192: lines through half the LDS (variant 1) for the chirp-scaling row
//   passes (two rows per workgroup, two workgroups per CU: 319 against 388
//   us with four rows per workgroup at 8192 x 8192) and the first forward
//   and the inverse column passes (four-column tiles: 738 against 786 us);
//   the update and residual passes run variant 0 (two-column tiles, 16
//   elements per thread, 1024 threads: 515 and 478 us against 533 and 503
//   us with variant 1 for the residual pass and 32 elements per thread for
//   the update pass).
// (The threshold adjoint recomputes the update pass's V: same plan, same
// support decisions.)
int row_variant(int n) { return n == 8192 ? 1 : 0; }
int column_variant(int n, int which) {
  if (n == 8192) return (which == CK_FWD || which == CK_INV) ? 1 : 0;
  if (n == 4096 && which == CK_R) return 1;
  if (n == 4096 && (which == CK_A || which == CK_AS || which == CK_VB)) return 2;
  if (n == 2048 && (which == CK_A || which == CK_AS || which == CK_VB || which == CK_R)) return 1;
  return 0;
}

int grid_for(int work, int cus, int per_cu) {
  int g = std::min(work, cus * per_cu);
  if (g >= 16) g -= g % 8;  // lets the kernels renumber blocks per XCD
  return std::max(g, 1);
}

ColArgs col_args(const cssar_op* op) {
  ColArgs a{};
  a.tw = op->tw_a;
  a.na = op->na;
  a.nr = op->nr;
  a.scale = 1.0f / (float)op->na;
  a.mu = 1.0f;
  a.partials = op->partials;
  a.status = op->counter + 1;
  return a;
}

RowArgs row_args(const cssar_op* op, const void* in, void* out, int conj) {
  RowArgs a{};
  a.in = (const float2*)in;
  a.out = (float2*)out;
  a.rowc1 = op->rowc1;
  a.rowc2 = op->rowc2;
  a.rowc3 = op->rowc3;
  a.tw = op->tw_r;
  a.na = op->na;
  a.conj = conj;
  a.scale = 1.0f / (float)op->nr;
  a.inv_fs = 1.0 / op->p.fs;
  a.fc_fs = op->p.fc / op->p.fs;
  a.p_c = op->p.fc * 2.0 * op->p.r_ref / kC;
  const double df = op->p.fs / op->nr;
  a.c_tau = 0.5 * df * df / op->p.Kr;
  a.taps = op->taps;
  return a;
}

hipEvent_t take_event(cssar_op* op) {
  if (!op->pool.empty()) {
    hipEvent_t e = op->pool.back();
    op->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

const char* const kPassKindName[CSSAR_PROFILE_KINDS] = {
    "cssar row M", "cssar row G", "cssar col forward", "cssar col inverse", "cssar col update",
    "cssar col residual", "cssar col threshold adjoint", "cssar col data adjoint",
    "cssar col iterate adjoint", "cssar col restricted step", "cssar col step norm",
    "cssar col value", "cssar col threshold selected", "cssar row adjoint M", "cssar row adjoint G",
    "cssar select kth", "cssar col update sparse"};

int launch_row(cssar_op* op, const RowArgs& a, hipStream_t s) {
  if (op->chain == CSSAR_CHAIN_RDA)
    return timed(op, a.conj ? 1 : 0, s, [&] { return op->kr->row_rda[a.conj ? 1 : 0](a, op->grid_rda, s); });
  return timed(op, a.conj ? 1 : 0, s, [&] { return op->krow->row(a, op->grid_row, s); });
}

int launch_col(cssar_op* op, int which, const ColArgs& a, hipStream_t s) {
  const int kind = which == CK_AS ? 16 : 2 + which;
  return timed(op, kind, s, [&] { return op->kcol[which]->col[which](a, op->grid_col[which], s); });
}

SparseLayout sparse_layout(const cssar_op* op, const KernelTable* kt) {
  if (!kt) kt = op->kcol[CK_AS];
  SparseLayout L;
  const size_t ntiles = (size_t)(op->nr / kt->C);
  L.wmask = align256(ntiles * kt->CT * 32);             // after the 32-byte records
  L.bytes = L.wmask + align256(ntiles * (kt->CT / 64) * 8);  // one 8-byte mask per wave
  return L;
}

size_t sparse_bytes_max(const cssar_op* op) {
  size_t m = 0;
  for (int v = 0; v < kMaxVariants; ++v) {
    const KernelTable* kt = table_for(op->na, v);
    if (kt && op->nr % kt->C == 0) m = std::max(m, sparse_layout(op, kt).bytes);
  }
  return m;
}

void set_sparse(const cssar_op* op, ColArgs& a, void* dense, void* base, const KernelTable* kt) {
  const SparseLayout L = sparse_layout(op, kt);
  a.xrec = (float4*)base;
  a.xwmask = (uint64_t*)((char*)base + L.wmask);
  a.xdense = (float2*)dense;
}

// ||R||^2 of the residual pass (or ||m o y||^2 of the first forward pass)
// from its per-block partials (FP64, in the
// order of the last-block reduction of the other passes), into out (if not
// NULL), and bit 0 of status when it is not finite.
__global__ __launch_bounds__(256) void residual_total_kernel(const float* __restrict__ part, int nblocks,
                                                             float* out, unsigned* status) {
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
    if (out) out[0] = (float)t;
    if (!isfinite(t)) atomicOr(status, 1u);
  }
}

int residual_total(cssar_op* op, int ck, const ColArgs& a, bool check, hipStream_t s) {
  if (!(check || a.hist_out)) return CSSAR_OK;
  hipLaunchKernelGGL(residual_total_kernel, dim3(1), dim3(256), 0, s, (const float*)a.partials,
                     op->grid_col[ck], a.hist_out, a.status);
  HIP_TRY(hipGetLastError());
  return CSSAR_OK;
}

// ||X||_1 and the nonzero count of an iterate, per block (FP64 sum, count)
// into part[2 block], part[2 block + 1]; a one-block kernel totals them.
// The sparse iterate: one thread per record slot of a wave's area (slots
// below the wave's record count hold records, packed in lane order); a
// dense record's thread is the lane of that rank in the wave mask, whose E
// values lie in the dense tiles at the positions of the update plan
// (tiles of C columns, T threads per column).
__global__ __launch_bounds__(256) void sparse_metrics_kernel(const float4* __restrict__ rec,
                                                             const uint64_t* __restrict__ wmask,
                                                             const float2* __restrict__ xdense, long long nwaves,
                                                             int CT, int C, int T, int E, int nr,
                                                             double* __restrict__ part) {
  __shared__ double sl[256], sn[256];
  double l1 = 0.0, nn = 0.0;
  const long long n = nwaves * 64;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (long long)gridDim.x * blockDim.x) {
    const long long w = g >> 6;
    const int slot = (int)(g & 63);
    const uint64_t m = wmask[w];
    if (slot >= __builtin_popcountll(m)) continue;
    const float4 r0 = rec[2 * g], r1 = rec[2 * g + 1];
    const uint32_t word = __float_as_uint(r0.x);
    if (word == kDenseWord) {
      uint64_t mm = m;  // the lane of rank slot
      for (int q = 0; q < slot; ++q) mm &= mm - 1;
      const int lane = __builtin_ctzll(mm);
      const int W = CT / 64;
      const int tile = (int)(w / W), th = (int)(w % W) * 64 + lane;
      const Addr ab = col_addr(B4, th / C, tile * C + th % C, T, nr);
      for (int k = 0; k < E; ++k) {
        const float2 x = xdense[(ab.voff + (size_t)k * ab.kstep) / 8];
        const double a = sqrt((double)x.x * x.x + (double)x.y * x.y);
        l1 += a;
        nn += a > 0.0 ? 1.0 : 0.0;
      }
    } else {
      const double a0 = sqrt((double)r0.y * r0.y + (double)r0.z * r0.z);
      const double a1 = __builtin_popcount(word) > 1 ? sqrt((double)r1.x * r1.x + (double)r1.y * r1.y) : 0.0;
      l1 += a0 + a1;
      nn += (a0 > 0.0 ? 1.0 : 0.0) + (a1 > 0.0 ? 1.0 : 0.0);
    }
  }
  sl[threadIdx.x] = l1;
  sn[threadIdx.x] = nn;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sl[threadIdx.x] += sl[threadIdx.x + h];
      sn[threadIdx.x] += sn[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sl[0];
    part[2 * blockIdx.x + 1] = sn[0];
  }
}

// The same for a row-major (or any dense) array of n complex values.
__global__ __launch_bounds__(256) void dense_metrics_kernel(const float2* __restrict__ x, long long n,
                                                            double* __restrict__ part) {
  __shared__ double sl[256], sn[256];
  double l1 = 0.0, nn = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float2 v = x[i];
    const double a = sqrt((double)v.x * v.x + (double)v.y * v.y);
    l1 += a;
    nn += a > 0.0 ? 1.0 : 0.0;
  }
  sl[threadIdx.x] = l1;
  sn[threadIdx.x] = nn;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sl[threadIdx.x] += sl[threadIdx.x + h];
      sn[threadIdx.x] += sn[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sl[0];
    part[2 * blockIdx.x + 1] = sn[0];
  }
}

constexpr int kMetricBlocks = 256;

__global__ __launch_bounds__(256) void metrics_total_kernel(const double* __restrict__ part, float* l1_out,
                                                            int* nnz_out) {
  __shared__ double sl[256], sn[256];
  sl[threadIdx.x] = part[2 * threadIdx.x];
  sn[threadIdx.x] = part[2 * threadIdx.x + 1];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sl[threadIdx.x] += sl[threadIdx.x + h];
      sn[threadIdx.x] += sn[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (l1_out) l1_out[0] = (float)sl[0];
    if (nnz_out) nnz_out[0] = (int)sn[0];
  }
}

// ||X||_1 and the nonzero count of the sparse iterate (dense == NULL) or of
// the dense array x (n values) into l1_out / nnz_out (either may be NULL).
int iterate_metrics(cssar_op* op, const ColArgs& a, const float2* dense, long long n, float* l1_out,
                    int* nnz_out, hipStream_t s) {
  if (!l1_out && !nnz_out) return CSSAR_OK;
  double* part = (double*)op->partials;  // (the pass partials are consumed by now)
  if (dense) {
    hipLaunchKernelGGL(dense_metrics_kernel, dim3(kMetricBlocks), dim3(256), 0, s, dense, n, part);
  } else {
    const KernelTable* kt = op->kcol[CK_AS];
    const long long nwaves = (long long)(op->nr / kt->C) * (kt->CT / 64);
    hipLaunchKernelGGL(sparse_metrics_kernel, dim3(kMetricBlocks), dim3(256), 0, s, (const float4*)a.xrec,
                       (const uint64_t*)a.xwmask, (const float2*)a.xdense, nwaves, kt->CT, kt->C, kt->T, kt->E,
                       op->nr, part);
  }
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(metrics_total_kernel, dim3(1), dim3(kMetricBlocks), 0, s, (const double*)part, l1_out, nnz_out);
  HIP_TRY(hipGetLastError());
  return CSSAR_OK;
}

int launch_row_adj(cssar_op* op, int conj, const RowArgs& a, hipStream_t s) {
  return timed(op, 13 + conj, s, [&] { return op->kr->row_adj[conj](a, op->grid_adj[conj], s); });
}

}  // namespace detail
}  // namespace cssar

extern "C" {

double cssar_azimuth_fm_rate(const cssar_params* p) {
  if (!p || !(p->fc > 0.0) || !(p->r_ref > 0.0)) return 0.0;
  return 2.0 * p->v * p->v / ((kC / p->fc) * p->r_ref);
}

int cssar_params_with_rates(const cssar_params* in, double Ka, double Kr, cssar_params* out) {
  if (!in || !out) return fail(CSSAR_EINVAL, "NULL parameters");
  if (!(Ka > 0.0) || !(Kr > 0.0) || !std::isfinite(Ka) || !std::isfinite(Kr))
    return fail(CSSAR_EINVAL, "the rates must be positive and finite");
  if (!(in->fc > 0.0) || !(in->r_ref > 0.0)) return fail(CSSAR_EINVAL, "fc and r_ref must be positive");
  const cssar_params p = *in;
  *out = p;
  out->v = std::sqrt(Ka * (kC / p.fc) * p.r_ref / 2.0);
  out->Kr = Kr;
  return CSSAR_OK;
}

int cssar_supported_length(int n) { return table_for(n) != nullptr; }

int cssar_plan_info(int n, int* elems_per_thread, int* n_passes, int* radices) {
  const KernelTable* t = table_for(n);
  if (!t) return fail(CSSAR_EUNSUPPORTED, "length %d is not supported", n);
  if (elems_per_thread) *elems_per_thread = t->E;
  if (n_passes) *n_passes = t->passes;
  if (radices)
    for (int i = 0; i < 8; ++i) radices[i] = t->radices[i];
  return CSSAR_OK;
}

const char* cssar_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace cssar {
namespace detail {

int make_operator_impl(const cssar_params* p, int n_az, int n_rg, int chain, int taps, cssar_op** out) {
  if (!out) return fail(CSSAR_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_params(p);
  if (rc) return rc;
  if (n_az <= 0 || n_rg <= 0) return fail(CSSAR_EINVAL, "grid sizes must be positive");
  const KernelTable* ka = table_for(n_az);
  const KernelTable* kr = table_for(n_rg);
  if (!ka) return fail(CSSAR_EUNSUPPORTED, "azimuth length %d is not supported", n_az);
  if (!kr) return fail(CSSAR_EUNSUPPORTED, "range length %d is not supported", n_rg);
  if (n_rg % ka->C != 0 || n_rg % 32 != 0)
    return fail(CSSAR_EUNSUPPORTED, "range length %d incompatible with the column tile", n_rg);

  if (chain == CSSAR_CHAIN_RDA && (taps < 2 || taps > 32 || taps % 2 != 0 || taps > n_rg))
    return fail(CSSAR_EINVAL, "taps must be even, in 2..32 and at most N_r (got %d)", taps);
  std::vector<double2> r1, r2, r3;
  build_coefficients(*p, n_az, n_rg, r1, r2, r3);
  for (int k = 0; k < n_az; ++k)
    if (!std::isfinite(r1[k].x) || !std::isfinite(r2[k].x) || !std::isfinite(r3[k].y))
      return fail(CSSAR_EINVAL, "parameters give non-finite phase coefficients");
  if (chain == CSSAR_CHAIN_RDA) {
    // the range-Doppler tables take the places of Phi1 and Phi3
    build_rda_coefficients(*p, n_az, n_rg, r1, r3);
    // a migration beyond the range extent has no meaning on the periodic
    // grid (and would let the interpolation windows wrap more than once)
    for (int k = 0; k < n_az; ++k)
      if (!(std::fabs(r1[k].x) + std::fabs(r1[k].y) * n_rg < 0.5 * n_rg))
        return fail(CSSAR_EINVAL, "range migration exceeds half the range extent (%d samples)", n_rg);
  }
  std::vector<float2> ta, tr;
  build_twiddles(n_az, ta);
  build_twiddles(n_rg, tr);

  cssar_op* op = new cssar_op();
  op->na = n_az;
  op->nr = n_rg;
  op->p = *p;
  op->chain = chain;
  op->taps = chain == CSSAR_CHAIN_RDA ? taps : 0;
  op->ka = ka;
  op->kr = kr;
  auto cleanup = [&](int code) {
    cssar_destroy_operator(op);
    return code;
  };
  if (hipGetDevice(&op->device) != hipSuccess) return cleanup(fail(CSSAR_EHIP, "hipGetDevice failed"));
  if (hipDeviceGetAttribute(&op->cus, hipDeviceAttributeMultiprocessorCount, op->device) != hipSuccess)
    return cleanup(fail(CSSAR_EHIP, "cannot query the compute unit count"));
  const size_t rowb = sizeof(double2) * n_az;
  void* mem = nullptr;
  std::vector<float> rd;
  build_derivatives(*p, n_az, n_rg, rd);
  const size_t total = 3 * rowb + sizeof(float2) * (n_az + n_rg) +
                       sizeof(float) * kMaxPartials + 4 * sizeof(unsigned) + 256 +
                       sizeof(float) * rd.size() + 1024;
  if (hipMalloc(&mem, total) != hipSuccess) return cleanup(fail(CSSAR_ENOMEM, "hipMalloc of %zu bytes failed", total));
  char* base = (char*)mem;
  op->rowc1 = (double2*)base;
  op->rowc2 = (double2*)(base + rowb);
  op->rowc3 = (double2*)(base + 2 * rowb);
  op->tw_a = (float2*)(base + 3 * rowb);
  op->tw_r = op->tw_a + n_az;
  op->partials = (float*)(op->tw_r + n_rg);
  op->counter = (unsigned*)(op->partials + kMaxPartials);
  op->rowd = (float*)((char*)op->counter + 256);
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(op->rowc1, r1.data(), rowb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(op->rowc2, r2.data(), rowb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(op->rowc3, r3.data(), rowb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(op->tw_a, ta.data(), sizeof(float2) * n_az, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(op->tw_r, tr.data(), sizeof(float2) * n_rg, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(op->rowd, rd.data(), sizeof(float) * rd.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(op->counter, 0, 4 * sizeof(unsigned));
  if (e != hipSuccess) return cleanup(fail(CSSAR_EHIP, "uploading operator tables: %s", hipGetErrorString(e)));

  // the chirp-scaling row passes may run another plan variant; the
  // range-Doppler and adjoint row passes keep variant 0
  op->krow = table_for(n_rg, row_variant(n_rg));
  if (!op->krow || n_az % op->krow->LR != 0) op->krow = kr;
  const int row_work = (n_az + kr->LR - 1) / kr->LR;
  op->grid_row = grid_for((n_az + op->krow->LR - 1) / op->krow->LR, op->cus,
                          occupancy(op->krow->row_fn, op->krow->RT));
  op->grid_rda = grid_for(row_work, op->cus, occupancy(kr->row_rda_fn[0], kr->RT));
  for (int c = 0; c < 2; ++c)
    op->grid_adj[c] = std::min(grid_for(row_work, op->cus, occupancy(kr->row_adj_fn[c], kr->RT)), kMaxPartials / 2);
  for (int w = 0; w < CK_COUNT; ++w) {
    const KernelTable* kt = table_for(n_az, column_variant(n_az, w));
    if (!kt || n_rg % kt->C != 0) kt = ka;
    op->kcol[w] = kt;
    op->grid_col[w] = grid_for(n_rg / kt->C, op->cus, occupancy(kt->col_fn[w], kt->CT));
    if (op->grid_col[w] > kMaxPartials) op->grid_col[w] = kMaxPartials;
  }
  *out = op;
  return CSSAR_OK;
}

}  // namespace detail
}  // namespace cssar

extern "C" {

int cssar_make_operator(const cssar_params* p, int n_az, int n_rg, cssar_op** out) {
  return make_operator_impl(p, n_az, n_rg, CSSAR_CHAIN_CSA, 0, out);
}

int cssar_make_operator_rda(const cssar_params* p, int n_az, int n_rg, int taps, cssar_op** out) {
  return make_operator_impl(p, n_az, n_rg, CSSAR_CHAIN_RDA, taps, out);
}

int cssar_operator_chain(const cssar_op* op) { return op ? op->chain : CSSAR_EINVAL; }

int cssar_destroy_operator(cssar_op* op) {
  if (!op) return CSSAR_OK;
  for (auto& r : op->recs) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto e : op->pool) (void)hipEventDestroy(e);
  if (op->rowc1) (void)hipFree(op->rowc1);
  delete op;
  return CSSAR_OK;
}

size_t cssar_workspace_size(const cssar_op* op, int mode) {
  if (!op) return 0;
  const size_t blk = align256(b4_bytes(op->na, op->nr));
  switch (mode) {
    case 0:
      return blk;
    case 1:
      return 3 * blk + sparse_layout(op).bytes;
    case 2:
      return 4 * blk + align256(support_bytes(op)) + adapt_state_bytes(op);
    case 3:
      return 6 * blk + 2 * align256(support_bytes(op)) + adapt_state_bytes(op);
    default:
      return 0;
  }
}

int cssar_apply_GH(cssar_op* op, const void* y, void* x_out, void* ws, void* stream) {
  const TraceRange tr("cssar_apply_GH");
  int rc = check_op(op);
  if (rc) return rc;
  if (!y || !x_out || !ws) return fail(CSSAR_EINVAL, "NULL array or workspace");
  if (y == x_out || ws == y || ws == x_out) return fail(CSSAR_EINVAL, "arrays must not alias");
  hipStream_t s = (hipStream_t)stream;
  // x = F_eta^-1 [Phi3 o F_tau^-1 [Phi2 o F_tau [Phi1 o F_eta y]]]
  ColArgs a = col_args(op);
  a.in0 = (const float2*)y;
  a.out = (float2*)ws;
  if ((rc = launch_col(op, CK_FWD, a, s))) return rc;
  if ((rc = launch_row(op, row_args(op, ws, ws, 0), s))) return rc;
  a.in0 = (const float2*)ws;
  a.out = (float2*)x_out;
  return launch_col(op, CK_INV, a, s);
}

int cssar_apply_G(cssar_op* op, const void* x, void* y_out, void* ws, void* stream) {
  const TraceRange tr("cssar_apply_G");
  int rc = check_op(op);
  if (rc) return rc;
  if (!x || !y_out || !ws) return fail(CSSAR_EINVAL, "NULL array or workspace");
  if (x == y_out || ws == x || ws == y_out) return fail(CSSAR_EINVAL, "arrays must not alias");
  hipStream_t s = (hipStream_t)stream;
  // y = F_eta^-1 [Phi1* o F_tau^-1 [Phi2* o F_tau [Phi3* o F_eta x]]]
  ColArgs a = col_args(op);
  a.in0 = (const float2*)x;
  a.out = (float2*)ws;
  if ((rc = launch_col(op, CK_FWD, a, s))) return rc;
  if ((rc = launch_row(op, row_args(op, ws, ws, 1), s))) return rc;
  a.in0 = (const float2*)ws;
  a.out = (float2*)y_out;
  return launch_col(op, CK_INV, a, s);
}

int cssar_ita_solve_ex(cssar_op* op, const void* y, const void* mask_bits, float lambda, int iters,
                       const cssar_solve_opts* opts, void* x_out, void* ws, void* stream) {
  const TraceRange tr("cssar_ita_solve");
  int rc = check_op(op);
  if (rc) return rc;
  if (!y || !mask_bits || !x_out || !ws) return fail(CSSAR_EINVAL, "NULL array");
  if (iters < 1) return fail(CSSAR_EINVAL, "iters must be >= 1");
  if (!(lambda >= 0.0f) || !std::isfinite(lambda)) return fail(CSSAR_EINVAL, "lambda must be finite and >= 0");
  if (x_out == y || x_out == ws || ws == y) return fail(CSSAR_EINVAL, "x_out, y and ws must not alias");
  const cssar_solve_opts o = opts ? *opts : cssar_solve_opts{};
  if (o.x0 && (o.x0 == ws || o.x0 == y)) return fail(CSSAR_EINVAL, "x0 must not alias y or ws");
  hipStream_t s = (hipStream_t)stream;
  const size_t blk = align256(b4_bytes(op->na, op->nr));
  float2* Xd = (float2*)ws;                      // dense tiles of the sparse iterate (blocked layout)
  float2* P = (float2*)((char*)ws + blk);        // pass buffer (in place)
  float2* Y = (float2*)((char*)ws + 2 * blk);    // m o y (blocked layout, unsampled marked)
  ColArgs a = col_args(op);
  a.y = Y;
  a.mask = (const uint32_t*)mask_bits;
  a.sigma = lambda * a.mu;
  set_sparse(op, a, Xd, (char*)ws + 3 * blk);
  const long long npx = (long long)op->na * op->nr;
  // R(0) = m o y - m o G X(0): the first pass keeps m o y (Y) for every
  // residual; from X(0) = 0 it is also F_eta R(0) (P)
  {
    ColArgs f = a;
    f.in0 = (const float2*)y;
    f.out = P;
    f.out2 = Y;
    f.flags = 1 | 4;
    f.hist_out = o.x0 ? nullptr : o.resid_hist;
    if ((rc = launch_col(op, CK_FWD, f, s))) return rc;
    if ((rc = residual_total(op, CK_FWD, f, !o.x0, s))) return rc;
  }
  if (o.x0) {
    // warm start: X(0) as the sparse iterate and F_eta X(0) into P, as an
    // update pass would have left them
    ColArgs w = a;
    w.in0 = (const float2*)o.x0;
    w.out = P;
    w.flags = 8;
    if ((rc = launch_col(op, CK_AS, w, s))) return rc;
  }
  for (int t = 0; t < iters; ++t) {
    const bool last = t == iters - 1;
    a.hist_out = o.resid_hist ? o.resid_hist + t : nullptr;
    if (t > 0 || o.x0) {
      // P = F_eta G X (row chain of G on F_eta X, which the update pass left
      // in P); then R = m o y - m o G X, P = F_eta R
      if ((rc = launch_row(op, row_args(op, P, P, 1), s))) return rc;
      ColArgs r = a;
      r.in0 = P;
      r.out = P;
      if ((rc = launch_col(op, CK_R, r, s))) return rc;
      if ((rc = residual_total(op, CK_R, r, last, s))) return rc;  // (the last one: non-finite check)
    }
    // P = F_eta M R (row chain of M)
    if ((rc = launch_row(op, row_args(op, P, P, 0), s))) return rc;
    // X+ = S(X + F_eta^-1 P / N_a): the sparse iterate, and F_eta X+ into P
    // (or X+ into x_out in the last iteration)
    ColArgs u = a;
    u.in1 = P;
    u.out = last ? (float2*)x_out : P;
    u.flags = (t == 0 && !o.x0 ? 1 : 0) | (last ? 2 : 0);
    u.hist_out = nullptr;
    if ((rc = launch_col(op, CK_AS, u, s))) return rc;
    float* l1 = o.l1_hist ? o.l1_hist + t : nullptr;
    int* nnz = o.nnz_hist ? o.nnz_hist + t : nullptr;
    if ((rc = iterate_metrics(op, u, last ? (const float2*)x_out : nullptr, npx, l1, nnz, s))) return rc;
  }
  return CSSAR_OK;
}

int cssar_ita_solve(cssar_op* op, const void* y, const void* mask_bits, float lambda, int iters,
                    void* x_out, float* resid_hist, void* ws, void* stream) {
  cssar_solve_opts o{};
  o.resid_hist = resid_hist;
  return cssar_ita_solve_ex(op, y, mask_bits, lambda, iters, &o, x_out, ws, stream);
}

int cssar_profile_enable(cssar_op* op, int on) {
  int rc = check_op(op);
  if (rc) return rc;
  op->profiling = on != 0;
  return CSSAR_OK;
}

int cssar_profile_read(cssar_op* op, double* ms_sum, long* counts) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!ms_sum || !counts) return fail(CSSAR_EINVAL, "NULL output");
  for (int k = 0; k < CSSAR_PROFILE_KINDS; ++k) {
    ms_sum[k] = 0.0;
    counts[k] = 0;
  }
  for (auto& r : op->recs) {
    HIP_TRY(hipEventSynchronize(r.stop));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.start, r.stop));
    if (r.kind >= 0 && r.kind < CSSAR_PROFILE_KINDS) {
      ms_sum[r.kind] += ms;
      counts[r.kind] += 1;
    }
    op->pool.push_back(r.start);
    op->pool.push_back(r.stop);
  }
  op->recs.clear();
  return CSSAR_OK;
}

int cssar_sync_status(cssar_op* op, void* stream) {
  int rc = check_op(op);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  unsigned st = 0;
  HIP_TRY(hipMemcpy(&st, op->counter + 1, sizeof st, hipMemcpyDeviceToHost));
  if (st) {
    unsigned zero = 0;
    HIP_TRY(hipMemcpy(op->counter + 1, &zero, sizeof zero, hipMemcpyHostToDevice));
    if (st & 1u) return fail(CSSAR_ENONFINITE, "non-finite residual norm");
  }
  return CSSAR_OK;
}

}  // extern "C"

// ------------------------------------------------------------ mask packing --
namespace {
// Word w of the packed mask holds blocked element indices 32 w .. 32 w + 31:
// e = ((i/4) (N_r/4) + j/4) 16 + (i%4) 4 + j%4, i.e. two 4 x 4 blocks.
__global__ void pack_mask_kernel(const unsigned char* __restrict__ m, uint32_t* __restrict__ bits, int na, int nr) {
  const size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nw = ((size_t)na * nr + 31) / 32;
  if (w >= nw) return;
  uint32_t word = 0;
  for (int q = 0; q < 32; ++q) {
    const size_t e = w * 32 + q;
    const size_t blk = e >> 4;
    const size_t bi = blk / (size_t)(nr / 4), bj = blk % (size_t)(nr / 4);
    const size_t i = bi * 4 + ((e >> 2) & 3), j = bj * 4 + (e & 3);
    if (i < (size_t)na && m[i * nr + j]) word |= 1u << q;
  }
  bits[w] = word;
}
}  // namespace

extern "C" int cssar_pack_mask(const cssar_op* op, const void* mask_bytes, void* mask_bits, void* stream) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!mask_bytes || !mask_bits) return fail(CSSAR_EINVAL, "NULL array");
  const size_t n = (size_t)op->na * op->nr;
  const size_t nw = (n + 31) / 32;
  const int block = 256;
  const unsigned grid = (unsigned)((nw + block - 1) / block);
  hipLaunchKernelGGL(pack_mask_kernel, dim3(grid), dim3(block), 0, (hipStream_t)stream,
                     (const unsigned char*)mask_bytes, (uint32_t*)mask_bits, op->na, op->nr);
  HIP_TRY(hipGetLastError());
  return CSSAR_OK;
}
