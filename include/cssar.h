/*
 * cssar.h -- C ABI of the MI355X (gfx950) library for fast compressed-sensing
 * SAR imaging with an approximated observation operator.
 *
 * Method (Fang, Xu, Zhang, Hong, Wu, "Fast Compressed Sensing SAR Imaging
 * based on Approximated Observation"):
 *   - M is a matched-filter focusing chain (Section III.B, eq. (focus)); here
 *     the chirp-scaling algorithm named in Section III.D.1:
 *         M(Y) = F_eta^-1 [ Phi3 o F_tau^-1 [ Phi2 o F_tau [ Phi1 o F_eta Y ] ] ]
 *   - G = M^-1 is the approximated observation (Section III.B), obtained by
 *     inverting every step (Section III.C rules i) and ii)):
 *         G(X) = F_eta^-1 [ Phi1* o F_tau^-1 [ Phi2* o F_tau [ Phi3* o F_eta X ] ] ]
 *     With unitary DFTs and unimodular phases, G^H = M exactly (Theorem 1).
 *   - The solver is the iterative thresholding algorithm eq. (th2d) /
 *     Algorithm 1 with X^(0) = 0, step mu = 1 and complex soft threshold
 *     eq. (L12) at lambda.
 *   Phase screens (turns = radians / 2 pi), with D(f) = sqrt(1 - (c f/(2 fc v))^2),
 *   Km(f) = Kr / (1 - Kr c r_ref f^2 / (2 v^2 fc^3 D^3)) (Km = Kr if src = 0),
 *   tau_j = 2 r_ref / c + (j - N_r/2) / fs, R0_j = c tau_j / 2:
 *     Phi1 = exp(i pi Km (1/D - 1) (tau_j - 2 r_ref / (c D))^2)
 *     Phi2 = exp(i pi D / Km f_tau^2) exp(i 4 pi r_ref f_tau (1/D - 1) / c)
 *     Phi3 = exp(i 4 pi fc R0_j D / c) exp(-i 4 pi Km / c^2 (1 - D) (R0_j - r_ref)^2 / D^2)
 *   with f_eta = prf nu(k)/N_a, f_tau = fs nu(l)/N_r, nu the signed (fftfreq
 *   order) frequency index.
 *
 * Data layout: a scene or raw-data array is N_a x N_r complex64 (interleaved
 * float re, im; torch.complex64), row-major, row = one range line (azimuth
 * index i), column = one azimuth line (range index j).  All array pointers
 * are DEVICE pointers on the current HIP device unless stated otherwise.
 * Supported lengths: N in {64, 128, ..., 8192} and {768, 1536, 3072} for
 * both N_a and N_r.
 *
 * Ownership: the caller owns every array (inputs, outputs, workspace).  The
 * operator owns only its O(N_a + N_r) coefficient and twiddle tables and a
 * small status block, released by cssar_destroy_operator.  Inputs are never
 * written.  Outputs must not alias inputs or the workspace unless stated.
 *
 * Errors: every call returns CSSAR_OK (0) or a negative code; arguments are
 * validated on the host before any HIP call.  Kernels are enqueued
 * asynchronously on the given stream (a hipStream_t, passed as void*; NULL =
 * the null stream).  Errors found on the device (a non-finite residual norm)
 * are reported by cssar_sync_status.  cssar_last_error returns a thread-local
 * message for the last non-zero status.  Calls sharing one operator must not
 * run concurrently on different streams (they share its status block).
 */
#ifndef CSSAR_H
#define CSSAR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CSSAR_OK = 0,
  CSSAR_EINVAL = -1,       /* null pointer, non-positive size or parameter, lambda < 0 */
  CSSAR_EUNSUPPORTED = -2, /* a length outside the supported set, f_dc != 0 */
  CSSAR_EHIP = -3,         /* HIP runtime error (message in cssar_last_error) */
  CSSAR_ENONFINITE = -4,   /* NaN or Inf met in a residual norm */
  CSSAR_ENOMEM = -5        /* device allocation of the operator tables failed */
};

/* Radar parameters, SI units, double precision (stripmap model, Section
 * II.A; Table 2 lists the same fields). */
typedef struct cssar_params {
  double fc;    /* carrier frequency f0 [Hz] */
  double Kr;    /* range chirp rate [Hz/s] (bandwidth / pulse duration) */
  double Tp;    /* pulse duration [s] (not used by G or M) */
  double fs;    /* range sampling rate [Hz] */
  double prf;   /* pulse repetition frequency [Hz] */
  double v;     /* effective radar velocity [m/s] */
  double r_ref; /* reference (scene-centre) slant range [m], at column N_r/2 */
  double ba;    /* processed Doppler bandwidth [Hz] (not used by G or M) */
  double f_dc;  /* Doppler centroid [Hz]; must be 0 */
  int src;      /* 1: secondary range compression in Km; 0: Km = Kr */
} cssar_params;

typedef struct cssar_op cssar_op;

/* Azimuth FM rate at the reference range, K_a = 2 v^2 / (lambda_w r_ref)
 * with lambda_w = c / fc (the rate of the azimuth matched filter of eq.
 * (amf)); 0 for NULL or non-positive fc, r_ref.  Host call. */
double cssar_azimuth_fm_rate(const cssar_params* p);

/* *out = *in with the azimuth FM rate set to Ka (through the velocity,
 * v = sqrt(Ka lambda_w r_ref / 2)) and the range chirp rate set to Kr: the
 * parameterisation (K_a, K_r) in which cssar_ita_backward reports its
 * parameter gradients.  CSSAR_EINVAL for NULL pointers or non-positive or
 * non-finite rates.  Host call. */
int cssar_params_with_rates(const cssar_params* in, double Ka, double Kr, cssar_params* out);

/* Build an operator for an n_az x n_rg grid: FP64 per-Doppler-bin and
 * per-range-column coefficient vectors, FP32 twiddle tables, kernel plan.
 * Host call; allocates the operator's small device tables on the current
 * device.  *out is set only on success. */
int cssar_make_operator(const cssar_params* p, int n_az, int n_rg, cssar_op** out);

/* Focusing chains of an operator (cssar_operator_chain). */
#define CSSAR_CHAIN_CSA 0
#define CSSAR_CHAIN_RDA 1

/* Build an operator whose M is the range-Doppler algorithm the paper works
 * as its example (Section III.C, eq. (RDA)) and whose G is built from it by
 * the inversion rules with D = C^T for the interpolation (eqs. (CD),
 * (apob)), so G^H = M exactly (Theorem 1) and G is close to M^-1:
 *     M(Y) = F_eta^-1 [ P_eta o C[ F_tau^-1 [ P_tau o F_tau [ F_eta Y ] ] ] ]
 *     G(X) = F_tau^-1 [ P_tau* o F_tau [ D[ P_eta* o F_eta X ] ] ], then F_eta^-1
 *   P_tau = exp(i pi f_tau^2 / Kr); P_eta = exp(-i pi f_eta^2 / Ka(tau_j)),
 *   Ka = 2 v^2 / (lambda_w R0_j) (no constant phase);
 *   C (eq. (RCMCs)): U[j] = sum_{t = -K/2+1}^{K/2} V[(p + t) mod N_r] sinc(t - fr),
 *   p + fr = j + delta_j (p integer, 0 <= fr < 1), delta_j = tau_j (1/D - 1) fs
 *   range samples, sinc(x) = sin(pi x) / (pi x), K = taps.
 * taps: even, 2..32 and at most n_rg (CSSAR_EINVAL otherwise).  Every
 * operator entry point accepts such an operator except the batched and the
 * gradient ones (CSSAR_EUNSUPPORTED). */
int cssar_make_operator_rda(const cssar_params* p, int n_az, int n_rg, int taps, cssar_op** out);

/* CSSAR_CHAIN_CSA or CSSAR_CHAIN_RDA; CSSAR_EINVAL for NULL. */
int cssar_operator_chain(const cssar_op* op);

/* Release an operator and its tables (NULL is accepted). */
int cssar_destroy_operator(cssar_op* op);

/* Workspace bytes the caller must provide (device memory, 256-byte aligned
 * start; contents need not be initialised and are clobbered):
 *   mode 0: cssar_apply_G / cssar_apply_GH   (one array in the blocked layout)
 *   mode 1: cssar_ita_solve                  (three arrays in the blocked layout, and
 *           the sparse iterate: 4 N_a N_r / E bytes of support words, E the
 *           update plan's elements per thread, a count per column tile and
 *           2 N_a N_r bytes of value slots)
 *   mode 2: cssar_ita_solve_adaptive         (four arrays in the blocked layout, the
 *           support bits (4 N_a N_r / E bytes, E the column plan's elements per
 *           thread), 8.6 KB of selection state and its candidate keys, one
 *           4-byte key per 16 pixels, at least 4096)
 *   mode 3: cssar_ita_solve_safeguarded      (six arrays in the blocked layout, two
 *           sets of support bits and the selection state with its keys)
 * The blocked layout holds 4 x 4 blocks of 128 bytes with a 128-byte pad per
 * block row: (N_a/4) (32 N_r + 128) bytes per array.  Returns 0 for a NULL
 * operator or an unknown mode. */
size_t cssar_workspace_size(const cssar_op* op, int mode);

/* y_out = G x (approximated observation, Section III.B).  x and y_out are
 * N_a x N_r complex64 (row-major); ws: cssar_workspace_size(op, 0) bytes.
 * No two of x, y_out, ws may alias. */
int cssar_apply_G(cssar_op* op, const void* x, void* y_out, void* ws, void* stream);

/* x_out = G^H y = M y (focusing chain, Theorem 1).  Same layout rules. */
int cssar_apply_GH(cssar_op* op, const void* y, void* x_out, void* ws, void* stream);

/* Pack a row-major N_a x N_r byte mask (nonzero = sampled) into the bit
 * layout the solver reads: 32-bit words, LSB first, bit e set for the
 * element with blocked index e = ((i/4) (N_r/4) + j/4) 16 + (i%4) 4 + j%4.
 * mask_bits must hold ceil(N_a N_r / 32) words. */
int cssar_pack_mask(const cssar_op* op, const void* mask_bytes, void* mask_bits, void* stream);

/* Iterative thresholding, eq. (th2d) / Algorithm 1:
 *   X^(0) = 0;  for t < iters:  R = m o (y - G X^(t));  X^(t+1) = S_lambda(X^(t) + M R)
 * y: N_a x N_r complex64 raw data (entries outside the mask are ignored);
 * mask_bits: packed mask (cssar_pack_mask); lambda >= 0; iters >= 1;
 * x_out: N_a x N_r complex64 result X^(iters);
 * resid_hist: NULL or a device array of iters floats receiving ||R^(t)||^2;
 * ws: cssar_workspace_size(op, 1) bytes.  No two of y, x_out, ws may alias.
 * The iterate is kept spatially and sparsely: per group of E elements of a
 * column (one thread of the update pass), its support and its first two
 * nonzeros, or all E values where it holds more than two; so a sparse
 * iterate costs the update pass a read and a write of one array instead of
 * two reads and a write. */
int cssar_ita_solve(cssar_op* op, const void* y, const void* mask_bits, float lambda,
                    int iters, void* x_out, float* resid_hist, void* ws, void* stream);

/* Options of cssar_ita_solve_ex (zero-initialise; a NULL field keeps the
 * plain solver's behaviour). */
typedef struct cssar_solve_opts {
  const void* x0;     /* starting iterate X^(0) (N_a x N_r complex64, row-major,
                         device), or NULL for X^(0) = 0 (Algorithm 1) */
  float* resid_hist;  /* NULL or iters floats: ||R^(t)||^2, t = 0 .. iters-1 */
  float* l1_hist;     /* NULL or iters floats: ||X^(t+1)||_1 = sum |X_ij| */
  int* nnz_hist;      /* NULL or iters ints: nonzero count of X^(t+1) */
} cssar_solve_opts;

/* cssar_ita_solve with the options above.  Warm start: the iteration of
 * eq. (th2d) / Algorithm 1 goes on from X^(0) = opts->x0, so a solve of
 * n1 iterations followed by one of n2 from its result gives the image and
 * residual norms of a solve of n1 + n2 iterations bit for bit (the iterate
 * kept between passes is rebuilt from x0 exactly as the update pass leaves
 * it).  Per-iteration metrics: a small pass after each update reads the
 * sparse iterate (the last one reads x_out) and totals |X_ij| in FP64 in a
 * fixed order.  opts may be NULL; x0 must not alias y or ws (it may be
 * x_out: it is read before x_out is written). */
int cssar_ita_solve_ex(cssar_op* op, const void* y, const void* mask_bits, float lambda, int iters,
                       const cssar_solve_opts* opts, void* x_out, void* ws, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid allocation): cssar_ita_solve with its
 * workspace in a fixed device array of the library, CSSAR_STATIC_WORKSPACE_BYTES
 * per device, which each device holds from the library's load until the
 * process ends; the call allocates nothing.  Arguments as cssar_ita_solve,
 * without ws.  CSSAR_EINVAL when the solve needs a larger workspace
 * (cssar_workspace_size(op, 1) > CSSAR_STATIC_WORKSPACE_BYTES: beyond about
 * 1536 x 1536 pixels), when the current device is not the operator's, or
 * while per-launch timing is enabled (it creates events).  Every call on a
 * device shares that device's array: calls that overlap on one device (on two
 * streams, or from two host threads) race and corrupt each other's results. */
#define CSSAR_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int cssar_ita_solve_static(cssar_op* op, const void* y, const void* mask_bits, float lambda,
                           int iters, void* x_out, float* resid_hist, void* stream);

/* Iterative thresholding with both parameters set per iteration as Section
 * IV.B suggests (eq. (mure) and the threshold rule after it):
 *   R = m o (y - G X);  dX = M R;
 *   mu_t = ||dX_G||^2 / ||m o G(dX_G)||^2, dX_G = dX on the support of X
 *          (the normalized step of the cited iterative hard thresholding; the
 *          printed ratio is inverted), mu_t = 1 when the support is empty or
 *          either norm is 0;
 *   V = X + mu_t dX;  lambda_t mu_t = the (k+1)-th largest |V| (0 when k >= N_a N_r);
 *   X+ = S_{lambda_t mu_t}(V), which keeps the k largest entries of V.
 * The selection compares |V|^2 in FP32 (ties at the (k+1)-th value are not
 * kept).  y, mask_bits, x_out, resid_hist, iters: as cssar_ita_solve; k >= 0
 * the sparsity (CSSAR_EINVAL if negative); mu_hist, lambda_hist: NULL or
 * device arrays of iters floats receiving mu_t and lambda_t;
 * ws: cssar_workspace_size(op, 2) bytes.  No two of y, x_out, ws may alias.
 * Every step runs on the device; nothing is read back between iterations. */
int cssar_ita_solve_adaptive(cssar_op* op, const void* y, const void* mask_bits, long k, int iters,
                             void* x_out, float* mu_hist, float* lambda_hist, float* resid_hist,
                             void* ws, void* stream);

/* Largest max_shrinks of cssar_ita_solve_safeguarded. */
#define CSSAR_MAX_SHRINKS 16

/* cssar_ita_solve_adaptive with the support-change safeguard of the
 * normalized iterative hard thresholding that Section IV.B cites for its
 * step (the paper states no safeguard; the bound is that method's): after
 * the step X+ = S_{lambda_t mu_t}(X + mu_t dX), if the support of X+ differs
 * from that of X,
 *   omega = (1 - c) ||X+ - X||^2 / ||m o G(X+ - X)||^2   (no bound if the
 *           denominator is 0),
 * and while mu_t > omega, mu_t <- mu_t / (kappa (1 - c)) and the step
 * (V, lambda_t, X+) is taken again, at most max_shrinks times per
 * iteration.  An accepted step lowers 1/2 ||m o (y - G X)||^2 + lambda_t ||X||_1.
 * The loop runs on the device: each iteration launches the passes of
 * max_shrinks further rounds, which return at once when the loop has ended
 * (support unchanged or mu_t <= omega).  c in (0, 1), kappa (1 - c) > 1
 * (the Python binding defaults to c = 0.01, kappa = 2, max_shrinks = 2),
 * 0 <= max_shrinks <= CSSAR_MAX_SHRINKS; CSSAR_EINVAL otherwise.  mu_hist, lambda_hist receive
 * the accepted step and threshold; shrink_hist: NULL or a device array of
 * iters ints receiving the shrinks of each iteration.  Other arguments as
 * cssar_ita_solve_adaptive; ws: cssar_workspace_size(op, 3) bytes. */
int cssar_ita_solve_safeguarded(cssar_op* op, const void* y, const void* mask_bits, long k, int iters,
                                double c, double kappa, int max_shrinks, void* x_out, float* mu_hist,
                                float* lambda_hist, float* resid_hist, int* shrink_hist, void* ws,
                                void* stream);

/* ---------------------------------------------------------------- batch --
 * Many independent scenes (any supported shapes) solved together.  The
 * paper's method is single-scene; batching is an execution strategy: each
 * ITA step of eq. (th2d) / Algorithm 1 is applied to every scene by grouped
 * persistent kernels, one launch per pass kind and line length (a table of
 * per-scene arguments maps a global work index to (scene, line group)), so
 * an iteration over 64 scenes of four sizes takes 16 launches instead of 256.
 * The middle iterations can be replayed from a captured HIP graph, and an
 * autotuner picks, per line length and pass kind, the kernel plan variant
 * and the number of resident workgroups per compute unit by measuring them.
 * Results equal those of cssar_ita_solve on each scene (bit for bit with
 * the default plans, within rounding with tuned plans).  Residual norms are
 * not formed; each call checks every X^(iters) for NaN or Inf instead
 * (cssar_batch_sync_status). */
typedef struct cssar_batch cssar_batch;

/* Group count >= 1 operators (all made on the current device).  The
 * operators must outlive the batch.  Allocates the batch's small device
 * argument tables and a pinned host staging buffer. */
int cssar_make_batch(cssar_op* const* ops, int count, cssar_batch** out);

/* Release a batch (NULL is accepted; the operators are not released). */
int cssar_destroy_batch(cssar_batch* b);

/* Workspace bytes of cssar_ita_solve_batched: three blocked arrays per scene
 * (cssar_workspace_size(op, 1) each, 256-byte aligned).  0 for NULL. */
size_t cssar_batch_workspace_size(const cssar_batch* b);

/* Launch mode of the middle iterations: 0 direct launches, 1 replay of a HIP
 * graph of one iteration (captured on first use on a private stream,
 * launched on the caller's stream).  The autotuner also sets it. */
int cssar_batch_set_graph(cssar_batch* b, int on);

/* Measure the plan variants and workgroups-per-CU choices of the row pass
 * and of the residual and update column passes for every line length of the
 * batch, and graph versus direct launches; keep the fastest.  Before any
 * timing, every plan variant runs the pass on a seeded input beside the
 * default plan (the single-array solver's): a variant whose output lies
 * more than 1e-5 (relative L2 over the group's scenes) from the default's
 * is never chosen, also when the cache names it; cssar_batch_describe
 * reports each distance.  ws: a batch
 * workspace (cssar_batch_workspace_size bytes; clobbered).  cache_path:
 * NULL, or a text file of earlier results (one line per choice, keyed by the
 * device, pass, length and amount of work); matching lines are used without
 * measuring and new results are appended.  Synchronises the stream. */
int cssar_batch_autotune(cssar_batch* b, void* ws, const char* cache_path, void* stream);

/* Current choices as text (one line per pass kind and length, with the
 * parity-gate distance of every plan variant, "-" where not measured; then
 * the launch mode) into buf (NUL-terminated, truncated to len).  Returns the
 * full length. */
int cssar_batch_describe(const cssar_batch* b, char* buf, int len);

/* Iterative thresholding on every scene s (the iteration of cssar_ita_solve):
 * ys[s], mask_bits[s] (cssar_pack_mask with that scene's operator),
 * lambdas[s] >= 0 and x_outs[s] as for cssar_ita_solve; host arrays of
 * count device pointers / floats; ws: cssar_batch_workspace_size bytes.
 * Calls sharing one batch must be ordered on one stream. */
int cssar_ita_solve_batched(cssar_batch* b, const void* const* ys, const void* const* mask_bits,
                            const float* lambdas, int iters, void* const* x_outs, void* ws,
                            void* stream);

/* Wait for the stream; if a call since the last check left NaN or Inf in
 * some scene's X^(iters), return CSSAR_ENONFINITE with *scene (if not NULL)
 * the first such scene (else -1), and clear the flags. */
int cssar_batch_sync_status(cssar_batch* b, void* stream, int* scene);

/* ------------------------------------------------------------- gradient --
 * Derivatives of a loss L(X^(K)) of K unrolled iterations of eq. (th2d) /
 * Algorithm 1 (X^(0) = 0, mu = 1) with respect to the raw data y, the
 * threshold lambda and the radar parameters K_a = 2 v^2 / (lambda_w r_ref)
 * (the azimuth FM rate at the reference range, Section II.A) and K_r.  Not
 * in the paper: plain calculus on the iteration, using G^H = M (Theorem 1)
 * for the adjoints of the operators.  Convention: for a complex array the
 * gradient is dL/dRe + i dL/dIm (what torch returns for a real loss). */

/* Bytes of the checkpoint buffer of cssar_ita_forward: one blocked array
 * (cssar_workspace_size(op, 0)) per iterate X^(c every), 0 < c every < iters.
 * 0 for NULL or non-positive arguments. */
size_t cssar_checkpoint_size(const cssar_op* op, int iters, int every);

/* Workspace bytes of cssar_ita_backward: every + 4 blocked arrays. */
size_t cssar_grad_workspace_size(const cssar_op* op, int every);

/* cssar_ita_solve that also stores the azimuth spectra of the iterates
 * X^(every), X^(2 every), ... (before the last) in ckpt (device,
 * cssar_checkpoint_size bytes; may be NULL if that is 0).  x_out equals
 * cssar_ita_solve's bit for bit.  ws: cssar_workspace_size(op, 1) bytes. */
int cssar_ita_forward(cssar_op* op, const void* y, const void* mask_bits, float lambda, int iters,
                      int every, void* x_out, void* ckpt, void* ws, void* stream);

/* Reverse pass: given grad_x = dL/dX^(K) (N_a x N_r complex64, row-major)
 * and the checkpoints of cssar_ita_forward with the same y, mask, lambda,
 * iters and every, writes grad_y = dL/dy (row-major complex64; zero off the
 * mask) and grad_scalars (device, 3 doubles) = (dL/dlambda, dL/dK_a,
 * dL/dK_r).  Each checkpoint segment is recomputed once.  ws:
 * cssar_grad_workspace_size(op, every) bytes.  grad_y must not alias y,
 * grad_x or ws.  The operator's partial-sum buffer is used: calls sharing
 * an operator must be ordered on one stream. */
int cssar_ita_backward(cssar_op* op, const void* y, const void* mask_bits, float lambda, int iters,
                       int every, const void* ckpt, const void* grad_x, void* grad_y,
                       double* grad_scalars, void* ws, void* stream);

/* Synchronise the stream and report a deferred device-side error of this
 * operator (CSSAR_ENONFINITE if a residual norm was NaN/Inf), clearing it. */
int cssar_sync_status(cssar_op* op, void* stream);

/* Thread-local message for the last non-zero status returned on this thread. */
const char* cssar_last_error(void);

/* Per-launch timing, for measurement only.  While enabled, every pass kernel
 * an operator enqueues is bracketed by two HIP events on its stream.
 * cssar_profile_read waits for those events, returns the summed elapsed
 * milliseconds and launch counts per pass kind, and forgets them.  Kinds:
 * 0 row pass of M (Phi1, range FFT, Phi2, inverse, Phi3), 1 row pass of G
 * (conjugate screens, reverse order), 2 column forward azimuth FFT (with
 * optional mask and residual norm), 3 column inverse azimuth FFT, 4 column
 * update + soft-threshold pass, 5 column residual pass, 6 column threshold
 * adjoint, 7 column data adjoint, 8 column iterate adjoint, 9 column
 * restricted step (adaptive solver), 10 column masked norm and step, 11
 * column pre-threshold value, 12 column threshold at the selected value,
 * 13 adjoint row pass with M forward, 14 adjoint row pass with G forward,
 * 15 selection of the (k+1)-th largest magnitude (all its launches), 16
 * column update + soft-threshold pass of the sparse iterate (cssar_ita_solve).
 * ms_sum and counts hold CSSAR_PROFILE_KINDS entries. */
#define CSSAR_PROFILE_KINDS 17
int cssar_profile_enable(cssar_op* op, int on);
int cssar_profile_read(cssar_op* op, double* ms_sum, long* counts);

/* Whether a length is supported (1) or not (0). */
int cssar_supported_length(int n);

/* Kernel plan of a length, for inspection: elements per thread, number of
 * radix passes and the radices (radices must hold 8 ints).  Returns 0 or
 * CSSAR_EUNSUPPORTED. */
int cssar_plan_info(int n, int* elems_per_thread, int* n_passes, int* radices);

#ifdef __cplusplus
}
#endif

#endif /* CSSAR_H */
