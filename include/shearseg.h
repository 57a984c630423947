/*
 * shearseg.h - C ABI of the MI355X (gfx950) library for shearlet-regularised convex
 * multi-label image segmentation (Haeuser & Steidl, "Convex Multiclass Segmentation
 * with Shearlet Regularization", arXiv 1112.1805).
 *
 * The library computes, on one GPU, the ADMM iteration of Section 3 for the model
 *
 *     min_u  <u, s> + || Lambda (I_q (x) S) u ||_1 + iota_C(u)     (problemSegmentation)
 *
 * where S is the FFT-based, translation-invariant discrete shearlet transform of
 * Section 2 (a Parseval frame, S^T S = I), s the data term of eq. (computationOfs) and
 * C the per-pixel probability simplex.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call returns shs_status (0 = SHS_OK, < 0 = error); nothing throws across the ABI.
 *   shs_last_error() returns a thread-local message for the last failing call.
 * - d_* pointers are caller-owned DEVICE memory on the plan's device, contiguous and
 *   row-major; h_* pointers are caller-owned HOST memory.  The library never frees or
 *   retains caller memory beyond the call.
 * - Images are square N x N arrays indexed [y][x]; axis 0 carries the frequency omega_1 of
 *   the paper (the paper vectorises column-wise: a layout choice only).  Label-indexed
 *   arrays are label-major ([q][N][N], the "q layers" of Section 3).
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  All work is enqueued
 *   asynchronously on it; only calls that return host results (h_stats, h_energy)
 *   synchronise that stream before returning.
 * - Inputs are never written.  Outputs are defined only when the call returns SHS_OK.
 * - Filter order (used by d_c and d_psi layouts and by per-filter weights):
 *     0 = low-pass; then for each scale j = 0..J-1: the horizontal-cone shears
 *     k = -(2^j-1)..(2^j-1), the vertical-cone shears in the same order, then the two
 *     glued seam filters k = -2^j and k = +2^j.  eta = 1 + 4 (2^J - 1) filters
 *     (5, 13, 29, 61 for J = 1..4; Theorem 2.2's system, Remark 2.3's "61 images").
 * - Frequency scaling: filters are evaluated at xi = (4^J / N) * omega (omega the integer
 *   frequency of Section 2), which is the paper's integer grid when N = 4^J and keeps the
 *   J-scale radial partition exact up to the Nyquist frequency otherwise.  For even N the
 *   Nyquist bins hold sqrt((psi(w)^2 + psi(-w)^2)/2), which keeps sum_j psi_j^2 = 1 and
 *   the coefficients real.
 */
#ifndef SHEARSEG_H
#define SHEARSEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SHS_OK = 0,
  SHS_E_INVALID = -1,      /* bad argument (null pointer, size, parameter out of range) */
  SHS_E_UNSUPPORTED = -2,  /* valid per the paper but not implemented (e.g. image size) */
  SHS_E_NOMEM = -3,        /* device allocation for plan constants failed */
  SHS_E_DEVICE = -4,       /* a HIP runtime call or kernel launch failed */
  SHS_E_NUMERIC = -5,      /* NaN/Inf met in the FP64 residual reduction */
  SHS_E_WORKSPACE = -6     /* workspace missing or smaller than shs_workspace_bytes() */
} shs_status;

/* Storage type of the dominant ADMM state (the eta*q coefficient images); arithmetic is
 * FP32 throughout, residual and energy reductions FP64.  SHS_STORE_F16 holds |g| < 65504 for
 * the stored g = b_v + S u; since |b_v| <= gamma lambda_j and the first iterate is
 * u = -gamma s / 2, keep gamma * max(s) well below 1e4 (e.g. scale 8-bit images to [0, 1]).
 * shs_solve on an F16 plan always checks the last iteration for non-finite values (one
 * synchronisation) and returns SHS_E_NUMERIC if the state overflowed. */
typedef enum { SHS_STORE_F32 = 0, SHS_STORE_BF16 = 1, SHS_STORE_F16 = 2 } shs_store;

#define SHS_MAX_LABELS 8
#define SHS_MAX_CHANNELS 4

typedef struct shs_plan shs_plan;   /* opaque: filter bank, twiddles, sizes, device */

typedef struct {
  int32_t n;         /* image side N (square images, Section 2): a power of two in 64..2048, or a
                        multiple of 8 in 64..1024 whose prime factors are all <= 23 (mixed radix) */
  int32_t channels;  /* 1 = gray, 3 = RGB (data term only); 1..SHS_MAX_CHANNELS */
  int32_t q;         /* number of labels, 1..SHS_MAX_LABELS */
  int32_t J;         /* number of shearlet scales, J >= 1 and 4^J <= 2N */
  int32_t store;     /* shs_store */
} shs_shape;

typedef struct {
  const float* lambda;  /* HOST array: J+1 weights Lambda = (lambda_0 low-pass, lambda_1..lambda_J
                           per scale) as in Section 3, or eta per-filter weights; all >= 0 */
  int32_t lambda_len;   /* J+1 or eta */
  float gamma;          /* ADMM penalty gamma > 0 (Section 3, general ADMM) */
  int32_t iters;        /* maximum number of ADMM iterations, >= 0 */
  double tol;           /* 0: run exactly `iters`; > 0: stop after the first checked iteration
                           whose combined residual sqrt(|dy|^2 + |db|^2) <= tol * sqrt(q N^2) */
  int32_t check_every;  /* residual check period when tol > 0 (>= 1) */
  int32_t resume;       /* 0: start from v = w = b = 0; 1: continue from the state left in the
                           workspace by a previous shs_solve on the same plan and workspace */
} shs_params;

typedef struct {
  int32_t iters_done;
  double energy;            /* F(u*) = <u*, s> + sum_l sum_j lambda_j ||S_j u*_l||_1, exact (FP64 sum) */
  double energy_surrogate;  /* <w, s> + sum lambda_j |v| of the last iterate (free by-product) */
  double r_primal;          /* ||b^K - b^(K-1)||                 (b = (b_v, b_w)) */
  double r_dual;            /* ||y^K - y^(K-1)|| / gamma           (y = (v, w))     */
  double r_combined;        /* ||y^K - y^(K-1)||^2 + ||b^K - b^(K-1)||^2            */
} shs_stats;

/* ---- plan ------------------------------------------------------------------------
 * shs_plan_create validates the shape, selects `device` (HIP ordinal), allocates the plan's
 * constants in device memory (the eta filter spectra and FFT twiddles) and fills them on
 * the device.  Errors: SHS_E_INVALID (null, q/channels/J out of range),
 * SHS_E_UNSUPPORTED (N not a supported size), SHS_E_NOMEM, SHS_E_DEVICE.
 * The plan is immutable after creation and may be shared by concurrent calls that use
 * distinct workspaces. */
shs_status shs_plan_create(const shs_shape* shape, int device, shs_plan** out);
shs_status shs_plan_destroy(shs_plan* plan);

/* Bytes of device workspace every compute call on this plan needs (0 for a null plan).
 * The workspace starts with the ADMM state (shs_state_bytes bytes): copying that prefix
 * out and back is a checkpoint of a solve (see shs_params.resume). */
size_t shs_workspace_bytes(const shs_plan* plan);
size_t shs_state_bytes(const shs_plan* plan);

/* The plan's launch schedule as text (stable for the plan's life; "" for a null plan).
 * Mixed-radix plans (N not a power of two) choose it at creation by timing candidates on
 * their own kernels: rows per wave and waves per block of the row pass, the stage order of
 * the row and column FFTs, and the filters per synthesis work item; the choice is cached per
 * (GPU arch, N, J, q, store) for the process and, if the environment variable
 * SHEARSEG_TUNE_CACHE names a file, there too (SHEARSEG_TUNE=0 keeps the default schedule).
 * The stage order changes the FFT's rounding, so results are reproducible for a given
 * schedule. */
const char* shs_plan_describe(const shs_plan* plan);

/* eta = 1 + 4 (2^J - 1) (Theorem 2.2's system); -1 for J < 1. */
int32_t shs_num_filters(int32_t J);

/* Copy the plan's filter bank to d_psi, float32 [eta][N][N/2+1]: filter j at the FFT bins
 * (k0, k1), k1 <= N/2 (the other half follows from psi(-w) = psi(w)). */
shs_status shs_filters(const shs_plan* plan, float* d_psi, void* stream);

/* Data term of eq. (computationOfs), colour form of Section 4:
 * s[k][y][x] = sum_c |f[c][y][x] - codebook[k][c]|^p.
 * d_img: float32 [channels][N][N]; h_codebook: HOST float32 [q][channels]; p > 0;
 * d_s: float32 [q][N][N]. */
shs_status shs_datacost(const shs_plan* plan, const float* d_img, const float* h_codebook, float p,
                        float* d_s, void* stream);

/* Discrete shearlet transform S (Section 2, eq. (wichtig)) of `count` images (any
 * count >= 1; processed in groups of at most q): d_f float32 [count][N][N]  ->
 * d_c float32 [count][eta][N][N], c_j = ifft2(psi_j * fft2(f)).  Uses the workspace. */
shs_status shs_shearlet_forward(const shs_plan* plan, int32_t count, const float* d_f, float* d_c,
                                void* d_ws, size_t ws_bytes, void* stream);

/* Adjoint (= inverse, by the Parseval property) transform S^T (Section 2, inverse
 * paragraph): d_c float32 [count][eta][N][N]  ->  d_f float32 [count][N][N],
 * f = ifft2(sum_j psi_j * fft2(c_j)); any count >= 1. */
shs_status shs_shearlet_adjoint(const shs_plan* plan, int32_t count, const float* d_c, float* d_f,
                                void* d_ws, size_t ws_bytes, void* stream);

/* Shrinkage denoising S^T S_lambda S of `count` images (any count >= 1): the transform of
 * Section 2, the componentwise soft shrinkage of Section 3 (S_lambda(x) = x - clip(x,
 * +-lambda), zero for |x| <= lambda) with threshold lambda_j on every coefficient of
 * filter j, and the adjoint; with all lambda = 0 it returns f (Theorem 2.2).
 * h_lambda: HOST float32, lambda_len = J+1 (per scale, low-pass first, as shs_params) or
 * eta (per filter), entries finite and >= 0.  d_f, d_out: float32 [count][N][N] (may be
 * the same buffer).  The coefficient images are never stored: the shrinkage runs inside
 * the row pass between the forward and the adjoint column passes.  Uses the workspace. */
shs_status shs_shearlet_denoise(const shs_plan* plan, int32_t count, const float* h_lambda, int32_t lambda_len,
                                const float* d_f, float* d_out, void* d_ws, size_t ws_bytes, void* stream);

/* ADMM for (problemSegmentationADMM) (Section 3): starting from v = w = b = 0 (or the
 * workspace state if params->resume), run params->iters iterations of
 *   u = 1/2 [ S^T (v - b_v) + (w - b_w) - gamma s ]
 *   v = shrink_{gamma Lambda}(b_v + S u),  w = P_C(b_w + u),
 *   b_v += S u - v,  b_w += u - w
 * (S applied per label).  d_s: float32 [q][N][N] data term.
 * Outputs: d_u float32 [q][N][N] = w^K (the relaxed labelling, in C); d_labels int32 [N][N]
 * = index of the largest entry of w^K per pixel, lowest index on ties, 0-based (either may
 * be NULL).  d_hist: NULL or float64 [iters][4] = (r_primal, r_dual, r_combined,
 * energy_surrogate) per iteration.  h_stats: NULL (no synchronisation) or receives the final
 * statistics, including the exact energy (one extra forward transform of w^K).
 * Launches: with tol = 0 and at least 10 iterations, the iterations between the first and
 * the last few are replayed from a captured HIP graph of 8 iterations (captured on a stream
 * of the plan's own at first use for a given workspace, data term, history buffer and
 * parameters, and kept by the plan, a few per plan); while kernel timing is on
 * (shs_profile_begin) every launch is eager.  Results are the same either way.
 * Errors: SHS_E_INVALID, SHS_E_WORKSPACE, SHS_E_DEVICE, SHS_E_NUMERIC (non-finite residual
 * at a checked iteration; with SHS_STORE_F16 the last iteration is always checked, which
 * synchronises the stream). */
shs_status shs_solve(const shs_plan* plan, const shs_params* params, const float* d_s, void* d_ws,
                     size_t ws_bytes, float* d_u, int32_t* d_labels, double* d_hist, shs_stats* h_stats,
                     void* stream);

/* Allocation-free variant of shs_solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and results as shs_solve except the workspace: the library keeps one
 * device array of SHS_NOALLOC_MAX_BYTES per GPU for the life of the process and uses it
 * in place of d_ws; the call itself allocates nothing (no hipMalloc / hipFree, and no graph
 * capture: every launch is eager).  Plans
 * whose shs_workspace_bytes() exceeds SHS_NOALLOC_MAX_BYTES are rejected with
 * SHS_E_WORKSPACE (at 64 MiB: e.g. 128^2 with q = 3, J = 2 fits; 512^2 with q = 4, J = 3
 * does not).  All calls on one GPU share that array and it keeps the last call's contents
 * (params->resume = 1 continues from the state the previous call on this GPU left there):
 * calls that overlap on one GPU race, so serialise them (one stream, or host-side order). */
#define SHS_NOALLOC_MAX_BYTES (64ull << 20)
shs_status shs_solve_noalloc(const shs_plan* plan, const shs_params* params, const float* d_s, float* d_u,
                             int32_t* d_labels, double* d_hist, shs_stats* h_stats, void* stream);

/* Parameters of the primal-dual solver.  lambda/lambda_len as in shs_params (the weights
 * of the regulariser, low-pass first); tau (primal) and sigma (dual) step sizes, finite,
 * > 0, tau * sigma <= 1 (the operator I_q (x) S has norm 1 by Theorem 2.2). */
typedef struct {
  const float* lambda;   /* HOST */
  int32_t lambda_len;
  float tau, sigma;
  int32_t iters;         /* >= 0 (0 returns the zero start) */
} shs_pd_params;

/* Primal-dual (Chambolle-Pock) solver for the same functional as shs_solve, the
 * alternative the paper names at the end of Section 3: from u = ubar = y = 0,
 *   y    = clip(y + sigma S ubar, +-lambda_j)          (per label and filter)
 *   u'   = P_C(u - tau (S^T y + s)),   ubar = 2 u' - u,   u = u'
 * The dual variable y takes the place of the ADMM state (same workspace, same storage
 * type); the dual step is fused into the row pass between the transform's column passes.
 * Outputs as shs_solve with u^K in place of w^K (it lies in C).  d_hist: NULL or float64
 * [iters][4] = (||u' - u||, ||y' - y||, ||u' - u||^2 + ||y' - y||^2,
 * <u', s> + sum_j lambda_j ||(S ubar)_j||_1) per iteration.  h_stats: as shs_solve
 * (r_primal = ||u' - u||, r_dual = ||y' - y|| of the last iteration, exact energy of u^K).
 * Errors: SHS_E_INVALID (bad steps or lambda), SHS_E_WORKSPACE, SHS_E_DEVICE,
 * SHS_E_NUMERIC (non-finite value seen by the last iteration's reduction). */
shs_status shs_solve_pd(const shs_plan* plan, const shs_pd_params* params, const float* d_s, void* d_ws,
                        size_t ws_bytes, float* d_u, int32_t* d_labels, double* d_hist, shs_stats* h_stats,
                        void* stream);

/* TV comparison model of Section 4 (the labels' gradients coupled per pixel):
 *   min_u <u, s> + lambda sum_pixels (sum_l |grad u_l|^2)^(1/2) + iota_C(u),
 * with the periodic forward-difference gradient, solved by the ADMM of Section 3 with grad
 * in place of S (the paper names no solver for it):
 *   u = (I + grad^T grad)^{-1} [grad^T (v - b_v) + (w - b_w) - gamma s]   (on the DFT)
 *   v = shrink_{gamma lambda}(b_v + grad u) per pixel over the 2q-vector,  w = P_C(b_w + u),
 *   b_v += grad u - v,  b_w += u - w,   from the zero state.
 * params: lambda_len must be 1 (one weight), gamma > 0, iters, tol/check_every as for
 * shs_solve; resume must be 0.  q <= 8.  The state (2q images in the plan's storage type)
 * uses the workspace of the shearlet solver.  Outputs, d_hist rows and h_stats as
 * shs_solve (energy = <w^K, s> + lambda TV(w^K); the surrogate uses lambda sum |v|).
 * Errors: SHS_E_INVALID, SHS_E_UNSUPPORTED, SHS_E_WORKSPACE, SHS_E_DEVICE, SHS_E_NUMERIC. */
shs_status shs_solve_tv(const shs_plan* plan, const shs_params* params, const float* d_s, void* d_ws,
                        size_t ws_bytes, float* d_u, int32_t* d_labels, double* d_hist, shs_stats* h_stats,
                        void* stream);

/* Nonlocal comparison model of Section 4: the NL-means graph replaces the gradient.
 * Graph parameters (Section 4's values: patch 5, window 15, a = 2, m = 5). */
typedef struct {
  int32_t patch;    /* odd patch side p */
  int32_t window;   /* odd search-window side (<= N) */
  float a;          /* standard deviation of the patch Gaussian */
  int32_t m;        /* neighbours picked per pixel, 1..8 (D has 2m blocks) */
} shs_nl_graph_params;

/* Builds the neighbour graph on the HOST (no device, no plan): for every pixel i in
 * row-major order, with l its weights already set, the k = min(m, 2m - l) eligible pixels
 * j of smallest Gaussian-weighted patch distance in the window get w(i, j) = w(j, i) = 1
 * (eligible: j != i, not yet a neighbour of i, fewer than 2m weights; ties to the smaller
 * linear index; periodic boundary; colour images sum the distance over channels).
 * h_img: HOST float32 [channels][N][N].  Outputs (HOST int32 [2m][N][N]): h_nbr[b][i] =
 * linear index of the b-th neighbour of i (order in which the weights were set) or -1;
 * h_rev[b][i] = the block b' with h_nbr[b'][h_nbr[b][i]] = i, or -1.  *h_max_degree (may
 * be NULL) = the largest number of neighbours.  Uses up to 16 host threads. */
shs_status shs_nl_graph(int32_t n, int32_t channels, const float* h_img, const shs_nl_graph_params* params,
                        int32_t* h_nbr, int32_t* h_rev, int32_t* h_max_degree);

/* Parameters of the NL solver.  blocks = 2m (rows of the graph arrays), max_degree from
 * shs_nl_graph; tau, sigma > 0 with tau * sigma * 4 * max_degree <= 1 (||D||^2 <= 4 max degree). */
typedef struct {
  float lambda, tau, sigma;
  int32_t iters;
  int32_t blocks;
  int32_t max_degree;
} shs_nl_params;

/* min <u, s> + lambda sum_i (sum_l sum_b (D_b u_l)(i)^2)^(1/2) + iota_C(u) with the graph
 * operator D ((D_b u)(i) = u(nbr[b][i]) - u(i), 0 without a b-th neighbour), by the
 * primal-dual iteration (I + D^T D is not diagonal in the DFT): from u = ubar = y = 0,
 *   y = P_ball(y + sigma D ubar) per pixel over labels and blocks (radius lambda),
 *   u' = P_C(u - tau (D^T y + s)),  ubar = 2 u' - u.
 * d_nbr, d_rev: DEVICE int32 [blocks][N][N] (shs_nl_graph's output).  The dual variable
 * (q * blocks images, the plan's storage type) lives in the state part of the workspace,
 * so the plan needs eta >= blocks (J >= 2 for m = 5).  q <= 8.  Outputs, d_hist rows and
 * h_stats as shs_solve_pd (energy = <u^K, s> + lambda NL-TV(u^K)).
 * Errors: SHS_E_INVALID, SHS_E_UNSUPPORTED, SHS_E_WORKSPACE, SHS_E_DEVICE, SHS_E_NUMERIC. */
shs_status shs_solve_nl(const shs_plan* plan, const shs_nl_params* params, const float* d_s, const int32_t* d_nbr,
                        const int32_t* d_rev, void* d_ws, size_t ws_bytes, float* d_u, int32_t* d_labels,
                        double* d_hist, shs_stats* h_stats, void* stream);

/* Energy F(u) = <u, s> + sum_l sum_j lambda_j ||S_j u_l||_1 of (problemSegmentation) for a
 * given u (float32 [q][N][N]; the indicator term is not evaluated).  Uses params->lambda /
 * lambda_len only.  Synchronises the stream; result in *h_energy (FP64 accumulation). */
shs_status shs_energy(const shs_plan* plan, const shs_params* params, const float* d_s, const float* d_u,
                      void* d_ws, size_t ws_bytes, double* h_energy, void* stream);

/* ---- batches of images --------------------------------------------------------------
 * A batch solves `count` independent problems of the model above (Section 3) whose images
 * may differ in size N, label count q, channel count and storage type; each element of
 * `shapes` follows the rules of shs_plan_create (one plan per distinct shape is created
 * inside the batch).  Image i uses its own region of one workspace
 * (shs_batch_workspace_bytes).
 *
 * shs_solve_batch runs params[i] on image i from the zero state (tol and resume are not
 * supported: SHS_E_UNSUPPORTED; every image runs the same number of iterations).  Each step
 * of an ADMM iteration is one grouped launch per kernel configuration covering all images
 * that use it (the blocks of every image's grid laid end to end, each block running exactly
 * the single-image kernel's code), and the whole solve (zero start, all iterations,
 * epilogue, statistics) is captured once into one HIP graph, replayed on `stream` with a
 * single graph launch.  Results equal separate shs_solve calls bit for bit.  The graph and
 * its task tables (device memory owned by the batch) are rebuilt whenever a pointer or
 * parameter differs from the previous call.  The call returns without synchronising.
 * d_s, d_u, d_labels: HOST arrays of `count` device pointers (d_u / d_labels and their
 * entries may be NULL); layouts as in shs_solve.  d_stats: NULL or DEVICE float64
 * [count][5] receiving, per image, the last iteration's |dy|^2, |db|^2, <w,s>,
 * sum lambda|v| and a non-finite flag (1.0 if any of them is not finite); all zeros
 * when iters = 0.
 * A batch object is not thread-safe (it owns its captured graphs). */
typedef struct shs_batch shs_batch;
/* count: 1..65535 images. */
shs_status shs_batch_create(int32_t count, const shs_shape* shapes, int device, shs_batch** out);
shs_status shs_batch_destroy(shs_batch* batch);
size_t shs_batch_workspace_bytes(const shs_batch* batch);
shs_status shs_solve_batch(shs_batch* batch, const shs_params* params, const float* const* d_s, void* d_ws,
                           size_t ws_bytes, float* const* d_u, int32_t* const* d_labels, double* d_stats,
                           void* stream);

/* ---- optional kernel timing (benchmarks) ------------------------------------------
 * Between shs_profile_begin() and shs_profile_end(), every kernel the library enqueues is
 * bracketed by a pair of HIP events recorded on the stream it is launched on.
 * shs_profile_end() waits for those events and returns, per kernel class, the number of
 * launches and the summed event-measured duration; it returns the number of classes
 * written (<= max_entries) or -1 on error.  Process-wide; not for concurrent solves.
 * shs_profile_begin_classes(list) times only the kernel classes named in the
 * comma-separated list (NULL or "" = all, as shs_profile_begin); each event pair sits on
 * the launch stream, so timing fewer classes disturbs the stream less.  An unknown name
 * returns SHS_E_INVALID and leaves the profiling state unchanged. */
typedef struct {
  char name[32];       /* kernel class: row_solve, col_syn, col_ana, col_final, row_c2r, ... */
  int64_t launches;
  double total_ms;
} shs_kernel_time;
shs_status shs_profile_begin(void);
shs_status shs_profile_begin_classes(const char* classes);
int32_t shs_profile_end(shs_kernel_time* out, int32_t max_entries);

const char* shs_status_str(shs_status status);
const char* shs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SHEARSEG_H */
