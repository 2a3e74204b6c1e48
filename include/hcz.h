/*
 * hcz.h - C ABI of libhcz, the MI355X (gfx950) implementation of the per-histogram hot
 * path of the hybrid compressor of Banerjee et al., "Scalable Hybrid Learning Techniques
 * for Scientific Data Compression" (arXiv 2212.10733).
 *
 * Pipeline (paper Section III, Fig. 1), per velocity-space histogram f[j][i]
 * (j = v_perp row, i = v_par column):
 *   moments b = A f                     (Section II, Eq. 1-4)
 *   encode z = encoder((f - mu) / sigma) (Stages 2-3)
 *   quantize codes = PQ(z)               (Stage 3, Section IV-E)
 *   decode fhat = sigma decoder(C[codes]) + mu
 *   residual r = f - fhat, coded under a per-histogram bound tau_h by a multilevel coder
 *   with a binary search over its quantisation ladder (Stage 4)
 *   Newton projection of ft = fhat + rhat onto {A x = b, x >= 0}; 4 multipliers lambda
 *   per histogram (Stage 5, Eq. 6)
 * Decompress rebuilds ft and applies f_c = max(0, ft - A^T lambda).
 *
 * Conventions
 *   - Pointers are device pointers unless marked (host).  Every call that takes a
 *     hipStream_t enqueues work on that stream and returns without synchronising,
 *     except hcz_stats_read, which synchronises the stream.
 *   - Buffers passed in are owned by the caller; the library never frees them.  Objects
 *     created by hcz_*_create / hcz_model_load own device memory of their own and are
 *     released by the matching destroy/free call.
 *   - Every entry point returns an hcz_status.  Argument errors are detected before any
 *     launch; a failed HIP call returns HCZ_EHIP.  hcz_last_error() gives the message of
 *     the calling thread's last failure.  No C++ exception crosses this interface.
 *   - Data-dependent outcomes (verbatim records, Newton fallbacks) are not errors: they
 *     are reported in the per-histogram flags and in hcz_stats.
 *   - A context is bound to one device; calls on one context may come from one host
 *     thread at a time.  Calls that overlap on one stream are ordered by the stream.
 */
#ifndef HCZ_H
#define HCZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hcz_stream_t;   /* a hipStream_t; NULL = the null stream */

typedef enum {
  HCZ_OK = 0,
  HCZ_EINVAL = -1,        /* bad argument (null pointer, size, mode, shape mismatch) */
  HCZ_ENOMEM = -2,        /* library-owned allocation failed */
  HCZ_EHIP = -3,          /* a HIP runtime call failed */
  HCZ_EUNSUPPORTED = -4,  /* valid request the library does not implement */
  HCZ_ECAPACITY = -5,     /* residual stream larger than the caller's capacity */
  HCZ_EWORKSPACE = -6     /* workspace smaller than the size query returned */
} hcz_status;

enum { HCZ_F32 = 0, HCZ_F64 = 1 };                       /* element types */
enum { HCZ_ARCH_DENSE = 1, HCZ_ARCH_CONV = 2 };           /* autoencoder architectures */
enum { HCZ_COMPUTE_FP32 = 0, HCZ_COMPUTE_BF16 = 1, HCZ_COMPUTE_FP64 = 2 };  /* autoencoder arithmetic */
enum { HCZ_TAU_REL_L2 = 0, HCZ_TAU_NRMSE = 1 };          /* tau_h = tau ||f||, tau sqrt(N)(max-min) */
enum { HCZ_FALLBACK_BACKTRACK = 0, HCZ_FALLBACK_PAPER = 1 };
enum { HCZ_BOUND_AB = 0, HCZ_BOUND_UB = 1 };                /* coder step: searched, user-specified */
enum { HCZ_SEARCH_GUIDED = 0, HCZ_SEARCH_BISECT = 1 };      /* how the coder step is searched */
enum { HCZ_FLAG_CODED = 1, HCZ_FLAG_ROUND2 = 2, HCZ_FLAG_RAW = 4, HCZ_FLAG_WARM_REJECTED = 8,
       HCZ_FLAG_NOCLIP = 16, HCZ_FLAG_KL = 32 };
enum { HCZ_WARM_COLD = 0, HCZ_WARM_MLP = 1, HCZ_WARM_ANALYTIC = 2 };

typedef struct hcz_ctx hcz_ctx;
typedef struct hcz_plan hcz_plan;
typedef struct hcz_model hcz_model;
typedef struct hcz_mlp hcz_mlp;

/* Velocity grid (Section II).  v_par_i = vpar_lo + i (vpar_hi - vpar_lo)/(n_par - 1),
 * likewise v_perp_j.  vol (host, [n_perp][n_par], copied) gives the cell volumes of
 * Eq. 1-4; NULL means dv_par * dv_perp for every cell.  mass is m of Eq. 3-4.
 * Supported sizes: 3 <= n_par, n_perp <= 128 and n_par * n_perp <= 4608. */
typedef struct {
  int32_t n_par, n_perp;
  double vpar_lo, vpar_hi, vperp_lo, vperp_hi;
  double mass;
  const double* vol;
} hcz_grid;

/* Dense autoencoder N -> hidden -> latent -> hidden -> N, ReLU after each hidden layer,
 * linear latent and output (Stage 2).  weights (host, FP32, copied) holds
 * W1[hidden][N], b1[hidden], W2[latent][hidden], b2[latent], W3[hidden][latent],
 * b3[hidden], W4[N][hidden], b4[N] back to back (y = x W^T + b).  norm_mean and
 * norm_std (host, [N]) are the per-pixel z-score statistics (Section IV-D).
 * Supported: hidden = 128, latent = 16.
 * compute: HCZ_COMPUTE_FP32 evaluates both products on FP32 matrix cores.
 *   HCZ_COMPUTE_BF16 (an arithmetic form of this library, not the paper's) gives the two
 *   large products bfloat16 operands with FP32 accumulation: x = (f - mean) * (1 / std)
 *   formed in FP32 (FP64 input rounded to FP32 first) and rounded to nearest-even
 *   bfloat16 against W1 rounded at load; h3 = relu(b3 + sum_d zhat_d W3[:, d]) as FP32
 *   fused multiply-adds in order d = 0..15, rounded likewise, against W4 rounded at load.
 *   The 128 -> latent and latent -> 128 layers stay FP32.
 *   HCZ_COMPUTE_FP64 (a checking form, one workgroup per histogram on the vector ALUs)
 *   evaluates every layer in FP64 with the weights and statistics widened exactly:
 *   x = (f - mean) / std (non-finite inputs as 0), every sum in index order with fused
 *   multiply-adds, fhat = std y + mean; z and fhat are stored rounded to FP32 where the
 *   other forms store them, so the quantiser and the residual stage see FP32 values.
 *   Compression and decompression evaluate the decoder with the same kernel, so they
 *   agree bit for bit in every form.
 * arch = HCZ_ARCH_CONV: the convolutional autoencoder of 39 x 39 grids (latent 16,
 *   compute = HCZ_COMPUTE_BF16; hidden is ignored).  weights (host, FP32) holds, back to
 *   back: c1w[32][1][3][3], c1b[32], c2w[64][32][3][3], c2b[64], fw[16][6400], fb[16],
 *   dw[6400][16], db[6400], t1w[64][32][3][3], t1b[32], t2w[32][1][3][3], t2b[1]
 *   (248,785 values).  Encoder: relu(conv1) 3x3 1 -> 32 stride 2 padding 1 (39 -> 20),
 *   relu(conv2) 32 -> 64 (20 -> 10), z = fw h2 + fb with h2 flattened channel-major;
 *   decoder: hd = relu(dw zhat + db) as 64 x 10 x 10, relu(transposed conv) 64 -> 32
 *   stride 2 padding 1 output padding 1 (10 -> 20), transposed conv 32 -> 1 (20 -> 39),
 *   fhat = std * y + mean.  conv1 and the decoder's dense layer are FP32 fused
 *   multiply-add chains (conv1 over the in-range taps in row-major order, the dense layer
 *   over d = 0..15); their ReLU outputs and the weights of conv2 and of the first
 *   transposed conv are rounded to nearest-even bfloat16 for the matrix cores (FP32
 *   accumulation); the rest is FP32.  Other grids or compute forms: HCZ_EUNSUPPORTED.
 *   The model owns a 419 MB device scratch buffer through which encode and decode pass
 *   their intermediate layer in chunks of 16,384 histograms: calls that use one
 *   convolutional model must not overlap (calls ordered on one stream are fine). */
typedef struct {
  int32_t arch;
  int32_t latent, hidden;
  const float* weights;
  const float* norm_mean;
  const float* norm_std;
  int32_t compute;
} hcz_model_desc;

/* Product-quantizer codebook (Section III Stage 3): centroids [latent][1 << bits]
 * (device, FP32), sorted within each latent dimension.  1 <= bits <= 8. */
typedef struct {
  int32_t bits;
  float* centroids;
} hcz_codebook;

/* Compression parameters.
 * tau, tau_mode    per-histogram bound tau_h (tau >= 0; tau = 0 makes every histogram
 *                  that needs a residual a verbatim record)
 * newton_s         Eq. 6 step size of round 1 (paper default 1.0)
 * newton_max_iter  round-1 update cap (paper: 50); newton_max_iter2: round-2 cap
 * fallback         round 2: Armijo backtracking, or the fixed step 0.01
 * fit_codebook     1: hcz_compress fits the codebook from the latents of every
 *                  sample_every-th histogram before quantising and writes it to the
 *                  codebook argument; 0: it uses the codebook given.
 * warm_start, mlp  HCZ_WARM_MLP: round 1 of the Newton solve starts from the warm-start
 *                  network's multipliers (hcz_compress with a model only); the start is
 *                  rejected, and the solve restarts cold, if its first Newton step makes
 *                  max_k |g_k| / sum_j |A_kj| x_j grow (flag HCZ_FLAG_WARM_REJECTED).
 *                  HCZ_WARM_ANALYTIC: round 1 starts from the multipliers of the projection
 *                  without positivity, lam0 = (A A^T)^-1 (A f~ - b), computed in the kernel
 *                  by one Newton step at lam = 0 over every cell; under the same acceptance
 *                  rule (and the same flag when it is dropped).  Exact when no cell of
 *                  f~ - A^T lam0 is negative.  mlp is not read.  Not combined with
 *                  no_positivity or kl (HCZ_EINVAL).
 * lambda_fp32      1: store the multipliers as FP32 (the paper's float multipliers,
 *                  Section I and Fig. 7: QoIs to about 1e-8 instead of 1e-14); the
 *                  compressed batch's lambda_fp32 must say the same.
 * no_positivity    1: the correction drops x >= 0 and becomes the orthogonal projection
 *                  onto {A x = b}, f_c = f~ - A^T lam with (A A^T) lam = A f~ - b (one
 *                  Newton step; flag HCZ_FLAG_NOCLIP); 0: the Stage-5 projection onto
 *                  {A x = b, x >= 0}.
 * kl               1: the KL (I-divergence) reading of Stage 5 first: f_c = argmin
 *                  sum x log(x / ft) - x + ft subject to A x = b over the cells with ft > 0,
 *                  i.e. f_c = max(ft, 0) exp(-A^T lam), solved by the same Newton rounds on
 *                  its dual.  It is not non-expansive, so it is kept (flag HCZ_FLAG_KL) only
 *                  where ||f - f_c|| <= (1 - 2^-20) tau_h; elsewhere the histogram gets the
 *                  L2 projection.  Runs on the wave-per-histogram kernels for grids that
 *                  fit one wave, on the workgroup-per-histogram kernel otherwise.
 *                  Not combined with no_positivity or a warm start (HCZ_EINVAL).
 * lambda_bits      0: multipliers stored as computed; 1..52: rounded (nearest, ties to
 *                  even) to that many mantissa bits before storage, the truncation of the
 *                  multipliers the paper allows to raise the compression level (Section I);
 *                  the QoI error grows like 2^-lambda_bits, and the PD bound holds up to
 *                  the change the rounding makes to f_c.  At most 23 with lambda_fp32.
 * tau_hist         NULL: every histogram uses tau.  Otherwise (device, FP64, [H]) histogram
 *                  h uses tau_hist[h] in place of tau (tau is then not read): per-subdomain
 *                  bounds in one call, see hcz_segment_tau.  A negative, infinite or NaN
 *                  entry makes that histogram a verbatim record.
 * bound_mode       HCZ_BOUND_AB (0): the coder's step is searched per histogram by the
 *                  search over the ladder below (the paper's 'ab', automatic error-bound
 *                  determination, Section IV-F).  HCZ_BOUND_UB (1): the step is the user's
 *                  ('ub', user-specified error bound): every coded histogram is quantised
 *                  with ladder step ub_level, without a search.  ub_level 0 is the step
 *                  whose a-priori error estimate ((L+1) Delta / 2 per cell) meets tau_h, so
 *                  the bound still holds; a larger ub_level trades the bound for ratio and
 *                  nothing checks ||f - f~|| against tau_h.  The selection (coded iff
 *                  ||r|| > (1 - 2^-20) tau_h) is the same in both modes.
 * ub_level         0..40, read only with HCZ_BOUND_UB.
 * search           how HCZ_BOUND_AB searches the ladder.  HCZ_SEARCH_GUIDED (0): an
 *                  exponential search from the predicted index round(4 log2(L+1)) (where an
 *                  estimate of independent quantisation errors meets tau_h): probe it, then
 *                  climb (+1, +3, +7, ...) while feasible or descend (-1, -3, ...) while
 *                  infeasible, and bisect the bracket; about half the probes of a plain
 *                  bisection on smooth data.  HCZ_SEARCH_BISECT (1): bisection over [0, 41).
 *                  Both end on a feasible k* whose successor is infeasible (or k* = 40);
 *                  where feasibility is not monotone in k they may end on different k*. */
typedef struct {
  double tau;
  int32_t tau_mode;
  double newton_s;
  int32_t newton_max_iter;
  int32_t newton_max_iter2;
  int32_t fallback;
  int32_t fit_codebook;
  int32_t sample_every;
  int32_t warm_start;
  const hcz_mlp* mlp;
  int32_t lambda_fp32;
  int32_t no_positivity;
  const double* tau_hist;
  int32_t kl;
  int32_t lambda_bits;
  int32_t bound_mode;
  int32_t ub_level;
  int32_t search;
} hcz_params;

/* Run statistics, written to device memory by compress and read with hcz_stats_read. */
typedef struct {
  uint64_t n_hist, n_coded, n_round2, n_raw;
  uint64_t stream_bytes;          /* bytes the residual stream needs */
  uint64_t overflow;              /* 1 if stream_bytes > res_capacity (nothing written past it) */
  uint64_t newton_max_iters;
  uint64_t newton_iters_total;
  uint64_t newton_iter_hist[64];  /* updates per histogram (last bin: >= 63) */
  uint64_t kstar_hist[48];        /* chosen ladder index of coded histograms */
} hcz_stats;

/* Compressed batch.  codes [H][latent] (u8; unused without a model), lambda [H][4]
 * (FP64, or FP32 when lambda_fp32 = 1), flags [H] (u8, HCZ_FLAG_*), res_offset [H+1]
 * (u64, exclusive scan of record sizes), res_bytes [res_capacity] (records in histogram
 * order), stats (device).  t_done: NULL, or (device, u64, [H]) the device wall clock
 * (hcz_wall_clock_hz ticks per second) at which the residual stage finished histogram h,
 * for per-subdomain completion times (hcz_segment_max, hcz_timestamp). */
typedef struct {
  uint8_t* codes;
  void* lambda;
  uint8_t* flags;
  uint64_t* res_offset;
  uint8_t* res_bytes;
  uint64_t res_capacity;
  hcz_stats* stats;
  int32_t lambda_fp32;
  uint64_t* t_done;
} hcz_compressed;

/* ---- context, plan, model ------------------------------------------------------- */

/* Create a context on HIP device `device` (sets it current on the calling thread). */
hcz_status hcz_create(int device, hcz_ctx** out);
void hcz_destroy(hcz_ctx* ctx);
/* Message of the calling thread's last failed call ("" if none); valid until the next call. */
const char* hcz_last_error(void);
/* Library version string, e.g. "hcz 0.1 gfx950". */
const char* hcz_version(void);

/* Device tables for one grid: basis phi_k of the four moments (Eq. 1-4; phi = 1,
 * v_par/V_par, (v_perp/V_perp)^2, (v_par/V_par)^2 with V = the grid's half extent) and
 * the multilevel node layout of the residual coder (Stage 4). */
hcz_status hcz_plan_create(hcz_ctx* ctx, const hcz_grid* grid, hcz_plan** out);
void hcz_plan_destroy(hcz_plan* plan);

/* Which per-histogram kernels serve `plan`'s grid (host only, no GPU work):
   HCZ_PATH_BLOCK one workgroup per histogram (the generic kernel; the KL reading),
   HCZ_PATH_WAVE one wave per histogram with the slot structure read at run time,
   HCZ_PATH_WAVE_FIXED one wave per histogram with a slot structure compiled in
   (the 39 x 39 grid with uniform cell volumes),
   HCZ_PATH_TEAM2 / HCZ_PATH_TEAM4 a team of two / four waves per histogram (grids too
   large for one wave whose nodes fit the team's slots, e.g. 49 x 49 / 65 x 65).  Records and flags are identical on every
   path; multipliers agree to the Newton stopping rule.
   Errors: HCZ_EINVAL for a NULL argument. */
enum { HCZ_PATH_BLOCK = 0, HCZ_PATH_WAVE = 1, HCZ_PATH_WAVE_FIXED = 2, HCZ_PATH_TEAM2 = 3, HCZ_PATH_TEAM4 = 4 };
hcz_status hcz_plan_path(const hcz_plan* plan, int32_t* path);

/* Launch variants of the residual stage (hcz_compress, hcz_residual) for tuning: the
 * kernel family and its shape, i.e. waves per histogram and nodes per thread.
 *   HCZ_VARIANT_AUTO          the default choice of hcz_plan_path (on the workgroup kernel
 *                             256 x 6, 512 x 5 or 512 x 9 threads x nodes per thread, the
 *                             smallest that holds the grid);
 *   HCZ_VARIANT_WAVE_FIXED    one wave per histogram, slot structure compiled in (the 39 x 39
 *                             grid with uniform cell volumes only);
 *   HCZ_VARIANT_WAVE          one wave per histogram, slot structure read at run time
 *                             (grids whose nodes fit 26 slots of 64);
 *   HCZ_VARIANT_BLOCK_256x6, _512x5, _512x9   the workgroup kernel with that many threads and
 *                             nodes per thread (N at most 1,536, 2,560, 4,608);
 *   HCZ_VARIANT_TEAM2, _TEAM4 a team of two or four waves per histogram with the wave
 *                             kernels' slot layout widened to 128 or 256 lanes (grids whose
 *                             nodes fit 22 slots of 128, resp. 20 slots of 256, e.g. 49 x 49
 *                             and 65 x 65).
 * Every variant gives the same records, offsets and flags; the multipliers agree to the
 * Newton stopping rule (the kernel families sum in different orders, so their last bits
 * may differ).  The KL reading runs on the wave kernels and the workgroup kernel; a
 * team variant then means the workgroup kernel.  hcz_plan_variants writes the variants valid for the
 * plan's grid (at most 8) to list (host) and their count to *n; hcz_plan_set_variant makes
 * one of them the plan's choice for later calls (not thread-safe against calls in flight
 * on other threads).  Errors: HCZ_EINVAL for a NULL argument, HCZ_EUNSUPPORTED for a
 * variant the grid does not allow. */
enum { HCZ_VARIANT_AUTO = 0, HCZ_VARIANT_WAVE_FIXED = 1, HCZ_VARIANT_WAVE = 2, HCZ_VARIANT_BLOCK_256x6 = 3,
       HCZ_VARIANT_BLOCK_512x5 = 4, HCZ_VARIANT_BLOCK_512x9 = 5, HCZ_VARIANT_TEAM2 = 6, HCZ_VARIANT_TEAM4 = 7 };
hcz_status hcz_plan_variants(const hcz_plan* plan, int32_t* list, int32_t* n);
hcz_status hcz_plan_set_variant(hcz_plan* plan, int32_t variant);

/* Copy an autoencoder to the device for `plan`'s grid (N = n_par * n_perp). */
hcz_status hcz_model_load(hcz_plan* plan, const hcz_model_desc* desc, hcz_model** out);
void hcz_model_free(hcz_model* model);

/* ---- stages (each one step of Section III, callable on its own) ------------------- */

/* Moments b[H][4] = A f and QoIs qoi[H][4] = (n, u_par, T_perp, T_par) (Eq. 1-4), and
 * norm[H] = ||f||_2 (correctly rounded sum of the rounded squares).  hist: H histograms,
 * element (h, j, i) at hist[h*hist_stride + j*row_stride + i] (elements); any output
 * pointer may be NULL. */
hcz_status hcz_qoi(const hcz_plan* plan, const void* hist, int32_t dtype, int64_t H,
                   int64_t hist_stride, int64_t row_stride, double* b, double* qoi,
                   double* norm, hcz_stream_t stream);

/* Encoder (Stages 2-3): z[H][latent] (FP32) of the z-scored histograms. */
hcz_status hcz_encode(const hcz_model* model, const void* hist, int32_t dtype, int64_t H,
                      int64_t hist_stride, int64_t row_stride, float* z, hcz_stream_t stream);

/* Codebook fit (Section IV-E): per latent dimension, 1-D k-means with k = 1 << bits on
 * the rows z[s * sample_every], s = 0..ceil(n/sample_every)-1, of z[n][latent]; initial
 * centroids at the (2c+1)/(2k) quantiles of the sorted sample; Lloyd updates until no
 * assignment changes (at most 25); empty clusters keep their centroid.  Writes
 * cb->centroids.  Workspace: hcz_codebook_fit_workspace. */
hcz_status hcz_codebook_fit_workspace(int64_t n, int32_t latent, int64_t sample_every,
                                      size_t* bytes);
hcz_status hcz_codebook_fit(const float* z, int64_t n, int32_t latent, int64_t sample_every,
                            hcz_codebook* cb, void* ws, size_t ws_bytes, hcz_stream_t stream);

/* Quantize (Stage 3): codes[n][latent] = #{c : (C[d][c] + C[d][c+1]) / 2 < z[n][d]}
 * (midpoints in FP64), the nearest centroid value with exact midpoints going low. */
hcz_status hcz_quantize(const float* z, int64_t n, int32_t latent, const hcz_codebook* cb,
                        uint8_t* codes, hcz_stream_t stream);

/* Decode (Stage 3): fhat[H][N] (FP32, row-major [j][i]) = sigma * decoder(C[codes]) + mu. */
hcz_status hcz_decode(const hcz_model* model, const uint8_t* codes, const hcz_codebook* cb,
                      int64_t H, float* fhat, hcz_stream_t stream);

/* Residual coding + QoI correction of H histograms against a given reconstruction
 * (Stages 4-5): fhat [H][N] FP32 row-major, or NULL for fhat = 0 (the coder-only
 * pipeline); lam0 [H][4] (FP64) warm-start multipliers or NULL (params->warm_start
 * HCZ_WARM_MLP is not used here; HCZ_WARM_ANALYTIC is, and then lam0 must be NULL).  Fills out->lambda, flags, res_offset, res_bytes, stats (codes
 * untouched).  Workspace: hcz_compress_workspace. */
hcz_status hcz_residual(const hcz_plan* plan, const hcz_params* params, const void* hist,
                        int32_t dtype, int64_t H, int64_t hist_stride, int64_t row_stride,
                        const float* fhat, const double* lam0, hcz_compressed* out, void* ws,
                        size_t ws_bytes, hcz_stream_t stream);

/* ---- whole path --------------------------------------------------------------------- */

/* Workspace bytes for hcz_compress / hcz_residual / hcz_decompress of H histograms. */
hcz_status hcz_compress_workspace(const hcz_plan* plan, const hcz_model* model, int64_t H,
                                  const hcz_params* params, size_t* bytes);
hcz_status hcz_decompress_workspace(const hcz_plan* plan, const hcz_model* model, int64_t H,
                                    size_t* bytes);

/* Compress H histograms: encode, (fit and) quantize, decode, residual coding, Newton.
 * model may be NULL (fhat = 0; cb unused).  The stream needs at most
 * H * (header + 4 N) bytes for FP32 input (H * 8 N for FP64). */
hcz_status hcz_compress(const hcz_plan* plan, const hcz_model* model, hcz_codebook* cb,
                        const hcz_params* params, const void* hist, int32_t dtype, int64_t H,
                        int64_t hist_stride, int64_t row_stride, hcz_compressed* out,
                        void* ws, size_t ws_bytes, hcz_stream_t stream);

/* Compression that allocates nothing, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results as hcz_compress, without the workspace: the
 * workspace is a scratch array of HCZ_STATIC_SCRATCH_BYTES (64 MiB) that the library holds
 * on every device it has a context on, from hcz_create until the process ends.  A batch is
 * accepted while the workspace hcz_compress would need for it (the layout for this dtype,
 * model and codebook fit) fits that array: about 5,000 FP32 or 3,500 FP64 histograms of
 * 39 x 39 with a model; larger batches return HCZ_EWORKSPACE, before any launch, with the
 * largest batch that fits in the message.  Every call on a device shares that device's
 * array and the array keeps the last call's contents (nothing in it needs to start at
 * zero): calls that overlap on one device, e.g. on two streams, race and give undefined
 * results; calls ordered on one stream are fine.  The caller still owns and passes the
 * input and every output buffer.  Errors: as hcz_compress. */
#define HCZ_STATIC_SCRATCH_BYTES (64u << 20)
hcz_status hcz_compress_static(const hcz_plan* plan, const hcz_model* model, hcz_codebook* cb,
                               const hcz_params* params, const void* hist, int32_t dtype, int64_t H,
                               int64_t hist_stride, int64_t row_stride, hcz_compressed* out,
                               hcz_stream_t stream);

/* Decompress (Section III, last paragraph): out[H][N] in out_dtype, row-major.
 * in_dtype is the element type the batch was compressed from (verbatim records).
 * A histogram whose record ends past in->res_capacity decodes to NaN. */
hcz_status hcz_decompress(const hcz_plan* plan, const hcz_model* model,
                          const hcz_codebook* cb, const hcz_compressed* in, int32_t in_dtype,
                          int64_t H, void* out, int32_t out_dtype, void* ws, size_t ws_bytes,
                          hcz_stream_t stream);

/* Synchronise `stream`, copy the device stats to host_out (host); returns
 * HCZ_ECAPACITY if the stream overflowed its capacity. */
hcz_status hcz_stats_read(const hcz_stats* dev_stats, hcz_stats* host_out, hcz_stream_t stream);

/* ---- batches of subdomains (one call per grid size, per-subdomain bounds) -----------
 * A batch of nseg subdomains laid out back to back: subdomain s holds histograms
 * [seg_start[s], seg_start[s+1]) (device, i64, [nseg+1], non-decreasing, seg_start[0] = 0,
 * seg_start[nseg] = H).  Entries out of that order are clamped to [0, H], so no access
 * leaves the arrays; the results are then unspecified.  nseg >= 1. */

/* tau_hist[h] = seg_tau[s] for seg_start[s] <= h < seg_start[s+1] (device arrays). */
hcz_status hcz_segment_tau(const int64_t* seg_start, const double* seg_tau, int32_t nseg, int64_t H,
                           double* tau_hist, hcz_stream_t stream);
/* seg_max[s] = max of t[h] over subdomain s (0 for an empty one): with hcz_compressed.t_done
 * the moment the subdomain's last histogram finished. */
hcz_status hcz_segment_max(const int64_t* seg_start, int32_t nseg, int64_t H, const uint64_t* t,
                           uint64_t* seg_max, hcz_stream_t stream);
/* *dst = the device wall clock when the stream reaches this call (device, u64). */
hcz_status hcz_timestamp(uint64_t* dst, hcz_stream_t stream);
/* Ticks per second of the device wall clock of HIP device `device`. */
hcz_status hcz_wall_clock_hz(int device, double* hz);

/* ---- one launch for the subdomains of several grids ----------------------------------
 * Compresses nseg batches whose grids may differ (a rank's subdomains at several
 * resolutions: Section III-A compresses every subdomain's histograms on their own) with
 * one launch of the residual stage (Stages 4-5) for all of them.  Segment k holds the
 * arguments of one hcz_compress call, with their meaning there (ws: that segment's
 * hcz_compress_workspace).  The model stages of the segments run first, in order, on
 * `stream`; then one persistent launch of as many workgroups as stay resident takes the
 * segments' histograms from one work list (four histograms of a grid whose nodes fit 26
 * slots of 64 lanes per item, one wave each; one histogram of a grid that fits 20 slots of
 * 256 lanes per item, a team of four waves), so the histograms of a small grid and of a
 * large one share the device instead of running launch after launch; then each segment's
 * records are compacted as hcz_compress compacts them.  Every segment gets the records,
 * offsets, flags, multipliers and stats that hcz_compress gives it with the variant
 * HCZ_VARIANT_WAVE (resp. HCZ_VARIANT_TEAM4), byte for byte; params->variant is not read.
 * batch_ws: device memory of at least HCZ_BATCH_WORKSPACE_BYTES bytes for the work counter,
 * reset by the call itself on `stream` (calls that overlap on one batch_ws race).
 * Errors: HCZ_EINVAL for nseg outside [1, HCZ_BATCH_MAX_SEGMENTS], plans of different
 * contexts or different dtypes; HCZ_EUNSUPPORTED for a batch mixing uniform and
 * non-uniform cell volumes, the KL reading, or a grid that fits neither layout;
 * HCZ_EWORKSPACE for a short batch_ws; otherwise as hcz_compress.  Every segment is checked
 * before the first launch.  With profiling on, a batch call times its residual launch only
 * (HCZ_STAGE_RESIDUAL). */
#define HCZ_BATCH_MAX_SEGMENTS 4
#define HCZ_BATCH_WORKSPACE_BYTES 256
typedef struct {
  const hcz_plan* plan;
  const hcz_model* model;     /* NULL: coder-only, as in hcz_compress */
  hcz_codebook* codebook;
  const hcz_params* params;
  const void* hist;           /* device */
  int32_t dtype;
  int64_t H, hist_stride, row_stride;
  hcz_compressed* out;
  void* ws;                   /* device, hcz_compress_workspace bytes for this segment */
  size_t ws_bytes;
} hcz_batch_segment;
hcz_status hcz_compress_batch(const hcz_batch_segment* seg, int32_t nseg, void* batch_ws, size_t batch_ws_bytes,
                              hcz_stream_t stream);

/* ---- output container and entropy coding (host) ------------------------------------
 * The buffer of one compressed batch in the order the paper gives (Section III, end of
 * Stage 5): a 44-byte header (scheme, sizes, byte boundaries, total size), the autoencoder
 * weights with the z-score statistics, the quantized codes, the PQ table, the residual
 * bytes (flags, record sizes, records) and the Lagrange multipliers.  entropy = 1 codes
 * the codes, the residual bytes and the multipliers with an order-0 byte-wise rANS coder
 * (12-bit frequencies, one table per section); entropy = 2 codes the residual records
 * by their integers instead: the headers and verbatim records as one byte stream, every
 * zigzag integer's bit length as a byte symbol in the stream of its coefficient group
 * (each stream with its own rANS table) and its bits below the leading one raw; unpacking
 * re-packs the integers with the records' widths, byte for byte (packing refuses a coded
 * record not in the coder's format).  Every pointer here is a host pointer; the caller
 * copies the device arrays of hcz_compressed to the host first.  Unpacking checks every
 * size against the buffer and fails with HCZ_EINVAL on a malformed or truncated buffer,
 * without reading past it. */
typedef struct {
  int64_t H;
  int32_t n_par, n_perp;
  int32_t arch;            /* 0: no model (coder-only), HCZ_ARCH_DENSE or HCZ_ARCH_CONV */
  int32_t compute;         /* HCZ_COMPUTE_* of the model */
  int32_t latent, bits;    /* codes per histogram and bits per code (model only) */
  int32_t lambda_fp32;     /* multipliers stored as FP32 */
  int32_t entropy;         /* 0: none; 1: rANS-coded codes, residual bytes and multipliers;
                              2: as 1, with the residual records coded by their integers
                              (per-group magnitude classes plus raw low bits) */
  int64_t n_weights;       /* floats in the weight blob of hcz_model_desc */
  uint64_t res_bytes;      /* residual record bytes (read_info output) */
  uint64_t total_bytes;    /* container size (read_info output) */
} hcz_container_info;

typedef struct {
  hcz_container_info info;
  const float* weights;       /* [n_weights] (the hcz_model_desc blob) */
  const float* norm_mean;     /* [N] */
  const float* norm_std;      /* [N] */
  const uint8_t* codes;       /* [H][latent] */
  const float* centroids;     /* [latent][1 << bits] */
  const uint8_t* flags;       /* [H] */
  const uint64_t* res_offset; /* [H+1] exclusive scan of record sizes */
  const uint8_t* res_bytes;   /* [res_offset[H]] */
  const void* lambda;         /* [H][4] FP64, or FP32 when lambda_fp32 */
} hcz_container_in;

typedef struct {              /* arrays of the sizes hcz_container_read_info implies */
  float* weights;
  float* norm_mean;
  float* norm_std;
  uint8_t* codes;
  float* centroids;
  uint8_t* flags;
  uint64_t* res_offset;       /* [H+1] */
  uint8_t* res_bytes;
  void* lambda;
} hcz_container_out;

/* Upper bound of the packed size, then the packing itself (*written = the size). */
hcz_status hcz_container_bound(const hcz_container_in* c, size_t* bytes);
hcz_status hcz_container_pack(const hcz_container_in* c, void* out, size_t capacity, size_t* written);
/* Header fields, the residual byte count and the total size of a packed buffer. */
hcz_status hcz_container_read_info(const void* buf, size_t n, hcz_container_info* info);
hcz_status hcz_container_unpack(const void* buf, size_t n, const hcz_container_out* out);
/* The rANS coder on its own: a block of n bytes needs at most hcz_rans_bound(n) bytes. */
hcz_status hcz_rans_bound(size_t n, size_t* bytes);
hcz_status hcz_rans_encode(const void* in, size_t n, void* out, size_t capacity, size_t* written);
hcz_status hcz_rans_decode(const void* in, size_t avail, void* out, size_t n);

/* ---- autoencoder training (Section III Stage 2, Eq. 5; Section IV-C) -------------------
 * The dense model of hcz_model_desc, trained with these kernels from torch.autograd.
 * params / grad: FP32 device vectors in the hcz_model_desc weights layout
 * (hcz_ae_param_count elements).  x: z-scored inputs [B][N] (device, FP32).
 * hcz_ae_forward writes z [B][latent], xhat [B][N] and the activations the backward
 * pass needs into `saved` (hcz_ae_saved_bytes; also the backward's scratch).
 * hcz_ae_backward takes dL/dz (or NULL for 0) and dL/dxhat and writes dL/dparams to
 * grad and, if dx is not NULL, dL/dx [B][N].  compute: HCZ_COMPUTE_FP32, every product on
 * FP32 matrix cores; HCZ_COMPUTE_BF16, both operands of every product (forward and
 * backward) rounded to the nearest bfloat16 and multiplied on BF16 matrix cores with FP32
 * accumulation, while parameters, gradients, biases, ReLU and the loss stay FP32 (FP32
 * master weights under hcz_adam_step).  Fixed reduction order (no atomics); any other
 * compute value is HCZ_EINVAL.  saved layout (FP32): h1 [B][128], h3 [B][128], then the
 * backward's dL/da3 [B][128], dL/da1 [B][128] and dL/dz [B][latent]. */
hcz_status hcz_ae_param_count(int32_t N, int64_t* count);
hcz_status hcz_ae_saved_bytes(int32_t N, int64_t B, size_t* bytes);
hcz_status hcz_ae_forward(int32_t N, int32_t compute, const float* params, const float* x, int64_t B,
                          float* z, float* xhat, void* saved, size_t saved_bytes, hcz_stream_t stream);
hcz_status hcz_ae_backward(int32_t N, int32_t compute, const float* params, const float* x, int64_t B,
                           const float* dz, const float* dxhat, void* saved, size_t saved_bytes,
                           float* grad, float* dx, hcz_stream_t stream);
/* Convolutional model (39 x 39; the parameter blob in the hcz_model_desc order, 248,785
 * floats): forward writes z [B][16] and xhat [B][1521] for z-scored x [B][1521] and keeps
 * the pre-activations in `saved`; backward accumulates nothing: it writes grad [248,785]
 * (dL/dparams for dL/dxhat = dxhat and, if dz is not NULL, an extra dL/dz) from the same
 * saved buffer.  Sizes: hcz_conv_ae_saved_bytes.  compute HCZ_COMPUTE_FP32: FP32
 * operands; HCZ_COMPUTE_BF16: both operands of every product of both passes (convolutions,
 * transposed convolutions, dense layers, weight gradients) rounded to the nearest bfloat16,
 * exact products, FP32 accumulation (FP64 in the convolution weight gradients); biases,
 * ReLU, bias gradients, the loss and Adam stay FP32 on FP32 master weights (Section III
 * Stage 2 trains the autoencoder; reduced precision is this library's option).  Both
 * passes of one step take the same compute. */
hcz_status hcz_conv_ae_param_count(int64_t* count);
hcz_status hcz_conv_ae_saved_bytes(int64_t B, size_t* bytes);
hcz_status hcz_conv_ae_forward(int32_t compute, const float* params, const float* x, int64_t B, float* z,
                               float* xhat, void* saved, size_t saved_bytes, hcz_stream_t stream);
hcz_status hcz_conv_ae_backward(int32_t compute, const float* params, const float* x, int64_t B,
                                const float* dz, const float* dxhat, void* saved, size_t saved_bytes,
                                float* grad, hcz_stream_t stream);
/* MSE of Eq. 5: *loss (device) = mean((xhat - x)^2) over n values; dxhat (or NULL) =
 * 2 (xhat - x) / n.  Workspace: hcz_mse_workspace bytes. */
hcz_status hcz_mse_workspace(size_t* bytes);
hcz_status hcz_mse(const float* xhat, const float* x, int64_t n, float* loss, float* dxhat,
                   void* ws, size_t ws_bytes, hcz_stream_t stream);
/* One Adam update (Kingma & Ba) of n parameters in place; step counts from 1. */
hcz_status hcz_adam_step(float* params, const float* grad, float* m, float* v, int64_t n,
                         double lr, double beta1, double beta2, double eps, int64_t step,
                         hcz_stream_t stream);
/* Per-pixel z-score statistics (Section IV-D): mean and population std over H
 * histograms (FP64 two-pass), std floored at 1e-12 * max std; written as FP32 [N]. */
hcz_status hcz_norm_stats_workspace(const hcz_plan* plan, int64_t H, size_t* bytes);
hcz_status hcz_norm_stats(const hcz_plan* plan, const void* hist, int32_t dtype, int64_t H,
                          int64_t hist_stride, int64_t row_stride, float* mean, float* std,
                          void* ws, size_t ws_bytes, hcz_stream_t stream);

/* The same statistics for any matrix x [rows][cols] (row stride ld >= cols elements, FP32
 * or FP64): per-column mean and population std (FP64 two-pass), std floored at 1e-12 times
 * the largest std, written as FP32 [cols]; e.g. the scales of the warm-start targets.
 * Workspace: hcz_column_stats_workspace bytes.  Errors: HCZ_EINVAL for NULL pointers, an
 * unknown dtype or a bad shape, HCZ_EWORKSPACE for a short workspace. */
hcz_status hcz_column_stats_workspace(int64_t rows, int64_t cols, size_t* bytes);
hcz_status hcz_column_stats(const void* x, int32_t dtype, int64_t rows, int64_t cols, int64_t ld, float* mean,
                            float* std, void* ws, size_t ws_bytes, hcz_stream_t stream);
/* z-scoring of training rows (Section IV-D: inputs are normalised before training):
 * out[r][c] = (x[r][c] - mean[c]) / std[c] (out dense [rows][cols], FP32), x rounded to FP32
 * first, then one FP32 subtraction and one FP32 division (round to nearest); mean NULL
 * means 0 (pure scaling).  x may be FP32 or FP64 with row stride ld.  Errors: HCZ_EINVAL. */
hcz_status hcz_column_normalize(const void* x, int32_t dtype, int64_t rows, int64_t cols, int64_t ld,
                                const float* mean, const float* std, float* out, hcz_stream_t stream);

/* ---- warm-start network (learned addition to Section III Stage 5) ----------------------
 * lam0 = scale * (W3 relu(W2 relu(W1 zhat + b1) + b2) + b3), 16 -> 64 -> 64 -> 4, with
 * zhat the dequantised latent.  params (host for hcz_mlp_load, device for training):
 * W1[64][16], b1[64], W2[64][64], b2[64], W3[4][64], b3[4] back to back (5,508 FP32);
 * scale (host) [4].  Training entry points mirror the autoencoder's: saved holds the
 * activations (hcz_mlp_saved_bytes), grad receives dL/dparams for dL/dout given. */
hcz_status hcz_mlp_load(hcz_ctx* ctx, const float* params, const double* scale, hcz_mlp** out);
void hcz_mlp_free(hcz_mlp* mlp);
hcz_status hcz_mlp_param_count(int64_t* count);
hcz_status hcz_mlp_saved_bytes(int64_t B, size_t* bytes);
hcz_status hcz_mlp_forward(const float* params, const float* z, int64_t B, float* out, void* saved,
                           size_t saved_bytes, hcz_stream_t stream);
hcz_status hcz_mlp_backward(const float* params, const float* z, int64_t B, const float* dout,
                            void* saved, size_t saved_bytes, float* grad, hcz_stream_t stream);
/* Dequantise codes [n][latent] with a codebook: z[n][d] = C[d][code[n][d]] (FP32). */
hcz_status hcz_dequantize(const uint8_t* codes, int64_t n, int32_t latent, const hcz_codebook* cb,
                          float* z, hcz_stream_t stream);
/* Warm-start multipliers lam0 [H][4] (FP64) of the network for codes [H][16]. */
hcz_status hcz_mlp_predict(const hcz_mlp* mlp, const uint8_t* codes, const hcz_codebook* cb, int64_t H,
                           double* lam0, hcz_stream_t stream);

/* ---- measured ceilings (measurement infrastructure, not part of compression) ----------
 * hcz_probe_copy: a streaming device-to-device copy of `bytes` (a multiple of 16, both
 * pointers 16-byte aligned; device), for the practical HBM rate.  hcz_probe_compute: a
 * launch of 2,048 workgroups of 256 threads whose loops keep every SIMD busy with
 * independent FP64 fused multiply-adds (8 chains per lane), FP32 matrix-core operations
 * (v_mfma_f32_32x32x2f32, 4 chains per wave) or BF16 matrix-core operations
 * (v_mfma_f32_32x32x16_bf16), `iters` times; *flops (host) receives the launch's operation
 * count (FMA = 2).  sink: device scratch of hcz_probe_sink_bytes bytes; its contents are
 * meaningless.  Errors: HCZ_EINVAL for NULL, misaligned or negative arguments or an unknown
 * kind, HCZ_EHIP when the launch fails. */
enum { HCZ_PROBE_FP64_FMA = 0, HCZ_PROBE_FP32_MFMA = 1, HCZ_PROBE_BF16_MFMA = 2 };
hcz_status hcz_probe_sink_bytes(size_t* bytes);
hcz_status hcz_probe_copy(const void* src, void* dst, size_t bytes, hcz_stream_t stream);
hcz_status hcz_probe_compute(int32_t kind, int64_t iters, void* sink, double* flops, hcz_stream_t stream);

/* ---- stage timing ---------------------------------------------------------------------
 * With profiling on, hcz_compress and hcz_decompress record a HIP event pair around every
 * kernel stage, on the caller's stream.  hcz_profile_read waits for the recorded events
 * and returns, per stage, the summed milliseconds (ms[HCZ_NSTAGES], host) and the number
 * of calls (calls[HCZ_NSTAGES], host) since the previous read, then resets. */
enum { HCZ_STAGE_ENCODE = 0, HCZ_STAGE_CODEBOOK, HCZ_STAGE_QUANTIZE, HCZ_STAGE_DECODE,
       HCZ_STAGE_RESIDUAL, HCZ_STAGE_SCAN, HCZ_STAGE_COMPACT, HCZ_STAGE_STATS,
       HCZ_STAGE_DECOMPRESS, HCZ_STAGE_WARMSTART, HCZ_NSTAGES };
hcz_status hcz_profile_enable(hcz_ctx* ctx, int enable);
hcz_status hcz_profile_read(hcz_ctx* ctx, double* ms, int64_t* calls);

#ifdef __cplusplus
}
#endif
#endif /* HCZ_H */
