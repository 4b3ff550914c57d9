/*
 * ehi.h - data-space Hessian build and inversion on one MI355X (gfx950).
 *
 * Implements the direct inversion of the data-space Hessian of time-domain
 * extended-source waveform inversion (Sonbolestan & Gholami, arXiv 2512.16642):
 * the multipliers delta d^e = Q^{-1} delta d of the deblurring system, with
 * Q = S S^T + mu I (Theory section, the Hessian definition and the deblurring
 * system), solved one frequency at a time on the block-diagonal Fourier form
 * (frequency-domain inversion).
 *
 * Pipeline (one survey = one model, one receiver set, one time axis):
 *   ehi_build_green    Nr Green functions by 2D acoustic FD (one impulse source
 *                      per receiver, block equation of the Hessian) with the DFT
 *                      at the nf requested frequencies accumulated during the
 *                      time loop; the time samples are never stored in full.
 *   ehi_build_hessian  Hhat(w) = Ghat(w) Ghat(w)^H over the grid for every w
 *                      (the Fourier diagonal of each block, taken in the long
 *                      record limit where the finite-record weighting is a
 *                      constant; computation of the Fourier diagonals).
 *   ehi_factor         Qhat(w) = Hhat(w) + mu I, Cholesky Qhat = L L^H in FP64,
 *                      kept resident (the paper inverts and stores each block).
 *   ehi_apply_multipliers
 *                      X(w) = Qhat(w)^{-1} R(w) for many sources at once.
 *
 * Conventions
 *   - All device pointers are hipMalloc'd (or torch-allocated) memory on the
 *     device that was current at ehi_create.  The library never allocates
 *     device memory: every buffer lives in the caller's workspace or in the
 *     caller's input/output arrays.
 *   - "stream" arguments are hipStream_t values passed as void*; NULL is the
 *     default stream.  Work is enqueued asynchronously; only ehi_factor and
 *     ehi_lambda_max wait on the stream (to read back a status or a value).
 *   - Complex arrays are interleaved (re, im): complex64 = 2 x float,
 *     complex128 = 2 x double.
 *   - Every entry point returns an ehi_status; on failure ehi_last_error()
 *     gives a message (thread-local, valid until the next call on the thread).
 *     Functions never throw and never abort.
 *   - A survey handle is not thread-safe: calls on one handle must not overlap.
 *     Different handles are independent.
 */
#ifndef EHI_H
#define EHI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EHI_OK = 0,
  EHI_EINVAL = 1,   /* bad argument or descriptor */
  EHI_ENOMEM = 2,   /* workspace smaller than ehi_workspace_bytes() */
  EHI_EHIP = 3,     /* a HIP runtime call failed (message names it) */
  EHI_ENOTPD = 4,   /* Qhat(w) not positive definite; index reported */
  EHI_ESTATE = 5    /* call out of order (e.g. factor before build_hessian) */
} ehi_status;

/* Arithmetic of the Hessian contraction, the factorisation and the solves. */
typedef enum {
  /* FP32 contraction, FP32 Cholesky, FP32 solves without refinement */
  EHI_PREC_PLAIN_FP32 = 0,
  /* split-BF16 (hi+lo) MFMA contraction with FP32 accumulation, FP64
     Cholesky, FP32 triangular solves + FP64 iterative refinement (one step
     by default, ehi_set_refinement) */
  EHI_PREC_SPLIT_BF16 = 1
} ehi_precision;

/* Weighting of the time-domain cross-correlations in the Fourier diagonals
 * (the weighting function of the algorithm for the Fourier block-diagonal
 * Hessian). */
typedef enum {
  /* W constant (long-record limit): Hhat(w) = Ghat(w) Ghat(w)^H with the final
     spectra (sum over the subgrid) */
  EHI_WEIGHT_LONG_RECORD = 0,
  /* W(m, n) = min(Nt - m, Nt - n): Hhat(w) = (1/Nt) sum_{p=1}^{Nt}
     Ghat_p(w) Ghat_p(w)^H, Ghat_p the DFT truncated after sample p.
     Requires EHI_PREC_SPLIT_BF16 and all receivers stepped together
     (nr_batch 0 or >= nr); computed during ehi_build_green. */
  EHI_WEIGHT_FINITE_RECORD = 1
} ehi_weighting;

/*
 * Survey descriptor.  Host memory; copied by ehi_create.
 *   nz, nx    interior grid, row-major [nz][nx], z pointing down.  >= 4 each.
 *   nb        absorbing layer width in cells on all four sides (0..512).
 *   h         grid spacing (m), dt time step (s); the FD scheme needs
 *             vmax*dt/h <= sqrt(3/8) for stability (not checked: vmax is
 *             only known on the device).
 *   nt        number of time steps; samples u^1..u^nt enter the DFT.
 *   stride    the Hessian contraction runs over interior cells (iz, ix) with
 *             iz % stride == 0 and ix % stride == 0 (stride 1, 2, 4 or 8).
 *   nr        receivers (1..1024); rec_iz/rec_ix are interior indices (host arrays of
 *             nr entries), 0 <= rec_iz < nz, 0 <= rec_ix < nx.
 *   nf        frequencies (1..64); freq_hz: host array of nf values >= 0 (Hz).  Any
 *             frequencies are allowed (not only 2nt-point transform bins).
 *   precision an ehi_precision value.
 *   max_ns    largest number of sources one apply launch processes; larger
 *             calls are split.  Sizes the refinement scratch.  >= 1.
 *   nr_batch  receivers time-stepped together (0 = all).  Sizes the
 *             wavefield buffers.
 *   weighting an ehi_weighting value.
 *   chunk     time samples per staging window of the DFT (0 = 256; 256, 512
 *             or 1024).  Each doubling halves the accumulator traffic of the
 *             DFT and doubles the staging buffer (nr_batch x chunk x subgrid
 *             floats).
 *   keep_z, keep_x  spatial compression of the contraction (the orthonormal
 *             transform of the spatial axis the paper's discussion proposes):
 *             0, 0 = contract over the subgrid points; otherwise each
 *             spectrum row, as an nzs x nxs image, is transformed by the
 *             orthonormal 2D DCT-II and only the leading keep_z x keep_x
 *             coefficients enter Hhat (exact when all are kept).  Long-record
 *             weighting only.
 *   windows   staging windows (0 = 1; 1 or 2).  With 2, the DFT of a full
 *             window runs on a second, library-owned stream while the time
 *             steps fill the other window, at twice the staging memory.
 *             Results do not depend on it.
 *   decim     time-axis resampling of the finite-record weighting (0 or 1 =
 *             every sample; D = 2..64 keeps every D-th sample; the paper's
 *             numerical examples resample the record in time before forming
 *             the Hessian).  The record is low-pass filtered first (zero-phase
 *             Kaiser-windowed sinc, 120 dB: passband up to the highest
 *             frequency f_max, stopband from 1/(D dt) - f_max, half-length
 *             K = ceil((120 - 7.95) / (2 * 14.36 * (1/D - 2 f_max dt))),
 *             unit sum), kept at the times n_q = 1 - K + q D, and
 *               Hhat(w) = (D / Nt) sum_{q: 1 <= n_q <= Nt} Gt_q(w) Gt_q(w)^H,
 *               Gt_q(w) = (D / H(w)) sum_{m <= q} y_m exp(-i w n_m dt),
 *             H(w) the filter's response; the spectra of ehi_copy_green_dft
 *             are Gt_last.  Requires EHI_WEIGHT_FINITE_RECORD, windows 1,
 *             1/(D dt) > 2 f_max, K <= 512 and 2K <= chunk, D <= chunk / 2.
 *   herk_split  partitions of the grid sum in the contraction (0 = chosen
 *             from the sizes, at least enough that no partition adds more
 *             than 40 stages of 32 grid points into its FP32 running sums;
 *             1..64).  Changes the order of the FP32 partial sums only
 *             (partitions are reduced in FP64 in a fixed order); fewer
 *             partitions than the default leave a larger rounding error,
 *             which grows about linearly with the stages per partition.
 *   herk_form   final-spectrum contraction: 0 = chosen from the sizes;
 *             split-BF16: 1 = whole-matrix form (the rows of a grid stage
 *             staged once per group of 32 x 32 block pairs: every row up to
 *             224 receivers, the eight row blocks of a 4 x 4 tile of block
 *             pairs above), 2 = 64 x 64 tile pairs; plain FP32: 0-2 = 64 x 64 tile pairs on the FP32
 *             matrix cores, 3 = FP32 products on the vector units.  Ignored by
 *             the other contractions.
 */
typedef struct {
  int32_t nz, nx, nb;
  double h, dt;
  int32_t nt;
  int32_t stride;
  int32_t nr;
  const int32_t* rec_iz;
  const int32_t* rec_ix;
  int32_t nf;
  const double* freq_hz;
  int32_t precision;
  int32_t max_ns;
  int32_t nr_batch;
  int32_t weighting;
  int32_t chunk;
  int32_t keep_z, keep_x;
  int32_t windows;
  int32_t decim;
  int32_t herk_split;
  int32_t herk_form;
} ehi_survey_desc;

typedef struct ehi_survey ehi_survey;

/* Bytes of device workspace the survey needs (256-byte aligned start
 * required).  Returns 0 for an invalid descriptor (see ehi_last_error). */
size_t ehi_workspace_bytes(const ehi_survey_desc* desc);

/* Creates a survey handle over a caller-owned workspace of ws_bytes bytes at
 * workspace_dev (device memory, 256-byte aligned, kept alive until
 * ehi_destroy).  Copies the descriptor's host arrays.  Enqueues the twiddle
 * table set-up (FP64 exp(-i w n dt) rounded to complex64, n = 1..nt) on
 * stream and waits for it.  *out receives the handle. */
ehi_status ehi_create(const ehi_survey_desc* desc, void* workspace_dev, size_t ws_bytes,
                      void* stream, ehi_survey** out);

/* Time-steps the nr Green functions through the velocity model vel_dev
 * (device, float32 [nz][nx] in m/s, read-only, caller-owned, only read by work
 * enqueued by this call) and accumulates
 *   Ghat[f][r][x'] = sum_{n=1}^{nt} g_r(n, x') exp(-i 2 pi freq_hz[f] n dt)
 * on the stride subgrid x' (interior only).  Medium set-up (sponge, padded
 * coefficients) runs on the device in FP64 and is rounded to FP32 once.
 * Asynchronous. */
ehi_status ehi_build_green(ehi_survey* s, const float* vel_dev);

/* Hhat(w_f)[i][j] = sum_x' Ghat[f][i][x'] conj(Ghat[f][j][x']) for all f,
 * Hermitian by construction (upper tiles computed, lower mirrored, imaginary
 * part of the diagonal zero).  Requires ehi_build_green or
 * ehi_load_green_dft first.  Asynchronous. */
ehi_status ehi_build_hessian(ehi_survey* s);

/* Qhat(w) = Hhat(w) + mu I (mu > 0, absolute), Cholesky factor of every
 * frequency, resident in the workspace.  Waits for the stream.  On a
 * non-positive pivot returns EHI_ENOTPD and stores the first failing
 * frequency index in *bad_freq (if non-NULL; -1 on success). */
ehi_status ehi_factor(ehi_survey* s, double mu, int32_t* bad_freq);

/* Batched factorisation of several surveys in one launch (uneven sizes and
 * either precision form): Qhat_k(w) = Hhat_k(w) + mu[k] I and the Cholesky
 * factor of every frequency of every survey, one workgroup per (survey,
 * frequency).  batch_ws: device memory of ehi_batch_workspace_bytes() bytes
 * for the job table (caller-owned, reusable once the call returns).  Work is
 * enqueued on stream, which the caller must order after the surveys' own
 * streams (e.g. by synchronising them); waits for the stream.  On a
 * non-positive pivot returns EHI_ENOTPD with the first failing (survey,
 * frequency) in *bad_survey, *bad_freq (either may be NULL); the other surveys
 * are factored. */
size_t ehi_batch_workspace_bytes(ehi_survey* const* surveys, int32_t n);
ehi_status ehi_factor_batch(ehi_survey* const* surveys, int32_t n, const double* mu,
                            void* batch_ws, size_t ws_bytes, void* stream, int32_t* bad_survey,
                            int32_t* bad_freq);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batched factorisation as ehi_factor_batch, with the job table in a static
 * device array of the library instead of a caller-provided batch_ws.  The
 * array holds up to 4096 (survey, frequency) jobs (288 KiB); each device the
 * library runs on keeps its own copy until the process ends.  Every survey
 * must live on the current device.  EHI_EINVAL if the batch has more jobs
 * than the table holds or a survey is on another device; otherwise the
 * arguments, stream ordering, waiting and EHI_ENOTPD reporting are those of
 * ehi_factor_batch, and the results are identical.  Allocates nothing.  The
 * table is shared by every call on a device: calls that overlap on one device
 * (from several host threads, before the previous call has returned) race and
 * must be serialised by the caller. */
ehi_status ehi_factor_batch_static(ehi_survey* const* surveys, int32_t n, const double* mu,
                                   void* stream, int32_t* bad_survey, int32_t* bad_freq);

/* Measurement aid (the roofline of the stepping kernel): a plain streaming
 * kernel over device buffers of `bytes` bytes each (a multiple of 16), to
 * measure the HBM rate the memory system delivers for an access mix.
 * mode 0: c = a + a (copy-like, 1 read + 1 write); 1: read a (sums to sink);
 * 2: read a, b, write c, d; 3: as 2 plus e over its first e_frac * bytes
 * (0 <= e_frac <= 2; e holds that many bytes) (the stepping kernel's mix:
 * u, w read; u, w and the staged samples written);
 * 4: read a, b (sums to sink).  sink: device float4 [grid * 256] (modes 1
 * and 4).  grid: workgroups of 256 threads (grid-stride loop).  Enqueued on
 * stream; the caller times it. */
ehi_status ehi_hbm_probe(int32_t mode, const void* a, const void* b, void* c, void* d, void* e, size_t bytes,
                         double e_frac, int32_t grid, void* sink, void* stream);

/* Refinement steps of ehi_apply_multipliers in the split-BF16 form (default
 * 1; 0..4): each step forms r = R - Qhat X in FP64 (X kept in FP64) and adds
 * the FP32 solve of r.  One step leaves an error of about (cond(Qhat) 2^-24)^2
 * of the solution; more steps matter only for very ill-conditioned systems.
 * EHI_EINVAL for steps > 0 in the plain FP32 form (no FP64 factors). */
ehi_status ehi_set_refinement(ehi_survey* s, int32_t steps);

/* Routes all later work of the survey to stream (a hipStream_t; NULL = the
 * default stream), e.g. to capture a build into a HIP graph or to run surveys
 * concurrently. */
ehi_status ehi_set_stream(ehi_survey* s, void* stream);

/* Launch shape of the Green-function stepping: time levels per launch
 * (4 or 8; 0 keeps the current value), rows per marching segment (16..512;
 * 0 keeps), and columns per marching workgroup (256, 384, 448 or 512; 0 picks
 * the width that covers the padded grid with the fewest lanes for the chosen
 * time levels; -1 keeps the current request).  Results do not depend on them
 * (used by the autotuner).  EHI_EINVAL for any other value. */
ehi_status ehi_set_launch(ehi_survey* s, int32_t tblock, int32_t seg_rows, int32_t band);

/* The current launch shape (host outputs; any pointer may be NULL). */
ehi_status ehi_get_launch(const ehi_survey* s, int32_t* tblock, int32_t* seg_rows, int32_t* band);

/* X(w) = Qhat(w)^{-1} R(w) for ns sources: resid_dev and mult_dev are device
 * complex64 arrays [nf][ns][nr] (frequency-major, one row of nr receiver
 * values per source).  They may not alias.  Enqueued on stream (NULL = the
 * survey's stream); asynchronous.  Requires a successful ehi_factor. */
ehi_status ehi_apply_multipliers(ehi_survey* s, const void* resid_dev, void* mult_dev,
                                 int32_t ns, void* stream);

/* max over frequencies of the largest eigenvalue of Hhat(w) (power
 * iteration in FP64), for choosing mu = eps * lambda_max.  Requires
 * ehi_build_hessian.  Waits for the stream. */
ehi_status ehi_lambda_max(ehi_survey* s, double* out);

/* Copies Ghat, complex64 [nf][nr][nzs][nxs] (nzs = ceil(nz/stride),
 * nxs = ceil(nx/stride)), to the device buffer out_dev.  Asynchronous.
 * EHI_EINVAL for a compressed survey (keep_z > 0), which holds one receiver
 * batch's spectra at a time and keeps only their compressed form. */
ehi_status ehi_copy_green_dft(ehi_survey* s, void* out_dev);

/* Compressed surveys: copies the compressed spectra (the leading keep_z x
 * keep_x coefficients of the orthonormal 2D DCT-II of every spectrum row,
 * the orthonormal spatial transform of the paper's discussion), complex64
 * [nf][nr][keep_z][keep_x], to out_dev.  They are formed batch by batch
 * during ehi_build_green (or from the input of ehi_load_green_dft), so the
 * full spectra are never held.  EHI_EINVAL if the survey is not compressed.
 * Asynchronous. */
ehi_status ehi_copy_compressed(ehi_survey* s, void* out_dev);

/* Replaces Ghat by the caller's complex64 [nf][nr][nzs][nxs] device array, so
 * the later stages can be run on given spectra.  Asynchronous.  EHI_ESTATE for
 * a finite-record survey (its Hessian needs the time samples). */
ehi_status ehi_load_green_dft(ehi_survey* s, const void* in_dev);

/* Copies Hhat (no penalty), complex128 [nf][nr][nr] (full Hermitian), to
 * out_dev.  Requires ehi_build_hessian.  Asynchronous. */
ehi_status ehi_copy_hessian(ehi_survey* s, void* out_dev);

/* Replaces Hhat by the caller's complex128 [nf][nr][nr] device array, which
 * must be Hermitian (it is used as given).  Asynchronous. */
ehi_status ehi_load_hessian(ehi_survey* s, const void* in_dev);

/* Copies the Cholesky factors, complex128 [nf][nr][nr] lower-triangular
 * (upper part zero), to out_dev.  Requires ehi_factor.  Asynchronous. */
ehi_status ehi_copy_factor(ehi_survey* s, void* out_dev);

/* ---- Steps either side of the deblur and the Hessian accuracy test ---------
 *
 * The paper's extended-source algorithm deblurs time-domain residuals:
 * delta d^e = Q^{-1} delta d, back-propagates them as the source extension
 * delta b = S^T delta d^e, and its Hessian accuracy test compares the data with
 * the prediction of the extended wavefield, d - P u^e = delta d - S S^T
 * delta d^e (Theory: S = P A(m)^{-1}, Q = S S^T + mu I; numerical examples,
 * Hessian accuracy test).  The frequency-domain inversion carries the
 * residuals over with a transform of length 2 nt and the multipliers back
 * with its inverse, cropped to the record.
 *
 * S here is the forward operator of the Green functions' own scheme with its
 * source side on the stride subgrid (the grid points the Hessian contraction
 * runs over), so S S^T is the time-domain Hessian that Hhat approximates:
 *   S: f [nt][nzs][nxs] -> traces d [nr][nt], f^n entering the step that
 *      produces u^{n+1} (a u^{n+1} = 2u^n - b u^{n-1} + kappa (L4 u^n + f^n)),
 *      d[r][n-1] = u^n at receiver r, n = 1..nt;
 *   S^T: its transpose, a run in reversed time with the traces injected at the
 *      receivers.
 * Both time-step every field one level per launch in FP32 on the survey's
 * stream, using the wavefield buffers of the workspace (no allocation), in
 * batches of nr_batch fields. */

/* Loads the medium (sponge and padded coefficients of vel_dev, float32
 * [nz][nx] m/s) for ehi_forward_subgrid / ehi_backpropagate without time-
 * stepping the Green functions (ehi_build_green loads it too).  Leaves the
 * spectra, Hhat and the factors as they are.  Asynchronous. */
ehi_status ehi_set_medium(ehi_survey* s, const float* vel_dev);

/* data = S src for ns fields: src_dev float32 [ns][nt][nzs][nxs], data_dev
 * float32 [ns][nr][nt] (device, caller-owned, not aliased).  EHI_ESTATE if no
 * medium is loaded.  Asynchronous on the survey's stream. */
ehi_status ehi_forward_subgrid(ehi_survey* s, const float* src_dev, int32_t ns, float* data_dev);

/* src = S^T data for ns fields (the back-propagated source extension
 * delta b = S^T delta d^e): data_dev float32 [ns][nr][nt], src_dev float32
 * [ns][nt][nzs][nxs].  Receivers sharing a cell add.  EHI_ESTATE if no medium
 * is loaded.  Asynchronous on the survey's stream. */
ehi_status ehi_backpropagate(ehi_survey* s, const float* data_dev, int32_t ns, float* src_dev);

/* Residual spectra R[f][s][r] = sum_{n=1}^{nt} dres[s][r][n-1]
 * exp(-i 2 pi freq_hz[f] n dt) (the Green functions' sign and sample origin;
 * at a bin k = freq 2 nt dt it is bin k of the 2nt-point DFT of the zero-padded
 * record): dres_dev float32 [ns][nr][nt], resid_dev complex64 [nf][ns][nr],
 * ready for ehi_apply_multipliers.  Sums in FP64 over the complex64 twiddle
 * table.  Any frequencies.  Enqueued on stream (NULL = the survey's). */
ehi_status ehi_residual_spectra(ehi_survey* s, const float* dres_dev, int32_t ns, void* resid_dev,
                                void* stream);

/* Multipliers back to time: the inverse 2nt-point transform of the bins held
 * in mult_dev (complex64 [nf][ns][nr]; bins not among the survey's frequencies
 * count as zero; the record is real, so bin k stands for itself and its
 * conjugate 2nt - k), cropped to samples 1..nt:
 *   out[s][r][n-1] = (1/2nt) sum_f c_f Re(X[f][s][r] exp(+i 2 pi freq_hz[f] n dt)),
 * c_f = 1 for bins 0 and nt, 2 otherwise; out_dev float32 [ns][nr][nt].  Sums
 * in FP64.  EHI_EINVAL unless every frequency is a distinct bin k = freq_hz 2
 * nt dt in 0..nt (within 1e-6 of an integer).  Enqueued on stream (NULL = the
 * survey's). */
ehi_status ehi_multipliers_to_time(ehi_survey* s, const void* mult_dev, int32_t ns, float* out_dev,
                                   void* stream);

/* Misfit of the accuracy test for ns records of len values each (float32,
 * device): err = dd - pred (err_dev may be NULL) and relerr[s] = sum err^2 /
 * sum obs^2 (FP64, relerr_dev double [ns], device).  Enqueued on stream (NULL
 * = the default stream). */
ehi_status ehi_misfit(const float* dd_dev, const float* pred_dev, const float* obs_dev, int32_t ns,
                      int64_t len, float* err_dev, double* relerr_dev, void* stream);

/* ---- The Krylov baseline: conjugate gradients on Q x = dd ------------------
 *
 * The paper's comparison method (Introduction; Hessian accuracy test; Table of
 * PDE solves and CPU times): CG on the time-domain system Q x = dd with
 * Q = S S^T + mu I applied through one ehi_backpropagate and one
 * ehi_forward_subgrid per iteration (two PDE solves per source).  These four
 * calls are the vector arithmetic of one batched CG, ns independent records of
 * len float32 values each (device arrays [ns][len]); the per-record scalars
 * rr, pAp, rr_new, fit are device double [ns].  Each call is one launch, one
 * workgroup per record, FP64 sums in a fixed order; enqueued on stream (NULL =
 * the default stream).  EHI_EINVAL for ns < 0, len < 1 or a NULL pointer.
 * An iteration:  Ap = S (S^T p);  ehi_cg_shift_dot;  ehi_cg_update;
 *                ehi_cg_direction;  rr <- rr_new.  */

/* x = 0, r = p = dd, rr = r.r */
ehi_status ehi_cg_init(const float* dd_dev, int32_t ns, int64_t len, float* x_dev, float* r_dev,
                       float* p_dev, double* rr_dev, void* stream);

/* Ap += mu p (Ap holds S S^T p on entry), pAp = p.Ap */
ehi_status ehi_cg_shift_dot(float* ap_dev, const float* p_dev, double mu, int32_t ns, int64_t len,
                            double* pap_dev, void* stream);

/* alpha = rr / pAp (0 if pAp <= 0); x += alpha p; r -= alpha Ap;
 * rr_new = r.r; fit = |r + mu x|^2, which equals |dd - S S^T x|^2, the
 * accuracy test's misfit of the current iterate. */
ehi_status ehi_cg_update(float* x_dev, float* r_dev, const float* p_dev, const float* ap_dev,
                         const double* rr_dev, const double* pap_dev, double mu, int32_t ns, int64_t len,
                         double* rr_new_dev, double* fit_dev, void* stream);

/* p = r + (rr_new / rr) p (beta 0 if rr <= 0) */
ehi_status ehi_cg_direction(float* p_dev, const float* r_dev, const double* rr_new_dev, const double* rr_dev,
                            int32_t ns, int64_t len, void* stream);

/* Block operations of a Krylov basis (GMRES, the paper's second iterative
 * baseline): nvec float32 vectors of ns records of len values, vector j of
 * record s at v_dev + j * vstride + s * len (vstride >= len elements).  One
 * launch each, FP64 sums, enqueued on stream (NULL = the default stream).
 * EHI_EINVAL for negative or oversized counts or a NULL pointer. */

/* out[s][j] = V_j[s] . w[s] for j < nvec (out double [ns][nvec], device);
 * nvec, ns <= 65535. */
ehi_status ehi_mdot(const float* v_dev, int64_t vstride, int32_t nvec, const float* w_dev, int32_t ns,
                    int64_t len, double* out_dev, void* stream);

/* dst[s] = beta dst[s] + sum_j coef[s][j] V_j[s] (coef double [ns][nvec],
 * device; nvec <= 1024; dst [ns][len] must not overlap the V_j). */
ehi_status ehi_combine(const float* v_dev, int64_t vstride, int32_t nvec, const double* coef_dev, int32_t ns,
                       int64_t len, double beta, float* dst_dev, void* stream);

/* Event-based timing of the kernels a survey launches.  Kinds: */
enum {
  EHI_PROF_SETUP = 0,   /* medium, twiddle and wavefield set-up */
  EHI_PROF_STEP = 1,    /* Green-function time steps */
  EHI_PROF_DFT = 2,     /* DFT accumulation of the staged samples */
  EHI_PROF_HERK = 3,    /* Hessian contraction and its reduction */
  EHI_PROF_FACTOR = 4,  /* penalty and Cholesky */
  EHI_PROF_SOLVE = 5,   /* triangular solves and refinement */
  EHI_PROF_MODEL = 6,   /* forward/adjoint modelling and time/frequency transfer */
  EHI_PROF_KINDS = 8
};

/* enable != 0: from now on, every run of consecutive launches of one kind is
 * bracketed by a pair of HIP events recorded on the stream it is launched
 * on.  Events are host-side objects; no device memory is allocated.
 * enable == 0 stops recording (recorded pairs are kept until read). */
ehi_status ehi_profile_enable(ehi_survey* s, int enable);

/* Waits for every recorded event, adds the elapsed milliseconds of each kind
 * into ms[EHI_PROF_KINDS] and the number of kernel launches covered into
 * launches[EHI_PROF_KINDS] (both zeroed first), then releases the events. */
ehi_status ehi_profile_read(ehi_survey* s, double* ms, int64_t* launches);

/* Releases the handle (not the workspace) without waiting for the device:
 * the caller ensures no enqueued work still uses the survey before it frees
 * or reuses the workspace.  NULL is accepted. */
ehi_status ehi_destroy(ehi_survey* s);

/* Message of the last failing call on this thread ("" if none). */
const char* ehi_last_error(void);

/* Library version string. */
const char* ehi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EHI_H */
