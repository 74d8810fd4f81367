/*
 * slicq.h - C ABI of the MI355X (gfx950) sliCQ library.
 *
 * The sliced constant-Q nonstationary Gabor transform (sliCQ) of Holighaus,
 * Doerfler, Velasco and Grill, "A framework for invertible, real-time
 * constant-Q transforms": a real signal is cut into Tukey-windowed slices of
 * length 2N at hop N (Section 4, Algorithm 3); each slice is transformed by the
 * painless constant-Q NSG frame (Section 3, Table 1; Algorithm 1):
 *
 *     c^m_{n,k} = <F x_m, M_{-n a_k} g_k> = sum_{j in J_k} X_m[j] g_k[j] e^{2 pi i j n / M_k}
 *
 * (equation CQ_coeff with the unitary DFT of Section 2.1), and synthesis
 * (Algorithm 2 per slice, Algorithm 4 across slices) reconstructs the signal
 * exactly with the canonical dual windows g~_k = g_k / sum_l M_l g_l^2
 * (Proposition 2) and the dual slicing window (equation dualwincond).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every int-returning call returns SLICQ_OK (0) or a negative
 *   slicq_status; slicq_last_error() then gives a message (thread-local).
 *   No exception crosses the ABI.
 * - Memory: all device buffers (signals, coefficients, outputs, workspace,
 *   tables) are owned by the caller and must be device memory of the current
 *   HIP device (coarse-grained, e.g. hipMalloc). The library allocates no
 *   device memory in any transform call.
 * - Streams: transform calls only enqueue work on `hip_stream` (a hipStream_t,
 *   NULL for the default stream) and never synchronise; launch failures are
 *   reported as SLICQ_EHIP.
 * - Plans are immutable after nsgt_plan_upload and may be shared between
 *   threads; concurrent calls must use distinct output and workspace buffers.
 * - Real signals: bands 0..K+1 (DC, K constant-Q bands, Nyquist) are stored.
 *   Bands K+2..2K+1 mirror bands K..1 and carry conjugate coefficients.
 * - Coefficient layout (complex interleaved re/im of the dtype), chosen per
 *   plan: band-major puts band k, slice m, index n < M_k at element
 *   S * off_k + m * M_k + n (each band a contiguous S x M_k array); slice-major
 *   puts it at m * C + off_k + n (each slice's c^m contiguous, Section 4.1),
 *   with off_k = sum_{k' < k} M_k', C = sum_k M_k, S = slices of the signal.
 */
#ifndef SLICQ_H
#define SLICQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slicq_plan_s* slicq_plan;

typedef enum {
  SLICQ_OK = 0,
  SLICQ_EINVAL = -1, /* invalid parameter or plan design (message says which) */
  SLICQ_ENOMEM = -2, /* host allocation failed */
  SLICQ_EHIP = -3,   /* a HIP runtime call or kernel launch failed */
  SLICQ_ESIZE = -4,  /* a caller buffer is too small */
  SLICQ_EBUSY = -5,  /* streaming server: admission refused (memory budget) */
  SLICQ_ESTATE = -6  /* call not valid in the current state (e.g. tables not uploaded) */
} slicq_status;

typedef enum { SLICQ_F32 = 0, SLICQ_F64 = 1 } slicq_dtype;

/* Plan parameters (Section 3: xi_min, xi_max, xi_s, B; Section 4.3: N, M). */
typedef struct {
  double fs;                /* sampling rate xi_s in Hz, > 0 */
  double fmin;              /* xi_min in Hz, 0 < fmin < fs/2 */
  double fmax;              /* xi_max in Hz, > fmin; >= fs/2 is clamped below Nyquist */
  int32_t bins_per_octave;  /* B >= 1 */
  int64_t slice_len;        /* 2N, a power of two in [16, 2^20] */
  int64_t transition_len;   /* Tukey transition M, 0 < M < N, N - M even */
  double min_win;           /* minimal band support in bins (Section 5.3), default 16 */
  int32_t dual_slice;       /* 0: canonical dual h_0 / sum_m T_mN h_0^2, 1: indicator of supp h_0 */
  int32_t group_cap;        /* tuning: coefficients per analysis work item (power of two, 16..4096), default 2048 */
  int32_t lds_cap;          /* tuning: target complex values per synthesis work item, own and overlapping
                               bands (64..16384), default 4096; a single band with the bands reaching
                               into its bins may exceed it, up to 16384 */
  int32_t pass_cap;         /* tuning: complex values per slice-FFT work item (power of two), default 4096 */
  int32_t coef_layout;      /* SLICQ_BAND_MAJOR (0) or SLICQ_SLICE_MAJOR (1), see below */
  int32_t window;           /* band window on |x| < 1/2: 0 Hann (default), 1 Blackman-Harris
                               (4 terms, the window of the approximation study, Section 5.3) */
  int32_t scale;            /* centre frequencies: 0 constant-Q (geometric, Section 3), 1 mel, 2 Bark
                               (Section 7): as many bands as constant-Q would place between fmin and
                               fmax, equally spaced on the scale, bandwidth = distance of the two
                               neighbouring centres (xi_k / Q for constant-Q) */
  int32_t slicing;          /* slicing window: 0 Tukey with sum_m h_m = 1 (default), 1 its square root,
                               sum_m h_m^2 = 1, so that the same windows serve in the overlap-add
                               (the other design of Section 4.3) */
  int32_t m_policy;         /* coefficients per band: 0 the smallest power of two >= |J_k| (default),
                               1 one M for every band, the largest of those (the rectangular
                               representation of Section 6), 2 the smallest even 2^a, 3 2^a or
                               5 2^a >= |J_k| (equation framecond1 asks only M_k >= |J_k|; Algorithm
                               3's layers need M_k even): fewer coefficients (c2: 76,476 instead of
                               94,416 per slice), hops 2N / M_k of a fraction of a sample where M_k
                               does not divide 2N, band transforms with radix-3 and radix-5 steps,
                               and never one workgroup per slice */
  int32_t fused;            /* 0 (default): the multi-kernel pipeline; 1: where a slice's half
                               spectrum and its largest band transform fit one workgroup's LDS,
                               each slice's analysis (and synthesis) runs in one workgroup with no
                               intermediate in HBM (the same results to rounding; about 1.1x the
                               algorithmic HBM bytes instead of about 2.6x, but bound by LDS
                               latency and barriers at one workgroup per CU, and slower on
                               MI355X for 2N = 16384 and 32768) */
} slicq_plan_opts;

enum { SLICQ_BAND_MAJOR = 0, SLICQ_SLICE_MAJOR = 1 };

typedef struct {
  int32_t K;                /* constant-Q bands 1..K */
  int32_t nbands;           /* stored bands K + 2 */
  int64_t slice_len;        /* 2N */
  int64_t transition_len;   /* M */
  int64_t coefs_per_slice;  /* sum_k M_k over stored bands */
  double Q;                 /* Q = (2^{1/B} - 2^{-1/B})^{-1} */
  int32_t max_M;            /* largest M_k */
  int32_t n_ana_items;      /* analysis work items per slice */
  int32_t n_syn_items;      /* synthesis work items per slice */
  int32_t coef_layout;      /* SLICQ_BAND_MAJOR or SLICQ_SLICE_MAJOR */
  int32_t fused;            /* bit d set: dtype d (SLICQ_F32 = 0, SLICQ_F64 = 1) runs one workgroup per slice */
  int64_t coefs_per_slice_all;  /* sum_k M_k over all 2K+2 bands (complex-signal calls) */
} slicq_plan_info;

/* Design a plan from the paper's parameters (Section 3, Table 1; Section
 * 4.3), with min_win = 16 and the canonical dual slicing window. Host only.
 * Returns SLICQ_EINVAL for parameters outside the ranges in slicq_plan_opts
 * or a frame that fails Proposition 2's condition. *out receives the plan,
 * owned by the caller (nsgt_plan_destroy). */
int nsgt_plan(double fs, double fmin, double fmax, int bins_per_octave, int64_t slice_len_2N,
              int64_t transition_len, slicq_plan* out);

/* As nsgt_plan with every option explicit; zero tuning fields take defaults.
 * nsgt_plan uses the band-major layout. */
int nsgt_plan_ex(const slicq_plan_opts* opts, slicq_plan* out);

/* Frees the plan's host memory. The caller still owns the device tables. */
void nsgt_plan_destroy(slicq_plan plan);

int nsgt_plan_info(slicq_plan plan, slicq_plan_info* info);

/* Per stored band k (arrays of nbands entries, any may be NULL): M_k, packing
 * offset off_k, signed first bin of J_k, |J_k|, centre and bandwidth in Hz
 * (Table 1). */
int nsgt_plan_bands(slicq_plan plan, int32_t* M, int64_t* off, int64_t* start, int32_t* len,
                    double* fc_hz, double* bw_hz);

/* The plan's FP64 tables (any may be NULL): g_k and g~_k over each J_k
 * concatenated in band order (sum_k |J_k| values each), h_0 and h~_0 over
 * j = t + N, t in [-N, N) (2N values each), frame-operator diagonal D (2N). */
int nsgt_plan_windows(slicq_plan plan, double* g, double* gd, double* h0, double* hd, double* D);

/* Bytes of device tables for dtype. */
int nsgt_plan_table_bytes(slicq_plan plan, slicq_dtype dtype, size_t* bytes);

/* Copies the tables for dtype into caller-owned device memory `dev_tables`
 * (at least nsgt_plan_table_bytes bytes, 256-byte aligned) on hip_stream and
 * records the address in the plan. The memory must stay valid while the plan
 * is used with this dtype. */
int nsgt_plan_upload(slicq_plan plan, slicq_dtype dtype, void* dev_tables, size_t bytes, void* hip_stream);

/* S = 2 ceil(T / 2N): slices of a signal of T samples (Algorithm 3, L = 2N ceil(T/2N)). */
int64_t slicq_num_slices(slicq_plan plan, int64_t T);

/* Workspace bytes to process n_slices slices in one pass. Any workspace of at
 * least the size for one slice (plus the task table of all slices) is
 * accepted; smaller ones are processed in several passes. */
int slicq_workspace_size(slicq_plan plan, slicq_dtype dtype, int64_t n_slices, size_t* bytes);

/* Analysis (Algorithm 3 with Algorithm 1 per slice) of x: T real samples of
 * dtype. coef: coef_count complex values of dtype, band-major (see above),
 * needs coef_count >= S * coefs_per_slice (else SLICQ_ESIZE). The signal is
 * zero padded to L = 2N ceil(T/2N) and sliced circularly. */
int slicq_analyze(slicq_plan plan, slicq_dtype dtype, const void* x, int64_t T, void* coef,
                  int64_t coef_count, void* work, size_t work_bytes, void* hip_stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The same
 * analysis as slicq_analyze (bitwise the same coefficients), with the
 * workspace taken from a fixed device array inside the library instead of a
 * caller buffer: slicq_static_scratch_bytes() bytes (32 MiB) per device,
 * held until the process ends. x and coef are the caller's device buffers as
 * for slicq_analyze. The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine (its first call on a device looks up the
 * array's address once). Signals whose S = slicq_num_slices(T) slices need a
 * task table plus one slice's workspace beyond the array fail with
 * SLICQ_ESIZE; otherwise the slices run in as many chunks as the array
 * holds. Every call on one device shares that device's array: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller. Nothing in the array needs clearing between
 * calls (each call writes what it reads). */
size_t slicq_static_scratch_bytes(void);
int slicq_analyze_static(slicq_plan plan, slicq_dtype dtype, const void* x, int64_t T, void* coef,
                         int64_t coef_count, void* hip_stream);

/* Synthesis (Algorithm 4 with Algorithm 2 per slice, canonical duals) from
 * coef (S = slicq_num_slices(T) slices, band-major) into y: T real samples.
 * For real signals the mirrored bands take conjugate coefficients and y is
 * the real part of the full synthesis. Overwrites all of y. */
int slicq_synthesize(slicq_plan plan, slicq_dtype dtype, const void* coef, int64_t coef_count, void* y,
                     int64_t T, void* work, size_t work_bytes, void* hip_stream);

/* Adjoint of the real-input analysis: y = Re(A^H coef), the transpose of
 * slicq_analyze for the real inner product. Same arguments as synthesis. */
int slicq_adjoint(slicq_plan plan, slicq_dtype dtype, const void* coef, int64_t coef_count, void* y,
                  int64_t T, void* work, size_t work_bytes, void* hip_stream);

/* Adjoint of synthesis (the gradient of a loss of the synthesised signal with
 * respect to the coefficients, for the real inner products): with w_k = 2 on
 * bands 1..K (each also synthesises through its conjugate mirror) and 1 on the
 * DC and Nyquist bands, coef = w_k <y, gamma_k> for the dual atoms gamma_k of
 * Algorithm 4 (dual windows g~_k = g_k / D of Proposition 2, dual slicing
 * window h~_0 of equation dualwincond): the analysis of y (T real samples)
 * with h~_0 in place of h_0 and w_k g~_k in place of g_k. Arguments as for
 * slicq_analyze. */
int slicq_synthesize_adjoint(slicq_plan plan, slicq_dtype dtype, const void* y, int64_t T, void* coef,
                             int64_t coef_count, void* work, size_t work_bytes, void* hip_stream);

/* Log-magnitude loss of coefficients against target log-magnitudes t (the
 * differentiable workload's loss, not part of the paper's transform): with
 * d = log(1 + |c|^2) - t over n complex coefficients, *loss = sum d^2 and
 * grad = 4 d c / (1 + |c|^2) (the derivative with respect to the real and
 * imaginary parts), in one pass over c and t. partial: device scratch of at
 * least slicq_logmag_loss_partials(n) values of the dtype; loss: one value of
 * the dtype in device memory. Blocks sum fixed strides and the partials are
 * added in order: the result is the same on every run. */
int64_t slicq_logmag_loss_partials(int64_t n);
int slicq_logmag_loss(slicq_dtype dtype, const void* coef, const void* target, int64_t n, void* grad, void* partial,
                      int64_t partial_count, void* loss, void* hip_stream);

/* Complex signals (the transform of Sections 2-4 before the restriction to
 * real signals): analysis onto all 2K+2 bands, band-major in the order
 * 0..K+1 (the stored bands, same offsets as for real signals) then the
 * mirrored bands K+2..2K+1 (band 2K+2-k has M_k coefficients per slice),
 * slicq_plan_info.coefs_per_slice_all per slice. x and y are T complex values
 * of the dtype, interleaved. The transform is complex linear: analysis runs
 * the real analysis on the real and imaginary parts and combines them
 * (mirror bands take conj c_k(Re x) + i conj c_k(Im x)); synthesis splits the
 * coefficients into the two Hermitian-symmetric sets whose real syntheses are
 * the real and imaginary parts of y. The workspace (at least
 * slicq_complex_workspace_size bytes) holds the real workspace, the two parts
 * and two coefficient sets. Band-major plans only (SLICQ_EINVAL otherwise). */
int slicq_complex_workspace_size(slicq_plan plan, slicq_dtype dtype, int64_t T, size_t* bytes);
int slicq_analyze_complex(slicq_plan plan, slicq_dtype dtype, const void* x, int64_t T, void* coef,
                          int64_t coef_count, void* work, size_t work_bytes, void* hip_stream);
int slicq_synthesize_complex(slicq_plan plan, slicq_dtype dtype, const void* coef, int64_t coef_count, void* y,
                             int64_t T, void* work, size_t work_bytes, void* hip_stream);

/* Coefficient domain (Algorithm 3's 2-layer array; Sections 4.3 and 6), for
 * the coefficients of one signal of S (even) slices in the plan's layout.
 * Slice m's coefficients of band k belong to layer m mod 2 at positions
 * (m - 1) M_k / 2 + n, n < M_k, circular modulo S M_k / 2. Layer-grid arrays
 * are band-major: band k's S M_k / 2 values start at (S / 2) off_k.
 * slicq_layers writes s^0 + s^1 (mode 0, complex) or the sliCQ spectrogram
 * |s^0 + s^1|^2 (mode 1, real) into out ((S / 2) coefs_per_slice values).
 * slicq_mask_db scales every coefficient in place by 10^{5 (v - 1)}, v in
 * [0, 1] the mask value of its layer position (mask on the layer grid: 0 is
 * -100 dB, 1 is 0 dB; one value serves both layers). slicq_transpose writes
 * out band t = in band t - d for constant-Q bands 1..K (d bands up: 8 bands
 * are 2 semitones at 48 bands per octave), zero for vacated bands and for the
 * DC and Nyquist bands; every moved band must have the M_k of its target
 * (SLICQ_EINVAL otherwise: use m_policy 1 or a shift inside a run of equal
 * M_k). in and out must not alias. */
int slicq_layers(slicq_plan plan, slicq_dtype dtype, const void* coef, int64_t S, int mode, void* out,
                 int64_t out_count, void* hip_stream);
int slicq_mask_db(slicq_plan plan, slicq_dtype dtype, void* coef, int64_t S, const void* mask, int64_t mask_count,
                  void* hip_stream);
int slicq_transpose(slicq_plan plan, slicq_dtype dtype, const void* in, void* out, int64_t S, int32_t d,
                    void* hip_stream);

/* Ragged batches. Signal b holds samples x_off[b] .. x_off[b+1]-1 of the
 * packed x (x_off: nsig + 1 int64 in device memory, x_len = packed length)
 * and its coefficients start at coef_off[b] (nsig int64, device memory) with
 * the single-signal layout. total_slices must equal sum_b S_b. The offsets
 * live in device memory, so these calls cannot check them on the host and
 * never synchronise: a signal whose samples or coefficients fall outside
 * x_len / coef_len (or beyond total_slices) is skipped and the task builder
 * flags it in the workspace; slicq_batched_status reads that flag back.
 * Every slice of every signal is processed by the same launches (one per
 * kernel). Per-signal results are identical to the single-signal calls. */
int slicq_analyze_batched(slicq_plan plan, slicq_dtype dtype, const void* x, int64_t x_len,
                          const int64_t* x_off, int32_t nsig, int64_t total_slices, void* coef,
                          int64_t coef_len, const int64_t* coef_off, void* work, size_t work_bytes,
                          void* hip_stream);
int slicq_synthesize_batched(slicq_plan plan, slicq_dtype dtype, const void* coef, int64_t coef_len,
                             const int64_t* coef_off, void* y, int64_t y_len, const int64_t* y_off,
                             int32_t nsig, int64_t total_slices, void* work, size_t work_bytes,
                             void* hip_stream);
int slicq_adjoint_batched(slicq_plan plan, slicq_dtype dtype, const void* coef, int64_t coef_len,
                          const int64_t* coef_off, void* y, int64_t y_len, const int64_t* y_off,
                          int32_t nsig, int64_t total_slices, void* work, size_t work_bytes,
                          void* hip_stream);
/* Validity of the last batched call that used `work` (same plan, dtype and
 * total_slices): waits for hip_stream, then *bad = 1 if that call skipped a
 * signal whose ranges fell outside its buffers (and returns SLICQ_ESIZE),
 * else *bad = 0 and SLICQ_OK; *slices (may be NULL) receives the slice count
 * the task builder found. Synchronises the stream: call it when the caller
 * chooses, never inside graph capture. */
int slicq_batched_status(slicq_plan plan, slicq_dtype dtype, int64_t total_slices, const void* work,
                         size_t work_bytes, int32_t* bad, int64_t* slices, void* hip_stream);

/* Prepared batches: the slice task table of a ragged batch built once and
 * reused by any number of transforms of batches with the same offsets (the
 * batched calls above rebuild it on every call). slicq_batch_tasks_bytes
 * gives the size of the caller-owned device buffer `tasks`.
 * slicq_batch_create builds the table on hip_stream (offsets as for the
 * batched calls; x_len and coef_len bound the signal and coefficient ranges
 * the tasks may address), waits for it once and checks it: a signal whose
 * samples or coefficients fall outside those bounds, or a slice count other
 * than total_slices, fails the call with SLICQ_ESIZE (no handle). On success
 * it returns a host handle that keeps the plan, the tasks pointer and these
 * bounds; the offsets may be freed. slicq_*_batch then run the transform with the prepared tasks: buffers
 * must be at least x_len / coef_len long (SLICQ_ESIZE otherwise) and the
 * tasks buffer must stay alive and unmodified. A workspace smaller than
 * slicq_workspace_size(total_slices) is processed in chunks. The handle is
 * immutable after creation; destroy it with slicq_batch_destroy (host memory
 * only). Per-signal results are identical to the other calls. */
typedef struct slicq_batch_s* slicq_batch;
size_t slicq_batch_tasks_bytes(int64_t total_slices);
int slicq_batch_create(slicq_plan plan, const int64_t* x_off, const int64_t* coef_off, int32_t nsig,
                       int64_t total_slices, int64_t x_len, int64_t coef_len, void* tasks, size_t tasks_bytes,
                       void* hip_stream, slicq_batch* out);
void slicq_batch_destroy(slicq_batch batch);
int slicq_analyze_batch(slicq_batch batch, slicq_dtype dtype, const void* x, int64_t x_len, void* coef,
                        int64_t coef_len, void* work, size_t work_bytes, void* hip_stream);
int slicq_synthesize_batch(slicq_batch batch, slicq_dtype dtype, const void* coef, int64_t coef_len, void* y,
                           int64_t y_len, void* work, size_t work_bytes, void* hip_stream);
int slicq_adjoint_batch(slicq_batch batch, slicq_dtype dtype, const void* coef, int64_t coef_len, void* y,
                        int64_t y_len, void* work, size_t work_bytes, void* hip_stream);

/* ---- Streaming service (real-time streams, continuously batched) ----------
 * Each stream is the linear sliCQ of an unbounded signal that is zero before
 * sample 0: slice m is centred on sample mN (Algorithm 3) and becomes ready
 * once mN + (N+M)/2 samples have been pushed; its output samples are final
 * once slice m is done for t <= mN + (N-M)/2 (Algorithm 4 overlap-add), and
 * equal the input samples (Proposition 3). Each tick processes every ready
 * slice of every open stream in one launch sequence on the server's own HIP
 * stream and synchronises with it; pushes, polls, opens and closes from other
 * threads proceed meanwhile and join the next tick. Per-stream state (input
 * and output rings of 4N samples) lives in device memory allocated once at
 * creation; admission is limited by max_streams and hbm_budget_bytes
 * (0 = no budget): every device buffer the server allocates, fixed
 * (workspace and coefficients for max_batch slices) or per stream (two rings
 * and the staging share), is counted against the budget. Each tick serves
 * the ready slices of the streams round robin, starting after the last
 * stream the previous tick reached when max_batch cut it short, so no stream
 * waits more than a bounded number of ticks under overload. Samples passed to push/poll are host memory of the
 * server's dtype. A device error fences the server (SLICQ_EHIP on every later
 * call). */
typedef struct slicq_stream_server_s* slicq_stream_server;

typedef struct {
  int64_t ticks, slices, samples_in, samples_out;
  int64_t admitted, rejected, closed, gap_samples;
  double latency_p50_s, latency_p99_s, latency_max_s;  /* ready-hop arrival to tick completion */
  int64_t latency_count;
  double busy_s;             /* host time spent inside ticks */
  int32_t slots;             /* streams the budget admits */
  int32_t pad_;
  int64_t ring_len;          /* samples per ring (4N) */
  int64_t bytes_per_stream;  /* device bytes per admitted stream (two rings, staging, copy records) */
  int64_t fixed_bytes;       /* device bytes independent of the stream count (workspace, coefficients) */
} slicq_stream_stats;

int slicq_stream_server_create(slicq_plan plan, slicq_dtype dtype, int32_t max_streams, int32_t max_batch,
                               size_t hbm_budget_bytes, slicq_stream_server* out);
void slicq_stream_server_destroy(slicq_stream_server server);
/* Admits a stream: *id >= 0, or SLICQ_EBUSY when no slot fits the budget. */
int slicq_stream_open(slicq_stream_server server, int32_t* id);
/* Appends n samples; push_gap appends n zeros for a hop that never arrived. */
int slicq_stream_push(slicq_stream_server server, int32_t id, const void* samples, int64_t n);
int slicq_stream_push_gap(slicq_stream_server server, int32_t id, int64_t n);
/* A whole round of hops in one call: stream ids[i] receives counts[i]
 * samples, taken in order from the packed `samples`. Every id and count is
 * checked before any sample is appended. */
int slicq_stream_push_many(slicq_stream_server server, int32_t n_ids, const int32_t* ids, const void* samples,
                           const int64_t* counts);
/* One batch over all streams; *n_slices receives the slices processed. */
int slicq_stream_tick(slicq_stream_server server, int64_t* n_slices);
/* Moves up to max final output samples of stream id into out; *n receives the count. */
int slicq_stream_poll(slicq_stream_server server, int32_t id, void* out, int64_t max, int64_t* n);
/* The final output of streams ids[i], packed in order into out (host memory
 * of cap samples); counts[i] receives each stream's count. Streams past the
 * capacity get what still fits (possibly 0) and keep the rest. */
int slicq_stream_poll_many(slicq_stream_server server, int32_t n_ids, const int32_t* ids, void* out, int64_t cap,
                           int64_t* counts);
/* Ends a stream (also mid-slice); its slot is cleared before reuse. */
int slicq_stream_close(slicq_stream_server server, int32_t id);
/* Coefficients of stream id's most recent slice (slice-major c^m: band k at
 * off_k, coefs_per_slice complex values of the dtype, host memory of at least
 * cap values), when the last tick processed it; *m receives the slice index,
 * or -1 if the last tick did not process this stream. */
int slicq_stream_coefs(slicq_stream_server server, int32_t id, void* out, int64_t cap, int64_t* m);
int slicq_stream_stats_get(slicq_stream_server server, slicq_stream_stats* stats);
int slicq_stream_stats_reset(slicq_stream_server server);
/* Per-stream checkpoint: counters, queued samples and both rings. With
 * buf == NULL only *bytes is set. restore() loads a snapshot of the same plan
 * and dtype into an open stream; outputs then continue bit for bit. */
int slicq_stream_snapshot(slicq_stream_server server, int32_t id, void* buf, size_t cap, size_t* bytes);
int slicq_stream_restore(slicq_stream_server server, int32_t id, const void* buf, size_t bytes);

/* Measurement hook: enqueues one kernel of the pipeline of the preceding
 * transform call made with the same plan, dtype, buffers and workspace (which
 * must hold all n_slices slices at once), so that a profiler can time it
 * alone. Stages: 0 slice FFT pass 1, 1 slice FFT pass 2 and real split,
 * 2 band analysis, 3 band synthesis, 4 inverse FFT pass A, 5 inverse FFT pass B
 * with overlap-add (and the fix-up kernel that adds the second contribution
 * of every output sample two slices share). The stage reads what the
 * preceding call left in the workspace; outputs are overwritten (stage 5
 * rewrites y in full, so it may be repeated; it overwrites the workspace
 * region that stage 4 reads). For a dtype that runs one workgroup per slice
 * (slicq_plan_info.fused), stage 0 is the whole analysis, stage 3 the whole
 * synthesis before the overlap fix-up, stage 5 the fix-up, and stages 1, 2
 * and 4 enqueue nothing. */
int slicq_profile_stage(slicq_plan plan, slicq_dtype dtype, int stage, int64_t n_slices, const void* x,
                        void* coef, void* y, void* work, size_t work_bytes, void* hip_stream);
/* The same for a prepared batch: re-launches one stage over all of its
 * slices, reading what the preceding slicq_*_batch call left in `work`
 * (buffers at least as long as the batch was prepared for). */
int slicq_profile_stage_batch(slicq_batch batch, slicq_dtype dtype, int stage, const void* x, int64_t x_len,
                              void* coef, int64_t coef_len, void* y, int64_t y_len, void* work, size_t work_bytes,
                              void* hip_stream);

/* ---------------------------------------------------------------------------
 * Full-length CQ-NSGT: Algorithms 1 and 2 run at the signal length L instead
 * of the slice length (Section 3), on a complex signal, onto all 2K+2 bands.
 * The band windows are the sliCQ plan's (same centres, bandwidths after the
 * minimal filter length, plateaus, window shape) sampled on the L-point grid,
 * so that g_k[j] = g^L_k[j L / 2N] (the relation of Proposition 4). Bands
 * 0..K+1 come first, then the mirrors K+2..2K+1 of bands K..1.
 *
 * lattice 0: M^L_k = M_k L / 2N coefficients per band, the sliCQ's
 *   time-frequency lattice (what Proposition 4 and the approximation study of
 *   Section 5.3 compare s^0 + s^1 with, after rescaling by sqrt(2N / L) with
 *   unitary DFTs). A band may alias (|J^L_k| > M^L_k): analysis is still the
 *   inner products of equation CQ_coeff, but synthesis is refused.
 * lattice 1: M^L_k the smallest power of two >= |J^L_k| (>= 2; one M for all
 *   bands on a rectangular plan): the painless case of Proposition 2, whose
 *   canonical dual g^L_k / D^L, D^L = sum_k M^L_k |g^L_k|^2, gives perfect
 *   reconstruction.
 *
 * L must be a power of two, at least 2N and at most 2^24; every M^L_k at most
 * 2^24. Coefficients are complex interleaved (f32 or f64), band k at
 * off_k .. off_k + M^L_k - 1 (nsgt_full_bands):
 *   c_{n,k} = sum_j (F_L f)[j] g^L_k[j] e^{2 pi i j n / M^L_k}
 * with the unitary DFT F_L. Signals are L complex values, interleaved.
 * Tables are uploaded once per dtype into caller-owned device memory
 * (256-byte aligned, kept alive while the plan is used), as for the sliCQ
 * plan. The transforms enqueue on hip_stream, never synchronise and never
 * allocate; the workspace (nsgt_full_workspace_size) is caller-owned and
 * may be reused once the call's work is complete. */
typedef struct slicq_full_s* slicq_full;

typedef struct {
  int64_t L;              /* signal length */
  int32_t nbands;         /* 2K + 2 */
  int32_t lattice;        /* 0 sliCQ hops, 1 painless */
  int32_t painless;       /* 1 when every band has M^L_k >= |J^L_k| (synthesis allowed) */
  int32_t pad_;
  int64_t coef_count;     /* sum_k M^L_k */
  int64_t max_M;          /* largest M^L_k */
  int64_t entries;        /* sum_k |J^L_k| (synthesis overlap-add entries) */
} slicq_full_info;

/* Builds the full-length plan of `plan` at length L (host only; FP64).
 * SLICQ_EINVAL for L or lattice out of range, a band with no bin on the
 * L-point grid, a zero of D^L, or coefficient counts reaching 2^31. */
int nsgt_full_plan(slicq_plan plan, int64_t L, int32_t lattice, slicq_full* out);
void nsgt_full_destroy(slicq_full full);
int nsgt_full_info(slicq_full full, slicq_full_info* info);
/* Per band (arrays of nbands, any may be NULL): first signed bin of J^L_k,
 * |J^L_k|, M^L_k and the coefficient offset. */
int nsgt_full_bands(slicq_full full, int64_t* start, int32_t* len, int32_t* M, int64_t* off);
/* g^L_k and the canonical dual g^L_k / D^L over each J^L_k, concatenated in
 * band order (entries doubles each; either may be NULL). */
int nsgt_full_windows(slicq_full full, double* g, double* gd);
int nsgt_full_table_bytes(slicq_full full, slicq_dtype dtype, size_t* bytes);
int nsgt_full_upload(slicq_full full, slicq_dtype dtype, void* dev_tables, size_t bytes, void* hip_stream);
/* Bytes of workspace for either transform: complex values for the band
 * spectra (coef_count), one length-L spectrum and the scratch of the
 * four-step FFTs (max(L, coef_count)). */
int nsgt_full_workspace_size(slicq_full full, slicq_dtype dtype, size_t* bytes);
/* Analysis (Algorithm 1 at length L): unitary DFT of x (L complex values),
 * X g^L_k wrapped modulo M^L_k, inverse DFTs of length M^L_k (unnormalised)
 * into coef (coef_count >= info.coef_count complex values, else
 * SLICQ_ESIZE). */
int nsgt_full_analyze(slicq_full full, slicq_dtype dtype, const void* x, void* coef, int64_t coef_count, void* work,
                      size_t work_bytes, void* hip_stream);
/* Synthesis (Algorithm 2 at length L): DFTs of length M^L_k, overlap-add of
 * g^L_k / D^L times each band's spectrum at j mod M^L_k, unitary inverse DFT
 * into y (L complex values). The inverse of nsgt_full_analyze; SLICQ_EINVAL
 * on a plan whose lattice aliases a band (info.painless == 0). */
int nsgt_full_synthesize(slicq_full full, slicq_dtype dtype, const void* coef, int64_t coef_count, void* y,
                         void* work, size_t work_bytes, void* hip_stream);

/* Message of the last failing call on this thread ("" if none). */
const char* slicq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SLICQ_H */
