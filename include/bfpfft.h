/*
 * bfpfft.h -- C ABI of the block-floating-point half-precision FFT and the
 * range-Doppler SAR chain built on it, for AMD Instinct MI355X (gfx950).
 *
 * Method (arXiv 2605.28451, "Range, Not Precision"):
 *   * matched-filter compression y = (1/N) IFFT(FFT(x) . H) with the inverse
 *     realised as conj-FFT-conj (Sec. III-B);
 *   * fixed-shift block floating point: the exact factor 1/N = 2^-log2(N) is
 *     folded into the conjugate that precedes every inverse transform
 *     (Eq. (1), Sec. IV-A), so every intermediate stays within O(N) and the
 *     result equals the conventionally scaled inverse;
 *   * the cascade of Sec. IV-B: range compression emits O(1) data, so the
 *     azimuth FFT emits O(N) spectra and its own BFP inverse stays in range.
 *
 * Conventions shared by every entry point
 *   - Data pointers are HIP device pointers owned by the caller.  Host
 *     pointers are marked "(host)".  Streams are hipStream_t passed as void*
 *     (NULL = the legacy default stream).
 *   - Complex data is interleaved (re, im); rows are contiguous, row-major.
 *     The element type follows the precision mode (bfp_storage_bytes).
 *   - Execution calls are asynchronous on the given stream: they validate
 *     their arguments, enqueue kernels and return.  Device faults surface at
 *     the next synchronisation.  in == out is allowed for fft_exec_* (each
 *     row is read completely before any of it is written).
 *   - Every function returns BFP_OK (0) or a negative bfp_status; none
 *     throws across the ABI.  bfp_last_error() returns a message for the
 *     last failure on the calling thread.
 *   - Plans are immutable after creation and may be used concurrently from
 *     several streams; a plan's non-finite counter is shared by all of them.
 *     Exception: a plan's phasor table, its entropy and autofocus
 *     workspaces and an uneven plan's work-queue counter are written by
 *     the calls that use them (an azimuth compression given a phase
 *     vector, sar_image_entropy, sar_azimuth_image_entropy,
 *     sar_azimuth_phase_grad, fft_exec_uneven); such calls must not overlap
 *     on one plan (give each stream its own plan for them).
 */
#ifndef BFPFFT_H
#define BFPFFT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfp_plan_s *bfp_plan;

/* ------------------------------------------------------------ status --- */
enum bfp_status {
  BFP_OK = 0,
  BFP_EINVAL = -1,        /* bad argument (size, pointer, mode, flag) */
  BFP_EUNSUPPORTED = -2,  /* valid request this build does not implement */
  BFP_ENOMEM = -3,        /* device or host allocation failed */
  BFP_EHIP = -4,          /* a HIP runtime call failed (see bfp_last_error) */
  BFP_ENODEV = -5         /* no gfx950 device visible */
};

/* ------------------------------------------------------ precision --- */
/* Precision modes (paper Sec. VI lists four; FP8 storage is Sec. VII).
 * "storage" = HBM element type; on-chip (LDS) intermediates between radix
 * passes are stored as noted; arithmetic as noted.                         */
enum bfp_precision {
  BFP_FP32 = 0,                    /* FP32 storage, LDS, twiddles, arithmetic  */
  BFP_FP16 = 1,                    /* pure FP16: packed half2 arithmetic, FP16
                                      twiddles, FP16 LDS and storage           */
  BFP_FP16_STORE_FP32_COMPUTE = 2, /* FP16 storage and LDS, FP32 twiddles and
                                      arithmetic                              */
  BFP_FP16_MUL_FP32_ACC = 3,       /* FP16 storage, LDS and twiddles; every
                                      twiddle/filter product takes FP16
                                      operands and accumulates in FP32         */
  BFP_FP8_E4M3_STORE = 4,          /* OCP FP8 E4M3 storage (saturating RNE),
                                      FP32 LDS, twiddles and arithmetic        */
  BFP_FP8_E5M2_STORE = 5           /* OCP FP8 E5M2 storage, otherwise as above */
};

/* Storage formats for bfp_convert and for tables. */
enum bfp_format {
  BFP_FMT_F32 = 0,   /* 8 bytes per complex  */
  BFP_FMT_F16 = 1,   /* 4 bytes per complex  */
  BFP_FMT_E4M3 = 2,  /* 2 bytes per complex  */
  BFP_FMT_E5M2 = 3   /* 2 bytes per complex  */
};

/* ----------------------------------------------------------- flags --- */
enum bfp_flags {
  /* Debug: conventional output scaling instead of the BFP fold.  The
   * unscaled inverse is rounded to the storage format first and multiplied
   * by 2^-log2(N) afterwards, which overflows FP16 storage (Sec. III-B). */
  BFP_FLAG_NAIVE_POSTSCALE = 1u,
  /* Count non-finite output values into the plan's counter
   * (read with fft_plan_nonfinite). */
  BFP_FLAG_CHECK_FINITE = 2u,
  /* sar_range_compress only: store the result corner-turned, rc_t[range]
   * [pulse] (n x n_pulses), as sar_corner_turn would leave it (the corner
   * turn fused into the compression's store). */
  BFP_FLAG_TRANSPOSED_STORE = 4u,
  /* Output stored as interleaved FP32 whatever the precision mode. */
  BFP_FLAG_OUT_FP32 = 8u,
  /* Use conj(filter): the adjoint of the compression chain. */
  BFP_FLAG_CONJ_FILTER = 16u,
  /* Plan flag: allocate the autofocus workspace (FP32 twiddles and the
   * phase-gradient partial sums: 1024 workgroups x n floats per transform
   * a workgroup holds, 16 MiB at n = 4096, 64 MiB at n = 16384). */
  BFP_FLAG_AUTOFOCUS = 32u
};

/* Bytes per complex element in HBM for a precision mode (-1 if invalid). */
int bfp_storage_bytes(int prec);
/* Storage format of filters for a precision mode: BFP_FMT_F16 for the FP16
 * modes, BFP_FMT_F32 for FP32 and the FP8-storage modes. */
int bfp_filter_format(int prec);
/* Bytes per complex element of a storage format (-1 if invalid). */
int bfp_format_bytes(int fmt);

const char *bfp_status_string(int status);
const char *bfp_last_error(void);

/* Number of visible gfx950 devices (0 when none).  Never fails. */
int bfp_device_count(void);

/* ------------------------------------------------------------ plans --- */
/* Plan for `batch` independent transforms of length n = 2^k, 2^3..2^14, in
 * precision mode `prec` (below 256 points a workgroup holds 256 * E / n
 * transforms, E = 8 or 16 points per thread; n = 8 and 16 take one thread
 * each).  flags: BFP_FLAG_CHECK_FINITE, BFP_FLAG_OUT_FP32,
 * BFP_FLAG_CONJ_FILTER (every filtered call uses conj(filter); an azimuth
 * compression's `adjoint` then reverts to the filter itself),
 * BFP_FLAG_NAIVE_POSTSCALE, BFP_FLAG_AUTOFOCUS (n >= 256).
 * The plan owns its device twiddle tables (built on the host in FP64 with
 * exact argument reduction and rounded once, never by recurrence: Sec.
 * III-A) and its non-finite counter; it is bound to the device current at
 * creation.  Errors: BFP_EINVAL (n not a supported power of two, batch < 0,
 * bad mode), BFP_ENODEV, BFP_ENOMEM, BFP_EHIP. */
int fft_plan(bfp_plan *out, int n, int batch, int prec, unsigned flags);
int fft_destroy(bfp_plan p);
/* Query: any output pointer may be NULL. */
int fft_plan_info(bfp_plan p, int *n, int *batch, int *prec, unsigned *flags);

/* X = DFT_N(x) per row, unscaled (exponent 0): X[k] = sum x[n] e^{-2 pi i nk/N}
 * (Sec. III-B).  in/out: batch x n elements of the plan's storage type
 * (BFP_FLAG_OUT_FP32: out is FP32 pairs). */
int fft_exec_fwd(bfp_plan p, const void *in, void *out, void *stream);

/* BFP inverse, Eq. (1): y = conj(DFT_N(conj(in . filter) . 2^-log2N)), i.e.
 * the normalised IDFT of in . filter.  filter: n elements in
 * bfp_filter_format(prec), shared by every row, or NULL for none.  The
 * 2^-log2N multiply is exact for normal results and rounds to nearest-even
 * into subnormals.  BFP_FLAG_NAIVE_POSTSCALE in the plan flags or in
 * `flags` selects the conventional scaling instead. */
int fft_exec_inv_bfp(bfp_plan p, const void *in, void *out, const void *filter,
                     void *stream);
int fft_exec_inv_bfp_flags(bfp_plan p, const void *in, void *out, const void *filter,
                           unsigned flags, void *stream);

/* Tuning knobs of a plan.  engine: 0 = matrix cores where the mode and size
 * have them (BFP_FP16_MUL_FP32_ACC at n = 4096: forward, BFP inverse with
 * or without a filter, and the compressions with a filter, its conjugate, a
 * phase applied before the chain, FP32 output or the naive schedule; the
 * output-phase adjoint, the transposed store, the adaptive shift and the
 * migration correction always run on the vector ALU), 1 = vector ALU only
 * (the default of a new plan: the faster engine on MI355X at every measured
 * size; fft_autotune may still select 0).
 * blocks_per_cu: rows plans: -1 = automatic (the default of a new plan:
 * the fused compression of pure FP16 at n <= 4096 uses k = 3, or 8 from
 * 4096 rows of 4096 points; the FP32-output image of
 * sar_azimuth_image_entropy one round of its kernel's resident workgroups;
 * everything else 0), 0 = one workgroup per group of rows, k > 0 = a persistent grid of
 * k workgroups per CU looping over the rows (in pure FP16 at n <= 4096 this
 * grid overlaps the next rows' loads with the current rows' transforms); uneven plans:
 * workgroups per CU of the launch, 0 = the resident maximum (the default: a
 * persistent grid whose workgroups pull tiles from the work queue), k in
 * [1, 64] = k per CU; above the resident maximum the hardware queues the
 * extra workgroups, and a grid with one workgroup per tile or more takes
 * every tile by workgroup index, without the queue.  Results do not depend
 * on blocks_per_cu. */
int fft_plan_set_tuning(bfp_plan p, int engine, int blocks_per_cu);
int fft_plan_get_tuning(bfp_plan p, int *engine, int *blocks_per_cu);

/* All tuning knobs: engine and blocks_per_cu as above, radix_plan and
 * rows_per_thread.  radix_plan (0 or 1, sizes 32..16384; n <= 16 has one
 * plan): the factorisation of n into radix passes, 0 the default (radix-16
 * passes where they fit), 1 the second plan (radix-8 passes with 8 values
 * per thread from 32 to 4096 points except 512, which takes 16 16 2; 16 16
 * 8 4 at 8192; 4 16 16 16 at 16384).  The plan changes the order of the
 * arithmetic, hence the rounding (both stay within the same accuracy); it
 * applies to the variants rows_per_thread covers (below), with storage-type
 * output, and the others run plan 0.  rows_per_thread
 * (1 or 2): with 2, the forward transform, the BFP inverse (with a filter,
 * its conjugate or none) and the compression (with a filter, its conjugate,
 * or a phase applied before the chain) transform two rows per thread
 * together, sharing twiddles and one barrier per LDS exchange; the other
 * variants, the matrix-core engine and sizes whose two rows would not leave
 * LDS for two workgroups per CU (FP32 exchanges above 4096 points, FP16
 * above 8192) ignore it.  For one radix plan, results are the same bits for
 * every engine-independent setting (blocks_per_cu, rows_per_thread).
 * Uneven plans take rows_per_thread = 1 and radix_plan = 0.  A new plan has
 * {1, -1, 2, 0} in the modes with FP32 arithmetic (BFP_FP32,
 * BFP_FP16_STORE_FP32_COMPUTE and the FP8-storage modes) and {1, -1, 1, 0}
 * in BFP_FP16 and BFP_FP16_MUL_FP32_ACC; a plan made with
 * BFP_FLAG_AUTOFOCUS takes radix_plan 1 where its size has two plans (the
 * phase gradient, sar_azimuth_phase_grad, runs that plan where its
 * workgroups hold no more transforms than plan 0's, and plan 0 otherwise;
 * the FP32-output image of sar_azimuth_image_entropy always runs plan 0).
 * Errors: BFP_EINVAL. */
typedef struct {
  int engine;
  int blocks_per_cu;
  int rows_per_thread;
  int radix_plan;
} bfp_tuning;
int fft_plan_set_tuning_ex(bfp_plan p, const bfp_tuning *t);
int fft_plan_get_tuning_ex(bfp_plan p, bfp_tuning *t);

/* Times every tuning candidate of the plan (engine x blocks_per_cu x
 * rows_per_thread x radix_plan for rows plans, blocks_per_cu for uneven
 * plans) on the
 * caller's buffers (op: 0
 * forward, 1 BFP inverse with `filter` (may be NULL), 2 fused compression
 * with `filter`; ignored for uneven plans), `reps` calls each after two
 * warm-up calls, keeps the fastest in the plan and returns its mean time per
 * call in *best_ms (may be NULL).  `out` is overwritten; synchronises
 * `stream`. */
int fft_autotune(bfp_plan p, int op, const void *in, void *out, const void *filter, int reps,
                 float *best_ms, void *stream);
/* fft_autotune over n_sets buffer pairs, call k using (host arrays of device
 * pointers) ins[k % n_sets] and outs[k % n_sets]: with sets that together
 * exceed the last-level cache (256 MB on MI355X) every candidate is timed
 * streaming from HBM, as it will run.  n_sets in [1, 4096]. */
int fft_autotune_sets(bfp_plan p, int op, const void *const *ins, void *const *outs, int n_sets,
                      const void *filter, int reps, float *best_ms, void *stream);

/* Reads and clears the plan's non-finite counter; synchronises `stream`. */
int fft_plan_nonfinite(bfp_plan p, void *stream, unsigned long long *count);

/* -------------------------------------------------- uneven batches --- */
/* One persistent launch over `count` transforms of mixed length
 * (n_i = 2^log2n[i], 8 <= log2n[i] <= 14) and per-transform direction
 * (inverse[i] = 0: forward; 1: BFP inverse without filter), packed back to
 * back in the given order.  log2n and inverse are (host) arrays copied into
 * the plan.  Work is split into equal-size tiles of 16384 complex elements
 * (one transform of 16384, two of 8192, ..., 64 of 256) dispatched longest-
 * first from a device work queue. */
int fft_plan_uneven(bfp_plan *out, int count, const int *log2n,
                    const unsigned char *inverse, int prec, unsigned flags);
/* (host) offsets[count]: element offset of each transform in the packing. */
int fft_uneven_offsets(bfp_plan p, long long *offsets);
/* Total complex elements of the packed buffer. */
int fft_uneven_total(bfp_plan p, long long *total);
/* One launch over the packed batch (in, out: device, fft_uneven_total
 * complex elements in the plan's storage format).  With a grid smaller
 * than the tile count a one-thread kernel zeroes the plan's work-queue
 * counter first, so calls on one plan must not overlap. */
int fft_exec_uneven(bfp_plan p, const void *in, void *out, void *stream);

/* ------------------------------------------------------------ tables --- */
/* Matched filter for a replica (host) h[len] (interleaved FP64 pairs),
 * zero-padded to n: H = conj(DFT_n(h)) / max_k |DFT_n(h)|, so |H| <= 1
 * (Sec. III-B).  Computed on the host in FP64 and rounded once to `fmt`
 * into (host) out_host[n]. */
int bfp_make_filter(const double *h, int len, int n, int fmt, void *out_host);

/* Amplitude taper for weighted apertures: the paper's limitations paragraph
 * (Sec. VIII) names deeply weighted apertures (-40 dB sidelobes) as the case
 * where the FP16 noise floor comes near and the FP32-accumulate mode is the
 * remedy.  A weighted matched filter is bfp_make_filter of the replica
 * multiplied point by point by this taper over the replica's support.
 * Writes (host) out_host[len] in FP64, centred on the middle of the
 * aperture:
 *   BFP_WINDOW_RECT    1;
 *   BFP_WINDOW_HAMMING 0.54 - 0.46 cos(2 pi n / (len - 1));
 *   BFP_WINDOW_TAYLOR  Taylor taper with nbar terms whose nearest sidelobes
 *                      sit near -sll_db dB (0 < sll_db <= 300, nbar >= 1),
 *                      scaled to 1 at the aperture centre.
 * nbar and sll_db are ignored for the other kinds.  Errors: BFP_EINVAL. */
enum bfp_window_kind { BFP_WINDOW_RECT = 0, BFP_WINDOW_HAMMING = 1, BFP_WINDOW_TAYLOR = 2 };
int bfp_window(int kind, int len, int nbar, double sll_db, double *out_host);

/* Element-wise storage conversion of `count` complex values on the device,
 * rounding to nearest-even; FP8 targets saturate at their largest finite
 * value (E4M3: 448, E5M2: 57344).  in != out. */
int bfp_convert(const void *in, int in_fmt, void *out, int out_fmt, long long count,
                void *stream);

/* Adaptive block shift (the per-block exponents the paper leaves as future
 * work, Sec. VIII).  The fixed shift 2^-log2N of Eq. (1) keeps the inverse
 * in range for every input but pushes weak rows toward the FP16
 * subnormals.  These variants choose the shift per row: with z the
 * inverse's input (after the filter product) and M the largest |Re z| or
 * |Im z| of the row, k is the smallest integer in [-15, 14] with
 * sqrt(2) N M 2^-k < 2^15 (-15 for an all-zero row), which bounds every
 * partial sum of the inverse by 2^15 and scales weak rows up.  Each output row holds the normalised result times 2^(log2N - k);
 * (device) row_exp[r] = k - log2N, so the true row is out[r] * 2^row_exp[r].
 * FP16-storage modes only (BFP_FP16, BFP_FP16_STORE_FP32_COMPUTE,
 * BFP_FP16_MUL_FP32_ACC; else BFP_EUNSUPPORTED); flags: BFP_FLAG_CHECK_FINITE
 * only, and the plan may not carry NAIVE_POSTSCALE, CONJ_FILTER or OUT_FP32.
 * row_exp holds the plan's batch (inverse) or n_pulses (compression) ints.
 * Each row's maximum is a workgroup reduction (one LDS atomic per thread
 * and one barrier per row). */
int fft_exec_inv_bfp_adaptive(bfp_plan p, const void *in, void *out, const void *filter,
                              int *row_exp, unsigned flags, void *stream);
int sar_range_compress_adaptive(bfp_plan range_plan, const void *echo, void *rc,
                                const void *h_range, int n_pulses, int *row_exp, unsigned flags,
                                void *stream);

/* Range compression with range cell migration correction (the RCMC step of
 * the range-Doppler pipeline, Sec. VI), for data already in the Doppler
 * domain: row r of in (n_rows x n, one Doppler bin per row) becomes
 *   IDFT( DFT(in_r) . H . exp(+2 pi i k' s_r / n) ),  k' = k or k - n (k >= n/2),
 * with the BFP fold of Eq. (1): the row compressed by H and moved s_r bins
 * toward smaller range by band-limited (periodic sinc) interpolation.
 * (device) shift[n_rows]: s_r in range bins (FP32, any real value).  All
 * precision modes; flags: BFP_FLAG_CHECK_FINITE only; in != out.  The
 * linear phase is evaluated per element in FP32 (sincospif of the phase
 * reduced to [-1/2, 1/2] cycles) and multiplied into H before the filter
 * product. */
int sar_range_compress_rcmc(bfp_plan range_plan, const void *in, void *out, const void *h_range,
                            const float *shift, int n_rows, unsigned flags, void *stream);

/* Plain streaming copy of `bytes` (multiple of 16; 16-byte aligned
 * pointers), 16 bytes per lane: the reference for achievable HBM bandwidth
 * and for calibrating hardware memory counters against known traffic. */
int bfp_device_copy(const void *in, void *out, long long bytes, void *stream);

/* --------------------------------------------------------------- SAR --- */
/* Fused range compression (Fig. 1, left group): per pulse row,
 * rc = conj(DFT(conj(DFT(echo) . H_r) . 2^-log2N)), one HBM read and one
 * write per row.  range_plan: n = range samples, its mode sets the storage
 * type; n_pulses <= plan batch is the number of rows processed.  h_range:
 * n elements in bfp_filter_format(prec).  flags: BFP_FLAG_NAIVE_POSTSCALE,
 * BFP_FLAG_CONJ_FILTER, BFP_FLAG_OUT_FP32, BFP_FLAG_CHECK_FINITE,
 * BFP_FLAG_TRANSPOSED_STORE (rc is then n x n_pulses, range-major: the
 * layout sar_azimuth_compress reads, with no separate corner turn). */
int sar_range_compress(bfp_plan range_plan, const void *echo, void *rc, const void *h_range,
                       int n_pulses, unsigned flags, void *stream);

/* Corner turn: out[c][r] = in[r][c] for a rows x cols complex matrix in
 * storage format `fmt`, staged through LDS tiles.  in != out. */
int sar_corner_turn(const void *in, void *out, int rows, int cols, int fmt, void *stream);

/* Fused azimuth compression (Fig. 1, right group) of range-compressed data
 * laid out [range][pulse]: per range bin, the azimuth FFT, x H_a, the BFP
 * fold and the inverse.  phase: NULL, or (device) n_az FP32 radians; when
 * given, pulse m is first multiplied by exp(i phase[m]) (autofocus
 * correction).  adjoint != 0 applies the adjoint of that chain: with
 * A(x) = IDFT(DFT(x e^{i phase}) H_a), A^H(y) = e^{-i phase} IDFT(DFT(y)
 * conj(H_a)), i.e. the conjugated filter and exp(-i phase[m]) multiplied
 * into the output instead of the input.  The filter used is conj(H_a) when
 * exactly one of (BFP_FLAG_CONJ_FILTER in the call or the plan, adjoint)
 * holds.  flags: BFP_FLAG_CHECK_FINITE, BFP_FLAG_CONJ_FILTER,
 * BFP_FLAG_OUT_FP32 (with a phase only for the forward chain with H_a),
 * BFP_FLAG_NAIVE_POSTSCALE (without a phase and without the conjugated
 * filter); other combinations give BFP_EUNSUPPORTED before any launch.
 * az_plan: n = pulses; n_range <= plan batch rows are processed.  The image
 * is [range][azimuth]; the phase table is the plan's (calls with a phase
 * must not overlap on one plan). */
int sar_azimuth_compress(bfp_plan az_plan, const void *rc_t, void *image, const void *h_az,
                         const float *phase, int n_range, int adjoint, unsigned flags,
                         void *stream);

/* ---------------------------------------------------------- autofocus --- */
/* Entropy autofocus of the azimuth chain (gradient of the image entropy with
 * respect to a per-pulse phase vector).  Images and image gradients are
 * interleaved FP32 pairs.  stats is (device) 3 doubles: S = sum |I|^2,
 * Q = sum |I|^2 ln |I|^2, E = ln S - Q / S = -sum p ln p with p = |I|^2 / S
 * (0 ln 0 = 0).  The reductions run in a fixed order (deterministic). */
int sar_image_entropy(bfp_plan plan, const void *image, long long count, double *stats,
                      void *stream);

/* sar_image_entropy without a plan and without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid it): the same kernels and the same
 * fixed-order sums, so the result equals sar_image_entropy's bit for bit.
 * The per-workgroup partial sums live in a library-owned device array of
 * 1024 (S, Q) pairs (16 KiB, held on each GPU the library runs on until the
 * process ends); a launch uses min(ceil(count / 256), 1024) workgroups.
 * count in [1, 2^40] (else BFP_EINVAL); image: count FP32 pairs; stats:
 * (device) 3 doubles.  Calls that overlap on one GPU share the array and
 * race: serialise them (one stream, or events). */
int sar_image_entropy_noalloc(const void *image, long long count, double *stats, void *stream);

/* The image of sar_azimuth_compress (phase applied before the chain, output
 * FP32 pairs) and its entropy statistics in one pass: each workgroup of the
 * compression reduces |I|^2 and |I|^2 ln |I|^2 of the rows it wrote
 * (FP32 logarithms, FP64 sums), and the workgroup partials are added in a
 * fixed order into stats (device, 3 doubles as above).  The image is the
 * one sar_azimuth_compress writes; the statistics agree with
 * sar_image_entropy up to the order of the FP64 sums.  A phase vector
 * leaves exp(+i phase) in the plan's phasor table, which
 * sar_azimuth_phase_grad can reuse.  az_plan: precision BFP_FP32 or
 * BFP_FP16_STORE_FP32_COMPUTE; n_range <= plan batch; calls on one plan
 * must not overlap. */
int sar_azimuth_image_entropy(bfp_plan az_plan, const void *rc_t, void *image, const void *h_az,
                              const float *phase, int n_range, double *stats, void *stream);

/* grad = scale . dE/dI as a real pair (dE/dRe I + i dE/dIm I)
 *      = scale . (-2/S)(ln p + E) I;  scale: (device) one float or NULL (1). */
int sar_entropy_grad(const void *image, const double *stats, const float *scale, void *grad,
                     long long count, void *stream);

/* Gradient with respect to phase[m] of a real loss L of the image
 * I = A_az(rc_t . exp(i phase)), given dL/dI as FP32 pairs in g (stats ==
 * NULL), or, fused, given the image itself in g and its entropy stats
 * (L = E).  Per range bin the adjoint chain A^H = IDFT diag(conj H_a) DFT is
 * applied in FP32 and grad_phase[m] = sum_r Im(G_z[r][m] conj(z[r][m])) with
 * z = rc_t . exp(i phase) (device, n_az floats out).  phase NULL: the
 * plan's phasor table as the last call on the plan that took a phase vector
 * left it (sar_azimuth_image_entropy, sar_azimuth_compress without adjoint
 * or this call), i.e. exp(+i phase) of that call's phase as it was when the
 * call ran, so an autofocus iteration's image and gradient share one table;
 * BFP_EINVAL if that last call was an adjoint compression or there was none.
 * az_plan: precision BFP_FP32 or BFP_FP16_STORE_FP32_COMPUTE, created with
 * BFP_FLAG_AUTOFOCUS; n_range <= plan batch.  Calls on one plan must not
 * overlap (they share the plan's workspace). */
int sar_azimuth_phase_grad(bfp_plan az_plan, const void *rc_t, const void *g, const double *stats,
                           const void *h_az, const float *phase, float *grad_phase, int n_range,
                           void *stream);

/* One Adam step (Kingma & Ba, 2015, Algorithm 1) of the autofocus phase:
 *   k = *step + 1;  m = beta1 m + (1 - beta1) g;  v = beta2 v + (1 - beta2) g^2;
 *   phase -= lr (m / (1 - beta1^k)) / (sqrt(v / (1 - beta2^k)) + eps);  *step = k.
 * phase, grad, m, v: device, n floats each (m and v zeroed by the caller
 * before the first step); step: device, one unsigned (zeroed before the
 * first step).  All state stays on the device, so a whole autofocus
 * iteration (sar_azimuth_image_entropy, sar_azimuth_phase_grad, this call)
 * can be captured in a graph and replayed.  n in [1, 2^20]; lr finite and
 * >= 0; beta1, beta2 in [0, 1); eps finite and > 0; otherwise BFP_EINVAL
 * before any launch.  Calls on the same state must not overlap. */
int sar_autofocus_adam(float *phase, const float *grad, float *m, float *v, unsigned *step, int n,
                       float lr, float beta1, float beta2, float eps, void *stream);

/* sar_autofocus_adam with a learning-rate schedule read on the device, so a
 * graph-captured iteration follows it on every replay: step k (the updated
 * *step) uses lr_schedule[min(k, schedule_len) - 1]; (device) lr_schedule
 * holds schedule_len floats, each finite and >= 0 (any other entry gives a
 * zero step).  schedule_len in [1, 2^20]; the other arguments as for
 * sar_autofocus_adam.  Errors: BFP_EINVAL before any launch. */
int sar_autofocus_adam_schedule(float *phase, const float *grad, float *m, float *v, unsigned *step,
                                int n, const float *lr_schedule, int schedule_len, float beta1,
                                float beta2, float eps, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BFPFFT_H */
