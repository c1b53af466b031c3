/*
 * sonar.h -- C ABI of the MI355X energyscape library.
 *
 * One multi-microphone recording of a broadband FM sweep's echoes becomes one
 * energyscape E[d][q]: the reflector intensity along range bin q for
 * direction of interest d.  The pipeline is the one of the paper's processing
 * chain (Fig. 3 caption; §4.1 Signal Processing; §4.3 GPU Algorithm
 * Implementation): a matched filter against the emitted sweep, delay-and-sum
 * beamforming toward every direction, and an envelope detector whose output
 * is subsampled.  The exact arithmetic each call performs is written next to
 * it below.
 *
 * DFT convention: X[k] = sum_n x[n] exp(-2 pi i k n / P),
 *                 IDFT(X)[n] = (1/P) sum_k X[k] exp(+2 pi i k n / P).
 *
 * Conventions shared by every call
 *  - Host arrays in the plan descriptor are copied by sonar_plan_create; the
 *    caller may free them afterwards.
 *  - Every pointer passed to an execution call is caller-owned DEVICE memory on
 *    the device that was current when the plan was created, contiguous, 16-byte
 *    aligned, laid out as stated.  The library never allocates during
 *    execution: the plan owns all workspace, allocated once at creation (the
 *    paper preallocates device memory for the same reason, §4.3).
 *  - Execution calls only enqueue work on the given stream (no implicit
 *    synchronisation).  One plan serves one stream at a time because its
 *    workspace is shared between calls.
 *  - Errors are negative status codes; nothing is thrown or aborted across the
 *    ABI.  sonar_last_error() returns a thread-local message for the last
 *    failing call on the calling thread.  Launch failures map to SONAR_E_HIP;
 *    asynchronous device faults surface at the caller's next synchronisation.
 *    NaN or Inf in the samples propagate unchecked.
 */
#ifndef SONAR_H
#define SONAR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sonar_plan_s* sonar_plan;

enum sonar_status {
  SONAR_OK = 0,
  SONAR_E_INVALID = -1,      /* bad argument (null pointer, size, range)            */
  SONAR_E_NOMEM = -2,        /* device allocation failed, or above max_workspace    */
  SONAR_E_HIP = -3,          /* a HIP runtime call or kernel launch failed          */
  SONAR_E_UNSUPPORTED = -4   /* valid per the definition, not supported by the build */
};

/* Beamformer (§4.1: delay-and-sum steering toward each direction).
 *  TD_LINEAR : fractional delay by linear interpolation between samples.
 *  FD_FP32   : exact fractional delay as a per-frequency-bin phase; the
 *              per-bin complex product over microphones runs in FP32.
 *  FD_BF16   : as FD_FP32 on BF16 MFMA with FP32 accumulation: the
 *              steering operand is rounded to one BF16 term, the sample
 *              operand is carried as two BF16 terms (hi + lo), two products.
 *  FD_BF16X3 : as FD_BF16 with each operand split into two BF16 terms
 *              (hi + lo) and three products (hi*hi + hi*lo + lo*hi).
 *  TD_BF16   : the TD_LINEAR result computed on BF16 MFMA with FP32
 *              accumulation: directions are tiled 32 at a time and the
 *              interpolation becomes a dense product of a tap-weight matrix
 *              with a Hankel matrix of samples; weights and samples are each
 *              split into two BF16 terms (hi + lo), three products.  Only the
 *              fused beamformer + envelope runs on MFMA; sonar_beamform in
 *              this mode returns the FP32 beam.
 *  TD_NEAREST: integer delays (the delay rounded to the nearest sample, ties
 *              toward the later sample): o = floor(-Dl + 1/2),
 *              b_d[n] = (1/M) sum_m yhat_m[(n + o) mod P]; FP32, same kernels
 *              and buffers as TD_LINEAR with the second weight zero.
 *  TD_BF16X2 : as TD_BF16 with the samples carried as one BF16 term (the
 *              weights still split): two products, four MFMAs per K-chunk,
 *              two BF16 planes per microphone.  Its error is the samples'
 *              BF16 rounding averaged over the microphones: within 1e-3 for
 *              arrays of 32 or more microphones (SONAR_PREC_BF16 picks it only
 *              there).  In TD_BF16X2 and TD_F16 the envelope's low-pass runs on
 *              FP16 MFMA: |b| as one FP16 term scaled per tile of 32 directions
 *              by a power of two (largest scaled value below 2^14), the taps as
 *              two FP16 terms after a plan-time power-of-two scale that puts the
 *              largest tap in [2^13, 2^14) (undone in FP32 at the store, so
 *              filters of any gain keep about 22 bits per tap).
 *  TD_CUBIC  : 4-point Lagrange (cubic) fractional delay: o = floor(-Dl),
 *              a = -Dl - o, b_d[n] = (1/M) sum_m sum_{k=-1..2} L_k(a) yhat_m[n+o+k],
 *              L_k(a) = prod_{j != k} (a - j)/(k - j); FP32 on the TD_LINEAR
 *              kernels, each microphone taken as two two-tap entries.  M <= 64.
 *  TD_F16    : TD_LINEAR with the fractional delay on a grid of 1/2048
 *              sample (alpha = rint(2048 (-Dl - o)) / 2048, o = floor(-Dl),
 *              alpha = 1 taken as o + 1, alpha = 0), computed on FP16 MFMA
 *              with FP32 accumulation: the weights 1 - alpha and alpha are
 *              exact in FP16, the samples are one FP16 term scaled per frame
 *              by a power of two 2^e chosen from a bound on |yhat| (so the
 *              scaled samples stay below 2^14), and E is scaled back by
 *              2^-e / M in FP32.  Two products (re, im), two MFMAs per
 *              K-chunk, two FP16 planes per microphone.  The grid moves a
 *              delay by at most 1/4096 sample; with the samples' FP16
 *              rounding the result is within about 1e-4 of TD_LINEAR.
 *              Samples below 2^-28 of the frame's bound are FP16 subnormals
 *              (less relative precision, far below the 1e-4 scale of the
 *              error); e is clamped to [-100, 100], so frames whose bound
 *              lies outside [2^-86, 2^114] overflow or underflow.
 *  TD_BF16G  : TD_LINEAR with the fractional delay on a grid of 1/256 sample
 *              (alpha = rint(256 (-Dl - o)) / 256, alpha = 1 taken as o + 1,
 *              alpha = 0), computed on BF16 MFMA with FP32 accumulation: the
 *              weights 1 - alpha and alpha are exact in one BF16 term, the
 *              samples are one BF16 term (two BF16 planes per microphone, as in
 *              TD_BF16X2): two products (re, im), two MFMAs per K-chunk.  The
 *              grid moves a delay by at most 1/512 sample; with the samples'
 *              BF16 rounding the result is within 1e-3 of TD_LINEAR for arrays
 *              of 32 or more microphones (SONAR_PREC_BF16 offers it only there).
 *              The low-pass runs as in TD_BF16X2. */
enum sonar_bf_mode {
  SONAR_BF_TD_LINEAR = 0, SONAR_BF_FD_FP32 = 1, SONAR_BF_FD_BF16 = 2, SONAR_BF_FD_BF16X3 = 3,
  SONAR_BF_TD_BF16 = 4, SONAR_BF_TD_NEAREST = 5, SONAR_BF_TD_CUBIC = 6, SONAR_BF_TD_BF16X2 = 7,
  SONAR_BF_TD_F16 = 8, SONAR_BF_TD_BF16G = 9
};

/* Element type of the microphone samples x. */
enum sonar_dtype { SONAR_F32 = 0, SONAR_F16 = 1, SONAR_BF16 = 2 };

typedef struct {
  int32_t n_mics;            /* M >= 1 (the eRTIS has 32, §2)                               */
  const double* mic_pos;     /* [M][3] microphone positions, metres                          */
  int32_t chirp_len;         /* L >= 1                                                       */
  const double* chirp;       /* [L] emitted sweep sampled at fs (the matched-filter template) */
  double fs_hz;              /* sample rate (450 kHz on the eRTIS, §2)                       */
  double c_mps;              /* speed of sound                                               */
  int32_t n_dirs;            /* D >= 1                                                       */
  const double* dirs;        /* [D][3] unit vectors, | |u| - 1 | <= 1e-9                      */
  int32_t n_samples;         /* N samples per channel, N >= L                                */
  int32_t gate_begin;        /* range gate [n0, n1) in matched-filter samples;              */
  int32_t gate_end;          /*   0, 0 selects [0, N)                                        */
  int32_t decim;             /* R >= 1, subsampling factor after the envelope (§4.3)        */
  int32_t lpf_len;           /* K, odd; 0 selects the default low-pass (K = 8R + 1)          */
  const double* lpf_taps;    /* [K] envelope low-pass taps, or NULL for the default          */
  double band_lo_hz;         /* matched-filter band mask [lo, hi] in Hz;                    */
  double band_hi_hz;         /*   0, 0 disables the mask                                     */
  int32_t fft_len;           /* P: even, >= N + L - 1; 0 selects the smallest power of two  */
                             /*   (the library transforms powers of two 32 .. 524288 only)   */
  int32_t bf_mode;           /* enum sonar_bf_mode                                            */
  int32_t sample_dtype;      /* enum sonar_dtype of x                                         */
  int32_t max_frames;        /* F_max >= 1: the workspace is sized for this batch            */
} sonar_plan_desc;

/* Keys for sonar_plan_query. */
enum sonar_query {
  SONAR_Q_RANGE_BINS = 0,     /* Q = ceil((n1 - n0) / R)                                   */
  SONAR_Q_BEAM_LEN = 1,       /* G' = (Q - 1) R + K: beam samples per direction            */
  SONAR_Q_FFT_LEN = 2,        /* P                                                          */
  SONAR_Q_MF_ROW = 3,         /* complex elements per microphone row of the MF buffer      */
  SONAR_Q_MF_ORIGIN = 4,      /* TD: sample index n of MF row element 0 (may be negative)  */
  SONAR_Q_BAND_LO_BIN = 5,    /* FD: first stored frequency bin                            */
  SONAR_Q_BAND_BINS = 6,      /* FD: number of stored frequency bins Kb                    */
  SONAR_Q_WORKSPACE_BYTES = 7,/* device bytes owned by the plan                            */
  SONAR_Q_LPF_LEN = 8,        /* K                                                          */
  SONAR_Q_MF_FRAME_ELEMS = 9, /* complex elements per frame of the MF buffer               */
  SONAR_Q_MATRIX_FLOP_PER_FRAME = 10, /* MFMA TD modes: matrix-core flops issued per frame by the
                                         fused beamformer (padding included); 0 otherwise  */
  SONAR_Q_MT_WAVES = 11               /* MFMA TD modes: wavefronts per beamformer workgroup
                                         (4: two workgroups per CU; 8: wide apertures); else 0 */,
  SONAR_Q_BEAM_SPEC_STRIDE = 12,      /* FD modes: complex elements per direction row of sonar_beam_spectrum's
                                         output (the stored bins, padded to a multiple of 16); else 0 */
  SONAR_Q_FD_PHASE_LEN = 13,          /* FD modes: points L of each phase of the per-direction inverse; else 0 */
  SONAR_Q_FD_FUSED = 14               /* FD modes: 1 when inverse, magnitude and low-pass are one kernel; else 0 */
};

/*
 * sonar_plan_create -- validate the descriptor, copy it, allocate the plan's
 * whole device workspace for max_frames frames, and build the plan tables on
 * the device in FP64 (§4.1: the delay of every direction relative to every
 * channel is computed up front):
 *   Dl[d][m] = fs * (p_m . u_d) / c  samples;
 *   TD: o = floor(-Dl), alpha = -Dl - o;
 *   C[k] = beta[k] W[k] conj(S[k]), S = DFT_P(chirp), W the one-sided analytic
 *   weights (1, 2, ..., 2, 1, 0, ...), beta the band mask;
 *   FFT twiddles.
 * The tables are built with work enqueued on `stream`; the call synchronises
 * that stream before returning.  Returns SONAR_E_INVALID for a descriptor that
 * breaks a rule stated above (an odd P or P < N + L - 1 among them);
 * SONAR_E_UNSUPPORTED for an even P >= N + L - 1 that is not a power of two
 * or lies outside [32, 524288], and for array apertures whose delay spread
 * exceeds the beamformer tiles; SONAR_E_NOMEM when allocation fails.  *out is
 * set only on success.  The frequency-domain modes run their per-direction
 * inverse as P / L transforms of L <= 16384 points with the stored bins folded
 * modulo L; when at most two bins fold onto a slot and Q <= L / 2 the inverse,
 * magnitude and low-pass are one kernel (no beam window in memory), otherwise
 * the beam window is kept in the plan's workspace ([max_frames][D][G']).
 */
int sonar_plan_create(const sonar_plan_desc* desc, hipStream_t stream, sonar_plan* out);

/* Free every device buffer of the plan.  NULL is accepted.  The caller must
 * make sure no work that uses the plan is still pending. */
int sonar_plan_destroy(sonar_plan plan);

/* Read one derived size of the plan (enum sonar_query) into *value. */
int sonar_plan_query(sonar_plan plan, int32_t what, int64_t* value);

/*
 * sonar_matched_filter -- §4.1 matched filter, realised as an FFT filter with
 * its group delay removed (§4.3):
 *   yhat_m[n] = IDFT_P( beta W X_m conj(S) )[n],  X_m = DFT_P(x_m zero-padded),
 * i.e. the analytic signal of the correlation sum_l s[l] x_m[n + l], circular
 * in P.
 *   x      : [F][M][N] samples of sample_dtype.
 *   mf_out : complex64 (float re, im) buffer, SONAR_Q_MF_FRAME_ELEMS per frame.
 *            TD modes: [F][M][row] with row = SONAR_Q_MF_ROW, element i holding
 *            yhat_m[(origin + i) mod P], origin = SONAR_Q_MF_ORIGIN.  TD_BF16
 *            appends to each frame the same samples as BF16 planes
 *            [M][4][row] (re hi, re lo, im hi, im lo; hi = bf16(v),
 *            lo = bf16(v - hi), round to nearest even), so a frame holds
 *            2*M*row complex64 elements; TD_BF16X2 appends [M][2][row]
 *            (re hi, im hi), 1.5*M*row complex64 elements per frame;
 *            TD_F16 appends [M][2][row] FP16 planes (re, im of 2^e yhat)
 *            and one 16-byte frame header whose first float is 2^-e / M,
 *            1.5*M*row + 2 complex64 elements per frame (the beamformer
 *            reads the scale from there, so a buffer stays valid for
 *            sonar_beamform_envelope after later matched-filter calls).
 *            FD modes: [F][Kb][M] (bin-major), element (j, m) holding the
 *            spectrum Yhat_m[k] = beta W X_m conj(S) at bin k = band_lo_bin + j
 *            (Kb = SONAR_Q_BAND_BINS; bins outside are zero by definition).
 *   F      : 1 <= F <= max_frames.
 */
int sonar_matched_filter(sonar_plan plan, const void* x, int32_t F, void* mf_out,
                         hipStream_t stream);

/*
 * sonar_beamform -- §4.1 delay-and-sum toward every direction, evaluated on the
 * beam window n = n0 - (K-1)/2 + i, i in [0, G'):
 *   TD: b_d[n] = (1/M) sum_m (1 - a) yhat_m[n + o] + a yhat_m[n + o + 1],
 *       (o, a) = (o[d][m], alpha[d][m]), indices mod P;
 *   FD: b_d = IDFT_P( (1/M) sum_m Yhat_m[k] exp(-2 pi i k Dl[d][m] / P) ).
 *   mf_in    : a buffer written by sonar_matched_filter with this plan.
 *   beam_out : complex64 [F][D][G'].
 */
int sonar_beamform(sonar_plan plan, const void* mf_in, int32_t F, void* beam_out,
                   hipStream_t stream);

/*
 * sonar_beam_spectrum -- the first half of the frequency-domain beamformer
 * (§4.1 delay-and-sum with each channel's delay applied as a per-bin phase),
 * for FD plans only: the per-bin product over microphones
 *   B_d[k] = (1/M) sum_m Yhat_m[k] exp(-2 pi i k Dl[d][m] / P)
 * on the stored bins k = band_lo_bin + j, j < Kb (SONAR_Q_BAND_BINS).
 *   mf_in    : a buffer written by sonar_matched_filter with this plan.
 *   spec_out : complex64 [F][D][S], S = SONAR_Q_BEAM_SPEC_STRIDE; element (f, d, j)
 *              holds B_d at bin band_lo_bin + j for j < Kb (S - Kb padding
 *              elements per row are written with unspecified values).
 * SONAR_E_INVALID for a time-domain plan.
 */
int sonar_beam_spectrum(sonar_plan plan, const void* mf_in, int32_t F, void* spec_out, hipStream_t stream);

/*
 * sonar_envelope -- §4.1 envelope and §4.3 subsampling:
 *   E[d][q] = sum_{j<K} h[j] |b_d[n0 + q R + (K-1)/2 - j]|,  q in [0, Q),
 * a zero-phase FIR low-pass of the beam magnitude read at every R-th sample.
 *   beam_in : complex64 [F][D][G'] as written by sonar_beamform.
 *   E       : float [F][D][Q].
 */
int sonar_envelope(sonar_plan plan, const void* beam_in, int32_t F, float* E,
                   hipStream_t stream);

/*
 * sonar_beamform_envelope -- sonar_beamform followed by sonar_envelope with
 * the beam kept on chip (it is never written to memory):
 *   E[d][q] = sum_{j<K} h[j] |b_d[n0 + q R + (K-1)/2 - j]|,  b as in sonar_beamform.
 *   mf_in : a buffer written by sonar_matched_filter with this plan.
 *   E     : float [F][D][Q].
 */
int sonar_beamform_envelope(sonar_plan plan, const void* mf_in, int32_t F, float* E,
                            hipStream_t stream);

/*
 * sonar_energyscape_batch -- the whole chain for F recordings that share the
 * plan (geometry, directions, sweep): the result equals sonar_envelope(
 * sonar_beamform(sonar_matched_filter(x))) up to floating-point reordering, but
 * the beam is never written to memory.
 *   x : [F][M][N] samples of sample_dtype;  E : float [F][D][Q].
 */
int sonar_energyscape_batch(sonar_plan plan, const void* x, int32_t F, float* E,
                            hipStream_t stream);

/*
 * sonar_energyscape_batch_static -- for callers that cannot allocate device
 * memory or touch allocation calls at all (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the result of
 * sonar_energyscape_batch bit for bit (the same kernels), with every
 * per-frame buffer beyond x and E (matched-filter spectra and rows or planes,
 * band and beam spectra, transform scratch, frame bounds) taken from a
 * 128 MiB static device array of the library instead of the plan's
 * workspace.  The call allocates and frees nothing.  Each device holds its
 * own copy of the array from the time the library is loaded until the process
 * ends; its device address is taken when the first plan is created on that
 * device.  Every call on a device shares that device's array and leaves its
 * contents behind (nothing in it needs to start at zero): calls that overlap
 * on one device, on any streams, race, and must be ordered by the caller.
 *   x : [F][M][N] samples of sample_dtype;  E : float [F][D][Q].
 * SONAR_E_INVALID (nothing enqueued) when F frames of this plan need more than
 * the 128 MiB (the message states how many frames fit).
 */
int sonar_energyscape_batch_static(sonar_plan plan, const void* x, int32_t F, float* E,
                                   hipStream_t stream);

/*
 * sonar_energyscape_multi -- the whole chain for n independent items, each
 * with its own plan (its own sensor geometry, recording length, direction
 * grid and mode): E_i = sonar_energyscape_batch(plans[i], x[i], frames[i]).
 * This is the sensor network's batch (§3: many sensors' measurements are
 * processed by the same GPU service; §5).  All items are validated before any
 * work is enqueued.  Items whose plans are MFMA time-domain modes (TD_BF16,
 * TD_BF16X2, TD_F16, TD_BF16G) with the FIR envelope, each plan once in the call, run
 * first, on `stream`: their matched filters, then ONE persistent
 * beamformer + envelope launch per group of up to 16 items with the same mode
 * and workgroup shape (a fixed grid of workgroups walks a work list of every
 * item's tiles of 32 directions x range; item descriptors travel as kernel
 * arguments), bit-identical to the items' own batch calls.  The other items
 * then run concurrently: forked from `stream` onto
 * it and up to three library-owned side streams of the device (created with
 * its first plan, default priority), largest items first onto the least
 * loaded stream, items sharing a plan on one stream in order, and joined back
 * into `stream` by events, so work enqueued on `stream` afterwards sees every
 * E_i.  The call enqueues kernels and event records/waits only (no
 * allocation, no synchronisation, no memset), so a caller may capture it in a
 * HIP graph on `stream` (the branches become parallel graph nodes) and replay
 * it; replays reuse the plans' workspaces, so replays of graphs that share a
 * plan must not overlap.  Concurrent calls on one device are serialised on
 * the host while they enqueue.  Side streams that joined a capture stay in it
 * until that capture ends: while they are joined to a capture other than the
 * one `stream` belongs to (a graph still being recorded on another stream, or
 * an eager call during such a recording), the call runs its items in order on
 * `stream` alone (same results, no concurrency).
 *   plans  : n plan handles (a plan may appear more than once).
 *   x      : n device pointers, x[i] = [frames[i]][M_i][N_i] samples.
 *   frames : n frame counts, 1 <= frames[i] <= max_frames of plans[i].
 *   E      : n device pointers, E[i] = float [frames[i]][D_i][Q_i].
 * Returns SONAR_E_INVALID (nothing enqueued) when any item is invalid.
 */
int sonar_energyscape_multi(const sonar_plan* plans, const void* const* x, const int32_t* frames,
                            float* const* E, int32_t n, hipStream_t stream);

/* Precision classes for sonar_plan_create_tuned. */
enum sonar_precision {
  SONAR_PREC_FP32 = 0,   /* modes within 1e-5 of the definition: TD_LINEAR, FD_FP32, FD_BF16X3  */
  SONAR_PREC_BF16 = 1    /* modes within 1e-3: the above, TD_BF16, TD_F16, and FD_BF16, TD_BF16X2 and TD_BF16G for >= 32 mics */
};

/*
 * sonar_plan_create_tuned -- picks the beamformer mode for a descriptor by
 * measurement: every mode of the precision class that the build supports for
 * the descriptor is planned and timed on max_frames frames of zero samples
 * (the kernels' time does not depend on the sample values), and the fastest
 * plan is returned; desc->bf_mode is ignored.  The MFMA time-domain modes are
 * tried with both workgroup shapes (4 and 8 wavefronts of 32 directions x 128
 * samples each; SONAR_Q_MT_WAVES reports the one kept), the frequency-domain
 * modes with their default phase length and half and twice it where the fused
 * inverse allows (SONAR_Q_FD_PHASE_LEN reports the one kept).  The call synchronises
 * `stream`.
 *   *chosen_mode (may be NULL) receives the selected enum sonar_bf_mode.
 * Returns the status of sonar_plan_create when no mode can be planned.
 */
int sonar_plan_create_tuned(const sonar_plan_desc* desc, int32_t precision, hipStream_t stream,
                            sonar_plan* out, int32_t* chosen_mode);

/*
 * sonar_tune_cache -- persist the choices of sonar_plan_create_tuned: with a
 * path set, a tuned creation first looks the descriptor up in that file and,
 * when found, creates the recorded plan (mode, MFMA workgroup size, frequency-
 * domain phase length) without timing anything; otherwise it tunes and appends
 * one JSON object per line, {"key": ..., "mode": m, "mt_waves": w,
 * "fd_logl": l, "ms": t}, the key naming every descriptor size, the precision
 * class, the device architecture and a hash of the geometry, directions,
 * sweep and taps.  NULL or "" switches the cache off (the default).  Process-
 * wide; the file is read and appended under a lock.
 */
int sonar_tune_cache(const char* path);

/*
 * Reverse-mode derivatives of the pipeline (the adjoint used to self-calibrate
 * the array: the delays of §4.1 depend on the microphone positions).  For a
 * real loss L with dE = dL/dE [F][D][Q], complex quantities z carry gradients
 * G_z = dL/dRe z + i dL/dIm z:
 *   envelope        G_b = (FIR^T dE) * b / |b|            (0 where b = 0)
 *   TD delay-and-sum
 *                   dL/dDl[d][m] = (1/M) sum_n Re(conj(G_b[n]) (yhat_m[n+o] - yhat_m[n+o+1]))
 *                   G_yhat_m  = the transposed interpolation of G_b
 *                   (o = floor(-Dl) is piecewise constant: derivatives almost everywhere)
 *   FD delay-and-sum
 *                   G_B[d][k] = DFT_P(G_b[d] on its window)[k] / P
 *                   dL/dDl[d][m] = (1/M) sum_k Re(conj(G_B[d][k]) Yhat_m[k] (-2 pi i k/P) e^{-2 pi i k Dl/P})
 *                   G_Yhat_m[k] = (1/M) sum_d e^{+2 pi i k Dl[d][m]/P} G_B[d][k]
 *                   (smooth in the delays: exact derivatives)
 *   delays          dL/dp_m = fs/c sum_{f,d} dL/dDl[f][d][m] u_d
 *   matched filter  dL/dx = Re sum_k conj(C[k]) G_Yhat[k] e^{2 pi i k n/P}, cut to N
 *                   (TD: G_Yhat = DFT_P(G_yhat) / P)
 * All gradient arithmetic is FP32 (dL/dp accumulated in FP64) on the buffers of
 * the forward pass given.
 *
 * sonar_plan_enable_gradients -- allocates the gradient workspace of the plan
 * (once; the bytes are added to SONAR_Q_WORKSPACE_BYTES), including the beam
 * window [max_frames][D][G'] that sonar_energyscape_backward fills.  Every FFT length
 * the plan accepts is supported: the P-point transforms of the adjoint run as P / L
 * phase transforms of L = min(P / 2, 16384) points, through a scratch of at most
 * 4 GiB (channels of P complex64 values, max_frames * D of them for frequency-domain
 * plans and max_frames * M for time-domain ones, or as many as fit; the adjoint then
 * takes them in chunks).
 */
int sonar_plan_enable_gradients(sonar_plan plan);

/*
 * sonar_energyscape_vjp -- the derivatives above for F frames, ordered on
 * `stream`.
 *   mf_in      : the matched-filter buffer of the forward pass (sonar_matched_filter).
 *   beam_inout : the beam window of the forward pass (sonar_beamform),
 *                complex64 [F][D][G']; overwritten with G_b.
 *   dE         : float [F][D][Q].
 *   dyhat_out  : gradient of the matched-filter output, or NULL.  TD modes:
 *                complex64 [F][M][P] G_yhat over Z_P (sample n at index n).
 *                FD modes: complex64 [F][Kb][M], G_Yhat on the band bins in
 *                the layout of the FD matched-filter buffer.
 *   dx_out     : float [F][M][N], or NULL (needs dyhat_out).
 *   dpos_out   : double [M][3] dL/dp_m summed over the F frames, or NULL.
 * SONAR_E_INVALID before sonar_plan_enable_gradients.
 */
int sonar_energyscape_vjp(sonar_plan plan, const void* mf_in, void* beam_inout, const float* dE,
                          int32_t F, void* dyhat_out, float* dx_out, double* dpos_out,
                          hipStream_t stream);

/*
 * sonar_energyscape_backward -- the whole backward pass from the samples:
 * matched filter, beam window (both in the plan's workspace) and the
 * derivatives above, for F frames of x [F][M][N] (sample_dtype) and
 * dE [F][D][Q].  dx_out float [F][M][N] or NULL, dpos_out double [M][3] or NULL
 * (summed over the frames).  Needs sonar_plan_enable_gradients (which also
 * allocates the beam window and matched-filter gradient this call uses).
 */
int sonar_energyscape_backward(sonar_plan plan, const void* x, const float* dE, int32_t F, float* dx_out,
                               double* dpos_out, hipStream_t stream);

/*
 * sonar_energyscape_cells -- selected energyscape cells and the position
 * derivative of a loss that reads only them, for calibration losses whose dE
 * vanishes elsewhere (a few reflector cells of a whole energyscape).  Each cell
 * c = (f, d, q) is computed by the definitions of sonar_energyscape (section 4.1
 * beamformer, envelope and subsampling) on its K window samples
 * n_i = n0 - (K-1)/2 + qR + i only:
 *   frequency-domain plans (FD_FP32, FD_BF16, FD_BF16X3; exact phase, section 4.3):
 *     B[k] = (1/M) sum_m Y_m[k] e^{-2 pi i k Dl[d][m]/P} on the band bins and
 *     b_i = IDFT_P(B) at n_i, from the band spectra alone (no P-point transform);
 *   FP32 time-domain plans (TD_LINEAR, TD_NEAREST, TD_CUBIC): b_i = the plan's
 *     interpolated delay-and-sum at n_i from the matched-filter rows;
 *   E_c = sum_i h[K-1-i] |b_i|,
 * and for L = sum_c dE[c] E_c the chain of sonar_energyscape_vjp restricted to
 * the cells' windows gives dL/dp (TD_NEAREST: refused, as in the dense call).
 *   mf_in     : the matched-filter buffer of the F frames (sonar_matched_filter):
 *               FD complex64 [F][Kb][M], TD the rows with their halo.
 *   cells     : int32 [n_cells][3] (f, d, q) in device memory; a cell outside
 *               [0, F) x [0, D) x [0, Q) yields E = NaN and adds nothing to dL/dp.
 *   dE        : float [n_cells] in device memory (the weights dL/dE_c).
 *   E_out     : float [n_cells], or NULL.
 *   dpos_out  : double [M][3], or NULL.
 * Repeated cells count once each.  Needs sonar_plan_enable_gradients (its
 * workspace holds the per-cell partial sums, so n_cells <= max_frames * D),
 * K <= 256, and for FD plans M <= 256 and 2K + M <= 2P (SONAR_E_UNSUPPORTED
 * otherwise, and for the BF16 / FP16 time-domain modes).  FP32 arithmetic with the steering phases reduced in FP64, as the
 * dense derivative.  Uses the same workspace as sonar_energyscape_vjp: calls on
 * one plan must be ordered (one stream).
 */
int sonar_energyscape_cells(sonar_plan plan, const void* mf_in, const int32_t* cells, int32_t n_cells,
                            const float* dE, int32_t F, float* E_out, double* dpos_out, hipStream_t stream);

/*
 * sonar_plan_set_positions -- new microphone positions [M][3] (metres): the
 * delay tables (§4.1 delays) are rebuilt on `stream` without reallocating,
 * ordered after the work already queued there.  A time-domain plan whose new
 * geometry needs delays outside the plan's range returns SONAR_E_UNSUPPORTED
 * and keeps its old positions (the plan keeps 3 samples of slack on each side
 * of the geometry it was created with).
 * MFMA TD modes (TD_BF16, TD_BF16X2, TD_F16, TD_BF16G): their direction tiles,
 * tap groups and weight fragments follow the geometry, so the call also
 * synchronizes `stream`, rebuilds those tables on the host and replaces them
 * (device allocations: not for graph capture or no-allocation callers).  The
 * plan must not be in use on another stream meanwhile.  If the rebuild fails
 * (SONAR_E_NOMEM, SONAR_E_HIP), the delay table already holds the new
 * positions while the tiles keep the old ones: set the positions again or
 * create a new plan.
 */
int sonar_plan_set_positions(sonar_plan plan, const double* mic_pos, hipStream_t stream);
/* (TD_NEAREST and TD_CUBIC plans move like TD_LINEAR ones.  TD_NEAREST's dL/dp is zero
 * almost everywhere, so sonar_energyscape_vjp returns SONAR_E_UNSUPPORTED for dpos_out on
 * it, and on TD_F16 and TD_BF16G, whose delays lie on a 1/2048- or 1/256-sample grid; dx_out
 * of those plans is the adjoint of TD_LINEAR on the gridded delays.  TD_CUBIC's gradients are
 * those of its 4-point Lagrange reading: dx from the four taps' weights, dpos from their
 * slopes in the fractional delay.) */

/*
 * PDM front end (§2: the microphones deliver 1-bit sigma-delta pulse-density
 * modulation; §4.3: the binary data are unpacked, demodulated by a low-pass
 * filter and subsampled before the matched filter):
 *   x[m][n] = sum_{j<K} h[j] s_m[n D + (K-1)/2 - j],  n < N,
 * with s_m[t] = +1 (bit set) or -1 (bit clear) for the T = N D recorded ticks and
 * 0 outside them: a zero-phase FIR low-pass at the PDM rate evaluated at every
 * D-th tick.  Packing: each tick is W = ceil(M/32) little-endian 32-bit words,
 * microphone m in bit m % 32 of word m / 32.
 */
typedef struct sonar_pdm_s* sonar_pdm;

typedef struct {
  int32_t n_mics;          /* M, 1 <= M <= 128                                            */
  int32_t n_out;           /* N >= 1 output samples per microphone                        */
  int32_t decim;           /* D >= 1 PDM ticks per output sample (10: 4.5 MHz -> 450 kHz)  */
  int32_t n_taps;          /* K, odd, <= 513; 0 selects the default                       */
  const double* taps;      /* [K] host taps h, or NULL for the default: Hamming-windowed   */
                           /* sinc, K = 32 D + 1, cutoff 1/(4 D) of the PDM rate, unit DC  */
                           /* gain (passband flat to 0.05 dB below 85 kHz at D = 10)       */
  int32_t max_frames;      /* F per call, >= 1                                             */
} sonar_pdm_desc;

/* sonar_pdm_create -- builds the filter's tables on the current device (on
 * `stream`, synchronised before returning).  SONAR_E_UNSUPPORTED when the
 * staging of one workgroup would not fit in LDS (very large D or K). */
int sonar_pdm_create(const sonar_pdm_desc* desc, hipStream_t stream, sonar_pdm* out);
int sonar_pdm_destroy(sonar_pdm pdm);

/*
 * sonar_pdm_demodulate -- F frames: words [F][N D][W] uint32 (device) ->
 * x [F][M][N] float (device), the sample layout sonar_matched_filter and
 * sonar_energyscape_batch take with SONAR_DTYPE_F32.  Enqueues one kernel.
 */
int sonar_pdm_demodulate(sonar_pdm pdm, const uint32_t* words, int32_t F, float* x, hipStream_t stream);

/*
 * sonar_plan_set_envelope_iir -- the IIR reading of the envelope filter (§4.3:
 * the CPU implementation runs Butterworth filters through a causal lfilter).
 * Afterwards every envelope of the plan (sonar_envelope, sonar_beamform_envelope,
 * sonar_energyscape_batch) is
 *   y_d = causal IIR of |b_d| over the beam window from zero state at its first
 *         sample n0 - (K-1)/2,      E[d][q] = y_d at sample n0 + qR,
 * with the beam window materialised in the plan's workspace (allocated here, once)
 * instead of the fused FIR epilogue.
 *   n_sections : 1..4 second-order sections, or 0 to return to the FIR envelope.
 *   sos        : [n_sections][6] host array {b0, b1, b2, a0, a1, a2} per section (the
 *                cascade's transfer function is the product), or NULL for the
 *                Butterworth low-pass of order 2 n_sections with -3 dB at fs/(2R)
 *                (bilinear transform with prewarping, unit DC gain).
 * The cascade runs as one state-space recurrence in FP32, evaluated in parallel
 * over 64 chunks of each row by a scan of chunk end states.  Gradients
 * (sonar_energyscape_vjp) are built for the FIR envelope only.
 */
int sonar_plan_set_envelope_iir(sonar_plan plan, int32_t n_sections, const double* sos, hipStream_t stream);

/* Static text for a status code. */
const char* sonar_status_string(int status);

/* Thread-local detail message of the last failing call on this thread ("" if none). */
const char* sonar_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SONAR_H */
