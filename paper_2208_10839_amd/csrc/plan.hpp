// Internal plan object and kernel launchers of the energyscape library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <vector>

#include "sonar.h"

// Tile shape of the time-domain beamformer: one wavefront per direction,
// TD_NW directions per workgroup, TD_NB blocks of 64 consecutive beam samples
// per wavefront (one sample per lane).
constexpr int TD_NB = 16;
constexpr int TD_NW = 8;
constexpr int TD_XCDS = 8;       // accelerator dies (each with its own L2) that workgroups are spread over
constexpr int TD_FIR_DIRS = 2;   // directions per thread in the fused low-pass stage
constexpr int TD_WAVES_PER_EU = 4;   // two workgroups per CU (80 KiB LDS each): 128 VGPRs per lane
constexpr int TD_LDS_BYTES = 80 * 1024;    // LDS budget of one beamformer workgroup
constexpr int TD_MAX_MICS = 128;
constexpr int TD_MAX_ROW_PAIRS = 640;   // staged row = 1280 samples: delay spread <= 1280 - 64 * TD_NB - 1

struct sonar_plan_s {
  // descriptor (copied)
  int M = 0, L = 0, D = 0, N = 0;
  int n0 = 0, n1 = 0, R = 1, K = 0;
  int P = 0, NF = 0, logNF = 0;
  int bf_mode = 0, dtype = 0, max_frames = 1;
  double fs = 0, c = 0, band_lo = 0, band_hi = 0;
  bool band_on = false;

  // derived sizes
  int Q = 0;            // range bins
  int G = 0;            // beam window length G' = (Q-1)R + K
  int hk = 0;           // (K-1)/2
  int omin = 0, omax = 0, spread = 0;   // bounds of o = floor(-Dl) over all (d, m)
  int64_t origin = 0;   // sample index of MF row element 0 (TD)
  int row = 0;          // complex elements per MF row (TD), a multiple of 8
  long long mf_fstride = 0;   // complex64 elements per frame of the TD MF buffer: M*row, or 2*M*row
                              // when the BF16 planes [M][4][row] follow the complex rows (TD BF16)

  // time-domain beamformer tiling
  int td_ws = 0;        // staged samples per microphone
  int td_mc = 0;        // microphones staged per pass
  int td_tn = 0;        // valid beam samples per wavefront tile (64*NB - 1)
  int td_qc = 0;        // range bins per tile
  int td_nqc = 0;       // range-bin tiles
  int td_nbc = 0;       // beam-sample tiles (beamform-only kernel)
  int td_vshift = 0;    // delay-table entries per microphone = 1 << td_vshift (2 for TD_CUBIC)

  // frequency-domain layout: stored band bins [k_lo, k_lo + kb); the
  // per-direction inverse transform runs as fd_R polyphase transforms of
  // fd_L = P / fd_R points, the stored bins folded modulo fd_L (fd_nfold = ceil(kb / fd_L))
  int k_lo = 0, kb = 0;
  int kb_pad = 0;       // row stride (bins) of the per-direction spectra
  int fd_L = 0, fd_logL = 0, fd_R = 0, fd_nfold = 0;
  bool fd_fused = false;   // the fused inverse + envelope kernel serves this plan (else beam window + envelope)
  bool fd_win = false;     // fused, with the whole beam window in LDS (the window fits beside the transform)

  // time-domain BF16-MFMA beamformer tiling (see k_das_mfma.hip)
  int mt_ntiles = 0, mt_nmc = 0, mt_qc = 0, mt_nqt = 0, mt_wrow = 0, mt_gmax = 0, mt_kcmax = 0;
  int mt_nwave = 0;     // wavefronts per workgroup (MT_NWAVE_SMALL or MT_NWAVE_LARGE)
  long long mt_flop_per_frame = 0;   // matrix-core flops issued per frame
  float mt_fir_unscale = 1.f;          // 2^-ts (two-plane modes: taps stored times 2^ts), times 1/M for TD_BF16G
                                       // (its exact weights leave out the array mean's 1/M)
  std::vector<double> h_dirs;          // [D][3] and [K] host copies of the directions and FP64 taps: the
  std::vector<double> h_taps;          // MFMA tiles are rebuilt from them when the positions change

  int device = 0;
  int cu_count = 0;     // compute units of the device
  size_t ws_bytes = 0;

  // device buffers (owned)
  int4* d_dtab = nullptr;      // [D][M] {o - omin, bits((1-a)/M), bits(a/M), 0}
  double* d_dl = nullptr;      // [D][M] delays in samples (FP64)
  double* d_pos = nullptr;     // [M][3]
  double* d_dirs = nullptr;    // [D][3]
  double* d_chirp = nullptr;   // [L]
  float* d_taps = nullptr;     // [K]
  float2* d_cspec = nullptr;   // [NF+1] beta W conj(S)
  float2* d_tw = nullptr;      // FFT twiddle tables (see fft layout)
  float2* d_mf = nullptr;      // MF workspace, [max_frames][M][row]
  float2* d_spec = nullptr;    // one-sided MF spectra, [max_frames][M][NF+1]
  float2* d_fdspec = nullptr;  // FD: band spectra of the MF output, [max_frames][kb][M]
  float2* d_bspec = nullptr;   // FD: beam spectra, [max_frames][D][kb_pad]
  float2* d_fdtw = nullptr;    // FD: twiddles for fd_L and P (layout: fd_tw_len)
  float2* d_big = nullptr;     // NF > 2^MB_LOGN2: matched-filter scratch, [max_frames][M][2 NF]
  float2* d_tw2 = nullptr;     // NF > 2^MB_LOGN2: twiddles of the 2^MB_LOGN2-point row transforms
  float2* d_fdstep = nullptr;  // FD: per-bin steering rotation exp(-2 pi i Dl / P), [D][M]
  float2* d_beam = nullptr;    // beam window [max_frames][D][G'] (unfused FD plans, IIR envelope), else a placeholder
  size_t beam_cap = 0;         // complex elements d_beam holds
  int* d_mt_g = nullptr;       // TD BF16: tap groups as their first sample's offset in the staging buffer, [tiles][GT][gmax]
  unsigned short* d_mt_w = nullptr;   // TD BF16: weight fragments, [tiles][GT][kcmax][hi, lo][64 lanes][8] BF16
  int2* d_mt_kcr = nullptr;    // TD BF16: K-chunk range per microphone group, [tiles][nmc][GT]
  int* d_mt_perm = nullptr;    // TD BF16: tile slot -> direction (-1: empty), [tiles][32]
  unsigned short* d_mt_fir = nullptr;   // TD BF16: low-pass B fragments, [K-steps][hi, lo][64 lanes][8] BF16
  void* d_aux = nullptr;       // plan-build scratch
  float* d_gdl = nullptr;      // gradients (TD): dL/dDl, [max_frames][D][M]
  float2* d_gscr = nullptr;    // gradients: phase transforms of G_yhat (TD) or G_b (FD), gscr_chans
                               // channels of P values at a time (at most GSCR_MAX_BYTES)
  long long gscr_chans = 0;
  float2* d_gband = nullptr;   // gradients (FD): beam-spectrum gradient G_B, [max_frames][D][kb]
  float2* d_gspec = nullptr;   // gradients (FD): conj(C) G_Y on [0, NF], [max_frames][M][NF + 1]
  float2* d_gy = nullptr;      // gradients: matched-filter gradient for sonar_energyscape_backward
                               // ([max_frames][M][P] TD, [max_frames][kb][M] FD)
  bool grad_on = false;
  int iir_ns = 0;              // IIR envelope: state dimension (2 per section); 0 = the FIR envelope
  int iir_chunk = 0;           // IIR envelope: window samples per lane (multiple of 16, 64 L >= G' + 15)
  float* d_iir = nullptr;      // IIR envelope tables (layout: IIR_TAB_LEN below)
  float* d_fbound = nullptr;   // TD_F16: per channel bound (1/P) sum_k |Yhat[k]| >= max |yhat|, [max_frames][M]
};

// 16-bit sample planes per microphone the matched filter appends for the MFMA
// time-domain beamformer: 4 BF16 (re hi, re lo, im hi, im lo) for TD_BF16, 2 (re, im)
// for TD_BF16X2 (BF16) and TD_F16 (FP16, scaled per frame), 0 for the other modes
inline int mt_planes(const sonar_plan_s* p) {
  return p->bf_mode == SONAR_BF_TD_BF16 ? 4
         : (p->bf_mode == SONAR_BF_TD_BF16X2 || p->bf_mode == SONAR_BF_TD_F16 || p->bf_mode == SONAR_BF_TD_BF16G ? 2 : 0);
}

inline bool mt_f16(const sonar_plan_s* p) { return p->bf_mode == SONAR_BF_TD_F16; }
// MFMA TD modes whose interpolation weights are exact in one 16-bit term (delays on a grid):
// TD_F16 (1/2048 sample, FP16) and TD_BF16G (1/256 sample, BF16); one product per sample plane
inline bool mt_w1(const sonar_plan_s* p) { return p->bf_mode == SONAR_BF_TD_F16 || p->bf_mode == SONAR_BF_TD_BF16G; }
inline int mt_grid_steps(const sonar_plan_s* p) {
  return p->bf_mode == SONAR_BF_TD_F16 ? 2048 : (p->bf_mode == SONAR_BF_TD_BF16G ? 256 : 0);
}
// TD_F16 frame header after the planes: complex64 elements (16 bytes, keeps frames 16-byte aligned);
// float 0 = 2^-e / M, the factor that takes the energyscape of the scaled FP16 samples back
constexpr int MF_F16_HEADER = 2;
// TD_F16 sample scale: 2^e with e = MF_F16_TOP - exponent of the frame's bound, |e| <= MF_F16_EMAX
constexpr int MF_F16_TOP = 14;
constexpr int MF_F16_EMAX = 100;
// complex64 offset of the TD_F16 frame header within a frame: after M rows and 2 M 16-bit rows
__host__ __device__ inline long long mf_f16_header(int M, int row) { return static_cast<long long>(M) * row * 3 / 2; }
#ifdef __HIPCC__
// TD_F16 sample exponent of frame f from its channels' bounds
__device__ inline int mf_f16_exponent(const float* fbound, long long f, int M) {
  float b = 0.f;
  for (int i = 0; i < M; ++i) b = fmaxf(b, fbound[f * M + i]);
  int ex = 0;
  (void)frexpf(b, &ex);   // b = mant 2^ex, mant in [0.5, 1) (ex = 0 for b = 0)
  const int e = MF_F16_TOP - ex;
  return e < -MF_F16_EMAX ? -MF_F16_EMAX : (e > MF_F16_EMAX ? MF_F16_EMAX : e);
}
// 16-bit plane words of a matched-filter value v: FP16 of sc v (sc != 0, TD_F16) or BF16 of v
__device__ __forceinline__ unsigned short mf_plane_word(float v, float sc) {
  return sc != 0.f ? __builtin_bit_cast(unsigned short, static_cast<_Float16>(v * sc))
                   : __builtin_bit_cast(unsigned short, static_cast<__bf16>(v));
}
#endif

// IIR envelope tables: A [ns][ns], B [ns], C [ns], D at offset 0 (packed for the
// section count in use), then A^(chunk 2^k), k < 6, [6][ns][ns] from IIR_POW_OFFSET
constexpr int IIR_MAX_SECTIONS = 4;
constexpr int IIR_POW_OFFSET = 96;
constexpr int IIR_TAB_LEN = IIR_POW_OFFSET + 6 * 64;

// PDM front end (k_pdm.hip): PDM_THREADS threads per workgroup, each workgroup makes
// NB outputs of every microphone of one frame
constexpr int PDM_THREADS = 256;
constexpr int PDM_MAX_MICS = 128;
constexpr int PDM_MAX_TAPS = 513;
constexpr size_t PDM_LDS_LIMIT = 150 * 1024;

// Matrix-core variant: 16-output x 16-microphone tiles on int8 MFMA (16x16x64), PDM_MT_THREADS
// threads per workgroup; used where the tile's tap operand (4 PDM_MT_KS_MAX KB at most) fits
constexpr int PDM_MT_THREADS = 512;
constexpr int PDM_MT_KS_MAX = 16;   // 64-tick K-steps per tile: 15 D + K <= 1024
constexpr size_t PDM_MT_LDS_PAIR = 80 * 1024;   // two workgroups per CU below this

struct sonar_pdm_s {
  int M = 0, N = 0, D = 1, K = 0, C = 0, W = 1, max_frames = 1, device = 0;
  int NB = 0, SW = 0;          // outputs per workgroup, staged words per microphone
  float* d_lut = nullptr;      // [C][256] byte tables of the reversed taps (C = 4 ceil(K/32), zero past K)
  float* d_gcum = nullptr;     // [K + 1] prefix sums of the reversed taps (windows at the recording's edges)
  // matrix-core variant (mt = true): taps as integers r = round(g 2^qshift), |r| < 2^29, split into
  // four signed base-256 digits
  bool mt = false;
  int KS = 0, qshift = 0, rows = 0;   // K-steps per tile, tap scale, staged microphone rows (16 ceil(M/16))
  unsigned* d_qtab = nullptr;   // [KS][4 digits][64 lanes][4 words]: the Toeplitz tap operand of a tile
  long long* d_rcum = nullptr;  // [K + 1] prefix sums of r
};

int pdm_span_words(int NB, int D, int K);
int pdm_tables(int K);
size_t pdm_lds_bytes(int M, int SW, int C);
int pdm_mt_ksteps(int D, int K);
int pdm_mt_span_words(int NB, int D, int KS);
size_t pdm_mt_lds_bytes(int rows, int SW, int KS);
hipError_t launch_pdm_tables(sonar_pdm_s* p, const double* d_taps64, hipStream_t s);
hipError_t init_pdm_kernel_attributes(const sonar_pdm_s* p, size_t lds);
hipError_t launch_pdm_demod(const sonar_pdm_s* p, const unsigned* words, int F, float* x, hipStream_t s);

// FFT twiddle table layout inside d_tw (all FP32 values built from FP64):
//   [0, nhi)              : exp(-2 pi i * 64 * t / NF)   t < nhi = max(NF/64, 1)
//   [nhi, nhi+64)         : exp(-2 pi i * t / NF)        t < 64
//   [nhi+64, +nhp)        : exp(-2 pi i * 64 * t / P)    t < nhp = NF/64 + 1
//   [.., +64)             : exp(-2 pi i * t / P)         t < 64
__host__ __device__ inline int fft_nhi(int NF) { return NF / 64 > 0 ? NF / 64 : 1; }
__host__ __device__ inline int fft_nhp(int NF) { return NF / 64 + 1; }
__host__ __device__ inline int fft_tw_len(int NF) { return fft_nhi(NF) + 64 + fft_nhp(NF) + 64; }

// FD twiddle layout inside d_fdtw:
//   [0, lh)            : exp(-2 pi i * 64 * t / L)   t < lh = max(L/64, 1)
//   [lh, lh+64)        : exp(-2 pi i * t / L)        t < 64
//   [lh+64, +P/64+1)   : exp(-2 pi i * 64 * t / P)   t <= P/64
//   [.., +64)          : exp(-2 pi i * t / P)        t < 64
__host__ __device__ inline int fd_tw_len(int L, int P) { return (L / 64 > 0 ? L / 64 : 1) + 64 + P / 64 + 1 + 64; }

// time-domain beamformer on BF16 MFMA: tiles of 32 directions x nwave * 128
// beam samples per workgroup; wavefront w computes the samples of residue
// w % GT (mod GT, the tap-group width below) in block w / GT; MT_MICS microphones staged at a time.
// Plans take 4-wave workgroups (two share a CU) and fall back to 8 waves when the
// staged window of a wide aperture does not fit the 4-wave staging budget.
constexpr int DELAY_MARGIN = 3;   // samples of delay range kept beyond the geometry's bound
constexpr int MT_NWAVE_SMALL = 4;
constexpr int MT_NWAVE_LARGE = 8;
// matched filters with NF > 2^MB_LOGN2 run as a radix-(NF / 2^MB_LOGN2) pass over
// global memory plus 2^MB_LOGN2-point transforms in LDS (k_mf_big.hip)
constexpr int MB_LOGN2 = 14;
constexpr int MB_MAX_R = 16;
// gradient transform scratch: at most this many bytes (the adjoint runs its channels in chunks)
constexpr long long GSCR_MAX_BYTES = 4LL << 30;
constexpr int MT_MICS = 8;      // microphones staged per group with four planes (16 with two)
// microphones staged per group: the staged bytes per group stay the same for both plane counts
inline int mt_mics(const sonar_plan_s* p) { return mt_planes(p) == 2 ? 2 * MT_MICS : MT_MICS; }
constexpr int MT_SPT = 10;   // 16-byte staging chunks per thread: planes x MT_MICS rows x wrow / 8 <= MT_SPT x threads
// Tap groups of the MFMA beamformer: GT consecutive taps of one microphone per group (one 2 GT-byte
// LDS read per output column), GT sample residues per block (a column reads its group where sample +
// first tap = 0 mod GT, so every read is aligned), 16 / GT groups per 16-row K-chunk.  Two sample
// planes take groups of 2 (fewer taps issued past each microphone's span: about 4.1x the two taps a
// direction needs instead of 5.0x with groups of 4 at 32 x 16384 x 1500); four planes keep groups of
// 4 in pairs (taps t, t + 4 read as 8 consecutive samples).
__host__ __device__ constexpr int mt_gt_of(int npl) { return npl == 2 ? 2 : 4; }
inline int mt_gt(const sonar_plan_s* p) { return mt_gt_of(mt_planes(p)); }
constexpr int MT_XCDS = 8;      // accelerator dies (each with its own L2) that workgroups are spread over
// |b| rows in LDS for the matrix-core low-pass (one 32-bit word per sample): nwave * 128
// samples + a zeroed tail, padded so that a row is 16 bytes past a multiple of 256 (bank spread)
__host__ __device__ constexpr int mt_nsp(int nwave) { return nwave * 128 + 4; }
constexpr int MT_FIR_TAIL = 64;   // zero words after the last |b| row
constexpr int MT_MULTI_MAX_ITEMS = 16;   // items of one persistent multi launch (descriptors travel as kernel arguments)

constexpr int FD_MAX_LOGL = 14;        // largest per-phase transform of the FD inverse (LDS): 16384 points
constexpr int FD_MAX_FOLD = 3;         // stored bins per slot held in registers by the fused FD inverse
constexpr int FD_FOLD1_MAX_L = 8192;   // the default layout keeps one bin per slot up to this transform length
constexpr int FD_GEMM_DIRS = 64;       // directions per FD GEMM workgroup (16 per wavefront)
constexpr int FD_GEMM_FRAMES = 16;     // frames per FD GEMM workgroup
constexpr int FD_XCDS = 8;             // accelerator dies the FD GEMM's sample tiles are grouped by
constexpr int FD_MAX_TAPS = 4096;       // low-pass taps of the fused FD inverse (LDS)
constexpr int FD_MAX_PHASES = 64;       // phases R' = P / L of the fused FD inverse (16 R' rotations in LDS)

hipError_t launch_build_tables(sonar_plan_s* p, hipStream_t s);
hipError_t init_mt_kernel_attributes();
hipError_t launch_mf_big_td(const sonar_plan_s* p, const void* x, int F, float2* yext, hipStream_t s, bool rows);
hipError_t launch_mf_big_fd(const sonar_plan_s* p, const void* x, int F, float2* band, hipStream_t s);
// out[ch][n] = Re IDFT_P(V[ch]) for n < N from one-sided spectra V[ch][0..NF] (chans <= max_frames * M)
hipError_t launch_big_inv_real(const sonar_plan_s* p, const float2* V, int chans, float* out, hipStream_t s);
size_t mt_smem_bytes(const sonar_plan_s* p);
hipError_t launch_das_mfma_env(const sonar_plan_s* p, const float2* yext, int F, float* E, hipStream_t s);
// persistent beamformer + envelope over n <= MT_MULTI_MAX_ITEMS items of compatible MFMA TD plans
bool mt_multi_compatible(const sonar_plan_s* a, const sonar_plan_s* b);
hipError_t launch_das_mfma_env_multi(const sonar_plan_s* const* plans, const float2* const* yext, const int* frames,
                                     float* const* E, int n, hipStream_t s);
hipError_t launch_build_fd_tables(sonar_plan_s* p, hipStream_t s);
hipError_t launch_mf_fd(const sonar_plan_s* p, const void* x, int F, float2* band, hipStream_t s);
hipError_t launch_fd_gemm(const sonar_plan_s* p, const float2* band, int F, float2* bspec, hipStream_t s);
size_t fd_envw_static_lds(int logL);
size_t fd_envw_dyn_lds(const sonar_plan_s* p);
size_t fd_env_dyn_lds(const sonar_plan_s* p);     // per-phase variant: 16 R' factors, classed taps, Q range-bin sums
hipError_t launch_fd_ifft_env(const sonar_plan_s* p, const float2* bspec, int F, float* E, hipStream_t s);
hipError_t launch_fd_ifft_beam(const sonar_plan_s* p, const float2* bspec, int F, float2* beam, hipStream_t s);
// rows = false skips the complex64 rows (MFMA modes whose beamformer reads only the 16-bit planes)
hipError_t launch_mf_td(const sonar_plan_s* p, const void* x, int F, float2* yext, hipStream_t s, bool rows = true);
hipError_t launch_mf_bound(const sonar_plan_s* p, int F, hipStream_t s);
hipError_t launch_delay_tables(sonar_plan_s* p, hipStream_t s);
hipError_t launch_fd_step_table(sonar_plan_s* p, hipStream_t s);
// energyscape cells (f, d, q) of an exact-phase plan and dL/dp for L = sum_c dE[c] E_c (scratch: d_gscr)
bool cells_supported(const sonar_plan_s* p);
hipError_t launch_energyscape_cells(const sonar_plan_s* p, const float2* mf, int F, const int* cells,
                                    const float* dE, int n, float* E_out, double* dpos, hipStream_t s);
hipError_t launch_energyscape_vjp(const sonar_plan_s* p, const float2* mf, float2* beam_grad, const float* dE, int F,
                                  float2* dyhat, float* dx, double* dpos, hipStream_t s);
hipError_t launch_das_td_env(const sonar_plan_s* p, const float2* yext, int F, float* E, hipStream_t s);
hipError_t launch_das_td_beam(const sonar_plan_s* p, const float2* yext, int F, float2* beam, hipStream_t s);
hipError_t launch_envelope(const sonar_plan_s* p, const float2* beam, int F, float* E, hipStream_t s);
hipError_t launch_iir_envelope(const sonar_plan_s* p, const float2* beam, int F, float* E, hipStream_t s);
hipError_t init_td_kernel_attributes();
