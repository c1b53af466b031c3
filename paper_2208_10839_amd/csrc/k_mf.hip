// Matched-filter kernels (§4.1 matched filter; §4.3 FFT-convolution filters
// with the group delay removed).
//
// Per channel (frame f, microphone m) one workgroup computes
//   Yhat[k] = X[k] C[k],  X = DFT_P(x zero-padded),  C = beta W conj(S),
// for k in [0, P/2] (C vanishes above P/2), and, for the time-domain
// beamformer, the analytic matched-filter output
//   yhat[n] = IDFT_P(Yhat)[n].
// The real input is packed as z[n] = x[2n] + i x[2n+1] into an NF = P/2 point
// complex FFT and split afterwards (X[k] = E[k] + exp(-2 pi i k/P) O[k]).
// Because Yhat vanishes above NF, the inverse splits by output parity:
//   yhat[2a + r] = (1/P) ( sum_{k<NF} Yhat[k] exp(2 pi i k r/P) exp(2 pi i k a/NF)
//                          + Yhat[NF] (-1)^r ),
// two NF-point inverse FFTs, one workgroup each, reading the spectrum that the
// forward kernel left in the plan's workspace (L2/MALL resident at these sizes).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include "fft_lds.hpp"
#include "plan.hpp"

using namespace fftk;

namespace {

template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<__half>(__half v) { return __half2float(v); }
template <>
__device__ __forceinline__ float to_f32<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }

// Loads the twiddle tables of the plan into LDS.
// round-to-nearest-even BF16 bits of a finite float
__device__ __forceinline__ unsigned short bf16_rne(float v) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(v));
}

template <int LOGNF>
__device__ __forceinline__ void load_tw(float2* tw, const float2* __restrict__ tw_g, int tid, int nthreads) {
  constexpr int NF = 1 << LOGNF;
  constexpr int NHI = NF / 64 > 0 ? NF / 64 : 1;
  constexpr int LEN = NHI + 64 + (NF / 64 + 1) + 64;
  for (int i = tid; i < LEN; i += nthreads) tw[i] = tw_g[i];
}

// Forward transform of one channel and the matched-filter product.  On return
// lds holds Yhat[k] (padded layout) for the band bins k in [k_lo, k_lo + kb), k < NF, and
// *nyq holds Yhat[NF]; C is zero at every other bin, whose entries are left unspecified.
template <int LOGNF, typename TIn>
__device__ __forceinline__ void forward_mf(const TIn* __restrict__ x, int N,
                                           const float2* __restrict__ cspec, float2* lds,
                                           const float2* tw, float2* nyq, int tid, int k_lo, int kb) {
  using S = FftShape<LOGNF>;
  constexpr int NF = S::NF;
  constexpr int T = S::T;
  constexpr int NHI = NF / 64 > 0 ? NF / 64 : 1;
  const float2* tw_hi = tw;
  const float2* tw_lo = tw + NHI;
  const float2* twp_hi = tw + NHI + 64;                 // exp(-2 pi i 64 t / P)
  const float2* twp_lo = tw + NHI + 64 + (NF / 64 + 1);   // exp(-2 pi i t / P)

  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int n = tid + r * (NF / 16);
    const int i0 = 2 * n;
    const float a = i0 < N ? to_f32<TIn>(x[i0]) : 0.0f;
    const float b = i0 + 1 < N ? to_f32<TIn>(x[i0 + 1]) : 0.0f;
    v[r] = make_float2(a, b);
  }
  fft_lds<LOGNF, false>(v, lds, tw_hi, tw_lo, tid);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) lds[padi(S::out_index(tid, i))] = v[i];
  __syncthreads();
  // split the packed transform into the real signal's spectrum and apply C, for the pairs
  // (k, NF - k) with a bin in the band (bin 0 pairs with the Nyquist bin NF)
  for (int k = tid; k <= NF / 2; k += T) {
    const bool in_k = static_cast<unsigned>(k - k_lo) < static_cast<unsigned>(kb);
    const bool in_m = static_cast<unsigned>(NF - k - k_lo) < static_cast<unsigned>(kb);
    if (!in_k && !in_m && k != 0) continue;
    const float2 A = lds[padi(k)];
    const float2 B = lds[padi((NF - k) & (NF - 1))];
    const float2 Ek = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));      // (A + conj B)/2
    const float2 Ok = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));     // (A - conj B)/(2i)
    const float2 wk = cmul(twp_hi[k >> 6], twp_lo[k & 63]);                     // exp(-2 pi i k / P)
    const float2 wo = cmul(wk, Ok);
    const float2 Xk = cadd(Ek, wo);
    const float2 Xm = cconj(csub(Ek, wo));                                      // X[NF - k]
    lds[padi(k)] = cmul(Xk, cspec[k]);
    if (k == 0) {
      *nyq = cmul(Xm, cspec[NF]);
    } else if (k != NF / 2) {
      lds[padi(NF - k)] = cmul(Xm, cspec[NF - k]);
    }
  }
  __syncthreads();
}

// Forward transform and matched-filter product of one channel per workgroup;
// writes the one-sided spectrum Yhat[k] for the band bins k in [k_lo, k_lo + kb) to
// spec[ch][k] (C, hence Yhat, is zero at every other bin of [0, NF], which the inverse
// takes as zero without reading) and, when bound is given (TD_F16), (1/P) sum_k |Yhat[k]|
// to bound[ch] (the sample-scale bound; the bins outside the band add zeros).
template <int LOGNF, typename TIn>
__global__ __launch_bounds__((1 << LOGNF) / 16) void mf_fwd_kernel(
    const TIn* __restrict__ x, int N, const float2* __restrict__ cspec,
    const float2* __restrict__ tw_g, float2* __restrict__ spec, float* __restrict__ bound, float inv_p,
    int k_lo, int kb) {
  using S = FftShape<LOGNF>;
  constexpr int NF = S::NF;
  constexpr int T = S::T;
  constexpr int NHI = NF / 64 > 0 ? NF / 64 : 1;
  constexpr int TWLEN = NHI + 64 + (NF / 64 + 1) + 64;
  __shared__ float2 lds[S::LDS_ELEMS];
  __shared__ float2 tw[TWLEN];
  __shared__ float2 nyq;
  const int tid = threadIdx.x;
  const long long ch = blockIdx.x;                       // f * M + m
  load_tw<LOGNF>(tw, tw_g, tid, T);
  __syncthreads();
  forward_mf<LOGNF, TIn>(x + ch * N, N, cspec, lds, tw, &nyq, tid, k_lo, kb);
  float2* out = spec + ch * (NF + 1);
  float acc = 0.f;
  // thread tid keeps bins k = tid mod T (its first one at or above k_lo), so each partial sum of
  // the bound adds the same nonzero terms in the same order as over every bin
  const int k_end = k_lo + kb;   // <= NF + 1
  int k0 = tid;
  if (k0 < k_lo) k0 += (k_lo - k0 + T - 1) / T * T;
  for (int k = k0; k < (k_end < NF ? k_end : NF); k += T) {
    const float2 v = lds[padi(k)];
    out[k] = v;
    acc += sqrtf(v.x * v.x + v.y * v.y);
  }
  if (tid == 0 && k_end > NF) {
    out[NF] = nyq;
    acc += sqrtf(nyq.x * nyq.x + nyq.y * nyq.y);
  }
  if (bound) {   // a kernel argument: the whole workgroup takes this branch
    __syncthreads();   // every read of the spectrum in LDS is done: reuse it for the sum
    float* red = reinterpret_cast<float*>(lds);
    red[tid] = acc;
    __syncthreads();
    for (int w = T / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) bound[ch] = red[0] * inv_p;
  }
}

// Forward transform and matched-filter product of one channel split over two workgroups by
// the parity s of the bin (NF = 2 H):
//   Z[2k' + s] = DFT_H(u_s)[k'],   u_s[n] = (z[n] + (-1)^s z[n + H]) exp(-2 pi i s n / NF),
// and the real split pairs bin k with NF - k, of the same parity, so each workgroup finishes its
// bins alone; two such workgroups share a CU.  Writes the band bins of Yhat (as mf_fwd_kernel
// does) straight from the split; no sample bound (TD_F16 keeps mf_fwd_kernel).
template <int LOGH, typename TIn>
__global__ __launch_bounds__((1 << LOGH) / 16) void mf_fwd2_kernel(
    const TIn* __restrict__ x, int N, const float2* __restrict__ cspec,
    const float2* __restrict__ tw_g, float2* __restrict__ spec, long long chans, int k_lo, int kb) {
  static_assert(LOGH >= 6, "H-point tables assume H >= 64");
  using S = FftShape<LOGH>;
  constexpr int H = S::NF;
  constexpr int NF = 2 * H;
  constexpr int T = S::T;
  constexpr int NHI_H = H / 64;            // H-point table, built here as the plan builds its own
  constexpr int NHI = NF / 64;             // plan table: NF-point entries, then the P-point ones
  constexpr int NHP = NF / 64 + 1;
  constexpr int TWLEN = NHI_H + 64 + NHI + 64 + NHP + 64;
  __shared__ float2 lds[S::LDS_ELEMS];
  __shared__ float2 tw[TWLEN];
  const int tid = threadIdx.x;
  // workgroups 16 j + 8 s + x are the two parities of channel 8 j + x: both on XCD x
  const unsigned bi = blockIdx.x;
  const int sp = (bi >> 3) & 1;
  const long long ch = static_cast<long long>(bi >> 4) * 8 + (bi & 7);
  if (ch >= chans) return;
  for (int i = tid; i < NHI_H + 64; i += T) {
    const double num = i < NHI_H ? 64.0 * i : static_cast<double>(i - NHI_H);
    double sn, cs;
    sincospi(-2.0 * num / H, &sn, &cs);
    tw[i] = make_float2(static_cast<float>(cs), static_cast<float>(sn));
  }
  for (int i = tid; i < NHI + 64 + NHP + 64; i += T) tw[NHI_H + 64 + i] = tw_g[i];
  __syncthreads();
  const float2* tw_hi = tw;                      // exp(-2 pi i 64 t / H)
  const float2* tw_lo = tw + NHI_H;              // exp(-2 pi i t / H)
  const float2* twn_hi = tw + NHI_H + 64;        // exp(-2 pi i 64 t / NF)
  const float2* twn_lo = twn_hi + NHI;           // exp(-2 pi i t / NF)
  const float2* twp_hi = twn_lo + 64;            // exp(-2 pi i 64 t / P)
  const float2* twp_lo = twp_hi + NHP;           // exp(-2 pi i t / P)
  const TIn* xc = x + ch * N;
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int n = tid + r * (H / 16);
    const int i0 = 2 * n, i1 = 2 * (n + H);
    const float2 a = make_float2(i0 < N ? to_f32<TIn>(xc[i0]) : 0.0f, i0 + 1 < N ? to_f32<TIn>(xc[i0 + 1]) : 0.0f);
    const float2 b = make_float2(i1 < N ? to_f32<TIn>(xc[i1]) : 0.0f, i1 + 1 < N ? to_f32<TIn>(xc[i1 + 1]) : 0.0f);
    v[r] = sp ? cmul(csub(a, b), cmul(twn_hi[n >> 6], twn_lo[n & 63])) : cadd(a, b);
  }
  fft_lds<LOGH, false>(v, lds, tw_hi, tw_lo, tid);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) lds[padi(S::out_index(tid, i))] = v[i];   // Z[2 k' + s] at k'
  __syncthreads();
  float2* out = spec + ch * (NF + 1);
  for (int kq = tid; 2 * kq + sp <= NF / 2; kq += T) {
    const int k = 2 * kq + sp;
    const bool in_k = static_cast<unsigned>(k - k_lo) < static_cast<unsigned>(kb);
    const bool in_m = static_cast<unsigned>(NF - k - k_lo) < static_cast<unsigned>(kb);
    if (!in_k && !in_m) continue;           // (bin 0 pairs with the Nyquist bin NF)
    const int km = (NF - k) & (NF - 1);     // same parity as k
    const float2 A = lds[padi(kq)];
    const float2 B = lds[padi((km - sp) >> 1)];
    const float2 Ek = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));      // (A + conj B)/2
    const float2 Ok = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));     // (A - conj B)/(2i)
    const float2 wk = cmul(twp_hi[k >> 6], twp_lo[k & 63]);                     // exp(-2 pi i k / P)
    const float2 wo = cmul(wk, Ok);
    const float2 Xk = cadd(Ek, wo);
    const float2 Xm = cconj(csub(Ek, wo));                                      // X[NF - k]
    if (in_k) out[k] = cmul(Xk, cspec[k]);
    if (in_m && k != NF / 2) out[NF - k] = cmul(Xm, cspec[NF - k]);
  }
}

// Inverse transform of one output parity of one channel per workgroup:
//   yhat[2a + par] = (1/P) (IDFT'_NF(Yhat[k] exp(2 pi i k par / P))[a] + Yhat[NF] (-1)^par)
// written to the MF rows: element j of a row holds yhat[(origin + j) mod P].
// PLANES (0, 2 or 4 16-bit planes after the complex rows) and F16 (FP16 planes of 2^e yhat
// instead of BF16) are compile-time, so each output format is its own kernel without the
// other formats' live registers (the one kernel for all formats spilled at NF = 16384).
template <int LOGNF, int PLANES, bool F16>
__global__ __launch_bounds__((1 << LOGNF) / 16) void mf_inv_kernel(
    const float2* __restrict__ spec, const float2* __restrict__ tw_g, float2* __restrict__ yext,
    long long fstride, int M, int row, int origin, int P, const float* __restrict__ fbound, int rows,
    long long chans, int k_lo, int kb) {
  static_assert(PLANES == 0 || PLANES == 2 || PLANES == 4, "no planes, two or four");
  static_assert(!F16 || PLANES == 2, "FP16 samples come as two planes");
  constexpr int planes = PLANES;
  using S = FftShape<LOGNF>;
  constexpr int NF = S::NF;
  constexpr int T = S::T;
  constexpr int NHI = NF / 64 > 0 ? NF / 64 : 1;
  constexpr int TWLEN = NHI + 64 + (NF / 64 + 1) + 64;
  __shared__ float2 lds[S::LDS_ELEMS];
  __shared__ float2 tw[TWLEN];
  const int tid = threadIdx.x;
  // workgroups 16 j + x and 16 j + 8 + x are the two parities of channel 8 j + x: both on XCD x
  // (workgroups go to the XCDs round-robin), so the second reads the spectrum from that L2
  const unsigned bi = blockIdx.x;
  const int par = (bi >> 3) & 1;
  const long long ch = static_cast<long long>(bi >> 4) * 8 + (bi & 7);
  if (ch >= chans) return;
  load_tw<LOGNF>(tw, tw_g, tid, T);
  __syncthreads();
  const float2* tw_hi = tw;
  const float2* tw_lo = tw + NHI;
  const float2* twp_hi = tw + NHI + 64;
  const float2* twp_lo = tw + NHI + 64 + (NF / 64 + 1);
  const float2* in = spec + ch * (NF + 1);
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k = tid + r * (NF / 16);
    // bins outside [k_lo, k_lo + kb) are zero (the forward kernel stores the band only)
    v[r] = static_cast<unsigned>(k - k_lo) < static_cast<unsigned>(kb) ? in[k] : make_float2(0.f, 0.f);
    if (par) v[r] = cmul(v[r], cconj(cmul(twp_hi[k >> 6], twp_lo[k & 63])));   // exp(+2 pi i k / P)
  }
  const float2 ny = k_lo + kb > NF ? in[NF] : make_float2(0.f, 0.f);
  fft_lds<LOGNF, true>(v, lds, tw_hi, tw_lo, tid);
  const float inv_p = 1.0f / static_cast<float>(P);
  const float sgn = par ? -1.0f : 1.0f;
  const long long f = ch / M;
  const int m = static_cast<int>(ch - f * M);
  float2* out = yext + f * fstride + static_cast<long long>(m) * row;
  // 16-bit planes of the same samples after the complex rows of the frame:
  // [M][4][row] (re hi, re lo, im hi, im lo) or [M][2][row] (re, im)
  unsigned short* pl = reinterpret_cast<unsigned short*>(yext + f * fstride + static_cast<long long>(M) * row) +
                       static_cast<long long>(m) * planes * row;
  // TD_F16: FP16 planes of 2^e yhat (e from the frame's channel bounds), 2^-e / M in the frame header
  float sc = 0.f;
  if constexpr (F16) {
    const int e = mf_f16_exponent(fbound, f, M);
    sc = ldexpf(1.0f, e);
    if (m == 0 && par == 0 && tid == 0)
      *reinterpret_cast<float*>(yext + f * fstride + mf_f16_header(M, row)) = ldexpf(1.0f / static_cast<float>(M), -e);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int n = 2 * S::out_index(tid, i) + par;
    const float2 y = make_float2((v[i].x + sgn * ny.x) * inv_p, (v[i].y + sgn * ny.y) * inv_p);
    unsigned short rh = 0, rl = 0, ih = 0, il = 0;
    if constexpr (planes != 0) {
      rh = mf_plane_word(y.x, F16 ? sc : 0.f);
      ih = mf_plane_word(y.y, F16 ? sc : 0.f);
      if constexpr (planes == 4) {
        rl = bf16_rne(y.x - __uint_as_float(static_cast<unsigned>(rh) << 16));
        il = bf16_rne(y.y - __uint_as_float(static_cast<unsigned>(ih) << 16));
      }
    }
    for (int j = (n - origin) & (P - 1); j < row; j += P) {
      if (rows) out[j] = y;
      if constexpr (planes == 4) {
        pl[j] = rh;
        pl[row + j] = rl;
        pl[2 * row + j] = ih;
        pl[3 * row + j] = il;
      } else if constexpr (planes == 2) {
        pl[j] = rh;
        pl[row + j] = ih;
      }
    }
  }
}

// Inverse transform of one output residue mod 4 of one channel per workgroup, with
// H = NF / 2 point transforms (P = 4 H):
//   yhat[4a + r] = (1/P) (IDFT'_H(V_r)[a] + Yhat[NF] (-1)^r),
//   V_r[k0] = sum_{q = 0, 1} Yhat[k0 + q H] exp(2 pi i (k0 + q H) r / P),   k0 < H,
// (exp(2 pi i k a / H) depends on k mod H only), so the four workgroups of a channel hold half
// the LDS of one NF-point transform each and two of them share a CU.  Output formats as in
// mf_inv_kernel; the H-point twiddle tables are built here the way the plan builds its own.
template <int LOGH, int PLANES, bool F16>
__global__ __launch_bounds__((1 << LOGH) / 16) void mf_inv4_kernel(
    const float2* __restrict__ spec, const float2* __restrict__ tw_g, float2* __restrict__ yext,
    long long fstride, int M, int row, int origin, int P, const float* __restrict__ fbound, int rows,
    long long chans, int k_lo, int kb) {
  static_assert(PLANES == 0 || PLANES == 2 || PLANES == 4, "no planes, two or four");
  static_assert(!F16 || PLANES == 2, "FP16 samples come as two planes");
  static_assert(LOGH >= 6, "H-point tables assume H >= 64");
  constexpr int planes = PLANES;
  using S = FftShape<LOGH>;
  constexpr int H = S::NF;
  constexpr int NF = 2 * H;
  constexpr int T = S::T;
  constexpr int NHI_H = H / 64;            // H-point table: exp(-2 pi i 64 t / H), exp(-2 pi i t / H)
  constexpr int NHI = NF / 64;             // plan table: NF-point entries, then the P-point ones
  constexpr int NHP = NF / 64 + 1;
  __shared__ float2 lds[S::LDS_ELEMS];
  __shared__ float2 tw[NHI_H + 64 + NHP + 64];
  const int tid = threadIdx.x;
  // workgroups 32 j + 8 r + x, r < 4, are the four residues of channel 8 j + x: all on XCD x
  // (workgroups go to the XCDs round-robin), so three of them read the spectrum from that L2
  const unsigned bi = blockIdx.x;
  const int par = (bi >> 3) & 3;
  const long long ch = static_cast<long long>(bi >> 5) * 8 + (bi & 7);
  if (ch >= chans) return;
  for (int i = tid; i < NHI_H + 64; i += T) {
    const double num = i < NHI_H ? 64.0 * i : static_cast<double>(i - NHI_H);
    double sn, cs;
    sincospi(-2.0 * num / H, &sn, &cs);
    tw[i] = make_float2(static_cast<float>(cs), static_cast<float>(sn));
  }
  for (int i = tid; i < NHP + 64; i += T) tw[NHI_H + 64 + i] = tw_g[NHI + 64 + i];
  __syncthreads();
  const float2* tw_hi = tw;
  const float2* tw_lo = tw + NHI_H;
  const float2* twp_hi = tw + NHI_H + 64;   // exp(-2 pi i 64 t / P), t <= NF / 64
  const float2* twp_lo = twp_hi + NHP;      // exp(-2 pi i t / P), t < 64
  const float2* in = spec + ch * (NF + 1);
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k0 = tid + r * (H / 16);
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = k0 + q * H;
      // bins outside [k_lo, k_lo + kb) are zero (the forward kernel stores the band only)
      if (static_cast<unsigned>(k - k_lo) < static_cast<unsigned>(kb)) {
        float2 y = in[k];
        if (par) {
          int e = k * par;                  // < 3 NF = 1.5 P
          if (e >= P) e -= P;
          const bool neg = e >= NF;         // exp(2 pi i e / P) = -exp(2 pi i (e - NF) / P)
          if (neg) e -= NF;
          float2 w = cconj(cmul(twp_hi[e >> 6], twp_lo[e & 63]));
          if (neg) w = make_float2(-w.x, -w.y);
          y = cmul(y, w);
        }
        acc = cadd(acc, y);
      }
    }
    v[r] = acc;
  }
  const float2 ny = k_lo + kb > NF ? in[NF] : make_float2(0.f, 0.f);
  fft_lds<LOGH, true>(v, lds, tw_hi, tw_lo, tid);
  const float inv_p = 1.0f / static_cast<float>(P);
  const float sgn = (par & 1) ? -1.0f : 1.0f;
  const long long f = ch / M;
  const int m = static_cast<int>(ch - f * M);
  float2* out = yext + f * fstride + static_cast<long long>(m) * row;
  unsigned short* pl = reinterpret_cast<unsigned short*>(yext + f * fstride + static_cast<long long>(M) * row) +
                       static_cast<long long>(m) * planes * row;
  float sc = 0.f;
  if constexpr (F16) {
    const int e = mf_f16_exponent(fbound, f, M);
    sc = ldexpf(1.0f, e);
    if (m == 0 && par == 0 && tid == 0)
      *reinterpret_cast<float*>(yext + f * fstride + mf_f16_header(M, row)) = ldexpf(1.0f / static_cast<float>(M), -e);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int n = 4 * S::out_index(tid, i) + par;
    const float2 y = make_float2((v[i].x + sgn * ny.x) * inv_p, (v[i].y + sgn * ny.y) * inv_p);
    unsigned short rh = 0, rl = 0, ih = 0, il = 0;
    if constexpr (planes != 0) {
      rh = mf_plane_word(y.x, F16 ? sc : 0.f);
      ih = mf_plane_word(y.y, F16 ? sc : 0.f);
      if constexpr (planes == 4) {
        rl = bf16_rne(y.x - __uint_as_float(static_cast<unsigned>(rh) << 16));
        il = bf16_rne(y.y - __uint_as_float(static_cast<unsigned>(ih) << 16));
      }
    }
    for (int j = (n - origin) & (P - 1); j < row; j += P) {
      if (rows) out[j] = y;
      if constexpr (planes == 4) {
        pl[j] = rh;
        pl[row + j] = rl;
        pl[2 * row + j] = ih;
        pl[3 * row + j] = il;
      } else if constexpr (planes == 2) {
        pl[j] = rh;
        pl[row + j] = ih;
      }
    }
  }
}

// Forward transform and matched-filter product of one channel per workgroup;
// writes the band bins [k_lo, k_lo + kb) bin-major: band[f][k'][m].
template <int LOGNF, typename TIn>
__global__ __launch_bounds__((1 << LOGNF) / 16) void mf_fwd_band_kernel(
    const TIn* __restrict__ x, int N, const float2* __restrict__ cspec,
    const float2* __restrict__ tw_g, float2* __restrict__ band, int M, int F, int k_lo, int kb) {
  using S = FftShape<LOGNF>;
  constexpr int NF = S::NF;
  constexpr int T = S::T;
  constexpr int NHI = NF / 64 > 0 ? NF / 64 : 1;
  constexpr int TWLEN = NHI + 64 + (NF / 64 + 1) + 64;
  __shared__ float2 lds[S::LDS_ELEMS];
  __shared__ float2 tw[TWLEN];
  __shared__ float2 nyq;
  const int tid = threadIdx.x;
  // The M channels of a frame interleave in every stored bin row (8 M bytes), so all of them
  // run on one XCD (workgroups go to the XCDs round-robin by index): workgroup 8 j + xc
  // takes microphone j mod M of frame xc + 8 (j / M), and that L2 merges the rows before HBM.
  const unsigned bi = blockIdx.x;
  const long long jb = bi / MT_XCDS;
  const int m = static_cast<int>(jb % M);
  const long long f = static_cast<long long>(bi % MT_XCDS) + MT_XCDS * (jb / M);
  if (f >= F) return;
  const long long ch = f * M + m;
  load_tw<LOGNF>(tw, tw_g, tid, T);
  __syncthreads();
  forward_mf<LOGNF, TIn>(x + ch * N, N, cspec, lds, tw, &nyq, tid, k_lo, kb);
  float2* out = band + f * kb * M + m;
  for (int j = tid; j < kb; j += T) {
    const int k = k_lo + j;
    out[static_cast<long long>(j) * M] = k < NF ? lds[padi(k)] : nyq;
  }
}

template <int LOGNF, typename TIn>
hipError_t launch_mf_band_t(const sonar_plan_s* p, const void* x, int F, float2* band, hipStream_t s) {
  constexpr int T = (1 << LOGNF) / 16;
  const unsigned blocks = static_cast<unsigned>(MT_XCDS * p->M * ((F + MT_XCDS - 1) / MT_XCDS));
  hipLaunchKernelGGL((mf_fwd_band_kernel<LOGNF, TIn>), dim3(blocks), dim3(T), 0, s,
                     static_cast<const TIn*>(x), p->N, p->d_cspec, p->d_tw, band, p->M, F, p->k_lo, p->kb);
  return hipGetLastError();
}

template <typename TIn>
hipError_t launch_mf_band_dt(const sonar_plan_s* p, const void* x, int F, float2* band, hipStream_t s) {
  switch (p->logNF) {
    case 4: return launch_mf_band_t<4, TIn>(p, x, F, band, s);
    case 5: return launch_mf_band_t<5, TIn>(p, x, F, band, s);
    case 6: return launch_mf_band_t<6, TIn>(p, x, F, band, s);
    case 7: return launch_mf_band_t<7, TIn>(p, x, F, band, s);
    case 8: return launch_mf_band_t<8, TIn>(p, x, F, band, s);
    case 9: return launch_mf_band_t<9, TIn>(p, x, F, band, s);
    case 10: return launch_mf_band_t<10, TIn>(p, x, F, band, s);
    case 11: return launch_mf_band_t<11, TIn>(p, x, F, band, s);
    case 12: return launch_mf_band_t<12, TIn>(p, x, F, band, s);
    case 13: return launch_mf_band_t<13, TIn>(p, x, F, band, s);
    case 14: return launch_mf_band_t<14, TIn>(p, x, F, band, s);
    default: return hipErrorInvalidValue;
  }
}

template <int LOGNF, typename TIn>
hipError_t launch_mf_td_t(const sonar_plan_s* p, const void* x, int F, float2* yext, hipStream_t s, bool rows) {
  constexpr int T = (1 << LOGNF) / 16;
  bool split = false;
  if constexpr (LOGNF == 14) {
    if (!mt_f16(p)) {   // two parities of 8192-point transforms per channel (two workgroups per CU)
      const long long ch2 = static_cast<long long>(F) * p->M;
      hipLaunchKernelGGL((mf_fwd2_kernel<LOGNF - 1, TIn>), dim3(static_cast<unsigned>((ch2 + 7) / 8 * 16)),
                         dim3(T / 2), 0, s, static_cast<const TIn*>(x), p->N, p->d_cspec, p->d_tw, p->d_spec, ch2,
                         p->k_lo, p->kb);
      split = true;
    }
  }
  if (!split)
    hipLaunchKernelGGL((mf_fwd_kernel<LOGNF, TIn>), dim3(F * p->M), dim3(T), 0, s,
                       static_cast<const TIn*>(x), p->N, p->d_cspec, p->d_tw, p->d_spec,
                       mt_f16(p) ? p->d_fbound : nullptr, 1.0f / static_cast<float>(p->P), p->k_lo, p->kb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long chans = static_cast<long long>(F) * p->M;
  const int org = static_cast<int>(p->origin), rw = rows ? 1 : 0;
  const int planes = mt_planes(p);
  if constexpr (LOGNF == 14) {
    // NF = 16384: four residues mod 4 per channel with 8192-point transforms (two workgroups per
    // CU, twice the workgroups of the two-parity split for small batches)
    constexpr int T4 = (1 << (LOGNF - 1)) / 16;
    const dim3 grid4(static_cast<unsigned>((chans + 7) / 8 * 32));
    if (mt_f16(p)) {
      if (planes != 2) return hipErrorInvalidValue;
      hipLaunchKernelGGL((mf_inv4_kernel<LOGNF - 1, 2, true>), grid4, dim3(T4), 0, s, p->d_spec, p->d_tw, yext,
                         p->mf_fstride, p->M, p->row, org, p->P, p->d_fbound, rw, chans, p->k_lo, p->kb);
    } else if (planes == 4) {
      hipLaunchKernelGGL((mf_inv4_kernel<LOGNF - 1, 4, false>), grid4, dim3(T4), 0, s, p->d_spec, p->d_tw, yext,
                         p->mf_fstride, p->M, p->row, org, p->P, nullptr, rw, chans, p->k_lo, p->kb);
    } else if (planes == 2) {
      hipLaunchKernelGGL((mf_inv4_kernel<LOGNF - 1, 2, false>), grid4, dim3(T4), 0, s, p->d_spec, p->d_tw, yext,
                         p->mf_fstride, p->M, p->row, org, p->P, nullptr, rw, chans, p->k_lo, p->kb);
    } else if (planes == 0) {
      hipLaunchKernelGGL((mf_inv4_kernel<LOGNF - 1, 0, false>), grid4, dim3(T4), 0, s, p->d_spec, p->d_tw, yext,
                         p->mf_fstride, p->M, p->row, org, p->P, nullptr, rw, chans, p->k_lo, p->kb);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const dim3 grid(static_cast<unsigned>((chans + 7) / 8 * 16));
  if (mt_f16(p)) {
    if (planes != 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL((mf_inv_kernel<LOGNF, 2, true>), grid, dim3(T), 0, s, p->d_spec, p->d_tw, yext,
                       p->mf_fstride, p->M, p->row, org, p->P, p->d_fbound, rw, chans, p->k_lo, p->kb);
  } else if (planes == 4) {
    hipLaunchKernelGGL((mf_inv_kernel<LOGNF, 4, false>), grid, dim3(T), 0, s, p->d_spec, p->d_tw, yext,
                       p->mf_fstride, p->M, p->row, org, p->P, nullptr, rw, chans, p->k_lo, p->kb);
  } else if (planes == 2) {
    hipLaunchKernelGGL((mf_inv_kernel<LOGNF, 2, false>), grid, dim3(T), 0, s, p->d_spec, p->d_tw, yext,
                       p->mf_fstride, p->M, p->row, org, p->P, nullptr, rw, chans, p->k_lo, p->kb);
  } else if (planes == 0) {
    hipLaunchKernelGGL((mf_inv_kernel<LOGNF, 0, false>), grid, dim3(T), 0, s, p->d_spec, p->d_tw, yext,
                       p->mf_fstride, p->M, p->row, org, p->P, nullptr, rw, chans, p->k_lo, p->kb);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TIn>
hipError_t launch_mf_td_dt(const sonar_plan_s* p, const void* x, int F, float2* yext, hipStream_t s, bool rows) {
  switch (p->logNF) {
    case 4: return launch_mf_td_t<4, TIn>(p, x, F, yext, s, rows);
    case 5: return launch_mf_td_t<5, TIn>(p, x, F, yext, s, rows);
    case 6: return launch_mf_td_t<6, TIn>(p, x, F, yext, s, rows);
    case 7: return launch_mf_td_t<7, TIn>(p, x, F, yext, s, rows);
    case 8: return launch_mf_td_t<8, TIn>(p, x, F, yext, s, rows);
    case 9: return launch_mf_td_t<9, TIn>(p, x, F, yext, s, rows);
    case 10: return launch_mf_td_t<10, TIn>(p, x, F, yext, s, rows);
    case 11: return launch_mf_td_t<11, TIn>(p, x, F, yext, s, rows);
    case 12: return launch_mf_td_t<12, TIn>(p, x, F, yext, s, rows);
    case 13: return launch_mf_td_t<13, TIn>(p, x, F, yext, s, rows);
    case 14: return launch_mf_td_t<14, TIn>(p, x, F, yext, s, rows);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

namespace {

// (1/P) sum_{k <= NF} |Yhat[k]| per channel: the inverse transform sums NF + 1 terms of these
// magnitudes (times unit phases) over P, so this bounds |yhat[n]| for every n
__global__ __launch_bounds__(256) void mf_bound_kernel(const float2* __restrict__ spec, int NF, float inv_p,
                                                       float* __restrict__ bound) {
  __shared__ float part[4];
  const long long ch = blockIdx.x;
  const float2* sp = spec + ch * (NF + 1);
  float acc = 0.f;
  for (int k = threadIdx.x; k <= NF; k += 256) {
    const float2 v = sp[k];
    acc += sqrtf(v.x * v.x + v.y * v.y);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) bound[ch] = ((part[0] + part[1]) + (part[2] + part[3])) * inv_p;
}

}  // namespace

hipError_t launch_mf_bound(const sonar_plan_s* p, int F, hipStream_t s) {
  hipLaunchKernelGGL(mf_bound_kernel, dim3(static_cast<unsigned>(F) * p->M), dim3(256), 0, s, p->d_spec, p->NF,
                     1.0f / static_cast<float>(p->P), p->d_fbound);
  return hipGetLastError();
}

hipError_t launch_mf_td(const sonar_plan_s* p, const void* x, int F, float2* yext, hipStream_t s, bool rows) {
  if (p->NF > (1 << MB_LOGN2)) return launch_mf_big_td(p, x, F, yext, s, rows);
  switch (p->dtype) {
    case SONAR_F32: return launch_mf_td_dt<float>(p, x, F, yext, s, rows);
    case SONAR_F16: return launch_mf_td_dt<__half>(p, x, F, yext, s, rows);
    case SONAR_BF16: return launch_mf_td_dt<__hip_bfloat16>(p, x, F, yext, s, rows);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mf_fd(const sonar_plan_s* p, const void* x, int F, float2* band, hipStream_t s) {
  if (p->NF > (1 << MB_LOGN2)) return launch_mf_big_fd(p, x, F, band, s);
  switch (p->dtype) {
    case SONAR_F32: return launch_mf_band_dt<float>(p, x, F, band, s);
    case SONAR_F16: return launch_mf_band_dt<__half>(p, x, F, band, s);
    case SONAR_BF16: return launch_mf_band_dt<__hip_bfloat16>(p, x, F, band, s);
    default: return hipErrorInvalidValue;
  }
}
