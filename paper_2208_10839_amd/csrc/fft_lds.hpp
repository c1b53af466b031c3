// Radix-16 Stockham FFT held in one workgroup's LDS (device code).
//
// The matched filter of the pipeline is an FFT filter (§4.3 replaces SciPy's
// lfilter by FFT convolution on the GPU).  This header provides the transform
// used by the matched-filter kernels: a complex FFT of NF = 2^LOGNF points
// (16 <= NF <= 16384) computed by NF/16 threads that each hold 16 points in
// registers.  Passes are radix 16, with one final radix-2/4/8 pass when LOGNF
// is not a multiple of 4.  Between passes the data goes through LDS in place
// (every thread reads its inputs, barrier, every thread writes its outputs),
// with one pad slot after every 16 points so that the stride-16 stores of the
// early passes spread over the banks.  Twiddles come from two small FP32
// tables built in FP64 (exp(-2 pi i 64 t / NF) and exp(-2 pi i t / NF)), so
// each twiddle is one complex product of two correctly rounded values.
//
// Data layout contract:
//  * input : thread t holds x[t + r NF/16] in v[r], r < 16;
//  * output: thread t holds X[j + r NF/LASTR] in v[b LASTR + r] with
//            j = t + b NF/16 (b < 16/LASTR), LASTR the radix of the last pass.
#pragma once

#include <hip/hip_runtime.h>

namespace fftk {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// a * (-i) for the forward transform, a * (+i) for the inverse.
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// exp(-+ 2 pi i e / 16) for a compile-time e (sign: - forward, + inverse).
template <bool INV>
__device__ __forceinline__ float2 w16(int e) {
  const float c4[5] = {1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f, 0.0f};
  e &= 15;
  const int q = e >> 2, r = e & 3;
  float c = c4[r], s = c4[4 - r];   // cos, sin of r*pi/8
  float cc, ss;                     // rotate by q quarter turns
  if (q == 0) { cc = c; ss = s; }
  else if (q == 1) { cc = -s; ss = c; }
  else if (q == 2) { cc = -c; ss = -s; }
  else { cc = s; ss = -c; }
  return INV ? make_float2(cc, ss) : make_float2(cc, -ss);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
  const float2 t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// 8-point DFT in place (natural order in and out): 8 = 4 x 2 split.
template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
#pragma unroll
  for (int n2 = 0; n2 < 2; ++n2) dft4<INV>(v[n2], v[n2 + 2], v[n2 + 4], v[n2 + 6]);
#pragma unroll
  for (int k1 = 1; k1 < 4; ++k1) v[1 + 2 * k1] = cmul(v[1 + 2 * k1], w16<INV>(2 * k1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft2<INV>(v[2 * k1], v[2 * k1 + 1]);
  float2 t[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) t[k1 + 4 * k2] = v[2 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = t[i];
}

// 16-point DFT in place (natural order in and out): 16 = 4 x 4 split.
template <bool INV>
__device__ __forceinline__ void dft16(float2* v) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) v[n2 + 4 * k1] = cmul(v[n2 + 4 * k1], w16<INV>(n2 * k1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  float2 t[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = t[i];
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 16) dft16<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 2) dft2<INV>(v[0], v[1]);
}

__device__ __forceinline__ int padi(int i) { return i + (i >> 4); }

// exp(-+ 2 pi i e / NF) from the two-level table in LDS (hi: 64-step, lo: unit step).
template <bool INV>
__device__ __forceinline__ float2 twiddle(const float2* tw_hi, const float2* tw_lo, int e) {
  const float2 w = cmul(tw_hi[e >> 6], tw_lo[e & 63]);
  return INV ? cconj(w) : w;
}

template <int LOGNF>
struct FftShape {
  static constexpr int NF = 1 << LOGNF;
  static constexpr int T = NF / 16;                       // threads
  static constexpr int N16 = LOGNF / 4;                   // radix-16 passes
  static constexpr int RL = 1 << (LOGNF % 4);             // last radix if < 16 (1: none)
  static constexpr int LASTR = RL > 1 ? RL : 16;
  static constexpr int LDS_ELEMS = NF + NF / 16;          // padded data
  static_assert(LOGNF >= 4 && LOGNF <= 14, "FFT size out of range");
  // index of the output held in v[i] by thread t
  __device__ static __forceinline__ int out_index(int t, int i) {
    return t + (i / LASTR) * T + (i % LASTR) * (NF / LASTR);
  }
};

// Full transform.  v holds the input in the contract layout and receives the
// output; lds must hold LDS_ELEMS float2 and is clobbered.  Starts with a
// barrier, so the caller may still be reading lds when it calls this.
// With TW1 (NF >= 256), the twiddles of the second pass (Ns = 16), which
// depend only on k = tid mod 16 and r, are read from tw1[16 r + k] (the same
// products, precomputed by the caller, see pass1_twiddles) instead of being
// rebuilt from the two-level table; k runs fastest, so the 16 values of k a
// wavefront reads lie in consecutive banks.
// With TWR, the twiddles of the third radix-16 pass (Ns = 256) and of the final
// radix-2/4/8 pass, which depend only on the thread, come from twr (filled by
// fft_thread_twiddles, e.g. once for many transforms and kept in registers).
template <int LOGNF>
struct FftTwr {
  using S = FftShape<LOGNF>;
  static constexpr int N_P2 = S::N16 >= 3 ? 15 : 0;
  static constexpr int N_LAST = S::RL > 1 ? (16 / S::RL) * (S::RL - 1) : 0;
  static constexpr int N = N_P2 + N_LAST > 0 ? N_P2 + N_LAST : 1;
};

template <int LOGNF, bool INV, bool TW1 = false, bool TWR = false>
__device__ __forceinline__ void fft_lds(float2 (&v)[16], float2* lds, const float2* tw_hi,
                                        const float2* tw_lo, int tid, const float2* tw1 = nullptr,
                                        const float2* twr = nullptr) {
  using S = FftShape<LOGNF>;
  constexpr int NF = S::NF;
  constexpr int T = S::T;
  dft16<INV>(v);                                  // first pass: radix 16, Ns = 1, no twiddles
  if constexpr (S::N16 == 1 && S::RL == 1) {
    return;
  } else {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[padi(16 * tid + r)] = v[r];
    __syncthreads();
    int Ns = 16;
#pragma unroll
    for (int p = 1; p < S::N16; ++p) {
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = lds[padi(tid + r * (NF / 16))];
      const int k = tid & (Ns - 1);
      const int estep = k * (NF / (Ns * 16));
      if (TW1 && p == 1) {
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], tw1[16 * r + k]);
      } else if (TWR && p == 2) {
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twr[r - 1]);
      } else {
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twiddle<INV>(tw_hi, tw_lo, estep * r));
      }
      dft16<INV>(v);
      if (S::RL == 1 && p == S::N16 - 1) return;   // last pass: outputs stay in registers
      __syncthreads();
      const int idxd = (tid - k) * 16 + k;
#pragma unroll
      for (int r = 0; r < 16; ++r) lds[padi(idxd + r * Ns)] = v[r];
      __syncthreads();
      Ns *= 16;
    }
    if constexpr (S::RL > 1) {
      constexpr int R = S::RL;
#pragma unroll
      for (int b = 0; b < 16 / R; ++b) {
        const int j = tid + b * T;
#pragma unroll
        for (int r = 0; r < R; ++r) v[b * R + r] = lds[padi(j + r * (NF / R))];
      }
#pragma unroll
      for (int b = 0; b < 16 / R; ++b) {
        const int j = tid + b * T;                // Ns * R == NF, so k == j
#pragma unroll
        for (int r = 1; r < R; ++r) {
          if constexpr (TWR)
            v[b * R + r] = cmul(v[b * R + r], twr[FftTwr<LOGNF>::N_P2 + b * (R - 1) + r - 1]);
          else
            v[b * R + r] = cmul(v[b * R + r], twiddle<INV>(tw_hi, tw_lo, j * r));
        }
        dftR<R, INV>(&v[b * R]);
      }
    }
  }
}

// The table fft_lds<LOGNF, INV, true> reads: entry 16 r + k is the twiddle of
// pass 1 (Ns = 16) for k = tid mod 16 and r, exactly as that pass would build
// it from the two-level table (tw_hi, tw_lo may be the global copies).
template <int LOGNF, bool INV>
__device__ __forceinline__ void pass1_twiddles(float2* tw1, const float2* tw_hi, const float2* tw_lo, int tid,
                                               int nthreads) {
  constexpr int NF = 1 << LOGNF;
  static_assert(NF >= 256, "pass 1 exists for NF >= 256");
  for (int i = tid; i < 256; i += nthreads) tw1[i] = twiddle<INV>(tw_hi, tw_lo, (i & 15) * (NF / 256) * (i >> 4));
}

// The per-thread twiddles fft_lds<LOGNF, INV, TW1, true> reads, exactly as the
// passes would build them.
template <int LOGNF, bool INV>
__device__ __forceinline__ void fft_thread_twiddles(float2 (&twr)[FftTwr<LOGNF>::N], const float2* tw_hi,
                                                    const float2* tw_lo, int tid) {
  using S = FftShape<LOGNF>;
  constexpr int NF = S::NF;
  if constexpr (S::N16 >= 3) {
    const int estep = (tid & 255) * (NF / 4096);
#pragma unroll
    for (int r = 1; r < 16; ++r) twr[r - 1] = twiddle<INV>(tw_hi, tw_lo, estep * r);
  }
  if constexpr (S::RL > 1) {
    constexpr int R = S::RL;
#pragma unroll
    for (int b = 0; b < 16 / R; ++b)
#pragma unroll
      for (int r = 1; r < R; ++r)
        twr[FftTwr<LOGNF>::N_P2 + b * (R - 1) + r - 1] = twiddle<INV>(tw_hi, tw_lo, (tid + b * S::T) * r);
  }
}

}  // namespace fftk
