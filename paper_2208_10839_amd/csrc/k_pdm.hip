// PDM front end (§2: 1-bit sigma-delta pulse-density modulated microphones;
// §4.3: the binary data are unpacked, demodulated by a low-pass filter and
// subsampled on the GPU before the matched filter):
//
//   x[m][n] = sum_{j<K} h[j] s_m[n D + (K-1)/2 - j],   s_m[t] = +1 / -1 for a set / clear bit,
//                                                      0 outside the T = N D recorded ticks,
//
// ticks packed W = ceil(M/32) 32-bit words per tick, microphone m in bit m % 32 of
// word m / 32.
//
// One workgroup makes PDM_NB consecutive outputs of every microphone of one frame:
//  1. transpose: each wavefront takes 64 consecutive ticks (one per lane) and turns
//     them into one 64-bit mask per microphone with a wave ballot, so LDS holds each
//     microphone's bits as a time-ordered bit string;
//  2. filter: with the taps reversed (g[i] = h[K-1-i], i = tick - first tick of the
//     window), the sum over K taps is a sum over ceil(K/8) byte lookups: table c maps
//     the 8 bits of ticks 8c..8c+7 of the window to sum_i g[8c+i] (+-1).  A lane aligns
//     its window with v_alignbit on pairs of LDS words and adds one table entry per
//     byte (the tables are built once per filter, in FP64, rounded to FP32);
//  3. windows that reach outside [0, T) take the tap-by-tap sum with bounds checks.
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace {

// lut[c][b] = sum_{i<8, 8c+i<K} g[8c+i] (bit i of b ? 1 : -1), g[i] = h[K-1-i]
__global__ void pdm_lut_kernel(const double* __restrict__ taps, int K, int C, float* __restrict__ lut) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= C * 256) return;
  const int c = e >> 8, b = e & 255;
  double s = 0.0;
  for (int i = 0; i < 8; ++i) {
    const int k = 8 * c + i;
    if (k >= K) break;
    const double g = taps[K - 1 - k];
    s += ((b >> i) & 1) ? g : -g;
  }
  lut[e] = static_cast<float>(s);
}

__global__ void pdm_taps_f32_kernel(const double* __restrict__ taps, int K, float* __restrict__ rev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) rev[i] = static_cast<float>(taps[K - 1 - i]);
}

__global__ __launch_bounds__(PDM_THREADS) void pdm_demod_kernel(
    const unsigned* __restrict__ words, const float* __restrict__ lut_g, const float* __restrict__ grev,
    float* __restrict__ x, int M, int W, int N, int D, int K, int C, int NB, int SW, int ntile) {
  extern __shared__ unsigned smem[];
  unsigned* bits = smem;                                  // [M][SW]
  float* lut = reinterpret_cast<float*>(smem + M * SW);   // [C][256]
  const int tile = blockIdx.x % ntile;
  const long long f = blockIdx.x / ntile;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long T = static_cast<long long>(N) * D;
  const int hk = (K - 1) >> 1;
  const int n0 = tile * NB;
  const long long t_lo = static_cast<long long>(n0) * D - hk;
  const long long tb = t_lo >= 0 ? (t_lo & ~31LL) : -((-t_lo + 31) & ~31LL);   // floor to a multiple of 32
  const unsigned* wf = words + f * T * W;

  for (int i = threadIdx.x; i < C * 256; i += PDM_THREADS) lut[i] = lut_g[i];

  // 1. bit transpose: 64-tick chunks, wave-strided
  const int nchunk = SW >> 1;
  for (int ch = wv; ch < nchunk; ch += PDM_THREADS / 64) {
    const long long t = tb + 64LL * ch + lane;
    const bool in = t >= 0 && t < T;
    unsigned long long keep0 = 0, keep1 = 0;
    for (int w = 0; w < W; ++w) {
      const unsigned word = in ? wf[t * W + w] : 0u;
      const int mend = M - 32 * w < 32 ? M - 32 * w : 32;
      for (int b = 0; b < mend; ++b) {
        const unsigned long long mask = __ballot((word >> b) & 1u);
        const int m = 32 * w + b;
        if (lane == (m & 63)) {
          if (m < 64) keep0 = mask;
          else keep1 = mask;
        }
      }
    }
    if (lane < M) {
      bits[lane * SW + 2 * ch] = static_cast<unsigned>(keep0);
      bits[lane * SW + 2 * ch + 1] = static_cast<unsigned>(keep0 >> 32);
    }
    if (lane + 64 < M) {
      bits[(lane + 64) * SW + 2 * ch] = static_cast<unsigned>(keep1);
      bits[(lane + 64) * SW + 2 * ch + 1] = static_cast<unsigned>(keep1 >> 32);
    }
  }
  __syncthreads();

  // 2./3. filter and subsample: wave w takes microphones w, w+4, ...; lanes take samples
  const int nw = (K + 31) >> 5;   // aligned words covering the window
  float* xf = x + f * static_cast<long long>(M) * N;
  for (int m = wv; m < M; m += PDM_THREADS / 64) {
    const unsigned* bm = bits + m * SW;
    for (int nb = lane; nb < NB; nb += 64) {
      const int n = n0 + nb;
      if (n >= N) break;
      const long long ts = static_cast<long long>(n) * D - hk;   // first tick of the window
      const int a = static_cast<int>(ts - tb);                   // its bit offset in the staged string
      float acc = 0.f;
      if (ts >= 0 && ts + K <= T) {
        const int w0 = a >> 5, sh = a & 31;
        for (int k = 0; k < nw; ++k) {
          const unsigned al = __builtin_amdgcn_alignbit(bm[w0 + k + 1], bm[w0 + k], sh);
          const int c0 = 4 * k;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            if (c0 + cc < C) acc += lut[(c0 + cc) * 256 + ((al >> (8 * cc)) & 255u)];
          }
        }
      } else {
        for (int i = 0; i < K; ++i) {
          const long long t = ts + i;
          if (t < 0 || t >= T) continue;
          const int p = a + i;
          const float g = grev[i];
          acc += ((bm[p >> 5] >> (p & 31)) & 1u) ? g : -g;
        }
      }
      xf[static_cast<long long>(m) * N + n] = acc;
    }
  }
}

}  // namespace

// staged 32-bit words per microphone for NB outputs (window of the last output plus the
// alignment slack and the word read past the end by the funnel shift), rounded to 64 ticks
int pdm_span_words(int NB, int D, int K) {
  const long long ticks = static_cast<long long>(NB - 1) * D + K + 31;
  const long long words = (ticks + 31) / 32 + 1;
  return static_cast<int>((words + 1) & ~1LL);
}

size_t pdm_lds_bytes(int M, int SW, int C) {
  return (static_cast<size_t>(M) * SW + static_cast<size_t>(C) * 256) * 4;
}

hipError_t launch_pdm_tables(sonar_pdm_s* p, const double* d_taps64, hipStream_t s) {
  const int n = p->C * 256;
  hipLaunchKernelGGL(pdm_lut_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_taps64, p->K, p->C, p->d_lut);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pdm_taps_f32_kernel, dim3((p->K + 255) / 256), dim3(256), 0, s, d_taps64, p->K, p->d_grev);
  return hipGetLastError();
}

hipError_t init_pdm_kernel_attributes(size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(pdm_demod_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
}

hipError_t launch_pdm_demod(const sonar_pdm_s* p, const unsigned* words, int F, float* x, hipStream_t s) {
  const int ntile = (p->N + p->NB - 1) / p->NB;
  const size_t lds = pdm_lds_bytes(p->M, p->SW, p->C);
  hipLaunchKernelGGL(pdm_demod_kernel, dim3(static_cast<unsigned>(F) * ntile), dim3(PDM_THREADS), lds, s, words,
                     p->d_lut, p->d_grev, x, p->M, p->W, p->N, p->D, p->K, p->C, p->NB, p->SW, ntile);
  return hipGetLastError();
}
