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
//     the 8 bits of ticks 8c..8c+7 of the window to sum_i g[8c+i] (+-1).  A lane loads
//     the NW + 1 words under its window, aligns them with v_alignbit and issues all
//     4 NW table reads at once into four partial sums (tables past the filter's end
//     are zero); the tables are built once per filter, in FP64, rounded to FP32;
//  3. ticks outside [0, T) are staged as clear bits, so the tables count them as -1;
//     a window that reaches outside adds back g over its outside prefix and suffix
//     (prefix sums of g, built in FP64 with the tables).
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

// gcum[i] = sum_{j<i} g[j], i <= K (one thread: K is at most a few hundred)
__global__ void pdm_prefix_kernel(const double* __restrict__ taps, int K, float* __restrict__ gcum) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  gcum[0] = 0.f;
  for (int i = 0; i < K; ++i) {
    s += taps[K - 1 - i];
    gcum[i + 1] = static_cast<float>(s);
  }
}

template <int NW>
__global__ __launch_bounds__(PDM_THREADS) void pdm_demod_kernel(
    const unsigned* __restrict__ words, const float* __restrict__ lut_g, const float* __restrict__ gcum,
    float* __restrict__ x, int M, int W, int N, int D, int K, int NB, int SW, int ntile) {
  constexpr int C = 4 * NW;                               // byte tables, zero past the filter
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

  // 1. bit transpose: 64-tick chunks, wave-strided; the next chunk's first word is
  //    loaded while the current one is turned into masks
  const int nchunk = SW >> 1;
  auto load_word = [&](int ch, int w) -> unsigned {
    const long long t = tb + 64LL * ch + lane;
    return (ch < nchunk && t >= 0 && t < T) ? wf[t * W + w] : 0u;
  };
  unsigned next0 = load_word(wv, 0);
  for (int ch = wv; ch < nchunk; ch += PDM_THREADS / 64) {
    const unsigned first = next0;
    next0 = load_word(ch + PDM_THREADS / 64, 0);
    unsigned long long keep0 = 0, keep1 = 0;
    for (int w = 0; w < W; ++w) {
      const unsigned word = w == 0 ? first : load_word(ch, w);
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
  float* xf = x + f * static_cast<long long>(M) * N;
  for (int m = wv; m < M; m += PDM_THREADS / 64) {
    const unsigned* bm = bits + m * SW;
    for (int nb = lane; nb < NB; nb += 64) {
      const int n = n0 + nb;
      if (n >= N) break;
      const long long ts = static_cast<long long>(n) * D - hk;   // first tick of the window
      const int a = static_cast<int>(ts - tb);                   // its bit offset in the staged string
      const int w0 = a >> 5, sh = a & 31;
      unsigned wd[NW + 1];
#pragma unroll
      for (int k = 0; k <= NW; ++k) wd[k] = bm[w0 + k];
      float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const unsigned al = __builtin_amdgcn_alignbit(wd[k + 1], wd[k], sh);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) part[cc] += lut[(4 * k + cc) * 256 + ((al >> (8 * cc)) & 255u)];
      }
      float acc = (part[0] + part[1]) + (part[2] + part[3]);
      if (ts < 0 || ts + K > T) {
        // window positions i < lo and i >= hi lie outside the recording
        const int lo = ts < 0 ? static_cast<int>(ts < -K ? K : -ts) : 0;
        const int hi = ts + K > T ? static_cast<int>(T - ts > 0 ? T - ts : 0) : K;
        acc += gcum[lo] + (gcum[K] - gcum[hi > lo ? hi : lo]);
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

// byte tables per filter length: 4 per aligned 32-bit word of the window
int pdm_tables(int K) { return 4 * ((K + 31) / 32); }

size_t pdm_lds_bytes(int M, int SW, int C) {
  return (static_cast<size_t>(M) * SW + static_cast<size_t>(C) * 256) * 4;
}

hipError_t launch_pdm_tables(sonar_pdm_s* p, const double* d_taps64, hipStream_t s) {
  const int n = p->C * 256;
  hipLaunchKernelGGL(pdm_lut_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_taps64, p->K, p->C, p->d_lut);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pdm_prefix_kernel, dim3(1), dim3(64), 0, s, d_taps64, p->K, p->d_gcum);
  return hipGetLastError();
}

namespace {

template <int NW>
hipError_t set_attr(size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(pdm_demod_kernel<NW>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
}

template <int NW>
hipError_t launch_nw(const sonar_pdm_s* p, const unsigned* words, int F, float* x, hipStream_t s) {
  const int ntile = (p->N + p->NB - 1) / p->NB;
  const size_t lds = pdm_lds_bytes(p->M, p->SW, p->C);
  hipLaunchKernelGGL(pdm_demod_kernel<NW>, dim3(static_cast<unsigned>(F) * ntile), dim3(PDM_THREADS), lds, s, words,
                     p->d_lut, p->d_gcum, x, p->M, p->W, p->N, p->D, p->K, p->NB, p->SW, ntile);
  return hipGetLastError();
}

}  // namespace

#define SONAR_PDM_NW_DISPATCH(NAME, NWV, ...)                                            \
  switch (NWV) {                                                                          \
    case 1: return NAME<1>(__VA_ARGS__);   case 2: return NAME<2>(__VA_ARGS__);           \
    case 3: return NAME<3>(__VA_ARGS__);   case 4: return NAME<4>(__VA_ARGS__);           \
    case 5: return NAME<5>(__VA_ARGS__);   case 6: return NAME<6>(__VA_ARGS__);           \
    case 7: return NAME<7>(__VA_ARGS__);   case 8: return NAME<8>(__VA_ARGS__);           \
    case 9: return NAME<9>(__VA_ARGS__);   case 10: return NAME<10>(__VA_ARGS__);         \
    case 11: return NAME<11>(__VA_ARGS__); case 12: return NAME<12>(__VA_ARGS__);         \
    case 13: return NAME<13>(__VA_ARGS__); case 14: return NAME<14>(__VA_ARGS__);         \
    case 15: return NAME<15>(__VA_ARGS__); case 16: return NAME<16>(__VA_ARGS__);         \
    case 17: return NAME<17>(__VA_ARGS__);                                                \
    default: return hipErrorInvalidValue;                                                 \
  }

hipError_t init_pdm_kernel_attributes(const sonar_pdm_s* p, size_t lds) {
  SONAR_PDM_NW_DISPATCH(set_attr, p->C / 4, lds)
}

hipError_t launch_pdm_demod(const sonar_pdm_s* p, const unsigned* words, int F, float* x, hipStream_t s) {
  SONAR_PDM_NW_DISPATCH(launch_nw, p->C / 4, p, words, F, x, s)
}
