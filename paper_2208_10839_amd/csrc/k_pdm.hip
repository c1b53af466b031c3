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
//
// Matrix-core variant (where a tile's tap operand fits LDS, 15 D + K <= 1024): the filter
// of 16 consecutive outputs n0.. of 16 microphones is one banded product over the ticks of
// their windows, X[m][n0 + c] = sum_k bit_m[ts(n0) + k] A[k][c] with A[k][c] = g[k - D c],
// taken on int8 matrix cores (16x16x64).  The taps enter as integers r = round(g 2^qshift)
// (|r| < 2^29) in four signed base-256 digits, one product per digit, and the bits as 0 / 1,
// so the sums are exact integers and
//     x = (2 sum_i r[i] bit[ts + i] - sum_{i inside the recording} r[i]) 2^-qshift
// (s = 2 bit - 1 inside, 0 outside) is rounded once.  The bit strings come from a 32 x 32
// bit-matrix transpose in registers (five exchange steps between lanes) instead of ballots.
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

typedef int pdm_i32x4 __attribute__((ext_vector_type(4)));

// signed base-256 digit t (0 = most significant) of r, |r| < 2^29: r = sum_t d_t 256^(3-t)
__device__ int pdm_digit(long long r, int t) {
  int d3 = static_cast<signed char>(r & 0xFF);
  r = (r - d3) / 256;
  int d2 = static_cast<signed char>(r & 0xFF);
  r = (r - d2) / 256;
  int d1 = static_cast<signed char>(r & 0xFF);
  r = (r - d1) / 256;
  return t == 0 ? static_cast<int>(r) : (t == 1 ? d1 : (t == 2 ? d2 : d3));
}

// tap operand of a 16-output tile, in the B-fragment order of the 16x16x64 int8 product:
// word (ks, t, lane, j), byte i holds digit t of r[k - D c], k = 64 ks + 16 (lane / 16) + 4 j + i,
// c = lane % 16 (zero outside the filter), r[i] = round(2^qshift h[K-1-i]) in FP64
__global__ void pdm_qtab_kernel(const double* __restrict__ taps, int K, int D, int KS, int qshift,
                                unsigned* __restrict__ qtab) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= KS * 1024) return;
  const int j = e & 3, lane = (e >> 2) & 63, t = (e >> 8) & 3, ks = e >> 10;
  unsigned word = 0;
  for (int i = 0; i < 4; ++i) {
    const int ig = 64 * ks + 16 * (lane >> 4) + 4 * j + i - D * (lane & 15);
    if (ig >= 0 && ig < K) {
      const long long r = llrint(ldexp(taps[K - 1 - ig], qshift));
      word |= (static_cast<unsigned>(pdm_digit(r, t)) & 0xFFu) << (8 * i);
    }
  }
  qtab[e] = word;
}

// rcum[i] = sum_{j<i} r[j], i <= K
__global__ void pdm_rcum_kernel(const double* __restrict__ taps, int K, int qshift, long long* __restrict__ rcum) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  long long s = 0;
  rcum[0] = 0;
  for (int i = 0; i < K; ++i) {
    s += llrint(ldexp(taps[K - 1 - i], qshift));
    rcum[i + 1] = s;
  }
}

// 32 x 32 bit transpose within each half-wavefront: lane r holds row r (bit c = element (r, c))
// on entry and column r (bit c = element (c, r)) on return; step j swaps the off-diagonal
// j x j blocks of every 2j x 2j block between lanes r and r ^ j
template <int J, unsigned MASK>
__device__ __forceinline__ unsigned pdm_transpose_step(unsigned x, int lane) {
  const unsigned y = static_cast<unsigned>(__shfl_xor(static_cast<int>(x), J));
  return (lane & J) ? ((x & ~MASK) | ((y >> J) & MASK)) : ((x & MASK) | ((y << J) & ~MASK));
}

__device__ __forceinline__ unsigned pdm_transpose32(unsigned x, int lane) {
  x = pdm_transpose_step<16, 0x0000FFFFu>(x, lane);
  x = pdm_transpose_step<8, 0x00FF00FFu>(x, lane);
  x = pdm_transpose_step<4, 0x0F0F0F0Fu>(x, lane);
  x = pdm_transpose_step<2, 0x33333333u>(x, lane);
  return pdm_transpose_step<1, 0x55555555u>(x, lane);
}

// bits 0..15 of b as 16 bytes of 0 / 1 (byte 4 j + i = bit 4 j + i)
__device__ __forceinline__ pdm_i32x4 pdm_bytes01(unsigned b) {
  pdm_i32x4 v;
  v.x = static_cast<int>(((b & 15u) * 0x204081u) & 0x01010101u);
  v.y = static_cast<int>((((b >> 4) & 15u) * 0x204081u) & 0x01010101u);
  v.z = static_cast<int>((((b >> 8) & 15u) * 0x204081u) & 0x01010101u);
  v.w = static_cast<int>((((b >> 12) & 15u) * 0x204081u) & 0x01010101u);
  return v;
}

__global__ __launch_bounds__(PDM_MT_THREADS) void pdm_mfma_kernel(
    const unsigned* __restrict__ words, const pdm_i32x4* __restrict__ qtab_g, const long long* __restrict__ rcum,
    float* __restrict__ x, int M, int W, int N, int D, int K, int NB, int SW, int ntile, int KS, int rows,
    int qshift, int vec4) {
  constexpr int NWAVE = PDM_MT_THREADS / 64;
  extern __shared__ unsigned smem[];
  pdm_i32x4* qtab = reinterpret_cast<pdm_i32x4*>(smem);   // [KS][4][64]
  unsigned* bits = smem + KS * 1024;                      // [rows][SW]
  const int tile = blockIdx.x % ntile;
  const long long f = blockIdx.x / ntile;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long T = static_cast<long long>(N) * D;
  const int hk = (K - 1) >> 1;
  const int n0 = tile * NB;
  const long long t_lo = static_cast<long long>(n0) * D - hk;
  const long long tb = t_lo >= 0 ? (t_lo & ~31LL) : -((-t_lo + 31) & ~31LL);   // floor to a multiple of 32
  const unsigned* wf = words + f * T * W;
  for (int i = threadIdx.x; i < KS * 256; i += PDM_MT_THREADS) qtab[i] = qtab_g[i];

  // 1. 64-tick chunks: lane l loads tick 64 ch + l, the transpose leaves microphone
  //    32 w + l % 32's bits of ticks 64 ch + 32 (l / 32) + 0..31 in lane l.  A wavefront
  //    takes chunks wv, wv + NWAVE, ..., loading PF of them before transposing any
  constexpr int PF = 8;
  const int nchunk = SW >> 1;
  for (int c0 = wv; c0 < nchunk; c0 += PF * NWAVE) {
    for (int w = 0; 32 * w < rows; ++w) {
      unsigned v[PF];
#pragma unroll
      for (int i = 0; i < PF; ++i) {
        const int ch = c0 + i * NWAVE;
        const long long t = tb + 64LL * ch + lane;
        v[i] = (ch < nchunk && t >= 0 && t < T) ? wf[t * W + w] : 0u;
      }
      const int m = 32 * w + (lane & 31);
#pragma unroll
      for (int i = 0; i < PF; ++i) {
        const int ch = c0 + i * NWAVE;
        const unsigned col = pdm_transpose32(v[i], lane);
        if (ch < nchunk && m < rows) bits[m * SW + 2 * ch + (lane >> 5)] = col;
      }
    }
  }
  __syncthreads();

  // 2. tiles of 16 outputs x 16 microphones, four per wavefront at a time (they share the
  //    tap operand, which does not depend on the tile): A = the tap digits (row = output,
  //    lane % 16), B = the bits (column = microphone, lane % 16); lane l reads 16 ticks from
  //    bit 64 ks + 16 (l / 16) of its tile's span
  constexpr int G = 4;
  const int ntl = NB / 16;
  const int items = ntl * (rows / 16);
  const int r16 = lane & 15, kh = lane >> 4;
  float* xf = x + f * static_cast<long long>(M) * N;
  const long long rtot = rcum[K];
  for (int i0 = wv; i0 < items; i0 += G * NWAVE) {
    const unsigned* bm[G];
    int sh[G], nt0[G];
    bool ok[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int it = i0 + g * NWAVE;
      const int tl = it % ntl, mb = it / ntl;
      nt0[g] = n0 + 16 * tl;
      ok[g] = it < items && nt0[g] < N;   // wave-uniform
      const int a = ok[g] ? static_cast<int>(static_cast<long long>(nt0[g]) * D - hk - tb) + 16 * kh : 0;
      bm[g] = bits + (ok[g] ? (16 * mb + r16) * SW + (a >> 5) : 0);
      sh[g] = a & 31;
    }
    pdm_i32x4 acc[G][4];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[g][t] = pdm_i32x4{0, 0, 0, 0};
    for (int ks = 0; ks < KS; ++ks) {
      const pdm_i32x4* q = qtab + ks * 256 + lane;
      const pdm_i32x4 q0 = q[0], q1 = q[64], q2 = q[128], q3 = q[192];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (!ok[g]) continue;
        const pdm_i32x4 bv = pdm_bytes01(__builtin_amdgcn_alignbit(bm[g][2 * ks + 1], bm[g][2 * ks], sh[g]));
        acc[g][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(q0, bv, acc[g][0], 0, 0, 0);
        acc[g][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(q1, bv, acc[g][1], 0, 0, 0);
        acc[g][2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(q2, bv, acc[g][2], 0, 0, 0);
        acc[g][3] = __builtin_amdgcn_mfma_i32_16x16x64_i8(q3, bv, acc[g][3], 0, 0, 0);
      }
    }
    // lane l holds outputs nt0 + 4 (l / 16) + v of microphone 16 mb + l % 16
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (!ok[g]) continue;
      const int mb = (i0 + g * NWAVE) / ntl;
      const int m = 16 * mb + r16;
      const int nb = nt0[g] + 4 * kh;
      if (m >= M || nb >= N) continue;
      float o[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long long ts = static_cast<long long>(nb + v) * D - hk;
        long long rin = rtot;
        if (ts < 0 || ts + K > T) {
          const int lo = ts < 0 ? static_cast<int>(ts < -K ? K : -ts) : 0;
          const int hi = ts + K > T ? static_cast<int>(T - ts > 0 ? T - ts : 0) : K;
          rin = rcum[hi > lo ? hi : lo] - rcum[lo];
        }
        const long long sum = (static_cast<long long>(acc[g][0][v]) << 24) +
                              (static_cast<long long>(acc[g][1][v]) << 16) +
                              (static_cast<long long>(acc[g][2][v]) << 8) + static_cast<long long>(acc[g][3][v]);
        o[v] = ldexpf(static_cast<float>(2 * sum - rin), -qshift);
      }
      float* dst = xf + static_cast<long long>(m) * N + nb;
      if (vec4 && nb + 3 < N) {
        *reinterpret_cast<float4*>(dst) = make_float4(o[0], o[1], o[2], o[3]);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (nb + v < N) dst[v] = o[v];
      }
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

// 64-tick K-steps of a 16-output tile: the ticks of its windows, 15 D + K
int pdm_mt_ksteps(int D, int K) { return (15 * D + K + 63) / 64; }

// staged words per microphone row of the matrix-core variant: the last tile's reads (its first
// tick at most 31 past the 32-aligned start, lanes offset by up to 48 ticks, KS K-steps of two
// words), rounded to 64 ticks
int pdm_mt_span_words(int NB, int D, int KS) {
  const long long words = (static_cast<long long>(NB - 16) * D + 79) / 32 + 2LL * KS;
  return static_cast<int>((words + 1) & ~1LL);
}

size_t pdm_mt_lds_bytes(int rows, int SW, int KS) {
  return (static_cast<size_t>(KS) * 1024 + static_cast<size_t>(rows) * SW) * 4;
}

hipError_t launch_pdm_tables(sonar_pdm_s* p, const double* d_taps64, hipStream_t s) {
  if (p->mt) {
    const int n = p->KS * 1024;
    hipLaunchKernelGGL(pdm_qtab_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_taps64, p->K, p->D, p->KS,
                       p->qshift, p->d_qtab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pdm_rcum_kernel, dim3(1), dim3(64), 0, s, d_taps64, p->K, p->qshift, p->d_rcum);
    return hipGetLastError();
  }
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
  if (p->mt)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(pdm_mfma_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  SONAR_PDM_NW_DISPATCH(set_attr, p->C / 4, lds)
}

hipError_t launch_pdm_demod(const sonar_pdm_s* p, const unsigned* words, int F, float* x, hipStream_t s) {
  if (p->mt) {
    const int ntile = (p->N + p->NB - 1) / p->NB;
    hipLaunchKernelGGL(pdm_mfma_kernel, dim3(static_cast<unsigned>(F) * ntile), dim3(PDM_MT_THREADS),
                       pdm_mt_lds_bytes(p->rows, p->SW, p->KS), s, words, reinterpret_cast<const pdm_i32x4*>(p->d_qtab),
                       p->d_rcum, x, p->M, p->W, p->N, p->D, p->K, p->NB, p->SW, ntile, p->KS, p->rows, p->qshift,
                       (p->N & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0 ? 1 : 0);
    return hipGetLastError();
  }
  SONAR_PDM_NW_DISPATCH(launch_nw, p->C / 4, p, words, F, x, s)
}
