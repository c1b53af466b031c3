// Matched filter for FFT lengths beyond one workgroup's LDS (§4.1 matched
// filter; §4.3 FFT-convolution filters with the group delay removed).
//
// Same result as k_mf.hip: Yhat[k] = X[k] C[k] for k in [0, NF] and, for the
// time-domain beamformers, yhat[n] = IDFT_P(Yhat)[n], with the real input
// packed as z[n] = x[2n] + i x[2n+1] into an NF = P/2 point complex FFT.
// Here NF = R * N2 with N2 = 2^MB_LOGN2 held in LDS and a radix-R pass over
// global memory (four-step decomposition, n = N2 n1 + n2, k = k1 + R k2):
//
//   X[k1 + R k2] = sum_n2 W_N2^(n2 k2) [ W_NF^(n2 k1) sum_n1 z[N2 n1 + n2] W_R^(n1 k1) ]
//   y[N2 n1 + n2] = sum_k1 W_R^(-n1 k1) W_NF^(-n2 k1) sum_k2 v[k1 + R k2] W_N2^(-n2 k2)
//
// Kernels per launch:
//   forward  : big_fwd_radix (z -> t, radix R + twiddle), big_fwd_rows (N2-point
//              FFT of each t row -> Z in natural order), big_split (real split,
//              x C -> one-sided spectrum, or the band bins bin-major);
//   inverse  : big_inv_rows (per output parity and k1: parity twiddle,
//              N2-point inverse FFT -> u), big_inv_radix (twiddle, radix-R
//              inverse, Nyquist term, 1/P, scatter into the halo'd rows and
//              the BF16 planes);
//   real inverse: big_inv_rows, then big_inv_real (the real part cut to N samples:
//              the adjoint of the matched filter in the gradient path).
// Scratch (plan workspace): per channel 2 NF complex values; t and Z first,
// then the two parities of u.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include "fft_lds.hpp"
#include "plan.hpp"

using namespace fftk;

namespace {

constexpr int LOGN2 = MB_LOGN2;
constexpr int N2 = 1 << LOGN2;

template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<__half>(__half v) { return __half2float(v); }
template <>
__device__ __forceinline__ float to_f32<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }

__device__ __forceinline__ unsigned short bf16_rne(float v) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(v));
}

// Twiddles from the plan's two-level tables in global memory (layout in plan.hpp)
struct BigTw {
  const float2* hi;    // exp(-2 pi i 64 t / NF)
  const float2* lo;    // exp(-2 pi i t / NF)
  const float2* phi;   // exp(-2 pi i 64 t / P)
  const float2* plo;   // exp(-2 pi i t / P)
  __device__ __forceinline__ float2 nf(int e) const { return cmul(hi[e >> 6], lo[e & 63]); }
  __device__ __forceinline__ float2 p(int e) const { return cmul(phi[e >> 6], plo[e & 63]); }
};

__device__ __forceinline__ BigTw big_tw(const float2* __restrict__ tw, int NF) {
  BigTw t;
  t.hi = tw;
  t.lo = tw + NF / 64;
  t.phi = tw + NF / 64 + 64;
  t.plo = tw + NF / 64 + 64 + NF / 64 + 1;
  return t;
}

// z (packed real samples) -> t[k1][n2] = W_NF^(n2 k1) sum_n1 z[N2 n1 + n2] W_R^(n1 k1)
template <int R, typename TIn>
__global__ __launch_bounds__(256) void big_fwd_radix(const TIn* __restrict__ x, int N,
                                                     const float2* __restrict__ tw_g,
                                                     float2* __restrict__ scratch) {
  constexpr int NF = R * N2;
  const int n2 = blockIdx.x * 256 + threadIdx.x;
  const long long ch = blockIdx.y;
  const TIn* xc = x + ch * N;
  const BigTw tw = big_tw(tw_g, NF);
  float2 v[R];
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) {
    const int i0 = 2 * (N2 * n1 + n2);
    const float a = i0 < N ? to_f32<TIn>(xc[i0]) : 0.0f;
    const float b = i0 + 1 < N ? to_f32<TIn>(xc[i0 + 1]) : 0.0f;
    v[n1] = make_float2(a, b);
  }
  dftR<R, false>(v);
  float2* t = scratch + ch * 2 * NF;
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) t[k1 * N2 + n2] = k1 == 0 ? v[0] : cmul(v[k1], tw.nf(n2 * k1));
}

// one row t[k1][.] per workgroup: N2-point FFT, written as Z[k1 + R k2]
template <int R>
__global__ __launch_bounds__(N2 / 16) void big_fwd_rows(const float2* __restrict__ tw2_g,
                                                        float2* __restrict__ scratch) {
  using S = FftShape<LOGN2>;
  constexpr int NF = R * N2;
  constexpr int T = S::T;
  constexpr int NHI = N2 / 64;
  __shared__ float2 lds[S::LDS_ELEMS];
  __shared__ float2 tw[NHI + 64];
  const int tid = threadIdx.x;
  const long long ch = blockIdx.x / R;
  const int k1 = blockIdx.x % R;
  for (int i = tid; i < NHI + 64; i += T) tw[i] = tw2_g[i];
  const float2* row = scratch + ch * 2 * NF + static_cast<long long>(k1) * N2;
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = row[tid + r * (N2 / 16)];
  __syncthreads();
  fft_lds<LOGN2, false>(v, lds, tw, tw + NHI, tid);
  float2* Z = scratch + ch * 2 * NF + NF;
#pragma unroll
  for (int i = 0; i < 16; ++i) Z[k1 + R * S::out_index(tid, i)] = v[i];
}

// Real split and matched-filter product of one channel's packed transform Z:
// X[k] = E[k] + exp(-2 pi i k / P) O[k]; writes the one-sided spectrum
// spec[ch][0..NF] (TD) or the band bins band[f][k - k_lo][m] (FD).
__global__ __launch_bounds__(256) void big_split(const float2* __restrict__ scratch, const float2* __restrict__ tw_g,
                                                 const float2* __restrict__ cspec, int NF, int M,
                                                 float2* __restrict__ spec, float2* __restrict__ band, int k_lo,
                                                 int kb) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k > NF / 2) return;
  const long long ch = blockIdx.y;
  const BigTw tw = big_tw(tw_g, NF);
  const float2* Z = scratch + ch * 2 * NF + NF;
  const float2 A = Z[k];
  const float2 B = Z[(NF - k) & (NF - 1)];
  const float2 Ek = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));      // (A + conj B)/2
  const float2 Ok = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));     // (A - conj B)/(2i)
  const float2 wo = cmul(tw.p(k), Ok);
  const float2 Xk = cadd(Ek, wo);
  const float2 Xm = cconj(csub(Ek, wo));                                      // X[NF - k]
  const float2 yk = cmul(Xk, cspec[k]);
  const float2 ym = cmul(Xm, cspec[NF - k]);                                  // k = 0: the Nyquist bin
  if (spec) {
    float2* out = spec + ch * (NF + 1);
    out[k] = yk;
    if (k != NF / 2) out[NF - k] = ym;
  } else {
    const long long f = ch / M;
    const int m = static_cast<int>(ch - f * M);
    float2* out = band + f * static_cast<long long>(kb) * M + m;
    if (k >= k_lo && k < k_lo + kb) out[static_cast<long long>(k - k_lo) * M] = yk;
    const int km = NF - k;
    if (k != NF / 2 && km >= k_lo && km < k_lo + kb) out[static_cast<long long>(km - k_lo) * M] = ym;
  }
}

// per (channel, output parity, k1): u[par][k1][n2] = sum_k2 v[k1 + R k2] W_N2^(-n2 k2),
// v[k] = Yhat[k] exp(2 pi i k par / P)
template <int R>
__global__ __launch_bounds__(N2 / 16) void big_inv_rows(const float2* __restrict__ spec,
                                                        const float2* __restrict__ tw_g,
                                                        const float2* __restrict__ tw2_g,
                                                        float2* __restrict__ scratch, long long chans) {
  using S = FftShape<LOGN2>;
  constexpr int NF = R * N2;
  constexpr int T = S::T;
  constexpr int NHI = N2 / 64;
  __shared__ float2 lds[S::LDS_ELEMS];
  __shared__ float2 tw[NHI + 64];
  const int tid = threadIdx.x;
  // the 2R workgroups of channel 8 j + x (every k1, both parities: each reads a strided share of
  // the channel's spectrum, together every line 2R times) are blocks 16 R j + 8 s + x, s < 2R:
  // all on XCD x (workgroups go to the XCDs round-robin), so the lines come from that L2
  const int s8 = (blockIdx.x / 8) % (2 * R);
  const int k1 = s8 % R;
  const int par = s8 / R;
  const long long ch = static_cast<long long>(blockIdx.x / (16 * R)) * 8 + blockIdx.x % 8;
  if (ch >= chans) return;
  for (int i = tid; i < NHI + 64; i += T) tw[i] = tw2_g[i];
  const BigTw twb = big_tw(tw_g, NF);
  const float2* in = spec + ch * (NF + 1);
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k = k1 + R * (tid + r * (N2 / 16));
    v[r] = in[k];
    if (par) v[r] = cmul(v[r], cconj(twb.p(k)));   // exp(+2 pi i k / P)
  }
  __syncthreads();
  fft_lds<LOGN2, true>(v, lds, tw, tw + NHI, tid);
  float2* u = scratch + ch * 2 * NF + static_cast<long long>(par) * NF + static_cast<long long>(k1) * N2;
#pragma unroll
  for (int i = 0; i < 16; ++i) u[S::out_index(tid, i)] = v[i];
}

// per (channel, parity, n2): y[N2 n1 + n2] = sum_k1 W_R^(-n1 k1) W_NF^(-n2 k1) u[k1][n2];
// yhat[2 (N2 n1 + n2) + par] = (y + (-1)^par Yhat[NF]) / P, scattered into the rows
template <int R>
__global__ __launch_bounds__(256) void big_inv_radix(const float2* __restrict__ spec, const float2* __restrict__ tw_g,
                                                     const float2* __restrict__ scratch, float2* __restrict__ yext,
                                                     long long fstride, int M, int row, int origin, int P,
                                                     int planes, const float* __restrict__ fbound, int rows) {
  constexpr int NF = R * N2;
  const int n2 = blockIdx.x * 256 + threadIdx.x;
  const int par = blockIdx.y & 1;
  const long long ch = blockIdx.y >> 1;
  const BigTw tw = big_tw(tw_g, NF);
  const float2* u = scratch + ch * 2 * NF + static_cast<long long>(par) * NF;
  float2 v[R];
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) {
    const float2 a = u[static_cast<long long>(k1) * N2 + n2];
    v[k1] = k1 == 0 ? a : cmul(a, cconj(tw.nf(n2 * k1)));
  }
  dftR<R, true>(v);
  const float2 ny = spec[ch * (NF + 1) + NF];
  const float inv_p = 1.0f / static_cast<float>(P);
  const float sgn = par ? -1.0f : 1.0f;
  const long long f = ch / M;
  const int m = static_cast<int>(ch - f * M);
  float2* out = yext + f * fstride + static_cast<long long>(m) * row;
  unsigned short* pl = reinterpret_cast<unsigned short*>(yext + f * fstride + static_cast<long long>(M) * row) +
                       static_cast<long long>(m) * planes * row;
  // TD_F16: FP16 planes of 2^e yhat (e from the frame's channel bounds), 2^-e / M in the frame header
  float sc = 0.f;
  if (fbound) {
    const int e = mf_f16_exponent(fbound, f, M);
    sc = ldexpf(1.0f, e);
    if (m == 0 && par == 0 && n2 == 0)
      *reinterpret_cast<float*>(yext + f * fstride + mf_f16_header(M, row)) = ldexpf(1.0f / static_cast<float>(M), -e);
  }
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) {
    const int n = 2 * (N2 * n1 + n2) + par;
    const float2 y = make_float2((v[n1].x + sgn * ny.x) * inv_p, (v[n1].y + sgn * ny.y) * inv_p);
    unsigned short rh = 0, rl = 0, ih = 0, il = 0;
    if (planes) {
      rh = mf_plane_word(y.x, sc);
      ih = mf_plane_word(y.y, sc);
      if (planes == 4) {
        rl = bf16_rne(y.x - __uint_as_float(static_cast<unsigned>(rh) << 16));
        il = bf16_rne(y.y - __uint_as_float(static_cast<unsigned>(ih) << 16));
      }
    }
    for (int j = (n - origin) & (P - 1); j < row; j += P) {
      if (rows) out[j] = y;
      if (planes == 4) {
        pl[j] = rh;
        pl[row + j] = rl;
        pl[2 * row + j] = ih;
        pl[3 * row + j] = il;
      } else if (planes == 2) {
        pl[j] = rh;
        pl[row + j] = ih;
      }
    }
  }
}

// Real part of the same inverse, cut to n < N: out[ch][n] = Re (y + (-1)^par V[NF]) / P
// (the matched filter's adjoint, whose one-sided spectrum V is conjugate-symmetric only in
// what the real part keeps)
template <int R>
__global__ __launch_bounds__(256) void big_inv_real(const float2* __restrict__ V, const float2* __restrict__ tw_g,
                                                    const float2* __restrict__ scratch, float* __restrict__ out,
                                                    int N, int P) {
  constexpr int NF = R * N2;
  const int n2 = blockIdx.x * 256 + threadIdx.x;
  const int par = blockIdx.y & 1;
  const long long ch = blockIdx.y >> 1;
  const BigTw tw = big_tw(tw_g, NF);
  const float2* u = scratch + ch * 2 * NF + static_cast<long long>(par) * NF;
  float2 v[R];
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) {
    const float2 a = u[static_cast<long long>(k1) * N2 + n2];
    v[k1] = k1 == 0 ? a : cmul(a, cconj(tw.nf(n2 * k1)));
  }
  dftR<R, true>(v);
  const float ny = V[ch * (NF + 1) + NF].x;
  const float inv_p = 1.0f / static_cast<float>(P);
  const float sgn = par ? -1.0f : 1.0f;
  float* o = out + ch * N;
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) {
    const int n = 2 * (N2 * n1 + n2) + par;
    if (n < N) o[n] = (v[n1].x + sgn * ny) * inv_p;
  }
}

template <int R>
hipError_t inverse_real_t(const sonar_plan_s* p, const float2* V, int chans, float* out, hipStream_t s) {
  hipLaunchKernelGGL((big_inv_rows<R>), dim3((chans + 7) / 8 * 16 * R), dim3(N2 / 16), 0, s, V, p->d_tw, p->d_tw2,
                     p->d_big, static_cast<long long>(chans));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((big_inv_real<R>), dim3(N2 / 256, 2 * chans), dim3(256), 0, s, V, p->d_tw, p->d_big, out, p->N,
                     p->P);
  return hipGetLastError();
}

template <int R, typename TIn>
hipError_t forward_t(const sonar_plan_s* p, const void* x, int F, float2* spec, float2* band, hipStream_t s) {
  constexpr int NF = R * N2;
  const int chans = F * p->M;
  hipLaunchKernelGGL((big_fwd_radix<R, TIn>), dim3(N2 / 256, chans), dim3(256), 0, s, static_cast<const TIn*>(x),
                     p->N, p->d_tw, p->d_big);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((big_fwd_rows<R>), dim3(chans * R), dim3(N2 / 16), 0, s, p->d_tw2, p->d_big);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(big_split, dim3((NF / 2 + 1 + 255) / 256, chans), dim3(256), 0, s, p->d_big, p->d_tw,
                     p->d_cspec, NF, p->M, spec, band, p->k_lo, p->kb);
  return hipGetLastError();
}

template <int R>
hipError_t inverse_t(const sonar_plan_s* p, int F, float2* yext, hipStream_t s, bool rows) {
  const int chans = F * p->M;
  hipLaunchKernelGGL((big_inv_rows<R>), dim3((chans + 7) / 8 * 16 * R), dim3(N2 / 16), 0, s, p->d_spec, p->d_tw,
                     p->d_tw2, p->d_big, static_cast<long long>(chans));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((big_inv_radix<R>), dim3(N2 / 256, 2 * chans), dim3(256), 0, s, p->d_spec, p->d_tw, p->d_big,
                     yext, p->mf_fstride, p->M, p->row, static_cast<int>(p->origin), p->P,
                     mt_planes(p), mt_f16(p) ? p->d_fbound : nullptr, rows ? 1 : 0);
  return hipGetLastError();
}

template <typename TIn>
hipError_t forward_dt(const sonar_plan_s* p, const void* x, int F, float2* spec, float2* band, hipStream_t s) {
  switch (p->NF / N2) {
    case 2: return forward_t<2, TIn>(p, x, F, spec, band, s);
    case 4: return forward_t<4, TIn>(p, x, F, spec, band, s);
    case 8: return forward_t<8, TIn>(p, x, F, spec, band, s);
    case 16: return forward_t<16, TIn>(p, x, F, spec, band, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t forward(const sonar_plan_s* p, const void* x, int F, float2* spec, float2* band, hipStream_t s) {
  switch (p->dtype) {
    case SONAR_F32: return forward_dt<float>(p, x, F, spec, band, s);
    case SONAR_F16: return forward_dt<__half>(p, x, F, spec, band, s);
    case SONAR_BF16: return forward_dt<__hip_bfloat16>(p, x, F, spec, band, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_mf_big_td(const sonar_plan_s* p, const void* x, int F, float2* yext, hipStream_t s, bool rows) {
  hipError_t e = forward(p, x, F, p->d_spec, nullptr, s);
  if (e == hipSuccess && mt_f16(p)) e = launch_mf_bound(p, F, s);
  if (e != hipSuccess) return e;
  switch (p->NF / N2) {
    case 2: return inverse_t<2>(p, F, yext, s, rows);
    case 4: return inverse_t<4>(p, F, yext, s, rows);
    case 8: return inverse_t<8>(p, F, yext, s, rows);
    case 16: return inverse_t<16>(p, F, yext, s, rows);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_big_inv_real(const sonar_plan_s* p, const float2* V, int chans, float* out, hipStream_t s) {
  if (!p->d_big || !p->d_tw2) return hipErrorInvalidValue;
  switch (p->NF / N2) {
    case 2: return inverse_real_t<2>(p, V, chans, out, s);
    case 4: return inverse_real_t<4>(p, V, chans, out, s);
    case 8: return inverse_real_t<8>(p, V, chans, out, s);
    case 16: return inverse_real_t<16>(p, V, chans, out, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mf_big_fd(const sonar_plan_s* p, const void* x, int F, float2* band, hipStream_t s) {
  return forward(p, x, F, nullptr, band, s);
}
