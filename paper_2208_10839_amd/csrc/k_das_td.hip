// Time-domain delay-and-sum beamformer (§4.1 delay-and-sum toward every
// direction of interest; §4.3 a device kernel) fused with the envelope
// detector and subsampling (§4.1 envelope; §4.3 subsampling after envelope
// detection):
//
//   b_d[n]  = sum_m w0[d][m] yhat_m[n + o] + w1[d][m] yhat_m[n + o + 1],
//             w0 = (1 - alpha)/M, w1 = alpha/M,
//   E[d][q] = sum_j h[j] |b_d[n0 + qR + (K-1)/2 - j]|.
//
// Mapping: a workgroup owns TD_NW directions (one wavefront each) and a tile
// of beam samples; lane l of a wavefront handles samples 64 t + l, t < TD_NB.
// The workgroup stages the matched-filter rows of a group of microphones in
// LDS (contiguous, coalesced), then each wavefront reads yhat_m[n + o] once
// per sample and microphone and accumulates two sums
//   A[n] = sum_m w0 yhat_m[n + o],   C[n] = sum_m w1 yhat_m[n + o]
// so that b[n] = A[n] + C[n + 1]: the one-sample neighbour of the linear
// interpolation is taken once per direction from the adjacent lane after the
// microphone loop, instead of once per microphone.  Per (direction, mic,
// sample) that is one 8-byte LDS read and four FMAs, with (o, w0, w1) in
// scalar registers because a wavefront has one direction.  The beam never
// leaves the chip: |b| goes to LDS and the FIR reads it there at the
// decimated positions.
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace {

// lane i receives v of lane (i + 1) mod 64
__device__ __forceinline__ float from_next_lane(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(((lane + 1) & 63) << 2, __float_as_int(v)));
}

// Accumulates A[n] = sum_m w0 yhat_m[n + o] and C[n] = sum_m w1 yhat_m[n + o]
// for this wavefront's direction over all microphones.  Microphones are
// consumed in groups of at most NW rows held in LDS; wavefront w copies row w
// of a group with back-to-back 16-byte loads (one address register plus
// immediate offsets), then stores them.  The table entries (o - omin, w0, w1)
// of the wavefront's direction sit one microphone per lane (up to 128 mics)
// and are broadcast with readlane.
// M counts table entries; entry m reads matched-filter row m >> vshift (TD_CUBIC
// takes each microphone as two two-tap entries).
template <int NB, int NW>
__device__ __forceinline__ void das_accumulate(const float2* __restrict__ yrow0, long long row,
                                               const int4* __restrict__ dtab_d, int M, int vshift, int mc, int ws,
                                               bool active, float2 (&A)[NB], float2 (&C)[NB],
                                               int wv, int lane) {
  extern __shared__ float2 smem[];
  constexpr int MAXL = TD_MAX_ROW_PAIRS / 64;   // 16-byte loads per lane for the longest row
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    A[t] = make_float2(0.f, 0.f);
    C[t] = make_float2(0.f, 0.f);
  }
  int4 ent0 = make_int4(0, 0, 0, 0), ent1 = make_int4(0, 0, 0, 0);
  if (active) {
    if (lane < M) ent0 = dtab_d[lane];
    if (lane + 64 < M) ent1 = dtab_d[lane + 64];
  }
  for (int m0 = 0; m0 < M; m0 += mc) {
    const int rows = M - m0 < mc ? M - m0 : mc;
    if (wv < rows) {
      // rows are staged whole: 64 * MAXL pairs per row (ws = 128 * MAXL samples);
      // the matched-filter rows are padded so these loads stay in the allocation
      const float4* src = reinterpret_cast<const float4*>(yrow0 + static_cast<long long>((m0 + wv) >> vshift) * row) + lane;
      float4* dst = reinterpret_cast<float4*>(smem + wv * ws) + lane;
      float4 stage[MAXL];
#pragma unroll
      for (int j = 0; j < MAXL; ++j) stage[j] = src[64 * j];
#pragma unroll
      for (int j = 0; j < MAXL; ++j) dst[64 * j] = stage[j];
    }
    __syncthreads();
    if (active) {
      const float2* cur = smem + lane;
      for (int ml = 0; ml < rows; ++ml) {
        const int m = m0 + ml;
        const int src_lane = m & 63;
        const int4 e4 = m < 64 ? ent0 : ent1;
        const int rel = __builtin_amdgcn_readlane(e4.x, src_lane);
        const float w0 = __int_as_float(__builtin_amdgcn_readlane(e4.y, src_lane));
        const float w1 = __int_as_float(__builtin_amdgcn_readlane(e4.z, src_lane));
        const float2* p = cur + ml * ws + rel;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const float2 y = p[64 * t];
          A[t].x = fmaf(w0, y.x, A[t].x);
          A[t].y = fmaf(w0, y.y, A[t].y);
          C[t].x = fmaf(w1, y.x, C[t].x);
          C[t].y = fmaf(w1, y.y, C[t].y);
        }
      }
    }
    __syncthreads();
  }
}

// b for block t: A[t] + C shifted one sample later (lane 63 takes lane 0 of block t+1).
template <int NB>
__device__ __forceinline__ float2 beam_sample(const float2 (&A)[NB], const float2 (&C)[NB], int t, int lane) {
  const float2 src = (lane == 0 && t + 1 < NB) ? C[t + 1] : C[t];
  return make_float2(A[t].x + from_next_lane(src.x, lane), A[t].y + from_next_lane(src.y, lane));
}

template <int NB, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(TD_WAVES_PER_EU, TD_WAVES_PER_EU))) void das_td_env_kernel(
    const float2* __restrict__ yext, const int4* __restrict__ dtab, const float* __restrict__ taps,
    float* __restrict__ E, long long fstride, int M, int vshift, int D, int Q, int row, int R, int K, int qc, int nqc,
    int ws, int mc, int nwin) {
  extern __shared__ float2 smem[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ndt = (D + NW - 1) / NW;
  // Workgroups are handed to the XCDs round-robin by index: XCD x runs every
  // direction tile of windows (frame, range tile) x, x + TD_XCDS, ... so each
  // staged window is fetched into one L2 only.
  const int bx = blockIdx.x % TD_XCDS;
  int bid = blockIdx.x / TD_XCDS;
  const int dt = bid % ndt;
  const int win = bx + TD_XCDS * (bid / ndt);
  if (win >= nwin) return;
  const int qi = win % nqc;
  const int f = win / nqc;
  const int d = dt * NW + wv;
  const bool active = d < D;
  const long long i0 = static_cast<long long>(qi) * qc * R;

  float2 A[NB], C[NB];
  das_accumulate<NB, NW>(yext + f * fstride + i0, row,
                         dtab + static_cast<long long>(active ? d : 0) * M, M, vshift, mc, ws, active,
                         A, C, wv, lane);

  float* absb = reinterpret_cast<float*>(smem);
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const float2 b = beam_sample<NB>(A, C, t, lane);
    absb[wv * 64 * NB + 64 * t + lane] = __builtin_amdgcn_sqrtf(b.x * b.x + b.y * b.y);
  }
  __syncthreads();
  // low-pass + decimation: lanes over range bins, TD_FIR_DIRS directions per thread
  constexpr int NG = NW / TD_FIR_DIRS;
  for (int idx = threadIdx.x; idx < NG * qc; idx += NW * 64) {
    const int g = idx / qc, q = idx - g * qc;
    const int qq = qi * qc + q;
    if (qq >= Q) continue;
    const float* a = absb + g * 64 * NB + q * R + K - 1;
    float acc[TD_FIR_DIRS];
#pragma unroll
    for (int i = 0; i < TD_FIR_DIRS; ++i) acc[i] = 0.f;
    for (int j = 0; j < K; ++j) {
      const float h = taps[j];
#pragma unroll
      for (int i = 0; i < TD_FIR_DIRS; ++i) acc[i] = fmaf(h, a[i * NG * 64 * NB - j], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < TD_FIR_DIRS; ++i) {
      const int dd = dt * NW + g + NG * i;
      if (dd < D) E[(static_cast<long long>(f) * D + dd) * Q + qq] = acc[i];
    }
  }
}

template <int NB, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(TD_WAVES_PER_EU, TD_WAVES_PER_EU))) void das_td_beam_kernel(
    const float2* __restrict__ yext, const int4* __restrict__ dtab, float2* __restrict__ beam,
    long long fstride, int M, int vshift, int D, int G, int row, int tc, int nbc, int ws, int mc) {
  extern __shared__ float2 smem[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ndt = (D + NW - 1) / NW;
  int bid = blockIdx.x;
  const int dt = bid % ndt;
  bid /= ndt;
  const int ci = bid % nbc;
  const int f = bid / nbc;
  const int d = dt * NW + wv;
  const bool active = d < D;
  const long long i0 = static_cast<long long>(ci) * tc;

  float2 A[NB], C[NB];
  das_accumulate<NB, NW>(yext + f * fstride + i0, row,
                         dtab + static_cast<long long>(active ? d : 0) * M, M, vshift, mc, ws, active,
                         A, C, wv, lane);
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const float2 b = beam_sample<NB>(A, C, t, lane);
    const int s = 64 * t + lane;
    const long long gi = i0 + s;
    if (active && s < tc && gi < G) beam[(static_cast<long long>(f) * D + d) * G + gi] = b;
  }
}

// Envelope of a materialised beam: |b| of a window into LDS, FIR at the
// decimated positions.  One workgroup per (frame, direction, range-bin tile).
constexpr int ENV_WINDOW = 32768;   // floats of |b| staged per workgroup (128 KiB)

__global__ __launch_bounds__(256) void envelope_kernel(const float2* __restrict__ beam,
                                                       const float* __restrict__ taps,
                                                       float* __restrict__ E, int D, int Q, int G,
                                                       int R, int K, int qt_len, int nqt) {
  extern __shared__ float ebuf[];
  const int qt = blockIdx.x % nqt;
  const long long fd = blockIdx.x / nqt;          // f * D + d
  const int q0 = qt * qt_len;
  const int nq = Q - q0 < qt_len ? Q - q0 : qt_len;
  const int w0 = q0 * R;
  const int wl = (nq - 1) * R + K;
  const float2* b = beam + fd * G + w0;
  for (int i = threadIdx.x; i < wl; i += blockDim.x) {
    const float2 v = b[i];
    ebuf[i] = __builtin_amdgcn_sqrtf(v.x * v.x + v.y * v.y);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    const float* a = ebuf + q * R + K - 1;
    float acc = 0.f;
    for (int j = 0; j < K; ++j) acc = fmaf(taps[j], a[-j], acc);
    E[fd * Q + q0 + q] = acc;
  }
}

size_t td_smem_bytes(const sonar_plan_s* p) {
  const size_t stage = static_cast<size_t>(p->td_mc) * p->td_ws * sizeof(float2);
  const size_t absb = static_cast<size_t>(TD_NW) * 64 * TD_NB * sizeof(float);
  return stage > absb ? stage : absb;
}

}  // namespace

hipError_t init_td_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(das_td_env_kernel<TD_NB, TD_NW>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(das_td_beam_kernel<TD_NB, TD_NW>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(envelope_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

hipError_t launch_das_td_env(const sonar_plan_s* p, const float2* yext, int F, float* E, hipStream_t s) {
  const int ndt = (p->D + TD_NW - 1) / TD_NW;
  const size_t smem = td_smem_bytes(p);
  const int nwin = F * p->td_nqc;
  const long long nblk = static_cast<long long>((nwin + TD_XCDS - 1) / TD_XCDS) * TD_XCDS * ndt;
  hipLaunchKernelGGL((das_td_env_kernel<TD_NB, TD_NW>), dim3(static_cast<unsigned>(nblk)), dim3(TD_NW * 64),
                     smem, s, yext, p->d_dtab, p->d_taps, E, p->mf_fstride, p->M << p->td_vshift, p->td_vshift, p->D,
                     p->Q, p->row, p->R, p->K,
                     p->td_qc, p->td_nqc, p->td_ws, p->td_mc, nwin);
  return hipGetLastError();
}

hipError_t launch_das_td_beam(const sonar_plan_s* p, const float2* yext, int F, float2* beam, hipStream_t s) {
  const int ndt = (p->D + TD_NW - 1) / TD_NW;
  const size_t smem = td_smem_bytes(p);
  const long long nblk = static_cast<long long>(F) * p->td_nbc * ndt;
  hipLaunchKernelGGL((das_td_beam_kernel<TD_NB, TD_NW>), dim3(static_cast<unsigned>(nblk)), dim3(TD_NW * 64),
                     smem, s, yext, p->d_dtab, beam, p->mf_fstride, p->M << p->td_vshift, p->td_vshift, p->D, p->G,
                     p->row, p->td_tn, p->td_nbc,
                     p->td_ws, p->td_mc);
  return hipGetLastError();
}

hipError_t launch_envelope(const sonar_plan_s* p, const float2* beam, int F, float* E, hipStream_t s) {
  // K <= ENV_WINDOW is checked at plan creation
  int qt_len = (ENV_WINDOW - p->K) / p->R + 1;
  if (qt_len > p->Q) qt_len = p->Q;
  const int nqt = (p->Q + qt_len - 1) / qt_len;
  const size_t smem = static_cast<size_t>((qt_len - 1) * p->R + p->K) * sizeof(float);
  const long long nblk = static_cast<long long>(F) * p->D * nqt;
  hipLaunchKernelGGL(envelope_kernel, dim3(static_cast<unsigned>(nblk)), dim3(256), smem, s, beam,
                     p->d_taps, E, p->D, p->Q, p->G, p->R, p->K, qt_len, nqt);
  return hipGetLastError();
}
