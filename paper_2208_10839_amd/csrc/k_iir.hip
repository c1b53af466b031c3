// IIR reading of the envelope filter (§4.3: the CPU implementation filters with
// Butterworth designs run by a causal lfilter): for every beam-window row,
//   y = causal IIR of |b| from zero state at window position 0,  E[q] = y[qR + (K-1)/2].
// The filter is a cascade of second-order sections, held as one state-space system
// s[i+1] = A s[i] + B x[i], y[i] = C s[i] + D x[i] of dimension NS (2 per section),
// built and raised to powers on the host in FP64.
//
// One wavefront per row: lane c owns the chunk [c L - o, c L + L - o) of the window, where
// L is a multiple of IIR_TB with 64 L >= G' + 15 and o < 16 is the row's offset from a
// 128-byte boundary in samples, so every chunk starts on a 128-byte boundary (positions
// below 0 are zero input, which leaves the zero start state as it is).  The row is read
// in steps of IIR_TB samples per chunk: the wave loads 64 chunks x IIR_TB consecutive
// samples (16 lanes per aligned 128-byte line) into LDS, then each lane runs its chunk's
// IIR_TB samples from there, the next step's loads in flight meanwhile.  Pass 1 runs
// each chunk from zero state to get its end state e_c; a Hillis-Steele scan over the lanes with the tables A^(L 2^k) turns these into the
// true start state of every chunk (start_c = sum_{j<c} A^(L (c-1-j)) e_j); pass 2 reruns
// each chunk from its start state and writes the subsampled outputs.
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace {

constexpr int IIR_TB = 16;

// samples [t0, t0 + IIR_TB) of every chunk into registers (0 outside the row): value j of
// lane l is sample t0 + l % 16 of chunk 4 j + l / 16
__device__ __forceinline__ void load_stage(const float2* __restrict__ b, float2* v, int t0, int L, int G, int off,
                                           int lane) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int c = 4 * j + (lane >> 4), tt = lane & 15;
    const int i = c * L - off + t0 + tt;
    v[j] = (i >= 0 && i < G) ? b[i] : make_float2(0.f, 0.f);
  }
}

// their magnitudes into seg[chunk][.]
__device__ __forceinline__ void store_abs(const float2* v, float (*seg)[IIR_TB + 1], int lane) {
#pragma unroll
  for (int j = 0; j < 16; ++j) seg[4 * j + (lane >> 4)][lane & 15] = sqrtf(v[j].x * v[j].x + v[j].y * v[j].y);
}

template <int NS>
__device__ __forceinline__ void step(const float* A, const float* B, float* s, float x) {
  float t[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    float acc = B[i] * x;
#pragma unroll
    for (int j = 0; j < NS; ++j) acc = fmaf(A[i * NS + j], s[j], acc);
    t[i] = acc;
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) s[i] = t[i];
}

template <int NS>
__global__ __launch_bounds__(64) void iir_env_kernel(const float2* __restrict__ beam, const float* __restrict__ tab,
                                                     float* __restrict__ E, int G, int Q, int R, int hk, int L) {
  __shared__ float t[IIR_TAB_LEN];
  __shared__ float seg[64][IIR_TB + 1];
  const int lane = threadIdx.x;
  for (int i = lane; i < IIR_TAB_LEN; i += 64) t[i] = tab[i];
  __syncthreads();
  const float* A = t;
  const float* B = t + NS * NS;
  const float* C = B + NS;
  const float Dd = C[NS];
  const float* Apow = t + IIR_POW_OFFSET;   // [6][NS][NS]
  const long long row = blockIdx.x;
  const float2* b = beam + row * G;
  const int off = static_cast<int>((reinterpret_cast<uintptr_t>(b) >> 3) & 15);
  const int i0 = lane * L - off;
  const int i1 = i0 + L < G ? i0 + L : G;

  float s[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) s[i] = 0.f;
  // each stage's loads are issued before the previous stage's recurrence runs
  float2 v[16];
  load_stage(b, v, 0, L, G, off, lane);
  for (int t0 = 0; t0 < L; t0 += IIR_TB) {
    store_abs(v, seg, lane);
    __syncthreads();
    if (t0 + IIR_TB < L) load_stage(b, v, t0 + IIR_TB, L, G, off, lane);
    for (int tt = 0; tt < IIR_TB; ++tt)
      if (i0 + t0 + tt >= 0 && i0 + t0 + tt < i1) step<NS>(A, B, s, seg[lane][tt]);
    __syncthreads();
  }
  // inclusive scan of the chunk end states: V_c = sum_{j<=c} A^(L (c-j)) e_j
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int off = 1 << k;
    float o[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) o[i] = __shfl_up(s[i], off);
    if (lane >= off) {
      const float* P = Apow + k * NS * NS;
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        float acc = s[i];
#pragma unroll
        for (int j = 0; j < NS; ++j) acc = fmaf(P[i * NS + j], o[j], acc);
        s[i] = acc;
      }
    }
  }
  // start state of chunk c = V_{c-1}
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const float v = __shfl_up(s[i], 1);
    s[i] = lane == 0 ? 0.f : v;
  }
  float* e = E + row * Q;
  load_stage(b, v, 0, L, G, off, lane);
  for (int t0 = 0; t0 < L; t0 += IIR_TB) {
    store_abs(v, seg, lane);
    __syncthreads();
    if (t0 + IIR_TB < L) load_stage(b, v, t0 + IIR_TB, L, G, off, lane);
    for (int tt = 0; tt < IIR_TB; ++tt) {
      const int i = i0 + t0 + tt;
      if (i >= i1) break;
      const float x = seg[lane][tt];
      if (i >= hk && (i - hk) % R == 0) {
        const int q = (i - hk) / R;
        if (q < Q) {
          float y = Dd * x;
#pragma unroll
          for (int j = 0; j < NS; ++j) y = fmaf(C[j], s[j], y);
          e[q] = y;
        }
      }
      step<NS>(A, B, s, x);
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_iir_envelope(const sonar_plan_s* p, const float2* beam, int F, float* E, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(static_cast<long long>(F) * p->D));
  const int L = p->iir_chunk;
  switch (p->iir_ns) {
    case 2: hipLaunchKernelGGL(iir_env_kernel<2>, grid, dim3(64), 0, s, beam, p->d_iir, E, p->G, p->Q, p->R, p->hk, L); break;
    case 4: hipLaunchKernelGGL(iir_env_kernel<4>, grid, dim3(64), 0, s, beam, p->d_iir, E, p->G, p->Q, p->R, p->hk, L); break;
    case 6: hipLaunchKernelGGL(iir_env_kernel<6>, grid, dim3(64), 0, s, beam, p->d_iir, E, p->G, p->Q, p->R, p->hk, L); break;
    case 8: hipLaunchKernelGGL(iir_env_kernel<8>, grid, dim3(64), 0, s, beam, p->d_iir, E, p->G, p->Q, p->R, p->hk, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
