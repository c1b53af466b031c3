// Time-domain delay-and-sum on BF16 MFMA (§4.1 delay-and-sum toward every
// direction; §4.3 subsampling after the envelope), fused with the envelope:
//
//   b_d[n]  = sum_m w0[d][m] yhat_m[n + o] + w1[d][m] yhat_m[n + o + 1]
//   E[d][q] = sum_j h[j] |b_d[n0 + qR + (K-1)/2 - j]|
//
// The same linear-interpolation result as the FP32 beamformer, computed as a
// dense product.  Directions are grouped into tiles of 32 neighbours (plan
// time, along a Hilbert curve of the direction grid), so within a tile the
// integer offsets o[d][m] of one microphone span only a few samples.  For
// each microphone the tile covers that span with groups of 8 consecutive
// taps; the tap weights form a sparse 32 x K matrix W (two nonzeros per
// direction and microphone) and the samples a Hankel matrix
//   Y[(m, toff + j)][n] = yhat_m[n + toff + j],
// so b = W Y runs on v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  A
// B-operand fragment (8 consecutive taps of one sample) is 8 consecutive
// samples of one row.  The 32 columns of an output tile are samples
// 4c + rho of one residue rho, and the tap groups used for residue rho start
// at t0 with t0 + rho = 0 mod 4, so every fragment read starts on an 8-byte
// boundary.
//
// Precision: weights and samples are each carried as two BF16 terms
// (hi = bf16(v), lo = bf16(v - hi)); the product keeps hi*hi + hi*lo + lo*hi
// (the dropped lo*lo term is below 2^-16 relative), real and imaginary parts
// separately, so each K-chunk costs six MFMAs per 32 x 32 output tile.  The
// matched filter writes the samples already split, as four BF16 planes per
// microphone (re hi, re lo, im hi, im lo), so staging a tile is a plain copy.
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int MT_FIR_DIRS = 4;   // directions per thread in the low-pass stage

// 8 BF16 values at an 8-byte aligned LDS address
__device__ __forceinline__ bf16x8 lds_frag(const unsigned short* p) {
  const uint2 a = *reinterpret_cast<const uint2*>(p);
  const uint2 b = *reinterpret_cast<const uint2*>(p + 4);
  return __builtin_bit_cast(bf16x8, make_uint4(a.x, a.y, b.x, b.y));
}

// Workgroup: one tile of 32 directions x NWAVE * 128 beam samples of one frame.
// Wavefront wv owns residue rho = wv % MT_RES of the 512-sample block
// wv / MT_RES: 4 output tiles of 32 samples (4c + rho).
template <int NWAVE>
__global__ __launch_bounds__(NWAVE * 64) void das_mfma_env_kernel(
    const unsigned short* __restrict__ planes, long long fstride, const int2* __restrict__ gtab,
    const uint4* __restrict__ wtab, const int2* __restrict__ kcr, const int* __restrict__ perm,
    const float* __restrict__ taps, float* __restrict__ E, int M, int D, int Q, int row, int R, int K, int qc,
    int nqt, int ntiles, int nx, int tpx, int gmax, int kcmax, int nmc, int wrow) {
  extern __shared__ unsigned short sm[];    // 4 planes x MT_MICS rows x wrow (re hi, re lo, im hi, im lo)
  constexpr int NS = NWAVE * 128;            // beam samples per workgroup
  constexpr int NT = NWAVE * 64;
  static_assert(NWAVE % MT_RES == 0, "wavefronts come in groups of MT_RES residues");
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int rho = wv % MT_RES;
  // Workgroups are handed to the XCDs round-robin by index: XCD x = index % nx
  // keeps the weights of its own tpx direction tiles in its L2 and runs them
  // back to back on each staged window (frame f, range tile qt).
  const int bx = blockIdx.x % nx;
  int bid = blockIdx.x / nx;
  const int tile = bx * tpx + bid % tpx;
  if (tile >= ntiles) return;
  bid /= tpx;
  const int qt = bid % nqt;
  const int f = bid / nqt;
  const int s0 = qt * qc * R;                // first window sample of the tile (a multiple of 4)
  const int s0a = s0 & ~7;                   // staged from here: 16-byte aligned rows
  // first sample of the wavefront, as an index into the staged rows
  const int sb = (wv / MT_RES) * (32 * 4 * MT_RES) + rho + (s0 - s0a);
  const int plane = MT_MICS * wrow;
  const unsigned short* src = planes + f * fstride + s0a;

  f32x16 cre[4], cim[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    cre[nt] = f32x16{};
    cim[nt] = f32x16{};
  }

  for (int mc = 0; mc < nmc; ++mc) {
    const int m0 = mc * MT_MICS;
    const int rows = M - m0 < MT_MICS ? M - m0 : MT_MICS;
    // stage rows m0.. of this frame, samples [s0a, s0a + wrow) of each BF16 plane:
    // segment sg = 4 ml + c is plane c of microphone m0 + ml, copied in 16-byte chunks
    {
      constexpr int B = 8;
      const int cw = wrow >> 3;
      const int nseg = 4 * rows;
      const int total = nseg * cw;
      const int dq = NT / cw, dr = NT % cw;
      int sg = threadIdx.x / cw, k = threadIdx.x - sg * cw;
      for (int base = threadIdx.x; base < total; base += NT * B) {
        uint4 v[B];
        int dst[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
          const bool ok = base + i * NT < total;
          const int sgc = ok ? sg : nseg - 1, kc = ok ? k : cw - 1;
          v[i] = *reinterpret_cast<const uint4*>(src + static_cast<long long>(m0 * 4 + sgc) * row + 8 * kc);
          dst[i] = ok ? (sgc & 3) * plane + (sgc >> 2) * wrow + 8 * kc : -1;
          k += dr;
          sg += dq;
          if (k >= cw) {
            k -= cw;
            sg += 1;
          }
        }
#pragma unroll
        for (int i = 0; i < B; ++i)
          if (dst[i] >= 0) *reinterpret_cast<uint4*>(sm + dst[i]) = v[i];
      }
    }
    __syncthreads();
    const int li = tile * MT_RES + rho;
    const int2 kr = kcr[(tile * nmc + mc) * MT_RES + rho];
    if (kr.x < kr.y) {
      const uint4* wt = wtab + static_cast<long long>(li) * kcmax * 128 + lane;
      const int2* gt = gtab + static_cast<long long>(li) * gmax + (lane >> 5);
      uint4 ah_next = wt[kr.x * 128], al_next = wt[kr.x * 128 + 64];
      int2 g_next = gt[2 * kr.x];
      for (int kc = kr.x; kc < kr.y; ++kc) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, ah_next);
        const bf16x8 al = __builtin_bit_cast(bf16x8, al_next);
        const int2 g = g_next;
        if (kc + 1 < kr.y) {
          ah_next = wt[(kc + 1) * 128];
          al_next = wt[(kc + 1) * 128 + 64];
          g_next = gt[2 * (kc + 1)];
        }
        const unsigned short* p = sm + (g.x - m0) * wrow + g.y + sb + 4 * (lane & 31);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const bf16x8 brh = lds_frag(p + 128 * nt);
          const bf16x8 brl = lds_frag(p + plane + 128 * nt);
          const bf16x8 bih = lds_frag(p + 2 * plane + 128 * nt);
          const bf16x8 bil = lds_frag(p + 3 * plane + 128 * nt);
          cre[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, brh, cre[nt], 0, 0, 0);
          cim[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bih, cim[nt], 0, 0, 0);
          cre[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, brl, cre[nt], 0, 0, 0);
          cim[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bil, cim[nt], 0, 0, 0);
          cre[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, brh, cre[nt], 0, 0, 0);
          cim[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bih, cim[nt], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  // |b| of the tile into LDS: lane holds rows 8(v/4) + 4(lane/32) + v%4 (directions)
  // of column lane%32 (window sample sw + 128 nt + 4 column) for each output tile
  float* absb = reinterpret_cast<float*>(sm);
  const int sw = (wv / MT_RES) * (32 * 4 * MT_RES) + rho;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int s = sw + 128 * nt + 4 * (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int dl = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      absb[dl * NS + s] = __builtin_amdgcn_sqrtf(cre[nt][v] * cre[nt][v] + cim[nt][v] * cim[nt][v]);
    }
  }
  __syncthreads();
  // low-pass + decimation: lanes run over range bins (coalesced stores), each
  // thread accumulates MT_FIR_DIRS directions dl = g + 8 i at once
  constexpr int NG = 32 / MT_FIR_DIRS;
  for (int it = threadIdx.x; it < NG * qc; it += NWAVE * 64) {
    const int g = it / qc, q = it - g * qc;
    const int qq = qt * qc + q;
    if (qq >= Q) continue;
    const float* a = absb + g * NS + q * R + K - 1;
    float acc[MT_FIR_DIRS];
#pragma unroll
    for (int i = 0; i < MT_FIR_DIRS; ++i) acc[i] = 0.f;
    for (int j = 0; j < K; ++j) {
      const float h = taps[j];
#pragma unroll
      for (int i = 0; i < MT_FIR_DIRS; ++i) acc[i] = fmaf(h, a[i * NG * NS - j], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < MT_FIR_DIRS; ++i) {
      const int d = perm[tile * 32 + g + NG * i];
      if (d >= 0) E[(static_cast<long long>(f) * D + d) * Q + qq] = acc[i];
    }
  }
}

}  // namespace

size_t mt_smem_bytes(const sonar_plan_s* p) {
  const size_t planes = 4 * static_cast<size_t>(MT_MICS) * p->mt_wrow * sizeof(unsigned short);
  const size_t absb = 32 * static_cast<size_t>(MT_NWAVE * 128) * sizeof(float);
  return planes > absb ? planes : absb;
}

hipError_t init_mt_kernel_attributes() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(das_mfma_env_kernel<MT_NWAVE>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

hipError_t launch_das_mfma_env(const sonar_plan_s* p, const float2* yext, int F, float* E, hipStream_t s) {
  const int nx = p->mt_ntiles < MT_XCDS ? p->mt_ntiles : MT_XCDS;
  const int tpx = (p->mt_ntiles + nx - 1) / nx;
  const long long nblk = static_cast<long long>(F) * p->mt_nqt * nx * tpx;
  // the BF16 planes of frame f follow its M complex rows
  const unsigned short* planes = reinterpret_cast<const unsigned short*>(yext + static_cast<long long>(p->M) * p->row);
  hipLaunchKernelGGL((das_mfma_env_kernel<MT_NWAVE>), dim3(static_cast<unsigned>(nblk)), dim3(MT_NWAVE * 64),
                     mt_smem_bytes(p), s, planes, 4 * p->mf_fstride, p->d_mt_g,
                     reinterpret_cast<const uint4*>(p->d_mt_w), p->d_mt_kcr,
                     p->d_mt_perm, p->d_taps, E, p->M, p->D, p->Q, p->row, p->R, p->K, p->mt_qc, p->mt_nqt,
                     p->mt_ntiles, nx, tpx, p->mt_gmax, p->mt_kcmax, p->mt_nmc, p->mt_wrow);
  return hipGetLastError();
}
