// Frequency-domain beamformer (§4.1 delay-and-sum toward every direction of
// interest, with each channel's delay applied exactly as a per-bin phase) and
// its envelope (§4.1 envelope; §4.3 subsampling after envelope detection):
//
//   B_d[k]  = sum_m (1/M) exp(-2 pi i k Dl[d][m] / P) Yhat_m[k]      (per-bin GEMM)
//   b_d[n]  = IDFT_P(B_d)[n]                                          (per direction)
//   E[d][q] = sum_j h[j] |b_d[n0 + qR + (K-1)/2 - j]|
//
// Per frequency bin the product over microphones is a small complex GEMM
// (directions x microphones) x (microphones x frames): it is dense when many
// frames share one geometry, and runs on MFMA.  The steering matrix is never
// stored: each lane rebuilds its slice bin by bin from an FP64-anchored phasor
// and an FP64-derived per-bin rotation.
//
// The stored spectra are band-limited to kb bins starting at k_lo, so the
// inverse transform of one direction runs as R' = P / L polyphase transforms
// of L points (L >= kb - 1):
//   b_d[R' a + r] = (1/P) exp(2 pi i k_lo n / P)
//                   ( IDFT'_L( B'[k'] exp(2 pi i k' r / P) )[a] + B'[L] exp(2 pi i r / R') ),
// with B'[k'] = B_d[k_lo + k'] and IDFT' unnormalised; the last term exists
// only when kb = L + 1.  The envelope needs |b| only, so the exp(2 pi i k_lo n/P)
// factor drops out of the fused kernel.
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "plan.hpp"


using namespace fftk;

namespace {

int ilog2_host(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int MODE_FP32 = SONAR_BF_FD_FP32;
constexpr int MODE_BF16 = SONAR_BF_FD_BF16;
constexpr int MODE_BF16X3 = SONAR_BF_FD_BF16X3;

// ---------------------------------------------------------------------------
// Per-bin GEMM.  Workgroup: 4 wavefronts x 16 directions, FD_GEMM_BINS_WG bins,
// up to 16 frames.  Lane l builds the steering values of direction l % 16 of
// its wavefront for 8 microphones and supplies the samples of frame l % 16 for
// the same 8 microphones, matching the MFMA operand layouts:
//   v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16) + j], B[8(l/16) + j][l%16]
//   v_mfma_f32_16x16x4_f32:   lane l holds A[l%16][l/16],        B[l/16][l%16]
// (microphone of slot j: 8(l/16) + j for BF16, 4j + l/16 for FP32 MFMA), and
// receives D[4(l/16) + i][l%16] (direction 4(l/16) + i, frame l%16).
// Real embedding: Cr = Ar Yr - Ai Yi, Ci = Ai Yr + Ar Yi.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bf16x8 to_bf16x8(const float (&v)[8]) {
  bf16x8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = static_cast<__bf16>(v[j]);
  return r;
}

// hi = bf16(v), lo = bf16(v - hi)
__device__ __forceinline__ void split_bf16x8(const float (&v)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 h = static_cast<__bf16>(v[j]);
    hi[j] = h;
    lo[j] = static_cast<__bf16>(v[j] - static_cast<float>(h));
  }
}

// Lane exchanges inside a quad (4 consecutive lanes) by DPP: the value of lane q ^ 1, resp. q ^ 2.
__device__ __forceinline__ float dpp_xor1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_xor2(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, true));
}

// 4 x 4 transpose of 16-byte elements over the lanes of a quad: afterwards lane q holds in e[j] what
// lane j held in e[q].  Two butterfly steps; in step b a lane takes from lane q ^ b the element p ^ b
// for every p whose bit b differs from q's.  All four lanes of every quad must be active.
__device__ __forceinline__ void quad_transpose(f32x4 (&e)[4], int q) {
  const bool o1 = (q & 1) != 0, o2 = (q & 2) != 0;
#pragma unroll
  for (int p = 0; p < 4; p += 2) {
    f32x4 lo = e[p], hi = e[p + 1];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float plo = dpp_xor1(lo[c]), phi = dpp_xor1(hi[c]);
      e[p][c] = o1 ? phi : lo[c];
      e[p + 1][c] = o1 ? hi[c] : plo;
    }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    f32x4 lo = e[p], hi = e[p + 2];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float plo = dpp_xor2(lo[c]), phi = dpp_xor2(hi[c]);
      e[p][c] = o2 ? phi : lo[c];
      e[p + 2][c] = o2 ? hi[c] : plo;
    }
  }
}

// Workgroup: 4 wavefronts x 16 directions, FD_GEMM_BINS_WG bins in chunks of 8,
// 16 frames.  The samples of a chunk (16 frames x 8 bins x 32 microphones)
// are staged once in LDS and shared by the four wavefronts.  Steering values
// restart at every chunk from an anchor exp(-2 pi i k Dl / P) whose phase is
// reduced in FP64, then advance bin by bin with the per-(d, m) rotation
// exp(-2 pi i Dl / P) taken from the plan table (at most 7 FP32 rotations).
constexpr int CHB = 8;                  // bins per chunk
// bins per workgroup: one chunk, so a workgroup's stores drain while other workgroups compute (a
// workgroup that looped over chunks would wait for its stores before loading the next chunk's samples,
// since loads and stores retire in issue order)
constexpr int FD_GEMM_BINS_WG = CHB;
constexpr int YS_FRAME = CHB * 32 + 2;  // float2 per frame row in LDS (padded)
// BF16 modes: the staged samples are split once into four BF16 planes (re hi, re lo, im hi, im lo),
// [plane][frame][bin][mic] with a 16-byte pad per frame row, so every wavefront reads its operands as
// 16-byte fragments instead of converting them itself
constexpr int YB_FRAME = CHB * 32 + 8;  // 16-bit words per frame row
constexpr int YB_PLANE = FD_GEMM_FRAMES * YB_FRAME;

template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void fd_gemm_kernel(
    const float2* __restrict__ band, const double* __restrict__ dl, const float2* __restrict__ step,
    float2* __restrict__ bspec, int F, int D, int M, int kb, int kb_pad, int k_lo, int P, int nbt, int ndt,
    int nyt) {
  constexpr bool SPLIT = MODE != MODE_FP32;   // samples as BF16 hi + lo terms
  __shared__ float2 ys[SPLIT ? 1 : FD_GEMM_FRAMES * YS_FRAME];
  __shared__ uint4 ybv[SPLIT ? 4 * YB_PLANE / 8 : 1];
  unsigned short* yb = reinterpret_cast<unsigned short*>(ybv);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  // Workgroups go to the XCDs round-robin by index.  Each XCD takes a contiguous block of sample
  // tiles (bin tile bt, frame tile ft) in pairs of neighbouring bin tiles, and runs every direction
  // tile of a pair back to back, the two sample tiles alternating: the XCD reads each sample tile
  // from HBM once (its other ndt - 1 readers find it in the XCD's L2), and the two 64-byte halves of
  // each 128-byte line of the beam spectra are written by consecutive workgroups of one L2, so whole
  // lines reach HBM (a lone half costs a fill read).
  const int xcd = blockIdx.x % FD_XCDS;
  const int jx = blockIdx.x / FD_XCDS;       // position in this XCD's sequence
  const int pr = jx % (2 * ndt);             // position within the pair's run
  const int dt = pr >> 1;
  const int yt = xcd * (static_cast<int>(gridDim.x) / ndt / FD_XCDS) + 2 * (jx / (2 * ndt)) + (pr & 1);
  if (yt >= nyt) return;
  const int bt = yt % nbt;
  const int ft = yt / nbt;
  const int r16 = lane & 15, grp = lane >> 4;
  const int d_st = dt * FD_GEMM_DIRS + wv * 16 + r16;    // direction this lane steers
  const bool d_ok = d_st < D;
  const double invP = 1.0 / static_cast<double>(P);
  const float invM = 1.0f / static_cast<float>(M);   // the array mean's 1/M (one rounding, as the steering's)

  for (int k0 = bt * FD_GEMM_BINS_WG; k0 < (bt + 1) * FD_GEMM_BINS_WG && k0 < kb; k0 += CHB) {
    f32x4 cr[CHB], ci[CHB];
#pragma unroll
    for (int b = 0; b < CHB; ++b) {
      cr[b] = f32x4{0.f, 0.f, 0.f, 0.f};
      ci[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    for (int mc = 0; mc < M; mc += 32) {
      // stage samples: ys[f][b][m] = band[frame][k0 + b][mc + m].  Each thread
      // issues its 16 loads back to back; out-of-range slots read a clamped
      // (valid) address and are zeroed, so no load sits behind a branch.
      __syncthreads();
      {
        float2 y[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int e = threadIdx.x + 256 * i;
          const int f = e / (CHB * 32), b = (e / 32) % CHB, m = e % 32;
          const int fg = ft * FD_GEMM_FRAMES + f;
          const int fc = fg < F ? fg : F - 1;
          const int kc = k0 + b < kb ? k0 + b : kb - 1;
          const int mcl = mc + m < M ? mc + m : M - 1;
          y[i] = band[(static_cast<long long>(fc) * kb + kc) * M + mcl];
          if (!(fg < F && k0 + b < kb && mc + m < M)) y[i] = make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int e = threadIdx.x + 256 * i;
          const int f = e / (CHB * 32), b = (e / 32) % CHB, m = e % 32;
          if constexpr (SPLIT) {
            const __bf16 rh = static_cast<__bf16>(y[i].x), ih = static_cast<__bf16>(y[i].y);
            const __bf16 rl = static_cast<__bf16>(y[i].x - static_cast<float>(rh));
            const __bf16 il = static_cast<__bf16>(y[i].y - static_cast<float>(ih));
            const int at = f * YB_FRAME + b * 32 + m;
            yb[at] = __builtin_bit_cast(unsigned short, rh);
            yb[YB_PLANE + at] = __builtin_bit_cast(unsigned short, rl);
            yb[2 * YB_PLANE + at] = __builtin_bit_cast(unsigned short, ih);
            yb[3 * YB_PLANE + at] = __builtin_bit_cast(unsigned short, il);
          } else {
            ys[f * YS_FRAME + b * 32 + m] = y[i];
          }
        }
      }
      __syncthreads();
      // the delays and rotations of this lane's 8 microphones, all loads issued before any is used
      // (a slot outside the array reads a valid entry and is zeroed)
      float phr[8], phi[8], str[8], sti[8];
      double dlv[8];
      float2 stv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int m = mc + (MODE == MODE_FP32 ? 4 * j + grp : 8 * grp + j);
        const long long at = static_cast<long long>(d_ok ? d_st : 0) * M + (m < M ? m : 0);
        dlv[j] = dl[at];
        stv[j] = step[at];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int m = mc + (MODE == MODE_FP32 ? 4 * j + grp : 8 * grp + j);
        const double tt = static_cast<double>(k_lo + k0) * dlv[j] * invP;
        const float fr = static_cast<float>(tt - floor(tt));
        float s, c;
        sincospif(-2.0f * fr, &s, &c);
        const bool ok = d_ok && m < M;
        phr[j] = ok ? c * invM : 0.f;
        phi[j] = ok ? s * invM : 0.f;
        str[j] = ok ? stv[j].x : 0.f;
        sti[j] = ok ? stv[j].y : 0.f;
      }
#pragma unroll
      for (int b = 0; b < CHB; ++b) {
        float ar[8], ai[8], nai[8], yr[8], yi[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          ar[j] = phr[j];
          ai[j] = phi[j];
          nai[j] = -phi[j];
          const float nr = phr[j] * str[j] - phi[j] * sti[j];
          const float ni = phr[j] * sti[j] + phi[j] * str[j];
          phr[j] = nr;
          phi[j] = ni;
          if constexpr (!SPLIT) {
            const float2 y = ys[r16 * YS_FRAME + b * 32 + 4 * j + grp];
            yr[j] = y.x;
            yi[j] = y.y;
          }
        }
        // BF16 modes: this lane's 8 microphones of frame r16, bin b, from each plane
        const unsigned short* yp = yb + r16 * YB_FRAME + b * 32 + 8 * grp;
        auto yfrag = [&](int plane) { return *reinterpret_cast<const bf16x8*>(yp + plane * YB_PLANE); };
        if constexpr (MODE == MODE_FP32) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            cr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[j], yr[j], cr[b], 0, 0, 0);
            cr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai[j], yi[j], cr[b], 0, 0, 0);
            ci[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[j], yr[j], ci[b], 0, 0, 0);
            ci[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[j], yi[j], ci[b], 0, 0, 0);
          }
        } else if constexpr (MODE == MODE_BF16) {
          // steering in one BF16 term, samples in two (hi + lo): two products
          const bf16x8 Ar = to_bf16x8(ar), Ai = to_bf16x8(ai), nAi = to_bf16x8(nai);
          const bf16x8 Yrh = yfrag(0), Yrl = yfrag(1), Yih = yfrag(2), Yil = yfrag(3);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar, Yrh, cr[b], 0, 0, 0);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar, Yrl, cr[b], 0, 0, 0);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nAi, Yih, cr[b], 0, 0, 0);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nAi, Yil, cr[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ai, Yrh, ci[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ai, Yrl, ci[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar, Yih, ci[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar, Yil, ci[b], 0, 0, 0);
        } else {
          bf16x8 Arh, Arl, Aih, Ail, nAih, nAil;
          split_bf16x8(ar, Arh, Arl);
          split_bf16x8(ai, Aih, Ail);
          split_bf16x8(nai, nAih, nAil);
          const bf16x8 Yrh = yfrag(0), Yrl = yfrag(1), Yih = yfrag(2), Yil = yfrag(3);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Arh, Yrh, cr[b], 0, 0, 0);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Arh, Yrl, cr[b], 0, 0, 0);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Arl, Yrh, cr[b], 0, 0, 0);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nAih, Yih, cr[b], 0, 0, 0);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nAih, Yil, cr[b], 0, 0, 0);
          cr[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nAil, Yih, cr[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aih, Yrh, ci[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aih, Yrl, ci[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ail, Yrh, ci[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Arh, Yih, ci[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Arh, Yil, ci[b], 0, 0, 0);
          ci[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Arl, Yih, ci[b], 0, 0, 0);
        }
      }
    }
    // Lane holds (direction 4 grp + i, frame r16) for the chunk's CHB = 8 bins: one 64-byte segment of
    // each of 4 output rows.  A quad transpose gives lane q of each quad the bins 2q, 2q + 1 of the
    // quad's rows (its 4 frames x the same direction), so each store writes 16 whole 64-byte segments
    // (4 lanes each) instead of 64 scattered 16-byte pieces.  The stores are non-temporal: the beam
    // spectra stream out without evicting the band spectra that the sample tile's other direction
    // tiles still read from L2.
    static_assert(CHB == 8, "one 16-byte bin pair per quad lane");
    const int q = lane & 3;
    const int f_quad = ft * FD_GEMM_FRAMES + (r16 & ~3);   // frame held by lane 0 of the quad
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f32x4 e[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) e[b] = f32x4{cr[2 * b][i], ci[2 * b][i], cr[2 * b + 1][i], ci[2 * b + 1][i]};
      quad_transpose(e, q);                                  // e[j]: frame f_quad + j, bins 2q, 2q + 1
      const int d_out = dt * FD_GEMM_DIRS + wv * 16 + 4 * grp + i;
      if (d_out < D) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int f = f_quad + j;
          if (f < F)
            __builtin_nontemporal_store(e[j], reinterpret_cast<f32x4*>(bspec + (static_cast<long long>(f) * D + d_out) * kb_pad + k0 + 2 * q));
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Polyphase inverse transforms.
// ---------------------------------------------------------------------------

template <int LOGL>
struct FdTw {
  static constexpr int L = 1 << LOGL;
  static constexpr int LH = L / 64 > 0 ? L / 64 : 1;
};

// exp(-2 pi i e / P) from the plan's two-level P tables (in global memory)
__device__ __forceinline__ float2 twp(const float2* __restrict__ twp_hi, const float2* __restrict__ twp_lo, int e) {
  return cmul(twp_hi[e >> 6], twp_lo[e & 63]);
}

// Loads the phase-r input of one direction: thread t holds, for slot s (k' = t + s L/16),
// the fold sum_f B'[k' + f L] exp(2 pi i (k' + f L) r / P) over every stored bin of that class.
template <int LOGL>
__device__ __forceinline__ void load_phase(const float2* __restrict__ in, int kb, int r, int P,
                                           const float2* twp_hi, const float2* twp_lo, float2 (&v)[16], int tid) {
  constexpr int L = 1 << LOGL;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    float2 acc = make_float2(0.f, 0.f);
    for (int k = tid + s * (L / 16); k < kb; k += L) {
      float2 x = in[k];
      if (r != 0) x = cmul(x, cconj(twp(twp_hi, twp_lo, (k * r) & (P - 1))));
      acc = cadd(acc, x);
    }
    v[s] = acc;
  }
}

// One direction of one frame per workgroup: the fused inverse transform and envelope.
// The stored bins are read once into registers (NFOLD per slot, k' = t + s L/16 + f L).  For each
// phase r the folded, rotated spectrum goes through one L-point inverse transform in LDS; the
// magnitudes |b[R' a + r]| of that phase replace the transform's data in LDS, and each range bin q
// (owned by thread q mod T, its sum kept in LDS) adds the low-pass taps j that read phase r:
//   E[q] = sum_j h[j] |b[n_start + qR + K - 1 - j]|,   tap j reads phase (n_start + qR + K - 1 - j) mod R'.
// No copy of the whole beam window is kept, so the window length is not bounded by LDS (Q floats
// are: the range-bin sums).
//
// Costs kept off the vector ALUs:
//  * the phase rotation exp(+2 pi i k r / P) of slot s, fold f is A_t exp(+2 pi i s r / (16 R'))
//    exp(+2 pi i f r / R'), with A_t = exp(+2 pi i t r / P) (one lookup per thread and phase), the
//    second factor from an LDS table of 16 R' entries and the third the same for every thread, so the
//    folds are combined first (a short DFT over f with uniform factors) and rotated once;
//  * the taps are rearranged by phase class, hc[c][u] = h[c + R' u] (zero past K), and the phase's
//    magnitudes carry a circular halo of H entries on both sides, so range bin q reads its taps and
//    samples as two runs, hc[c_q][u] and mag[a_q - u] for u < ceil(K / R'), with no index wrapping.
template <int LOGL, int NFOLD>
__global__ __launch_bounds__((1 << LOGL) / 16) void fd_ifft_env_kernel(
    const float2* __restrict__ bspec, const float2* __restrict__ tw_g, const float* __restrict__ taps,
    float* __restrict__ E, int kb, int kb_pad, int Rp, int logRp, int P, int n_start, int Q, int R, int K) {
  using S = FftShape<LOGL>;
  constexpr int L = S::NF;
  constexpr int T = S::T;
  constexpr int LH = FdTw<LOGL>::LH;
  constexpr bool TW1 = L >= 256;              // pass-1 twiddles from a table (built once per workgroup)
  __shared__ float2 buf[S::LDS_ELEMS];
  __shared__ float2 tw[LH + 64];
  __shared__ float2 tw1[TW1 ? 256 : 1];
  extern __shared__ float2 dyn[];             // 16 R' phase factors, the classed taps / P, the Q range-bin sums
  float2* tws = dyn;
  const int nu = (K + Rp - 1) >> logRp;      // taps per phase class
  float* hc = reinterpret_cast<float*>(dyn + 16 * Rp);
  float* accq = hc + Rp * nu;
  const int H = ((K - 1) / 2 >> logRp) + 2;  // halo of the phase magnitudes (samples read past [0, L))
  const int tid = threadIdx.x;
  const long long fd = blockIdx.x;            // f * D + d
  for (int i = tid; i < LH + 64; i += T) tw[i] = tw_g[i];
  if constexpr (TW1) pass1_twiddles<LOGL, true>(tw1, tw_g, tw_g + LH, tid, T);
  const float2* twp_hi = tw_g + LH + 64;
  const float2* twp_lo = twp_hi + P / 64 + 1;
  for (int i = tid; i < 16 * Rp; i += T) tws[i] = cconj(twp(twp_hi, twp_lo, i * (L / 16)));   // exp(+2 pi i i / (16 R'))
  // the taps carry the transform's 1/P (a power of two: the products are exactly those of h[j] |b| / P)
  const float invP = 1.0f / static_cast<float>(P);
  for (int i = tid; i < Rp * nu; i += T) {
    const int c = i / nu, u = i - c * nu, j = c + Rp * u;
    hc[i] = j < K ? taps[j] * invP : 0.f;
  }
  for (int q = tid; q < Q; q += T) accq[q] = 0.f;
  const float2* in = bspec + fd * kb_pad;
  float2 bin[NFOLD][16];
#pragma unroll
  for (int f = 0; f < NFOLD; ++f)
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int k = tid + s * (L / 16) + f * L;
      bin[f][s] = k < kb ? in[k] : make_float2(0.f, 0.f);
    }
  float* mr = reinterpret_cast<float*>(buf) + H;   // |b| of the current phase, index a in [-H, L + H)
  __syncthreads();                                  // tables in LDS

  for (int r = 0; r < Rp; ++r) {
    float2 v[16];
    if (r == 0) {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        float2 x = bin[0][s];
#pragma unroll
        for (int f = 1; f < NFOLD; ++f) x = cadd(x, bin[f][s]);
        v[s] = x;
      }
    } else {
      const float2 at = cconj(twp(twp_hi, twp_lo, (tid * r) & (P - 1)));   // exp(+2 pi i t r / P)
      const int m16 = 16 * Rp - 1;
      float2 om[NFOLD];                                                    // exp(+2 pi i f r / R')
#pragma unroll
      for (int f = 1; f < NFOLD; ++f) om[f] = tws[(16 * f * r) & m16];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        float2 x = bin[0][s];
#pragma unroll
        for (int f = 1; f < NFOLD; ++f) x = cadd(x, cmul(bin[f][s], om[f]));
        v[s] = cmul(x, cmul(at, tws[(s * r) & m16]));
      }
    }
    fft_lds<LOGL, true, TW1>(v, buf, tw, tw + LH, tid, tw1);   // starts with a barrier
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int oi = S::out_index(tid, i);
      const float m = __builtin_amdgcn_sqrtf(v[i].x * v[i].x + v[i].y * v[i].y);
      mr[oi] = m;
      if (oi < H) mr[oi + L] = m;
      if (oi >= L - H) mr[oi - L] = m;
    }
    __syncthreads();
    for (int q = tid; q < Q; q += T) {
      const int base = n_start + q * R + K - 1;        // sample read by tap j = 0
      const int c = (base - r) & (Rp - 1);               // taps j = c + R' u read this phase
      const float* hp = hc + c * nu;
      const float* mp = mr + ((base - c - r) >> logRp);  // sample of tap c, then one back per u
      float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
      int u = 0;
      for (; u + 4 <= nu; u += 4) {
        s0 = fmaf(hp[u], mp[-u], s0);
        s1 = fmaf(hp[u + 1], mp[-u - 1], s1);
        s2 = fmaf(hp[u + 2], mp[-u - 2], s2);
        s3 = fmaf(hp[u + 3], mp[-u - 3], s3);
      }
      for (; u < nu; ++u) s0 = fmaf(hp[u], mp[-u], s0);
      accq[q] += (s0 + s1) + (s2 + s3);                  // this thread's own range bin
    }
  }
  for (int q = tid; q < Q; q += T) E[fd * Q + q] = accq[q];
}

// The same result with the whole beam window in LDS, where it fits (G floats beside the transform):
// each phase's magnitudes land at their window positions w = (R' a + r - n_start) mod P, w < G, and
// the low-pass runs once over the window at the end (contiguous taps per range bin, no per-phase
// work).  Rotations as above.
template <int LOGL, int NFOLD>
__global__ __launch_bounds__((1 << LOGL) / 16) void fd_ifft_envw_kernel(
    const float2* __restrict__ bspec, const float2* __restrict__ tw_g, const float* __restrict__ taps,
    float* __restrict__ E, int kb, int kb_pad, int Rp, int P, int n_start, int G, int Q, int R, int K) {
  using S = FftShape<LOGL>;
  constexpr int L = S::NF;
  constexpr int T = S::T;
  constexpr int LH = FdTw<LOGL>::LH;
  constexpr bool TW1 = L >= 256;              // pass-1 twiddles from a table (built once per workgroup)
  __shared__ float2 buf[S::LDS_ELEMS];
  __shared__ float2 tw[LH + 64];
  __shared__ float2 tw1[TW1 ? 256 : 1];
  extern __shared__ float2 dyn[];             // 16 R' phase factors, K taps / P, the G-sample window
  float2* tws = dyn;
  float* hs = reinterpret_cast<float*>(dyn + 16 * Rp);
  float* mag = hs + ((K + 3) & ~3);
  const int tid = threadIdx.x;
  const long long fd = blockIdx.x;            // f * D + d
  for (int i = tid; i < LH + 64; i += T) tw[i] = tw_g[i];
  if constexpr (TW1) pass1_twiddles<LOGL, true>(tw1, tw_g, tw_g + LH, tid, T);
  const float2* twp_hi = tw_g + LH + 64;
  const float2* twp_lo = twp_hi + P / 64 + 1;
  for (int i = tid; i < 16 * Rp; i += T) tws[i] = cconj(twp(twp_hi, twp_lo, i * (L / 16)));   // exp(+2 pi i i / (16 R'))
  // the taps carry the transform's 1/P (a power of two: the products are exactly those of h[j] |b| / P)
  const float invP = 1.0f / static_cast<float>(P);
  for (int j = tid; j < K; j += T) hs[j] = taps[j] * invP;
  const float2* in = bspec + fd * kb_pad;
  float2 bin[NFOLD][16];
#pragma unroll
  for (int f = 0; f < NFOLD; ++f)
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int k = tid + s * (L / 16) + f * L;
      bin[f][s] = k < kb ? in[k] : make_float2(0.f, 0.f);
    }
  __syncthreads();                            // tables in LDS
  // the twiddles of the later passes depend only on the thread: built once, kept across the phases
  // (one bin per slot leaves the registers for them)
  constexpr bool TWR = NFOLD == 1;
  float2 twr[FftTwr<LOGL>::N];
  if constexpr (TWR) fft_thread_twiddles<LOGL, true>(twr, tw, tw + LH, tid);

  for (int r = 0; r < Rp; ++r) {
    float2 v[16];
    if (r == 0) {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        float2 x = bin[0][s];
#pragma unroll
        for (int f = 1; f < NFOLD; ++f) x = cadd(x, bin[f][s]);
        v[s] = x;
      }
    } else {
      const float2 at = cconj(twp(twp_hi, twp_lo, (tid * r) & (P - 1)));   // exp(+2 pi i t r / P)
      const int m16 = 16 * Rp - 1;
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        float2 x = cmul(bin[0][s], cmul(at, tws[(s * r) & m16]));
#pragma unroll
        for (int f = 1; f < NFOLD; ++f) x = cadd(x, cmul(bin[f][s], cmul(at, tws[((s + 16 * f) * r) & m16])));
        v[s] = x;
      }
    }
    fft_lds<LOGL, true, TW1, TWR>(v, buf, tw, tw + LH, tid, tw1, twr);   // starts with a barrier
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int w = (Rp * S::out_index(tid, i) + r - n_start) & (P - 1);   // window position of the sample
      if (w < G) mag[w] = __builtin_amdgcn_sqrtf(v[i].x * v[i].x + v[i].y * v[i].y);
    }
  }
  __syncthreads();
  for (int q = tid; q < Q; q += T) {
    const float* a = mag + q * R + K - 1;
    float acc = 0.f;
    for (int j = 0; j < K; ++j) acc = fmaf(hs[j], a[-j], acc);
    E[fd * Q + q] = acc;
  }
}

template <int LOGL>
__global__ __launch_bounds__((1 << LOGL) / 16) void fd_ifft_beam_kernel(
    const float2* __restrict__ bspec, const float2* __restrict__ tw_g, float2* __restrict__ beam,
    int kb, int kb_pad, int Rp, int P, int k_lo, int n_start, int G) {
  using S = FftShape<LOGL>;
  constexpr int T = S::T;
  constexpr int LH = FdTw<LOGL>::LH;
  __shared__ float2 lds[S::LDS_ELEMS];
  __shared__ float2 tw[LH + 64];
  const int tid = threadIdx.x;
  const int r = blockIdx.x % Rp;
  const long long fd = blockIdx.x / Rp;
  for (int i = tid; i < LH + 64; i += T) tw[i] = tw_g[i];
  const float2* twp_hi = tw_g + LH + 64;
  const float2* twp_lo = twp_hi + P / 64 + 1;
  float2 v[16];
  load_phase<LOGL>(bspec + fd * kb_pad, kb, r, P, twp_hi, twp_lo, v, tid);
  fft_lds<LOGL, true>(v, lds, tw, tw + LH, tid);   // starts with a barrier (after the twiddle copy)
  const float invP = 1.0f / static_cast<float>(P);
  float2* out = beam + fd * G;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const long long n = static_cast<long long>(Rp) * S::out_index(tid, i) + r;
    const int e = static_cast<int>((static_cast<long long>(k_lo) * n) % P);   // exp(2 pi i k_lo n / P)
    const float2 rot = cconj(twp(twp_hi, twp_lo, e));
    const float2 y = cmul(make_float2(v[i].x * invP, v[i].y * invP), rot);
    for (int j = static_cast<int>((n - n_start) & (P - 1)); j < G; j += P) out[j] = y;
  }
}

}  // namespace

hipError_t launch_fd_gemm(const sonar_plan_s* p, const float2* band, int F, float2* bspec, hipStream_t s) {
  const int nbt = (p->kb_pad + FD_GEMM_BINS_WG - 1) / FD_GEMM_BINS_WG;
  const int ndt = (p->D + FD_GEMM_DIRS - 1) / FD_GEMM_DIRS;
  const int nft = (F + FD_GEMM_FRAMES - 1) / FD_GEMM_FRAMES;
  const int nyt = nbt * nft;                                  // sample tiles
  const int nyt8 = (nyt + 2 * FD_XCDS - 1) / (2 * FD_XCDS) * (2 * FD_XCDS);   // whole pairs on every XCD
  const dim3 grid(static_cast<unsigned>(nyt8) * ndt);
  switch (p->bf_mode) {
    case SONAR_BF_FD_FP32:
      hipLaunchKernelGGL(fd_gemm_kernel<MODE_FP32>, grid, dim3(256), 0, s, band, p->d_dl, p->d_fdstep, bspec, F, p->D, p->M,
                         p->kb, p->kb_pad, p->k_lo, p->P, nbt, ndt, nyt);
      break;
    case SONAR_BF_FD_BF16:
      hipLaunchKernelGGL(fd_gemm_kernel<MODE_BF16>, grid, dim3(256), 0, s, band, p->d_dl, p->d_fdstep, bspec, F, p->D, p->M,
                         p->kb, p->kb_pad, p->k_lo, p->P, nbt, ndt, nyt);
      break;
    case SONAR_BF_FD_BF16X3:
      hipLaunchKernelGGL(fd_gemm_kernel<MODE_BF16X3>, grid, dim3(256), 0, s, band, p->d_dl, p->d_fdstep, bspec, F, p->D, p->M,
                         p->kb, p->kb_pad, p->k_lo, p->P, nbt, ndt, nyt);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int LOGL, int NFOLD>
hipError_t launch_env_t(const sonar_plan_s* p, const float2* bspec, int F, float* E, hipStream_t s) {
  const size_t smem = fd_env_dyn_lds(p);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fd_ifft_env_kernel<LOGL, NFOLD>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fd_ifft_env_kernel<LOGL, NFOLD>), dim3(static_cast<unsigned>(F) * p->D), dim3((1 << LOGL) / 16),
                     smem, s, bspec, p->d_fdtw, p->d_taps, E, p->kb, p->kb_pad, p->fd_R, ilog2_host(p->fd_R), p->P,
                     p->n0 - p->hk, p->Q, p->R, p->K);
  return hipGetLastError();
}

template <int LOGL, int NFOLD>
hipError_t launch_envw_t(const sonar_plan_s* p, const float2* bspec, int F, float* E, hipStream_t s) {
  const size_t smem = fd_envw_dyn_lds(p);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fd_ifft_envw_kernel<LOGL, NFOLD>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fd_ifft_envw_kernel<LOGL, NFOLD>), dim3(static_cast<unsigned>(F) * p->D), dim3((1 << LOGL) / 16),
                     smem, s, bspec, p->d_fdtw, p->d_taps, E, p->kb, p->kb_pad, p->fd_R, p->P, p->n0 - p->hk, p->G,
                     p->Q, p->R, p->K);
  return hipGetLastError();
}

template <int LOGL>
hipError_t launch_env_f(const sonar_plan_s* p, const float2* bspec, int F, float* E, hipStream_t s) {
  if (p->fd_win) {
    if (p->fd_nfold == 1) return launch_envw_t<LOGL, 1>(p, bspec, F, E, s);
    return p->fd_nfold == 2 ? launch_envw_t<LOGL, 2>(p, bspec, F, E, s) : launch_envw_t<LOGL, 3>(p, bspec, F, E, s);
  }
  if (p->fd_nfold == 1) return launch_env_t<LOGL, 1>(p, bspec, F, E, s);
  return p->fd_nfold == 2 ? launch_env_t<LOGL, 2>(p, bspec, F, E, s) : launch_env_t<LOGL, 3>(p, bspec, F, E, s);
}

hipError_t launch_fd_ifft_env(const sonar_plan_s* p, const float2* bspec, int F, float* E, hipStream_t s) {
  if (!p->fd_fused || p->fd_nfold < 1 || p->fd_nfold > FD_MAX_FOLD) return hipErrorInvalidValue;
  switch (p->fd_logL) {
    case 4: return launch_env_f<4>(p, bspec, F, E, s);
    case 5: return launch_env_f<5>(p, bspec, F, E, s);
    case 6: return launch_env_f<6>(p, bspec, F, E, s);
    case 7: return launch_env_f<7>(p, bspec, F, E, s);
    case 8: return launch_env_f<8>(p, bspec, F, E, s);
    case 9: return launch_env_f<9>(p, bspec, F, E, s);
    case 10: return launch_env_f<10>(p, bspec, F, E, s);
    case 11: return launch_env_f<11>(p, bspec, F, E, s);
    case 12: return launch_env_f<12>(p, bspec, F, E, s);
    case 13: return launch_env_f<13>(p, bspec, F, E, s);
    case 14: return launch_env_f<14>(p, bspec, F, E, s);
    default: return hipErrorInvalidValue;
  }
}

template <int LOGL>
hipError_t launch_beam_t(const sonar_plan_s* p, const float2* bspec, int F, float2* beam, hipStream_t s) {
  hipLaunchKernelGGL((fd_ifft_beam_kernel<LOGL>), dim3(static_cast<unsigned>(F) * p->D * p->fd_R),
                     dim3((1 << LOGL) / 16), 0, s, bspec, p->d_fdtw, beam, p->kb, p->kb_pad, p->fd_R, p->P,
                     p->k_lo, p->n0 - p->hk, p->G);
  return hipGetLastError();
}

hipError_t launch_fd_ifft_beam(const sonar_plan_s* p, const float2* bspec, int F, float2* beam, hipStream_t s) {
  switch (p->fd_logL) {
    case 4: return launch_beam_t<4>(p, bspec, F, beam, s);
    case 5: return launch_beam_t<5>(p, bspec, F, beam, s);
    case 6: return launch_beam_t<6>(p, bspec, F, beam, s);
    case 7: return launch_beam_t<7>(p, bspec, F, beam, s);
    case 8: return launch_beam_t<8>(p, bspec, F, beam, s);
    case 9: return launch_beam_t<9>(p, bspec, F, beam, s);
    case 10: return launch_beam_t<10>(p, bspec, F, beam, s);
    case 11: return launch_beam_t<11>(p, bspec, F, beam, s);
    case 12: return launch_beam_t<12>(p, bspec, F, beam, s);
    case 13: return launch_beam_t<13>(p, bspec, F, beam, s);
    case 14: return launch_beam_t<14>(p, bspec, F, beam, s);
    default: return hipErrorInvalidValue;
  }
}

// LDS of the window variant of the fused inverse: static (transform buffer, transform twiddles) and
// dynamic (16 R' phase factors, taps, the beam window)
size_t fd_env_dyn_lds(const sonar_plan_s* p) {
  const int nu = (p->K + p->fd_R - 1) / p->fd_R;
  return static_cast<size_t>(16) * p->fd_R * sizeof(float2) + static_cast<size_t>(p->fd_R) * nu * sizeof(float) +
         static_cast<size_t>(p->Q) * sizeof(float);
}
size_t fd_envw_static_lds(int logL) {
  const int L = 1 << logL;
  return static_cast<size_t>(L + L / 16 + (L / 64 > 0 ? L / 64 : 1) + 64 + (L >= 256 ? 256 : 1)) * sizeof(float2);
}
size_t fd_envw_dyn_lds(const sonar_plan_s* p) {
  return static_cast<size_t>(16) * p->fd_R * sizeof(float2) + static_cast<size_t>((p->K + 3) & ~3) * sizeof(float) +
         static_cast<size_t>(p->G) * sizeof(float);
}
