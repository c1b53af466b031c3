// Reverse-mode derivatives of the time-domain pipeline (the adjoint used to
// self-calibrate the array geometry; the forward steps are §4.1 matched
// filter, delay-and-sum and envelope, §4.3 subsampling).  For a real loss L of
// the energyscape with dE = dL/dE, complex quantities z carry
// G_z = dL/dRe z + i dL/dIm z:
//
//   envelope      G_b[w]   = (sum_{q, j: qR + K-1-j = w} dE[q] h[j]) * b[w] / |b[w]|
//   delay-and-sum dDl[d][m] = sum_w Re(conj(G_b[w]) (y_m[w+rel] - y_m[w+rel+1])) / M
//                 G_y[m][r] = sum_d w0[d][m] G_b[d][r-rel] + w1[d][m] G_b[d][r-rel-1]
//   (4-point Lagrange reading, TD_CUBIC: taps k = -1 .. 2 with weights L_k(alpha) / M, so
//    G_y collects all four and dDl[d][m] = -sum_w Re(conj(G_b[w]) sum_k L_k'(alpha) y_m[w+rel_k]) / M)
//   delays        dpos[m]   = fs/c * sum_{f,d} dDl[f][d][m] u_d
//   matched filter dx       = Re IDFT_P(conj(C) . DFT_P(G_yhat)), cut to N
//
// (w is the beam-window position, r the position in a matched-filter row, rel
// the row offset of tap 0; the row layout and weights are those of the forward
// kernels.)  The complex P-point DFTs of G_yhat and G_b run as P / L transforms of
// L points, one per phase (samples nph a + ph), recombined with exp(-2 pi i k ph / P):
// L = NF (even and odd samples) while it fits one workgroup's LDS, else the big
// matched filter's 2^MB_LOGN2-point rows; the inverse is the forward matched
// filter's two-parity inverse (in LDS, or over global memory for the big rows).
//
// The exact-phase (frequency-domain) beamformer b_d = IDFT_P(B_d) on the window,
// B_d[k] = (1/M) sum_m Y_m[k] exp(-2 pi i k Dl[d][m] / P) over the band bins, has
//   G_B[d][k]  = DFT_P(G_b[d] placed on its window positions)[k] / P
//   dDl[d][m]  = (1/M) sum_k Re(conj(G_B[d][k]) Y_m[k] (-2 pi i k / P) exp(-2 pi i k Dl / P))
//   G_Y[m][k]  = (1/M) sum_d exp(+2 pi i k Dl[d][m] / P) G_B[d][k]
//   dx         = Re sum_k conj(C[k]) G_Y[k] exp(2 pi i k n / P), cut to N.
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "plan.hpp"

using namespace fftk;

namespace {

// G_b over the beam window, in place: beam[f][d][w] -> G_b[f][d][w]
__global__ void env_vjp_kernel(float2* __restrict__ beam, const float* __restrict__ dE,
                               const float* __restrict__ taps, long long rows, int G, int Q, int R, int K) {
  const int w = blockIdx.y * blockDim.x + threadIdx.x;
  const long long fd = blockIdx.x;
  if (w >= G || fd >= rows) return;
  // outputs q reading position w: 0 <= qR + K-1-w < K
  int qlo = w - K + 1 > 0 ? (w - K + 1 + R - 1) / R : 0;
  int qhi = w / R;
  if (qhi > Q - 1) qhi = Q - 1;
  const float* e = dE + fd * Q;
  float g = 0.f;
  for (int q = qlo; q <= qhi; ++q) g = fmaf(e[q], taps[q * R + K - 1 - w], g);
  const float2 b = beam[fd * G + w];
  const float mag = sqrtf(b.x * b.x + b.y * b.y);
  const float s = mag > 0.f ? g / mag : 0.f;
  beam[fd * G + w] = make_float2(s * b.x, s * b.y);
}

// dDl[f][d][m]: one workgroup per (frame, direction), a block reduction per microphone.  Linear
// readings: one table entry {rel, w0, w1} per microphone, slopes (1, -1) on y[rel], y[rel + 1].
// Cubic: two entries {o - 1 - omin, ..}, {o + 1 - omin, ..} per microphone; the slopes -L_k'(alpha)
// of the four taps come from the FP64 delay dl (alpha = -Dl - floor(-Dl)).
__global__ __launch_bounds__(256) void dl_vjp_kernel(const float2* __restrict__ gb, const float2* __restrict__ yext,
                                                     const int4* __restrict__ dtab, const double* __restrict__ dl,
                                                     float* __restrict__ ddl, long long fstride, int M, int D, int G,
                                                     int row, int cubic) {
  __shared__ float red[256 / 64];
  const int d = blockIdx.x % D;
  const long long f = blockIdx.x / D;
  const float2* g = gb + (f * D + d) * G;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int m = 0; m < M; ++m) {
    const long long i = static_cast<long long>(d) * M + m;
    // taps y[rel_k + w] with slopes s_k (k = 0 .. 3); the linear readings use the first two
    int rel0, rel2 = 0;
    float s0 = 1.f, s1 = -1.f, s2 = 0.f, s3 = 0.f;
    if (cubic) {
      rel0 = dtab[2 * i].x;
      rel2 = dtab[2 * i + 1].x;
      const double Dl = dl[i];
      const double a = -Dl - floor(-Dl), a2 = a * a;
      // -L_k'(a) for the nodes -1, 0, 1, 2
      s0 = static_cast<float>((3.0 * a2 - 6.0 * a + 2.0) / 6.0);
      s1 = static_cast<float>(-(3.0 * a2 - 4.0 * a - 1.0) / 2.0);
      s2 = static_cast<float>((3.0 * a2 - 2.0 * a - 2.0) / 2.0);
      s3 = static_cast<float>(-(3.0 * a2 - 1.0) / 6.0);
    } else {
      rel0 = dtab[i].x;
    }
    const float2* y = yext + f * fstride + static_cast<long long>(m) * row + rel0;
    const float2* y2 = yext + f * fstride + static_cast<long long>(m) * row + rel2;
    float acc = 0.f;
    if (cubic) {
      for (int w = threadIdx.x; w < G; w += 256) {
        const float2 gw = g[w], a = y[w], b = y[w + 1], c = y2[w], e = y2[w + 1];
        const float tx = s0 * a.x + s1 * b.x + s2 * c.x + s3 * e.x;
        const float ty = s0 * a.y + s1 * b.y + s2 * c.y + s3 * e.y;
        acc = fmaf(gw.x, tx, acc);
        acc = fmaf(gw.y, ty, acc);
      }
    } else {
      for (int w = threadIdx.x; w < G; w += 256) {
        const float2 gw = g[w], a = y[w], b = y[w + 1];
        acc = fmaf(gw.x, a.x - b.x, acc);
        acc = fmaf(gw.y, a.y - b.y, acc);
      }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
      ddl[(f * D + d) * M + m] = (red[0] + red[1] + red[2] + red[3]) / static_cast<float>(M);
    __syncthreads();
  }
}

// dpos[m][k] = fs/c * sum_{f,d} dDl[f][d][m] u_d[k] (FP64 accumulation), one workgroup per microphone
__global__ __launch_bounds__(256) void pos_vjp_kernel(const float* __restrict__ ddl, const double* __restrict__ dirs,
                                                      double* __restrict__ dpos, int F, int M, int D, double scale) {
  __shared__ double red[3][256];
  const int m = blockIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (long long i = threadIdx.x; i < static_cast<long long>(F) * D; i += 256) {
    const int d = static_cast<int>(i % D);
    const double v = ddl[i * M + m];
    a0 += v * dirs[3 * d];
    a1 += v * dirs[3 * d + 1];
    a2 += v * dirs[3 * d + 2];
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  red[2][threadIdx.x] = a2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 3) dpos[3 * m + threadIdx.x] = scale * red[threadIdx.x][0];
}

// G_yhat[f][m][n], n in Z_P: every row position r = (n - origin) mod P, r + P, ... below row
// collects the taps that read it
// (TD_CUBIC: 1 << vshift = 2 two-tap table entries per microphone, each handled as a linear one)
__global__ __launch_bounds__(256) void yhat_vjp_kernel(const float2* __restrict__ gb, const int4* __restrict__ dtab,
                                                       float2* __restrict__ gy, int M, int D, int G, int row, int P,
                                                       int origin, int vshift) {
  const int n = blockIdx.y * 256 + threadIdx.x;
  const long long fm = blockIdx.x;
  if (n >= P) return;
  const long long f = fm / M;
  const int m = static_cast<int>(fm - f * M);
  const float2* g = gb + f * D * G;
  const int ne = 1 << vshift;
  float2 acc = make_float2(0.f, 0.f);
  for (int r = (n - origin) & (P - 1); r < row; r += P) {
    for (int de = 0; de < D * ne; ++de) {
      const int d = de >> vshift;
      const int4 e = dtab[((static_cast<long long>(d) * M + m) << vshift) + (de & (ne - 1))];
      const int w = r - e.x;
      const float w0 = __int_as_float(e.y), w1 = __int_as_float(e.z);
      if (w >= 0 && w < G) {
        const float2 v = g[static_cast<long long>(d) * G + w];
        acc.x = fmaf(w0, v.x, acc.x);
        acc.y = fmaf(w0, v.y, acc.y);
      }
      if (w >= 1 && w <= G) {
        const float2 v = g[static_cast<long long>(d) * G + w - 1];
        acc.x = fmaf(w1, v.x, acc.x);
        acc.y = fmaf(w1, v.y, acc.y);
      }
    }
  }
  gy[fm * P + n] = acc;
}

// Two-level twiddle tables of the plan in LDS (layout in plan.hpp)
template <int LOGNF>
__device__ __forceinline__ void load_tw(float2* tw, const float2* __restrict__ tw_g, int tid, int nthreads) {
  constexpr int NF = 1 << LOGNF;
  constexpr int NHI = NF / 64 > 0 ? NF / 64 : 1;
  constexpr int LEN = NHI + 64 + (NF / 64 + 1) + 64;
  for (int i = tid; i < LEN; i += nthreads) tw[i] = tw_g[i];
}

// Polyphase split of a P-point DFT, P = nph L:
//   DFT_P(g)[k] = sum_ph exp(-2 pi i k ph / P) S_ph[k mod L],  S_ph = DFT_L(g[nph a + ph]), a < L.
// S[ch][ph][j] = DFT_L(g[nph a + ph])[j] for the row of channel ch placed on Z_P: row position i
// (i < G) sits at sample (wstart + i) mod P, every other sample is zero.  twl holds the L-point
// two-level table (exp(-2 pi i 64 t / L), t < max(L/64, 1), then exp(-2 pi i t / L), t < 64).
template <int LOGL>
__global__ __launch_bounds__((1 << LOGL) / 16) void phase_fft_kernel(const float2* __restrict__ g, long long gstride,
                                                                     const float2* __restrict__ twl,
                                                                     float2* __restrict__ S, int G, int P, int wstart,
                                                                     int nph) {
  using Sh = FftShape<LOGL>;
  constexpr int L = Sh::NF;
  constexpr int T = Sh::T;
  constexpr int NHI = L / 64 > 0 ? L / 64 : 1;
  __shared__ float2 lds[Sh::LDS_ELEMS];
  __shared__ float2 tw[NHI + 64];
  const int tid = threadIdx.x;
  const int ph = blockIdx.x % nph;
  const long long ch = blockIdx.x / nph;
  for (int i = tid; i < NHI + 64; i += T) tw[i] = twl[i];
  __syncthreads();
  const float2* in = g + ch * gstride;
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int n = nph * (tid + r * (L / 16)) + ph;
    const int i = (n - wstart) & (P - 1);
    v[r] = i < G ? in[i] : make_float2(0.f, 0.f);
  }
  fft_lds<LOGL, false>(v, lds, tw, tw + NHI, tid);
  float2* out = S + (ch * nph + ph) * L;
#pragma unroll
  for (int i = 0; i < 16; ++i) out[Sh::out_index(tid, i)] = v[i];
}

// exp(-2 pi i e / P), 0 <= e < P, from the plan's table of exp(-2 pi i t / P) for t <= NF + 63
// (tw_g: the two-level table of d_tw; e > NF by the half-turn symmetry)
__device__ __forceinline__ float2 tw_p(const float2* __restrict__ tw_g, int NF, int e) {
  const float2* hi = tw_g + fft_nhi(NF) + 64;          // exp(-2 pi i 64 t / P)
  const float2* lo = hi + fft_nhp(NF);                 // exp(-2 pi i t / P)
  if (e <= NF) return cmul(hi[e >> 6], lo[e & 63]);
  const float2 w = cmul(hi[(e - NF) >> 6], lo[(e - NF) & 63]);
  return make_float2(-w.x, -w.y);
}

// DFT_P(g)[k] of channel ch from its nph phase transforms (layout of phase_fft_kernel)
__device__ __forceinline__ float2 phase_sum(const float2* __restrict__ S, const float2* __restrict__ tw_g,
                                            long long ch, int nph, int L, int NF, int P, int k) {
  const int km = k & (L - 1);
  const float2* s = S + ch * nph * static_cast<long long>(L) + km;
  float2 acc = s[0];
  for (int ph = 1; ph < nph; ++ph)
    acc = cadd(acc, cmul(tw_p(tw_g, NF, (k * ph) & (P - 1)), s[static_cast<long long>(ph) * L]));
  return acc;
}

// V[ch][k] = conj(C[k]) DFT_P(G_yhat[ch])[k], k in [0, NF]
__global__ void mfadj_mul_kernel(const float2* __restrict__ S, const float2* __restrict__ cspec,
                                 const float2* __restrict__ tw_g, float2* __restrict__ V, int NF, int nph, int L) {
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  const long long ch = blockIdx.x;
  if (k > NF) return;
  const float2 gk = phase_sum(S, tw_g, ch, nph, L, NF, 2 * NF, k);
  V[ch * (NF + 1) + k] = cmul(cconj(cspec[k]), gk);
}

// dx[ch][2a + par] = Re (1/P) (sum_{k<NF} V[k] exp(2 pi i k par / P) exp(2 pi i k a / NF) + V[NF] (-1)^par)
template <int LOGNF>
__global__ __launch_bounds__((1 << LOGNF) / 16) void mfadj_inv_kernel(const float2* __restrict__ V,
                                                                      const float2* __restrict__ tw_g,
                                                                      float* __restrict__ dx, int N, int P) {
  using Sh = FftShape<LOGNF>;
  constexpr int NF = Sh::NF;
  constexpr int T = Sh::T;
  constexpr int NHI = NF / 64 > 0 ? NF / 64 : 1;
  constexpr int TWLEN = NHI + 64 + (NF / 64 + 1) + 64;
  __shared__ float2 lds[Sh::LDS_ELEMS];
  __shared__ float2 tw[TWLEN];
  const int tid = threadIdx.x;
  const int par = blockIdx.x & 1;
  const long long ch = blockIdx.x >> 1;
  load_tw<LOGNF>(tw, tw_g, tid, T);
  __syncthreads();
  const float2* twp_hi = tw + NHI + 64;
  const float2* twp_lo = tw + NHI + 64 + (NF / 64 + 1);
  const float2* in = V + ch * (NF + 1);
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k = tid + r * (NF / 16);
    v[r] = in[k];
    if (par) v[r] = cmul(v[r], cconj(cmul(twp_hi[k >> 6], twp_lo[k & 63])));
  }
  const float2 ny = in[NF];
  fft_lds<LOGNF, true>(v, lds, tw, tw + NHI, tid);
  const float inv_p = 1.0f / static_cast<float>(P);
  const float sgn = par ? -1.0f : 1.0f;
  float* out = dx + ch * N;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int n = 2 * Sh::out_index(tid, i) + par;
    if (n < N) out[n] = (v[i].x + sgn * ny.x) * inv_p;
  }
}

// exp(-2 pi i k Dl / P) with the phase k Dl / P reduced to [-1/2, 1/2] in FP64
__device__ __forceinline__ float2 steer(int k, double dl_over_p) {
  const double a = static_cast<double>(k) * dl_over_p;
  const float r = static_cast<float>(a - rint(a));
  float s, c;
  sincospif(-2.0f * r, &s, &c);
  return make_float2(c, s);
}

// G_B[ch][j] = DFT_P(G_b[ch] on its window positions)[k] / P, k = k_lo + j
__global__ void gfd_band_kernel(const float2* __restrict__ S, const float2* __restrict__ tw_g,
                                float2* __restrict__ GB, int NF, int P, int k_lo, int kb, int nph, int L) {
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  const long long ch = blockIdx.x;
  if (j >= kb) return;
  const float2 g = phase_sum(S, tw_g, ch, nph, L, NF, P, k_lo + j);
  const float inv_p = 1.0f / static_cast<float>(P);
  GB[ch * kb + j] = make_float2(g.x * inv_p, g.y * inv_p);
}

// dDl[f][d][m], one workgroup per (frame, direction): lane l of a wavefront takes microphone
// m0 + l % ms and bins j = jsub + (4 waves x 64/ms) t, where ms = min(64, next pow2 >= M)
__global__ __launch_bounds__(256) void gfd_dl_kernel(const float2* __restrict__ GB, const float2* __restrict__ Y,
                                                     const double* __restrict__ dl, float* __restrict__ ddl,
                                                     int M, int D, int kb, int k_lo, int P, int ms) {
  __shared__ float red[256];
  const int d = blockIdx.x % D;
  const long long f = blockIdx.x / D;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int per_wave = 64 / ms;
  const int jsub = wv * per_wave + lane / ms;
  const int jstep = 4 * per_wave;
  const float2* gb = GB + (f * D + d) * kb;
  const float2* y = Y + f * static_cast<long long>(kb) * M;
  const float two_pi_over_p = 6.283185307179586f / static_cast<float>(P);
  for (int m0 = 0; m0 < M; m0 += ms) {
    const int m = m0 + lane % ms;
    float acc = 0.f;
    if (m < M) {
      const double dlp = dl[static_cast<long long>(d) * M + m] / static_cast<double>(P);
      for (int j = jsub; j < kb; j += jstep) {
        const int k = k_lo + j;
        const float2 g = gb[j];
        const float2 yv = y[static_cast<long long>(j) * M + m];
        const float2 ph = steer(k, dlp);
        // Re(conj(g) * yv * ph * (-i w)) = w Im(conj(g) * yv * ph), w = 2 pi k / P
        const float2 t = cmul(cconj(g), cmul(yv, ph));
        acc = fmaf(two_pi_over_p * static_cast<float>(k), t.y, acc);
      }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < ms && m0 + static_cast<int>(threadIdx.x) < M) {
      float s = 0.f;
      for (int i = threadIdx.x; i < 256; i += ms) s += red[i];
      ddl[(f * D + d) * M + m0 + threadIdx.x] = s / static_cast<float>(M);
    }
    __syncthreads();
  }
}

// G_Y[f][j][m] = (1/M) sum_d exp(+2 pi i k Dl[d][m] / P) G_B[f][d][j], one thread per (j, m)
__global__ __launch_bounds__(256) void gfd_gy_kernel(const float2* __restrict__ GB, const double* __restrict__ dl,
                                                     float2* __restrict__ GY, int M, int D, int kb, int k_lo, int P) {
  const long long t = static_cast<long long>(blockIdx.y) * 256 + threadIdx.x;
  const long long f = blockIdx.x;
  if (t >= static_cast<long long>(kb) * M) return;
  const int j = static_cast<int>(t / M), m = static_cast<int>(t - static_cast<long long>(j) * M);
  const int k = k_lo + j;
  const float2* gb = GB + f * D * static_cast<long long>(kb) + j;
  float2 acc = make_float2(0.f, 0.f);
  for (int d = 0; d < D; ++d) {
    const float2 ph = steer(k, dl[static_cast<long long>(d) * M + m] / static_cast<double>(P));
    acc = cadd(acc, cmul(cconj(ph), gb[static_cast<long long>(d) * kb]));
  }
  const float inv_m = 1.0f / static_cast<float>(M);
  GY[f * static_cast<long long>(kb) * M + t] = make_float2(acc.x * inv_m, acc.y * inv_m);
}

// V[f][m][k] = P conj(C[k]) G_Y[f][k - k_lo][m] on the band bins, 0 elsewhere, k in [0, NF]
__global__ void gfd_spec_kernel(const float2* __restrict__ GY, const float2* __restrict__ cspec,
                                float2* __restrict__ V, int M, int NF, int P, int k_lo, int kb) {
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  const long long ch = blockIdx.x;   // f * M + m
  if (k > NF) return;
  const long long f = ch / M;
  const int m = static_cast<int>(ch - f * M);
  const int j = k - k_lo;
  float2 v = make_float2(0.f, 0.f);
  if (j >= 0 && j < kb) {
    const float2 g = GY[(f * kb + j) * M + m];
    v = cmul(cconj(cspec[k]), g);
    v.x *= static_cast<float>(P);
    v.y *= static_cast<float>(P);
  }
  V[ch * (NF + 1) + k] = v;
}

// Transform length of the polyphase split: L = NF (two phases) while an NF-point transform fits
// one workgroup's LDS, else L = 2^MB_LOGN2 and P / L phases (the big matched filter's row length,
// whose table is d_tw2)
int adj_logl(const sonar_plan_s* p) { return p->NF > (1 << MB_LOGN2) ? MB_LOGN2 : p->logNF; }

template <int LOGL>
hipError_t launch_phase_fft_t(const sonar_plan_s* p, const float2* g, long long gstride, long long chans, int G,
                              int wstart, hipStream_t s) {
  constexpr int T = (1 << LOGL) / 16;
  const int nph = p->P >> LOGL;
  const float2* twl = LOGL == p->logNF ? p->d_tw : p->d_tw2;
  hipLaunchKernelGGL((phase_fft_kernel<LOGL>), dim3(static_cast<unsigned>(chans * nph)), dim3(T), 0, s, g, gstride,
                     twl, p->d_gscr, G, p->P, wstart, nph);
  return hipGetLastError();
}

template <int LOGNF>
hipError_t launch_mfinv_t(const sonar_plan_s* p, const float2* V, int F, float* dx, hipStream_t s) {
  constexpr int T = (1 << LOGNF) / 16;
  hipLaunchKernelGGL((mfadj_inv_kernel<LOGNF>), dim3(2 * F * p->M), dim3(T), 0, s, V, p->d_tw, dx, p->N, p->P);
  return hipGetLastError();
}

#define SONAR_LOG_DISPATCH(LOG, NAME, ...)       \
  switch (LOG) {                                  \
    case 4: return NAME<4>(__VA_ARGS__);          \
    case 5: return NAME<5>(__VA_ARGS__);          \
    case 6: return NAME<6>(__VA_ARGS__);          \
    case 7: return NAME<7>(__VA_ARGS__);          \
    case 8: return NAME<8>(__VA_ARGS__);          \
    case 9: return NAME<9>(__VA_ARGS__);          \
    case 10: return NAME<10>(__VA_ARGS__);        \
    case 11: return NAME<11>(__VA_ARGS__);        \
    case 12: return NAME<12>(__VA_ARGS__);        \
    case 13: return NAME<13>(__VA_ARGS__);        \
    case 14: return NAME<14>(__VA_ARGS__);        \
    default: return hipErrorInvalidValue;         \
  }

// phase transforms of chans rows (stride gstride, G values from window sample wstart) into d_gscr
hipError_t phase_fft(const sonar_plan_s* p, const float2* g, long long gstride, long long chans, int G, int wstart,
                     hipStream_t s) {
  SONAR_LOG_DISPATCH(adj_logl(p), launch_phase_fft_t, p, g, gstride, chans, G, wstart, s)
}

// dx = Re IDFT_P(V) cut to N, V one-sided per (frame, microphone)
hipError_t mfinv(const sonar_plan_s* p, const float2* V, int F, float* dx, hipStream_t s) {
  if (p->NF > (1 << MB_LOGN2)) return launch_big_inv_real(p, V, F * p->M, dx, s);
  SONAR_LOG_DISPATCH(p->logNF, launch_mfinv_t, p, V, F, dx, s)
}

// matched-filter adjoint of the time-domain path: dx from G_yhat over Z_P (the phase transforms
// of gscr_chans channels at a time through the scratch)
hipError_t mfadj(const sonar_plan_s* p, const float2* gy, int F, float* dx, hipStream_t s) {
  const long long chans = static_cast<long long>(F) * p->M;
  const int L = 1 << adj_logl(p);
  for (long long c0 = 0; c0 < chans; c0 += p->gscr_chans) {
    const long long n = chans - c0 < p->gscr_chans ? chans - c0 : p->gscr_chans;
    hipError_t e = phase_fft(p, gy + c0 * p->P, p->P, n, p->P, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mfadj_mul_kernel, dim3(static_cast<unsigned>(n), (p->NF + 1 + 255) / 256), dim3(256), 0, s,
                       p->d_gscr, p->d_cspec, p->d_tw, p->d_spec + c0 * (p->NF + 1), p->NF, p->P / L, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return mfinv(p, p->d_spec, F, dx, s);
}

// exact-phase beamformer: G_B, then dDl / dpos and G_Y / dx
hipError_t vjp_fd(const sonar_plan_s* p, const float2* mf, const float2* gb, int F, float2* dyhat, float* dx,
                  double* dpos, hipStream_t s) {
  hipError_t e = hipSuccess;
  const long long chans = static_cast<long long>(F) * p->D;
  const int L = 1 << adj_logl(p);
  for (long long c0 = 0; c0 < chans; c0 += p->gscr_chans) {
    const long long n = chans - c0 < p->gscr_chans ? chans - c0 : p->gscr_chans;
    if ((e = phase_fft(p, gb + c0 * p->G, p->G, n, p->G, p->n0 - p->hk, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(gfd_band_kernel, dim3(static_cast<unsigned>(n), (p->kb + 255) / 256), dim3(256), 0, s, p->d_gscr,
                       p->d_tw, p->d_gband + c0 * p->kb, p->NF, p->P, p->k_lo, p->kb, p->P / L, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (dpos) {
    int ms = 1;
    while (ms < p->M && ms < 64) ms *= 2;
    hipLaunchKernelGGL(gfd_dl_kernel, dim3(F * p->D), dim3(256), 0, s, p->d_gband, mf, p->d_dl, p->d_gdl, p->M,
                       p->D, p->kb, p->k_lo, p->P, ms);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(pos_vjp_kernel, dim3(p->M), dim3(256), 0, s, p->d_gdl, p->d_dirs, dpos, F, p->M, p->D,
                       p->fs / p->c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (dyhat) {
    const long long items = static_cast<long long>(p->kb) * p->M;
    hipLaunchKernelGGL(gfd_gy_kernel, dim3(F, static_cast<unsigned>((items + 255) / 256)), dim3(256), 0, s,
                       p->d_gband, p->d_dl, dyhat, p->M, p->D, p->kb, p->k_lo, p->P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (dx) {
      hipLaunchKernelGGL(gfd_spec_kernel, dim3(F * p->M, (p->NF + 1 + 255) / 256), dim3(256), 0, s, dyhat,
                         p->d_cspec, p->d_gspec, p->M, p->NF, p->P, p->k_lo, p->kb);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      return mfinv(p, p->d_gspec, F, dx, s);
    }
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Energyscape cells of the exact-phase beamformer and their adjoint, for a loss
// L = sum_c w_c E_c over cells c = (f, d, q), from the band spectra Y[f][j][m] alone: no
// beam window and no P-point transform.  With n_i = n0 - hk + qR + i (i < K, window
// position qR + i, tap K-1-i):
//   B[k]    = (1/M) sum_m Y_m[k] exp(-2 pi i k Dl[d][m] / P)            (band bins k)
//   b_i     = (1/P) sum_k B[k] exp(+2 pi i k n_i / P)
//   E_c     = sum_i h[K-1-i] |b_i|
//   G_b,i   = w_c h[K-1-i] b_i / |b_i|
//   G_B[k]  = (1/P) sum_i G_b,i exp(-2 pi i k n_i / P)
//   dDl[m]  = (1/M) sum_k Re(conj(G_B[k]) Y_m[k] (-2 pi i k / P) exp(-2 pi i k Dl[d][m] / P))
// (the chain of the dense derivative restricted to the cells' windows).  The band bins of a
// cell are split into S ranges, one workgroup each: cells_b_kernel writes each range's share
// of the sums b_i, cells_g_kernel adds them up (every range's workgroup the same way), forms
// E and G_b, and writes its range's share of dDl; pos_cells_kernel adds the shares.  B and G_B
// go through LDS in chunks of CELL_CHUNK bins.
constexpr int CELL_THREADS = 1024;
constexpr int CELL_WAVES = CELL_THREADS / 64;
constexpr int CELL_CHUNK = 4096;
constexpr int CELL_SPW = 16;    // window samples per wavefront: K <= CELL_WAVES * CELL_SPW
constexpr int CELL_MG = 4;      // groups of 64 microphones: M <= 256

struct CellArgs {
  const float2* Y;
  const int* cells;
  const float* wgt;
  const double* dl;
  const float* taps;
  const float2* tw;
  float* E_out;
  float2* bpart;   // [n][S][K]
  float* dpart;    // [n][S][M]
  int n, S, F, M, D, Q, R, K, n0, hk, k_lo, kb, NF, P;
};

__device__ __forceinline__ bool cell_valid(const CellArgs& a, int c, int* f, int* d, int* q) {
  *f = a.cells[3 * c];
  *d = a.cells[3 * c + 1];
  *q = a.cells[3 * c + 2];
  return *f >= 0 && *f < a.F && *d >= 0 && *d < a.D && *q >= 0 && *q < a.Q;
}

// bins [jb, je) of range sp of the cell
__device__ __forceinline__ void cell_range(const CellArgs& a, int sp, int* jb, int* je) {
  const int per = (a.kb + a.S - 1) / a.S;
  *jb = sp * per < a.kb ? sp * per : a.kb;
  *je = *jb + per < a.kb ? *jb + per : a.kb;
}

__global__ __launch_bounds__(CELL_THREADS) void cells_b_kernel(const CellArgs a) {
  __shared__ float2 chunk[CELL_CHUNK];
  const int c = blockIdx.x / a.S, sp = blockIdx.x % a.S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int f, d, q;
  if (!cell_valid(a, c, &f, &d, &q)) return;   // uniform: cells_g_kernel handles the cell
  int jb, je;
  cell_range(a, sp, &jb, &je);
  const int M = a.M, P = a.P;
  const float2* y = a.Y + static_cast<long long>(f) * a.kb * M;
  const double* dlr = a.dl + static_cast<long long>(d) * M;
  const double inv_pd = 1.0 / static_cast<double>(P);
  const float inv_m = 1.0f / static_cast<float>(M);
  const int nbase = a.n0 - a.hk + q * a.R;
  // wavefront wv accumulates the window samples i = wv + CELL_WAVES s over its lanes' bins
  float2 bacc[CELL_SPW];
#pragma unroll
  for (int s = 0; s < CELL_SPW; ++s) bacc[s] = make_float2(0.f, 0.f);
  for (int c0 = jb; c0 < je; c0 += CELL_CHUNK) {
    const int nb = je - c0 < CELL_CHUNK ? je - c0 : CELL_CHUNK;
    for (int jj = tid; jj < nb; jj += CELL_THREADS) {
      const int j = c0 + jj;
      const int k = a.k_lo + j;
      float2 acc = make_float2(0.f, 0.f);
      for (int m = 0; m < M; ++m) acc = cadd(acc, cmul(y[static_cast<long long>(j) * M + m], steer(k, dlr[m] * inv_pd)));
      chunk[jj] = make_float2(acc.x * inv_m, acc.y * inv_m);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < CELL_SPW; ++s) {
      const int i = wv + CELL_WAVES * s;
      if (i < a.K) {
        const unsigned ni = static_cast<unsigned>((nbase + i) & (P - 1));
        for (int jj = lane; jj < nb; jj += 64) {
          const unsigned e = (static_cast<unsigned>(a.k_lo + c0 + jj) * ni) & static_cast<unsigned>(P - 1);
          bacc[s] = cadd(bacc[s], cmul(chunk[jj], cconj(tw_p(a.tw, a.NF, static_cast<int>(e)))));
        }
      }
    }
    __syncthreads();
  }
  float2* out = a.bpart + (static_cast<long long>(c) * a.S + sp) * a.K;
#pragma unroll
  for (int s = 0; s < CELL_SPW; ++s) {
    float2 v = bacc[s];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      v.x += __shfl_xor(v.x, off);
      v.y += __shfl_xor(v.y, off);
    }
    const int i = wv + CELL_WAVES * s;
    if (lane == 0 && i < a.K) out[i] = v;
  }
}

__global__ __launch_bounds__(CELL_THREADS) void cells_g_kernel(const CellArgs a) {
  __shared__ float2 chunk[CELL_CHUNK];
  __shared__ float2 gw[CELL_WAVES * CELL_SPW];
  __shared__ float red[CELL_THREADS];
  const int c = blockIdx.x / a.S, sp = blockIdx.x % a.S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int M = a.M, P = a.P, K = a.K;
  float* dout = a.dpart + (static_cast<long long>(c) * a.S + sp) * M;
  int f, d, q;
  if (!cell_valid(a, c, &f, &d, &q)) {
    if (a.E_out && sp == 0 && tid == 0) a.E_out[c] = __builtin_nanf("");
    for (int m = tid; m < M; m += CELL_THREADS) dout[m] = 0.f;
    return;
  }
  int jb, je;
  cell_range(a, sp, &jb, &je);
  const float2* y = a.Y + static_cast<long long>(f) * a.kb * M;
  const double* dlr = a.dl + static_cast<long long>(d) * M;
  const double inv_pd = 1.0 / static_cast<double>(P);
  const float inv_m = 1.0f / static_cast<float>(M), inv_p = 1.0f / static_cast<float>(P);
  const int nbase = a.n0 - a.hk + q * a.R;

  // b from the ranges' shares, E and G_b (wavefront 0; every range's workgroup alike)
  if (wv == 0) {
    const float wc = a.wgt[c];
    float e = 0.f;
    for (int i = lane; i < K; i += 64) {
      float2 b = make_float2(0.f, 0.f);
      for (int r = 0; r < a.S; ++r) b = cadd(b, a.bpart[(static_cast<long long>(c) * a.S + r) * K + i]);
      b = make_float2(b.x * inv_p, b.y * inv_p);
      const float am = sqrtf(b.x * b.x + b.y * b.y);
      const float h = a.taps[K - 1 - i];
      e = fmaf(h, am, e);
      const float g = am > 0.f ? wc * h / am : 0.f;
      gw[i] = make_float2(g * b.x, g * b.y);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if (lane == 0 && sp == 0 && a.E_out) a.E_out[c] = e;
  }
  __syncthreads();

  // G_B chunk by chunk, then dDl: lane l takes microphones m0 + l % ms and bins
  // jsub + jstep t of the chunk (as the dense kernel)
  int ms = 1;
  while (ms < M && ms < 64) ms *= 2;
  const int per_wave = 64 / ms;
  const int jsub = wv * per_wave + lane / ms, jstep = CELL_WAVES * per_wave;
  const float two_pi_over_p = 6.283185307179586f / static_cast<float>(P);
  float dacc[CELL_MG];
#pragma unroll
  for (int g = 0; g < CELL_MG; ++g) dacc[g] = 0.f;
  for (int c0 = jb; c0 < je; c0 += CELL_CHUNK) {
    const int nb = je - c0 < CELL_CHUNK ? je - c0 : CELL_CHUNK;
    for (int jj = tid; jj < nb; jj += CELL_THREADS) {
      const unsigned k = static_cast<unsigned>(a.k_lo + c0 + jj);
      float2 acc = make_float2(0.f, 0.f);
      for (int i = 0; i < K; ++i) {
        const unsigned e = (k * static_cast<unsigned>((nbase + i) & (P - 1))) & static_cast<unsigned>(P - 1);
        acc = cadd(acc, cmul(gw[i], tw_p(a.tw, a.NF, static_cast<int>(e))));
      }
      chunk[jj] = make_float2(acc.x * inv_p, acc.y * inv_p);
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < CELL_MG; ++g) {
      const int m = 64 * g + lane % ms;
      if (64 * g < M && m < M) {
        const double dlp = dlr[m] * inv_pd;
        for (int jj = jsub; jj < nb; jj += jstep) {
          const int k = a.k_lo + c0 + jj;
          const float2 t = cmul(cconj(chunk[jj]), cmul(y[static_cast<long long>(c0 + jj) * M + m], steer(k, dlp)));
          dacc[g] = fmaf(two_pi_over_p * static_cast<float>(k), t.y, dacc[g]);
        }
      }
    }
    __syncthreads();
  }
  for (int g = 0; g < CELL_MG && 64 * g < M; ++g) {
    red[tid] = dacc[g];
    __syncthreads();
    const int m = 64 * g + tid;
    if (tid < ms && m < M) {
      float sum = 0.f;
      for (int i = tid; i < CELL_THREADS; i += ms) sum += red[i];
      dout[m] = sum * inv_m;
    }
    __syncthreads();
  }
}

// Time-domain readings (linear, nearest, cubic) of the same cells, one 256-thread workgroup per
// cell from the matched-filter rows: b_i = sum over the delay-table entries of the two weighted
// taps at window position qR + i (the weights carry 1/M), E_c, G_b, and dDl[m] with the slopes of
// the dense kernel ((1, -1) on the linear pair; -L_k'(alpha) on the four cubic taps)
__global__ __launch_bounds__(256) void cells_td_kernel(const float2* __restrict__ yext, long long fstride, int row,
                                                       const int4* __restrict__ dtab, const double* __restrict__ dl,
                                                       const int* __restrict__ cells, const float* __restrict__ wgt,
                                                       const float* __restrict__ taps, float* __restrict__ E_out,
                                                       float* __restrict__ dpart, int F, int M, int D, int Q, int R,
                                                       int K, int cubic) {
  __shared__ float2 gw[256];
  __shared__ float red[4];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int f = cells[3 * c], d = cells[3 * c + 1], q = cells[3 * c + 2];
  float* dout = dpart + static_cast<long long>(c) * M;
  if (!(f >= 0 && f < F && d >= 0 && d < D && q >= 0 && q < Q)) {
    if (E_out && tid == 0) E_out[c] = __builtin_nanf("");
    for (int m = tid; m < M; m += 256) dout[m] = 0.f;
    return;
  }
  const float2* yf = yext + static_cast<long long>(f) * fstride;
  const int ne = cubic ? 2 * M : M;   // table entries of the direction, entry e reading row e / (1 + cubic)
  const int4* dt = dtab + static_cast<long long>(d) * ne;
  float e = 0.f;
  if (tid < K) {
    const int w = q * R + tid;
    float2 b = make_float2(0.f, 0.f);
    for (int en = 0; en < ne; ++en) {
      const int4 t = dt[en];
      const float2* y = yf + static_cast<long long>(cubic ? en >> 1 : en) * row + t.x + w;
      const float w0 = __int_as_float(t.y), w1 = __int_as_float(t.z);
      const float2 a0 = y[0], a1 = y[1];
      b.x = fmaf(w0, a0.x, fmaf(w1, a1.x, b.x));
      b.y = fmaf(w0, a0.y, fmaf(w1, a1.y, b.y));
    }
    const float am = sqrtf(b.x * b.x + b.y * b.y);
    const float h = taps[K - 1 - tid];
    e = h * am;
    const float g = am > 0.f ? wgt[c] * h / am : 0.f;
    gw[tid] = make_float2(g * b.x, g * b.y);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
  if (lane == 0) red[wv] = e;
  __syncthreads();
  if (tid == 0 && E_out) E_out[c] = red[0] + red[1] + red[2] + red[3];
  const float inv_m = 1.0f / static_cast<float>(M);
  for (int m = tid; m < M; m += 256) {
    const long long i = static_cast<long long>(d) * M + m;
    int rel0, rel2 = 0;
    float s0 = 1.f, s1 = -1.f, s2 = 0.f, s3 = 0.f;
    if (cubic) {
      rel0 = dtab[2 * i].x;
      rel2 = dtab[2 * i + 1].x;
      const double Dl = dl[i];
      const double a = -Dl - floor(-Dl), a2 = a * a;
      s0 = static_cast<float>((3.0 * a2 - 6.0 * a + 2.0) / 6.0);
      s1 = static_cast<float>(-(3.0 * a2 - 4.0 * a - 1.0) / 2.0);
      s2 = static_cast<float>((3.0 * a2 - 2.0 * a - 2.0) / 2.0);
      s3 = static_cast<float>(-(3.0 * a2 - 1.0) / 6.0);
    } else {
      rel0 = dtab[i].x;
    }
    const float2* y = yf + static_cast<long long>(m) * row + rel0 + q * R;
    const float2* y2 = yf + static_cast<long long>(m) * row + rel2 + q * R;
    float acc = 0.f;
    for (int k = 0; k < K; ++k) {
      const float2 g = gw[k], a = y[k], b = y[k + 1];
      float tx = s0 * a.x + s1 * b.x, ty = s0 * a.y + s1 * b.y;
      if (cubic) {
        const float2 cc = y2[k], ee = y2[k + 1];
        tx += s2 * cc.x + s3 * ee.x;
        ty += s2 * cc.y + s3 * ee.y;
      }
      acc = fmaf(g.x, tx, acc);
      acc = fmaf(g.y, ty, acc);
    }
    dout[m] = acc * inv_m;
  }
}

// dpos[m] = fs/c sum_cells (sum of the ranges' dDl shares)[m] u_{d_c} (cells outside the plan add
// nothing: their shares are zero)
__global__ __launch_bounds__(256) void pos_cells_kernel(const float* __restrict__ dpart, const int* __restrict__ cells,
                                                        int n, int S, const double* __restrict__ dirs,
                                                        double* __restrict__ dpos, int M, int D, double scale) {
  __shared__ double red[3][256];
  const int m = blockIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    int d = cells[3 * i + 1];
    d = d < 0 ? 0 : (d >= D ? D - 1 : d);
    double v = 0.0;
    for (int r = 0; r < S; ++r) v += dpart[(static_cast<long long>(i) * S + r) * M + m];
    a0 += v * dirs[3 * d];
    a1 += v * dirs[3 * d + 1];
    a2 += v * dirs[3 * d + 2];
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  red[2][threadIdx.x] = a2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 3) dpos[3 * m + threadIdx.x] = scale * red[threadIdx.x][0];
}

}  // namespace

hipError_t launch_energyscape_vjp(const sonar_plan_s* p, const float2* mf, float2* beam_grad, const float* dE, int F,
                                  float2* dyhat, float* dx, double* dpos, hipStream_t s) {
  const long long rows = static_cast<long long>(F) * p->D;
  hipLaunchKernelGGL(env_vjp_kernel, dim3(static_cast<unsigned>(rows), (p->G + 255) / 256), dim3(256), 0, s,
                     beam_grad, dE, p->d_taps, rows, p->G, p->Q, p->R, p->K);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p->bf_mode != SONAR_BF_TD_LINEAR && p->bf_mode != SONAR_BF_TD_BF16 && p->bf_mode != SONAR_BF_TD_NEAREST &&
      p->bf_mode != SONAR_BF_TD_BF16X2 && p->bf_mode != SONAR_BF_TD_F16 && p->bf_mode != SONAR_BF_TD_BF16G &&
      p->bf_mode != SONAR_BF_TD_CUBIC)
    return vjp_fd(p, mf, beam_grad, F, dyhat, dx, dpos, s);
  const int cubic = p->bf_mode == SONAR_BF_TD_CUBIC ? 1 : 0;
  if (dpos) {
    hipLaunchKernelGGL(dl_vjp_kernel, dim3(static_cast<unsigned>(rows)), dim3(256), 0, s, beam_grad, mf, p->d_dtab,
                       p->d_dl, p->d_gdl, p->mf_fstride, p->M, p->D, p->G, p->row, cubic);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(pos_vjp_kernel, dim3(p->M), dim3(256), 0, s, p->d_gdl, p->d_dirs, dpos, F, p->M, p->D,
                       p->fs / p->c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (dyhat) {
    hipLaunchKernelGGL(yhat_vjp_kernel, dim3(F * p->M, (p->P + 255) / 256), dim3(256), 0, s, beam_grad, p->d_dtab,
                       dyhat, p->M, p->D, p->G, p->row, p->P, static_cast<int>(p->origin), cubic);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (dx) return mfadj(p, dyhat, F, dx, s);
  }
  return hipSuccess;
}

bool cells_supported(const sonar_plan_s* p) {
  if (p->bf_mode == SONAR_BF_TD_LINEAR || p->bf_mode == SONAR_BF_TD_NEAREST || p->bf_mode == SONAR_BF_TD_CUBIC)
    return p->K <= 256;
  if (p->bf_mode != SONAR_BF_FD_FP32 && p->bf_mode != SONAR_BF_FD_BF16 && p->bf_mode != SONAR_BF_FD_BF16X3) return false;
  return p->K <= CELL_WAVES * CELL_SPW && p->M <= 64 * CELL_MG && 2 * p->K + p->M <= 2 * p->P;
}

hipError_t launch_energyscape_cells(const sonar_plan_s* p, const float2* mf, int F, const int* cells,
                                    const float* dE, int n, float* E_out, double* dpos, hipStream_t s) {
  if (p->bf_mode == SONAR_BF_TD_LINEAR || p->bf_mode == SONAR_BF_TD_NEAREST || p->bf_mode == SONAR_BF_TD_CUBIC) {
    // the delay-derivative shares go to the plan's [max_frames][D][M] table (n <= max_frames D)
    hipLaunchKernelGGL(cells_td_kernel, dim3(n), dim3(256), 0, s, mf, p->mf_fstride, p->row, p->d_dtab, p->d_dl, cells,
                       dE, p->d_taps, E_out, p->d_gdl, F, p->M, p->D, p->Q, p->R, p->K,
                       p->bf_mode == SONAR_BF_TD_CUBIC ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !dpos) return e;
    hipLaunchKernelGGL(pos_cells_kernel, dim3(p->M), dim3(256), 0, s, p->d_gdl, cells, n, 1, p->d_dirs, dpos, p->M,
                       p->D, p->fs / p->c);
    return hipGetLastError();
  }
  // S bin ranges per cell (about 1024 bins each, at most 8), with the shares of b and dDl in the
  // plan's transform scratch (P complex values per cell slot: S (K + M) floats must fit 2 P)
  int S = p->kb / 1024;
  S = S < 1 ? 1 : (S > 8 ? 8 : S);
  const long long room = 2LL * p->gscr_chans * p->P;   // floats of scratch
  while (S > 1 && static_cast<long long>(n) * S * (2 * p->K + p->M) > room) --S;
  if (static_cast<long long>(n) * S * (2 * p->K + p->M) > room) return hipErrorInvalidValue;
  CellArgs a;
  a.Y = mf;
  a.cells = cells;
  a.wgt = dE;
  a.dl = p->d_dl;
  a.taps = p->d_taps;
  a.tw = p->d_tw;
  a.E_out = E_out;
  a.bpart = p->d_gscr;
  a.dpart = reinterpret_cast<float*>(p->d_gscr + static_cast<long long>(n) * S * p->K);
  a.n = n;
  a.S = S;
  a.F = F;
  a.M = p->M;
  a.D = p->D;
  a.Q = p->Q;
  a.R = p->R;
  a.K = p->K;
  a.n0 = p->n0;
  a.hk = p->hk;
  a.k_lo = p->k_lo;
  a.kb = p->kb;
  a.NF = p->NF;
  a.P = p->P;
  const dim3 grid(static_cast<unsigned>(static_cast<long long>(n) * S));
  hipLaunchKernelGGL(cells_b_kernel, grid, dim3(CELL_THREADS), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cells_g_kernel, grid, dim3(CELL_THREADS), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess || !dpos) return e;
  hipLaunchKernelGGL(pos_cells_kernel, dim3(p->M), dim3(256), 0, s, a.dpart, cells, n, S, p->d_dirs, dpos, p->M, p->D,
                     p->fs / p->c);
  return hipGetLastError();
}
