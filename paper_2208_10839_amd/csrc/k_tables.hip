// Plan tables built on the device in FP64 (§4.1: the delay of each direction
// relative to each channel is computed ahead of beamforming; §4.3: all device
// memory is prepared once before processing starts).
//
//  * delays      Dl[d][m] = fs (p_m . u_d) / c, and for the time-domain
//                beamformer o = floor(-Dl), alpha = -Dl - o, stored as
//                {o - omin, (1-alpha)/M, alpha/M} (integer delays: o = floor(-Dl + 1/2),
//                alpha = 0; cubic: two entries per microphone, {o - 1 - omin, L_-1/M, L_0/M}
//                and {o + 1 - omin, L_1/M, L_2/M}, the 4-point Lagrange weights; gridded
//                (TD_F16, TD_BF16G): alpha rounded to a multiple of 1/2048 or 1/256, alpha = 1
//                taken as o + 1);
//  * chirp       C[k] = beta[k] W[k] conj(S[k]), S[k] = sum_l s[l] exp(-2 pi i k l/P),
//                with the phase index k l reduced mod P exactly in integers;
//  * twiddles    FFT tables (layout in plan.hpp), exp(-2 pi i e / NF) and
//                exp(-2 pi i e / P) rounded once from FP64.
#include <hip/hip_runtime.h>
#include <math.h>

#include "plan.hpp"

namespace {

__global__ void delay_table_kernel(const double* __restrict__ pos, const double* __restrict__ dirs,
                                   int M, int D, double fs, double c, int omin, int spread, int interp,
                                   int4* __restrict__ dtab, double* __restrict__ dl) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<long long>(D) * M) return;
  const int d = static_cast<int>(i / M), m = static_cast<int>(i % M);
  const double pu = pos[3 * m] * dirs[3 * d] + pos[3 * m + 1] * dirs[3 * d + 1] + pos[3 * m + 2] * dirs[3 * d + 2];
  const double Dl = fs * pu / c;
  const bool nearest = interp == 1;
  double o = nearest ? floor(-Dl + 0.5) : floor(-Dl);
  double a = nearest ? 0.0 : -Dl - o;
  if (interp == 3 || interp == 4) {
    const double steps = interp == 3 ? 2048.0 : 256.0;
    a = rint(a * steps) / steps;
    if (a >= 1.0) {
      o += 1.0;
      a = 0.0;
    }
  }
  dl[i] = Dl;
  if (interp == 2) {
    // 4-point Lagrange weights at a for the samples o - 1 .. o + 2
    const double lm = -a * (a - 1.0) * (a - 2.0) / 6.0, l0 = (a + 1.0) * (a - 1.0) * (a - 2.0) / 2.0;
    const double l1 = -(a + 1.0) * a * (a - 2.0) / 2.0, l2 = (a + 1.0) * a * (a - 1.0) / 6.0;
    int r0 = static_cast<int>(o) - 1 - omin, r1 = static_cast<int>(o) + 1 - omin;
    r0 = r0 < 0 ? 0 : (r0 > spread ? spread : r0);
    r1 = r1 < 0 ? 0 : (r1 > spread ? spread : r1);
    dtab[2 * i] = make_int4(r0, __float_as_int(static_cast<float>(lm / M)), __float_as_int(static_cast<float>(l0 / M)), 0);
    dtab[2 * i + 1] = make_int4(r1, __float_as_int(static_cast<float>(l1 / M)), __float_as_int(static_cast<float>(l2 / M)), 0);
    return;
  }
  int rel = static_cast<int>(o) - omin;
  rel = rel < 0 ? 0 : (rel > spread ? spread : rel);
  const float w0 = static_cast<float>((1.0 - a) / M);
  const float w1 = static_cast<float>(a / M);
  dtab[i] = make_int4(rel, __float_as_int(w0), __float_as_int(w1), 0);
}

// roots[t] = exp(-2 pi i t / P), t < P
__global__ void roots_kernel(double2* __restrict__ roots, int P) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P) return;
  double s, c;
  sincospi(-2.0 * static_cast<double>(t) / static_cast<double>(P), &s, &c);
  roots[t] = make_double2(c, s);
}

__global__ void chirp_spectrum_kernel(const double* __restrict__ chirp, int L,
                                      const double2* __restrict__ roots, int P, int NF,
                                      double fs, double lo, double hi, int band_on,
                                      float2* __restrict__ cspec) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > NF) return;
  double re = 0.0, im = 0.0;
  for (int l = 0; l < L; ++l) {
    const int t = static_cast<int>((static_cast<long long>(k) * l) % P);
    re += chirp[l] * roots[t].x;
    im += chirp[l] * roots[t].y;
  }
  const double W = (k == 0 || k == NF) ? 1.0 : 2.0;
  double beta = 1.0;
  if (band_on) {
    const double f = static_cast<double>(k) * (fs / static_cast<double>(P));
    beta = (f >= lo && f <= hi) ? 1.0 : 0.0;
  }
  const double g = beta * W;
  cspec[k] = make_float2(static_cast<float>(g * re), static_cast<float>(-g * im));
}

__global__ void fft_twiddle_kernel(float2* __restrict__ tw, int NF, int P) {
  const int nhi = fft_nhi(NF), nhp = fft_nhp(NF);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nhi + 64 + nhp + 64) return;
  double num, den;
  if (i < nhi) { num = 64.0 * i; den = NF; }
  else if (i < nhi + 64) { num = i - nhi; den = NF; }
  else if (i < nhi + 64 + nhp) { num = 64.0 * (i - nhi - 64); den = P; }
  else { num = i - nhi - 64 - nhp; den = P; }
  double s, c;
  sincospi(-2.0 * num / den, &s, &c);
  tw[i] = make_float2(static_cast<float>(c), static_cast<float>(s));
}

// FD twiddles (layout: fd_tw_len in plan.hpp)
__global__ void fd_twiddle_kernel(float2* __restrict__ tw, int L, int P) {
  const int lh = L / 64 > 0 ? L / 64 : 1;
  const int ph = P / 64 + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= lh + 64 + ph + 64) return;
  double num, den;
  if (i < lh) { num = 64.0 * i; den = L; }
  else if (i < lh + 64) { num = i - lh; den = L; }
  else if (i < lh + 64 + ph) { num = 64.0 * (i - lh - 64); den = P; }
  else { num = i - lh - 64 - ph; den = P; }
  double s, c;
  sincospi(-2.0 * num / den, &s, &c);
  tw[i] = make_float2(static_cast<float>(c), static_cast<float>(s));
}

// FD steering rotation per bin: exp(-2 pi i Dl / P) from the FP64 delays
__global__ void fd_step_kernel(const double* __restrict__ dl, long long n, int P, float2* __restrict__ step) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c;
  sincospi(-2.0 * dl[i] / static_cast<double>(P), &s, &c);
  step[i] = make_float2(static_cast<float>(c), static_cast<float>(s));
}

}  // namespace

hipError_t launch_fd_step_table(sonar_plan_s* p, hipStream_t s) {
  const long long dm = static_cast<long long>(p->D) * p->M;
  hipLaunchKernelGGL(fd_step_kernel, dim3(static_cast<unsigned>((dm + 255) / 256)), dim3(256), 0, s, p->d_dl, dm,
                     p->P, p->d_fdstep);
  return hipGetLastError();
}

hipError_t launch_build_fd_tables(sonar_plan_s* p, hipStream_t s) {
  const int n = fd_tw_len(p->fd_L, p->P);
  hipLaunchKernelGGL(fd_twiddle_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p->d_fdtw, p->fd_L, p->P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_fd_step_table(p, s);
}

hipError_t launch_delay_tables(sonar_plan_s* p, hipStream_t s) {
  const long long dm = static_cast<long long>(p->D) * p->M;
  hipLaunchKernelGGL(delay_table_kernel, dim3(static_cast<unsigned>((dm + 255) / 256)), dim3(256), 0, s,
                     p->d_pos, p->d_dirs, p->M, p->D, p->fs, p->c, p->omin, p->spread,
                     p->bf_mode == SONAR_BF_TD_NEAREST ? 1
                     : p->bf_mode == SONAR_BF_TD_CUBIC ? 2
                     : p->bf_mode == SONAR_BF_TD_F16   ? 3
                     : p->bf_mode == SONAR_BF_TD_BF16G ? 4
                                                       : 0,
                     p->d_dtab, p->d_dl);
  return hipGetLastError();
}

hipError_t launch_build_tables(sonar_plan_s* p, hipStream_t s) {
  hipError_t e = launch_delay_tables(p, s);
  if (e != hipSuccess) return e;
  double2* roots = static_cast<double2*>(p->d_aux);
  hipLaunchKernelGGL(roots_kernel, dim3((p->P + 255) / 256), dim3(256), 0, s, roots, p->P);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(chirp_spectrum_kernel, dim3((p->NF + 1 + 255) / 256), dim3(256), 0, s,
                     p->d_chirp, p->L, roots, p->P, p->NF, p->fs, p->band_lo, p->band_hi,
                     p->band_on ? 1 : 0, p->d_cspec);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int twl = fft_tw_len(p->NF);
  hipLaunchKernelGGL(fft_twiddle_kernel, dim3((twl + 255) / 256), dim3(256), 0, s, p->d_tw, p->NF, p->P);
  // row-transform twiddles only for the four-step matched filter (d_tw2 is a 16-byte
  // placeholder allocation otherwise)
  if ((e = hipGetLastError()) != hipSuccess || p->NF <= (1 << MB_LOGN2)) return e;
  const int tw2l = fft_tw_len(1 << MB_LOGN2);
  hipLaunchKernelGGL(fft_twiddle_kernel, dim3((tw2l + 255) / 256), dim3(256), 0, s, p->d_tw2, 1 << MB_LOGN2, p->P);
  return hipGetLastError();
}
