// C ABI of the energyscape library: plan creation (validation, derived sizes,
// one-time allocation of all device memory, FP64 table build) and the
// execution entry points, which only enqueue kernels.
//
// The paper preallocates every device buffer once when the processing node
// starts and frees it at shutdown, because per-measurement allocation cost
// performance (§4.3); the plan object is that preallocation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "plan.hpp"
#include "sonar.h"

// Static scratch of sonar_energyscape_batch_static (128 MiB per device, see below).
constexpr size_t STATIC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SONAR_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Default envelope low-pass: K = 8R + 1 Hamming-windowed sinc with cutoff
// fs/(2R), normalised to unit DC gain (zero phase about its centre tap).
std::vector<double> default_lowpass(int R) {
  const int K = 8 * R + 1;
  std::vector<double> h(K);
  const double pi = 3.14159265358979323846;
  double sum = 0.0;
  for (int j = 0; j < K; ++j) {
    const double w = 0.54 - 0.46 * std::cos(2.0 * pi * j / (K - 1));
    const double t = (j - (K - 1) / 2.0) / R;
    const double sinc = t == 0.0 ? 1.0 : std::sin(pi * t) / (pi * t);
    h[j] = w * sinc;
    sum += h[j];
  }
  for (double& v : h) v /= sum;
  return h;
}

void free_plan(sonar_plan_s* p) {
  if (!p) return;
  (void)hipFree(p->d_dtab);
  (void)hipFree(p->d_dl);
  (void)hipFree(p->d_pos);
  (void)hipFree(p->d_dirs);
  (void)hipFree(p->d_chirp);
  (void)hipFree(p->d_taps);
  (void)hipFree(p->d_cspec);
  (void)hipFree(p->d_tw);
  (void)hipFree(p->d_mf);
  (void)hipFree(p->d_spec);
  (void)hipFree(p->d_fdspec);
  (void)hipFree(p->d_bspec);
  (void)hipFree(p->d_beam);
  (void)hipFree(p->d_fdtw);
  (void)hipFree(p->d_fdstep);
  (void)hipFree(p->d_big);
  (void)hipFree(p->d_gdl);
  (void)hipFree(p->d_gscr);
  (void)hipFree(p->d_gband);
  (void)hipFree(p->d_gspec);
  (void)hipFree(p->d_gy);
  (void)hipFree(p->d_iir);
  (void)hipFree(p->d_fbound);
  (void)hipFree(p->d_tw2);
  (void)hipFree(p->d_mt_g);
  (void)hipFree(p->d_mt_w);
  (void)hipFree(p->d_mt_kcr);
  (void)hipFree(p->d_mt_perm);
  (void)hipFree(p->d_mt_fir);
  (void)hipFree(p->d_aux);
  delete p;
}

// count == 0 still allocates a 16-byte placeholder: never test a plan buffer pointer to
// decide whether a feature is enabled
template <typename T>
hipError_t dev_alloc(T** ptr, size_t count, size_t* total) {
  const size_t bytes = count * sizeof(T);
  *total += bytes;
  return hipMalloc(reinterpret_cast<void**>(ptr), bytes > 0 ? bytes : 16);
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

bool is_td(const sonar_plan_s* p) {
  return p->bf_mode == SONAR_BF_TD_LINEAR || p->bf_mode == SONAR_BF_TD_BF16 || p->bf_mode == SONAR_BF_TD_NEAREST ||
         p->bf_mode == SONAR_BF_TD_CUBIC || p->bf_mode == SONAR_BF_TD_BF16X2 || p->bf_mode == SONAR_BF_TD_F16 ||
         p->bf_mode == SONAR_BF_TD_BF16G;
}

// Coordinates z_d in which distances between directions equal distances between their
// delay vectors: |z_d - z_e| = |P (u_d - u_e)| for the microphone position matrix P
// (rows p_m).  With G = P^T P = V diag(l) V^T, z_d = diag(sqrt(l)) V^T u_d.  The 3 x 3
// eigenproblem is solved by cyclic Jacobi rotations.
void delay_space_coords(const double* pos, int M, const double* dirs, int D, std::vector<double>& z) {
  double G[3][3] = {};
  for (int m = 0; m < M; ++m)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) G[i][j] += pos[3 * m + i] * pos[3 * m + j];
  double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = std::fabs(G[0][1]) + std::fabs(G[0][2]) + std::fabs(G[1][2]);
    if (off < 1e-300) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int a = pq == 2 ? 1 : 0, b = pq == 0 ? 1 : 2;
      if (std::fabs(G[a][b]) < 1e-300) continue;
      const double th = 0.5 * std::atan2(2.0 * G[a][b], G[b][b] - G[a][a]);
      const double c = std::cos(th), s = std::sin(th);
      for (int k = 0; k < 3; ++k) {   // G <- G J
        const double gka = G[k][a], gkb = G[k][b];
        G[k][a] = c * gka - s * gkb;
        G[k][b] = s * gka + c * gkb;
      }
      for (int k = 0; k < 3; ++k) {   // G <- J^T G
        const double gak = G[a][k], gbk = G[b][k];
        G[a][k] = c * gak - s * gbk;
        G[b][k] = s * gak + c * gbk;
      }
      for (int k = 0; k < 3; ++k) {   // V <- V J
        const double vka = V[k][a], vkb = V[k][b];
        V[k][a] = c * vka - s * vkb;
        V[k][b] = s * vka + c * vkb;
      }
    }
  }
  z.assign(static_cast<size_t>(D) * 3, 0.0);
  for (int d = 0; d < D; ++d)
    for (int i = 0; i < 3; ++i) {
      const double sl = std::sqrt(std::max(G[i][i], 0.0));
      z[3 * d + i] = sl * (V[0][i] * dirs[3 * d] + V[1][i] * dirs[3 * d + 1] + V[2][i] * dirs[3 * d + 2]);
    }
}

// Orders idx[lo, hi) into runs of 32 that are compact in z: split along the widest axis of the
// set at a multiple of 32 near the middle, recursively.
void kd_tiles(std::vector<int>& idx, int lo, int hi, const std::vector<double>& z) {
  if (hi - lo <= 32) return;
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int i = lo; i < hi; ++i)
    for (int k = 0; k < 3; ++k) {
      mn[k] = std::min(mn[k], z[3 * idx[i] + k]);
      mx[k] = std::max(mx[k], z[3 * idx[i] + k]);
    }
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (mx[k] - mn[k] > mx[ax] - mn[ax]) ax = k;
  std::stable_sort(idx.begin() + lo, idx.begin() + hi,
                   [&](int a, int b) { return z[3 * a + ax] < z[3 * b + ax]; });
  const int n = hi - lo;
  const int half = ((n / 32 + 1) / 2) * 32;
  kd_tiles(idx, lo, lo + half, z);
  kd_tiles(idx, lo + half, hi, z);
}

uint16_t to_bf16_bits(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (finite values)
  return static_cast<uint16_t>(u >> 16);
}

// Tiles of the BF16-MFMA time-domain beamformer, built from the device's FP64
// delay table: directions cut into tiles of 32 that are compact in delay space
// (a k-d split of the coordinates of delay_space_coords).  Beam samples are
// split by residue mod GT (the group width: 2 taps with two sample planes, 4
// with four); for residue rho, per tile and microphone the span of integer
// offsets is covered by groups of GT taps whose first tap t0 has
// t0 + rho = 0 mod GT, so every sample group read by the kernel is one aligned
// 2 GT-byte load (four planes: groups in pairs, one microphone's taps t, t + 4,
// read as 8 consecutive samples).  16 / GT groups are one K-chunk of
// v_mfma_f32_32x32x16_bf16 (K rows GT i .. GT i + GT - 1 from group i), whose A
// fragments (tap weights as BF16 hi and lo terms) are stored in lane order.
int build_mt_tables(sonar_plan_s* p, const double* pos, const double* dirs, const std::vector<double>& taps,
                    hipStream_t stream, size_t* total) {
  // two sample planes: the low-pass runs on FP16 taps, scaled by 2^ts so that the largest lands in
  // [2^13, 2^14) (FP16 hi + lo terms keep ~22 bits of every tap whatever the filter's gain); the kernel
  // multiplies the result by 2^-ts at the store
  int ts = 0;
  if (mt_planes(p) == 2) {
    double hmax = 0.0;
    for (double h : taps) hmax = std::fmax(hmax, std::fabs(h));
    if (hmax > 0.0) {
      int ex = 0;
      (void)std::frexp(hmax, &ex);   // hmax = mant 2^ex, mant in [0.5, 1)
      ts = std::max(-100, std::min(100, 14 - ex));
    }
  }
  p->mt_fir_unscale = static_cast<float>(std::ldexp(1.0, -ts) / (p->bf_mode == SONAR_BF_TD_BF16G ? p->M : 1));
  const int D = p->D, M = p->M;
  std::vector<int4> dtab(static_cast<size_t>(D) * M);
  hipError_t e = hipMemcpyAsync(dtab.data(), p->d_dtab, dtab.size() * sizeof(int4), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "delay table read-back");
  std::vector<double> z;
  delay_space_coords(pos, M, dirs, D, z);
  std::vector<int> order(D);
  for (int d = 0; d < D; ++d) order[d] = d;
  kd_tiles(order, 0, D, z);
  const int mics = mt_mics(p);
  const int nt = (D + 31) / 32, nmc = (M + mics - 1) / mics;
  std::vector<int> perm(static_cast<size_t>(nt) * 32, -1);
  for (int i = 0; i < D; ++i) perm[i] = order[i];
  const int res = mt_gt(p), gtaps = mt_gt(p), gpc = 16 / mt_gt(p);   // residues, taps per group, groups per chunk
  const int nlist = nt * res;   // group list per (tile, residue)
  std::vector<std::vector<int2>> groups(nlist);
  std::vector<std::vector<char>> pad(nlist);   // zero-weight group completing a K-chunk
  std::vector<int2> kcr(static_cast<size_t>(nt) * nmc * res);
  int gmax = gpc;
  const bool f16 = mt_f16(p);
  const bool w1 = mt_w1(p);              // gridded delays: one exact 16-bit weight term
  const double steps = static_cast<double>(mt_grid_steps(p));
  // taps per microphone are allotted in runs of 4 (two planes) or 8 (four planes: the
  // kernel reads a group pair as 8 consecutive samples)
  const int span = mt_planes(p) == 4 ? 2 * gtaps : gtaps;
  for (int t = 0; t < nt; ++t) {
    for (int rho = 0; rho < res; ++rho) {
      std::vector<int2>& gl = groups[t * res + rho];
      std::vector<char>& pl = pad[t * res + rho];
      for (int mc = 0; mc < nmc; ++mc) {
        const int m0 = mc * mics, m1 = std::min(M, m0 + mics);
        const int g0 = static_cast<int>(gl.size());
        for (int m = m0; m < m1; ++m) {
          int rmin = 1 << 30, rmax = -(1 << 30);
          for (int s = 0; s < 32; ++s) {
            const int d = perm[t * 32 + s];
            if (d < 0) continue;
            rmin = std::min(rmin, dtab[static_cast<size_t>(d) * M + m].x);
            rmax = std::max(rmax, dtab[static_cast<size_t>(d) * M + m].x);
          }
          const int t0 = rmin - (rmin + rho) % res;   // rmin >= 0, so t0 + rho >= 0
          const int ng = (rmax + 2 - t0 + span - 1) / span;   // taps t0 .. rmax + 1
          for (int g = 0; g < ng * (span / gtaps); ++g) {
            gl.push_back(make_int2(m, t0 + gtaps * g));
            pl.push_back(0);
          }
        }
        while ((gl.size() - g0) % gpc) {
          gl.push_back(make_int2(m0, (res - rho) % res));
          pl.push_back(1);
        }
        kcr[(static_cast<size_t>(t) * nmc + mc) * res + rho] =
            make_int2(g0 / gpc, static_cast<int>(gl.size()) / gpc);
      }
      gmax = std::max(gmax, static_cast<int>(gl.size()));
    }
  }
  const int kcmax = gmax / gpc;
  std::vector<int> gtab(static_cast<size_t>(nlist) * gmax, 0);
  std::vector<uint16_t> wtab(static_cast<size_t>(nlist) * kcmax * 2 * 64 * 8, 0);
  for (int li = 0; li < nlist; ++li) {
    const int t = li / res;
    // the group's first sample: its microphone's row in the staging buffer, plus the first tap
    for (size_t g = 0; g < groups[li].size(); ++g) {
      const int2 gr = groups[li][g];
      gtab[static_cast<size_t>(li) * gmax + g] = (gr.x % mics) * p->mt_wrow + gr.y;
    }
    for (int kc = 0; kc < static_cast<int>(groups[li].size()) / gpc; ++kc) {
      for (int l = 0; l < 64; ++l) {
        const int d = perm[t * 32 + (l & 31)];
        for (int j = 0; j < 8; ++j) {
          // K row 8 (l / 32) + j: tap j % GT of group (16 / GT) kc + (8 / GT) (l / 32) + j / GT
          const int gi = gpc * kc + (gpc / 2) * (l >> 5) + j / gtaps;
          const int2 g = groups[li][gi];
          const int tap = g.y + j % gtaps;
          float w = 0.f;
          if (d >= 0 && !pad[li][gi]) {
            const int4 en = dtab[static_cast<size_t>(d) * M + g.x];
            float wa0, wa1;
            std::memcpy(&wa0, &en.y, 4);
            std::memcpy(&wa1, &en.z, 4);
            if (w1) {
              // gridded delay: alpha = k / steps recovered exactly from alpha / M
              const double a = std::rint(static_cast<double>(wa1) * M * steps) / steps;
              // 1 - alpha and alpha are exact in FP16 (1/2048 grid) and in BF16 (1/256 grid); the
              // 1/M of the array mean is applied in FP32 at the store (with the TD_F16 sample scale,
              // or with the low-pass scale for TD_BF16G)
              wa0 = static_cast<float>(1.0 - a);
              wa1 = static_cast<float>(a);
            }
            if (tap == en.x) w = wa0;
            else if (tap == en.x + 1) w = wa1;
          }
          if (w1 && !f16) {
            const size_t at = ((static_cast<size_t>(li) * kcmax + kc) * 128 + l) * 8 + j;
            wtab[at] = to_bf16_bits(w);
            wtab[at + 64 * 8] = 0;
            continue;
          }
          if (f16) {
            const _Float16 h = static_cast<_Float16>(w);
            uint16_t hb;
            std::memcpy(&hb, &h, 2);
            const size_t at = ((static_cast<size_t>(li) * kcmax + kc) * 128 + l) * 8 + j;
            wtab[at] = hb;
            wtab[at + 64 * 8] = 0;
            continue;
          }
          const uint16_t hi = to_bf16_bits(w);
          const uint32_t hb = static_cast<uint32_t>(hi) << 16;
          float hv;
          std::memcpy(&hv, &hb, 4);
          const size_t at = ((static_cast<size_t>(li) * kcmax + kc) * 128 + l) * 8 + j;
          wtab[at] = hi;
          wtab[at + 64 * 8] = to_bf16_bits(w - hv);
        }
      }
    }
  }
  // low-pass B fragments: K-step ks, lane l holds H[16 ks + 8 (l / 32) + j][l % 32],
  // H[k][n] = h[n R + K - 1 - k], as hi and lo terms (BF16 with four sample planes, FP16 with two)
  const int nks = (31 * p->R + p->K + 15) / 16;
  // rounded up to whole batches of 4 K-steps; the extra K-steps have zero taps
  std::vector<uint16_t> ftab(static_cast<size_t>((nks + 3) & ~3) * 2 * 64 * 8, 0);
  for (int ks = 0; ks < nks; ++ks) {
    for (int l = 0; l < 64; ++l) {
      for (int j = 0; j < 8; ++j) {
        const int idx = (l & 31) * p->R + p->K - 1 - (16 * ks + 8 * (l >> 5) + j);
        const float h = idx >= 0 && idx < p->K ? static_cast<float>(std::ldexp(taps[idx], ts)) : 0.f;
        uint16_t hi, lo;
        if (mt_planes(p) == 2) {
          // two sample planes: the low-pass runs on FP16 MFMA, taps as FP16 hi + lo
          const _Float16 h1 = static_cast<_Float16>(h);
          const _Float16 h2 = static_cast<_Float16>(h - static_cast<float>(h1));
          std::memcpy(&hi, &h1, 2);
          std::memcpy(&lo, &h2, 2);
        } else {
          hi = to_bf16_bits(h);
          const uint32_t hb = static_cast<uint32_t>(hi) << 16;
          float hv;
          std::memcpy(&hv, &hb, 4);
          lo = to_bf16_bits(h - hv);
        }
        ftab[((static_cast<size_t>(2 * ks) * 64) + l) * 8 + j] = hi;
        ftab[((static_cast<size_t>(2 * ks + 1) * 64) + l) * 8 + j] = lo;
      }
    }
  }
  p->mt_gmax = gmax;
  p->mt_kcmax = kcmax;
  // every (tile, residue) K-chunk runs on nwave / GT wavefronts x 4 output tiles
  long long chunks = 0;
  for (int li = 0; li < nlist; ++li) chunks += static_cast<long long>(groups[li].size()) / gpc;
  // per K-chunk and 32 x 32 output tile: 6 MFMAs (split samples), 4 (single-term samples) or 2 (FP16)
  const int mfma_per_chunk = mt_planes(p) == 4 ? 6 : (w1 ? 2 : 4);
  p->mt_flop_per_frame = chunks * (p->mt_nwave / res) * 4 * mfma_per_chunk * (2LL * 32 * 32 * 16) * p->mt_nqt;
  // low-pass: 3 MFMAs per K-step and column block (BF16 hi/lo x hi/lo), 2 with two sample planes
  // (FP16 taps hi + lo times one FP16 term of |b|)
  // (TD_BF16G: taps as one FP16 term, one product)
  const int fir_mfma = p->bf_mode == SONAR_BF_TD_BF16G ? 1 : (mt_planes(p) == 2 ? 2 : 3);
  for (int q0 = 0; q0 < p->mt_qc; q0 += 32) {
    const int nval = std::min(32, p->mt_qc - q0);
    p->mt_flop_per_frame += static_cast<long long>((nval - 1) * p->R + p->K + 15) / 16 * fir_mfma *
                            (2LL * 32 * 32 * 16) * nt * p->mt_nqt;
  }
  bool ok = dev_alloc(&p->d_mt_g, gtab.size(), total) == hipSuccess &&
            dev_alloc(&p->d_mt_w, wtab.size(), total) == hipSuccess &&
            dev_alloc(&p->d_mt_kcr, kcr.size(), total) == hipSuccess &&
            dev_alloc(&p->d_mt_perm, perm.size(), total) == hipSuccess &&
            dev_alloc(&p->d_mt_fir, ftab.size(), total) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return fail(SONAR_E_NOMEM, "device allocation of the MFMA beamformer tables failed");
  }
  e = hipMemcpy(p->d_mt_g, gtab.data(), gtab.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_mt_w, wtab.data(), wtab.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_mt_kcr, kcr.data(), kcr.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_mt_perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_mt_fir, ftab.data(), ftab.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "MFMA beamformer table upload");
}

// largest |p_m| fs / c over the microphones: the delay bound over all directions
double delay_bound(const double* pos, int M, double fs, double c) {
  double bmax = 0.0;
  for (int m = 0; m < M; ++m) {
    const double* q = pos + 3 * m;
    bmax = std::fmax(bmax, std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) * fs / c);
  }
  return bmax * (1.0 + 1e-9) + 1e-9;
}

// Side streams of sonar_energyscape_multi, one pool per device, created with the device's
// first plan (outside any graph capture) and kept until the process ends; default priority.
constexpr int MULTI_SIDE_STREAMS = 3;
constexpr int MULTI_MAX_DEVICES = 64;
struct side_pool {
  bool ready = false;
  hipStream_t s[MULTI_SIDE_STREAMS] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[MULTI_SIDE_STREAMS] = {};
  std::mutex mu;
};
side_pool g_side_pools[MULTI_MAX_DEVICES];
std::mutex g_side_pools_mu;

void create_side_pool(int dev) {
  if (dev < 0 || dev >= MULTI_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lk(g_side_pools_mu);
  side_pool& p = g_side_pools[dev];
  if (p.ready) return;
  hipError_t e = hipEventCreateWithFlags(&p.fork, hipEventDisableTiming);
  for (int i = 0; i < MULTI_SIDE_STREAMS && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&p.s[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p.join[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) p.ready = true;
  else (void)hipGetLastError();   // without the pool, multi enqueues everything on the caller's stream
}

side_pool* side_pool_of(int dev) {
  if (dev < 0 || dev >= MULTI_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_side_pools_mu);
  return g_side_pools[dev].ready ? &g_side_pools[dev] : nullptr;
}

// Static scratch of sonar_energyscape_batch_static: device memory that needs no allocation call.
// Each device holds its own copy from the time the code object is loaded until the process ends.
// Host code never uses the array's name as an address: the device address is taken once per
// device by hipGetSymbolAddress (with that device current) and kept in g_scratch_addr.
struct scratch_slot {
  bool tried = false;
  void* addr = nullptr;
  hipError_t err = hipSuccess;
};
scratch_slot g_scratch_addr[MULTI_MAX_DEVICES];
std::mutex g_scratch_mu;

// takes the device address of `scratch` on device dev (the current device), once
void resolve_scratch(int dev) {
  if (dev < 0 || dev >= MULTI_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  scratch_slot& s = g_scratch_addr[dev];
  if (s.tried) return;
  s.tried = true;
  void* ptr = nullptr;
  s.err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (s.err == hipSuccess) s.addr = ptr;
  else (void)hipGetLastError();
}

// workgroup size the next plan creation on this thread must give the MFMA beamformer
// (0: the largest-throughput rule, 4 waves where the staging fits, else 8); set only by
// sonar_plan_create_tuned while it tries the candidates
thread_local int g_mt_nwave_hint = 0;
// log2 of the smallest per-phase transform length the next frequency-domain plan on this thread
// must use (0: the default rule); set only by sonar_plan_create_tuned while it tries the candidates
thread_local int g_fd_logl_hint = 0;

int check_exec(const sonar_plan_s* p, const void* a, const void* b, int F) {
  if (!p) return fail(SONAR_E_INVALID, "plan is NULL");
  if (!a || !b) return fail(SONAR_E_INVALID, "NULL buffer");
  if (F < 1 || F > p->max_frames)
    return fail(SONAR_E_INVALID, "F=%d outside [1, max_frames=%d]", F, p->max_frames);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(SONAR_E_INVALID, "current device %d is not the plan's device %d", dev, p->device);
  return SONAR_OK;
}

}  // namespace

extern "C" {

const char* sonar_status_string(int status) {
  switch (status) {
    case SONAR_OK: return "success";
    case SONAR_E_INVALID: return "invalid argument";
    case SONAR_E_NOMEM: return "out of device memory";
    case SONAR_E_HIP: return "HIP runtime error";
    case SONAR_E_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

const char* sonar_last_error(void) { return g_last_error.c_str(); }

int sonar_plan_create(const sonar_plan_desc* desc, hipStream_t stream, sonar_plan* out) {
  g_last_error.clear();
  if (!desc || !out) return fail(SONAR_E_INVALID, "desc or out is NULL");
  const sonar_plan_desc& d = *desc;
  if (d.n_mics < 1 || !d.mic_pos) return fail(SONAR_E_INVALID, "n_mics must be >= 1 with mic_pos");
  if (d.chirp_len < 1 || !d.chirp) return fail(SONAR_E_INVALID, "chirp_len must be >= 1 with chirp");
  if (d.n_dirs < 1 || !d.dirs) return fail(SONAR_E_INVALID, "n_dirs must be >= 1 with dirs");
  if (!(d.fs_hz > 0) || !std::isfinite(d.fs_hz)) return fail(SONAR_E_INVALID, "fs_hz must be > 0");
  if (!(d.c_mps > 0) || !std::isfinite(d.c_mps)) return fail(SONAR_E_INVALID, "c_mps must be > 0");
  if (d.n_samples < d.chirp_len) return fail(SONAR_E_INVALID, "n_samples must be >= chirp_len");
  if (d.decim < 1) return fail(SONAR_E_INVALID, "decim must be >= 1");
  if (d.max_frames < 1) return fail(SONAR_E_INVALID, "max_frames must be >= 1");
  if (d.sample_dtype < SONAR_F32 || d.sample_dtype > SONAR_BF16)
    return fail(SONAR_E_INVALID, "unknown sample_dtype %d", d.sample_dtype);
  if (d.bf_mode < SONAR_BF_TD_LINEAR || d.bf_mode > SONAR_BF_TD_BF16G)
    return fail(SONAR_E_INVALID, "unknown bf_mode %d", d.bf_mode);
  if (!finite_all(d.mic_pos, 3 * static_cast<size_t>(d.n_mics)) ||
      !finite_all(d.dirs, 3 * static_cast<size_t>(d.n_dirs)) ||
      !finite_all(d.chirp, static_cast<size_t>(d.chirp_len)))
    return fail(SONAR_E_INVALID, "non-finite geometry, direction or chirp value");
  for (int i = 0; i < d.n_dirs; ++i) {
    const double* u = d.dirs + 3 * i;
    const double n = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (std::fabs(n - 1.0) > 1e-9) return fail(SONAR_E_INVALID, "direction %d is not a unit vector", i);
  }

  auto* p = new (std::nothrow) sonar_plan_s();
  if (!p) return fail(SONAR_E_NOMEM, "host allocation failed");
  p->M = d.n_mics;
  p->L = d.chirp_len;
  p->D = d.n_dirs;
  p->N = d.n_samples;
  p->R = d.decim;
  p->fs = d.fs_hz;
  p->c = d.c_mps;
  p->bf_mode = d.bf_mode;
  p->dtype = d.sample_dtype;
  p->max_frames = d.max_frames;
  p->n0 = d.gate_begin;
  p->n1 = d.gate_end;
  if (p->n0 == 0 && p->n1 == 0) p->n1 = p->N;
  if (p->n0 < 0 || p->n0 >= p->n1 || p->n1 > p->N) {
    delete p;
    return fail(SONAR_E_INVALID, "gate [%d, %d) outside [0, N=%d)", d.gate_begin, d.gate_end, d.n_samples);
  }
  p->band_lo = d.band_lo_hz;
  p->band_hi = d.band_hi_hz;
  p->band_on = !(d.band_lo_hz == 0.0 && d.band_hi_hz == 0.0);
  if (p->band_on && !(d.band_lo_hz >= 0.0 && d.band_hi_hz >= d.band_lo_hz)) {
    delete p;
    return fail(SONAR_E_INVALID, "band must satisfy 0 <= lo <= hi");
  }

  // FFT length
  const long long need = static_cast<long long>(p->N) + p->L - 1;
  long long P = d.fft_len;
  if (P == 0) {
    P = 32;
    while (P < need) P *= 2;
  } else if (P < need || (P % 2) != 0) {
    delete p;
    return fail(SONAR_E_INVALID, "fft_len %d must be even and >= N + L - 1 = %lld", d.fft_len, need);
  } else if (!is_pow2(P) || P < 32) {
    // a valid length (the definition only needs P even and >= N + L - 1) that the library's
    // transforms do not cover: they are radix-2^k
    delete p;
    return fail(SONAR_E_UNSUPPORTED, "fft_len %d: the library transforms powers of two >= 32 only", d.fft_len);
  }
  if (P > 2LL * MB_MAX_R * (1 << MB_LOGN2)) {
    delete p;
    return fail(SONAR_E_UNSUPPORTED, "FFT length %lld above %d is not supported", P, 2 * MB_MAX_R * (1 << MB_LOGN2));
  }
  p->P = static_cast<int>(P);
  p->NF = p->P / 2;
  p->logNF = ilog2(p->NF);

  // envelope low-pass
  std::vector<double> taps;
  if (d.lpf_len == 0) {
    taps = default_lowpass(p->R);
  } else {
    if (d.lpf_len < 1 || (d.lpf_len % 2) == 0 || !d.lpf_taps) {
      delete p;
      return fail(SONAR_E_INVALID, "lpf_len must be odd with lpf_taps (or 0 for the default)");
    }
    if (!finite_all(d.lpf_taps, static_cast<size_t>(d.lpf_len))) {
      delete p;
      return fail(SONAR_E_INVALID, "non-finite low-pass tap");
    }
    taps.assign(d.lpf_taps, d.lpf_taps + d.lpf_len);
  }
  p->K = static_cast<int>(taps.size());
  p->hk = (p->K - 1) / 2;
  p->Q = (p->n1 - p->n0 + p->R - 1) / p->R;
  p->G = (p->Q - 1) * p->R + p->K;

  // bounds of the integer offset o = floor(-Dl): |Dl| <= fs |p_m| / c (|u| = 1)
  const double bmax = delay_bound(d.mic_pos, p->M, p->fs, p->c);
  // DELAY_MARGIN extra samples on each side let sonar_plan_set_positions move the microphones
  p->omin = static_cast<int>(std::floor(-bmax)) - DELAY_MARGIN;
  p->omax = static_cast<int>(std::floor(bmax)) + DELAY_MARGIN;
  p->spread = p->omax - p->omin;

  // time-domain tiling
  p->td_tn = 64 * TD_NB - 1;
  if (p->K > p->td_tn) {
    delete p;
    return fail(SONAR_E_UNSUPPORTED, "low-pass length %d above %d is not supported", p->K, p->td_tn);
  }
  p->td_vshift = p->bf_mode == SONAR_BF_TD_CUBIC ? 1 : 0;
  if ((p->M << p->td_vshift) > TD_MAX_MICS) {
    delete p;
    return fail(SONAR_E_UNSUPPORTED, "more than %d microphones is not supported%s", TD_MAX_MICS >> p->td_vshift,
                p->td_vshift ? " by TD_CUBIC" : "");
  }
  if (64 * TD_NB + p->spread + 1 > 2 * TD_MAX_ROW_PAIRS) {
    delete p;
    return fail(SONAR_E_UNSUPPORTED, "array aperture too large (%d samples of delay spread)", p->spread);
  }
  // tile starts in the MF rows must be even (16-byte aligned copies into LDS)
  p->td_qc = (p->td_tn - p->K) / p->R + 1;
  if ((p->td_qc * p->R) & 1) p->td_qc -= 1;
  if (p->td_qc < 1) {
    delete p;
    return fail(SONAR_E_UNSUPPORTED, "low-pass length %d too long for decimation %d", p->K, p->R);
  }
  p->td_tn -= p->td_tn & 1;
  p->td_nqc = (p->Q + p->td_qc - 1) / p->td_qc;
  p->td_nbc = (p->G + p->td_tn - 1) / p->td_tn;
  // staged row length (LDS row stride): a fixed 2 * TD_MAX_ROW_PAIRS samples,
  // enough for 64 * TD_NB beam samples plus the delay spread
  p->td_ws = 2 * TD_MAX_ROW_PAIRS;
  // one LDS buffer holds mc microphone rows of ws samples, one row per wavefront
  int mc = TD_LDS_BYTES / (p->td_ws * static_cast<int>(sizeof(float2)));
  if (mc > TD_NW) mc = TD_NW;
  if (mc < 1) {
    delete p;
    return fail(SONAR_E_UNSUPPORTED, "array aperture too large for the beamformer tile");
  }
  p->td_mc = mc < p->M ? mc : p->M;
  // every staging copy reads 2 * TD_MAX_ROW_PAIRS samples from its tile start
  const long long need_env = static_cast<long long>(p->td_nqc - 1) * p->td_qc * p->R + 2 * TD_MAX_ROW_PAIRS;
  const long long need_beam = static_cast<long long>(p->td_nbc - 1) * p->td_tn + 2 * TD_MAX_ROW_PAIRS;
  long long row = need_env > need_beam ? need_env : need_beam;
  if (mt_planes(p)) {
    // MFMA tiles: nwave * 128 beam samples, rows staged over the tile plus the delay span;
    // 4-wave workgroups where the staging fits (two per CU), else 8 waves
    p->mt_ntiles = (p->D + 31) / 32;
    p->mt_nmc = (p->M + mt_mics(p) - 1) / mt_mics(p);
    p->mt_nwave = 0;
    for (const int nwave : {MT_NWAVE_SMALL, MT_NWAVE_LARGE}) {
      if (g_mt_nwave_hint != 0 && nwave != g_mt_nwave_hint) continue;
      const int ns = nwave * 128;
      int qc = (ns - p->K) / p->R + 1;
      while (qc > 0 && (qc * p->R) % 4 != 0) qc -= 1;
      if (qc < 1) continue;
      p->mt_nwave = nwave;
      p->mt_qc = qc;
      p->mt_nqt = (p->Q + qc - 1) / qc;
      p->mt_wrow = (4 + ns + p->spread + 16 + 7) / 8 * 8;   // window start aligned down by 0 or 4
      const size_t lds_cap = nwave == MT_NWAVE_SMALL ? 80 * 1024 : 160 * 1024;
      if (static_cast<long long>(mt_planes(p)) * mt_mics(p) * (p->mt_wrow / 8) <= static_cast<long long>(MT_SPT) * nwave * 64 &&
          mt_smem_bytes(p) <= lds_cap)
        break;
      p->mt_nwave = 0;
    }
    if (p->mt_nwave == 0) {
      delete p;
      return fail(SONAR_E_UNSUPPORTED, "array aperture or low-pass length too large for the BF16 time-domain beamformer");
    }
    const long long need_mt = static_cast<long long>(p->mt_nqt - 1) * p->mt_qc * p->R + p->mt_wrow;
    if (need_mt > row) row = need_mt;
  }
  row = (row + 7) / 8 * 8;
  p->row = static_cast<int>(row);
  // complex rows, then (MFMA modes) mt_planes(p) 16-bit planes per microphone: 4 16-bit values per
  // complex64; TD_F16 frames end with a 16-byte header (the sample scale)
  p->mf_fstride = static_cast<long long>(p->M) * p->row * (4 + mt_planes(p)) / 4 + (mt_f16(p) ? MF_F16_HEADER : 0);
  p->origin = static_cast<long long>(p->n0) - p->hk + p->omin;

  // frequency-domain layout: the stored bins are exactly those the band mask keeps
  if (p->band_on) {
    int lo = -1, hi = -1;
    for (int k = 0; k <= p->NF; ++k) {
      const double f = static_cast<double>(k) * (p->fs / static_cast<double>(p->P));
      if (f >= p->band_lo && f <= p->band_hi) {
        if (lo < 0) lo = k;
        hi = k;
      }
    }
    if (lo < 0) {
      delete p;
      return fail(SONAR_E_INVALID, "band [%g, %g] Hz holds no frequency bin", p->band_lo, p->band_hi);
    }
    p->k_lo = lo;
    p->kb = hi - lo + 1;
  } else {
    p->k_lo = 0;
    p->kb = p->NF + 1;
  }
  p->kb_pad = (p->kb + 15) / 16 * 16;
  {
    // Inverse layout: phases of L points with the stored bins folded modulo L.  The fused inverse +
    // envelope keeps at most FD_MAX_FOLD bins per slot in registers, so L >= kb / FD_MAX_FOLD; by
    // default the fewest folds whose L is at most FD_FOLD1_MAX_L (512-thread transforms).  The tuner
    // may ask for another L (g_fd_logl_hint).
    auto pow2_at_least = [](long long v) {
      long long l = 16;
      while (l < v) l *= 2;
      return l;
    };
    const long long hard = pow2_at_least((p->kb + FD_MAX_FOLD - 1) / FD_MAX_FOLD);
    long long L = 0;
    for (int nf = 1; nf <= FD_MAX_FOLD && L == 0; ++nf) {
      const long long l = pow2_at_least((p->kb + nf - 1) / nf);
      if (l <= FD_FOLD1_MAX_L) L = l;
    }
    if (L == 0) L = hard;
    if (g_fd_logl_hint > 0) L = std::max(hard, 1LL << g_fd_logl_hint);
    // the fused kernel keeps one phase's magnitudes with a circular halo of hk / R' + 2 entries on each
    // side inside its L-point transform buffer (2 (L + L / 16) floats)
    const long long halo = L <= p->P ? (p->K - 1) / 2 / (p->P / L) + 2 : 0;
    p->fd_fused = L <= (1LL << FD_MAX_LOGL) && L <= p->P && p->K <= FD_MAX_TAPS && p->P / L <= FD_MAX_PHASES &&
                  2 * halo + L <= 2 * (L + L / 16);
    if (!p->fd_fused) L = std::min<long long>(hard, std::min<long long>(1LL << FD_MAX_LOGL, p->P));
    p->fd_L = static_cast<int>(L);
    p->fd_logL = ilog2(p->fd_L);
    p->fd_R = p->P / p->fd_L;
    p->fd_nfold = (p->kb + p->fd_L - 1) / p->fd_L;
    // LDS: the per-phase variant holds the Q range-bin sums beside the transform; where the whole beam
    // window fits there too, the fused kernel keeps it and runs the low-pass once at the end instead
    p->fd_fused = p->fd_fused && fd_envw_static_lds(p->fd_logL) + fd_env_dyn_lds(p) <= 160 * 1024;
    p->fd_win = p->fd_fused && fd_envw_static_lds(p->fd_logL) + fd_envw_dyn_lds(p) <= 160 * 1024;
  }
  const bool fd = !is_td(p);

  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(SONAR_E_HIP, "hipGetDevice failed");
  }
  create_side_pool(p->device);
  resolve_scratch(p->device);
  if (hipDeviceGetAttribute(&p->cu_count, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
      p->cu_count < 1) {
    (void)hipGetLastError();
    p->cu_count = 256;
  }
  hipError_t e = init_td_kernel_attributes();
  if (e == hipSuccess) e = init_mt_kernel_attributes();
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "kernel attributes");
  }

  // one-time allocation of every device buffer
  size_t total = 0;
  const size_t dm = static_cast<size_t>(p->D) * p->M;
  const size_t dtab_elems = dm << p->td_vshift;
  const size_t mf_elems = fd ? 0 : static_cast<size_t>(p->max_frames) * p->mf_fstride;
  const size_t spec_elems = fd ? 0 : static_cast<size_t>(p->max_frames) * p->M * (p->NF + 1);
  const size_t band_elems = fd ? static_cast<size_t>(p->max_frames) * p->kb * p->M : 0;
  const size_t bspec_elems = fd ? static_cast<size_t>(p->max_frames) * p->D * p->kb_pad : 0;
  const size_t beam_elems = fd && !p->fd_fused ? static_cast<size_t>(p->max_frames) * p->D * p->G : 0;
  const size_t fdtw_elems = fd ? static_cast<size_t>(fd_tw_len(p->fd_L, p->P)) : 0;
  const size_t aux_bytes = static_cast<size_t>(p->P) * sizeof(double2);
  const bool big = p->NF > (1 << MB_LOGN2);
  const size_t big_elems = big ? static_cast<size_t>(p->max_frames) * p->M * 2 * p->NF : 0;
  const size_t tw2_elems = big ? static_cast<size_t>(fft_tw_len(1 << MB_LOGN2)) : 0;
  bool ok = dev_alloc(&p->d_dtab, dtab_elems, &total) == hipSuccess &&
            dev_alloc(&p->d_dl, dm, &total) == hipSuccess &&
            dev_alloc(&p->d_pos, 3 * static_cast<size_t>(p->M), &total) == hipSuccess &&
            dev_alloc(&p->d_dirs, 3 * static_cast<size_t>(p->D), &total) == hipSuccess &&
            dev_alloc(&p->d_chirp, static_cast<size_t>(p->L), &total) == hipSuccess &&
            dev_alloc(&p->d_taps, static_cast<size_t>(p->K), &total) == hipSuccess &&
            dev_alloc(&p->d_cspec, static_cast<size_t>(p->NF) + 1, &total) == hipSuccess &&
            dev_alloc(&p->d_tw, static_cast<size_t>(fft_tw_len(p->NF)), &total) == hipSuccess &&
            dev_alloc(&p->d_mf, mf_elems, &total) == hipSuccess &&
            dev_alloc(&p->d_spec, spec_elems, &total) == hipSuccess &&
            dev_alloc(&p->d_fdspec, band_elems, &total) == hipSuccess &&
            dev_alloc(&p->d_bspec, bspec_elems, &total) == hipSuccess &&
            dev_alloc(&p->d_beam, beam_elems, &total) == hipSuccess &&
            dev_alloc(&p->d_fdtw, fdtw_elems, &total) == hipSuccess &&
            dev_alloc(&p->d_fdstep, fd ? dm : 0, &total) == hipSuccess &&
            dev_alloc(&p->d_big, big_elems, &total) == hipSuccess &&
            dev_alloc(&p->d_tw2, tw2_elems, &total) == hipSuccess &&
            dev_alloc(&p->d_fbound, mt_f16(p) ? static_cast<size_t>(p->max_frames) * p->M : 0, &total) == hipSuccess &&
            dev_alloc(reinterpret_cast<char**>(&p->d_aux), aux_bytes, &total) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_plan(p);
    return fail(SONAR_E_NOMEM, "device allocation of %zu bytes failed", total);
  }
  p->ws_bytes = total;
  p->beam_cap = beam_elems;

  std::vector<float> taps_f(taps.begin(), taps.end());
  ok = hipMemcpyAsync(p->d_pos, d.mic_pos, 3 * sizeof(double) * p->M, hipMemcpyHostToDevice, stream) == hipSuccess &&
       hipMemcpyAsync(p->d_dirs, d.dirs, 3 * sizeof(double) * p->D, hipMemcpyHostToDevice, stream) == hipSuccess &&
       hipMemcpyAsync(p->d_chirp, d.chirp, sizeof(double) * p->L, hipMemcpyHostToDevice, stream) == hipSuccess &&
       hipMemcpyAsync(p->d_taps, taps_f.data(), sizeof(float) * p->K, hipMemcpyHostToDevice, stream) == hipSuccess;
  if (!ok) {
    e = hipGetLastError();
    free_plan(p);
    return hip_fail(e, "plan upload");
  }
  e = launch_build_tables(p, stream);
  if (e == hipSuccess && fd) e = launch_build_fd_tables(p, stream);
  if (e == hipSuccess && mt_planes(p)) {
    p->h_dirs.assign(d.dirs, d.dirs + 3 * static_cast<size_t>(p->D));
    p->h_taps = taps;
    const int st = build_mt_tables(p, d.mic_pos, d.dirs, taps, stream, &total);
    if (st != SONAR_OK) {
      free_plan(p);
      return st;
    }
    p->ws_bytes = total;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "plan table build");
  }
  *out = p;
  return SONAR_OK;
}

int sonar_plan_destroy(sonar_plan plan) {
  free_plan(plan);
  return SONAR_OK;
}

int sonar_plan_query(sonar_plan p, int32_t what, int64_t* value) {
  if (!p || !value) return fail(SONAR_E_INVALID, "plan or value is NULL");
  switch (what) {
    case SONAR_Q_RANGE_BINS: *value = p->Q; break;
    case SONAR_Q_BEAM_LEN: *value = p->G; break;
    case SONAR_Q_FFT_LEN: *value = p->P; break;
    case SONAR_Q_MF_ROW: *value = p->row; break;
    case SONAR_Q_MF_ORIGIN: *value = p->origin; break;
    case SONAR_Q_BAND_LO_BIN: *value = p->k_lo; break;
    case SONAR_Q_BAND_BINS: *value = p->kb; break;
    case SONAR_Q_WORKSPACE_BYTES: *value = static_cast<int64_t>(p->ws_bytes); break;
    case SONAR_Q_LPF_LEN: *value = p->K; break;
    case SONAR_Q_MATRIX_FLOP_PER_FRAME: *value = p->mt_flop_per_frame; break;
    case SONAR_Q_MT_WAVES: *value = p->mt_nwave; break;
    case SONAR_Q_BEAM_SPEC_STRIDE: *value = is_td(p) ? 0 : p->kb_pad; break;
    case SONAR_Q_FD_PHASE_LEN: *value = is_td(p) ? 0 : p->fd_L; break;
    case SONAR_Q_FD_FUSED: *value = is_td(p) ? 0 : (p->fd_fused ? 1 : 0); break;
    case SONAR_Q_MF_FRAME_ELEMS:
      *value = is_td(p) ? static_cast<int64_t>(p->mf_fstride)
                                                : static_cast<int64_t>(p->kb) * p->M;
      break;
    default: return fail(SONAR_E_INVALID, "unknown query key %d", what);
  }
  return SONAR_OK;
}

int sonar_matched_filter(sonar_plan p, const void* x, int32_t F, void* mf_out, hipStream_t stream) {
  int st = check_exec(p, x, mf_out, F);
  if (st != SONAR_OK) return st;
  hipError_t e = is_td(p) ? launch_mf_td(p, x, F, static_cast<float2*>(mf_out), stream)
                                                  : launch_mf_fd(p, x, F, static_cast<float2*>(mf_out), stream);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "matched filter launch");
}

int sonar_beamform(sonar_plan p, const void* mf_in, int32_t F, void* beam_out, hipStream_t stream) {
  int st = check_exec(p, mf_in, beam_out, F);
  if (st != SONAR_OK) return st;
  hipError_t e;
  if (is_td(p)) {
    e = launch_das_td_beam(p, static_cast<const float2*>(mf_in), F, static_cast<float2*>(beam_out), stream);
  } else {
    e = launch_fd_gemm(p, static_cast<const float2*>(mf_in), F, p->d_bspec, stream);
    if (e == hipSuccess) e = launch_fd_ifft_beam(p, p->d_bspec, F, static_cast<float2*>(beam_out), stream);
  }
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "beamform launch");
}

int sonar_beam_spectrum(sonar_plan p, const void* mf_in, int32_t F, void* spec_out, hipStream_t stream) {
  int st = check_exec(p, mf_in, spec_out, F);
  if (st != SONAR_OK) return st;
  if (is_td(p)) return fail(SONAR_E_INVALID, "sonar_beam_spectrum: the plan's beamformer is not frequency-domain");
  const hipError_t e = launch_fd_gemm(p, static_cast<const float2*>(mf_in), F, static_cast<float2*>(spec_out), stream);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "beam spectrum launch");
}

int sonar_envelope(sonar_plan p, const void* beam_in, int32_t F, float* E, hipStream_t stream) {
  int st = check_exec(p, beam_in, E, F);
  if (st != SONAR_OK) return st;
  hipError_t e = p->iir_ns > 0 ? launch_iir_envelope(p, static_cast<const float2*>(beam_in), F, E, stream)
                               : launch_envelope(p, static_cast<const float2*>(beam_in), F, E, stream);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "envelope launch");
}

namespace {

// beamformer + envelope from a matched-filter buffer of this plan's layout
hipError_t beam_env(const sonar_plan_s* p, const float2* mf, int F, float* E, hipStream_t s) {
  if (p->iir_ns > 0) {
    hipError_t e;
    if (is_td(p)) {
      e = launch_das_td_beam(p, mf, F, p->d_beam, s);
    } else {
      e = launch_fd_gemm(p, mf, F, p->d_bspec, s);
      if (e == hipSuccess) e = launch_fd_ifft_beam(p, p->d_bspec, F, p->d_beam, s);
    }
    return e == hipSuccess ? launch_iir_envelope(p, p->d_beam, F, E, s) : e;
  }
  if (p->bf_mode == SONAR_BF_TD_LINEAR || p->bf_mode == SONAR_BF_TD_NEAREST || p->bf_mode == SONAR_BF_TD_CUBIC)
    return launch_das_td_env(p, mf, F, E, s);
  if (mt_planes(p)) return launch_das_mfma_env(p, mf, F, E, s);
  hipError_t e = launch_fd_gemm(p, mf, F, p->d_bspec, s);
  if (e != hipSuccess) return e;
  if (p->fd_fused) return launch_fd_ifft_env(p, p->d_bspec, F, E, s);
  e = launch_fd_ifft_beam(p, p->d_bspec, F, p->d_beam, s);
  if (e != hipSuccess) return e;
  return launch_envelope(p, p->d_beam, F, E, s);
}

}  // namespace

int sonar_beamform_envelope(sonar_plan p, const void* mf_in, int32_t F, float* E, hipStream_t stream) {
  int st = check_exec(p, mf_in, E, F);
  if (st != SONAR_OK) return st;
  hipError_t e = beam_env(p, static_cast<const float2*>(mf_in), F, E, stream);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "beamform-envelope launch");
}

namespace {

// the whole chain for F frames on the workspace buffers that p points at
hipError_t energyscape_enqueue(const sonar_plan_s* p, const void* x, int F, float* E, hipStream_t stream) {
  hipError_t e;
  if (is_td(p)) {
    // the fused MFMA beamformer reads only the 16-bit planes: the complex rows are not written
    e = launch_mf_td(p, x, F, p->d_mf, stream, !(mt_planes(p) && p->iir_ns == 0));
    if (e == hipSuccess) e = beam_env(p, p->d_mf, F, E, stream);
  } else {
    e = launch_mf_fd(p, x, F, p->d_fdspec, stream);
    if (e == hipSuccess) e = beam_env(p, p->d_fdspec, F, E, stream);
  }
  return e;
}

// Per-frame workspace of sonar_energyscape_batch, laid out in `base` (256-byte aligned pieces)
// on a copy of the plan; returns the bytes F frames need (nothing is written when base is null).
size_t carve_workspace(sonar_plan_s* q, int F, unsigned char* base) {
  size_t off = 0;
  auto take = [&](auto** ptr, size_t elems, size_t elem_bytes) {
    off = (off + 255) / 256 * 256;
    if (base) *ptr = reinterpret_cast<std::remove_reference_t<decltype(**ptr)>*>(base + off);
    off += elems * elem_bytes;
  };
  const size_t f = static_cast<size_t>(F);
  const bool fd = !is_td(q);
  const bool big = q->NF > (1 << MB_LOGN2);
  if (!fd) {
    take(&q->d_mf, f * q->mf_fstride, sizeof(float2));
    take(&q->d_spec, f * q->M * (static_cast<size_t>(q->NF) + 1), sizeof(float2));
    if (mt_f16(q)) take(&q->d_fbound, f * q->M, sizeof(float));
  } else {
    take(&q->d_fdspec, f * q->kb * q->M, sizeof(float2));
    take(&q->d_bspec, f * q->D * q->kb_pad, sizeof(float2));
  }
  if ((fd && !q->fd_fused) || q->iir_ns > 0) take(&q->d_beam, f * q->D * q->G, sizeof(float2));
  if (big) take(&q->d_big, f * q->M * 2 * static_cast<size_t>(q->NF), sizeof(float2));
  return off;
}

}  // namespace

int sonar_energyscape_batch(sonar_plan p, const void* x, int32_t F, float* E, hipStream_t stream) {
  int st = check_exec(p, x, E, F);
  if (st != SONAR_OK) return st;
  const hipError_t e = energyscape_enqueue(p, x, F, E, stream);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "energyscape launch");
}

int sonar_energyscape_batch_static(sonar_plan p, const void* x, int32_t F, float* E, hipStream_t stream) {
  int st = check_exec(p, x, E, F);
  if (st != SONAR_OK) return st;
  const int dev = p->device;
  void* base = nullptr;
  hipError_t se = hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev >= 0 && dev < MULTI_MAX_DEVICES) {
      base = g_scratch_addr[dev].addr;
      se = g_scratch_addr[dev].err;
    }
  }
  if (!base)
    return se != hipSuccess ? hip_fail(se, "static scratch address")
                            : fail(SONAR_E_HIP, "static scratch of device %d has no address", dev);
  sonar_plan_s q = *p;   // same tables; per-frame buffers re-pointed into the static scratch
  const size_t need = carve_workspace(&q, F, nullptr);
  if (need > STATIC_SCRATCH_BYTES) {
    const size_t per = carve_workspace(&q, 1, nullptr);
    return fail(SONAR_E_INVALID, "F=%d needs %zu bytes of scratch; the static scratch holds %zu (%zu frames of this plan)",
                F, need, STATIC_SCRATCH_BYTES, per > 0 ? STATIC_SCRATCH_BYTES / per : 0);
  }
  carve_workspace(&q, F, static_cast<unsigned char*>(base));
  const hipError_t e = energyscape_enqueue(&q, x, F, E, stream);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "energyscape launch (static scratch)");
}

int sonar_energyscape_multi(const sonar_plan* plans, const void* const* x, const int32_t* frames,
                            float* const* E, int32_t n, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!plans || !x || !frames || !E)))
    return fail(SONAR_E_INVALID, "multi: NULL item arrays or n < 0");
  for (int i = 0; i < n; ++i) {
    const int st = check_exec(plans[i], x[i], E[i], frames[i]);
    if (st != SONAR_OK) {
      const std::string why = sonar_last_error();
      return fail(st, "multi item %d: %s", i, why.c_str());
    }
  }
  if (n == 0) return SONAR_OK;
  // Items of the MFMA time-domain modes (FIR envelope, each plan once in the call) run as one
  // persistent beamformer launch per compatible group of up to MT_MULTI_MAX_ITEMS items, after
  // their matched filters, all on the caller's stream; the other items follow below.
  std::vector<int> rest;
  {
    std::vector<int> elig;
    for (int i = 0; i < n; ++i) {
      bool unique = true;
      for (int j = 0; j < n; ++j)
        if (j != i && plans[j] == plans[i]) unique = false;
      if (unique && mt_planes(plans[i]) && plans[i]->iir_ns == 0) elig.push_back(i);
      else rest.push_back(i);
    }
    std::vector<char> done(n, 0);
    for (size_t a = 0; a < elig.size(); ++a) {
      const int i0 = elig[a];
      if (done[i0]) continue;
      std::vector<int> grp;
      for (size_t b = a; b < elig.size() && static_cast<int>(grp.size()) < MT_MULTI_MAX_ITEMS; ++b)
        if (!done[elig[b]] && mt_multi_compatible(plans[elig[b]], plans[i0])) {
          grp.push_back(elig[b]);
          done[elig[b]] = 1;
        }
      std::vector<const sonar_plan_s*> gp;
      std::vector<const float2*> gy;
      std::vector<int> gf;
      std::vector<float*> ge;
      hipError_t e = hipSuccess;
      for (int i : grp) {
        // the persistent beamformer reads only the 16-bit planes: the complex rows are not written
        if (e == hipSuccess) e = launch_mf_td(plans[i], x[i], frames[i], plans[i]->d_mf, stream, false);
        gp.push_back(plans[i]);
        gy.push_back(plans[i]->d_mf);
        gf.push_back(frames[i]);
        ge.push_back(E[i]);
      }
      if (e == hipSuccess)
        e = launch_das_mfma_env_multi(gp.data(), gy.data(), gf.data(), ge.data(), static_cast<int>(grp.size()), stream);
      if (e != hipSuccess) return hip_fail(e, "multi persistent launch");
    }
  }
  if (rest.empty()) return SONAR_OK;
  std::vector<sonar_plan> rp;
  std::vector<const void*> rx;
  std::vector<int32_t> rf;
  std::vector<float*> re;
  for (int i : rest) {
    rp.push_back(plans[i]);
    rx.push_back(x[i]);
    rf.push_back(frames[i]);
    re.push_back(E[i]);
  }
  plans = rp.data();
  x = rx.data();
  frames = rf.data();
  E = re.data();
  n = static_cast<int32_t>(rest.size());
  side_pool* pool = side_pool_of(plans[0]->device);
  if (n < 2 || !pool) {
    for (int i = 0; i < n; ++i) {
      const int st = sonar_energyscape_batch(plans[i], x[i], frames[i], E[i], stream);
      if (st != SONAR_OK) return st;
    }
    return SONAR_OK;
  }
  // Independent items run on the caller's stream and the device's side streams, forked from
  // and joined back into the caller's stream (a graph captured on it gets parallel branches).
  // Items of one plan share its workspace and stay on one stream, in order.  Items go
  // largest first to the least loaded stream (load = frames x directions x samples).
  constexpr int NL = MULTI_SIDE_STREAMS + 1;
  std::vector<int> order(n), lane(n, -1);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto cost = [&](int i) { return static_cast<double>(frames[i]) * plans[i]->D * plans[i]->N; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  double load[NL] = {0.0};
  for (int i : order) {
    for (int j = 0; j < n; ++j)
      if (lane[j] >= 0 && plans[j] == plans[i]) lane[i] = lane[j];
    if (lane[i] < 0) lane[i] = static_cast<int>(std::min_element(load, load + NL) - load);
    load[lane[i]] += cost(i);
  }
  std::lock_guard<std::mutex> lk(pool->mu);   // the pool's events are reused by every call
  // A side stream that joined a capture stays in it until that capture ends.  If one is joined to
  // a capture other than the caller's (another stream's graph still being recorded, or the caller
  // is eager while some capture is open), the items run in order on the caller's stream instead.
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    unsigned long long cid = 0;
    hipError_t ec = hipStreamGetCaptureInfo(stream, &cs, &cid);
    bool clash = ec != hipSuccess;
    for (int k = 0; k < MULTI_SIDE_STREAMS && !clash; ++k) {
      hipStreamCaptureStatus ss = hipStreamCaptureStatusNone;
      unsigned long long sid = 0;
      ec = hipStreamGetCaptureInfo(pool->s[k], &ss, &sid);
      if (ec != hipSuccess) clash = true;
      else if (ss != hipStreamCaptureStatusNone && !(cs == hipStreamCaptureStatusActive && sid == cid)) clash = true;
    }
    if (ec != hipSuccess) (void)hipGetLastError();
    if (clash) {
      for (int i = 0; i < n; ++i) {
        const int st = sonar_energyscape_batch(plans[i], x[i], frames[i], E[i], stream);
        if (st != SONAR_OK) return st;
      }
      return SONAR_OK;
    }
  }
  bool used[NL] = {false};
  for (int i = 0; i < n; ++i) used[lane[i]] = true;
  hipError_t e = hipEventRecord(pool->fork, stream);
  for (int k = 1; k < NL && e == hipSuccess; ++k)
    if (used[k]) e = hipStreamWaitEvent(pool->s[k - 1], pool->fork, 0);
  if (e != hipSuccess) return hip_fail(e, "multi fork");
  int st = SONAR_OK;
  for (int i = 0; i < n && st == SONAR_OK; ++i)
    st = sonar_energyscape_batch(plans[i], x[i], frames[i], E[i], lane[i] == 0 ? stream : pool->s[lane[i] - 1]);
  // join every branch, also after a failed enqueue, so the caller's stream (and a capture) stays whole
  for (int k = 1; k < NL; ++k) {
    if (!used[k]) continue;
    hipError_t ej = hipEventRecord(pool->join[k - 1], pool->s[k - 1]);
    if (ej == hipSuccess) ej = hipStreamWaitEvent(stream, pool->join[k - 1], 0);
    if (ej != hipSuccess && st == SONAR_OK) st = hip_fail(ej, "multi join");
  }
  return st;
}

namespace {

// Tuning cache: one JSON object per line, {"key": "...", "mode": m, "mt_waves": w, "fd_logl": l, "ms": t},
// keyed by every descriptor field that shapes the plan, the precision class, the device's architecture and
// a hash of the geometry, directions, sweep and taps (the choice depends on all of them).  Read at every
// tuned creation (the last line of a key wins), appended after each tuning.
std::string g_tune_cache_path;
std::mutex g_tune_mu;

struct tune_choice {
  int mode = -1, nwave = 0, logl = 0;
};

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ULL;
  }
  return h;
}

void tune_key(const sonar_plan_desc& d, int precision, std::string* key) {
  uint64_t h = 14695981039346656037ULL;
  if (d.mic_pos && d.n_mics > 0) h = fnv1a(h, d.mic_pos, sizeof(double) * 3 * static_cast<size_t>(d.n_mics));
  if (d.dirs && d.n_dirs > 0) h = fnv1a(h, d.dirs, sizeof(double) * 3 * static_cast<size_t>(d.n_dirs));
  if (d.chirp && d.chirp_len > 0) h = fnv1a(h, d.chirp, sizeof(double) * static_cast<size_t>(d.chirp_len));
  if (d.lpf_taps && d.lpf_len > 0) h = fnv1a(h, d.lpf_taps, sizeof(double) * static_cast<size_t>(d.lpf_len));
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  else (void)hipGetLastError();
  char buf[512];
  snprintf(buf, sizeof(buf),
           "%s M%d L%d D%d N%d gate%d-%d R%d K%d P%d band%.9g-%.9g fs%.9g c%.9g dtype%d F%d prec%d h%016llx",
           arch.c_str(), d.n_mics, d.chirp_len, d.n_dirs, d.n_samples, d.gate_begin, d.gate_end, d.decim, d.lpf_len,
           d.fft_len, d.band_lo_hz, d.band_hi_hz, d.fs_hz, d.c_mps, d.sample_dtype, d.max_frames, precision,
           static_cast<unsigned long long>(h));
  *key = buf;
}

// integer field "name": value of a cache line
bool json_int(const std::string& line, const char* name, int* v) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return false;
  char* end = nullptr;
  const long x = std::strtol(line.c_str() + at + pat.size(), &end, 10);
  if (end == line.c_str() + at + pat.size()) return false;
  *v = static_cast<int>(x);
  return true;
}

bool cache_lookup(const std::string& path, const std::string& key, tune_choice* c) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  const std::string want = "\"key\":\"" + key + "\"";
  bool found = false;
  char buf[2048];
  while (std::fgets(buf, sizeof(buf), f)) {
    const std::string line(buf);
    if (line.find(want) == std::string::npos) continue;
    tune_choice t;
    if (json_int(line, "mode", &t.mode) && json_int(line, "mt_waves", &t.nwave) && json_int(line, "fd_logl", &t.logl)) {
      *c = t;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_append(const std::string& path, const std::string& key, const tune_choice& c, float ms) {
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "{\"key\":\"%s\",\"mode\":%d,\"mt_waves\":%d,\"fd_logl\":%d,\"ms\":%.4f}\n", key.c_str(), c.mode,
               c.nwave, c.logl, ms);
  std::fclose(f);
}

// sonar_plan_create with the tile hints of a choice
int create_with_choice(const sonar_plan_desc* desc, const tune_choice& c, hipStream_t stream, sonar_plan* out) {
  sonar_plan_desc d = *desc;
  d.bf_mode = c.mode;
  g_mt_nwave_hint = c.nwave;
  g_fd_logl_hint = c.logl;
  const int st = sonar_plan_create(&d, stream, out);
  g_mt_nwave_hint = 0;
  g_fd_logl_hint = 0;
  return st;
}

bool is_mt_mode(int m) {
  return m == SONAR_BF_TD_BF16 || m == SONAR_BF_TD_BF16X2 || m == SONAR_BF_TD_F16 || m == SONAR_BF_TD_BF16G;
}
bool is_fd_mode(int m) { return m == SONAR_BF_FD_FP32 || m == SONAR_BF_FD_BF16 || m == SONAR_BF_FD_BF16X3; }

}  // namespace

int sonar_tune_cache(const char* path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache_path = path ? path : "";
  return SONAR_OK;
}

int sonar_plan_create_tuned(const sonar_plan_desc* desc, int32_t precision, hipStream_t stream,
                            sonar_plan* out, int32_t* chosen_mode) {
  if (!desc || !out) return fail(SONAR_E_INVALID, "desc and out must not be NULL");
  if (precision != SONAR_PREC_FP32 && precision != SONAR_PREC_BF16)
    return fail(SONAR_E_INVALID, "precision %d is not a sonar_precision", precision);
  std::string cache;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    cache = g_tune_cache_path;
  }
  std::string key;
  if (!cache.empty()) tune_key(*desc, precision, &key);
  tune_choice hit;
  if (!cache.empty() && cache_lookup(cache, key, &hit)) {
    sonar_plan p = nullptr;
    if (create_with_choice(desc, hit, stream, &p) == SONAR_OK) {
      *out = p;
      if (chosen_mode) *chosen_mode = hit.mode;
      return SONAR_OK;
    }
    g_last_error.clear();   // a stale entry: tune again
  }
  std::vector<int> modes = {SONAR_BF_TD_LINEAR, SONAR_BF_FD_FP32, SONAR_BF_FD_BF16X3};
  if (precision == SONAR_PREC_BF16) {
    modes.push_back(SONAR_BF_TD_BF16);
    modes.push_back(SONAR_BF_TD_F16);
    if (desc->n_mics >= 32) {
      modes.push_back(SONAR_BF_FD_BF16);
      modes.push_back(SONAR_BF_TD_BF16X2);
      modes.push_back(SONAR_BF_TD_BF16G);
    }
  }
  // candidates: the MFMA time-domain modes with both workgroup shapes; the frequency-domain modes
  // with their default phase length, then half and twice it (added once the default is known)
  std::vector<tune_choice> cands;
  for (int m : modes) {
    if (is_mt_mode(m)) {
      cands.push_back({m, MT_NWAVE_SMALL, 0});
      cands.push_back({m, MT_NWAVE_LARGE, 0});
    } else {
      cands.push_back({m, 0, 0});
    }
  }
  const int F = desc->max_frames > 0 ? desc->max_frames : 1;
  const size_t in_bytes = static_cast<size_t>(F) * (desc->n_mics > 0 ? desc->n_mics : 1) *
                          (desc->n_samples > 0 ? desc->n_samples : 1) *
                          (desc->sample_dtype == SONAR_F32 ? 4 : 2);
  void* xin = nullptr;
  float* eout = nullptr;
  sonar_plan best = nullptr;
  tune_choice best_c;
  int last_status = SONAR_E_UNSUPPORTED;
  float best_ms = 0.f;
  std::string last_msg = "no beamformer mode could be planned";
  std::vector<std::pair<int, int>> fd_seen;   // (mode, phase length) already timed
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he == hipSuccess) he = hipMalloc(&xin, in_bytes);
  if (he == hipSuccess) he = hipMemsetAsync(xin, 0, in_bytes, stream);
  for (size_t i = 0; he == hipSuccess && i < cands.size(); ++i) {
    const tune_choice c = cands[i];
    sonar_plan p = nullptr;
    const int st = create_with_choice(desc, c, stream, &p);
    if (st != SONAR_OK) {
      last_status = st;
      last_msg = sonar_last_error();
      if (st == SONAR_E_INVALID) break;   // the descriptor itself is bad
      continue;
    }
    tune_choice got = c;
    got.nwave = is_mt_mode(c.mode) ? p->mt_nwave : 0;
    got.logl = is_fd_mode(c.mode) ? p->fd_logL : 0;
    if (is_fd_mode(c.mode)) {
      if (std::find(fd_seen.begin(), fd_seen.end(), std::make_pair(c.mode, p->fd_logL)) != fd_seen.end()) {
        sonar_plan_destroy(p);   // the hint was clamped to a length already timed
        continue;
      }
      fd_seen.push_back({c.mode, p->fd_logL});
      if (c.logl == 0 && p->fd_fused) {
        if (p->fd_logL > 4) cands.push_back({c.mode, 0, p->fd_logL - 1});
        if (p->fd_logL < FD_MAX_LOGL) cands.push_back({c.mode, 0, p->fd_logL + 1});
      }
    }
    if (!eout) he = hipMalloc(reinterpret_cast<void**>(&eout), static_cast<size_t>(F) * p->D * p->Q * sizeof(float));
    float ms = 0.f;
    int rs = he == hipSuccess ? sonar_energyscape_batch(p, xin, F, eout, stream) : SONAR_E_HIP;   // warm-up
    if (rs == SONAR_OK) he = hipEventRecord(e0, stream);
    for (int r = 0; rs == SONAR_OK && he == hipSuccess && r < 3; ++r) rs = sonar_energyscape_batch(p, xin, F, eout, stream);
    if (rs == SONAR_OK && he == hipSuccess) he = hipEventRecord(e1, stream);
    if (rs == SONAR_OK && he == hipSuccess) he = hipEventSynchronize(e1);
    if (rs == SONAR_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (rs != SONAR_OK || he != hipSuccess) {
      sonar_plan_destroy(p);
      last_status = rs != SONAR_OK ? rs : SONAR_E_HIP;
      break;
    }
    if (!best || ms < best_ms) {
      if (best) sonar_plan_destroy(best);
      best = p;
      best_ms = ms;
      best_c = got;
    } else {
      sonar_plan_destroy(p);
    }
  }
  if (he == hipSuccess) he = hipStreamSynchronize(stream);
  (void)hipFree(xin);
  (void)hipFree(eout);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (he != hipSuccess) {
    if (best) sonar_plan_destroy(best);
    return hip_fail(he, "mode tuning");
  }
  if (!best) return fail(last_status, "%s", last_msg.c_str());
  if (!cache.empty()) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    cache_append(cache, key, best_c, best_ms / 3.0f);
  }
  *out = best;
  if (chosen_mode) *chosen_mode = best_c.mode;
  return SONAR_OK;
}


namespace {

// the beam window workspace [max_frames][D][G'] (plans with a fused envelope hold only a placeholder)
int ensure_beam_workspace(sonar_plan_s* p, size_t* total) {
  const size_t need = static_cast<size_t>(p->max_frames) * p->D * p->G;
  if (p->beam_cap >= need) return SONAR_OK;
  float2* nb = nullptr;
  if (dev_alloc(&nb, need, total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SONAR_E_NOMEM, "beam window workspace (%zu bytes) failed", sizeof(float2) * need);
  }
  (void)hipFree(p->d_beam);
  p->d_beam = nb;
  p->beam_cap = need;
  return SONAR_OK;
}

}  // namespace

int sonar_plan_enable_gradients(sonar_plan p) {
  if (!p) return fail(SONAR_E_INVALID, "plan is NULL");
  const bool td = is_td(p);
  if (p->grad_on) return SONAR_OK;
  const size_t mf = static_cast<size_t>(p->max_frames);
  size_t total = 0;
  // transform scratch: every channel of a batch, or as many as GSCR_MAX_BYTES hold (the adjoint then
  // runs its channels in chunks)
  const long long all_chans = static_cast<long long>(mf) * (td ? p->M : p->D);
  const long long cap_chans = std::max(1LL, GSCR_MAX_BYTES / (static_cast<long long>(p->P) * 8));
  p->gscr_chans = std::min(all_chans, cap_chans);
  bool ok = dev_alloc(&p->d_gdl, mf * p->D * p->M, &total) == hipSuccess &&
            dev_alloc(&p->d_gscr, static_cast<size_t>(p->gscr_chans) * p->P, &total) == hipSuccess;
  if (ok && !td)
    ok = dev_alloc(&p->d_gband, mf * p->D * p->kb, &total) == hipSuccess &&
         dev_alloc(&p->d_gspec, mf * p->M * (static_cast<size_t>(p->NF) + 1), &total) == hipSuccess;
  if (ok)
    ok = dev_alloc(&p->d_gy, mf * (td ? static_cast<size_t>(p->M) * p->P : static_cast<size_t>(p->kb) * p->M),
                   &total) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    (void)hipFree(p->d_gdl);
    (void)hipFree(p->d_gscr);
    (void)hipFree(p->d_gband);
    (void)hipFree(p->d_gspec);
    (void)hipFree(p->d_gy);
    p->d_gdl = nullptr;
    p->d_gscr = nullptr;
    p->d_gband = nullptr;
    p->d_gspec = nullptr;
    p->d_gy = nullptr;
    return fail(SONAR_E_NOMEM, "gradient workspace allocation (%zu bytes) failed", total);
  }
  const int st = ensure_beam_workspace(p, &total);
  if (st != SONAR_OK) return st;
  p->ws_bytes += total;
  p->grad_on = true;
  return SONAR_OK;
}

int sonar_energyscape_vjp(sonar_plan p, const void* mf_in, void* beam_inout, const float* dE, int32_t F,
                          void* dyhat_out, float* dx_out, double* dpos_out, hipStream_t stream) {
  int st = check_exec(p, mf_in, dE, F);
  if (st != SONAR_OK) return st;
  if (!beam_inout) return fail(SONAR_E_INVALID, "beam_inout is NULL");
  if (!p->grad_on) return fail(SONAR_E_INVALID, "call sonar_plan_enable_gradients first");
  if (p->iir_ns > 0) return fail(SONAR_E_UNSUPPORTED, "gradients are built for the FIR envelope only");
  if (dx_out && !dyhat_out) return fail(SONAR_E_INVALID, "dx_out needs dyhat_out (the matched filter's gradient)");
  if (dpos_out && p->bf_mode == SONAR_BF_TD_NEAREST)
    return fail(SONAR_E_UNSUPPORTED, "TD_NEAREST: integer delays are piecewise constant in the positions");
  if (dpos_out && (p->bf_mode == SONAR_BF_TD_F16 || p->bf_mode == SONAR_BF_TD_BF16G))
    return fail(SONAR_E_UNSUPPORTED, "TD_F16 / TD_BF16G: gridded delays are piecewise constant in the positions");
  const hipError_t e = launch_energyscape_vjp(p, static_cast<const float2*>(mf_in), static_cast<float2*>(beam_inout),
                                              dE, F, static_cast<float2*>(dyhat_out), dx_out, dpos_out, stream);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "gradient launch");
}

int sonar_energyscape_cells(sonar_plan p, const void* mf_in, const int32_t* cells, int32_t n_cells, const float* dE,
                            int32_t F, float* E_out, double* dpos_out, hipStream_t stream) {
  int st = check_exec(p, mf_in, cells, F);
  if (st != SONAR_OK) return st;
  if (!dE) return fail(SONAR_E_INVALID, "dE is NULL");
  if (!p->grad_on) return fail(SONAR_E_INVALID, "call sonar_plan_enable_gradients first");
  if (!cells_supported(p))
    return fail(SONAR_E_UNSUPPORTED,
                "energyscape cells: FP32 time-domain (linear, nearest, cubic) or frequency-domain plans with K <= 256 "
                "(and M <= 256, 2K + M <= 2P for frequency-domain plans)");
  if (dpos_out && p->bf_mode == SONAR_BF_TD_NEAREST)
    return fail(SONAR_E_UNSUPPORTED, "TD_NEAREST: integer delays are piecewise constant in the positions");
  if (n_cells < 0 || static_cast<long long>(n_cells) > static_cast<long long>(p->max_frames) * p->D)
    return fail(SONAR_E_INVALID, "n_cells=%d outside [0, max_frames * D = %lld]", n_cells,
                static_cast<long long>(p->max_frames) * p->D);
  if (!is_td(p)) {
    const long long need = static_cast<long long>(n_cells) * (2 * p->K + p->M);   // floats, one range per cell
    if (need > 2LL * p->gscr_chans * p->P)
      return fail(SONAR_E_INVALID, "n_cells=%d needs more scratch than the plan's gradient workspace: pass fewer cells",
                  n_cells);
  }
  if (n_cells == 0) {
    if (dpos_out) {
      const hipError_t e = hipMemsetAsync(dpos_out, 0, sizeof(double) * 3 * p->M, stream);
      if (e != hipSuccess) return hip_fail(e, "energyscape cells");
    }
    return SONAR_OK;
  }
  const hipError_t e = launch_energyscape_cells(p, static_cast<const float2*>(mf_in), F, cells, dE, n_cells, E_out,
                                                dpos_out, stream);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "energyscape cells launch");
}

int sonar_energyscape_backward(sonar_plan p, const void* x, const float* dE, int32_t F, float* dx_out,
                               double* dpos_out, hipStream_t stream) {
  int st = check_exec(p, x, dE, F);
  if (st != SONAR_OK) return st;
  if (!p->grad_on) return fail(SONAR_E_INVALID, "call sonar_plan_enable_gradients first");
  hipError_t e;
  const float2* mf;
  if (is_td(p)) {
    e = launch_mf_td(p, x, F, p->d_mf, stream);
    mf = p->d_mf;
    if (e == hipSuccess) e = launch_das_td_beam(p, mf, F, p->d_beam, stream);
  } else {
    e = launch_mf_fd(p, x, F, p->d_fdspec, stream);
    mf = p->d_fdspec;
    if (e == hipSuccess) e = launch_fd_gemm(p, mf, F, p->d_bspec, stream);
    if (e == hipSuccess) e = launch_fd_ifft_beam(p, p->d_bspec, F, p->d_beam, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "backward forward pass");
  return sonar_energyscape_vjp(p, mf, p->d_beam, dE, F, dx_out ? p->d_gy : nullptr, dx_out, dpos_out, stream);
}

int sonar_plan_set_positions(sonar_plan p, const double* mic_pos, hipStream_t stream) {
  if (!p || !mic_pos) return fail(SONAR_E_INVALID, "plan and mic_pos must not be NULL");
  for (int i = 0; i < 3 * p->M; ++i)
    if (!std::isfinite(mic_pos[i])) return fail(SONAR_E_INVALID, "mic_pos must be finite");
  if (is_td(p)) {
    // offsets o in [floor(-bmax), floor(bmax) + 1] (nearest rounds up by one at most); the taps read
    // o .. o + 1 (linear), o - 1 .. o + 2 (cubic)
    const double bmax = delay_bound(mic_pos, p->M, p->fs, p->c);
    if (static_cast<int>(std::floor(-bmax)) - 1 < p->omin || static_cast<int>(std::floor(bmax)) + 2 > p->omax)
      return fail(SONAR_E_UNSUPPORTED, "new positions need delays beyond the plan's range [%d, %d]: create a new plan",
                  p->omin, p->omax);
  }
  hipError_t e = hipMemcpyAsync(p->d_pos, mic_pos, 3 * sizeof(double) * p->M, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = launch_delay_tables(p, stream);
  if (e == hipSuccess && !is_td(p)) e = launch_fd_step_table(p, stream);
  if (e != hipSuccess) return hip_fail(e, "position update");
  if (!mt_planes(p)) return SONAR_OK;
  // MFMA time-domain modes: the direction tiles, tap groups and weights follow the geometry and are
  // rebuilt on the host from the new delay table (the staged window already spans the plan's whole
  // delay range).  The new tables replace the old ones only once they are complete; on failure the
  // plan keeps the old tables, which then no longer match the delay table.
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "position update");
  int* old_g = p->d_mt_g;
  unsigned short* old_w = p->d_mt_w;
  int2* old_kcr = p->d_mt_kcr;
  int* old_perm = p->d_mt_perm;
  unsigned short* old_fir = p->d_mt_fir;
  const int old_gmax = p->mt_gmax, old_kcmax = p->mt_kcmax;
  const long long old_flop = p->mt_flop_per_frame;
  const float old_unscale = p->mt_fir_unscale;
  p->d_mt_g = nullptr;
  p->d_mt_w = nullptr;
  p->d_mt_kcr = nullptr;
  p->d_mt_perm = nullptr;
  p->d_mt_fir = nullptr;
  size_t total = 0;
  const int st = build_mt_tables(p, mic_pos, p->h_dirs.data(), p->h_taps, stream, &total);
  int* const fr_g = st == SONAR_OK ? old_g : p->d_mt_g;
  unsigned short* const fr_w = st == SONAR_OK ? old_w : p->d_mt_w;
  int2* const fr_kcr = st == SONAR_OK ? old_kcr : p->d_mt_kcr;
  int* const fr_perm = st == SONAR_OK ? old_perm : p->d_mt_perm;
  unsigned short* const fr_fir = st == SONAR_OK ? old_fir : p->d_mt_fir;
  (void)hipFree(fr_g);
  (void)hipFree(fr_w);
  (void)hipFree(fr_kcr);
  (void)hipFree(fr_perm);
  (void)hipFree(fr_fir);
  if (st != SONAR_OK) {
    p->d_mt_g = old_g;
    p->d_mt_w = old_w;
    p->d_mt_kcr = old_kcr;
    p->d_mt_perm = old_perm;
    p->d_mt_fir = old_fir;
    p->mt_gmax = old_gmax;
    p->mt_kcmax = old_kcmax;
    p->mt_flop_per_frame = old_flop;
    p->mt_fir_unscale = old_unscale;
  }
  return st;
}

namespace {

// default sections: Butterworth of order 2 S, -3 dB at fc / fs; the analog poles
// W exp(i pi (2k + 2S + 1) / (4S)), k < S (one of each conjugate pair), prewarped
// W = 2 tan(pi fc / fs) (fs = 1), bilinear z = (2 + p) / (2 - p), double zero at -1,
// each section scaled to unit gain at DC
void butterworth_sections(int S, double fc_over_fs, std::vector<double>& sos) {
  const int order = 2 * S;
  const double W = 2.0 * std::tan(M_PI * fc_over_fs);
  sos.assign(6 * static_cast<size_t>(S), 0.0);
  for (int k = 0; k < S; ++k) {
    const double th = M_PI * (2.0 * k + order + 1) / (2.0 * order);
    const double pr = W * std::cos(th), pi = W * std::sin(th);
    // z = (2 + p) / (2 - p)
    const double nr = 2.0 + pr, ni = pi, dr = 2.0 - pr, di = -pi;
    const double den = dr * dr + di * di;
    const double zr = (nr * dr + ni * di) / den, zi = (ni * dr - nr * di) / den;
    const double a1 = -2.0 * zr, a2 = zr * zr + zi * zi;
    const double g = (1.0 + a1 + a2) / 4.0;
    double* s = &sos[6 * static_cast<size_t>(k)];
    s[0] = g; s[1] = 2.0 * g; s[2] = g; s[3] = 1.0; s[4] = a1; s[5] = a2;
  }
}

}  // namespace

int sonar_plan_set_envelope_iir(sonar_plan p, int32_t n_sections, const double* sos_in, hipStream_t stream) {
  if (!p) return fail(SONAR_E_INVALID, "plan is NULL");
  if (n_sections < 0 || n_sections > IIR_MAX_SECTIONS)
    return fail(SONAR_E_INVALID, "n_sections=%d outside [0, %d]", n_sections, IIR_MAX_SECTIONS);
  if (n_sections == 0) {
    p->iir_ns = 0;
    return SONAR_OK;
  }
  std::vector<double> sos;
  if (sos_in) {
    sos.assign(sos_in, sos_in + 6 * static_cast<size_t>(n_sections));
  } else {
    butterworth_sections(n_sections, 1.0 / (2.0 * p->R), sos);
  }
  for (double v : sos)
    if (!std::isfinite(v)) return fail(SONAR_E_INVALID, "sos must be finite");
  const int ns = 2 * n_sections;
  // cascade -> one state-space system (x: input |b|, u_s: input of section s)
  std::vector<double> A(ns * ns, 0.0), B(ns, 0.0), Cu(ns, 0.0);
  double Du = 1.0;
  for (int s = 0; s < n_sections; ++s) {
    const double* q = &sos[6 * static_cast<size_t>(s)];
    if (q[3] == 0.0) return fail(SONAR_E_INVALID, "section %d has a0 = 0", s);
    const double b0 = q[0] / q[3], b1 = q[1] / q[3], b2 = q[2] / q[3], a1 = q[4] / q[3], a2 = q[5] / q[3];
    const double Bs[2] = {b1 - a1 * b0, b2 - a2 * b0};
    const int r = 2 * s;
    // x_s' = A_s x_s + B_s u_s, u_s = Cu . x + Du x_in (transposed direct form II)
    for (int i = 0; i < 2; ++i) {
      for (int j = 0; j < ns; ++j) A[(r + i) * ns + j] += Bs[i] * Cu[j];
      B[r + i] = Bs[i] * Du;
    }
    A[r * ns + r] += -a1;
    A[r * ns + r + 1] += 1.0;
    A[(r + 1) * ns + r] += -a2;
    // y_s = x_s[0] + b0 u_s becomes the next section's input
    for (int j = 0; j < ns; ++j) Cu[j] *= b0;
    Cu[r] += 1.0;
    Du *= b0;
  }
  // chunk length: a multiple of 16 samples with 64 L >= G' + 15 (chunks start on 128-byte boundaries)
  const int L = ((p->G + 15 + 63) / 64 + 15) / 16 * 16;
  std::vector<float> tab(IIR_TAB_LEN, 0.0f);
  for (int i = 0; i < ns * ns; ++i) tab[i] = static_cast<float>(A[i]);
  for (int i = 0; i < ns; ++i) {
    tab[ns * ns + i] = static_cast<float>(B[i]);
    tab[ns * ns + ns + i] = static_cast<float>(Cu[i]);
  }
  tab[ns * ns + 2 * ns] = static_cast<float>(Du);
  // P = A^L by squaring, then A^(L 2^k) by repeated squaring
  auto mul = [ns](const std::vector<double>& X, const std::vector<double>& Y) {
    std::vector<double> Z(ns * ns, 0.0);
    for (int i = 0; i < ns; ++i)
      for (int k = 0; k < ns; ++k)
        for (int j = 0; j < ns; ++j) Z[i * ns + j] += X[i * ns + k] * Y[k * ns + j];
    return Z;
  };
  std::vector<double> P(ns * ns, 0.0), base = A;
  for (int i = 0; i < ns; ++i) P[i * ns + i] = 1.0;
  for (int e = L; e > 0; e >>= 1) {
    if (e & 1) P = mul(P, base);
    base = mul(base, base);
  }
  for (int k = 0; k < 6; ++k) {
    for (int i = 0; i < ns * ns; ++i) tab[IIR_POW_OFFSET + k * ns * ns + i] = static_cast<float>(P[i]);
    P = mul(P, P);
  }
  size_t total = 0;
  if (!p->d_iir && dev_alloc(&p->d_iir, static_cast<size_t>(IIR_TAB_LEN), &total) != hipSuccess)
    return fail(SONAR_E_NOMEM, "IIR table allocation failed");
  const int st = ensure_beam_workspace(p, &total);
  if (st != SONAR_OK) return st;
  p->ws_bytes += total;
  hipError_t e = hipMemcpyAsync(p->d_iir, tab.data(), sizeof(float) * IIR_TAB_LEN, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "IIR table upload");
  p->iir_ns = ns;
  p->iir_chunk = L;
  return SONAR_OK;
}

int sonar_pdm_destroy(sonar_pdm p) {
  if (!p) return SONAR_OK;
  (void)hipFree(p->d_lut);
  (void)hipFree(p->d_gcum);
  (void)hipFree(p->d_qtab);
  (void)hipFree(p->d_rcum);
  delete p;
  return SONAR_OK;
}

int sonar_pdm_create(const sonar_pdm_desc* desc, hipStream_t stream, sonar_pdm* out) {
  if (!desc || !out) return fail(SONAR_E_INVALID, "desc and out must not be NULL");
  *out = nullptr;
  const sonar_pdm_desc& d = *desc;
  if (d.n_mics < 1 || d.n_mics > PDM_MAX_MICS) return fail(SONAR_E_INVALID, "n_mics=%d outside [1, %d]", d.n_mics, PDM_MAX_MICS);
  if (d.n_out < 1 || d.decim < 1 || d.max_frames < 1) return fail(SONAR_E_INVALID, "n_out, decim and max_frames must be >= 1");
  if (static_cast<long long>(d.n_out) * d.decim > (1LL << 31) / 4)
    return fail(SONAR_E_UNSUPPORTED, "n_out * decim = %lld ticks is above the supported 2^29", static_cast<long long>(d.n_out) * d.decim);
  std::vector<double> taps;
  if (d.n_taps == 0 && !d.taps) {
    const int K = 32 * d.decim + 1;
    taps.resize(K);
    const double hk = 0.5 * (K - 1);
    double sum = 0.0;
    for (int j = 0; j < K; ++j) {
      const double w = 0.54 - 0.46 * std::cos(2.0 * M_PI * j / (K - 1));
      const double arg = (j - hk) / (2.0 * d.decim);
      const double sinc = arg == 0.0 ? 1.0 : std::sin(M_PI * arg) / (M_PI * arg);
      taps[j] = w * sinc;
      sum += taps[j];
    }
    for (double& v : taps) v /= sum;
  } else {
    if (!d.taps || d.n_taps < 1) return fail(SONAR_E_INVALID, "n_taps > 0 needs taps (or n_taps = 0 and taps = NULL)");
    taps.assign(d.taps, d.taps + d.n_taps);
  }
  const int K = static_cast<int>(taps.size());
  if (K % 2 == 0) return fail(SONAR_E_INVALID, "the PDM filter length must be odd (zero phase), got %d", K);
  if (K > PDM_MAX_TAPS) return fail(SONAR_E_UNSUPPORTED, "PDM filter length %d above %d", K, PDM_MAX_TAPS);
  for (double v : taps)
    if (!std::isfinite(v)) return fail(SONAR_E_INVALID, "PDM taps must be finite");

  auto* p = new sonar_pdm_s();
  p->M = d.n_mics;
  p->N = d.n_out;
  p->D = d.decim;
  p->K = K;
  p->C = pdm_tables(K);
  p->W = (d.n_mics + 31) / 32;
  p->max_frames = d.max_frames;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(SONAR_E_HIP, "hipGetDevice failed");
  }
  // matrix-core variant where a tile's tap operand fits: the largest tile of outputs that
  // leaves room for two workgroups per CU, else the largest that fits one
  const int KS = pdm_mt_ksteps(p->D, K);
  p->rows = 16 * ((p->M + 15) / 16);
  if (KS <= PDM_MT_KS_MAX) {
    for (const size_t cap : {PDM_MT_LDS_PAIR, PDM_LDS_LIMIT}) {
      for (int nb = 512; nb >= 64 && !p->mt; nb /= 2) {
        const int sw = pdm_mt_span_words(nb, p->D, KS);
        if (pdm_mt_lds_bytes(p->rows, sw, KS) <= cap) {
          p->mt = true;
          p->NB = nb;
          p->SW = sw;
          p->KS = KS;
        }
      }
      if (p->mt) break;
    }
  }
  if (p->mt) {
    // integer taps r = round(g 2^qshift) with |r| <= 2^29: four signed base-256 digits
    double amax = 0.0;
    for (double v : taps) amax = std::max(amax, std::fabs(v));
    int ex = 0;
    if (amax > 0.0) (void)std::frexp(amax, &ex);
    p->qshift = amax > 0.0 ? 29 - ex : 0;
  } else {
    for (int nb = 256; nb >= 64; nb /= 2) {
      const int sw = pdm_span_words(nb, p->D, K);
      if (pdm_lds_bytes(p->M, sw, p->C) <= PDM_LDS_LIMIT) {
        p->NB = nb;
        p->SW = sw;
        break;
      }
    }
  }
  if (p->NB == 0) {
    delete p;
    return fail(SONAR_E_UNSUPPORTED, "decim=%d with %d taps needs more LDS than a workgroup has", d.decim, K);
  }
  size_t total = 0;
  double* d_taps64 = nullptr;
  bool ok = (p->mt ? dev_alloc(&p->d_qtab, static_cast<size_t>(p->KS) * 1024, &total) == hipSuccess &&
                         dev_alloc(&p->d_rcum, static_cast<size_t>(K) + 1, &total) == hipSuccess
                   : dev_alloc(&p->d_lut, static_cast<size_t>(p->C) * 256, &total) == hipSuccess &&
                         dev_alloc(&p->d_gcum, static_cast<size_t>(K) + 1, &total) == hipSuccess) &&
            hipMalloc(&d_taps64, sizeof(double) * K) == hipSuccess;
  hipError_t e = ok ? hipMemcpyAsync(d_taps64, taps.data(), sizeof(double) * K, hipMemcpyHostToDevice, stream)
                    : hipErrorOutOfMemory;
  if (e == hipSuccess) e = launch_pdm_tables(p, d_taps64, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e == hipSuccess)
    e = init_pdm_kernel_attributes(p, p->mt ? pdm_mt_lds_bytes(p->rows, p->SW, p->KS)
                                            : pdm_lds_bytes(p->M, p->SW, p->C));
  (void)hipFree(d_taps64);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    sonar_pdm_destroy(p);
    return e == hipErrorOutOfMemory ? fail(SONAR_E_NOMEM, "PDM tables allocation failed") : hip_fail(e, "PDM tables");
  }
  *out = p;
  return SONAR_OK;
}

int sonar_pdm_demodulate(sonar_pdm p, const uint32_t* words, int32_t F, float* x, hipStream_t stream) {
  if (!p) return fail(SONAR_E_INVALID, "pdm is NULL");
  if (!words || !x) return fail(SONAR_E_INVALID, "NULL buffer");
  if (F < 1 || F > p->max_frames) return fail(SONAR_E_INVALID, "F=%d outside [1, max_frames=%d]", F, p->max_frames);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(SONAR_E_INVALID, "current device %d is not the device %d the PDM filter was created on", dev, p->device);
  const hipError_t e = launch_pdm_demod(p, words, F, x, stream);
  return e == hipSuccess ? SONAR_OK : hip_fail(e, "PDM demodulation launch");
}

}  // extern "C"
