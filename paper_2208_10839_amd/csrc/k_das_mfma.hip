// Time-domain delay-and-sum on BF16 or FP16 MFMA (§4.1 delay-and-sum toward
// every direction; §4.3 subsampling after the envelope), fused with the envelope:
//
//   b_d[n]  = sum_m w0[d][m] yhat_m[n + o] + w1[d][m] yhat_m[n + o + 1]
//   E[d][q] = sum_j h[j] |b_d[n0 + qR + (K-1)/2 - j]|
//
// The same linear-interpolation result as the FP32 beamformer, computed as a
// dense product.  Directions are grouped into tiles of 32 neighbours (plan
// time, compact in delay space), so within a tile the
// integer offsets o[d][m] of one microphone span only a few samples.  For
// each microphone the tile covers that span with groups of GT consecutive
// taps (GT = 2 with two sample planes, 4 with four); the tap weights form a
// sparse 32 x K matrix W (two nonzeros per direction and microphone) and the
// samples a Hankel matrix
//   Y[(m, toff + j)][n] = yhat_m[n + toff + j],
// so b = W Y runs on v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  A
// B-operand fragment (8 consecutive K rows of one sample) is 8 / GT groups of
// GT consecutive samples of one row each (with four planes, 8 consecutive
// samples of one row: the groups come in pairs).  The 32 columns of an output
// tile are samples GT c + rho of one residue rho, and the tap groups used for
// residue rho start at t0 with t0 + rho = 0 mod GT, so every group read is
// one aligned 2 GT-byte load.
//
// Precision: weights and samples are each carried as two BF16 terms
// (hi = bf16(v), lo = bf16(v - hi)); the product keeps hi*hi + hi*lo + lo*hi
// (the dropped lo*lo term is below 2^-16 relative), real and imaginary parts
// separately, so each K-chunk costs six MFMAs per 32 x 32 output tile.  The
// matched filter writes the samples already split, as four BF16 planes per
// microphone (re hi, re lo, im hi, im lo), so staging a tile is a plain copy.
// With NPL = 2 planes (re, im: TD_BF16X2) the samples are one BF16 term and
// the product is hi*s + lo*s: four MFMAs per K-chunk.  A weight's rounding is
// the same for every sample and would add up coherently, so the weights stay
// split; the samples' rounding is independent from sample to sample and
// microphone to microphone and averages down in the sum over the array.
//
// F16 (TD_F16): the fractional delays lie on a 1/2048-sample grid, so the
// weights 1 - alpha and alpha are exact in FP16; the samples are one FP16
// term of 2^e yhat (e per frame, from the matched filter's bound on |yhat|),
// and v_mfma_f32_32x32x16_f16 takes two MFMAs per K-chunk (re, im).  The
// energyscape is scaled back by the frame header's 2^-e / M at the store.
//
// Envelope: |b| goes through LDS (the samples of one output tile are spread over
// the four residue wavefronts) and the low-pass + decimation runs as a banded
// Toeplitz product on MFMA: with four planes on BF16 (|b| and taps as hi + lo
// terms, three products), with two planes on FP16 (|b| as one FP16 term scaled
// per workgroup by a power of two, taps as hi + lo, two products; TD_BF16G: the taps
// as one FP16 term, one product).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "plan.hpp"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));


// 4 + 4 16-bit values at two 8-byte aligned LDS addresses
__device__ __forceinline__ uint4 lds_frag(const unsigned short* p, const unsigned short* q) {
  const uint2 a = *reinterpret_cast<const uint2*>(p);
  const uint2 b = *reinterpret_cast<const uint2*>(q);
  return make_uint4(a.x, a.y, b.x, b.y);
}

__device__ __forceinline__ f32x16 mfma_bf16(uint4 a, uint4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                 0);
}

__device__ __forceinline__ f32x16 mfma_f16(uint4 a, uint4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// Workgroup: one tile of 32 directions x NWAVE * 128 beam samples of one frame.
// Wavefront wv owns residue rho = wv % GT of the 128 GT-sample block wv / GT: 4 output
// tiles of 32 samples (GT c + rho).  `block` is the tile's index in the
// plan's grid (the workgroup index of a one-plan launch, a work-list position of the persistent one).
template <int NWAVE, int NPL, bool F16, bool W1>
__device__ __forceinline__ void mt_tile(
    const unsigned short* __restrict__ planes, long long fstride, const int4* __restrict__ gtab,
    const uint4* __restrict__ wtab, const int2* __restrict__ kcr, const int* __restrict__ perm,
    const uint4* __restrict__ ftab, float* __restrict__ E, int M, int D, int Q, int row, int R, int K, int qc,
    int nqt, int ntiles, int tg, int nwin, int gmax, int kcmax, int nmc, int wrow, int perm_off,
    float fir_unscale,
    int block) {
  constexpr int MICS = NPL == 2 ? 2 * MT_MICS : MT_MICS;   // microphones staged per group
  extern __shared__ unsigned short sm[];    // NPL planes x MICS rows x wrow (re hi, re lo, im hi, im lo / re, im)
  constexpr int NS = NWAVE * 128;            // beam samples per workgroup
  constexpr int NT = NWAVE * 64;
  constexpr int GT = mt_gt_of(NPL);          // taps per group = sample residues per block
  constexpr int RES = GT;
  constexpr int GPC = 16 / GT;               // groups per K-chunk
  static_assert(NWAVE % RES == 0, "wavefronts come in groups of RES residues");
  static_assert(NPL == 4 || NPL == 2, "four split planes or two single ones");
  static_assert(!F16 || NPL == 2, "FP16 samples come as two planes");
  static_assert(!F16 || W1, "FP16 weights are single terms");
  static_assert(!W1 || NPL == 2, "single-term weights go with single-term samples");
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int rho = wv % RES;
  // Workgroups are handed to the XCDs round-robin by index (XCD x = index % MT_XCDS).  The
  // direction tiles are cut into tg groups (tg divides MT_XCDS) and XCD x serves group
  // x / (MT_XCDS / tg) on the windows (frame f, range tile qt) congruent to x mod MT_XCDS / tg,
  // running the group's tiles back to back on each window: each window is staged from HBM into
  // tg L2s and each L2 holds the weight fragments of 1/tg of the tiles.  tg = 1 (window-major)
  // where all the fragments fit one L2 (single-term weights), larger with split weights.
  int tile, win;
  {
    const int xpg = MT_XCDS / tg;
    const int ntg = (ntiles + tg - 1) / tg;
    const int x = block % MT_XCDS, jb = block / MT_XCDS;
    tile = (x / xpg) * ntg + jb % ntg;
    win = x % xpg + xpg * (jb / ntg);
    if (tile >= ntiles || win >= nwin) return;   // padding of the last round
  }
  const int qt = win % nqt;
  const int f = win / nqt;
  const int s0 = qt * qc * R;                // first window sample of the tile (a multiple of 4)
  const int s0a = s0 & ~7;                   // staged from here: 16-byte aligned rows
  // first sample of the wavefront, as an index into the staged rows
  // (a block of 128 RES samples holds RES residues x 4 output tiles of 32 columns, column c of tile
  // nt being sample 32 RES nt + RES c + rho)
  const int sb = (wv / RES) * (32 * 4 * RES) + rho + (s0 - s0a);
  const int sbl = sb + RES * (lane & 31);    // this lane's first sample (column) in a staged row
  // Offsets of output tiles 1-3 (32 RES samples apart), opaque to the compiler: with constant offsets
  // it pairs the reads of tiles nt and nt + 1 into one two-address LDS read whose registers then have
  // to be moved into the fragment order (four moves per product); separate reads land in place.
  int ntoff1 = 32 * RES, ntoff2 = 64 * RES, ntoff3 = 96 * RES;
  asm volatile("" : "+v"(ntoff1), "+v"(ntoff2), "+v"(ntoff3));
  auto ntoff = [&](int nt) { return nt == 0 ? 0 : (nt == 1 ? ntoff1 : (nt == 2 ? ntoff2 : ntoff3)); };
  const int plane = MICS * wrow;
  const int bufsz = NPL * plane;             // one staging buffer: NPL planes x MICS rows
  const unsigned short* src = planes + f * fstride + s0a;
  // slot -> direction of this tile, kept in LDS past every other region (read by the stores)
  int* permL = reinterpret_cast<int*>(reinterpret_cast<char*>(sm) + perm_off);
  if (threadIdx.x < 32) permL[threadIdx.x] = perm[tile * 32 + threadIdx.x];

  f32x16 cre[4], cim[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    cre[nt] = f32x16{};
    cim[nt] = f32x16{};
  }

  // Staging: rows m0.. of this frame, samples [s0a, s0a + wrow) of each BF16 plane,
  // copied in 16-byte chunks; chunk i of a microphone group is segment sg = NPL ml + c
  // (plane c of microphone m0 + ml), column k.  Thread t owns chunks t + NT j, j < MT_SPT.
  // Two LDS buffers: the loads for group mc + 1 are in flight while group mc runs.
  const int cw = wrow >> 3;
  const int dq = NT / cw, dr = NT % cw;
  const int sg0 = threadIdx.x / cw, k0 = threadIdx.x - sg0 * cw;
  static_assert(MT_SPT == 10, "the staging registers below are written out for 5 chunks per half");
  uint4 st0, st1, st2, st3, st4;
  int sgh = sg0, kh = k0;                    // chunk position of st0 within the group
  // one half (5 chunks per thread) of the staging of a microphone group
#define MT_ADV                                                                                         \
  k += dr;                                                                                             \
  sg += dq;                                                                                            \
  if (k >= cw) {                                                                                       \
    k -= cw;                                                                                           \
    sg += 1;                                                                                           \
  }
#define MT_LD(R_)                                                                                      \
  R_ = *reinterpret_cast<const uint4*>(src + static_cast<long long>(m0n * NPL + (sg < nseg ? sg : 0)) * row + \
                                        8 * (sg < nseg ? k : 0));                                       \
  MT_ADV
#define MT_ST(R_)                                                                                      \
  if (sg < nseg) *reinterpret_cast<uint4*>(dstb + (sg % NPL) * plane + (sg / NPL) * wrow + 8 * k) = R_; \
  MT_ADV
#define MT_STAGE_LOAD(MC)                                                                              \
  {                                                                                                    \
    const int m0n = (MC) * MICS;                                                                       \
    const int nseg = NPL * (M - m0n < MICS ? M - m0n : MICS);                                          \
    int sg = sgh, k = kh;                                                                              \
    MT_LD(st0) MT_LD(st1) MT_LD(st2) MT_LD(st3) MT_LD(st4)                                             \
  }
#define MT_STAGE_STORE(MC, BUF)                                                                        \
  {                                                                                                    \
    const int m0n = (MC) * MICS;                                                                       \
    const int nseg = NPL * (M - m0n < MICS ? M - m0n : MICS);                                          \
    unsigned short* dstb = (BUF);                                                                      \
    int sg = sgh, k = kh;                                                                              \
    MT_ST(st0) MT_ST(st1) MT_ST(st2) MT_ST(st3) MT_ST(st4)                                             \
    sgh = sg;                                                                                          \
    kh = k;                                                                                            \
  }

  MT_STAGE_LOAD(0)
  MT_STAGE_STORE(0, sm)
  MT_STAGE_LOAD(0)
  MT_STAGE_STORE(0, sm)
  // The wavefront's K-chunks of all microphone groups are consecutive in the tables, so the
  // prefetch runs across group and half boundaries.  Chunk kc's operands sit in register set
  // (kc - kfirst) & 1 and are loaded two chunks ahead, after the products of the body that last
  // reads that set, so no register copy has to wait for a load (a one-ahead prefetch into a
  // single set needed one).  The group table is read through the scalar cache (its address is
  // wave-uniform), so only the weight fragments use vector loads.
  const int li = tile * RES + rho;
  const uint4* wt = wtab + static_cast<long long>(li) * kcmax * 128 + lane;
  // K-chunk kc: groups GPC kc .. GPC kc + GPC - 1, each as its first sample's offset in the staging
  // buffer, (mic - first mic of its group) * wrow + first tap; lanes 0-31 use the first half of the
  // groups, lanes 32-63 the others, each lane reading its half with one vector load
  const int* gs = reinterpret_cast<const int*>(gtab) + static_cast<long long>(li) * gmax + (GPC / 2) * (lane >> 5);
  const int kend = kcr[(tile * nmc + nmc - 1) * RES + rho].y;
  int kfirst = kcr[tile * nmc * RES + rho].x;
  if (kfirst >= kend) kfirst = 0;            // no chunks at all: harmless in-table prefetch
  struct Operands {
    uint4 ah, al;                            // weight fragments: BF16 hi and lo terms, or one FP16 term
    int4 g;                                  // offsets of this lane half's groups (two or four)
  };
  // every body issues the same loads (past the last chunk, an in-table one)
  auto load_ops = [&](Operands& o, int kc) {
    const int kl = kc < kend ? kc : kfirst;
    o.ah = wt[kl * 128];
    if constexpr (!W1) o.al = wt[kl * 128 + 64];
    if constexpr (GPC == 8) {
      o.g = *reinterpret_cast<const int4*>(gs + 8 * kl);
    } else {
      const int2 q = *reinterpret_cast<const int2*>(gs + 4 * kl);
      o.g = make_int4(q.x, q.y, 0, 0);
    }
  };
  Operands op0, op1;
  op0.al = op1.al = make_uint4(0, 0, 0, 0);
  load_ops(op0, kfirst);
  load_ops(op1, kfirst + 1);
  for (int mc = 0; mc < nmc; ++mc) {
    unsigned short* buf = sm + (mc & 1) * bufsz;
    unsigned short* nbuf = sm + ((mc + 1) & 1) * bufsz;
    const bool next = mc + 1 < nmc;
    __syncthreads();                         // group mc staged; group mc - 1 no longer read
    sgh = sg0;
    kh = k0;
    const int2 kr = kcr[(tile * nmc + mc) * RES + rho];
    const int kmid = (kr.x + kr.y) >> 1;
    auto kbody = [&](int kc, Operands& o) {
      const unsigned short* p = buf + o.g.x + sbl;
      // four planes: the two groups are always taps t, t + 4 of one microphone (registers are short)
      const unsigned short* p2 = NPL == 4 ? p + 4 : buf + o.g.y + sbl;
      // two planes: four groups of 2 taps, one 4-byte read each
      const unsigned short* p3 = buf + o.g.z + sbl;
      const unsigned short* p4 = buf + o.g.w + sbl;
      auto frag = [&](int off) {
        return make_uint4(*reinterpret_cast<const unsigned*>(p + off), *reinterpret_cast<const unsigned*>(p2 + off),
                          *reinterpret_cast<const unsigned*>(p3 + off), *reinterpret_cast<const unsigned*>(p4 + off));
      };
      if constexpr (NPL == 4) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const uint4 brh = lds_frag(p + 128 * nt, p2 + 128 * nt);
          const uint4 brl = lds_frag(p + plane + 128 * nt, p2 + plane + 128 * nt);
          const uint4 bih = lds_frag(p + 2 * plane + 128 * nt, p2 + 2 * plane + 128 * nt);
          const uint4 bil = lds_frag(p + 3 * plane + 128 * nt, p2 + 3 * plane + 128 * nt);
          cre[nt] = mfma_bf16(o.ah, brh, cre[nt]);
          cim[nt] = mfma_bf16(o.ah, bih, cim[nt]);
          cre[nt] = mfma_bf16(o.ah, brl, cre[nt]);
          cim[nt] = mfma_bf16(o.ah, bil, cim[nt]);
          cre[nt] = mfma_bf16(o.al, brh, cre[nt]);
          cim[nt] = mfma_bf16(o.al, bih, cim[nt]);
        }
      } else if constexpr (F16) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const uint4 br = frag(ntoff(nt));
          const uint4 bi = frag(plane + ntoff(nt));
          cre[nt] = mfma_f16(o.ah, br, cre[nt]);
          cim[nt] = mfma_f16(o.ah, bi, cim[nt]);
        }
      } else if constexpr (W1) {
        // exact single-term BF16 weights (delays on a 1/256 grid): one product per plane
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const uint4 br = frag(ntoff(nt));
          const uint4 bi = frag(plane + ntoff(nt));
          cre[nt] = mfma_bf16(o.ah, br, cre[nt]);
          cim[nt] = mfma_bf16(o.ah, bi, cim[nt]);
        }
      } else {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const uint4 br = frag(ntoff(nt));
          const uint4 bi = frag(plane + ntoff(nt));
          cre[nt] = mfma_bf16(o.ah, br, cre[nt]);
          cim[nt] = mfma_bf16(o.ah, bi, cim[nt]);
          cre[nt] = mfma_bf16(o.al, br, cre[nt]);
          cim[nt] = mfma_bf16(o.al, bi, cim[nt]);
        }
      }
      load_ops(o, kc + 2);
    };
    // the next group is staged in two halves, each loaded during one half of the K-chunks
    for (int hk = 0; hk < 2; ++hk) {
      if (next) {
        if (hk == 1) MT_STAGE_STORE(mc + 1, nbuf)
        MT_STAGE_LOAD(mc + 1)
      }
      const int ka = hk ? kmid : kr.x, kb = hk ? kr.y : kmid;
      int kc = ka;
      if (kc < kb && ((kc - kfirst) & 1)) kbody(kc++, op1);
      for (; kc + 1 < kb; kc += 2) {
        kbody(kc, op0);
        kbody(kc + 1, op1);
      }
      if (kc < kb) kbody(kc, op0);
    }
    if (next) MT_STAGE_STORE(mc + 1, nbuf)
  }
#undef MT_STAGE_LOAD
#undef MT_STAGE_STORE
#undef MT_LD
#undef MT_ST
#undef MT_ADV
  __syncthreads();

  // |b| of the tile into LDS: lane holds rows 8(v/4) + 4(lane/32) + v%4 (directions) of
  // column lane%32 (window sample sw + 32 RES nt + RES column) for each output tile.
  //  * two sample planes (FIR16): [32][NSP16] FP16 of 2^e |b|, e per workgroup from the tile's
  //    largest |b| (so every scaled value is below 2^14); the low-pass runs on FP16 MFMA with
  //    the taps (scaled by the plan's power of two) as two FP16 terms, and E is scaled back by
  //    2^-e and the taps' 2^-ts;
  //  * four planes: [32][NSP] words {bf16 hi, bf16 lo}, the taps as two BF16 terms.
  constexpr bool FIR16 = NPL == 2;
  constexpr int NSP = mt_nsp(NWAVE);
  constexpr int NSP16 = NS + 8;            // 16 bytes past a multiple of 256 per row (bank spread)
  unsigned int* bw = reinterpret_cast<unsigned int*>(sm);
  unsigned short* b16 = reinterpret_cast<unsigned short*>(sm);
  float* wmax = reinterpret_cast<float*>(permL + 32);   // [NWAVE] largest |b| per wavefront
  const int sw = (wv / RES) * (32 * 4 * RES) + rho;
  float inv_scale = 1.f;
  if constexpr (FIR16) {
    float mx = 0.f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        cre[nt][v] = __builtin_amdgcn_sqrtf(cre[nt][v] * cre[nt][v] + cim[nt][v] * cim[nt][v]);
        mx = fmaxf(mx, cre[nt][v]);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0) wmax[wv] = mx;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) mx = fmaxf(mx, wmax[w]);
    int ex = 0;
    (void)frexpf(mx, &ex);                 // mx = mant 2^ex, mant in [0.5, 1) (ex = 0 for mx = 0)
    int e = 14 - ex;
    e = e < -MF_F16_EMAX ? -MF_F16_EMAX : (e > MF_F16_EMAX ? MF_F16_EMAX : e);
    const float sc = ldexpf(1.0f, e);
    inv_scale = ldexpf(1.0f, -e);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int s = sw + 32 * RES * nt + RES * (lane & 31);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int dl = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        b16[dl * NSP16 + s] = __builtin_bit_cast(unsigned short, static_cast<_Float16>(cre[nt][v] * sc));
      }
    }
    // the K-steps of a column block (rounded up to a multiple of 4) read up to 63 samples past
    // the window: those of each row's tail, the next row's first ones, and after the last
    // row MT_FIR_TAIL zeros; their tap fragments are zero
    for (int i = threadIdx.x; i < 32 * (NSP16 - NS) + MT_FIR_TAIL; i += NT) {
      const int r = i / (NSP16 - NS), c = i - r * (NSP16 - NS);
      b16[r < 32 ? r * NSP16 + NS + c : 32 * NSP16 + (i - 32 * (NSP16 - NS))] = 0;
    }
  } else {
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int s = sw + 32 * RES * nt + RES * (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; v += 2) {
      const int dl = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);   // dl + 1 for v + 1
      const f32x2 a = {__builtin_amdgcn_sqrtf(cre[nt][v] * cre[nt][v] + cim[nt][v] * cim[nt][v]),
                       __builtin_amdgcn_sqrtf(cre[nt][v + 1] * cre[nt][v + 1] + cim[nt][v + 1] * cim[nt][v + 1])};
      const unsigned int hp = __builtin_bit_cast(unsigned int, __builtin_convertvector(a, bf16x2));
      const f32x2 l = {a.x - __builtin_bit_cast(float, hp << 16), a.y - __builtin_bit_cast(float, hp & 0xFFFF0000u)};
      const unsigned int lp = __builtin_bit_cast(unsigned int, __builtin_convertvector(l, bf16x2));
      bw[dl * NSP + s] = __builtin_amdgcn_perm(lp, hp, 0x05040100u);         // {hi, lo} of a.x
      bw[(dl + 1) * NSP + s] = __builtin_amdgcn_perm(lp, hp, 0x07060302u);   // {hi, lo} of a.y
    }
  }
  // the K-steps of a column block (rounded up to a multiple of 4) read up to 63 samples past
  // the window: those of each row's tail, the next row's first ones, and after the last
  // row MT_FIR_TAIL zeros; their tap fragments are zero
  for (int i = threadIdx.x; i < 32 * (NSP - NS) + MT_FIR_TAIL; i += NT) {
    const int r = i / (NSP - NS), c = i - r * (NSP - NS);
    bw[r < 32 ? r * NSP + NS + c : 32 * NSP + (i - 32 * (NSP - NS))] = 0;
  }
  }
  __syncthreads();
  // low-pass + decimation on MFMA: E[d][q] = sum_s |b|[d][s] H[s][q], H[s][q] = h[qR + K-1 - s],
  // a banded Toeplitz operand.  A column block of 32 range bins q0.. needs samples
  // q0 R .. (q0 + 31) R + K - 1; with s = q0 R + 16 ks + k the B fragments
  // h[nR + K-1 - 16 ks - k] do not depend on q0 and come from the plan (hi, lo terms),
  // loaded four K-steps at a time, one batch ahead.
  const int nqb = (qc + 31) / 32;
  // The product is taken as E^T = H^T |b|^T: the same fragments with the operands swapped,
  // so lane l receives range bins 8 g + 4 (l / 32) + 0..3 (g = v / 4) of direction l % 32
  // and writes them with one 16-byte store per g.
  // TD_BF16G: the taps as one FP16 term (the largest scaled into [2^13, 2^14), so every tap keeps 11
  // significant bits): one product per K-step instead of the hi + lo pair
  constexpr bool FIR1 = W1 && !F16;
#define MT_FIR_LOAD(H0, L0, H1, L1, H2, L2, H3, L3, KB)                                               \
  {                                                                                                    \
    const uint4* fp = ftab + 2 * (KB) * 64 + lane;                                                     \
    H0 = fp[0];                                                                                        \
    H1 = fp[128];                                                                                      \
    H2 = fp[256];                                                                                      \
    H3 = fp[384];                                                                                      \
    if constexpr (!FIR1) {                                                                             \
      L0 = fp[64];                                                                                     \
      L1 = fp[192];                                                                                    \
      L2 = fp[320];                                                                                    \
      L3 = fp[448];                                                                                    \
    }                                                                                                  \
  }
#define MT_FIR_STEP16(H, L, KS, ACC)                                                                   \
  {                                                                                                    \
    const uint4 bb = *reinterpret_cast<const uint4*>(bh + 16 * (KS));                                  \
    ACC = mfma_f16(H, bb, ACC);                                                                        \
    if constexpr (!FIR1) ACC = mfma_f16(L, bb, ACC);                                                   \
  }
#define MT_FIR_STEP(H, L, KS, ACC)                                                                     \
  if constexpr (FIR16) MT_FIR_STEP16(H, L, KS, ACC) else                                               \
  {                                                                                                    \
    const uint4 w0 = *reinterpret_cast<const uint4*>(ah + 16 * (KS));                                  \
    const uint4 w1 = *reinterpret_cast<const uint4*>(ah + 16 * (KS) + 4);                              \
    const uint4 ahi = make_uint4(__builtin_amdgcn_perm(w0.y, w0.x, 0x05040100u),                       \
                                 __builtin_amdgcn_perm(w0.w, w0.z, 0x05040100u),                       \
                                 __builtin_amdgcn_perm(w1.y, w1.x, 0x05040100u),                       \
                                 __builtin_amdgcn_perm(w1.w, w1.z, 0x05040100u));                      \
    const uint4 alo = make_uint4(__builtin_amdgcn_perm(w0.y, w0.x, 0x07060302u),                       \
                                 __builtin_amdgcn_perm(w0.w, w0.z, 0x07060302u),                       \
                                 __builtin_amdgcn_perm(w1.y, w1.x, 0x07060302u),                       \
                                 __builtin_amdgcn_perm(w1.w, w1.z, 0x07060302u));                      \
    const bf16x8 h_hi = __builtin_bit_cast(bf16x8, H);                                                 \
    const bf16x8 h_lo = __builtin_bit_cast(bf16x8, L);                                                 \
    ACC = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h_hi, __builtin_bit_cast(bf16x8, ahi), ACC, 0, 0, 0); \
    ACC = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h_lo, __builtin_bit_cast(bf16x8, ahi), ACC, 0, 0, 0); \
    ACC = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h_hi, __builtin_bit_cast(bf16x8, alo), ACC, 0, 0, 0); \
  }
  // K-steps [k0, k1) (multiples of 4) of column block cb into acc (even K-steps) and acc2 (odd):
  // two independent MFMA chains
  auto fir_block = [&](int cb, int k0, int k1, f32x16& acc, f32x16& acc2) {
    const unsigned int* ah = bw + (lane & 31) * NSP + 32 * cb * R + 8 * (lane >> 5);
    const unsigned short* bh = b16 + (lane & 31) * NSP16 + 32 * cb * R + 8 * (lane >> 5);
    (void)ah;
    (void)bh;
    uint4 ah0, al0 = {}, ah1, al1 = {}, ah2, al2 = {}, ah3, al3 = {};   // tap fragments, batch A
    uint4 bh0, bl0 = {}, bh1, bl1 = {}, bh2, bl2 = {}, bh3, bl3 = {};   // batch B
    MT_FIR_LOAD(ah0, al0, ah1, al1, ah2, al2, ah3, al3, k0)
    for (int kb = k0; kb < k1; kb += 8) {
      const bool more = kb + 4 < k1;
      if (more) MT_FIR_LOAD(bh0, bl0, bh1, bl1, bh2, bl2, bh3, bl3, kb + 4)
      MT_FIR_STEP(ah0, al0, kb, acc)
      MT_FIR_STEP(ah1, al1, kb + 1, acc2)
      MT_FIR_STEP(ah2, al2, kb + 2, acc)
      MT_FIR_STEP(ah3, al3, kb + 3, acc2)
      if (more) {
        if (kb + 8 < k1) MT_FIR_LOAD(ah0, al0, ah1, al1, ah2, al2, ah3, al3, kb + 8)
        MT_FIR_STEP(bh0, bl0, kb + 4, acc)
        MT_FIR_STEP(bh1, bl1, kb + 5, acc2)
        MT_FIR_STEP(bh2, bl2, kb + 6, acc)
        MT_FIR_STEP(bh3, bl3, kb + 7, acc2)
      }
    }
  };
  // K-steps of column block cb (rounded up to a multiple of 4)
  auto fir_ksteps = [&](int cb) {
    const int nval = qc - 32 * cb < 32 ? qc - 32 * cb : 32;
    return (((nval - 1) * R + K + 15) / 16 + 3) & ~3;
  };
  auto store_block = [&](int cb, f32x16 acc, const f32x16& acc2) {
    const int q0 = 32 * cb;
    const int d = permL[lane & 31];
    if constexpr (F16) {
      // frame header: 2^-e / M
      const float esc = *reinterpret_cast<const float*>(planes + f * fstride + 2LL * M * row);
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = (acc[v] + acc2[v]) * esc;
    } else {
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] += acc2[v];
    }
    if constexpr (FIR16) {
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = acc[v] * inv_scale * fir_unscale;   // two steps: each factor >= 2^-100
    }
    if (d >= 0) {
      float* erow = E + (static_cast<long long>(f) * D + d) * Q + static_cast<long long>(qt) * qc;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int q = q0 + 8 * g + 4 * (lane >> 5);
        const float4 o = make_float4(acc[4 * g], acc[4 * g + 1], acc[4 * g + 2], acc[4 * g + 3]);
        const int lim = (qc < Q - qt * qc ? qc : Q - qt * qc) - q;   // valid bins from q on
        if (lim >= 4) {
          __builtin_memcpy(erow + q, &o, 16);
        } else {
          if (lim > 0) erow[q] = o.x;
          if (lim > 1) erow[q + 1] = o.y;
          if (lim > 2) erow[q + 2] = o.z;
        }
      }
    }
  };
  if (2 * nqb <= NWAVE) {
    // few column blocks: each block's K-steps are split over two wavefronts; the second half's
    // sums go through LDS (after the |b| rows and their zero tail, which the products never read)
    float* part = reinterpret_cast<float*>(bw + 32 * NSP + MT_FIR_TAIL);   // [NWAVE / 2][16][64 lanes]
    const int cb = wv % nqb, half = wv / nqb;
    f32x16 acc = f32x16{}, acc2 = f32x16{};
    if (wv < 2 * nqb) {
      const int nks4 = fir_ksteps(cb);
      const int kmid = (nks4 / 2) & ~3;
      fir_block(cb, half ? kmid : 0, half ? nks4 : kmid, acc, acc2);
      if (half) {
#pragma unroll
        for (int v = 0; v < 16; ++v) part[(cb * 16 + v) * 64 + lane] = acc[v] + acc2[v];
      }
    }
    __syncthreads();
    if (wv < nqb) {
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] += part[(cb * 16 + v) * 64 + lane];
      store_block(cb, acc, acc2);
    }
  } else {
    for (int cb = wv; cb < nqb; cb += NWAVE) {
      f32x16 acc = f32x16{}, acc2 = f32x16{};
      fir_block(cb, 0, fir_ksteps(cb), acc, acc2);
      store_block(cb, acc, acc2);
    }
  }
#undef MT_FIR_LOAD
#undef MT_FIR_STEP
#undef MT_FIR_STEP16
}

template <int NWAVE, int NPL, bool F16, bool W1>
__global__ __launch_bounds__(NWAVE * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void das_mfma_env_kernel(
    const unsigned short* __restrict__ planes, long long fstride, const int4* __restrict__ gtab,
    const uint4* __restrict__ wtab, const int2* __restrict__ kcr, const int* __restrict__ perm,
    const uint4* __restrict__ ftab, float* __restrict__ E, int M, int D, int Q, int row, int R, int K, int qc,
    int nqt, int ntiles, int tg, int nwin, int gmax, int kcmax, int nmc, int wrow, int perm_off,
    float fir_unscale) {
  mt_tile<NWAVE, NPL, F16, W1>(planes, fstride, gtab, wtab, kcr, perm, ftab, E, M, D, Q, row, R, K, qc, nqt, ntiles, tg, nwin,
                           gmax, kcmax, nmc, wrow, perm_off, fir_unscale, static_cast<int>(blockIdx.x));
}

// Persistent launch over the items of a sensor-network batch (each item: one plan, its frames):
// a work list of every item's tiles, item after item, each item's run padded to whole rounds of
// MT_XCDS so that the XCD mapping of one-plan launches is kept (window x mod MT_XCDS of every item
// on XCD x; the grid is a multiple of MT_XCDS).  A fixed grid of workgroups (a few per CU) walks
// the list with a stride of its size.
struct MtItem {
  const unsigned short* planes;
  const int4* gtab;
  const uint4* wtab;
  const int2* kcr;
  const int* perm;
  const uint4* ftab;
  float* E;
  long long fstride;
  int M, D, Q, row, R, K, qc, nqt, ntiles, tg, nwin, gmax, kcmax, nmc, wrow, perm_off;
  float fir_unscale;
  int work_begin;   // first work-list position of the item (a multiple of MT_XCDS)
  int work_count;   // its positions (mt_grid_blocks), nwin = frames x nqt
};
struct MtWork {
  MtItem item[MT_MULTI_MAX_ITEMS];
  int n_items;
  int total;        // work-list length
};

template <int NWAVE, int NPL, bool F16, bool W1>
__global__ __launch_bounds__(NWAVE * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void das_mfma_env_multi_kernel(
    const MtWork work) {
  for (int w = blockIdx.x; w < work.total; w += gridDim.x) {
    int i = 0;
    while (i + 1 < work.n_items && work.item[i + 1].work_begin <= w) ++i;   // wave-uniform
    const MtItem& it = work.item[i];
    if (w - it.work_begin >= it.work_count) continue;   // padding up to the next item (uniform)
    mt_tile<NWAVE, NPL, F16, W1>(it.planes, it.fstride, it.gtab, it.wtab, it.kcr, it.perm, it.ftab, it.E, it.M, it.D, it.Q,
                             it.row, it.R, it.K, it.qc, it.nqt, it.ntiles, it.tg, it.nwin, it.gmax, it.kcmax, it.nmc,
                             it.wrow, it.perm_off, it.fir_unscale, w - it.work_begin);
    __syncthreads();   // the next tile's staging rewrites the LDS this tile's epilogue reads
  }
}

}  // namespace

// tile groups of the workgroup order and the workgroups of a launch over nwin windows: one group
// (window-major) for single-term weights, 2 for split weights on two planes, 8 (tile-major) for
// four planes, as measured best at 32 x 16384 x 1500; at most the tile count (a power of two)
static long long mt_grid_blocks(const sonar_plan_s* p, int nwin, int* tg) {
  int g = mt_w1(p) ? 1 : (mt_planes(p) == 2 ? 2 : MT_XCDS);
  while (g > 1 && g > p->mt_ntiles) g /= 2;
  *tg = g;
  const int xpg = MT_XCDS / g;
  return static_cast<long long>(MT_XCDS) * ((p->mt_ntiles + g - 1) / g) * ((nwin + xpg - 1) / xpg);
}

// byte offset of the tile's slot -> direction table, after the staging and low-pass regions
// (|b| rows, their zero tail, and the split low-pass partial sums [nwave / 2][16][64] floats)
static size_t mt_perm_offset(const sonar_plan_s* p) {
  const size_t planes = 2 * static_cast<size_t>(mt_planes(p)) * mt_mics(p) * p->mt_wrow * sizeof(unsigned short);
  const size_t absb = (32 * static_cast<size_t>(mt_nsp(p->mt_nwave)) + MT_FIR_TAIL) * sizeof(unsigned int) +
                      static_cast<size_t>(p->mt_nwave / 2) * 16 * 64 * sizeof(float);
  return ((planes > absb ? planes : absb) + 15) / 16 * 16;
}

// slot -> direction table (32 ints), then the per-wavefront largest |b| (up to 16 floats)
size_t mt_smem_bytes(const sonar_plan_s* p) { return mt_perm_offset(p) + 32 * sizeof(int) + 16 * sizeof(float); }

namespace {

template <int NWAVE, int NPL, bool F16, bool W1>
hipError_t set_mt_attr() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(das_mfma_env_kernel<NWAVE, NPL, F16, W1>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(das_mfma_env_multi_kernel<NWAVE, NPL, F16, W1>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  return e;
}

template <int NWAVE, int NPL, bool F16, bool W1>
hipError_t launch_mt(const sonar_plan_s* p, const unsigned short* planes, int F, float* E, hipStream_t s) {
  int tg;
  const int nwin = F * p->mt_nqt;   // windows (frame, range tile)
  const long long nblk = mt_grid_blocks(p, nwin, &tg);
  hipLaunchKernelGGL((das_mfma_env_kernel<NWAVE, NPL, F16, W1>), dim3(static_cast<unsigned>(nblk)), dim3(NWAVE * 64),
                     mt_smem_bytes(p), s, planes, 4 * p->mf_fstride, reinterpret_cast<const int4*>(p->d_mt_g),
                     reinterpret_cast<const uint4*>(p->d_mt_w), p->d_mt_kcr,
                     p->d_mt_perm, reinterpret_cast<const uint4*>(p->d_mt_fir), E, p->M, p->D, p->Q, p->row, p->R, p->K,
                     p->mt_qc, p->mt_nqt, p->mt_ntiles, tg, nwin, p->mt_gmax, p->mt_kcmax, p->mt_nmc, p->mt_wrow,
                     static_cast<int>(mt_perm_offset(p)), p->mt_fir_unscale);
  return hipGetLastError();
}

template <int NWAVE, int NPL, bool F16, bool W1>
hipError_t launch_mt_multi(const MtWork& work, size_t smem, int grid, hipStream_t s) {
  hipLaunchKernelGGL((das_mfma_env_multi_kernel<NWAVE, NPL, F16, W1>), dim3(static_cast<unsigned>(grid)),
                     dim3(NWAVE * 64), smem, s, work);
  return hipGetLastError();
}

// the kernel variant of a plan: four split planes (TD_BF16), two BF16 planes with split weights
// (TD_BF16X2), FP16 (TD_F16), two BF16 planes with exact single-term weights (TD_BF16G)
enum MtVariant { MT_V_BF16X4, MT_V_BF16X2, MT_V_F16, MT_V_BF16G };
MtVariant mt_variant(const sonar_plan_s* p) {
  if (mt_planes(p) == 4) return MT_V_BF16X4;
  if (mt_f16(p)) return MT_V_F16;
  return mt_w1(p) ? MT_V_BF16G : MT_V_BF16X2;
}

template <int NWAVE>
hipError_t set_mt_attrs() {
  hipError_t e = set_mt_attr<NWAVE, 4, false, false>();
  if (e == hipSuccess) e = set_mt_attr<NWAVE, 2, false, false>();
  if (e == hipSuccess) e = set_mt_attr<NWAVE, 2, true, true>();
  if (e == hipSuccess) e = set_mt_attr<NWAVE, 2, false, true>();
  return e;
}

template <int NWAVE>
hipError_t launch_mt_v(const sonar_plan_s* p, const unsigned short* planes, int F, float* E, hipStream_t s) {
  switch (mt_variant(p)) {
    case MT_V_BF16X4: return launch_mt<NWAVE, 4, false, false>(p, planes, F, E, s);
    case MT_V_BF16X2: return launch_mt<NWAVE, 2, false, false>(p, planes, F, E, s);
    case MT_V_F16: return launch_mt<NWAVE, 2, true, true>(p, planes, F, E, s);
    default: return launch_mt<NWAVE, 2, false, true>(p, planes, F, E, s);
  }
}

template <int NWAVE>
hipError_t launch_mt_multi_v(const sonar_plan_s* p0, const MtWork& work, size_t smem, int grid, hipStream_t s) {
  switch (mt_variant(p0)) {
    case MT_V_BF16X4: return launch_mt_multi<NWAVE, 4, false, false>(work, smem, grid, s);
    case MT_V_BF16X2: return launch_mt_multi<NWAVE, 2, false, false>(work, smem, grid, s);
    case MT_V_F16: return launch_mt_multi<NWAVE, 2, true, true>(work, smem, grid, s);
    default: return launch_mt_multi<NWAVE, 2, false, true>(work, smem, grid, s);
  }
}

}  // namespace

hipError_t init_mt_kernel_attributes() {
  hipError_t e = set_mt_attrs<MT_NWAVE_SMALL>();
  if (e == hipSuccess) e = set_mt_attrs<MT_NWAVE_LARGE>();
  return e;
}

bool mt_multi_compatible(const sonar_plan_s* a, const sonar_plan_s* b) {
  return mt_planes(a) == mt_planes(b) && mt_variant(a) == mt_variant(b) && a->mt_nwave == b->mt_nwave &&
         a->device == b->device;
}

hipError_t launch_das_mfma_env_multi(const sonar_plan_s* const* plans, const float2* const* yext, const int* frames,
                                     float* const* E, int n, hipStream_t s) {
  if (n < 1 || n > MT_MULTI_MAX_ITEMS) return hipErrorInvalidValue;
  MtWork work{};
  size_t smem = 0;
  int pos = 0;
  for (int i = 0; i < n; ++i) {
    const sonar_plan_s* p = plans[i];
    if (!mt_planes(p) || !mt_multi_compatible(p, plans[0])) return hipErrorInvalidValue;
    MtItem& it = work.item[i];
    it.planes = reinterpret_cast<const unsigned short*>(yext[i] + static_cast<long long>(p->M) * p->row);
    it.gtab = reinterpret_cast<const int4*>(p->d_mt_g);
    it.wtab = reinterpret_cast<const uint4*>(p->d_mt_w);
    it.kcr = p->d_mt_kcr;
    it.perm = p->d_mt_perm;
    it.ftab = reinterpret_cast<const uint4*>(p->d_mt_fir);
    it.E = E[i];
    it.fstride = 4 * p->mf_fstride;
    it.M = p->M;
    it.D = p->D;
    it.Q = p->Q;
    it.row = p->row;
    it.R = p->R;
    it.K = p->K;
    it.qc = p->mt_qc;
    it.nqt = p->mt_nqt;
    it.ntiles = p->mt_ntiles;
    it.nwin = frames[i] * p->mt_nqt;
    const long long blocks = mt_grid_blocks(p, it.nwin, &it.tg);
    it.gmax = p->mt_gmax;
    it.kcmax = p->mt_kcmax;
    it.nmc = p->mt_nmc;
    it.wrow = p->mt_wrow;
    it.perm_off = static_cast<int>(mt_perm_offset(p));
    it.fir_unscale = p->mt_fir_unscale;
    it.work_begin = pos;
    it.work_count = static_cast<int>(blocks);
    pos += (it.work_count + MT_XCDS - 1) / MT_XCDS * MT_XCDS;
    smem = std::max(smem, mt_smem_bytes(p));
  }
  work.n_items = n;
  work.total = pos;
  // a fixed grid: the workgroups the CUs hold at once (two 4-wave or one 8-wave workgroup per CU
  // at two waves per SIMD), a whole number of rounds over the XCDs, no more than the work
  const sonar_plan_s* p0 = plans[0];
  int grid = p0->cu_count * (p0->mt_nwave == MT_NWAVE_SMALL ? 2 : 1);
  grid = grid / MT_XCDS * MT_XCDS;
  if (grid < MT_XCDS) grid = MT_XCDS;
  if (grid > pos) grid = pos;
  if (grid < 1) return hipSuccess;
  return p0->mt_nwave == MT_NWAVE_SMALL ? launch_mt_multi_v<MT_NWAVE_SMALL>(p0, work, smem, grid, s)
                                        : launch_mt_multi_v<MT_NWAVE_LARGE>(p0, work, smem, grid, s);
}

hipError_t launch_das_mfma_env(const sonar_plan_s* p, const float2* yext, int F, float* E, hipStream_t s) {
  // the 16-bit planes of frame f follow its M complex rows
  const unsigned short* planes = reinterpret_cast<const unsigned short*>(yext + static_cast<long long>(p->M) * p->row);
  if (p->mt_nwave == MT_NWAVE_SMALL) return launch_mt_v<MT_NWAVE_SMALL>(p, planes, F, E, s);
  if (p->mt_nwave == MT_NWAVE_LARGE) return launch_mt_v<MT_NWAVE_LARGE>(p, planes, F, E, s);
  return hipErrorInvalidValue;
}
