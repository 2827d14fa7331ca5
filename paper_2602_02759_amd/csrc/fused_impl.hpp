#pragma once
// Fused pass of libnnef for gfx950 (CDNA4): device code shared by the
// per-width translation units fused16.hip, fused32.hip, fused64.hip.
//
// Device kernels of libnnef for gfx950 (CDNA4).
//
// fused_pass  - one block update's pass over Y (Algorithm 1, Sec. 3): rebuild a
//               16 x (16*PT) tile of Yhat on MFMA, form the masked weights
//               a(Y,Yhat), b(Y,Yhat) (App. B; mask per Sec. 6) in registers and
//               contract them against the other side on MFMA into the
//               numerator and denominator of eq. 3.4.  Yhat never leaves the
//               register file.
// update      - fixed-order reduction of the fused pass partials, then the
//               update Theta <- max(eps, Theta * g^{-1}(N/D)) (eq. 3.4).
// einsum      - generic small contraction for side operands and chain-back.
//
// MFMA layout used throughout (v_mfma_f32_16x16x4_f32): lane l = 16*g + c
// supplies A[row c][k g] and B[k g][col c]; the accumulator holds
// C[row 4g + r][col c], r = 0..3.  The tile is computed transposed,
// Yhat^T[q][p], so that each lane's accumulator rows r are four q values of
// one p: they feed the next MFMA directly as its B operand (K = q), with no
// LDS round trip.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "nnef_internal.hpp"

namespace nnef {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// forward use in the load helpers below
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Loads at a 32-bit element offset from a wave-uniform base pointer.  The
// offset is turned into a 32-bit byte offset so that the compiler can address
// through the scalar base (no 64-bit address arithmetic per lane); every
// buffer the kernels index this way holds fewer than 2^30 elements.
__device__ __forceinline__ float ldf(const float* base, uint32_t off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (off << 2));
}
typedef float f4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4_t ldf4(const float* base, uint32_t off) {
  return *reinterpret_cast<const f4_t*>(reinterpret_cast<const char*>(base) + (off << 2));
}
__device__ __forceinline__ uint32_t ldu32(const uint8_t* base, uint32_t off) {
  return *reinterpret_cast<const uint32_t*>(base + off);
}

__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// x^p for x >= 0 with 0^p = 0 (p > 0), through log2/exp2.
__device__ __forceinline__ float powpos(float x, float p) {
  return x > 0.f ? fast_exp2(p * fast_log2(x)) : (p > 0.f ? 0.f : (p == 0.f ? 1.f : INFINITY));
}

// Weights a(y, yh), b(y, yh) of App. B for an observed entry (yh > 0).
template <int WK>
__device__ __forceinline__ void ab_weights(float y, float yh, float al, float be, float& wa,
                                           float& wb) {
  if constexpr (WK == WK_KL) {
    wa = y * fast_rcp(yh);
    wb = 1.f;
  } else if constexpr (WK == WK_EUC) {
    wa = y;
    wb = yh;
  } else if constexpr (WK == WK_SQRT) {
    wa = __builtin_sqrtf(y);
    wb = __builtin_sqrtf(yh);
  } else if constexpr (WK == WK_IS) {
    float r = fast_rcp(yh);
    wb = r;
    wa = y * r * r;
  } else if constexpr (WK == WK_GEN) {
    float ly = fast_log2(yh);
    wb = fast_exp2((al + be - 1.f) * ly);
    wa = powpos(y, al) * fast_exp2((be - 1.f) * ly);
  } else {  // WK_RKL
    wa = fast_log2(y * fast_rcp(yh)) * 0.69314718055994531f;
    wb = 1.f;
  }
}

// (1+u) log(1+u) - u, accurate near u = 0 (series below |u| < 1/4).
__device__ __forceinline__ float xlogx_m(float u) {
  if (fabsf(u) < 0.25f) {
    // sum_{n>=2} (-1)^n u^n / (n (n-1))
    float s = 0.f, un = u * u;
    const float inv[9] = {1.f / 2, 1.f / 6, 1.f / 12, 1.f / 20, 1.f / 30, 1.f / 42, 1.f / 56,
                          1.f / 72, 1.f / 90};
#pragma unroll
    for (int n = 0; n < 9; ++n) {
      s += ((n & 1) ? -inv[n] : inv[n]) * un;
      un *= u;
    }
    return s;
  }
  float t = 1.f + u;
  return t * (fast_log2(t) * 0.69314718055994531f) - u;
}

// u - log(1+u), accurate near u = 0.
__device__ __forceinline__ float u_mlog(float u) {
  if (fabsf(u) < 0.25f) {
    float s = 0.f, un = u * u;
#pragma unroll
    for (int n = 2; n < 11; ++n) {
      s += ((n & 1) ? -1.f : 1.f) * un / (float)n;
      un *= u;
    }
    return s;
  }
  return u - fast_log2(1.f + u) * 0.69314718055994531f;
}

// D_{alpha,beta}(y, yh) of App. B for one observed entry, as float.  The
// specialised weight kinds fix the case; WK_GEN selects it at run time.
template <int WK>
__device__ __forceinline__ float ab_loss(float y, float yh, const FusedArgs& a) {
  const float ln2 = 0.69314718055994531f;
  if constexpr (WK == WK_KL) {  // y log(y/yh) - y + yh = yh [(1+u) log(1+u) - u], u = y/yh - 1
    return y > 0.f ? yh * xlogx_m(y / yh - 1.f) : yh;
  } else if constexpr (WK == WK_EUC) {
    const float d = y - yh;
    return 0.5f * d * d;
  } else if constexpr (WK == WK_IS) {  // y/yh - log(y/yh) - 1 = u - log(1+u)
    return u_mlog(y / yh - 1.f);
  } else if constexpr (WK == WK_SQRT) {  // (1/2, 1): (2/3)(sqrt y - sqrt yh)^2 (sqrt y + 2 sqrt yh)
    const float sy = __builtin_sqrtf(y), v = __builtin_sqrtf(yh), d = sy - v;
    return (2.f / 3.f) * d * d * (sy + 2.f * v);
  } else if constexpr (WK == WK_RKL) {  // (0, 1): yh log(yh/y) - yh + y
    return y > 0.f ? y * xlogx_m(yh / y - 1.f) : INFINITY;
  } else {
    const float al = a.alpha, be = a.beta;
    if (a.lk == LK_GENERIC)
      return a.ab_inv * (al * a.apb_inv * powpos(y, al + be) + be * a.apb_inv * powpos(yh, al + be) -
                         powpos(y, al) * powpos(yh, be));
    if (a.lk == LK_BETA0) {
      const float ya = powpos(y, al);
      const float lg = y > 0.f ? ya * fast_log2(y / yh) * ln2 : 0.f;
      return (powpos(yh, al) - ya + al * lg) / (al * al);
    }
    // alpha = -beta
    return (powpos(y, al) / powpos(yh, al) - 1.f + al * fast_log2(yh / y) * ln2) / (al * al);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

#ifndef NNEF_PT32
#define NNEF_PT32 2
#endif
template <int KP>
struct Tile {
  static constexpr int PT = KP == 16 ? 4 : (KP == 32 ? NNEF_PT32 : 1);  // 16-wide p subtiles per wave
  static constexpr int ROWS = 16 * PT;                          // rows of a panel
  static constexpr int KS = KP / 4;                             // reconstruction K steps
  static constexpr int KT = KP / 16;                            // kappa tiles of N and D
  static constexpr int RST = KP + 4;                            // LDS row stride (floats)
};

// Accumulator element (t, kt, r) is X^T[k = 16kt + 4g + r][p = 16t + c].  Waves
// 1..3 stash theirs in LDS; wave 0 adds them in a fixed order and stores the
// workgroup's partial rows.
template <int KP>
__device__ __forceinline__ void store_partial(const f4 (&acc)[Tile<KP>::PT][Tile<KP>::KT], float* dst,
                                              float* red, const FusedArgs& a, int wave, int g, int c,
                                              int p0, int chunk) {
  constexpr int PT = Tile<KP>::PT, KT = Tile<KP>::KT, ROWS = Tile<KP>::ROWS, RST = Tile<KP>::RST;
  if (wave > 0) {
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
        *reinterpret_cast<f4*>(&red[(wave - 1) * ROWS * RST + (16 * t + c) * RST + 16 * kt + 4 * g]) =
            acc[t][kt];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int p = p0 + 16 * t + c;
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        f4 v = acc[t][kt];
#pragma unroll
        for (int w = 0; w < 3; ++w)
          v += *reinterpret_cast<const f4*>(&red[w * ROWS * RST + (16 * t + c) * RST + 16 * kt + 4 * g]);
        if (p < a.nP) *reinterpret_cast<f4*>(&dst[((size_t)chunk * a.nP + p) * KP + 16 * kt + 4 * g]) = v;
      }
    }
  }
  __syncthreads();
}

template <int KP, int WK, bool VECQ, int MODE, bool FULL>
__global__ __launch_bounds__(256) void fused_pass(FusedArgs a) {
  using T = Tile<KP>;
  constexpr int PT = T::PT, ROWS = T::ROWS, KS = T::KS, KT = T::KT, RST = T::RST;
  constexpr bool LOSS = MODE >= 1, ND = MODE <= 1;
  __shared__ f4 red4[ND ? 3 * ROWS * RST / 4 : 1];
  __shared__ double lred[4];
  float* red = reinterpret_cast<float*>(red4);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, c = lane & 15;
  int b = blockIdx.x;
  if (a.xcd_remap) b = (b & 7) * (a.n_wg >> 3) + (b >> 3);
  const int panel = b % a.n_panels, chunk = b / a.n_panels;
  const int p0 = panel * ROWS;
  const int64_t s_beg = ((int64_t)chunk * 4 + wave) * a.steps_per_wave;
  const int64_t s_end = s_beg + a.steps_per_wave < a.n_steps ? s_beg + a.steps_per_wave : a.n_steps;

  // ---- row side, in registers for the whole pass: lane holds L[p][g*KS + s]
  float Lop[PT][KS];
  uint32_t poff[PT];
  bool pval[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int p = p0 + 16 * t + c;
    pval[t] = FULL || p < a.nP;
    poff[t] = pval[t] ? a.p_off[p] : 0u;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = g * KS + s;
      Lop[t][s] = (pval[t] && k < a.K) ? a.L[(size_t)p * a.ldL + k] : 0.f;
    }
  }
  // lane-constant kappa indices, clamped in range (out-of-range lanes are zeroed)
  int kA[KS], kB[KT];
#pragma unroll
  for (int s = 0; s < KS; ++s) kA[s] = min(g * KS + s, a.K - 1);
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) kB[kt] = min(16 * kt + c, a.K - 1);

  f4 accN[PT][KT], accD[PT][KT];
#pragma unroll
  for (int t = 0; t < PT; ++t)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      accN[t][kt] = f4{0.f, 0.f, 0.f, 0.f};
      accD[t][kt] = f4{0.f, 0.f, 0.f, 0.f};
    }
  double lsum = 0.0;
  const bool has_mask = a.M != nullptr;

  // ---- per-qo state: outer product u at this lane's kappa positions, inner base row
  int cur_qo = -1;
  float uA[KS], uB[KT];
  uint32_t ibase = 0;
  const bool vec_in = a.K == KP && (a.ld_in & 3) == 0;  // float4 loads of inner rows

  auto load_qo = [&](int qo) {
#pragma unroll
    for (int s = 0; s < KS; ++s) uA[s] = 1.f;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) uB[kt] = 1.f;
    for (int m = 0; m < a.nouter; ++m) {
      const float* ob = a.outer[m];
      const uint32_t roff = a.orow[m][qo] * (uint32_t)a.ld_out[m];
      if (FULL && (a.ld_out[m] & 3) == 0) {
#pragma unroll
        for (int s = 0; s < KS; s += 4) {
          const f4 v = ldf4(ob, roff + g * KS + s);
          uA[s] *= v[0];
          uA[s + 1] *= v[1];
          uA[s + 2] *= v[2];
          uA[s + 3] *= v[3];
        }
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) uA[s] *= ldf(ob, roff + kA[s]);
      }
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) uB[kt] *= ldf(ob, roff + kB[kt]);
    }
    ibase = a.in_base ? a.in_base[qo] : 0u;
  };

  // column side of one step, in both MFMA layouts
  struct Cols {
    float Ra[KS];     // R[qi0 + c][g*KS + s]
    float Rb[KT][4];  // R[qi0 + 4g + r][16 kt + c]
  };
  const uint32_t ld_in = (uint32_t)a.ld_in, in_stride = (uint32_t)a.in_stride;
  auto load_cols = [&](int qi0, Cols& d) {
    const int qa = qi0 + c;
    if constexpr (FULL) {
      const uint32_t ra = (ibase + (uint32_t)qa * in_stride) * ld_in;
      if (vec_in) {
#pragma unroll
        for (int s = 0; s < KS; s += 4) {
          const f4 v = ldf4(a.inner, ra + g * KS + s);
#pragma unroll
          for (int j = 0; j < 4; ++j) d.Ra[s + j] = v[j] * uA[s + j];
        }
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) d.Ra[s] = ldf(a.inner, ra + g * KS + s) * uA[s];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t rb = (ibase + (uint32_t)(qi0 + 4 * g + r) * in_stride) * ld_in;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) d.Rb[kt][r] = ldf(a.inner, rb + 16 * kt + c) * uB[kt];
      }
    } else {
      const int qac = qa < a.nqi ? qa : a.nqi - 1;
      const uint32_t ra = (ibase + (uint32_t)qac * in_stride) * ld_in;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const float v = ldf(a.inner, ra + kA[s]);
        d.Ra[s] = (qa < a.nqi && g * KS + s < a.K) ? v * uA[s] : 0.f;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int qb = qi0 + 4 * g + r;
        const int qbc = qb < a.nqi ? qb : a.nqi - 1;
        const uint32_t rb = (ibase + (uint32_t)qbc * in_stride) * ld_in;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          const float v = ldf(a.inner, rb + kB[kt]);
          d.Rb[kt][r] = (qb < a.nqi && 16 * kt + c < a.K) ? v * uB[kt] : 0.f;
        }
      }
    }
  };

  // data and mask of one step (the HBM stream)
  struct YM {
    f4 y[PT];         // y[p0 + 16t + c][qi0 + 4g + r]
    uint32_t m[PT];   // mask bytes, r = 0..3
  };
  const uint32_t qys = (uint32_t)a.qi_ystride;
  auto load_ym = [&](int qo, int qi0, YM& d) {
    const uint32_t ybase = a.qo_yoff[qo];
    const int q4 = qi0 + 4 * g;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      if constexpr (VECQ) {
        const bool ok = FULL || (pval[t] && q4 < a.nqi);
        const int q4c = FULL ? q4 : (q4 < a.nqi ? q4 : a.nqi - 4);
        const uint32_t off = ybase + poff[t] + (uint32_t)q4c;
        const f4 v = ldf4(a.Y, off);
        const uint32_t mm = has_mask ? ldu32(a.M, off) : 0x01010101u;
        d.y[t] = ok ? v : f4{0.f, 0.f, 0.f, 0.f};
        d.m[t] = ok ? mm : 0u;
      } else {
        uint32_t mm = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = q4 + r;
          const bool ok = FULL || (pval[t] && q < a.nqi);
          const int qc = FULL ? q : (q < a.nqi ? q : a.nqi - 1);
          const uint32_t off = ybase + poff[t] + (uint32_t)qc * qys;
          const float v = ldf(a.Y, off);
          const uint32_t mb = has_mask ? (uint32_t)a.M[off] : 1u;
          d.y[t][r] = ok ? v : 0.f;
          mm |= (ok ? mb : 0u) << (8 * r);
        }
        d.m[t] = mm;
      }
    }
  };

  auto compute = [&](const YM& ym, const Cols& cl) {
    // reconstruction tile, transposed: yh[t][r] = yhat[p0+16t+c][q = (qo, qi0+4g+r)]
    f4 yh[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s2 = 0; s2 < KS; ++s2) acc = mfma4(cl.Ra[s2], Lop[t][s2], acc);
      yh[t] = acc;
    }
    // masked weights (and loss)
    f4 wa[PT], wb[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool obs = (ym.m[t] >> (8 * r)) & 0xffu;
        const float y = ym.y[t][r];
        const float yhat = fmaxf(yh[t][r], FLT_MIN);
        if constexpr (ND) {
          float xa, xb;
          ab_weights<WK>(y, yhat, a.alpha, a.beta, xa, xb);
          wa[t][r] = obs ? xa : 0.f;
          wb[t][r] = obs ? xb : 0.f;
        }
        if constexpr (LOSS) {
          const float l = ab_loss<WK>(obs ? y : 1.f, obs ? yhat : 1.f, a);
          lsum += obs ? (double)l : 0.0;
        }
      }
    }
    if constexpr (ND) {
      // contractions: X^T[k][p] += sum_q R^T[k][q] W^T[q][p]
#pragma unroll
      for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int r = 0; r < 4; ++r) accN[t][kt] = mfma4(cl.Rb[kt][r], wa[t][r], accN[t][kt]);
      if (!a.no_d) {
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
          for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int r = 0; r < 4; ++r) accD[t][kt] = mfma4(cl.Rb[kt][r], wb[t][r], accD[t][kt]);
      }
    }
  };

  // ---- software pipeline: the HBM stream runs two steps ahead, the column
  // side one step ahead; three-stage rings, unrolled so indices are static.
  const int64_t nst = s_end > s_beg ? s_end - s_beg : 0;
  int yq = 0, yqi = 0;
  if (nst > 0) {
    yq = (int)(s_beg / a.nqis);
    yqi = (int)(s_beg - (int64_t)yq * a.nqis);
  }
  int cq = yq, cqi = yqi;
  auto adv = [&](int& qo, int& qis) {
    if (++qis == a.nqis) {
      qis = 0;
      ++qo;
    }
  };
  YM ym0, ym1, ym2;
  Cols c0, c1, c2;
  if (nst > 0) {
    load_ym(yq, 16 * yqi, ym0);
    adv(yq, yqi);
    load_qo(cq);
    cur_qo = cq;
    load_cols(16 * cqi, c0);
    adv(cq, cqi);
  }
  if (nst > 1) {
    load_ym(yq, 16 * yqi, ym1);
    adv(yq, yqi);
  }
  auto step = [&](int64_t i, const YM& cy, YM& py, const Cols& cc, Cols& pc) {
    if (i + 2 < nst) {
      load_ym(yq, 16 * yqi, py);
      adv(yq, yqi);
    }
    if (i + 1 < nst) {
      if (cq != cur_qo) {
        load_qo(cq);
        cur_qo = cq;
      }
      load_cols(16 * cqi, pc);
      adv(cq, cqi);
    }
    compute(cy, cc);
  };
  for (int64_t i = 0; i < nst; i += 3) {
    step(i, ym0, ym2, c0, c1);
    if (i + 1 < nst) step(i + 1, ym1, ym0, c1, c2);
    if (i + 2 < nst) step(i + 2, ym2, ym1, c2, c0);
  }

  if constexpr (LOSS) {
    const double w = wave_sum(lsum);
    if (lane == 0) lred[wave] = w;
    __syncthreads();
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
  }
  if constexpr (ND) {
    store_partial<KP>(accN, a.partN, red, a, wave, g, c, p0, chunk);
    if (!a.no_d) store_partial<KP>(accD, a.partD, red, a, wave, g, c, p0, chunk);
  }
}

template <int KP, int WK, bool VECQ, int MODE>
int launch_fused_t(const FusedArgs& a, hipStream_t s) {
  if (a.full)
    hipLaunchKernelGGL((fused_pass<KP, WK, VECQ, MODE, true>), dim3(a.n_wg), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((fused_pass<KP, WK, VECQ, MODE, false>), dim3(a.n_wg), dim3(256), 0, s, a);
  return (int)hipGetLastError();
}

template <int KP, int WK, bool VECQ>
int launch_fused_m(const FusedArgs& a, int mode, hipStream_t s) {
  switch (mode) {
    case 0: return launch_fused_t<KP, WK, VECQ, 0>(a, s);
    case 1: return launch_fused_t<KP, WK, VECQ, 1>(a, s);
    default: return launch_fused_t<KP, WK, VECQ, 2>(a, s);
  }
}

template <int KP, int WK>
int launch_fused_v(const FusedArgs& a, bool vecq, int mode, hipStream_t s) {
  return vecq ? launch_fused_m<KP, WK, true>(a, mode, s) : launch_fused_m<KP, WK, false>(a, mode, s);
}

template <int KP>
int launch_fused_w(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  switch (wk) {
    case WK_KL: return launch_fused_v<KP, WK_KL>(a, vecq, mode, s);
    case WK_EUC: return launch_fused_v<KP, WK_EUC>(a, vecq, mode, s);
    case WK_SQRT: return launch_fused_v<KP, WK_SQRT>(a, vecq, mode, s);
    case WK_IS: return launch_fused_v<KP, WK_IS>(a, vecq, mode, s);
    case WK_GEN: return launch_fused_v<KP, WK_GEN>(a, vecq, mode, s);
    default: return launch_fused_v<KP, WK_RKL>(a, vecq, mode, s);
  }
}

}  // namespace
}  // namespace nnef
