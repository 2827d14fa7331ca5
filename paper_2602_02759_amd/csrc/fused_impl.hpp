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
#include <hip/hip_ext.h>

#include <cfloat>
#include <cmath>

#include "nnef_internal.hpp"

// A pass launch that records g_pass_events at the kernel's start and end when
// they are set (see nnef_internal.hpp).
#define NNEF_LAUNCH_PASS(kern, grid, block, stream, ...)                                            \
  do {                                                                                             \
    if (::nnef::g_pass_events.start)                                                               \
      hipExtLaunchKernelGGL(kern, grid, block, 0, stream, (hipEvent_t)::nnef::g_pass_events.start, \
                            (hipEvent_t)::nnef::g_pass_events.stop, 0, __VA_ARGS__);              \
    else                                                                                           \
      hipLaunchKernelGGL(kern, grid, block, 0, stream, __VA_ARGS__);                               \
  } while (0)

namespace nnef {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// forward use in the load helpers below
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

typedef short s4v __attribute__((ext_vector_type(4)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));

// 16x16x16 MFMA with BF16 (LP 1) or FP16 (LP 2) inputs rounded from FP32 and
// FP32 accumulation: lane (g, c) supplies A[row c][k 4g + j] and
// B[k 4g + j][col c], j = 0..3, from four converted values each.  An operand
// is converted once and may feed several MFMA.
template <int LP>
struct Lp4T {
  typedef s4v v4;  // BF16 bit patterns
};
template <>
struct Lp4T<2> {
  typedef h4v v4;
};

template <int LP>
__device__ __forceinline__ typename Lp4T<LP>::v4 cvt4(float v0, float v1, float v2, float v3) {
  typename Lp4T<LP>::v4 x;
  const float v[4] = {v0, v1, v2, v3};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if constexpr (LP == 2) x[j] = (_Float16)v[j];
    else x[j] = __builtin_bit_cast(short, (__bf16)v[j]);
  }
  return x;
}

template <int LP>
__device__ __forceinline__ f4 mfma4v(const typename Lp4T<LP>::v4& a, const typename Lp4T<LP>::v4& b, f4 c) {
  if constexpr (LP == 2) return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Packed data hold an observed value with its sign bit clear (data are
// nonnegative); a validation entry of a split as the value with the sign bit
// set (-0 for a zero), everything else (missing entries, tile padding) as -inf.
__device__ __forceinline__ bool observed(float yv) { return __builtin_bit_cast(int, yv) >= 0; }
__device__ __forceinline__ bool validation(float yv) { return !observed(yv) && yv != -INFINITY; }

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
  } else if constexpr (WK == WK_RKL) {
    wa = fast_log2(y * fast_rcp(yh)) * 0.69314718055994531f;
    wb = 1.f;
  } else {  // WK_FAM: al carries the family parameter, be the LossKind
    const int lk = (int)be;
    if (lk == LK_JS) {
      wa = fast_log2((y + yh) * 0.5f * fast_rcp(yh)) * 0.69314718055994531f;
      wb = 1.f;
    } else {
      wa = y * fast_rcp(yh);
      wb = lk == LK_NB ? (al + y) * fast_rcp(al + yh) : al * fast_rcp(1.f + yh);
    }
  }
}

constexpr float kLn2 = 0.69314718055994531f;
constexpr float kLog2e = 1.44269504088896341f;

// log(1 + u) for u > -1, accurate near u = 0: below |u| < 1/4 through
// 2 atanh(s), s = u / (2 + u), by its odd series (|s| < 1/7, error < 1e-9
// relative); elsewhere 1 + u is far from 1 and the hardware logarithm is
// accurate relative to its result.
__device__ __forceinline__ float log1p_acc(float u) {
  if (fabsf(u) < 0.25f) {
    const float s = u * fast_rcp(2.f + u), s2 = s * s;
    return 2.f * s * (1.f + s2 * (1.f / 3 + s2 * (1.f / 5 + s2 * (1.f / 7 + s2 * (1.f / 9)))));
  }
  return fast_log2(1.f + u) * kLn2;
}

// e^z - 1 - z, accurate near z = 0 (Taylor series through z^10 below |z| < 1/2).
__device__ __forceinline__ float expm1_m(float z) {
  if (fabsf(z) < 0.5f) {
    float s = 1.f / 3628800;
    const float inv[8] = {1.f / 362880, 1.f / 40320, 1.f / 5040, 1.f / 720, 1.f / 120, 1.f / 24, 1.f / 6,
                          1.f / 2};
#pragma unroll
    for (int n = 0; n < 8; ++n) s = s * z + inv[n];
    return s * z * z;
  }
  return fast_exp2(z * kLog2e) - 1.f - z;
}

// 1 - e^z + z e^z = sum_{m >= 2} (m - 1) z^m / m!, accurate near z = 0.
__device__ __forceinline__ float xexp_m(float z) {
  if (fabsf(z) < 0.5f) {
    // coefficients (m - 1)/m! for m = 10 .. 3, then 1/2 for m = 2
    const float c[8] = {9.f / 3628800, 8.f / 362880, 7.f / 40320, 6.f / 5040, 5.f / 720, 4.f / 120,
                        3.f / 24, 2.f / 6};
    float s = c[0];
#pragma unroll
    for (int n = 1; n < 8; ++n) s = s * z + c[n];
    return (s * z + 0.5f) * z * z;
  }
  return 1.f + (z - 1.f) * fast_exp2(z * kLog2e);
}

// (1+u) log(1+u) - u for u >= -1, accurate near u = 0 (series below |u| < 1/4).
__device__ __forceinline__ float xlogx_m(float u) {
  if (fabsf(u) < 0.25f) {
    // sum_{n>=2} (-1)^n u^n / (n (n-1)), through n = 12
    float s = 0.f, un = u * u;
#pragma unroll
    for (int n = 2; n <= 12; ++n) {
      s += ((n & 1) ? -1.f : 1.f) / (float)(n * (n - 1)) * un;
      un *= u;
    }
    return s;
  }
  const float t = 1.f + u;
  return (t > 0.f ? t * (fast_log2(t) * kLn2) : 0.f) - u;
}

// u - log(1+u), accurate near u = 0.
__device__ __forceinline__ float u_mlog(float u) {
  if (fabsf(u) < 0.25f) {
    float s = 0.f, un = u * u;
#pragma unroll
    for (int n = 2; n <= 12; ++n) {
      s += ((n & 1) ? -1.f : 1.f) / (float)n * un;
      un *= u;
    }
    return s;
  }
  return u - fast_log2(1.f + u) * kLn2;
}

// D_{alpha,beta}(y, yh) of App. B for one observed entry, as float.  The
// specialised weight kinds fix the case; WK_GEN selects it at run time.
// Near a fit (y close to yh) every case is written so that no two large
// terms cancel: the relative residual u = (y - yh)/yh is formed from the
// difference y - yh (exact when y and yh are within a factor of two), and
// the cases that are differences of powers are rewritten through
// t = log(y/yh) with series for e^z - 1 - z and 1 - e^z + z e^z:
//   generic:     yh^(a+b)/(a b) [a/(a+b) E((a+b) t) - E(a t)],  E(z) = e^z - 1 - z
//   beta = 0:    yh^a/a^2 F(a t),  F(z) = 1 - e^z + z e^z
//   alpha = -b:  E(a t)/a^2
// (algebraically identical to the definitions; used while |t| <= 1, where no
// overflow can occur, the definitions as written beyond).
template <int WK>
__device__ __forceinline__ float ab_loss(float y, float yh, const FusedArgs& a) {
  if constexpr (WK == WK_KL) {  // y log(y/yh) - y + yh = yh [(1+u) log(1+u) - u]
    return y > 0.f ? yh * xlogx_m((y - yh) * fast_rcp(yh)) : yh;
  } else if constexpr (WK == WK_EUC) {
    const float d = y - yh;
    return 0.5f * d * d;
  } else if constexpr (WK == WK_IS) {  // y/yh - log(y/yh) - 1 = u - log(1+u)
    return u_mlog((y - yh) * fast_rcp(yh));
  } else if constexpr (WK == WK_SQRT) {  // (1/2, 1): (2/3)(sqrt y - sqrt yh)^2 (sqrt y + 2 sqrt yh)
    const float sy = __builtin_sqrtf(y), v = __builtin_sqrtf(yh), d = sy - v;
    return (2.f / 3.f) * d * d * (sy + 2.f * v);
  } else if constexpr (WK == WK_RKL) {  // (0, 1): yh log(yh/y) - yh + y
    return y > 0.f ? y * xlogx_m((yh - y) * fast_rcp(y)) : INFINITY;
  } else if constexpr (WK == WK_FAM) {
    const float ph = a.fparam;
    if (a.lk == LK_NB)  // (phi + y) log(phi + yh) - y log yh
      return ((ph + y) * fast_log2(ph + yh) - (y > 0.f ? y * fast_log2(yh) : 0.f)) * kLn2;
    if (a.lk == LK_BIN)  // n log(1 + yh) - y log yh
      return ph * log1pf(yh) - (y > 0.f ? y * fast_log2(yh) * kLn2 : 0.f);
    // Jensen-Shannon: (y log(y/m) + yh log(yh/m))/2, m = (y + yh)/2.  With
    // y = m (1 + v), yh = m (1 - v): (m/2) [h(v) + h(-v)], h(u) = (1+u) log(1+u) - u >= 0
    const float s = y + yh, v = (y - yh) * fast_rcp(s);
    return 0.25f * s * (xlogx_m(v) + xlogx_m(-v));
  } else {
    const float al = a.alpha, be = a.beta;
    float t = 0.f;
    bool near = false;
    if (y > 0.f) {
      t = log1p_acc((y - yh) * fast_rcp(yh));
      near = fabsf(t) <= 1.f;
    }
    if (a.lk == LK_GENERIC) {
      if (near)
        return a.ab_inv * powpos(yh, al + be) * (al * a.apb_inv * expm1_m((al + be) * t) - expm1_m(al * t));
      return a.ab_inv * (al * a.apb_inv * powpos(y, al + be) + be * a.apb_inv * powpos(yh, al + be) -
                         powpos(y, al) * powpos(yh, be));
    }
    if (a.lk == LK_BETA0) {
      if (near) return powpos(yh, al) * xexp_m(al * t) / (al * al);
      const float ya = powpos(y, al);
      const float lg = y > 0.f ? ya * fast_log2(y / yh) * kLn2 : 0.f;
      return (powpos(yh, al) - ya + al * lg) / (al * al);
    }
    // alpha = -beta
    if (near) return expm1_m(al * t) / (al * al);
    return (powpos(y, al) / powpos(yh, al) - 1.f + al * fast_log2(yh / y) * kLn2) / (al * al);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int KP>
struct Tile {
  static constexpr int PT = KP == 16 ? 4 : (KP == 32 ? 2 : 1);  // 16-wide p subtiles per wave
  static constexpr int ROWS = 16 * PT;                          // rows of a panel
  static constexpr int KS = KP / 4;                             // reconstruction K steps
  static constexpr int KT = KP / 16;                            // kappa tiles of N and D
  static constexpr int RST = KP + 4;                            // LDS row stride (floats)
};


// Weight kinds that divide by yhat or raise it to a negative power need
// yhat >= FLT_MIN (exact arithmetic keeps yhat > 0; FP32 may underflow).
template <int WK>
__device__ constexpr bool needs_floor() {
  return WK == WK_KL || WK == WK_IS || WK == WK_GEN || WK == WK_RKL || WK == WK_FAM;
}

// Weight kinds whose a(y, yhat) vanishes at y = 0 (alpha > 0), so a missing
// entry stored as y = 0 needs no select for Wa.
template <int WK>
__device__ constexpr bool a_zero_at_zero() {
  return WK == WK_KL || WK == WK_EUC || WK == WK_SQRT || WK == WK_IS;
}

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

// One workgroup's tile: braw is the workgroup index within the problem's
// grid (before the XCD remap), slot its loss-partial index.
// PREC: input precision of the contractions (0 = FP32 on 16x16x4 f32 MFMA;
// 1 = BF16, 2 = FP16 numerator/denominator on one 16x16x16 MFMA per kappa tile,
// FP32 accumulation; 3 = BF16, 4 = FP16 for the reconstruction as well, one
// 16x16x16 MFMA per subtile, in the passes without a loss).
template <int KP, int WK, bool VECQ, int MODE, bool FULL, int PREC>
__device__ __forceinline__ void fused_pass_body(const FusedArgs& a, int braw, int slot) {
  using T = Tile<KP>;
  constexpr int PT = T::PT, ROWS = T::ROWS, KS = T::KS, KT = T::KT, RST = T::RST;
  constexpr bool LOSS = MODE >= 1, ND = MODE <= 1;
  constexpr int LP = PREC > 2 ? PREC - 2 : PREC;
  constexpr bool LPREC = PREC > 2 && KS == 4;  // reduced-precision reconstruction (width 16)
  static_assert(PREC <= 2 || !LOSS, "a loss pass keeps an FP32 reconstruction");
  __shared__ f4 red4[ND ? 3 * ROWS * RST / 4 : 1];
  __shared__ double lred[8];
  float* red = reinterpret_cast<float*>(red4);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, c = lane & 15;
  int b = braw;
  if (a.xcd_remap) b = (b & 7) * (a.n_wg >> 3) + (b >> 3);
  const int panel = b % a.n_panels, chunk = b / a.n_panels;
  const int p0 = panel * ROWS;
  const int64_t s_beg = ((int64_t)chunk * 4 + wave) * a.steps_per_wave;
  const int64_t s_end = s_beg + a.steps_per_wave < a.n_steps ? s_beg + a.steps_per_wave : a.n_steps;

  // ---- row side: lane holds Lu[t][s] = L[p][g*KS + s] * u[g*KS + s], p = p0 + 16t + c
  uint32_t poff[PT];
  bool pval[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int p = p0 + 16 * t + c;
    pval[t] = FULL || p < a.nP;
    poff[t] = pval[t] ? a.p_off[p] : 0u;
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
  double lsum = 0.0, vsum = 0.0;

  // ---- outer factors: u[k] = prod_m outer_m[orow_m[qo]][k] is folded into the
  // row operand (Lu = L * u) for the reconstruction, and into the contraction
  // by accumulating per-qo partials tN, tD that are scaled by u and added to
  // accN, accD whenever qo changes.  Column-side values stay raw loads.
  float Lu[PT][KS];
  typename Lp4T<(LP > 0 ? LP : 1)>::v4 LuL[PT];  // Lu converted once per qo (reduced-precision reconstruction)
  f4 uN[KT];  // u at the accumulator rows k = 16 kt + 4g + r
  f4 tN[PT][KT], tD[PT][KT];
  const bool has_outer = a.nouter > 0;
  auto zero_t = [&]() {
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        tN[t][kt] = f4{0.f, 0.f, 0.f, 0.f};
        tD[t][kt] = f4{0.f, 0.f, 0.f, 0.f};
      }
  };
  auto set_u = [&](int qo) {
    float uA[KS];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int p = p0 + 16 * t + c;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = g * KS + s;
        Lu[t][s] = (pval[t] && k < a.K) ? ldf(a.L, (uint32_t)p * (uint32_t)a.ldL + (uint32_t)k) : 0.f;
      }
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) uA[s] = 1.f;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) uN[kt] = f4{1.f, 1.f, 1.f, 1.f};
    for (int m = 0; m < a.nouter; ++m) {
      const float* ob = a.outer[m];
      const uint32_t roff = a.orow[m][qo] * (uint32_t)a.ld_out[m];
#pragma unroll
      for (int s = 0; s < KS; ++s) uA[s] *= ldf(ob, roff + kA[s]);
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r) uN[kt][r] *= ldf(ob, roff + min(16 * kt + 4 * g + r, a.K - 1));
    }
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
      for (int s = 0; s < KS; ++s) Lu[t][s] *= uA[s];
    if constexpr (LPREC) {
#pragma unroll
      for (int t = 0; t < PT; ++t) LuL[t] = cvt4<LP>(Lu[t][0], Lu[t][1], Lu[t][2], Lu[t][3]);
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        accN[t][kt] += uN[kt] * tN[t][kt];
        if (!a.no_d) accD[t][kt] += uN[kt] * tD[t][kt];
      }
    zero_t();
  };

  // column side of one step, raw, in both MFMA layouts
  struct Cols {
    float Ra[KS];     // C[qi0 + c][g*KS + s]
    float Rb[KT][4];  // C[qi0 + 4g + r][16 kt + c]
  };
  const uint32_t ld_in = (uint32_t)a.ld_in, in_stride = (uint32_t)a.in_stride;
  const bool vec_in = a.K == KP && (a.ld_in & 3) == 0;  // float4 loads of inner rows
  auto load_cols = [&](int qo, int qi0, Cols& d) {
    const uint32_t ibase = a.in_base ? a.in_base[qo] : 0u;
    const int qa = qi0 + c;
    if constexpr (FULL) {
      const uint32_t ra = (ibase + (uint32_t)qa * in_stride) * ld_in;
      if (vec_in) {
#pragma unroll
        for (int s = 0; s < KS; s += 4) {
          const f4 v = ldf4(a.inner, ra + g * KS + s);
#pragma unroll
          for (int j = 0; j < 4; ++j) d.Ra[s + j] = v[j];
        }
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) d.Ra[s] = ldf(a.inner, ra + g * KS + s);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t rb = (ibase + (uint32_t)(qi0 + 4 * g + r) * in_stride) * ld_in;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) d.Rb[kt][r] = ldf(a.inner, rb + 16 * kt + c);
      }
    } else {
      // ragged edges: clamp the address, zero the value
      const int qac = qa < a.nqi ? qa : a.nqi - 1;
      const uint32_t ra = (ibase + (uint32_t)qac * in_stride) * ld_in;
      const bool va = qa < a.nqi;
      if (vec_in) {  // full-width rows: float4 loads, only the row is clamped
#pragma unroll
        for (int s = 0; s < KS; s += 4) {
          const f4 v = ldf4(a.inner, ra + g * KS + s);
#pragma unroll
          for (int j = 0; j < 4; ++j) d.Ra[s + j] = va ? v[j] : 0.f;
        }
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const float v = ldf(a.inner, ra + kA[s]);
          d.Ra[s] = (va && g * KS + s < a.K) ? v : 0.f;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int qb = qi0 + 4 * g + r;
        const int qbc = qb < a.nqi ? qb : a.nqi - 1;
        const uint32_t rb = (ibase + (uint32_t)qbc * in_stride) * ld_in;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          const float v = ldf(a.inner, rb + kB[kt]);
          d.Rb[kt][r] = (qb < a.nqi && 16 * kt + c < a.K) ? v : 0.f;
        }
      }
    }
  };

  // data of one step (the HBM stream); a missing entry is stored as -1
  struct YM {
    f4 y[PT];  // y[p0 + 16t + c][qi0 + 4g + r]
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
        const f4 v = ldf4(a.Y, ybase + poff[t] + (uint32_t)q4c);
        d.y[t] = ok ? v : f4{-INFINITY, -INFINITY, -INFINITY, -INFINITY};
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = q4 + r;
          const bool ok = FULL || (pval[t] && q < a.nqi);
          const int qc = FULL ? q : (q < a.nqi ? q : a.nqi - 1);
          const float v = ldf(a.Y, ybase + poff[t] + (uint32_t)qc * qys);
          d.y[t][r] = ok ? v : -INFINITY;
        }
      }
    }
  };

  const bool masked = a.masked != 0;  // else every entry is observed (y >= 0 by contract)
  const bool vmode = LOSS && a.vloss_part != nullptr;
  // One step: reconstruction R(t), weights W(t), contractions ND(t) for the
  // p subtiles t, ordered R(0) R(1)|W(0) ND(0)|W(1) ND(1) ... so that the
  // weight arithmetic of one subtile issues in the shadow of the MFMAs of
  // another (scheduling hints below keep that interleave).
  // reduced-precision column operands of a step, converted once for all subtiles
  typename Lp4T<(LP > 0 ? LP : 1)>::v4 raL, rbL[KT];
  auto recon = [&](int t, const Cols& cl) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (LPREC) {
      // lane (g, c) holds kappa 4g .. 4g+3 of its row and column: the K = 16 form
      acc = mfma4v<LP>(raL, LuL[t], acc);
    } else {
#pragma unroll
      for (int s2 = 0; s2 < KS; ++s2) acc = mfma4(cl.Ra[s2], Lu[t][s2], acc);
    }
    return acc;
  };
  auto weights = [&](int t, const YM& ym, const f4& yh, f4& wa, f4& wb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float yv = ym.y[t][r];
      // ragged tiles pad out-of-range entries with -inf as well: they count as
      // missing whether or not the caller passed a mask
      const bool obs = (FULL && !masked) || observed(yv);
      const float y = (masked || !FULL) ? fmaxf(yv, 0.f) : yv;
      const float yhat = needs_floor<WK>() ? __builtin_amdgcn_fmed3f(yh[r], FLT_MIN, FLT_MAX) : yh[r];
      if constexpr (ND) {
        float xa, xb;
        ab_weights<WK>(y, yhat, WK == WK_FAM ? a.fparam : a.alpha, WK == WK_FAM ? (float)a.lk : a.beta,
                       xa, xb);
        wa[r] = obs ? xa : 0.f;
        wb[r] = obs ? xb : 0.f;
      }
      if constexpr (LOSS) {
        const bool val = vmode && validation(yv);
        const float l = ab_loss<WK>(obs ? y : (val ? -yv : 1.f), (obs || val) ? yhat : 1.f, a);
        lsum += obs ? (double)l : 0.0;
        vsum += val ? (double)l : 0.0;
      }
    }
  };
  auto contract = [&](int t, const Cols& cl, const f4& wa, const f4& wb) {
    if constexpr (ND) {
      // X^T[k][p] += sum_q C^T[k][q] W^T[q][p]   (scaled by u at flush)
      if constexpr (PREC == 0) {
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int r = 0; r < 4; ++r) tN[t][kt] = mfma4(cl.Rb[kt][r], wa[r], tN[t][kt]);
        if (!a.no_d) {
#pragma unroll
          for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int r = 0; r < 4; ++r) tD[t][kt] = mfma4(cl.Rb[kt][r], wb[r], tD[t][kt]);
        }
      } else {
        // the K = 16 form sums the step's 16 columns q = 4g + r in one
        // instruction: lane (g, c) supplies exactly its four r values
        const auto waL = cvt4<LP>(wa[0], wa[1], wa[2], wa[3]);
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) tN[t][kt] = mfma4v<LP>(rbL[kt], waL, tN[t][kt]);
        if (!a.no_d) {
          const auto wbL = cvt4<LP>(wb[0], wb[1], wb[2], wb[3]);
#pragma unroll
          for (int kt = 0; kt < KT; ++kt) tD[t][kt] = mfma4v<LP>(rbL[kt], wbL, tD[t][kt]);
        }
      }
    }
  };
  auto compute = [&](const YM& ym, const Cols& cl) {
    f4 yh[PT], wa[PT], wb[PT];
    if constexpr (LPREC) raL = cvt4<LP>(cl.Ra[0], cl.Ra[1], cl.Ra[2], cl.Ra[3]);
    if constexpr (ND && PREC > 0) {
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) rbL[kt] = cvt4<LP>(cl.Rb[kt][0], cl.Rb[kt][1], cl.Rb[kt][2], cl.Rb[kt][3]);
    }
    yh[0] = recon(0, cl);
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      if (t + 1 < PT) yh[t + 1] = recon(t + 1, cl);
      weights(t, ym, yh[t], wa[t], wb[t]);
      contract(t, cl, wa[t], wb[t]);
    }
    // MFMA/VALU interleave: R(0); then per subtile its successor's R (KS
    // MFMAs) or its own ND (8 KT MFMAs) alternating with the weight VALU.
    __builtin_amdgcn_sched_group_barrier(0x008, LPREC ? 1 : KS, 0);
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int nm = (t + 1 < PT ? (LPREC ? 1 : KS) : 0) + (ND ? (PREC == 0 ? 8 : 2) * KT : 0);
#pragma unroll
      for (int j = 0; j < nm; ++j) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
      }
    }
  };

  // ---- software pipeline: the HBM stream runs two steps ahead, the column
  // side one step ahead; loads of a step are issued column side first so that
  // waiting for them leaves the later Y loads in flight.  Three-stage rings,
  // unrolled so that indices stay static.
  const int64_t nst = s_end > s_beg ? s_end - s_beg : 0;
  int q0 = 0, qis0 = 0;
  if (nst > 0) {
    q0 = (int)(s_beg / a.nqis);
    qis0 = (int)(s_beg - (int64_t)q0 * a.nqis);
  }
  int yq = q0, yqi = qis0;   // next Y step to load
  int cq = q0, cqi = qis0;   // next column step to load
  int kq = q0, kqi = qis0;   // next step to compute
  auto adv = [&](int& qo, int& qis) {
    if (++qis == a.nqis) {
      qis = 0;
      ++qo;
    }
  };
  zero_t();
  int comp_qo = q0;
  if (nst > 0) set_u(q0);
  else {
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
      for (int s = 0; s < KS; ++s) Lu[t][s] = 0.f;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) uN[kt] = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (LPREC) {
#pragma unroll
      for (int t = 0; t < PT; ++t) LuL[t] = cvt4<LP>(0.f, 0.f, 0.f, 0.f);
    }
  }
  YM ym0, ym1, ym2;
  Cols c0, c1, c2;
  if (nst > 0) {
    load_cols(cq, 16 * cqi, c0);
    adv(cq, cqi);
    load_ym(yq, 16 * yqi, ym0);
    adv(yq, yqi);
  }
  if (nst > 1) {
    load_ym(yq, 16 * yqi, ym1);
    adv(yq, yqi);
  }
  auto step = [&](int64_t i, const YM& cy, YM& py, const Cols& cc, Cols& pc) {
    if (i + 1 < nst) {
      load_cols(cq, 16 * cqi, pc);
      adv(cq, cqi);
    }
    if (i + 2 < nst) {
      load_ym(yq, 16 * yqi, py);
      adv(yq, yqi);
    }
    if (kq != comp_qo) {  // entering a new qo: fold the finished one
      if (has_outer) {
        flush();
        set_u(kq);
      }
      comp_qo = kq;
    }
    compute(cy, cc);
    adv(kq, kqi);
  };
  for (int64_t i = 0; i < nst; i += 3) {
    step(i, ym0, ym2, c0, c1);
    if (i + 1 < nst) step(i + 1, ym1, ym0, c1, c2);
    if (i + 2 < nst) step(i + 2, ym2, ym1, c2, c0);
  }
  flush();

  if constexpr (LOSS) {
    const double w = wave_sum(lsum);
    if (lane == 0) lred[wave] = w;
    if (vmode) {  // uniform: the split pack's validation entries
      const double wv = wave_sum(vsum);
      if (lane == 0) lred[4 + wave] = wv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.loss_part[slot] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
      if (vmode) a.vloss_part[slot] = ((lred[4] + lred[5]) + lred[6]) + lred[7];
    }
  }
  if constexpr (ND) {
    store_partial<KP>(accN, a.partN, red, a, wave, g, c, p0, chunk);
    if (!a.no_d) store_partial<KP>(accD, a.partD, red, a, wave, g, c, p0, chunk);
  }
}

template <int KP, int WK, bool VECQ, int MODE, bool FULL, int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void fused_pass(FusedArgs a) {
  fused_pass_body<KP, WK, VECQ, MODE, FULL, PREC>(a, blockIdx.x, blockIdx.x);
}

// Persistent form over many problems (see fused_x32_batched).
template <int KP, int WK, bool VECQ, int MODE, bool FULL, int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void fused_pass_batched(
    const FusedArgs* __restrict__ args, const WorkItem* __restrict__ work, int n_work) {
  for (int w = blockIdx.x; w < n_work; w += gridDim.x) {
    const WorkItem it = work[w];
    const FusedArgs a = args[it.run];
    fused_pass_body<KP, WK, VECQ, MODE, FULL, PREC>(a, it.blk, it.blk);
    __syncthreads();
  }
}

#ifndef NNEF_BATCHED_TU
template <int KP, int WK, bool VECQ, int MODE, int PREC>
int launch_fused_t(const FusedArgs& a, hipStream_t s) {
  if (a.full)
    NNEF_LAUNCH_PASS((fused_pass<KP, WK, VECQ, MODE, true, PREC>), dim3(a.n_wg), dim3(256), s, a);
  else
    NNEF_LAUNCH_PASS((fused_pass<KP, WK, VECQ, MODE, false, PREC>), dim3(a.n_wg), dim3(256), s, a);
  return (int)hipGetLastError();
}

// PREC != 0 is instantiated for the passes with contractions only (modes 0,
// 1); with a reduced-precision reconstruction (PREC > 2) the pass that also
// computes the loss keeps it FP32 (PREC - 2)
template <int KP, int WK, bool VECQ, int PREC>
int launch_fused_m(const FusedArgs& a, int mode, hipStream_t s) {
  if constexpr (PREC != 0) {
    constexpr int P1 = PREC > 2 ? PREC - 2 : PREC;
    return mode == 0 ? launch_fused_t<KP, WK, VECQ, 0, PREC>(a, s) : launch_fused_t<KP, WK, VECQ, 1, P1>(a, s);
  } else {
    switch (mode) {
      case 0: return launch_fused_t<KP, WK, VECQ, 0, 0>(a, s);
      case 1: return launch_fused_t<KP, WK, VECQ, 1, 0>(a, s);
      default: return launch_fused_t<KP, WK, VECQ, 2, 0>(a, s);
    }
  }
}

template <int KP, int WK, int PREC>
int launch_fused_v(const FusedArgs& a, bool vecq, int mode, hipStream_t s) {
  return vecq ? launch_fused_m<KP, WK, true, PREC>(a, mode, s) : launch_fused_m<KP, WK, false, PREC>(a, mode, s);
}

template <int KP, int PREC>
int launch_fused_w(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  switch (wk) {
    case WK_KL: return launch_fused_v<KP, WK_KL, PREC>(a, vecq, mode, s);
    case WK_EUC: return launch_fused_v<KP, WK_EUC, PREC>(a, vecq, mode, s);
    case WK_SQRT: return launch_fused_v<KP, WK_SQRT, PREC>(a, vecq, mode, s);
    case WK_IS: return launch_fused_v<KP, WK_IS, PREC>(a, vecq, mode, s);
    case WK_GEN: return launch_fused_v<KP, WK_GEN, PREC>(a, vecq, mode, s);
    case WK_RKL: return launch_fused_v<KP, WK_RKL, PREC>(a, vecq, mode, s);
    default: return launch_fused_v<KP, WK_FAM, PREC>(a, vecq, mode, s);
  }
}

#else
template <int KP, int WK, bool VECQ, int MODE>
int launch_fused_batched_t(const BatchedLaunch& L, hipStream_t s) {
  if (L.full)
    hipLaunchKernelGGL((fused_pass_batched<KP, WK, VECQ, MODE, true, 0>), dim3(L.grid), dim3(256), 0, s,
                       L.args, L.work, L.n_work);
  else
    hipLaunchKernelGGL((fused_pass_batched<KP, WK, VECQ, MODE, false, 0>), dim3(L.grid), dim3(256), 0, s,
                       L.args, L.work, L.n_work);
  return (int)hipGetLastError();
}

template <int KP, int WK>
int launch_fused_batched_v(const BatchedLaunch& L, hipStream_t s) {
  if (L.vecq)
    return L.mode ? launch_fused_batched_t<KP, WK, true, 1>(L, s) : launch_fused_batched_t<KP, WK, true, 0>(L, s);
  return L.mode ? launch_fused_batched_t<KP, WK, false, 1>(L, s) : launch_fused_batched_t<KP, WK, false, 0>(L, s);
}

template <int KP>
int launch_fused_batched_w(const BatchedLaunch& L, hipStream_t s) {
  switch (L.wk) {
    case WK_KL: return launch_fused_batched_v<KP, WK_KL>(L, s);
    case WK_EUC: return launch_fused_batched_v<KP, WK_EUC>(L, s);
    case WK_SQRT: return launch_fused_batched_v<KP, WK_SQRT>(L, s);
    case WK_IS: return launch_fused_batched_v<KP, WK_IS>(L, s);
    case WK_GEN: return launch_fused_batched_v<KP, WK_GEN>(L, s);
    case WK_RKL: return launch_fused_batched_v<KP, WK_RKL>(L, s);
    default: return launch_fused_batched_v<KP, WK_FAM>(L, s);
  }
}

#endif
}  // namespace
}  // namespace nnef
