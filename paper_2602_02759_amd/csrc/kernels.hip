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

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
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

// D_{alpha,beta}(y, yh) of App. B for one observed entry, as float.
__device__ __forceinline__ float ab_loss(float y, float yh, const FusedArgs& a) {
  const float ln2 = 0.69314718055994531f;
  switch (a.lk) {
    case LK_KL:  // y log(y/yh) - y + yh = yh [(1+u) log(1+u) - u], u = y/yh - 1
      return y > 0.f ? yh * xlogx_m(y / yh - 1.f) : yh;
    case LK_EUC: {
      float d = y - yh;
      return 0.5f * d * d;
    }
    case LK_IS:  // y/yh - log(y/yh) - 1 = u - log(1+u)
      return u_mlog(y / yh - 1.f);
    case LK_SQRT: {  // (alpha,beta) = (1/2, 1): (2/3) (sqrt y - sqrt yh)^2 (sqrt y + 2 sqrt yh)
      float s = __builtin_sqrtf(y), v = __builtin_sqrtf(yh), d = s - v;
      return (2.f / 3.f) * d * d * (s + 2.f * v);
    }
    case LK_GENERIC: {
      float al = a.alpha, be = a.beta;
      return a.ab_inv * (al * a.apb_inv * powpos(y, al + be) + be * a.apb_inv * powpos(yh, al + be) -
                         powpos(y, al) * powpos(yh, be));
    }
    case LK_BETA0: {
      float al = a.alpha, ya = powpos(y, al);
      float lg = y > 0.f ? ya * fast_log2(y / yh) * ln2 : 0.f;
      return (powpos(yh, al) - ya + al * lg) / (al * al);
    }
    case LK_AMB: {
      float al = a.alpha;
      return (powpos(y, al) / powpos(yh, al) - 1.f + al * fast_log2(yh / y) * ln2) / (al * al);
    }
    case LK_ALPHA0: {
      float be = a.beta, yb = powpos(yh, be);
      return (be * yb * fast_log2(yh / y) * ln2 - yb + powpos(y, be)) / (be * be);
    }
    default: {
      float d = (fast_log2(y) - fast_log2(yh)) * ln2;
      return 0.5f * d * d;
    }
  }
}

// Row of the column side: R[q][k] = prod_m piece_m[idx_m(q) * ld_m + k].
__device__ __forceinline__ float side_val(const FusedArgs& a, const uint32_t* rows, int k) {
  float v = 1.f;
#pragma unroll
  for (int m = 0; m < kMaxPieces; ++m)
    if (m < a.npieces) v *= a.piece[m][(size_t)rows[m] * a.ldpiece[m] + k];
  return v;
}

__device__ __forceinline__ void side_rows(const FusedArgs& a, int q, uint32_t* rows) {
#pragma unroll
  for (int m = 0; m < kMaxPieces; ++m)
    rows[m] = (m < a.npieces) ? (a.pidx[m] ? a.pidx[m][q] : (uint32_t)q) : 0u;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Accumulator element (t, kt, r) is X^T[k = 16kt + 4g + r][p = 16t + c].  Waves
// 1..3 stash theirs in LDS; wave 0 adds them in a fixed order and stores the
// workgroup's partial row block.
template <int KP, int PT, int KT, int RST>
__device__ __forceinline__ void store_partial(const f4 (&acc)[PT][KT], float* dst, float* red,
                                              const FusedArgs& a, int wave, int g, int c, int p0,
                                              int chunk) {
  constexpr int ROWS = 16 * PT;
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

template <int KP, int WK, bool VECQ>
__global__ __launch_bounds__(256) void fused_pass(FusedArgs a) {
  constexpr int PT = (KP == 64) ? 2 : 4;  // 16-wide p subtiles per wave
  constexpr int ROWS = 16 * PT;           // p rows of a panel
  constexpr int KS = KP / 4;              // reconstruction K steps
  constexpr int KT = KP / 16;             // kappa tiles of N and D
  constexpr int RST = KP + 4;             // LDS row stride (floats)
  __shared__ f4 red4[3 * ROWS * RST / 4];
  __shared__ double lred[4];
  float* red = reinterpret_cast<float*>(red4);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  int b = blockIdx.x;
  if (a.xcd_remap) b = (b & 7) * (a.n_wg >> 3) + (b >> 3);
  const int panel = b % a.n_panels, chunk = b / a.n_panels;
  const int p0 = panel * ROWS;
  const int qbeg = (chunk * 4 + wave) * a.q_per_wave;
  const int qend = min(qbeg + a.q_per_wave, a.nQ);

  // Row side, kept in registers for the whole pass: lane holds L[p][g*KS + s].
  float Lop[PT][KS];
  uint32_t poff[PT];
  bool pval[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int p = p0 + 16 * t + c;
    pval[t] = p < a.nP;
    poff[t] = pval[t] ? a.p_off[p] : 0u;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = g * KS + s;
      Lop[t][s] = (pval[t] && k < a.K) ? a.L[(size_t)p * a.ldL + k] : 0.f;
    }
  }

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

  for (int q0 = qbeg; q0 < qend; q0 += 16) {
    // ---- column side operands
    // Ra[s] = R[q0 + c][g*KS + s]   (A operand of the reconstruction)
    // Rb[kt][r] = R[q0 + 4g + r][16 kt + c]   (A operand of N and D)
    float Ra[KS], Rb[KT][4];
    {
      const int qa = q0 + c;
      uint32_t rows[kMaxPieces];
      const bool va = qa < a.nQ;
      side_rows(a, va ? qa : 0, rows);
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = g * KS + s;
        Ra[s] = (va && k < a.K) ? side_val(a, rows, k) : 0.f;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int qb = q0 + 4 * g + r;
        const bool vb = qb < a.nQ;
        side_rows(a, vb ? qb : 0, rows);
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          const int k = 16 * kt + c;
          Rb[kt][r] = (vb && k < a.K) ? side_val(a, rows, k) : 0.f;
        }
      }
    }
    // ---- data: y and mask for rows q0 + 4g + r of each p subtile
    f4 yv[PT];
    uint32_t mv[PT];
    uint32_t qo[4];
    bool qv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = q0 + 4 * g + r;
      qv[r] = q < a.nQ;
      if (!VECQ || r == 0) qo[r] = qv[r] ? a.q_off[q] : 0u;
      else qo[r] = qo[0] + r;
    }
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      if constexpr (VECQ) {
        const bool ok = pval[t] && qv[0];
        const size_t off = (size_t)poff[t] + qo[0];
        yv[t] = ok ? *reinterpret_cast<const f4*>(a.Y + off) : f4{0.f, 0.f, 0.f, 0.f};
        if (has_mask) mv[t] = ok ? *reinterpret_cast<const uint32_t*>(a.M + off) : 0u;
        else mv[t] = ok ? 0x01010101u : 0u;
      } else {
        uint32_t m = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const bool ok = pval[t] && qv[r];
          const size_t off = (size_t)poff[t] + qo[r];
          yv[t][r] = ok ? a.Y[off] : 0.f;
          uint32_t mb = ok ? (has_mask ? (uint32_t)a.M[off] : 1u) : 0u;
          m |= mb << (8 * r);
        }
        mv[t] = m;
      }
    }
    // ---- reconstruction tile, transposed: acc[t][r] = yhat[p0+16t+c][q0+4g+r]
    f4 yh[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) acc = mfma4(Ra[s], Lop[t][s], acc);
      yh[t] = acc;
    }
    // ---- weights (and loss)
    f4 wa[PT], wb[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool obs = (mv[t] >> (8 * r)) & 0xffu;
        const float y = yv[t][r];
        const float yhat = fmaxf(yh[t][r], FLT_MIN);
        float xa, xb;
        ab_weights<WK>(y, yhat, a.alpha, a.beta, xa, xb);
        wa[t][r] = obs ? xa : 0.f;
        wb[t][r] = obs ? xb : 0.f;
        if (a.loss_part && obs) lsum += (double)ab_loss(y, yhat, a);
      }
    }
    if (a.loss_only) continue;
    // ---- contractions: N^T[k][p] += sum_q R^T[k][q] Wa^T[q][p]
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r) accN[t][kt] = mfma4(Rb[kt][r], wa[t][r], accN[t][kt]);
    if (!a.no_d) {
#pragma unroll
      for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int r = 0; r < 4; ++r) accD[t][kt] = mfma4(Rb[kt][r], wb[t][r], accD[t][kt]);
    }
  }

  // ---- loss: wave sum, then the four waves in fixed order
  if (a.loss_part) {
    double w = wave_sum(lsum);
    if (lane == 0) lred[wave] = w;
    __syncthreads();
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
  }
  if (a.loss_only) return;

  // ---- partial N, D: waves 1..3 stash, wave 0 adds in fixed order and stores
  store_partial<KP, PT, KT, RST>(accN, a.partN, red, a, wave, g, c, p0, chunk);
  if (!a.no_d) store_partial<KP, PT, KT, RST>(accD, a.partD, red, a, wave, g, c, p0, chunk);
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ float mu_rule(float th, float n, float d, int upd, float gamma,
                                         float eps) {
  if (!(d > 0.f)) return th;  // every entry depending on theta is missing: keep it
  const float r = n / d;
  float s;
  switch (upd) {
    case UP_ONE: s = r; break;
    case UP_SQR: s = r * r; break;
    case UP_SQRT: s = __builtin_sqrtf(r); break;
    case UP_EXP: s = expf(r); break;
    default: s = r > 0.f ? exp2f(gamma * log2f(r)) : (gamma > 0.f ? 0.f : INFINITY); break;
  }
  return fmaxf(eps, th * s);
}

__global__ __launch_bounds__(256) void colsum_kernel(UpdateArgs a, float* dcol) {
  // dcol[k] = prod_m sum_rows piece_m[row][k]; one workgroup, K <= 64
  __shared__ double part[4][64];
  const int k = threadIdx.x & 63, w = threadIdx.x >> 6;
  double prod = 1.0;
  for (int m = 0; m < a.npieces; ++m) {
    double s = 0.0;
    if (k < a.K)
      for (int64_t row = w; row < a.nrows[m]; row += 4) s += a.piece[m][row * a.ldpiece[m] + k];
    part[w][k] = s;
    __syncthreads();
    if (w == 0) prod *= ((part[0][k] + part[1][k]) + part[2][k]) + part[3][k];
    __syncthreads();
  }
  if (w == 0 && k < a.K) dcol[k] = (float)prod;
}

__global__ __launch_bounds__(256) void update_kernel(UpdateArgs a, const float* dcol) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)a.nP * a.K;
  if (idx < n) {
    const int p = (int)(idx / a.K), k = (int)(idx % a.K);
    double N = 0.0, D = 0.0;
    for (int ch = 0; ch < a.n_chunks; ++ch) N += a.partN[((size_t)ch * a.nP + p) * a.KP + k];
    if (a.no_d) {
      D = dcol[k];
    } else {
      for (int ch = 0; ch < a.n_chunks; ++ch) D += a.partD[((size_t)ch * a.nP + p) * a.KP + k];
    }
    if (a.theta) {
      float* th = a.theta + (size_t)p * a.ldT + k;
      *th = mu_rule(*th, (float)N, (float)D, a.upd, a.gamma, a.eps);
    } else {
      a.NL[idx] = (float)N;
      a.DL[idx] = (float)D;
    }
  }
  if (a.loss_out && blockIdx.x == 0 && threadIdx.x < 64) {
    double s = 0.0;
    for (int i = threadIdx.x; i < a.n_loss_part; i += 64) s += a.loss_part[i];
    s = wave_sum(s);
    if (threadIdx.x == 0) *a.loss_out = s;
  }
}

__global__ __launch_bounds__(64) void loss_final_kernel(const double* part, int n, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += part[i];
  s = wave_sum(s);
  if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(256) void apply_kernel(ApplyArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n) a.theta[i] = mu_rule(a.theta[i], a.N[i], a.D[i], a.upd, a.gamma, a.eps);
}

__global__ __launch_bounds__(256) void einsum_kernel(EinsumArgs a) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= a.n_out_total) return;
  int64_t off[kMaxEinsumIn] = {0, 0, 0, 0};
  int64_t ooff = 0, rem = o;
  for (int d = a.n_out - 1; d >= 0; --d) {
    const int64_t v = rem % a.out_size[d];
    rem /= a.out_size[d];
    ooff += v * a.out_stride[d];
    for (int i = 0; i < a.n_in; ++i) off[i] += v * a.in_out_stride[i][d];
  }
  int64_t n_sum = 1;
  for (int d = 0; d < a.n_sum; ++d) n_sum *= a.sum_size[d];
  int64_t cnt[kMaxEinsumLetters] = {0};
  double acc = 0.0;
  for (int64_t cidx = 0; cidx < n_sum; ++cidx) {
    float prod = 1.f;
    for (int i = 0; i < a.n_in; ++i) prod *= a.in[i][off[i]];
    acc += (double)prod;
    for (int d = a.n_sum - 1; d >= 0; --d) {
      ++cnt[d];
      for (int i = 0; i < a.n_in; ++i) off[i] += a.in_sum_stride[i][d];
      if (cnt[d] < a.sum_size[d]) break;
      for (int i = 0; i < a.n_in; ++i) off[i] -= a.sum_size[d] * a.in_sum_stride[i][d];
      cnt[d] = 0;
    }
  }
  a.out[ooff] = (float)acc;
}

__global__ __launch_bounds__(256) void zero_kernel(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <int KP, int WK, bool VECQ>
static int launch_fused_t(const FusedArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((fused_pass<KP, WK, VECQ>), dim3(a.n_wg), dim3(256), 0, s, a);
  return (int)hipGetLastError();
}

template <int KP, int WK>
static int launch_fused_v(const FusedArgs& a, bool vecq, hipStream_t s) {
  return vecq ? launch_fused_t<KP, WK, true>(a, s) : launch_fused_t<KP, WK, false>(a, s);
}

template <int KP>
static int launch_fused_w(const FusedArgs& a, int wk, bool vecq, hipStream_t s) {
  switch (wk) {
    case WK_KL: return launch_fused_v<KP, WK_KL>(a, vecq, s);
    case WK_EUC: return launch_fused_v<KP, WK_EUC>(a, vecq, s);
    case WK_SQRT: return launch_fused_v<KP, WK_SQRT>(a, vecq, s);
    case WK_IS: return launch_fused_v<KP, WK_IS>(a, vecq, s);
    case WK_GEN: return launch_fused_v<KP, WK_GEN>(a, vecq, s);
    default: return launch_fused_v<KP, WK_RKL>(a, vecq, s);
  }
}

int launch_fused(const FusedArgs& a, int KP, int wk, bool vecq, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (KP) {
    case 16: return launch_fused_w<16>(a, wk, vecq, s);
    case 32: return launch_fused_w<32>(a, wk, vecq, s);
    case 64: return launch_fused_w<64>(a, wk, vecq, s);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_update(const UpdateArgs& a, float* dcol, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (a.no_d) {
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, a, dcol);
  }
  const int64_t n = (int64_t)a.nP * a.K;
  const int grid = (int)((n + 255) / 256);
  hipLaunchKernelGGL(update_kernel, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, a, dcol);
  return (int)hipGetLastError();
}


int launch_einsum(const EinsumArgs& a, void* stream) {
  if (a.n_out_total <= 0) return 0;
  const int64_t grid = (a.n_out_total + 255) / 256;
  hipLaunchKernelGGL(einsum_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_apply(const ApplyArgs& a, void* stream) {
  if (a.n <= 0) return 0;
  hipLaunchKernelGGL(apply_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_loss_final(const double* part, int n, double* out, void* stream) {
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, part, n, out);
  return (int)hipGetLastError();
}

int launch_zero(float* p, int64_t n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, p, n);
  return (int)hipGetLastError();
}

}  // namespace nnef
