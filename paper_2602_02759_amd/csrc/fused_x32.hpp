// Fused pass for contraction widths 32 (NT = 1) and 64 (NT = 2) on
// v_mfma_f32_32x32x2_f32.
//
// Same computation as fused_pass in fused_impl.hpp (one block update's pass
// over Y: reconstruction tile, masked (alpha, beta) weights, numerator and
// denominator contractions), with 32 x 32 tiles: this MFMA form sustains the
// full FP32 matrix rate of the chip, the 16x16x4 form does not.  The
// contraction width is NT tiles of 32: the reconstruction sums all of them
// into one 32 x 32 tile, and N, D keep one accumulator tile each per kappa
// tile (width 64 runs one wave per SIMD to hold them without spills).
//
// MFMA layout (32x32x2): lane l = 32*g + c supplies A[row c][k g] and
// B[k g][col c]; the accumulator register v holds C[row 8(v/4) + 4g + v%4][col c].
// The tile is computed transposed, Yhat^T[q][p], so each lane owns one p and
// 16 q values, which feed the contraction MFMAs directly as the B operand
// (K = q).  A wave covers 32 rows p and steps of 32 columns q.
#pragma once
#include "fused_impl.hpp"

namespace nnef {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f16v mfma32(float a, float b, const f16v& c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Reduced-precision contraction operands: MFMA m (0, 1) of the K = 16 form
// takes this lane's accumulator rows v = 8m .. 8m+7 as its eight K slots; the
// A and B operands use the same permutation of q, so the sum is unchanged.
// LP = 1: BF16, 2: FP16.  An operand is converted once and may feed several
// MFMA (the column operand of N and D, the factor rows of every step of a qo).
template <int LP>
struct LpT {
  typedef bf16x8 v8;
};
template <>
struct LpT<2> {
  typedef f16x8 v8;
};

template <int LP>
__device__ __forceinline__ typename LpT<LP>::v8 cvt8(const float* v) {
  typename LpT<LP>::v8 x;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if constexpr (LP == 2) x[j] = (_Float16)v[j];
    else x[j] = (__bf16)v[j];
  }
  return x;
}

template <int LP>
__device__ __forceinline__ f16v mfma8(const typename LpT<LP>::v8& a, const typename LpT<LP>::v8& b, const f16v& c) {
  if constexpr (LP == 2) return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// PREC: input precision of the contractions: 0 = FP32; 1 = BF16, 2 = FP16
// for the numerator and denominator; 3 = BF16, 4 = FP16 for the
// reconstruction as well (instantiated for the passes without a loss only).
// One workgroup's tile: braw is the workgroup index within the problem's
// grid (before the XCD remap), slot its loss-partial index.
template <int NT, int WK, bool VECQ, int MODE, bool FULL, int PREC>
__device__ __forceinline__ void fused_x32_body(const FusedArgs& a, int braw, int slot) {
  constexpr int KP = 32 * NT, ROWS = 32, RST = KP + 4;
  constexpr bool LOSS = MODE >= 1, ND = MODE <= 1;
  constexpr int LP = PREC > 2 ? PREC - 2 : PREC;  // MFMA input type of the reduced-precision forms
  static_assert(PREC <= 2 || !LOSS, "a loss pass keeps an FP32 reconstruction");
  // Y ring for the direct-to-LDS prefetch of full tiles: kStages stages of 4 KB
  // per wave; after the main loop the same memory holds the partial reduction.
  constexpr int kStages = 4;
  constexpr int kRing = FULL ? 4 * kStages * 256 : 0;     // f4 elements
  constexpr int kRed = ND ? 3 * ROWS * RST / 4 : 1;       // f4 elements
  __shared__ f4 lds4[kRing > kRed ? kRing : kRed];
  __shared__ double lred[8];
  float* red = reinterpret_cast<float*>(lds4);

  // Every argument the prologue reads, requested in one batch: left to
  // themselves the scalar loads follow the control flow below, one
  // round trip to cold caches at a time, before the first data move.
  {
    const int i0 = a.xcd_remap, i1 = a.n_wg, i2 = a.n_panels, i3 = a.wave_rows, i4 = a.steps_per_wave,
              i5 = a.nqis, i6 = a.nP, i7 = a.masked, i8 = a.nouter, i9 = a.K, i10 = a.ldL, i11 = a.ld_out[0];
    const int64_t l0 = a.n_steps;
    const void *p0 = a.Y, *p1 = a.p_off, *p2 = a.qo_yoff, *p3 = a.in_base, *p4 = a.inner, *p5 = a.outer[0],
               *p6 = a.orow[0], *p7 = a.L;
    __asm__ volatile("" ::"s"(i0), "s"(i1), "s"(i2), "s"(i3), "s"(i4), "s"(i5), "s"(i6), "s"(i7), "s"(i8), "s"(i9),
                     "s"(i10), "s"(i11), "s"(l0), "s"(p0), "s"(p1), "s"(p2), "s"(p3), "s"(p4), "s"(p5), "s"(p6),
                     "s"(p7));
  }

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 5, c = lane & 31;
  int b = braw;
  if (a.xcd_remap) b = (b & 7) * (a.n_wg >> 3) + (b >> 3);
  const int panel = b % a.n_panels, chunk = b / a.n_panels;
  // wave_rows: the four waves take four consecutive 32-row panels over the same
  // steps (for blocks with many rows and few column steps); otherwise they
  // share one panel and split the steps
  const bool wrows = a.wave_rows != 0;
  const int p0 = wrows ? (panel * 4 + wave) * ROWS : panel * ROWS;
  const int64_t s_beg = wrows ? (int64_t)chunk * a.steps_per_wave
                              : ((int64_t)chunk * 4 + wave) * a.steps_per_wave;
  const int64_t s_end = s_beg + a.steps_per_wave < a.n_steps ? s_beg + a.steps_per_wave : a.n_steps;

  const int p = p0 + c;
  const bool pval = FULL || p < a.nP;
  const uint32_t poff = pval ? a.p_off[p] : 0u;
  const bool masked = a.masked != 0;
  const bool vmode = LOSS && a.vloss_part != nullptr;

  f16v accN[NT], accD[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    accN[t] = f16v{};
    accD[t] = f16v{};
  }
  double lsum = 0.0, vsum = 0.0;

  // ---- row operand: Lr[t][s] = L[p][32t + 16g + s] (0 past K or the last
  // row); loaded once in the ragged path, with each new qo for full tiles.
  float Lr[NT][16];
  auto load_L = [&]() {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int k = 32 * t + 16 * g + s;
        Lr[t][s] = (pval && k < a.K) ? ldf(a.L, (uint32_t)p * (uint32_t)a.ldL + (uint32_t)k) : 0.f;
      }
  };

  // ---- outer factors of a step's column index qo: u[k] = prod_m
  // outer_m[orow_m[qo]][k].  In the ragged path their rows are moved into a
  // per-wave LDS slot (qo mod 4) by direct-to-LDS loads that need no
  // registers, one step ahead of the step that starts the qo, which reads
  // them back: short inner modes start a new qo every few steps.
  __shared__ float ulds[FULL ? 1 : 4][4][2 * KP];  // [wave][slot][piece * KP + k] (ragged path)
  float* ub = &ulds[FULL ? 0 : wave][0][0];
  const int nout = a.nouter;
  auto dma_u = [&](int qo) {
    if (nout == 0) return;
    qo = __builtin_amdgcn_readfirstlane(qo);
    const uint32_t r0 = a.orow[0][qo] * (uint32_t)a.ld_out[0];
    const uint32_t r1 = nout > 1 ? a.orow[1][qo] * (uint32_t)a.ld_out[1] : r0;
    const float* o1 = nout > 1 ? a.outer[1] : a.outer[0];
    float* dst = ub + (qo & 3) * (2 * KP);
    if constexpr (NT == 1) {  // lanes 0..31: piece 0, lanes 32..63: piece 1 (or piece 0 again)
      const uint32_t e = (uint32_t)min(lane & 31, a.K - 1);
      // the two row addresses as integers, selected per lane (no pointer array)
      const uint64_t b0 = (uint64_t)(uintptr_t)(a.outer[0] + r0), b1 = (uint64_t)(uintptr_t)(o1 + r1);
      const uint64_t src = (lane < 32 ? b0 : b1) + 4ull * e;
      __builtin_amdgcn_global_load_lds((const void*)(uintptr_t)src, (__attribute__((address_space(3))) void*)dst, 4,
                                       0, 0);
    } else {
      const uint32_t e = (uint32_t)min(lane, a.K - 1);
      __builtin_amdgcn_global_load_lds((const void*)(a.outer[0] + r0 + e),
                                       (__attribute__((address_space(3))) void*)dst, 4, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(o1 + r1 + e),
                                       (__attribute__((address_space(3))) void*)(dst + KP), 4, 0, 0);
    }
  };
  // per-qo state, formed when a step starts a new qo: Lu[t][s] = L[p][32t +
  // 16g + s] u[32t + 16g + s] (the reconstruction's B operand) and ul[t] =
  // u[32t + c] (scales the contraction's A operand of kappa tile t).  Full
  // tiles read the rows from memory there (their steps per qo are many);
  // ragged tiles read the rows moved into LDS and the row operand Lr.
  float Lu[NT][16], ul[NT];
  typename LpT<(PREC > 2 ? PREC - 2 : 1)>::v8 LuL[NT][2];  // Lu converted (PREC > 2)
  auto set_u = [&](int qo) {
    float uA[NT][16];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int s = 0; s < 16; ++s) uA[t][s] = 1.f;
      ul[t] = 1.f;
    }
    if constexpr (FULL) {
      for (int m = 0; m < nout; ++m) {
        const float* ob = a.outer[m];
        const uint32_t roff = a.orow[m][qo] * (uint32_t)a.ld_out[m];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
          for (int s = 0; s < 16; ++s) uA[t][s] *= ldf(ob, roff + min(32 * t + 16 * g + s, a.K - 1));
          ul[t] *= ldf(ob, roff + min(32 * t + c, a.K - 1));
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const int k = 32 * t + 16 * g + s;
          const float lv = (pval && k < a.K) ? ldf(a.L, (uint32_t)p * (uint32_t)a.ldL + (uint32_t)k) : 0.f;
          Lu[t][s] = lv * uA[t][s];
        }
    } else {
      if (nout > 0) {
        const float* us = ub + (qo & 3) * (2 * KP);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
          for (int s = 0; s < 16; ++s) uA[t][s] = us[32 * t + 16 * g + s];
          ul[t] = us[32 * t + c];
        }
        if (nout > 1) {
#pragma unroll
          for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int s = 0; s < 16; ++s) uA[t][s] *= us[KP + 32 * t + 16 * g + s];
            ul[t] *= us[KP + 32 * t + c];
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 16; ++s) Lu[t][s] = Lr[t][s] * uA[t][s];
    }
    if constexpr (PREC > 2) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        LuL[t][0] = cvt8<LP>(Lu[t]);
        LuL[t][1] = cvt8<LP>(Lu[t] + 8);
      }
    }
  };

  // ---- column side of one step (raw inner rows).  Every load is a
  // wave-uniform pointer plus a loop-invariant lane offset, so a step's
  // addressing is scalar arithmetic only.
  struct Cols {
    float Ra[NT][16];  // C[qi0 + c][32t + 16g + s]             (A of the reconstruction)
    float Rb[NT][16];  // C[qi0 + 8(v/4) + 4g + v%4][32t + c]   (A of N and D, MFMA step v)
  };
  const uint32_t ld_in = (uint32_t)a.ld_in, in_stride = (uint32_t)a.in_stride;
  // full tiles: inner rows are KP floats apart (K = ld = KP, in_stride = 1), so
  // every offset inside a step is a compile-time immediate on one base pointer
  const uint32_t offA = (uint32_t)c * KP + 16u * g;         // lane part of Ra addresses
  const uint32_t offB = (uint32_t)(4 * g) * KP + (uint32_t)c;  // lane part of Rb addresses
  auto load_cols = [&](uint32_t ibase, int qi0, Cols& d) {
    if constexpr (FULL) {
      const float* base = a.inner + (size_t)(ibase + (uint32_t)qi0) * KP;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 16; s += 4) {
          const f4 v = ldf4(base, offA + 32 * t + s);
          d.Ra[t][s] = v[0];
          d.Ra[t][s + 1] = v[1];
          d.Ra[t][s + 2] = v[2];
          d.Ra[t][s + 3] = v[3];
        }
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          d.Rb[t][v] = ldf(base, offB + 32 * t + (uint32_t)(8 * (v >> 2) + (v & 3)) * KP);
    } else {
      const int qa = qi0 + c;
      const bool va = qa < a.nqi;
      const uint32_t ra = (ibase + (uint32_t)(va ? qa : a.nqi - 1) * in_stride) * ld_in;
      if (a.K == KP && (ld_in & 3u) == 0) {  // full-width rows: float4 loads
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int s = 0; s < 16; s += 4) {
            const f4 v = ldf4(a.inner, ra + 32u * t + 16u * g + s);
#pragma unroll
            for (int j = 0; j < 4; ++j) d.Ra[t][s + j] = va ? v[j] : 0.f;
          }
      } else {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            const int k = 32 * t + 16 * g + s;
            const float v = ldf(a.inner, ra + (uint32_t)min(k, a.K - 1));
            d.Ra[t][s] = (va && k < a.K) ? v : 0.f;
          }
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int qb = qi0 + 8 * (v >> 2) + 4 * g + (v & 3);
        const uint32_t rb = (ibase + (uint32_t)(qb < a.nqi ? qb : a.nqi - 1) * in_stride) * ld_in;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const bool vb = qb < a.nqi && 32 * t + c < a.K;
          const float x = ldf(a.inner, rb + (uint32_t)min(32 * t + c, a.K - 1));
          d.Rb[t][v] = vb ? x : 0.f;
        }
      }
    }
  };

  // ---- data of one step: y[q0 + 8(v/4) + 4g + v%4][p]; a missing entry holds -1
  struct YM {
    f4 y[4];
  };
  const uint32_t qys = (uint32_t)a.qi_ystride;
  const uint32_t offY = poff + 4u * g;               // lane part of Y addresses (VECQ)
  const uint32_t offYs = poff + (uint32_t)(4 * g) * qys;  // lane part of Y addresses (strided q)
  auto load_ym = [&](uint32_t ybase, int qi0, YM& d) {
#pragma unroll
    for (int bq = 0; bq < 4; ++bq) {
      const int q4 = qi0 + 8 * bq + 4 * g;
      if constexpr (VECQ) {
        if constexpr (FULL) {
          d.y[bq] = ldf4(a.Y + ybase + (uint32_t)qi0, offY + 8u * bq);
        } else {
          const bool ok = pval && q4 < a.nqi;
          const int q4c = q4 < a.nqi ? q4 : a.nqi - 4;
          const f4 v = ldf4(a.Y, ybase + poff + (uint32_t)q4c);
          d.y[bq] = ok ? v : f4{-INFINITY, -INFINITY, -INFINITY, -INFINITY};
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = q4 + r;
          if constexpr (FULL) {
            d.y[bq][r] = ldf(a.Y + ybase + (size_t)(qi0 + 8 * bq + r) * qys, offYs);
          } else {
            const bool ok = pval && q < a.nqi;
            const float v = ldf(a.Y, ybase + poff + (uint32_t)(q < a.nqi ? q : a.nqi - 1) * qys);
            d.y[bq][r] = ok ? v : -INFINITY;
          }
        }
      }
    }
  };

  // ---- direct-to-LDS prefetch of Y for full tiles.  Every lane moves its own
  // 16 B (VECQ) or 4 B (strided q) and reads back exactly what it moved, so
  // the ring is private to the wave and needs no barrier; completion is a
  // vmcnt wait (the LDS DMA counts as a vector memory operation).
  f4* ring = lds4 + wave * (kStages * 256);
  auto dma_ym = [&](uint32_t ybase, int qi0, int stage) {
    if constexpr (FULL) {
      f4* st = ring + stage * 256;
      if constexpr (VECQ) {
        const float* src = a.Y + ybase + (uint32_t)qi0 + offY;
#pragma unroll
        for (int bq = 0; bq < 4; ++bq)
          __builtin_amdgcn_global_load_lds((const void*)(src + 8 * bq),
                                           (__attribute__((address_space(3))) void*)(st + 64 * bq), 16, 0, 0);
      } else {
        float* stf = reinterpret_cast<float*>(st);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const float* src = a.Y + ybase + (size_t)(qi0 + 8 * (v >> 2) + (v & 3)) * qys + offYs;
          __builtin_amdgcn_global_load_lds((const void*)src,
                                           (__attribute__((address_space(3))) void*)(stf + 64 * v), 4, 0, 0);
        }
      }
    }
  };
  auto read_ym = [&](int stage, YM& d) {
    const f4* st = ring + stage * 256;
    if constexpr (VECQ) {
#pragma unroll
      for (int bq = 0; bq < 4; ++bq) d.y[bq] = st[64 * bq + lane];
    } else {
      const float* stf = reinterpret_cast<const float*>(st);
#pragma unroll
      for (int v = 0; v < 16; ++v) d.y[v >> 2][v & 3] = stf[64 * v + lane];
    }
  };

  auto compute = [&](const YM& ym, const Cols& cl) {
    f16v yh = {};
    if constexpr (PREC > 2) {
      // K = 16 form: MFMA m takes the lane's kappa values 8m .. 8m+7 of each tile
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        yh = mfma8<LP>(cvt8<LP>(cl.Ra[t]), LuL[t][0], yh);
        yh = mfma8<LP>(cvt8<LP>(cl.Ra[t] + 8), LuL[t][1], yh);
      }
    } else {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 16; ++s) yh = mfma32(cl.Ra[t][s], Lu[t][s], yh);
    }
    f16v wa, wb;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float yv = ym.y[v >> 2][v & 3];
      // ragged tiles pad out-of-range entries with -inf as well: they count as
      // missing whether or not the caller passed a mask
      const bool obs = (FULL && !masked) || observed(yv);
      // a missing entry (negative) becomes 0: a(0, yhat) = 0 for alpha > 0
      const float y = (masked || !FULL) ? __builtin_amdgcn_fmed3f(yv, 0.f, FLT_MAX) : yv;
      const float yhat = needs_floor<WK>() ? __builtin_amdgcn_fmed3f(yh[v], FLT_MIN, FLT_MAX) : yh[v];
      if constexpr (ND) {
        float xa, xb;
        ab_weights<WK>(y, yhat, WK == WK_FAM ? a.fparam : a.alpha, WK == WK_FAM ? (float)a.lk : a.beta,
                       xa, xb);
        wa[v] = (a_zero_at_zero<WK>() || obs) ? xa : 0.f;
        wb[v] = obs ? xb : 0.f;
      }
      if constexpr (LOSS) {
        const bool val = vmode && validation(yv);
        const float l = ab_loss<WK>(obs ? y : (val ? -yv : 1.f), (obs || val) ? yhat : 1.f, a);
        lsum += obs ? (double)l : 0.0;
        vsum += val ? (double)l : 0.0;
      }
    }
    if constexpr (ND) {
      // N^T[k][p] += sum_q (u[k] C[q][k]) W^T[q][p], one accumulator tile per kappa tile
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        float rb[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) rb[v] = cl.Rb[t][v] * ul[t];
        if constexpr (PREC == 0) {
#pragma unroll
          for (int v = 0; v < 16; ++v) accN[t] = mfma32(rb[v], wa[v], accN[t]);
          if (!a.no_d) {
#pragma unroll
            for (int v = 0; v < 16; ++v) accD[t] = mfma32(rb[v], wb[v], accD[t]);
          }
        } else {
          float wav[16], wbv[16];
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            wav[v] = wa[v];
            wbv[v] = wb[v];
          }
          const auto r0 = cvt8<LP>(rb), r1 = cvt8<LP>(rb + 8);
          accN[t] = mfma8<LP>(r0, cvt8<LP>(wav), accN[t]);
          accN[t] = mfma8<LP>(r1, cvt8<LP>(wav + 8), accN[t]);
          if (!a.no_d) {
            accD[t] = mfma8<LP>(r0, cvt8<LP>(wbv), accD[t]);
            accD[t] = mfma8<LP>(r1, cvt8<LP>(wbv + 8), accD[t]);
          }
        }
      }
    }
  };

  // ---- software pipeline: column side and data one step ahead (two-stage rings);
  // per-qo bases are refreshed only when the load iterator enters a new qo
  const int64_t nst = s_end > s_beg ? s_end - s_beg : 0;
  int q0 = 0, qis0 = 0;
  if (nst > 0) {
    q0 = (int)(s_beg / a.nqis);
    qis0 = (int)(s_beg - (int64_t)q0 * a.nqis);
  }
  int lq = q0, lqi = qis0;  // next step to load
  int kq = q0, kqi = qis0;  // next step to compute
  uint32_t ybase = 0, ibase = 0;
  auto set_bases = [&](int qo) {
    ybase = a.qo_yoff[qo];
    ibase = a.in_base ? a.in_base[qo] : 0u;
  };
  auto adv_load = [&]() {
    if (++lqi == a.nqis) {
      lqi = 0;
      ++lq;
      set_bases(lq);
    }
  };
  if (nst > 0) {
    if constexpr (!FULL) load_L();  // full tiles read their rows in set_u
    set_bases(q0);
  }
  int comp_qo = -1;  // qo whose Lu, ul are formed
  if constexpr (FULL) {
   if (nst > 0) {
    // Y: direct-to-LDS ring, kStages - 1 steps ahead; column side: registers,
    // one step ahead.  Issue order per step: Y DMA (nY ops), then column loads
    // (nC ops).  Before reading stage j at least kWait ops issued after its DMA
    // exist in every non-tail step, so vmcnt <= kWait implies it landed.
    constexpr int nY = VECQ ? 4 : 16, nC = NT * (4 + 16);
    constexpr int kMin = (kStages - 1) * nY + 2 * nC < nC + (kStages - 1) * (nY + nC)
                             ? (kStages - 1) * nY + 2 * nC
                             : nC + (kStages - 1) * (nY + nC);
    constexpr int kWait = kMin < 63 ? kMin : 63;  // vmcnt holds 6 bits; smaller is safe
    constexpr int kWaitImm = (kWait & 15) | ((kWait >> 4) << 14) | (7 << 4) | (15 << 8);
    constexpr int kWait0 = (7 << 4) | (15 << 8);  // vmcnt(0)
    (void)kWait0;
    int dq = lq, dqi = lqi;  // next Y step to move (lq, lqi: next column step)
    uint32_t dybase = ybase;
    auto adv_dma = [&]() {
      if (++dqi == a.nqis) {
        dqi = 0;
        ++dq;
        dybase = a.qo_yoff[dq];
      }
    };
    // Every path issues the same loads: past the end of the range the
    // iterators stay on the last step and re-issue it (an L2 hit).  Equal
    // counts keep the waitcnt analysis exact at every join, so prefetches
    // stay in flight.
    Cols c0, c1;
    for (int j = 0; j < kStages - 1; ++j) {
      dma_ym(dybase, 32 * dqi, j);
      if (j + 1 < nst) adv_dma();
    }
    __builtin_amdgcn_sched_barrier(0);
    load_cols(ibase, 32 * lqi, c0);
    if (nst > 1) adv_load();
    set_u(q0);
    comp_qo = q0;
    auto stepf = [&](int64_t i, const Cols& cc, Cols& pc) {
      dma_ym(dybase, 32 * dqi, (int)((i + kStages - 1) % kStages));
      if (i + kStages < nst) adv_dma();
      __builtin_amdgcn_sched_barrier(0);  // keep the issue order: Y DMA, then column loads
      load_cols(ibase, 32 * lqi, pc);
      if (i + 2 < nst) adv_load();
      if (kq != comp_qo) {
        if (nout > 0) set_u(kq);
        comp_qo = kq;
      }
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_waitcnt(kWaitImm);
      __builtin_amdgcn_sched_barrier(0);
      YM cy;
      read_ym((int)(i % kStages), cy);
      compute(cy, cc);
      if (++kqi == a.nqis) {
        kqi = 0;
        ++kq;
      }
    };
    for (int64_t i = 0; i < nst; i += 2) {
      stepf(i, c0, c1);
      if (i + 1 < nst) stepf(i + 1, c1, c0);
    }
    __builtin_amdgcn_s_waitcnt(kWait0);  // retire the trailing re-issued loads
   }
    __syncthreads();  // the ring memory is reused for the partial reduction
  } else {
    // Outer-factor rows of a step are moved with the step's column and data
    // loads, one step ahead; a step starts by waiting for everything issued
    // so far (its own operands, which it needs anyway), then forms Lu, ul if
    // it starts a new qo.
    YM y0, y1;
    Cols c0, c1;
    int u_last = -1;  // qo whose rows were moved last
    if (nst > 0) {
      load_cols(ibase, 32 * lqi, c0);
      load_ym(ybase, 32 * lqi, y0);
      dma_u(lq);
      u_last = lq;
      if (nst > 1) adv_load();
    }
    constexpr int kWait0 = (7 << 4) | (15 << 8);  // vmcnt(0)
    auto step = [&](int64_t i, const YM& cy, YM& py, const Cols& cc, Cols& pc) {
      __builtin_amdgcn_s_waitcnt(kWait0);
      if (kq != comp_qo) {
        set_u(kq);
        comp_qo = kq;
      }
      if (i + 1 < nst) {
        load_cols(ibase, 32 * lqi, pc);
        load_ym(ybase, 32 * lqi, py);
        if (lq != u_last) {
          dma_u(lq);
          u_last = lq;
        }
        if (i + 2 < nst) adv_load();
      }
      compute(cy, cc);
      if (++kqi == a.nqis) {
        kqi = 0;
        ++kq;
      }
    };
    for (int64_t i = 0; i < nst; i += 2) {
      step(i, y0, y1, c0, c1);
      if (i + 1 < nst) step(i + 1, y1, y0, c1, c0);
    }
  }

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
    // accumulator register v of tile t holds X^T[k = 32t + 8(v/4) + 4g + v%4][p = p0 + c];
    // waves 1..3 stash theirs, wave 0 adds them in a fixed order and stores the partial
    auto store = [&](const f16v (&acc)[NT], float* dst) {
      if (wrows) {  // each wave owns its rows
        if (p < a.nP) {
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int bq = 0; bq < 4; ++bq)
              *reinterpret_cast<f4*>(&dst[((size_t)chunk * a.nP + p) * KP + 32 * t + 8 * bq + 4 * g]) =
                  f4{acc[t][4 * bq], acc[t][4 * bq + 1], acc[t][4 * bq + 2], acc[t][4 * bq + 3]};
        }
        return;
      }
      if (wave > 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int bq = 0; bq < 4; ++bq)
            *reinterpret_cast<f4*>(&red[(wave - 1) * ROWS * RST + c * RST + 32 * t + 8 * bq + 4 * g]) =
                f4{acc[t][4 * bq], acc[t][4 * bq + 1], acc[t][4 * bq + 2], acc[t][4 * bq + 3]};
      }
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int bq = 0; bq < 4; ++bq) {
            f4 v = f4{acc[t][4 * bq], acc[t][4 * bq + 1], acc[t][4 * bq + 2], acc[t][4 * bq + 3]};
#pragma unroll
            for (int w = 0; w < 3; ++w)
              v += *reinterpret_cast<const f4*>(&red[w * ROWS * RST + c * RST + 32 * t + 8 * bq + 4 * g]);
            if (p < a.nP)
              *reinterpret_cast<f4*>(&dst[((size_t)chunk * a.nP + p) * KP + 32 * t + 8 * bq + 4 * g]) = v;
          }
      }
      __syncthreads();
    };
    store(accN, a.partN);
    if (!a.no_d) store(accD, a.partD);
  }
}

// Width 32 runs two waves per SIMD; width 64 holds twice the accumulators and
// column operands and runs one (its registers then include the accumulation
// registers, so nothing spills).
template <int NT, int WK, bool VECQ, int MODE, bool FULL, int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT == 1 ? 2 : 1, NT == 1 ? 2 : 1))) void
fused_x32(FusedArgs a) {
  fused_x32_body<NT, WK, VECQ, MODE, FULL, PREC>(a, blockIdx.x, blockIdx.x);
}

// Persistent form over many problems: work item w = (problem, workgroup index
// in that problem's grid); each workgroup walks the items w = blockIdx.x,
// blockIdx.x + gridDim.x, ...
template <int NT, int WK, bool VECQ, int MODE, bool FULL, int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT == 1 ? 2 : 1, NT == 1 ? 2 : 1))) void
fused_x32_batched(const FusedArgs* __restrict__ args, const WorkItem* __restrict__ work, int n_work) {
  for (int w = blockIdx.x; w < n_work; w += gridDim.x) {
    const WorkItem it = work[w];
    const FusedArgs a = args[it.run];
    fused_x32_body<NT, WK, VECQ, MODE, FULL, PREC>(a, it.blk, it.blk);
    __syncthreads();
  }
}

#ifndef NNEF_BATCHED_TU
template <int NT, int WK, bool VECQ, int MODE, int PREC>
int launch_x32_p(const FusedArgs& a, hipStream_t s) {
  if (a.full)
    NNEF_LAUNCH_PASS((fused_x32<NT, WK, VECQ, MODE, true, PREC>), dim3(a.n_wg), dim3(256), s, a);
  else
    NNEF_LAUNCH_PASS((fused_x32<NT, WK, VECQ, MODE, false, PREC>), dim3(a.n_wg), dim3(256), s, a);
  return (int)hipGetLastError();
}

// PREC != 0 is instantiated for the passes with contractions only (modes 0,
// 1); with a reduced-precision reconstruction (PREC > 2) the pass that also
// computes the loss keeps it FP32 (PREC - 2)
template <int NT, int WK, bool VECQ, int PREC>
int launch_x32_m(const FusedArgs& a, int mode, hipStream_t s) {
  if constexpr (PREC != 0) {
    constexpr int P1 = PREC > 2 ? PREC - 2 : PREC;
    return mode == 0 ? launch_x32_p<NT, WK, VECQ, 0, PREC>(a, s) : launch_x32_p<NT, WK, VECQ, 1, P1>(a, s);
  } else {
    switch (mode) {
      case 0: return launch_x32_p<NT, WK, VECQ, 0, 0>(a, s);
      case 1: return launch_x32_p<NT, WK, VECQ, 1, 0>(a, s);
      default: return launch_x32_p<NT, WK, VECQ, 2, 0>(a, s);
    }
  }
}

template <int NT, int WK, int PREC>
int launch_x32_v(const FusedArgs& a, bool vecq, int mode, hipStream_t s) {
  return vecq ? launch_x32_m<NT, WK, true, PREC>(a, mode, s) : launch_x32_m<NT, WK, false, PREC>(a, mode, s);
}

// One contraction width and input precision: the weight kind, data layout and
// mode are dispatched at run time.
template <int NT, int PREC>
int launch_x32(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  switch (wk) {
    case WK_KL: return launch_x32_v<NT, WK_KL, PREC>(a, vecq, mode, s);
    case WK_EUC: return launch_x32_v<NT, WK_EUC, PREC>(a, vecq, mode, s);
    case WK_SQRT: return launch_x32_v<NT, WK_SQRT, PREC>(a, vecq, mode, s);
    case WK_IS: return launch_x32_v<NT, WK_IS, PREC>(a, vecq, mode, s);
    case WK_GEN: return launch_x32_v<NT, WK_GEN, PREC>(a, vecq, mode, s);
    case WK_RKL: return launch_x32_v<NT, WK_RKL, PREC>(a, vecq, mode, s);
    default: return launch_x32_v<NT, WK_FAM, PREC>(a, vecq, mode, s);
  }
}

#else
template <int NT, int WK, bool VECQ, int MODE, int PREC>
int launch_x32_batched_p(const BatchedLaunch& L, hipStream_t s) {
  if (L.full)
    hipLaunchKernelGGL((fused_x32_batched<NT, WK, VECQ, MODE, true, PREC>), dim3(L.grid), dim3(256), 0, s,
                       L.args, L.work, L.n_work);
  else
    hipLaunchKernelGGL((fused_x32_batched<NT, WK, VECQ, MODE, false, PREC>), dim3(L.grid), dim3(256), 0,
                       s, L.args, L.work, L.n_work);
  return (int)hipGetLastError();
}

template <int NT, int WK, bool VECQ, int MODE>
int launch_x32_batched_m(const BatchedLaunch& L, hipStream_t s) {
  if constexpr (NT == 1) {
    if (L.prec == 1) return launch_x32_batched_p<NT, WK, VECQ, MODE, 1>(L, s);
    if (L.prec == 2) return launch_x32_batched_p<NT, WK, VECQ, MODE, 2>(L, s);
  }
  return launch_x32_batched_p<NT, WK, VECQ, MODE, 0>(L, s);
}

template <int NT, int WK>
int launch_x32_batched_w(const BatchedLaunch& L, hipStream_t s) {
  if (L.vecq)
    return L.mode ? launch_x32_batched_m<NT, WK, true, 1>(L, s) : launch_x32_batched_m<NT, WK, true, 0>(L, s);
  return L.mode ? launch_x32_batched_m<NT, WK, false, 1>(L, s) : launch_x32_batched_m<NT, WK, false, 0>(L, s);
}

// Batched passes: width 32 (NT = 1) in every input precision, width 64 in FP32.
template <int NT>
int launch_x32_batched(const BatchedLaunch& L, hipStream_t s) {
  switch (L.wk) {
    case WK_KL: return launch_x32_batched_w<NT, WK_KL>(L, s);
    case WK_EUC: return launch_x32_batched_w<NT, WK_EUC>(L, s);
    case WK_SQRT: return launch_x32_batched_w<NT, WK_SQRT>(L, s);
    case WK_IS: return launch_x32_batched_w<NT, WK_IS>(L, s);
    case WK_GEN: return launch_x32_batched_w<NT, WK_GEN>(L, s);
    case WK_RKL: return launch_x32_batched_w<NT, WK_RKL>(L, s);
    default: return launch_x32_batched_w<NT, WK_FAM>(L, s);
  }
}

#endif
}  // namespace
}  // namespace nnef
