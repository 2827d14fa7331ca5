// Direct pass of libnnef for gfx950: one block update's pass over Y for model
// strings that have no bilinear split with a contraction width of at most 64
// (the many-body models of Sec. 2, whose operands pair every observed mode
// with every other, and CP-like strings of rank above 64).
//
// For every observed entry (p, q) the reconstruction is the explicit sum of
// eq. 2.1 over latent combinations, in registers (Yhat is never stored):
//   c[r] = sum_s prod_j op_j[entry, r, s],   yhat = sum_r theta[p, r] c[r],
// then the masked weights of App. B, and the numerator and denominator of
// eq. 3.6 for operand l accumulate per thread as Wa c[r] and Wb c[r] (the
// entry's row p is fixed for a thread, so no atomics).  The work is FP32
// vector arithmetic: at most sixteen latent combinations per thread, G
// threads per entry combined with a butterfly (every lane ends with the same
// sum), 256 threads covering rows_per_wg rows x qlanes column lanes.  The
// column lanes of a row are summed in lane order into the partial of the
// workgroup's column chunk, the layout the update kernel reduces.
#include "fused_impl.hpp"

namespace nnef {
namespace {

template <int WK, int MODE, int KPT>
__global__ __launch_bounds__(256) void direct_pass(DirectArgs a) {
  constexpr bool LOSS = MODE >= 1, ND = MODE <= 1;
  __shared__ uint32_t slat[kDirectMaxLat];
  __shared__ float red[ND ? 256 * KPT : 1];
  __shared__ double lred[8];
  const int tid = threadIdx.x;
  const int G = a.G;
  const int gi = tid & (G - 1), eg = tid / G;
  const int rl = eg % a.rows_per_wg, ql = eg / a.rows_per_wg;
  const int panel = blockIdx.x % a.n_panels, chunk = blockIdx.x / a.n_panels;
  const int p = panel * a.rows_per_wg + rl;
  const bool pval = p < a.nP;
  const int K = a.K, KS = a.KS, nlat = a.K * a.KS, nops = a.n_ops;

  for (int j = 0; j < nops; ++j)
    for (int i = tid; i < nlat; i += 256) slat[j * nlat + i] = a.oplat[j][i];
  __syncthreads();

  FusedArgs fa;
  fa.alpha = a.alpha;
  fa.beta = a.beta;
  fa.ab_inv = a.ab_inv;
  fa.apb_inv = a.apb_inv;
  fa.lk = a.lk;
  fa.fparam = a.fparam;

  float th[KPT], accN[KPT], accD[KPT];
  const uint32_t yrow = pval ? a.yp[p] : 0u;
  const uint32_t trow = pval ? a.thp[p] : 0u;
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    const int r = gi + G * i;
    th[i] = (pval && r < K) ? ldf(a.theta, trow + a.thr[r]) : 0.f;
    accN[i] = 0.f;
    accD[i] = 0.f;
  }
  uint32_t pb[kMaxDirectOps];
#pragma unroll
  for (int j = 0; j < kMaxDirectOps; ++j) pb[j] = (j < nops && pval) ? a.opp[j][p] : 0u;

  double lsum = 0.0, vsum = 0.0;
  const bool vmode = LOSS && a.vloss_part != nullptr;
  const int q0 = chunk * a.q_per_chunk;
  const int q1 = min(a.nQ, q0 + a.q_per_chunk);
  for (int q = q0 + ql; q < q1; q += a.qlanes) {
    const float yv = pval ? ldf(a.Y, yrow + a.yq[q]) : -INFINITY;
    // rows past the end and (with a mask) missing entries are negative
    const bool obs = (!a.masked && pval) || observed(yv);
    uint32_t qb[kMaxDirectOps];
#pragma unroll
    for (int j = 0; j < kMaxDirectOps; ++j) qb[j] = j < nops ? pb[j] + a.opq[j][q] : 0u;
    float c[KPT];
    float part = 0.f;
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int r = gi + G * i;
      float cs = 0.f;
      if (r < K) {
        for (int s = 0; s < KS; ++s) {
          const int li = r * KS + s;
          float prod = 1.f;
#pragma unroll
          for (int j = 0; j < kMaxDirectOps; ++j)
            if (j < nops) prod *= ldf(a.op[j], qb[j] + slat[j * nlat + li]);
          cs += prod;
        }
      }
      c[i] = cs;
      part = fmaf(th[i], cs, part);
    }
    for (int o = 1; o < G; o <<= 1) part += __shfl_xor(part, o, 64);
    const float y = (a.masked || !pval) ? __builtin_amdgcn_fmed3f(yv, 0.f, FLT_MAX) : yv;
    const float yhat = needs_floor<WK>() ? __builtin_amdgcn_fmed3f(part, FLT_MIN, FLT_MAX) : part;
    if constexpr (ND) {
      float xa, xb;
      ab_weights<WK>(y, yhat, WK == WK_FAM ? a.fparam : a.alpha, WK == WK_FAM ? (float)a.lk : a.beta, xa, xb);
      const float wa = (a_zero_at_zero<WK>() || obs) ? xa : 0.f;
      const float wb = obs ? xb : 0.f;
#pragma unroll
      for (int i = 0; i < KPT; ++i) {
        accN[i] = fmaf(wa, c[i], accN[i]);
        accD[i] = fmaf(wb, c[i], accD[i]);
      }
    }
    if constexpr (LOSS) {
      const bool val = vmode && validation(yv);
      if (gi == 0 && (obs || val)) {
        const double l = (double)ab_loss<WK>(obs ? y : -yv, yhat, fa);
        if (obs) lsum += l;
        else vsum += l;
      }
    }
  }

  if constexpr (LOSS) {
    const double w = wave_sum(lsum);
    if ((tid & 63) == 0) lred[tid >> 6] = w;
    if (vmode) {
      const double wv = wave_sum(vsum);
      if ((tid & 63) == 0) lred[4 + (tid >> 6)] = wv;
    }
    __syncthreads();
    if (tid == 0) {
      a.loss_part[blockIdx.x] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
      if (vmode) a.vloss_part[blockIdx.x] = ((lred[4] + lred[5]) + lred[6]) + lred[7];
    }
  }
  if constexpr (ND) {
    // thread tid = ((ql * rows_per_wg + rl) * G + gi) holds r = gi + G i of its
    // row.  The column lanes of a row that share a wave are summed first by a
    // butterfly over the lane bits at and above span = rows_per_wg * G (all of
    // them end with the same sum); the lanes below span then hold one value per
    // group of 64 / span column lanes, and every output (row, r) sums those
    // groups in lane order.
    const int nout = a.rows_per_wg * K;
    const int span = a.rows_per_wg * G;
    const int grp = span < 64 ? 64 / span : 1;
    auto reduce = [&](float (&acc)[KPT], float* dst) {
      for (int o = span; o < 64; o <<= 1) {
#pragma unroll
        for (int i = 0; i < KPT; ++i) acc[i] += __shfl_xor(acc[i], o, 64);
      }
#pragma unroll
      for (int i = 0; i < KPT; ++i) red[tid * KPT + i] = acc[i];
      __syncthreads();
      for (int o = tid; o < nout; o += 256) {
        const int rr = o / K, r = o - rr * K;
        const int g2 = r & (G - 1), i2 = r / G;
        float v = 0.f;
        for (int l = 0; l < a.qlanes; l += grp) v += red[((l * a.rows_per_wg + rr) * G + g2) * KPT + i2];
        const int pp = panel * a.rows_per_wg + rr;
        if (pp < a.nP) dst[((size_t)chunk * a.nP + pp) * K + r] = v;
      }
      __syncthreads();
    };
    reduce(accN, a.partN);
    reduce(accD, a.partD);
  }
}

template <int WK, int MODE>
int launch_direct_m(const DirectArgs& a, hipStream_t s) {
  const int grid = a.n_panels * a.n_chunks;
  if (a.K == 1)
    NNEF_LAUNCH_PASS((direct_pass<WK, MODE, 1>), dim3(grid), dim3(256), s, a);
  else
    NNEF_LAUNCH_PASS((direct_pass<WK, MODE, kDirectKPT>), dim3(grid), dim3(256), s, a);
  return (int)hipGetLastError();
}

template <int WK>
int launch_direct_w(const DirectArgs& a, int mode, hipStream_t s) {
  switch (mode) {
    case 0: return launch_direct_m<WK, 0>(a, s);
    case 1: return launch_direct_m<WK, 1>(a, s);
    default: return launch_direct_m<WK, 2>(a, s);
  }
}

}  // namespace

int launch_direct(const DirectArgs& a, int wk, int mode, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (wk) {
    case WK_KL: return launch_direct_w<WK_KL>(a, mode, s);
    case WK_EUC: return launch_direct_w<WK_EUC>(a, mode, s);
    case WK_SQRT: return launch_direct_w<WK_SQRT>(a, mode, s);
    case WK_IS: return launch_direct_w<WK_IS>(a, mode, s);
    case WK_GEN: return launch_direct_w<WK_GEN>(a, mode, s);
    case WK_RKL: return launch_direct_w<WK_RKL>(a, mode, s);
    default: return launch_direct_w<WK_FAM>(a, mode, s);
  }
}

}  // namespace nnef
