// Device kernels of libnnef for gfx950 (CDNA4), apart from the fused pass
// (fused_impl.hpp):
// update  - fixed-order reduction of the fused pass partials, then the update
//           Theta <- max(eps, Theta * g^{-1}(N/D)) (eq. 3.4);
// einsum  - generic small contraction for side operands and chain-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstdint>
#include <cmath>

#include "nnef_internal.hpp"

namespace nnef {

thread_local PassEvents g_pass_events;

int launch_fused_kp16(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_kp32(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_kp64(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_batched_kp16(const BatchedLaunch& L, hipStream_t s);
int launch_fused_batched_kp32(const BatchedLaunch& L, hipStream_t s);
int launch_fused_batched_kp64(const BatchedLaunch& L, hipStream_t s);

namespace {
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
}  // namespace

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

__device__ __forceinline__ void colsum_body(const UpdateArgs& a, float* dcol) {
  // dcol[k] = prod_m sum_rows piece_m[row][k]; one workgroup, K <= 64.  With
  // KQ = K rounded up to a power of two, thread t takes column t % KQ and the
  // rows t / KQ + j * (256 / KQ), four loads in flight; the row lanes of a
  // column are then added in a fixed tree in LDS (deterministic).
  __shared__ double part[256];
  const int t = threadIdx.x;
  int kq = 1;
  while (kq < a.K) kq <<= 1;
  const int k = t & (kq - 1), r0 = t / kq, rstep = 256 / kq;
  double prod = 1.0;
  for (int m = 0; m < a.npieces; ++m) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (k < a.K) {
      const float* col = a.piece[m] + k;
      const int64_t ld = a.ldpiece[m], n = a.nrows[m];
      int64_t row = r0;
      for (; row + 3 * rstep < n; row += 4 * rstep) {
        s0 += col[row * ld];
        s1 += col[(row + rstep) * ld];
        s2 += col[(row + 2 * rstep) * ld];
        s3 += col[(row + 3 * rstep) * ld];
      }
      for (; row < n; row += rstep) s0 += col[row * ld];
    }
    part[t] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int h = rstep / 2; h > 0; h >>= 1) {
      if (r0 < h) part[t] += part[t + h * kq];
      __syncthreads();
    }
    if (t < kq) prod *= part[t];
    __syncthreads();
  }
  if (t < a.K) dcol[t] = (float)prod;
}

__global__ __launch_bounds__(256) void colsum_kernel(UpdateArgs a, float* dcol) { colsum_body(a, dcol); }

// One workgroup of NW waves per 64 consecutive (p, k) outputs.  Wave w sums
// the partial slots w, w + NW, w + 2 NW, ... with U independent running sums
// (U loads in flight per lane for each of N and D), then wave 0 adds the waves'
// sums in wave order (deterministic) and applies the update.
template <int NW, int U>
__device__ __forceinline__ void update_body(const UpdateArgs& a, const float* dcol, int blk) {
  __shared__ double sN[NW][64], sD[NW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = (int64_t)a.nP * a.K;
  const int64_t idx = (int64_t)blk * 64 + lane;
  const bool valid = idx < n;
  const int p = valid ? (int)(idx / a.K) : 0, k = valid ? (int)(idx % a.K) : 0;
  double N = 0.0, D = 0.0;
  if (valid) {
    const size_t stride = (size_t)a.nP * a.KP;
    const float* pn = a.partN + (size_t)p * a.KP + k;
    const float* pd = a.partD + (size_t)p * a.KP + k;
    double sn[U], sd[U];
#pragma unroll
    for (int j = 0; j < U; ++j) sn[j] = sd[j] = 0.0;
    int ch = w;
    for (; ch + (U - 1) * NW < a.n_chunks; ch += U * NW) {
#pragma unroll
      for (int j = 0; j < U; ++j) sn[j] += pn[(size_t)(ch + NW * j) * stride];
      if (!a.no_d) {
#pragma unroll
        for (int j = 0; j < U; ++j) sd[j] += pd[(size_t)(ch + NW * j) * stride];
      }
    }
    for (; ch < a.n_chunks; ch += NW) {
      sn[0] += pn[(size_t)ch * stride];
      if (!a.no_d) sd[0] += pd[(size_t)ch * stride];
    }
    // pairwise in a fixed pattern
#pragma unroll
    for (int h = U / 2; h > 0; h /= 2)
#pragma unroll
      for (int j = 0; j < h; ++j) {
        sn[j] += sn[j + h];
        sd[j] += sd[j + h];
      }
    N = sn[0];
    D = sd[0];
  }
  sN[w][lane] = N;
  sD[w][lane] = D;
  __syncthreads();
  if (w == 0 && valid) {
    N = 0.0;
    D = 0.0;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      N += sN[j][lane];
      D += sD[j][lane];
    }
    if (a.no_d) D = (double)dcol[k];
    if (a.theta) {
      float* th = a.theta + (size_t)p * a.ldT + k;
      *th = mu_rule(*th, (float)N, (float)D, a.upd, a.gamma, a.eps);
    } else {
      a.NL[idx] = (float)N;
      a.DL[idx] = (float)D;
    }
  }
  if (a.loss_out && blk == 0 && w == (NW > 1 ? 1 : 0)) {
    double sl = 0.0;
    for (int i = lane; i < a.n_loss_part; i += 64) sl += a.loss_part[i];
    sl = wave_sum(sl);
    if (lane == 0) *a.loss_out = sl;
    if (a.vloss_out) {
      double sv = 0.0;
      for (int i = lane; i < a.n_loss_part; i += 64) sv += a.vloss_part[i];
      sv = wave_sum(sv);
      if (lane == 0) *a.vloss_out = sv;
    }
  }
}

// Single plans: the waves per workgroup follow the number of partial slots,
// so that every lane's loads are in flight at once (sixteen waves at the usual
// 64 slots) and blocks with few slots (many rows) do not idle waves.  With
// the closed-form D and no dcol given, each 256-thread workgroup forms the
// column sums itself in LDS (small outer pieces: one launch fewer).
template <int NW, int U>
__global__ __launch_bounds__(64 * NW) void update_kernel(UpdateArgs a, const float* dcol) {
  if constexpr (NW == 4) {
    __shared__ float dloc[64];
    if (a.no_d && dcol == nullptr) {
      colsum_body(a, dloc);
      __syncthreads();
      dcol = dloc;
    }
  }
  update_body<NW, U>(a, dcol, blockIdx.x);
}

// Few partial slots (blocks with many rows): one output per thread, the slots
// summed in slot order; the first workgroup's first wave also finishes the
// loss.
__global__ __launch_bounds__(256) void update_flat_kernel(UpdateArgs a, const float* dcol) {
  __shared__ float dloc[64];
  if (a.no_d && dcol == nullptr) {
    colsum_body(a, dloc);
    __syncthreads();
    dcol = dloc;
  }
  const int64_t n = (int64_t)a.nP * a.K;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx < n) {
    const int p = (int)(idx / a.K), k = (int)(idx % a.K);
    const size_t stride = (size_t)a.nP * a.KP;
    const size_t o = (size_t)p * a.KP + k;
    double N = 0.0, D = 0.0;
    for (int ch = 0; ch < a.n_chunks; ++ch) {
      N += a.partN[(size_t)ch * stride + o];
      if (!a.no_d) D += a.partD[(size_t)ch * stride + o];
    }
    if (a.no_d) D = (double)dcol[k];
    if (a.theta) {
      float* th = a.theta + (size_t)p * a.ldT + k;
      *th = mu_rule(*th, (float)N, (float)D, a.upd, a.gamma, a.eps);
    } else {
      a.NL[idx] = (float)N;
      a.DL[idx] = (float)D;
    }
  }
  if (a.loss_out && blockIdx.x == 0 && threadIdx.x < 64) {
    double sl = 0.0;
    for (int i = (int)threadIdx.x; i < a.n_loss_part; i += 64) sl += a.loss_part[i];
    sl = wave_sum(sl);
    if (threadIdx.x == 0) *a.loss_out = sl;
    if (a.vloss_out) {
      double sv = 0.0;
      for (int i = (int)threadIdx.x; i < a.n_loss_part; i += 64) sv += a.vloss_part[i];
      sv = wave_sum(sv);
      if (threadIdx.x == 0) *a.vloss_out = sv;
    }
  }
}

__global__ __launch_bounds__(256) void colsum_batched(const UpdateArgs* __restrict__ args,
                                                      const int* __restrict__ runs) {
  const UpdateArgs a = args[runs[blockIdx.x]];
  colsum_body(a, a.dcol);
}

__global__ __launch_bounds__(256) void update_batched(const UpdateArgs* __restrict__ args,
                                                      const WorkItem* __restrict__ work, int n_work) {
  for (int w = blockIdx.x; w < n_work; w += gridDim.x) {
    const WorkItem it = work[w];
    const UpdateArgs a = args[it.run];
    update_body<4, 8>(a, a.dcol, it.blk);
    __syncthreads();
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

// Operand and output pointers of a second contraction with the same shapes
// (the denominator chain beside the numerator's): workgroups with
// blockIdx.y = 1 take these.
struct EinsumPtrs {
  const float* in[kMaxEinsumIn];
  float* out;
};

// One thread per output; NIN inputs (loops over inputs unrolled, offsets in
// registers).  With no summed letter the output is a plain product.
template <int NIN>
__global__ __launch_bounds__(256) void einsum_kernel(EinsumArgs a, EinsumPtrs b) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= a.n_out_total) return;
  const bool second = blockIdx.y != 0;
  const float* src[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) src[i] = second ? b.in[i] : a.in[i];
  float* const dst = second ? b.out : a.out;
  int64_t off[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) off[i] = 0;
  int64_t ooff = 0;
  if (a.n_out_total <= (int64_t)UINT32_MAX) {  // 32-bit division where it suffices
    uint32_t rem = (uint32_t)o;
    for (int d = a.n_out - 1; d >= 0; --d) {
      const uint32_t sz = (uint32_t)a.out_size[d];
      const int64_t v = (int64_t)(rem % sz);
      rem /= sz;
      ooff += v * a.out_stride[d];
#pragma unroll
      for (int i = 0; i < NIN; ++i) off[i] += v * a.in_out_stride[i][d];
    }
  } else {
    int64_t rem = o;
    for (int d = a.n_out - 1; d >= 0; --d) {
      const int64_t v = rem % a.out_size[d];
      rem /= a.out_size[d];
      ooff += v * a.out_stride[d];
#pragma unroll
      for (int i = 0; i < NIN; ++i) off[i] += v * a.in_out_stride[i][d];
    }
  }
  if (a.n_sum == 0) {
    float prod = 1.f;
#pragma unroll
    for (int i = 0; i < NIN; ++i) prod *= src[i][off[i]];
    dst[ooff] = prod;
    return;
  }
  int64_t n_sum = 1;
  for (int d = 0; d < a.n_sum; ++d) n_sum *= a.sum_size[d];
  int64_t cnt[kMaxEinsumLetters] = {0};
  double acc = 0.0;
  for (int64_t cidx = 0; cidx < n_sum; ++cidx) {
    float prod = 1.f;
#pragma unroll
    for (int i = 0; i < NIN; ++i) prod *= src[i][off[i]];
    acc += (double)prod;
    for (int d = a.n_sum - 1; d >= 0; --d) {
      ++cnt[d];
#pragma unroll
      for (int i = 0; i < NIN; ++i) off[i] += a.in_sum_stride[i][d];
      if (cnt[d] < a.sum_size[d]) break;
#pragma unroll
      for (int i = 0; i < NIN; ++i) off[i] -= a.sum_size[d] * a.in_sum_stride[i][d];
      cnt[d] = 0;
    }
  }
  dst[ooff] = (float)acc;
}

// The same contraction with G lanes per output (G a power of two <= 64): lane
// g of an output's group sums the flattened summed indices c = g, g + G, ...,
// four at a time so that several loads are in flight, and the group adds its
// lanes' sums with a fixed butterfly (deterministic).  Used when there are
// few outputs with long sums, where one thread per output leaves the chip
// idle and every thread waits on one load per term.
template <int NIN, bool ONE_SUM>
__global__ __launch_bounds__(256) void einsum_split_kernel(EinsumArgs a, EinsumPtrs b, int log2g,
                                                           uint32_t n_sum) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool second = blockIdx.y != 0;
  const float* src[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) src[i] = second ? b.in[i] : a.in[i];
  float* const dst = second ? b.out : a.out;
  const int G = 1 << log2g;
  const int64_t o = t >> log2g;
  const uint32_t g = (uint32_t)(t & (G - 1));
  const bool valid = o < a.n_out_total;
  int64_t off[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) off[i] = 0;
  int64_t ooff = 0;
  if (valid) {
    if (a.n_out_total <= (int64_t)UINT32_MAX) {  // 32-bit division where it suffices
      uint32_t rem = (uint32_t)o;
      for (int d = a.n_out - 1; d >= 0; --d) {
        const uint32_t sz = (uint32_t)a.out_size[d];
        const int64_t v = (int64_t)(rem % sz);
        rem /= sz;
        ooff += v * a.out_stride[d];
#pragma unroll
        for (int i = 0; i < NIN; ++i) off[i] += v * a.in_out_stride[i][d];
      }
    } else {
      int64_t rem = o;
      for (int d = a.n_out - 1; d >= 0; --d) {
        const int64_t v = rem % a.out_size[d];
        rem /= a.out_size[d];
        ooff += v * a.out_stride[d];
#pragma unroll
        for (int i = 0; i < NIN; ++i) off[i] += v * a.in_out_stride[i][d];
      }
    }
  }
  double acc = 0.0;
  if constexpr (ONE_SUM) {
    // one summed letter: walk each input with a pointer step per term
    if (valid) {
      const float* ptr[NIN];
      int64_t step[NIN];
#pragma unroll
      for (int i = 0; i < NIN; ++i) {
        const int64_t st = a.in_sum_stride[i][0];
        ptr[i] = src[i] + off[i] + (int64_t)g * st;
        step[i] = (int64_t)G * st;
      }
      uint32_t c = g;
      for (; c + 3u * (uint32_t)G < n_sum; c += 4u * (uint32_t)G) {
        float pr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          pr[u] = 1.f;
#pragma unroll
          for (int i = 0; i < NIN; ++i) pr[u] *= ptr[i][u * step[i]];
        }
        acc += ((double)pr[0] + (double)pr[1]) + ((double)pr[2] + (double)pr[3]);
#pragma unroll
        for (int i = 0; i < NIN; ++i) ptr[i] += 4 * step[i];
      }
      for (; c < n_sum; c += (uint32_t)G) {
        float pr = 1.f;
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
          pr *= ptr[i][0];
          ptr[i] += step[i];
        }
        acc += (double)pr;
      }
    }
  } else if (valid && a.n_sum == 2) {
    // two summed letters, c = v0 * size1 + v1: the inner digit and the input
    // offsets advance by G per term with at most one carry into the outer
    // digit (G = g0 * size1 + g1, g1 < size1), so no division per term; the
    // terms, products and grouping of the sums are those of the general path
    const uint32_t s1 = (uint32_t)a.sum_size[1];
    const uint32_t g0 = (uint32_t)G / s1, g1 = (uint32_t)G % s1;
    uint32_t v1 = g % s1;
    const int64_t v0 = (int64_t)(g / s1);
    int64_t o[NIN], inc[NIN], wrap[NIN];
#pragma unroll
    for (int i = 0; i < NIN; ++i) {
      const int64_t st0 = a.in_sum_stride[i][0], st1 = a.in_sum_stride[i][1];
      o[i] = off[i] + v0 * st0 + (int64_t)v1 * st1;
      inc[i] = (int64_t)g0 * st0 + (int64_t)g1 * st1;
      wrap[i] = st0 - (int64_t)s1 * st1;
    }
    for (uint32_t c0 = g; c0 < n_sum; c0 += 4u * (uint32_t)G) {
      float prod[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool in_range = c0 + (uint32_t)u * (uint32_t)G < n_sum;
        float pr = 1.f;
#pragma unroll
        for (int i = 0; i < NIN; ++i) pr *= src[i][in_range ? o[i] : off[i]];
        prod[u] = in_range ? pr : 0.f;
        v1 += g1;
        const bool carry = v1 >= s1;
        v1 = carry ? v1 - s1 : v1;
#pragma unroll
        for (int i = 0; i < NIN; ++i) o[i] += inc[i] + (carry ? wrap[i] : 0);
      }
      acc += ((double)prod[0] + (double)prod[1]) + ((double)prod[2] + (double)prod[3]);
    }
  } else if (valid) {
    for (uint32_t c0 = g; c0 < n_sum; c0 += 4u * (uint32_t)G) {
      float prod[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t c = c0 + (uint32_t)u * (uint32_t)G;
        prod[u] = 0.f;
        if (c < n_sum) {
          int64_t so[NIN];
#pragma unroll
          for (int i = 0; i < NIN; ++i) so[i] = off[i];
          uint32_t rem = c;
          for (int d = a.n_sum - 1; d >= 0; --d) {
            const uint32_t sz = (uint32_t)a.sum_size[d];
            const uint32_t v = rem % sz;
            rem /= sz;
#pragma unroll
            for (int i = 0; i < NIN; ++i) so[i] += (int64_t)v * a.in_sum_stride[i][d];
          }
          float pr = 1.f;
#pragma unroll
          for (int i = 0; i < NIN; ++i) pr *= src[i][so[i]];
          prod[u] = pr;
        }
      }
      acc += ((double)prod[0] + (double)prod[1]) + ((double)prod[2] + (double)prod[3]);
    }
  }
  for (int m = G >> 1; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if (valid && g == 0) dst[ooff] = (float)acc;
}

// Missing entries become -1 (observed data are nonnegative); the value stored
// at a missing entry is never read into arithmetic, only replaced.
__device__ __forceinline__ float pack_one(float y, uint32_t m, uint32_t value, uint32_t vvalue) {
  return m == value ? y : (m == vvalue ? __builtin_copysignf(y, -1.f) : -INFINITY);
}

__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ Y,
                                                   const uint8_t* __restrict__ M,
                                                   float* __restrict__ Yp, int64_t n, uint32_t value,
                                                   uint32_t vvalue) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i + 3 < n) {
    const v4 y = *reinterpret_cast<const v4*>(Y + i);
    const uint32_t m = *reinterpret_cast<const uint32_t*>(M + i);
    v4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = pack_one(y[j], (m >> (8 * j)) & 0xffu, value, vvalue);
    *reinterpret_cast<v4*>(Yp + i) = o;
  } else {
    for (int64_t j = i; j < n; ++j) Yp[j] = pack_one(Y[j], M[j], value, vvalue);
  }
}

__global__ __launch_bounds__(256) void copy_f64_kernel(double* dst, const double* src, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void zero_kernel(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
int launch_fused(const FusedArgs& a, int KP, int wk, bool vecq, int mode, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (a.n_wg <= 0) return 0;
  switch (KP) {
    case 16: return launch_fused_kp16(a, wk, vecq, mode, s);
    case 32: return launch_fused_kp32(a, wk, vecq, mode, s);
    case 64: return launch_fused_kp64(a, wk, vecq, mode, s);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_fused_batched(const BatchedLaunch& L, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (L.n_work <= 0) return 0;
  switch (L.KP) {
    case 16: return launch_fused_batched_kp16(L, s);
    case 32: return launch_fused_batched_kp32(L, s);
    case 64: return launch_fused_batched_kp64(L, s);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_update(const UpdateArgs& a, float* dcol, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  // small outer pieces: the 256-thread update workgroups form the closed-form
  // D themselves (a null dcol tells them to), saving the column-sum launch
  int64_t piece_elems = 0;
  for (int m = 0; m < a.npieces; ++m) piece_elems += a.nrows[m] * a.K;
  const bool inline_d = a.no_d && a.n_chunks < 32 && piece_elems <= 65536;
  if (a.no_d && !inline_d) {
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, a, dcol);
  }
  const float* dc = inline_d ? nullptr : dcol;
  const int64_t n = (int64_t)a.nP * a.K;
  const int grid = (int)((n + 63) / 64);
  const dim3 g(grid > 0 ? grid : 1);
  if (a.n_chunks >= 32)
    hipLaunchKernelGGL((update_kernel<16, 4>), g, dim3(1024), 0, s, a, dc);
  else if (a.n_chunks >= 4)
    hipLaunchKernelGGL((update_kernel<4, 8>), g, dim3(256), 0, s, a, dc);
  else
    hipLaunchKernelGGL(update_flat_kernel, dim3((unsigned)std::max<int64_t>(1, (n + 255) / 256)), dim3(256), 0, s, a,
                       dc);
  return (int)hipGetLastError();
}


int launch_update_batched(const UpdateArgs* args, const int* colsum_runs, int n_colsum,
                          const WorkItem* work, int n_work, int grid, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (n_colsum > 0) hipLaunchKernelGGL(colsum_batched, dim3(n_colsum), dim3(256), 0, s, args, colsum_runs);
  if (n_work > 0) hipLaunchKernelGGL(update_batched, dim3(grid), dim3(256), 0, s, args, work, n_work);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// A two-input contraction with one summed letter k, written as a batched
// matrix product out[b][m][n] = sum_k X[b][m][k] Y[b][k][n]: output letters
// found only in X form the row index m, those only in Y the column index n,
// those in both the batch index b (each a row-major combination of its
// letters, in output order).  One wave computes a 32 x 32 tile of one batch on
// v_mfma_f32_32x32x2_f32 (FP32 accumulate); lane l = 32 g + c supplies
// A[row c][k g] and B[k g][col c], and accumulator register v holds
// C[row 8(v/4) + 4g + v%4][col c].
struct GemmGroup {
  int n;                               // letters in the group
  int64_t size[kMaxEinsumLetters];
  int64_t sx[kMaxEinsumLetters];       // stride in X (0 when absent)
  int64_t sy[kMaxEinsumLetters];       // stride in Y
  int64_t so[kMaxEinsumLetters];       // stride in the output
};

struct GemmArgs {
  const float* X;
  const float* Y;
  float* out;
  const float* X2;                     // a second problem of the same shape (blockIdx.y = 1)
  const float* Y2;
  float* out2;
  GemmGroup gm, gn, gb;
  int64_t M, N, B, K;
  int64_t kx, ky;                      // strides of the summed letter in X and Y
  int64_t tiles_m, tiles_n;
};

struct Off3 {
  int64_t x, y, o;
};

__device__ __forceinline__ Off3 group_offsets(const GemmGroup& g, int64_t idx64) {
  Off3 r{0, 0, 0};
  uint32_t idx = (uint32_t)idx64;  // the host keeps M, N and B below 2^31
  for (int d = g.n - 1; d >= 0; --d) {
    const uint32_t sz = (uint32_t)g.size[d];
    const int64_t v = (int64_t)(idx % sz);
    idx /= sz;
    r.x += v * g.sx[d];
    r.y += v * g.sy[d];
    r.o += v * g.so[d];
  }
  return r;
}

// WPT waves share one 32 x 32 tile and split the sum into WPT even shares
// (WPT = 1: four tiles per 256-thread workgroup, each wave the whole sum);
// wave 0 adds the other waves' sums in wave order (deterministic) and stores
// the tile.  Each wave keeps the loads of its next sixteen k in flight while
// it issues the eight MFMA of the current ones.
template <int WPT>
__global__ __launch_bounds__(WPT == 1 ? 256 : 64 * WPT) void einsum_gemm_kernel(GemmArgs a) {
  typedef float f16v __attribute__((ext_vector_type(16)));
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t w = WPT == 1 ? (int64_t)blockIdx.x * 4 + wv : (int64_t)blockIdx.x;
  const int64_t n_tiles = a.tiles_m * a.tiles_n * a.B;
  if (w >= n_tiles) return;  // whole waves (whole workgroups when WPT > 1), before any barrier
  const int g = lane >> 5, c = lane & 31;
  const int64_t tn = w % a.tiles_n, tm = (w / a.tiles_n) % a.tiles_m, bb = w / (a.tiles_n * a.tiles_m);
  const int64_t m = tm * 32 + c, n = tn * 32 + c;
  const bool mv = m < a.M, nv = n < a.N;
  const Off3 ob = group_offsets(a.gb, bb);
  const Off3 om = group_offsets(a.gm, mv ? m : 0);
  const Off3 on = group_offsets(a.gn, nv ? n : 0);
  const bool second = blockIdx.y != 0;
  const float* X = second ? a.X2 : a.X;
  const float* Y = second ? a.Y2 : a.Y;
  float* out = second ? a.out2 : a.out;
  int64_t kb = 0, ke = a.K;
  if constexpr (WPT > 1) {
    const int64_t kq = (a.K + 2 * WPT - 1) / (2 * WPT) * 2;  // a share of the sum, rounded up to even
    kb = wv * kq < a.K ? wv * kq : a.K;
    ke = kb + kq < a.K ? kb + kq : a.K;
  }
  const float* xp = X + ob.x + om.x + g * a.kx;
  const float* yp = Y + ob.y + on.y + g * a.ky;
  const int64_t kx = a.kx, ky = a.ky;
  auto load = [&](int64_t k0, float (&av)[8], float (&bv)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t kk = k0 + 2 * j;
      const bool kv = kk + g < ke;
      av[j] = (mv && kv) ? xp[kk * kx] : 0.f;
      bv[j] = (nv && kv) ? yp[kk * ky] : 0.f;
    }
  };
  f16v acc = {};
  float an[8], bn[8];
  if (kb < ke) load(kb, an, bn);
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
    float ac[8], bc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ac[j] = an[j];
      bc[j] = bn[j];
    }
    if (k0 + 16 < ke) load(k0 + 16, an, bn);
#pragma unroll
    for (int j = 0; j < 8; ++j) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[j], bc[j], acc, 0, 0, 0);
  }
  if constexpr (WPT > 1) {
    __shared__ float red[WPT - 1][16][64];
    if (wv > 0) {
#pragma unroll
      for (int v = 0; v < 16; ++v) red[wv - 1][v][lane] = acc[v];
    }
    __syncthreads();
    if (wv != 0) return;
    for (int q = 0; q < WPT - 1; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] += red[q][v][lane];
  }
  // rows of this lane's accumulator registers: their output offsets come from
  // the lanes that own those rows (every lane of the wave takes part)
  const int64_t base = ob.o + on.o;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = 8 * (v >> 2) + 4 * g + (v & 3);
    const int lo = __shfl((int)(uint32_t)om.o, r, 64);
    const int hi = __shfl((int)(uint32_t)((uint64_t)om.o >> 32), r, 64);
    const int64_t rowo = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    if (nv && tm * 32 + r < a.M) out[base + rowo] = acc[v];
  }
}

// Classify the letters of a two-input, one-summed-letter step; false when
// the step does not have that form (or an output letter is in neither input).
bool gemm_args(const EinsumArgs& e, GemmArgs& g) {
  if (e.n_in != 2 || e.n_sum != 1) return false;
  g.X = e.in[0];
  g.Y = e.in[1];
  g.out = e.out;
  g.X2 = g.Y2 = nullptr;
  g.out2 = nullptr;
  g.gm.n = g.gn.n = g.gb.n = 0;
  g.M = g.N = g.B = 1;
  for (int d = 0; d < e.n_out; ++d) {
    const int64_t sx = e.in_out_stride[0][d], sy = e.in_out_stride[1][d];
    GemmGroup* grp;
    int64_t* tot;
    if (sx != 0 && sy == 0) {
      grp = &g.gm;
      tot = &g.M;
    } else if (sx == 0 && sy != 0) {
      grp = &g.gn;
      tot = &g.N;
    } else if (sx != 0 && sy != 0) {
      grp = &g.gb;
      tot = &g.B;
    } else {
      if (e.out_size[d] != 1) return false;
      continue;  // a size-1 letter adds nothing
    }
    const int i = grp->n++;
    grp->size[i] = e.out_size[d];
    grp->sx[i] = sx;
    grp->sy[i] = sy;
    grp->so[i] = e.out_stride[d];
    *tot *= e.out_size[d];
  }
  g.K = e.sum_size[0];
  g.kx = e.in_sum_stride[0][0];
  g.ky = e.in_sum_stride[1][0];
  g.tiles_m = (g.M + 31) / 32;
  g.tiles_n = (g.N + 31) / 32;
  return true;
}

template <int NIN>
void launch_split(const EinsumArgs& a, const EinsumPtrs& b, dim3 grid, int log2g, uint32_t n_sum, hipStream_t s) {
  if (a.n_sum == 1)
    hipLaunchKernelGGL((einsum_split_kernel<NIN, true>), grid, dim3(256), 0, s, a, b, log2g, n_sum);
  else
    hipLaunchKernelGGL((einsum_split_kernel<NIN, false>), grid, dim3(256), 0, s, a, b, log2g, n_sum);
}

// Two summed letters d, e whose strides satisfy stride(d) = size(e) * stride(e)
// in every input are one letter of size size(d) * size(e) and stride stride(e).
static EinsumArgs merge_sum_letters(EinsumArgs a) {
  bool merged = true;
  while (merged && a.n_sum > 1) {
    merged = false;
    for (int d = 0; d < a.n_sum && !merged; ++d)
      for (int e = 0; e < a.n_sum && !merged; ++e) {
        if (d == e) continue;
        bool ok = true;
        for (int i = 0; i < a.n_in; ++i)
          ok = ok && a.in_sum_stride[i][d] == a.sum_size[e] * a.in_sum_stride[i][e];
        if (!ok) continue;
        a.sum_size[e] *= a.sum_size[d];  // letter e now spans both; d is removed
        for (int j = d; j + 1 < a.n_sum; ++j) {
          a.sum_size[j] = a.sum_size[j + 1];
          for (int i = 0; i < a.n_in; ++i) a.in_sum_stride[i][j] = a.in_sum_stride[i][j + 1];
        }
        --a.n_sum;
        merged = true;
      }
  }
  return a;
}

// Two contractions that differ only in their operand and output pointers
// (the numerator and denominator chains of one block) go out as one launch,
// the second on blockIdx.y = 1.
int launch_einsum(const EinsumArgs& a_in, void* stream, const EinsumArgs* second) {
  const EinsumArgs a = merge_sum_letters(a_in);
  if (a.n_out_total <= 0) return 0;
  int64_t n_sum = 1;
  for (int d = 0; d < a.n_sum; ++d) n_sum *= a.sum_size[d];
  GemmArgs ga;
  if (gemm_args(a, ga) && ga.M >= 8 && ga.N >= 8 && ga.M * ga.N * ga.B * ga.K >= (int64_t(1) << 20) &&
      ga.M < (int64_t(1) << 31) && ga.N < (int64_t(1) << 31) && ga.B < (int64_t(1) << 31)) {
    const int64_t tiles = ga.tiles_m * ga.tiles_n * ga.B;
    const unsigned pairs = second ? 2u : 1u;
    if (second) {
      ga.X2 = second->in[0];
      ga.Y2 = second->in[1];
      ga.out2 = second->out;
    }
    // too few tiles to fill the chip: the waves of a workgroup split the sum
    if (tiles < 512 && ga.K >= 256) {
      hipLaunchKernelGGL(einsum_gemm_kernel<8>, dim3((unsigned)tiles, pairs), dim3(512), 0, (hipStream_t)stream,
                         ga);
      return (int)hipGetLastError();
    }
    if (tiles < 2048 && ga.K >= 64) {
      hipLaunchKernelGGL(einsum_gemm_kernel<4>, dim3((unsigned)tiles, pairs), dim3(256), 0, (hipStream_t)stream,
                         ga);
      return (int)hipGetLastError();
    }
    if ((tiles + 3) / 4 < (int64_t(1) << 31)) {
      hipLaunchKernelGGL(einsum_gemm_kernel<1>, dim3((unsigned)((tiles + 3) / 4), pairs), dim3(256), 0,
                         (hipStream_t)stream, ga);
      return (int)hipGetLastError();
    }
  }
  // otherwise the second contraction's pointers (same shapes, so the same
  // merged letters) go out in the same launch as blockIdx.y = 1
  EinsumPtrs b;
  for (int i = 0; i < kMaxEinsumIn; ++i) b.in[i] = second ? second->in[i] : a.in[i];
  b.out = second ? second->out : a.out;
  const unsigned pairs = second ? 2u : 1u;
  if (n_sum >= 16 && n_sum < (int64_t(1) << 31) && a.n_in >= 1 && a.n_in <= 4) {
    // lanes per output: enough threads to fill the chip, at most 64
    int log2g = 0;
    while (log2g < 6 && (a.n_out_total << log2g) < (int64_t(1) << 19) && (int64_t(4) << log2g) < n_sum)
      ++log2g;
    const int64_t threads = a.n_out_total << log2g;
    const dim3 grid((unsigned)((threads + 255) / 256), pairs);
    hipStream_t s = (hipStream_t)stream;
    switch (a.n_in) {
      case 1: launch_split<1>(a, b, grid, log2g, (uint32_t)n_sum, s); break;
      case 2: launch_split<2>(a, b, grid, log2g, (uint32_t)n_sum, s); break;
      case 3: launch_split<3>(a, b, grid, log2g, (uint32_t)n_sum, s); break;
      default: launch_split<4>(a, b, grid, log2g, (uint32_t)n_sum, s); break;
    }
    return (int)hipGetLastError();
  }
  const dim3 grid((unsigned)((a.n_out_total + 255) / 256), pairs);
  hipStream_t s = (hipStream_t)stream;
  switch (a.n_in) {
    case 1: hipLaunchKernelGGL(einsum_kernel<1>, grid, dim3(256), 0, s, a, b); break;
    case 2: hipLaunchKernelGGL(einsum_kernel<2>, grid, dim3(256), 0, s, a, b); break;
    case 3: hipLaunchKernelGGL(einsum_kernel<3>, grid, dim3(256), 0, s, a, b); break;
    default: hipLaunchKernelGGL(einsum_kernel<4>, grid, dim3(256), 0, s, a, b); break;
  }
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

int launch_pack(const float* Y, const uint8_t* M, float* Yp, int64_t n, void* stream, int value, int vvalue) {
  if (n <= 0) return 0;
  const int64_t threads = (n + 3) / 4;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, Y, M, Yp, n, (uint32_t)value, (uint32_t)vvalue);
  return (int)hipGetLastError();
}

int launch_copy_f64(double* dst, const double* src, int n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(copy_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, dst, src, n);
  return (int)hipGetLastError();
}

int launch_zero(float* p, int64_t n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, p, n);
  return (int)hipGetLastError();
}

}  // namespace nnef
