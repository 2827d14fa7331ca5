// Learned extrapolation of multiplicative-update iterates on gfx950.
//
// A three-layer MLP (8 -> 128 -> 128 -> 1, ReLU, softplus output) maps
// per-element features of a factor's recent iterates to a step multiplier s;
// the proposal is theta' = max(eps, theta_t * exp(s * d1)) with d1 the last
// log step.  The 128 x 128 layer (the only real matrix product) runs on
// v_mfma_f32_32x32x16_bf16 with BF16 inputs and FP32 accumulation, forward and
// backward; the 8 -> 128 and 128 -> 1 layers, the features, the loss and Adam
// are FP32 VALU work.  Gradients are reduced over workgroups in a fixed order
// (deterministic).  The paper has no learned component: the features, targets
// and network are this library's own specification.
//
// MFMA 32x32x16 operand layout used here: lane l = 32 g + c supplies
// A[row c][k slots (g, 0..7)] and B[k slots (g, 0..7)][col c]; both operands
// map slot (g, j) to k = 8 g + j, so the hardware's own slot order cancels.
// The accumulator register v of lane (g, c) holds C[8 (v / 4) + 4 g + v % 4][c].
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "nnef_internal.hpp"

namespace nnef {
namespace {

constexpr int NIN = kMlpIn, WD = kMlpWidth, RB = 32;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f16v mfma_bf16(const bf16x8& a, const bf16x8& b, const f16v& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int acc_row(int v, int g) { return 8 * (v >> 2) + 4 * g + (v & 3); }

__device__ __forceinline__ float softplus(float z) { return z > 20.f ? z : log1pf(expf(z)); }
__device__ __forceinline__ float sigmoid(float z) { return 1.f / (1.f + expf(-z)); }

// log(a / b) for positive a, b, accurate when a is close to b.
__device__ __forceinline__ float log_ratio(float a, float b) {
  const float r = a / b;
  return fabsf(r - 1.f) < 0.5f ? log1pf((a - b) / b) : logf(a) - logf(b);
}

__device__ __forceinline__ int factor_of(const FeatArgs& f, int64_t e) {
  int k = 0;
  while (k + 1 < f.n_fac && e >= f.off[k + 1]) ++k;
  return k;
}

// The eight features of element e (see the MLP oracle for the definition).
__device__ void features(const FeatArgs& f, int64_t e, float* x, float& th_t, float& d1, int& k,
                         int64_t& i) {
  k = factor_of(f, e);
  i = e - f.off[k];
  const float a = f.th[k][i], b = f.tm1[k][i], c = f.tm2[k][i];
  d1 = log_ratio(a, b);
  const float d2 = log_ratio(b, c);
  const float sig = (float)f.sigma[k];
  const float inv = 1.f / sig;
  double rel = f.rel_dec;
  if (f.loss_prev) rel = (*f.loss_prev - *f.loss_cur) / *f.loss_cur;
  x[0] = d1 * inv;
  x[1] = d2 * inv;
  x[2] = log10f(sig) * 0.125f;
  x[3] = (logf(a) - f.log_eps) * f.inv_abs_log_eps;
  x[4] = log10f((float)fmax(rel, 1e-30)) * 0.125f;
  x[5] = f.gamma;
  x[6] = f.logK8[k];
  x[7] = 1.f;
  th_t = a;
}

// LDS layout (bytes) of the MLP kernel.
template <int MODE>
struct Lds {
  static constexpr int W2T = 0;                                 // bf16 [j][i] = W2[i][j]
  static constexpr int W2 = W2T + WD * WD * 2;                  // bf16 [i][j] (backward only)
  static constexpr int W1 = W2 + (MODE == 1 ? WD * WD * 2 : 0);  // f32 [in][i]
  static constexpr int B1 = W1 + NIN * WD * 4;
  static constexpr int B2 = B1 + WD * 4;
  static constexpr int W3 = B2 + WD * 4;
  static constexpr int X = W3 + WD * 4;                          // f32 [row][in]
  static constexpr int H1 = X + RB * NIN * 4;                    // f32 [row][i]
  static constexpr int P = H1 + RB * WD * 4;                     // f32 [row][j]: z terms, then dA2
  static constexpr int DA1 = P + RB * WD * 4;                    // f32 [row][i] (backward only)
  static constexpr int Z = DA1 + (MODE == 1 ? RB * WD * 4 : 0);  // f32 [row]
  static constexpr int AUX = Z + RB * 4;                         // f32 [3][row]: tau | theta_t, d1
  static constexpr int AUXI = AUX + 3 * RB * 4;                  // int64 [row]: element index
  static constexpr int TOTAL = AUXI + RB * 8;
};

// MODE 0: s for rows of X.  MODE 1: gradient partials of the mean row loss
// (s x0 - tau)^2.  MODE 2: proposals for the factor elements of a.f.
template <int MODE>
__global__ __launch_bounds__(256) void mlp_kernel(MlpArgs a) {
  using L = Lds<MODE>;
  __shared__ __attribute__((aligned(16))) unsigned char lds[L::TOTAL];
  __bf16* sW2T = reinterpret_cast<__bf16*>(lds + L::W2T);
  __bf16* sW2 = reinterpret_cast<__bf16*>(lds + L::W2);
  float* sW1 = reinterpret_cast<float*>(lds + L::W1);
  float* sB1 = reinterpret_cast<float*>(lds + L::B1);
  float* sB2 = reinterpret_cast<float*>(lds + L::B2);
  float* sW3 = reinterpret_cast<float*>(lds + L::W3);
  float* sX = reinterpret_cast<float*>(lds + L::X);
  float* sH1 = reinterpret_cast<float*>(lds + L::H1);
  float* sP = reinterpret_cast<float*>(lds + L::P);
  float* sDA1 = reinterpret_cast<float*>(lds + L::DA1);
  float* sZ = reinterpret_cast<float*>(lds + L::Z);
  float* sAux = reinterpret_cast<float*>(lds + L::AUX);
  int64_t* sIdx = reinterpret_cast<int64_t*>(lds + L::AUXI);

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int g = lane >> 5, c = lane & 31;
  const float* prm = a.params;

  // ---- parameters into LDS (W2 as BF16, both orientations for the backward)
  for (int e = t; e < WD * WD; e += 256) {
    const int i = e / WD, j = e % WD;
    const __bf16 w = (__bf16)prm[kMlpOffW2 + e];
    sW2T[j * WD + i] = w;
    if constexpr (MODE == 1) sW2[e] = w;
  }
  for (int e = t; e < NIN * WD; e += 256) sW1[e] = prm[kMlpOffW1 + e];
  if (t < WD) {
    sB1[t] = prm[kMlpOffB1 + t];
    sB2[t] = prm[kMlpOffB2 + t];
    sW3[t] = prm[kMlpOffW3 + t];
  }
  const float b3 = prm[kMlpOffB3];
  __syncthreads();

  // layer-1 weights of this thread's hidden unit
  const int hu = t & (WD - 1), rhalf = t >> 7;
  float w1[NIN];
#pragma unroll
  for (int in = 0; in < NIN; ++in) w1[in] = sW1[in * WD + hu];
  const float b1u = sB1[hu];
  const int jw = 32 * wave + c;  // this lane's unit in the wave's column tile
  const float b2j = sB2[jw], w3j = sW3[jw];

  // gradient accumulators (MODE 1)
  f16v gW2[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) gW2[q][v] = 0.f;
  float gW1[4] = {0.f, 0.f, 0.f, 0.f};
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f;
  double lsum = 0.0;

  const int64_t n_blocks = (a.n_rows + RB - 1) / RB;
  for (int64_t blk = blockIdx.x; blk < n_blocks; blk += gridDim.x) {
    const int64_t r0 = blk * RB;
    // ---- rows of this block
    if constexpr (MODE == 2) {
      if (t < RB) {
        float x[NIN];
        const int64_t e = r0 + t;
        if (e < a.n_rows) {
          float th_t, d1;
          int k;
          int64_t i;
          features(a.f, e, x, th_t, d1, k, i);
          sAux[RB + t] = th_t;
          sAux[2 * RB + t] = d1;
          sIdx[t] = e;
        } else {
#pragma unroll
          for (int in = 0; in < NIN; ++in) x[in] = 0.f;
          sIdx[t] = -1;
        }
#pragma unroll
        for (int in = 0; in < NIN; ++in) sX[t * NIN + in] = x[in];
      }
    } else {
      const int r = t >> 3;
      const int64_t row = r0 + r;
      float xv = 0.f;
      if (row < a.n_rows) {
        const int64_t src = a.idx ? (int64_t)a.idx[row] : row;
        xv = a.X[src * NIN + (t & 7)];
        if (MODE == 1 && (t & 7) == 0) sAux[r] = a.tau[src];
      }
      sX[t] = xv;
    }
    __syncthreads();

    // ---- layer 1 (VALU): h1 = relu(x W1 + b1)
#pragma unroll 4
    for (int q = 0; q < RB / 2; ++q) {
      const int r = rhalf + 2 * q;
      float s = b1u;
#pragma unroll
      for (int in = 0; in < NIN; ++in) s = fmaf(sX[r * NIN + in], w1[in], s);
      sH1[r * WD + hu] = fmaxf(s, 0.f);
    }
    __syncthreads();

    // ---- layer 2 (MFMA): a2[row][j] for the wave's 32 units j
    f16v acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
    for (int ks = 0; ks < WD / 16; ++ks) {
      bf16x8 av, bv;
      const float* hrow = sH1 + c * WD + 16 * ks + 8 * g;
      const __bf16* wrow = sW2T + jw * WD + 16 * ks + 8 * g;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        av[j] = (__bf16)hrow[j];
        bv[j] = wrow[j];
      }
      acc = mfma_bf16(av, bv, acc);
    }
    // layer 3 terms h2 * w3, summed per row below
#pragma unroll
    for (int v = 0; v < 16; ++v) sP[acc_row(v, g) * WD + jw] = fmaxf(acc[v] + b2j, 0.f) * w3j;
    __syncthreads();
    {
      const int r = t >> 3, part = t & 7;
      float s = 0.f;
#pragma unroll
      for (int q = 0; q < 16; ++q) s += sP[r * WD + part * 16 + q];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      if (part == 0) sZ[r] = s + b3;
    }
    __syncthreads();

    if constexpr (MODE == 0) {
      if (t < RB && r0 + t < a.n_rows) a.s_out[r0 + t] = softplus(sZ[t]);
    } else if constexpr (MODE == 2) {
      if (t < RB && sIdx[t] >= 0) {
        const float s = softplus(sZ[t]);
        const int64_t e = sIdx[t];
        const int k = factor_of(a.f, e);
        a.f.cand[k][e - a.f.off[k]] = fmaxf(a.f.eps, sAux[RB + t] * expf(s * sAux[2 * RB + t]));
      }
    } else {
      // ---- loss and d/dz
      if (t < RB) {
        float dz = 0.f;
        if (r0 + t < a.n_rows) {
          const float z = sZ[t], x0 = sX[t * NIN];
          const float s = softplus(z);
          const float r = s * x0 - sAux[t];
          lsum += (double)r * r;
          dz = 2.f * r * x0 * sigmoid(z) * a.inv_n;
          gb3 += dz;
        }
        sZ[t] = dz;
      }
      __syncthreads();
      // ---- layer 3 and 2 backward in the accumulator layout
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = acc_row(v, g);
        const float dz = sZ[m];
        const float a2 = acc[v] + b2j;
        gw3 = fmaf(dz, fmaxf(a2, 0.f), gw3);
        const float da2 = a2 > 0.f ? dz * w3j : 0.f;
        gb2 += da2;
        sP[m * WD + jw] = da2;
      }
      __syncthreads();
      // ---- dH1 = dA2 W2^T (MFMA): the wave's 32 hidden units i = 32 wave + c
      f16v dh;
#pragma unroll
      for (int v = 0; v < 16; ++v) dh[v] = 0.f;
#pragma unroll
      for (int ks = 0; ks < WD / 16; ++ks) {
        bf16x8 av, bv;
        const float* drow = sP + c * WD + 16 * ks + 8 * g;
        const __bf16* wrow = sW2 + jw * WD + 16 * ks + 8 * g;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          av[j] = (__bf16)drow[j];
          bv[j] = wrow[j];
        }
        dh = mfma_bf16(av, bv, dh);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = acc_row(v, g);
        const float da1 = sH1[m * WD + jw] > 0.f ? dh[v] : 0.f;
        gb1 += da1;
        sDA1[m * WD + jw] = da1;
      }
      // ---- gW2[i][j] += sum_rows H1[row][i] dA2[row][j] (MFMA, K = rows)
#pragma unroll
      for (int ks = 0; ks < RB / 16; ++ks) {
        bf16x8 av;
#pragma unroll
        for (int j = 0; j < 8; ++j) av[j] = (__bf16)sH1[(16 * ks + 8 * g + j) * WD + jw];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bf16x8 bv;
#pragma unroll
          for (int j = 0; j < 8; ++j) bv[j] = (__bf16)sP[(16 * ks + 8 * g + j) * WD + 32 * q + c];
          gW2[q] = mfma_bf16(av, bv, gW2[q]);
        }
      }
      __syncthreads();
      // ---- gW1[in][i] += sum_rows x[row][in] dA1[row][i]
      {
        const int in0 = 4 * rhalf;
#pragma unroll 4
        for (int r = 0; r < RB; ++r) {
          const float d = sDA1[r * WD + hu];
#pragma unroll
          for (int q = 0; q < 4; ++q) gW1[q] = fmaf(sX[r * NIN + in0 + q], d, gW1[q]);
        }
      }
    }
    __syncthreads();
  }

  if constexpr (MODE == 1) {
    float* gp = a.gpart + (int64_t)blockIdx.x * kMlpParams;
#pragma unroll
    for (int q = 0; q < 4; ++q) gp[kMlpOffW1 + (4 * rhalf + q) * WD + hu] = gW1[q];
    const float b1s = gb1 + __shfl_xor(gb1, 32, 64);
    const float b2s = gb2 + __shfl_xor(gb2, 32, 64);
    const float w3s = gw3 + __shfl_xor(gw3, 32, 64);
    if (g == 0) {
      gp[kMlpOffB1 + jw] = b1s;
      gp[kMlpOffB2 + jw] = b2s;
      gp[kMlpOffW3 + jw] = w3s;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        gp[kMlpOffW2 + (32 * wave + acc_row(v, g)) * WD + 32 * q + c] = gW2[q][v];
    if (wave == 0) {
      float b = gb3;
      double l = lsum;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        b += __shfl_xor(b, o, 64);
        l += __shfl_xor(l, o, 64);
      }
      if (lane == 0) {
        gp[kMlpOffB3] = b;
        a.lpart[blockIdx.x] = l;
      }
    }
  }
}

// Fixed-order sum of the gradient partials; optional Adam step on the FP32
// master parameters (m, v: FP32 moments; bc1, bc2: bias corrections).  One
// workgroup per 64 parameters: wave w sums partials w, w + 4, ... with eight
// independent accumulators (eight loads in flight), then wave 0 adds the four
// wave sums in a fixed order.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* gpart, const double* lpart,
                                                         int grid, float inv_n, float* grad_out,
                                                         double* loss_out, float* params, float* m,
                                                         float* v, float lr, float b1, float b2,
                                                         float eps, float bc1, float bc2, int adam) {
  __shared__ double sw[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const bool valid = k < kMlpParams;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (valid) {
    int r = w;
    for (; r + 28 < grid; r += 32) {
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] += (double)gpart[(int64_t)(r + 4 * j) * kMlpParams + k];
    }
    for (; r < grid; r += 4) acc[0] += (double)gpart[(int64_t)r * kMlpParams + k];
  }
  sw[w][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (w == 0 && valid) {
    const float gk = (float)(((sw[0][lane] + sw[1][lane]) + sw[2][lane]) + sw[3][lane]);
    if (grad_out) grad_out[k] = gk;
    if (adam) {
      const float mk = b1 * m[k] + (1.f - b1) * gk;
      const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
      m[k] = mk;
      v[k] = vk;
      params[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
    }
  }
  if (blockIdx.x == 0 && w == 1 && loss_out) {
    double l = 0.0;
    for (int i = lane; i < grid; i += 64) l += lpart[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
    if (lane == 0) *loss_out = l * (double)inv_n;
  }
}

// sigma_k = rms over factor k of d1 (one workgroup per factor, FP64 sums).
__global__ __launch_bounds__(256) void sigma_kernel(FeatArgs f, double* sigma) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  const int64_t n = f.off[k + 1] - f.off[k];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double d = log_ratio(f.th[k][i], f.tm1[k][i]);
    s += d * d;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) sigma[k] = sqrt((red[0] + red[1] + red[2] + red[3]) / (double)n) + 1e-30;
}

// Training rows: features and targets tau = clip(log(theta_{t+h}/theta_t)/sigma, +-64).
__global__ __launch_bounds__(256) void rows_kernel(FeatArgs f, float* X, float* tau) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= f.off[f.n_fac]) return;
  float x[NIN], th_t, d1;
  int k;
  int64_t i;
  features(f, e, x, th_t, d1, k, i);
#pragma unroll
  for (int in = 0; in < NIN; ++in) X[e * NIN + in] = x[in];
  if (tau && f.tth[k]) {
    const float r = log_ratio(f.tth[k][i], th_t) / (float)f.sigma[k];
    tau[e] = fminf(64.f, fmaxf(-64.f, r));
  }
}

// Accept a proposal iff its loss is strictly lower (FP64 compare) and it is
// >= eps everywhere (true by construction); then copy it over the factors.
__global__ __launch_bounds__(256) void accept_kernel(FeatArgs f, const double* loss_cand,
                                                     const double* loss_cur, int* n_acc) {
  const double lc = *loss_cand, lu = *loss_cur;
  const bool ok = lc < lu;  // false for NaN
  if (blockIdx.x == 0 && threadIdx.x == 0 && ok && n_acc) n_acc[0] += 1;
  if (!ok) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= f.off[f.n_fac]) return;
  const int k = factor_of(f, e);
  const int64_t i = e - f.off[k];
  f.dst[k][i] = f.cand[k][i];
}

__global__ __launch_bounds__(256) void copy_factors_kernel(FeatArgs f) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= f.off[f.n_fac]) return;
  const int k = factor_of(f, e);
  const int64_t i = e - f.off[k];
  const_cast<float*>(f.tm1[k])[i] = f.th[k][i];
}

int grid_of(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace

int mlp_grid(int64_t n_rows) {
  const int64_t blocks = (n_rows + RB - 1) / RB;
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, 256));
}

int launch_mlp(const MlpArgs& a, int mode, int grid, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (a.n_rows <= 0) return 0;
  if (mode == 0) mlp_kernel<0><<<grid, 256, 0, s>>>(a);
  else if (mode == 1) mlp_kernel<1><<<grid, 256, 0, s>>>(a);
  else mlp_kernel<2><<<grid, 256, 0, s>>>(a);
  return (int)hipGetLastError();
}

int launch_mlp_reduce(const float* gpart, const double* lpart, int grid, float inv_n, float* grad_out,
                      double* loss_out, float* params, float* m, float* v, float lr, float b1, float b2,
                      float eps, float bc1, float bc2, int adam, void* stream) {
  mlp_reduce_kernel<<<(kMlpParams + 63) / 64, 256, 0, (hipStream_t)stream>>>(
      gpart, lpart, grid, inv_n, grad_out, loss_out, params, m, v, lr, b1, b2, eps, bc1, bc2, adam);
  return (int)hipGetLastError();
}

int launch_sigma(const FeatArgs& f, void* stream) {
  sigma_kernel<<<f.n_fac, 256, 0, (hipStream_t)stream>>>(f, const_cast<double*>(f.sigma));
  return (int)hipGetLastError();
}

int launch_rows(const FeatArgs& f, float* X, float* tau, void* stream) {
  const int64_t n = f.off[f.n_fac];
  if (n <= 0) return 0;
  rows_kernel<<<grid_of(n), 256, 0, (hipStream_t)stream>>>(f, X, tau);
  return (int)hipGetLastError();
}

int launch_accept(const FeatArgs& f, const double* loss_cand, const double* loss_cur, int* n_acc,
                  void* stream) {
  const int64_t n = f.off[f.n_fac];
  accept_kernel<<<grid_of(std::max<int64_t>(n, 1)), 256, 0, (hipStream_t)stream>>>(f, loss_cand,
                                                                                    loss_cur, n_acc);
  return (int)hipGetLastError();
}

int launch_copy_factors(const FeatArgs& f, void* stream) {
  const int64_t n = f.off[f.n_fac];
  if (n <= 0) return 0;
  copy_factors_kernel<<<grid_of(n), 256, 0, (hipStream_t)stream>>>(f);
  return (int)hipGetLastError();
}

}  // namespace nnef
