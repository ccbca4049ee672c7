// Per-element MLP behind the learned Newton initial guess of an implicit
// stage (not in the paper, which starts Newton from S_m, Eq. 21):
// y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3 per element, x the
// element's last two step-to-step changes of the converged stage increment
// (scaled per variable), y two blend weights; the guess takes the mean of y
// over the elements.  Weights are held as an FP32 master copy and a BF16
// copy; the products run on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32
// accumulate) in one strided GEMM kernel used for the forward pass and for
// the transposed products of the backward pass.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace dgj {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x) {
  __hip_bfloat16 b = __float2bfloat16(x);
  uint16_t r;
  __builtin_memcpy(&r, &b, 2);
  return r;
}

struct GemmArgs {
  const uint16_t* A;   // A(i,k) = A[i*a_i + k*a_k]   (bf16 bits)
  long a_i, a_k;
  const uint16_t* B;   // B(k,j) = B[k*b_k + j*b_j]
  long b_k, b_j;
  int M, N, K;
  const float* bias;   // [N] or null
  int act;             // 0 identity, 1 tanh
  float* Cf;           // C(i,j) = Cf[i*c_ld + j] or null
  uint16_t* Cb;        // bf16 copy with the same layout, or null
  long c_ld;
  int k_chunk;         // split K: workgroup z sums k in [z k_chunk, (z+1) k_chunk) (0: all of K)
  float* part;         // split K: raw partial sums part[z][i][j] (M x N each) instead of the epilogue
};

// 64x64 output tile per workgroup of 4 wavefronts, 32x32 per wavefront as
// 2x2 MFMA tiles; K in steps of 16 with zero fill at the edges.  MFMA lane
// layout: A row = lane%16, k = 4*(lane/16)+t; B column = lane%16,
// k = 4*(lane/16)+t; D row = 4*(lane/16)+r, column = lane%16.
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ti = blockIdx.y * 64 + (wave >> 1) * 32;
  const int tj = blockIdx.x * 64 + (wave & 1) * 32;
  const int r16 = lane & 15, kq = (lane >> 4) * 4;
  f32x4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const int kb0 = g.k_chunk > 0 ? (int)blockIdx.z * g.k_chunk : 0;
  const int kb1 = g.k_chunk > 0 ? min(g.K, kb0 + g.k_chunk) : g.K;
  for (int k0 = kb0; k0 < kb1; k0 += 16) {
    bf16x4_t av[2], bv[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int i = ti + s * 16 + r16;
      const int j = tj + s * 16 + r16;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = k0 + kq + t;
        av[s][t] = (i < g.M && k < kb1) ? (short)g.A[(long)i * g.a_i + (long)k * g.a_k] : (short)0;
        bv[s][t] = (j < g.N && k < kb1) ? (short)g.B[(long)k * g.b_k + (long)j * g.b_j] : (short)0;
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ti + a * 16 + kq + r;
        const int j = tj + b * 16 + r16;
        if (i < g.M && j < g.N) {
          float v = acc[a][b][r];
          if (g.part) {
            g.part[((long)blockIdx.z * g.M + i) * g.N + j] = v;
            continue;
          }
          if (g.bias) v += g.bias[j];
          if (g.act == 1) v = tanhf(v);
          if (g.Cf) g.Cf[(long)i * g.c_ld + j] = v;
          if (g.Cb) g.Cb[(long)i * g.c_ld + j] = f2bf(v);
        }
      }
}

// sum of the split-K partials in a fixed order, then the GEMM epilogue
__global__ void k_splitk_reduce(const float* __restrict__ part, int S, int M, int N, const float* __restrict__ bias,
                                int act, float* __restrict__ Cf, uint16_t* __restrict__ Cb, long c_ld) {
  const long total = (long)M * N;
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (long)gridDim.x * blockDim.x) {
    float v = 0.f;
    for (int z = 0; z < S; ++z) v += part[(long)z * total + q];
    const long i = q / N, j = q - i * N;
    if (bias) v += bias[j];
    if (act == 1) v = tanhf(v);
    if (Cf) Cf[i * c_ld + j] = v;
    if (Cb) Cb[i * c_ld + j] = f2bf(v);
  }
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = f2bf(x[i]);
}

// dZ = dH * (1 - H^2) from dH (fp32) and the tanh output H (fp32); bf16 and fp32 out
__global__ void k_tanh_back(const float* __restrict__ dH, const float* __restrict__ H, float* __restrict__ dZ,
                            uint16_t* __restrict__ dZb, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float h = H[i];
    const float z = dH[i] * (1.f - h * h);
    dZ[i] = z;
    dZb[i] = f2bf(z);
  }
}

// dY = 2 (Y - T) / n (fp32 and bf16), squared error per block for the loss
__global__ void k_mse_grad(const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY,
                           uint16_t* __restrict__ dYb, long n, double* __restrict__ part) {
  __shared__ double red[16];
  double s = 0.0;
  const float sc = 2.f / (float)n;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    s += (double)d * (double)d;
    dY[i] = sc * d;
    dYb[i] = f2bf(sc * d);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// column sums of a [R][N] fp32 matrix (bias gradients), fixed order
__global__ void k_colsum(const float* __restrict__ X, long R, int N, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double s = 0.0;
  for (long r = 0; r < R; ++r) s += X[r * N + j];
  out[j] = (float)s;
}

__global__ void k_adam(float* __restrict__ w, uint16_t* __restrict__ wb, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
  }
}

// x rows [(i1 - i2)/s | (i2 - i3)/s] from the three previous stage
// increments i1, i2, i3 ([e][v][m]), s the per-variable scale
__global__ void k_mlp_features(const double* __restrict__ i1, const double* __restrict__ i2,
                               const double* __restrict__ i3, long n_elem, int nv, int nm,
                               const double* __restrict__ s, float* __restrict__ X) {
  const long nb = (long)nv * nm;
  const long total = n_elem * nb;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long e = i / nb, r = i % nb;
    const int v = (int)(r / nm);
    X[e * 2 * nb + r] = (float)((i1[i] - i2[i]) / s[v]);
    X[e * 2 * nb + nb + r] = (float)((i2[i] - i3[i]) / s[v]);
  }
}

// g = S + 2 i1 - i2 + c0 (i1 - i2) + c1 (i1 - 2 i2 + i3): the extrapolated
// guess plus the learned blend of the first and second differences
__global__ void k_blend_guess(double* __restrict__ g, const double* __restrict__ S, const double* __restrict__ i1,
                              const double* __restrict__ i2, const double* __restrict__ i3, double c0, double c1,
                              long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double d1 = i1[i] - i2[i], d2 = i2[i] - i3[i];
    g[i] = S[i] + (2.0 * i1[i] - i2[i]) + c0 * d1 + c1 * (d1 - d2);
  }
}

// training terms of one recorded stage: F0 = i1 - i2, F1 = i1 - 2 i2 + i3
// (the blend directions) and r = inc - 2 i1 + i2 (the extrapolated guess's error)
__global__ void k_blend_terms(const double* __restrict__ inc, const double* __restrict__ i1,
                              const double* __restrict__ i2, const double* __restrict__ i3, double* __restrict__ F0,
                              double* __restrict__ F1, double* __restrict__ r, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double d1 = i1[i] - i2[i], d2 = i2[i] - i3[i];
    F0[i] = d1;
    F1[i] = d1 - d2;
    r[i] = inc[i] - (2.0 * i1[i] - i2[i]);
  }
}

// out[j] = mean over the R rows of Y[r][j]: one workgroup of 256 threads per
// column, FP64 partial sums over rows t, t + 256, ..., then a fixed-order tree
__global__ __launch_bounds__(256) void k_colmean(const float* __restrict__ Y, long R, int N, double* __restrict__ out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (long r = threadIdx.x; r < R; r += 256) s += (double)Y[r * N + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0] / (double)R;
}

// every row of the upstream gradient dY[R][N] = dv[0..N) (FP32 and BF16 copies)
__global__ void k_fill_rows(float* __restrict__ dY, uint16_t* __restrict__ dYb, long R, int N,
                            const double* __restrict__ dv) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < R * N; i += (long)gridDim.x * blockDim.x) {
    const float x = (float)dv[i % N];
    dY[i] = x;
    dYb[i] = f2bf(x);
  }
}

// per-variable sums of squares of (a - b) (b may be null): part[block][v]
__global__ void k_varsq_diff(const double* __restrict__ a, const double* __restrict__ b, long n_elem, int nv, int nm,
                             double* __restrict__ part) {
  __shared__ double red[16];
  for (int v = 0; v < nv; ++v) {
    double s = 0.0;
    const long total = n_elem * nm;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
      const long e = i / nm, m = i % nm;
      const long k = (e * nv + v) * nm + m;
      const double x = b ? a[k] - b[k] : a[k];
      s += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
      part[blockIdx.x * nv + v] = t;
    }
    __syncthreads();
  }
}

}  // namespace dgj
