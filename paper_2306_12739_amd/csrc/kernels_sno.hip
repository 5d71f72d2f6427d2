// Kernels of the spectral neural operator used for the learned spin-up.
//
// Every linear map of the network -- the pointwise channel mixes, the
// truncated x-z DFT and its inverse (dense real matrices), the per-mode complex
// channel mixes and all their gradients -- is one strided, batched GEMM:
//   C[b][m][n] = alpha * sum_k A[b][m][k] B[b][k][n] + beta * C[b][m][n],
// each operand addressed by its own (row, column, batch) strides, so transposes
// and interleaved layouts need no copies.  Two arithmetic modes:
//   * BF16: operands rounded to bfloat16 (nearest even) as they enter the
//     matrix cores, v_mfma_f32_16x16x16bf16_1k with FP32 accumulation;
//   * FP32: the same tiles through FP32 fused multiply-adds (for parity checks).
// Elementwise work (bias, GELU and its derivative), per-channel sums, the
// relative-L2 loss and AdamW are plain FP32 kernels.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dns {

namespace {

constexpr int kTile = 64;   // output tile (rows and columns) per workgroup
constexpr int kKT = 32;     // K depth of one LDS stage
constexpr int kGT = 256;    // threads per GEMM workgroup

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return static_cast<short>(u >> 16);
}

template <bool kBF16>
__global__ void __launch_bounds__(kGT) gemm_kernel(GemmArgs g) {
  __shared__ float As[kTile][kKT + 1];
  __shared__ float Bs[kKT][kTile + 1];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  const int nb = g.reduce_batch ? g.batch : 1;
  const int b0 = g.reduce_batch ? 0 : blockIdx.z;
  const int lane = tid & 63, wave = tid >> 6;
  // BF16: wave w owns rows 32 (w / 2).., cols 32 (w % 2).. as 2 x 2 MFMA tiles
  f32x4 acc[2][2];
  // FP32: thread owns a 4 x 4 block
  float accs[4][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) accs[i][j] = 0.f;

  for (int bb = 0; bb < nb; ++bb) {
    const int b = b0 + bb;
    const float* A = g.A + b * g.sab;
    const float* B = g.B + b * g.sbb;
    for (int k0 = 0; k0 < g.K; k0 += kKT) {
      for (int q = tid; q < kTile * kKT; q += kGT) {
        const int r = q / kKT, c = q - r * kKT;
        const int m = m0 + r, k = k0 + c;
        As[r][c] = (m < g.M && k < g.K) ? A[m * g.sam + k * g.sak] : 0.f;
      }
      for (int q = tid; q < kKT * kTile; q += kGT) {
        const int r = q / kTile, c = q - r * kTile;
        const int k = k0 + r, n = n0 + c;
        Bs[r][c] = (k < g.K && n < g.N) ? B[k * g.sbk + n * g.sbn] : 0.f;
      }
      __syncthreads();
      if constexpr (kBF16) {
        const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
        const int lr = lane & 15, lk = (lane >> 4) * 4;
#pragma unroll
        for (int ks = 0; ks < kKT; ks += 16) {
          bf16x4 a[2], bv[2];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              a[i][t] = to_bf16(As[wr + 16 * i + lr][ks + lk + t]);
              bv[i][t] = to_bf16(Bs[ks + lk + t][wc + 16 * i + lr]);
            }
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], bv[j], acc[i][j], 0, 0, 0);
        }
      } else {
        const int tr = (tid >> 4) * 4, tc = (tid & 15) * 4;
        for (int k = 0; k < kKT; ++k) {
          float av[4], bw[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) av[i] = As[tr + i][k];
#pragma unroll
          for (int j = 0; j < 4; ++j) bw[j] = Bs[k][tc + j];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) accs[i][j] = fmaf(av[i], bw[j], accs[i][j]);
        }
      }
      __syncthreads();
    }
  }

  float* C = g.C + (g.reduce_batch ? 0 : b0 * g.scb);
  auto put = [&](int m, int n, float v) {
    if (m >= g.M || n >= g.N) return;
    float* p = C + m * g.scm + n * g.scn;
    *p = g.beta != 0.f ? g.alpha * v + g.beta * *p : g.alpha * v;
  };
  if constexpr (kBF16) {
    // D layout of the 16x16 MFMA: lane l, register r -> row 4 (l / 16) + r, col l % 16
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          put(m0 + wr + 16 * i + 4 * (lane >> 4) + r, n0 + wc + 16 * j + (lane & 15), acc[i][j][r]);
  } else {
    const int tr = (tid >> 4) * 4, tc = (tid & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) put(m0 + tr + i, n0 + tc + j, accs[i][j]);
  }
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.3989422804014327f * expf(-0.5f * z * z);
}

// x[b][c][p] += bias[c]; optionally h = GELU(x)
__global__ void bias_act_kernel(float* x, float* h, const float* bias, int C, int P, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int c = int((i / P) % C);
    const float z = x[i] + bias[c];
    x[i] = z;
    if (h) h[i] = gelu_f(z);
  }
}

// dz = dh * GELU'(z), in place on dh
__global__ void gelu_bwd_kernel(float* dh, const float* z, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dh[i] *= gelu_grad_f(z[i]);
}

// out[c] = sum_{b, p} x[b][c][p]; one workgroup per channel, fixed order
__global__ void channel_sum_kernel(const float* x, float* out, int B, int C, int P) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int b = 0; b < B; ++b)
    for (int p = threadIdx.x; p < P; p += blockDim.x) s += x[(size_t(b) * C + c) * P + p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// per sample: sq[2 b] = ||yhat_b - y_b||^2, sq[2 b + 1] = ||y_b||^2 (FP64 sums)
__global__ void loss_norms_kernel(const float* yhat, const float* y, double* sq, long long per) {
  __shared__ double r1[256], r2[256];
  const int b = blockIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (long long i = threadIdx.x; i < per; i += blockDim.x) {
    const double t = double(y[b * per + i]);
    const double d = double(yhat[b * per + i]) - t;
    s1 += d * d;
    s2 += t * t;
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sq[2 * b] = r1[0];
    sq[2 * b + 1] = r2[0];
  }
}

// loss = mean_b sqrt(sq_d / sq_y); dy = (yhat - y) / (||d|| ||y|| B)
__global__ void loss_grad_kernel(const float* yhat, const float* y, const double* sq, float* dy, float* loss,
                                 int B, long long per) {
  const long long n = per * B;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += sqrt(sq[2 * b] / sq[2 * b + 1]);
    *loss = float(s / B);
  }
  if (!dy) return;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int b = int(i / per);
    const double nd = sqrt(sq[2 * b]), ny = sqrt(sq[2 * b + 1]);
    dy[i] = nd > 0.0 ? float((double(yhat[i]) - double(y[i])) / (nd * ny * B)) : 0.f;
  }
}

__global__ void adamw_kernel(float* w, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                             float eps, float wd, float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    w[i] = w[i] - lr * wd * w[i] - lr * mh / (sqrtf(vh) + eps);
  }
}

// c[i] = sum_b t[b * n + i], b in order
__global__ void batch_sum_kernel(const float* t, float* c, int batch, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int b = 0; b < batch; ++b) acc += t[b * n + i];
    c[i] = acc;
  }
}

int grid_for(long long n) {
  long long b = (n + 255) / 256;
  return int(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& g, bool bf16, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  dim3 grid((g.N + kTile - 1) / kTile, (g.M + kTile - 1) / kTile, g.reduce_batch ? 1 : g.batch);
  if (bf16)
    hipLaunchKernelGGL(gemm_kernel<true>, grid, dim3(kGT), 0, s, g);
  else
    hipLaunchKernelGGL(gemm_kernel<false>, grid, dim3(kGT), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_bias_act(float* x, float* h, const float* bias, int B, int C, int P, hipStream_t s) {
  const long long n = (long long)B * C * P;
  hipLaunchKernelGGL(bias_act_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, h, bias, C, P, n);
  return hipGetLastError();
}

hipError_t launch_gelu_bwd(float* dh, const float* z, long long n, hipStream_t s) {
  hipLaunchKernelGGL(gelu_bwd_kernel, dim3(grid_for(n)), dim3(256), 0, s, dh, z, n);
  return hipGetLastError();
}

hipError_t launch_channel_sum(const float* x, float* out, int B, int C, int P, hipStream_t s) {
  hipLaunchKernelGGL(channel_sum_kernel, dim3(C), dim3(256), 0, s, x, out, B, C, P);
  return hipGetLastError();
}

hipError_t launch_loss(const float* yhat, const float* y, double* sq, float* dy, float* loss, int B, long long per,
                       hipStream_t s) {
  hipLaunchKernelGGL(loss_norms_kernel, dim3(B), dim3(256), 0, s, yhat, y, sq, per);
  hipLaunchKernelGGL(loss_grad_kernel, dim3(grid_for(per * B)), dim3(256), 0, s, yhat, y, sq, dy, loss, B, per);
  return hipGetLastError();
}

hipError_t launch_batch_sum(const float* t, float* c, int batch, long long n, hipStream_t s) {
  hipLaunchKernelGGL(batch_sum_kernel, dim3(grid_for(n)), dim3(256), 0, s, t, c, batch, n);
  return hipGetLastError();
}

hipError_t launch_adamw(float* w, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                        float eps, float wd, int t, hipStream_t s) {
  const float c1 = 1.f - powf(b1, float(t)), c2 = 1.f - powf(b2, float(t));
  hipLaunchKernelGGL(adamw_kernel, dim3(grid_for(n)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, wd, c1, c2);
  return hipGetLastError();
}

}  // namespace dns
