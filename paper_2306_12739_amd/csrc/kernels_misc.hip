// Layout transposes between the host state layout and the member-innermost
// device layout, and the per-step diagnostics / one-point statistics kernel.
//
// Statistics follow Sec. 4 of the paper (one-point statistics: mean profile,
// rms fluctuations about it, tangential Reynolds stress); energy, dissipation
// and power input follow from the momentum equation between walls (Sec. 2).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace dns {

namespace {

// host layout [mem][m][j] (complex) <-> device [m][j][e] (complex)
__global__ void state_to_device(const double* __restrict__ src, double* __restrict__ dst, int E0,
                                int count, int E, int K, int N) {
  const size_t total = size_t(count) * K * N;
  for (size_t idx = blockIdx.x * size_t(blockDim.x) + threadIdx.x; idx < total;
       idx += size_t(gridDim.x) * blockDim.x) {
    const int jj = int(idx % N);
    const size_t t = idx / N;
    const int m = int(t % K);
    const int mem = int(t / K);
    const size_t d = (size_t(m) * N + jj) * E + (E0 + mem);
    dst[2 * d] = src[2 * idx];
    dst[2 * d + 1] = src[2 * idx + 1];
  }
}

__global__ void state_from_device(const double* __restrict__ src, double* __restrict__ dst, int E0,
                                  int count, int E, int K, int N) {
  const size_t total = size_t(count) * K * N;
  for (size_t idx = blockIdx.x * size_t(blockDim.x) + threadIdx.x; idx < total;
       idx += size_t(gridDim.x) * blockDim.x) {
    const int jj = int(idx % N);
    const size_t t = idx / N;
    const int m = int(t % K);
    const int mem = int(t / K);
    const size_t d = (size_t(m) * N + jj) * E + (E0 + mem);
    dst[2 * idx] = src[2 * d];
    dst[2 * idx + 1] = src[2 * d + 1];
  }
}

// host [mem][j] <-> device [j][e]
__global__ void profile_to_device(const double* __restrict__ src, double* __restrict__ dst, int E0,
                                  int count, int E, int My) {
  const int total = count * My;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const int j = idx % My, mem = idx / My;
    dst[size_t(j) * E + E0 + mem] = src[idx];
  }
}

__global__ void profile_from_device(const double* __restrict__ src, double* __restrict__ dst, int E0,
                                    int count, int E, int My) {
  const int total = count * My;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const int j = idx % My, mem = idx / My;
    dst[idx] = src[size_t(j) * E + E0 + mem];
  }
}

int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return int(b);
}

// Sum of x over the workgroup in a fixed order (a butterfly within each wave,
// then the waves in order): the same value in every thread after the call.
constexpr int kStatsThreads = 256;
template <int NV>
__device__ __forceinline__ void block_sum(double (&x)[NV], double (*red)[kStatsThreads / 64]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    for (int off = 32; off > 0; off >>= 1) x[c] += __shfl_xor(x[c], off, 64);
    if (lane == 0) red[c][wv] = x[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double t = 0.0;
    for (int w = 0; w < kStatsThreads / 64; ++w) t += red[c][w];
    x[c] = t;
  }
}

// One workgroup per member, one node per thread: volume integrals with
// Clenshaw-Curtis weights (fixed summation order), wall shear, power input,
// finiteness, and the optional time accumulation of the plane profiles.
__global__ void __launch_bounds__(kStatsThreads) stats_kernel(StatsArgs a, int accumulate) {
  const int e = a.e0 + int(blockIdx.x);
  const int My = a.My, E = a.E;
  const size_t ME = size_t(My) * E;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // energy, dissipation, flux, lower and upper shear
  for (int j = threadIdx.x; j < My; j += kStatsThreads) {
    const size_t je = size_t(j) * E + e;
    const double w = a.ccw[j], U = a.U[je];
    s[0] += w * (a.psum[size_t(PS_UU) * ME + je] + a.psum[size_t(PS_VV) * ME + je] +
                 a.psum[size_t(PS_WW) * ME + je]);
    s[1] += w * a.psum[size_t(PS_GRAD) * ME + je];
    s[2] += w * U;
    s[3] += a.D1[j] * U;
    s[4] += a.D1[size_t(My - 1) * My + j] * U;
    if (accumulate) {
      const double W = a.W[je];
      a.acc[size_t(PA_U) * ME + je] += U;
      a.acc[size_t(PA_W) * ME + je] += W;
      a.acc[size_t(PA_U2) * ME + je] += U * U;
      a.acc[size_t(PA_W2) * ME + je] += W * W;
      a.acc[size_t(PA_UU) * ME + je] += a.psum[size_t(PS_UU) * ME + je];
      a.acc[size_t(PA_VV) * ME + je] += a.psum[size_t(PS_VV) * ME + je];
      a.acc[size_t(PA_WW) * ME + je] += a.psum[size_t(PS_WW) * ME + je];
      a.acc[size_t(PA_UV) * ME + je] += a.means[je];
    }
  }
  __shared__ double red[5][kStatsThreads / 64];
  block_sum(s, red);
  if (threadIdx.x != 0) return;
  const double Ly = 2.0;
  const double en = 0.5 * s[0] / Ly, ds = s[1] / (a.Re * Ly), q = s[2], dlo = s[3], dhi = s[4];
  const double pin = a.poiseuille != 0.0 ? a.gamma[e] * q / Ly : a.Uw * (dhi + dlo) / (a.Re * Ly);
  double* inst = a.inst;
  inst[DI_E * E + e] = en;
  inst[DI_EPS * E + e] = ds;
  inst[DI_PI * E + e] = pin;
  inst[DI_Q * E + e] = q;
  inst[DI_TLO * E + e] = dlo / a.Re;
  inst[DI_THI * E + e] = dhi / a.Re;
  if (!isfinite(en) || !isfinite(ds) || !isfinite(q)) a.failed[e] = 1;
  if (accumulate) {
    // wall shear for tau_w: accumulate in the extra slot after the profiles
    a.acc[size_t(NPA) * ME + e] += dlo;
    a.acc[size_t(NPA) * ME + E + e] += dhi;
  }
}

// Shared-mean ensembles (Sec. 4, statistical-state-dynamics paragraph): every
// member's streamwise mean is the member average.  member_mean replaces the
// n_x = 0 column (modes k < NZ) of each plane's advection terms and the plane
// means by their member averages, summed in member order; share_columns does the
// same for the n_x = 0 column of state-shaped buffers [K][N][E] (complex) and,
// when U is given, for the mean profiles [My][E].
template <typename VT>
__global__ void member_mean(VT* __restrict__ nl, double* __restrict__ means, int My, int E, int K,
                            int NZ) {
  const size_t ncol = size_t(3) * My * NZ, total = ncol + size_t(2) * My;
  const double inv = 1.0 / E;
  for (size_t idx = blockIdx.x * size_t(blockDim.x) + threadIdx.x; idx < total;
       idx += size_t(gridDim.x) * blockDim.x) {
    if (idx < ncol) {
      const int k = int(idx % NZ);
      const size_t fj = idx / NZ;  // f * My + j
      const int lb = stage_block_log2(E);
      double re = 0.0, im = 0.0;
      for (int e = 0; e < E; ++e) {
        const VT* p = nl + 2 * stage_off(fj, e, k, E, K, lb);
        re += double(p[0]);
        im += double(p[1]);
      }
      const VT r = VT(re * inv), i = VT(im * inv);
      for (int e = 0; e < E; ++e) {
        VT* p = nl + 2 * stage_off(fj, e, k, E, K, lb);
        p[0] = r;
        p[1] = i;
      }
    } else {
      double* row = means + (idx - ncol) * E;  // [2][My] rows of E members
      double sum = 0.0;
      for (int e = 0; e < E; ++e) sum += row[e];
      for (int e = 0; e < E; ++e) row[e] = sum * inv;
    }
  }
}

__global__ void share_columns(double* __restrict__ v, double* __restrict__ eta, double* __restrict__ U,
                              double* __restrict__ W, int E, int N, int NZ, int My) {
  const size_t ncol = size_t(NZ) * N;  // complex elements of the n_x = 0 column
  const size_t total = 2 * ncol + (U ? size_t(2) * My : 0);
  const double inv = 1.0 / E;
  for (size_t idx = blockIdx.x * size_t(blockDim.x) + threadIdx.x; idx < total;
       idx += size_t(gridDim.x) * blockDim.x) {
    if (idx < 2 * ncol) {
      double* base = (idx < ncol ? v : eta) + 2 * (idx % ncol) * E;  // [k][j] row of E members
      double re = 0.0, im = 0.0;
      for (int e = 0; e < E; ++e) {
        re += base[2 * e];
        im += base[2 * e + 1];
      }
      re *= inv;
      im *= inv;
      for (int e = 0; e < E; ++e) {
        base[2 * e] = re;
        base[2 * e + 1] = im;
      }
    } else {
      const size_t r = idx - 2 * ncol;
      double* row = (r < size_t(My) ? U : W) + (r % My) * E;
      double sum = 0.0;
      for (int e = 0; e < E; ++e) sum += row[e];
      for (int e = 0; e < E; ++e) row[e] = sum * inv;
    }
  }
}

// Plane sums of the two wall planes from the spectral stage fields (Parseval
// over the stored half spectrum, weight 1 for n_x = 0 and 2 otherwise), so
// that the advection kernel never has to visit them: <u^2>, <v^2>, <w^2>,
// <|grad u|^2> (with dv/dy = -(du/dx + dw/dz)) and the means <uv>, <wv>.  At a
// no-slip wall only U00 and the wall shears du/dy, dw/dy contribute; the
// general expressions are evaluated anyway.  One workgroup per (member, wall),
// fixed-order reduction.
constexpr int kWallThreads = 256;
template <typename VT>
__global__ void __launch_bounds__(kWallThreads) wall_sums(const VT* __restrict__ vel, double* __restrict__ psum,
                                                          double* __restrict__ means, int My, int E, int K, int NZ,
                                                          int P, double kxs, double kzs, int e0) {
  typedef typename std::conditional<sizeof(VT) == 4, float2, double2>::type P2;
  const int e = e0 + int(blockIdx.x >> 1);
  const int j = (blockIdx.x & 1) ? My - 1 : 0;
  const size_t FS = 2 * size_t(My) * E * K;  // field stride (VT units)
  const int lb = stage_block_log2(E);
  const VT* row = vel + 2 * stage_off(j, e, 0, E, K, lb);  // mode k at row + (2 k << lb)
  double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // uu vv ww grad uv wv
  auto add = [&](int k, const P2 (&g)[5]) {
    const int nx = k / NZ;
    const int nz = stage_kz(k - nx * NZ);
    const double m = nx == 0 ? 1.0 : 2.0;
    const double kx = kxs * nx, kz = kzs * nz, k2 = kx * kx + kz * kz;
    double f[5][2];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      f[c][0] = double(g[c].x);
      f[c][1] = double(g[c].y);
    }
    const double uu = f[0][0] * f[0][0] + f[0][1] * f[0][1];
    const double vv = f[1][0] * f[1][0] + f[1][1] * f[1][1];
    const double ww = f[2][0] * f[2][0] + f[2][1] * f[2][1];
    const double uy = f[3][0] * f[3][0] + f[3][1] * f[3][1];
    const double wy = f[4][0] * f[4][0] + f[4][1] * f[4][1];
    const double vr = kx * f[0][0] + kz * f[2][0], vi = kx * f[0][1] + kz * f[2][1];  // |dv/dy|
    q[0] += m * uu;
    q[1] += m * vv;
    q[2] += m * ww;
    q[3] += m * (k2 * (uu + vv + ww) + uy + wy + vr * vr + vi * vi);
    q[4] += m * (f[0][0] * f[1][0] + f[0][1] * f[1][1]);
    q[5] += m * (f[2][0] * f[1][0] + f[2][1] * f[1][1]);
  };
  // two modes per thread loaded together (the second clamped to mode 0 and
  // not summed when it is past K)
  for (int k = threadIdx.x; k < K; k += 2 * kWallThreads) {
    const int k2 = k + kWallThreads < K ? k + kWallThreads : 0;
    P2 ga[5], gb[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      ga[c] = *reinterpret_cast<const P2*>(row + c * FS + (2 * size_t(k) << lb));
      gb[c] = *reinterpret_cast<const P2*>(row + c * FS + (2 * size_t(k2) << lb));
    }
    add(k, ga);
    if (k + kWallThreads < K) add(k2, gb);
  }
  __shared__ double red[6][kWallThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double x = q[c];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[c][wv] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[6];
    for (int c = 0; c < 6; ++c) {
      t[c] = 0.0;
      for (int w = 0; w < kWallThreads / 64; ++w) t[c] += red[c][w];
    }
    const size_t je = size_t(j) * E + e, ME = size_t(My) * E;
    psum[size_t(PS_UU) * ME + je] = t[0];
    psum[size_t(PS_VV) * ME + je] = t[1];
    psum[size_t(PS_WW) * ME + je] = t[2];
    psum[size_t(PS_GRAD) * ME + je] = t[3];
    means[je] = t[4];
    means[ME + je] = t[5];
  }
}

}  // namespace

hipError_t launch_wall_sums(int precision, const void* vel, double* psum, double* means, int My, int E, int K,
                            int NZ, int P, double kxs, double kzs, int e0, int ec, hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(wall_sums<double>, dim3(2 * ec), dim3(kWallThreads), 0, s, static_cast<const double*>(vel), psum,
                       means, My, E, K, NZ, P, kxs, kzs, e0);
  else
    hipLaunchKernelGGL(wall_sums<float>, dim3(2 * ec), dim3(kWallThreads), 0, s, static_cast<const float*>(vel), psum,
                       means, My, E, K, NZ, P, kxs, kzs, e0);
  return hipGetLastError();
}

hipError_t launch_member_mean(int precision, void* nl, double* means, int My, int E, int K, int NZ,
                              hipStream_t s) {
  const size_t total = size_t(3) * My * NZ + size_t(2) * My;
  if (precision == 0)
    hipLaunchKernelGGL(member_mean<double>, dim3(grid_for(total)), dim3(256), 0, s,
                       static_cast<double*>(nl), means, My, E, K, NZ);
  else
    hipLaunchKernelGGL(member_mean<float>, dim3(grid_for(total)), dim3(256), 0, s,
                       static_cast<float*>(nl), means, My, E, K, NZ);
  return hipGetLastError();
}

hipError_t launch_share_columns(double* v, double* eta, double* U, double* W, int E, int N, int NZ,
                                int My, hipStream_t s) {
  const size_t total = 2 * size_t(NZ) * N + (U ? size_t(2) * My : 0);
  hipLaunchKernelGGL(share_columns, dim3(grid_for(total)), dim3(256), 0, s, v, eta, U, W, E, N, NZ, My);
  return hipGetLastError();
}

hipError_t launch_state_to_device(const double* src, double* dst, int E0, int count, int E, int K,
                                  int N, hipStream_t s) {
  hipLaunchKernelGGL(state_to_device, dim3(grid_for(size_t(count) * K * N)), dim3(256), 0, s, src,
                     dst, E0, count, E, K, N);
  return hipGetLastError();
}

hipError_t launch_state_from_device(const double* src, double* dst, int E0, int count, int E, int K,
                                    int N, hipStream_t s) {
  hipLaunchKernelGGL(state_from_device, dim3(grid_for(size_t(count) * K * N)), dim3(256), 0, s,
                     src, dst, E0, count, E, K, N);
  return hipGetLastError();
}

hipError_t launch_profile_to_device(const double* src, double* dst, int E0, int count, int E,
                                    int My, hipStream_t s) {
  hipLaunchKernelGGL(profile_to_device, dim3(grid_for(size_t(count) * My)), dim3(256), 0, s, src,
                     dst, E0, count, E, My);
  return hipGetLastError();
}

hipError_t launch_profile_from_device(const double* src, double* dst, int E0, int count, int E,
                                      int My, hipStream_t s) {
  hipLaunchKernelGGL(profile_from_device, dim3(grid_for(size_t(count) * My)), dim3(256), 0, s,
                     src, dst, E0, count, E, My);
  return hipGetLastError();
}

// Resolve the statistics and layout kernels on the current device.
hipError_t misc_preload() {
  const void* fns[10] = {reinterpret_cast<const void*>(&stats_kernel),
                        reinterpret_cast<const void*>(&wall_sums<double>),
                        reinterpret_cast<const void*>(&wall_sums<float>),
                        reinterpret_cast<const void*>(&state_to_device),
                        reinterpret_cast<const void*>(&state_from_device),
                        reinterpret_cast<const void*>(&profile_to_device),
                        reinterpret_cast<const void*>(&profile_from_device),
                        reinterpret_cast<const void*>(&member_mean<double>),
                        reinterpret_cast<const void*>(&member_mean<float>),
                        reinterpret_cast<const void*>(&share_columns)};
  for (const void* fn : fns) {
    hipFuncAttributes attr;
    const hipError_t err = hipFuncGetAttributes(&attr, fn);
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_stats(const StatsArgs& a, int accumulate, hipStream_t s) {
  if (a.ec < 1) return hipSuccess;
  hipLaunchKernelGGL(stats_kernel, dim3(a.ec), dim3(kStatsThreads), 0, s, a, accumulate);
  return hipGetLastError();
}

}  // namespace dns
