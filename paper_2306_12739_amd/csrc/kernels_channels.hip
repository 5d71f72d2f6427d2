// Channel form of ensemble states (learned spin-up; layout in include/sno.h).
//
// To channels: the velocity spectra u, v, w at every Chebyshev node (the stage
// buffer the per-mode kernel writes) are transformed to the 3/2-padded x-z
// grid (Sec. 3.2) and, along y, to the coefficients of the Chebyshev
// interpolant through the nodes (Sec. 2).  From channels: the reverse maps,
// then an admissible state -- v at the interior nodes, eta = i kz u - i kx w,
// the (0, 0) modes as the mean profiles with the boundary values at the walls,
// the n_x = 0 column made Hermitian (Appendix A's half spectrum).
//
// The x-z transforms here are separable direct sums in FP64 (one workgroup per
// (member, field, node)); they run once per hand-off, not per time step.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace dns {

namespace {

constexpr int kCT = 256;

struct cd {
  double x, y;
};

__device__ __forceinline__ cd cexp_frac(long long num, long long den, double sign) {
  // e^{sign 2 pi i num / den} with num reduced exactly modulo den
  long long r = num % den;
  if (r < 0) r += den;
  double s, c;
  sincospi(2.0 * double(r) / double(den), &s, &c);
  return cd{c, sign * s};
}

// spectra (stage buffer, fields 0..2) -> physical planes phys[e][f][j][iz][ix]
template <typename VT>
__global__ void __launch_bounds__(kCT) spec_to_phys_kernel(const VT* vel, double* phys, int My, int E, int K, int L,
                                                           int NZ, int Mx, int Mz, int member0) {
  extern __shared__ double sm[];
  cd* spec = reinterpret_cast<cd*>(sm);       // [L][NZ]
  cd* T = spec + size_t(L) * NZ;              // [L][Mz]
  const int blk = blockIdx.x;
  const int j = blk % My, f = (blk / My) % 3, el = blk / (3 * My);
  const int e = member0 + el;
  const int P = (NZ + 1) / 2;
  const size_t FS = 2 * size_t(My) * E * K;
  for (int q = threadIdx.x; q < L * NZ; q += kCT) {
    const size_t off = f * FS + 2 * stage_off(j, e, q, E, K, stage_block_log2(E));
    const int nx = q / NZ, nz = stage_kz(q - nx * NZ);
    spec[nx * NZ + (nz >= 0 ? nz : nz + NZ)] = cd{double(vel[off]), double(vel[off + 1])};
  }
  __syncthreads();
  for (int q = threadIdx.x; q < L * Mz; q += kCT) {
    const int kx = q / Mz, iz = q - kx * Mz;
    double ar = 0.0, ai = 0.0;
    for (int izp = 0; izp < NZ; ++izp) {
      const int nz = izp < P ? izp : izp - NZ;
      const cd w = cexp_frac((long long)nz * iz, Mz, 1.0);
      const cd a = spec[kx * NZ + izp];
      ar += a.x * w.x - a.y * w.y;
      ai += a.x * w.y + a.y * w.x;
    }
    T[q] = cd{ar, ai};
  }
  __syncthreads();
  double* out = phys + ((size_t(el) * 3 + f) * My + j) * size_t(Mx) * Mz;
  for (int q = threadIdx.x; q < Mx * Mz; q += kCT) {
    const int iz = q / Mx, ix = q - iz * Mx;
    double s = 0.0;
    for (int kx = 0; kx < L; ++kx) {
      const cd w = cexp_frac((long long)kx * ix, Mx, 1.0);
      const cd a = T[kx * Mz + iz];
      s += (kx == 0 ? 1.0 : 2.0) * (a.x * w.x - a.y * w.y);
    }
    out[q] = s;
  }
}

// dst[c][k][p] = sum_j M[k][j] src[c][j][p], c over count*3 columns of My rows
template <typename SRC, typename DST>
__global__ void ymap_kernel(const SRC* src, const double* Mt, DST* dst, int My, long long P, long long ncol) {
  const long long n = ncol * P;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long c = i / P, p = i - c * P;
    const SRC* s = src + c * My * P + p;
    DST* d = dst + c * My * P + p;
    for (int k = 0; k < My; ++k) {
      double acc = 0.0;
      for (int j = 0; j < My; ++j) acc += Mt[k * My + j] * double(s[j * P]);
      d[k * P] = DST(acc);
    }
  }
}

// physical planes -> kept modes spec[e][f][j][K] (complex FP64)
__global__ void __launch_bounds__(kCT) phys_to_spec_kernel(const double* phys, double* spec, int My, int L, int NZ,
                                                           int Mx, int Mz) {
  extern __shared__ double sm[];
  double* plane = sm;                                   // [Mz][Mx]
  cd* S = reinterpret_cast<cd*>(sm + size_t(Mx) * Mz);   // [Mz][L]
  const int blk = blockIdx.x;
  const size_t PL = size_t(Mx) * Mz;
  const double* in = phys + size_t(blk) * PL;
  for (size_t q = threadIdx.x; q < PL; q += kCT) plane[q] = in[q];
  __syncthreads();
  for (int q = threadIdx.x; q < Mz * L; q += kCT) {
    const int iz = q / L, kx = q - iz * L;
    double ar = 0.0, ai = 0.0;
    for (int ix = 0; ix < Mx; ++ix) {
      const cd w = cexp_frac((long long)kx * ix, Mx, -1.0);
      const double v = plane[iz * Mx + ix];
      ar += v * w.x;
      ai += v * w.y;
    }
    S[q] = cd{ar, ai};
  }
  __syncthreads();
  const int P = (NZ + 1) / 2;
  const double norm = 1.0 / (double(Mx) * Mz);
  double* out = spec + size_t(blk) * 2 * L * NZ;
  for (int q = threadIdx.x; q < L * NZ; q += kCT) {
    const int kx = q / NZ, izp = q - kx * NZ;
    const int nz = izp < P ? izp : izp - NZ;
    double ar = 0.0, ai = 0.0;
    for (int iz = 0; iz < Mz; ++iz) {
      const cd w = cexp_frac((long long)nz * iz, Mz, -1.0);
      const cd a = S[iz * L + kx];
      ar += a.x * w.x - a.y * w.y;
      ai += a.x * w.y + a.y * w.x;
    }
    out[2 * q] = ar * norm;
    out[2 * q + 1] = ai * norm;
  }
}

// admissible state from the spectra of u, v, w at every node
__global__ void assemble_state_kernel(const double* spec, double* v, double* eta, double* U, double* W, int My,
                                      int E, int L, int NZ, int member0, int count, double kxs, double kzs,
                                      double Ubot, double Utop) {
  const int N = My - 2, K = L * NZ, P = (NZ + 1) / 2;
  const long long nst = (long long)K * N * count;
  const long long total = nst + (long long)My * count;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    if (i < nst) {
      const int el = int(i % count);
      const long long r = i / count;
      const int jj = int(r % N), mode = int(r / N);
      const int nx = mode / NZ, izp = mode - nx * NZ;
      auto at = [&](int f, int md) {
        const double* p = spec + 2 * ((((size_t(el) * 3 + f) * My) + jj + 1) * K + md);
        return cd{p[0], p[1]};
      };
      auto vort = [&](int md) {
        const int mx = md / NZ, mz = md - mx * NZ;
        const double kx = kxs * mx, kz = kzs * (mz < P ? mz : mz - NZ);
        const cd u = at(0, md), w = at(2, md);
        // i kz u - i kx w
        return cd{-kz * u.y + kx * w.y, kz * u.x - kx * w.x};
      };
      cd vv = at(1, mode), ee = vort(mode);
      if (nx == 0) {
        const int nz = izp < P ? izp : izp - NZ;
        const int mir = nz > 0 ? NZ - nz : (nz < 0 ? -nz : 0);
        const cd vm = at(1, mir), em = vort(mir);
        vv = cd{0.5 * (vv.x + vm.x), 0.5 * (vv.y - vm.y)};
        ee = cd{0.5 * (ee.x + em.x), 0.5 * (ee.y - em.y)};
        if (izp == 0) vv = ee = cd{0.0, 0.0};
      }
      const size_t o = 2 * ((size_t(mode) * N + jj) * E + member0 + el);
      v[o] = vv.x;
      v[o + 1] = vv.y;
      eta[o] = ee.x;
      eta[o + 1] = ee.y;
    } else {
      const long long r = i - nst;
      const int el = int(r % count), j = int(r / count);
      double u = spec[2 * (((size_t(el) * 3 + 0) * My + j) * K)];
      double w = spec[2 * (((size_t(el) * 3 + 2) * My + j) * K)];
      if (j == 0) u = Ubot, w = 0.0;
      if (j == My - 1) u = Utop, w = 0.0;
      U[size_t(j) * E + member0 + el] = u;
      W[size_t(j) * E + member0 + el] = w;
    }
  }
}

int grid_of(long long n) {
  const long long b = (n + 255) / 256;
  return int(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

__global__ void clear_ints_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

// ---- scratch of the allocation-free hand-off -----------------------------------
// dns_set_channels_noalloc keeps its FP64 intermediates in this fixed array
// instead of the handle's staging buffer.  Every GPU the library runs on holds
// its own copy until the process ends.  In host code the array's name is only a
// stand-in: the device address comes from hipGetSymbolAddress, looked up once
// per device (with that device current) and kept in g_scratch_ptr.
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (err != hipSuccess) return err;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return static_cast<double*>(g_scratch_ptr[device]);
}

hipError_t launch_clear_ints(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(clear_ints_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_to_channels(int precision, const void* vel, double* phys, const double* cinv, float* out, int My,
                              int E, int K, int L, int NZ, int Mx, int Mz, int member0, int count, hipStream_t s) {
  const size_t lds = (size_t(L) * NZ + size_t(L) * Mz) * sizeof(cd);
  const void* fn = precision == 0 ? reinterpret_cast<const void*>(&spec_to_phys_kernel<double>)
                                  : reinterpret_cast<const void*>(&spec_to_phys_kernel<float>);
  hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (err != hipSuccess) return err;
  const dim3 grid(3 * My * count);
  if (precision == 0)
    hipLaunchKernelGGL(spec_to_phys_kernel<double>, grid, dim3(kCT), lds, s, static_cast<const double*>(vel), phys,
                       My, E, K, L, NZ, Mx, Mz, member0);
  else
    hipLaunchKernelGGL(spec_to_phys_kernel<float>, grid, dim3(kCT), lds, s, static_cast<const float*>(vel), phys, My,
                       E, K, L, NZ, Mx, Mz, member0);
  const long long P = (long long)Mx * Mz, ncol = 3LL * count;
  hipLaunchKernelGGL((ymap_kernel<double, float>), dim3(grid_of(ncol * P)), dim3(256), 0, s, phys, cinv, out, My, P,
                     ncol);
  return hipGetLastError();
}

hipError_t launch_from_channels(const float* in, double* phys, double* spec, const double* tmat, double* v,
                                double* eta, double* U, double* W, int My, int E, int L, int NZ, int Mx, int Mz,
                                int member0, int count, double kxs, double kzs, double Ubot, double Utop,
                                hipStream_t s) {
  const long long P = (long long)Mx * Mz, ncol = 3LL * count;
  hipLaunchKernelGGL((ymap_kernel<float, double>), dim3(grid_of(ncol * P)), dim3(256), 0, s, in, tmat, phys, My, P,
                     ncol);
  const size_t lds = size_t(Mx) * Mz * sizeof(double) + size_t(Mz) * L * sizeof(cd);
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&phys_to_spec_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(phys_to_spec_kernel, dim3(3 * My * count), dim3(kCT), lds, s, phys, spec, My, L, NZ, Mx, Mz);
  const long long total = (long long)L * NZ * (My - 2) * count + (long long)My * count;
  hipLaunchKernelGGL(assemble_state_kernel, dim3(grid_of(total)), dim3(256), 0, s, spec, v, eta, U, W, My, E, L, NZ,
                     member0, count, kxs, kzs, Ubot, Utop);
  return hipGetLastError();
}

}  // namespace dns
