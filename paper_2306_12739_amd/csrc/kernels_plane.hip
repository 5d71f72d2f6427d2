// Pseudo-spectral advection stage: one workgroup per (Chebyshev plane j, member e).
//
// Paper Sec. 3.1-3.2: the advection term u . grad u_i is formed pointwise on a
// 3/2-padded physical grid (2/3-rule dealiasing), its x-z transform truncated
// back to the kept modes; the mean-flow equations need the plane means <uv>
// and <wv> (Eqs. (U00), (W00)).
//
// Inputs per (j, e): spectral u, v, w, du/dy, dw/dy (the derivative fields
// d/dx = i kx, d/dz = i kz are formed on the fly; dv/dy = -(du/dx + dw/dz) by
// continuity, exact at every node).  The physical plane (Mz x Mx) is processed
// in R chunks of PP rows z_p, p = R q + r: a chunk's rows are the output of a
// PP-point inverse FFT of the Mz-point column folded onto PP points with
// twiddles e^{2 pi i n r / Mz}.  Each chunk does
//   Z1 z-iFFT(u, v, w) -> X1 x-iFFT(u, v, w) -> phys u, v, w
//   XA x-iFFT(ux, vx, wx)      -> Nu = u ux, Nv = u vx, Nw = u wx, VY = -ux
//   Z2 z-iFFT(uz, vz, wz) -> XB -> Nu += w uz, Nv += w vz, Nw += w wz, VY -= wz
//   Z3 z-iFFT(uy, wy)     -> XC -> Nu += v uy, Nw += v wy
//   P  Nv += v VY, plane sums
//   XF x-FFT(Nu, Nv, Nw) -> ZF z-FFT of the chunk -> accumulate
//      N_hat(nz) += e^{-2 pi i r nz / Mz} Y_r[nz mod PP] in registers.
// Pairs of physical rows share one complex x transform (real + i imag).
//
// Rotational form (kRot): the advection term is taken as omega x u, which
// differs from u . grad u by a gradient that the curl operators of the v-eta
// equations annihilate (momentum equation, Sec. 2).  The vorticity
//   omega = (dw/dy - i kz v, i kz u - i kx w, i kx v - du/dy)
// is formed in the z fold, so a chunk needs 6 z- and 6 x-transforms:
//   Z1 -> X1 phys u, v, w;  ZW z-iFFT(omega) -> XW phys omega;
//   P  N = (oy w - oz v, oz u - ox w, ox v - oy u), plane sums.
//
// Quasi-linear form (kForm 2, the perturbation dynamics of a shared-mean
// ensemble): with U_m the streamwise mean (n_x = 0 part) of each field and
// u' = u - U_m, the n_x >= 1 output is U_m . grad u' + u' . grad U_m and the
// n_x = 0 output is the full advection's.  On a physical row (fixed y, z) the
// streamwise mean of a field is the real part of its n_x = 0 z-transformed
// value, so the chunk keeps those row means of u, v, w and of the z- and
// y-derivatives, accumulates the linear terms
//   Lin_i = U_m du_i/dx + W_m (du_i/dz - <du_i/dz>) + (w - W_m) <du_i/dz>
//         + V_m (du_i/dy - <du_i/dy>) + (v - V_m) <du_i/dy>
// (their row means vanish) beside the full products, and hands the forward
// transform Lin_i + (row mean of the full product): its n_x = 0 mode is the
// full advection's and every other mode is the linear term's.
//
// Adjoint form (kForm 3, optimal disturbances of a frozen mean): for a velocity
// lambda' of the n_x >= 1 modes the term is -(U_m . grad) lambda' + (grad U_m)^T
// lambda', i.e. Lin_i = -U_m dl_i/dx - W_m (dl_i/dz - <dl_i/dz>) - V_m (dl_i/dy -
// <dl_i/dy>) plus, for i = y and z, sum_j lambda'_j <d u_j/dy> and sum_j
// lambda'_j <d u_j/dz> (row means of the derivatives are those of the mean).
#include <type_traits>

#include "fft.h"
#include "internal.h"

namespace dns {

namespace {

// Spread consecutive logical block indices over one XCD: hardware dispatches
// block b to XCD b % 8, so logical neighbours (same plane, adjacent members,
// which share cache lines of the member-innermost layout) land on one L2.
__device__ __forceinline__ int xcd_logical(int b, int nblk) {
  const int q = nblk >> 3, rem = nblk & 7;
  const int x = b & 7, local = b >> 3;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + local;
}

template <typename VT>
struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename T, typename VT>
__device__ __forceinline__ cx<T> ldc(const VT* p) {
  using V = typename Vec2<VT>::type;
  const V v = *reinterpret_cast<const V*>(p);
  return cx<T>{T(v.x), T(v.y)};
}

template <typename T, typename VT>
__device__ __forceinline__ void stc(VT* p, cx<T> c) {
  using V = typename Vec2<VT>::type;
  V v;
  v.x = VT(c.x);
  v.y = VT(c.y);
  *reinterpret_cast<V*>(p) = v;
}

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int kNT = 512;

enum Phys { PU = 0, PV, PW, PNU, PNV, PNW, PVY, NPHYS };

template <typename T, int L, int P, int PP>
struct PlaneCfg {
  static constexpr int MX = 3 * L, MZ = 3 * P, NZ = 2 * P - 1;
  static constexpr int R = MZ / PP, PH = PP / 2;
  static constexpr int RAX = Split<MX>::A, RBX = Split<MX>::B;
  // LDS pitches, chosen so that the lanes of a wavefront spread over the banks
  static constexpr int ZP = L + 1;                             // z-transform rows [q][nx]
  static constexpr int FP = lds_pitch(2 * L, RAX, 0, 2);       // forward x rows [pair][kx]
  static constexpr int MXP = lds_pitch(MX, RAX, RBX, 1);       // physical rows [q][x]
  static constexpr int PPP = lds_pitch(PP, 1, 0, 2);           // forward z output [(f, nx)][k]
  static constexpr int ZB0 = 3 * PP * ZP, ZB1 = 3 * PH * FP, ZB2 = 3 * L * PPP;
  static constexpr int ZB = ZB0 > ZB1 ? (ZB0 > ZB2 ? ZB0 : ZB2) : (ZB1 > ZB2 ? ZB1 : ZB2);
  static constexpr int MIDZ = 3 * L * MidPitch<PP>::value, MIDX = 3 * PH * MidPitch<MX>::value;
  static constexpr int MID = MIDZ > MIDX ? MIDZ : MIDX;
  static constexpr int NPT = PP * MX;                          // physical points per chunk
  static constexpr int NPTS = PP * MXP;                        // their LDS footprint per field
  static constexpr int NACC = (3 * L * NZ + kNT - 1) / kNT;
  // static LDS of plane_kernel: roots, zb, mid, phys and the reduction scratch
  static constexpr size_t kLdsBytes =
      (MX + MZ + PP + ZB + MID) * 2 * sizeof(T) + NPHYS * NPTS * sizeof(T) + 8 * (kNT / 64) * sizeof(double);
  static_assert(MZ % PP == 0 && PP % 2 == 0, "chunk rows must divide Mz and pair up");
};

}  // namespace

template <typename T, typename VT, int L, int P, int PP, int kForm>
__global__ void __launch_bounds__(kNT) plane_kernel(PlaneArgs a) {
  constexpr bool kRot = kForm == 1, kQL = kForm == 2 || kForm == 3, kAdj = kForm == 3;
  using C = cx<T>;
  using Cfg = PlaneCfg<T, L, P, PP>;
  constexpr int MX = Cfg::MX, MZ = Cfg::MZ, NZ = Cfg::NZ, R = Cfg::R, PH = Cfg::PH;
  __shared__ C rootX[MX];
  __shared__ C rootZ[MZ];
  __shared__ C rootP[PP];
  __shared__ C zb[Cfg::ZB];
  __shared__ C mid[Cfg::MID];
  __shared__ T phys[NPHYS][Cfg::NPTS];
  __shared__ double red[8][kNT / 64];
  // quasi-linear form: linear terms and row means (1-element stand-ins otherwise)
  __shared__ T lin[kQL ? 3 : 1][kQL ? Cfg::NPTS : 1];
  __shared__ T rmean[kQL ? 8 : 1][kQL ? PP : 1];   // U_m V_m W_m, <d/dz> x3, <du/dy> <dw/dy>
  __shared__ T rsum[kQL ? 3 : 1][kQL ? PP : 1];

  const int tid = threadIdx.x;
  const int flat = xcd_logical(blockIdx.x, gridDim.x);
  const int E = a.E, K = a.K, My = a.My;
  const int slb = stage_block_log2(E);  // stage-buffer member blocks
  const int jl = flat / a.ec;
  const int j = a.j0 + jl, e = a.e0 + (flat - jl * a.ec);
  const VT* vel = static_cast<const VT*>(a.vel);
  const bool want_stats = a.psum != nullptr;
  const T kxs = T(a.kxs), kzs = T(a.kzs);

  for (int t = tid; t < MX; t += kNT) {
    T s, c;
    if constexpr (sizeof(T) == 8) sincospi(-2.0 * t / MX, &s, &c); else sincospif(-2.0f * t / MX, &s, &c);
    rootX[t] = C{c, s};
  }
  for (int t = tid; t < MZ; t += kNT) {
    T s, c;
    if constexpr (sizeof(T) == 8) sincospi(-2.0 * t / MZ, &s, &c); else sincospif(-2.0f * t / MZ, &s, &c);
    rootZ[t] = C{c, s};
  }
  __syncthreads();
  for (int t = tid; t < PP; t += kNT) rootP[t] = rootZ[t * R];
  __syncthreads();

  // spectral input element (field f, nx, stage slot iz) of this (j, e), as complex T
  auto vel_at = [&](int f, int nx, int iz) -> C {
    const size_t off = stage_off(size_t(f) * My + j, e, nx * NZ + iz, E, K, slb);
    return ldc<T>(vel + 2 * off);
  };

  // register accumulators of the forward transform: flat (f, stage-buffer position)
  C acc[Cfg::NACC];
#pragma unroll
  for (int k = 0; k < Cfg::NACC; ++k) acc[k] = C{T(0), T(0)};
  double s_uv = 0.0, s_wv = 0.0, s_uu = 0.0, s_vv = 0.0, s_ww = 0.0, s_grad = 0.0;

  for (int r = 0; r < R; ++r) {
    // ---- z inverse of NF spectral fields into zb[fi][q][nx] ----------------
    // The fold y[n'] = sum_a x[n' + PP a] e^{2 pi i (n' + PP a) r / Mz} is done
    // first, by the whole workgroup with consecutive threads on consecutive kz
    // (a short-stride run of the member-outer stage buffer), into zb[fi][n'][nx]; the
    // transform then reads LDS only and writes its output back to zb.
    // kind 0: fields fbase.. as stored; 1: times i kz; 2: the vorticity
    auto zinv = [&](auto nf_tag, int fbase, auto kind_tag) {
      constexpr int NF = decltype(nf_tag)::value;
      constexpr int kind = decltype(kind_tag)::value;
#pragma unroll 1
      for (int it = tid; it < NF * L * PP; it += kNT) {
        const int np = it % PP;
        const int rest = it / PP;
        const int nx = rest % L, fi = rest / L;
        C acc_f{T(0), T(0)};
#pragma unroll
        for (int fold = 0; fold < R; ++fold) {
          const int n = np + PP * fold;
          int nz;
          if (n < P) nz = n;
          else if (n > MZ - P) nz = n - MZ;
          else continue;
          const int izs = stage_slot(nz);
          C x;
          if constexpr (kind == 2) {
            const T kz = kzs * T(nz), kx = kxs * T(nx);
            if (fi == 0) {         // dw/dy - i kz v
              const C vv = vel_at(1, nx, izs), wy = vel_at(4, nx, izs);
              x = C{wy.x + kz * vv.y, wy.y - kz * vv.x};
            } else if (fi == 1) {  // i (kz u - kx w)
              const C uu = vel_at(0, nx, izs), ww = vel_at(2, nx, izs);
              x = cmuli<1>(C{kz * uu.x - kx * ww.x, kz * uu.y - kx * ww.y});
            } else {               // i kx v - du/dy
              const C vv = vel_at(1, nx, izs), uy = vel_at(3, nx, izs);
              x = C{-kx * vv.y - uy.x, kx * vv.x - uy.y};
            }
          } else {
            x = vel_at(fbase + fi, nx, izs);
            if constexpr (kind == 1) x = cmuli<1>(cscale(x, kzs * T(nz)));
          }
          acc_f = cadd(acc_f, cmul(x, cconj(rootZ[(n * r) % MZ])));
        }
        zb[(fi * PP + np) * Cfg::ZP + nx] = acc_f;
      }
      __syncthreads();
      auto load = [&](int b, int np) -> C {
        const int fi = b / L, nx = b - fi * L;
        return zb[(fi * PP + np) * Cfg::ZP + nx];
      };
      auto store = [&](int b, int q, C v) {
        const int fi = b / L, nx = b - fi * L;
        zb[(fi * PP + q) * Cfg::ZP + nx] = v;
      };
      fft2pass<T, PP, +1, NF * L, kNT, true>(mid, rootP, load, store);
    };
    // ---- x inverse of NF fields held in zb, rows paired (q, q + PH) -------
    auto xinv = [&](auto nf_tag, bool dx, auto action) {
      constexpr int NF = decltype(nf_tag)::value;
      auto load = [&](int b, int n) -> C {
        const int fi = b / PH, qp = b - fi * PH;
        const C* col = zb + fi * PP * Cfg::ZP;
        auto cval = [&](int nx, int q) -> C {
          C c = col[q * Cfg::ZP + nx];
          if (dx) c = cmuli<1>(cscale(c, kxs * T(nx)));
          return c;
        };
        if (n == 0) {
          if (dx) return C{T(0), T(0)};
          return C{col[qp * Cfg::ZP].x, col[(PH + qp) * Cfg::ZP].x};
        }
        if (n < L) {
          const C c0 = cval(n, qp), c1 = cval(n, qp + PH);
          return C{c0.x - c1.y, c0.y + c1.x};
        }
        if (n > MX - L) {
          const C c0 = cconj(cval(MX - n, qp)), c1 = cconj(cval(MX - n, qp + PH));
          return C{c0.x - c1.y, c0.y + c1.x};
        }
        return C{T(0), T(0)};
      };
      auto store = [&](int b, int n, C v) {
        const int fi = b / PH, qp = b - fi * PH;
        action(fi, qp * Cfg::MXP + n, v.x);
        action(fi, (qp + PH) * Cfg::MXP + n, v.y);
      };
      fft2pass<T, MX, +1, NF * PH, kNT>(mid, rootX, load, store);
    };
    std::integral_constant<int, 3> three;
    std::integral_constant<int, 2> two;
    std::integral_constant<int, 0> plain;
    std::integral_constant<int, 1> dz;
    std::integral_constant<int, 2> vort;

    // quasi-linear form: row means of NF fields from the n_x = 0 entries of zb
    auto keep_row_means = [&](int nf, int slot) {
      if constexpr (kQL) {
        for (int t = tid; t < nf * PP; t += kNT) {
          const int fi = t / PP, q = t - fi * PP;
          rmean[slot + fi][q] = zb[(fi * PP + q) * Cfg::ZP].x;
        }
        __syncthreads();
      }
    };

    zinv(three, 0, plain);
    __syncthreads();
    keep_row_means(3, 0);
    xinv(three, false, [&](int fi, int p, T val) { phys[PU + fi][p] = val; });
    __syncthreads();
    if constexpr (kRot) {
      zinv(three, 0, vort);
      __syncthreads();
      xinv(three, false, [&](int fi, int p, T val) {
        phys[PNU + fi][p] = val;
        if (want_stats) s_grad += double(val) * double(val);
      });
      __syncthreads();
      for (int pl = tid; pl < Cfg::NPT; pl += kNT) {
        const int q = pl / MX;
        const int p = q * Cfg::MXP + (pl - q * MX);
        const T u = phys[PU][p], v = phys[PV][p], w = phys[PW][p];
        const T ox = phys[PNU][p], oy = phys[PNV][p], oz = phys[PNW][p];
        phys[PNU][p] = oy * w - oz * v;
        phys[PNV][p] = oz * u - ox * w;
        phys[PNW][p] = ox * v - oy * u;
        s_uv += double(u) * double(v);
        s_wv += double(w) * double(v);
        if (want_stats) {
          s_uu += double(u) * double(u);
          s_vv += double(v) * double(v);
          s_ww += double(w) * double(w);
        }
      }
    } else {
    xinv(three, true, [&](int fi, int p, T val) {
      const T u = phys[PU][p];
      if constexpr (kQL) lin[fi][p] = (kAdj ? -rmean[0][p / Cfg::MXP] : rmean[0][p / Cfg::MXP]) * val;
      if (fi == 0) {
        phys[PNU][p] = u * val;
        phys[PVY][p] = -val;
      } else if (fi == 1) {
        phys[PNV][p] = u * val;
      } else {
        phys[PNW][p] = u * val;
      }
      if (want_stats) s_grad += double(val) * double(val);
    });
    __syncthreads();
    zinv(three, 0, dz);
    __syncthreads();
    keep_row_means(3, 3);
    xinv(three, false, [&](int fi, int p, T val) {
      const T w = phys[PW][p];
      if constexpr (kQL) {
        const int q = p / Cfg::MXP;
        const T Wm = rmean[2][q], Zm = rmean[3 + fi][q];
        if constexpr (kAdj) lin[fi][p] -= Wm * (val - Zm);
        else lin[fi][p] += Wm * (val - Zm) + (w - Wm) * Zm;
      }
      if (fi == 0) {
        phys[PNU][p] += w * val;
      } else if (fi == 1) {
        phys[PNV][p] += w * val;
      } else {
        phys[PNW][p] += w * val;
        phys[PVY][p] -= val;
      }
      if (want_stats) s_grad += double(val) * double(val);
    });
    __syncthreads();
    zinv(two, 3, plain);
    __syncthreads();
    keep_row_means(2, 6);
    xinv(two, false, [&](int fi, int p, T val) {
      const T v = phys[PV][p];
      if constexpr (kQL) {
        const int q = p / Cfg::MXP;
        const T Vm = rmean[1][q], Ym = rmean[6 + fi][q];
        if constexpr (kAdj) lin[fi == 0 ? 0 : 2][p] -= Vm * (val - Ym);
        else lin[fi == 0 ? 0 : 2][p] += Vm * (val - Ym) + (v - Vm) * Ym;
      }
      if (fi == 0) phys[PNU][p] += v * val; else phys[PNW][p] += v * val;
      if (want_stats) s_grad += double(val) * double(val);
    });
    __syncthreads();
    for (int pl = tid; pl < Cfg::NPT; pl += kNT) {
      const int q = pl / MX;
      const int p = q * Cfg::MXP + (pl - q * MX);
      const T u = phys[PU][p], v = phys[PV][p], w = phys[PW][p], vy = phys[PVY][p];
      phys[PNV][p] += v * vy;
      if constexpr (kQL) {  // <dv/dy> = -<dw/dz> by continuity (<du/dx> = 0)
        const T Vm = rmean[1][q], Ym = -rmean[5][q];
        if constexpr (kAdj) {
          const T up = u - rmean[0][q], vp = v - Vm, wp = w - rmean[2][q];
          lin[1][p] += -Vm * (vy - Ym) + up * rmean[6][q] + vp * Ym + wp * rmean[7][q];
          lin[2][p] += up * rmean[3][q] + vp * rmean[4][q] + wp * rmean[5][q];
        } else {
          lin[1][p] += Vm * (vy - Ym) + (v - Vm) * Ym;
        }
      }
      s_uv += double(u) * double(v);
      s_wv += double(w) * double(v);
      if (want_stats) {
        s_uu += double(u) * double(u);
        s_vv += double(v) * double(v);
        s_ww += double(w) * double(w);
        s_grad += double(vy) * double(vy);
      }
    }
    }  // advective form
    __syncthreads();
    if constexpr (kQL) {
      static_assert(MX <= 128, "row sums take at most two values per lane");
      // row sums of the full products, one wavefront per row, fixed order
      const int lane = tid & 63, wvi = tid >> 6;
      for (int rr = wvi; rr < 3 * PP; rr += kNT / 64) {
        const int i = rr / PP, q = rr - i * PP;
        const T* row = &phys[PNU + i][q * Cfg::MXP];
        T x = lane < MX ? row[lane] : T(0);
        if (lane + 64 < MX) x += row[lane + 64];
        x = wave_sum(x);
        if (lane == 0) rsum[i][q] = x;
      }
      __syncthreads();
      for (int pl = tid; pl < Cfg::NPT; pl += kNT) {
        const int q = pl / MX;
        const int p = q * Cfg::MXP + (pl - q * MX);
#pragma unroll
        for (int i = 0; i < 3; ++i) phys[PNU + i][p] = lin[i][p] + rsum[i][q] * (T(1) / T(MX));
      }
      __syncthreads();
    }
    // ---- forward x transform of (Nu, Nv, Nw); keep |kx| < L ----------------
    {
      auto load = [&](int b, int n) -> C {
        const int f = b / PH, qp = b - f * PH;
        return C{phys[PNU + f][qp * Cfg::MXP + n], phys[PNU + f][(qp + PH) * Cfg::MXP + n]};
      };
      auto store = [&](int b, int k, C v) {
        if (k < L) zb[b * Cfg::FP + k] = v;
        else if (k > MX - L) zb[b * Cfg::FP + k - MX + 2 * L] = v;
      };
      fft2pass<T, MX, -1, 3 * PH, kNT>(mid, rootX, load, store);
    }
    __syncthreads();
    // ---- forward z transform of the chunk (unpacking the row pairs) ------------
    {
      auto load = [&](int b, int q) -> C {
        const int f = b / L, nx = b - f * L;
        const int qp = q < PH ? q : q - PH;
        const C* row = zb + (f * PH + qp) * Cfg::FP;
        const C zk = row[nx];
        const C zm = cconj(row[nx == 0 ? 0 : 2 * L - nx]);
        if (q < PH) return C{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y + zm.y)};
        // (zk - zm) / (2 i)
        return C{T(0.5) * (zk.y - zm.y), T(-0.5) * (zk.x - zm.x)};
      };
      // Y is written to zb after pass 1 has consumed it (pass 2 reads only mid)
      auto storeY = [&](int b, int k, C v) { zb[b * Cfg::PPP + k] = v; };
      fft2pass<T, PP, -1, 3 * L, kNT, true>(mid, rootP, load, storeY);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < Cfg::NACC; ++k) {
      const int idx = tid + k * kNT;
      if (idx < 3 * L * NZ) {
        const int f = idx / (L * NZ);
        const int rem = idx - f * L * NZ;
        const int nx = rem / NZ;
        const int nz = stage_kz(rem - nx * NZ);  // rem: the mode's stage-buffer position
        const int kk = ((nz % PP) + PP) % PP;
        const int t = (((r * nz) % MZ) + MZ) % MZ;
        acc[k] = cadd(acc[k], cmul(zb[(f * L + nx) * Cfg::PPP + kk], rootZ[t]));
      }
    }
    __syncthreads();
  }

  // ---- write the truncated advection spectrum --------------------------------
  VT* nl = static_cast<VT*>(a.nl);
  const T inv = T(1.0 / (double(MX) * double(MZ)));
#pragma unroll
  for (int k = 0; k < Cfg::NACC; ++k) {
    const int idx = tid + k * kNT;
    if (idx < 3 * L * NZ) {
      const int f = idx / (L * NZ);
      const int m = idx - f * L * NZ;
      const size_t off = stage_off(size_t(f) * My + j, e, m, E, K, slb);
      stc<T>(nl + 2 * off, cscale(acc[k], inv));
    }
  }

  // ---- plane means (fixed-order reductions) -------------------------------------
  const double vals[6] = {s_uv, s_wv, s_uu, s_vv, s_ww, s_grad};
  const int nq = want_stats ? 6 : 2;
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int qi = 0; qi < 6; ++qi) {
    if (qi < nq) {
      const double sred = wave_sum(vals[qi]);
      if (lane == 0) red[qi][wv] = sred;
    }
  }
  __syncthreads();
  if (tid == 0) {
    const double norm = 1.0 / (double(MX) * double(MZ));
    double tot[6];
    for (int qi = 0; qi < nq; ++qi) {
      double s = 0.0;
      for (int w = 0; w < kNT / 64; ++w) s += red[qi][w];
      tot[qi] = s * norm;
    }
    a.means[(size_t(0) * My + j) * E + e] = tot[0];
    a.means[(size_t(1) * My + j) * E + e] = tot[1];
    if (want_stats) {
      a.psum[(size_t(PS_UU) * My + j) * E + e] = tot[2];
      a.psum[(size_t(PS_VV) * My + j) * E + e] = tot[3];
      a.psum[(size_t(PS_WW) * My + j) * E + e] = tot[4];
      a.psum[(size_t(PS_GRAD) * My + j) * E + e] = tot[5];
    }
  }
}

// Chunk-row variants (PP) built for each precision and grid; index 0 is the
// default, the others are candidates for the tuner.  Every variant keeps the
// workgroup's LDS within 160 KB.
namespace {
constexpr int kVar64[6][3] = {{24, 12, 8}, {16, 24, 8}, {12, 8, 0}, {16, 12, 8}, {18, 12, 0}, {8, 0, 0}};
constexpr int kVar32[6][3] = {{24, 12, 8}, {16, 24, 48}, {12, 24, 36}, {32, 24, 16}, {36, 18, 12}, {16, 12, 8}};
int grid_index(int Nx) {
  return Nx == 16 ? 0 : Nx == 32 ? 1 : Nx == 48 ? 2 : Nx == 64 ? 3 : Nx == 72 ? 4 : Nx == 96 ? 5 : -1;
}

template <typename T, int L, int PP, int Form>
constexpr bool variant_built() {
  constexpr int gi = L == 8 ? 0 : L == 16 ? 1 : L == 24 ? 2 : L == 32 ? 3 : L == 36 ? 4 : L == 48 ? 5 : -1;
  if constexpr (gi < 0 || (3 * L) % PP != 0 || (Form >= 2 && 3 * L > 128)) {
    return false;  // (the quasi-linear row sums take at most two values per lane)
  } else {
    using Cfg = PlaneCfg<T, L, L, PP>;
    const size_t extra = Form >= 2 ? (3 * Cfg::NPTS + 11 * PP) * sizeof(T) : 0;
    if (Cfg::kLdsBytes + extra > 160 * 1024) return false;
    for (int v = 0; v < 3; ++v)
      if ((sizeof(T) == 8 ? kVar64 : kVar32)[gi][v] == PP) return true;
    return false;
  }
}

template <typename T, int L, int PP, int Form>
const void* plane_fn_if_built() {
  if constexpr (variant_built<T, L, PP, Form>())
    return reinterpret_cast<const void*>(&plane_kernel<T, T, L, L, PP, Form>);
  return nullptr;
}

template <typename T, int L, int Form>
const void* plane_fn_rows(int pp) {
  switch (pp) {
    case 8: return plane_fn_if_built<T, L, 8, Form>();
    case 12: return plane_fn_if_built<T, L, 12, Form>();
    case 16: return plane_fn_if_built<T, L, 16, Form>();
    case 18: return plane_fn_if_built<T, L, 18, Form>();
    case 24: return plane_fn_if_built<T, L, 24, Form>();
    case 32: return plane_fn_if_built<T, L, 32, Form>();
    case 36: return plane_fn_if_built<T, L, 36, Form>();
    case 48: return plane_fn_if_built<T, L, 48, Form>();
  }
  return nullptr;
}

template <typename T, int Form>
const void* plane_fn_grid(int Nx, int pp) {
  switch (Nx) {
    case 16: return plane_fn_rows<T, 8, Form>(pp);
    case 32: return plane_fn_rows<T, 16, Form>(pp);
    case 48: return plane_fn_rows<T, 24, Form>(pp);
    case 64: return plane_fn_rows<T, 32, Form>(pp);
    case 72: return plane_fn_rows<T, 36, Form>(pp);
    case 96: return plane_fn_rows<T, 48, Form>(pp);
  }
  return nullptr;
}

template <typename T>
const void* plane_fn_t(int form, int Nx, int pp) {
  switch (form) {
    case 0: return plane_fn_grid<T, 0>(Nx, pp);
    case 1: return plane_fn_grid<T, 1>(Nx, pp);
    case 2: return plane_fn_grid<T, 2>(Nx, pp);
    case 3: return plane_fn_grid<T, 3>(Nx, pp);
  }
  return nullptr;
}

// The kernel of (precision, form, grid, chunk rows); nullptr if not built.
const void* plane_fn(int precision, int form, int Nx, int pp) {
  return precision == 0 ? plane_fn_t<double>(form, Nx, pp) : plane_fn_t<float>(form, Nx, pp);
}

// chunk-row counts of the table row for (precision, Nx), built or not
int table_rows(int precision, int Nx, int* rows) {
  const int gi = grid_index(Nx);
  if (gi < 0) return 0;
  const int(*tab)[3] = precision == 0 ? kVar64 : kVar32;
  int n = 0;
  for (int v = 0; v < 3; ++v)
    if (tab[gi][v]) rows[n++] = tab[gi][v];
  return n;
}
}  // namespace

// Grids with an advective-form variant: the general kernel's square grids,
// and the lane-parallel kernel's (square or not).
bool plane_supported(int Nx, int Nz) {
  int rows[kMaxPlaneVariants];
  return plane_variants(1, 0, Nx, Nz, rows) > 0;
}

// Resolve every built plane-kernel variant of grid Nx (both precisions, every
// form) on the current device, so that a later graph capture never holds a
// kernel's first launch.
hipError_t plane_preload(int Nx, int Nz) {
  for (int prec = 0; prec < 2; ++prec) {
    for (int form = 0; form < kPlaneForms; ++form) {
      int rows[kMaxPlaneVariants];
      const int n = plane_variants(prec, form, Nx, Nz, rows);  // 0: this form does not fit this grid
      for (int v = 0; v < n; ++v) {
        const void* fn = rows[v] > kWaveRows ? plane_wave_fn(prec, Nx, Nz, rows[v] - kWaveRows)
                                             : plane_fn(prec, form, Nx, rows[v]);
        if (!fn) return hipErrorInvalidValue;
        hipFuncAttributes attr;
        const hipError_t err = hipFuncGetAttributes(&attr, fn);
        if (err != hipSuccess) return err;
      }
    }
  }
  return hipSuccess;
}

// The lane-parallel advective variants first (advective form, grids with a
// power-of-two Nx/2), then the table's variants that are built for this form
// (the quasi-linear form needs more LDS and drops the largest chunks).
int plane_variants(int precision, int form, int Nx, int Nz, int* rows) {
  int n = 0;
  if (form == 0) {
    int wave[6];
    const int nw = plane_wave_rows(precision, Nx, Nz, wave);
    for (int v = 0; v < nw; ++v) rows[n++] = kWaveRows + wave[v];
  }
  if (Nx != Nz) return n;  // the general kernel is built for square grids
  int all[3];
  const int n_all = table_rows(precision, Nx, all);
  for (int v = 0; v < n_all; ++v)
    if (plane_fn(precision, form, Nx, all[v])) rows[n++] = all[v];
  return n;
}

// precision 0: FP64 storage and arithmetic; 1: FP32 storage and FFT arithmetic.
// form 0: advective u . grad u; 1: rotational omega x u; 2: quasi-linear advective;
// 3: adjoint of the quasi-linear advection.
hipError_t launch_plane(int precision, int form, int Nx, int Nz, int variant, const PlaneArgs& a,
                        hipStream_t s) {
  if (!plane_supported(Nx, Nz) || form < 0 || form >= kPlaneForms) return hipErrorInvalidValue;
  int rows[kMaxPlaneVariants];
  const int n = plane_variants(precision, form, Nx, Nz, rows);
  if (variant < 0 || variant >= n) return hipErrorInvalidValue;
  const bool wave = rows[variant] > kWaveRows;
  const void* fn = wave ? plane_wave_fn(precision, Nx, Nz, rows[variant] - kWaveRows)
                        : plane_fn(precision, form, Nx, rows[variant]);
  if (!fn) return hipErrorInvalidValue;
  const int nt = wave ? plane_wave_threads(Nx, rows[variant] - kWaveRows) : kNT;
  void* args[] = {const_cast<PlaneArgs*>(&a)};
  const hipError_t err = hipLaunchKernel(fn, dim3(a.nj * a.ec), dim3(nt), args, 0, s);
  return err != hipSuccess ? err : hipGetLastError();
}

}  // namespace dns
