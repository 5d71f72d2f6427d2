// Pseudo-spectral advection stage with lane-parallel x transforms: one
// workgroup per (Chebyshev plane j, member e), advective form u . grad u_i
// (paper Sec. 3.1-3.2: products on the 3/2-padded physical grid, the 2/3-rule
// truncation of their x-z transform, and the plane means <uv>, <wv> of the
// mean-flow equations (U00), (W00)).  It computes what plane_kernel computes
// for the advective form (kernels_plane.hip) with a different organisation,
// built for grids whose Nx/2 is a power of two.
//
// The physical plane (Mz x Mx, Mx = 3L with L = Nx/2) is processed in R chunks
// of PP z rows p = R q + r, as in plane_kernel.  Per chunk:
//   fold  : the five stage fields u, v, w, du/dy, dw/dy are folded onto PP
//           points, y_f[nx][n'] = sum_a X_f[nx][n' + PP a] e^{2 pi i n r/Mz}
//           (n = n' + PP a), with i kz applied on the way for du/dz, dv/dz,
//           dw/dz -- eight columns per kx, coalesced loads, into LDS;
//   z     : each column's PP-point inverse transform, S = PP/16 threads per
//           column (a radix-S split, then a 16-point DFT in registers), the
//           rows written to LDS in (field, row, kx) order;
//   x     : each row pair (q, q + PP/2) is owned by a group of L lanes, each
//           lane holding three complex points of a 3L-point complex transform
//           (real part row q, imaginary part row q + PP/2): a radix-3 step in
//           registers, then log2 L radix-2 steps across the lanes (DPP and
//           ds_swizzle exchanges, no LDS traffic, no workgroup barrier).  The
//           eleven inverse transforms (u, v, w and their x, z, y derivatives,
//           dv/dy = -(du/dx + dw/dz) by continuity) leave every physical value
//           in the lane that forms the products, so u . grad u_i and the plane
//           sums are accumulated in registers; the forward x transforms of the
//           three products run the same network backwards and the kept
//           |kx| < L modes go to LDS;
//   zf    : the PP-point forward transform of each (product, kx) column
//           (radix-S split, 16-point DFT in registers), then every thread adds
//           its share of N_hat(nz) += e^{-2 pi i r nz/Mz} Y_r[nz mod PP] in
//           registers.
// Six workgroup barriers per chunk.  The lane of row-pair lane l holds the
// physical points x = n1 + 3 bitrev(l), n1 < 3.
#include "fft.h"
#include "internal.h"

namespace dns {

namespace {

__device__ __forceinline__ int xcd_remap(int b, int nblk) {
  const int q = nblk >> 3, rem = nblk & 7;
  const int x = b & 7, local = b >> 3;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + local;
}

// value of lane (l ^ MASK), MASK < 32: DPP quad permutes for 1 and 2, a
// ds_swizzle bit-mask permute (within 32-lane halves) otherwise
template <int MASK>
__device__ __forceinline__ int lane_xor_i(int v) {
  static_assert(MASK == 1 || MASK == 2 || MASK == 4 || MASK == 8 || MASK == 16, "xor mask");
  if constexpr (MASK == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
  else if constexpr (MASK == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
  else return __builtin_amdgcn_ds_swizzle(v, 0x1F | (MASK << 10));
}
template <int MASK>
__device__ __forceinline__ float lane_xor(float v) {
  return __int_as_float(lane_xor_i<MASK>(__float_as_int(v)));
}
template <int MASK>
__device__ __forceinline__ double lane_xor(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_xor_i<MASK>(int(b & 0xffffffffLL)), hi = lane_xor_i<MASK>(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

template <typename T, typename VT>
__device__ __forceinline__ cx<T> ld2(const VT* p) {
  if constexpr (sizeof(VT) == 8) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    return cx<T>{T(v.x), T(v.y)};
  } else {
    const float2 v = *reinterpret_cast<const float2*>(p);
    return cx<T>{T(v.x), T(v.y)};
  }
}

template <typename T, typename VT>
__device__ __forceinline__ void st2(VT* p, cx<T> c) {
  if constexpr (sizeof(VT) == 8) {
    *reinterpret_cast<double2*>(p) = double2{double(c.x), double(c.y)};
  } else {
    *reinterpret_cast<float2*>(p) = float2{float(c.x), float(c.y)};
  }
}

template <typename V>
__device__ __forceinline__ V wsum(V v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int L>
constexpr int log2i() {
  int s = 0;
  while ((1 << s) < L) ++s;
  return s;
}

template <typename T, int L, int P, int PP>
struct WaveCfg {
  static constexpr int MX = 3 * L, MZ = 3 * P, NZ = 2 * P - 1, K = L * NZ;
  static constexpr int R = MZ / PP, PH = PP / 2, S = PP / 16;
  static constexpr int NT = PH * L;                 // one lane per (row pair, l)
  static constexpr int LOGL = log2i<L>();
  static constexpr int ZYP = PP + 1;                // fold output [f][nx][n'] pitch
  static constexpr int ZP = L + 1;                  // z output rows [f][q][nx] pitch
  static constexpr int FP = 2 * L + 1;              // forward x rows [f][qp][k] pitch
  static constexpr int YP = PP + 1;                 // forward z output [f][nx][k] pitch
  static constexpr int AZY = 8 * L * ZYP, AZB = 8 * PP * ZP, AZF = 3 * PH * FP, AY = 3 * L * YP;
  static constexpr int A = AZY > AZB ? (AZY > AZF + AY ? AZY : AZF + AY) : (AZB > AZF + AY ? AZB : AZF + AY);
  static constexpr int NM = (K + NT - 1) / NT;      // kept modes per thread
  static constexpr int NACC = 3 * NM;               // (field, mode) accumulators per thread
  static constexpr size_t kLdsBytes = size_t(A + MX + MZ) * 2 * sizeof(T) + 6 * (NT / 64) * sizeof(double);
  static_assert((L & (L - 1)) == 0 && L >= 8 && L <= 32, "row-pair lanes: a power of two, 8..32");
  static_assert(PP % 16 == 0 && MZ % PP == 0 && S >= 1 && S <= 3, "chunk rows: 16, 32 or 48 dividing Mz");
  static_assert(NT % 64 == 0 && NT <= 1024, "whole wavefronts");
};

// e^{sgn 2 pi i b c / S} for S <= 3
template <typename T, int S>
__device__ __forceinline__ cx<T> root_s(int bc, int sgn) {
  if constexpr (S == 1) {
    return cx<T>{T(1), T(0)};
  } else if constexpr (S == 2) {
    return cx<T>{(bc & 1) ? T(-1) : T(1), T(0)};
  } else {
    const int m = bc % 3;
    return m == 0 ? cx<T>{T(1), T(0)} : cx<T>{T(-0.5), T(sgn * (m == 1 ? 1 : -1) * 0.86602540378443864676373)};
  }
}

// One radix-2 exchange stage of span H across the lanes of a row-pair group,
// applied to the three values of the lane.
//   inverse (decimation in frequency): v <- (sgn v + v[l ^ H]) * tw
//   forward (decimation in time):      t = v * conj(tw); v <- sgn t + t[l ^ H]
// with sgn = -1, tw = e^{2 pi i (l mod H) / (2H)} in the upper lane of a pair
// and sgn = +1, tw = 1 in the lower one.  At span 1 the twiddle is 1 in every
// lane and is not applied.
template <typename T, int H>
__device__ __forceinline__ void stage_inv(cx<T>* v, cx<T> tw, T sgn) {
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    const T px = lane_xor<H>(v[n].x), py = lane_xor<H>(v[n].y);
    const cx<T> s{sgn * v[n].x + px, sgn * v[n].y + py};
    if constexpr (H == 1)
      v[n] = s;
    else
      v[n] = cmul(s, tw);
  }
}
template <typename T, int H>
__device__ __forceinline__ void stage_fwd(cx<T>* v, cx<T> tw, T sgn) {
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    cx<T> t = v[n];
    if constexpr (H != 1) t = cmul(t, cconj(tw));
    const T px = lane_xor<H>(t.x), py = lane_xor<H>(t.y);
    v[n] = cx<T>{sgn * t.x + px, sgn * t.y + py};
  }
}

template <typename T, int L, int S>
__device__ __forceinline__ void stages_inv(cx<T>* v, const cx<T>* tw, const T* sg) {
  if constexpr (S < log2i<L>()) {
    constexpr int H = L >> (S + 1);
    stage_inv<T, H>(v, tw[S], sg[S]);
    stages_inv<T, L, S + 1>(v, tw, sg);
  }
}
template <typename T, int L, int S>
__device__ __forceinline__ void stages_fwd(cx<T>* v, const cx<T>* tw, const T* sg) {
  if constexpr (S >= 0) {
    constexpr int H = L >> (S + 1);
    stage_fwd<T, H>(v, tw[S], sg[S]);
    stages_fwd<T, L, S - 1>(v, tw, sg);
  }
}

}  // namespace

template <typename T, typename VT, int L, int P, int PP, bool kGAcc>
__global__ void __launch_bounds__((PP / 2) * L) plane_wave_kernel(PlaneArgs a) {
  using C = cx<T>;
  using Cfg = WaveCfg<T, L, P, PP>;
  constexpr int MX = Cfg::MX, MZ = Cfg::MZ, NZ = Cfg::NZ, K = Cfg::K, R = Cfg::R, PH = Cfg::PH, S = Cfg::S;
  constexpr int NT = Cfg::NT, LOGL = Cfg::LOGL;
  __shared__ C lds[Cfg::A];
  __shared__ C rootX[MX];
  __shared__ C rootZ[MZ];
  __shared__ double red[6][NT / 64];

  const int tid = threadIdx.x;
  const int flat = xcd_remap(blockIdx.x, gridDim.x);
  const int E = a.E, My = a.My;
  const int slb = stage_block_log2(E);  // stage-buffer member blocks
  const int jl = flat / a.ec;
  const int j = a.j0 + jl, e = a.e0 + (flat - jl * a.ec);
  const VT* vel = static_cast<const VT*>(a.vel);
  const bool want_stats = a.psum != nullptr;
  const T kxs = T(a.kxs), kzs = T(a.kzs);

  for (int t = tid; t < MX; t += NT) {
    T s, c;
    if constexpr (sizeof(T) == 8) sincospi(-2.0 * t / MX, &s, &c); else sincospif(-2.0f * t / MX, &s, &c);
    rootX[t] = C{c, s};
  }
  for (int t = tid; t < MZ; t += NT) {
    T s, c;
    if constexpr (sizeof(T) == 8) sincospi(-2.0 * t / MZ, &s, &c); else sincospif(-2.0f * t / MZ, &s, &c);
    rootZ[t] = C{c, s};
  }
  if (tid < 6 * (NT / 64)) (&red[0][0])[tid] = 0.0;
  __syncthreads();

  const int lane0 = tid % L, qp = tid / L;
  constexpr T c3 = T(-0.5), s3 = T(0.86602540378443864676373);  // e^{2 pi i/3}

  // forward-z sums: in registers, or (kGAcc) in the output buffer itself,
  // read back and updated by the same thread in every chunk
  constexpr int NACC = kGAcc ? 1 : Cfg::NACC;
  C acc[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = C{T(0), T(0)};
  VT* const nl = static_cast<VT*>(a.nl);
  const T inv = T(1.0 / (double(MX) * double(MZ)));

  C* const zy = lds;                 // fold output   [f][nx][n']
  C* const zb = lds;                 // z output rows [f][q][nx]
  C* const zf = lds;                 // forward x     [f][qp][k]
  C* const Yb = lds + Cfg::AZF;      // forward z     [f][nx][k]

  for (int r = 0; r < R; ++r) {
    // ---- fold of the five stage fields (eight columns per kx) ----------------
#pragma unroll 1
    for (int it = tid; it < 5 * L * PP; it += NT) {
      const int np = it % PP;
      const int rest = it / PP;
      const int nx = rest % L, src = rest / L;
      C y0{T(0), T(0)}, y1{T(0), T(0)};
      const VT* col = vel + 2 * stage_off(size_t(src) * My + j, e, nx * NZ, E, K, slb);
#pragma unroll
      for (int fa = 0; fa < R; ++fa) {
        const int n = np + PP * fa;
        int nz;
        if (n < P) nz = n;
        else if (n > MZ - P) nz = n - MZ;
        else continue;
        const C x = ld2<T>(col + (2 * stage_slot(nz) << slb));
        const C xt = cmul(x, cconj(rootZ[(n * r) % MZ]));
        y0 = cadd(y0, xt);
        if (src < 3) y1 = cadd(y1, cmuli<1>(cscale(xt, kzs * T(nz))));
      }
      const int f0 = src < 3 ? src : src + 3;   // u v w | uy wy -> 0 1 2 | 6 7
      zy[(f0 * L + nx) * Cfg::ZYP + np] = y0;
      if (src < 3) zy[((src + 3) * L + nx) * Cfg::ZYP + np] = y1;   // uz vz wz -> 3 4 5
    }
    __syncthreads();
    // ---- PP-point inverse z transform of each column -------------------------
    {
      const int nx = tid % L, c = (tid / L) % S, f = tid / (L * S);
      const C* colp = zy + (f * L + nx) * Cfg::ZYP;
      C z[16];
#pragma unroll
      for (int n = 0; n < 16; ++n) {
        C s = colp[n];
#pragma unroll
        for (int b = 1; b < S; ++b) s = cadd(s, cmul(colp[n + 16 * b], root_s<T, S>(b * c, 1)));
        z[n] = (c == 0 || n == 0) ? s : cmul(s, cconj(rootZ[(n * c * R) % MZ]));
      }
      SmallDft<T, 16, 1>::run(z);
      __syncthreads();
#pragma unroll
      for (int qq = 0; qq < 16; ++qq) zb[(f * PP + S * qq + c) * Cfg::ZP + nx] = z[qq];
    }
    __syncthreads();
    // ---- x transforms of the row pair (qp, qp + PH), products ------------------
    {
      // The lane constants are rebuilt in every chunk (the empty asm keeps the
      // compiler from holding them in registers across the other phases).
      int lane = lane0;
      asm volatile("" : "+v"(lane));
      // row-pair lane constants: radix-3 twiddles e^{2 pi i n1 l / Mx} and the
      // exchange-stage twiddles and signs (stage s has span L >> (s + 1))
      const C tw1 = cconj(rootX[lane]), tw2 = cconj(rootX[2 * lane]);
      C stw[LOGL];
      T ssg[LOGL];
#pragma unroll
      for (int s = 0; s < LOGL; ++s) {
        const int H = L >> (s + 1);
        const bool upper = (lane & H) != 0;
        stw[s] = upper ? cconj(rootX[(lane % H) * (MX / (2 * H))]) : C{T(1), T(0)};
        ssg[s] = upper ? T(-1) : T(1);
      }
      const T kxa = kxs * T(lane), kxb = kxs * T(L - lane);
      const int lane2 = lane == 0 ? 0 : L - lane;   // conjugate partner column
      const T nz0 = lane == 0 ? T(0) : T(1);

      // inverse transform of field f (dx: times i kx) into this lane's 3 points
      auto xinv = [&](int f, bool dx, C* v) {
        const C* ra = zb + (f * PP + qp) * Cfg::ZP;
        const C* rb = ra + PH * Cfg::ZP;
        // lane 0 (kx = 0) takes the real parts only and has no conjugate
        // partner: the 0/1 factor nz0 masks it without a branch
        C p = ra[lane], q = rb[lane], p2 = ra[lane2], q2 = rb[lane2];
        if (dx) {
          p = cmuli<1>(cscale(p, kxa));
          q = cmuli<1>(cscale(q, kxa));
          p2 = cmuli<1>(cscale(p2, kxb));
          q2 = cmuli<1>(cscale(q2, kxb));
        }
        const C x0 = C{p.x - nz0 * q.y, nz0 * p.y + q.x};            // p + i q
        const C x2 = C{nz0 * (p2.x + q2.y), nz0 * (q2.x - p2.y)};    // conj(p2) + i conj(q2)
        // radix 3 with a zero middle input: Y[n1] = x0 + w3^{2 n1} x2, with
        // w3^{2}, w3^{4} = c3 -/+ i s3 sharing x0 + c3 x2 and s3 x2
        v[0] = cadd(x0, x2);
        const C m{x0.x + c3 * x2.x, x0.y + c3 * x2.y};
        const T sx = s3 * x2.x, sy = s3 * x2.y;
        v[1] = cmul(C{m.x + sy, m.y - sx}, tw1);
        v[2] = cmul(C{m.x - sy, m.y + sx}, tw2);
        stages_inv<T, L, 0>(v, stw, ssg);
      };
      // forward transform of this lane's 3 points; kept modes kx = lane and
      // the index 2L + lane (kx = lane - L) go to zf[f][qp][lane], [L + lane]
      auto xfwd = [&](int f, C* v) {
        stages_fwd<T, L, LOGL - 1>(v, stw, ssg);
        const C y0 = v[0], y1 = cmul(v[1], cconj(tw1)), y2 = cmul(v[2], cconj(tw2));
        const C o0 = cadd(cadd(y0, y1), y2);
        // y1 w3 + y2 w3^{-1} = c3 (y1 + y2) + i s3 (y1 - y2)
        const C sp = cadd(y1, y2), dm = csub(y1, y2);
        const C o2{y0.x + c3 * sp.x - s3 * dm.y, y0.y + c3 * sp.y + s3 * dm.x};
        C* row = zf + (f * PH + qp) * Cfg::FP;
        row[lane] = o0;
        row[L + lane] = o2;
      };
      auto prod = [](C a, C b) { return C{a.x * b.x, a.y * b.y}; };
      auto sq = [](C a) { return a.x * a.x + a.y * a.y; };
      C U[3], V[3], W[3], NU[3], NV[3], NW[3], VY[3], t[3];
      T g = T(0);
      __builtin_amdgcn_sched_barrier(0);
      xinv(0, false, U);
      __builtin_amdgcn_sched_barrier(0);
      xinv(1, false, V);
      __builtin_amdgcn_sched_barrier(0);
      xinv(2, false, W);
      __builtin_amdgcn_sched_barrier(0);
      xinv(0, true, t);
#pragma unroll
      for (int n = 0; n < 3; ++n) NU[n] = prod(U[n], t[n]), VY[n] = C{-t[n].x, -t[n].y}, g += sq(t[n]);
      __builtin_amdgcn_sched_barrier(0);
      xinv(1, true, t);
#pragma unroll
      for (int n = 0; n < 3; ++n) NV[n] = prod(U[n], t[n]), g += sq(t[n]);
      __builtin_amdgcn_sched_barrier(0);
      xinv(2, true, t);
#pragma unroll
      for (int n = 0; n < 3; ++n) NW[n] = prod(U[n], t[n]), g += sq(t[n]);
      __builtin_amdgcn_sched_barrier(0);
      xinv(3, false, t);
#pragma unroll
      for (int n = 0; n < 3; ++n) NU[n] = cadd(NU[n], prod(W[n], t[n])), g += sq(t[n]);
      __builtin_amdgcn_sched_barrier(0);
      xinv(4, false, t);
#pragma unroll
      for (int n = 0; n < 3; ++n) NV[n] = cadd(NV[n], prod(W[n], t[n])), g += sq(t[n]);
      __builtin_amdgcn_sched_barrier(0);
      xinv(5, false, t);
#pragma unroll
      for (int n = 0; n < 3; ++n) NW[n] = cadd(NW[n], prod(W[n], t[n])), VY[n] = csub(VY[n], t[n]), g += sq(t[n]);
      __builtin_amdgcn_sched_barrier(0);
      xinv(6, false, t);
#pragma unroll
      for (int n = 0; n < 3; ++n) NU[n] = cadd(NU[n], prod(V[n], t[n])), g += sq(t[n]);
      __builtin_amdgcn_sched_barrier(0);
      xinv(7, false, t);
#pragma unroll
      for (int n = 0; n < 3; ++n) NW[n] = cadd(NW[n], prod(V[n], t[n])), g += sq(t[n]);
      T suv = T(0), swv = T(0), suu = T(0), svv = T(0), sww = T(0);
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        NV[n] = cadd(NV[n], prod(V[n], VY[n]));
        g += sq(VY[n]);
        suv += U[n].x * V[n].x + U[n].y * V[n].y;
        swv += W[n].x * V[n].x + W[n].y * V[n].y;
        suu += sq(U[n]);
        svv += sq(V[n]);
        sww += sq(W[n]);
      }
      // the products and sums are complete before the barrier (the empty asm
      // keeps the compiler from deferring their arithmetic past it, which
      // would hold the loaded spectra in registers)
#pragma unroll
      for (int n = 0; n < 3; ++n)
        asm volatile("" : "+v"(NU[n].x), "+v"(NU[n].y), "+v"(NV[n].x), "+v"(NV[n].y), "+v"(NW[n].x), "+v"(NW[n].y));
      asm volatile("" : "+v"(suv), "+v"(swv), "+v"(suu), "+v"(svv), "+v"(sww), "+v"(g));
      __syncthreads();   // every lane has read zb before zf overwrites it
      __builtin_amdgcn_sched_barrier(0);
      xfwd(0, NU);
      __builtin_amdgcn_sched_barrier(0);
      xfwd(1, NV);
      __builtin_amdgcn_sched_barrier(0);
      xfwd(2, NW);
      // this chunk's plane sums, one fixed-order wavefront sum each
      const int wl = tid & 63, wv = tid >> 6;
      const T vals[6] = {suv, swv, suu, svv, sww, g};
#pragma unroll
      for (int qi = 0; qi < 6; ++qi) {
        if (qi < 2 || want_stats) {
          const double s = wsum(double(vals[qi]));
          if (wl == 0) red[qi][wv] += s;
        }
      }
    }
    __syncthreads();
    // ---- PP-point forward z transform of each (product, kx) column ------------
    if (tid < 3 * L * S) {
      const int nx = tid % L, c = (tid / L) % S, f = tid / (L * S);
      const C* rows = zf + f * PH * Cfg::FP;
      // row q of the column: unpack the complex row pairs
      auto yq = [&](int q) -> C {
        const int p = q < PH ? q : q - PH;
        const C zk = rows[p * Cfg::FP + nx];
        const C zm = cconj(rows[p * Cfg::FP + (nx == 0 ? 0 : 2 * L - nx)]);
        if (q < PH) return C{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y + zm.y)};
        return C{T(0.5) * (zk.y - zm.y), T(-0.5) * (zk.x - zm.x)};
      };
      C z[16];
#pragma unroll
      for (int n = 0; n < 16; ++n) {
        C s = yq(n);
#pragma unroll
        for (int b = 1; b < S; ++b) s = cadd(s, cmul(yq(n + 16 * b), root_s<T, S>(b * c, -1)));
        z[n] = (c == 0 || n == 0) ? s : cmul(s, rootZ[(n * c * R) % MZ]);
      }
      SmallDft<T, 16, -1>::run(z);
      C* out = Yb + (f * L + nx) * Cfg::YP;
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) out[S * kk + c] = z[kk];
    }
    __syncthreads();
    // the accumulators' mode indices are recomputed in every chunk rather than
    // held in registers across the chunk loop; one mode's index arithmetic and
    // twiddle serve its three fields
    int tbase = tid;
    asm volatile("" : "+v"(tbase));
#pragma unroll
    for (int km = 0; km < Cfg::NM; ++km) {
      const int m = tbase + km * NT;
      if (m < K) {
        const int nx = m / NZ;
        const int nz = stage_kz(m - nx * NZ);  // m: the mode's stage-buffer position
        const int kk = ((nz % PP) + PP) % PP;
        const int tt = (((r * nz) % MZ) + MZ) % MZ;
        const C w = rootZ[tt];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const C term = cmul(Yb[(f * L + nx) * Cfg::YP + kk], w);
          if constexpr (kGAcc) {
            VT* pn = nl + 2 * stage_off(size_t(f) * My + j, e, m, E, K, slb);
            C v = r > 0 ? cadd(ld2<T>(pn), term) : term;
            if (r == R - 1) v = cscale(v, inv);
            st2<T>(pn, v);
          } else {
            acc[f * Cfg::NM + km] = cadd(acc[f * Cfg::NM + km], term);
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- truncated advection spectrum ----------------------------------------------
  if constexpr (!kGAcc) {
#pragma unroll
    for (int km = 0; km < Cfg::NM; ++km) {
      const int m = tid + km * NT;
      if (m < K) {
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const size_t off = stage_off(size_t(f) * My + j, e, m, E, K, slb);
          st2<T>(nl + 2 * off, cscale(acc[f * Cfg::NM + km], inv));
        }
      }
    }
  }
  // ---- plane means: per-wavefront sums added in wavefront order ----------------
  if (tid == 0) {
    const double norm = 1.0 / (double(MX) * double(MZ));
    double tot[6];
    for (int qi = 0; qi < 6; ++qi) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[qi][w];
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

namespace {

// Built (precision, L, chunk rows), default first per grid: the variants whose
// registers fit without spilling.
// Built (precision, L = Nx/2, P = Nz/2, chunk rows): on the square grids the
// variants whose registers fit without spilling; on the non-square grids
// (Nx, Nz) = (64, 32) and (32, 64) the 16-row chunks.
template <typename T, int L, int P, int PP>
constexpr bool wave_built() {
  if constexpr (L != P) return PP == 16 && ((L == 32 && P == 16) || (L == 16 && P == 32));
  else if constexpr (sizeof(T) == 4) return (L == 32 && (PP == 32 || PP == 16)) || (L == 16 && (PP == 48 || PP == 16));
  else return (L == 32 && PP == 16) || (L == 16 && (PP == 16 || PP == 48));
}

template <typename T, int L, int P, int PP>
const void* wave_fn_if_built(bool gacc) {
  if constexpr (!wave_built<T, L, P, PP>()) {
    return nullptr;
  } else {
    using Cfg = WaveCfg<T, L, P, PP>;
    static_assert(Cfg::kLdsBytes <= 160 * 1024, "LDS of a built variant");
    return gacc ? reinterpret_cast<const void*>(&plane_wave_kernel<T, T, L, P, PP, true>)
                : reinterpret_cast<const void*>(&plane_wave_kernel<T, T, L, P, PP, false>);
  }
}

template <typename T, int L, int P>
const void* wave_fn_rows(int pp, bool gacc) {
  switch (pp) {
    case 16: return wave_fn_if_built<T, L, P, 16>(gacc);
    case 32: return wave_fn_if_built<T, L, P, 32>(gacc);
    case 48: return wave_fn_if_built<T, L, P, 48>(gacc);
  }
  return nullptr;
}

template <typename T>
const void* wave_fn_t(int Nx, int Nz, int pp, bool gacc) {
  if (Nx == 32 && Nz == 32) return wave_fn_rows<T, 16, 16>(pp, gacc);
  if (Nx == 64 && Nz == 64) return wave_fn_rows<T, 32, 32>(pp, gacc);
  if (Nx == 64 && Nz == 32) return wave_fn_rows<T, 32, 16>(pp, gacc);
  if (Nx == 32 && Nz == 64) return wave_fn_rows<T, 16, 32>(pp, gacc);
  return nullptr;
}

}  // namespace

// code: chunk rows, plus kWaveGlobalAcc for the variant that accumulates the
// forward z transform in the output buffer
const void* plane_wave_fn(int precision, int Nx, int Nz, int code) {
  const bool gacc = code >= kWaveGlobalAcc;
  const int pp = code % kWaveGlobalAcc;
  return precision == 0 ? wave_fn_t<double>(Nx, Nz, pp, gacc) : wave_fn_t<float>(Nx, Nz, pp, gacc);
}

// Built codes, fastest first as measured on the MI355X (per-launch times of
// the 16-member 64x97x64 and 64-member 32x49x32 ensembles): FP32 at Nx = 64
// the 512-lane 32-row chunks with the sums in the output buffer (their 126
// VGPRs admit two workgroups per CU), FP64 at Nx = 64 the 16-row chunks with
// the sums in the output buffer; at Nx = 32 the 16-row chunks with register
// sums.  The tuner times them all.
int plane_wave_rows(int precision, int Nx, int Nz, int* codes) {
  constexpr int G = kWaveGlobalAcc;
  static constexpr int fp32_64[6] = {32 + G, 16, 16 + G, 32, 48 + G, 48};
  static constexpr int fp64_64[6] = {16 + G, 16, 32 + G, 32, 48 + G, 48};
  static constexpr int other[6] = {16, 16 + G, 48, 48 + G, 32 + G, 32};
  const int* order = Nx == 64 && Nz == 64 ? (precision == 0 ? fp64_64 : fp32_64) : other;
  int n = 0;
  for (int i = 0; i < 6; ++i)
    if (plane_wave_fn(precision, Nx, Nz, order[i])) codes[n++] = order[i];
  return n;
}

int plane_wave_threads(int Nx, int code) { return (code % kWaveGlobalAcc / 2) * (Nx / 2); }

}  // namespace dns
