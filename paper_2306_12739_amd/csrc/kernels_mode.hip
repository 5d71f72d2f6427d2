// Per-(kx, kz) stage: right-hand sides, RK3 combination, implicit CN solves
// and velocity recovery.  One workgroup per operator group (nx, |nz|) -- the
// modes (nx, +nz) and (nx, -nz) share every y operator -- and member tile.
//
// Paper references:
//  * F and G, Eqs. (Dv), (eta), (Dv_F): d_t Lap v = -F + LapLap v / Re,
//    d_t eta = -G + Lap eta / Re, with F = -k^2 N_v - D1 (i kx N_u + i kz N_w)
//    and G = i kz N_u - i kx N_w;
//  * Sec. 3.1: sub-step forcing F^0, 2F^1 - F^0, (F^0 + 4F^1 + F^2)/6 with
//    h = 1/2, 1, 1, every sub-step restarting from the state at t;
//  * Eqs. (CN1)-(CN4) and Sec. 3.2: pre-inverted operators applied to all
//    ensemble members at once (members are extra columns);
//  * Sec. 3.2, u/w recovery: u = (i kx dv/dy - i kz eta)/k^2,
//    w = (i kx eta + i kz dv/dy)/k^2 with dv/dy from the clamped interpolant;
//  * Eqs. (U00), (W00) with the Couette wall lift and, for the channel, a
//    pressure gradient gamma that holds the bulk flux at its target.
// Columns of the per-group matrices are (mode slot, member) pairs; rows are
// Chebyshev nodes.  All arithmetic here is FP64.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dns {

namespace {

__device__ __forceinline__ int xcd_logical_m(int b, int nblk) {
  const int q = nblk >> 3, rem = nblk & 7;
  const int x = b & 7, local = b >> 3;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + local;
}

constexpr int kNT = 256;
constexpr int kMaxR = 16;  // rows per thread

struct dc {
  double x, y;
};
__device__ __forceinline__ dc dadd(dc a, dc b) { return dc{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ dc dsub(dc a, dc b) { return dc{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ dc dscale(dc a, double s) { return dc{a.x * s, a.y * s}; }
__device__ __forceinline__ dc dmuli(dc a, double s) { return dc{-a.y * s, a.x * s}; }  // i s a
__device__ __forceinline__ dc dconj(dc a) { return dc{a.x, -a.y}; }

template <typename VT>
__device__ __forceinline__ dc ld_vt(const VT* p) {
  return dc{double(p[0]), double(p[1])};
}
template <typename VT>
__device__ __forceinline__ void st_vt(VT* p, dc v) {
  p[0] = VT(v.x);
  p[1] = VT(v.y);
}

// acc[r] += sum_k M[(row_r + roff) * ldm + k + koff] * B[k][c], k in [k0, k1)
// for the rows this thread owns (row_r = rg + r * nrg < nrows).
__device__ __forceinline__ void contract(dc* acc, const double* __restrict__ M, int ldm, int roff,
                                         int koff, const dc* B, int C, int c, int rg, int nrg,
                                         int nrows, int row0, int k0, int k1) {
#pragma unroll 1
  for (int k = k0; k < k1; ++k) {
    const dc x = B[k * C + c];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int row = row0 + rg + r * nrg;
      if (row < nrows) {
        const double m = M[size_t(row + roff) * ldm + k + koff];
        acc[r].x = fma(m, x.x, acc[r].x);
        acc[r].y = fma(m, x.y, acc[r].y);
      }
    }
  }
}

}  // namespace

template <typename VT>
__global__ void __launch_bounds__(kNT) mode_kernel(ModeArgs a) {
  extern __shared__ dc smem[];
  const int tid = threadIdx.x;
  const int My = a.My, N = a.N, K = a.K, E = a.E, NZ = a.NZ, P = a.P, ET = a.ET;
  const int C = 2 * ET;
  const int nrg = kNT / C;
  const int c = tid % C;
  const int rg = tid / C;
  const bool active_thread = rg < nrg;
  dc* B0 = smem;
  dc* B1 = smem + My * C;
  dc* B2 = smem + 2 * My * C;
  __shared__ double red[kNT];

  const int flat = xcd_logical_m(blockIdx.x, gridDim.x);
  const int g = flat / a.ntiles;
  const int tile = flat - g * a.ntiles;
  const int nx = g / P, az = g - nx * P;
  const int slot = c / ET;
  const int e = tile * ET + (c - slot * ET);
  const bool colvalid = active_thread && e < E && (slot == 0 || az > 0);
  const double kx = a.kxs * nx;
  const double kz = (slot == 0 ? 1.0 : -1.0) * a.kzs * az;
  const double k2 = kx * kx + kz * kz;
  const int iz = slot == 0 ? az : NZ - az;
  const int m = nx * NZ + iz;
  const bool mean_group = (g == 0);
  VT* vel = static_cast<VT*>(a.vel);
  const VT* nl = static_cast<const VT*>(a.nl);
  const int s = a.stage;
  const double hdt = a.hdt;

  auto velp = [&](int f, int i) -> VT* {
    return vel + 2 * ((size_t(f) * My + i) * K * E + size_t(m) * E + e);
  };
  auto nlp = [&](int f, int i) -> const VT* {
    return nl + 2 * ((size_t(f) * My + i) * K * E + size_t(m) * E + e);
  };
  auto stp = [&](double* base, int i) -> double* {  // interior row i in [1, N]
    return base + 2 * ((size_t(m) * N + (i - 1)) * E + e);
  };

  dc acc[kMaxR];
  auto zero_acc = [&]() {
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) acc[r] = dc{0.0, 0.0};
  };

  if (!mean_group) {
    // ===================== fluctuation modes (k^2 > 0) =====================
    if (s >= 0) {
      // right-hand-side ingredients on every node
      for (int i = rg; i < My; i += nrg) {
        if (!active_thread) break;
        dc q{0.0, 0.0}, nv{0.0, 0.0}, gg{0.0, 0.0};
        if (colvalid) {
          const dc Nu = ld_vt(nlp(0, i)), Nv = ld_vt(nlp(1, i)), Nw = ld_vt(nlp(2, i));
          q = dadd(dmuli(Nu, kx), dmuli(Nw, kz));
          nv = dscale(Nv, -k2);
          gg = dsub(dmuli(Nu, kz), dmuli(Nw, kx));
        }
        B0[i * C + c] = q;
        B1[i * C + c] = nv;
        B2[i * C + c] = gg;
      }
      __syncthreads();
      // F = -k^2 N_v - D1 (i kx N_u + i kz N_w) on interior rows, in place in B1
      zero_acc();
      if (active_thread) contract(acc, a.D1, My, 0, 0, B0, C, c, rg, nrg, My - 1, 1, 0, My);
      __syncthreads();
      if (active_thread) {
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
          const int i = 1 + rg + r * nrg;
          if (i < My - 1) B1[i * C + c] = dsub(B1[i * C + c], acc[r]);
        }
      }
      __syncthreads();
      // RK3 combination, history update, -h dt scaling; state v0 into B0
      for (int i = 1 + rg; i < My - 1; i += nrg) {
        if (!active_thread) break;
        dc F = B1[i * C + c], G = B2[i * C + c];
        dc v0{0.0, 0.0};
        if (colvalid) {
          double* hf = stp(a.hF, i);
          double* hg = stp(a.hG, i);
          if (s == 0) {
            hf[0] = F.x; hf[1] = F.y;
            hg[0] = G.x; hg[1] = G.y;
          } else if (s == 1) {
            const dc H{hf[0], hf[1]}, HG{hg[0], hg[1]};
            const dc Fc = dsub(dscale(F, 2.0), H), Gc = dsub(dscale(G, 2.0), HG);
            const dc Hn = dadd(H, dscale(F, 4.0)), HGn = dadd(HG, dscale(G, 4.0));
            hf[0] = Hn.x; hf[1] = Hn.y;
            hg[0] = HGn.x; hg[1] = HGn.y;
            F = Fc;
            G = Gc;
          } else {
            const dc H{hf[0], hf[1]}, HG{hg[0], hg[1]};
            F = dscale(dadd(H, F), 1.0 / 6.0);
            G = dscale(dadd(HG, G), 1.0 / 6.0);
          }
          const double* vp = stp(a.v, i);
          v0 = dc{vp[0], vp[1]};
        } else {
          F = dc{0.0, 0.0};
          G = dc{0.0, 0.0};
        }
        B1[i * C + c] = dscale(F, -hdt);
        B2[i * C + c] = dscale(G, -hdt);
        B0[i * C + c] = v0;
      }
      __syncthreads();
      // v = A_v v0 + B_v (-h dt F_c)
      const double* opg = a.ops + size_t(g) * 4 * N * N;
      zero_acc();
      if (active_thread) {
        contract(acc, opg, N, -1, -1, B0, C, c, rg, nrg, My - 1, 1, 1, My - 1);
        contract(acc, opg + size_t(N) * N, N, -1, -1, B1, C, c, rg, nrg, My - 1, 1, 1, My - 1);
      }
      __syncthreads();
      if (active_thread) {
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
          const int i = 1 + rg + r * nrg;
          if (i < My - 1) {
            B0[i * C + c] = acc[r];
            dc e0{0.0, 0.0};
            if (colvalid) {
              const double* ep = stp(a.eta, i);
              e0 = dc{ep[0], ep[1]};
            }
            B1[i * C + c] = e0;
          }
        }
      }
      __syncthreads();
      // eta = A_eta eta0 + B_eta (-h dt G_c)
      zero_acc();
      if (active_thread) {
        contract(acc, opg + size_t(2) * N * N, N, -1, -1, B1, C, c, rg, nrg, My - 1, 1, 1, My - 1);
        contract(acc, opg + size_t(3) * N * N, N, -1, -1, B2, C, c, rg, nrg, My - 1, 1, 1, My - 1);
      }
      __syncthreads();
      if (active_thread) {
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
          const int i = 1 + rg + r * nrg;
          if (i < My - 1) B1[i * C + c] = acc[r];
        }
      }
      __syncthreads();
      if (s == 2) {
        // Hermitian projection of the n_x = 0 column: (0, nz) and (0, -nz)
        if (nx == 0 && az > 0 && active_thread && slot == 0) {
          for (int i = 1 + rg; i < My - 1; i += nrg) {
            const int cp = c + ET;
            const dc va = B0[i * C + c], vb = B0[i * C + cp];
            const dc ea = B1[i * C + c], eb = B1[i * C + cp];
            const dc pv = dscale(dadd(va, dconj(vb)), 0.5);
            const dc pe = dscale(dadd(ea, dconj(eb)), 0.5);
            B0[i * C + c] = pv;
            B0[i * C + cp] = dconj(pv);
            B1[i * C + c] = pe;
            B1[i * C + cp] = dconj(pe);
          }
        }
        __syncthreads();
        if (colvalid) {
          for (int i = 1 + rg; i < My - 1; i += nrg) {
            double* vp = stp(a.v, i);
            double* ep = stp(a.eta, i);
            const dc vv = B0[i * C + c], ee = B1[i * C + c];
            vp[0] = vv.x; vp[1] = vv.y;
            ep[0] = ee.x; ep[1] = ee.y;
          }
        }
      }
    } else {
      // velocities of the stored state only
      for (int i = rg; i < My; i += nrg) {
        if (!active_thread) break;
        dc v0{0.0, 0.0}, e0{0.0, 0.0};
        if (colvalid && i >= 1 && i < My - 1) {
          const double* vp = stp(a.v, i);
          const double* ep = stp(a.eta, i);
          v0 = dc{vp[0], vp[1]};
          e0 = dc{ep[0], ep[1]};
        }
        B0[i * C + c] = v0;
        B1[i * C + c] = e0;
      }
      __syncthreads();
    }
    // ---- velocity recovery: dv/dy = D1c v, u, w, then du/dy, dw/dy ----------
    zero_acc();
    if (active_thread) contract(acc, a.D1c, N, 0, -1, B0, C, c, rg, nrg, My, 0, 1, My - 1);
    dc ur[kMaxR], wr[kMaxR];
    double dmax = 0.0;
    const double ik2 = k2 > 0.0 ? 1.0 / k2 : 0.0;
    if (active_thread) {
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int i = rg + r * nrg;
        if (i < My) {
          const dc dv = acc[r];
          const bool inner = i >= 1 && i < My - 1;
          const dc et = inner ? B1[i * C + c] : dc{0.0, 0.0};
          const dc vv = inner ? B0[i * C + c] : dc{0.0, 0.0};
          const dc u = dscale(dsub(dmuli(dv, kx), dmuli(et, kz)), ik2);
          const dc w = dscale(dadd(dmuli(et, kx), dmuli(dv, kz)), ik2);
          ur[r] = u;
          wr[r] = w;
          if (colvalid) {
            st_vt(velp(0, i), u);
            st_vt(velp(1, i), vv);
            st_vt(velp(2, i), w);
            const dc dv_s = dadd(dadd(dmuli(u, kx), dv), dmuli(w, kz));
            dmax = fmax(dmax, sqrt(dv_s.x * dv_s.x + dv_s.y * dv_s.y));
          }
        }
      }
    }
    __syncthreads();
    if (active_thread) {
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int i = rg + r * nrg;
        if (i < My) {
          B0[i * C + c] = ur[r];
          B1[i * C + c] = wr[r];
        }
      }
    }
    __syncthreads();
    zero_acc();
    if (active_thread) contract(acc, a.D1, My, 0, 0, B0, C, c, rg, nrg, My, 0, 0, My);
    if (colvalid) {
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int i = rg + r * nrg;
        if (i < My) st_vt(velp(3, i), acc[r]);
      }
    }
    zero_acc();
    if (active_thread) contract(acc, a.D1, My, 0, 0, B1, C, c, rg, nrg, My, 0, 0, My);
    if (colvalid) {
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int i = rg + r * nrg;
        if (i < My) st_vt(velp(4, i), acc[r]);
      }
    }
    // per-member divergence maximum of this group (stage 2 and state-only calls)
    if (s == 2 || s < 0) {
      red[tid] = dmax;
      __syncthreads();
      if (tid < C && colvalid) {
        double mx = 0.0;
        for (int q = 0; q < nrg; ++q) mx = fmax(mx, red[q * C + tid]);
        atomicMax(&a.divmax[e], __double_as_longlong(mx));
      }
    }
    return;
  }

  // ========================= mean profiles (0, 0) ===========================
  // Columns 0..ET-1 are members; U and W travel together as (re, im) of one
  // complex column because they share the operators A_U, B_U (Eqs. (CN3), (CN4)).
  const bool mcol = active_thread && slot == 0 && e < E;
  if (s >= 0) {
    for (int i = rg; i < My; i += nrg) {
      if (!active_thread) break;
      dc uw{0.0, 0.0}, u0{0.0, 0.0};
      if (mcol) {
        uw = dc{a.means[(size_t(0) * My + i) * E + e], a.means[(size_t(1) * My + i) * E + e]};
        u0 = dc{a.U[size_t(i) * E + e], a.W[size_t(i) * E + e]};
      }
      B0[i * C + c] = uw;
      B2[i * C + c] = u0;
    }
    __syncthreads();
    // E_U + i E_W = -D1 (<uv> + i <wv>) on interior rows
    zero_acc();
    if (active_thread) contract(acc, a.D1, My, 0, 0, B0, C, c, rg, nrg, My - 1, 1, 0, My);
    __syncthreads();
    if (active_thread) {
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int i = 1 + rg + r * nrg;
        if (i < My - 1) {
          dc X = dscale(acc[r], -1.0);
          if (mcol) {
            double* hu = a.hEU + size_t(i - 1) * E + e;
            double* hw = a.hEW + size_t(i - 1) * E + e;
            if (s == 0) {
              *hu = X.x;
              *hw = X.y;
            } else if (s == 1) {
              const dc H{*hu, *hw};
              *hu = H.x + 4.0 * X.x;
              *hw = H.y + 4.0 * X.y;
              X = dsub(dscale(X, 2.0), H);
            } else {
              const dc H{*hu, *hw};
              X = dscale(dadd(H, X), 1.0 / 6.0);
            }
          } else {
            X = dc{0.0, 0.0};
          }
          B1[i * C + c] = dscale(X, hdt);
        }
      }
    }
    __syncthreads();
    // (U, W) = A_U (U0, W0) + B_U h dt (E_U,c, E_W,c) + (lift, 0)
    zero_acc();
    if (active_thread) {
      contract(acc, a.mean_ops, N, -1, -1, B2, C, c, rg, nrg, My - 1, 1, 1, My - 1);
      contract(acc, a.mean_ops + size_t(N) * N, N, -1, -1, B1, C, c, rg, nrg, My - 1, 1, 1, My - 1);
    }
    double qpart = 0.0;
    if (active_thread) {
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int i = 1 + rg + r * nrg;
        if (i < My - 1) {
          acc[r].x += a.lift[i - 1];
          qpart += a.ccw[i] * acc[r].x;
        }
      }
    }
    // bulk flux of the provisional U, reduced over rows in a fixed order
    red[tid] = qpart;
    __syncthreads();
    double gam = 0.0;
    if (a.poiseuille) {
      double qa = a.ccw[0] * a.Ubot + a.ccw[My - 1] * a.Utop;
      double wg = 0.0;
      for (int q = 0; q < nrg; ++q) qa += red[q * C + c];
      for (int i = 1; i < My - 1; ++i) wg += a.ccw[i] * a.green[i - 1];
      gam = (a.Qtarget - qa) / wg;
    }
    __syncthreads();
    if (active_thread) {
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int i = 1 + rg + r * nrg;
        if (i < My - 1) {
          dc uw = acc[r];
          uw.x += gam * a.green[i - 1];
          B0[i * C + c] = uw;
        }
      }
      if (rg == 0) {
        B0[c] = dc{a.Ubot, 0.0};
        B0[(My - 1) * C + c] = dc{a.Utop, 0.0};
      }
      if (mcol && rg == 0) a.gamma[e] = gam;
    }
    __syncthreads();
    if (s == 2 && mcol) {
      for (int i = rg; i < My; i += nrg) {
        const dc uw = B0[i * C + c];
        a.U[size_t(i) * E + e] = uw.x;
        a.W[size_t(i) * E + e] = uw.y;
      }
    }
  } else {
    for (int i = rg; i < My; i += nrg) {
      if (!active_thread) break;
      B0[i * C + c] = mcol ? dc{a.U[size_t(i) * E + e], a.W[size_t(i) * E + e]} : dc{0.0, 0.0};
    }
    __syncthreads();
  }
  // velocity fields of the (0, 0) mode: u = U, v = 0, w = W, du/dy, dw/dy
  zero_acc();
  if (active_thread) contract(acc, a.D1, My, 0, 0, B0, C, c, rg, nrg, My, 0, 0, My);
  if (mcol) {
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int i = rg + r * nrg;
      if (i < My) {
        const dc uw = B0[i * C + c];
        st_vt(velp(0, i), dc{uw.x, 0.0});
        st_vt(velp(1, i), dc{0.0, 0.0});
        st_vt(velp(2, i), dc{uw.y, 0.0});
        st_vt(velp(3, i), dc{acc[r].x, 0.0});
        st_vt(velp(4, i), dc{acc[r].y, 0.0});
      }
    }
  }
}

int mode_member_tile(int My, int E) {
  // columns C = 2 * ET; keep three My x C complex-double buffers within ~80 KB
  // and every thread's row count within kMaxR.
  int et = 1;
  while (et * 2 <= E && et * 2 <= 32) {
    const int cand = et * 2;
    const size_t lds = size_t(3) * My * 2 * cand * 16;
    const int nrg = kNT / (2 * cand);
    const int rows = (My + nrg - 1) / nrg;
    if (lds > 80 * 1024 || rows > kMaxR) break;
    et = cand;
  }
  return et;
}

hipError_t launch_mode(int precision, const ModeArgs& a, hipStream_t s) {
  const int nblk = a.G * a.ntiles;
  const size_t lds = size_t(3) * a.My * 2 * a.ET * sizeof(dc);
  const void* fn = precision == 0 ? reinterpret_cast<const void*>(&mode_kernel<double>)
                                  : reinterpret_cast<const void*>(&mode_kernel<float>);
  hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (err != hipSuccess) return err;
  if (precision == 0) {
    hipLaunchKernelGGL(mode_kernel<double>, dim3(nblk), dim3(kNT), lds, s, a);
  } else {
    hipLaunchKernelGGL(mode_kernel<float>, dim3(nblk), dim3(kNT), lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace dns
