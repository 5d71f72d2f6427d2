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
//
// Every y contraction Y = M X is a real matrix (an operator or a Chebyshev
// derivative) times real columns (re/im of every (mode, member) pair) and runs
// on the FP64 matrix cores: v_mfma_f64_16x16x4f64, one 16x16 output tile per
// wavefront, K in steps of 4.  Operators are stored pre-tiled in the MFMA A
// lane order (tile (rt, kt) = 64 consecutive doubles, lane l holding
// M[16 rt + l % 16][4 kt + l / 16]) so each A fragment is one coalesced 512 B
// load; X lives in LDS as [k][column] so each B fragment is four 128 B rows.
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
constexpr int kWaves = kNT / 64;

typedef double d4 __attribute__((ext_vector_type(4)));

// Y = M X over every output tile of this workgroup; store(row, col, value) is
// called once per element with row < 16 RT, col < 16 CT (the caller ignores
// padding rows).  M: tiled operator (RT x KT tiles), X: LDS, row stride ldx.
// D layout of v_mfma_f64_16x16x4f64: lane l, register r -> row l/16 + 4r, col l%16.
template <class Store>
__device__ __forceinline__ void mfma_contract(const double* __restrict__ Mt, int RT, int KT,
                                              const double* X, int ldx, int CT, Store store) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  for (int t = wave; t < RT * CT; t += kWaves) {
    const int rt = t / CT, ct = t - rt * CT;
    const double* a = Mt + size_t(rt) * KT * 64 + lane;
    const double* b = X + lk * ldx + ct * 16 + lr;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    int kt = 0;
    for (; kt + 4 <= KT; kt += 4) {
      const double a0 = a[(kt + 0) * 64], a1 = a[(kt + 1) * 64];
      const double a2 = a[(kt + 2) * 64], a3 = a[(kt + 3) * 64];
      const double b0 = b[(4 * kt + 0) * ldx], b1 = b[(4 * kt + 4) * ldx];
      const double b2 = b[(4 * kt + 8) * ldx], b3 = b[(4 * kt + 12) * ldx];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b2, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, b3, acc, 0, 0, 0);
    }
    for (; kt < KT; ++kt)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kt * 64], b[4 * kt * ldx], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) store(rt * 16 + lk + 4 * r, ct * 16 + lr, acc[r]);
  }
}

template <typename VT>
__device__ __forceinline__ void st_c(VT* p, double re, double im) {
  p[0] = VT(re);
  p[1] = VT(im);
}

}  // namespace

// LDS (doubles, row stride CRP = real columns padded to 16):
//   S  [SR][CRP]  v-solve stack [v0; -h dt F_c], later eta (rows 0..My-1)
//   S2 [SR][CRP]  eta-solve stack [eta0; -h dt G_c], later dv/dy then u
//   T  [TR][CRP]  Q = i kx N_u + i kz N_w, later v (rows 0..My-1)
// SR >= max(4 KT(2N), My), TR >= 4 KT(My); padding rows are zero.
template <typename VT>
__global__ void __launch_bounds__(kNT) mode_kernel(ModeArgs a) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int My = a.My, N = a.N, K = a.K, E = a.E, NZ = a.NZ, P = a.P, ET = a.ET;
  const int C = 2 * ET;           // complex columns: (slot, member)
  const int CRP = a.CRP;          // real columns, padded to 16
  const int CT = CRP / 16;
  const int SR = a.SR, TR = a.TR;
  double* S = smem;
  double* S2 = S + size_t(SR) * CRP;
  double* T = S2 + size_t(SR) * CRP;
  __shared__ double red[kNT];
  __shared__ double gam_s[64];

  const int flat = xcd_logical_m(blockIdx.x, gridDim.x);
  const int g = flat / a.ntiles;
  const int tile = flat - g * a.ntiles;
  const int nx = g / P, az = g - nx * P;
  const bool mean_group = (g == 0);
  VT* vel = static_cast<VT*>(a.vel);
  const VT* nl = static_cast<const VT*>(a.nl);
  const int s = a.stage;
  const double hdt = a.hdt;
  const size_t KE = size_t(K) * E;

  // column c -> (slot, member); real column 2c (re), 2c + 1 (im)
  auto col_slot = [&](int c) { return c / ET; };
  auto col_member = [&](int c) { return tile * ET + (c - (c / ET) * ET); };
  auto col_valid = [&](int c) {
    const int sl = c / ET;
    return tile * ET + (c - sl * ET) < E && (sl == 0 || az > 0);
  };
  auto col_mode = [&](int c) { return nx * NZ + (c / ET == 0 ? az : NZ - az); };
  auto col_kz = [&](int c) { return (c / ET == 0 ? 1.0 : -1.0) * a.kzs * az; };
  const double kx = a.kxs * nx;

  // zero all buffers (padding rows and columns must hold zeros)
  for (int q = tid; q < (2 * SR + TR) * CRP; q += kNT) smem[q] = 0.0;
  __syncthreads();

  const int RTn = (N + 15) / 16, RTm = (My + 15) / 16;
  const int KT2n = (2 * N + 3) / 4, KTm = (My + 3) / 4, KTn = (N + 3) / 4;

  if (!mean_group) {
    // ===================== fluctuation modes (k^2 > 0) =====================
    if (s >= 0) {
      for (int q = tid; q < My * C; q += kNT) {
        const int i = q / C, c = q - i * C;
        if (!col_valid(c)) continue;
        const size_t off = 2 * ((size_t(i) * E + col_member(c)) * K + col_mode(c));
        const size_t fs = 2 * size_t(My) * KE;
        const double kz = col_kz(c), k2 = kx * kx + kz * kz;
        const double nur = nl[off], nui = nl[off + 1];
        const double nvr = nl[off + fs], nvi = nl[off + fs + 1];
        const double nwr = nl[off + 2 * fs], nwi = nl[off + 2 * fs + 1];
        // Q = i kx N_u + i kz N_w
        T[i * CRP + 2 * c] = -(kx * nui + kz * nwi);
        T[i * CRP + 2 * c + 1] = kx * nur + kz * nwr;
        if (i >= 1 && i < My - 1) {
          // -k^2 N_v into the lower half of S; G = i kz N_u - i kx N_w into S2
          S[(N + i - 1) * CRP + 2 * c] = -k2 * nvr;
          S[(N + i - 1) * CRP + 2 * c + 1] = -k2 * nvi;
          S2[(N + i - 1) * CRP + 2 * c] = -(kz * nui - kx * nwi);
          S2[(N + i - 1) * CRP + 2 * c + 1] = kz * nur - kx * nwr;
        }
      }
      __syncthreads();
      // F = -k^2 N_v - D1 Q on interior rows (D1int = D1[1:My-1, :])
      mfma_contract(a.D1intT, RTn, KTm, T, CRP, CT, [&](int r, int cc, double v) {
        if (r < N) S[(N + r) * CRP + cc] -= v;
      });
      __syncthreads();
      // RK3 combination, history, -h dt scaling; v0 and eta0 into the stacks
      for (int q = tid; q < N * C; q += kNT) {
        const int ii = q / C, c = q - ii * C;
        if (!col_valid(c)) continue;
        const size_t so = 2 * ((size_t(col_mode(c)) * N + ii) * E + col_member(c));
        double Fr = S[(N + ii) * CRP + 2 * c], Fi = S[(N + ii) * CRP + 2 * c + 1];
        double Gr = S2[(N + ii) * CRP + 2 * c], Gi = S2[(N + ii) * CRP + 2 * c + 1];
        double* hf = a.hF + so;
        double* hg = a.hG + so;
        if (s == 0) {
          hf[0] = Fr; hf[1] = Fi;
          hg[0] = Gr; hg[1] = Gi;
        } else if (s == 1) {
          const double Hr = hf[0], Hi = hf[1], HGr = hg[0], HGi = hg[1];
          hf[0] = Hr + 4.0 * Fr; hf[1] = Hi + 4.0 * Fi;
          hg[0] = HGr + 4.0 * Gr; hg[1] = HGi + 4.0 * Gi;
          Fr = 2.0 * Fr - Hr; Fi = 2.0 * Fi - Hi;
          Gr = 2.0 * Gr - HGr; Gi = 2.0 * Gi - HGi;
        } else {
          Fr = (hf[0] + Fr) * (1.0 / 6.0); Fi = (hf[1] + Fi) * (1.0 / 6.0);
          Gr = (hg[0] + Gr) * (1.0 / 6.0); Gi = (hg[1] + Gi) * (1.0 / 6.0);
        }
        S[(N + ii) * CRP + 2 * c] = -hdt * Fr;
        S[(N + ii) * CRP + 2 * c + 1] = -hdt * Fi;
        S2[(N + ii) * CRP + 2 * c] = -hdt * Gr;
        S2[(N + ii) * CRP + 2 * c + 1] = -hdt * Gi;
        S[ii * CRP + 2 * c] = a.v[so];
        S[ii * CRP + 2 * c + 1] = a.v[so + 1];
        S2[ii * CRP + 2 * c] = a.eta[so];
        S2[ii * CRP + 2 * c + 1] = a.eta[so + 1];
      }
      __syncthreads();
      const double* opg = a.opsT + size_t(g) * 2 * RTn * KT2n * 64;
      // v = [A_v | B_v] [v0; -h dt F_c] -> T rows 1..N (Q no longer needed;
      // its wall rows 0 and My-1 must read as v = 0 later)
      for (int q = tid; q < CRP; q += kNT) {
        T[q] = 0.0;
        T[(My - 1) * CRP + q] = 0.0;
      }
      mfma_contract(opg, RTn, KT2n, S, CRP, CT, [&](int r, int cc, double v) {
        if (r < N) T[(1 + r) * CRP + cc] = v;
      });
      __syncthreads();
      // eta = [A_eta | B_eta] [eta0; -h dt G_c] -> S rows 1..N; S rows 0 and
      // My-1 become the eta wall values (zero).  Rows beyond My keep finite
      // stack data that only meets the zero padding columns of D1.
      for (int q = tid; q < CRP; q += kNT) {
        S[q] = 0.0;
        S[(My - 1) * CRP + q] = 0.0;
      }
      mfma_contract(opg + size_t(RTn) * KT2n * 64, RTn, KT2n, S2, CRP, CT, [&](int r, int cc, double v) {
        if (r < N) S[(1 + r) * CRP + cc] = v;
      });
      __syncthreads();
      if (s == 2) {
        // Hermitian projection of the n_x = 0 column: (0, nz) and (0, -nz)
        if (nx == 0 && az > 0) {
          for (int q = tid; q < N * ET; q += kNT) {
            const int ii = q / ET, c0 = q - ii * ET, c1 = c0 + ET;
            const int i = ii + 1;
            double* bufs[2] = {T, S};
#pragma unroll
            for (int bsel = 0; bsel < 2; ++bsel) {
              double* B = bufs[bsel];
              const double ar = B[i * CRP + 2 * c0], ai = B[i * CRP + 2 * c0 + 1];
              const double br = B[i * CRP + 2 * c1], bi = B[i * CRP + 2 * c1 + 1];
              const double pr = 0.5 * (ar + br), pi = 0.5 * (ai - bi);
              B[i * CRP + 2 * c0] = pr;
              B[i * CRP + 2 * c0 + 1] = pi;
              B[i * CRP + 2 * c1] = pr;
              B[i * CRP + 2 * c1 + 1] = -pi;
            }
          }
          __syncthreads();
        }
        for (int q = tid; q < N * C; q += kNT) {
          const int ii = q / C, c = q - ii * C;
          if (!col_valid(c)) continue;
          const size_t so = 2 * ((size_t(col_mode(c)) * N + ii) * E + col_member(c));
          a.v[so] = T[(ii + 1) * CRP + 2 * c];
          a.v[so + 1] = T[(ii + 1) * CRP + 2 * c + 1];
          a.eta[so] = S[(ii + 1) * CRP + 2 * c];
          a.eta[so + 1] = S[(ii + 1) * CRP + 2 * c + 1];
        }
      }
    } else {
      // velocities of the stored state: v -> T rows 1..N, eta -> S rows 1..N
      for (int q = tid; q < N * C; q += kNT) {
        const int ii = q / C, c = q - ii * C;
        if (!col_valid(c)) continue;
        const size_t so = 2 * ((size_t(col_mode(c)) * N + ii) * E + col_member(c));
        T[(ii + 1) * CRP + 2 * c] = a.v[so];
        T[(ii + 1) * CRP + 2 * c + 1] = a.v[so + 1];
        S[(ii + 1) * CRP + 2 * c] = a.eta[so];
        S[(ii + 1) * CRP + 2 * c + 1] = a.eta[so + 1];
      }
    }
    __syncthreads();
    // ---- velocity recovery: dv/dy = D1c v -> S2 rows 0..My-1 ---------------
    mfma_contract(a.D1cT, RTm, KTn, T + CRP, CRP, CT, [&](int r, int cc, double v) {
      if (r < My) S2[r * CRP + cc] = v;
    });
    __syncthreads();
    double dmax = 0.0;
    for (int q = tid; q < My * C; q += kNT) {
      const int i = q / C, c = q - i * C;
      const double kz = col_kz(c), k2 = kx * kx + kz * kz;
      const double ik2 = k2 > 0.0 ? 1.0 / k2 : 0.0;
      const double dr = S2[i * CRP + 2 * c], di = S2[i * CRP + 2 * c + 1];
      const double er = S[i * CRP + 2 * c], ei = S[i * CRP + 2 * c + 1];
      const double vr = T[i * CRP + 2 * c], vi = T[i * CRP + 2 * c + 1];
      // u = (i kx dv - i kz eta) / k^2 ; w = (i kx eta + i kz dv) / k^2
      const double ur = (-kx * di + kz * ei) * ik2, ui = (kx * dr - kz * er) * ik2;
      const double wr = (-kx * ei - kz * di) * ik2, wi = (kx * er + kz * dr) * ik2;
      S2[i * CRP + 2 * c] = ur;
      S2[i * CRP + 2 * c + 1] = ui;
      S[i * CRP + 2 * c] = wr;
      S[i * CRP + 2 * c + 1] = wi;
      if (col_valid(c)) {
        const size_t off = 2 * ((size_t(i) * E + col_member(c)) * K + col_mode(c));
        const size_t fs = 2 * size_t(My) * KE;
        st_c(vel + off, ur, ui);
        st_c(vel + off + fs, vr, vi);
        st_c(vel + off + 2 * fs, wr, wi);
        // divergence i kx u + dv/dy + i kz w
        const double xr = -kx * ui + dr - kz * wi, xi = kx * ur + di + kz * wr;
        dmax = fmax(dmax, sqrt(xr * xr + xi * xi));
      }
    }
    __syncthreads();
    // du/dy = D1 u, dw/dy = D1 w -> velocity fields 3 and 4
    auto store_y = [&](int f, const double* Xsrc) {
      mfma_contract(a.D1T, RTm, KTm, Xsrc, CRP, CT, [&](int r, int cc, double v) {
        const int c = cc >> 1;
        if (r < My && c < C && col_valid(c)) {
          const size_t off = 2 * (((size_t(f) * My + r) * E + col_member(c)) * K + col_mode(c));
          vel[off + (cc & 1)] = VT(v);
        }
      });
    };
    store_y(3, S2);
    store_y(4, S);
    if (s == 2 || s < 0) {
      red[tid] = dmax;
      __syncthreads();
      // per member: max over the threads that saw its columns
      if (tid < C && col_valid(tid)) {
        double mx = 0.0;
        for (int q = 0; q < kNT; ++q)
          if ((q % C) == tid) mx = fmax(mx, red[q]);
        atomicMax(&a.divmax[col_member(tid)], (unsigned long long)__double_as_longlong(mx));
      }
    }
    return;
  }

  // ========================= mean profiles (0, 0) ===========================
  // Real columns 2e (U or <uv> or E_U) and 2e + 1 (W or <wv> or E_W), e < ET;
  // U and W share A_U, B_U (Eqs. (CN3), (CN4)).
  const int NM = ET;  // members in this tile (slot 0 only)
  if (s >= 0) {
    for (int q = tid; q < My * NM; q += kNT) {
      const int i = q / NM, el = q - i * NM, e = tile * ET + el;
      if (e >= E) continue;
      T[i * CRP + 2 * el] = a.means[(size_t(0) * My + i) * E + e];
      T[i * CRP + 2 * el + 1] = a.means[(size_t(1) * My + i) * E + e];
    }
    __syncthreads();
    // E_U + E_W = -D1 (<uv>, <wv>) on interior rows -> S rows N..2N-1
    mfma_contract(a.D1intT, RTn, KTm, T, CRP, CT, [&](int r, int cc, double v) {
      if (r < N) S[(N + r) * CRP + cc] = -v;
    });
    __syncthreads();
    for (int q = tid; q < N * NM; q += kNT) {
      const int ii = q / NM, el = q - ii * NM, e = tile * ET + el;
      if (e >= E) continue;
      double xu = S[(N + ii) * CRP + 2 * el], xw = S[(N + ii) * CRP + 2 * el + 1];
      double* hu = a.hEU + size_t(ii) * E + e;
      double* hw = a.hEW + size_t(ii) * E + e;
      if (s == 0) {
        *hu = xu;
        *hw = xw;
      } else if (s == 1) {
        const double Hu = *hu, Hw = *hw;
        *hu = Hu + 4.0 * xu;
        *hw = Hw + 4.0 * xw;
        xu = 2.0 * xu - Hu;
        xw = 2.0 * xw - Hw;
      } else {
        xu = (*hu + xu) * (1.0 / 6.0);
        xw = (*hw + xw) * (1.0 / 6.0);
      }
      S[(N + ii) * CRP + 2 * el] = hdt * xu;
      S[(N + ii) * CRP + 2 * el + 1] = hdt * xw;
      S[ii * CRP + 2 * el] = a.U[size_t(ii + 1) * E + e];
      S[ii * CRP + 2 * el + 1] = a.W[size_t(ii + 1) * E + e];
    }
    __syncthreads();
    // (U_a, W) = [A_U | B_U] [(U0, W0); h dt (E_U,c, E_W,c)] -> T rows 1..N
    mfma_contract(a.meanT, RTn, KT2n, S, CRP, CT, [&](int r, int cc, double v) {
      if (r < N) T[(1 + r) * CRP + cc] = v;
    });
    __syncthreads();
    // lift, bulk flux of the provisional U and gamma, one thread per member
    if (tid < NM) {
      const int el = tid, e = tile * ET + el;
      double gam = 0.0;
      if (a.poiseuille) {
        double qa = a.ccw[0] * a.Ubot + a.ccw[My - 1] * a.Utop;
        double wg = 0.0;
        for (int i = 1; i < My - 1; ++i) {
          qa += a.ccw[i] * (T[i * CRP + 2 * el] + a.lift[i - 1]);
          wg += a.ccw[i] * a.green[i - 1];
        }
        gam = (a.Qtarget - qa) / wg;
      }
      gam_s[el] = gam;
      if (e < E) a.gamma[e] = gam;
    }
    __syncthreads();
    for (int q = tid; q < My * NM; q += kNT) {
      const int i = q / NM, el = q - i * NM;
      if (i == 0) {
        T[2 * el] = a.Ubot;
        T[2 * el + 1] = 0.0;
      } else if (i == My - 1) {
        T[i * CRP + 2 * el] = a.Utop;
        T[i * CRP + 2 * el + 1] = 0.0;
      } else {
        T[i * CRP + 2 * el] += a.lift[i - 1] + gam_s[el] * a.green[i - 1];
      }
    }
    __syncthreads();
    if (s == 2) {
      for (int q = tid; q < My * NM; q += kNT) {
        const int i = q / NM, el = q - i * NM, e = tile * ET + el;
        if (e >= E) continue;
        a.U[size_t(i) * E + e] = T[i * CRP + 2 * el];
        a.W[size_t(i) * E + e] = T[i * CRP + 2 * el + 1];
      }
    }
  } else {
    for (int q = tid; q < My * NM; q += kNT) {
      const int i = q / NM, el = q - i * NM, e = tile * ET + el;
      if (e >= E) continue;
      T[i * CRP + 2 * el] = a.U[size_t(i) * E + e];
      T[i * CRP + 2 * el + 1] = a.W[size_t(i) * E + e];
    }
    __syncthreads();
  }
  // velocity fields of the (0, 0) mode: u = U, v = 0, w = W, du/dy, dw/dy
  for (int q = tid; q < My * NM; q += kNT) {
    const int i = q / NM, el = q - i * NM, e = tile * ET + el;
    if (e >= E) continue;
    const size_t off = 2 * ((size_t(i) * E + e) * K);
    const size_t fs = 2 * size_t(My) * KE;
    st_c(vel + off, T[i * CRP + 2 * el], 0.0);
    st_c(vel + off + fs, 0.0, 0.0);
    st_c(vel + off + 2 * fs, T[i * CRP + 2 * el + 1], 0.0);
  }
  mfma_contract(a.D1T, RTm, KTm, T, CRP, CT, [&](int r, int cc, double v) {
    const int el = cc >> 1, e = tile * ET + el;
    if (r < My && el < NM && e < E) {
      const int f = 3 + (cc & 1);
      const size_t off = 2 * (((size_t(f) * My + r) * E + e) * K);
      st_c(vel + off, v, 0.0);
    }
  });
}

// LDS geometry of one workgroup; shared with the host launcher.
void mode_lds_geometry(int My, int ET, int* CRP, int* SR, int* TR) {
  const int N = My - 2;
  *CRP = ((4 * ET + 15) / 16) * 16;
  const int k2n = 4 * ((2 * N + 3) / 4);
  const int km = 4 * ((My + 3) / 4);
  int sr = k2n > My ? k2n : My;
  // D1c reads T rows 1..4*KT(N); D1 reads rows 0..4*KT(My)-1
  *SR = sr > km ? sr : km;
  const int kn1 = 1 + 4 * ((N + 3) / 4);
  *TR = km > kn1 ? km : kn1;
}

int mode_member_tile(int My, int E) {
  // largest ET in {1, 2, 4, 8} (<= E) whose LDS allows two workgroups per CU
  int best = 1;
  for (int et = 1; et <= 8 && et <= E; et *= 2) {
    int crp, sr, tr;
    mode_lds_geometry(My, et, &crp, &sr, &tr);
    const size_t lds = size_t(2 * sr + tr) * crp * sizeof(double);
    if (lds <= 78 * 1024) best = et;
  }
  return best;
}

hipError_t launch_mode(int precision, const ModeArgs& a, hipStream_t s) {
  const int nblk = a.G * a.ntiles;
  const size_t lds = size_t(2 * a.SR + a.TR) * a.CRP * sizeof(double);
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
