// Host construction of the pre-inverted Crank-Nicolson operators.
//
// Paper Sec. 3.2 (Eqs. (CN1)-(CN4), Listings 1 and 3): for every (kx, kz)
// pair and each sub-step fraction h in {1/2, 1} the left-hand-side matrix of
// the CN difference equation is inverted once and folded into the constant
// right-hand-side matrix.  Only two operator sets are needed because the last
// two RK3 sub-steps share h = 1 (Sec. 1).  The clamped fourth derivative
// (Sec. 2, Weideman-Reddy) has entries growing like N^8, so everything here is
// built in 80-bit long double and rounded to FP64 at the end.
//
// With Lap = D2_D - k^2 I (Dirichlet walls) and LapLap = D4c - 2k^2 D2c + k^4 I
// (clamped walls), c = h dt / (2 Re), Eq. (CN1) multiplied through by Lap gives
//   (Lap - c LapLap) v_new = (Lap + c LapLap) v_0 - h dt F,
// so A_v = (Lap - c LapLap)^{-1} (Lap + c LapLap) and B_v = (Lap - c LapLap)^{-1};
// Eq. (CN2): A_eta = (I - c Lap)^{-1} (I + c Lap), B_eta = (I - c Lap)^{-1}.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.h"

namespace dns {

namespace {

using ld = long double;
using Mat = std::vector<ld>;  // row-major n x n

const ld kPi = 3.14159265358979323846264338327950288L;

// LU with partial pivoting, in place; returns false if singular.
bool lu_factor(Mat& A, std::vector<int>& piv, int n) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    ld best = std::fabs(A[size_t(k) * n + k]);
    for (int i = k + 1; i < n; ++i) {
      const ld v = std::fabs(A[size_t(i) * n + k]);
      if (v > best) { best = v; p = i; }
    }
    if (best == 0.0L) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A[size_t(k) * n + j], A[size_t(p) * n + j]);
    const ld inv = 1.0L / A[size_t(k) * n + k];
    for (int i = k + 1; i < n; ++i) {
      const ld f = A[size_t(i) * n + k] * inv;
      A[size_t(i) * n + k] = f;
      if (f != 0.0L)
        for (int j = k + 1; j < n; ++j) A[size_t(i) * n + j] -= f * A[size_t(k) * n + j];
    }
  }
  return true;
}

// Solve A X = B for X (n x m, row-major), B overwritten.
void lu_solve(const Mat& LU, const std::vector<int>& piv, int n, Mat& B, int m) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k)
      for (int j = 0; j < m; ++j) std::swap(B[size_t(k) * m + j], B[size_t(piv[k]) * m + j]);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < i; ++k) {
      const ld f = LU[size_t(i) * n + k];
      if (f != 0.0L)
        for (int j = 0; j < m; ++j) B[size_t(i) * m + j] -= f * B[size_t(k) * m + j];
    }
  for (int i = n - 1; i >= 0; --i) {
    const ld inv = 1.0L / LU[size_t(i) * n + i];
    for (int k = i + 1; k < n; ++k) {
      const ld f = LU[size_t(i) * n + k];
      if (f != 0.0L)
        for (int j = 0; j < m; ++j) B[size_t(i) * m + j] -= f * B[size_t(k) * m + j];
    }
    for (int j = 0; j < m; ++j) B[size_t(i) * m + j] *= inv;
  }
}

Mat matmul(const Mat& A, const Mat& B, int n) {
  Mat C(size_t(n) * n, 0.0L);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const ld a = A[size_t(i) * n + k];
      if (a == 0.0L) continue;
      for (int j = 0; j < n; ++j) C[size_t(i) * n + j] += a * B[size_t(k) * n + j];
    }
  return C;
}

ld inf_norm(const Mat& A, int n) {
  ld best = 0.0L;
  for (int i = 0; i < n; ++i) {
    ld s = 0.0L;
    for (int j = 0; j < n; ++j) s += std::fabs(A[size_t(i) * n + j]);
    best = std::max(best, s);
  }
  return best;
}

struct Cheb {
  int My, N;
  std::vector<ld> y;
  Mat D1, D2;         // My x My
  Mat D2D, D2c, D4c;  // N x N
  Mat D1c;            // My x N (stored My*N)
};

// First-derivative collocation matrix on the Gauss-Lobatto points (ascending),
// D_ij = (c_i/c_j)(-1)^(i+j)/(y_i - y_j), c = 2 at the ends, negative-sum diagonal.
void build_cheb(int My, Cheb* ch) {
  const int n = My;
  ch->My = My;
  ch->N = My - 2;
  ch->y.resize(n);
  for (int j = 0; j < n; ++j) ch->y[j] = -std::cos(kPi * ld(j) / ld(n - 1));
  ch->D1.assign(size_t(n) * n, 0.0L);
  std::vector<ld> c(n, 1.0L);
  c[0] = c[n - 1] = 2.0L;
  for (int i = 0; i < n; ++i) {
    ld rowsum = 0.0L;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      const ld sgn = ((i + j) % 2) ? -1.0L : 1.0L;
      const ld v = (c[i] / c[j]) * sgn / (ch->y[i] - ch->y[j]);
      ch->D1[size_t(i) * n + j] = v;
      rowsum += v;
    }
    ch->D1[size_t(i) * n + i] = -rowsum;
  }
  ch->D2 = matmul(ch->D1, ch->D1, n);
  const int N = n - 2;
  ch->D2D.assign(size_t(N) * N, 0.0L);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) ch->D2D[size_t(i) * N + j] = ch->D2[size_t(i + 1) * n + (j + 1)];

  // Clamped operators: p(y) = sum_j w(y) l_j(y) / w(y_j) v_j, w = (1 - y^2)^2,
  // l_j Lagrange on the N interior nodes; derivatives by the Leibniz rule.
  std::vector<ld> x(ch->y.begin() + 1, ch->y.end() - 1);
  std::vector<ld> bw(N, 1.0L);
  for (int j = 0; j < N; ++j)
    for (int k = 0; k < N; ++k)
      if (k != j) bw[j] *= (x[j] - x[k]);
  Mat Dt(size_t(N) * N, 0.0L);
  for (int i = 0; i < N; ++i) {
    ld rs = 0.0L;
    for (int j = 0; j < N; ++j) {
      if (i == j) continue;
      const ld v = (bw[i] / bw[j]) / (x[i] - x[j]);
      Dt[size_t(i) * N + j] = v;
      rs += v;
    }
    Dt[size_t(i) * N + i] = -rs;
  }
  const Mat Dt2 = matmul(Dt, Dt, N);
  const Mat Dt3 = matmul(Dt2, Dt, N);
  const Mat Dt4 = matmul(Dt3, Dt, N);
  ch->D2c.assign(size_t(N) * N, 0.0L);
  ch->D4c.assign(size_t(N) * N, 0.0L);
  Mat D1ci(size_t(N) * N, 0.0L);
  for (int i = 0; i < N; ++i) {
    const ld yi = x[i];
    const ld w0 = (1 - yi * yi) * (1 - yi * yi);
    const ld w1 = -4 * yi + 4 * yi * yi * yi;
    const ld w2 = -4 + 12 * yi * yi;
    const ld w3 = 24 * yi;
    const ld w4 = 24;
    for (int j = 0; j < N; ++j) {
      const ld s = 1.0L / ((1 - x[j] * x[j]) * (1 - x[j] * x[j]));
      const ld id = (i == j) ? 1.0L : 0.0L;
      const size_t ij = size_t(i) * N + j;
      D1ci[ij] = (w1 * id + w0 * Dt[ij]) * s;
      ch->D2c[ij] = (w2 * id + 2 * w1 * Dt[ij] + w0 * Dt2[ij]) * s;
      ch->D4c[ij] = (w4 * id + 4 * w3 * Dt[ij] + 6 * w2 * Dt2[ij] + 4 * w1 * Dt3[ij] + w0 * Dt4[ij]) * s;
    }
  }
  ch->D1c.assign(size_t(n) * N, 0.0L);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) ch->D1c[size_t(i + 1) * N + j] = D1ci[size_t(i) * N + j];
}

// Clenshaw-Curtis weights on the Gauss-Lobatto points (closed form).
std::vector<ld> cc_weights(int My) {
  const int n = My - 1;
  std::vector<ld> w(My, 0.0L);
  std::vector<ld> v(n - 1 > 0 ? n - 1 : 0, 1.0L);
  if (n % 2 == 0) {
    w[0] = w[n] = 1.0L / (ld(n) * n - 1);
    for (int k = 1; k < n / 2; ++k)
      for (int j = 1; j < n; ++j) v[j - 1] -= 2 * std::cos(2 * k * kPi * j / n) / (4 * ld(k) * k - 1);
    for (int j = 1; j < n; ++j) v[j - 1] -= std::cos(n * kPi * j / n) / (ld(n) * n - 1);
  } else {
    w[0] = w[n] = 1.0L / (ld(n) * n);
    for (int k = 1; k <= (n - 1) / 2; ++k)
      for (int j = 1; j < n; ++j) v[j - 1] -= 2 * std::cos(2 * k * kPi * j / n) / (4 * ld(k) * k - 1);
  }
  for (int j = 1; j < n; ++j) w[j] = 2 * v[j - 1] / n;
  return w;
}

// A = lhs^{-1} rhs and B = lhs^{-1}; returns an estimate of cond_inf(lhs).
ld fold_pair(const Mat& lhs, const Mat& rhs, int n, double* A, double* B) {
  Mat LU = lhs;
  std::vector<int> piv;
  if (!lu_factor(LU, piv, n)) return INFINITY;
  Mat X = rhs;
  lu_solve(LU, piv, n, X, n);
  Mat I(size_t(n) * n, 0.0L);
  for (int i = 0; i < n; ++i) I[size_t(i) * n + i] = 1.0L;
  lu_solve(LU, piv, n, I, n);
  for (size_t q = 0; q < size_t(n) * n; ++q) {
    A[q] = double(X[q]);
    B[q] = double(I[q]);
  }
  return inf_norm(lhs, n) * inf_norm(I, n);
}

// Helmholtz-Poisson (Kim-Moin-Moser) form of the v step: with phi = Lap v a
// polynomial on all My nodes,
//   [I - c Lap] phi_new = [I + c Lap] Lap v_0 - h dt F   (interior nodes)
//   Lap v_new = phi_new                                   (interior nodes)
//   v_new = 0 and d v_new/dy = 0                          (walls)
// solved as one block system for (phi, v); A = S Q and B = S with S the
// v-rows of its inverse on the Helmholtz right-hand side and Q = [I + c Lap]
// Lap restricted to interior rows and columns.  Returns a lower-bound estimate
// of cond_inf of the block matrix.
ld kmm_pair(const Cheb& ch, ld k2, ld c, double* A, double* B) {
  const int My = ch.My, N = ch.N, n = My + N;
  Mat lapf(size_t(My) * My);
  for (int i = 0; i < My; ++i)
    for (int j = 0; j < My; ++j) lapf[size_t(i) * My + j] = ch.D2[size_t(i) * My + j] - (i == j ? k2 : 0.0L);
  Mat M(size_t(n) * n, 0.0L);
  for (int i = 0; i < N; ++i) {
    const int r = i + 1;  // interior node
    for (int j = 0; j < My; ++j) {
      M[size_t(i) * n + j] = (r == j ? 1.0L : 0.0L) - c * lapf[size_t(r) * My + j];  // Helmholtz
    }
    M[size_t(N + i) * n + r] = -1.0L;                                                   // Poisson: -phi
    for (int j = 0; j < N; ++j) M[size_t(N + i) * n + My + j] = lapf[size_t(r) * My + j + 1];
  }
  for (int j = 0; j < N; ++j) {
    M[size_t(2 * N) * n + My + j] = ch.D1[size_t(0) * My + j + 1];
    M[size_t(2 * N + 1) * n + My + j] = ch.D1[size_t(My - 1) * My + j + 1];
  }
  Mat LU = M;
  std::vector<int> piv;
  if (!lu_factor(LU, piv, n)) return INFINITY;
  Mat X(size_t(n) * N, 0.0L);  // columns: unit right-hand sides of the Helmholtz rows
  for (int i = 0; i < N; ++i) X[size_t(i) * N + i] = 1.0L;
  lu_solve(LU, piv, n, X, N);
  // Q = ([I + c Lap] Lap[:, interior])[interior rows]
  Mat Q(size_t(N) * N, 0.0L);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const int r = i + 1;
      ld q = lapf[size_t(r) * My + j + 1];
      for (int m = 0; m < My; ++m) q += c * lapf[size_t(r) * My + m] * lapf[size_t(m) * My + j + 1];
      Q[size_t(i) * N + j] = q;
    }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      ld a = 0.0L;
      for (int m = 0; m < N; ++m) a += X[size_t(My + i) * N + m] * Q[size_t(m) * N + j];
      A[size_t(i) * N + j] = double(a);
      B[size_t(i) * N + j] = double(X[size_t(My + i) * N + j]);
    }
  // conditioning estimate from the inverse columns already at hand (a lower
  // bound of cond_inf(M); a full inverse would cost n^3 per mode)
  ld xmax = 0.0L;
  for (int i = 0; i < n; ++i) {
    ld row = 0.0L;
    for (int j = 0; j < N; ++j) row += std::fabs(X[size_t(i) * N + j]);
    xmax = std::max(xmax, row);
  }
  return inf_norm(M, n) * xmax;
}

}  // namespace

std::vector<double> tile_for_mfma(const double* M, int R, int Kd, int ldm) {
  const int RT = (R + 15) / 16, KT = (Kd + 3) / 4;
  std::vector<double> out(size_t(RT) * KT * 64, 0.0);
  for (int rt = 0; rt < RT; ++rt)
    for (int kt = 0; kt < KT; ++kt)
      for (int l = 0; l < 64; ++l) {
        const int r = rt * 16 + l % 16, k = kt * 4 + l / 16;
        if (r < R && k < Kd) out[(size_t(rt) * KT + kt) * 64 + l] = M[size_t(r) * ldm + k];
      }
  return out;
}

namespace {
unsigned short bf16_rne(float f) {
  unsigned int u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}
float bf16_value(unsigned short h) {
  const unsigned int u = static_cast<unsigned int>(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
}  // namespace

void tile_for_mfma_bf16(const double* M, int R, int Kd, int ldm, std::vector<unsigned short>* hi,
                        std::vector<unsigned short>* lo) {
  const int RT = (R + 15) / 16, KT = (Kd + 15) / 16;
  hi->assign(size_t(RT) * KT * 256, 0);
  lo->assign(size_t(RT) * KT * 256, 0);
  for (int rt = 0; rt < RT; ++rt)
    for (int kt = 0; kt < KT; ++kt)
      for (int l = 0; l < 64; ++l)
        for (int t = 0; t < 4; ++t) {
          const int r = rt * 16 + l % 16, k = kt * 16 + 4 * (l / 16) + t;
          if (r >= R || k >= Kd) continue;
          const double m = M[size_t(r) * ldm + k];
          const unsigned short h = bf16_rne(float(m));
          const size_t o = ((size_t(rt) * KT + kt) * 64 + l) * 4 + t;
          (*hi)[o] = h;
          (*lo)[o] = bf16_rne(float(m - double(bf16_value(h))));
        }
}

std::vector<double> half_block(const double* M, int rows_out, int Cn, int ldm, bool even_in) {
  const int ncol = even_in ? (Cn + 1) / 2 : Cn / 2;
  std::vector<double> out(size_t(rows_out) * ncol, 0.0);
  for (int i = 0; i < rows_out; ++i)
    for (int k = 0; k < ncol; ++k) {
      const double a = M[size_t(i) * ldm + k];
      const double b = M[size_t(i) * ldm + (Cn - 1 - k)];
      double v;
      if (even_in) v = (k < Cn / 2) ? a + b : a;  // centre column when Cn is odd
      else v = a - b;
      out[size_t(i) * ncol + k] = v;
    }
  return out;
}

int build_operators(int My, int L, int P, double kxs, double kzs, double Re, double dt, double Ubot,
                    double Utop, HostOperators* out, int v_discretization) {
  Cheb ch;
  build_cheb(My, &ch);
  const int N = My - 2;
  const int G = L * P;
  out->My = My;
  out->N = N;
  out->G = G;
  out->D1.resize(size_t(My) * My);
  for (size_t q = 0; q < out->D1.size(); ++q) out->D1[q] = double(ch.D1[q]);
  out->D1c.resize(size_t(My) * N);
  for (size_t q = 0; q < out->D1c.size(); ++q) out->D1c[q] = double(ch.D1c[q]);
  const std::vector<ld> w = cc_weights(My);
  out->ccw.assign(w.begin(), w.end());

  const ld hs[2] = {0.5L, 1.0L};
  std::vector<ld> conds(size_t(2) * G, 0.0L);
  for (int hi = 0; hi < 2; ++hi) {
    const ld c = hs[hi] * ld(dt) / (2.0L * ld(Re));
    out->ops[hi].assign(size_t(G) * 4 * N * N, 0.0);
    // mean operators (k = 0), Eqs. (CN3)-(CN4)
    {
      Mat lhs(size_t(N) * N), rhs(size_t(N) * N);
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          const ld id = i == j ? 1.0L : 0.0L;
          lhs[size_t(i) * N + j] = id - c * ch.D2D[size_t(i) * N + j];
          rhs[size_t(i) * N + j] = id + c * ch.D2D[size_t(i) * N + j];
        }
      out->mean_ops[hi].assign(size_t(2) * N * N, 0.0);
      fold_pair(lhs, rhs, N, out->mean_ops[hi].data(), out->mean_ops[hi].data() + size_t(N) * N);
      Mat LU = lhs;
      std::vector<int> piv;
      lu_factor(LU, piv, N);
      Mat rl(size_t(N) * 2, 0.0L);
      for (int i = 0; i < N; ++i) {
        rl[size_t(i) * 2 + 0] = 2.0L * c * (ch.D2[size_t(i + 1) * My + 0] * ld(Ubot) +
                                             ch.D2[size_t(i + 1) * My + (My - 1)] * ld(Utop));
        rl[size_t(i) * 2 + 1] = hs[hi] * ld(dt);
      }
      lu_solve(LU, piv, N, rl, 2);
      out->lift[hi].resize(N);
      out->green[hi].resize(N);
      for (int i = 0; i < N; ++i) {
        out->lift[hi][i] = double(rl[size_t(i) * 2 + 0]);
        out->green[hi][i] = double(rl[size_t(i) * 2 + 1]);
      }
    }
    // fluctuation operators per group g = nx * P + |nz|, g > 0
    auto work = [&](int g0, int g1) {
      Mat lhs(size_t(N) * N), rhs(size_t(N) * N), lhe(size_t(N) * N), rhe(size_t(N) * N);
      for (int g = std::max(g0, 1); g < g1; ++g) {
        const int nx = g / P, az = g % P;
        const ld kx = ld(kxs) * nx, kz = ld(kzs) * az;
        const ld k2 = kx * kx + kz * kz;
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j) {
            const size_t ij = size_t(i) * N + j;
            const ld id = i == j ? 1.0L : 0.0L;
            const ld lap = ch.D2D[ij] - k2 * id;
            const ld laplap = ch.D4c[ij] - 2.0L * k2 * ch.D2c[ij] + k2 * k2 * id;
            lhs[ij] = lap - c * laplap;
            rhs[ij] = lap + c * laplap;
            lhe[ij] = id - c * lap;
            rhe[ij] = id + c * lap;
          }
        double* base = out->ops[hi].data() + size_t(g) * 4 * N * N;
        const ld cv = v_discretization == 1 ? kmm_pair(ch, k2, c, base, base + size_t(N) * N)
                                            : fold_pair(lhs, rhs, N, base, base + size_t(N) * N);
        const ld ce = fold_pair(lhe, rhe, N, base + size_t(2) * N * N, base + size_t(3) * N * N);
        conds[size_t(hi) * G + g] = std::max(cv, ce);
      }
    };
    unsigned nth = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    const int per = (G + int(nth) - 1) / int(nth);
    for (unsigned t = 0; t < nth; ++t) {
      const int g0 = int(t) * per, g1 = std::min(G, g0 + per);
      if (g0 < g1) pool.emplace_back(work, g0, g1);
    }
    for (auto& th : pool) th.join();
  }
  ld mc = 0.0L;
  for (ld v : conds) mc = std::max(mc, v);
  out->max_cond = double(mc);
  return std::isfinite(out->max_cond) ? 0 : -1;
}

}  // namespace dns
