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
// y-parity split.  The Gauss-Lobatto grid is symmetric under y -> -y (node j
// <-> My-1-j).  Every CN operator commutes with that reflection and D1, D1c
// anticommute with it, so in the basis of even halves e[k] = (x[k] +
// x[n-1-k])/2 and odd halves o[k] = (x[k] - x[n-1-k])/2 each product splits
// into two half-size products (even -> even and odd -> odd for the operators,
// even -> odd and odd -> even for the derivatives).  This halves the matrix
// work and the operator stream; the pointwise steps act on halves unchanged
// because their coefficients do not depend on y.
//
// Every half-size contraction Y = M X runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64, one 16x16 output tile per wavefront, K in steps of
// 4).  Matrices are stored pre-tiled in the MFMA A lane order (tile (rt, kt) =
// 64 consecutive doubles, lane l holding M[16 rt + l % 16][4 kt + l / 16]), so
// each A fragment is one coalesced 512 B load; X lives in LDS as [k][column].
// With the split-BF16 precision the six y-derivative contractions instead run
// as three bfloat16 products on v_mfma_f32_16x16x16bf16_1k, and with the FP32
// matrix-core precision on v_mfma_f32_16x16x4f32 (the solves stay FP64).
#include <hip/hip_runtime.h>

#include "internal.h"

// Multiply-adds are fused only within one source expression, so that the same
// arithmetic inlined into the single-ensemble and the grouped kernel rounds
// the same way (fusion across statements follows instruction scheduling).
#pragma clang fp contract(on)

namespace dns {

namespace {

__device__ __forceinline__ int xcd_logical_m(int b, int nblk) {
  const int q = nblk >> 3, rem = nblk & 7;
  const int x = b & 7, local = b >> 3;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + local;
}

// The workgroup size NT (512 or 1024 threads: kModeThreadsNarrow, kModeThreadsWide) is a
// template parameter of the kernel and of every helper below; NT / 64 waves.
static_assert(mode_static_lds(kModeThreadsNarrow) == (kModeThreadsNarrow / 64 * 16 + 64) * sizeof(double) &&
                  mode_static_lds(kModeThreadsWide) == (kModeThreadsWide / 64 * 16 + 64) * sizeof(double),
              "static LDS of mode_body");

typedef double d4 __attribute__((ext_vector_type(4)));

// Dynamic LDS of the per-mode kernel: its work buffers, rows of ld doubles.
// With 32-double rows the two 16-column halves of every odd row (rows counted
// from the start of the LDS) trade places.  At a 256-byte row stride two
// consecutive rows would put the same columns in the same banks, and a
// matrix-core fragment reads (and its result writes) consecutive rows from the
// two half-waves of one LDS pass; 16-double rows already put consecutive rows
// in different banks and stay as they are.
extern __shared__ double mode_smem[];
__device__ __forceinline__ int lds_swz_mask(int ld) { return ld == 32 ? 16 : 0; }
__device__ __forceinline__ int lds_swz(int i, int m) { return i ^ ((i >> 1) & m); }
// Address of logical element i of the LDS, in a buffer with rows of ld doubles.
__device__ __forceinline__ const double* lds_at(int i, int ld) { return mode_smem + lds_swz(i, lds_swz_mask(ld)); }

// One work buffer: rows of ld doubles from element off of the dynamic LDS.
struct LdsBuf {
  int off, ld, m;
  __device__ double& operator[](int i) const { return mode_smem[lds_swz(off + i, m)]; }
  // elements i and i + 1 for even i (the swizzle keeps them adjacent)
  __device__ double* pair(int i) const { return mode_smem + lds_swz(off + i, m); }
  // logical element offset of row r, an operand of the contractions (which swizzle)
  __device__ int row(int r) const { return off + r * ld; }
};

// Y = M X over every output tile of this workgroup; store(row, col, value) is
// called once per element with row < 16 RT, col < 16 CT (the caller ignores
// padding rows).  M: tiled matrix with K = 4 KT columns (zero padded),
// X: logical element offset of the first row of an LDS buffer (LdsBuf
// layout), row stride ldx, at least 4 KT finite rows.
// D layout of v_mfma_f64_16x16x4f64: lane l, register r -> row l/16 + 4r, col l%16.
template <int NT, class Store>
__device__ __forceinline__ void mfma_contract(const double* __restrict__ Mt, int RT, int KT,
                                              int X, int ldx, int CT, Store store) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar tile arithmetic
  const int lr = lane & 15, lk = lane >> 4;
  for (int t = wave; t < RT * CT; t += (NT / 64)) {
    const int rt = t / CT, ct = t - rt * CT;
    const double* a = Mt + size_t(rt) * KT * 64 + lane;
    const double* b = lds_at(X + lk * ldx + ct * 16 + lr, ldx);  // rows lk + 4 kt: one parity
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

// One job of a multi-job contraction: Y = M X for a tiled M (RT row tiles, KT
// k-steps) and an LDS operand X.
struct CJob {
  const double* Mt;
  int RT, KT;
  int X;  // logical LDS element offset of the operand's first row
};

// U k-steps of one tile (or of two tiles, interleaved) from k-step kt while
// kt + U <= kend: all U fragment loads are issued before the first product,
// and every tile's products accumulate in ascending k.
template <int U>
__device__ __forceinline__ void tile_steps(const double* a, const double* b, int ldx, d4& acc, int& kt, int kend) {
  for (; kt + U <= kend; kt += U) {
    double p[U], x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) p[u] = a[(kt + u) * 64];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = b[(4 * (kt + u)) * ldx];
#pragma unroll
    for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(p[u], x[u], acc, 0, 0, 0);
  }
}

template <int U>
__device__ __forceinline__ void tile_pair_steps(const double* a1, const double* b1, d4& acc1, const double* a2,
                                                const double* b2, d4& acc2, int ldx, int& kt, int kend) {
  for (; kt + U <= kend; kt += U) {
    double p[U], q[U], x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      p[u] = a1[(kt + u) * 64];
      q[u] = a2[(kt + u) * 64];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x[u] = b1[(4 * (kt + u)) * ldx];
      y[u] = b2[(4 * (kt + u)) * ldx];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(p[u], x[u], acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(q[u], y[u], acc2, 0, 0, 0);
    }
  }
}

// k-steps whose fragment loads a wave keeps in flight per tile
constexpr int kKUnroll = 8;

template <int U>
__device__ __forceinline__ void tile_tail(const double* a, const double* b, int ldx, d4& acc, int& kt, int kend) {
  tile_steps<U>(a, b, ldx, acc, kt, kend);
  if constexpr (U > 1) tile_tail<U / 2>(a, b, ldx, acc, kt, kend);
}

template <int U>
__device__ __forceinline__ void tile_pair_tail(const double* a1, const double* b1, d4& acc1, const double* a2,
                                               const double* b2, d4& acc2, int ldx, int& kt, int kend) {
  tile_pair_steps<U>(a1, b1, acc1, a2, b2, acc2, ldx, kt, kend);
  if constexpr (U > 1) tile_pair_tail<U / 2>(a1, b1, acc1, a2, b2, acc2, ldx, kt, kend);
}

// Output tiles (rt1, ct1) of J1 and, if has2, (rt2, ct2) of J2, with their
// fragment loads interleaved so that a wave keeps twice as many loads in
// flight; each tile's products accumulate in ascending k from zero, as in
// mfma_contract, so the results equal its results.
__device__ __forceinline__ void mfma_tile_pair(const CJob J1, int rt1, int ct1, bool has2, const CJob J2, int rt2,
                                               int ct2, int ldx, d4& acc1, d4& acc2) {
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const double* a1 = J1.Mt + size_t(rt1) * J1.KT * 64 + lane;
  const double* b1 = lds_at(J1.X + lk * ldx + ct1 * 16 + lr, ldx);
  acc1 = d4{0.0, 0.0, 0.0, 0.0};
  acc2 = d4{0.0, 0.0, 0.0, 0.0};
  int kt = 0;
  if (has2) {
    const double* a2 = J2.Mt + size_t(rt2) * J2.KT * 64 + lane;
    const double* b2 = lds_at(J2.X + lk * ldx + ct2 * 16 + lr, ldx);
    const int kc = J1.KT < J2.KT ? J1.KT : J2.KT;
    tile_pair_tail<kKUnroll>(a1, b1, acc1, a2, b2, acc2, ldx, kt, kc);
    int k2 = kt;
    tile_tail<kKUnroll>(a2, b2, ldx, acc2, k2, J2.KT);
  }
  tile_tail<kKUnroll>(a1, b1, ldx, acc1, kt, J1.KT);
}

// Every output tile of NJ jobs that share the column tiling (CT) and the
// operand row stride ldx: tiles are numbered job-major and wave w takes tiles
// w, w + (waves), ... two at a time.  store(job, row, col, value) as in
// mfma_contract.  kDefer: every wave first computes all its tiles (at most
// kMaxHeld) into registers, the workgroup synchronises, then the stores run,
// so a job may overwrite any job's operand; the caller checks the tile count
// (mfma_jobs_fit).
constexpr int kMaxHeld = 4;
template <int NT, int NJ>
__device__ __forceinline__ bool mfma_jobs_fit(const CJob (&job)[NJ], int CT) {
  int total = 0;
#pragma unroll
  for (int j = 0; j < NJ; ++j) total += job[j].RT * CT;
  return total <= kMaxHeld * (NT / 64);
}

template <int NT, bool kDefer, int NJ, class Store>
__device__ __forceinline__ void mfma_jobs(const CJob (&job)[NJ], int ldx, int CT, Store store) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar tile arithmetic
  const int lr = lane & 15, lk = lane >> 4;
  int base[NJ + 1];
  base[0] = 0;
#pragma unroll
  for (int j = 0; j < NJ; ++j) base[j + 1] = base[j] + job[j].RT * CT;
  const int total = base[NJ];
  // tile t -> job, row tile, column tile; t is uniform over the wave, so the
  // job is chosen by selects rather than by indexing (no stack copy)
  auto decode = [&](int t, CJob* J, int* j, int* rt, int* ct) {
    int jj = 0, b0 = 0;
    CJob sel = job[0];
#pragma unroll
    for (int q = 1; q < NJ; ++q) {
      if (t >= base[q]) {
        jj = q;
        b0 = base[q];
        sel = job[q];
      }
    }
    const int local = t - b0;
    *J = sel;
    *j = jj;
    *rt = local / CT;
    *ct = local - *rt * CT;
  };
  auto put = [&](int t, const d4& acc) {
    CJob J;
    int j, rt, ct;
    decode(t, &J, &j, &rt, &ct);
#pragma unroll
    for (int r = 0; r < 4; ++r) store(j, rt * 16 + lk + 4 * r, ct * 16 + lr, acc[r]);
  };
  if constexpr (kDefer) {
    d4 held[kMaxHeld];
#pragma unroll
    for (int i = 0; i < kMaxHeld; i += 2) {
      const int t1 = wave + i * (NT / 64), t2 = t1 + (NT / 64);
      if (t1 < total) {
        CJob J1, J2 = job[0];
        int j1, rt1, ct1, j2 = 0, rt2 = 0, ct2 = 0;
        decode(t1, &J1, &j1, &rt1, &ct1);
        if (t2 < total) decode(t2, &J2, &j2, &rt2, &ct2);
        mfma_tile_pair(J1, rt1, ct1, t2 < total, J2, rt2, ct2, ldx, held[i], held[i + 1]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMaxHeld; ++i) {
      const int t = wave + i * (NT / 64);
      if (t < total) put(t, held[i]);
    }
  } else {
    for (int t1 = wave; t1 < total; t1 += 2 * (NT / 64)) {
      const int t2 = t1 + (NT / 64);
      CJob J1, J2 = job[0];
      int j1, rt1, ct1, j2 = 0, rt2 = 0, ct2 = 0;
      decode(t1, &J1, &j1, &rt1, &ct1);
      if (t2 < total) decode(t2, &J2, &j2, &rt2, &ct2);
      d4 acc1, acc2;
      mfma_tile_pair(J1, rt1, ct1, t2 < total, J2, rt2, ct2, ldx, acc1, acc2);
      put(t1, acc1);
      if (t2 < total) put(t2, acc2);
    }
  }
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return static_cast<short>(u >> 16);
}
__device__ __forceinline__ float bf16_value(short h) {
  return __uint_as_float(static_cast<unsigned int>(static_cast<unsigned short>(h)) << 16);
}

// Split-BF16 variant of mfma_contract: M = Mhi + Mlo (pre-tiled bfloat16 pairs,
// K in steps of 16), X rounded to FP32 and split the same way on the fly;
// M X ~ Mhi Xhi + Mhi Xlo + Mlo Xhi on v_mfma_f32_16x16x16bf16_1k with FP32
// accumulation (the Mlo Xlo term is below FP32 resolution).  X needs 16 KT
// finite rows.  D layout: lane l, register r -> row 4 (l / 16) + r, col l % 16.
template <int NT, class Store>
__device__ __forceinline__ void mfma_contract_split(const unsigned short* __restrict__ Hi,
                                                    const unsigned short* __restrict__ Lo, int RT, int KT,
                                                    int X, int ldx, int CT, Store store) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar tile arithmetic
  const int lr = lane & 15, lk = (lane >> 4) * 4;
  for (int t = wave; t < RT * CT; t += (NT / 64)) {
    const int rt = t / CT, ct = t - rt * CT;
    const bf16x4* ah = reinterpret_cast<const bf16x4*>(Hi) + size_t(rt) * KT * 64 + lane;
    const bf16x4* al = reinterpret_cast<const bf16x4*>(Lo) + size_t(rt) * KT * 64 + lane;
    // rows lk + q + 16 kt: even q on b0's parity, odd q on b1's
    const double* b0 = lds_at(X + lk * ldx + ct * 16 + lr, ldx);
    const double* b1 = lds_at(X + (lk + 1) * ldx + ct * 16 + lr, ldx);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < KT; ++kt) {
      const bf16x4 a_hi = ah[kt * 64], a_lo = al[kt * 64];
      bf16x4 b_hi, b_lo;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float x = float((q & 1 ? b1 : b0)[(16 * kt + (q & ~1)) * ldx]);
        const short h = bf16_bits(x);
        b_hi[q] = h;
        b_lo[q] = bf16_bits(x - bf16_value(h));
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_hi, b_hi, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_hi, b_lo, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_lo, b_hi, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) store(rt * 16 + lk + r, ct * 16 + lr, double(acc[r]));
  }
}

// FP32 variant of mfma_contract: M in FP32, in the A lane order of the FP64
// tiles (K = 4 KT), X rounded to FP32, FP32 accumulation on
// v_mfma_f32_16x16x4f32.  D layout: lane l, register r -> row 4 (l / 16) + r,
// col l % 16.
template <int NT, class Store>
__device__ __forceinline__ void mfma_contract_f32(const float* __restrict__ Mt, int RT, int KT, int X,
                                                  int ldx, int CT, Store store) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar tile arithmetic
  const int lr = lane & 15, lk = lane >> 4;
  for (int t = wave; t < RT * CT; t += (NT / 64)) {
    const int rt = t / CT, ct = t - rt * CT;
    const float* a = Mt + size_t(rt) * KT * 64 + lane;
    const double* b = lds_at(X + lk * ldx + ct * 16 + lr, ldx);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    int kt = 0;
    for (; kt + 4 <= KT; kt += 4) {
      float p[4], x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) p[u] = a[(kt + u) * 64];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = float(b[(4 * (kt + u)) * ldx]);
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(p[u], x[u], acc, 0, 0, 0);
    }
    for (; kt < KT; ++kt)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kt * 64], float(b[4 * kt * ldx]), acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) store(rt * 16 + 4 * lk + r, ct * 16 + lr, double(acc[r]));
  }
}

// y-derivative arithmetic of the per-mode kernel: FP64 matrix cores, split
// BF16 (three bfloat16 products) or FP32 matrix cores
constexpr int kDerFP64 = 0, kDerSplitBF16 = 1, kDerFP32 = 2;

// A y-derivative contraction (one of the six parity halves, index `which`).
// Kd is the K dimension.
template <int kDer, int NT, class Store>
__device__ __forceinline__ void dcontract(const ModeArgs& a, int which, const double* Mt, int RT, int Kd,
                                          int X, int ldx, int CT, Store store) {
  if constexpr (kDer == kDerSplitBF16)
    mfma_contract_split<NT>(a.Dhi[which], a.Dlo[which], RT, (Kd + 15) / 16, X, ldx, CT, store);
  else if constexpr (kDer == kDerFP32)
    mfma_contract_f32<NT>(a.Df[which], RT, (Kd + 3) / 4, X, ldx, CT, store);
  else
    mfma_contract<NT>(Mt, RT, (Kd + 3) / 4, X, ldx, CT, store);
}

template <typename VT>
struct Pair;
template <> struct Pair<float> { typedef float2 type; };
template <> struct Pair<double> { typedef double2 type; };

// One complex value as one vector store (p is even in VT units, so aligned to
// the pair): the real and imaginary parts never reach memory separately.
template <typename VT>
__device__ __forceinline__ void st_c(VT* p, double re, double im) {
  typename Pair<VT>::type v;
  v.x = VT(re);
  v.y = VT(im);
  *reinterpret_cast<typename Pair<VT>::type*>(p) = v;
}

}  // namespace

// Half sizes: interior N = My - 2 splits into He = ceil(N/2) even and Ho =
// floor(N/2) odd rows; the full grid into Fe = He + 1 and Fo = Ho + 1 (the
// wall pair adds one row to each parity).
//
// LDS buffers (doubles, row stride CRP = real columns padded to 16):
//   full-half layout FH : rows [0, Fe) even, [Fe, My) odd; row 0 / Fe = walls
//   S  : solve stack [v0_e; F'_e; v0_o; F'_o] (interior halves), later eta (FH)
//   S2 : solve stack [eta0_e; G'_e; eta0_o; G'_o], later dv/dy, u, dw/dy (FH)
//   T  : Q = i kx N_u + i kz N_w (FH), later v (FH), later du/dy (FH)
// The per-mode work of workgroup `flat` (a group and member tile) of the
// launch described by `a`.
template <typename VT, int kDer, bool kForce, int NT>
__device__ __forceinline__ void mode_body(const ModeArgs& a, int flat) {
  const int tid = threadIdx.x;
  const int My = a.My, N = a.N, K = a.K, E = a.E, NZ = a.NZ, P = a.P, ET = a.ET;
  const int He = (N + 1) / 2, Ho = N / 2, Fe = He + 1, Fo = Ho + 1;
  const int C = 2 * ET;           // complex columns: (slot, member)
  const int CRP = a.CRP;          // real columns, padded to 16
  const int CT = CRP / 16;
  const int SR = a.SR, TR = a.TR;
  const int swm = lds_swz_mask(CRP);
  const LdsBuf S{0, CRP, swm}, S2{SR * CRP, CRP, swm}, T{2 * SR * CRP, CRP, swm};
  __shared__ double red[(NT / 64) * 16];  // per-wave maxima of <= 16 columns
  __shared__ double gam_s[64];

  const int g = flat / a.ntiles;
  const int tile = flat - g * a.ntiles;
  const int nx = g / P, az = g - nx * P;
  const bool mean_group = (g == 0);
  // a frozen streamwise mean: its groups keep their state and stage velocities
  if (a.freeze_mean && nx == 0 && a.stage >= 0) return;
  VT* vel = static_cast<VT*>(a.vel);
  const VT* nl = static_cast<const VT*>(a.nl);
  const int s = a.stage;
  const double hdt = a.hdt;
  const size_t KE = size_t(K) * E;
  const size_t FS = 2 * size_t(My) * KE;  // stage-buffer field stride (VT units)

  const int m0 = a.e0, mend = a.e0 + a.ec;  // members of this launch
  // ET is a power of two: index arithmetic by shifts and masks
  const int ets = __ffs(ET) - 1, cs = ets + 1;  // C = 2 ET = 1 << cs
  auto col_member = [&](int c) { return m0 + tile * ET + (c & (ET - 1)); };
  auto col_valid = [&](int c) {
    const int sl = c >> ets;
    return m0 + tile * ET + (c - sl * ET) < mend && (sl == 0 || az > 0);
  };
  auto col_mode = [&](int c) { return nx * NZ + (c < ET ? az : NZ - az); };  // state arrays
  auto col_slot = [&](int c) { return nx * NZ + stage_slot(c < ET ? az : -az); };  // stage buffers
  auto col_kz = [&](int c) { return (c < ET ? 1.0 : -1.0) * a.kzs * az; };
  // stage-buffer element (node j, column c) in VT units
  const int slb = stage_block_log2(E);
  auto sb = [&](int j, int c) { return 2 * stage_off(j, col_member(c), col_slot(c), E, K, slb); };
  // state element (interior node i in [0, N), column c)
  auto st = [&](int i, int c) { return 2 * ((size_t(col_mode(c)) * N + i) * E + col_member(c)); };
  const double kx = a.kxs * nx;

  // zero all buffers once (padding rows and columns must hold finite zeros)
  for (int q = tid; q < (2 * SR + TR) * CRP; q += NT) mode_smem[q] = 0.0;
  __syncthreads();

  // tile counts of the half-size matrices
  const int RTe = (He + 15) / 16, RTo = (Ho + 15) / 16, RFe = (Fe + 15) / 16, RFo = (Fo + 15) / 16;
  const int KSe = (2 * He + 3) / 4, KSo = (2 * Ho + 3) / 4;

  // write the FH pair k of buffer B (re/im columns 2c, 2c+1) to stage field f
  // (node k takes even + odd, node My-1-k even - odd).  Both stores are
  // unconditional so that each stays one vector store: at the centre node of
  // an odd grid (k = Fo, no odd part) both address node k, and the second,
  // in program order, leaves er - 0 = er exactly.
  auto write_pair = [&](const LdsBuf& B, int k, int c, int f) {
    const double er = B.pair(k * CRP + 2 * c)[0], ei = B.pair(k * CRP + 2 * c)[1];
    double orr = 0.0, oi = 0.0;
    if (k < Fo) {
      orr = B.pair((Fe + k) * CRP + 2 * c)[0];
      oi = B.pair((Fe + k) * CRP + 2 * c)[1];
    }
    st_c(vel + f * FS + sb(k, c), er + orr, ei + oi);
    st_c(vel + f * FS + sb(My - 1 - k, c), er - orr, ei - oi);
  };

  if (!mean_group) {
    // ===================== fluctuation modes (k^2 > 0) =====================
    if (s >= 0) {
      // Q on every node (FH), -k^2 N_v and G on interior nodes (solve stacks).
      // Both nodes are loaded unconditionally (at the centre node of an odd
      // grid they coincide, giving he = x, ho = 0), one complex value per
      // load; a thread issues the loads of two items before either's stores
      // (an item outside the tile loads element 0 and stores nothing).
      typedef typename Pair<VT>::type P2;
      auto nl_load = [&](int q, P2 (&x1)[3], P2 (&x2)[3]) {
        const int k = q >> cs, c = q & (C - 1);
        const bool ok = q < Fe * C && col_valid(c);
        const size_t o1 = ok ? sb(k, c) : 0, o2 = ok ? sb(My - 1 - k, c) : 0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          x1[f] = *reinterpret_cast<const P2*>(nl + f * FS + o1);
          x2[f] = *reinterpret_cast<const P2*>(nl + f * FS + o2);
        }
        return ok;
      };
      auto nl_item = [&](int q, const P2 (&x1)[3], const P2 (&x2)[3]) {
        const int k = q >> cs, c = q & (C - 1);
        const double kz = col_kz(c), k2 = kx * kx + kz * kz;
        const bool pair = k < Fo;
        double he[6], ho[6];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          he[2 * f] = 0.5 * (double(x1[f].x) + double(x2[f].x));
          ho[2 * f] = 0.5 * (double(x1[f].x) - double(x2[f].x));
          he[2 * f + 1] = 0.5 * (double(x1[f].y) + double(x2[f].y));
          ho[2 * f + 1] = 0.5 * (double(x1[f].y) - double(x2[f].y));
        }
        // Q = i kx N_u + i kz N_w
        T.pair(k * CRP + 2 * c)[0] = -(kx * he[1] + kz * he[5]);
        T.pair(k * CRP + 2 * c)[1] = kx * he[0] + kz * he[4];
        if (pair) {
          T.pair((Fe + k) * CRP + 2 * c)[0] = -(kx * ho[1] + kz * ho[5]);
          T.pair((Fe + k) * CRP + 2 * c)[1] = kx * ho[0] + kz * ho[4];
        }
        if (k >= 1) {
          const int kk = k - 1;  // interior half index
          S.pair((He + kk) * CRP + 2 * c)[0] = -k2 * he[2];
          S.pair((He + kk) * CRP + 2 * c)[1] = -k2 * he[3];
          S2.pair((He + kk) * CRP + 2 * c)[0] = -(kz * he[1] - kx * he[5]);
          S2.pair((He + kk) * CRP + 2 * c)[1] = kz * he[0] - kx * he[4];
          if (kk < Ho) {
            S.pair((2 * He + Ho + kk) * CRP + 2 * c)[0] = -k2 * ho[2];
            S.pair((2 * He + Ho + kk) * CRP + 2 * c)[1] = -k2 * ho[3];
            S2.pair((2 * He + Ho + kk) * CRP + 2 * c)[0] = -(kz * ho[1] - kx * ho[5]);
            S2.pair((2 * He + Ho + kk) * CRP + 2 * c)[1] = kz * ho[0] - kx * ho[4];
          }
        }
      };
      for (int q = tid; q < Fe * C; q += 2 * NT) {
        P2 a1[3], a2[3], b1[3], b2[3];
        const bool oka = nl_load(q, a1, a2);
        const bool okb = nl_load(q + NT, b1, b2);
        if (oka) nl_item(q, a1, a2);
        if (okb) nl_item(q + NT, b1, b2);
      }
      __syncthreads();
      // F = -k^2 N_v - D1 Q: odd F from even Q, even F from odd Q
      if constexpr (kDer != kDerFP64) {
        dcontract<kDer, NT>(a, 0, a.D1intT_e, RTo, Fe, T.row(0), CRP, CT, [&](int r, int cc, double v) {
          if (r < Ho) S[(2 * He + Ho + r) * CRP + cc] -= v;
        });
        dcontract<kDer, NT>(a, 1, a.D1intT_o, RTe, Fo, T.row(Fe), CRP, CT, [&](int r, int cc, double v) {
          if (r < He) S[(He + r) * CRP + cc] -= v;
        });
      } else {
        const CJob jf[2] = {{a.D1intT_e, RTo, (Fe + 3) / 4, T.row(0)}, {a.D1intT_o, RTe, (Fo + 3) / 4, T.row(Fe)}};
        mfma_jobs<NT, false>(jf, CRP, CT, [&](int j, int r, int cc, double v) {
          if (j == 0) {
            if (r < Ho) S[(2 * He + Ho + r) * CRP + cc] -= v;
          } else if (r < He) {
            S[(He + r) * CRP + cc] -= v;
          }
        });
      }
      __syncthreads();
      // RK3 combination on halves (history kept in half layout); v0, eta0
      // halves.  Half of interior nodes kk and N-1-kk: 0.5 (x1 + sg x2); at the
      // centre node of an odd N the two nodes coincide (sg = 1) and this is
      // x1 exactly, so every load is unconditional; two items per thread.
      // (an item outside the tile loads element 0 and stores nothing)
      struct RkIn {
        double2 v1, v2, e1, e2, hf, hg;
        bool ok;
      };
      auto rk_offsets = [&](int q, size_t* s1, size_t* s2, size_t* so) {
        const int hr = q >> cs, c = q & (C - 1);
        const bool ok = q < N * C && col_valid(c);
        const int kk = hr < He ? hr : hr - He;
        *s1 = ok ? st(kk, c) : 0;
        *s2 = ok ? st(N - 1 - kk, c) : 0;
        *so = ok ? st(hr, c) : 0;
        return ok;
      };
      auto rk_load = [&](int q, RkIn& in) {
        size_t s1, s2, so;
        in.ok = rk_offsets(q, &s1, &s2, &so);
        in.v1 = *reinterpret_cast<const double2*>(a.v + s1);
        in.v2 = *reinterpret_cast<const double2*>(a.v + s2);
        in.e1 = *reinterpret_cast<const double2*>(a.eta + s1);
        in.e2 = *reinterpret_cast<const double2*>(a.eta + s2);
      };
      auto rk_load_hist = [&](int q, RkIn& in) {
        size_t s1, s2, so;
        rk_offsets(q, &s1, &s2, &so);
        in.hf = *reinterpret_cast<const double2*>(a.hF + so);
        in.hg = *reinterpret_cast<const double2*>(a.hG + so);
      };
      auto rk_item = [&](int q, const RkIn& in) {
        const int hr = q >> cs, c = q & (C - 1);
        const bool even = hr < He;
        const int kk = even ? hr : hr - He;
        const int rowF = even ? He + kk : 2 * He + Ho + kk;
        const int rowX = even ? kk : 2 * He + kk;
        const size_t s1 = st(kk, c), s2 = st(N - 1 - kk, c);
        const double sg = even ? 1.0 : -1.0;
        const double2 v1 = in.v1, v2 = in.v2, e1 = in.e1, e2 = in.e2, Hf = in.hf, Hg = in.hg;
        const size_t so = st(hr, c);
        double2* hf = reinterpret_cast<double2*>(a.hF + so);
        double2* hg = reinterpret_cast<double2*>(a.hG + so);
        double Fr = S.pair(rowF * CRP + 2 * c)[0], Fi = S.pair(rowF * CRP + 2 * c)[1];
        double Gr = S2.pair(rowF * CRP + 2 * c)[0], Gi = S2.pair(rowF * CRP + 2 * c)[1];
        if constexpr (kForce) {
          // external forcing held over the step enters every sub-step's terms
          // as F - f_lapv, G - f_eta (y-parity halves of the interior values)
          const double2 p1 = *reinterpret_cast<const double2*>(a.fv + s1);
          const double2 p2 = *reinterpret_cast<const double2*>(a.fv + s2);
          const double2 g1 = *reinterpret_cast<const double2*>(a.feta + s1);
          const double2 g2 = *reinterpret_cast<const double2*>(a.feta + s2);
          Fr -= 0.5 * (p1.x + sg * p2.x);
          Fi -= 0.5 * (p1.y + sg * p2.y);
          Gr -= 0.5 * (g1.x + sg * g2.x);
          Gi -= 0.5 * (g1.y + sg * g2.y);
        }
        if (s == 0) {
          *hf = double2{Fr, Fi};
          *hg = double2{Gr, Gi};
        } else if (s == 1) {
          *hf = double2{Hf.x + 4.0 * Fr, Hf.y + 4.0 * Fi};
          *hg = double2{Hg.x + 4.0 * Gr, Hg.y + 4.0 * Gi};
          Fr = 2.0 * Fr - Hf.x; Fi = 2.0 * Fi - Hf.y;
          Gr = 2.0 * Gr - Hg.x; Gi = 2.0 * Gi - Hg.y;
        } else {
          Fr = (Hf.x + Fr) * (1.0 / 6.0); Fi = (Hf.y + Fi) * (1.0 / 6.0);
          Gr = (Hg.x + Gr) * (1.0 / 6.0); Gi = (Hg.y + Gi) * (1.0 / 6.0);
        }
        S.pair(rowF * CRP + 2 * c)[0] = -hdt * Fr;
        S.pair(rowF * CRP + 2 * c)[1] = -hdt * Fi;
        S2.pair(rowF * CRP + 2 * c)[0] = -hdt * Gr;
        S2.pair(rowF * CRP + 2 * c)[1] = -hdt * Gi;
        S.pair(rowX * CRP + 2 * c)[0] = 0.5 * (v1.x + sg * v2.x);
        S.pair(rowX * CRP + 2 * c)[1] = 0.5 * (v1.y + sg * v2.y);
        S2.pair(rowX * CRP + 2 * c)[0] = 0.5 * (e1.x + sg * e2.x);
        S2.pair(rowX * CRP + 2 * c)[1] = 0.5 * (e1.y + sg * e2.y);
      };
      for (int q = tid; q < N * C; q += 2 * NT) {
        RkIn ia, ib;
        rk_load(q, ia);
        rk_load(q + NT, ib);
        ia.hf = ib.hf = ia.hg = ib.hg = double2{0.0, 0.0};
        if (s > 0) {
          rk_load_hist(q, ia);
          rk_load_hist(q + NT, ib);
        }
        if (ia.ok) rk_item(q, ia);
        if (ib.ok) rk_item(q + NT, ib);
      }
      __syncthreads();
      const double* opve = a.opsT + size_t(g) * a.op_group_stride;
      const double* opvo = opve + size_t(RTe) * KSe * 64;
      const double* opee = opvo + size_t(RTo) * KSo * 64;
      const double* opeo = opee + size_t(RTe) * KSe * 64;
      // v halves -> T (FH, interior rows from 1); the wall rows read as v = 0.
      // eta halves -> S (FH); rows beyond My keep finite stack data that only
      // meets zero padding columns of D1.  Both solves in one pass when every
      // wave can hold its tiles until the v stack in S has been read.
      for (int q = tid; q < CRP; q += NT) {
        T[q] = 0.0;
        T[Fe * CRP + q] = 0.0;
      }
      const CJob js[4] = {{opve, RTe, KSe, S.row(0)}, {opvo, RTo, KSo, S.row(2 * He)},
                          {opee, RTe, KSe, S2.row(0)}, {opeo, RTo, KSo, S2.row(2 * He)}};
      if (mfma_jobs_fit<NT>(js, CT)) {
        mfma_jobs<NT, true>(js, CRP, CT, [&](int j, int r, int cc, double v) {
          const int lim = (j & 1) ? Ho : He;
          if (r < lim) ((j < 2) ? T : S)[((j & 1) ? Fe + 1 + r : 1 + r) * CRP + cc] = v;
        });
        for (int q = tid; q < CRP; q += NT) {
          S[q] = 0.0;
          S[Fe * CRP + q] = 0.0;
        }
      } else {
        mfma_contract<NT>(opve, RTe, KSe, S.row(0), CRP, CT, [&](int r, int cc, double v) {
          if (r < He) T[(1 + r) * CRP + cc] = v;
        });
        mfma_contract<NT>(opvo, RTo, KSo, S.row(2 * He), CRP, CT, [&](int r, int cc, double v) {
          if (r < Ho) T[(Fe + 1 + r) * CRP + cc] = v;
        });
        __syncthreads();
        for (int q = tid; q < CRP; q += NT) {
          S[q] = 0.0;
          S[Fe * CRP + q] = 0.0;
        }
        mfma_contract<NT>(opee, RTe, KSe, S2.row(0), CRP, CT, [&](int r, int cc, double v) {
          if (r < He) S[(1 + r) * CRP + cc] = v;
        });
        mfma_contract<NT>(opeo, RTo, KSo, S2.row(2 * He), CRP, CT, [&](int r, int cc, double v) {
          if (r < Ho) S[(Fe + 1 + r) * CRP + cc] = v;
        });
      }
      __syncthreads();
      if (s == 2) {
        // Hermitian projection of the n_x = 0 column: (0, nz) and (0, -nz);
        // a per-node combination of two columns, so it acts on halves as is
        if (nx == 0 && az > 0) {
          for (int q = tid; q < My * ET; q += NT) {
            const int i = q >> ets, c0 = q & (ET - 1), c1 = c0 + ET;
#pragma unroll
            for (int bsel = 0; bsel < 2; ++bsel) {
              const LdsBuf B = bsel == 0 ? T : S;
              const double ar = B.pair(i * CRP + 2 * c0)[0], ai = B.pair(i * CRP + 2 * c0)[1];
              const double br = B.pair(i * CRP + 2 * c1)[0], bi = B.pair(i * CRP + 2 * c1)[1];
              const double pr = 0.5 * (ar + br), pi = 0.5 * (ai - bi);
              B.pair(i * CRP + 2 * c0)[0] = pr;
              B.pair(i * CRP + 2 * c0)[1] = pi;
              B.pair(i * CRP + 2 * c1)[0] = pr;
              B.pair(i * CRP + 2 * c1)[1] = -pi;
            }
          }
          __syncthreads();
        }
        // state: interior node pairs (kk, N-1-kk) from FH rows 1 + kk, Fe + 1 + kk
        for (int q = tid; q < He * C; q += NT) {
          const int kk = q >> cs, c = q & (C - 1);
          if (!col_valid(c)) continue;
          const int re = 1 + kk, ro = Fe + 1 + kk;
          const double ver = T.pair(re * CRP + 2 * c)[0], vei = T.pair(re * CRP + 2 * c)[1];
          const double eer = S.pair(re * CRP + 2 * c)[0], eei = S.pair(re * CRP + 2 * c)[1];
          const size_t s1 = st(kk, c);
          if (kk < Ho) {
            const double vor = T.pair(ro * CRP + 2 * c)[0], voi = T.pair(ro * CRP + 2 * c)[1];
            const double eor = S.pair(ro * CRP + 2 * c)[0], eoi = S.pair(ro * CRP + 2 * c)[1];
            const size_t s2 = st(N - 1 - kk, c);
            const double v1r = ver + vor, v1i = vei + voi, v2r = ver - vor, v2i = vei - voi;
            const double e1r = eer + eor, e1i = eei + eoi, e2r = eer - eor, e2i = eei - eoi;
            a.v[s1] = v1r; a.v[s1 + 1] = v1i;
            a.v[s2] = v2r; a.v[s2 + 1] = v2i;
            a.eta[s1] = e1r; a.eta[s1 + 1] = e1i;
            a.eta[s2] = e2r; a.eta[s2 + 1] = e2i;
            // halves of the stored (rounded) values, formed exactly as a restart
            // from this state forms them, so that a resumed run is bitwise equal
            T.pair(re * CRP + 2 * c)[0] = 0.5 * (v1r + v2r);
            T.pair(re * CRP + 2 * c)[1] = 0.5 * (v1i + v2i);
            T.pair(ro * CRP + 2 * c)[0] = 0.5 * (v1r - v2r);
            T.pair(ro * CRP + 2 * c)[1] = 0.5 * (v1i - v2i);
            S.pair(re * CRP + 2 * c)[0] = 0.5 * (e1r + e2r);
            S.pair(re * CRP + 2 * c)[1] = 0.5 * (e1i + e2i);
            S.pair(ro * CRP + 2 * c)[0] = 0.5 * (e1r - e2r);
            S.pair(ro * CRP + 2 * c)[1] = 0.5 * (e1i - e2i);
          } else {
            a.v[s1] = ver; a.v[s1 + 1] = vei;
            a.eta[s1] = eer; a.eta[s1 + 1] = eei;
          }
        }
      }
    } else {
      // velocities of the stored state: v -> T (FH), eta -> S (FH)
      for (int q = tid; q < He * C; q += NT) {
        const int kk = q >> cs, c = q & (C - 1);
        if (!col_valid(c)) continue;
        const size_t s1 = st(kk, c);
        const int re = 1 + kk, ro = Fe + 1 + kk;
        if (kk < Ho) {
          const size_t s2 = st(N - 1 - kk, c);
          T.pair(re * CRP + 2 * c)[0] = 0.5 * (a.v[s1] + a.v[s2]);
          T.pair(re * CRP + 2 * c)[1] = 0.5 * (a.v[s1 + 1] + a.v[s2 + 1]);
          T.pair(ro * CRP + 2 * c)[0] = 0.5 * (a.v[s1] - a.v[s2]);
          T.pair(ro * CRP + 2 * c)[1] = 0.5 * (a.v[s1 + 1] - a.v[s2 + 1]);
          S.pair(re * CRP + 2 * c)[0] = 0.5 * (a.eta[s1] + a.eta[s2]);
          S.pair(re * CRP + 2 * c)[1] = 0.5 * (a.eta[s1 + 1] + a.eta[s2 + 1]);
          S.pair(ro * CRP + 2 * c)[0] = 0.5 * (a.eta[s1] - a.eta[s2]);
          S.pair(ro * CRP + 2 * c)[1] = 0.5 * (a.eta[s1 + 1] - a.eta[s2 + 1]);
        } else {
          T.pair(re * CRP + 2 * c)[0] = a.v[s1];
          T.pair(re * CRP + 2 * c)[1] = a.v[s1 + 1];
          S.pair(re * CRP + 2 * c)[0] = a.eta[s1];
          S.pair(re * CRP + 2 * c)[1] = a.eta[s1 + 1];
        }
      }
    }
    __syncthreads();
    // ---- velocity recovery: dv/dy = D1c v (odd <- even, even <- odd) -> S2 FH
    if constexpr (kDer != kDerFP64) {
      dcontract<kDer, NT>(a, 2, a.D1cT_e, RFo, He, T.row(1), CRP, CT, [&](int r, int cc, double v) {
        if (r < Fo) S2[(Fe + r) * CRP + cc] = v;
      });
      dcontract<kDer, NT>(a, 3, a.D1cT_o, RFe, Ho, T.row(Fe + 1), CRP, CT, [&](int r, int cc, double v) {
        if (r < Fe) S2[r * CRP + cc] = v;
      });
    } else {
      const CJob jc[2] = {{a.D1cT_e, RFo, (He + 3) / 4, T.row(1)}, {a.D1cT_o, RFe, (Ho + 3) / 4, T.row(Fe + 1)}};
      mfma_jobs<NT, false>(jc, CRP, CT, [&](int j, int r, int cc, double v) {
        if (j == 0) {
          if (r < Fo) S2[(Fe + r) * CRP + cc] = v;
        } else if (r < Fe) {
          S2[r * CRP + cc] = v;
        }
      });
    }
    __syncthreads();
    double dmax = 0.0;
    for (int q = tid; q < Fe * C; q += NT) {
      const int k = q >> cs, c = q & (C - 1);
      const double kz = col_kz(c), k2 = kx * kx + kz * kz;
      const double ik2 = k2 > 0.0 ? 1.0 / k2 : 0.0;
      const bool pair = k < Fo;
      double uh[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, wh[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
      double dh[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        if (par == 1 && !pair) continue;
        const int row = par == 0 ? k : Fe + k;
        const double dr = S2.pair(row * CRP + 2 * c)[0], di = S2.pair(row * CRP + 2 * c)[1];
        const double er = S.pair(row * CRP + 2 * c)[0], ei = S.pair(row * CRP + 2 * c)[1];
        // u = (i kx dv - i kz eta) / k^2 ; w = (i kx eta + i kz dv) / k^2
        const double ur = (-kx * di + kz * ei) * ik2, ui = (kx * dr - kz * er) * ik2;
        const double wr = (-kx * ei - kz * di) * ik2, wi = (kx * er + kz * dr) * ik2;
        S2.pair(row * CRP + 2 * c)[0] = ur;
        S2.pair(row * CRP + 2 * c)[1] = ui;
        S.pair(row * CRP + 2 * c)[0] = wr;
        S.pair(row * CRP + 2 * c)[1] = wi;
        uh[par][0] = ur; uh[par][1] = ui;
        wh[par][0] = wr; wh[par][1] = wi;
        dh[par][0] = dr; dh[par][1] = di;
      }
      if (col_valid(c)) {
        write_pair(T, k, c, 1);  // v
        // u, w and the divergence i kx u + dv/dy + i kz w at both nodes
        for (int side = 0; side < (pair ? 2 : 1); ++side) {
          const double sg = side == 0 ? 1.0 : -1.0;
          const int j = side == 0 ? k : My - 1 - k;
          const double ur = uh[0][0] + sg * uh[1][0], ui = uh[0][1] + sg * uh[1][1];
          const double wr = wh[0][0] + sg * wh[1][0], wi = wh[0][1] + sg * wh[1][1];
          const double dr = dh[0][0] + sg * dh[1][0], di = dh[0][1] + sg * dh[1][1];
          st_c(vel + 0 * FS + sb(j, c), ur, ui);
          st_c(vel + 2 * FS + sb(j, c), wr, wi);
          const double xr = -kx * ui + dr - kz * wi, xi = kx * ur + di + kz * wr;
          dmax = fmax(dmax, sqrt(xr * xr + xi * xi));
        }
      }
    }
    __syncthreads();
    // du/dy = D1 u -> T (FH) and dw/dy = D1 w -> S2 (FH): in one pass when
    // every wave can hold its tiles until u in S2 has been read
    const CJob jd[4] = {{a.D1T_e, RFo, (Fe + 3) / 4, S2.row(0)}, {a.D1T_o, RFe, (Fo + 3) / 4, S2.row(Fe)},
                        {a.D1T_e, RFo, (Fe + 3) / 4, S.row(0)}, {a.D1T_o, RFe, (Fo + 3) / 4, S.row(Fe)}};
    bool merged = false;
    if constexpr (kDer == kDerFP64) {
      if (mfma_jobs_fit<NT>(jd, CT)) {
        mfma_jobs<NT, true>(jd, CRP, CT, [&](int j, int r, int cc, double v) {
          const int lim = (j & 1) ? Fe : Fo;
          if (r < lim) ((j < 2) ? T : S2)[((j & 1) ? r : Fe + r) * CRP + cc] = v;
        });
        merged = true;
      }
    }
    if (!merged) {
      dcontract<kDer, NT>(a, 4, a.D1T_e, RFo, Fe, S2.row(0), CRP, CT, [&](int r, int cc, double v) {
        if (r < Fo) T[(Fe + r) * CRP + cc] = v;
      });
      dcontract<kDer, NT>(a, 5, a.D1T_o, RFe, Fo, S2.row(Fe), CRP, CT, [&](int r, int cc, double v) {
        if (r < Fe) T[r * CRP + cc] = v;
      });
      __syncthreads();
      dcontract<kDer, NT>(a, 4, a.D1T_e, RFo, Fe, S.row(0), CRP, CT, [&](int r, int cc, double v) {
        if (r < Fo) S2[(Fe + r) * CRP + cc] = v;
      });
      dcontract<kDer, NT>(a, 5, a.D1T_o, RFe, Fo, S.row(Fe), CRP, CT, [&](int r, int cc, double v) {
        if (r < Fe) S2[r * CRP + cc] = v;
      });
    }
    __syncthreads();
    for (int q = tid; q < Fe * C; q += NT) {
      const int k = q >> cs, c = q & (C - 1);
      if (!col_valid(c)) continue;
      write_pair(T, k, c, 3);
      write_pair(S2, k, c, 4);
    }
    if (s == 2 || s < 0) {
      // thread tid's maximum belongs to column tid mod C: lanes that differ
      // in bits >= log2 C share it; then one value per wave and column
      for (int off = C; off < 64; off <<= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
      const int lane = tid & 63, wave = tid >> 6;
      if (lane < C) red[wave * C + lane] = dmax;
      __syncthreads();
      if (tid < C && col_valid(tid)) {
        double mx = 0.0;
        for (int w = 0; w < (NT / 64); ++w) mx = fmax(mx, red[w * C + tid]);
        atomicMax(&a.divmax[col_member(tid)], (unsigned long long)__double_as_longlong(mx));
      }
    }
    return;
  }

  // ========================= mean profiles (0, 0) ===========================
  // Real columns 2e (U, <uv>, E_U) and 2e + 1 (W, <wv>, E_W), e < ET; U and W
  // share A_U, B_U (Eqs. (CN3), (CN4)), which commute with the reflection.
  const int NM = ET;
  if (s >= 0) {
    // plane means (FH halves)
    for (int q = tid; q < Fe * NM; q += NT) {
      const int k = q >> ets, el = q & (NM - 1), e = m0 + tile * ET + el;
      if (e >= mend) continue;
      const int j2 = My - 1 - k;
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
        const double x1 = a.means[(size_t(comp) * My + k) * E + e];
        const double x2 = a.means[(size_t(comp) * My + j2) * E + e];
        if (k < Fo) {
          T.pair(k * CRP + 2 * el)[comp] = 0.5 * (x1 + x2);
          T.pair((Fe + k) * CRP + 2 * el)[comp] = 0.5 * (x1 - x2);
        } else {
          T.pair(k * CRP + 2 * el)[comp] = x1;
        }
      }
    }
    __syncthreads();
    // (E_U, E_W) = -D1 (<uv>, <wv>) on interior halves
    dcontract<kDer, NT>(a, 0, a.D1intT_e, RTo, Fe, T.row(0), CRP, CT, [&](int r, int cc, double v) {
      if (r < Ho) S[(2 * He + Ho + r) * CRP + cc] = -v;
    });
    dcontract<kDer, NT>(a, 1, a.D1intT_o, RTe, Fo, T.row(Fe), CRP, CT, [&](int r, int cc, double v) {
      if (r < He) S[(He + r) * CRP + cc] = -v;
    });
    __syncthreads();
    for (int q = tid; q < N * NM; q += NT) {
      const int hr = q >> ets, el = q & (NM - 1), e = m0 + tile * ET + el;
      if (e >= mend) continue;
      const bool even = hr < He;
      const int kk = even ? hr : hr - He;
      const int rowF = even ? He + kk : 2 * He + Ho + kk;
      const int rowX = even ? kk : 2 * He + kk;
      double xu = S.pair(rowF * CRP + 2 * el)[0], xw = S.pair(rowF * CRP + 2 * el)[1];
      double* hu = a.hEU + size_t(hr) * E + e;
      double* hw = a.hEW + size_t(hr) * E + e;
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
      S.pair(rowF * CRP + 2 * el)[0] = hdt * xu;
      S.pair(rowF * CRP + 2 * el)[1] = hdt * xw;
      // interior nodes 1 + kk and My - 2 - kk of U0, W0
      const size_t j1 = size_t(1 + kk) * E + e, j2 = size_t(My - 2 - kk) * E + e;
      const bool center = even && kk == Ho;
      const double sg = even ? 1.0 : -1.0;
      S.pair(rowX * CRP + 2 * el)[0] = center ? a.U[j1] : 0.5 * (a.U[j1] + sg * a.U[j2]);
      S.pair(rowX * CRP + 2 * el)[1] = center ? a.W[j1] : 0.5 * (a.W[j1] + sg * a.W[j2]);
    }
    __syncthreads();
    // (U_a, W) halves = [A_U | B_U] halves -> T (FH)
    const double* me = a.meanT;
    const double* mo = me + size_t(RTe) * KSe * 64;
    mfma_contract<NT>(me, RTe, KSe, S.row(0), CRP, CT, [&](int r, int cc, double v) {
      if (r < He) T[(1 + r) * CRP + cc] = v;
    });
    mfma_contract<NT>(mo, RTo, KSo, S.row(2 * He), CRP, CT, [&](int r, int cc, double v) {
      if (r < Ho) T[(Fe + 1 + r) * CRP + cc] = v;
    });
    __syncthreads();
    // wall pair, lift on the interior halves
    for (int q = tid; q < Fe * NM; q += NT) {
      const int k = q >> ets, el = q & (NM - 1);
      if (k == 0) {
        T.pair(2 * el)[0] = 0.5 * (a.Ubot + a.Utop);
        T.pair(2 * el)[1] = 0.0;
        T.pair(Fe * CRP + 2 * el)[0] = 0.5 * (a.Ubot - a.Utop);
        T.pair(Fe * CRP + 2 * el)[1] = 0.0;
      } else {
        T.pair(k * CRP + 2 * el)[0] += a.lift_h[k - 1];
        if (k - 1 < Ho) T.pair((Fe + k) * CRP + 2 * el)[0] += a.lift_h[He + k - 1];
      }
    }
    __syncthreads();
    // bulk flux of the provisional U (even half only) and gamma per member
    if (tid < NM) {
      const int el = tid, e = m0 + tile * ET + el;
      double gam = 0.0;
      if (a.poiseuille) {
        double qa = 0.0, wg = 0.0;
        for (int k = 0; k < Fe; ++k) {
          qa += a.ccw_h[k] * T.pair(k * CRP + 2 * el)[0];
          if (k >= 1) wg += a.ccw_h[k] * a.green_h[k - 1];
        }
        gam = (a.Qtarget - qa) / wg;
      }
      gam_s[el] = gam;
      if (e < mend) a.gamma[e] = gam;
    }
    __syncthreads();
    // gamma response is even (the green function is symmetric)
    for (int q = tid; q < He * NM; q += NT) {
      const int kk = q >> ets, el = q & (NM - 1);
      T.pair((1 + kk) * CRP + 2 * el)[0] += gam_s[el] * a.green_h[kk];
    }
    __syncthreads();
    if (s == 2) {
      for (int q = tid; q < Fe * NM; q += NT) {
        const int k = q >> ets, el = q & (NM - 1), e = m0 + tile * ET + el;
        if (e >= mend) continue;
        const double ue = T.pair(k * CRP + 2 * el)[0], we = T.pair(k * CRP + 2 * el)[1];
        if (k < Fo) {
          const double uo = T.pair((Fe + k) * CRP + 2 * el)[0], wo = T.pair((Fe + k) * CRP + 2 * el)[1];
          const double u1 = ue + uo, w1 = we + wo, u2 = ue - uo, w2 = we - wo;
          a.U[size_t(k) * E + e] = u1;
          a.W[size_t(k) * E + e] = w1;
          a.U[size_t(My - 1 - k) * E + e] = u2;
          a.W[size_t(My - 1 - k) * E + e] = w2;
          // halves of the stored values, as a restart forms them
          T.pair(k * CRP + 2 * el)[0] = 0.5 * (u1 + u2);
          T.pair(k * CRP + 2 * el)[1] = 0.5 * (w1 + w2);
          T.pair((Fe + k) * CRP + 2 * el)[0] = 0.5 * (u1 - u2);
          T.pair((Fe + k) * CRP + 2 * el)[1] = 0.5 * (w1 - w2);
        } else {
          a.U[size_t(k) * E + e] = ue;
          a.W[size_t(k) * E + e] = we;
        }
      }
    }
  } else {
    for (int q = tid; q < Fe * NM; q += NT) {
      const int k = q >> ets, el = q & (NM - 1), e = m0 + tile * ET + el;
      if (e >= mend) continue;
      const size_t j1 = size_t(k) * E + e, j2 = size_t(My - 1 - k) * E + e;
      if (k < Fo) {
        T.pair(k * CRP + 2 * el)[0] = 0.5 * (a.U[j1] + a.U[j2]);
        T.pair(k * CRP + 2 * el)[1] = 0.5 * (a.W[j1] + a.W[j2]);
        T.pair((Fe + k) * CRP + 2 * el)[0] = 0.5 * (a.U[j1] - a.U[j2]);
        T.pair((Fe + k) * CRP + 2 * el)[1] = 0.5 * (a.W[j1] - a.W[j2]);
      } else {
        T.pair(k * CRP + 2 * el)[0] = a.U[j1];
        T.pair(k * CRP + 2 * el)[1] = a.W[j1];
      }
    }
  }
  __syncthreads();
  // (0,0) velocity fields: u = U, v = 0, w = W, du/dy = D1 U, dw/dy = D1 W
  dcontract<kDer, NT>(a, 4, a.D1T_e, RFo, Fe, T.row(0), CRP, CT, [&](int r, int cc, double v) {
    if (r < Fo) S2[(Fe + r) * CRP + cc] = v;
  });
  dcontract<kDer, NT>(a, 5, a.D1T_o, RFe, Fo, T.row(Fe), CRP, CT, [&](int r, int cc, double v) {
    if (r < Fe) S2[r * CRP + cc] = v;
  });
  __syncthreads();
  for (int q = tid; q < Fe * NM; q += NT) {
    const int k = q >> ets, el = q & (NM - 1), e = m0 + tile * ET + el;
    if (e >= mend) continue;
    const bool pair = k < Fo;
    for (int side = 0; side < (pair ? 2 : 1); ++side) {
      const double sg = side == 0 ? 1.0 : -1.0;
      const int j = side == 0 ? k : My - 1 - k;
      const size_t off = 2 * stage_off(j, e, 0, E, K, stage_block_log2(E));
      const double U = T.pair(k * CRP + 2 * el)[0] + (pair ? sg * T.pair((Fe + k) * CRP + 2 * el)[0] : 0.0);
      const double W = T.pair(k * CRP + 2 * el)[1] + (pair ? sg * T.pair((Fe + k) * CRP + 2 * el)[1] : 0.0);
      const double dU = S2.pair(k * CRP + 2 * el)[0] + (pair ? sg * S2.pair((Fe + k) * CRP + 2 * el)[0] : 0.0);
      const double dW = S2.pair(k * CRP + 2 * el)[1] + (pair ? sg * S2.pair((Fe + k) * CRP + 2 * el)[1] : 0.0);
      st_c(vel + off, U, 0.0);
      st_c(vel + off + FS, 0.0, 0.0);
      st_c(vel + off + 2 * FS, W, 0.0);
      st_c(vel + off + 3 * FS, dU, 0.0);
      st_c(vel + off + 4 * FS, dW, 0.0);
    }
  }
}

// Four waves per SIMD (registers <= 128): sixteen waves per CU, as two
// workgroups of 512 threads or one of 1024.
template <typename VT, int kDer, bool kForce, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) mode_kernel(ModeArgs a) {
  mode_body<VT, kDer, kForce, NT>(a, xcd_logical_m(blockIdx.x, gridDim.x));
}

// Several ensembles' per-mode work in one launch (uneven grouped ensembles,
// members of different Re and grid): workgroups [first[d], first[d + 1]) run
// descriptor d, each with the launch shape it would have alone.
template <typename VT, int kDer, bool kForce>
__global__ void __launch_bounds__(kModeThreadsNarrow) __attribute__((amdgpu_waves_per_eu(4))) mode_grouped_kernel(const ModeArgs* __restrict__ descs,
                                                           const int* __restrict__ first, int ndesc) {
  const int b = blockIdx.x;
  int d = 0;
  while (d + 1 < ndesc && b >= first[d + 1]) ++d;
  mode_body<VT, kDer, kForce, kModeThreadsNarrow>(descs[d], xcd_logical_m(b - first[d], first[d + 1] - first[d]));
}

// LDS geometry of one workgroup; shared with the host launcher.
void mode_lds_geometry(int My, int ET, int* CRP, int* SR, int* TR) {
  const int N = My - 2;
  const int He = (N + 1) / 2, Ho = N / 2, Fe = He + 1, Fo = Ho + 1;
  auto t4 = [](int n) { return 4 * ((n + 3) / 4); };
  auto t16 = [](int n) { return 16 * ((n + 15) / 16); };  // K steps of the split-BF16 contractions
  auto mx = [](int a, int b) { return a > b ? a : b; };
  *CRP = ((4 * ET + 15) / 16) * 16;
  // S/S2: even solve reads rows < t4(2He), odd solve from 2He; D1 halves read
  // rows < t16(Fe) and from Fe
  int sr = mx(t4(2 * He), 2 * He + t4(2 * Ho));
  sr = mx(sr, Fe + t16(Fo));
  sr = mx(sr, mx(t16(Fe), My));
  // T: D1int/D1 halves as above; D1c halves from row 1 and from row Fe + 1
  int tr = mx(Fe + t16(Fo), t16(Fe));
  tr = mx(tr, mx(1 + t16(He), Fe + 1 + t16(Ho)));
  *SR = sr;
  *TR = mx(tr, My);
}

// Workgroup size of member tile ET: 512 threads when two workgroups fit a
// CU's LDS, else 1024 when one does (either way sixteen waves per CU), else 512.
int mode_tile_threads(int My, int ET) {
  int crp, sr, tr;
  mode_lds_geometry(My, ET, &crp, &sr, &tr);
  const size_t dyn = size_t(2 * sr + tr) * crp * sizeof(double);
  if (2 * (dyn + mode_static_lds(kModeThreadsNarrow)) <= kLdsPerCU) return kModeThreadsNarrow;
  if (dyn + mode_static_lds(kModeThreadsWide) <= kLdsPerCU) return kModeThreadsWide;
  return kModeThreadsNarrow;
}

// Default member tile: the largest ET in {1, 2, 4, 8} (<= E) of which two
// 512-thread workgroups fit a CU's LDS (sixteen waves per CU; measured faster
// than one 1024-thread workgroup of twice the tile, or level with it); when
// no tile allows two, the largest that fits one 1024-thread workgroup (with
// narrow_only: ET = 1).
int mode_member_tile(int My, int E, bool narrow_only) {
  int two_best = 0, wide_best = 1;
  for (int et = 1; et <= 8 && et <= E; et *= 2) {
    int crp, sr, tr;
    mode_lds_geometry(My, et, &crp, &sr, &tr);
    const size_t dyn = size_t(2 * sr + tr) * crp * sizeof(double);
    if (2 * (dyn + mode_static_lds(kModeThreadsNarrow)) <= kLdsPerCU) two_best = et;
    if (dyn + mode_static_lds(kModeThreadsWide) <= kLdsPerCU) wide_best = et;
  }
  if (two_best > 0) return two_best;
  return narrow_only ? 1 : wide_best;
}

namespace {
// precision 0: FP64 stage buffers; 1: FP32 stage buffers; 2: FP32 stage
// buffers and split-BF16 derivative products; 3: FP32 stage buffers and FP32
// matrix-core derivative products
template <bool kForce, int NT>
const void* mode_fn_t(int precision) {
  switch (precision) {
    case 0: return reinterpret_cast<const void*>(&mode_kernel<double, kDerFP64, kForce, NT>);
    case 1: return reinterpret_cast<const void*>(&mode_kernel<float, kDerFP64, kForce, NT>);
    case 2: return reinterpret_cast<const void*>(&mode_kernel<float, kDerSplitBF16, kForce, NT>);
    default: return reinterpret_cast<const void*>(&mode_kernel<float, kDerFP32, kForce, NT>);
  }
}
template <bool kForce>
const void* mode_fn(int precision, int threads) {
  return threads == kModeThreadsWide ? mode_fn_t<kForce, kModeThreadsWide>(precision)
                                     : mode_fn_t<kForce, kModeThreadsNarrow>(precision);
}
template <bool kForce>
const void* mode_grouped_fn(int precision) {
  switch (precision) {
    case 0: return reinterpret_cast<const void*>(&mode_grouped_kernel<double, kDerFP64, kForce>);
    case 1: return reinterpret_cast<const void*>(&mode_grouped_kernel<float, kDerFP64, kForce>);
    case 2: return reinterpret_cast<const void*>(&mode_grouped_kernel<float, kDerSplitBF16, kForce>);
    default: return reinterpret_cast<const void*>(&mode_grouped_kernel<float, kDerFP32, kForce>);
  }
}
}  // namespace

// Resolve the per-mode kernel instantiations on the current device.
hipError_t mode_preload() {
  for (int prec = 0; prec < 4; ++prec) {
    for (const void* fn : {mode_fn<false>(prec, kModeThreadsNarrow), mode_fn<true>(prec, kModeThreadsNarrow),
                           mode_fn<false>(prec, kModeThreadsWide), mode_fn<true>(prec, kModeThreadsWide),
                           mode_grouped_fn<false>(prec), mode_grouped_fn<true>(prec)}) {
      hipFuncAttributes attr;
      const hipError_t err = hipFuncGetAttributes(&attr, fn);
      if (err != hipSuccess) return err;
    }
  }
  return hipSuccess;
}

// The kernel of the precision and a.threads (as mode_fn); a forcing (a.fv)
// selects the variant that subtracts it.
hipError_t launch_mode(int precision, const ModeArgs& a, hipStream_t s) {
  const int nblk = a.G * a.ntiles;
  const int threads = a.threads == kModeThreadsWide ? kModeThreadsWide : kModeThreadsNarrow;
  const size_t lds = size_t(2 * a.SR + a.TR) * a.CRP * sizeof(double);
  const void* fn = a.fv ? mode_fn<true>(precision, threads) : mode_fn<false>(precision, threads);
  hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (err != hipSuccess) return err;
  void* args[] = {const_cast<ModeArgs*>(&a)};
  err = hipLaunchKernel(fn, dim3(nblk), dim3(threads), args, lds, s);
  return err != hipSuccess ? err : hipGetLastError();
}

// Every descriptor of descs (device, ndesc entries; first: device, ndesc + 1
// block offsets) in one launch of nblk workgroups of 512 threads with lds bytes
// of dynamic LDS (the largest of the descriptors'); forced selects the variant
// that subtracts an external forcing (each descriptor then needs one).
hipError_t launch_mode_grouped(int precision, bool forced, const ModeArgs* descs, const int* first, int ndesc,
                               int nblk, size_t lds, hipStream_t s) {
  const void* fn = forced ? mode_grouped_fn<true>(precision) : mode_grouped_fn<false>(precision);
  hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (err != hipSuccess) return err;
  void* args[] = {const_cast<ModeArgs**>(&descs), const_cast<int**>(&first), &ndesc};
  err = hipLaunchKernel(fn, dim3(nblk), dim3(kModeThreadsNarrow), args, lds, s);
  return err != hipSuccess ? err : hipGetLastError();
}

}  // namespace dns
