// Small-transform building blocks for the x-z pseudo-spectral stage.
//
// The paper evaluates the advection term on a 3/2-padded physical grid
// (Sec. 3.2, 2/3-rule dealiasing) with 2-D FFTs of every ensemble member.
// Here every transform length is 2^a 3^b and at most a few hundred points, so
// each transform is done as two Stockham passes of in-register radix-R1 and
// radix-R2 butterflies (R1 * R2 = N, R <= 16) with one LDS round trip between
// them.  The first pass reads its inputs through a caller functor (so zero
// padding, Hermitian extension, derivative factors and folds are fused into
// it) and the last pass hands every output element to a caller functor
// exactly once (so pointwise products are fused into it).
#pragma once

#include <hip/hip_runtime.h>

namespace dns {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cmk(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return cx<T>{a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return cx<T>{a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return cx<T>{a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return cx<T>{a.x * s, a.y * s}; }
// multiply by +i (DIR = +1) or -i (DIR = -1)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> cmuli(cx<T> a) {
  return DIR > 0 ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

// cos(2 pi t / 144) for the quarter-wave angles used by radices 6, 8, 9, 12, 16.
constexpr double qcos144(int t) {
  return t == 0 ? 1.0
       : t == 4 ? 0.98480775301220805936674
       : t == 8 ? 0.93969262078590838405410
       : t == 9 ? 0.92387953251128675612818
       : t == 12 ? 0.86602540378443864676373
       : t == 16 ? 0.76604444311897803520240
       : t == 18 ? 0.70710678118654752440084
       : t == 20 ? 0.64278760968653932632264
       : t == 24 ? 0.5
       : t == 27 ? 0.38268343236508977172846
       : t == 28 ? 0.34202014332566873304410
       : t == 32 ? 0.17364817766693034885172
       : t == 36 ? 0.0
       : 2.0;  // not a supported angle: an impossible cosine flags misuse
}
constexpr double cos144(int t) {
  t = ((t % 144) + 144) % 144;
  return t <= 36 ? qcos144(t)
       : t <= 72 ? -qcos144(72 - t)
       : t <= 108 ? -qcos144(t - 72)
       : qcos144(144 - t);
}
constexpr double sin144(int t) { return cos144(t - 36); }

// e^{DIR 2 pi i t / R} for R dividing 144.
template <typename T, int R, int DIR>
__device__ __forceinline__ cx<T> unit_root(int t) {
  static_assert(144 % R == 0, "radix must divide 144");
  return cx<T>{T(cos144(t * (144 / R))), T(DIR * sin144(t * (144 / R)))};
}

// In-place DFT of R elements, natural order in and out:
//   v[k] <- sum_n v[n] e^{DIR 2 pi i n k / R}
template <typename T, int R, int DIR>
struct SmallDft;

template <typename T, int DIR>
struct SmallDft<T, 1, DIR> {
  static __device__ __forceinline__ void run(cx<T>*) {}
};

template <typename T, int DIR>
struct SmallDft<T, 2, DIR> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename T, int DIR>
struct SmallDft<T, 3, DIR> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const T c = T(-0.5);
    const T s = T(DIR * 0.86602540378443864676373);
    cx<T> a = v[0], b = v[1], d = v[2];
    cx<T> t1 = cadd(b, d);
    cx<T> t2 = csub(b, d);
    cx<T> m = cx<T>{a.x + c * t1.x, a.y + c * t1.y};
    cx<T> r = cx<T>{-s * t2.y, s * t2.x};  // i s (b - d)
    v[0] = cadd(a, t1);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  }
};

template <typename T, int DIR>
struct SmallDft<T, 4, DIR> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1], c = v[2], d = v[3];
    cx<T> s0 = cadd(a, c), s1 = csub(a, c);
    cx<T> s2 = cadd(b, d), s3 = cmuli<DIR>(csub(b, d));
    v[0] = cadd(s0, s2);
    v[2] = csub(s0, s2);
    v[1] = cadd(s1, s3);
    v[3] = csub(s1, s3);
  }
};

// Composite radix R = R1 * R2 with R1 in {2, 3, 4}: Cooley-Tukey in registers.
template <int R>
struct FirstFactor {
  static constexpr int value = (R % 4 == 0 && R != 4 && R != 8) ? 4 : (R % 2 == 0 && R != 2) ? 2 : 3;
};

template <typename T, int R, int DIR>
struct SmallDft {
  static constexpr int R1 = FirstFactor<R>::value;
  static constexpr int R2 = R / R1;
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> t[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      cx<T> a[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) a[n1] = v[n1 * R2 + n2];
      SmallDft<T, R1, DIR>::run(a);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1)
        t[k1 * R2 + n2] = (k1 * n2 == 0) ? a[k1] : cmul(a[k1], unit_root<T, R, DIR>(k1 * n2));
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cx<T> b[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) b[n2] = t[k1 * R2 + n2];
      SmallDft<T, R2, DIR>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = b[k2];
    }
  }
};

// Two-pass split of a transform length: N = RA * RB with both radices <= 16.
template <int N>
struct Split;
template <> struct Split<8> { static constexpr int A = 2, B = 4; };
template <> struct Split<12> { static constexpr int A = 3, B = 4; };
template <> struct Split<16> { static constexpr int A = 4, B = 4; };
template <> struct Split<18> { static constexpr int A = 2, B = 9; };
template <> struct Split<24> { static constexpr int A = 4, B = 6; };
template <> struct Split<32> { static constexpr int A = 4, B = 8; };
template <> struct Split<36> { static constexpr int A = 6, B = 6; };
template <> struct Split<48> { static constexpr int A = 6, B = 8; };
template <> struct Split<54> { static constexpr int A = 6, B = 9; };
template <> struct Split<64> { static constexpr int A = 8, B = 8; };
template <> struct Split<72> { static constexpr int A = 8, B = 9; };
template <> struct Split<96> { static constexpr int A = 8, B = 12; };
template <> struct Split<108> { static constexpr int A = 12, B = 9; };
template <> struct Split<144> { static constexpr int A = 12, B = 12; };

// Batched length-N transform, sign DIR, over NBATCH independent sequences,
// executed by the whole workgroup (NT threads).  Stockham autosort:
//   pass 1 (radix RA):  butterfly j < RB reads x[j + r*RB], r < RA, and keeps
//                       its output r at mid[b][r][j]
//   pass 2 (radix RB):  butterfly k < RA reads output k of every pass-1
//                       butterfly, twiddles e^{DIR 2 pi i t k / N}, and hands
//                       element k + RA*t of the transform to store()
// The intermediate rows have an odd pitch (RB + 1) and the per-sequence pitch
// is odd as well, so both passes touch distinct LDS banks across a wavefront.
// load(b, n) returns input element n of sequence b; store(b, k, val) receives
// output element k of sequence b exactly once.  mid holds NBATCH * MidPitch<N>
// elements; root[t] = e^{-2 pi i t / N}.  One barrier separates the passes; the
// caller places barriers around the call when load/store touch shared memory.
// Most lanes of one wavefront that meet in one LDS bank when lane l touches
// element (l / G) * S + l % G of W 4-byte words, for NB banks of 4 bytes.
constexpr int lds_bank_load(int S, int G, int W, int NB) {
  int cnt[64] = {};
  int mx = 0;
  for (int l = 0; l < 64; ++l) {
    const int e = (l / G) * S + l % G;
    for (int w = 0; w < W; ++w) {
      const int b = (e * W + w) % NB;
      if (++cnt[b] > mx) mx = cnt[b];
    }
  }
  return mx;
}

// Row pitch in [base, base + 16] with the fewest bank collisions for rows read
// in groups of G1 (and G2, if non-zero) consecutive lanes, under 32 and 64 banks;
// each extra element of pitch costs a quarter of a collision.
constexpr int lds_pitch(int base, int G1, int G2, int W) {
  int best = base, load = 1 << 30;
  for (int s = base; s <= base + 16; ++s) {
    int v = lds_bank_load(s, G1, W, 32) + lds_bank_load(s, G1, W, 64);
    if (G2) v += lds_bank_load(s, G2, W, 32) + lds_bank_load(s, G2, W, 64);
    v = 4 * v + (s - base);
    if (v < load) load = v, best = s;
  }
  return best;
}

template <int N>
struct MidPitch {
  static constexpr int row = Split<N>::B + 1;
  static constexpr int raw = Split<N>::A * row;
  static constexpr int value = (raw % 2) ? raw : raw + 1;
};

// kBatchFast selects which index consecutive threads step through: the
// butterfly index within a sequence (false) or the sequence index (true).  The
// caller picks the one along which its load/store addresses are contiguous.
template <typename T, int N, int DIR, int NBATCH, int NT, bool kBatchFast = false, class Load, class Store>
__device__ __forceinline__ void fft2pass(cx<T>* mid, const cx<T>* root, Load load, Store store) {
  constexpr int RA = Split<N>::A;
  constexpr int RB = Split<N>::B;
  constexpr int RP = MidPitch<N>::row;
  constexpr int SP = MidPitch<N>::value;
  const int tid = threadIdx.x;
#pragma unroll 1
  for (int it = tid; it < NBATCH * RB; it += NT) {
    const int b = kBatchFast ? it % NBATCH : it / RB;
    const int j = kBatchFast ? it / NBATCH : it - b * RB;
    cx<T> v[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) v[r] = load(b, j + r * RB);
    SmallDft<T, RA, DIR>::run(v);
#pragma unroll
    for (int r = 0; r < RA; ++r) mid[b * SP + r * RP + j] = v[r];
  }
  __syncthreads();
#pragma unroll 1
  for (int it = tid; it < NBATCH * RA; it += NT) {
    const int b = kBatchFast ? it % NBATCH : it / RA;
    const int k = kBatchFast ? it / NBATCH : it - b * RA;
    cx<T> v[RB];
#pragma unroll
    for (int t = 0; t < RB; ++t) v[t] = mid[b * SP + k * RP + t];
#pragma unroll
    for (int t = 1; t < RB; ++t) {
      const cx<T> w = root[t * k];  // t*k < N
      v[t] = cmul(v[t], DIR > 0 ? cconj(w) : w);
    }
    SmallDft<T, RB, DIR>::run(v);
#pragma unroll
    for (int t = 0; t < RB; ++t) store(b, k + RA * t, v[t]);
  }
}

}  // namespace dns
