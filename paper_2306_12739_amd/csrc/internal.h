// Internal interfaces between the host orchestration (dns_api.cpp), the host
// operator builder (operators.cpp) and the HIP kernels.
//
// Device layouts (members innermost, "E" = ensemble size):
//   state v, eta   : complex double [K][N][E]       K = Nx/2 * (Nz-1) modes
//   state U, W     : double         [My][E]         walls included
//   vel            : complex VT     [5][My][E/B][K][B]  u, v, w, du/dy, dw/dy
//   nl             : complex VT     [3][My][E/B][K][B]  advection N_u, N_v, N_w
// (the two stage buffers are member-outer in blocks of B = 2 members when E is
// even, below: [f][My][E/B][K][B], so that one plane workgroup's spectral input
// is a stride-B run; within an n_x row their modes are in stage_slot order)
//   means          : double         [2][My][E]      <uv>, <wv>
//   psum           : double         [NPS][My][E]    plane means for statistics
//   hist F, G      : complex double [K][N][E]       RK3 forcing history
//   hist EU, EW    : double         [N][E]
//   ops            : double [2 h][G][4][N][N]       A_v, B_v, A_eta, B_eta
// Mode index m = nx*(Nz-1) + iz with iz in FFT order; operator group
// g = nx*(Nz/2) + |nz| holds the modes (nx, +nz) and (nx, -nz).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

namespace dns {

// Order of the kz modes within an n_x row of the stage buffers: kz = 0, then
// +1, -1, +2, -2, ...  A per-mode workgroup owns the pair (+|kz|, -|kz|) of
// every row, so its loads and stores of the pair fall in one cache line.
__host__ __device__ constexpr int stage_slot(int nz) { return nz > 0 ? 2 * nz - 1 : -2 * nz; }
__host__ __device__ constexpr int stage_kz(int slot) { return (slot & 1) ? (slot + 1) >> 1 : -(slot >> 1); }
static_assert(stage_slot(0) == 0 && stage_slot(1) == 1 && stage_slot(-1) == 2 && stage_slot(-3) == 6 &&
                  stage_kz(5) == 3 && stage_kz(6) == -3 && stage_kz(0) == 0,
              "stage slot order");

// Members of the stage buffers come in pairs when E is even (log2 of the block
// returned), innermost: a per-mode workgroup's values of one mode, node and
// field for two members then share a cache line, while an advection workgroup's
// row of modes (one member) keeps a stride of two elements.  Blocks of four
// made the advection kernel's strided rows cost more than the per-mode kernel
// saved.
__host__ __device__ constexpr int stage_block_log2(int E) { return E % 2 == 0 ? 1 : 0; }
// Complex-element offset of (row r = field * My + node, member e, stage
// position k) in a stage buffer of E members and K modes, blocks of 1 << lb.
__host__ __device__ constexpr size_t stage_off(size_t r, int e, int k, int E, int K, int lb) {
  return (((r * size_t(E >> lb) + size_t(e >> lb)) * size_t(K) + size_t(k)) << lb) + size_t(e & ((1 << lb) - 1));
}

enum PlaneSum { PS_UU = 0, PS_VV = 1, PS_WW = 2, PS_GRAD = 3, NPS = 4 };

struct PlaneArgs {
  const void* vel;
  void* nl;
  double* means;
  double* psum;   // nullptr: skip statistics sums
  int My, K, E;
  int e0, ec;       // members [e0, e0 + ec) of this launch
  int j0, nj;       // planes [j0, j0 + nj) of this launch
  double kxs, kzs;  // 2 pi / Lx, 2 pi / Lz
};

struct ModeArgs {
  // state (FP64)
  double* v;     // complex [K][N][E]
  double* eta;   // complex [K][N][E]
  double* U;     // [My][E]
  double* W;
  // RK3 history (FP64)
  double* hF;
  double* hG;
  double* hEU;   // [N][E]
  double* hEW;
  // pseudo-spectral stage buffers
  void* vel;          // complex VT [5][My][E/B][K][B] (written; B = stage member block)
  const void* nl;     // complex VT [3][My][E/B][K][B] (read)
  const double* means;  // [2][My][E]
  // operators, split by y parity and pre-tiled for v_mfma_f64_16x16x4f64 (see
  // tile_for_mfma): He = ceil(N/2), Ho = floor(N/2), Fe = He + 1, Fo = Ho + 1
  const double* opsT;      // per group: [A_v|B_v] even (He x 2He), odd (Ho x 2Ho),
                           // then [A_eta|B_eta] even, odd
  size_t op_group_stride;  // doubles per group
  const double* meanT;     // [A_U|B_U] even, odd
  const double* D1intT_e;  // D1 interior rows: even full half -> odd interior half (Ho x Fe)
  const double* D1intT_o;  // odd full half -> even interior half (He x Fo)
  const double* D1cT_e;    // D1c: even interior half -> odd full half (Fo x He)
  const double* D1cT_o;    // odd interior half -> even full half (Fe x Ho)
  const double* D1T_e;     // D1: even full half -> odd full half (Fo x Fe)
  const double* D1T_o;     // odd full half -> even full half (Fe x Fo)
  // the same six derivative halves as bfloat16 pairs (hi + lo), tiled for
  // v_mfma_f32_16x16x16bf16_1k (see tile_for_mfma_bf16); used by the split-BF16
  // precision, index order D1int_e, D1int_o, D1c_e, D1c_o, D1_e, D1_o
  const unsigned short* Dhi[6];
  const unsigned short* Dlo[6];
  // the same six halves in FP32, in the A lane order of the FP64 tiles (the
  // FP32 matrix-core precision)
  const float* Df[6];
  const double* lift_h;    // [N]: even half (He) then odd half (Ho) of the Couette lift
  const double* green_h;   // [N]: halves of the pressure-gradient response
  const double* ccw_h;     // [Fe]: Clenshaw-Curtis weights summed over node pairs
  // per-member outputs
  // external forcing of Lap v and eta, state layout (nullptr: none)
  const double* fv;
  const double* feta;
  double* gamma;        // [E]
  int* failed;          // [E]
  unsigned long long* divmax;  // [E] (bit pattern of a non-negative double)
  // sizes and parameters
  int My, N, K, E, L, P, NZ, G, ET, ntiles;
  int e0, ec;           // members [e0, e0 + ec) of this launch (ntiles covers ec)
  int CRP, SR, TR;      // LDS geometry (mode_lds_geometry)
  int threads;          // workgroup size of launch_mode: 512 or 1024 (mode_tile_threads)
  double kxs, kzs, hdt, Ubot, Utop, Qtarget;
  int stage;      // 0, 1, 2: sub-step index; -1: velocities of the state only
  int freeze_mean;  // 1: sub-steps leave the n_x = 0 modes and U, W untouched
  int poiseuille;
};

// Kernel launchers (kernels_*.hip).  Return hipSuccess or the launch error.
// form 0: advective u . grad u; 1: rotational omega x u; 2: quasi-linear
// advective (n_x >= 1 output linearised about the streamwise mean); 3: adjoint
// of the linearised advection
constexpr int kPlaneForms = 4;
hipError_t launch_plane(int precision, int form, int Nx, int Nz, int variant, const PlaneArgs& a,
                        hipStream_t s);
// Plane-kernel variants built for (precision, form, Nx, Nz), index 0 being the
// default: returns how many (<= kMaxPlaneVariants).  rows[v] is the chunk-row
// count of variant v, plus kWaveRows for the lane-parallel advective kernel.
constexpr int kMaxPlaneVariants = 12;
constexpr int kWaveRows = 100;
constexpr int kWaveGlobalAcc = 50;
int plane_variants(int precision, int form, int Nx, int Nz, int* rows);
// Lane-parallel advective kernel (kernels_plane_wave.hip): the kernel of
// (precision, grid, code) or nullptr, where code is the chunk-row count plus
// kWaveGlobalAcc for the variant whose forward-z sums live in the output
// buffer; the built codes (default first); the workgroup size of a code.
const void* plane_wave_fn(int precision, int Nx, int Nz, int code);
int plane_wave_rows(int precision, int Nx, int Nz, int* codes);
int plane_wave_threads(int Nx, int code);
bool plane_supported(int Nx, int Nz);
hipError_t launch_mode(int precision, const ModeArgs& a, hipStream_t s);
// Several ensembles' per-mode kernels in one launch (kernels_mode.hip):
// descriptor d (device array descs) covers workgroups [first[d], first[d+1]).
hipError_t launch_mode_grouped(int precision, bool forced, const ModeArgs* descs, const int* first, int ndesc,
                               int nblk, size_t lds, hipStream_t s);
// Resolve kernels on the current device before any graph capture uses them.
hipError_t plane_preload(int Nx, int Nz);
hipError_t mode_preload();
hipError_t misc_preload();
int mode_member_tile(int My, int E, bool narrow_only);
void mode_lds_geometry(int My, int ET, int* CRP, int* SR, int* TR);
// per-mode workgroup sizes (512 threads; 1024 for member tiles whose LDS fits
// one workgroup per CU), the static LDS of a workgroup of that size (per-wave
// reduction slots of up to 16 columns, per-member gamma); LDS of one CU
constexpr int kModeThreadsNarrow = 512, kModeThreadsWide = 1024;
constexpr size_t mode_static_lds(int threads) { return size_t(threads / 64 * 16 + 64) * sizeof(double); }
constexpr size_t kLdsPerCU = 160 * 1024;
int mode_tile_threads(int My, int ET);

// Row-major R x Kd matrix -> bfloat16 A-operand tiles of the 16x16x16 BF16 MFMA,
// split M = hi + lo (each rounded to nearest even): tile (rt, kt), kt <
// ceil(Kd/16), is 64 lanes x 4 values, lane l holding M[16 rt + l % 16][16 kt +
// 4 (l / 16) + t], t < 4 (zero outside the matrix).
void tile_for_mfma_bf16(const double* M, int R, int Kd, int ldm, std::vector<unsigned short>* hi,
                        std::vector<unsigned short>* lo);

// Row-major R x Kd matrix (row stride ldm) -> MFMA A-operand tiles: tile
// (rt, kt), rt < ceil(R/16), kt < ceil(Kd/4), is 64 consecutive values with
// lane l holding M[16 rt + l % 16][4 kt + l / 16] (zero outside the matrix).
std::vector<double> tile_for_mfma(const double* M, int R, int Kd, int ldm);

// Half-size block of a matrix M (row stride ldm, Cn columns) for inputs of one
// y parity: columns k < ceil(Cn/2) (even) or floor(Cn/2) (odd) hold
// M[i][k] +/- M[i][Cn-1-k] (the centre column alone for even, odd Cn), rows
// i < rows_out are the first-half rows of M.
std::vector<double> half_block(const double* M, int rows_out, int Cn, int ldm, bool even_in);

// Plane sums (statistics) and plane means <uv>, <wv> of the two wall planes of
// members [e0, e0 + ec), computed spectrally from the stage fields.
hipError_t launch_wall_sums(int precision, const void* vel, double* psum, double* means, int My, int E, int K,
                            int NZ, int P, double kxs, double kzs, int e0, int ec, hipStream_t s);

// Shared-mean ensembles: member averages of the n_x = 0 column (modes k < NZ)
// of the advection terms and plane means (in place, every member), and of the
// n_x = 0 column of two state-shaped buffers plus, if U is non-null, the mean
// profiles U, W.
hipError_t launch_member_mean(int precision, void* nl, double* means, int My, int E, int K, int NZ,
                              hipStream_t s);
hipError_t launch_share_columns(double* v, double* eta, double* U, double* W, int E, int N, int NZ,
                                int My, hipStream_t s);

// layout transposes between the host state layout and the device layout
hipError_t launch_state_to_device(const double* host_layout_dev, double* dev, int E0, int count,
                                  int E, int K, int N, hipStream_t s);
hipError_t launch_state_from_device(const double* dev, double* host_layout_dev, int E0, int count,
                                    int E, int K, int N, hipStream_t s);
hipError_t launch_profile_to_device(const double* host_layout_dev, double* dev, int E0, int count,
                                    int E, int My, hipStream_t s);
hipError_t launch_profile_from_device(const double* dev, double* host_layout_dev, int E0, int count,
                                      int E, int My, hipStream_t s);

struct StatsArgs {
  const double* psum;    // [NPS][My][E]
  const double* means;   // [2][My][E]
  const double* U;       // [My][E]
  const double* W;
  const double* ccw;     // [My]
  const double* D1;      // [My][My]
  const double* gamma;   // [E]
  double* acc;           // [NPA][My][E] time sums, then [2][E] wall shear sums
  double* inst;          // [NDI][E] instantaneous per-member diagnostics
  int* failed;           // [E] sticky non-finite flag
  int My, E;
  int e0, ec;            // members [e0, e0 + ec) of this launch
  double Re, Uw, poiseuille, Qtarget;
};
enum ProfileAcc { PA_U = 0, PA_W, PA_U2, PA_W2, PA_UU, PA_VV, PA_WW, PA_UV, NPA };
enum InstDiag { DI_E = 0, DI_EPS, DI_PI, DI_Q, DI_TLO, DI_THI, NDI };
hipError_t launch_stats(const StatsArgs& a, int accumulate, hipStream_t s);

// Host operator builder (operators.cpp), long double internally.
struct HostOperators {
  int My = 0, N = 0, G = 0;
  std::vector<double> D1;      // My*My
  std::vector<double> D1c;     // My*N
  std::vector<double> ccw;     // My
  std::vector<double> ops[2];  // per h: G*4*N*N
  std::vector<double> mean_ops[2];  // per h: 2*N*N
  std::vector<double> lift[2];      // per h: N
  std::vector<double> green[2];     // per h: N
  double max_cond = 0.0;
};
// h index 0 is h = 1/2, index 1 is h = 1.  v_discretization 0: clamped fourth-
// derivative operator; 1: Helmholtz-Poisson system with clamped walls.
int build_operators(int My, int L, int P, double kxs, double kzs, double Re, double dt,
                    double Ubot, double Utop, HostOperators* out, int v_discretization = 0);

// ---- channel form of states (learned spin-up) -------------------------------------
// cinv: Chebyshev coefficients from node values (My x My); tmat: node values
// from coefficients (My x My); phys: count * 3 * My planes of Mz x Mx doubles;
// spec: count * 3 * My * K complex doubles.
hipError_t launch_to_channels(int precision, const void* vel, double* phys, const double* cinv, float* out, int My,
                              int E, int K, int L, int NZ, int Mx, int Mz, int member0, int count, hipStream_t s);
hipError_t launch_from_channels(const float* in, double* phys, double* spec, const double* tmat, double* v,
                                double* eta, double* U, double* W, int My, int E, int L, int NZ, int Mx, int Mz,
                                int member0, int count, double kxs, double kzs, double Ubot, double Utop,
                                hipStream_t s);
// Fixed per-device scratch of the allocation-free hand-off (a __device__ array
// of kNoAllocScratchBytes).  noalloc_scratch_init looks up its address on
// `device`, which must be current, once per device; noalloc_scratch returns
// that address (nullptr before the lookup).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch_init(int device);
double* noalloc_scratch(int device);
// p[0..n) = 0 by a kernel (no memset node in a captured stream)
hipError_t launch_clear_ints(int* p, int n, hipStream_t s);

// ---- spectral neural operator (learned spin-up) --------------------------------
// C[b][m][n] = alpha * sum_k A[b][m][k] B[b][k][n] + beta * C[b][m][n]; element
// (m, k) of batch b of A sits at A + b * sab + m * sam + k * sak (likewise B, C).
// reduce_batch: C has no batch index and receives the sum over all batches.
// beta == 0 never reads C.
struct GemmArgs {
  const float* A;
  long long sam, sak, sab;
  const float* B;
  long long sbk, sbn, sbb;
  float* C;
  long long scm, scn, scb;
  int M, N, K, batch;
  float alpha, beta;
  int reduce_batch;
};
hipError_t launch_gemm(const GemmArgs& g, bool bf16, hipStream_t s);
hipError_t launch_bias_act(float* x, float* h, const float* bias, int B, int C, int P, hipStream_t s);
hipError_t launch_gelu_bwd(float* dh, const float* z, long long n, hipStream_t s);
hipError_t launch_channel_sum(const float* x, float* out, int B, int C, int P, hipStream_t s);
hipError_t launch_loss(const float* yhat, const float* y, double* sq, float* dy, float* loss, int B, long long per,
                       hipStream_t s);
hipError_t launch_batch_sum(const float* t, float* c, int batch, long long n, hipStream_t s);
hipError_t launch_adamw(float* w, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                        float eps, float wd, int t, hipStream_t s);

}  // namespace dns
