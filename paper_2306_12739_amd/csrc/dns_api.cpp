// C ABI of the ensemble DNS library: handle lifetime, state I/O, the CN/RK3
// step orchestration and statistics.  See include/dns.h for the contract.
//
// One time step (paper Sec. 3.1) is three sub-steps s = 0, 1, 2 with
// h = 1/2, 1, 1.  Each sub-step is two kernels:
//   plane kernel  (one workgroup per Chebyshev plane and member): velocity
//                 fields -> 3/2-padded physical grid -> u.grad u -> truncated
//                 spectrum, plane means <uv>, <wv>;
//   mode kernel   (one workgroup per (nx, |nz|) operator group and member
//                 tile): F, G, RK3 combination, FP64 CN solves, velocities of
//                 the next sub-step's state.
// After sub-step 0's plane kernel a small kernel evaluates per-member
// diagnostics (and, when enabled, accumulates one-point statistics) of the
// state at the start of the step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dns.h"
#include "../../include/sno.h"
#include "internal.h"

using namespace dns;

static_assert(kNoAllocScratchBytes == DNS_NOALLOC_SCRATCH_BYTES, "scratch size of the header and the library");

struct dns_handle {
  // problem
  int flow = 0;
  double Lx = 0, Lz = 0, Uw = 1, flux = 4.0 / 3.0, Re = 0, dt = 0;
  int Nx = 0, Ny = 0, Nz = 0, E = 0;
  int L = 0, P = 0, NZ = 0, K = 0, N = 0, My = 0, G = 0;
  double kxs = 0, kzs = 0, Ubot = 0, Utop = 0;
  // options
  int precision = DNS_PREC_FP64;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  bool use_graph = false;
  bool stats_on = false;
  // device buffers
  double *v = nullptr, *eta = nullptr, *U = nullptr, *W = nullptr;
  double *hF = nullptr, *hG = nullptr, *hEU = nullptr, *hEW = nullptr;
  void *vel = nullptr, *nl = nullptr;
  double *means = nullptr, *psum = nullptr;
  double *opsT[2] = {nullptr, nullptr}, *meanT[2] = {nullptr, nullptr};
  size_t op_group_stride = 0;
  double *D1intT_e = nullptr, *D1intT_o = nullptr, *D1cT_e = nullptr, *D1cT_o = nullptr;
  double *D1T_e = nullptr, *D1T_o = nullptr;
  unsigned short *Dhi[6] = {}, *Dlo[6] = {};  // split-BF16 tiles of the six derivative halves
  float* Df[6] = {};                            // FP32 tiles of the six derivative halves
  int CRP = 16, SR = 0, TR = 0;
  double *lift_h[2] = {nullptr, nullptr}, *green_h[2] = {nullptr, nullptr};
  double *ccw_h = nullptr, *D1 = nullptr, *ccw = nullptr;
  double *cheb_cinv = nullptr, *cheb_t = nullptr;  // channel form: coefficients <-> node values
  double* gamma = nullptr;
  int* failed = nullptr;
  unsigned long long* divmax = nullptr;
  double *acc = nullptr, *inst = nullptr;
  double* staging = nullptr;
  size_t staging_bytes = 0;
  int ET = 1, ntiles = 1;
  int mode_threads = kModeThreadsNarrow;  // per-mode workgroup size of tile ET (mode_tile_threads)
  int plane_var[2][kPlaneForms] = {};  // plane-kernel variant per precision (FP64, mixed) and form
  int advection = DNS_ADV_ADVECTIVE;
  // shared-mean ensemble: one streamwise mean for all members, optionally
  // quasi-linear perturbations, and an additive (Lap v, eta) forcing
  bool shared_mean = false;
  int quasilinear = 0;        // 0 full advection, 1 linearised, 2 adjoint of the linearised
  bool frozen_mean = false;   // sub-steps leave the n_x = 0 modes and U, W untouched
  int v_discretization = DNS_VDISC_CLAMPED;
  std::vector<double> host_D1c, host_ccw;  // for energy inner products on the host
  bool forcing_on = false;
  double *fv = nullptr, *feta = nullptr;
  // member chains advanced concurrently within a step
  int nchain = 1;
  std::vector<hipStream_t> chain_stream;
  std::vector<hipEvent_t> chain_join;
  hipEvent_t chain_fork = nullptr;
  // progress
  long long steps = 0, samples = 0;
  bool vel_fresh = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_valid = false;
  double max_cond = 0.0;
  int device = 0;  // the device current at creation
  std::string err;
  // grouped handle: ensembles of different grid, Re, box or dt advanced by one
  // dns_step (members numbered group-major); each group runs on its own stream,
  // forked from and joined back into this handle's stream
  std::vector<dns_handle*> sub;
  std::vector<int> sub_base;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  dns_handle* parent = nullptr;
  // grouped handle: every group's per-mode work in one launch per sub-step
  // (descriptors [sub-step][group] and block offsets on the device, their host
  // copy to detect changes); group_streams = true runs each group's kernels on
  // its own stream instead
  bool group_streams = false;
  ModeArgs* gdesc = nullptr;
  int* gfirst = nullptr;
  std::vector<ModeArgs> gdesc_host;
  std::vector<int> gfirst_host;
  size_t glds = 0;
  std::vector<hipEvent_t> gfork;  // per member chain: start of a sub-step's advection work
  bool grouped() const { return !sub.empty(); }
};

namespace {

thread_local std::string g_thread_err;

int fail(dns_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_thread_err = msg;
  return code;
}

#define HIP_OR_FAIL(h, call)                                                              \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((h), DNS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

size_t vt_size(int precision) { return precision == DNS_PREC_FP64 ? sizeof(double) : sizeof(float); }

void destroy_one(dns_handle* h);

void free_all(dns_handle* h) {
  if (h->gexec) hipGraphExecDestroy(h->gexec);
  if (h->graph) hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  for (dns_handle* s : h->sub) {
    s->parent = nullptr;
    destroy_one(s);
  }
  h->sub.clear();
  for (hipEvent_t e : h->join)
    if (e) hipEventDestroy(e);
  h->join.clear();
  for (hipEvent_t e : h->gfork)
    if (e) hipEventDestroy(e);
  h->gfork.clear();
  for (hipStream_t st : h->chain_stream)
    if (st) hipStreamDestroy(st);
  h->chain_stream.clear();
  for (hipEvent_t e : h->chain_join)
    if (e) hipEventDestroy(e);
  h->chain_join.clear();
  if (h->chain_fork) hipEventDestroy(h->chain_fork);
  h->chain_fork = nullptr;
  if (h->fork) hipEventDestroy(h->fork);
  h->fork = nullptr;
  void* bufs[] = {h->v, h->eta, h->U, h->W, h->hF, h->hG, h->hEU, h->hEW, h->vel, h->nl,
                  h->means, h->psum, h->opsT[0], h->opsT[1], h->meanT[0], h->meanT[1],
                  h->D1intT_e, h->D1intT_o, h->D1cT_e, h->D1cT_o, h->D1T_e, h->D1T_o,
                  h->lift_h[0], h->lift_h[1], h->green_h[0], h->green_h[1], h->ccw_h,
                  h->D1, h->ccw, h->cheb_cinv, h->cheb_t,
                  h->gamma, h->failed, h->divmax, h->acc, h->inst, h->staging, h->fv, h->feta,
                  h->gdesc, h->gfirst};
  for (void* p : bufs)
    if (p) hipFree(p);
  for (int i = 0; i < 6; ++i) {
    if (h->Dhi[i]) hipFree(h->Dhi[i]);
    if (h->Dlo[i]) hipFree(h->Dlo[i]);
    if (h->Df[i]) hipFree(h->Df[i]);
  }
  if (h->own_stream) hipStreamDestroy(h->own_stream);
}

// Chebyshev interpolation on the ascending nodes y_j = -cos(pi j / n), n = My - 1:
// T_k(y_j) = (-1)^k cos(pi k j / n); coefficients by the discrete cosine
// (DCT-I) orthogonality, a_k = 2 / (n c_k) sum_j T_k(y_j) f_j / c_j, c_0 = c_n = 2.
int ensure_cheb(dns_handle* h) {
  if (h->cheb_cinv) return DNS_OK;
  const int My = h->My, n = My - 1;
  std::vector<double> T(size_t(My) * My), Ci(size_t(My) * My);
  auto Tk = [&](int k, int j) {
    const long long r = (long long)k * j % (2 * n);
    return ((k & 1) ? -1.0 : 1.0) * std::cos(M_PI * double(r) / n);
  };
  for (int j = 0; j < My; ++j)
    for (int k = 0; k < My; ++k) T[size_t(j) * My + k] = Tk(k, j);
  for (int k = 0; k < My; ++k)
    for (int j = 0; j < My; ++j) {
      const double ck = (k == 0 || k == n) ? 2.0 : 1.0, cj = (j == 0 || j == n) ? 2.0 : 1.0;
      Ci[size_t(k) * My + j] = 2.0 / (n * ck) * Tk(k, j) / cj;
    }
  if (dalloc(&h->cheb_cinv, Ci.size()) != hipSuccess || dalloc(&h->cheb_t, T.size()) != hipSuccess)
    return fail(h, DNS_E_NOMEM, "hipMalloc Chebyshev matrices");
  HIP_OR_FAIL(h, hipMemcpy(h->cheb_cinv, Ci.data(), Ci.size() * 8, hipMemcpyHostToDevice));
  HIP_OR_FAIL(h, hipMemcpy(h->cheb_t, T.data(), T.size() * 8, hipMemcpyHostToDevice));
  return DNS_OK;
}

int ensure_staging(dns_handle* h, size_t bytes) {
  if (bytes <= h->staging_bytes) return DNS_OK;
  if (h->staging) hipFree(h->staging);
  h->staging = nullptr;
  h->staging_bytes = 0;
  HIP_OR_FAIL(h, hipMalloc(reinterpret_cast<void**>(&h->staging), bytes));
  h->staging_bytes = bytes;
  return DNS_OK;
}

ModeArgs mode_args(dns_handle* h, int stage, int e0 = 0, int ec = -1) {
  ModeArgs a{};
  if (ec < 0) ec = h->E;
  a.e0 = e0;
  a.ec = ec;
  const int hi = stage == 0 ? 0 : 1;
  const double hval = stage == 0 ? 0.5 : 1.0;
  a.v = h->v;
  a.eta = h->eta;
  a.U = h->U;
  a.W = h->W;
  a.hF = h->hF;
  a.hG = h->hG;
  a.fv = h->forcing_on ? h->fv : nullptr;
  a.feta = h->forcing_on ? h->feta : nullptr;
  a.hEU = h->hEU;
  a.hEW = h->hEW;
  a.vel = h->vel;
  a.nl = h->nl;
  a.means = h->means;
  a.opsT = h->opsT[hi];
  a.op_group_stride = h->op_group_stride;
  a.meanT = h->meanT[hi];
  a.D1intT_e = h->D1intT_e;
  a.D1intT_o = h->D1intT_o;
  a.D1cT_e = h->D1cT_e;
  a.D1cT_o = h->D1cT_o;
  a.D1T_e = h->D1T_e;
  a.D1T_o = h->D1T_o;
  for (int i = 0; i < 6; ++i) {
    a.Dhi[i] = h->Dhi[i];
    a.Dlo[i] = h->Dlo[i];
    a.Df[i] = h->Df[i];
  }
  a.lift_h = h->lift_h[hi];
  a.green_h = h->green_h[hi];
  a.ccw_h = h->ccw_h;
  a.CRP = h->CRP;
  a.SR = h->SR;
  a.TR = h->TR;
  a.threads = h->mode_threads;
  a.gamma = h->gamma;
  a.failed = h->failed;
  a.divmax = h->divmax;
  a.My = h->My;
  a.N = h->N;
  a.K = h->K;
  a.E = h->E;
  a.L = h->L;
  a.P = h->P;
  a.NZ = h->NZ;
  a.G = h->G;
  a.ET = h->ET;
  a.ntiles = (ec + h->ET - 1) / h->ET;
  a.kxs = h->kxs;
  a.kzs = h->kzs;
  a.hdt = hval * h->dt;
  a.Ubot = h->Ubot;
  a.Utop = h->Utop;
  a.Qtarget = h->flux;
  a.stage = stage;
  a.freeze_mean = h->frozen_mean ? 1 : 0;
  a.poiseuille = h->flow == DNS_FLOW_POISEUILLE;
  return a;
}

// [A | B] of N x N operators restricted to one y parity (n x 2n, n = ceil(N/2)
// even or floor(N/2) odd), tiled for the FP64 MFMA.
std::vector<double> parity_pair_block(const double* A, const double* B, int N, bool even) {
  const int n = even ? (N + 1) / 2 : N / 2;
  const std::vector<double> a = half_block(A, n, N, N, even);
  const std::vector<double> b = half_block(B, n, N, N, even);
  std::vector<double> cat(size_t(n) * 2 * n);
  for (int r = 0; r < n; ++r)
    for (int k = 0; k < n; ++k) {
      cat[size_t(r) * 2 * n + k] = a[size_t(r) * n + k];
      cat[size_t(r) * 2 * n + n + k] = b[size_t(r) * n + k];
    }
  return tile_for_mfma(cat.data(), n, 2 * n, 2 * n);
}

// Every fluctuation group's [A_v|B_v] (even, odd) then [A_eta|B_eta] (even,
// odd) for sub-step fraction index hi, in the layout of dns_handle::opsT.
std::vector<double> tile_group_operators(const HostOperators& ho, int hi, int N, int G, size_t stride) {
  const size_t nn = size_t(N) * N;
  std::vector<double> out(size_t(G) * stride, 0.0);
  for (int g = 1; g < G; ++g) {
    const double* base = ho.ops[hi].data() + size_t(g) * 4 * nn;
    auto dst = out.begin() + size_t(g) * stride;
    for (int blk = 0; blk < 4; ++blk) {  // v even, v odd, eta even, eta odd
      const double* A = base + (blk < 2 ? 0 : 2 * nn);
      const std::vector<double> t = parity_pair_block(A, A + nn, N, (blk & 1) == 0);
      dst = std::copy(t.begin(), t.end(), dst);
    }
  }
  return out;
}

// walls = false leaves out the two wall planes.  There, no-slip (v = 0 and u,
// w uniform in x-z) makes the plane means and the terms N_u, N_w vanish
// exactly in every advection form; N_v at a wall (zero in the advective form,
// -u du/dy in the rotational one) enters no interior equation.  Steps never
// visit them (the stage buffers start zeroed) and take their statistics sums
// from launch_wall_sums.
PlaneArgs plane_args(dns_handle* h, bool sums, int e0 = 0, int ec = -1, bool walls = true) {
  PlaneArgs a{};
  a.e0 = e0;
  a.ec = ec < 0 ? h->E : ec;
  a.j0 = walls ? 0 : 1;
  a.nj = walls ? h->My : h->My - 2;
  a.vel = h->vel;
  a.nl = h->nl;
  a.means = h->means;
  a.psum = sums ? h->psum : nullptr;
  a.My = h->My;
  a.K = h->K;
  a.E = h->E;
  a.kxs = h->kxs;
  a.kzs = h->kzs;
  return a;
}

// plane-kernel form: 0 advective, 1 rotational, 2 quasi-linear advective
int plane_form(const dns_handle* h) { return h->quasilinear ? 1 + h->quasilinear : h->advection; }
// some (form, precision) pairs have no chunk variant within the LDS of the larger grids
bool form_fits(const dns_handle* h, int precision, int form) {
  int rows[kMaxPlaneVariants];
  return plane_variants(precision == DNS_PREC_FP64 ? 0 : 1, form, h->Nx, h->Nz, rows) > 0;
}

int& plane_var(dns_handle* h) { return h->plane_var[h->precision == DNS_PREC_FP64 ? 0 : 1][plane_form(h)]; }

hipError_t plane_launch(dns_handle* h, bool sums, int e0 = 0, int ec = -1, hipStream_t st = nullptr,
                        bool walls = true) {
  return launch_plane(h->precision, plane_form(h), h->Nx, h->Nz, plane_var(h),
                      plane_args(h, sums, e0, ec, walls), st ? st : h->stream);
}

// Members per mode-kernel workgroup: 1, 2, 4 or 8, at most the ensemble size
// (rounded up to a power of two) and within 160 KB of LDS at the workgroup size
// the tile uses.
bool mode_tile_ok(const dns_handle* h, int et) {
  if (et != 1 && et != 2 && et != 4 && et != 8) return false;
  if (et > 1 && et / 2 >= h->E) return false;
  int crp, sr, tr;
  mode_lds_geometry(h->My, et, &crp, &sr, &tr);
  return size_t(2 * sr + tr) * crp * sizeof(double) + mode_static_lds(mode_tile_threads(h->My, et)) <= kLdsPerCU;
}

void set_mode_tile(dns_handle* h, int et) {
  h->ET = et;
  h->ntiles = (h->E + et - 1) / et;
  h->mode_threads = mode_tile_threads(h->My, et);
  mode_lds_geometry(h->My, et, &h->CRP, &h->SR, &h->TR);
}

StatsArgs stats_args(dns_handle* h, int e0 = 0, int ec = -1) {
  StatsArgs a{};
  a.e0 = e0;
  a.ec = ec < 0 ? h->E : ec;
  a.psum = h->psum;
  a.means = h->means;
  a.U = h->U;
  a.W = h->W;
  a.ccw = h->ccw;
  a.D1 = h->D1;
  a.gamma = h->gamma;
  a.acc = h->acc;
  a.inst = h->inst;
  a.failed = h->failed;
  a.My = h->My;
  a.E = h->E;
  a.Re = h->Re;
  a.Uw = h->Uw;
  a.poiseuille = h->flow == DNS_FLOW_POISEUILLE ? 1.0 : 0.0;
  a.Qtarget = h->flux;
  return a;
}

// Velocity fields of the current state (no time advance).
int refresh_velocities(dns_handle* h) {
  HIP_OR_FAIL(h, launch_mode(h->precision, mode_args(h, -1), h->stream));
  h->vel_fresh = true;
  return DNS_OK;
}

// Enqueue one time step; requires the velocity buffer to hold the state's velocities.
void invalidate_graph(dns_handle* h);

// Advance the members in n contiguous chains (streams and events made on first use).
int set_chains(dns_handle* h, int n) {
  if (n < 1 || n > DNS_MAX_CHAINS || n > h->E)
    return fail(h, DNS_E_INVALID, "member chains must be 1..DNS_MAX_CHAINS and at most the ensemble size");
  while (int(h->chain_stream.size()) < n) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    HIP_OR_FAIL(h, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    h->chain_stream.push_back(st);
    HIP_OR_FAIL(h, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    h->chain_join.push_back(ev);
  }
  if (!h->chain_fork) HIP_OR_FAIL(h, hipEventCreateWithFlags(&h->chain_fork, hipEventDisableTiming));
  h->nchain = n;
  invalidate_graph(h);
  return DNS_OK;
}

// One step of members [e0, e0 + ec) on stream st.
int enqueue_members(dns_handle* h, int e0, int ec, hipStream_t st) {
  for (int s = 0; s < 3; ++s) {
    // the wall planes' advection terms and means are exact zeros (the buffers
    // start zeroed); their statistics sums come from the spectral fields
    HIP_OR_FAIL(h, plane_launch(h, s == 0, e0, ec, st, false));
    if (s == 0)
      HIP_OR_FAIL(h, launch_wall_sums(h->precision == DNS_PREC_FP64 ? 0 : 1, h->vel, h->psum, h->means, h->My,
                                      h->E, h->K, h->NZ, h->P, h->kxs, h->kzs, e0, ec < 0 ? h->E : ec, st));
    if (h->shared_mean)  // one chain holds every member (set_chains)
      HIP_OR_FAIL(h, launch_member_mean(h->precision == DNS_PREC_FP64 ? 0 : 1, h->nl, h->means, h->My, h->E,
                                        h->K, h->NZ, st));
    if (s == 0) HIP_OR_FAIL(h, launch_stats(stats_args(h, e0, ec), h->stats_on ? 1 : 0, st));
    HIP_OR_FAIL(h, launch_mode(h->precision, mode_args(h, s, e0, ec), st));
  }
  return DNS_OK;
}

// Enqueue one time step; requires the velocity buffer to hold the state's
// velocities.  With several member chains, each chain's kernels run on a stream
// of its own (forked from and joined back into h->stream), so the advection
// kernel of one chain overlaps the per-mode kernel of another.
int enqueue_step(dns_handle* h) {
  const int nc = h->nchain;
  if (nc <= 1) return enqueue_members(h, 0, h->E, h->stream);
  HIP_OR_FAIL(h, hipEventRecord(h->chain_fork, h->stream));
  for (int c = 0; c < nc; ++c) {
    const int e0 = int((long long)h->E * c / nc), e1 = int((long long)h->E * (c + 1) / nc);
    hipStream_t st = h->chain_stream[c];
    HIP_OR_FAIL(h, hipStreamWaitEvent(st, h->chain_fork, 0));
    const int rc = enqueue_members(h, e0, e1 - e0, st);
    if (rc) return rc;
    HIP_OR_FAIL(h, hipEventRecord(h->chain_join[c], st));
    HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->chain_join[c], 0));
  }
  return DNS_OK;
}

void invalidate_graph(dns_handle* h) {
  if (h->gexec) hipGraphExecDestroy(h->gexec);
  if (h->graph) hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  h->graph_valid = false;
  if (h->parent) invalidate_graph(h->parent);  // a group's change stales the joint graph
}

// One step of every group: fork from h->stream, each group's kernels on its own
// stream (independent, so the device overlaps them), join back.
int enqueue_grouped(dns_handle* h) {
  HIP_OR_FAIL(h, hipEventRecord(h->fork, h->stream));
  for (size_t g = 0; g < h->sub.size(); ++g) {
    dns_handle* s = h->sub[g];
    HIP_OR_FAIL(h, hipStreamWaitEvent(s->stream, h->fork, 0));
    const int rc = enqueue_step(s);
    if (rc) return fail(h, rc, "group " + std::to_string(g) + ": " + s->err);
    HIP_OR_FAIL(h, hipEventRecord(h->join[g], s->stream));
    HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->join[g], 0));
  }
  return DNS_OK;
}

// The grouped one-launch path applies unless asked for per-group streams, a
// group carries an external forcing or the groups' precisions differ (a
// group's own handle can set one).
bool grouped_one_launch(const dns_handle* h) {
  if (h->group_streams) return false;
  for (const dns_handle* sh : h->sub)
    if (sh->forcing_on || sh->precision != h->sub[0]->precision) return false;
  return true;
}

// Member chains of the grouped one-launch path: two (each group's members
// split in halves, so that one chain's advection kernels overlap the other's
// per-mode launch), one when a group shares its streamwise mean across members.
int grouped_chains(const dns_handle* h) {
  for (const dns_handle* sh : h->sub)
    if (sh->shared_mean) return 1;
  return h->chain_stream.size() >= 2 ? 2 : 1;
}

// members [e0, e0 + ec) of group g in chain c of nc
void chain_slice(const dns_handle* sh, int c, int nc, int* e0, int* ec) {
  const int a = int((long long)sh->E * c / nc), b = int((long long)sh->E * (c + 1) / nc);
  *e0 = a;
  *ec = b - a;
}

// Per-mode descriptors [chain][sub-step][group] (each group's chain slice, its
// own tile shape) and block offsets [chain][group + 1], uploaded in stream
// order when they differ from the last upload.
int update_group_descs(dns_handle* h) {
  const int ng = int(h->sub.size());
  const int nc = grouped_chains(h);
  std::vector<ModeArgs> d(size_t(nc) * 3 * ng);
  std::vector<int> first(size_t(nc) * (ng + 1), 0);
  size_t lds = 0;
  for (int c = 0; c < nc; ++c) {
    int* fc = first.data() + size_t(c) * (ng + 1);
    for (int g = 0; g < ng; ++g) {
      dns_handle* sh = h->sub[g];
      int e0, ec;
      chain_slice(sh, c, nc, &e0, &ec);
      // the shared launch runs 512-thread workgroups: a group whose own tile
      // needs 1024 threads takes the largest tile of two such workgroups per CU
      // (results do not depend on the tile)
      int et = sh->ET, crp = sh->CRP, sr = sh->SR, tr = sh->TR;
      if (sh->mode_threads != kModeThreadsNarrow) {
        et = mode_member_tile(sh->My, sh->E, true);
        mode_lds_geometry(sh->My, et, &crp, &sr, &tr);
      }
      for (int st = 0; st < 3; ++st) {
        ModeArgs a = mode_args(sh, st, e0, ec);
        a.ET = et;
        a.ntiles = (ec + et - 1) / et;
        a.CRP = crp;
        a.SR = sr;
        a.TR = tr;
        a.threads = kModeThreadsNarrow;
        d[(size_t(c) * 3 + st) * ng + g] = a;
      }
      fc[g + 1] = fc[g] + sh->G * ((ec + et - 1) / et);
      lds = std::max(lds, size_t(2 * sr + tr) * crp * sizeof(double));
    }
  }
  const bool same = h->gdesc_host.size() == d.size() &&
                    std::memcmp(h->gdesc_host.data(), d.data(), d.size() * sizeof(ModeArgs)) == 0 &&
                    h->gfirst_host == first;
  if (same) return DNS_OK;
  if (h->gdesc_host.size() != d.size() || h->gfirst_host.size() != first.size()) {
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    if (h->gdesc) hipFree(h->gdesc);
    if (h->gfirst) hipFree(h->gfirst);
    h->gdesc = nullptr;
    h->gfirst = nullptr;
    HIP_OR_FAIL(h, dalloc(&h->gdesc, d.size()));
    HIP_OR_FAIL(h, dalloc(&h->gfirst, first.size()));
  }
  h->gdesc_host = d;
  h->gfirst_host = first;
  h->glds = lds;
  HIP_OR_FAIL(h, hipMemcpyAsync(h->gdesc, h->gdesc_host.data(), d.size() * sizeof(ModeArgs), hipMemcpyHostToDevice,
                                h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->gfirst, h->gfirst_host.data(), first.size() * sizeof(int),
                                hipMemcpyHostToDevice, h->stream));
  // the host copies must outlive the transfers
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  return DNS_OK;
}

// The stream that runs group sh's advection work for member chain c of the
// grouped one-launch path: the group's own chain stream, or its main stream.
hipStream_t group_chain_stream(const dns_handle* sh, int c) {
  return c < int(sh->chain_stream.size()) ? sh->chain_stream[c] : sh->stream;
}
hipEvent_t group_chain_event(const dns_handle* sh, int c) {
  return c < int(sh->chain_join.size()) ? sh->chain_join[c] : nullptr;
}

// One step of every group with one per-mode launch per sub-step and member
// chain.  Each chain runs on a stream of its own forked from and joined into
// h->stream; in each sub-step it forks again onto every group's stream for
// that chain, where the group's advection work for the chain's members runs
// (and, at the first sub-step, their wall sums and diagnostics), joins back
// and launches the per-mode kernel once over every group's workgroups of
// those members.
int enqueue_grouped_one_launch(dns_handle* h) {
  const int ng = int(h->sub.size());
  const int nc = int(h->gfirst_host.size()) / (ng + 1);
  HIP_OR_FAIL(h, hipEventRecord(h->chain_fork, h->stream));
  for (int c = 0; c < nc; ++c) HIP_OR_FAIL(h, hipStreamWaitEvent(h->chain_stream[c], h->chain_fork, 0));
  for (int st = 0; st < 3; ++st) {
    for (int c = 0; c < nc; ++c) {
      hipStream_t cs = h->chain_stream[c];
      const int* fc = h->gfirst_host.data() + size_t(c) * (ng + 1);
      HIP_OR_FAIL(h, hipEventRecord(h->gfork[c], cs));
      for (int g = 0; g < ng; ++g) {
        dns_handle* sh = h->sub[g];
        int e0, ec;
        chain_slice(sh, c, nc, &e0, &ec);
        if (ec == 0) continue;
        hipStream_t gs = group_chain_stream(sh, c);
        hipEvent_t ge = group_chain_event(sh, c);
        if (ge) HIP_OR_FAIL(h, hipStreamWaitEvent(gs, h->gfork[c], 0));
        else gs = cs;  // no stream of its own for this chain: run on the chain's
        HIP_OR_FAIL(h, plane_launch(sh, st == 0, e0, ec, gs, false));
        if (st == 0)
          HIP_OR_FAIL(h, launch_wall_sums(sh->precision == DNS_PREC_FP64 ? 0 : 1, sh->vel, sh->psum, sh->means,
                                          sh->My, sh->E, sh->K, sh->NZ, sh->P, sh->kxs, sh->kzs, e0, ec, gs));
        if (sh->shared_mean)  // one chain holds every member (grouped_chains)
          HIP_OR_FAIL(h, launch_member_mean(sh->precision == DNS_PREC_FP64 ? 0 : 1, sh->nl, sh->means, sh->My,
                                            sh->E, sh->K, sh->NZ, gs));
        if (st == 0) HIP_OR_FAIL(h, launch_stats(stats_args(sh, e0, ec), sh->stats_on ? 1 : 0, gs));
        if (ge) {
          HIP_OR_FAIL(h, hipEventRecord(ge, gs));
          HIP_OR_FAIL(h, hipStreamWaitEvent(cs, ge, 0));
        }
      }
      // every group has the precision of the grouped handle's options (set on all groups)
      if (fc[ng] > 0)
        HIP_OR_FAIL(h, launch_mode_grouped(h->sub[0]->precision, false, h->gdesc + (size_t(c) * 3 + st) * ng,
                                           h->gfirst + size_t(c) * (ng + 1), ng, fc[ng], h->glds, cs));
    }
  }
  for (int c = 0; c < nc; ++c) {
    HIP_OR_FAIL(h, hipEventRecord(h->chain_join[c], h->chain_stream[c]));
    HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->chain_join[c], 0));
  }
  return DNS_OK;
}

int enqueue_any(dns_handle* h) {
  if (!h->grouped()) return enqueue_step(h);
  return grouped_one_launch(h) ? enqueue_grouped_one_launch(h) : enqueue_grouped(h);
}

int build_graph(dns_handle* h) {
  invalidate_graph(h);
  HIP_OR_FAIL(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_any(h);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (rc != DNS_OK) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(h, DNS_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  h->graph = g;
  HIP_OR_FAIL(h, hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
  h->graph_valid = true;
  return DNS_OK;
}

int any_failed(dns_handle* h, std::vector<int>* flags) {
  std::vector<int> f(h->E, 0);
  if (hipMemcpyAsync(f.data(), h->failed, sizeof(int) * h->E, hipMemcpyDeviceToHost, h->stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return -1;
  int any = 0;
  for (int x : f) any |= x;
  if (flags) *flags = f;
  return any;
}

void destroy_one(dns_handle* h) {
  if (!h) return;
  if (h->stream) hipStreamSynchronize(h->stream);
  free_all(h);
  delete h;
}

// Group g holding member m of a grouped handle, or -1.
int group_of(const dns_handle* h, int m) {
  for (size_t g = 0; g < h->sub.size(); ++g)
    if (m >= h->sub_base[g] && m < h->sub_base[g] + h->sub[g]->E) return int(g);
  return -1;
}

// Route a member range of a grouped handle to its group; the range must lie in one group.
int route(dns_handle* h, int member0, int count, dns_handle** s, int* local0) {
  const int g = member0 >= 0 && count >= 1 ? group_of(h, member0) : -1;
  if (g < 0 || member0 + count > h->sub_base[g] + h->sub[g]->E)
    return fail(h, DNS_E_INVALID, "member range must lie inside one group");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  *s = h->sub[g];
  *local0 = member0 - h->sub_base[g];
  return DNS_OK;
}

// Calls on a group's handle are ordered after the work its grouped handle has queued.
int after_parent(dns_handle* h) {
  if (h->parent) HIP_OR_FAIL(h, hipStreamSynchronize(h->parent->stream));
  return DNS_OK;
}

#define ORDER_AFTER_PARENT(h)       \
  do {                              \
    const int rc_ = after_parent(h); \
    if (rc_) return rc_;            \
  } while (0)

int forward(dns_handle* h, dns_handle* s, int rc) {
  if (rc != DNS_OK) return fail(h, rc, s->err);
  return DNS_OK;
}

int check_dims(int Nx, int Ny, int Nz, int E) {
  if (Nx <= 0 || Nz <= 0 || (Nx % 2) || (Nz % 2)) return DNS_E_INVALID;
  if (Ny < 5 || Ny > 257) return DNS_E_INVALID;
  if (E < 1) return DNS_E_INVALID;
  if (!plane_supported(Nx, Nz)) return DNS_E_UNSUPPORTED;
  return DNS_OK;
}

// Requirements of a state on its n_x = 0 column (Appendix A stores half of
// the conjugate pairs: f(0, -n_z) = conj f(0, n_z); the (0,0) mode of v and
// eta is zero, the mean flow living in U00, W00).  col: one member's column,
// NZ x N interleaved complex values with n_z in FFT order.  Both rules hold
// within 1e-12 of the column's largest entry; a NaN fails every comparison.
const char* column_violation(const double* col, int NZ, int N) {
  const int P = (NZ + 1) / 2;
  double top = 0.0;
  for (size_t q = 0; q < size_t(NZ) * N * 2; ++q) top = std::fmax(top, std::fabs(col[q]));
  const double tol = 1e-12 * top;
  for (int j = 0; j < N; ++j)
    if (!(std::hypot(col[2 * j], col[2 * j + 1]) <= tol)) return "the (0,0) mode is not zero";
  for (int iz = 1; iz < NZ; ++iz) {
    const int nz = iz < P ? iz : iz - NZ;
    const int mirror = (NZ - nz) % NZ;
    for (int j = 0; j < N; ++j) {
      const double* a = col + 2 * (size_t(iz) * N + j);
      const double* b = col + 2 * (size_t(mirror) * N + j);
      if (!(std::hypot(a[0] - b[0], a[1] + b[1]) <= tol)) return "the n_x = 0 column is not Hermitian";
    }
  }
  return nullptr;
}

// Wall values of one member's U00, W00 (My nodes) against the boundary
// conditions (Eq. (b_ve) and the wall speeds of Sec. 2); NaN fails.
const char* wall_violation(const double* U, const double* W, int My, double Ubot, double Utop) {
  if (!(std::fabs(U[0] - Ubot) <= 1e-12) || !(std::fabs(U[My - 1] - Utop) <= 1e-12) ||
      !(std::fabs(W[0]) <= 1e-12) || !(std::fabs(W[My - 1]) <= 1e-12))
    return "U00/W00 wall values do not match the boundary conditions";
  return nullptr;
}

// Host state view (host layout of dns_state_view) of count members.
int check_host_state(dns_handle* h, int L, int NZ, int N, int My, double Ubot, double Utop, int count,
                     const dns_state_view* s) {
  const size_t per = size_t(L) * NZ * N * 2;
  for (int m = 0; m < count; ++m) {
    std::string why;
    if (const char* w = wall_violation(s->U00 + size_t(m) * My, s->W00 + size_t(m) * My, My, Ubot, Utop))
      why = w;
    else if (const char* c = column_violation(s->v_hat + m * per, NZ, N))
      why = std::string("v_hat: ") + c;
    else if (const char* c2 = column_violation(s->eta_hat + m * per, NZ, N))
      why = std::string("eta_hat: ") + c2;
    if (!why.empty()) return fail(h, DNS_E_INVALID, "member " + std::to_string(m) + ": " + why);
  }
  return DNS_OK;
}

}  // namespace

extern "C" {

int dns_check_state(const dns_geometry* g, int Nx, int Ny, int Nz, int count, const dns_state_view* s) {
  if (!g || !s || !s->v_hat || !s->eta_hat || !s->U00 || !s->W00)
    return fail(nullptr, DNS_E_INVALID, "geometry or state view is NULL");
  if (s->on_device) return fail(nullptr, DNS_E_INVALID, "dns_check_state reads host views only");
  if (g->flow != DNS_FLOW_COUETTE && g->flow != DNS_FLOW_POISEUILLE)
    return fail(nullptr, DNS_E_INVALID, "unknown flow type");
  if (Nx <= 0 || Nz <= 0 || (Nx % 2) || (Nz % 2) || Ny < 5 || count < 1)
    return fail(nullptr, DNS_E_INVALID, "need even Nx, Nz > 0, Ny >= 5 and count >= 1");
  const double Uw = g->Uw > 0 ? g->Uw : 1.0;
  const double Ubot = g->flow == DNS_FLOW_COUETTE ? -Uw : 0.0, Utop = g->flow == DNS_FLOW_COUETTE ? Uw : 0.0;
  return check_host_state(nullptr, Nx / 2, Nz - 1, Ny - 2, Ny, Ubot, Utop, count, s);
}

int dns_create(const dns_geometry* g, double Re, int Nx, int Ny, int Nz, int ensemble, double dt,
               dns_handle** out) {
  if (!out) return fail(nullptr, DNS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!g) return fail(nullptr, DNS_E_INVALID, "geometry is NULL");
  if (g->flow != DNS_FLOW_COUETTE && g->flow != DNS_FLOW_POISEUILLE)
    return fail(nullptr, DNS_E_INVALID, "unknown flow type");
  if (!(g->Lx > 0) || !(g->Lz > 0) || !(Re > 0) || !(dt > 0) || !std::isfinite(Re) ||
      !std::isfinite(dt))
    return fail(nullptr, DNS_E_INVALID, "Lx, Lz, Re and dt must be positive and finite");
  const int dc = check_dims(Nx, Ny, Nz, ensemble);
  if (dc == DNS_E_INVALID)
    return fail(nullptr, dc, "need even Nx, Nz > 0, 5 <= Ny <= 257 and ensemble >= 1");
  if (dc == DNS_E_UNSUPPORTED)
    return fail(nullptr, dc,
                "grid not built: Nx == Nz in {16, 32, 48, 64, 72, 96}, and (Nx, Nz) = (64, 32) or (32, 64) "
                "for the advective form, are supported");
  {
    // one member per per-mode workgroup must fit the workgroup LDS (Ny <= 254)
    int crp, sr, tr;
    mode_lds_geometry(Ny, 1, &crp, &sr, &tr);
    if (size_t(2 * sr + tr) * crp * sizeof(double) + mode_static_lds(kModeThreadsNarrow) > kLdsPerCU)
      return fail(nullptr, DNS_E_UNSUPPORTED, "Ny too large: the per-mode kernel's LDS holds Ny <= 254");
  }

  dns_handle* h = new dns_handle();
  h->flow = g->flow;
  h->Lx = g->Lx;
  h->Lz = g->Lz;
  h->Uw = g->Uw > 0 ? g->Uw : 1.0;
  h->flux = g->flux > 0 ? g->flux : 4.0 / 3.0;
  h->Re = Re;
  h->dt = dt;
  h->Nx = Nx;
  h->Ny = Ny;
  h->Nz = Nz;
  h->E = ensemble;
  h->L = Nx / 2;
  h->P = Nz / 2;
  h->NZ = Nz - 1;
  h->K = h->L * h->NZ;
  h->My = Ny;
  h->N = Ny - 2;
  h->G = h->L * h->P;
  h->kxs = 2.0 * M_PI / g->Lx;
  h->kzs = 2.0 * M_PI / g->Lz;
  if (h->flow == DNS_FLOW_COUETTE) {
    h->Ubot = -h->Uw;
    h->Utop = h->Uw;
  }
  set_mode_tile(h, mode_member_tile(h->My, h->E, false));

  HostOperators ho;
  if (build_operators(h->My, h->L, h->P, h->kxs, h->kzs, Re, dt, h->Ubot, h->Utop, &ho) != 0) {
    delete h;
    return fail(nullptr, DNS_E_INVALID, "a Crank-Nicolson operator is singular");
  }
  h->max_cond = ho.max_cond;
  h->host_D1c = ho.D1c;
  h->host_ccw = ho.ccw;

  auto fail_free = [&](int code, const std::string& msg) {
    free_all(h);
    delete h;
    return fail(nullptr, code, msg);
  };
#define ALLOC(ptr, n)                                                      \
  if (dalloc(&(ptr), (n)) != hipSuccess) return fail_free(DNS_E_NOMEM, "hipMalloc " #ptr);
  const size_t KNE = size_t(h->K) * h->N * h->E;
  const size_t MyE = size_t(h->My) * h->E;
  ALLOC(h->v, 2 * KNE);
  ALLOC(h->eta, 2 * KNE);
  ALLOC(h->U, MyE);
  ALLOC(h->W, MyE);
  ALLOC(h->hF, 2 * KNE);
  ALLOC(h->hG, 2 * KNE);
  ALLOC(h->hEU, size_t(h->N) * h->E);
  ALLOC(h->hEW, size_t(h->N) * h->E);
  {
    const size_t velb = size_t(5) * h->My * h->K * h->E * 2 * sizeof(double);
    const size_t nlb = size_t(3) * h->My * h->K * h->E * 2 * sizeof(double);
    if (hipMalloc(&h->vel, velb) != hipSuccess) return fail_free(DNS_E_NOMEM, "hipMalloc vel");
    if (hipMalloc(&h->nl, nlb) != hipSuccess) return fail_free(DNS_E_NOMEM, "hipMalloc nl");
  }
  ALLOC(h->means, 2 * MyE);
  ALLOC(h->psum, size_t(NPS) * MyE);
  // Operators split by y parity (each CN operator commutes with the reflection
  // y -> -y, each D1 anticommutes with it), in MFMA A-operand tile order.
  const int N = h->N, My = h->My;
  const int He = (N + 1) / 2, Ho = N / 2, Fe = He + 1, Fo = Ho + 1;
  auto ntile = [](int r, int k) { return size_t((r + 15) / 16) * ((k + 3) / 4) * 64; };
  const size_t per_e = ntile(He, 2 * He), per_o = ntile(Ho, 2 * Ho);
  h->op_group_stride = 2 * (per_e + per_o);
  auto pair_block = [&](const double* A, const double* B, bool even) { return parity_pair_block(A, B, N, even); };
  // halves of an interior vector: even (He) then odd (Ho)
  auto halves = [&](const std::vector<double>& x) {
    std::vector<double> out(size_t(N), 0.0);
    for (int k = 0; k < He; ++k) out[k] = (k < Ho) ? 0.5 * (x[k] + x[N - 1 - k]) : x[k];
    for (int k = 0; k < Ho; ++k) out[He + k] = 0.5 * (x[k] - x[N - 1 - k]);
    return out;
  };
  std::vector<double> opsT[2], meanT[2], lift_h[2], green_h[2];
  const size_t nn = size_t(N) * N;
  for (int hi = 0; hi < 2; ++hi) {
    opsT[hi] = tile_group_operators(ho, hi, N, h->G, h->op_group_stride);
    meanT[hi] = pair_block(ho.mean_ops[hi].data(), ho.mean_ops[hi].data() + nn, true);
    const std::vector<double> mo = pair_block(ho.mean_ops[hi].data(), ho.mean_ops[hi].data() + nn, false);
    meanT[hi].insert(meanT[hi].end(), mo.begin(), mo.end());
    lift_h[hi] = halves(ho.lift[hi]);
    green_h[hi] = halves(ho.green[hi]);
  }
  // derivative halves: even input -> odd output and odd input -> even output,
  // FP64 tiles, split-BF16 tiles and FP32 tiles (index order of ModeArgs::Dhi)
  std::vector<unsigned short> bhi[6], blo[6];
  std::vector<float> bf32[6];
  int nsplit = 0;
  auto dhalf = [&](const double* M, int rows_out, int Cn, int ldm, bool even_in) {
    const std::vector<double> b = half_block(M, rows_out, Cn, ldm, even_in);
    const int ncol = even_in ? (Cn + 1) / 2 : Cn / 2;
    tile_for_mfma_bf16(b.data(), rows_out, ncol, ncol, &bhi[nsplit], &blo[nsplit]);
    std::vector<double> t = tile_for_mfma(b.data(), rows_out, ncol, ncol);
    bf32[nsplit].assign(t.begin(), t.end());  // the same A lane order, rounded to FP32
    ++nsplit;
    return t;
  };
  const double* D1int = ho.D1.data() + My;  // interior rows of D1
  const std::vector<double> D1intT_e = dhalf(D1int, Ho, My, My, true);
  const std::vector<double> D1intT_o = dhalf(D1int, He, My, My, false);
  const std::vector<double> D1cT_e = dhalf(ho.D1c.data(), Fo, N, N, true);
  const std::vector<double> D1cT_o = dhalf(ho.D1c.data(), Fe, N, N, false);
  const std::vector<double> D1T_e = dhalf(ho.D1.data(), Fo, My, My, true);
  const std::vector<double> D1T_o = dhalf(ho.D1.data(), Fe, My, My, false);
  // Clenshaw-Curtis weights over node pairs (the weights are symmetric)
  std::vector<double> ccw_h(size_t(Fe), 0.0);
  for (int k = 0; k < Fe; ++k) ccw_h[k] = k < Fo ? 2.0 * ho.ccw[k] : ho.ccw[k];
  for (int hi = 0; hi < 2; ++hi) {
    ALLOC(h->opsT[hi], opsT[hi].size());
    ALLOC(h->meanT[hi], meanT[hi].size());
    ALLOC(h->lift_h[hi], lift_h[hi].size());
    ALLOC(h->green_h[hi], green_h[hi].size());
  }
  ALLOC(h->D1intT_e, D1intT_e.size());
  ALLOC(h->D1intT_o, D1intT_o.size());
  ALLOC(h->D1cT_e, D1cT_e.size());
  ALLOC(h->D1cT_o, D1cT_o.size());
  ALLOC(h->D1T_e, D1T_e.size());
  ALLOC(h->D1T_o, D1T_o.size());
  ALLOC(h->ccw_h, ccw_h.size());
  for (int i = 0; i < 6; ++i) {
    ALLOC(h->Dhi[i], bhi[i].size());
    ALLOC(h->Dlo[i], blo[i].size());
    ALLOC(h->Df[i], bf32[i].size());
  }
  ALLOC(h->D1, ho.D1.size());
  ALLOC(h->ccw, ho.ccw.size());
  ALLOC(h->gamma, size_t(h->E));
  ALLOC(h->failed, size_t(h->E));
  ALLOC(h->divmax, size_t(h->E));
  ALLOC(h->acc, size_t(NPA) * MyE + 2 * size_t(h->E));
  ALLOC(h->inst, size_t(NDI) * h->E);
#undef ALLOC
  if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess)
    return fail_free(DNS_E_HIP, "hipStreamCreate");
  h->stream = h->own_stream;
  if (hipGetDevice(&h->device) != hipSuccess) return fail_free(DNS_E_HIP, "hipGetDevice");
  // the allocation-free hand-off needs this device's scratch address and the
  // Chebyshev tables of the channel form, so both exist from creation on
  if (noalloc_scratch_init(h->device) != hipSuccess)
    return fail_free(DNS_E_HIP, "looking up the allocation-free scratch");
  {
    const int rc = ensure_cheb(h);
    if (rc != DNS_OK) return fail_free(rc, h->err);
  }
  // every kernel a step uses is resolved now, so that no captured step holds a
  // kernel's first launch
  if (plane_preload(Nx, Nz) != hipSuccess || mode_preload() != hipSuccess || misc_preload() != hipSuccess)
    return fail_free(DNS_E_HIP, "resolving kernels");
  // one member chain: every launch of a step covers the whole ensemble
  // (DNS_OPT_CHAINS splits it so that chains overlap each other's kernels)
  if (set_chains(h, 1) != DNS_OK) return fail_free(DNS_E_HIP, "creating chain streams");

  auto up = [&](double* dst, const std::vector<double>& src) {
    return hipMemcpy(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice);
  };
  bool ok = true;
  for (int hi = 0; hi < 2; ++hi) {
    ok &= up(h->opsT[hi], opsT[hi]) == hipSuccess;
    ok &= up(h->meanT[hi], meanT[hi]) == hipSuccess;
    ok &= up(h->lift_h[hi], lift_h[hi]) == hipSuccess;
    ok &= up(h->green_h[hi], green_h[hi]) == hipSuccess;
  }
  ok &= up(h->D1intT_e, D1intT_e) == hipSuccess;
  ok &= up(h->D1intT_o, D1intT_o) == hipSuccess;
  ok &= up(h->D1cT_e, D1cT_e) == hipSuccess;
  ok &= up(h->D1cT_o, D1cT_o) == hipSuccess;
  ok &= up(h->D1T_e, D1T_e) == hipSuccess;
  ok &= up(h->D1T_o, D1T_o) == hipSuccess;
  ok &= up(h->ccw_h, ccw_h) == hipSuccess;
  for (int i = 0; i < 6; ++i) {
    ok &= hipMemcpy(h->Dhi[i], bhi[i].data(), bhi[i].size() * 2, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(h->Dlo[i], blo[i].data(), blo[i].size() * 2, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(h->Df[i], bf32[i].data(), bf32[i].size() * sizeof(float), hipMemcpyHostToDevice) ==
          hipSuccess;
  }
  ok &= up(h->D1, ho.D1) == hipSuccess;
  ok &= up(h->ccw, ho.ccw) == hipSuccess;
  // laminar state, zero history
  std::vector<double> Ul(MyE, 0.0);
  for (int j = 0; j < h->My; ++j) {
    const double y = -std::cos(M_PI * j / (h->My - 1));
    const double u = h->flow == DNS_FLOW_COUETTE ? h->Uw * y : 1.0 - y * y;
    for (int e = 0; e < h->E; ++e) Ul[size_t(j) * h->E + e] = u;
  }
  if (h->flow == DNS_FLOW_POISEUILLE) {
    for (int e = 0; e < h->E; ++e) {
      Ul[e] = 0.0;
      Ul[size_t(h->My - 1) * h->E + e] = 0.0;
    }
  }
  ok &= up(h->U, Ul) == hipSuccess;
  ok &= hipMemset(h->v, 0, 2 * KNE * sizeof(double)) == hipSuccess;
  ok &= hipMemset(h->eta, 0, 2 * KNE * sizeof(double)) == hipSuccess;
  ok &= hipMemset(h->W, 0, MyE * sizeof(double)) == hipSuccess;
  ok &= hipMemset(h->hF, 0, 2 * KNE * sizeof(double)) == hipSuccess;
  ok &= hipMemset(h->hG, 0, 2 * KNE * sizeof(double)) == hipSuccess;
  ok &= hipMemset(h->gamma, 0, h->E * sizeof(double)) == hipSuccess;
  ok &= hipMemset(h->failed, 0, h->E * sizeof(int)) == hipSuccess;
  ok &= hipMemset(h->divmax, 0, h->E * sizeof(unsigned long long)) == hipSuccess;
  ok &= hipMemset(h->acc, 0, (size_t(NPA) * MyE + 2 * h->E) * sizeof(double)) == hipSuccess;
  ok &= hipMemset(h->means, 0, 2 * MyE * sizeof(double)) == hipSuccess;
  ok &= hipMemset(h->nl, 0, size_t(3) * h->My * h->K * h->E * 2 * vt_size(DNS_PREC_FP64)) == hipSuccess;
  ok &= hipMemset(h->psum, 0, size_t(NPS) * MyE * sizeof(double)) == hipSuccess;
  if (!ok) return fail_free(DNS_E_HIP, "uploading operators / initial state failed");
  if (hipDeviceSynchronize() != hipSuccess) return fail_free(DNS_E_HIP, "hipDeviceSynchronize");
  *out = h;
  return DNS_OK;
}

int dns_create_grouped(const dns_group* groups, int ngroups, dns_handle** out) {
  if (!out) return fail(nullptr, DNS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!groups || ngroups < 1 || ngroups > DNS_MAX_GROUPS)
    return fail(nullptr, DNS_E_INVALID, "need 1 <= ngroups <= DNS_MAX_GROUPS and a group array");
  dns_handle* h = new dns_handle();
  auto bail = [&](int code, const std::string& msg) {
    free_all(h);
    delete h;
    return fail(nullptr, code, msg);
  };
  int total = 0;
  for (int g = 0; g < ngroups; ++g) {
    const dns_group& q = groups[g];
    dns_handle* sh = nullptr;
    const int rc = dns_create(&q.g, q.Re, q.Nx, q.Ny, q.Nz, q.members, q.dt, &sh);
    if (rc) return bail(rc, "group " + std::to_string(g) + ": " + g_thread_err);
    sh->parent = h;
    h->sub.push_back(sh);
    h->sub_base.push_back(total);
    total += q.members;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
      return bail(DNS_E_HIP, "hipEventCreate");
    h->join.push_back(ev);
  }
  if (hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) != hipSuccess)
    return bail(DNS_E_HIP, "hipEventCreate");
  if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(DNS_E_HIP, "hipStreamCreate");
  h->stream = h->own_stream;
  h->E = total;
  // member chains of the one-launch path (two streams, a fork event each)
  if (set_chains(h, std::min(2, total)) != DNS_OK) return bail(DNS_E_HIP, "creating chain streams");
  for (size_t c = 0; c < h->chain_stream.size(); ++c) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return bail(DNS_E_HIP, "hipEventCreate");
    h->gfork.push_back(ev);
  }
  *out = h;
  return DNS_OK;
}

int dns_group_handle(dns_handle* h, int group, dns_handle** out) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  if (!out) return fail(h, DNS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!h->grouped()) return fail(h, DNS_E_INVALID, "not a grouped handle");
  if (group < 0 || group >= int(h->sub.size())) return fail(h, DNS_E_INVALID, "group out of range");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  *out = h->sub[group];
  return DNS_OK;
}

int dns_set_option(dns_handle* h, int key, long long value) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped() && (key == DNS_OPT_PRECISION || key == DNS_OPT_STATS || key == DNS_OPT_CHAINS ||
                       key == DNS_OPT_ADVECTION || key == DNS_OPT_SHARED_MEAN ||
                       key == DNS_OPT_QUASILINEAR || key == DNS_OPT_FROZEN_MEAN ||
                       key == DNS_OPT_V_DISCRETIZATION)) {
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    for (dns_handle* sh : h->sub) {
      const int rc = dns_set_option(sh, key, value);
      if (rc) return forward(h, sh, rc);
    }
    invalidate_graph(h);
    return DNS_OK;
  }
  switch (key) {
    case DNS_OPT_PRECISION:
      if (value != DNS_PREC_FP64 && value != DNS_PREC_MIXED_FP32 && value != DNS_PREC_MIXED_3XBF16 &&
          value != DNS_PREC_MIXED_FP32MM)
        return fail(h, DNS_E_INVALID, "unknown precision");
      if (!form_fits(h, int(value), plane_form(h)))
        return fail(h, DNS_E_UNSUPPORTED, "no advection-kernel variant of this form fits this grid at that precision");
      if (value != h->precision) {
        h->precision = int(value);
        h->vel_fresh = false;
        invalidate_graph(h);
      }
      return DNS_OK;
    case DNS_OPT_STREAM:
      h->stream = value ? reinterpret_cast<hipStream_t>(value) : h->own_stream;
      invalidate_graph(h);
      return DNS_OK;
    case DNS_OPT_GRAPH:
      // A grouped step captured as one graph (nested forks over the groups' and
      // their member chains' streams) crashed the host process inside dns_step
      // now and then, with no cause found in this library; grouped handles step
      // eagerly.  Each group's handle can still capture its own step.
      if (h->grouped() && value != 0)
        return fail(h, DNS_E_UNSUPPORTED, "graph capture of a grouped step is not supported; it steps eagerly");
      h->use_graph = value != 0;
      invalidate_graph(h);
      return DNS_OK;
    case DNS_OPT_STATS:
      h->stats_on = value != 0;
      invalidate_graph(h);
      return DNS_OK;
    case DNS_OPT_GROUP_STREAMS:
      if (!h->grouped()) return fail(h, DNS_E_INVALID, "DNS_OPT_GROUP_STREAMS applies to grouped handles");
      HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
      h->group_streams = value != 0;
      return DNS_OK;
    case DNS_OPT_PLANE_ROWS: {
      if (h->grouped()) return fail(h, DNS_E_INVALID, "set tile shapes on a group's handle");
      int rows[kMaxPlaneVariants];
      const int n = plane_variants(h->precision, plane_form(h), h->Nx, h->Nz, rows);
      for (int v = 0; v < n; ++v)
        if (rows[v] == value) {
          plane_var(h) = v;
          invalidate_graph(h);
          return DNS_OK;
        }
      return fail(h, DNS_E_UNSUPPORTED, "no plane-kernel variant with that many chunk rows");
    }
    case DNS_OPT_CHAINS:
      if (value < 1 || value > DNS_MAX_CHAINS || value > h->E)
        return fail(h, DNS_E_INVALID, "member chains must be 1..DNS_MAX_CHAINS and at most the ensemble size");
      if (value > 1 && h->shared_mean)
        return fail(h, DNS_E_INVALID, "a shared-mean ensemble advances its members in one chain");
      HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
      return set_chains(h, int(value));
    case DNS_OPT_ADVECTION:
      if (value != DNS_ADV_ADVECTIVE && value != DNS_ADV_ROTATIONAL)
        return fail(h, DNS_E_INVALID, "unknown advection form");
      if (value != DNS_ADV_ADVECTIVE && h->quasilinear)
        return fail(h, DNS_E_INVALID, "the quasi-linear dynamics use the advective form");
      if (!form_fits(h, h->precision, int(value)))
        return fail(h, DNS_E_UNSUPPORTED, "no advection-kernel variant of this form is built for this grid");
      if (value != h->advection) {
        h->advection = int(value);
        invalidate_graph(h);
      }
      return DNS_OK;
    case DNS_OPT_SHARED_MEAN: {
      if (value != 0 && value != 1) return fail(h, DNS_E_INVALID, "shared mean is 0 or 1");
      HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
      if (value && h->nchain > 1) {
        const int rc = set_chains(h, 1);
        if (rc) return rc;
      }
      h->shared_mean = value != 0;
      if (h->shared_mean) {
        HIP_OR_FAIL(h, launch_share_columns(h->v, h->eta, h->U, h->W, h->E, h->N, h->NZ, h->My, h->stream));
        if (h->fv)
          HIP_OR_FAIL(h, launch_share_columns(h->fv, h->feta, nullptr, nullptr, h->E, h->N, h->NZ, h->My,
                                              h->stream));
        HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
        h->vel_fresh = false;
      }
      invalidate_graph(h);
      return DNS_OK;
    }
    case DNS_OPT_QUASILINEAR:
      if (value < 0 || value > 2) return fail(h, DNS_E_INVALID, "quasi-linear is 0, 1 or 2 (adjoint)");
      if (value && h->advection != DNS_ADV_ADVECTIVE)
        return fail(h, DNS_E_INVALID, "the quasi-linear dynamics use the advective form");
      if (!form_fits(h, h->precision, value ? 1 + int(value) : h->advection))
        return fail(h, DNS_E_UNSUPPORTED, "no quasi-linear advection-kernel variant fits this grid at this precision");
      h->quasilinear = int(value);
      invalidate_graph(h);
      return DNS_OK;
    case DNS_OPT_V_DISCRETIZATION: {
      if (value != DNS_VDISC_CLAMPED && value != DNS_VDISC_KMM)
        return fail(h, DNS_E_INVALID, "unknown v discretization");
      if (value == h->v_discretization) return DNS_OK;
      HostOperators ho;
      if (build_operators(h->My, h->L, h->P, h->kxs, h->kzs, h->Re, h->dt, h->Ubot, h->Utop, &ho,
                          int(value)) != 0)
        return fail(h, DNS_E_INVALID, "a Crank-Nicolson operator is singular");
      HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
      for (int hi = 0; hi < 2; ++hi) {
        const std::vector<double> t = tile_group_operators(ho, hi, h->N, h->G, h->op_group_stride);
        HIP_OR_FAIL(h, hipMemcpy(h->opsT[hi], t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
      }
      h->max_cond = ho.max_cond;
      h->v_discretization = int(value);
      invalidate_graph(h);
      return DNS_OK;
    }
    case DNS_OPT_FROZEN_MEAN:
      if (value != 0 && value != 1) return fail(h, DNS_E_INVALID, "frozen mean is 0 or 1");
      h->frozen_mean = value != 0;
      invalidate_graph(h);
      return DNS_OK;
    case DNS_OPT_MODE_TILE:
      if (h->grouped()) return fail(h, DNS_E_INVALID, "set tile shapes on a group's handle");
      if (!mode_tile_ok(h, int(value)))
        return fail(h, DNS_E_INVALID, "mode tile must be 1, 2, 4 or 8 members and fit in LDS");
      set_mode_tile(h, int(value));
      invalidate_graph(h);
      return DNS_OK;
  }
  return fail(h, DNS_E_INVALID, "unknown option key");
}

int dns_set_state(dns_handle* h, int member0, int count, const dns_state_view* s) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) {
    dns_handle* sh;
    int m0;
    const int rc = route(h, member0, count, &sh, &m0);
    return rc ? rc : forward(h, sh, dns_set_state(sh, m0, count, s));
  }
  if (!s || !s->v_hat || !s->eta_hat || !s->U00 || !s->W00)
    return fail(h, DNS_E_INVALID, "state view has NULL buffers");
  if (member0 < 0 || count < 1 || member0 + count > h->E)
    return fail(h, DNS_E_INVALID, "member range out of bounds");
  const size_t nspec = size_t(count) * h->K * h->N * 2;
  const size_t nprof = size_t(count) * h->My;
  // validate on the host: profiles and the n_x = 0 columns (copied back from
  // device views first; the other modes carry no requirement)
  std::vector<double> U(nprof), W(nprof);
  if (s->on_device) {
    const size_t col = size_t(h->NZ) * h->N * 2, per = size_t(h->K) * h->N * 2;
    std::vector<double> vc(count * col), ec(count * col);
    HIP_OR_FAIL(h, hipMemcpy(U.data(), s->U00, nprof * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(h, hipMemcpy(W.data(), s->W00, nprof * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(h, hipMemcpy2D(vc.data(), col * sizeof(double), s->v_hat, per * sizeof(double),
                               col * sizeof(double), count, hipMemcpyDeviceToHost));
    HIP_OR_FAIL(h, hipMemcpy2D(ec.data(), col * sizeof(double), s->eta_hat, per * sizeof(double),
                               col * sizeof(double), count, hipMemcpyDeviceToHost));
    const dns_state_view hv{vc.data(), ec.data(), U.data(), W.data(), 0};
    const int rc = check_host_state(h, 1, h->NZ, h->N, h->My, h->Ubot, h->Utop, count, &hv);
    if (rc) return rc;
  } else {
    std::memcpy(U.data(), s->U00, nprof * sizeof(double));
    std::memcpy(W.data(), s->W00, nprof * sizeof(double));
    const int rc = check_host_state(h, h->L, h->NZ, h->N, h->My, h->Ubot, h->Utop, count, s);
    if (rc) return rc;
  }
  int rc = ensure_staging(h, 2 * nspec * sizeof(double));
  if (rc) return rc;
  const hipMemcpyKind kind = s->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  double* st = h->staging;
  HIP_OR_FAIL(h, hipMemcpyAsync(st, s->v_hat, nspec * sizeof(double), kind, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(st + nspec, s->eta_hat, nspec * sizeof(double), kind, h->stream));
  HIP_OR_FAIL(h, launch_state_to_device(st, h->v, member0, count, h->E, h->K, h->N, h->stream));
  HIP_OR_FAIL(h, launch_state_to_device(st + nspec, h->eta, member0, count, h->E, h->K, h->N, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(st, U.data(), nprof * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(st + nprof, W.data(), nprof * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, launch_profile_to_device(st, h->U, member0, count, h->E, h->My, h->stream));
  HIP_OR_FAIL(h, launch_profile_to_device(st + nprof, h->W, member0, count, h->E, h->My, h->stream));
  HIP_OR_FAIL(h, hipMemsetAsync(h->failed + member0, 0, sizeof(int) * count, h->stream));
  if (h->shared_mean)
    HIP_OR_FAIL(h, launch_share_columns(h->v, h->eta, h->U, h->W, h->E, h->N, h->NZ, h->My, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  h->vel_fresh = false;
  return DNS_OK;
}

int dns_set_forcing(dns_handle* h, int member0, int count, const double* f_lapv, const double* f_eta,
                    int on_device) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) {
    dns_handle* sh;
    int m0;
    const int rc = route(h, member0, count, &sh, &m0);
    return rc ? rc : forward(h, sh, dns_set_forcing(sh, m0, count, f_lapv, f_eta, on_device));
  }
  if (!f_lapv && !f_eta) {
    if (h->forcing_on) {
      HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
      h->forcing_on = false;
      invalidate_graph(h);
    }
    return DNS_OK;
  }
  if (member0 < 0 || count < 1 || member0 + count > h->E)
    return fail(h, DNS_E_INVALID, "member range out of bounds");
  const size_t full = size_t(h->E) * h->K * h->N * 2 * sizeof(double);
  // the stream may still run a step that reads the forcing or the staging buffer
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  if (!h->fv) {
    HIP_OR_FAIL(h, hipMalloc(reinterpret_cast<void**>(&h->fv), full));
    HIP_OR_FAIL(h, hipMalloc(reinterpret_cast<void**>(&h->feta), full));
    HIP_OR_FAIL(h, hipMemsetAsync(h->fv, 0, full, h->stream));
    HIP_OR_FAIL(h, hipMemsetAsync(h->feta, 0, full, h->stream));
  }
  const size_t nspec = size_t(count) * h->K * h->N * 2;
  const int rc = ensure_staging(h, 2 * nspec * sizeof(double));
  if (rc) return rc;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  double* st = h->staging;
  if (f_lapv) HIP_OR_FAIL(h, hipMemcpyAsync(st, f_lapv, nspec * sizeof(double), kind, h->stream));
  else HIP_OR_FAIL(h, hipMemsetAsync(st, 0, nspec * sizeof(double), h->stream));
  if (f_eta) HIP_OR_FAIL(h, hipMemcpyAsync(st + nspec, f_eta, nspec * sizeof(double), kind, h->stream));
  else HIP_OR_FAIL(h, hipMemsetAsync(st + nspec, 0, nspec * sizeof(double), h->stream));
  HIP_OR_FAIL(h, launch_state_to_device(st, h->fv, member0, count, h->E, h->K, h->N, h->stream));
  HIP_OR_FAIL(h, launch_state_to_device(st + nspec, h->feta, member0, count, h->E, h->K, h->N, h->stream));
  if (h->shared_mean)
    HIP_OR_FAIL(h, launch_share_columns(h->fv, h->feta, nullptr, nullptr, h->E, h->N, h->NZ, h->My, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  if (!h->forcing_on) {
    h->forcing_on = true;
    invalidate_graph(h);
  }
  return DNS_OK;
}

}  // extern "C"

namespace {

// Perturbation part (n_x >= 1 modes) of the members' states on the host, with
// dv/dy = D1c v at every node, for energy inner products:
//   <a, b> = (1/Ly) int dy sum_k m_k Re(u_a . conj u_b),
//   |u|^2 + |w|^2 = (|dv/dy|^2 + |eta|^2) / k^2 per mode, m_k = 2 (n_x >= 1),
// so that the kinetic energy density is E = <a, a> / 2.
struct Perturbations {
  int E = 0, K0 = 0, K = 0, N = 0, My = 0, L = 0, NZ = 0;
  std::vector<double> v, eta, dv;  // device layout [K][N][E] (dv: [K][My][E]) complex
  std::vector<double> k2;          // per mode
  std::vector<unsigned char> col;  // [E][L]: member has content in streamwise column n_x
};

int load_perturbations(dns_handle* h, Perturbations* P) {
  P->E = h->E;
  P->K0 = h->NZ;  // first mode with n_x = 1
  P->K = h->K;
  P->N = h->N;
  P->My = h->My;
  const size_t n = size_t(h->K) * h->N * h->E * 2;
  P->v.resize(n);
  P->eta.resize(n);
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  HIP_OR_FAIL(h, hipMemcpy(P->v.data(), h->v, n * sizeof(double), hipMemcpyDeviceToHost));
  HIP_OR_FAIL(h, hipMemcpy(P->eta.data(), h->eta, n * sizeof(double), hipMemcpyDeviceToHost));
  P->k2.assign(h->K, 1.0);
  for (int m = 0; m < h->K; ++m) {
    const int nx = m / h->NZ, iz = m - nx * h->NZ;
    const int nz = iz < h->P ? iz : iz - h->NZ;
    const double kx = h->kxs * nx, kz = h->kzs * nz;
    if (nx > 0 || nz != 0) P->k2[m] = kx * kx + kz * kz;
  }
  P->dv.assign(size_t(h->K) * h->My * h->E * 2, 0.0);
  const int E = h->E, N = h->N, My = h->My;
  P->L = h->L;
  P->NZ = h->NZ;
  P->col.assign(size_t(E) * h->L, 0);
  for (int m = P->K0; m < h->K; ++m)
    for (int j = 0; j < N; ++j)
      for (int e = 0; e < E; ++e) {
        const size_t o = ((size_t(m) * N + j) * E + e) * 2;
        if (P->v[o] != 0.0 || P->v[o + 1] != 0.0 || P->eta[o] != 0.0 || P->eta[o + 1] != 0.0)
          P->col[size_t(e) * h->L + m / h->NZ] = 1;
      }
  for (int m = P->K0; m < h->K; ++m)
    for (int i = 0; i < My; ++i) {
      double* d = &P->dv[(size_t(m) * My + i) * E * 2];
      for (int j = 0; j < N; ++j) {
        const double c = h->host_D1c[size_t(i) * N + j];
        if (c == 0.0) continue;
        const double* vv = &P->v[(size_t(m) * N + j) * E * 2];
        for (int e = 0; e < 2 * E; ++e) d[e] += c * vv[e];
      }
    }
  return DNS_OK;
}

double pert_inner(const dns_handle* h, const Perturbations& P, int a, int b) {
  const int E = P.E, N = P.N, My = P.My;
  const std::vector<double>& w = h->host_ccw;
  double tot = 0.0;
  for (int m = P.K0; m < P.K; ++m) {
    const int nx = m / P.NZ;
    if (!P.col[size_t(a) * P.L + nx] || !P.col[size_t(b) * P.L + nx]) continue;  // disjoint supports
    double sv = 0.0, se = 0.0, sd = 0.0;
    for (int j = 0; j < N; ++j) {
      const size_t o = (size_t(m) * N + j) * E * 2;
      sv += w[j + 1] * (P.v[o + 2 * a] * P.v[o + 2 * b] + P.v[o + 2 * a + 1] * P.v[o + 2 * b + 1]);
      se += w[j + 1] * (P.eta[o + 2 * a] * P.eta[o + 2 * b] + P.eta[o + 2 * a + 1] * P.eta[o + 2 * b + 1]);
    }
    for (int i = 0; i < My; ++i) {
      const size_t o = (size_t(m) * My + i) * E * 2;
      sd += w[i] * (P.dv[o + 2 * a] * P.dv[o + 2 * b] + P.dv[o + 2 * a + 1] * P.dv[o + 2 * b + 1]);
    }
    tot += 2.0 * (sv + (sd + se) / P.k2[m]);
  }
  return tot / 2.0;  // 1 / Ly
}

// x_a -= c x_b (perturbation modes, v, eta and dv)
void pert_axpy(Perturbations* P, int a, int b, double c) {
  const int E = P->E;
  auto upd = [&](std::vector<double>& x, size_t rows) {
    for (size_t r = size_t(P->K0) * rows; r < size_t(P->K) * rows; ++r) {
      double* row = &x[r * E * 2];
      row[2 * a] -= c * row[2 * b];
      row[2 * a + 1] -= c * row[2 * b + 1];
    }
  };
  upd(P->v, P->N);
  upd(P->eta, P->N);
  upd(P->dv, P->My);
  for (int nx = 0; nx < P->L; ++nx) P->col[size_t(a) * P->L + nx] |= P->col[size_t(b) * P->L + nx];
}

void pert_scale(Perturbations* P, int a, double c) {
  const int E = P->E;
  auto upd = [&](std::vector<double>& x, size_t rows) {
    for (size_t r = size_t(P->K0) * rows; r < size_t(P->K) * rows; ++r) {
      x[r * E * 2 + 2 * a] *= c;
      x[r * E * 2 + 2 * a + 1] *= c;
    }
  };
  upd(P->v, P->N);
  upd(P->eta, P->N);
  upd(P->dv, P->My);
}

}  // namespace

extern "C" {

int dns_perturbation_energy(dns_handle* h, double* out) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) return fail(h, DNS_E_INVALID, "call on a group's handle");
  if (!out) return fail(h, DNS_E_INVALID, "output is NULL");
  Perturbations P;
  const int rc = load_perturbations(h, &P);
  if (rc) return rc;
  for (int e = 0; e < h->E; ++e) out[e] = 0.5 * pert_inner(h, P, e, e);
  return DNS_OK;
}

int dns_orthonormalize(dns_handle* h) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) return fail(h, DNS_E_INVALID, "call on a group's handle");
  Perturbations P;
  int rc = load_perturbations(h, &P);
  if (rc) return rc;
  for (int i = 0; i < h->E; ++i) {
    for (int j = 0; j < i; ++j) {
      const double c = 0.5 * pert_inner(h, P, i, j);  // <x_j, x_j> = 2
      if (c != 0.0) pert_axpy(&P, i, j, c);
    }
    const double e = 0.5 * pert_inner(h, P, i, i);
    if (!(e > 0.0) || !std::isfinite(e))
      return fail(h, DNS_E_INVALID, "member " + std::to_string(i) + " has no independent perturbation");
    pert_scale(&P, i, 1.0 / std::sqrt(e));
  }
  const size_t n = P.v.size();
  HIP_OR_FAIL(h, hipMemcpy(h->v, P.v.data(), n * sizeof(double), hipMemcpyHostToDevice));
  HIP_OR_FAIL(h, hipMemcpy(h->eta, P.eta.data(), n * sizeof(double), hipMemcpyHostToDevice));
  h->vel_fresh = false;
  return DNS_OK;
}

int dns_get_state(dns_handle* h, int member0, int count, dns_state_view* s) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) {
    dns_handle* sh;
    int m0;
    const int rc = route(h, member0, count, &sh, &m0);
    return rc ? rc : forward(h, sh, dns_get_state(sh, m0, count, s));
  }
  if (!s || !s->v_hat || !s->eta_hat || !s->U00 || !s->W00)
    return fail(h, DNS_E_INVALID, "state view has NULL buffers");
  if (member0 < 0 || count < 1 || member0 + count > h->E)
    return fail(h, DNS_E_INVALID, "member range out of bounds");
  const size_t nspec = size_t(count) * h->K * h->N * 2;
  const size_t nprof = size_t(count) * h->My;
  int rc = ensure_staging(h, (2 * nspec + 2 * nprof) * sizeof(double));
  if (rc) return rc;
  double* st = h->staging;
  HIP_OR_FAIL(h, launch_state_from_device(h->v, st, member0, count, h->E, h->K, h->N, h->stream));
  HIP_OR_FAIL(h, launch_state_from_device(h->eta, st + nspec, member0, count, h->E, h->K, h->N, h->stream));
  HIP_OR_FAIL(h, launch_profile_from_device(h->U, st + 2 * nspec, member0, count, h->E, h->My, h->stream));
  HIP_OR_FAIL(h, launch_profile_from_device(h->W, st + 2 * nspec + nprof, member0, count, h->E, h->My, h->stream));
  const hipMemcpyKind kind = s->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIP_OR_FAIL(h, hipMemcpyAsync(s->v_hat, st, nspec * sizeof(double), kind, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(s->eta_hat, st + nspec, nspec * sizeof(double), kind, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(s->U00, st + 2 * nspec, nprof * sizeof(double), kind, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(s->W00, st + 2 * nspec + nprof, nprof * sizeof(double), kind, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  return DNS_OK;
}

int dns_step(dns_handle* h, int nsteps) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (nsteps < 0) return fail(h, DNS_E_INVALID, "nsteps must be >= 0");
  if (nsteps == 0) return DNS_OK;
  if (h->grouped()) {
    for (size_t g = 0; g < h->sub.size(); ++g) {
      HIP_OR_FAIL(h, hipEventRecord(h->join[g], h->sub[g]->stream));
      HIP_OR_FAIL(h, hipStreamWaitEvent(h->stream, h->join[g], 0));
    }
    bool stale = false;
    for (dns_handle* sh : h->sub) stale |= !sh->vel_fresh;
    if (stale) {
      HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
      for (dns_handle* sh : h->sub) {
        if (sh->vel_fresh) continue;
        const int rc = refresh_velocities(sh);
        if (rc) return forward(h, sh, rc);
        HIP_OR_FAIL(h, hipStreamSynchronize(sh->stream));
      }
    }
  } else if (!h->vel_fresh) {
    int rc = refresh_velocities(h);
    if (rc) return rc;
  }
  if (h->grouped() && grouped_one_launch(h)) {
    const int rc = update_group_descs(h);
    if (rc) return rc;
  }
  if (h->use_graph) {
    if (!h->graph_valid) {
      int rc = build_graph(h);
      if (rc) return rc;
    }
    for (int n = 0; n < nsteps; ++n) HIP_OR_FAIL(h, hipGraphLaunch(h->gexec, h->stream));
  } else {
    for (int n = 0; n < nsteps; ++n) {
      int rc = enqueue_any(h);
      if (rc) return rc;
    }
  }
  h->steps += nsteps;
  if (h->stats_on) h->samples += nsteps;
  for (dns_handle* sh : h->sub) {
    sh->steps += nsteps;
    if (sh->stats_on) sh->samples += nsteps;
  }
  return DNS_OK;
}

int dns_sync(dns_handle* h) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  if (h->grouped()) {
    int out = DNS_OK;
    for (dns_handle* sh : h->sub) {
      const int rc = dns_sync(sh);
      if (rc == DNS_E_NONFINITE) out = rc;
      else if (rc) return forward(h, sh, rc);
    }
    return out ? fail(h, out, "a member produced a non-finite value") : DNS_OK;
  }
  const int any = any_failed(h, nullptr);
  if (any < 0) return fail(h, DNS_E_HIP, "reading failure flags");
  if (any) return fail(h, DNS_E_NONFINITE, "a member produced a non-finite value");
  return DNS_OK;
}

int dns_stats(dns_handle* h, dns_stats_out* o) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (!o) return fail(h, DNS_E_INVALID, "output is NULL");
  if (h->grouped()) {
    if (o->U || o->W || o->urms || o->vrms || o->wrms || o->uv || o->member_profiles)
      return fail(h, DNS_E_INVALID,
                  "profiles of a grouped handle differ per group: read them from dns_group_handle");
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    int out = DNS_OK;
    for (size_t g = 0; g < h->sub.size(); ++g) {
      const int b = h->sub_base[g];
      auto at = [b](double* p) { return p ? p + b : nullptr; };
      dns_stats_out so{};
      so.energy = at(o->energy);
      so.dissipation = at(o->dissipation);
      so.power = at(o->power);
      so.flux = at(o->flux);
      so.gamma = at(o->gamma);
      so.div_max = at(o->div_max);
      so.tau_lower = at(o->tau_lower);
      so.tau_upper = at(o->tau_upper);
      so.failed = o->failed ? o->failed + b : nullptr;
      so.member_tau = o->member_tau ? o->member_tau + 2 * size_t(b) : nullptr;
      const int rc = dns_stats(h->sub[g], &so);
      if (rc == DNS_E_NONFINITE) out = rc;
      else if (rc) return forward(h, h->sub[g], rc);
    }
    o->tau_w = 0.0;
    o->re_tau = 0.0;
    o->samples = h->sub[0]->samples;
    o->steps = h->steps;
    return out ? fail(h, out, "a member produced a non-finite value") : DNS_OK;
  }
  // fresh diagnostics of the current state
  HIP_OR_FAIL(h, hipMemsetAsync(h->divmax, 0, sizeof(unsigned long long) * h->E, h->stream));
  int rc = refresh_velocities(h);
  if (rc) return rc;
  HIP_OR_FAIL(h, plane_launch(h, true));
  HIP_OR_FAIL(h, launch_stats(stats_args(h), 0, h->stream));
  const int E = h->E, My = h->My;
  std::vector<double> inst(size_t(NDI) * E), gam(E), acc(size_t(NPA) * My * E + 2 * E);
  std::vector<unsigned long long> dm(E);
  std::vector<int> fl(E);
  HIP_OR_FAIL(h, hipMemcpyAsync(inst.data(), h->inst, inst.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(gam.data(), h->gamma, gam.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(acc.data(), h->acc, acc.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(dm.data(), h->divmax, dm.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(fl.data(), h->failed, fl.size() * 4, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  int anyf = 0;
  for (int e = 0; e < E; ++e) {
    if (o->energy) o->energy[e] = inst[DI_E * E + e];
    if (o->dissipation) o->dissipation[e] = inst[DI_EPS * E + e];
    if (o->power) o->power[e] = inst[DI_PI * E + e];
    if (o->flux) o->flux[e] = inst[DI_Q * E + e];
    if (o->tau_lower) o->tau_lower[e] = inst[DI_TLO * E + e];
    if (o->tau_upper) o->tau_upper[e] = inst[DI_THI * E + e];
    if (o->gamma) o->gamma[e] = gam[e];
    if (o->div_max) {
      double d;
      std::memcpy(&d, &dm[e], sizeof(double));
      o->div_max[e] = d;
    }
    if (o->failed) o->failed[e] = fl[e];
    anyf |= fl[e];
  }
  o->samples = h->samples;
  o->steps = h->steps;
  // per-member time averages (zero before the first sample)
  const double inv_t = h->samples > 0 ? 1.0 / double(h->samples) : 0.0;
  if (o->member_profiles)
    for (int e = 0; e < E; ++e)
      for (int q = 0; q < NPA; ++q)
        for (int j = 0; j < My; ++j)
          o->member_profiles[(size_t(e) * NPA + q) * My + j] = acc[(size_t(q) * My + j) * E + e] * inv_t;
  if (o->member_tau)
    for (int e = 0; e < E; ++e)
      for (int side = 0; side < 2; ++side)
        o->member_tau[2 * size_t(e) + side] = acc[size_t(NPA) * My * E + size_t(side) * E + e] * inv_t / h->Re;
  if (h->samples > 0) {
    const double inv = 1.0 / (double(h->samples) * E);
    for (int j = 0; j < My; ++j) {
      double s[NPA] = {0};
      for (int q = 0; q < NPA; ++q)
        for (int e = 0; e < E; ++e) s[q] += acc[(size_t(q) * My + j) * E + e];
      for (int q = 0; q < NPA; ++q) s[q] *= inv;
      const double U = s[PA_U], W = s[PA_W];
      if (o->U) o->U[j] = U;
      if (o->W) o->W[j] = W;
      if (o->urms) o->urms[j] = std::sqrt(std::fmax(s[PA_UU] - U * U, 0.0));
      if (o->vrms) o->vrms[j] = std::sqrt(std::fmax(s[PA_VV], 0.0));
      if (o->wrms) o->wrms[j] = std::sqrt(std::fmax(s[PA_WW] - W * W, 0.0));
      if (o->uv) o->uv[j] = s[PA_UV];
    }
    double lo = 0, hi = 0;
    for (int e = 0; e < E; ++e) {
      lo += acc[size_t(NPA) * My * E + e];
      hi += acc[size_t(NPA) * My * E + E + e];
    }
    lo *= inv;
    hi *= inv;
    o->tau_w = h->flow == DNS_FLOW_COUETTE ? 0.5 * (std::fabs(lo) + std::fabs(hi)) / h->Re
                                           : (lo - hi) / (2.0 * h->Re);
    o->re_tau = h->Re * std::sqrt(std::fabs(o->tau_w));
  } else {
    o->tau_w = 0.0;
    o->re_tau = 0.0;
  }
  if (anyf) return fail(h, DNS_E_NONFINITE, "a member produced a non-finite value");
  return DNS_OK;
}

int dns_stats_reset(dns_handle* h) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) {
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    for (dns_handle* sh : h->sub) {
      const int rc = dns_stats_reset(sh);
      if (rc) return forward(h, sh, rc);
    }
    h->samples = 0;
    return DNS_OK;
  }
  HIP_OR_FAIL(h, hipMemsetAsync(h->acc, 0, (size_t(NPA) * h->My * h->E + 2 * h->E) * sizeof(double), h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  h->samples = 0;
  return DNS_OK;
}

void dns_destroy(dns_handle* h) {
  if (!h || h->parent) return;  // a group's handle belongs to its grouped handle
  destroy_one(h);
}

const char* dns_last_error(const dns_handle* h) {
  return h ? h->err.c_str() : g_thread_err.c_str();
}

// For every row length NZ = 2P - 1 the library builds: the kz in (-P, P) fill
// the stage slots [0, NZ) once each, stage_kz inverts stage_slot, and +kz and
// -kz sit in neighbouring slots (the per-mode kernel's paired accesses).
constexpr bool stage_order_ok() {
  for (int P = 1; P <= 256; ++P) {
    const int NZ = 2 * P - 1;
    for (int nz = 1 - P; nz < P; ++nz) {
      const int s = stage_slot(nz);
      if (s < 0 || s >= NZ || stage_kz(s) != nz) return false;
      if (nz > 0 && stage_slot(-nz) != s + 1) return false;
    }
  }
  return true;
}
static_assert(stage_order_ok(), "stage slot order");
// stage_off maps (row, member, mode) of small buffers onto [0, rows E K) once
// each, and a member's modes lie 1 << stage_block_log2(E) elements apart.
constexpr bool stage_off_ok() {
  for (int E = 1; E <= 9; ++E)
    for (int K = 1; K <= 7; ++K) {
      bool seen[2 * 9 * 7] = {};
      const int lb = stage_block_log2(E);
      for (int r = 0; r < 2; ++r)
        for (int e = 0; e < E; ++e)
          for (int k = 0; k < K; ++k) {
            const size_t o = stage_off(r, e, k, E, K, lb);
            if (o >= size_t(2 * E * K) || seen[o]) return false;
            seen[o] = true;
            if (k + 1 < K && stage_off(r, e, k + 1, E, K, lb) != o + (size_t(1) << lb)) return false;
          }
    }
  return true;
}
static_assert(stage_off_ok(), "stage member blocks");

int dns_debug_stage0(dns_handle* h, double* vel, double* nl, double* means) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) return fail(h, DNS_E_INVALID, "call this on a group's handle (dns_group_handle)");
  int rc = refresh_velocities(h);
  if (rc) return rc;
  HIP_OR_FAIL(h, plane_launch(h, false));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  const int E = h->E, My = h->My, K = h->K;
  const size_t vt = vt_size(h->precision);
  auto fetch = [&](const void* src, int nf, double* dst) -> int {
    const size_t n = size_t(nf) * My * K * E * 2;
    std::vector<unsigned char> raw(n * vt);
    if (hipMemcpy(raw.data(), src, raw.size(), hipMemcpyDeviceToHost) != hipSuccess) return -1;
    for (int f = 0; f < nf; ++f)
      for (int e = 0; e < E; ++e)
        for (int j = 0; j < My; ++j)
          for (int m = 0; m < K; ++m) {
            const int nx = m / h->NZ, iz = m - nx * h->NZ;
            const int slot = stage_slot(iz < h->P ? iz : iz - h->NZ);
            const size_t d = stage_off(size_t(f) * My + j, e, nx * h->NZ + slot, E, K, stage_block_log2(E)) * 2;
            const size_t o = (((size_t(f) * E + e) * My + j) * K + m) * 2;
            for (int c = 0; c < 2; ++c)
              dst[o + c] = vt == 8 ? reinterpret_cast<const double*>(raw.data())[d + c]
                                   : double(reinterpret_cast<const float*>(raw.data())[d + c]);
          }
    return 0;
  };
  if (vel && fetch(h->vel, 5, vel)) return fail(h, DNS_E_HIP, "copying velocity fields");
  if (nl && fetch(h->nl, 3, nl)) return fail(h, DNS_E_HIP, "copying advection fields");
  if (means) {
    std::vector<double> mm(size_t(2) * My * E);
    HIP_OR_FAIL(h, hipMemcpy(mm.data(), h->means, mm.size() * 8, hipMemcpyDeviceToHost));
    for (int q = 0; q < 2; ++q)
      for (int e = 0; e < E; ++e)
        for (int j = 0; j < My; ++j) means[(size_t(q) * E + e) * My + j] = mm[(size_t(q) * My + j) * E + e];
  }
  return DNS_OK;
}

}  // extern "C"

namespace {

// Average device time of nreps launches (after one untimed launch), HIP events.
template <class Launch>
int time_launches(dns_handle* h, int nreps, Launch launch, double* ms) {
  hipEvent_t e0, e1;
  HIP_OR_FAIL(h, hipEventCreate(&e0));
  HIP_OR_FAIL(h, hipEventCreate(&e1));
  hipError_t err = launch();
  if (err == hipSuccess) err = hipEventRecord(e0, h->stream);
  for (int r = 0; r < nreps && err == hipSuccess; ++r) err = launch();
  if (err == hipSuccess) err = hipEventRecord(e1, h->stream);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (err != hipSuccess) return fail(h, DNS_E_HIP, std::string("timing launches: ") + hipGetErrorString(err));
  *ms = double(t) / nreps;
  return DNS_OK;
}

std::string tune_key(const dns_handle* h) {
  return std::to_string(h->precision) + " " + std::to_string(h->Nx) + " " + std::to_string(h->Ny) + " " +
         std::to_string(h->Nz) + " " + std::to_string(h->E);
}

// Last cache line "<precision> <Nx> <Ny> <Nz> <E> <plane_rows> <mode_members> <plane_ms> <mode_ms>
// [<advection form>]" whose key matches h (a line without the form is the advective form's).
bool cache_lookup(const dns_handle* h, const char* path, dns_tuning* t) {
  if (!path) return false;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  int p, nx, ny, nz, e, rows, mem, form;
  double pm, mm;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    form = DNS_ADV_ADVECTIVE;
    const int got = std::sscanf(line, "%d %d %d %d %d %d %d %lf %lf %d", &p, &nx, &ny, &nz, &e, &rows, &mem,
                                &pm, &mm, &form);
    if (got != 9 && got != 10) continue;
    if (p == h->precision && nx == h->Nx && ny == h->Ny && nz == h->Nz && e == h->E && form == plane_form(h)) {
      t->plane_rows = rows;
      t->mode_members = mem;
      t->plane_ms = pm;
      t->mode_ms = mm;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

int tune_one(dns_handle* h, const char* cache, dns_tuning* out) {
  dns_tuning t{};
  if (cache_lookup(h, cache, &t)) {
    int rc = dns_set_option(h, DNS_OPT_PLANE_ROWS, t.plane_rows);
    if (rc == DNS_OK) rc = dns_set_option(h, DNS_OPT_MODE_TILE, t.mode_members);
    if (rc != DNS_OK) return fail(h, rc, "tune cache entry does not apply: " + h->err);
    t.from_cache = 1;
    if (out) *out = t;
    return DNS_OK;
  }
  constexpr int kReps = 5;
  if (!h->vel_fresh) {
    const int rc = refresh_velocities(h);
    if (rc) return rc;
  }
  int rows[kMaxPlaneVariants];
  const int nv = plane_variants(h->precision, plane_form(h), h->Nx, h->Nz, rows);
  int best_v = 0;
  double best_p = 1e30;
  for (int v = 0; v < nv; ++v) {
    plane_var(h) = v;
    double ms;
    const int rc = time_launches(h, kReps, [&] { return plane_launch(h, false, 0, -1, nullptr, false); }, &ms);
    if (rc) return rc;
    if (ms < best_p) best_p = ms, best_v = v;
  }
  plane_var(h) = best_v;
  // the mode kernel's second sub-step on the current stage buffers (the next
  // step rewrites its history first)
  // the current tile is timed first and another replaces it only when faster
  // by more than kTileMargin: member tiles often tie within timing noise, and
  // a choice that flips between runs would change what a run measures
  constexpr double kTileMargin = 0.02;
  const int et0 = h->ET;
  int best_et = et0;
  double best_m = 1e30;
  for (int i = 0; i <= 4; ++i) {
    const int et = i == 0 ? et0 : 1 << (i - 1);
    if ((i > 0 && et == et0) || !mode_tile_ok(h, et)) continue;
    set_mode_tile(h, et);
    double ms;
    const int rc = time_launches(h, kReps, [&] { return launch_mode(h->precision, mode_args(h, 1), h->stream); }, &ms);
    if (rc) return rc;
    if (i == 0 || ms < (1.0 - kTileMargin) * best_m) best_m = ms, best_et = et;
  }
  set_mode_tile(h, best_et);
  h->vel_fresh = false;
  invalidate_graph(h);
  t.plane_rows = rows[best_v];
  t.mode_members = best_et;
  t.plane_ms = best_p;
  t.mode_ms = best_m;
  t.from_cache = 0;
  if (cache) {
    std::FILE* f = std::fopen(cache, "a");
    if (!f) return fail(h, DNS_E_INVALID, std::string("cannot append to tune cache ") + cache);
    std::fprintf(f, "%s %d %d %.6f %.6f %d\n", tune_key(h).c_str(), t.plane_rows, t.mode_members, t.plane_ms,
                 t.mode_ms, plane_form(h));
    std::fclose(f);
  }
  if (out) *out = t;
  return DNS_OK;
}

}  // namespace

extern "C" {

int dns_tune(dns_handle* h, const char* cache_path, dns_tuning* out) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) {
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    for (size_t g = 0; g < h->sub.size(); ++g) {
      const int rc = tune_one(h->sub[g], cache_path, out ? out + g : nullptr);
      if (rc) return fail(h, rc, "group " + std::to_string(g) + ": " + h->sub[g]->err);
    }
    invalidate_graph(h);
    return DNS_OK;
  }
  return tune_one(h, cache_path, out);
}


int dns_get_channels(dns_handle* h, int member0, int count, float* out) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) {
    dns_handle* sh;
    int m0;
    const int rc = route(h, member0, count, &sh, &m0);
    return rc ? rc : forward(h, sh, dns_get_channels(sh, m0, count, out));
  }
  if (!out) return fail(h, DNS_E_INVALID, "out is NULL");
  if (member0 < 0 || count < 1 || member0 + count > h->E) return fail(h, DNS_E_INVALID, "member range out of bounds");
  int rc = ensure_cheb(h);
  if (rc) return rc;
  const int Mx = 3 * h->Nx / 2, Mz = 3 * h->Nz / 2;
  rc = ensure_staging(h, size_t(count) * 3 * h->My * Mx * Mz * sizeof(double));
  if (rc) return rc;
  rc = refresh_velocities(h);
  if (rc) return rc;
  HIP_OR_FAIL(h, launch_to_channels(h->precision, h->vel, h->staging, h->cheb_cinv, out, h->My, h->E, h->K, h->L,
                                    h->NZ, Mx, Mz, member0, count, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  return DNS_OK;
}

int dns_set_channels(dns_handle* h, int member0, int count, const float* in) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) {
    dns_handle* sh;
    int m0;
    const int rc = route(h, member0, count, &sh, &m0);
    return rc ? rc : forward(h, sh, dns_set_channels(sh, m0, count, in));
  }
  if (!in) return fail(h, DNS_E_INVALID, "in is NULL");
  if (member0 < 0 || count < 1 || member0 + count > h->E) return fail(h, DNS_E_INVALID, "member range out of bounds");
  int rc = ensure_cheb(h);
  if (rc) return rc;
  const int Mx = 3 * h->Nx / 2, Mz = 3 * h->Nz / 2;
  const size_t nphys = size_t(count) * 3 * h->My * Mx * Mz;
  const size_t nspec = size_t(count) * 3 * h->My * h->K * 2;
  rc = ensure_staging(h, (nphys + nspec) * sizeof(double));
  if (rc) return rc;
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  HIP_OR_FAIL(h, launch_from_channels(in, h->staging, h->staging + nphys, h->cheb_t, h->v, h->eta, h->U, h->W, h->My,
                                      h->E, h->L, h->NZ, Mx, Mz, member0, count, h->kxs, h->kzs, h->Ubot, h->Utop,
                                      h->stream));
  HIP_OR_FAIL(h, hipMemsetAsync(h->failed + member0, 0, sizeof(int) * count, h->stream));
  if (h->shared_mean)
    HIP_OR_FAIL(h, launch_share_columns(h->v, h->eta, h->U, h->W, h->E, h->N, h->NZ, h->My, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  h->vel_fresh = false;
  return DNS_OK;
}

int dns_set_channels_noalloc(dns_handle* h, int member0, int count, const float* in) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) {
    dns_handle* sh;
    int m0;
    const int rc = route(h, member0, count, &sh, &m0);
    return rc ? rc : forward(h, sh, dns_set_channels_noalloc(sh, m0, count, in));
  }
  if (!in) return fail(h, DNS_E_INVALID, "in is NULL");
  if (member0 < 0 || count < 1 || member0 + count > h->E) return fail(h, DNS_E_INVALID, "member range out of bounds");
  const int Mx = 3 * h->Nx / 2, Mz = 3 * h->Nz / 2;
  const size_t per_member = size_t(3) * h->My * (size_t(Mx) * Mz + 2 * size_t(h->K));
  const size_t max_count = kNoAllocScratchBytes / (per_member * sizeof(double));
  if (size_t(count) > max_count)
    return fail(h, DNS_E_INVALID,
                "count " + std::to_string(count) + " exceeds the allocation-free scratch (" +
                    std::to_string(kNoAllocScratchBytes >> 20) + " MiB): at most " + std::to_string(max_count) +
                    " members per call on this grid");
  double* scr = noalloc_scratch(h->device);
  if (!scr || !h->cheb_t) return fail(h, DNS_E_STATE, "allocation-free scratch not set up on this device");
  const size_t nphys = size_t(count) * 3 * h->My * Mx * Mz;
  HIP_OR_FAIL(h, launch_from_channels(in, scr, scr + nphys, h->cheb_t, h->v, h->eta, h->U, h->W, h->My, h->E, h->L,
                                      h->NZ, Mx, Mz, member0, count, h->kxs, h->kzs, h->Ubot, h->Utop, h->stream));
  HIP_OR_FAIL(h, launch_clear_ints(h->failed + member0, count, h->stream));
  if (h->shared_mean)
    HIP_OR_FAIL(h, launch_share_columns(h->v, h->eta, h->U, h->W, h->E, h->N, h->NZ, h->My, h->stream));
  h->vel_fresh = false;
  return DNS_OK;
}

int dns_kernel_times(dns_handle* h, int nreps, double* plane_ms, double* mode_ms) {
  if (!h) return fail(nullptr, DNS_E_STATE, "handle is NULL");
  ORDER_AFTER_PARENT(h);
  if (h->grouped()) return fail(h, DNS_E_INVALID, "call this on a group's handle (dns_group_handle)");
  if (nreps < 1) return fail(h, DNS_E_INVALID, "nreps must be >= 1");
  if (!h->vel_fresh) {
    int rc = refresh_velocities(h);
    if (rc) return rc;
  }
  hipEvent_t e0, e1, e2;
  HIP_OR_FAIL(h, hipEventCreate(&e0));
  HIP_OR_FAIL(h, hipEventCreate(&e1));
  HIP_OR_FAIL(h, hipEventCreate(&e2));
  // one untimed launch of each, then nreps timed launches of each, in the
  // launch shape of a step (interior planes, all members)
  HIP_OR_FAIL(h, plane_launch(h, false, 0, -1, nullptr, false));
  HIP_OR_FAIL(h, launch_mode(h->precision, mode_args(h, 1), h->stream));
  HIP_OR_FAIL(h, hipEventRecord(e0, h->stream));
  for (int r = 0; r < nreps; ++r)
    HIP_OR_FAIL(h, plane_launch(h, false, 0, -1, nullptr, false));
  HIP_OR_FAIL(h, hipEventRecord(e1, h->stream));
  for (int r = 0; r < nreps; ++r) HIP_OR_FAIL(h, launch_mode(h->precision, mode_args(h, 1), h->stream));
  HIP_OR_FAIL(h, hipEventRecord(e2, h->stream));
  HIP_OR_FAIL(h, hipEventSynchronize(e2));
  float t01 = 0.f, t12 = 0.f;
  HIP_OR_FAIL(h, hipEventElapsedTime(&t01, e0, e1));
  HIP_OR_FAIL(h, hipEventElapsedTime(&t12, e1, e2));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipEventDestroy(e2);
  if (plane_ms) *plane_ms = double(t01) / nreps;
  if (mode_ms) *mode_ms = double(t12) / nreps;
  // the mode kernel rewrote the stage buffers from sub-step-1 data
  h->vel_fresh = false;
  return DNS_OK;
}

int dns_host_operators(const dns_geometry* g, double Re, int Nx, int Ny, int Nz, double dt,
                       int h_index, int v_discretization, double* ops, double* mean_ops, double* lift,
                       double* green, double* D1, double* D1c, double* ccw) {
  if (!g || !(g->Lx > 0) || !(g->Lz > 0) || !(Re > 0) || !(dt > 0) || (h_index != 0 && h_index != 1) ||
      (v_discretization != DNS_VDISC_CLAMPED && v_discretization != DNS_VDISC_KMM))
    return fail(nullptr, DNS_E_INVALID, "invalid operator request");
  if (Nx <= 0 || Nz <= 0 || (Nx % 2) || (Nz % 2) || Ny < 5 || Ny > 257)
    return fail(nullptr, DNS_E_INVALID, "invalid grid");
  const double Uw = g->Uw > 0 ? g->Uw : 1.0;
  const double Ub = g->flow == DNS_FLOW_COUETTE ? -Uw : 0.0;
  const double Ut = g->flow == DNS_FLOW_COUETTE ? Uw : 0.0;
  HostOperators ho;
  if (build_operators(Ny, Nx / 2, Nz / 2, 2.0 * M_PI / g->Lx, 2.0 * M_PI / g->Lz, Re, dt, Ub, Ut, &ho,
                      v_discretization))
    return fail(nullptr, DNS_E_INVALID, "a Crank-Nicolson operator is singular");
  auto put = [](double* dst, const std::vector<double>& src) {
    if (dst) std::memcpy(dst, src.data(), src.size() * sizeof(double));
  };
  put(ops, ho.ops[h_index]);
  put(mean_ops, ho.mean_ops[h_index]);
  put(lift, ho.lift[h_index]);
  put(green, ho.green[h_index]);
  put(D1, ho.D1);
  put(D1c, ho.D1c);
  put(ccw, ho.ccw);
  return DNS_OK;
}

}  // extern "C"
