// Spectral neural operator of the learned spin-up: parameters, buffers, and
// the forward pass, gradient and AdamW step as sequences of the kernels in
// kernels_sno.hip (declarations and the parameter layout in include/sno.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sno.h"
#include "internal.h"

using dns::GemmArgs;

struct sno_handle {
  sno_config c{};
  int M = 0;             // retained modes
  long long P = 0, np = 0;
  bool bf16 = true;
  hipStream_t stream = nullptr, own_stream = nullptr;
  // parameters, gradient, AdamW moments
  float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  int t = 0;
  // truncated DFT (P x 2M) and inverse (2M x P)
  float *D = nullptr, *Dinv = nullptr;
  // activations for max_batch samples
  float *h = nullptr, *z = nullptr, *xh = nullptr, *yh = nullptr;
  float *dh = nullptr, *dh2 = nullptr, *dyh = nullptr, *dxh = nullptr, *y = nullptr, *dy = nullptr;
  double* sq = nullptr;
  float* loss = nullptr;
  float* red = nullptr;  // per-sample partial products of the weight gradients
  // parameter offsets
  long long o_lw = 0, o_lb = 0, o_qw = 0, o_qb = 0;
  std::vector<long long> o_w, o_b, o_rr, o_ri;
  std::string err;
};

namespace {

thread_local std::string g_sno_err;

int sfail(sno_handle* s, int code, const std::string& msg) {
  if (s) s->err = msg; else g_sno_err = msg;
  return code;
}

#define SNO_HIP(s, call)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return sfail((s), DNS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// uniform in [-1, 1) from (seed, index)
float uniform_pm1(uint64_t seed, uint64_t i) {
  const uint64_t r = splitmix64(seed * 0xD1B54A32D192ED03ull ^ splitmix64(i));
  return float(double(r >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0);
}

long long W_(const sno_handle* s) { return s->c.width; }

GemmArgs gemm(const float* A, long long sam, long long sak, long long sab, const float* B, long long sbk,
              long long sbn, long long sbb, float* C, long long scm, long long scn, long long scb, int M, int N,
              int K, int batch, float alpha = 1.f, float beta = 0.f, int reduce = 0) {
  GemmArgs g{};
  g.A = A; g.sam = sam; g.sak = sak; g.sab = sab;
  g.B = B; g.sbk = sbk; g.sbn = sbn; g.sbb = sbb;
  g.C = C; g.scm = scm; g.scn = scn; g.scb = scb;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.alpha = alpha; g.beta = beta; g.reduce_batch = reduce;
  return g;
}

#define GEMM(s, ...) SNO_HIP(s, dns::launch_gemm(gemm(__VA_ARGS__), (s)->bf16, (s)->stream))

// C (M x N, contiguous) = sum over the batch of A_b B_b: one GEMM per sample
// into s->red, then a fixed-order sum over samples (deterministic).
#define GEMM_SUM(s, A, sam, sak, sab, B, sbk, sbn, sbb, C, M, N, K, batch)                               \
  do {                                                                                                    \
    GEMM(s, A, sam, sak, sab, B, sbk, sbn, sbb, (s)->red, N, 1, (long long)(M) * (N), M, N, K, batch);  \
    SNO_HIP(s, dns::launch_batch_sum((s)->red, C, batch, (long long)(M) * (N), (s)->stream));            \
  } while (0)

float* H(sno_handle* s, int l, int B) { return s->h + size_t(l) * B * W_(s) * s->P; }
float* Z(sno_handle* s, int l, int B) { return s->z + size_t(l) * B * W_(s) * s->P; }
float* XH(sno_handle* s, int l, int B) { return s->xh + size_t(l) * B * W_(s) * 2 * s->M; }

// Y[b][o][m] = sum_i R[m][o][i] X[b][i][m] (complex, [Re | Im] halves of 2M)
int mix_forward(sno_handle* s, const float* rr, const float* ri, const float* X, float* Y, int B) {
  const long long W = W_(s), M = s->M, M2 = 2 * M;
  const float* Xr = X;
  const float* Xi = X + M;
  float* Yr = Y;
  float* Yi = Y + M;
  GEMM(s, rr, W, 1, W * W, Xr, M2, W * M2, 1, Yr, M2, W * M2, 1, int(W), B, int(W), int(M));
  GEMM(s, ri, W, 1, W * W, Xi, M2, W * M2, 1, Yr, M2, W * M2, 1, int(W), B, int(W), int(M), -1.f, 1.f);
  GEMM(s, ri, W, 1, W * W, Xr, M2, W * M2, 1, Yi, M2, W * M2, 1, int(W), B, int(W), int(M));
  GEMM(s, rr, W, 1, W * W, Xi, M2, W * M2, 1, Yi, M2, W * M2, 1, int(W), B, int(W), int(M), 1.f, 1.f);
  return DNS_OK;
}

int forward_impl(sno_handle* s, const float* x, float* yout, int B) {
  const long long W = W_(s), C = s->c.channels, P = s->P, M2 = 2LL * s->M;
  const float* th = s->theta;
  float* H0 = H(s, 0, B);
  GEMM(s, th + s->o_lw, C, 1, 0, x, P, 1, C * P, H0, P, 1, W * P, int(W), int(P), int(C), B);
  SNO_HIP(s, dns::launch_bias_act(H0, nullptr, th + s->o_lb, B, int(W), int(P), s->stream));
  for (int l = 0; l < s->c.layers; ++l) {
    float* Hin = H(s, l, B);
    float* Zl = Z(s, l, B);
    float* Xh = XH(s, l, B);
    GEMM(s, Hin, P, 1, 0, s->D, M2, 1, 0, Xh, M2, 1, 0, int(B * W), int(M2), int(P), 1);
    int rc = mix_forward(s, th + s->o_rr[l], th + s->o_ri[l], Xh, s->yh, B);
    if (rc) return rc;
    GEMM(s, th + s->o_w[l], W, 1, 0, Hin, P, 1, W * P, Zl, P, 1, W * P, int(W), int(P), int(W), B);
    GEMM(s, s->yh, M2, 1, 0, s->Dinv, P, 1, 0, Zl, P, 1, 0, int(B * W), int(P), int(M2), 1, 1.f, 1.f);
    SNO_HIP(s, dns::launch_bias_act(Zl, H(s, l + 1, B), th + s->o_b[l], B, int(W), int(P), s->stream));
  }
  SNO_HIP(s, hipMemcpyAsync(yout, x, sizeof(float) * B * C * P, hipMemcpyDeviceToDevice, s->stream));
  GEMM(s, th + s->o_qw, W, 1, 0, H(s, s->c.layers, B), P, 1, W * P, yout, P, 1, C * P, int(C), int(P), int(W), B,
       1.f, 1.f);
  SNO_HIP(s, dns::launch_bias_act(yout, nullptr, th + s->o_qb, B, int(C), int(P), s->stream));
  return DNS_OK;
}

// gradient of the loss into s->grad, from s->dy (dL/dy_hat) and the forward cache
int backward_impl(sno_handle* s, const float* x, int B) {
  const long long W = W_(s), C = s->c.channels, P = s->P, M = s->M, M2 = 2 * M;
  const float* th = s->theta;
  float* g = s->grad;
  const int L = s->c.layers;
  // projection
  GEMM_SUM(s, s->dy, P, 1, C * P, H(s, L, B), 1, P, W * P, g + s->o_qw, int(C), int(W), int(P), B);
  SNO_HIP(s, dns::launch_channel_sum(s->dy, g + s->o_qb, B, int(C), int(P), s->stream));
  GEMM(s, th + s->o_qw, 1, W, 0, s->dy, P, 1, C * P, s->dh, P, 1, W * P, int(W), int(P), int(C), B);
  for (int l = L - 1; l >= 0; --l) {
    const float* Hin = H(s, l, B);
    const float* Xh = XH(s, l, B);
    SNO_HIP(s, dns::launch_gelu_bwd(s->dh, Z(s, l, B), (long long)B * W * P, s->stream));
    SNO_HIP(s, dns::launch_channel_sum(s->dh, g + s->o_b[l], B, int(W), int(P), s->stream));
    GEMM_SUM(s, s->dh, P, 1, W * P, Hin, 1, P, W * P, g + s->o_w[l], int(W), int(W), int(P), B);
    GEMM(s, th + s->o_w[l], 1, W, 0, s->dh, P, 1, W * P, s->dh2, P, 1, W * P, int(W), int(P), int(W), B);
    GEMM(s, s->dh, P, 1, 0, s->Dinv, 1, P, 0, s->dyh, M2, 1, 0, int(B * W), int(M2), int(P), 1);
    const float* dYr = s->dyh;
    const float* dYi = s->dyh + M;
    const float* Xr = Xh;
    const float* Xi = Xh + M;
    float* gr = g + s->o_rr[l];
    float* gi = g + s->o_ri[l];
    // dRr = dYr Xr^T + dYi Xi^T ; dRi = -dYr Xi^T + dYi Xr^T   (sums over samples)
    GEMM(s, dYr, M2, W * M2, 1, Xr, W * M2, M2, 1, gr, W, 1, W * W, int(W), int(W), B, int(M));
    GEMM(s, dYi, M2, W * M2, 1, Xi, W * M2, M2, 1, gr, W, 1, W * W, int(W), int(W), B, int(M), 1.f, 1.f);
    GEMM(s, dYr, M2, W * M2, 1, Xi, W * M2, M2, 1, gi, W, 1, W * W, int(W), int(W), B, int(M), -1.f, 0.f);
    GEMM(s, dYi, M2, W * M2, 1, Xr, W * M2, M2, 1, gi, W, 1, W * W, int(W), int(W), B, int(M), 1.f, 1.f);
    // dXr = Rr^T dYr + Ri^T dYi ; dXi = -Ri^T dYr + Rr^T dYi
    const float* rr = th + s->o_rr[l];
    const float* ri = th + s->o_ri[l];
    float* dXr = s->dxh;
    float* dXi = s->dxh + M;
    GEMM(s, rr, 1, W, W * W, dYr, M2, W * M2, 1, dXr, M2, W * M2, 1, int(W), B, int(W), int(M));
    GEMM(s, ri, 1, W, W * W, dYi, M2, W * M2, 1, dXr, M2, W * M2, 1, int(W), B, int(W), int(M), 1.f, 1.f);
    GEMM(s, ri, 1, W, W * W, dYr, M2, W * M2, 1, dXi, M2, W * M2, 1, int(W), B, int(W), int(M), -1.f, 0.f);
    GEMM(s, rr, 1, W, W * W, dYi, M2, W * M2, 1, dXi, M2, W * M2, 1, int(W), B, int(W), int(M), 1.f, 1.f);
    GEMM(s, s->dxh, M2, 1, 0, s->D, 1, M2, 0, s->dh2, P, 1, 0, int(B * W), int(P), int(M2), 1, 1.f, 1.f);
    std::swap(s->dh, s->dh2);
  }
  GEMM_SUM(s, s->dh, P, 1, W * P, x, 1, P, C * P, g + s->o_lw, int(W), int(C), int(P), B);
  SNO_HIP(s, dns::launch_channel_sum(s->dh, g + s->o_lb, B, int(W), int(P), s->stream));
  return DNS_OK;
}

int check_batch(sno_handle* s, const void* a, const void* b, int batch) {
  if (!a || !b) return sfail(s, DNS_E_INVALID, "NULL tensor");
  if (batch < 1 || batch > s->c.max_batch) return sfail(s, DNS_E_INVALID, "batch must be in [1, max_batch]");
  return DNS_OK;
}

void free_sno(sno_handle* s) {
  void* bufs[] = {s->theta, s->grad, s->m1, s->m2, s->D, s->Dinv, s->h, s->z, s->xh, s->yh,
                  s->dh, s->dh2, s->dyh, s->dxh, s->y, s->dy, s->sq, s->loss, s->red};
  for (void* p : bufs)
    if (p) hipFree(p);
  if (s->own_stream) hipStreamDestroy(s->own_stream);
}

}  // namespace

extern "C" {

int sno_create(const sno_config* cfg, unsigned long long seed, sno_handle** out) {
  if (!out) return sfail(nullptr, DNS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg) return sfail(nullptr, DNS_E_INVALID, "config is NULL");
  const sno_config c = *cfg;
  if (c.channels < 1 || c.width < 1 || c.layers < 1 || c.Mx < 2 || c.Mz < 2 || c.modes_x < 1 ||
      c.modes_x > c.Mx / 2 || c.modes_z < 2 || c.modes_z > c.Mz || (c.modes_z % 2) || c.max_batch < 1)
    return sfail(nullptr, DNS_E_INVALID, "invalid SNO configuration");
  sno_handle* s = new sno_handle();
  s->c = c;
  s->M = c.modes_x * c.modes_z;
  s->P = (long long)c.Mx * c.Mz;
  const long long W = c.width, C = c.channels, M = s->M, P = s->P, B = c.max_batch;
  long long o = 0;
  s->o_lw = o; o += W * C;
  s->o_lb = o; o += W;
  for (int l = 0; l < c.layers; ++l) {
    s->o_w.push_back(o); o += W * W;
    s->o_b.push_back(o); o += W;
    s->o_rr.push_back(o); o += M * W * W;
    s->o_ri.push_back(o); o += M * W * W;
  }
  s->o_qw = o; o += C * W;
  s->o_qb = o; o += C;
  s->np = o;
  auto bail = [&](int code, const std::string& msg) {
    free_sno(s);
    delete s;
    return sfail(nullptr, code, msg);
  };
  auto alloc = [&](auto** p, size_t n) {
    return hipMalloc(reinterpret_cast<void**>(p), (n ? n : 1) * sizeof(**p)) == hipSuccess;
  };
  bool ok = alloc(&s->theta, s->np) && alloc(&s->grad, s->np) && alloc(&s->m1, s->np) && alloc(&s->m2, s->np) &&
            alloc(&s->D, size_t(P) * 2 * M) && alloc(&s->Dinv, size_t(P) * 2 * M) &&
            alloc(&s->h, size_t(c.layers + 1) * B * W * P) && alloc(&s->z, size_t(c.layers) * B * W * P) &&
            alloc(&s->xh, size_t(c.layers) * B * W * 2 * M) && alloc(&s->yh, size_t(B) * W * 2 * M) &&
            alloc(&s->dh, size_t(B) * W * P) && alloc(&s->dh2, size_t(B) * W * P) &&
            alloc(&s->dyh, size_t(B) * W * 2 * M) && alloc(&s->dxh, size_t(B) * W * 2 * M) &&
            alloc(&s->y, size_t(B) * C * P) && alloc(&s->dy, size_t(B) * C * P) && alloc(&s->sq, size_t(2 * B)) &&
            alloc(&s->loss, 1) && alloc(&s->red, size_t(B) * W * (C > W ? C : W));
  if (!ok) return bail(DNS_E_NOMEM, "hipMalloc of SNO buffers failed");
  if (hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(DNS_E_HIP, "hipStreamCreate");
  s->stream = s->own_stream;
  // parameters
  std::vector<float> th(size_t(s->np), 0.f);
  auto fill = [&](long long off, long long n, float scale) {
    for (long long i = 0; i < n; ++i) th[size_t(off + i)] = scale * uniform_pm1(seed, uint64_t(off + i));
  };
  fill(s->o_lw, W * C, float(1.0 / std::sqrt(double(C))));
  for (int l = 0; l < c.layers; ++l) {
    fill(s->o_w[l], W * W, float(1.0 / std::sqrt(double(W))));
    fill(s->o_rr[l], M * W * W, float(1.0 / double(W)));
    fill(s->o_ri[l], M * W * W, float(1.0 / double(W)));
  }
  fill(s->o_qw, C * W, float(0.1 / std::sqrt(double(W))));
  // truncated DFT matrices (exact integer phase reduction, FP64 trigonometry)
  std::vector<float> D(size_t(P) * 2 * M), Di(size_t(P) * 2 * M);
  for (long long p = 0; p < P; ++p) {
    const long long iz = p / c.Mx, ix = p - iz * c.Mx;
    for (long long m = 0; m < M; ++m) {
      const long long kx = m / c.modes_z, q = m - kx * c.modes_z;
      const long long kz = q < c.modes_z / 2 ? q : q - c.modes_z;
      const long long rx = (kx * ix) % c.Mx, rz = (((kz * iz) % c.Mz) + c.Mz) % c.Mz;
      const double th_ = 2.0 * M_PI * (double(rx) / c.Mx + double(rz) / c.Mz);
      const double cs = std::cos(th_), sn = std::sin(th_);
      const double w = kx == 0 ? 1.0 : 2.0;
      D[size_t(p) * 2 * M + m] = float(cs / double(P));
      D[size_t(p) * 2 * M + M + m] = float(-sn / double(P));
      Di[size_t(m) * P + p] = float(w * cs);
      Di[size_t(M + m) * P + p] = float(-w * sn);
    }
  }
  ok = hipMemcpy(s->theta, th.data(), th.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(s->D, D.data(), D.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(s->Dinv, Di.data(), Di.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(s->m1, 0, s->np * 4) == hipSuccess && hipMemset(s->m2, 0, s->np * 4) == hipSuccess &&
       hipMemset(s->grad, 0, s->np * 4) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  if (!ok) return bail(DNS_E_HIP, "uploading SNO parameters failed");
  *out = s;
  return DNS_OK;
}

int sno_set_option(sno_handle* s, int key, long long value) {
  if (!s) return sfail(nullptr, DNS_E_STATE, "handle is NULL");
  switch (key) {
    case SNO_OPT_MATH:
      if (value != SNO_MATH_BF16 && value != SNO_MATH_FP32) return sfail(s, DNS_E_INVALID, "unknown math mode");
      s->bf16 = value == SNO_MATH_BF16;
      return DNS_OK;
    case SNO_OPT_STREAM:
      s->stream = value ? reinterpret_cast<hipStream_t>(value) : s->own_stream;
      return DNS_OK;
  }
  return sfail(s, DNS_E_INVALID, "unknown option key");
}

long long sno_num_params(const sno_handle* s) { return s ? s->np : 0; }

int sno_set_params(sno_handle* s, const float* host, long long n) {
  if (!s) return sfail(nullptr, DNS_E_STATE, "handle is NULL");
  if (!host || n != s->np) return sfail(s, DNS_E_INVALID, "parameter count mismatch");
  SNO_HIP(s, hipStreamSynchronize(s->stream));
  SNO_HIP(s, hipMemcpy(s->theta, host, n * 4, hipMemcpyHostToDevice));
  SNO_HIP(s, hipMemset(s->m1, 0, n * 4));
  SNO_HIP(s, hipMemset(s->m2, 0, n * 4));
  SNO_HIP(s, hipDeviceSynchronize());
  s->t = 0;
  return DNS_OK;
}

int sno_get_params(sno_handle* s, float* host, long long n) {
  if (!s) return sfail(nullptr, DNS_E_STATE, "handle is NULL");
  if (!host || n != s->np) return sfail(s, DNS_E_INVALID, "parameter count mismatch");
  SNO_HIP(s, hipStreamSynchronize(s->stream));
  SNO_HIP(s, hipMemcpy(host, s->theta, n * 4, hipMemcpyDeviceToHost));
  return DNS_OK;
}

int sno_forward(sno_handle* s, const float* x, float* y, int batch) {
  if (!s) return sfail(nullptr, DNS_E_STATE, "handle is NULL");
  int rc = check_batch(s, x, y, batch);
  return rc ? rc : forward_impl(s, x, y, batch);
}

int sno_loss_grad(sno_handle* s, const float* x, const float* target, int batch, float* loss, float* grad_host) {
  if (!s) return sfail(nullptr, DNS_E_STATE, "handle is NULL");
  int rc = check_batch(s, x, target, batch);
  if (rc) return rc;
  if (!loss) return sfail(s, DNS_E_INVALID, "loss is NULL");
  rc = forward_impl(s, x, s->y, batch);
  if (rc) return rc;
  const long long per = (long long)s->c.channels * s->P;
  SNO_HIP(s, dns::launch_loss(s->y, target, s->sq, s->dy, s->loss, batch, per, s->stream));
  if (grad_host) {
    rc = backward_impl(s, x, batch);
    if (rc) return rc;
    SNO_HIP(s, hipMemcpyAsync(grad_host, s->grad, s->np * 4, hipMemcpyDeviceToHost, s->stream));
  }
  SNO_HIP(s, hipMemcpyAsync(loss, s->loss, 4, hipMemcpyDeviceToHost, s->stream));
  SNO_HIP(s, hipStreamSynchronize(s->stream));
  return DNS_OK;
}

int sno_train_step(sno_handle* s, const float* x, const float* target, int batch, const sno_adamw* opt,
                   float* loss) {
  if (!s) return sfail(nullptr, DNS_E_STATE, "handle is NULL");
  int rc = check_batch(s, x, target, batch);
  if (rc) return rc;
  if (!opt || !(opt->lr >= 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) ||
      !(opt->beta2 >= 0.f && opt->beta2 < 1.f) || !(opt->eps > 0.f))
    return sfail(s, DNS_E_INVALID, "invalid AdamW settings");
  rc = forward_impl(s, x, s->y, batch);
  if (rc) return rc;
  const long long per = (long long)s->c.channels * s->P;
  SNO_HIP(s, dns::launch_loss(s->y, target, s->sq, s->dy, s->loss, batch, per, s->stream));
  rc = backward_impl(s, x, batch);
  if (rc) return rc;
  s->t += 1;
  SNO_HIP(s, dns::launch_adamw(s->theta, s->grad, s->m1, s->m2, s->np, opt->lr, opt->beta1, opt->beta2, opt->eps,
                               opt->weight_decay, s->t, s->stream));
  if (loss) {
    SNO_HIP(s, hipMemcpyAsync(loss, s->loss, 4, hipMemcpyDeviceToHost, s->stream));
    SNO_HIP(s, hipStreamSynchronize(s->stream));
  }
  return DNS_OK;
}

int sno_sync(sno_handle* s) {
  if (!s) return sfail(nullptr, DNS_E_STATE, "handle is NULL");
  SNO_HIP(s, hipStreamSynchronize(s->stream));
  return DNS_OK;
}

const char* sno_last_error(const sno_handle* s) { return s ? s->err.c_str() : g_sno_err.c_str(); }

void sno_destroy(sno_handle* s) {
  if (!s) return;
  if (s->stream) hipStreamSynchronize(s->stream);
  free_sno(s);
  delete s;
}

}  // extern "C"
