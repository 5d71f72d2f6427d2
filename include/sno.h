/*
 * Learned spin-up of ensemble members (C ABI of libdns_ensemble.so, part 2).
 *
 * The paper starts each member from a perturbed state and lets the DNS run
 * through the transient to turbulence (Sec. 4 discards the transient before
 * accumulating statistics).  Here a small spectral neural operator (SNO), trained
 * on pairs of states that the DNS itself produces some steps apart, advances new
 * members through most of that transient; the plain DNS then continues from an
 * admissible state rebuilt from the prediction and checks every member.
 *
 * Channel form of a member's state: u, v, w on the 3/2-padded x-z grid
 * (Mx = 3Nx/2 by Mz = 3Nz/2 points, the grid of the advection term, Sec. 3.2)
 * at the Ny Chebyshev nodes (Sec. 2), each expanded along y in the Chebyshev
 * polynomials T_k, k < Ny, of its interpolant through the nodes.  Array layout
 * (float): [member][channel c = field * Ny + k][point p = iz * Mx + ix], field
 * 0, 1, 2 = u, v, w.
 *
 * SNO (width W, L layers, retained modes mx x mz), for one sample x (C
 * channels by P = Mx Mz points):
 *   h_0 = W_lift x + b_lift
 *   h_l = GELU(W_l h_{l-1} + b_l + IDFT(R_l[m] DFT(h_{l-1})[m])),  l = 1..L
 *   y   = x + Q h_L + b_Q
 * DFT: X[m] = 1/(Mx Mz) sum_p h[p] e^{-i theta}, theta = 2 pi (kx ix/Mx + kz iz/Mz),
 * modes m = kx mz + q with kx = 0..mx-1 and kz = q (q < mz/2) or q - mz;
 * IDFT: g[p] = sum_m w Re(Y[m] e^{+i theta}), w = 1 for kx = 0 and 2 otherwise;
 * R_l[m] is a complex W x W matrix per mode; GELU(z) = z Phi(z).
 * Loss: mean over samples of ||y_hat - y||_2 / ||y||_2.  Optimiser: AdamW
 * (decoupled weight decay, bias-corrected moments).
 * Parameters (float, flat, in this order): W_lift (W x C), b_lift (W); per
 * layer W_l (W x W), b_l (W), Re R_l (mx mz x W x W), Im R_l (same, [m][o][i]);
 * Q (C x W), b_Q (C).
 * Arithmetic: every linear map runs as a GEMM on the matrix cores with bfloat16
 * operands and FP32 accumulation (SNO_MATH_BF16, default) or in FP32
 * (SNO_MATH_FP32, for verification); activations, parameters and the
 * optimiser state are FP32.
 *
 * Return codes are those of dns.h.  All tensor arguments are device pointers
 * unless stated; calls are asynchronous on the handle's stream except where
 * they return host values.
 */
#ifndef DNS_SNO_H
#define DNS_SNO_H

#include "dns.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Channel form of members [member0, member0 + count) of h's current state into
 * out (device, float, count x 3 Ny x Mz Mx).  Synchronises.  Errors:
 * DNS_E_INVALID (range, NULL), DNS_E_HIP. */
int dns_get_channels(dns_handle* h, int member0, int count, float* out);

/* Replace the states of members [member0, member0 + count) by the admissible
 * states built from channel-form data in (device, float, same layout): v at the
 * interior nodes, eta = i kz u - i kx w, the (0, 0) modes as U00 and W00 with
 * the wall values of the boundary conditions, the n_x = 0 column made
 * Hermitian, v = eta = 0 at (0, 0).  Continuity and no-slip then hold exactly.
 * Clears the members' failure flags.  Synchronises.  Errors as above. */
int dns_set_channels(dns_handle* h, int member0, int count, const float* in);

/* Allocation-free dns_set_channels, for callers that cannot allocate device
 * memory during the call (work captured into a HIP graph, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and the same resulting
 * states, bitwise, as dns_set_channels.  It calls no allocating routine: its
 * FP64 intermediates (per member 3 Ny planes of Mx Mz values and 3 Ny x
 * Nx/2 (Nz-1) complex values) live in a fixed library array of
 * DNS_NOALLOC_SCRATCH_BYTES on each GPU, held until the process ends.
 * It queues its kernels on the handle's stream and returns without
 * synchronising (the failure flags are cleared by a kernel, not a memset);
 * `in` must stay valid until that work has run.  All calls on one GPU, from
 * every handle, share that array and leave the last call's intermediates in
 * it: calls whose queued work overlaps in time race, so order them (one
 * stream, or events).  Errors: DNS_E_INVALID (range, NULL, or count above
 * the members whose intermediates fit the array; the message gives that
 * number), DNS_E_STATE, DNS_E_HIP. */
#define DNS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int dns_set_channels_noalloc(dns_handle* h, int member0, int count, const float* in);

typedef struct sno_handle sno_handle;

typedef struct {
  int channels;   /* C: 3 Ny for the channel form of a grid with Ny nodes */
  int width;      /* W                                                   */
  int layers;     /* L >= 1                                              */
  int Mx, Mz;     /* physical grid points                                */
  int modes_x;    /* mx <= Mx / 2                                        */
  int modes_z;    /* mz <= Mz, even                                      */
  int max_batch;  /* largest batch passed to forward / training calls    */
} sno_config;

typedef struct {
  float lr, beta1, beta2, eps, weight_decay;
} sno_adamw;

#define SNO_MATH_BF16 0
#define SNO_MATH_FP32 1
#define SNO_OPT_MATH 1    /* value: SNO_MATH_*                             */
#define SNO_OPT_STREAM 2  /* value: hipStream_t as an integer (0: own)     */

/* Create an SNO with parameters drawn from a seeded counter-based generator
 * (uniform, scaled by 1/sqrt(fan-in); R by 1/W; Q by 0.1/sqrt(W); biases 0)
 * and zero optimiser state.  Errors: DNS_E_INVALID, DNS_E_NOMEM, DNS_E_HIP. */
int sno_create(const sno_config* cfg, unsigned long long seed, sno_handle** out);
int sno_set_option(sno_handle* s, int key, long long value);
/* Number of parameters (floats) of the flat parameter vector. */
long long sno_num_params(const sno_handle* s);
/* Copy the parameters from / to host memory (n must equal sno_num_params);
 * setting them also zeroes the optimiser state and step count.  Synchronise. */
int sno_set_params(sno_handle* s, const float* host, long long n);
int sno_get_params(sno_handle* s, float* host, long long n);
/* y = SNO(x) for batch samples (device, batch x C x P each). */
int sno_forward(sno_handle* s, const float* x, float* y, int batch);
/* Loss of SNO(x) against target (host *loss) and, if grad_host is not NULL,
 * its gradient with respect to the parameters (host, sno_num_params floats).
 * Synchronises. */
int sno_loss_grad(sno_handle* s, const float* x, const float* target, int batch, float* loss, float* grad_host);
/* One AdamW step on the loss of one batch; *loss (host, may be NULL) receives
 * the loss before the update (NULL: no synchronisation). */
int sno_train_step(sno_handle* s, const float* x, const float* target, int batch, const sno_adamw* opt,
                   float* loss);
int sno_sync(sno_handle* s);
const char* sno_last_error(const sno_handle* s);
void sno_destroy(sno_handle* s);

#ifdef __cplusplus
}
#endif

#endif /* DNS_SNO_H */
