/*
 * vqmc.h - C ABI of the MI355X (gfx950) hot path of autoregressive-model VQMC for
 * diagonal Ising / Max-Cut Hamiltonians (Zhao, De, Chen, Stokes, Veerapaneni,
 * "Overcoming barriers to scalability in variational quantum Monte Carlo",
 * arXiv:2106.13308).
 *
 * One optimisation step (paper Sec. 4, "Algorithm Parallelization": sample, measure,
 * back-propagate) is
 *   1. exact ancestral sampling of B spin strings from a MADE        (Algorithm 1)
 *   2. the diagonal local energy E(s) = sum_{i<j} J_ij s_i s_j          (eq. hamiltonian)
 *   3. batch statistics and the baseline coefficients c_b             (Sec. 2.1)
 *   4. the score-function gradient g = sum_b c_b grad log pi(s_b)      (Sec. 2.1)
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Spins are int8 in {-1,+1}; network input s = 1 - 2x for the binary x of eq. (e:tim).
 *  - The MADE (Sec. 2.3, MADE layer; Sec. 5.1 architecture) has one hidden layer of h
 *    units with sorted 1-based degrees m(k) in [1, n-1].  Unit k receives input site d
 *    (1-based) iff d <= m(k) and feeds output d iff d > m(k).  With 0-based sites and
 *    c[d] = #{k : m(k) <= d} (non-decreasing, c[0] = 0, c[n-1] = h), unit k feeds
 *    output d iff k < c[d] and receives input d iff k >= c[d]: the two masks are
 *    complementary, so all n*h unmasked weights fit one packed n x h matrix
 *        P[d][k] = W2[d][k] if k < c[d] else W1[k][d].
 *  - sigma(z_d) is P(s_d = +1 | s_<d); log pi(s) = sum_d log sigma(s_d z_d).
 *  - Uniform u[b][d] = (Philox4x32-10(ctr = (d/4, b+offset, step, tag), key = seed)
 *    word d%4 >> 8) * 2^-24 (Salmon et al., SC'11), and s_d = +1 iff u < sigma(z_d).
 *  - Leading dimensions: every row-major device array the library defines is padded
 *    to vqmc_ld(x) = x rounded up to VQMC_PAD elements.  A spin batch is B rows of
 *    vqmc_ld(n) int8 (columns >= n are written as 0 by the sampler and ignored by
 *    readers).
 *  - All pointers are DEVICE pointers owned by the caller unless stated "host".  The
 *    library allocates nothing persistent and never reads device data on the host.
 *  - `stream` is a hipStream_t (NULL = default stream).  Calls are asynchronous: they
 *    validate their arguments on the host, enqueue kernels and return.
 *  - Errors: return codes only.  Invalid arguments return VQMC_EINVAL (or EDTYPE /
 *    EWORKSPACE) and enqueue nothing; a failed launch returns VQMC_EHIP.
 *    vqmc_last_error() gives a thread-local message for the last failure.
 */
#ifndef VQMC_H
#define VQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VQMC_PAD 64

/* Working precisions of the weights.  VQMC_F64 names the precision of the reference
 * evaluation (the paper's equations in float64); no call of this library computes in it and
 * every call given it returns VQMC_EDTYPE. */
typedef enum { VQMC_F64 = 0, VQMC_F32 = 1, VQMC_BF16 = 2 } vqmc_dtype;

typedef enum {
  VQMC_OK = 0,
  VQMC_EINVAL = -1,     /* bad size, null pointer, unsorted degrees ...            */
  VQMC_EDTYPE = -2,     /* dtype not supported by this call                        */
  VQMC_EWORKSPACE = -3, /* workspace smaller than vqmc_workspace_bytes()           */
  VQMC_EHIP = -4,       /* a HIP launch or copy failed                             */
  VQMC_ENONFINITE = -5  /* a NaN or infinity among the parameters (vqmc_check_nonfinite) */
} vqmc_status;

/* MADE parameters in the kernels' working precision (produced by vqmc_cast).
 *   P  : n rows x vqmc_ld(h) columns, dtype wdtype, zero padding.
 *   Pt : h rows x vqmc_ld(n) columns, the transpose of P (same values), zero padding.
 *   b1 : h floats (hidden bias), b2 : n floats (output bias), c : n int32 (see above).
 *   band (nullable): the pipelined sampler's tables, vqmc_band_bytes(n, h, wdtype) bytes
 *   written by vqmc_band from P, Pt, b2 and c.  When present, vqmc_sample runs its
 *   pipelined kernel; it must be rebuilt whenever P or b2 changes. */
#define VQMC_BAND_REC 260
typedef struct {
  int32_t n, h;
  int32_t wdtype; /* VQMC_F32 or VQMC_BF16 */
  const void* P;
  const void* Pt;
  const float* b1;
  const float* b2;
  const int32_t* c;
  const float* band;
} vqmc_made;

typedef enum { VQMC_H_CSR_INT = 0, VQMC_H_CSR_F32 = 1, VQMC_H_DENSE_F32 = 2 } vqmc_hkind;

/* Diagonal Hamiltonian E(s) = sum_{i<j} J_ij s_i s_j (eq. hamiltonian with alpha_i =
 * beta_i = 0; Max-Cut: J_ij = w_ij and cut = (W_tot - E) / 2).
 *   CSR kinds: the strict upper triangle (each edge once, row i < col j), rowptr n+1
 *   int64, col nnz int32, w nnz int32 (CSR_INT) or float (CSR_F32).
 *   DENSE_F32: J is n x n float, row-major, symmetric with zero diagonal (only the
 *   strict upper triangle is read). */
typedef struct {
  int32_t n;
  int32_t kind;
  int64_t nnz;
  const int64_t* rowptr;
  const int32_t* col;
  const void* w;
  const float* J;
} vqmc_hamiltonian;

/* Batch statistics (Sec. 2.1 estimators, population variance), device-resident. */
typedef struct {
  double mean_E; /* sum_b E_b / B                 */
  double var_E;  /* sum_b (E_b - mean)^2 / B      */
  double min_E;  /* min_b E_b                     */
  int64_t argmin;/* first b attaining min_E       */
  double sum_E;
} vqmc_stats;

/* Transverse-field Ising model (eq. hamiltonian with the couplings of eq. (e:tim)):
 *   H = -sum_i (alpha_i X_i + beta_i Z_i) - sum_{i<j} beta_ij Z_i Z_j,
 * X_i and Z_i the Pauli matrices of site i.  In the basis of spin strings s (s_i = 1 - 2 x_i)
 * H_ss = -sum_i beta_i s_i - sum_{i<j} beta_ij s_i s_j and H_{s, s^(i)} = -alpha_i, s^(i) being s
 * with site i negated; every other entry is 0.
 *   alpha : n floats (transverse fields; alpha_i >= 0 keeps the ground state non-negative, as the
 *           trial state psi = sqrt(pi) of Sec. 2.3 assumes), beta : n floats,
 *   J     : n x n floats beta_ij, row-major, symmetric with zero diagonal (only the strict upper
 *           triangle is read).  All device pointers. */
typedef struct {
  int32_t n;
  const float* alpha;
  const float* beta;
  const float* J;
} vqmc_tim;

/* ------------------------------------------------------------------ sizes, errors */
int64_t vqmc_ld(int64_t x);
const char* vqmc_error_string(int status);
const char* vqmc_last_error(void);

enum {
  VQMC_WS_LOGPROB = 0,
  VQMC_WS_BACKWARD = 1,
  VQMC_WS_SAMPLE_PLAIN = 2,
  VQMC_WS_STEP = 3,
  VQMC_WS_BACKWARD_SAMPLED = 4,
  VQMC_WS_SR_GRAM = 5,
  VQMC_WS_SR_JVP = 6,
  VQMC_WS_SR_DIRECTION = 7,
  VQMC_WS_TIM_ENERGY = 8,
  VQMC_WS_TIM_STEP = 9
};
/* Workspace bytes needed by a call (host function, no device access). */
size_t vqmc_workspace_bytes(int which, int32_t n, int32_t h, int64_t B, int32_t wdtype);

/* ------------------------------------------------------------------ parameters */
/* Pack dense float32 MADE weights into the master packed matrix (Sec. 2.3 MADE layer;
 * masks by the degree rule above).  W1: h x n, W2: n x h (row-major, device).
 * degrees: HOST array of h sorted 1-based degrees in [1, n-1] (validated: EINVAL if
 * unsorted or out of range); it is read during the call (passed to the device as kernel
 * arguments), so the caller may free it on return and the call does not synchronise.
 * Writes P32 (n x h float, unpadded) and c (n int32). */
int vqmc_pack(int32_t n, int32_t h, const float* W1, const float* W2, const int32_t* degrees,
              float* P32, int32_t* c, void* stream);

/* Inverse of vqmc_pack: dense W1 (h x n) and W2 (n x h) with masked entries set to 0.
 * Used to export parameters or a packed gradient in the paper's W1/W2 form. */
int vqmc_unpack(int32_t n, int32_t h, const float* P32, const int32_t* c, float* W1, float* W2,
                void* stream);

/* Working-precision copies for the kernels: P (n x ld(h)) and Pt (h x ld(n)) in dtype
 * (F32: exact copy; BF16: round-to-nearest-even), padding zeroed.  P32 is n x h. */
int vqmc_cast(int32_t n, int32_t h, const float* P32, int32_t dtype, void* P, void* Pt,
              void* stream);

/* vqmc_cast followed by vqmc_band in one pass over the weights, as after every optimiser
 * update (Sec. 5.1: Adam on the FP32 master weights, then the kernels' working copies are
 * re-derived): writes P and Pt from P32 (as vqmc_cast) and, when band is not NULL, the
 * sampler's tables for the model (P, Pt, b1, b2, c) (as vqmc_band; band of
 * vqmc_band_bytes(n, h, dtype) bytes, 16-byte aligned).  The logit and push tiles are written
 * by the same workgroups that cast P32, from the tile they hold on chip.
 * nonfinite (nullable, device int32): the same pass sets it to 1 if any value of P32, b1 or
 * b2 is a NaN or an infinity (a diverged update); it is never cleared by the library, so
 * the caller zeroes it once and reads it back when convenient (vqmc_check_nonfinite turns
 * the value into a status).  Needs b1 and b2 when given. */
int vqmc_refresh(int32_t n, int32_t h, const float* P32, int32_t dtype, void* P, void* Pt, const float* b1,
                 const float* b2, const int32_t* c, float* band, int32_t* nonfinite, void* stream);

/* Status of a non-finite flag written by vqmc_refresh, after the caller copied it to the host:
 * VQMC_ENONFINITE (with a vqmc_last_error message) if flag != 0, else VQMC_OK. */
int vqmc_check_nonfinite(int32_t flag);

/* Size in bytes of the pipelined sampler's tables (the band) for n sites, h hidden units
 * and weights of type wdtype (VQMC_F32 or VQMC_BF16); 0 for invalid arguments. */
size_t vqmc_band_bytes(int32_t n, int32_t h, int32_t wdtype);

/* The sampler's per-unit band (Algorithm 1, incremental form; the MADE masks of Sec. 2.3
 * split each unit's weights by site).  Unit k completes inside the 64-site block
 * [64q, 64q + 64), q = floor(m(k) / 64) (0-based block of site m(k)).  Its record holds,
 * for j < 64 (entries whose site is < 0 or >= n are 0):
 *   rec[j]       = 2 W1[k][d] if site d = 64q + j feeds k (k >= c[d]), else 0
 *   rec[64 + j]  = W2[d][k]   if k feeds site d = 64q + j (k < c[d]),  else 0
 *   rec[128 + j] = 2 W1[k][d], d = 64(q-1) + j  (every site of the block before feeds k)
 *   rec[192 + j] = W2[d][k],   d = 64(q+1) + j  (k feeds every site of the block after)
 *   rec[256..259] = -(sum of the W1 entries above, halved back), four copies
 * with the values of P in its working precision, widened to float.  After the h records
 * (from byte offset round_up(4 * VQMC_BAND_REC * h, 256)) come the weights of the two
 * products of eq. (2.3) that the sampler's helper waves run, reordered so that each
 * fragment an MFMA lane group reads is one contiguous 1 KB row, zero past site n and unit h
 * (nb = ceil(n / 64) site blocks q, K = 32 units for BF16 and 4 for F32):
 *   logit tiles, nb x (1 + ceil(h / K)) tiles: tile 0 of block q holds b2 of sites 64q..+63
 *     (BF16: the exact split b2 = hi + mid + lo into BF16 terms in units 0-2; F32: b2 in
 *     unit 0), tile t >= 1 the second-layer weights P[64q + i][K (t-1) + u];
 *     BF16 [4][64 lanes][8 units], lane = 16 (u / 8) + i % 16, site i = 16 x first index
 *     + lane % 16; F32 [4][64 lanes] with u = lane / 16.
 *   push tiles, nb x ceil(h / 16) tiles: tile t of block q holds P[64q + d][16t + u] (the
 *     first-layer weights from the block's sites), [2 halves][64 lanes][8 sites], lane =
 *     16 g + u, sites 32 half + 8 g .. + 7.
 * BF16 only, after the push tiles (from the next multiple of 256 bytes): the masked copy of
 * P^T that the backward's hidden adjoint reads, h x ld(n) BF16, Pm[k][d] = P[d][k] where unit
 * k feeds site d (k < c[d]), else 0 (also for d >= n).
 * band: vqmc_band_bytes(n, h, m->wdtype) bytes (device, 16-byte aligned), overwritten.
 * Needs m->P, m->Pt, m->b2 and m->c; m->band is ignored. */
int vqmc_band(const vqmc_made* m, float* band, void* stream);

/* ------------------------------------------------------------------ the hot path */
/* Algorithm 1 (autoregressive sampling), incremental form: each sample keeps its h
 * hidden pre-activations on chip; after drawing s_d it adds s_d * W1[k][d] to the
 * units that receive site d, and each logit is a dot product over the units already
 * complete.  Exactly the conditionals of n full forward passes, O(nh) per sample.
 * Writes S (B x ld(n) int8, 8-byte aligned) and, if logp != NULL, log pi(S) (B floats).
 * With m->band set (see vqmc_band) the draw runs the pipelined kernel, else the blocked
 * one; both draw the same spins up to FP32 rounding of the logits. */
int vqmc_sample(const vqmc_made* m, int64_t B, uint64_t seed, uint64_t step, int64_t sample_offset,
                uint32_t tag, int8_t* S, float* logp, void* stream);

/* vqmc_sample (pipelined kernel; needs m->band) that also returns the forward quantities the
 * gradient needs, so that vqmc_backward_sampled does not recompute the forward pass
 * (Sec. 5.1 MaskedFC1 -> ReLU -> MaskedFC2 evaluated along the way by Algorithm 1):
 *   Zs (nullable): B x ld(n) floats, Zs[b][d] = s_d z_d, the drawn spin times its logit
 *                  (columns >= n are 0); log pi(s_b) = sum_d log sigma(Zs[b][d]).
 *   Rt (nullable): h x ld(B) values of type m->wdtype, Rt[k][b] = relu(A_k(s_b)), the hidden
 *                  activations, batch-contiguous (columns >= B are 0).
 * Zs and Rt 16-byte aligned.  EINVAL without a band or when h is too large for the kernel. */
int vqmc_sample_fwd(const vqmc_made* m, int64_t B, uint64_t seed, uint64_t step, int64_t sample_offset,
                    uint32_t tag, int8_t* S, float* logp, float* Zs, void* Rt, void* stream);

/* Measurement of the pipelined sampler (Algorithm 1 as vqmc_sample with a band, tag 0, sample
 * offset 0; same S and logp): every wave also counts its shader-clock cycles (s_memtime)
 * between the per-block barriers of the 64-site blocks.  *waves receives the waves per
 * workgroup W (waves 0 and 1 run the serial sweep of each block, the others its products and
 * I/O); workgroup g draws samples 8g .. 8g + 7.  cycles (device, ceil(B / 8) * W * 3 uint64):
 *   cycles[(g * W + w) * 3]     = cycles wave w spent from leaving one block's barrier to
 *                                 arriving at the next one's, summed over the blocks (its work,
 *                                 including the issue slots it waited for),
 *   cycles[(g * W + w) * 3 + 1] = cycles from its first departure to its last,
 *   cycles[(g * W + w) * 3 + 2] = that span in ticks of the 100 MHz constant clock
 *                                 (s_memrealtime), which gives the shader clock's rate.
 * The sweep's count per block is the serial chain's critical path per block. */
int vqmc_sample_cycles(const vqmc_made* m, int64_t B, uint64_t seed, uint64_t step, int8_t* S, float* logp,
                       uint64_t* cycles, int32_t* waves, void* stream);

/* Gradient of F = sum_b coef_b log pi(s_b) (as vqmc_logprob_backward) from the Zs and Rt that
 * vqmc_sample_fwd wrote for S: G = coef_b s sigma(-s z) directly from Zs, then the hidden
 * adjoint and the two weight-gradient halves.  Outputs overwritten.  Needs
 * VQMC_WS_BACKWARD_SAMPLED workspace. */
int vqmc_backward_sampled(const vqmc_made* m, const int8_t* S, int64_t B, const float* coef, const float* Zs,
                          const void* Rt, float* dP, float* db1, float* db2, void* ws, size_t ws_bytes,
                          void* stream);

/* Algorithm 1 as the paper runs it: n forward passes of the masked network over the
 * partially drawn batch, drawing site d after pass d (O(n^2 h) per sample).  Same
 * draws as vqmc_sample up to rounding.  Needs VQMC_WS_SAMPLE_PLAIN workspace. */
int vqmc_sample_plain(const vqmc_made* m, int64_t B, uint64_t seed, uint64_t step,
                      int64_t sample_offset, uint32_t tag, int8_t* S, float* logp, void* ws,
                      size_t ws_bytes, void* stream);

/* Local energy of a diagonal Hamiltonian (Sec. 2.1 local energy = H_xx).  E is int64
 * for CSR_INT (exact), double otherwise (FP64 accumulation of exact products).
 * S: B x ld(n) int8 spins (+1/-1; columns >= n are ignored), 16-byte aligned, else EINVAL.
 * The dense kind needs vqmc_energy_workspace_bytes() of workspace (CSR kinds need none;
 * ws may then be NULL). */
int vqmc_energy(const vqmc_hamiltonian* H, const int8_t* S, int64_t B, void* E, void* ws,
                size_t ws_bytes, void* stream);
size_t vqmc_energy_workspace_bytes(const vqmc_hamiltonian* H, int64_t B);

/* Batch statistics and baseline coefficients c_b = (E_b - mean) / B (Sec. 2.1 gradient
 * population form with the batch mean as baseline).  e_is_int: E is int64 (else
 * double).  Deterministic fixed-order FP64 reductions.  coef may be NULL. */
int vqmc_batch_stats(const void* E, int32_t e_is_int, int64_t B, vqmc_stats* stats, float* coef,
                     void* stream);

/* log pi(S) by one dense masked forward pass (MaskedFC1 -> ReLU -> MaskedFC2 ->
 * log-sigmoid, Sec. 5.1) on MFMA; skips the masked half of both products.
 * logp: B floats.  Z (nullable): B x ld(n) float logits. */
int vqmc_logprob(const vqmc_made* m, const int8_t* S, int64_t B, float* logp, float* Z, void* ws,
                 size_t ws_bytes, void* stream);

/* vqmc_logprob without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * kernels, arguments and results as vqmc_logprob; the call allocates nothing.  Its scratch is
 * a fixed array of VQMC_NOALLOC_SCRATCH_BYTES in the library's own device memory: one copy per
 * GPU the library runs on, held until the process ends.  Returns VQMC_EWORKSPACE (enqueueing
 * nothing) when vqmc_workspace_bytes(VQMC_WS_LOGPROB, n, h, B, wdtype) exceeds that size
 * (n = 10^4, h = 10^3, B = 2048 needs about 5 MiB, n = h = 2000, B = 8192 about 33 MiB).
 * Every call on one GPU uses the same array and leaves its contents behind (each call
 * overwrites all it reads, so nothing carries over): calls that may overlap on one GPU (on
 * unordered streams, or from several host threads) race, and the caller must order them.
 * The first call on each device looks up the array's address on that device. */
#define VQMC_NOALLOC_SCRATCH_BYTES (64u << 20)
int vqmc_logprob_noalloc(const vqmc_made* m, const int8_t* S, int64_t B, float* logp, float* Z, void* stream);

/* Gradient of F = sum_b coef_b log pi(s_b) (the surrogate whose gradient is the
 * score-function estimator of Sec. 2.1 when coef = c).  Recomputes the forward pass
 * (nothing is kept from vqmc_logprob).  dP: n x h float (packed like P32), db1: h,
 * db2: n.  Outputs are overwritten. */
int vqmc_logprob_backward(const vqmc_made* m, const int8_t* S, int64_t B, const float* coef,
                          float* dP, float* db1, float* db2, void* ws, size_t ws_bytes,
                          void* stream);

/* Sample-space Gram of the per-sample scores for stochastic reconfiguration (Sec. 2.1:
 * the Fisher information is the expectation of the outer product of grad log pi;
 * Sec. 5.1: SR with a ridge).  With O the B x (nh + h + n) matrix whose row b is
 * grad log pi(s_b) over every unmasked parameter (packed P, b1, b2), writes
 *   K = O O^T,   K[b][b'] = <grad log pi(s_b), grad log pi(s_b')>,
 * the matrix of the Woodbury form (lambda B I + K)^{-1} of the SR solve.  O is never
 * formed: the forward pass is recomputed and two staircase prefix sweeps build K in FP32.
 * S: B x ld(n) int8 spins (device).  K: B x B float, row-major, leading dimension B
 * (device, caller-owned, overwritten; symmetric).  1 <= B <= 65536, else EINVAL.  Needs
 * VQMC_WS_SR_GRAM workspace (it holds three B x B partial sums). */
int vqmc_sr_gram(const vqmc_made* m, const int8_t* S, int64_t B, float* K, void* ws, size_t ws_bytes,
                 void* stream);

/* vqmc_sr_gram for the spins vqmc_sample_fwd just drew, from its byproducts (the same
 * quantities as above, Sec. 2.1 / 5.1): Zs (B x ld(n) floats, s_d z_d) and Rt (h x ld(B)
 * values of type m->wdtype, relu(A), batch-contiguous) as vqmc_sample_fwd wrote them, both
 * 16-byte aligned, so the forward pass is not recomputed.  Same K, limits and
 * VQMC_WS_SR_GRAM workspace as vqmc_sr_gram; EINVAL for a misaligned Zs or Rt. */
int vqmc_sr_gram_sampled(const vqmc_made* m, const int8_t* S, int64_t B, const float* Zs, const void* Rt, float* K,
                         void* ws, size_t ws_bytes, void* stream);

/* The other product of the SR solve (Sec. 2.1 / 5.1, Woodbury form): v = O g, v[b] =
 * <grad log pi(s_b), g>, for a direction g in parameter space given like a gradient: gP
 * n x h float32 packed like P32 (and dP), gb1 h floats, gb2 n floats (device).  The two
 * masked layers are applied with g in place of the weights (the first without its ReLU)
 * and contracted with the score factors of each sample; g is rounded to the weight dtype
 * for the products.  v: B floats (device, overwritten).  Needs VQMC_WS_SR_JVP workspace.
 * With it the SR direction for any g is x = (g - O^T (lambda B I + K)^{-1} O g) / lambda
 * (Woodbury); for the batch gradient itself vqmc_sr_direction needs no O g. */
int vqmc_sr_jvp(const vqmc_made* m, const int8_t* S, int64_t B, const float* gP, const float* gb1, const float* gb2,
                float* v, void* ws, size_t ws_bytes, void* stream);

/* The B x B linear system of stochastic reconfiguration in sample space (Sec. 2.1 Fisher
 * information, Sec. 5.1 SR with a ridge):  (K + shift I) y = scale * rhs, solved in FP64 by a
 * blocked Cholesky factorisation with forward and back substitution, all on the device.
 * K: B x B float (device, row-major, leading dimension B), symmetric positive semi-definite;
 * only its lower triangle is read.  rhs: B floats (device).  y: B floats (device, overwritten;
 * NaN if K + shift I is not positive definite in FP64).  shift > 0 and finite, else EINVAL;
 * 1 <= B <= 65536.  Workspace: vqmc_sr_solve_workspace_bytes(B) bytes (device, 8-byte aligned;
 * it holds the FP64 factor, round_up(B, 64)^2 doubles). */
int vqmc_sr_solve(int64_t B, const float* K, double shift, const float* rhs, double scale, float* y, void* ws,
                  size_t ws_bytes, void* stream);
size_t vqmc_sr_solve_workspace_bytes(int64_t B);

/* The SR (natural-gradient) direction of the batch gradient (Sec. 2.1 gradient and Fisher
 * information; Sec. 5.1 SR with ridge lambda): x solves (O^T O / B + lambda I) x = g with
 * g = O^T coef the gradient vqmc_step returns for coefficients coef (O: per-sample scores over
 * every unmasked parameter, as for vqmc_sr_gram).  By the push-through identity
 * (O^T O / B + lambda I) O^T = O^T (O O^T / B + lambda I) this is
 *     x = O^T y,   (K + lambda B I) y = B coef,   K = O O^T,
 * computed as vqmc_sr_gram (or vqmc_sr_gram_sampled), vqmc_sr_solve and the gradient
 * kernels with coef = y; no d-dimensional system and no division by lambda.
 * S: B x ld(n) int8 spins; coef: B floats (device).  Zs, Rt (nullable together): vqmc_sample_fwd's
 * byproducts for S (then nothing of the forward pass is recomputed), 16-byte aligned.
 * xP (n x h float, packed like dP), xb1 (h), xb2 (n): outputs, overwritten.  K_out (nullable):
 * B x B floats receiving K, else K stays in the workspace.  lambda > 0; 1 <= B <= 65536.
 * Needs VQMC_WS_SR_DIRECTION workspace. */
int vqmc_sr_direction(const vqmc_made* m, const int8_t* S, int64_t B, const float* coef, const float* Zs,
                      const void* Rt, double lambda, float* xP, float* xb1, float* xb2, float* K_out, void* ws,
                      size_t ws_bytes, void* stream);

/* One optimisation step without the parameter update (Sec. 4): sample (algo 0 =
 * incremental, 1 = plain n-pass form), energy, statistics, gradient.  Writes S, logp,
 * E, stats, coef and the gradient (dP, db1, db2).  With algo 0 and a band this is
 * vqmc_sample_fwd, the energy, the statistics and vqmc_backward_sampled, all on `stream`;
 * otherwise the gradient recomputes the forward pass as vqmc_logprob_backward does, its
 * first product overlapping the energy and statistics, which then run on a library-owned
 * auxiliary stream (default priority). */
int vqmc_step(const vqmc_made* m, const vqmc_hamiltonian* H, int64_t B, uint64_t seed,
              uint64_t step, int64_t sample_offset, int32_t algo, int8_t* S, float* logp, void* E,
              vqmc_stats* stats, float* coef, float* dP, float* db1, float* db2, void* ws,
              size_t ws_bytes, void* stream);

/* Local energy of the transverse-field Ising model for the MADE trial state psi = sqrt(pi)
 * (Sec. 2.1 local energy l(x) = (H psi)(x) / psi(x); eq. (e:tim); Sec. 2.3 trial state):
 *     l(s) = H_ss - sum_i alpha_i exp(D_i / 2),   D_i = log pi(s^(i)) - log pi(s),
 * for every string of S.  The n single-flip ratios of a sample come from one forward pass: a flip
 * at site i changes only the pre-activations of the units site i feeds, and so only the
 * conditionals of the sites after i; their logit changes are one masked product per sample
 * (MFMA), its epilogue the sum of log-sigmoid differences.  H_ss in FP64 (its two-site part as
 * vqmc_energy's dense kind), the off-diagonal sum in FP64 from FP32 D_i.
 * S: B x ld(n) int8 spins, 16-byte aligned.  E: B doubles (device, overwritten).  D (nullable):
 * B x ld(n) floats receiving D_i (columns >= n untouched).  Needs VQMC_WS_TIM_ENERGY workspace.
 * EINVAL for H->n != m->n or h beyond 1024 (BF16 weights) / 512 (F32). */
int vqmc_tim_energy(const vqmc_made* m, const vqmc_tim* H, const int8_t* S, int64_t B, double* E, float* D,
                    void* ws, size_t ws_bytes, void* stream);

/* One optimisation step for the TIM (Sec. 4 iteration without the update, as vqmc_step): the
 * pipelined incremental sampler with its forward byproducts (needs m->band), vqmc_tim_energy,
 * the FP64 statistics with c_b = (l_b - mean) / B, and the gradient sum_b c_b grad log pi(s_b)
 * (Sec. 2.1: 2 grad log psi = grad log pi for psi = sqrt(pi)) from the sampler's byproducts.
 * Writes S, logp (nullable), E (B doubles), stats, coef, dP, db1, db2.  Needs VQMC_WS_TIM_STEP
 * workspace; all work on `stream`. */
int vqmc_tim_step(const vqmc_made* m, const vqmc_tim* H, int64_t B, uint64_t seed, uint64_t step,
                  int64_t sample_offset, int8_t* S, float* logp, double* E, vqmc_stats* stats, float* coef,
                  float* dP, float* db1, float* db2, void* ws, size_t ws_bytes, void* stream);

/* The uniforms the samplers consume (the Bernoulli draw of Algorithm 1, "Sample y_i"):
 * u[b][d] for b < B, d < n as defined above, written to u (B x n float, unpadded).
 * Exposed so that the device Philox4x32-10 can be checked against an independent
 * implementation; not needed on the hot path. */
int vqmc_uniforms(int32_t n, int64_t B, uint64_t seed, uint64_t step, int64_t sample_offset,
                  uint32_t tag, float* u, void* stream);

/* ------------------------------------------------------------------ host helper */
/* Build the strict-upper CSR of an undirected edge list (HOST pointers).  edges: m
 * pairs (i, j), i != j, each undirected edge once in either orientation; w: m int32
 * (wkind CSR_INT) or float (CSR_F32).  Outputs (host, caller-sized): rowptr n+1,
 * col m, w_out m, rows sorted by column.  EINVAL on out-of-range or self loops. */
int vqmc_csr_from_edges(int32_t n, int64_t m, const int32_t* edges, const void* w, int32_t wkind,
                        int64_t* rowptr, int32_t* col, void* w_out);

#ifdef __cplusplus
}
#endif
#endif /* VQMC_H */
