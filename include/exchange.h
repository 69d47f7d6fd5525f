/*
 * exchange.h -- C ABI of the MI355X (gfx950) nonlocal-exchange library.
 *
 * The library computes the Hartree-Fock exchange matrix of a hybrid functional
 * in the wavefunction basis, the hot path of the PBE0-in-FLAPW method of
 * Betzinger, Friedrich & Bluegel (arXiv:1003.0524):
 *
 *   V_{nn'}(k) = - sum_q w_q sum_{n'' occ} sum_{IJ} conj(M^{n n''}_I(k,q)) v_IJ(q) M^{n' n''}_J(k,q)
 *
 * (Sec. III.C, eq. "vec-mat-vec"; the q sum is the Brillouin-zone integration
 * on the k mesh of Sec. II; v is the Coulomb matrix of the mixed product basis,
 * eq. "coulomb matrix").
 *
 * Coulomb matrix layout (the transformed, sparse mixed product basis of
 * Sec. III.C and its Fig. 1): the basis index I runs over
 *   [ multipole-free MT functions, channel 0, channel 1, ... ]   N_s = sum_c (nrad_c - 1)
 *   [ one multipole-carrying MT function per channel ]            n_channels
 *   [ interstitial plane waves of q ]                            n_pw[q]
 * A channel is one (atom, L, M) combination. Nonzero blocks of v(q):
 *   D_c  (nrad_c-1)^2  among the multipole-free functions of channel c,
 *   C_c  (nrad_c-1)    between those and the channel's own multipole function,
 *   E(q) N_d(q)^2      dense block over [multipole functions | plane waves],
 *                      N_d(q) = n_channels + n_pw[q].
 * Multipole-free functions produce no potential outside their sphere, so only
 * the on-site (lattice translation T = 0) term of the Bloch sum contributes to
 * D_c and C_c: they are the same for every q and are passed once.
 *
 * All complex numbers are interleaved (re, im) pairs; matrices are column-major.
 *
 * Error behaviour: no function throws or aborts across the ABI. Every call
 * returns an exc_status; a human-readable message for the last failure is
 * available from exchange_last_error(ctx). On failure nothing is written to
 * the caller's outputs. Calls on a destroyed or never-initialised context
 * return EXC_ESTATE (a NULL ctx returns EXC_EINVAL).
 *
 * Asynchrony: exchange_matrix / exchange_matrix_all enqueue work on the given
 * HIP stream (hipStream_t passed as void*, NULL = the default stream) and
 * return without waiting when on_device = 1; inputs must stay valid and
 * outputs must not be read until the stream has reached that point. With
 * on_device = 0 the call copies from / to host memory and returns when the
 * result is on the host.
 *
 * Around the exchange matrix: exchange_energy[_device] (eq. "HF exchange
 * energy"); exchange_gamma_term (the q -> 0 term, Sec. III.E); the symmetry
 * reductions of Sec. III.D -- exc_desc.inversion (real v and bands),
 * exc_desc.w_kq (q sum over the extended irreducible wedge) and
 * exchange_band_mask (band pairs from the Theta^MT criterion);
 * exchange_back_transform (V in the LAPW basis, Sec. III.A); and the learned
 * extrapolator of V between exact evaluations (exchange_nn_*).
 */
#ifndef EXCHANGE_H
#define EXCHANGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EXC_OK = 0,
  EXC_EINVAL = -1,        /* NULL pointer, negative or inconsistent size, bad enum  */
  EXC_ENOMEM = -2,        /* device or host allocation failed                       */
  EXC_ENOTPD = -3,        /* Cholesky pivot <= 0: v(q) is not positive definite     */
  EXC_EHIP = -4,          /* a HIP runtime call failed                              */
  EXC_ESTATE = -5,        /* context destroyed, not initialised, or result missing  */
  EXC_EUNSUPPORTED = -6   /* valid request the library does not support            */
} exc_status;

/* Arithmetic of the bulk products (Cholesky, q sum and diagonal are always FP64). */
typedef enum {
  EXC_FP64 = 0,           /* FP64 MFMA throughout                                    */
  EXC_FP32 = 1,           /* operands rounded to FP32, FP32 MFMA, FP32 accumulate    */
  EXC_BF16X3 = 2,         /* x = hi + lo (bf16, RNE); hi*hi + hi*lo + lo*hi on BF16
                             MFMA with FP32 accumulate (Henry, Tang & Heinecke 2019) */
  EXC_BF16X6 = 3          /* x = hi + mid + lo; the six leading products             */
} exc_precision;

/* How the product with v(q) is organised. Both are exact re-arrangements of
 * the vector-matrix-vector form. */
typedef enum {
  EXC_FORM_GEMM = 0,      /* W = v A (sparse blocks + dense E), V -= w_q A^H W; FP64 only */
  EXC_FORM_CHOL_HERK = 1  /* v = L L^H once at init; Y = L^H A, V -= w_q Y^H Y            */
} exc_form;

typedef enum { EXC_C128 = 0, EXC_C64 = 1 } exc_dtype;   /* element type of M */

typedef struct exc_ctx exc_ctx;   /* opaque; owned by the library */

typedef struct {
  int32_t n_k;              /* number of irreducible k points (>= 1)                    */
  int32_t n_q;              /* number of q points of the mesh (>= 1)                     */
  int32_t n_occ;            /* occupied bands n'' summed at every k-q (>= 1)             */
  int32_t n_channels;       /* (atom, L, M) channels (>= 0)                              */
  const int32_t *n_bands;   /* [n_k] bands n_b(k) = n_max at k, 1..128 (the batched GEMM
                               form: 1..64, EXC_EUNSUPPORTED beyond; the unbatched GEMM
                               form takes 1..128)                                        */
  const int32_t *n_pw;      /* [n_q] interstitial plane waves of q (>= 0; with no
                               channels at least 1, else EXC_EINVAL: empty basis)        */
  const int32_t *ch_nrad;   /* [n_channels] radial functions per channel (>= 1):
                               one multipole function + (nrad - 1) multipole-free ones  */
  const double *w_q;        /* [n_q] q weights, host memory; NULL -> 1/n_q              */
  int32_t precision;        /* exc_precision                                             */
  int32_t form;             /* exc_form                                                  */
  int32_t batched;          /* exchange_matrix_all: 1 = one persistent launch over all
                               (k,q) work (EXC_GRAPH=1: replayed from a HIP graph); 0 =
                               one launch per (k,q) pair. Unbatched, the GEMM form runs per
                               pair the block-sparse rows of W = v A, W_d = E A_d + X and
                               A^H W on FP64 matrix cores, and accumulates V(k) in FP64 in
                               the order of q                                            */
  int32_t device;           /* HIP device ordinal                                        */
  int32_t inversion;        /* 1: inversion-symmetric system (Sec. III.D, symmetrized MT
                               functions): v(q) and the projections are real. Only the
                               real parts of E, D and C are read. M holds the n_occ real
                               bands in pairs: column j of a q block is the complex number
                               M_{2j} + i M_{2j+1} (M_{n_occ} = 0 when n_occ is odd), so a
                               q block is [ceil(n_occ/2)][n_b][N_MB] in the element type of
                               `dtype`. V(k) is real symmetric (stored complex128, Im = 0).
                               Since v is real, Re(Y^H Y) of a packed column is the sum of
                               the two bands' Y^T Y: half the columns, half the bytes.
                               0: general complex system                                 */
  const double *w_kq;       /* [n_k * n_q] (k-major) weight of each (k, q) pair, host
                               memory, or NULL for w_q of every k. A zero weight leaves
                               the pair out: its q block is then absent from M(k) (the
                               remaining blocks keep mesh order). For the q sum over the
                               extended irreducible wedge EIBZ(k) (Sec. III.D, eq. "rotate
                               APW"): w_q / N_{k,q} on the wedge, 0 elsewhere; summing the
                               result rotated by the operations of the little group of k
                               gives the full sum. Every k needs one nonzero weight
                               (EXC_EINVAL otherwise).                                   */
} exc_desc;

typedef struct {
  const void *const *E;     /* [n_q] -> N_d(q)^2 complex128, column-major, Hermitian     */
  const void *const *D;     /* [n_q] -> concat over channels of (nrad_c-1)^2 complex128,
                               column-major: the multipole-free blocks D_c of v(q)
                               (Sec. III.C, Fig. 1). Entries may alias: when all n_q
                               pointers are equal (the blocks do not depend on q, as a
                               function with no multipole produces no potential outside
                               its sphere) one copy is kept; otherwise one per q.
                               NULL (or NULL entries) allowed only without such functions */
  const void *const *C;     /* [n_q] -> concat over channels of (nrad_c-1) complex128: the
                               couplings C_c of each block to its channel's multipole
                               function; aliasing as for D (one copy only when both D and
                               C alias across q)                                         */
  int32_t on_device;        /* 0: host pointers, 1: device pointers (copied either way)   */
} exc_coulomb;

/*
 * exchange_init -- validate sizes, copy v(q) to device memory and prepare it.
 * The Coulomb matrix is independent of the wavefunctions and is prepared once
 * per self-consistency cycle (Sec. III.C, after eq. "coulomb matrix"). With
 * form = EXC_FORM_CHOL_HERK it is Cholesky-factored in FP64 on the GPU here;
 * a non-positive pivot returns EXC_ENOTPD (the message names q). The caller's
 * buffers may be freed after return. *out receives the new context (NULL on
 * failure). The call synchronises `stream`.
 */
exc_status exchange_init(const exc_desc *desc, const exc_coulomb *coulomb, void *stream,
                         exc_ctx **out);

/*
 * exchange_matrix -- V^x(k) for one irreducible k, summed over every q of the
 * mesh (eq. "vec-mat-vec" with the band cutoff n, n' < n_b(k), Sec. III).
 *   M  : the q blocks of k concatenated in mesh order; block q is
 *        [n''< n_occ][n < n_b(k)][I < N_MB(q)] (I fastest), element type `dtype`,
 *        holding M^{n n''}_I(k,q) = <M_I^q phi_{n'' k-q} | phi_{n k}>.
 *   Vx : n_b(k)^2 complex128, column-major. The upper triangle is computed, the
 *        lower triangle is its exact conjugate mirror and Im V_nn = 0.
 *   on_device: 1 -> M and Vx are device pointers; 0 -> host pointers.
 * The result also stays resident in the context for exchange_energy.
 */
exc_status exchange_matrix(exc_ctx *ctx, int32_t k, const void *M, int32_t dtype,
                           int32_t on_device, void *Vx, void *stream);

/*
 * exchange_matrix_noalloc -- exchange_matrix for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and result (bitwise), on device pointers M and Vx, with
 * the call's partial results and block-sparse workspace in a static per-GPU scratch
 * array of 64 MiB instead of context buffers. It calls no hipMalloc or hipFree.
 *   Batched contexts only (EXC_EUNSUPPORTED otherwise, and for complex128 M when the
 *   context's kernel reads complex64 only). EXC_EINVAL when this k needs more scratch
 *   than the array holds (the message gives both sizes). All calls on one GPU share the
 *   array: calls that overlap on one GPU (other streams, other threads) race.
 */
exc_status exchange_matrix_noalloc(exc_ctx *ctx, int32_t k, const void *M, int32_t dtype,
                                   void *Vx, void *stream);

/*
 * exchange_matrix_all -- V^x(k) for every irreducible k. M_k[k] and Vx_k[k] are
 * laid out as for exchange_matrix. With desc.batched = 1 all (k, q) work runs
 * in one persistent launch, followed by the FP64 q-sum, both enqueued on `stream`
 * (EXC_GRAPH=1: replayed from a HIP graph, re-captured when the pointers change);
 * otherwise one launch per (k, q) pair.
 */
exc_status exchange_matrix_all(exc_ctx *ctx, const void *const *M_k, int32_t dtype,
                               int32_t on_device, void *const *Vx_k, void *stream);

/*
 * exchange_energy -- E_x = 1/2 sum_k w_k Tr(rho_k V_k) over the resident V(k)
 * of the last exchange_matrix[_all] calls (eq. "HF exchange energy" with a
 * spin-degenerate density matrix rho = 2 P_occ).
 *   w_k   : [n_k] host weights, NULL -> 1/n_k
 *   rho_k : [n_k] device pointers to n_b(k)^2 complex128 column-major, or NULL
 *           for rho_k = diag(2 for n < n_occ, 0 otherwise)
 * Synchronises the context's stream. EXC_ESTATE if some V(k) was never computed.
 */
exc_status exchange_energy(exc_ctx *ctx, const double *w_k, const void *const *rho_k,
                           double *E_out);

/*
 * exchange_energy_device -- the same E_x as exchange_energy, left in device memory
 * without synchronising: for loops that keep results on the GPU.
 *   w_k, rho_k : as for exchange_energy (w_k host, rho_k device pointers); both
 *                arrays are copied before the call returns
 *   E_dev      : device pointer to one double, written on `stream` after the
 *                last exchange_matrix[_all] work (NULL stream: that work's stream;
 *                another stream is made to wait for it)
 * The sum over k is taken on the device in the order of k. Energy calls share the
 * context's staging buffers: each call (this one and exchange_energy) first makes
 * its stream wait for the previous energy call of the context, on whatever stream
 * that ran. Errors of the enqueued kernels surface on the next synchronising call.
 * EXC_ESTATE if some V(k) was never computed.
 */
exc_status exchange_energy_device(exc_ctx *ctx, const double *w_k, const void *const *rho_k,
                                  double *E_dev, void *stream);

/*
 * exchange_gamma_term -- the q -> 0 term of the exchange matrix (Sec. III.E,
 * eqs. "F(q)", "divergence" and "div final"). The divergent 1/q^2 part of the
 * Coulomb matrix, damped by exp(-beta q^2), is integrated analytically and the
 * part of that integral the q-mesh sum already holds is subtracted:
 *   C = erf(sqrt(beta) q0) / sqrt(pi beta)
 *       - 4 pi / (N Omega) * sum_{p, 0 < |p| <= q0} exp(-beta |p|^2) / |p|^2
 * with exp(-beta q0^2) = beta, p over every point q + G of the mesh (every G),
 * N = mesh[0] mesh[1] mesh[2] and Omega = (2 pi)^3 / |det B|. The prefactor
 * 4 pi / (N Omega) is the Riemann-sum weight that makes the bracket vanish as
 * the mesh is refined (the printed equation shows 1/(N Omega)). V_nn gains -C
 * for n < n_occ (occupation 1 per spin); off-diagonal elements are unchanged.
 *   recip : [9] host, row-major, rows = reciprocal lattice vectors b_i (bohr^-1)
 *   mesh  : [3] host, divisions of the Gamma-centred mesh (>= 1); its points are
 *           sum_i (j_i / mesh_i) b_i for integer j_i
 *   beta  : damping parameter, 0 < beta < 1 (the paper's choice is 0.005)
 *   apply : 1 -> every later exchange_matrix[_all] adds -C to the occupied diagonal
 *           of V(k) (and so to exchange_energy); 0 -> C is computed, no shift is applied.
 *           A context with per-pair weights (exc_desc.w_kq) returns EXC_EUNSUPPORTED
 *           for apply = 1: its q sum is restricted (EIBZ(k)), the rotation over the
 *           little group that completes it happens outside the library, and the shift
 *           must enter the completed sum once -- the caller adds -C after the rotation
 *   C_out : host, receives C (may be NULL)
 * The lattice sum runs on the GPU in FP64 in a fixed order (the same inputs give
 * the same bits). The call waits for earlier exchange_matrix[_all] work, runs on
 * `stream` and synchronises it. EXC_EINVAL for NULL arrays, mesh < 1, beta outside
 * (0, 1), linearly dependent b_i, or more than 2^40 candidate lattice points.
 */
exc_status exchange_gamma_term(exc_ctx *ctx, const double *recip, const int32_t *mesh, double beta,
                               int32_t apply, double *C_out, void *stream);

/*
 * exchange_back_transform -- V^x(k) in the LAPW basis (Sec. III.A, eq. "APW trafo"):
 *   VGG = Z V(k) Z^H,   Z = S(k) c(k),
 * S the overlap matrix and c the (generalized orthonormal, c^H S c = 1) eigenvectors of
 * the n_b(k) bands, so that Z V Z^H multiplies V by the inverse of c and its adjoint.
 * (The printed left factor carries S* with S's indices; for the Hermitian S its
 * adjoint's elements are read, which keeps VGG Hermitian.)
 *   Z   : device, n_G x n_b(k) complex128, column-major (leading dimension n_G)
 *   VGG : device, n_G x n_G complex128, column-major, every element written
 * V(k) is the resident result of the last exchange_matrix[_all]. Asynchronous on
 * `stream` (ordered after that work); Z and VGG must stay valid until it completes.
 * A workspace of n_G x n_b(k) complex128 is kept by the context and grown when a
 * larger one is needed (the growth synchronises the device). EXC_EINVAL for a bad k,
 * NULL pointers or n_G outside [1, 2^20]; EXC_ESTATE if V(k) was never computed.
 */
exc_status exchange_back_transform(exc_ctx *ctx, int32_t k, const void *Z, int32_t n_G, void *VGG,
                                   void *stream);

/*
 * exchange_band_mask -- band pairs (n, n') of V(k) to compute (Sec. III.D, eq. "MT
 * stepfuntion"): an element of V^x between bands of different irreducible
 * representations is zero, which the caller detects from the matrix elements of
 * Theta^MT = 1 - Theta between groups of degenerate bands and passes here.
 *   keep : host, n_b(k) x n_b(k) bytes, row-major (element (n, n') at keep[n n_b + n']),
 *          nonzero = compute; NULL = compute every pair (the default)
 * The work is skipped per 8 x 8 tile of band pairs: a tile (with its mirror) is left
 * out only if every element of both is 0, and then its elements of V(k) are 0; the
 * diagonal tiles (which hold V_nn) are always computed. Takes effect for later
 * exchange_matrix[_all] calls; it synchronises the device first.
 */
exc_status exchange_band_mask(exc_ctx *ctx, int32_t k, const uint8_t *keep);

/* Message of the last failure on ctx (never NULL; "" if none). With ctx == NULL,
 * the message of the last failed exchange_init on this thread. */
const char *exchange_last_error(const exc_ctx *ctx);

/* Release every resource of ctx. NULL is a no-op; a second destroy of the same
 * pointer is undefined (the memory is gone), as for free(). */
void exchange_destroy(exc_ctx *ctx);

/*
 * exchange_query -- introspection for tests and benchmarks.
 *   what = 0: number of work items of the batched launch
 *   what = 1: nominal flops of the method per exchange_matrix_all (sparse-aware,
 *             complex multiply-add = 8 flops, Hermitian upper triangle only)
 *   what = 2: flops the chosen form executes per exchange_matrix_all (padding included)
 *   what = 3: id of the main kernel's configuration (a fused instance, or the
 *             tile kernel of the block-sparse + tile path)
 *   what = 8: how it was chosen: 0 default, 1 timed by the autotuner on the first
 *             batched exchange_matrix_all, 2 read from the EXC_TUNE_CACHE file
 *   what = 9: bytes of the block-sparse workspace of the block-sparse + tile path
 *             (written once and read once per exchange_matrix_all on that path)
 *   what = 10: 1 if the fused kernel serves the batched path, else 0
 *   what = 4: algorithmic HBM bytes of one exchange_matrix_all
 *             (M read once, v(q) read once, Vx written once)
 *   what = 11: duration (ms, HIP events) of the lattice-sum kernel of the last
 *              exchange_gamma_term; what = 12: its number of terms
 *   what = 13: duration (ms, HIP events) of the product kernel of the last
 *              exchange_back_transform (waits for it)
 *   what = 14: how the fused kernel's work is split into items: 0 one item per (k, q)
 *              pair, 1 one per (pair, n'' chunk), 2 one per (pair, n'' chunk, row part)
 *              -- the block-sparse rows, or one dense row block (what = 19 rows); 1 and 2
 *              are chosen by the autotuner when few pairs leave the GPU short of work
 *              (one launch per k: at least 1)
 *   what = 15..18: how the reduced-precision main kernel accumulates the band
 *              contraction in binary32 (for error models; -1 in FP64 and for the
 *              unbatched GEMM form): 15 = band tiles per n'' pass; 16 = chain kind,
 *              0: one accumulator chain per work item, 1: one per row chunk of a pass,
 *              added into the item's binary32 partial, 2: one per n'' pass, added
 *              likewise, 3: a work item per n'' pass and row chunk (unbatched path);
 *              17 / 18 = rows per chunk in the block-sparse / dense rows
 *   what = 19: rows of a dense row block of the fused kernel (-1 without it)
 *   what = 5, 6, 7: see exchange_timing
 */
exc_status exchange_query(const exc_ctx *ctx, int32_t what, double *value);

/*
 * Autotuning (reduced-precision Cholesky/HERK contexts, batched path): the first
 * exchange_matrix_all times every main-kernel configuration that can serve the
 * context and the element type of M (fused instances with enough band tiles; for
 * complex64 M also the wide instances for large pairs; the block-sparse + tile
 * kernels; then, when the (k, q) pairs number fewer than 8 per CU, the fused
 * instances again with a work item per n'' chunk) on the caller's own inputs: one
 * untimed run, one timed run (a candidate more than twice as slow as the best so far
 * stops there) and five more timed runs, keeping the fastest (later candidates must
 * win by more than 3 %). Environment: EXC_TUNE=0
 * keeps the default choice; EXC_TUNE_CACHE=<file> looks the choice up / appends
 * it under a key of the problem's sizes; EXC_FUSED_CFG=<id> fixes a fused
 * instance (EXC_FUSED_SPLIT=1: an item per n'' chunk) and EXC_FUSED=0 the
 * block-sparse + tile path (neither is then tuned); EXC_SPARSE_NCW=1|2|4 fixes the
 * columns each wavefront of the block-sparse kernel takes (HERK form); EXC_GRAPH=1
 * replays the batched launch from a HIP graph instead of enqueueing its kernels.
 */

/*
 * exchange_timing -- live kernel timing of the batched exchange_matrix_all
 * path for benchmarks. n_slots > 0: events are recorded around the block-sparse
 * kernel and the tile kernel (event-record nodes of the next captured graph with
 * EXC_GRAPH=1), and each call records into its own slot of a pool of n_slots
 * event triples (the last n_slots calls are kept). n_slots = 0 switches timing
 * off. Both synchronise the device and drop the current graph. Read the means with
 * exchange_query: what = 5 tile kernel ms, 7 sparse kernel ms, 6 replays timed.
 */
exc_status exchange_timing(exc_ctx *ctx, int32_t n_slots);

/* ==========================================================================
 * Learned V^x extrapolator (extension of the nested self-consistency scheme
 * of Sec. IV, where V^x stays fixed between outer steps). V^x is linear in the
 * density matrix for fixed projections M, so between exact evaluations the
 * change dV(k) is predicted from the change dP of the density matrix by a
 * small network; the exact path stays the fallback and the judge.
 *
 * Network: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3, all
 * FP32; parameters flat as [W1 (hidden x in), b1, W2 (hidden x hidden), b2,
 * W3 (out x hidden), b3], row-major. Loss: mean squared error over samples and
 * outputs. Training: full-batch Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias
 * correction), one step per epoch. Samples are rows: X is n x in, Y is n x out.
 * The network belongs to the context (one per context) and lives on its GPU.
 * ========================================================================== */

/* exchange_nn_init -- create (or replace) the context's network. Weights are
 * (2u - 1)/sqrt(fan_in) with u the top 53 bits / 2^53 of output number
 * (flat index) of the SplitMix64 stream started at seed; biases 0; Adam state
 * zero. EXC_EINVAL for sizes < 1 or beyond 65536 (hidden: 8192, out: 2^20). */
exc_status exchange_nn_init(exc_ctx *ctx, int32_t in_dim, int32_t hidden, int32_t out_dim, uint64_t seed);

/* exchange_nn_params -- copy the n parameters out (set = 0) or in (set = 1;
 * also resets the Adam state). params is a host (on_device = 0) or device
 * pointer; n must equal the parameter count, else EXC_EINVAL. */
exc_status exchange_nn_params(exc_ctx *ctx, float *params, int64_t n, int32_t set, int32_t on_device);

/* exchange_nn_train -- epochs full-batch Adam steps on (X, Y), n samples; X, Y
 * host or device (on_device) FP32 rows. One epoch is a HIP graph replayed per
 * step. *loss_out (may be NULL) = the loss of the last step's forward pass.
 * Synchronous. EXC_ESTATE before exchange_nn_init. */
exc_status exchange_nn_train(exc_ctx *ctx, const float *X, const float *Y, int32_t n, int32_t epochs,
                             float lr, int32_t on_device, float *loss_out);

/* exchange_nn_grad -- the loss and its gradient with respect to the flat
 * parameters (same layout) at the current parameters, without an update.
 * grad_out host or device (on_device). Synchronous. */
exc_status exchange_nn_grad(exc_ctx *ctx, const float *X, const float *Y, int32_t n, int32_t on_device,
                            float *grad_out, float *loss_out);

/* exchange_nn_predict -- Y_out (n x out) = network(X). Host pointers: the
 * call returns when Y_out is written. Device pointers with a stream: ordered
 * on that stream, asynchronous. */
exc_status exchange_nn_predict(exc_ctx *ctx, const float *X, int32_t n, float *Y_out, int32_t on_device,
                               void *stream);

/* exchange_nn_features -- input encoding of a density-matrix change. P_new,
 * P_old: device arrays of n_real doubles (the complex n_b x n_b matrices of
 * every k', column-major, real and imaginary parts interleaved, k' outermost).
 * With v = P_new - P_old: x_out[i] = sum_j S_ij v_j / |v| (device, m floats,
 * zero if v = 0), S_ij = -1/sqrt(m) if the top bit of SplitMix64(seed) output
 * number i*n_real + j is set, else +1/sqrt(m); *norm_out (device double) =
 * |v|. 1 <= m <= 128. Asynchronous on stream (NULL: the context's stream,
 * synchronous). */
exc_status exchange_nn_features(exc_ctx *ctx, const double *P_new, const double *P_old, int64_t n_real,
                                uint64_t seed, int32_t m, float *x_out, double *norm_out, void *stream);

/* exchange_eigh -- eigen-decomposition of one Hermitian n_b(k) x n_b(k)
 * complex128 column-major matrix per k of the context (A_k: host array of n_k
 * device pointers; the Hermitian part is used). w_out: device, the ascending
 * eigenvalues packed k after k (sum n_b(k) doubles); Z_out: device, the
 * eigenvectors as columns, packed (sum n_b(k)^2 complex128). FP64 cyclic
 * Jacobi (off-diagonal norm below 1e-14 of the norm). n_b <= 256, else
 * EXC_EUNSUPPORTED. */
exc_status exchange_eigh(exc_ctx *ctx, const void *const *A_k, double *w_out, void *Z_out, void *stream);

/* exchange_nn_project -- output encoding: with B_k the first n_blk columns of
 * Z_k (as packed by exchange_eigh) and H = B_k^H (Va_k - Vb_k) B_k,
 * y_out[k][i*n_blk + j] = scale * Re H_ij (i <= j) and y_out[k][j*n_blk + i] =
 * scale * Im H_ij (i < j); y_out device, n_k * n_blk^2 floats. Va_k, Vb_k: host
 * arrays of device pointers to n_b(k)^2 complex128. Requires n_blk <= n_b(k)
 * and n_b * n_blk <= 4096 (EXC_EUNSUPPORTED). */
exc_status exchange_nn_project(exc_ctx *ctx, const void *const *Va_k, const void *const *Vb_k, const void *Z,
                               int32_t n_blk, double scale, float *y_out, void *stream);

/* exchange_nn_expand -- prediction: Vout_k = Vanchor_k + scale * B_k H_k B_k^H
 * with H_k decoded from y (device, layout of exchange_nn_project). Vout_k may
 * alias Vanchor_k. */
exc_status exchange_nn_expand(exc_ctx *ctx, const void *const *Vanchor_k, const void *Z, int32_t n_blk,
                              const float *y, double scale, void *const *Vout_k, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* EXCHANGE_H */
