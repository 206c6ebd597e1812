/*
 * floquet.h -- C ABI of the MI355X (gfx950) Floquet brickwork engine.
 *
 * The engine applies the Floquet unitary of a driven open spin chain,
 * |psi(nT)> = U_F^n |psi(0)>  (arXiv:2111.08044, Sec. III A, Eq. (3)),
 * where one period is two brickwork layers of nearest-neighbour two-qubit
 * gates (Eq. (4)), and reads energy observables between periods (Sec. IV,
 * Eq. (10)-(11)).  Every step runs in HIP kernels on one GPU; the host code
 * only builds the 4x4 gate exponentials in FP64 and plans the passes.
 *
 * Conventions
 *   Sites j = 0..L-1; bond b joins sites (b, b+1), b = 0..L-2 (the paper's
 *   1-indexed bond k = b+1).  State: 2^L interleaved complex amplitudes,
 *   amplitude index x = sum_j bit_j 2^(L-1-j) (site 0 is the most
 *   significant bit, as psi_{b1...bL} in Sec. II).  A bond operator acts on
 *   the local index 2*bit_b + bit_{b+1}.
 *   Gate: G_b = exp(-i (T/2) h_b) with h_b the Hermitian bond Hamiltonian
 *   acting during a half period (the paper's U_k = exp(-i H_k T), Eq. (5), is
 *   h_b = 2 H_k).  Period: the gates of odd b first, then those of even b
 *   (the rightmost product of Eq. (4) acts first).  Energy observable
 *   H0 = sum_b h_b.
 *   Matrices are row-major 4x4 complex, stored as 16 (re, im) double pairs.
 *
 * Ownership
 *   The caller owns every device buffer passed in (state vectors, checkpoints,
 *   workspaces): contiguous, 2^L elements of the context's dtype, 256-byte
 *   aligned.  The library never frees them.  The library owns the context,
 *   its device gate tables and its small reduction scratch.
 *
 * Streams
 *   All device work is enqueued on the context's HIP stream (given at
 *   creation or by fl_set_stream), in call order.  Uploads of parameters
 *   (fl_set_bonds, fl_set_gates) and of initial-state tables (fl_init_state,
 *   fl_init_pairs) are copied on that stream from pinned staging buffers the
 *   context owns, so they take effect after every kernel enqueued before
 *   them and before every kernel enqueued after them; these calls return
 *   without waiting for the device (they block only when all four staging
 *   buffers still feed copies that have not run).  When fl_set_stream
 *   changes the stream, work enqueued afterwards waits for the work already
 *   enqueued on the previous stream.  Calls that return host values
 *   (fl_expect_energy, fl_overlap, fl_energy_spread, fl_grad) synchronise
 *   the stream before returning.  A dense variant rebuilds its window plans
 *   when the gates change and synchronises the stream then, before it frees
 *   the old ones.

 * Errors
 *   Every int-returning call returns FL_OK (0) or a negative code; arguments
 *   are validated before anything is enqueued, so on FL_EINVAL / FL_ESTATE
 *   nothing was launched.  fl_last_error() returns a thread-local message
 *   describing the last failure of the calling thread.  No C++ exception
 *   crosses this interface.
 */
#ifndef FLOQUET_H
#define FLOQUET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FL_OK 0
#define FL_EINVAL (-1) /* invalid argument */
#define FL_ENOMEM (-2) /* device or host allocation failed */
#define FL_EHIP (-3)   /* a HIP runtime call or launch failed */
#define FL_ESTATE (-4) /* called before the context was ready (e.g. no bonds set) */
#define FL_ENODEV (-5) /* no usable gfx950 device */

#define FL_C64 0  /* complex64 state (FP32 arithmetic) */
#define FL_C128 1 /* complex128 state (FP64 arithmetic) */

#define FL_PLAIN 0           /* fused 4x4 gate sweep on the vector ALUs */
#define FL_DENSE6_FP32 1     /* 6-qubit windows pre-multiplied, FP32 MFMA (complex64 only) */
#define FL_DENSE6_BF16X3 2   /* 6-qubit windows pre-multiplied, split-BF16x3 MFMA, FP32 accumulation */
#define FL_DENSE4_FP32 3     /* 4-qubit windows pre-multiplied, FP32 MFMA (complex64, L >= 13) */

typedef struct fl_ctx fl_ctx;

/* Create a context for chains of L sites.  dtype: FL_C64 (L in [2, 34]) or
 * FL_C128 (L in [2, 33]); variant: FL_PLAIN, or a dense variant (FL_C64 only).
 * hip_stream: a hipStream_t (NULL = the default stream).  On success *ctx
 * receives a new context owned by the caller (release with fl_destroy).
 * Errors: FL_EINVAL (bad L, dtype, variant or ctx == NULL), FL_ENODEV,
 * FL_ENOMEM, FL_EHIP. */
int fl_create(fl_ctx **ctx, int L, int dtype, int variant, void *hip_stream);

/* Release a context and its device memory.  NULL is accepted (no-op). */
int fl_destroy(fl_ctx *ctx);

/* Make later calls enqueue their work on hip_stream. */
int fl_set_stream(fl_ctx *ctx, void *hip_stream);

/* Set the bond Hamiltonians and the period (Sec. III A, Eq. (5)).
 * h: host array [L-1][4][4] complex (double re, im), each Hermitian.
 * T: drive period (> 0).  Builds G_b = exp(-i (T/2) h_b) and G_b^dagger in
 * FP64 on the host and uploads them rounded to the context's precision, in
 * stream order (see Streams).
 * Errors: FL_EINVAL (NULL, non-finite or non-Hermitian h, T <= 0), FL_EHIP. */
int fl_set_bonds(fl_ctx *ctx, const double *h, double T);

/* Test hook: install FP64 gates G [L-1][4][4] (complex) and, optionally, the
 * bond Hamiltonians h [L-1][4][4] used by the energy (h may be NULL, then
 * fl_expect_energy reports <H0> = 0).  The period is recorded as T (used only
 * by fl_grad).  Errors: FL_EINVAL (NULL G, non-finite entries, a gate with
 * max |G^dagger G - I| > 1e-10, a non-Hermitian h), FL_EHIP. */
int fl_set_gates(fl_ctx *ctx, const double *G, const double *h, double T);

/* Write the product state psi[x] = prod_j s_j[bit_j(x)] (the form of the
 * initial state of Sec. IV, Eq. (9)), computed in FP64 and rounded.
 * psi: device, 2^L amplitudes of the context dtype.  spinors: host
 * [L][2] complex (double re, im), site-major.  Asynchronous: the factor
 * tables go through a staging buffer (see Streams), the host does not wait.
 * Errors: FL_EINVAL (NULL, misaligned or non-device psi, non-finite
 * spinors), FL_EHIP. */
int fl_init_state(fl_ctx *ctx, void *psi, const double *spinors);

/* Write the pair-product state of Sec. IV, Eq. (9): the sites (2m, 2m+1)
 * carry the two-site state pairs[m], so that
 *   psi[x] = prod_m pairs[m][2 bit(site 2m) + bit(site 2m+1)]
 * (the paper's initial state is the ground state of every odd-k term, i.e.
 * pairs[m] = ground state of h_{2m}; see fl_host_ground_states).  For odd L
 * the last site is unpaired and carries the spinor tail.  FP64, rounded.
 * psi: device, 2^L amplitudes of the context dtype.  pairs: host [L/2][4]
 * complex; tail: host [2] complex, required for odd L, ignored for even L.
 * Errors: FL_EINVAL (NULL, non-finite), FL_EHIP.  Asynchronous, as
 * fl_init_state. */
int fl_init_pairs(fl_ctx *ctx, void *psi, const double *pairs, const double *tail);

/* psi <- U_F^n psi (dagger = 0) or psi <- (U_F^dagger)^n psi (dagger = 1),
 * in place (Sec. III A, Eq. (3)-(4); the time-reversed evolution of the echo
 * of Sec. V).  n_periods >= 0.  Asynchronous. */
int fl_apply_period(fl_ctx *ctx, void *psi, int64_t n_periods, int dagger);

/* Energy of psi (Sec. IV, Eq. (10)): out[0] = <psi|H0|psi>,
 * out[1] = <psi|psi> (un-normalised), both FP64.  If rdm is not NULL it
 * receives the bond reduced density matrices
 * rho_b[i][j] = sum_rest psi_{..i..} conj(psi_{..j..}) as [L-1][4][4] complex.
 * Reductions: FP64 accumulation, deterministic order.  Synchronises. */
int fl_expect_energy(fl_ctx *ctx, const void *psi, double out[2], double *rdm);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the energy
 * readout of fl_expect_energy with every result left on the device and no
 * allocation and no host synchronisation in the call.
 *   out  device, 2 doubles: out[0] = <psi|H0|psi>, out[1] = <psi|psi>
 *   rdm  device, NULL or [L-1][4][4] complex doubles (the bond density
 *        matrices, as fl_expect_energy)
 * Both are written by kernels on the context stream; the call returns at
 * once.  The reduction partials live in a static 4 MiB device array (one per
 * GPU, kept until the process ends, set up by fl_create), sized for at least
 * 256 reduction workgroups: chains with (257 * 16 L) doubles > 4 MiB are
 * rejected with FL_EINVAL (no L <= 34 is).  All calls on one GPU share that
 * array, so calls that overlap on one GPU (two streams, two threads) race;
 * nothing in it needs clearing, each call writes every value it reads.
 * Errors: FL_EINVAL (bad psi, out or rdm not 8-byte aligned device memory,
 * another device current), FL_ESTATE (no bond Hamiltonians), FL_EHIP. */
int fl_expect_energy_noalloc(fl_ctx *ctx, const void *psi, double *out, double *rdm);

/* Energy spread (Sec. IV, Eq. (11)) of psi: out[0] = <H0>, out[1] = <H0^2>
 * (= ||H0 psi||^2), out[2] = <psi|psi>, all un-normalised FP64.  ws: device
 * workspace of 2^L amplitudes of the context dtype (receives H0 psi).
 * Synchronises. */
int fl_energy_spread(fl_ctx *ctx, const void *psi, void *ws, double out[3]);

/* Overlap of two states of the context's L (Eq. (1)): out[0] + i out[1] =
 * <phi|psi>, out[2] = <phi|phi>, out[3] = <psi|psi>, FP64 accumulation.
 * phi_dtype / psi_dtype: FL_C64 or FL_C128 each (mixed precision allowed).
 * Synchronises. */
int fl_overlap(fl_ctx *ctx, const void *phi, int phi_dtype, const void *psi, int psi_dtype, double out[4]);

/* Bytes of device workspace fl_grad needs (the adjoint state lambda):
 * 2^L amplitudes of the context dtype.  Returns a negative code on error. */
int64_t fl_grad_workspace_bytes(const fl_ctx *ctx);

/* Reverse-mode gradient of E_n = <psi_n|H0(theta)|psi_n>, psi_n = U_F^n psi_0,
 * with respect to per-bond parameters theta_{b,p} (dh_b/dtheta_{b,p} =
 * gens[b][p]) and the period T.
 *   psi_n     device, in: psi_n; clobbered (rebuilt backwards with G^dagger)
 *   ckpts     host array of n_periods/K device pointers: ckpts[s] = psi_{sK}
 *             (s = 0 .. n_periods/K - 1); psi is reset to ckpts[s] when the
 *             backward replay reaches period sK.  May be NULL if K == 0
 *             (pure G^dagger replay).
 *   n_periods >= 0; K >= 0 with K == 0 or n_periods % K == 0
 *   gens      host [L-1][P][4][4] complex, Hermitian generators
 *   lambda_ws device workspace of fl_grad_workspace_bytes()
 *   grad      host out, (L-1)*P + 1 doubles: d E_n / d theta_{b,p} at
 *             b*P + p, and d E_n / d T last.
 * The replay undoes the forward exactly up to arithmetic rounding when it
 * applies the adjoints of the very matrices the forward applied, so that a
 * reset from a checkpoint meets the state the replay reached.  The plain form
 * replays the FP32 gates' adjoints.  The 4-qubit-window form (complex64,
 * L >= 14) replays the adjoints of its FP32 window matrices, which matches
 * forwards run segment by segment as fl_apply_period(ctx, psi, K) (or one
 * fl_apply_period(n_periods) when K == 0).  The 6-qubit window forms (and
 * the 4-qubit one at L = 13) replay gate by gate; with K > 0 their dE/dT
 * carries ~1e-3 (FP32 windows) to ~1e-2 (split-BF16x3) relative error, so
 * take their gradients with K == 0.
 * Synchronises. */
int fl_grad(fl_ctx *ctx, void *psi_n, void *const *ckpts, int64_t n_periods, int64_t K, const double *gens, int P,
            void *lambda_ws, double *grad);

/* Thread-local description of the last error of the calling thread. */
const char *fl_last_error(void);

/* ---- host-only helpers (no device work; usable without a GPU) ---------- */

/* XYZ-plus-fields bond Hamiltonians:
 * h_b = Jx XX + Jy YY + Jz ZZ + (1/2) f_b.sigma (x) I + (1/2) I (x) f_{b+1}.sigma.
 * J: [L-1][3], fields: [L][3], h_out: [L-1][4][4] complex. */
int fl_xyz_bonds(int L, const double *J, const double *fields, double *h_out);

/* The FP64 gates the library builds: G_out[b] = exp(-i (T/2) h[b]), [n][4][4] complex. */
int fl_host_gates(int nbonds, const double *h, double T, double *G_out);

/* Ground states of n two-site Hamiltonians h [n][4][4] (complex, Hermitian):
 * g_out[k] = the eigenvector of the lowest eigenvalue of h[k] ([n][4]
 * complex, unit norm, largest component real and positive), e_out[k] (may
 * be NULL) = that eigenvalue.  FP64 Jacobi; errors: FL_EINVAL. */
int fl_host_ground_states(int n, const double *h, double *g_out, double *e_out);

/* d/dtheta exp(-i (T/2) h(theta)) in direction gen (4x4 complex each). */
int fl_host_gate_derivative(const double *h, const double *gen, double T, double *dG_out);

/* Generators of the XYZ couplings: gens_out[b][a] = d h_b / d J^a_b =
 * sigma^a (x) sigma^a (a = x, y, z), as [L-1][3][4][4] complex. */
int fl_xyz_generators(int L, double *gens_out);

/* Amplitude index of tile-local element j of tile t for window start h, for
 * the tile geometry of the plain sweep of dtype (complex64: 4 low bits and a
 * 9-bit window; complex128: 6 low bits and a 6-bit window; a single tile when
 * L is at most the tile size) (out: 2^L uint64 values, out[t * 2^K + j]).
 * Returns FL_EINVAL for L > 24 or an invalid window. */
int fl_tile_map(int L, int dtype, int h, uint64_t *out);

/* The window matrix a dense plan applies for one register group:
 * U = E(op_{n-1}) ... E(op_0), E(op_k) = the 4x4 gate G[k] ([nops][4][4]
 * complex) embedded at window bits (pos[k], pos[k]+1), window index bit i =
 * tile bit u0 + i, gate local index 2*bit(pos+1) + bit(pos).
 * mode -1, 0, 1: 6-bit window, U_out [64][64] complex; if frag_out is not
 * NULL it receives the MFMA fragments of the real 128x128 form: mode 0, 64 KiB
 * of FP32; mode 1, 32 KiB of bf16 hi/lo (Re, Im) pairs of U, each stored once
 * (the kernel forms the rows (Re, -Im) and (Im, Re)).  mode 2: 4-bit window, U_out [16][16]
 * complex, frag_out (if not NULL) the 4 KiB of FP32 fragments of the real
 * 32x32 form. */
int fl_host_window_matrix(const double *G, const int *pos, int nops, int mode, double *U_out, void *frag_out);

/* The overlap terms of the reverse pass for one 4-bit register group, from
 * its window overlap Q[x][y] = sum_r psi_{r,x} conj(lambda_{r,y}) ([16][16]
 * complex, taken before the group's first op; window index bit i = tile bit
 * u0 + i) and its ops: op k applies G[k] ([nops][4][4] complex, local index
 * 2 bit(pos+1) + bit(pos)) on window bits (pos[k], pos[k]+1), pos in [0, 2].
 * out[k][16]: the 16 reals of the op's bond at the state before its gate,
 * [0..3] = Im(conj(lambda_l) psi_l), then (re, im) of
 * sum conj(lambda_l) psi_m - conj(psi_l) lambda_m for the local index pairs
 * 01, 02, 03, 12, 13, 23 (the anti-Hermitian part of the bond's overlap
 * matrix, which the gradient of Sec. V's reverse replay needs).  FP64. */
int fl_host_window_overlaps(const double *Q, const double *G, const int *pos, int nops, double *out);

/* The plan fl_apply_period would run for n periods (kind 0 = sweep,
 * 1 = reverse sweep of the gradient, 2 = energy / density-matrix cover on
 * 12-bit tiles (complex128, and complex64 with L <= 13), 3 = cover used for
 * H0 psi by a plain-sweep context, 4 = dense 6-qubit-window sweep, 5 = dense 4-qubit-window sweep,
 * 6 = energy / density-matrix cover of complex64 states with L >= 14: 13-bit
 * tiles, bonds packed into 5-bit register groups), flattened as int32:
 * [C, W, R, npasses, {h, ngroups, flags, {u0, nops, {i, gate, slot}*}*}*].
 * Writes at most cap words to buf (may be NULL) and the required count to
 * *needed. */
int fl_plan_query(int L, int dtype, int kind, int64_t n_periods, int dagger, int32_t *buf, int64_t cap,
                  int64_t *needed);

#ifdef __cplusplus
}
#endif

#endif /* FLOQUET_H */
