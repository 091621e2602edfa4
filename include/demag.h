/*
 * demag.h -- C ABI of the MI355X (gfx950) stray-field library.
 *
 * Computes the collocated scalar potential and demagnetizing field of a
 * cell-wise constant magnetization on a uniform tensor grid with the separable
 * (Kronecker-product) sinc-quadrature operator of Exl et al., "FFT-based
 * Kronecker product approximation to micromagnetic long-range interactions"
 * (arXiv 1212.3509): Cor. kron_op, Eq. (kron_operator), with the Toeplitz
 * (convolution) structure of Sec. 4.2, Eqs. (conv_op)-(conv_pot).
 *
 * Conventions shared by every entry point
 *   - Physical sign: phi(x) = 1/(4 pi) int m(y).(x - y)/|x - y|^3 dy and
 *     h = -grad phi (Eq. (intop2) with the sign obtained by integrating
 *     Eq. (intop1) by parts).  A uniformly magnetized cube has h = -m/3 at its
 *     centre.
 *   - Full-format arrays are dense, x fastest: m[3][nz][ny][nx],
 *     phi[nz][ny][nx], h[3][nz][ny][nx] (component index first).
 *   - The field is the exact derivative of the separable potential with
 *     respect to the target point (not the finite differences of Sec. 4).
 *   - Device pointers are HIP device addresses on the context's device; host
 *     pointers are ordinary process memory.  The caller owns every buffer it
 *     passes; the library owns its handles and internal workspace.
 *   - All GPU work is enqueued on the context's stream and returns before it
 *     completes (the caller synchronizes).  Host outputs documented as such are
 *     complete on return.
 *   - Every call returns a status; arguments are validated before anything is
 *     launched, and on error nothing has been enqueued (except the Tucker-route
 *     calls, whose ranks are decided as they run: a failure there, e.g. a rank
 *     above rmax, comes after their GPU work has finished, with the outputs
 *     untouched).  demag_last_error() gives a message for the calling thread's
 *     last failure.
 */
#ifndef DEMAG_H
#define DEMAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DEMAG_OK = 0,
  DEMAG_E_INVAL = 1,        /* argument out of its documented range */
  DEMAG_E_NOMEM = 2,        /* device or host allocation failed */
  DEMAG_E_HIP = 3,          /* HIP runtime error */
  DEMAG_E_UNSUPPORTED = 4,  /* valid request this build does not support */
  DEMAG_E_ACCURACY = 5      /* no quadrature rule met the requested tolerance
                               (outputs hold the best rule found; see
                               demag_quad_predict) */
} demag_status;

/* Arithmetic of the mode products.  Factor assembly is always FP64.
 *   DEMAG_FP64    FP64 inputs/outputs, FP64 matrix-core products.
 *   DEMAG_FP32    FP32 inputs/outputs, FP32 matrix-core products.
 *   DEMAG_BF16X2  FP32 inputs/outputs; each operand split into two bfloat16
 *                 parts (hi, lo), products hi*hi + hi*lo + lo*hi accumulated
 *                 in FP32.
 *   DEMAG_BF16X3  as BF16X2 with a third part; six products, FP32 accumulate. */
typedef enum {
  DEMAG_FP64 = 0,
  DEMAG_FP32 = 1,
  DEMAG_BF16X2 = 2,
  DEMAG_BF16X3 = 3
} demag_prec;

/* Uniform tensor grid (Sec. 3.1): n[d] cells of size h[d] along x, y, z.
 * Requires 1 <= n[d] <= 4096 and h[d] > 0. */
typedef struct {
  int32_t n[3];
  double h[3];
} demag_grid;

/* Quadrature rule (Sec. 3.3, Cor. kron_op).  Nodes t_k = k*theta, k = 1..M,
 * tau_k = sinh t_k, weights alpha_k = 2 theta cosh t_k sinh^2 t_k (the folded
 * +-k pair of the symmetric sinc rule); the weight of node k in the potential
 * kernel is alpha_k / (2 pi^(3/2)).
 *   step_rule 0: theta = c0 ln(M)/M (Cor. kron_op; c0 = 2.15 in Sec. 3.5);
 *   step_rule 1: theta = ln(2 pi a M / b)/(a M) with a = 2, b = rho_min/4,
 *                rho_min = (h_min/2)^2 (Thm. sinc_theo), in the scaled domain.
 * If t and alpha are both non-NULL they give an explicit rule instead (host
 * arrays of length M, t_k > 0), e.g. a shortened learned rule.
 * The grid is scaled so its longest edge is 1 before the rule is applied
 * (Sec. 3.5); the potential is scaled back, the field is scale-free.
 * Requires 1 <= M <= 256. */
typedef struct {
  int32_t M;
  double c0;
  int32_t step_rule;
  const double *t;
  const double *alpha;
} demag_quad;

typedef struct demag_ctx demag_ctx;          /* opaque: device, stream, workspace */
typedef struct demag_factors demag_factors;  /* opaque: assembled 1D factors */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream). */
demag_status demag_create(int device, void *hip_stream, demag_ctx **out);
/* Release the context and its workspace (waits for the stream first). */
demag_status demag_destroy(demag_ctx *ctx);
/* Change the stream later calls enqueue on.  Work enqueued afterwards waits
 * for the work already enqueued on the previous stream (an event recorded
 * there), since both share the context's workspace. */
demag_status demag_set_stream(demag_ctx *ctx, void *hip_stream);
/* Input check (default off).  When on, demag_apply_full(_ws), demag_apply_fft,
 * demag_batch_apply and the structured applies first scan their input
 * magnetization / columns on the device and return DEMAG_E_INVAL, enqueueing
 * nothing else, if any value is NaN or infinite.  The scan synchronizes the
 * stream, so calls no longer return before the GPU work completes. */
demag_status demag_set_input_check(demag_ctx *ctx, int32_t enable);
/* Upper bound in bytes of the internal workspace of demag_apply_full (the
 * node loop is split into chunks that fit).  Default 16 GiB. */
demag_status demag_set_workspace_limit(demag_ctx *ctx, size_t bytes);
/* Tile shape of the full-format mode products: `rows` = 16-row blocks per
 * tile (1, 2, 4 or 8; 0 = chosen from the axis length), `cols` = 64-column
 * blocks per bfloat16 tile (1 or 2; 0 = automatic).  Results do not depend
 * on the shape.  DEMAG_E_INVAL for other values. */
demag_status demag_set_tiles(demag_ctx *ctx, int32_t rows, int32_t cols);
/* Message of the calling thread's most recent failure ("" if none). */
const char *demag_last_error(void);

/* Assemble the 1D factors of Cor. kron_op / Eq. (conv_pot) for every axis,
 * factor type and node, in FP64 on the GPU (erf/erfc differences, expm1
 * forms; Eq. (f_anal) and Sec. 4.2), plus their FP32 and bfloat16-split
 * copies.  Layout per axis d: [type][k][J + n_d - 1], J = -(n_d-1)..n_d-1,
 * types 0 = E~, 1 = X~, 2 = P~ = -X'~, 3 = Q~ = -E'~ = 2 tau^2 X~, each scaled
 * by w_k = (alpha_k / (2 pi^(3/2)))^(1/3) and computed in the scaled domain
 * (the potential's length factor is applied by the apply calls), where
 *   E(J)  = int_a^b exp(-tau^2 x^2) dx,  X(J) = int_a^b x exp(-tau^2 x^2) dx,
 *   X'(J) = b exp(-tau^2 b^2) - a exp(-tau^2 a^2),  [a, b] = [(J-1/2)h, (J+1/2)h].
 * On success *out is a new handle (free with demag_factors_free); the
 * assembly is enqueued on the context's stream. */
demag_status demag_assemble_factors(demag_ctx *ctx, const demag_grid *grid,
                                    const demag_quad *quad, demag_factors **out);
/* Factors of a non-uniform tensor-product grid (collocation at cell centres
 * and Lemma sinc_mumag hold for any partition; the factors lose the Toeplitz
 * structure).  edges[d]: n[d] + 1 strictly increasing cell boundaries
 * (host, physical units), 1 <= n[d] <= 1024.  The grid is scaled so that its
 * longest extent is 1 (the potential is scaled back); the theorem-step rule
 * uses the smallest scaled cell.  Factors are dense n x n matrices per type
 * and node, entry (i, j) integrating over source cell j seen from the centre
 * of cell i: E, X, P = -X', Q = 2 tau^2 X as for uniform grids, in FP64,
 * as an FP32 copy rounded once from them and as three bfloat16 parts of
 * that copy.  Such factors serve demag_apply_full in every precision (dense
 * mode products on the matrix cores: FP64, FP32, or split bfloat16 products
 * accumulated in FP32); the FFT, structured and batched paths need uniform
 * grids and reject them.
 * demag_factors_download returns [4][M][n][n]. */
demag_status demag_assemble_factors_grid(demag_ctx *ctx, const int32_t n[3], const double *const edges[3],
                                         const demag_quad *quad, demag_factors **out);
/* Waits for the last work enqueued (on any context) that reads f, then frees it. */
demag_status demag_factors_free(demag_factors *f);
/* Length scale L of the factor set: the longest grid extent, by which the
 * grid was scaled to unit size.  The full-format and FFT applies multiply the
 * potential by L themselves; the structured results are in the scaled domain,
 * so the potential of a structured result is L times its sum of terms (the
 * field is scale-free and needs no factor). */
demag_status demag_factors_length_scale(const demag_factors *f, double *L);
/* Number of nodes M of an assembled rule. */
demag_status demag_factors_count(const demag_factors *f, int32_t *M);
/* Host copies (length M) of t_k, tau_k and alpha_k in the scaled domain; any
 * pointer may be NULL. */
demag_status demag_factors_nodes(const demag_factors *f, double *t, double *tau,
                                 double *alpha);
/* Copy the FP64 factor table of axis d (0..2), [4][M][2 n_d - 1] doubles, to
 * host memory `dst`.  Synchronizes the context's stream. */
demag_status demag_factors_download(demag_ctx *ctx, const demag_factors *f, int32_t d,
                                    double *dst);

/* Full-format apply of the same separable operator by 3D FFT convolution
 * (Sec. 4.2's route for unstructured tensors): the kernel's 3D spectrum is
 * the sum over nodes of products of the 1D factor spectra (formed once per
 * factor set, 9 x Lz x Ly x (Lx/2+1) FP64 values, L_d = 2^p >= 2 n_d - 1);
 * each apply runs forward real/complex FFTs of m, the pointwise products and
 * the inverse FFTs, all FP64.  m: device [3][nz][ny][nx] FP64; phi: device
 * [nz][ny][nx]; h: device [3][nz][ny][nx] (FP64, non-overlapping).  Uses the
 * context workspace (4 x Lz x Ly x (Lx/2+1) complex values).  n <= 1024 per
 * axis, else DEMAG_E_INVAL. */
demag_status demag_apply_fft(demag_ctx *ctx, demag_factors *f, const double *m, double *phi, double *h);

/* Full-format apply, path (a): for every node, the 23 mode products of
 * Eq. (modemul) (6 along z, 9 along y, 8 along x, sharing partial products
 * between outputs), accumulated over nodes into
 *   phi = sum_k sum_q  m_q x_x F x_y F x_z F        (potential, Eq. (kron_operator))
 *   h_p = sum_k sum_q  (the same with axis p's factor differentiated).
 * m: device, [3][nz][ny][nx], FP64 if prec == DEMAG_FP64 else FP32.
 * phi: device [nz][ny][nx] or NULL; h: device [3][nz][ny][nx] or NULL (at
 * least one non-NULL), same element type as m.  Buffers must not overlap and
 * must be 16-byte aligned.  The grid is the one the factors were assembled
 * for; n <= 1024 per axis (the bfloat16 factor windows and the LDS-staged
 * factor rows are sized for it), else DEMAG_E_INVAL. */
demag_status demag_apply_full(demag_ctx *ctx, const demag_factors *f, demag_prec prec,
                              const void *m, void *phi, void *h);
/* Workspace of demag_apply_full(_ws) in bytes: *one_chunk runs the whole
 * node loop per stage launch ((12 M + 4) N elements of the precision's
 * element type: the per-node intermediates of the z and y stages plus four
 * scratch outputs), *minimum one node at a time ((12 + 4) N elements).
 * Either pointer may be NULL.  Host-only; enqueues nothing. */
demag_status demag_apply_full_workspace_size(const demag_factors *f, demag_prec prec, size_t *one_chunk,
                                             size_t *minimum);
/* demag_apply_full on a caller-owned device workspace of workspace_bytes
 * (16-byte aligned, at least the *minimum above, else DEMAG_E_NOMEM): the node
 * loop runs in the largest chunks that fit.  The workspace must not be used
 * by other work until this call's kernels complete (stream order). */
demag_status demag_apply_full_ws(demag_ctx *ctx, const demag_factors *f, demag_prec prec, const void *m,
                                 void *phi, void *h, void *workspace, size_t workspace_bytes);

/* ---------------------------------------------------------------- batches
 * Many states on uneven grids (same quadrature rule), FP64 or FP32.  All
 * states' intermediate products are formed by one persistent launch per
 * mode-product stage (a fixed, cost-sorted list of tiles walked by a fixed
 * set of workgroups: no atomics, reproducible), node chunks sized to the
 * context's workspace limit.  Fields are packed state after state:
 *   m   = concat_s m_s[3][nz][ny][nx],   phi = concat_s phi_s[nz][ny][nx],
 *   h   = concat_s h_s[3][nz][ny][nx];
 * state s starts at 3*off[s] in m and h and at off[s] in phi, with the
 * cell offsets off[] from demag_batch_offsets.  1 <= n <= 1024 per axis. */
typedef struct demag_batch demag_batch;
demag_status demag_batch_create(demag_ctx *ctx, int32_t count, const demag_grid *grids,
                                const demag_quad *quad, demag_prec prec, demag_batch **out);
demag_status demag_batch_free(demag_batch *b);
/* off: host array of count + 1 cell offsets (off[0] = 0, off[count] = total). */
demag_status demag_batch_offsets(const demag_batch *b, int64_t *off);
/* Nodes per chunk, persistent workgroups per launch, and the algorithmic
 * FLOPs of one apply (dense Toeplitz products); any pointer may be NULL. */
demag_status demag_batch_info(const demag_batch *b, int32_t *node_chunk, int32_t *persistent_groups,
                              double *flops_per_apply);
/* Apply to device buffers m, phi, h (element type of the batch precision,
 * 16-byte aligned).  use_graph != 0: the launch sequence is captured once as a
 * HIP graph for these buffers and this stream and replayed on later calls. */
demag_status demag_batch_apply(demag_ctx *ctx, demag_batch *b, const void *m, void *phi, void *h,
                               int32_t use_graph);
/* Autotuner: times each candidate row-block shape (16, 32, 64 or 128 rows
 * per wave) of the stage kernel for every (axis length, outputs) class of the
 * batch on the device (reps launches each), keeps the fastest and rebuilds
 * the batch.  With path != NULL the choices are read from and merged into a
 * JSON object there ({"fp32/n96/nout2": 8, ...}); cached entries are not
 * re-timed.  Synchronizes the stream. */
demag_status demag_batch_tune(demag_ctx *ctx, demag_batch *b, const char *path, int32_t reps);

/* ---------------------------------------------------------------- path (b)
 * Structured inputs (Sec. 2, Eqs. (CP), (tucker_rep); App. C, Eq. (tt_3d_2)).
 * Applying the Kronecker operator to a structured tensor needs only the
 * Toeplitz products of its factor columns (Eqs. (kron_eval_cp),
 * (kron_eval_tuck)), computed here through zero-padded FFTs of length
 * L = 2^p >= 2 n_d - 1 (Sec. 4, Eq. (fft_pot)).  Columns are read and written
 * in FP32; `prec` sets the transforms: DEMAG_FP64 runs every transform and
 * product in FP64; DEMAG_FP32 runs the forward transforms of the input
 * columns in FP64 and the kernel spectra, products and inverse transforms (one
 * per output column) in FP32.  DEMAG_BF16X2/X3 give DEMAG_E_UNSUPPORTED (the
 * butterflies are no matrix-core contractions).  Axis lengths up to 4096.
 * Results are in the scaled domain: multiply the potential by the length
 * scale (demag_factors_length_scale).
 *
 * Column sets per axis d, all device FP32, one column contiguous:
 *   in[d]:  [3 components q][R_d][n_d]
 *   out[d]: [3 q][2 s][M][R_d][n_d]
 * Output column (q, s, k, l) = T_{d,type,k} in[d][q][l], where for the
 * component's own axis (d == q) type = X~ (s = 0) or P~ (s = 1), and on the
 * other axes type = E~ (s = 0) or Q~ (s = 1).  Slot s = 1 is the factor
 * differentiated for the field component along d.  The caller owns all
 * buffers; out must not overlap in. */
demag_status demag_prepare_structured(demag_ctx *ctx, demag_factors *f);
demag_status demag_apply_columns(demag_ctx *ctx, demag_factors *f, demag_prec prec, const int32_t R[3],
                                 const float *const in[3], float *const out[3]);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as demag_apply_columns with DEMAG_FP64, bit for bit, with the column spectra in a
 * static 64 MiB device array per GPU instead of the context workspace; no
 * hipMalloc, hipFree or other allocating call.  Limits: the column spectra,
 * 16 (L_d/2 + 1) bytes per input column (3 R_d columns on axis d), must fit
 * in 64 MiB - 256 bytes (e.g. 1020 columns at n = 4096), else DEMAG_E_INVAL
 * with the sizes in the message; the factors' kernel spectra must already
 * exist (demag_prepare_structured, which allocates them), else DEMAG_E_INVAL.
 * All calls on one GPU share its array, which keeps the last call's
 * contents: calls that overlap in time on one GPU (other streams, other
 * threads, other contexts) race.  With profiling enabled the library may
 * create timing events. */
demag_status demag_apply_columns_noalloc(demag_ctx *ctx, const demag_factors *f, const int32_t R[3],
                                         const float *const in[3], float *const out[3]);

/* CP input, rank r per component (weights pass through unchanged):
 * U[d] = [3 q][r][n_d] holds column l of U^{(q,d)}.  Result: out[d] as above
 * with R_d = r, and (if table != NULL) the host int32 term table
 * [4 outputs (phi, h_x, h_y, h_z)][3 M r terms][3 axes]: term (q, k, l),
 * index (q M + k) r + l, of output o uses column ((q 2 + s) M + k) r + l of
 * out[d] with s = 1 exactly when o is the field along d.  Output o is
 * sum over its terms of lambda^q_l out[x][.] o out[y][.] o out[z][.], times
 * the length scale L for the potential (o = 0). */
demag_status demag_apply_cp(demag_ctx *ctx, demag_factors *f, demag_prec prec, int32_t r, const float *const U[3],
                            float *const out[3], int32_t *table);
/* Tucker input, ranks r[3]: U[d] = [3 q][r_d][n_d].  Result out[d] with
 * R_d = r_d and the host block table [4][3 M blocks][3 axes]: block (q, k),
 * index q M + k, of output o is [[C^q; out[x] cols c_x..c_x+r_x-1, ...]]
 * with first columns c_d = ((q 2 + s) M + k) r_d. */
demag_status demag_apply_tucker(demag_ctx *ctx, demag_factors *f, demag_prec prec, const int32_t r[3],
                                const float *const U[3], float *const out[3], int32_t *table);
/* TT input with ranks (1, r1, r2, 1): G1 = [3 q][r1][n_x] (columns of G1),
 * G2 = [3 q][r1][r2][n_y] (fibres G2[a, :, b]), G3 = [3 q][r2][n_z] (rows of
 * G3).  As Tucker with R = (r1, r1 r2, r2); block table as for Tucker. */
demag_status demag_apply_tt(demag_ctx *ctx, demag_factors *f, demag_prec prec, int32_t r1, int32_t r2,
                            const float *G1, const float *G2, const float *G3,
                            float *const out[3], int32_t *table);

/* ---------------------------------------------------------------- recompression
 * Tolerance-controlled recompression of a CP tensor to Tucker form by HOOI
 * (Sec. 2.2, Alg. HOOI), for the CP results of demag_apply_cp: the tensor
 *   X = sum_t lam[t] c0[table[t][0]] o c1[table[t][1]] o c2[table[t][2]]
 * (mode p column sets cols[p] = [ncols[p]][n[p]] FP32, device; table int32
 * [T][3] and lam FP64 [T], device) becomes [[core; U0, U1, U2]] with
 * orthonormal factor rows U_p [ranks[p]][n[p]] and core [r0][r1][r2]
 * (index (a r1 + b) r2 + c), FP64, device buffers of capacity rmax rows and
 * rmax^3.  Rank rule per mode and sweep: the smallest r whose discarded
 * singular values of the projected unfolding have a norm of at most
 * eps / sqrt(3) of all of them, capped at rmax (1..64).  Sweeps stop when the
 * squared core norm changes by at most 1e-13 relative, or after max_sweeps.
 * Singular subspaces come from a randomized range finder with K = rmax + 8
 * candidates: omega = three Gaussian test matrices [K][n_p] one after another
 * (initial factors, Khatri-Rao test vectors), gmat = a Gaussian [K*K][K]
 * matrix (sweeps), FP64 device, supplied by the caller.  Host outputs: ranks,
 * *rel_err = |X - [[core; U]]|_F / |X|_F (computed without cancellation),
 * *sweeps.  Synchronizes the stream; uses the context workspace (about
 * 8 (T (n0 + n1 + n2) + 6 T^2) bytes).  Errors: DEMAG_E_INVAL for NULL
 * pointers, sizes out of range, table entries outside the column sets or a
 * zero tensor. */
demag_status demag_recompress_cp(demag_ctx *ctx, const int32_t n[3], int32_t T, const float *const cols[3],
                                 const int32_t ncols[3], const int32_t *table, const double *lam, double eps,
                                 int32_t rmax, int32_t max_sweeps, const double *omega, const double *gmat,
                                 double *const U[3], double *core, int32_t ranks[3], double *rel_err,
                                 int32_t *sweeps);

/* ---------------------------------------------------------------- Tucker route
 * The scalar potential of a Tucker magnetization by structured DFTs
 * (Sec. 4.2, Alg. scpot_fft_tucker), the approximate summation of Tucker
 * tensors and TT rounding (App. C).  FP64 throughout; every pointer in these
 * calls is device memory except the rank arrays (host).  Layouts: a Tucker
 * tensor is a core [r0][r1][r2] (index (a r1 + b) r2 + c) and factor rows
 * rows[p] [r_p][n_p] (row i = the i-th factor column of mode p, contiguous).
 * Each recompression is HOOI (Alg. HOOI) with the rank rule of
 * demag_recompress_cp (discarded singular values of norm at most
 * tol / sqrt(3) of all of them, per mode), on the core of the tensor in
 * orthonormal bases of its factor rows; a factor-row set whose span exceeds
 * 128 dimensions in one mode gives DEMAG_E_UNSUPPORTED.  The calls allocate
 * device memory for their intermediates, synchronize the context's stream
 * and return ranks above rmax as DEMAG_E_UNSUPPORTED with the needed ranks in
 * rout and the outputs untouched.  Potentials are in the factors' scaled units
 * (multiply by demag_factors_length_scale), as for the structured applies. */
typedef struct demag_ktucker demag_ktucker;
typedef struct {
  int32_t r[3];             /* ranks, 1..128 each */
  const double *core;       /* [r0][r1][r2] */
  const double *rows[3];    /* [r_p][n_p] */
} demag_tucker_in;

/* Set-up of Alg. scpot_fft_tucker for the uniform-grid factors f (mode sizes
 * 1..4096, at most 512 nodes): the three CP kernels of Eq. (conv_pot), one
 * term per node with the X generator on axis q and E generators elsewhere
 * (length 2 n_p - 1, offset J at J + n_p - 1), compressed to Tucker with tol
 * in (0, 1), and the DFTs of their factor rows (length L_p = the smallest
 * power of two >= 2 n_p - 1, Lemma DFT_tucker).  *out owns device memory
 * until demag_ktucker_free; f may be freed afterwards. */
demag_status demag_ktucker_create(demag_ctx *ctx, const demag_factors *f, double tol, demag_ktucker **out);
/* Ranks of the compressed kernel of component q (0..2). */
demag_status demag_ktucker_ranks(const demag_ktucker *kt, int32_t q, int32_t r[3]);
/* Copy of the compressed kernel q: core (r0 r1 r2 values) and factor rows
 * rows[p] ([r_p][2 n_p - 1]), device buffers of the caller. */
demag_status demag_ktucker_copy(demag_ctx *ctx, const demag_ktucker *kt, int32_t q, double *core,
                                double *const rows[3]);
demag_status demag_ktucker_free(demag_ktucker *kt);
/* The loop and the closing step of Alg. scpot_fft_tucker for the magnetization
 * components m[0..2] (mode sizes those of the kernels): per component the DFT
 * of the factor rows, the Hadamard product with the kernel in Fourier space
 * (App. B, Eq. (t_had2); kernel rank times magnetization rank at most 512 per
 * mode), the inverse DFT cut to the convolution window, the product
 * recompressed with tol; then the approximate summation of the three
 * products with tol.  Output: ranks rout, core (capacity rmax^3) and rows[p]
 * (capacity rmax n_p). */
demag_status demag_potential_tucker(demag_ctx *ctx, const demag_ktucker *kt, const demag_tucker_in m[3], double tol,
                                    int32_t rmax, int32_t rout[3], double *core, double *const rows[3]);
/* Approximate summation: sum_t terms[t] (1..512 terms, mode sizes n[p] in
 * 1..16384, at most 512 factor rows per mode in all) recompressed with tol. */
demag_status demag_tucker_sum(demag_ctx *ctx, const int32_t n[3], int32_t nterms, const demag_tucker_in *terms,
                              double tol, int32_t rmax, int32_t rout[3], double *core, double *const rows[3]);
/* TT rounding (App. C) of the 3D tensor train G1 [r1][n0] (rows: the columns
 * of the first core), G2 [r1][r2][n1] (fibres G2[a, :, b] contiguous), G3
 * [r2][n2], ranks 1..128, mode sizes 1..16384: the outer cores are
 * orthonormalised, then two truncated SVDs from the left each discard
 * singular values of norm at most tol / sqrt(2) times the tensor norm, so
 * the result is within tol of the input in relative Frobenius norm.  Outputs
 * in the same layout: ranks rout[2], G1o (capacity rmax n0), G2o (rmax^2 n1),
 * G3o (rmax n2). */
demag_status demag_tt_round(demag_ctx *ctx, const int32_t n[3], int32_t r1, int32_t r2, const double *G1,
                            const double *G2, const double *G3, double tol, int32_t rmax, int32_t rout[2],
                            double *G1o, double *G2o, double *G3o);
/* Conversions between the formats (App. C), same layouts.  CP -> TT: the
 * rank-R CP tensor sum_a lam[a] U0[a] o U1[a] o U2[a] (lam [R], U[p]
 * [R][n_p]) as a TT with ranks (R, R) and the diagonal middle core
 * G2[a][b][j] = (a == b) lam[a] U1[a][j]; outputs G1 [R][n0], G2 [R][R][n1],
 * G3 [R][n2] (round it with demag_tt_round).  Enqueued only. */
demag_status demag_cp_to_tt(demag_ctx *ctx, const int32_t n[3], int32_t R, const double *lam,
                            const double *const U[3], double *G1, double *G2, double *G3);
/* Tucker -> TT (Eq. (tt_3d_2) read backwards): G1 = rows[0] [r0][n0],
 * G2[a][c][j] = sum_b core[a][b][c] rows[1][b][j] ([r0][r2][n1]), G3 =
 * rows[2] [r2][n2].  Enqueued only. */
demag_status demag_tucker_to_tt(demag_ctx *ctx, const int32_t n[3], const demag_tucker_in *t, double *G1,
                                double *G2, double *G3);
/* TT -> Tucker: the Tucker2 form of Eq. (tt_3d_2) with the middle mode in an
 * orthonormal basis of the r1 r2 fibres G2[a, b, :] (r1 r2 <= 512, spanning
 * at most 128 dimensions), recompressed by HOOI with tol as above. */
demag_status demag_tt_to_tucker(demag_ctx *ctx, const int32_t n[3], int32_t r1, int32_t r2, const double *G1,
                                const double *G2, const double *G3, double tol, int32_t rmax, int32_t rout[3],
                                double *core, double *const rows[3]);

/* ---------------------------------------------------------------- learned rule
 * A network proposes shortened rules (R' = 16..32 nodes); the operator error
 * of a rule is certified against an accurate reference rule; a theorem-step
 * rule with 33..64 nodes is the fallback.  Not part of the paper's method: it shortens the sinc rule
 * of Cor. kron_op.
 *
 * Network: 6 -> 64 -> 64 -> 64 -> 65, GELU hidden layers, FP32, parameters a
 * flat device array of demag_mlp_param_count() floats [W1 (64x6, row =
 * output), b1, W2, b2, W3, b3, W4 (65x64), b4].  Inputs per case (x[b][6],
 * demag_quad_features): n_x/n_max, n_y/n_max, n_z/n_max, log2(1/h)/6 - 1,
 * (log10 tol + 6.5)/2.5, (R' - 24)/8.  Outputs y[b][65]: 32 node offsets, 32
 * log-weight offsets, the predicted log10 error.
 * Rule from outputs, base = sinc rule with R' nodes and c0 = 2.15:
 *   t'_k = t_k + 0.45 theta tanh(y_k),
 *   alpha'_k = 2 theta cosh t'_k sinh^2 t'_k exp(tanh(y_{32+k})).
 * Kernel values at an offset J: [K^x, K^y, K^z, F_xx, F_yy, F_zz, F_xy, F_xz,
 * F_yz] (potential kernels of Cor. kron_op and the field kernels of h_p <-
 * m_q), reference = the sinc rule with the step of Thm. sinc_theo and 96
 * nodes, on unit-longest-edge grids with cubic cells hmin.
 * Certificate (demag_quad_certify): the relative Frobenius-norm errors of the
 * discrete potential operator (3N -> N) and field operator (3N -> 3N),
 *   e_phi^2 = sum_J c(J) sum_q dK^q(J)^2 / sum_J c(J) sum_q K^q_ref(J)^2,
 *   e_h^2   = the same over F_pq with multiplicity 2 off the diagonal,
 * summed over every offset J >= 0 with c(J) = prod_d (n_d - J_d) (J_d ? 2 : 1)
 * (exactly for axes up to 512 cells; past 512 cells an axis' offsets are
 * taken in blocks of 4, 8, 16, ... per octave, each block by its midpoint with
 * its summed weight).  It equals the relative L2 error of phi and h averaged
 * over inputs with independent, equal-variance cell values.
 * Judge (demag_quad_judge, the fit's objective): the same sums over S sampled
 * offsets with weights (demag_quad_offsets), err = sqrt(e_phi^2 + e_h^2).
 * All arrays below are device arrays unless marked host. */
int32_t demag_mlp_param_count(void);
/* y[B][65]; z, a (optional, [B][3][64]) hidden pre-activations/activations. */
demag_status demag_mlp_forward(demag_ctx *ctx, const float *params, const float *x, int32_t B, float *y,
                               float *z, float *a);
/* Gradient of sum_b <dy_b, y_b> w.r.t. params (grad[param_count]), summed over
 * samples in a fixed order; delta[B][3][64] is scratch. */
demag_status demag_mlp_backward(demag_ctx *ctx, const float *params, const float *x, const float *z,
                                const float *a, const float *dy, int32_t B, float *delta, float *grad);
/* One bias-corrected Adam update of count parameters (step >= 1). */
demag_status demag_adam_step(demag_ctx *ctx, float *params, const float *grad, float *m, float *v,
                             int32_t count, int32_t step, float lr, float b1, float b2, float eps);
/* Rules t, alpha [B][32] from outputs y (NULL: the base rules) and R[B]. */
demag_status demag_quad_rules(demag_ctx *ctx, const float *y, const int32_t *R, int32_t B, double *t,
                              double *alpha);
/* Host-only.  Offsets J[count][3] (0 <= J_d < n_d) and weights w[count] of
 * the judge on grid n: the near block J_d <= 3 with exact weights c(J), then
 * shells of max-norm 4..max(n) - 1 in G = min((count - near)/8, max(n) - 4)
 * geometric groups, each represented by 8 offsets along a cycle of
 * directions with 1/8 of the group's summed weight; padded with J = 0, w = 0.
 * The weights add up to prod_d n_d^2.  DEMAG_E_INVAL if count < near block. */
demag_status demag_quad_offsets(const int32_t n[3], int32_t count, int32_t *J, double *w);
/* Host-only.  Network input x[6] of one case (layout above). */
demag_status demag_quad_features(const int32_t n[3], double h, double log10_tol, int32_t R, float *x);
/* Judge B rules (t, alpha [B][KM], R[B] nodes used) on grids [B][3] with
 * cell sizes hmin[B] at offsets [B][S][3] with weights [B][S]: err[B]; with
 * parts != NULL also (e_phi, e_h) [B][2]; with dt, dalpha non-NULL
 * d err / d t_k, d err / d alpha_k [B][KM].  Synchronizes the stream. */
demag_status demag_quad_judge(demag_ctx *ctx, int32_t B, const int32_t *grids, const double *hmin,
                              const int32_t *sentinels, const double *weights, int32_t S, const double *t,
                              const double *alpha, const int32_t *R, int32_t KM, double *err, double *parts,
                              double *dt, double *dalpha);
/* Certificate of the rule (host t, alpha of length M, scaled domain) on the
 * grid (physical; scaled to unit longest extent): err[0] = e_phi,
 * err[1] = e_h (host).  Synchronizes the stream. */
demag_status demag_quad_certify(demag_ctx *ctx, const demag_grid *grid, int32_t M, const double *t,
                                const double *alpha, double err[2]);
/* Levenberg-Marquardt fit of B cases' outputs (rule parametrization of
 * demag_quad_rules) against the reference rule on their grids [B][3], cell
 * sizes hmin[B], offsets [B][S][3] and weights [B][S] (S <= 256), R[B]
 * nodes (16..32): `iters` damped Gauss-Newton steps on the judge's residuals
 * r_(s,c) = sqrt(w_s m_c / D_c) (K - K_ref)_c(J_s) in u_k = 0.45 tanh(y_k),
 * v_k = tanh(y_{32+k}) (projected onto |u| <= 0.44, |v| <= 0.99) from y0
 * ([B][65] device, NULL = zeros, the plain base rule) with initial damping
 * mu0.  Device outputs: yout [B][65] (fitted outputs; slot 64 = log10 of the
 * fitted err), xout [B][64] (u, v in double; may be NULL), H [B][64][64]
 * (J^T J / err^2 at the fit, zero outside the active outputs; may be NULL),
 * t, alpha [B][32] (the fitted rule, zero past R), err[B].  Synchronizes
 * the stream. */
demag_status demag_quad_fit(demag_ctx *ctx, int32_t B, const int32_t *grids, const double *hmin,
                            const int32_t *sentinels, const double *weights, int32_t S, const int32_t *R,
                            const float *y0, int32_t iters, double mu0, float *yout, double *xout, float *H,
                            double *t, double *alpha, double *err);
/* Training loss and its output gradient for network outputs y [B][65]
 * against fits (targets [B][65] = demag_quad_fit's yout, xfit [B][64],
 * H [B][64][64]):
 *   loss_b = ln(1 + d^T H d) + lambda (y_64 - t_64)^2,
 *   d = (0.45 tanh y_k, tanh y_{32+k}) - xfit over the active outputs;
 * with xfit = H = NULL instead loss_b = mean_k (y_k - clip(t_k, 3))^2 +
 * lambda (y_64 - t_64)^2.  dy [B][65] = d loss_b / d y / B; loss [B]. */
demag_status demag_quad_loss_grad(demag_ctx *ctx, const float *y, const float *targets, const double *xfit,
                                  const float *H, const int32_t *R, int32_t B, float lambda, float *dy,
                                  float *loss);
/* Train in place with Adam for `steps` minibatches of `batch` consecutive
 * cases (wrapping; shuffle the cases beforehand) on the mean of
 * demag_quad_loss_grad's loss over the batch ([count] rows of targets,
 * xfit, H, R); step0 = Adam steps already taken.  loss_host (host, length
 * steps, may be NULL) receives each step's mean loss. */
demag_status demag_quad_train(demag_ctx *ctx, float *params, float *adam_m, float *adam_v, const float *x,
                              const float *targets, const double *xfit, const float *H, const int32_t *R,
                              int32_t count, int32_t steps, int32_t batch, int32_t step0, float lr,
                              float lambda, float *loss_host);

/* Modes of demag_quad_predict. */
typedef enum {
  DEMAG_PREDICT_NETWORK = 0,           /* R' from the error head, fits from the plain base rule */
  DEMAG_PREDICT_NETWORK_PROPOSAL = 1,  /* R' from the error head, fits from the network's proposal */
  DEMAG_PREDICT_SEARCH = 2             /* no network: bisection over R', fits from the plain rule */
} demag_predict_mode;

/* Result of demag_quad_predict (host). */
typedef struct {
  int32_t R;          /* nodes of the returned rule (64 if fell back) */
  int32_t fell_back;  /* 1: the theorem-step rule (33..64 nodes) */
  int32_t fits;       /* Levenberg-Marquardt fits run */
  int32_t mode;
  double err_phi;     /* certificate of the returned rule */
  double err_h;
  double predicted;   /* network's log10 error for its first pick (NaN in the search mode) */
  double seconds;     /* wall time of the call */
  double t[64];       /* nodes, scaled domain (zero past R) */
  double alpha[64];
} demag_quad_result;

/* Shortened rule for a grid with cubic cells (DEMAG_E_UNSUPPORTED otherwise)
 * at tolerance tol on both certificates.  The library computes the
 * network's inputs and the fit's offsets and weights itself.  Per mode (see
 * demag_predict_mode) candidate rules get fit_iters Levenberg-Marquardt steps
 * on the weighted offsets and are certified; the network modes start at the
 * smallest R' whose predicted log10 error is <= log10 tol and step R' by 1 up
 * to 32 on a miss, the search mode bisects R' = 16..32.  If no candidate
 * meets tol, the sinc rule with the step of Thm. sinc_theo is returned with
 * the fewest nodes in 33..64 whose certificate meets tol (64 tried first,
 * then bisection; fell_back = 1), and if even 64 nodes miss tol the call
 * returns DEMAG_E_ACCURACY with *out filled by the 64-node rule.  params (device) may be
 * NULL in the search mode. */
demag_status demag_quad_predict(demag_ctx *ctx, const float *params, const demag_grid *grid, double tol,
                                int32_t fit_iters, int32_t mode, demag_quad_result *out);

/* The bfloat16 split used by DEMAG_BF16X2/X3 on the device, exposed for
 * checking: x (device, count floats) -> parts (device, [nparts][count]
 * uint16 bit patterns): hi = bf16(x), lo = bf16(x - hi), lo2 = bf16(x - hi -
 * lo), each rounded to nearest even.  1 <= nparts <= 3. */
demag_status demag_bf16_split(demag_ctx *ctx, const float *x, uint16_t *parts, size_t count,
                              int32_t nparts);

/* Kernel timing.  While enabled, every kernel launch of the library is
 * bracketed by HIP events on the context's stream and attributed to a label
 * (e.g. "fp64/x/nout2").  demag_profile_enable(ctx, 1) clears previous
 * records; 0 stops recording.  demag_profile_read synchronizes the stream and
 * writes, for up to `max` labels, the label (NUL-terminated, at most 47
 * chars, into labels + 48*i), the summed milliseconds, the number of launches,
 * and the algorithmic FLOPs and bytes of those launches (the operation count
 * and the compulsory HBM traffic defined by the work itself, not by the
 * tiling); *count receives the number of labels written. */
demag_status demag_profile_enable(demag_ctx *ctx, int32_t enable);
demag_status demag_profile_read(demag_ctx *ctx, int32_t max, char *labels, double *total_ms,
                                int64_t *launches, double *flops, double *bytes, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* DEMAG_H */
