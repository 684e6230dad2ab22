/*
 * pinv.h -- dense-inverse solves of the 5-point variable-permittivity Poisson
 * operator on one AMD Instinct MI355X (gfx950).
 *
 * The method (Dourbal & Pekker, "A New Numerical Method for Fast Solution of
 * Partial Integro-Differential Equations"): discretise Eq. 1,
 *     d/dx_i eps d u/dx_i = rho,
 * with the 5-point scheme of Eq. 2 and Dirichlet identity rows as in Fig. 3,
 * build the matrix once, invert it once ("The solution steps", steps 1-2), and
 * then obtain u at every time moment as one product of the (optionally
 * rounded) inverse with the source vector (step 3; the rounding experiment of
 * Table 1).
 *
 * Grid and layouts
 *   A grid is n_x by n_y nodes INCLUDING the boundary, spacing h.  Nodal
 *   arrays are row-major [n_y][n_x]: the first (slow) index runs over y, the
 *   second (fast) over x, exactly the unknown order of Fig. 3.  The N =
 *   (n_x-2)(n_y-2) interior unknowns are numbered row-major over the interior.
 *   Right-hand sides, solutions and adjoint vectors are "column-major N x nrhs":
 *   vector r starts at ptr + r*ld, its N entries contiguous, ld >= N.
 *
 * Operator (conservative form of Eq. 1, face permittivity = mean of the two
 * nodal values):  for interior p,  sum_f eps_f (u_p - u_q) = -h^2 rho_p, so
 *     u = -h^2 * G * rho + w,   G = K^{-1} (SPD),  w = G * b_B,
 * where b_B carries the Dirichlet data of boundary neighbours.  With eps = 1,
 * K is 4x the interior block of the Fig. 3 matrix, whose interior rows read
 * u - 0.25 * (sum of 4 neighbours) = -(h^2/4) rho.
 *
 * Precision modes of the apply (inputs and outputs are FP64 in every mode):
 *   PINV_FP64   G in FP64, FP64 matrix-core product.
 *   PINV_FP64_SYM  the same values from a symmetric-packed copy of G (the
 *               64 x 64 blocks on and above the diagonal): one pass over about
 *               half the bytes, for few right-hand sides.
 *   PINV_FIX16_TILE  G rounded to 16-bit fixed point with one power-of-two
 *               exponent per 64 x 64 tile (2-D tile scales instead of one per
 *               row), stored as int16: 2 bytes per entry; the stored integers
 *               times rho in FP64, for few right-hand sides.  The adjoint
 *               uses G^T quantised the same way, which is exactly the
 *               transpose of G's integers and exponents.
 *   PINV_FP32   G and rho rounded to FP32, FP32 products, FP32 accumulation.
 *   PINV_BF16X3 G and rho split into 2 bfloat16 parts each; hi*hi + hi*lo +
 *               lo*hi with FP32 accumulation.
 *   PINV_BF16X6 3 parts each; the 6 products of total order <= 2.
 *   PINV_INT8   G rounded to b-bit per-row fixed point (b = 8, 16, 24) held
 *               as 1-3 balanced int8 digit slices, rho rounded per column to
 *               rho_bits the same way; the integer product is exact (int32
 *               matrix-core accumulation per slice-pair class, int64
 *               recombination), then scaled once and added to w.  Given the
 *               same FP64 G the result is reproducible bit for bit.
 *   Fixed point: M_S = 127*(256^S-1)/255 for S digits; e_i = frexp exponent of
 *   max_k |G_ik|; q_ik = rint((G_ik * 2^-e_i) * M_S) (one rounded multiply,
 *   ties to even); G^_ik = q_ik 2^e_i / M_S.  u_ir = double(acc_ir) *
 *   (c * 2^(e_i+f_r)) + w_i with c = -h^2/(M_S M_Sr) (two roundings, no FMA).
 *
 * Conventions for every call
 *   Returns PINV_OK (0) or a negative status; nothing throws or aborts.
 *   "stream" is a hipStream_t passed as void*; NULL means the null stream.
 *   Device pointers are HIP device (or managed) memory on the current device.
 *   Apply, adjoint and grad calls are asynchronous on the stream; their
 *   argument checks are synchronous.  An op is read-only during apply /
 *   adjoint / grad, so such calls may run concurrently on several streams;
 *   build/import/quantize/prepare/destroy must not overlap other calls on the
 *   same op.
 */
#ifndef PINV_H
#define PINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define PINV_OK               0
#define PINV_E_INVALID_ARG   -1  /* bad size, NULL pointer, ld < N, bad enum   */
#define PINV_E_NOT_SPD       -2  /* Cholesky met a non-positive pivot (LU: singular matrix) */
#define PINV_E_OOM           -3  /* device allocation failed or would not fit  */
#define PINV_E_HIP           -4  /* a HIP runtime call failed                  */
#define PINV_E_UNSUPPORTED   -5  /* size beyond the integer headroom limits, or an operation the op does not support */
#define PINV_E_STATE         -6  /* representation needed by the call missing  */
#define PINV_E_IO            -7  /* a file could not be opened, read or written */

/* ---- enums -------------------------------------------------------------- */
#define PINV_FP64    0
#define PINV_FP32    1
#define PINV_BF16X3  2
#define PINV_BF16X6  3
#define PINV_INT8    4
#define PINV_FP64_SYM 5          /* FP64 from the symmetric-packed upper triangle */
#define PINV_FIX16_TILE 6        /* 16-bit fixed point, one exponent per 64 x 64 tile */

#define PINV_SCALE_ROW 0          /* one power-of-two exponent per row of G   */

typedef struct pinv_op_s* pinv_op; /* opaque; owns all of its device memory   */

typedef struct {
  int32_t nx;   /* grid points along x (fast axis), boundary included, >= 3    */
  int32_t ny;   /* grid points along y (slow axis), boundary included, >= 3    */
  double  h;    /* uniform spacing (Eq. 2: h = L/(n-1)), > 0                    */
} pinv_grid;

typedef struct {
  int32_t nx, ny, n;        /* grid and number of interior unknowns N          */
  double  h;
  int32_t has_fp64;         /* FP64 G resident                                  */
  int32_t int8_slices;      /* S (0 if not quantised)                           */
  int32_t has_fp32, has_bf16;
  int32_t has_lift;         /* nonzero Dirichlet data (w != 0)                  */
  int64_t device_bytes;     /* device memory held by the op                     */
  int32_t nz;               /* n_z for a 3-D op, 0 for a 2-D op                 */
  int32_t general;          /* built by pinv_build_inverse_general (h = 1)      */
  int32_t beta;             /* built by pinv_build_inverse_beta (h = 1)         */
  int32_t has_sym;          /* symmetric-packed FP64 copy held                  */
  int32_t has_tile16;       /* 16-bit tile-scaled copy held                     */
  int32_t fp64_symmetric;   /* G resident and equal to G^T bit for bit (checked
                               when G is built, imported or loaded; the FP64
                               adjoint then runs the forward product)          */
} pinv_info;

/* Steps 1-2 of "The solution steps": assemble the interior operator K from the
 * nodal permittivity (Eq. 1 in conservative form; Eq. 2 when eps = 1), factor
 * it by blocked FP64 Cholesky and form G = K^{-1} = L^{-T} L^{-1} on the GPU,
 * plus the lift w = G b_B.
 *   g           grid (host).
 *   eps_nodes   host [n_y][n_x] nodal permittivity, or NULL for eps = 1.
 *   u_boundary  host [n_y][n_x]; only boundary entries are read.  NULL = 0.
 *   out         receives the new op (NULL on failure).
 * Synchronises the stream once at the end.  PINV_E_NOT_SPD if a pivot <= 0
 * (e.g. eps <= 0 somewhere).  Device memory: about 3 N^2 doubles at peak,
 * N^2 doubles afterwards. */
int32_t pinv_build_inverse(const pinv_grid* g, const double* eps_nodes,
                           const double* u_boundary, void* stream, pinv_op* out);

/* The same for the 3-D operator (N = n_x n_y n_z in the problem statement;
 * 7-point conservative stencil, face eps = mean of the two nodal values):
 *   g           grid with n_z >= 3 (host).
 *   eps_nodes   host [n_z][n_y][n_x], or NULL for eps = 1.
 *   u_boundary  host [n_z][n_y][n_x]; only boundary entries are read.  NULL = 0.
 * Interior unknowns are ordered p = ((k-1)(n_y-2) + (i-1))(n_x-2) + (j-1)
 * (z slowest, x fastest).  The resulting op supports quantize, apply, the
 * adjoint and the eps-gradient (over the 6 faces of each node) like a 2-D op. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t _pad;
  double h;
} pinv_grid3;

int32_t pinv_build_inverse_3d(const pinv_grid3* g, const double* eps_nodes,
                              const double* u_boundary, void* stream, pinv_op* out);

/* Steps 1-2 for Eq. 1 with a permittivity per direction (eps_x, eps_y) on a
 * non-uniform tensor grid (node coordinates x[n_x], y[n_y], strictly
 * increasing), in finite-volume form: node (i, j) owns the control volume
 * A = (x[j+1]-x[j-1])/2 * (y[i+1]-y[i-1])/2; an x-face carries
 * eps_x,f * (y[i+1]-y[i-1])/2 / |x_q - x_j|, a y-face
 * eps_y,f * (x[j+1]-x[j-1])/2 / |y_q - y_i| (eps_f the mean of the two nodal
 * values), so K u = -A rho + b_B.  The op stores G = K^{-1} diag(A) with h = 1,
 * so pinv_apply_inverse gives u = -G rho + w as for the uniform forms (the
 * adjoint applies the transpose of this G).
 *   eps_x, eps_y  host [n_y][n_x]; NULL eps_x = 1, NULL eps_y = eps_x.
 *   u_boundary    host [n_y][n_x]; only boundary entries are read.  NULL = 0.
 * pinv_grad_eps returns PINV_E_UNSUPPORTED for the op (pinv_grad_eps_general
 * gives its gradients).  On a uniform grid with eps_x = eps_y this builds h^2
 * times the G of pinv_build_inverse. */
typedef struct {
  int32_t nx, ny;
  const double* x;    /* host [n_x] */
  const double* y;    /* host [n_y] */
} pinv_grid_general;

int32_t pinv_build_inverse_general(const pinv_grid_general* g, const double* eps_x,
                                   const double* eps_y, const double* u_boundary,
                                   void* stream, pinv_op* out);

/* Steps 1-2 for Eq. 3 with arbitrary neighbour coefficients (the relaxation
 * form of the discretisation, row-normalised and in general not symmetric),
 * restricted to the interior unknowns: row p = (i, j) reads
 *   u_p - sum_d beta[d][i][j] / 4 * u_{q_d} = rho_p,
 * d over the neighbours (i-1, j), (i+1, j), (i, j-1), (i, j+1) in that order;
 * a boundary neighbour's Dirichlet value moves to the right-hand side
 * (b_B[p] += beta[d][i][j] / 4 * u_B(q_d)), so u = A^{-1} (rho + b_B).  The
 * inverse is formed on the GPU by a blocked LU factorization with partial
 * pivoting, P A = L U (row exchanges chosen column by column: the first row of
 * largest magnitude), then A^{-1} = U^{-1} L^{-1} P.  The op stores G = -A^{-1} with h = 1,
 * so pinv_apply_inverse gives u = -G rho + w = A^{-1} rho + w with the lift
 * w = A^{-1} b_B; the adjoint applies the transpose.
 *   g           grid (host); g->h is not used (the op's h is 1).
 *   beta        host [4][n_y][n_x], finite; only interior nodes are read.
 *   u_boundary  host [n_y][n_x]; only boundary entries are read.  NULL = 0.
 * PINV_E_NOT_SPD if A is singular (a column with no non-zero finite pivot
 * candidate); pinv_grad_eps returns PINV_E_UNSUPPORTED for the op (the
 * coefficient gradient is pinv_grad_beta).  Synchronous; device memory about
 * 2 N^2 doubles at peak, N^2 afterwards. */
int32_t pinv_build_inverse_beta(const pinv_grid* g, const double* beta,
                                const double* u_boundary, void* stream, pinv_op* out);

/* Create an op from an inverse computed elsewhere (step 2 by "any standard
 * matrix inversion method"; also restores a saved op).
 *   G_host      host row-major N x N, row stride ldg >= N (copied).
 *   u_boundary  as in pinv_build_inverse (kept for pinv_grad_eps), or NULL.
 *   w_host      host [N] lift to use as is, or NULL: then w = G b_B is formed
 *               on the GPU when u_boundary is given (eps_nodes used for b_B),
 *               else w = 0. */
int32_t pinv_import_inverse(const pinv_grid* g, const double* G_host, int64_t ldg,
                            const double* eps_nodes, const double* u_boundary,
                            const double* w_host, void* stream, pinv_op* out);

/* Copy the FP64 inverse to host memory (row-major, row stride ldg >= N) and,
 * if w_host != NULL, the lift.  Synchronous.  PINV_E_STATE if G was freed. */
int32_t pinv_export_inverse(pinv_op op, double* G_host, int64_t ldg, double* w_host,
                            void* stream);

/* The rounding of the inverse (Table 1 experiment), in binary: per-row
 * fixed point with bits = 8, 16 or 24 (S = bits/8 int8 digit slices).
 * Replaces any previous quantisation.  keep_fp64 = 0 frees the FP64 G
 * afterwards (FP64/FP32/BF16 applies then return PINV_E_STATE).
 * scale_mode must be PINV_SCALE_ROW (64 x 64 tile scales are the separate
 * 16-bit storage PINV_FIX16_TILE of pinv_prepare_split).  Synchronous. */
int32_t pinv_quantize_inverse(pinv_op op, int32_t bits, int32_t scale_mode,
                              int32_t keep_fp64, void* stream);

/* Materialise the FP32 copy (mode PINV_FP32) or the bfloat16 parts (PINV_BF16X3
 * or PINV_BF16X6) of G, from the FP64 G.  Synchronous.
 * PINV_FP64_SYM: the symmetric-packed FP64 copy, for applies that are one pass
 * over G (few right-hand sides, HBM-bound): the 64 x 64 blocks on and above
 * the diagonal, about half the bytes of G.  G must be symmetric to within
 * 1e-12 sqrt(|G_ii G_jj|) in every entry (true of the inverses built by
 * pinv_build_inverse and pinv_build_inverse_3d, not of those from
 * pinv_build_inverse_general or pinv_build_inverse_beta): PINV_E_UNSUPPORTED
 * otherwise.  Applies in this mode use the upper triangle, and the adjoint
 * equals the forward product; each pass of up to 8 right-hand sides takes a
 * stream-ordered scratch of 8 N_b^2 64 doubles per right-hand side (N_b =
 * ceil(N/64)) from the device's memory pool.
 * PINV_FIX16_TILE (the rounding of Table 1 in binary with 2-D tile scales):
 * for each 64 x 64 tile (a, b), e_ab = the frexp exponent of its largest
 * |G_ik| (|G| < 2^e_ab; 0 for an all-zero tile) and
 * q_ik = rint(2^-e_ab G_ik M), M = 32639 (16-bit balanced fixed point, as
 * PINV_INT8 with 16 bits), held as int16 (N rows of 64 ceil(N/64) entries)
 * with the exponents; the apply forms u_i = -h^2 / M sum_b 2^e_(i/64,b)
 * sum_(k in b) q_ik rho_k + w_i in FP64 (deterministic order; within
 * 1e-12 of the exact value of that sum).  G^T is quantised alike into a
 * second copy for the adjoint (lambda = -h^2 G^T g in the same form; the
 * transposed tiles have the same maxima, so its integers and exponents are
 * exactly the transposes of G's): 4 N (64 ceil(N/64)) bytes in all.  Applies
 * and adjoints in this mode allocate nothing. */
int32_t pinv_prepare_split(pinv_op op, int32_t mode, void* stream);

/* Checkpoint (not in the paper, whose method precomputes once and applies at
 * every time moment): pinv_save writes the op's grid description and what it
 * holds of {FP64 G, the int8 digit slices with their row exponents, the lift
 * w, the Dirichlet data, a non-uniform grid's node coordinates} and its int8
 * variant choices to a file (host byte order; about 8 N^2 bytes for G and
 * S P^2 for the slices, P = 256 ceil(N / 256)).  Split-precision, packed and
 * tile-scaled copies are not written (pinv_prepare_split rebuilds them from
 * G).  pinv_load creates an op on the current device from such a file without
 * the O(N^3) build, bit for bit the same data (the transposed digit planes of
 * the adjoint are formed on the device).  The header and the file's length
 * are checked before anything is allocated: PINV_E_INVALID_ARG for a file
 * that is not such a checkpoint, PINV_E_IO if it cannot be opened, read or
 * written, PINV_E_STATE (save) for an op holding neither G nor slices.
 * Synchronous. */
int32_t pinv_save(pinv_op op, const char* path, void* stream);
int32_t pinv_load(const char* path, void* stream, pinv_op* out);

/* Export the 16-bit tile-scaled copy: q (host [N][N] int16, row-major) and
 * the tile exponents (host [ceil(N/64)][ceil(N/64)] int32, row-major).  Either
 * may be NULL.  Synchronous.  PINV_E_STATE if it was not prepared. */
int32_t pinv_export_tile16(pinv_op op, int16_t* q_host, int32_t* exponents_host, void* stream);

/* Export the int8 digit slices (host [S][N][N], most significant slice
 * first, row-major) and the per-row exponents (host [N]).  Either may be NULL.
 * Synchronous.  PINV_E_STATE if not quantised. */
int32_t pinv_export_quantized(pinv_op op, int8_t* slices_host, int32_t* exponents_host,
                              void* stream);

/* Step 3: u = L^{-1} rho for nrhs right-hand sides,  u = -h^2 G rho + w.
 *   mode      PINV_FP64 / FP64_SYM / FP32 / BF16X3 / BF16X6 / INT8 /
 *             FIX16_TILE (FP64_SYM, FP32, BF16X* and FIX16_TILE after
 *             pinv_prepare_split; INT8 after pinv_quantize_inverse).
 *   rho_bits  8, 16 or 24: fixed-point width of rho in INT8 mode (ignored
 *             otherwise).
 *   rho, u    device, column-major N x nrhs with strides ld_rho, ld_u >= N;
 *             must not overlap.  nrhs >= 0 (0 is a no-op).
 * Asynchronous.  PINV_E_STATE if the mode's representation is missing;
 * PINV_E_UNSUPPORTED in INT8 mode if N * M_S * M_Sr >= 2^63 (the exact int64
 * recombination).  Where one int32 class sum over all of k could overflow
 * (N * 16384 * pairs-per-class >= 2^31), k is split and the parts are added in
 * int64, taking a stream-ordered scratch of the class sums from the pool. */
int32_t pinv_apply_inverse(pinv_op op, int32_t mode, int32_t rho_bits,
                           const double* rho, int64_t ld_rho, int32_t nrhs,
                           double* u, int64_t ld_u, void* stream);

/* Bytes of device scratch that pinv_apply_inverse_noalloc holds per GPU. */
#define PINV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the INT8
 * apply of pinv_apply_inverse (same arguments, mode INT8), with identical
 * results, that calls no allocator.  Its scratch (the quantised right-hand
 * sides, SR * 128 ceil(nrhs / 128) * P bytes with P = 256 ceil(N / 256), plus
 * 4 bytes per padded right-hand side) is a fixed array of
 * PINV_NOALLOC_SCRATCH_BYTES per GPU, which the library holds until the
 * process ends; larger requests return PINV_E_OOM.  k is never split, so ops
 * whose int32 class sums would need a split (N * 16384 * pairs-per-class >=
 * 2^31) return PINV_E_UNSUPPORTED.  The current device must be the op's
 * (PINV_E_INVALID_ARG otherwise).  Every call on one GPU shares that GPU's
 * scratch: calls that overlap in time on one GPU (other streams, other ops)
 * race and must be ordered by the caller.  Asynchronous. */
int32_t pinv_apply_inverse_noalloc(pinv_op op, int32_t rho_bits,
                                   const double* rho, int64_t ld_rho, int32_t nrhs,
                                   double* u, int64_t ld_u, void* stream);

/* Adjoint of the apply's linear part (not in the paper; the derivative of
 * step 3):  lambda = dLoss/drho = -h^2 * G^T g  for the representation that
 * the mode selects (G^T of the rounded matrix in INT8 mode, where g's row
 * scaling 2^e_k is applied exactly before g is rounded to g_bits per column;
 * the transposed 16-bit copy in FIX16_TILE mode; the packed upper triangle
 * itself in FP64_SYM mode, G being symmetric; in FP64 mode the forward
 * product itself when G equals G^T bit for bit, see pinv_info).  Same layout
 * rules as pinv_apply_inverse.  Asynchronous. */
int32_t pinv_apply_inverse_adjoint(pinv_op op, int32_t mode, int32_t g_bits,
                                   const double* g, int64_t ld_g, int32_t nrhs,
                                   double* lambda, int64_t ld_lambda, void* stream);

/* Permittivity gradient (not in the paper): with u the forward solutions and
 * lambda the adjoint outputs of the same loss,
 *   dLoss/deps_f = (1/h^2) sum_r (lambda_p - lambda_q)(u_p - u_q)
 * over the faces f = (p, q) of the operator (lambda = 0 and u = u_B on the
 * boundary), and grad_nodes[i][j] = half the sum over the faces touching the
 * node.  grad_nodes: device [n_y][n_x] ([n_z][n_y][n_x] for a 3-D op),
 * overwritten (no accumulation).  Uniform-grid ops only (PINV_E_UNSUPPORTED
 * for ops from pinv_build_inverse_general and pinv_build_inverse_beta).
 * Deterministic (fixed summation order).  For nrhs > 16 a stream-ordered
 * scratch of ceil(nrhs/16) doubles per node is taken from the device's
 * memory pool for the duration of the call.  Asynchronous. */
int32_t pinv_grad_eps(pinv_op op, const double* u, int64_t ld_u,
                      const double* lambda, int64_t ld_lambda, int32_t nrhs,
                      double* grad_nodes, void* stream);

/* Per-direction permittivity gradients for an op from
 * pinv_build_inverse_general (not in the paper).  There the solve is
 * K u = -A rho + b_B and the adjoint output is lambda = -(K^{-1} diag(A))^T g,
 * so mu = K^{-1} g = -lambda / A.  A face f = (p, q) has the coefficient
 * eps_f * s_f (s_f = (y[i+1]-y[i-1])/2 / |x_q - x_p| for an x-face on row i,
 * (x[j+1]-x[j-1])/2 / |y_q - y_p| for a y-face on column j), and
 *   dLoss/d(eps_f s_f) = sum_r (lambda_p/A_p - lambda_q/A_q)(u_p - u_q)
 * (lambda = 0 and u = u_B on the boundary); each end node receives s_f/2 of it,
 * x-faces in grad_x and y-faces in grad_y.
 *   grad_x, grad_y  device [n_y][n_x], overwritten.  grad_y NULL: grad_x
 *                   receives the sum (the gradient with respect to one field
 *                   used for both directions, as when the op was built with
 *                   eps_y NULL).
 * PINV_E_UNSUPPORTED for other ops.  Deterministic; for nrhs > 16 a
 * stream-ordered scratch of 2 ceil(nrhs/16) doubles per node is taken from
 * the device's memory pool for the duration of the call.  Asynchronous. */
int32_t pinv_grad_eps_general(pinv_op op, const double* u, int64_t ld_u,
                              const double* lambda, int64_t ld_lambda, int32_t nrhs,
                              double* grad_x, double* grad_y, void* stream);

/* Gradient with respect to Eq. 3's coefficients (not in the paper), for an op
 * from pinv_build_inverse_beta: with u = A^{-1}(rho + b_B) the forward
 * solutions and lambda = A^{-T} g the adjoint outputs of the same loss
 * (pinv_apply_inverse_adjoint on the op),
 *   dLoss/dbeta_d(p) = (1/4) sum_r lambda_p U_{q_d},
 * U = u at interior nodes and u_B on the boundary (q_d: the neighbour of p in
 * direction d, in the order of pinv_build_inverse_beta).
 *   grad_beta  device [4][n_y][n_x], overwritten; zero at boundary nodes.
 * PINV_E_UNSUPPORTED for other ops.  Deterministic; for nrhs > 16 a
 * stream-ordered scratch of 4 ceil(nrhs/16) doubles per node is taken from the
 * device's memory pool for the duration of the call.  Asynchronous. */
int32_t pinv_grad_beta(pinv_op op, const double* u, int64_t ld_u,
                       const double* lambda, int64_t ld_lambda, int32_t nrhs,
                       double* grad_beta, void* stream);

/* Many solves against many ops in one call (batched uneven requests).
 * In PINV_INT8 mode the requests naming the same op are grouped and each group
 * runs as one product over all of its right-hand sides: one rho quantisation
 * reading the columns through a device pointer table and one slice GEMM whose
 * epilogue writes every column straight into its request's u (bit-identical
 * to one pinv_apply_inverse call per request); groups whose ops share a digit
 * count share one launch.  Other modes run the requests one by one.  Every request is checked before anything is
 * launched; requests must not write into each other's rho or u.
 * INT8 mode keeps a plan per request list (the device tables, the scratch of
 * the quantised right-hand sides and the pinned host image the tables were
 * uploaded from), keyed by the requests' ops, pointers, strides and column
 * counts, rho_bits, the ops' digit counts, and the stream.  The first call
 * with a key allocates the plan, uploads its tables (from the plan's own
 * pinned image, so nothing waits for the copy) and picks each launch's int8
 * kernel variant by timing every variant with 128-row tiles on that launch
 * (the call then waits for those timings; results are bit-identical whichever
 * variant runs); later calls with the same key only launch kernels, so such a call can be captured into a HIP graph, whose
 * replays stay valid while the plan is kept.  Under stream capture a key seen
 * for the first time gives PINV_E_STATE.  At most 4 plans are kept (the
 * least recently used is dropped first, after a device synchronisation); a
 * plan naming an op is dropped when the op is destroyed or re-quantised;
 * pinv_batched_release drops all of them.  In INT8 mode an op whose class
 * sums over all of k could overflow int32 (N * 16384 * pairs-per-class >=
 * 2^31; the grouped product does not split k) gives PINV_E_UNSUPPORTED, with
 * nothing launched. */
typedef struct {
  pinv_op        op;
  const double*  rho;     /* device, column-major N x nrhs, stride ld        */
  double*        u;       /* device, same layout                             */
  int64_t        ld;
  int32_t        nrhs;
  int32_t        _pad;
} pinv_request;

int32_t pinv_apply_batched(const pinv_request* reqs, int32_t nreq, int32_t mode,
                           int32_t rho_bits, void* stream);

/* Drops every plan of pinv_apply_batched (after a device synchronisation),
 * releasing their device and pinned host memory. */
int32_t pinv_batched_release(void);

int32_t pinv_get_info(pinv_op op, pinv_info* info);

/* Kernel selection for the int8 slice product (a performance choice only: every
 * variant computes the same exact integer classes, so results are bit-identical
 * whichever runs).  Variants differ in the k depth of an LDS stage (128 or 64
 * bytes, with 2 to 4 stages in flight) and in the order in which workgroups
 * take output tiles (grouped by the chip's eight L2 domains, or linear).
 *
 * pinv_int8_variants: number of variants (ids 0 .. count-1; 0 is the default).
 * pinv_set_int8_variant: use `variant` for this op's int8 products (forward
 *   and adjoint) at rho/g precision `rho_bits` (8, 16 or 24).
 * pinv_autotune_int8: times every variant on this op (which must be
 *   quantised) for `nrhs` right-hand sides at `rho_bits`: three rounds over
 *   the variants, `reps` launches each after one warm-up, each variant keeping
 *   its best round.  The digit planes timed are those of `rho` (device,
 *   column-major N x nrhs, stride ld_rho >= N: representative right-hand sides
 *   of the caller's workload; the matrix cores' clock depends on the data) or,
 *   if rho is NULL, uniformly random digits.  Scratch device memory is
 *   allocated and freed inside the call; the op's data is only read.  Selects
 *   the fastest variant for the op and writes its id to *best (may be NULL) and
 *   the mean milliseconds per launch of variant v to variant_ms[v] for
 *   v < n_ms (variant_ms may be NULL).  Synchronises the stream.
 *   E_STATE if the op is not quantised, E_INVALID_ARG for bad sizes.
 *   With the environment variable PINV_AUTOTUNE_CACHE naming a file, a choice
 *   stored there for the same device kind (architecture name and compute-unit
 *   count), unknowns, digit counts and padded right-hand-side count is taken
 *   without timing (variant_ms[v] is then the stored time for the chosen
 *   variant and -1 for the others); otherwise the choice is appended to the
 *   file as one text line "int8 <arch> <CUs> <N> <S> <SR> <Rpad> <variant>
 *   <ms>" (later lines win; lines that do not parse are ignored). */
int32_t pinv_int8_variants(void);
int32_t pinv_set_int8_variant(pinv_op op, int32_t rho_bits, int32_t variant);
int32_t pinv_autotune_int8(pinv_op op, int32_t rho_bits, const double* rho, int64_t ld_rho,
                           int32_t nrhs, int32_t reps, double* variant_ms, int32_t n_ms,
                           int32_t* best, void* stream);

/* Kernel tracing (profiling aid).  While enabled, every kernel launched by the
 * library is bracketed by a pair of HIP events recorded on the same stream.
 * pinv_trace_read sums the elapsed times of the recorded launches of one
 * kernel family -- "gemm_i8", "gemv_i8" (the int8 apply for at most 4
 * right-hand sides), "quantize_cols", "gemm_f64", "gemv_f64", "gemv_sym",
 * "gemv_tile16", "gemm_split", "grad_eps" -- waiting for their events, and
 * forgets them; total_ms and launches may be NULL.  pinv_trace_enable(0)
 * stops recording (recorded launches stay readable).  Thread-safe. */
int32_t pinv_trace_enable(int32_t on);
int32_t pinv_trace_read(const char* kernel, double* total_ms, int64_t* launches);
/* The same, also writing the elapsed milliseconds of each recorded launch, in
 * launch order, to ms_each[0 .. min(launches, cap) - 1] (ms_each may be NULL
 * when cap is 0). */
int32_t pinv_trace_read_each(const char* kernel, double* ms_each, int64_t cap,
                             double* total_ms, int64_t* launches);

/* Free the op and all of its device memory (waits for the device first). */
int32_t pinv_destroy(pinv_op op);

/* Static string for a status code. */
const char* pinv_status_string(int32_t status);

/* Library version string, "major.minor.patch". */
const char* pinv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PINV_H */
