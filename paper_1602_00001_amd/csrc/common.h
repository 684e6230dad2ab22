// Internal declarations of the pinv library (gfx950 / CDNA4 only).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <cstdint>
#include <cstddef>

#include "pinv.h"

typedef int    v4i  __attribute__((ext_vector_type(4)));
typedef int    v16i __attribute__((ext_vector_type(16)));
typedef double v4d  __attribute__((ext_vector_type(4)));
typedef float  v4f  __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

#define PINV_WAVE 64

// Workgroups for an element-wise kernel over `total` items with 256 threads
// and a grid-stride loop: at most 2^20 workgroups, so the launch stays far
// below the 2^32 work-items a dispatch can hold.
inline unsigned grid_1d(int64_t total) {
  const int64_t b = (total + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > (1 << 20) ? (1 << 20) : b));
}

// Padded square dimension of the int8 digit planes and of split-precision
// copies: a multiple of 256 so that every 128x128 (or 256-row) tile and every
// 64/128-byte k chunk lies inside the allocation; the padding holds zeros.
static inline int64_t pinv_pad_dim(int64_t n) { return (n + 255) / 256 * 256; }

struct pinv_op_s {
  int nx = 0, ny = 0, mx = 0, my = 0, n = 0;
  int nz = 0, mz = 1;        // 3-D grids: n_z nodes along z (0 for a 2-D grid)
  int general = 0;           // non-uniform grid / per-direction eps: G holds K^{-1} diag(A), h = 1
  int beta = 0;              // Eq. 3 with arbitrary coefficients: G holds -A^{-1}, h = 1
  double* xc = nullptr;      // non-uniform grid: device node coordinates [nx], [ny]
  double* yc = nullptr;
  double h = 0.0;
  int device = 0;

  // FP64 inverse, row-major [n][ldg] (ldg multiple of 32 doubles)
  double* G = nullptr;
  int64_t ldg = 0;
  int g_symmetric = 0;       // G is exactly symmetric (checked when G is formed or loaded)
  double* w = nullptr;       // lift [n] (nullptr when the Dirichlet data is zero)
  double* ub = nullptr;      // nodal Dirichlet data [ny*nx] (nullptr when zero)

  // per-row fixed point, S balanced int8 digit planes [S][P][P] (k fastest),
  // the transposed planes for the adjoint, and the row exponents [P]
  int S = 0;
  int64_t P = 0;
  int8_t* Q = nullptr;
  int8_t* QT = nullptr;
  int32_t* e = nullptr;
  int i8_variant[4] = {0, 0, 0, 0};   // int8 GEMM variant per rho slice count (autotuned)

  // split-precision copies, zero-padded row-major planes [P][P]
  float* G32 = nullptr;
  __bf16* Gb = nullptr;      // [nbf][P][P]
  int nbf = 0;               // number of bfloat16 parts held (2 or 3)

  // symmetric-packed FP64 copy: upper-triangle 64 x 64 blocks
  double* Gsym = nullptr;

  // 16-bit fixed point with one exponent per 64 x 64 tile: q [n][ldq] int16
  // (ldq = 64 ceil(n/64)), exponents [ceil(n/64)]^2
  int16_t* Gt16 = nullptr;
  int32_t* Et16 = nullptr;
  int16_t* Gt16T = nullptr;  // the same for G^T (the adjoint's operand)
  int32_t* Et16T = nullptr;

  int64_t bytes = 0;
};

// ---- error handling ---------------------------------------------------------
#define PINV_HIP_TRY(expr)                                   \
  do {                                                       \
    hipError_t e__ = (expr);                                 \
    if (e__ != hipSuccess) return pinv_hip_status(e__);      \
  } while (0)

int32_t pinv_hip_status(hipError_t e);
void pinv_log(const char* fmt, ...);

// Autotune cache (file named by PINV_AUTOTUNE_CACHE): device kind key
// ("<arch> <compute units>", empty if unknown), lookup of a stored int8
// variant choice, and appending one.
std::string tune_device_key(int device);
bool tune_cache_lookup(const char* path, const std::string& dkey, int n, int S, int SR, int Rpad, int nvariants,
                       int* variant, double* ms);
void tune_cache_store(const char* path, const std::string& dkey, int n, int S, int SR, int Rpad, int variant,
                      double ms);

// Records a pair of events around the launches in its scope when tracing is
// enabled (pinv_trace_enable) and name is not null; a no-op otherwise.
class TraceScope {
 public:
  TraceScope(const char* name, hipStream_t s);
  ~TraceScope();
  TraceScope(const TraceScope&) = delete;
  TraceScope& operator=(const TraceScope&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  bool on_ = false;
};

// ---- FP64 MFMA GEMM -----------------------------------------------------------
// C(m,n) = alpha * sum_{k in [kbeg, K)} A(m,k) B(k,n) + beta * C(m,n) + bias[m]
// A(m,k) = A[m*lda + k] if a_kcontig else A[k*lda + m]
// B(k,n) = B[n*ldb + k] if b_kcontig else B[k*ldb + n]
// C(m,n) = C[m*csm + n*csn]
// tri: 0 = full; 1 = skip tiles strictly above the diagonal (n0 > m0 + BM - 1)
// kdiag: if nonzero, the k range of a tile starts at max(m0, n0) rounded down to
//        the k step (both operands are zero for k below their own row/column
//        index, as for A(m,k) = W[k][m], B(k,n) = W[k][n] with W lower triangular).
struct GemmF64Args {
  const double* A; int64_t lda; int a_kcontig;
  const double* B; int64_t ldb; int b_kcontig;
  double* C; int64_t csm, csn;
  int M, N, K;
  double alpha, beta;
  const double* bias;
  int tri, kdiag;
  // split-K (both operands k-contiguous, no tri/kdiag): ksplit > 1 workgroups
  // share each output tile, each over k in [z*kchunk, (z+1)*kchunk); their raw
  // sums go to part[z][n][m] (column-major M x N per z) and a second kernel
  // adds them in order of z and applies alpha, beta and bias.
  int ksplit;
  int kchunk;
  double* part;
};
hipError_t launch_gemm_f64(const GemmF64Args& a, hipStream_t s);
// split count and k chunk for an M x N x K product (ksplit = 1: no split)
void gemm_f64_split_plan(int M, int N, int K, int* ksplit, int* kchunk);
// C = alpha * sum_z part[z] + beta * C + bias (column-major part, M x N per z)
hipError_t launch_splitk_reduce(const double* part, int ksplit, int M, int N, double alpha, double beta,
                                const double* bias, double* C, int64_t csm, int64_t csn, hipStream_t s);

// FP64 apply u = alpha * G X + bias for many right-hand sides (one wave per
// SIMD, 256 x 128 tiles; G row-major [M][lda] with zeros past column K up to
// the next multiple of 16, X column-major K x N with stride ldx).  Scratch:
// pack_bytes (zero-padded copy of X) + part_bytes (split-k partial sums).
struct ApplyF64Plan {
  int tilesM = 0, tilesN = 0, Npad = 0;
  int64_t ldp = 0;
  int ksplit = 1, kchunk = 0;
  size_t pack_bytes = 0, part_bytes = 0;
};
ApplyF64Plan apply_f64_plan(int M, int N, int K);
hipError_t launch_apply_f64(const ApplyF64Plan& p, const double* G, int64_t lda, int M, int K, const double* X,
                            int64_t ldx, int N, double alpha, const double* bias, double* U, int64_t ldu,
                            void* scratch, hipStream_t s);

// FP64 GEMV-style apply for few right-hand sides: u = alpha * G x + bias.
hipError_t launch_gemv_f64(const double* G, int64_t ldg, int n, const double* x, int64_t ldx,
                           int nrhs, double alpha, const double* bias, double* u, int64_t ldu,
                           hipStream_t s);

// ---- setup kernels ------------------------------------------------------------
// nz = 0: the 5-point operator of an n_y x n_x grid; nz >= 3: the 7-point
// operator of an n_z x n_y x n_x grid
hipError_t launch_assemble(int nx, int ny, int nz, const double* eps, const double* ub, double* K,
                           int64_t ldk, double* bB, hipStream_t s);
struct GeneralGrid {
  const double* x;       // node coordinates [nx] (device)
  const double* y;       // [ny]
  const double* eps_y;   // y-direction permittivity [ny][nx], or null (= eps_x)
  double* area;          // control volumes [n], written by the assembly (device scratch)
};
int32_t build_inverse_lu_device(pinv_op op, const double* beta_dev, const double* ub_dev, hipStream_t s);
int32_t build_inverse_device(pinv_op op, const double* eps_dev, const double* ub_dev, const GeneralGrid* gen,
                             hipStream_t s);

// ---- quantisation -------------------------------------------------------------
int64_t pinv_max_mag(int S);
hipError_t launch_quantize_rows(const double* G, int64_t ldg, int n, int S, int64_t P,
                                int8_t* Q, int32_t* e, hipStream_t s);
hipError_t launch_transpose_planes(const int8_t* Q, int8_t* QT, int S, int64_t P, hipStream_t s);
// digits of X (column-major n x nrhs, stride ldx) per column into [SR][Rpad][P];
// pre_exp (may be null) multiplies row k by 2^pre_exp[k] first.  If xcols is
// not null, column r is read from xcols[r] instead (X, ldx ignored).
hipError_t launch_quantize_cols(const double* X, int64_t ldx, const double* const* xcols, int n, int nrhs,
                                int Rpad, int SR, int64_t P, const int32_t* pre_exp, int8_t* Xq, int32_t* f,
                                hipStream_t s);

// ---- int8 digit-slice GEMM ------------------------------------------------------
struct GemmI8Args {
  const int8_t* Q; int S;          // [S][P][P]
  const int8_t* X; int SR;         // [SR][Rpad][P]
  int64_t P; int Rpad;
  int n, nrhs;
  const int32_t* row_exp;          // [P] or null
  const int32_t* col_exp;          // [nrhs]
  double c;                        // -h^2 / (M_S M_SR)
  const double* w;                 // [n] or null
  double* U; int64_t ldu;
  double* const* ucols;            // if not null, column r of the output is ucols[r]
  int variant;                     // kernel variant (0 .. gemm_i8_variants()-1)
  // split-K: ksplit > 1 workgroups share each tile, each over k in
  // [z*kchunk, (z+1)*kchunk) (kchunk a multiple of 128); their int32 class
  // sums go to part[z][class][Rpad][rows] (rows: the row tiles that run
  // split, times the tile height) and a second kernel adds them (exactly) and
  // applies the epilogue.  tail_rows > 0: only the last tail_rows row tiles
  // run split (the rest, whole rounds of resident workgroups, unsplit in a
  // launch of their own), so a short last round of tiles is spread over
  // ksplit times as many workgroups.
  int ksplit, kchunk;
  int32_t* part;
  int tail_rows;
  // row tiles of one launch: tiles mt0 .. mt0 + mtiles - 1 (mtiles = 0: all
  // from mt0 on); set by the launcher
  int mt0, mtiles;
  // bytes of k per operand row (the row stride); 0 means P (int8 digits)
  int64_t kbytes;
};
hipError_t launch_gemm_i8(const GemmI8Args& a, hipStream_t s);
// The same product for at most GEMV_I8_MAX_RHS right-hand sides as one pass
// over the digit planes (one wave per row; no k split needed, ksplit and part
// are ignored; ucols must be null).  Bit-identical to launch_gemm_i8.
constexpr int GEMV_I8_MAX_RHS = 4;
hipError_t launch_gemv_i8(const GemmI8Args& a, hipStream_t s);
// The same tiled product over bfloat16 split parts (G parts in Q as
// [S][P][P] bf16, right-hand-side parts in X as [S][Rpad][P] bf16, kbytes =
// 2P): products of parts p + q <= S-1 summed in two FP32 accumulators
// (leading part, corrections), u = c * (big + small) + w.  With ksplit > 1
// the splits' FP64 sums go to partf[z][r][m] and launch_splitk_reduce adds
// them.  col_exp and row_exp are unused.
hipError_t launch_gemm_bf16_parts(const GemmI8Args& a, double* partf, hipStream_t s);

// BF16x3 product on 128 x 256 tiles, one wave per SIMD (G parts [2+][P][P],
// rho parts [2][Rpad][P] with Rpad = 256 ceil(nrhs / 256)); with ksplit > 1
// the splits' FP64 sums go to part [ksplit][nrhs][nrows] and
// launch_splitk_reduce adds them.  u = alpha (hi hi + hi lo + lo hi) + w.
struct BF16W4Plan {
  int Rpad = 0, tilesM = 0, tilesN = 0, ksplit = 1, kchunk = 0;
};
BF16W4Plan bf16x3_w4_plan(int64_t P, int nrhs);
hipError_t launch_gemm_bf16x3_w4(const BF16W4Plan& p, const __bf16* Gb, int64_t P, const __bf16* Xb, int nrows,
                                 int nrhs, double alpha, const double* w, double* U, int64_t ldu, double* part,
                                 hipStream_t s);
int gemm_i8_variants();
// split plan for one apply with `variant` (ksplit = 1: none; tail_rows > 0:
// only the last tail_rows row tiles split, as in GemmI8Args)
void gemm_i8_split_plan(int64_t P, int Rpad, int variant, int* ksplit, int* kchunk, int* tail_rows);
// bytes of the int32 partial sums of such a plan (C classes)
size_t gemm_i8_part_bytes(int64_t P, int Rpad, int variant, int C, int ksplit, int tail_rows);

// Grouped int8 product: several operators (same S and SR) in one launch.
// Group g owns global tiles [tile0, tile0 + tilesM*tilesN) of the launch, tiles
// of gemm_i8_tile_rows(variant) rows x 128 right-hand sides; a.variant is
// ignored (the launch's variant applies to every group).
struct GemmI8Group {
  GemmI8Args a;
  int tilesM, tilesN;
  int tile0;
  int _pad;
};
int gemm_i8_tile_rows(int variant);
hipError_t launch_gemm_i8_grouped(const GemmI8Group* d_groups, int ngroups, int total_tiles, int S, int SR,
                                  int variant, hipStream_t s);

// Grouped rho quantisation: workgroups [col0, col0 + Rpad) serve group g.
struct QuantColsGroup {
  const double* const* xcols;   // nrhs column pointers
  int8_t* Xq;                   // [SR][Rpad][P]
  int32_t* f;                   // [Rpad]
  int64_t P;
  int n, nrhs, Rpad, col0;
};
// wide: every group's columns hold 16385 .. 40960 entries (quantize_cols_wide),
// read by 1024-thread workgroups; otherwise 256-thread workgroups
bool quantize_cols_wide(int n);
hipError_t launch_quantize_cols_grouped(const QuantColsGroup* groups, int ngroups, int total_cols, int SR, bool wide,
                                        hipStream_t s);
hipError_t launch_fill_random_i8(int8_t* p, size_t n, uint32_t seed, hipStream_t s);

// ---- split precision ----------------------------------------------------------
int64_t tile16_ld(int n);
int tile16_tiles(int n);
hipError_t launch_quantize_tiles16(const double* G, int64_t ldg, int n, int trans, int16_t* Q, int* E,
                                   hipStream_t s);
hipError_t launch_gemv_tile16(const int16_t* Q, const int* E, int n, const double* X, int64_t ldx, int nrhs,
                              double h, const double* bias, double* U, int64_t ldu, hipStream_t s);
hipError_t launch_make_fp32(const double* G, int64_t ldg, int n, float* G32, hipStream_t s);
hipError_t launch_make_bf16_parts(const double* G, int64_t ldg, int n, int parts, __bf16* Gb,
                                  hipStream_t s);
hipError_t launch_gemm_split(int mode, const pinv_op_s* op, const double* X, int64_t ldx,
                             int nrhs, double alpha, double* U, int64_t ldu, hipStream_t s,
                             void* scratch, size_t scratch_bytes);
size_t split_scratch_bytes(int mode, const pinv_op_s* op, int nrhs);

// ---- symmetric-packed FP64 ------------------------------------------------------
int sym_blocks_per_side(int n);
size_t sym_packed_elems(int n);
// scratch for launch_gemv_sym (partials of up to 8 right-hand sides)
size_t sym_scratch_bytes(int n, int nrhs);
hipError_t launch_sym_check(const double* G, int64_t ld, int n, double tol, int* flag, hipStream_t s);
hipError_t launch_pack_upper(const double* G, int64_t ld, int n, double* Gp, hipStream_t s);
// U = alpha * G X + bias from the packed copy; Y: sym_scratch_bytes(n, nrhs)
hipError_t launch_gemv_sym(const double* Gp, int n, const double* X, int64_t ldx, int nrhs, double alpha,
                           const double* bias, double* U, int64_t ldu, double* Y, hipStream_t s);

// ---- gradient ------------------------------------------------------------------
// nz = 0 for the 2-D operator.  part: scratch of grad_eps_chunks(nrhs) * (nodes)
// doubles (unused when that is <= 1)
int grad_eps_chunks(int nrhs);
// Eq. 3: dLoss/dbeta [4][ny][nx]; part: 4 * chunks * nodes doubles
hipError_t launch_grad_beta(int nx, int ny, const double* u, int64_t ldu, const double* lam, int64_t ldl, int nrhs,
                            const double* ub, double* part, double* grad, hipStream_t s);
// non-uniform grid (x, y: device node coordinates): per-direction gradients
// gx, gy [ny][nx], or their sum in gx when gy is null; part: 2 * chunks * nodes
hipError_t launch_grad_eps_general(int nx, int ny, const double* x, const double* y, const double* u, int64_t ldu,
                                   const double* lam, int64_t ldl, int nrhs, const double* ub, double* part,
                                   double* gx, double* gy, hipStream_t s);
hipError_t launch_grad_eps(int nx, int ny, int nz, double h, const double* u, int64_t ldu,
                           const double* lam, int64_t ldl, int nrhs, const double* ub,
                           double* part, double* grad, hipStream_t s);
