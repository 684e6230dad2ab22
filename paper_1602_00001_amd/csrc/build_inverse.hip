// One-time setup, steps 1-2 of "The solution steps": assemble the interior
// operator on the device and invert it.
//
// Step 1 (Eq. 1 in conservative form, Eq. 2 for eps = 1): for interior node p
// and each of its 4 faces f to node q, K[p][p] += eps_f and K[p][q] = -eps_f
// when q is interior; when q is a boundary node its Dirichlet value moves to
// the right-hand side, b_B[p] += eps_f * u_B(q).  eps_f is the mean of the two
// nodal permittivities.
//
// Step 2 ("any standard matrix inversion method"): K is symmetric positive
// definite, so it is factored K = L L^T by a right-looking blocked Cholesky
// (64-wide blocks; the diagonal block is factored and its triangular inverse
// formed in LDS by one workgroup, the panel and the trailing update are FP64
// matrix-core GEMMs), then W = L^{-1} is formed by blocked forward
// substitution and G = K^{-1} = W^T W by one more GEMM that skips the zero
// upper triangle of W.  A non-positive (or NaN) pivot raises a device flag
// that the host reads once at the end.
//
// Eq. 3 with arbitrary neighbour coefficients gives a unit-diagonal matrix
// that is not symmetric and, for mixed-sign coefficients, not diagonally
// dominant: it is factored P A = L U (L unit lower) with partial pivoting by
// the same right-looking blocking (each 64-column panel column by column:
// pivot search and row exchange, multipliers and the panel update; then the
// diagonal block's triangular inverses in LDS, the U panel and the trailing
// update as GEMMs), then X = L^{-1} by the forward substitution above,
// (P A)^{-1} = U^{-1} X by block back substitution, bottom block row first,
// and A^{-1} = (P A)^{-1} P by a column permutation.

#include "common.h"

namespace {

constexpr int NB = 64;

__global__ void assemble_kernel(int nx, int ny, const double* __restrict__ eps, const double* __restrict__ ub,
                                double* __restrict__ K, int64_t ldk, double* __restrict__ bB) {
  const int mx = nx - 2, my = ny - 2;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= mx * my) return;
  const int i = p / mx + 1, j = p % mx + 1;
  const int ni[4] = {i - 1, i + 1, i, i};
  const int nj[4] = {j, j, j - 1, j + 1};
  const double ep = eps ? eps[(int64_t)i * nx + j] : 1.0;
  double diag = 0.0, b = 0.0;
  for (int t = 0; t < 4; ++t) {
    const int k = ni[t], l = nj[t];
    const double eq = eps ? eps[(int64_t)k * nx + l] : 1.0;
    const double ef = 0.5 * (ep + eq);
    diag += ef;
    const bool bnd = (k == 0 || k == ny - 1 || l == 0 || l == nx - 1);
    if (bnd) {
      if (ub) b += ef * ub[(int64_t)k * nx + l];
    } else {
      const int q = (k - 1) * mx + (l - 1);
      if (K) K[(int64_t)p * ldk + q] = -ef;
    }
  }
  if (K) K[(int64_t)p * ldk + p] = diag;
  if (bB) bB[p] = b;
}

// The 7-point form on an n_z x n_y x n_x grid (nodal arrays [n_z][n_y][n_x];
// interior index p = ((k-1)(n_y-2) + (i-1))(n_x-2) + (j-1)): the same face
// rule over the 6 faces of each interior node.
__global__ void assemble_3d_kernel(int nx, int ny, int nz, const double* __restrict__ eps,
                                   const double* __restrict__ ub, double* __restrict__ K, int64_t ldk,
                                   double* __restrict__ bB) {
  const int mx = nx - 2, my = ny - 2, mz = nz - 2;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= mx * my * mz) return;
  const int k = p / (mx * my) + 1, i = (p / mx) % my + 1, j = p % mx + 1;
  const int nk[6] = {k - 1, k + 1, k, k, k, k};
  const int ni[6] = {i, i, i - 1, i + 1, i, i};
  const int nj[6] = {j, j, j, j, j - 1, j + 1};
  const int64_t node = ((int64_t)k * ny + i) * nx + j;
  const double ep = eps ? eps[node] : 1.0;
  double diag = 0.0, b = 0.0;
  for (int t = 0; t < 6; ++t) {
    const int a = nk[t], c = ni[t], d = nj[t];
    const int64_t q_node = ((int64_t)a * ny + c) * nx + d;
    const double eq = eps ? eps[q_node] : 1.0;
    const double ef = 0.5 * (ep + eq);
    diag += ef;
    const bool bnd = (a == 0 || a == nz - 1 || c == 0 || c == ny - 1 || d == 0 || d == nx - 1);
    if (bnd) {
      if (ub) b += ef * ub[q_node];
    } else {
      const int q = ((a - 1) * my + (c - 1)) * mx + (d - 1);
      if (K) K[(int64_t)p * ldk + q] = -ef;
    }
  }
  if (K) K[(int64_t)p * ldk + p] = diag;
  if (bB) bB[p] = b;
}

// Non-uniform tensor grid, permittivity per direction (finite-volume form):
// node (i, j) owns the control volume A = (x[j+1]-x[j-1])/2 * (y[i+1]-y[i-1])/2;
// an x-face carries eps_x,f * (y[i+1]-y[i-1])/2 / |x_q - x_j|, a y-face
// eps_y,f * (x[j+1]-x[j-1])/2 / |y_q - y_i|, eps_f the mean of the two nodal
// values of that direction's field.  Writes the areas to A.
__global__ void assemble_general_kernel(int nx, int ny, const double* __restrict__ x, const double* __restrict__ y,
                                        const double* __restrict__ epsx, const double* __restrict__ epsy,
                                        const double* __restrict__ ub, double* __restrict__ K, int64_t ldk,
                                        double* __restrict__ bB, double* __restrict__ A) {
  const int mx = nx - 2, my = ny - 2;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= mx * my) return;
  if (!epsy) epsy = epsx;  // one field for both directions (null: eps = 1)
  const int i = p / mx + 1, j = p % mx + 1;
  const double wx = 0.5 * (x[j + 1] - x[j - 1]);
  const double wy = 0.5 * (y[i + 1] - y[i - 1]);
  const int ni[4] = {i - 1, i + 1, i, i};
  const int nj[4] = {j, j, j - 1, j + 1};
  double diag = 0.0, b = 0.0;
  for (int t = 0; t < 4; ++t) {
    const int k = ni[t], l = nj[t];
    double c;
    if (k == i) {
      const double ep = epsx ? epsx[(int64_t)i * nx + j] : 1.0, eq = epsx ? epsx[(int64_t)k * nx + l] : 1.0;
      c = 0.5 * (ep + eq) * wy / fabs(x[l] - x[j]);
    } else {
      const double ep = epsy ? epsy[(int64_t)i * nx + j] : 1.0, eq = epsy ? epsy[(int64_t)k * nx + l] : 1.0;
      c = 0.5 * (ep + eq) * wx / fabs(y[k] - y[i]);
    }
    diag += c;
    const bool bnd = (k == 0 || k == ny - 1 || l == 0 || l == nx - 1);
    if (bnd) {
      if (ub) b += c * ub[(int64_t)k * nx + l];
    } else {
      K[(int64_t)p * ldk + (k - 1) * mx + (l - 1)] = -c;
    }
  }
  K[(int64_t)p * ldk + p] = diag;
  bB[p] = b;
  A[p] = wx * wy;
}

// G[i][q] *= A[q]: the inverse then maps rho straight to u (u = -G rho + w)
__global__ void scale_columns_kernel(double* __restrict__ G, int64_t ld, int n, const double* __restrict__ A) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), q = (int)(idx % n);
    G[(int64_t)i * ld + q] *= A[q];
  }
}

// Factor the kn x kn diagonal block at (k0, k0) in place (lower triangle, zero
// upper) and write its triangular inverse to Wd (64 x 64, zero padded).
__global__ __launch_bounds__(256) void diag_block_kernel(double* __restrict__ A, int64_t lda, int k0, int kn,
                                                         double* __restrict__ Wd, int* __restrict__ flag) {
  __shared__ double L[NB][NB + 1];
  __shared__ double tmp[NB];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int i = idx / NB, j = idx % NB;
    L[i][j] = (i < kn && j <= i) ? A[(int64_t)(k0 + i) * lda + k0 + j] : 0.0;
  }
  __syncthreads();
  // unblocked right-looking Cholesky
  for (int j = 0; j < kn; ++j) {
    if (tid == 0) {
      double d = L[j][j];
      if (!(d > 0.0)) {
        *flag = 1;
        d = 1.0;
      }
      L[j][j] = sqrt(d);
    }
    __syncthreads();
    const double piv = L[j][j];
    for (int i = j + 1 + tid; i < kn; i += 256) L[i][j] = L[i][j] / piv;
    __syncthreads();
    const int rem = kn - j - 1;
    for (int idx = tid; idx < rem * rem; idx += 256) {
      const int i = j + 1 + idx / rem, c = j + 1 + idx % rem;
      if (c <= i) L[i][c] -= L[i][j] * L[c][j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < kn * kn; idx += 256) {
    const int i = idx / kn, j = idx % kn;
    A[(int64_t)(k0 + i) * lda + k0 + j] = (j <= i) ? L[i][j] : 0.0;
  }
  __syncthreads();
  // in-place inverse of the lower triangular factor, last column first:
  // Linv[j][j] = 1/L[j][j];  Linv[j+1:, j] = -Linv[j+1:, j+1:] L[j+1:, j] / L[j][j]
  for (int j = kn - 1; j >= 0; --j) {
    const double ljj = L[j][j];
    const int i = j + 1 + tid;
    if (tid < NB && i < kn) {
      double x = 0.0;
      for (int k = j + 1; k <= i; ++k) x += L[i][k] * L[k][j];
      tmp[i] = x;
    }
    __syncthreads();
    if (tid < NB && i < kn) L[i][j] = -tmp[i] / ljj;
    if (tid == 0) L[j][j] = 1.0 / ljj;
    __syncthreads();
  }
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int i = idx / NB, j = idx % NB;
    Wd[idx] = (i < kn && j <= i) ? L[i][j] : 0.0;
  }
}

// Eq. 3 on the interior unknowns: A[p][p] = 1, A[p][q] = -beta_d(p)/4 for the
// interior neighbour q in direction d (i-1, i+1, j-1, j+1 in that order), and
// b_B[p] = sum of beta_d(p)/4 * u_B(q) over the boundary neighbours.
// beta: [4][n_y][n_x].
__global__ void assemble_beta_kernel(int nx, int ny, const double* __restrict__ beta, const double* __restrict__ ub,
                                     double* __restrict__ K, int64_t ldk, double* __restrict__ bB) {
  const int mx = nx - 2, my = ny - 2;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= mx * my) return;
  const int i = p / mx + 1, j = p % mx + 1;
  const int ni[4] = {i - 1, i + 1, i, i};
  const int nj[4] = {j, j, j - 1, j + 1};
  const int64_t plane = (int64_t)nx * ny;
  double b = 0.0;
  for (int d = 0; d < 4; ++d) {
    const int k = ni[d], l = nj[d];
    const double c = 0.25 * beta[d * plane + (int64_t)i * nx + j];
    if (k == 0 || k == ny - 1 || l == 0 || l == nx - 1) {
      if (ub) b += c * ub[(int64_t)k * nx + l];
    } else {
      K[(int64_t)p * ldk + (k - 1) * mx + (l - 1)] = -c;
    }
  }
  K[(int64_t)p * ldk + p] = 1.0;
  bB[p] = b;
}

// The kn x kn diagonal block at (k0, k0) holds its L (unit lower, below the
// diagonal) and U (on and above it); write L^{-1} (unit lower) to Wl and U^{-1}
// (upper) to Wu, 64 x 64, zero padded.
__global__ __launch_bounds__(256) void lu_diag_inverse_kernel(const double* __restrict__ A, int64_t lda, int k0,
                                                              int kn, double* __restrict__ Wl,
                                                              double* __restrict__ Wu) {
  __shared__ double F[NB][NB + 1];
  __shared__ double tmp[NB];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int i = idx / NB, j = idx % NB;
    F[i][j] = (i < kn && j < kn) ? A[(int64_t)(k0 + i) * lda + k0 + j] : 0.0;
  }
  __syncthreads();
  // L^{-1} in place below the diagonal, last column first:
  //   Linv[i][j] = -(L[i][j] + sum_{j<k<i} Linv[i][k] L[k][j])  (i > j)
  for (int j = kn - 1; j >= 0; --j) {
    const int i = j + 1 + tid;
    if (tid < NB && i < kn) {
      double x = F[i][j];
      for (int k = j + 1; k < i; ++k) x += F[i][k] * F[k][j];
      tmp[i] = x;
    }
    __syncthreads();
    if (tid < NB && i < kn) F[i][j] = -tmp[i];
    __syncthreads();
  }
  // U^{-1} in place on and above the diagonal, last row first:
  //   Uinv[i][i] = 1/U[i][i],  Uinv[i][j] = -(sum_{i<k<=j} U[i][k] Uinv[k][j]) / U[i][i]  (j > i)
  for (int i = kn - 1; i >= 0; --i) {
    const double uii = F[i][i];
    const int j = i + 1 + tid;
    if (tid < NB && j < kn) {
      double x = 0.0;
      for (int k = i + 1; k <= j; ++k) x += F[i][k] * F[k][j];
      tmp[j] = x;
    }
    __syncthreads();
    if (tid < NB && j < kn) F[i][j] = -tmp[j] / uii;
    if (tid == 0) F[i][i] = 1.0 / uii;
    __syncthreads();
  }
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int i = idx / NB, j = idx % NB;
    const bool in = i < kn && j < kn;
    Wl[idx] = in ? (i == j ? 1.0 : (j < i ? F[i][j] : 0.0)) : 0.0;
    Wu[idx] = (in && j >= i) ? F[i][j] : 0.0;
  }
}

// Partial pivoting at column c (LU with row exchanges, the standard way of
// inverting a general matrix): the pivot row p is the first row r >= c of
// largest |A[r][c]|; rows c and p are exchanged over all n columns (the L
// columns already formed to their left included, so the factors end up those
// of P A) and perm[c], perm[p] with them.  No finite non-zero candidate (a
// singular matrix) sets *flag and puts 1 on the diagonal so the remaining
// arithmetic stays finite.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void lu_pivot_kernel(double* __restrict__ A, int64_t lda, int n, int c,
                                                        int* __restrict__ perm, int* __restrict__ flag) {
  __shared__ double sv[16];
  __shared__ int si[16];
  __shared__ int sp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double best = -1.0;
  int bi = n;
  for (int r = c + tid; r < n; r += 1024) {
    const double v = fabs(A[(int64_t)r * lda + c]);
    if (v > best) {  // rows ascend per thread: the first of equal values is kept
      best = v;
      bi = r;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const double ov = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    sv[wave] = best;
    si[wave] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 16; ++w)
      if (sv[w] > best || (sv[w] == best && si[w] < bi)) {
        best = sv[w];
        bi = si[w];
      }
    if (!(best > 0.0 && best < INFINITY) || bi >= n) {
      *flag = 1;
      A[(int64_t)c * lda + c] = 1.0;
      bi = c;
    }
    sp = bi;
    if (bi != c) {
      const int t = perm[c];
      perm[c] = perm[bi];
      perm[bi] = t;
    }
  }
  __syncthreads();
  const int p = sp;
  if (p == c) return;
  double* rc = A + (int64_t)c * lda;
  double* rp = A + (int64_t)p * lda;
  for (int j = tid; j < n; j += 1024) {
    const double t = rc[j];
    rc[j] = rp[j];
    rp[j] = t;
  }
}

// Column c of the panel whose columns end at cend: every row r > c gets its
// multiplier l = A[r][c] / A[c][c] (stored in place) and the rank-one update
// A[r][j] -= l A[c][j] of the panel's columns right of c.  One thread per row.
__global__ __launch_bounds__(256) void lu_panel_column_kernel(double* __restrict__ A, int64_t lda, int n, int c,
                                                              int cend) {
  const int r = c + 1 + blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  double* row = A + (int64_t)r * lda;
  const double* prow = A + (int64_t)c * lda;
  const double l = row[c] / prow[c];
  row[c] = l;
  for (int j = c + 1; j < cend; ++j) row[j] -= l * prow[j];
}

__global__ void iota_kernel(int* __restrict__ perm, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) perm[i] = i;
}

// G[:, perm[i]] = -Y[:, i]: with P A = L U and Y = U^{-1} L^{-1} = (P A)^{-1},
// A^{-1} = Y P and G = -A^{-1}.
__global__ void permute_negate_kernel(const double* __restrict__ Y, int64_t ld, int n, const int* __restrict__ perm,
                                      double* __restrict__ G) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx / n), i = (int)(idx % n);
    G[(int64_t)r * ld + perm[i]] = -Y[(int64_t)r * ld + i];
  }
}

__global__ void set_identity_kernel(double* __restrict__ A, int64_t lda, int n) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx / n, j = idx % n;
  A[(int64_t)i * lda + j] = (i == j) ? 1.0 : 0.0;
}

}  // namespace

hipError_t launch_assemble(int nx, int ny, int nz, const double* eps, const double* ub, double* K, int64_t ldk,
                           double* bB, hipStream_t s) {
  if (nz > 0) {
    const int n = (nx - 2) * (ny - 2) * (nz - 2);
    hipLaunchKernelGGL(assemble_3d_kernel, dim3((n + 255) / 256), dim3(256), 0, s, nx, ny, nz, eps, ub, K, ldk, bB);
    return hipGetLastError();
  }
  const int n = (nx - 2) * (ny - 2);
  hipLaunchKernelGGL(assemble_kernel, dim3((n + 255) / 256), dim3(256), 0, s, nx, ny, eps, ub, K, ldk, bB);
  return hipGetLastError();
}

// Fills op->G (allocated here), op->w.  eps_dev / ub_dev: device nodal arrays or null.
// gen: non-uniform grid data (device), or null for the uniform 2-D / 3-D forms;
// then eps_dev is eps_x.
int32_t build_inverse_device(pinv_op op, const double* eps_dev, const double* ub_dev, const GeneralGrid* gen,
                             hipStream_t s) {
  const int n = op->n;
  const int64_t ld = op->ldg;
  const int nblk = (n + NB - 1) / NB;
  double *Kb = nullptr, *Wb = nullptr, *Wd = nullptr, *bB = nullptr;
  int* flag = nullptr;
  int32_t st = PINV_OK;
  hipError_t e;
  const size_t mat_bytes = (size_t)n * (size_t)ld * sizeof(double);

#define PINV_BAIL(expr)                 \
  do {                                  \
    e = (expr);                         \
    if (e != hipSuccess) {              \
      st = pinv_hip_status(e);          \
      goto done;                        \
    }                                   \
  } while (0)

  PINV_BAIL(hipMalloc(&Kb, mat_bytes));
  PINV_BAIL(hipMalloc(&Wb, mat_bytes));
  PINV_BAIL(hipMalloc(&Wd, (size_t)nblk * NB * NB * sizeof(double)));
  PINV_BAIL(hipMalloc(&bB, (size_t)n * sizeof(double)));
  PINV_BAIL(hipMalloc(&flag, sizeof(int)));
  PINV_BAIL(hipMemsetAsync(flag, 0, sizeof(int), s));
  PINV_BAIL(hipMemsetAsync(Kb, 0, mat_bytes, s));
  PINV_BAIL(hipMemsetAsync(Wb, 0, mat_bytes, s));
  if (gen) {
    hipLaunchKernelGGL(assemble_general_kernel, dim3((n + 255) / 256), dim3(256), 0, s, op->nx, op->ny, gen->x, gen->y,
                       eps_dev, gen->eps_y, ub_dev, Kb, ld, bB, gen->area);
    PINV_BAIL(hipGetLastError());
  } else {
    PINV_BAIL(launch_assemble(op->nx, op->ny, op->nz, eps_dev, ub_dev, Kb, ld, bB, s));
  }

  // Cholesky, L overwrites the lower triangle of Kb
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = kb * NB, kn = (n - k0 < NB) ? n - k0 : NB;
    double* wd = Wd + (size_t)kb * NB * NB;
    hipLaunchKernelGGL(diag_block_kernel, dim3(1), dim3(256), 0, s, Kb, ld, k0, kn, wd, flag);
    PINV_BAIL(hipGetLastError());
    const int r0 = k0 + kn, rn = n - r0;
    if (rn <= 0) continue;
    GemmF64Args p{};
    p.A = Kb + (int64_t)r0 * ld + k0; p.lda = ld; p.a_kcontig = 1;
    p.B = wd; p.ldb = NB; p.b_kcontig = 1;
    p.C = Kb + (int64_t)r0 * ld + k0; p.csm = ld; p.csn = 1;
    p.M = rn; p.N = kn; p.K = kn; p.alpha = 1.0; p.beta = 0.0;
    PINV_BAIL(launch_gemm_f64(p, s));
    GemmF64Args t{};
    t.A = Kb + (int64_t)r0 * ld + k0; t.lda = ld; t.a_kcontig = 1;
    t.B = Kb + (int64_t)r0 * ld + k0; t.ldb = ld; t.b_kcontig = 1;
    t.C = Kb + (int64_t)r0 * ld + r0; t.csm = ld; t.csn = 1;
    t.M = rn; t.N = rn; t.K = kn; t.alpha = -1.0; t.beta = 1.0; t.tri = 1;
    PINV_BAIL(launch_gemm_f64(t, s));
  }

  // W = L^{-1}: block row i is Wd_i (E_i - sum_{k<i} L_ik W_k), accumulated right-looking in Wb
  for (int ib = 0; ib < nblk; ++ib) {
    const int i0 = ib * NB, in_ = (n - i0 < NB) ? n - i0 : NB;
    const double* wd = Wd + (size_t)ib * NB * NB;
    hipLaunchKernelGGL(set_identity_kernel, dim3((in_ * in_ + 255) / 256), dim3(256), 0, s, Wb + (int64_t)i0 * ld + i0,
                       ld, in_);
    PINV_BAIL(hipGetLastError());
    GemmF64Args a{};
    a.A = wd; a.lda = NB; a.a_kcontig = 1;
    a.B = Wb + (int64_t)i0 * ld; a.ldb = ld; a.b_kcontig = 0;
    a.C = Wb + (int64_t)i0 * ld; a.csm = ld; a.csn = 1;
    a.M = in_; a.N = i0 + in_; a.K = in_; a.alpha = 1.0; a.beta = 0.0;
    PINV_BAIL(launch_gemm_f64(a, s));
    const int r0 = i0 + in_, rn = n - r0;
    if (rn <= 0) continue;
    GemmF64Args b{};
    b.A = Kb + (int64_t)r0 * ld + i0; b.lda = ld; b.a_kcontig = 1;
    b.B = Wb + (int64_t)i0 * ld; b.ldb = ld; b.b_kcontig = 0;
    b.C = Wb + (int64_t)r0 * ld; b.csm = ld; b.csn = 1;
    b.M = rn; b.N = r0; b.K = in_; b.alpha = -1.0; b.beta = 1.0;
    PINV_BAIL(launch_gemm_f64(b, s));
  }

  // G = W^T W (into Kb)
  {
    GemmF64Args g{};
    g.A = Wb; g.lda = ld; g.a_kcontig = 0;
    g.B = Wb; g.ldb = ld; g.b_kcontig = 0;
    g.C = Kb; g.csm = ld; g.csn = 1;
    g.M = n; g.N = n; g.K = n; g.alpha = 1.0; g.beta = 0.0; g.kdiag = 1;
    PINV_BAIL(launch_gemm_f64(g, s));
  }
  if (ub_dev) {
    PINV_BAIL(hipMalloc(&op->w, (size_t)n * sizeof(double)));
    op->bytes += (int64_t)n * sizeof(double);
    PINV_BAIL(launch_gemv_f64(Kb, ld, n, bB, n, 1, 1.0, nullptr, op->w, n, s));
  }
  if (gen) {
    // after the lift (w = K^{-1} b_B): fold the control volumes into G's columns
    hipLaunchKernelGGL(scale_columns_kernel, dim3(grid_1d((int64_t)n * n)), dim3(256), 0, s, Kb, ld,
                       n, (const double*)gen->area);
    PINV_BAIL(hipGetLastError());
  }
  {
    int hflag = 0;
    PINV_BAIL(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PINV_BAIL(hipStreamSynchronize(s));
    if (hflag) {
      st = PINV_E_NOT_SPD;
      goto done;
    }
  }
  op->G = Kb;
  op->bytes += (int64_t)mat_bytes;
  Kb = nullptr;

done:
#undef PINV_BAIL
  if (st != PINV_OK) (void)hipStreamSynchronize(s);
  if (Kb) (void)hipFree(Kb);
  if (Wb) (void)hipFree(Wb);
  if (Wd) (void)hipFree(Wd);
  if (bB) (void)hipFree(bB);
  if (flag) (void)hipFree(flag);
  return st;
}

// Eq. 3: fills op->G with -A^{-1} (so that u = -G rho + w = A^{-1}(rho + b_B)
// with h = 1) and op->w = A^{-1} b_B when ub_dev is given.  beta_dev: device
// [4][n_y][n_x].  P A = L U by a blocked right-looking factorization with
// partial pivoting: per 64-column panel, a pivot search and row exchange
// (lu_pivot_kernel) and a column update (lu_panel_column_kernel) per column,
// then the diagonal block's triangular inverses, the U panel L11^{-1} A12 and
// the trailing update as FP64 GEMMs.  PINV_E_NOT_SPD if A is singular (a
// column with no non-zero finite pivot).
int32_t build_inverse_lu_device(pinv_op op, const double* beta_dev, const double* ub_dev, hipStream_t s) {
  const int n = op->n;
  const int64_t ld = op->ldg;
  const int nblk = (n + NB - 1) / NB;
  double *Kb = nullptr, *Wb = nullptr, *Wl = nullptr, *Wu = nullptr, *bB = nullptr;
  int* flag = nullptr;
  int* perm = nullptr;
  int32_t st = PINV_OK;
  hipError_t e;
  const size_t mat_bytes = (size_t)n * (size_t)ld * sizeof(double);

#define PINV_BAIL(expr)                 \
  do {                                  \
    e = (expr);                         \
    if (e != hipSuccess) {              \
      st = pinv_hip_status(e);          \
      goto done;                        \
    }                                   \
  } while (0)

  PINV_BAIL(hipMalloc(&Kb, mat_bytes));
  PINV_BAIL(hipMalloc(&Wb, mat_bytes));
  PINV_BAIL(hipMalloc(&Wl, (size_t)nblk * NB * NB * sizeof(double)));
  PINV_BAIL(hipMalloc(&Wu, (size_t)nblk * NB * NB * sizeof(double)));
  PINV_BAIL(hipMalloc(&bB, (size_t)n * sizeof(double)));
  PINV_BAIL(hipMalloc(&flag, sizeof(int)));
  PINV_BAIL(hipMalloc(&perm, (size_t)n * sizeof(int)));
  PINV_BAIL(hipMemsetAsync(flag, 0, sizeof(int), s));
  PINV_BAIL(hipMemsetAsync(Kb, 0, mat_bytes, s));
  PINV_BAIL(hipMemsetAsync(Wb, 0, mat_bytes, s));
  hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, s, perm, n);
  PINV_BAIL(hipGetLastError());
  hipLaunchKernelGGL(assemble_beta_kernel, dim3((n + 255) / 256), dim3(256), 0, s, op->nx, op->ny, beta_dev, ub_dev, Kb,
                     ld, bB);
  PINV_BAIL(hipGetLastError());

  // P A = L U in place: L below the diagonal (unit diagonal implied), U on and above
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = kb * NB, kn = (n - k0 < NB) ? n - k0 : NB;
    double* wl = Wl + (size_t)kb * NB * NB;
    double* wu = Wu + (size_t)kb * NB * NB;
    // the panel's columns, one at a time: pivot and exchange, then multipliers
    // and the update of the panel's columns to the right (L21 is complete
    // after the last column)
    for (int c = k0; c < k0 + kn; ++c) {
      hipLaunchKernelGGL(lu_pivot_kernel, dim3(1), dim3(1024), 0, s, Kb, ld, n, c, perm, flag);
      PINV_BAIL(hipGetLastError());
      if (c + 1 < n) {
        hipLaunchKernelGGL(lu_panel_column_kernel, dim3((n - c - 1 + 255) / 256), dim3(256), 0, s, Kb, ld, n, c,
                           k0 + kn);
        PINV_BAIL(hipGetLastError());
      }
    }
    hipLaunchKernelGGL(lu_diag_inverse_kernel, dim3(1), dim3(256), 0, s, Kb, ld, k0, kn, wl, wu);
    PINV_BAIL(hipGetLastError());
    const int r0 = k0 + kn, rn = n - r0;
    if (rn <= 0) continue;
    // U panel: A[k, r0:] <- L_kk^{-1} A[k, r0:] (in place: one 128-row tile holds all kn <= 64 rows)
    GemmF64Args q{};
    q.A = wl; q.lda = NB; q.a_kcontig = 1;
    q.B = Kb + (int64_t)k0 * ld + r0; q.ldb = ld; q.b_kcontig = 0;
    q.C = Kb + (int64_t)k0 * ld + r0; q.csm = ld; q.csn = 1;
    q.M = kn; q.N = rn; q.K = kn; q.alpha = 1.0; q.beta = 0.0;
    PINV_BAIL(launch_gemm_f64(q, s));
    // trailing update A[r0:, r0:] -= L panel * U panel
    GemmF64Args t{};
    t.A = Kb + (int64_t)r0 * ld + k0; t.lda = ld; t.a_kcontig = 1;
    t.B = Kb + (int64_t)k0 * ld + r0; t.ldb = ld; t.b_kcontig = 0;
    t.C = Kb + (int64_t)r0 * ld + r0; t.csm = ld; t.csn = 1;
    t.M = rn; t.N = rn; t.K = kn; t.alpha = -1.0; t.beta = 1.0;
    PINV_BAIL(launch_gemm_f64(t, s));
  }

  // X = L^{-1} in Wb: block row i is Wl_i (E_i - sum_{k<i} L_ik X_k), accumulated right-looking
  for (int ib = 0; ib < nblk; ++ib) {
    const int i0 = ib * NB, in_ = (n - i0 < NB) ? n - i0 : NB;
    hipLaunchKernelGGL(set_identity_kernel, dim3((in_ * in_ + 255) / 256), dim3(256), 0, s, Wb + (int64_t)i0 * ld + i0,
                       ld, in_);
    PINV_BAIL(hipGetLastError());
    GemmF64Args a{};
    a.A = Wl + (size_t)ib * NB * NB; a.lda = NB; a.a_kcontig = 1;
    a.B = Wb + (int64_t)i0 * ld; a.ldb = ld; a.b_kcontig = 0;
    a.C = Wb + (int64_t)i0 * ld; a.csm = ld; a.csn = 1;
    a.M = in_; a.N = i0 + in_; a.K = in_; a.alpha = 1.0; a.beta = 0.0;
    PINV_BAIL(launch_gemm_f64(a, s));
    const int r0 = i0 + in_, rn = n - r0;
    if (rn <= 0) continue;
    GemmF64Args b{};
    b.A = Kb + (int64_t)r0 * ld + i0; b.lda = ld; b.a_kcontig = 1;
    b.B = Wb + (int64_t)i0 * ld; b.ldb = ld; b.b_kcontig = 0;
    b.C = Wb + (int64_t)r0 * ld; b.csm = ld; b.csn = 1;
    b.M = rn; b.N = r0; b.K = in_; b.alpha = -1.0; b.beta = 1.0;
    PINV_BAIL(launch_gemm_f64(b, s));
  }

  // A^{-1} = U^{-1} X in Wb, bottom block row first: row block i becomes
  // Wu_i Z_i, then Z[0:i0] -= U[0:i0, i] (row block i)
  for (int ib = nblk - 1; ib >= 0; --ib) {
    const int i0 = ib * NB, in_ = (n - i0 < NB) ? n - i0 : NB;
    GemmF64Args a{};
    a.A = Wu + (size_t)ib * NB * NB; a.lda = NB; a.a_kcontig = 1;
    a.B = Wb + (int64_t)i0 * ld; a.ldb = ld; a.b_kcontig = 0;
    a.C = Wb + (int64_t)i0 * ld; a.csm = ld; a.csn = 1;
    a.M = in_; a.N = n; a.K = in_; a.alpha = 1.0; a.beta = 0.0;
    PINV_BAIL(launch_gemm_f64(a, s));
    if (i0 == 0) continue;
    GemmF64Args b{};
    b.A = Kb + i0; b.lda = ld; b.a_kcontig = 1;
    b.B = Wb + (int64_t)i0 * ld; b.ldb = ld; b.b_kcontig = 0;
    b.C = Wb; b.csm = ld; b.csn = 1;
    b.M = i0; b.N = n; b.K = in_; b.alpha = -1.0; b.beta = 1.0;
    PINV_BAIL(launch_gemm_f64(b, s));
  }

  // G = -(P A)^{-1} P, into Kb (its factors are no longer read); w = -G b_B
  hipLaunchKernelGGL(permute_negate_kernel, dim3(grid_1d((int64_t)n * n)), dim3(256), 0, s, Wb, ld,
                     n, perm, Kb);
  PINV_BAIL(hipGetLastError());
  if (ub_dev) {
    PINV_BAIL(hipMalloc(&op->w, (size_t)n * sizeof(double)));
    op->bytes += (int64_t)n * sizeof(double);
    PINV_BAIL(launch_gemv_f64(Kb, ld, n, bB, n, 1, -1.0, nullptr, op->w, n, s));
  }
  {
    int hflag = 0;
    PINV_BAIL(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PINV_BAIL(hipStreamSynchronize(s));
    if (hflag) {
      st = PINV_E_NOT_SPD;
      goto done;
    }
  }
  op->G = Kb;
  op->bytes += (int64_t)mat_bytes;
  Kb = nullptr;

done:
#undef PINV_BAIL
  if (st != PINV_OK) (void)hipStreamSynchronize(s);
  if (Kb) (void)hipFree(Kb);
  if (Wb) (void)hipFree(Wb);
  if (Wl) (void)hipFree(Wl);
  if (Wu) (void)hipFree(Wu);
  if (bB) (void)hipFree(bB);
  if (flag) (void)hipFree(flag);
  if (perm) (void)hipFree(perm);
  return st;
}
