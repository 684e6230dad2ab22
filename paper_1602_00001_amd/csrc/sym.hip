// Symmetric-packed FP64 storage of the inverse for the pass-over-G regime
// (few right-hand sides, bound by HBM bandwidth): G = K^{-1} is symmetric
// (K is), so only the 64 x 64 blocks (I, J) with J >= I are kept, each
// row-major and zero padded past N, block row by block row:
//   packed index of (I, J) = I nb - I (I - 1) / 2 + (J - I),  nb = ceil(N / 64).
// That is about half the bytes of the full matrix.
//
// Apply (u = alpha G x + bias for up to 8 right-hand sides per pass): one
// workgroup per stored block reads it once and forms both of its products,
// B x_J (its contribution to rows I) and, off the diagonal, B^T x_I (to rows
// J), into a partial array Y[r][I][J][64]; a second kernel adds the partials
// of each block row in a fixed order, so the result is deterministic.

#include "common.h"

namespace {

constexpr int SB = 64;

__device__ inline int64_t block_row_start(int I, int nb) { return (int64_t)I * nb - (int64_t)I * (I - 1) / 2; }

// (I, J) of packed block b
__device__ inline void block_of(int64_t b, int nb, int& I, int& J) {
  const double t = 2.0 * nb + 1.0;
  int i = (int)((t - sqrt(t * t - 8.0 * (double)b)) * 0.5);
  if (i < 0) i = 0;
  if (i > nb - 1) i = nb - 1;
  while (i > 0 && block_row_start(i, nb) > b) --i;
  while (i + 1 < nb && block_row_start(i + 1, nb) <= b) ++i;
  I = i;
  J = i + (int)(b - block_row_start(i, nb));
}

// flag = 1 if some |G[i][j] - G[j][i]| with i < j exceeds tol sqrt(|G[i][i]
// G[j][j]|) (the scale of a symmetric positive definite matrix's entries;
// tol = 0 asks for exact symmetry; a NaN fails the test).  One workgroup per
// 64 x 64 block pair (I, J), J >= I: block (J, I) is read into LDS by rows
// (coalesced) and compared, transposed, with block (I, J).
__global__ __launch_bounds__(256) void sym_check_kernel(const double* __restrict__ G, int64_t ld, int n, int nb,
                                                        double tol, int* __restrict__ flag) {
  __shared__ double t[SB][SB + 1];
  int I, J;
  block_of(blockIdx.x, nb, I, J);
  for (int e = threadIdx.x; e < SB * SB; e += 256) {
    const int r = e / SB, c = e % SB;
    const int row = J * SB + r, col = I * SB + c;
    t[c][r] = (row < n && col < n) ? G[(int64_t)row * ld + col] : 0.0;
  }
  __syncthreads();
  bool bad = false;
  for (int e = threadIdx.x; e < SB * SB; e += 256) {
    const int r = e / SB, c = e % SB;
    const int i = I * SB + r, j = J * SB + c;
    if (i >= n || j >= n || i >= j) continue;
    const double d = fabs(G[(int64_t)i * ld + j] - t[r][c]);
    const double scale = sqrt(fabs(G[(int64_t)i * ld + i] * G[(int64_t)j * ld + j]));
    bad = bad || !(d <= tol * scale);
  }
  if (bad) *flag = 1;
}

__global__ __launch_bounds__(256) void pack_upper_kernel(const double* __restrict__ G, int64_t ld, int n, int nb,
                                                         double* __restrict__ Gp) {
  int I, J;
  block_of(blockIdx.x, nb, I, J);
  double* dst = Gp + (int64_t)blockIdx.x * SB * SB;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = threadIdx.x * 16 + k;
    const int gi = I * SB + e / SB, gj = J * SB + e % SB;
    dst[e] = (gi < n && gj < n) ? G[(int64_t)gi * ld + gj] : 0.0;
  }
}

// Thread t holds a 4 x 4 tile of the block: rows 4a .. 4a+3 and columns
// 4b .. 4b+3 with b = t % 16, a = t / 16, so the 16 lanes sharing a read the
// tile rows as 512 contiguous bytes each.  A row sum is 4 local products plus
// a reduction over the 16 lanes of b (lane bits 0-3); a column sum (blocks off
// the diagonal) is 4 local products plus a reduction over a: lane bits 4-5 by
// shuffles, then the 4 waves through LDS.
template <int NR>
__global__ __launch_bounds__(256) void sym_block_kernel(const double* __restrict__ Gp, int n, int nb,
                                                        const double* __restrict__ X, int64_t ldx,
                                                        double* __restrict__ Y) {
  __shared__ double part[4][NR][SB];
  int I, J;
  block_of(blockIdx.x, nb, I, J);
  const int tid = threadIdx.x;
  const int b = tid & 15, a = tid >> 4;
  const int wave = tid >> 6;
  const double* B = Gp + (int64_t)blockIdx.x * SB * SB + (4 * a) * SB + 4 * b;
  double t[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 v0 = *(const double2*)(B + i * SB);
    const double2 v1 = *(const double2*)(B + i * SB + 2);
    t[i][0] = v0.x;
    t[i][1] = v0.y;
    t[i][2] = v1.x;
    t[i][3] = v1.y;
  }
  const int64_t nbb = nb;
  const bool off = J != I;  // uniform per workgroup
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const double* x = X + (int64_t)q * ldx;
    // x_J at this thread's columns (zero past N), x_I at its rows
    double xj[4], xi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int col = J * SB + 4 * b + k;
      const double v = x[min(col, n - 1)];
      xj[k] = col < n ? v : 0.0;
      const int row = I * SB + 4 * a + k;
      const double w = x[min(row, n - 1)];
      xi[k] = row < n ? w : 0.0;
    }
    double rs[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double v = t[i][0] * xj[0];
#pragma unroll
      for (int k = 1; k < 4; ++k) v = fma(t[i][k], xj[k], v);
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
      rs[i] = v;
    }
    if (b == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) Y[(((int64_t)q * nbb + I) * nbb + J) * SB + 4 * a + i] = rs[i];
    }
    if (off) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double v = t[0][k] * xi[0];
#pragma unroll
        for (int i = 1; i < 4; ++i) v = fma(t[i][k], xi[i], v);
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if ((a & 3) == 0) part[wave][q][4 * b + k] = v;
      }
    }
  }
  if (!off) return;
  __syncthreads();
  if (tid < SB) {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const double v = ((part[0][q][tid] + part[1][q][tid]) + part[2][q][tid]) + part[3][q][tid];
      Y[(((int64_t)q * nbb + J) * nbb + I) * SB + tid] = v;
    }
  }
}

// u[q][i] = alpha * sum_J Y[q][i / 64][J][i % 64] (+ bias[i]).  Workgroup
// (I, q) covers the 64 rows of block row I; wave w adds the partials of J in
// its quarter of 0 .. nb-1 in order (eight loads in flight), then the four
// quarter sums are added in order: a fixed summation order.
__global__ __launch_bounds__(256) void sym_reduce_kernel(const double* __restrict__ Y, int n, int nb,
                                                         double alpha, const double* __restrict__ bias,
                                                         double* __restrict__ U, int64_t ldu) {
  __shared__ double qs[4][SB];
  const int I = blockIdx.x, q = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int per = (nb + 3) / 4;
  const int j0 = min(nb, w * per), j1 = min(nb, j0 + per);
  const double* y = Y + (((int64_t)q * nb + I) * nb) * SB + lane;
  double s = 0.0;
  int J = j0;
  for (; J + 8 <= j1; J += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = y[(int64_t)(J + k) * SB];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  for (; J < j1; ++J) s += y[(int64_t)J * SB];
  qs[w][lane] = s;
  __syncthreads();
  const int i = I * SB + threadIdx.x;
  if (threadIdx.x < SB && i < n) {
    const double t = ((qs[0][threadIdx.x] + qs[1][threadIdx.x]) + qs[2][threadIdx.x]) + qs[3][threadIdx.x];
    double v = alpha * t;
    if (bias) v += bias[i];
    U[(int64_t)q * ldu + i] = v;
  }
}

}  // namespace

int sym_blocks_per_side(int n) { return (n + SB - 1) / SB; }

size_t sym_packed_elems(int n) {
  const size_t nb = (size_t)sym_blocks_per_side(n);
  return nb * (nb + 1) / 2 * SB * SB;
}

size_t sym_scratch_bytes(int n, int nrhs) {
  const size_t nb = (size_t)sym_blocks_per_side(n);
  const size_t nr = nrhs < 8 ? (size_t)nrhs : 8;
  return nr * nb * nb * SB * sizeof(double);
}

hipError_t launch_sym_check(const double* G, int64_t ld, int n, double tol, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nb = sym_blocks_per_side(n);
  const int64_t blocks = (int64_t)nb * (nb + 1) / 2;
  hipLaunchKernelGGL(sym_check_kernel, dim3((unsigned)blocks), dim3(256), 0, s, G, ld, n, nb, tol, flag);
  return hipGetLastError();
}

hipError_t launch_pack_upper(const double* G, int64_t ld, int n, double* Gp, hipStream_t s) {
  const int nb = sym_blocks_per_side(n);
  const int64_t blocks = (int64_t)nb * (nb + 1) / 2;
  hipLaunchKernelGGL(pack_upper_kernel, dim3((unsigned)blocks), dim3(256), 0, s, G, ld, n, nb, Gp);
  return hipGetLastError();
}

hipError_t launch_gemv_sym(const double* Gp, int n, const double* X, int64_t ldx, int nrhs, double alpha,
                           const double* bias, double* U, int64_t ldu, double* Y, hipStream_t s) {
  const int nb = sym_blocks_per_side(n);
  const int64_t blocks = (int64_t)nb * (nb + 1) / 2;
  for (int r0 = 0; r0 < nrhs; r0 += 8) {
    const int nr = nrhs - r0 < 8 ? nrhs - r0 : 8;
    const double* xr = X + (int64_t)r0 * ldx;
    switch (nr) {
#define PINV_SYM_CASE(R)                                                                                     \
  case R:                                                                                                    \
    hipLaunchKernelGGL((sym_block_kernel<R>), dim3((unsigned)blocks), dim3(256), 0, s, Gp, n, nb, xr, ldx, Y); \
    break;
      PINV_SYM_CASE(1) PINV_SYM_CASE(2) PINV_SYM_CASE(3) PINV_SYM_CASE(4)
      PINV_SYM_CASE(5) PINV_SYM_CASE(6) PINV_SYM_CASE(7) PINV_SYM_CASE(8)
#undef PINV_SYM_CASE
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sym_reduce_kernel, dim3((unsigned)nb, (unsigned)nr), dim3(256), 0, s, Y, n, nb, alpha, bias,
                       U + (int64_t)r0 * ldu, ldu);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
