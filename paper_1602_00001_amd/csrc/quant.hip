// Rounding of the inverse's entries (the experiment behind Table 1), restated
// in binary fixed point so that the apply becomes an exact integer product.
//
// Rows of G (and columns of the right-hand sides) get one power-of-two scale
// each: e = frexp exponent of the largest magnitude, so every scaled entry is
// below 1 in magnitude.  An entry becomes q = rint((x * 2^-e) * M_S) with
// M_S = 127 (256^S - 1)/255; the scaling is exact, the multiply rounds once,
// rint rounds half to even.  q is stored as S balanced base-256 digits in
// [-128, 127] (most significant first), one int8 plane per digit, in padded
// P x P planes whose padding is zero.

#include "common.h"

namespace {

__device__ inline int frexp_exp(double x) {
  int e;
  (void)frexp(x, &e);
  return x == 0.0 ? 0 : e;
}

template <int S>
__device__ inline void digits(int q, int8_t* d) {
#pragma unroll
  for (int s = S - 1; s >= 0; --s) {
    const int lo = ((q + 128) & 255) - 128;
    d[s] = (int8_t)lo;
    q = (q - lo) >> 8;
  }
}

// maximum over the NW waves of the workgroup (red: NW doubles of LDS)
template <int NW>
__device__ inline double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  v = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) v = fmax(v, red[w]);
  __syncthreads();
  return v;
}

__device__ inline double block_max_256(double v, double* red) { return block_max<4>(v, red); }

// One wave per row: e[i] = exponent of max_k |G[i][k]| (0 for padding rows).
__global__ __launch_bounds__(256) void row_exponent_kernel(const double* __restrict__ G, int64_t ldg, int n,
                                                          int64_t P, int32_t* __restrict__ e) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= P) return;
  double m = 0.0;
  if (row < n) {
    const double* g = G + (int64_t)row * ldg;
    for (int k = lane; k < n; k += 64) m = fmax(m, fabs(g[k]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if (lane == 0) e[row] = frexp_exp(m);
}

// Each thread: 16 consecutive k of one row -> 16 bytes per digit plane.
template <int S>
__global__ __launch_bounds__(256) void quantize_rows_kernel(const double* __restrict__ G, int64_t ldg, int n,
                                                           int64_t P, const int32_t* __restrict__ e,
                                                           int8_t* __restrict__ Q) {
  const int64_t chunks = P / 16;
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= P * chunks) return;
  const int64_t row = gid / chunks;
  const int64_t k0 = (gid % chunks) * 16;
  const double M = (double)(127LL * ((1LL << (8 * S)) - 1) / 255);
  int8_t d[S][16];
  const int er = row < n ? e[row] : 0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int64_t k = k0 + t;
    int q = 0;
    if (row < n && k < n) {
      const double x = G[row * ldg + k];
      q = (int)rint(ldexp(x, -er) * M);
    }
    int8_t dd[S];
    digits<S>(q, dd);
#pragma unroll
    for (int s = 0; s < S; ++s) d[s][t] = dd[s];
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    v4i v;
    __builtin_memcpy(&v, d[s], 16);
    *(v4i*)(Q + (int64_t)s * P * P + row * P + k0) = v;
  }
}

// QT[s][k][i] = Q[s][i][k], 64x64 byte tiles through LDS.
__global__ __launch_bounds__(256) void transpose_planes_kernel(const int8_t* __restrict__ Q, int8_t* __restrict__ QT,
                                                              int64_t P) {
  __shared__ int8_t t[64][64 + 4];
  const int64_t tiles = P / 64;
  const int64_t bi = blockIdx.x / tiles, bk = blockIdx.x % tiles;
  const int s = blockIdx.y;
  const int8_t* src = Q + (int64_t)s * P * P;
  int8_t* dst = QT + (int64_t)s * P * P;
  const int r = threadIdx.x >> 2, c = (threadIdx.x & 3) * 16;
  v4i v = *(const v4i*)(src + (bi * 64 + r) * P + bk * 64 + c);
  const int8_t* pv = (const int8_t*)&v;
#pragma unroll
  for (int b = 0; b < 16; ++b) t[r][c + b] = pv[b];
  __syncthreads();
  int8_t o[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) o[b] = t[c + b][r];
  v4i ov;
  __builtin_memcpy(&ov, o, 16);
  *(v4i*)(dst + (bk * 64 + r) * P + bi * 64 + c) = ov;
}

// One workgroup per column r of X (column-major n x nrhs, stride ldx): the
// exponent of its largest magnitude, then its rows of the output
// [SR][Rpad][P] (rows n..P-1 and columns r >= nrhs are written as zeros).
// Each thread handles 4 consecutive k of every 4 x (threads) (32-byte reads,
// 4-byte writes per digit plane), so both the reads and the writes of a wave
// are contiguous.  Columns of up to 16384 entries (256 threads) or 40960
// (1024 threads) are read once into registers (all loads in flight together);
// longer ones are read twice, once for the maximum and once for the digits.
template <int SR>
__device__ __attribute__((always_inline)) inline void quantize_col_two_pass(const double* __restrict__ x, bool live, int n, int r, int Rpad, int64_t P,
                                    const int32_t* __restrict__ pre, int8_t* __restrict__ Xq,
                                    int32_t* __restrict__ f, double* red) {
  // Loads are unconditional from clamped indices (k < n selects the value
  // afterwards): a load under a per-lane condition makes the next write of its
  // register wait for it, which would serialise the loads of a pass.
  double m = 0.0;
  if (live)
    for (int64_t k0 = (int64_t)threadIdx.x * 4; k0 < n; k0 += 256 * 4) {
      double v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t k = min(k0 + t, (int64_t)n - 1);
        v[t] = pre ? ldexp(x[k], pre[k]) : x[k];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) m = fmax(m, k0 + t < n ? fabs(v[t]) : 0.0);
    }
  m = block_max_256(m, red);
  const int fr = frexp_exp(m);
  if (live && threadIdx.x == 0) f[r] = fr;
  const double M = (double)(127LL * ((1LL << (8 * SR)) - 1) / 255);
  for (int64_t k0 = (int64_t)threadIdx.x * 4; k0 < P; k0 += 256 * 4) {
    int8_t d[SR][4];
    double v[4];
    if (live) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t k = min(k0 + t, (int64_t)n - 1);
        v[t] = pre ? ldexp(x[k], pre[k]) : x[k];
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t k = k0 + t;
      int q = 0;
      if (live && k < n) q = (int)rint(ldexp(v[t], -fr) * M);
      int8_t dd[SR];
      digits<SR>(q, dd);
#pragma unroll
      for (int s = 0; s < SR; ++s) d[s][t] = dd[s];
    }
#pragma unroll
    for (int s = 0; s < SR; ++s) {
      int word;
      __builtin_memcpy(&word, d[s], 4);
      *(int*)(Xq + ((int64_t)s * Rpad + r) * P + k0) = word;
    }
  }
}

// Column in registers: NT threads, KR chunks of 4 NT entries (thread t holds
// entries 4t .. 4t+3 of every chunk); for columns of up to 4 NT KR entries.
template <int SR, int NT, int KR>
__device__ __attribute__((always_inline)) inline void quantize_col_regs(
    const double* __restrict__ x, bool live, int n, int r, int Rpad, int64_t P, const int32_t* __restrict__ pre,
    int8_t* __restrict__ Xq, int32_t* __restrict__ f, double* red) {
  constexpr int STR = 4 * NT;
  // (chunk c is read when it holds entries; the condition is uniform, and the
  // loads of a chunk are unconditional from clamped indices)
  double v[KR][4];
  double m = 0.0;
#pragma unroll
  for (int c = 0; c < KR; ++c) {
    const int64_t k0 = (int64_t)c * STR + threadIdx.x * 4;
    if (live && c * STR < n) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t k = min(k0 + t, (int64_t)n - 1);
        v[c][t] = pre ? ldexp(x[k], pre[k]) : x[k];
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) v[c][t] = 0.0;
    }
  }
#pragma unroll
  for (int c = 0; c < KR; ++c)
#pragma unroll
    for (int t = 0; t < 4; ++t) m = fmax(m, (int64_t)c * STR + threadIdx.x * 4 + t < n ? fabs(v[c][t]) : 0.0);
  m = block_max<NT / 64>(m, red);
  const int fr = frexp_exp(m);
  if (live && threadIdx.x == 0) f[r] = fr;
  const double M = (double)(127LL * ((1LL << (8 * SR)) - 1) / 255);
#pragma unroll
  for (int c = 0; c < KR; ++c) {
    const int64_t k0 = (int64_t)c * STR + threadIdx.x * 4;
    if (k0 >= P) break;
    int8_t d[SR][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      int q = 0;
      if (live && k0 + t < n) q = (int)rint(ldexp(v[c][t], -fr) * M);
      int8_t dd[SR];
      digits<SR>(q, dd);
#pragma unroll
      for (int s2 = 0; s2 < SR; ++s2) d[s2][t] = dd[s2];
    }
#pragma unroll
    for (int s2 = 0; s2 < SR; ++s2) {
      int word;
      __builtin_memcpy(&word, d[s2], 4);
      *(int*)(Xq + ((int64_t)s2 * Rpad + r) * P + k0) = word;
    }
  }
}

// 256 threads: columns of up to 16384 entries in registers, longer ones in
// two passes
constexpr int KR = 16;

template <int SR>
__device__ __attribute__((always_inline)) inline void quantize_col(const double* __restrict__ x, bool live, int n, int r, int Rpad, int64_t P,
                                    const int32_t* __restrict__ pre, int8_t* __restrict__ Xq,
                                    int32_t* __restrict__ f, double* red) {
  if (n > KR * 1024) {
    quantize_col_two_pass<SR>(x, live, n, r, Rpad, P, pre, Xq, f, red);
    return;
  }
  quantize_col_regs<SR, 256, KR>(x, live, n, r, Rpad, P, pre, Xq, f, red);
}

// 1024 threads: columns of 16385 to KRW * 4096 entries in registers
constexpr int KRW = 10;

template <int SR>
__global__ __launch_bounds__(256) void quantize_cols_kernel(const double* __restrict__ X, int64_t ldx,
                                                           const double* const* __restrict__ xcols, int n,
                                                           int nrhs, int Rpad, int64_t P,
                                                           const int32_t* __restrict__ pre, int8_t* __restrict__ Xq,
                                                           int32_t* __restrict__ f) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  const bool live = r < nrhs;
  const double* x = live ? (xcols ? xcols[r] : X + (int64_t)r * ldx) : X;
  quantize_col<SR>(x, live, n, r, Rpad, P, pre, Xq, f, red);
}

template <int SR>
__global__ __launch_bounds__(1024) void quantize_cols_wide_kernel(const double* __restrict__ X, int64_t ldx,
                                                                 const double* const* __restrict__ xcols, int n,
                                                                 int nrhs, int Rpad, int64_t P,
                                                                 const int32_t* __restrict__ pre,
                                                                 int8_t* __restrict__ Xq, int32_t* __restrict__ f) {
  __shared__ double red[16];
  const int r = blockIdx.x;
  const bool live = r < nrhs;
  const double* x = live ? (xcols ? xcols[r] : X + (int64_t)r * ldx) : X;
  quantize_col_regs<SR, 1024, KRW>(x, live, n, r, Rpad, P, pre, Xq, f, red);
}

// Grouped form: workgroup b serves group g with g.col0 <= b < next group's
// col0 (binary search over the table, uniform per workgroup).
template <int SR>
__global__ __launch_bounds__(256) void quantize_cols_grouped_kernel(const QuantColsGroup* __restrict__ groups,
                                                                   int ngroups) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  int lo = 0, hi = ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].col0 <= b) lo = mid; else hi = mid - 1;
  }
  const QuantColsGroup g = groups[lo];
  const int r = b - g.col0;
  const bool live = r < g.nrhs;
  const double* x = live ? g.xcols[r] : nullptr;
  quantize_col<SR>(x, live, g.n, r, g.Rpad, g.P, nullptr, g.Xq, g.f, red);
}

// Grouped form with 1024 threads, for groups whose columns hold 16385 to
// KRW * 4096 entries.
template <int SR>
__global__ __launch_bounds__(1024) void quantize_cols_grouped_wide_kernel(const QuantColsGroup* __restrict__ groups,
                                                                         int ngroups) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  int lo = 0, hi = ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].col0 <= b) lo = mid; else hi = mid - 1;
  }
  const QuantColsGroup g = groups[lo];
  const int r = b - g.col0;
  const bool live = r < g.nrhs;
  const double* x = live ? g.xcols[r] : nullptr;
  quantize_col_regs<SR, 1024, KRW>(x, live, g.n, r, g.Rpad, g.P, nullptr, g.Xq, g.f, red);
}

__global__ void fill_random_i8_kernel(int8_t* __restrict__ p, size_t n, uint32_t seed) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i * 2654435761u + seed;
    x ^= x >> 15;
    x *= 2246822519u;
    x ^= x >> 13;
    p[i] = (int8_t)(x >> 24);
  }
}

}  // namespace

hipError_t launch_fill_random_i8(int8_t* p, size_t n, uint32_t seed, hipStream_t s) {
  hipLaunchKernelGGL(fill_random_i8_kernel, dim3(grid_1d((int64_t)n)), dim3(256), 0, s, p, n, seed);
  return hipGetLastError();
}

int64_t pinv_max_mag(int S) { return 127LL * ((1LL << (8 * S)) - 1) / 255; }

bool quantize_cols_wide(int n) { return n > KR * 1024 && n <= KRW * 4096; }

hipError_t launch_quantize_cols_grouped(const QuantColsGroup* groups, int ngroups, int total_cols, int SR, bool wide,
                                        hipStream_t s) {
  if (ngroups <= 0 || total_cols <= 0) return hipSuccess;
  const dim3 grid((unsigned)total_cols);
  if (wide) {
    switch (SR) {
      case 1: hipLaunchKernelGGL(quantize_cols_grouped_wide_kernel<1>, grid, dim3(1024), 0, s, groups, ngroups); break;
      case 2: hipLaunchKernelGGL(quantize_cols_grouped_wide_kernel<2>, grid, dim3(1024), 0, s, groups, ngroups); break;
      case 3: hipLaunchKernelGGL(quantize_cols_grouped_wide_kernel<3>, grid, dim3(1024), 0, s, groups, ngroups); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (SR) {
    case 1: hipLaunchKernelGGL(quantize_cols_grouped_kernel<1>, grid, dim3(256), 0, s, groups, ngroups); break;
    case 2: hipLaunchKernelGGL(quantize_cols_grouped_kernel<2>, grid, dim3(256), 0, s, groups, ngroups); break;
    case 3: hipLaunchKernelGGL(quantize_cols_grouped_kernel<3>, grid, dim3(256), 0, s, groups, ngroups); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_quantize_rows(const double* G, int64_t ldg, int n, int S, int64_t P, int8_t* Q, int32_t* e,
                                hipStream_t s) {
  hipLaunchKernelGGL(row_exponent_kernel, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, s, G, ldg, n, P, e);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int64_t threads = P * (P / 16);
  const dim3 grid((unsigned)((threads + 255) / 256));
  switch (S) {
    case 1: hipLaunchKernelGGL(quantize_rows_kernel<1>, grid, dim3(256), 0, s, G, ldg, n, P, e, Q); break;
    case 2: hipLaunchKernelGGL(quantize_rows_kernel<2>, grid, dim3(256), 0, s, G, ldg, n, P, e, Q); break;
    case 3: hipLaunchKernelGGL(quantize_rows_kernel<3>, grid, dim3(256), 0, s, G, ldg, n, P, e, Q); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_transpose_planes(const int8_t* Q, int8_t* QT, int S, int64_t P, hipStream_t s) {
  const int64_t tiles = P / 64;
  hipLaunchKernelGGL(transpose_planes_kernel, dim3((unsigned)(tiles * tiles), (unsigned)S), dim3(256), 0, s, Q, QT, P);
  return hipGetLastError();
}

hipError_t launch_quantize_cols(const double* X, int64_t ldx, const double* const* xcols, int n, int nrhs, int Rpad,
                                int SR, int64_t P, const int32_t* pre_exp, int8_t* Xq, int32_t* f, hipStream_t s) {
  const dim3 grid((unsigned)Rpad);
  if (quantize_cols_wide(n)) {
    switch (SR) {
      case 1: hipLaunchKernelGGL(quantize_cols_wide_kernel<1>, grid, dim3(1024), 0, s, X, ldx, xcols, n, nrhs, Rpad, P, pre_exp, Xq, f); break;
      case 2: hipLaunchKernelGGL(quantize_cols_wide_kernel<2>, grid, dim3(1024), 0, s, X, ldx, xcols, n, nrhs, Rpad, P, pre_exp, Xq, f); break;
      case 3: hipLaunchKernelGGL(quantize_cols_wide_kernel<3>, grid, dim3(1024), 0, s, X, ldx, xcols, n, nrhs, Rpad, P, pre_exp, Xq, f); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (SR) {
    case 1: hipLaunchKernelGGL(quantize_cols_kernel<1>, grid, dim3(256), 0, s, X, ldx, xcols, n, nrhs, Rpad, P, pre_exp, Xq, f); break;
    case 2: hipLaunchKernelGGL(quantize_cols_kernel<2>, grid, dim3(256), 0, s, X, ldx, xcols, n, nrhs, Rpad, P, pre_exp, Xq, f); break;
    case 3: hipLaunchKernelGGL(quantize_cols_kernel<3>, grid, dim3(256), 0, s, X, ldx, xcols, n, nrhs, Rpad, P, pre_exp, Xq, f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
