// FP64 matrix-core GEMM and GEMV.
//
// The GEMM is the workhorse of the one-time inversion (Cholesky panel and
// trailing updates, the triangular inverse, G = L^{-T} L^{-1}) and of the plain
// FP64 apply u = -h^2 G rho + w (the N^2-per-vector product the paper's method
// repeats at every time moment).
//
// Tiling: 128x128 output tile per 256-thread workgroup (4 waves in 2x2, each
// 64x64 = 4x4 blocks of v_mfma_f64_16x16x4f64), k step 16, two LDS stages with
// register prefetch of the next stage (one barrier per step).  LDS holds both
// operands k-major ([k][m], [k][n]) padded by 16 doubles so that the two
// half-waves of a 64-bit read hit disjoint banks.
//
// v_mfma_f64_16x16x4f64 operand/result layout (lane l, result register r):
//   A(i = l%16, k = l/16), B(k = l/16, j = l%16), D(i = l/16 + 4r, j = l%16).
//
// Workgroup -> tile mapping is XCD-aware: workgroup b runs on XCD b % 8, and
// XCD x is handed a contiguous range of tiles (row-major over tiles), so the
// column tiles that share one row block of A run on the same XCD and share
// its L2.

#include "common.h"

namespace {

constexpr int BM = 128, BN = 128, BKK = 16, LDP = 128 + 16;
constexpr int NTHREADS = 256;

__device__ inline void tile_of(int bid, int tilesM, int tilesN, int& mt, int& nt, bool& valid) {
  const int T = tilesM * tilesN;
  const int per = (T + 7) / 8;
  const int tile = (bid % 8) * per + bid / 8;
  valid = tile < T;
  mt = valid ? tile / tilesN : 0;
  nt = valid ? tile % tilesN : 0;
}

template <bool AK, bool BKc>
__global__ __launch_bounds__(NTHREADS, 2) void gemm_f64_kernel(GemmF64Args a, int tilesM, int tilesN) {
  __shared__ double As[2][BKK][LDP];
  __shared__ double Bs[2][BKK][LDP];

  int mt, nt;
  bool valid;
  tile_of(blockIdx.x, tilesM, tilesN, mt, nt, valid);
  if (!valid) return;
  const int m0 = mt * BM, n0 = nt * BN;
  if (a.tri == 1 && n0 > m0 + BM - 1) return;
  int kbeg = 0;
  if (a.kdiag) kbeg = (max(m0, n0) / BKK) * BKK;
  const int K = a.K;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  double ra[8], rb[8];

  // Loads are unconditional, from indices clamped into the operands; values
  // outside them are zeroed when written to LDS (a load under a per-lane
  // condition would make later writes of its register wait for it).
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = i * NTHREADS + tid;
      int kk, mm;
      if (AK) { kk = idx & 15; mm = idx >> 4; } else { kk = idx >> 7; mm = idx & 127; }
      const int gm = min(m0 + mm, a.M - 1), gk = min(k0 + kk, K - 1);
      ra[i] = AK ? a.A[(int64_t)gm * a.lda + gk] : a.A[(int64_t)gk * a.lda + gm];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = i * NTHREADS + tid;
      int kk, nn;
      if (BKc) { kk = idx & 15; nn = idx >> 4; } else { kk = idx >> 7; nn = idx & 127; }
      const int gn = min(n0 + nn, a.N - 1), gk = min(k0 + kk, K - 1);
      rb[i] = BKc ? a.B[(int64_t)gn * a.ldb + gk] : a.B[(int64_t)gk * a.ldb + gn];
    }
  };
  auto store = [&](int st, int k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = i * NTHREADS + tid;
      int kk, mm;
      if (AK) { kk = idx & 15; mm = idx >> 4; } else { kk = idx >> 7; mm = idx & 127; }
      As[st][kk][mm] = (m0 + mm < a.M && k0 + kk < K) ? ra[i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = i * NTHREADS + tid;
      int kk, nn;
      if (BKc) { kk = idx & 15; nn = idx >> 4; } else { kk = idx >> 7; nn = idx & 127; }
      Bs[st][kk][nn] = (n0 + nn < a.N && k0 + kk < K) ? rb[i] : 0.0;
    }
  };

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  int st = 0;
  if (kbeg < K) {
    load(kbeg);
    store(0, kbeg);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < K; k0 += BKK) {
    const bool has_next = k0 + BKK < K;
    if (has_next) load(k0 + BKK);
#pragma unroll
    for (int k4 = 0; k4 < BKK / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      double fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[i] = As[st][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) fb[j] = Bs[st][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (has_next) store(st ^ 1, k0 + BKK);
    __syncthreads();
    st ^= 1;
  }

  // epilogue: C = alpha*acc + beta*C + bias
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + (lane >> 4) + 4 * r;
        if (m < a.M && n < a.N) {
          double* c = a.C + (int64_t)m * a.csm + (int64_t)n * a.csn;
          double v = a.alpha * acc[i][j][r];
          if (a.beta != 0.0) v += a.beta * *c;
          if (a.bias) v += a.bias[m];
          *c = v;
        }
      }
    }
  }
}

// Both operands k-contiguous (A(m,k) = A[m*lda + k], B(k,n) = B[n*ldb + k]):
// the plain FP64 apply and the Cholesky panel / trailing updates.
// LDS holds each 128 x 16 operand tile row-major (128 bytes per row) with its
// eight 16-byte chunks XOR-swizzled by (row >> 1) & 7: the 128-bit stores of a
// half-wave (two rows) and the 128-bit fragment reads (16 rows, one chunk) both
// cover all 64 banks exactly once.  The k index of the 16x16x4 instruction is
// permuted: on MFMA step s (0..3) lane group g = l/16 supplies k = 4g + s, so a
// lane reads its four k values of a row with two 128-bit reads per tile.
template <bool VEC>
__global__ __launch_bounds__(NTHREADS, 2) void gemm_f64_nt_kernel(GemmF64Args a, int tilesM, int tilesN) {
  __shared__ __attribute__((aligned(16))) double As[2][BM * BKK];
  __shared__ __attribute__((aligned(16))) double Bs[2][BN * BKK];

  int mt, nt;
  bool valid;
  tile_of(blockIdx.x, tilesM, tilesN, mt, nt, valid);
  if (!valid) return;
  const int m0 = mt * BM, n0 = nt * BN;
  if (a.tri == 1 && n0 > m0 + BM - 1) return;
  // k range of this workgroup (the whole of k unless split)
  const int kz = blockIdx.y;
  const int kb = a.ksplit > 1 ? kz * a.kchunk : 0;
  const int K = a.ksplit > 1 ? min(a.K, kb + a.kchunk) : a.K;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // loads: item it covers row (it*256 + tid) >> 3, 16-byte chunk (tid & 7).
  // The loads themselves are unconditional, from addresses clamped into the
  // operands; rows and k beyond the operands are zeroed when the registers are
  // written to LDS.  (Loads under per-lane conditions would make every later
  // write of the same registers wait for the load, serialising the loads.)
  const int lchunk = tid & 7;
  double2 ra[4], rb[4];
  // row offsets (elements) from the tile's first row, rows clamped into the
  // operand; 32-bit, since a tile spans 128 rows
  const double* Ab = a.A + (int64_t)m0 * a.lda;
  const double* Bb = a.B + (int64_t)n0 * a.ldb;
  uint32_t oa[4], ob[4];
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int row = (it * NTHREADS + tid) >> 3;
    oa[it] = (uint32_t)(min(m0 + row, a.M - 1) - m0) * (uint32_t)a.lda;
    ob[it] = (uint32_t)(min(n0 + row, a.N - 1) - n0) * (uint32_t)a.ldb;
  }
  auto load = [&](int k0) {
    const int gk = k0 + 2 * lchunk;
    // one uniform branch around all the loads of the step (a branch per load
    // would make each join wait for the loads before it)
    if (VEC && k0 + BKK <= K) {  // the whole k step lies inside the operands
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        ra[it] = *(const double2*)(Ab + (oa[it] + (uint32_t)gk));
        rb[it] = *(const double2*)(Bb + (ob[it] + (uint32_t)gk));
      }
    } else {
      const uint32_t k0c = (uint32_t)min(gk, K - 1), k1c = (uint32_t)min(gk + 1, K - 1);
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        ra[it].x = Ab[oa[it] + k0c];
        ra[it].y = Ab[oa[it] + k1c];
        rb[it].x = Bb[ob[it] + k0c];
        rb[it].y = Bb[ob[it] + k1c];
      }
    }
  };
  auto store = [&](int st, int k0) {
    const int gk = k0 + 2 * lchunk;
    const bool in0 = gk < K, in1 = gk + 1 < K;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int row = (it * NTHREADS + tid) >> 3;
      const int pc = lchunk ^ ((row >> 1) & 7);
      const bool okm = m0 + row < a.M, okn = n0 + row < a.N;
      double2 va, vb;
      va.x = (okm && in0) ? ra[it].x : 0.0;
      va.y = (okm && in1) ? ra[it].y : 0.0;
      vb.x = (okn && in0) ? rb[it].x : 0.0;
      vb.y = (okn && in1) ? rb[it].y : 0.0;
      *(double2*)(&As[st][row * BKK + pc * 2]) = va;
      *(double2*)(&Bs[st][row * BKK + pc * 2]) = vb;
    }
  };

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  const int fr = lane & 15, g = lane >> 4;
  int st = 0;
  if (K > kb) {
    load(kb);
    store(0, kb);
  }
  __syncthreads();
  for (int k0 = kb; k0 < K; k0 += BKK) {
    const bool has_next = k0 + BKK < K;
    if (has_next) load(k0 + BKK);
    double fa[4][4], fb[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wm * 64 + i * 16 + fr;
      const int sw = (row >> 1) & 7;
      const double2 lo = *(const double2*)(&As[st][row * BKK + ((2 * g) ^ sw) * 2]);
      const double2 hi = *(const double2*)(&As[st][row * BKK + ((2 * g + 1) ^ sw) * 2]);
      fa[i][0] = lo.x; fa[i][1] = lo.y; fa[i][2] = hi.x; fa[i][3] = hi.y;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = wn * 64 + j * 16 + fr;
      const int sw = (row >> 1) & 7;
      const double2 lo = *(const double2*)(&Bs[st][row * BKK + ((2 * g) ^ sw) * 2]);
      const double2 hi = *(const double2*)(&Bs[st][row * BKK + ((2 * g + 1) ^ sw) * 2]);
      fb[j][0] = lo.x; fb[j][1] = lo.y; fb[j][2] = hi.x; fb[j][3] = hi.y;
    }
#pragma unroll
    for (int sk = 0; sk < 4; ++sk)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][sk], fb[j][sk], acc[i][j], 0, 0, 0);
    if (has_next) store(st ^ 1, k0 + BKK);
    __syncthreads();
    st ^= 1;
  }

#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + (lane >> 4) + 4 * r;
        if (m < a.M && n < a.N) {
          if (a.ksplit > 1) {
            a.part[((int64_t)kz * a.N + n) * a.M + m] = acc[i][j][r];
            continue;
          }
          double* c = a.C + (int64_t)m * a.csm + (int64_t)n * a.csn;
          double v = a.alpha * acc[i][j][r];
          if (a.beta != 0.0) v += a.beta * *c;
          if (a.bias) v += a.bias[m];
          *c = v;
        }
      }
    }
  }
}

// One wave per row of G; lanes stride over k; up to 8 right-hand sides.
// VEC: the row is read as 16-byte pairs (rows start 16-byte aligned), so one
// load instruction of a wave covers 1 KB of the row.
template <int NR, bool VEC>
__global__ __launch_bounds__(256) void gemv_f64_kernel(const double* __restrict__ G, int64_t ldg, int n,
                                                      const double* __restrict__ x, int64_t ldx, double alpha,
                                                      const double* __restrict__ bias, double* __restrict__ u,
                                                      int64_t ldu) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* g = G + (int64_t)row * ldg;
  // four independent partial sums per right-hand side, so the loads of four
  // k blocks are in flight together (the loop would otherwise wait for each
  // load in turn; eight measured no faster)
  constexpr int U = 4;
  constexpr int W = VEC ? 2 : 1;           // doubles per lane and load
  double s[U][NR];
#pragma unroll
  for (int q = 0; q < U; ++q)
#pragma unroll
    for (int r = 0; r < NR; ++r) s[q][r] = 0.0;
  // whole blocks of 64 W U doubles (the same count for every lane), then the
  // rest one double per lane
  int b = 0;
  for (; b + 64 * W * U <= n; b += 64 * W * U) {
    const int k = b + lane * W;
    double gv[U][W];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if constexpr (VEC) {
        const double2 v = *(const double2*)(g + k + 64 * W * q);
        gv[q][0] = v.x;
        gv[q][W - 1] = v.y;
      } else {
        gv[q][0] = g[k + 64 * q];
      }
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int r = 0; r < NR; ++r)
          s[q][r] = fma(gv[q][w], x[(int64_t)r * ldx + k + 64 * W * q + w], s[q][r]);
  }
  for (int k = b + lane; k < n; k += 64) {
    const double gv = g[k];
#pragma unroll
    for (int r = 0; r < NR; ++r) s[0][r] = fma(gv, x[(int64_t)r * ldx + k], s[0][r]);
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    double v = s[0][r];
#pragma unroll
    for (int q = 1; q < U; ++q) v += s[q][r];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    s[0][r] = v;
  }
  if (lane < NR) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r == lane) v = s[0][r];
    v = alpha * v;
    if (bias) v += bias[row];
    u[(int64_t)lane * ldu + row] = v;
  }
}

// One thread per output element, threads along m (coalesced), the split parts
// added in order of z.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const double* __restrict__ part, int ksplit, int M, int N,
                                                           double alpha, double beta, const double* __restrict__ bias,
                                                           double* __restrict__ C, int64_t csm, int64_t csn) {
  const int64_t MN = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < MN; idx += (int64_t)gridDim.x * 256) {
    const int m = (int)(idx % M), n = (int)(idx / M);
    double acc = 0.0;
    for (int z = 0; z < ksplit; ++z) acc += part[(int64_t)z * MN + idx];
    double* c = C + (int64_t)m * csm + (int64_t)n * csn;
    double v = alpha * acc;
    if (beta != 0.0) v += beta * *c;
    if (bias) v += bias[m];
    *c = v;
  }
}

}  // namespace

void gemm_f64_split_plan(int M, int N, int K, int* ksplit, int* kchunk) {
  // two 128x128 workgroups fit per compute unit: aim for 512 in flight, with at
  // least 256 of k per split
  const int T = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int z = 512 / (T > 0 ? T : 1);
  const int zmax = K / 256;
  if (z > zmax) z = zmax;
  if (z > 16) z = 16;
  if (z < 2) {
    *ksplit = 1;
    *kchunk = K;
    return;
  }
  int chunk = (K + z - 1) / z;
  chunk = (chunk + BKK - 1) / BKK * BKK;
  *ksplit = (K + chunk - 1) / chunk;
  *kchunk = chunk;
}

hipError_t launch_splitk_reduce(const double* part, int ksplit, int M, int N, double alpha, double beta,
                                const double* bias, double* C, int64_t csm, int64_t csn, hipStream_t s) {
  const int64_t MN = (int64_t)M * N;
  if (MN == 0) return hipSuccess;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_1d(MN)), dim3(256), 0, s, part, ksplit, M, N,
                     alpha, beta, bias, C, csm, csn);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const GemmF64Args& a_in, hipStream_t s) {
  if (a_in.M <= 0 || a_in.N <= 0) return hipSuccess;
  const int tilesM = (a_in.M + BM - 1) / BM, tilesN = (a_in.N + BN - 1) / BN;
  const int T = tilesM * tilesN;
  const int grid = ((T + 7) / 8) * 8;
  // the NT kernel addresses a tile's rows with 32-bit element offsets
  // (row in tile * ld + k); operands with larger strides take the generic
  // kernel, unsplit
  const uint64_t ldmax = (uint64_t)(a_in.lda > a_in.ldb ? a_in.lda : a_in.ldb);
  const bool off32 = (uint64_t)(BM - 1) * ldmax + (uint64_t)a_in.K < (1ull << 32);
  GemmF64Args a = a_in;
  if (!off32) a.ksplit = 1;
  if (a.a_kcontig && a.b_kcontig && !a.kdiag && off32) {
    const bool vec = (a.lda % 2 == 0) && (a.ldb % 2 == 0) && ((uintptr_t)a.A % 16 == 0) && ((uintptr_t)a.B % 16 == 0);
    const bool split = a.ksplit > 1;
    if (split && (a.tri || !a.part || a.kchunk <= 0 || a.kchunk % BKK != 0 ||
                  (int64_t)a.kchunk * (a.ksplit - 1) >= a.K))
      return hipErrorInvalidValue;
    const dim3 g3(grid, split ? a.ksplit : 1);
    if (vec)
      hipLaunchKernelGGL((gemm_f64_nt_kernel<true>), g3, dim3(NTHREADS), 0, s, a, tilesM, tilesN);
    else
      hipLaunchKernelGGL((gemm_f64_nt_kernel<false>), g3, dim3(NTHREADS), 0, s, a, tilesM, tilesN);
    if (split) {
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      return launch_splitk_reduce(a.part, a.ksplit, a.M, a.N, a.alpha, a.beta, a.bias, a.C, a.csm, a.csn, s);
    }
  } else if (a.ksplit > 1) {
    return hipErrorInvalidValue;
  } else if (a.a_kcontig && a.b_kcontig)
    hipLaunchKernelGGL((gemm_f64_kernel<true, true>), dim3(grid), dim3(NTHREADS), 0, s, a, tilesM, tilesN);
  else if (a.a_kcontig && !a.b_kcontig)
    hipLaunchKernelGGL((gemm_f64_kernel<true, false>), dim3(grid), dim3(NTHREADS), 0, s, a, tilesM, tilesN);
  else if (!a.a_kcontig && !a.b_kcontig)
    hipLaunchKernelGGL((gemm_f64_kernel<false, false>), dim3(grid), dim3(NTHREADS), 0, s, a, tilesM, tilesN);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<false, true>), dim3(grid), dim3(NTHREADS), 0, s, a, tilesM, tilesN);
  return hipGetLastError();
}

hipError_t launch_gemv_f64(const double* G, int64_t ldg, int n, const double* x, int64_t ldx, int nrhs,
                           double alpha, const double* bias, double* u, int64_t ldu, hipStream_t s) {
  const int grid = (n + 3) / 4;
  const bool vec = ldg % 2 == 0 && (uintptr_t)G % 16 == 0;
  for (int r0 = 0; r0 < nrhs; r0 += 8) {
    const int nr = nrhs - r0 < 8 ? nrhs - r0 : 8;
    const double* xr = x + (int64_t)r0 * ldx;
    double* ur = u + (int64_t)r0 * ldu;
    switch (nr) {
#define PINV_GEMV_CASE(R)                                                                                       \
  case R:                                                                                                       \
    if (vec)                                                                                                    \
      hipLaunchKernelGGL((gemv_f64_kernel<R, true>), dim3(grid), dim3(256), 0, s, G, ldg, n, xr, ldx, alpha, bias, \
                         ur, ldu);                                                                              \
    else                                                                                                        \
      hipLaunchKernelGGL((gemv_f64_kernel<R, false>), dim3(grid), dim3(256), 0, s, G, ldg, n, xr, ldx, alpha,     \
                         bias, ur, ldu);                                                                        \
    break;
      PINV_GEMV_CASE(1) PINV_GEMV_CASE(2) PINV_GEMV_CASE(3) PINV_GEMV_CASE(4)
      PINV_GEMV_CASE(5) PINV_GEMV_CASE(6) PINV_GEMV_CASE(7) PINV_GEMV_CASE(8)
#undef PINV_GEMV_CASE
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
