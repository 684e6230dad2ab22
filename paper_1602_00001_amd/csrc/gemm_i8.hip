// Int8 digit-slice matrix-core product: the quantised form of step 3, u = L^{-1} rho.
//
// G^ = diag(2^e) Q / M_S with Q = sum_s 256^(S-1-s) Q_s (S int8 digit planes)
// and rho^ = X diag(2^f) / M_SR with X = sum_t 256^(SR-1-t) X_t, so
//   Q X = sum_c 256^(S+SR-2-c) A_c,   A_c = sum_{s+t=c} Q_s X_t.
// Each class accumulator A_c is an exact int32 sum of int8 x int8 products
// (v_mfma_i32_16x16x64_i8); the host checks that no class can overflow.  The
// epilogue recombines the classes exactly in int64 (Horner in base 256),
// converts once to double, multiplies by c * 2^(e_i + f_r) (c = -h^2/(M_S M_SR))
// and adds the lift w_i: two roundings, no fused multiply-add (the file is
// compiled with contraction off).
//
// Tiling: 128 (rows of G) x 128 (right-hand sides) per 256-thread workgroup,
// 4 waves in 2x2, each 64x64 = 4x4 MFMA blocks per class; k step 64 bytes;
// two LDS stages (one per k step) fed through registers, one barrier per step.
// LDS rows are 64 data bytes + 16 pad bytes: the 16 lanes of a 128-bit read
// (16 consecutive rows, same k chunk) then start on 16 distinct 4-bank groups.
// The digit planes and the quantised right-hand sides are zero-padded to the
// tile grid, so the main loop has no bounds checks.
//
// v_mfma_i32_16x16x64_i8 layout (lane l, result register r):
//   A(i = l%16, k = 16*(l/16) + b), B(k = 16*(l/16) + b, j = l%16),
//   D(i = 4*(l/16) + r, j = l%16).

#include "common.h"

namespace {

constexpr int BM = 128, BN = 128, BK = 64, ROWB = 80;  // bytes per LDS row (64 + 16 pad)
constexpr int NT = 256;

__device__ inline void tile_of(int bid, int tilesM, int tilesN, int& mt, int& nt, bool& valid) {
  const int T = tilesM * tilesN;
  const int per = (T + 7) / 8;
  const int tile = (bid % 8) * per + bid / 8;
  valid = tile < T;
  mt = valid ? tile / tilesN : 0;
  nt = valid ? tile % tilesN : 0;
}

template <int S, int SR>
__global__ __launch_bounds__(NT, 1) void gemm_i8_kernel(GemmI8Args a, int tilesM, int tilesN) {
  constexpr int C = S + SR - 1;
  constexpr int PLANE = BM * ROWB;                // bytes of one digit plane in LDS
  constexpr int STAGE = (S + SR) * PLANE;
  __shared__ __attribute__((aligned(16))) int8_t sm[2 * STAGE];

  int mt, nt;
  bool valid;
  tile_of(blockIdx.x, tilesM, tilesN, mt, nt, valid);
  if (!valid) return;
  const int m0 = mt * BM, n0 = nt * BN;
  const int64_t P = a.P;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // global -> register prefetch: 2 chunks of 16 bytes per plane per thread
  const int lrow0 = tid >> 2, lch = tid & 3;     // rows lrow0 and lrow0 + 64
  const int8_t* gq[S];
  const int8_t* gx[SR];
#pragma unroll
  for (int s = 0; s < S; ++s) gq[s] = a.Q + (int64_t)s * P * P + (int64_t)(m0 + lrow0) * P + lch * 16;
#pragma unroll
  for (int t = 0; t < SR; ++t) gx[t] = a.X + ((int64_t)t * a.Rpad + n0 + lrow0) * P + lch * 16;
  const int64_t step64 = 64 * P;                  // 64 rows further

  v4i pq[S][2], px[SR][2];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      pq[s][0] = *(const v4i*)(gq[s] + k0);
      pq[s][1] = *(const v4i*)(gq[s] + step64 + k0);
    }
#pragma unroll
    for (int t = 0; t < SR; ++t) {
      px[t][0] = *(const v4i*)(gx[t] + k0);
      px[t][1] = *(const v4i*)(gx[t] + step64 + k0);
    }
  };
  auto store = [&](int st) {
    int8_t* base = sm + st * STAGE;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      *(v4i*)(base + s * PLANE + lrow0 * ROWB + lch * 16) = pq[s][0];
      *(v4i*)(base + s * PLANE + (lrow0 + 64) * ROWB + lch * 16) = pq[s][1];
    }
#pragma unroll
    for (int t = 0; t < SR; ++t) {
      *(v4i*)(base + (S + t) * PLANE + lrow0 * ROWB + lch * 16) = px[t][0];
      *(v4i*)(base + (S + t) * PLANE + (lrow0 + 64) * ROWB + lch * 16) = px[t][1];
    }
  };

  v4i acc[C][4][4];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[c][i][j] = v4i{0, 0, 0, 0};

  const int frag_off = (lane & 15) * ROWB + (lane >> 4) * 16;
  int st = 0;
  load(0);
  store(0);
  __syncthreads();
  for (int64_t k0 = 0; k0 < P; k0 += BK) {
    const bool has_next = k0 + BK < P;
    if (has_next) load(k0 + BK);
    const int8_t* base = sm + st * STAGE;
    v4i fa[S][4], fb[SR][4];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[s][i] = *(const v4i*)(base + s * PLANE + (wm * 64 + i * 16) * ROWB + frag_off);
#pragma unroll
    for (int t = 0; t < SR; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) fb[t][j] = *(const v4i*)(base + (S + t) * PLANE + (wn * 64 + j * 16) * ROWB + frag_off);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int t = 0; t < SR; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[s + t][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[s][i], fb[t][j], acc[s + t][i][j], 0, 0, 0);
    if (has_next) store(st ^ 1);
    __syncthreads();
    st ^= 1;
  }

  // exact recombination and the single scaling
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + (lane & 15);
      if (n >= a.nrhs) continue;
      const int fn = a.col_exp[n];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        if (m >= a.n) continue;
        int64_t v = acc[0][i][j][r];
#pragma unroll
        for (int c = 1; c < C; ++c) v = v * 256 + (int64_t)acc[c][i][j][r];
        const int em = a.row_exp ? a.row_exp[m] : 0;
        const double scale = ldexp(a.c, em + fn);
        double u = (double)v * scale;
        if (a.w) u = u + a.w[m];
        a.U[(int64_t)n * a.ldu + m] = u;
      }
    }
  }
}

template <int S, int SR>
hipError_t launch_t(const GemmI8Args& a, hipStream_t s) {
  const int tilesM = (int)(a.P / BM), tilesN = a.Rpad / BN;
  const int T = tilesM * tilesN;
  const int grid = ((T + 7) / 8) * 8;
  hipLaunchKernelGGL((gemm_i8_kernel<S, SR>), dim3(grid), dim3(NT), 0, s, a, tilesM, tilesN);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_i8(const GemmI8Args& a, hipStream_t s) {
  if (a.nrhs <= 0) return hipSuccess;
  if (a.P % BM != 0 || a.Rpad % BN != 0) return hipErrorInvalidValue;
  switch (a.S * 4 + a.SR) {
    case 1 * 4 + 1: return launch_t<1, 1>(a, s);
    case 1 * 4 + 2: return launch_t<1, 2>(a, s);
    case 1 * 4 + 3: return launch_t<1, 3>(a, s);
    case 2 * 4 + 1: return launch_t<2, 1>(a, s);
    case 2 * 4 + 2: return launch_t<2, 2>(a, s);
    case 2 * 4 + 3: return launch_t<2, 3>(a, s);
    case 3 * 4 + 1: return launch_t<3, 1>(a, s);
    case 3 * 4 + 2: return launch_t<3, 2>(a, s);
    case 3 * 4 + 3: return launch_t<3, 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}
