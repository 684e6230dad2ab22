// The int8 digit-slice apply for few right-hand sides (step 3 with the inverse
// held as per-row-scaled fixed point, Table 1's rounding in base 2^8): a pass
// over the stored digit planes, bound by HBM.
//
// The tiled matrix-core product pads the right-hand sides to 128 columns, so at
// one right-hand side it does 128 times the needed products and reaches about
// half of HBM bandwidth on the digit planes.  Here one wave takes one row of G:
// each lane reads 16 bytes of every digit plane per 1 KB block of k (one load
// instruction covers 1 KB of the row, whole cache lines), the right-hand sides'
// digits at the same k (L2-resident, read by every row), and forms the digit
// products with v_dot4c_i32_i8 (four int8 products added into an int32 per
// instruction).  Products of G digit s and rho digit t go to class s + t, as
// in the tiled product.  Each lane's int32 class sums cover P / 64 values of k,
// so they cannot overflow; the lanes' sums are added in int64 (exact, any
// order), then recombined (Horner, base 256), converted once, scaled once and
// lifted once, exactly as the tiled product's epilogue: the result is
// bit-identical to it and to the oracle's integer apply.
//
// Layouts (those of the tiled product): Q [S][P][P] int8, row stride P, zero
// past column n; Xq [SR][Rpad][P] int8, zero past row n; row_exp [P] or null;
// col_exp [nrhs]; u column-major with stride ldu.

#include "common.h"

#include <type_traits>

namespace {

// v_dot4c_i32_i8: acc += sum of the four int8 products of a and b
__device__ inline int dot4(int a, int b, int acc) { return __builtin_amdgcn_sdot4(a, b, acc, false); }

template <int S, int SR, int NR>
__global__ __launch_bounds__(256) void gemv_i8_kernel(const int8_t* __restrict__ Q, const int8_t* __restrict__ Xq,
                                                      int64_t P, int Rpad, int n, const int32_t* __restrict__ row_exp,
                                                      const int32_t* __restrict__ col_exp, double c,
                                                      const double* __restrict__ w, double* __restrict__ U,
                                                      int64_t ldu) {
  constexpr int C = S + SR - 1;
  constexpr int UB = NR <= 2 ? 4 : 2;  // 1 KB blocks of k whose loads are in flight together
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const int64_t plane = P * P, xplane = (int64_t)Rpad * P;
  const int8_t* g = Q + (int64_t)row * P;

  int acc[C][NR];
#pragma unroll
  for (int q = 0; q < C; ++q)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[q][r] = 0;

  // the loads of NB blocks at k, k + 1024, ... are issued before any of their
  // products
  auto blocks = [&](int64_t k, auto nb) {
    constexpr int NB = decltype(nb)::value;
    v4i gd[NB][S], xd[NB][SR][NR];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
#pragma unroll
      for (int s = 0; s < S; ++s) gd[q][s] = *(const v4i*)(g + s * plane + k + 1024 * q);
#pragma unroll
      for (int t = 0; t < SR; ++t)
#pragma unroll
        for (int r = 0; r < NR; ++r) xd[q][t][r] = *(const v4i*)(Xq + t * xplane + (int64_t)r * P + k + 1024 * q);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int t = 0; t < SR; ++t)
#pragma unroll
          for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[s + t][r] = dot4(gd[q][s][e], xd[q][t][r][e], acc[s + t][r]);
  };

  // whole groups of UB blocks (the same count for every lane), then the
  // remaining 256-byte pieces of P (a multiple of 256) lane by lane
  int64_t b = 0;
  for (; b + 1024 * UB <= P; b += 1024 * UB) blocks(b + lane * 16, std::integral_constant<int, UB>{});
  for (int64_t k = b + lane * 16; k < P; k += 1024) blocks(k, std::integral_constant<int, 1>{});

  // lanes' class sums added in int64, recombined, scaled, lifted
  int64_t v[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    int64_t cls[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
      int64_t x = acc[q][r];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      cls[q] = x;
    }
    int64_t t = cls[0];
#pragma unroll
    for (int q = 1; q < C; ++q) t = t * 256 + cls[q];
    v[r] = t;
  }
  if (lane < NR) {
    int64_t mine = v[0];
#pragma unroll
    for (int r = 1; r < NR; ++r)
      if (r == lane) mine = v[r];
    const int em = row_exp ? row_exp[row] : 0;
    const double scale = ldexp(c, em + col_exp[lane]);
    double u = (double)mine * scale;
    if (w) u = u + w[row];
    U[(int64_t)lane * ldu + row] = u;
  }
}

template <int S, int SR>
hipError_t launch_sr(const GemmI8Args& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + 3) / 4));
  switch (a.nrhs) {
#define PINV_GEMV_I8(R)                                                                                          \
  case R:                                                                                                        \
    hipLaunchKernelGGL((gemv_i8_kernel<S, SR, R>), grid, dim3(256), 0, s, a.Q, a.X, a.P, a.Rpad, a.n, a.row_exp, \
                       a.col_exp, a.c, a.w, a.U, a.ldu);                                                         \
    break;
    PINV_GEMV_I8(1) PINV_GEMV_I8(2) PINV_GEMV_I8(3) PINV_GEMV_I8(4)
#undef PINV_GEMV_I8
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemv_i8(const GemmI8Args& a, hipStream_t s) {
  if (a.nrhs <= 0 || a.n <= 0) return hipSuccess;
  if (a.nrhs > GEMV_I8_MAX_RHS || a.P % 256 != 0 || a.n > a.P || a.Rpad < a.nrhs || a.ucols || a.kbytes)
    return hipErrorInvalidValue;
  if (((uintptr_t)a.Q % 16) != 0 || ((uintptr_t)a.X % 16) != 0) return hipErrorInvalidValue;
  switch (a.S * 4 + a.SR) {
    case 1 * 4 + 1: return launch_sr<1, 1>(a, s);
    case 1 * 4 + 2: return launch_sr<1, 2>(a, s);
    case 1 * 4 + 3: return launch_sr<1, 3>(a, s);
    case 2 * 4 + 1: return launch_sr<2, 1>(a, s);
    case 2 * 4 + 2: return launch_sr<2, 2>(a, s);
    case 2 * 4 + 3: return launch_sr<2, 3>(a, s);
    case 3 * 4 + 1: return launch_sr<3, 1>(a, s);
    case 3 * 4 + 2: return launch_sr<3, 2>(a, s);
    case 3 * 4 + 3: return launch_sr<3, 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}
