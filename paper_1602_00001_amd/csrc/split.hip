// Split-precision forms of step 3 (u = -h^2 G rho + w) on the matrix cores.
//
// FP32: G and rho rounded to float, v_mfma_f32_16x16x4f32, FP32 accumulation.
// BF16xNP (NP = 2 -> "BF16x3", NP = 3 -> "BF16x6"): every FP64 value x is
// written as x0 + x1 (+ x2) with x0 = bf16(x), x1 = bf16(x - x0), ... each
// rounded to nearest even directly from FP64 (the residuals are exact in FP64);
// the products a_i b_j with i + j <= NP - 1 are summed, the leading product in
// one FP32 accumulator and the correction products in a second, combined in
// FP64 at the end (the published bfloat16 split scheme of Henry, Tang and
// Heinecke, ARITH 2019).
//
// The bf16 products run on the tiled DMA kernel of the int8 digit GEMM
// (launch_gemm_bf16_parts): v_mfma_f32_16x16x32_bf16 takes its operands in the
// same 16-byte-per-lane layout as v_mfma_i32_16x16x64_i8 (lane l: A(i = l%16,
// k = 8*(l/16) + t), B(k = 8*(l/16) + t, j = l%16), D(i = 4*(l/16) + r,
// j = l%16)), 64 bytes of k per instruction, so the operand movement is the
// same byte for byte.  G's parts and the right-hand sides' parts are stored
// zero-padded to P x P and Rpad x P, so the main loops carry no bounds checks.

#include "common.h"

namespace {

__device__ inline double round_bf16_exact(double x) {
  // keep 8 significant bits, ties to even, directly from FP64
  if (x == 0.0) return 0.0;
  int e;
  const double m = frexp(x, &e);
  return ldexp(rint(ldexp(m, 8)), e - 8);
}

__device__ inline __bf16 to_bf16_exact(double v) {
  // v already holds a bfloat16 value: the conversion to float is exact and so
  // is float -> bf16 (any rounding mode)
  return (__bf16)(float)v;
}

__global__ __launch_bounds__(256) void make_fp32_kernel(const double* __restrict__ G, int64_t ldg, int n, int64_t P,
                                                       float* __restrict__ G32) {
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < P * P; idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx / P, k = idx % P;
    G32[idx] = (i < n && k < n) ? (float)G[i * ldg + k] : 0.0f;
  }
}

__global__ __launch_bounds__(256) void make_bf16_kernel(const double* __restrict__ G, int64_t ldg, int n, int64_t P,
                                                       int parts, __bf16* __restrict__ Gb) {
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < P * P; idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx / P, k = idx % P;
    double rest = (i < n && k < n) ? G[i * ldg + k] : 0.0;
    for (int p = 0; p < parts; ++p) {
      const double v = round_bf16_exact(rest);
      Gb[(int64_t)p * P * P + idx] = to_bf16_exact(v);
      rest = rest - v;
    }
  }
}

// right-hand sides (column-major n x nrhs, stride ldx) -> [parts][Rpad][P] bf16
__global__ __launch_bounds__(256) void pack_bf16_kernel(const double* __restrict__ X, int64_t ldx, int n, int nrhs,
                                                       int Rpad, int64_t P, int parts, __bf16* __restrict__ Xb) {
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < (int64_t)Rpad * P;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t r = idx / P, k = idx % P;
    double rest = (r < nrhs && k < n) ? X[r * ldx + k] : 0.0;
    for (int p = 0; p < parts; ++p) {
      const double v = round_bf16_exact(rest);
      Xb[(int64_t)p * Rpad * P + idx] = to_bf16_exact(v);
      rest = rest - v;
    }
  }
}

__global__ __launch_bounds__(256) void pack_fp32_kernel(const double* __restrict__ X, int64_t ldx, int n, int nrhs,
                                                       int Rpad, int64_t P, float* __restrict__ Xf) {
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < (int64_t)Rpad * P;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t r = idx / P, k = idx % P;
    Xf[idx] = (r < nrhs && k < n) ? (float)X[r * ldx + k] : 0.0f;
  }
}

__device__ inline void tile_of(int bid, int tilesM, int tilesN, int& mt, int& nt, bool& valid) {
  const int T = tilesM * tilesN;
  const int per = (T + 7) / 8;
  const int tile = (bid % 8) * per + bid / 8;
  valid = tile < T;
  mt = valid ? tile / tilesN : 0;
  nt = valid ? tile % tilesN : 0;
}

struct SplitArgs {
  const void* A;   // G parts [NP][P][P] (bf16) or G32 [P][P]
  const void* B;   // rhs parts [NP][Rpad][P] or [Rpad][P] float
  int64_t P;
  int Rpad, n, nrhs;
  double alpha;
  const double* w;
  double* U;
  int64_t ldu;
  // split-K: ksplit > 1 workgroups per tile, each over k in
  // [z*kchunk, (z+1)*kchunk); raw sums (FP64) to part[z][r][m] (n x nrhs per z)
  int ksplit;
  int64_t kchunk;
  double* part;
};

constexpr int BM = 128, BN = 128;

// FP32: 128x128 tiles, k step 16 floats, v_mfma_f32_16x16x4f32
// (lane l: A(i = l%16, k = l/16), B(k = l/16, j = l%16), D(i = 4*(l/16) + r, j = l%16)).
__global__ __launch_bounds__(256, 2) void gemm_fp32_kernel(SplitArgs a, int tilesM, int tilesN) {
  constexpr int BKK = 16, LDP = 128 + 32;
  __shared__ float As[2][BKK][LDP];
  __shared__ float Bs[2][BKK][LDP];
  int mt, nt;
  bool valid;
  tile_of(blockIdx.x, tilesM, tilesN, mt, nt, valid);
  if (!valid) return;
  const int m0 = mt * BM, n0 = nt * BN;
  const int64_t P = a.P;
  const float* A = (const float*)a.A;
  const float* B = (const float*)a.B;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // each thread loads 2 float4 of A and 2 of B per step: row = idx/4, k quad = idx%4
  float4 ra[2], rb[2];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int idx = t * 256 + tid;
      const int row = idx >> 2, kq = idx & 3;
      ra[t] = *(const float4*)(A + (int64_t)(m0 + row) * P + k0 + kq * 4);
      rb[t] = *(const float4*)(B + (int64_t)(n0 + row) * P + k0 + kq * 4);
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int idx = t * 256 + tid;
      const int row = idx >> 2, kq = idx & 3;
      As[st][kq * 4 + 0][row] = ra[t].x;
      As[st][kq * 4 + 1][row] = ra[t].y;
      As[st][kq * 4 + 2][row] = ra[t].z;
      As[st][kq * 4 + 3][row] = ra[t].w;
      Bs[st][kq * 4 + 0][row] = rb[t].x;
      Bs[st][kq * 4 + 1][row] = rb[t].y;
      Bs[st][kq * 4 + 2][row] = rb[t].z;
      Bs[st][kq * 4 + 3][row] = rb[t].w;
    }
  };
  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int kz = blockIdx.y;
  const int64_t K0 = a.ksplit > 1 ? kz * a.kchunk : 0;
  const int64_t K1 = a.ksplit > 1 ? min(P, (kz + 1) * a.kchunk) : P;
  int st = 0;
  load(K0);
  store(0);
  __syncthreads();
  for (int64_t k0 = K0; k0 < K1; k0 += BKK) {
    const bool has_next = k0 + BKK < K1;
    if (has_next) load(k0 + BKK);
#pragma unroll
    for (int k4 = 0; k4 < BKK / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      float fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[i] = As[st][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) fb[j] = Bs[st][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (has_next) store(st ^ 1);
    __syncthreads();
    st ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + (lane & 15);
      if (n >= a.nrhs) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        if (m >= a.n) continue;
        if (a.ksplit > 1) {
          a.part[((int64_t)kz * a.nrhs + n) * a.n + m] = (double)acc[i][j][r];
          continue;
        }
        double v = a.alpha * (double)acc[i][j][r];
        if (a.w) v += a.w[m];
        a.U[(int64_t)n * a.ldu + m] = v;
      }
    }
}

}  // namespace

hipError_t launch_make_fp32(const double* G, int64_t ldg, int n, float* G32, hipStream_t s) {
  const int64_t P = pinv_pad_dim(n);
  hipLaunchKernelGGL(make_fp32_kernel, dim3(grid_1d(P * P)), dim3(256), 0, s, G, ldg, n, P, G32);
  return hipGetLastError();
}

hipError_t launch_make_bf16_parts(const double* G, int64_t ldg, int n, int parts, __bf16* Gb, hipStream_t s) {
  const int64_t P = pinv_pad_dim(n);
  hipLaunchKernelGGL(make_bf16_kernel, dim3(grid_1d(P * P)), dim3(256), 0, s, G, ldg, n, P, parts,
                     Gb);
  return hipGetLastError();
}

namespace {

// split-K plan: enough workgroups for `target` in flight, at least 512 of k per
// split (kchunk a multiple of 256, so every split covers whole k steps of the
// zero-padded operands)
void split_plan(int64_t P, int Rpad, int target, int* ksplit, int64_t* kchunk) {
  const int T = (int)(P / BM) * (Rpad / BN);
  int z = target / (T > 0 ? T : 1);
  const int zmax = (int)(P / 512);
  if (z > zmax) z = zmax;
  if (z > 16) z = 16;
  if (z < 2) {
    *ksplit = 1;
    *kchunk = P;
    return;
  }
  int64_t chunk = (P + z - 1) / z;
  chunk = (chunk + 255) / 256 * 256;
  *ksplit = (int)((P + chunk - 1) / chunk);
  *kchunk = chunk;
}

int split_target(int mode) { return mode == PINV_FP32 ? 512 : 256; }

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// BF16x3 on the 128 x 256 one-wave-per-SIMD tiles where they fill at least
// half the chip without splitting k (126^2 x 1024: 1.62 -> 1.34 ms); smaller
// problems keep the 128 x 128 tiles, whose k splits are shorter (62^2 x 256:
// 52 us against 70 us)
bool bf16x3_wide(int64_t P, int nrhs) {
  const BF16W4Plan w = bf16x3_w4_plan(P, nrhs);
  return w.tilesM * w.tilesN >= 128;
}

}  // namespace

size_t split_scratch_bytes(int mode, const pinv_op_s* op, int nrhs) {
  const int64_t P = pinv_pad_dim(op->n);
  if (mode == PINV_BF16X3 && bf16x3_wide(P, nrhs)) {
    // 128 x 256 tiles, one wave per SIMD: rho parts padded to 256 columns
    const BF16W4Plan w = bf16x3_w4_plan(P, nrhs);
    const size_t part = w.ksplit > 1 ? (size_t)w.ksplit * op->n * nrhs * sizeof(double) : 0;
    return align256((size_t)2 * w.Rpad * P * sizeof(__bf16)) + part;
  }
  const int Rpad = (nrhs + 127) / 128 * 128;
  int ksplit;
  int64_t kchunk;
  split_plan(P, Rpad, split_target(mode), &ksplit, &kchunk);
  const size_t part = ksplit > 1 ? (size_t)ksplit * op->n * nrhs * sizeof(double) : 0;
  if (mode == PINV_FP32) return align256((size_t)Rpad * P * sizeof(float)) + part;
  const int parts = mode == PINV_BF16X3 ? 2 : 3;
  return align256((size_t)parts * Rpad * P * sizeof(__bf16)) + part;
}

hipError_t launch_gemm_split(int mode, const pinv_op_s* op, const double* X, int64_t ldx, int nrhs, double alpha,
                             double* U, int64_t ldu, hipStream_t s, void* scratch, size_t scratch_bytes) {
  const int64_t P = pinv_pad_dim(op->n);
  if (scratch_bytes < split_scratch_bytes(mode, op, nrhs)) return hipErrorInvalidValue;
  if (mode == PINV_BF16X3 && bf16x3_wide(P, nrhs)) {
    const BF16W4Plan w = bf16x3_w4_plan(P, nrhs);
    __bf16* Xb = (__bf16*)scratch;
    double* part = w.ksplit > 1 ? (double*)((char*)scratch + align256((size_t)2 * w.Rpad * P * sizeof(__bf16)))
                                : nullptr;
    hipLaunchKernelGGL(pack_bf16_kernel, dim3(grid_1d((int64_t)w.Rpad * P)), dim3(256), 0, s, X, ldx, op->n, nrhs,
                       w.Rpad, P, 2, Xb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_gemm_bf16x3_w4(w, op->Gb, P, Xb, op->n, nrhs, alpha, op->w, U, ldu, part, s);
  }
  const int Rpad = (nrhs + 127) / 128 * 128;
  const int tilesM = (int)(P / BM), tilesN = Rpad / BN;
  const int T = tilesM * tilesN;
  const int grid = ((T + 7) / 8) * 8;
  const unsigned pgrid = grid_1d((int64_t)Rpad * P);
  SplitArgs a{};
  a.P = P; a.Rpad = Rpad; a.n = op->n; a.nrhs = nrhs; a.alpha = alpha; a.w = op->w; a.U = U; a.ldu = ldu;
  a.B = scratch;
  split_plan(P, Rpad, split_target(mode), &a.ksplit, &a.kchunk);
  const size_t packed = mode == PINV_FP32 ? align256((size_t)Rpad * P * sizeof(float))
                                          : align256((size_t)(mode == PINV_BF16X3 ? 2 : 3) * Rpad * P * sizeof(__bf16));
  a.part = a.ksplit > 1 ? (double*)((char*)scratch + packed) : nullptr;
  const dim3 g3(grid, a.ksplit);
  if (mode == PINV_FP32) {
    hipLaunchKernelGGL(pack_fp32_kernel, dim3(pgrid), dim3(256), 0, s, X, ldx, op->n, nrhs, Rpad, P, (float*)scratch);
    a.A = op->G32;
    hipLaunchKernelGGL(gemm_fp32_kernel, g3, dim3(256), 0, s, a, tilesM, tilesN);
  } else {
    const int parts = mode == PINV_BF16X3 ? 2 : 3;
    hipLaunchKernelGGL(pack_bf16_kernel, dim3(pgrid), dim3(256), 0, s, X, ldx, op->n, nrhs, Rpad, P, parts,
                       (__bf16*)scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the parts' products on the tiled DMA kernel of the int8 slice GEMM (the
    // same byte layout: 128 x 128 tiles, 16-byte fragments, 64 bytes of k per
    // matrix-core instruction); G's parts are stored with op->nbf planes, the
    // first `parts` are read
    GemmI8Args g{};
    g.Q = (const int8_t*)op->Gb; g.S = parts;
    g.X = (const int8_t*)scratch; g.SR = parts;
    g.P = P; g.Rpad = Rpad; g.kbytes = 2 * P;
    g.n = op->n; g.nrhs = nrhs;
    g.c = alpha; g.w = op->w;
    g.U = U; g.ldu = ldu;
    g.ksplit = a.ksplit;
    g.kchunk = (int)(2 * a.kchunk);
    e = launch_gemm_bf16_parts(g, a.part, s);
    if (e != hipSuccess || a.ksplit <= 1) return e;
    return launch_splitk_reduce(a.part, a.ksplit, op->n, nrhs, alpha, 0.0, op->w, U, 1, ldu, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.ksplit <= 1) return e;
  return launch_splitk_reduce(a.part, a.ksplit, op->n, nrhs, alpha, 0.0, op->w, U, 1, ldu, s);
}
