// The plain FP64 apply u = alpha G X + bias (step 3 with the inverse held in
// FP64) for many right-hand sides, on the FP64 matrix cores.
//
// One wave per SIMD: 256-thread workgroups of 4 waves in 2 x 2, output tile
// 256 rows of G x 128 right-hand sides, each wave 128 x 64 = 8 x 4 blocks of
// v_mfma_f64_16x16x4_f64.  The 32 block accumulators (4 doubles each, 256
// registers per lane) fill the accumulation registers and are operands of
// inline-asm products that read and write them in place.  Operands move
// global -> LDS with global_load_lds_dwordx4 in 128-byte row pieces (16
// doubles of k), whose 16-byte chunks are XOR-swizzled so that a fragment read
// (16 consecutive rows, one chunk) is conflict-free; three LDS stages of 48 KB,
// two in flight.  Each step's products run in two halves (k slices 0-1, 2-3)
// while the other half's fragments are read into the registers just freed;
// one barrier per step.  A taller tile
// than the 128 x 128 of the general GEMM halves the number of workgroups that
// read each row block of G.
//
// Layouts: G row-major [M][lda], zero between column K and the next multiple
// of 16 (the operator's storage pads rows to 32 doubles with zeros); the
// right-hand sides are first copied into a zero-padded [Npad][ldp] block
// (Npad = 128 ceil(N / 128), ldp = 32 ceil(K / 32)), so the main loop has no
// bounds checks; rows of G beyond M are read from row M - 1 and their
// outputs dropped.
//
// v_mfma_f64_16x16x4_f64 (lane l, result register r):
//   A(i = l%16, k = l/16), B(k = l/16, j = l%16), D(i = l/16 + 4r, j = l%16).
// Each lane reads 4 consecutive k (two 16-byte chunks) of its fragment row
// once per step and feeds them to the step's 4 k-slices, so the k order
// inside a step is permuted the same way for both operands.

#include "common.h"

#include <type_traits>

#define PINV_LDS(p) ((__attribute__((address_space(3))) void*)(p))

namespace {

typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int FBM = 256, FBN = 128, FBK = 16, FNST = 3;
constexpr int FA_BYTES = FBM * FBK * 8;     // one stage of G: 32 KB
constexpr int FB_BYTES = FBN * FBK * 8;     // one stage of right-hand sides: 16 KB
constexpr int FSTAGE = FA_BYTES + FB_BYTES;

template <int V>
__device__ inline void wait_vm() {
  static_assert(V >= 0 && V < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((V & 15) | (((V >> 4) & 3) << 14) | (7 << 4) | (15 << 8));
}
__device__ inline void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4)); }
__device__ inline void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }

// 16-byte chunk c of tile row `row` sits at chunk position c ^ ((row >> 1) & 7)
__device__ inline int swz8(int row, int c) { return c ^ ((row >> 1) & 7); }

// acc += a * b on the matrix cores, accumulator in place
__device__ inline void mfma_f64_acc(v4d& acc, double a, double b) {
  asm volatile("v_mfma_f64_16x16x4_f64 %0, %1, %2, %0" : "+a"(acc) : "v"(a), "v"(b));
}

// right-hand sides (column-major K x N: vector n at X + n ldx, k contiguous)
// -> zero-padded [Npad][ldp]
__global__ __launch_bounds__(256) void pack_rhs_kernel(const double* __restrict__ X, int64_t ldx, int K, int N,
                                                       int64_t ldp, int Npad, double* __restrict__ Xp) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)Npad * ldp) return;
  const int64_t n = idx / ldp, k = idx % ldp;
  Xp[idx] = (n < N && k < K) ? X[n * ldx + k] : 0.0;
}

__global__ __launch_bounds__(256, 1) void apply_f64_w4_kernel(const double* __restrict__ A, int64_t lda, int M,
                                                              int K, const double* __restrict__ Bp, int64_t ldp,
                                                              int N, double alpha, const double* __restrict__ bias,
                                                              double* __restrict__ C, int64_t ldc, int tilesM,
                                                              int tilesN, int ksplit, int kchunk,
                                                              double* __restrict__ part) {
  __shared__ __attribute__((aligned(1024))) int8_t sm[FNST * FSTAGE];
  constexpr int IA = 8, IB = 4;              // DMA instructions per wave per stage (G, rhs)
  constexpr int ND = IA + IB;

  // XCD-aware tile order: XCD x (workgroups x, x + 8, ...) takes a contiguous
  // range of tiles, row-major, so the column tiles of one row block share an L2
  const int T = tilesM * tilesN;
  const int per = (T + 7) / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= T) return;
  const int mt = tile / tilesN, nt = tile % tilesN;
  const int m0 = mt * FBM, n0 = nt * FBN;
  const int kz = blockIdx.y;
  const int kb = ksplit > 1 ? kz * kchunk : 0;
  const int ke = ksplit > 1 ? min(K, kb + kchunk) : K;
  const int nsteps = (ke - kb + FBK - 1) / FBK;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;

  // DMA: instruction j of wave w fills 8 rows (1 KB) of a stage; lane l lands
  // at row l / 8, chunk position l % 8, and loads the logical chunk the swizzle
  // puts there.  32-bit byte offsets from the tile's first row.
  const int8_t* tA = (const int8_t*)(A + (int64_t)m0 * lda);
  const int8_t* tB = (const int8_t*)(Bp + (int64_t)n0 * ldp);
  uint32_t oa[IA], ob[IB];
#pragma unroll
  for (int j = 0; j < IA; ++j) {
    const int row = wave * 64 + j * 8 + lane / 8;
    const int rg = min(m0 + row, M - 1) - m0;
    oa[j] = (uint32_t)rg * (uint32_t)(lda * 8) + (uint32_t)(swz8(row, lane % 8) * 16);
  }
#pragma unroll
  for (int j = 0; j < IB; ++j) {
    const int row = wave * 32 + j * 8 + lane / 8;
    ob[j] = (uint32_t)row * (uint32_t)(ldp * 8) + (uint32_t)(swz8(row, lane % 8) * 16);
  }
  // DMA instruction d of stage `step` into LDS buffer `buf`
  auto dma = [&](int step, int buf, int d) {
    const int64_t k0 = (int64_t)__builtin_amdgcn_readfirstlane((kb + step * FBK) * 8);
    int8_t* dst = sm + buf * FSTAGE;
    if (d < IA) {
      __builtin_amdgcn_global_load_lds((const void*)(tA + k0 + oa[d]), PINV_LDS(dst + wave * 64 * 128 + d * 1024), 16,
                                       0, 0);
    } else {
      const int j = d - IA;
      __builtin_amdgcn_global_load_lds((const void*)(tB + k0 + ob[j]),
                                       PINV_LDS(dst + FA_BYTES + wave * 32 * 128 + j * 1024), 16, 0, 0);
    }
  };

  // fragment reads: lane group g = lane / 16 reads logical chunks 2g, 2g + 1
  // (k = 4g .. 4g + 3) of row lane % 16 of each 16-row block (block bases are
  // multiples of 16 rows, where the swizzle's row term is zero)
  const int fr = lane & 15, g = lane >> 4;
  const int sw = (fr >> 1) & 7;
  const int flo = fr * 128 + ((2 * g) ^ sw) * 16, fhi = fr * 128 + ((2 * g + 1) ^ sw) * 16;
  const int aoff = wm * 128 * 128, boff = FA_BYTES + wn * 64 * 128;

  // the accumulators start as 0 * 0 + 0 from a product written into the
  // accumulation registers, so the compiler keeps them there (zeros written
  // by ordinary instructions were given a home in the ordinary registers and
  // copied across on every step)
  v4d acc[8][4];
  const double zero = 0.0;
  asm volatile("s_nop 4" ::: "memory");  // (the zero operand was just written)
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) asm volatile("v_mfma_f64_16x16x4_f64 %0, %1, %1, 0" : "=a"(acc[i][j]) : "v"(zero));

  // one register set: fa[i][sk] (sk = k slice 0..3 of the step), fb[j][sk].
  // Slices 0-1 come from chunk 2g, slices 2-3 from chunk 2g + 1, so the first
  // half of a step (slices 0-1) can run while the second half's chunk is
  // read, and the second half while the next step's first chunk is read.
  double fa[8][4], fb[4][4];
  // read of fragment f (0..11: G block f for f < 8, else rhs block f - 8),
  // chunk h, of the stage at `base`
  auto read = [&](const int8_t* base, int f, int h) {
    if (f < 8) {
      const v2d v = *(const v2d*)(base + aoff + f * 16 * 128 + (h ? fhi : flo));
      fa[f][2 * h] = v.x;
      fa[f][2 * h + 1] = v.y;
    } else {
      const v2d v = *(const v2d*)(base + boff + (f - 8) * 16 * 128 + (h ? fhi : flo));
      fb[f - 8][2 * h] = v.x;
      fb[f - 8][2 * h + 1] = v.y;
    }
  };
  // half hh of a step: the 64 products of slices 2hh, 2hh + 1, with the 12
  // reads of chunk rh of the stage at `rbase` and (ND > 0) the DMA of stage
  // `dstep` spread between them
  auto half = [&](int hh, const int8_t* rbase, int rh, int dstep, int dbuf, auto nd) {
    constexpr int NDV = decltype(nd)::value;
    constexpr int M_ = 64, RR = 12;
#pragma unroll
    for (int q = 0; q < M_; ++q) {
      const int sk = 2 * hh + q / 32, i = (q / 4) % 8, j = q % 4;
      mfma_f64_acc(acc[i][j], fa[i][sk], fb[j][sk]);
#pragma unroll
      for (int r = (q * RR + M_ - 1) / M_; r < ((q + 1) * RR + M_ - 1) / M_; ++r) read(rbase, r, rh);
      if constexpr (NDV > 0) {
#pragma unroll
        for (int d = (q * NDV + M_ - 1) / M_; d < ((q + 1) * NDV + M_ - 1) / M_; ++d) dma(dstep, dbuf, d);
      }
    }
  };
  using DOn = std::integral_constant<int, ND>;
  using DOff = std::integral_constant<int, 0>;

  // prologue: stages 0-2 in flight; the first chunk of stage 0 read once it
  // has landed
#pragma unroll
  for (int p = 0; p < FNST; ++p)
#pragma unroll
    for (int d = 0; d < ND; ++d) dma(min(p, nsteps - 1), p, d);
  wait_vm<2 * ND>();
  lds_barrier();
#pragma unroll
  for (int f = 0; f < 12; ++f) read(sm, f, 0);

  // step k (its stage in LDS buffer B = k mod 3, a compile-time constant in
  // each copy of the loop body, so that the compiler can tell the DMA's
  // destination from the buffers being read and adds no waits on the DMA
  // before the LDS reads): first half (reads of stage k's second chunk
  // alongside); this wave's reads of stage k are complete and stage k + 1 has
  // landed (stage k + 2 may be in flight), barrier; second half (reads of
  // stage k + 1's first chunk, DMA of stage k + 3 into buffer B).  Past the end
  // the DMA loads the last stage again (in bounds; the buffer is not read
  // again), which keeps the wait counts fixed; the last step's reads of
  // "stage k + 1" read a buffer whose values go unused.
  auto step = [&](int k, auto bi) {
    constexpr int B = decltype(bi)::value;
    const int8_t* cur = sm + B * FSTAGE;
    const int8_t* nxt = sm + ((B + 1) % FNST) * FSTAGE;
    half(0, cur, 1, 0, 0, DOff{});
    wait_lgkm0();
    wait_vm<ND>();
    lds_barrier();
    half(1, nxt, 0, min(k + 3, nsteps - 1), B, DOn{});
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  using B2 = std::integral_constant<int, 2>;
  int k = 0;
  for (; k + 3 <= nsteps; k += 3) {
    step(k, B0{});
    step(k + 1, B1{});
    step(k + 2, B2{});
  }
  if (k < nsteps) step(k, B0{});
  if (k + 1 < nsteps) step(k + 1, B1{});
  wait_vm<0>();
  // the accumulators are read below by ordinary instructions: let the last
  // products retire first (the hazard checks do not see inside inline asm)
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");

#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + fr;
      if (n >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 128 + i * 16 + g + 4 * r;
        if (m >= M) continue;
        if (ksplit > 1) {
          part[((int64_t)kz * N + n) * M + m] = acc[i][j][r];
        } else {
          double v = alpha * acc[i][j][r];
          if (bias) v += bias[m];
          C[(int64_t)n * ldc + m] = v;
        }
      }
    }
  }
}

}  // namespace

ApplyF64Plan apply_f64_plan(int M, int N, int K) {
  ApplyF64Plan p;
  p.tilesM = (M + FBM - 1) / FBM;
  p.tilesN = (N + FBN - 1) / FBN;
  p.Npad = p.tilesN * FBN;
  p.ldp = ((int64_t)K + 31) / 32 * 32;
  // One workgroup per compute unit, so the tiles run in rounds of 256.  k is
  // split z ways (at least 512 of k per split, at most 16 splits, chunks of
  // whole 16-wide steps) where that shortens the estimate
  //   ceil(T z / 256) / z   rounds of whole-tile time
  //   + (z M N 16 bytes of partial sums written and read at ~4 TB/s + 10 us
  //      for the adding kernel) / whole-tile time,
  // whole-tile time being 2 * 256 * 128 * K flops at 90% of a compute unit's
  // share of the FP64 matrix peak: a grid smaller than the chip, or a last
  // round mostly empty (24^3 unknowns x 1024: 432 tiles), is then spread over
  // more workgroups, while 504 tiles (two nearly full rounds) stay unsplit.
  const int T = p.tilesM * p.tilesN;
  const double t_tile = 2.0 * FBM * FBN * (double)K / (0.9 * 78.6e12 / 256.0);
  int z = 1;
  double best = 1e300;
  for (int c = 1; c <= 16; ++c) {
    if (c > 1 && K / c < 512) break;
    const double rounds = (double)(((int64_t)T * c + 255) / 256) / c;
    const double extra = c > 1 ? ((double)c * M * N * 16.0 / 4e12 + 10e-6) / t_tile : 0.0;
    if (rounds + extra < best * 0.98) {
      best = rounds + extra;
      z = c;
    }
  }
  p.ksplit = 1;
  p.kchunk = K;
  if (z >= 2) {
    int chunk = (K + z - 1) / z;
    chunk = (chunk + FBK - 1) / FBK * FBK;
    p.ksplit = (K + chunk - 1) / chunk;
    p.kchunk = chunk;
  }
  p.pack_bytes = ((size_t)p.Npad * p.ldp * sizeof(double) + 255) / 256 * 256;
  p.part_bytes = p.ksplit > 1 ? (size_t)p.ksplit * M * N * sizeof(double) : 0;
  return p;
}

hipError_t launch_apply_f64(const ApplyF64Plan& p, const double* G, int64_t lda, int M, int K, const double* X,
                            int64_t ldx, int N, double alpha, const double* bias, double* U, int64_t ldu,
                            void* scratch, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  // 32-bit DMA offsets inside a tile: 256 rows of G, 128 rows of the packed
  // right-hand sides
  if ((uint64_t)FBM * (uint64_t)lda * 8 >= (1ull << 32) || (uint64_t)FBN * (uint64_t)p.ldp * 8 >= (1ull << 32) ||
      lda < p.ldp || lda % 2 != 0 || ((uintptr_t)G % 16) != 0)
    return hipErrorInvalidValue;
  double* Xp = (double*)scratch;
  double* part = p.ksplit > 1 ? (double*)((char*)scratch + p.pack_bytes) : nullptr;
  const int64_t packed = (int64_t)p.Npad * p.ldp;
  hipLaunchKernelGGL(pack_rhs_kernel, dim3((unsigned)((packed + 255) / 256)), dim3(256), 0, s, X, ldx, K, N, p.ldp,
                     p.Npad, Xp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int T = p.tilesM * p.tilesN;
  hipLaunchKernelGGL(apply_f64_w4_kernel, dim3((unsigned)(((T + 7) / 8) * 8), (unsigned)p.ksplit), dim3(256), 0, s,
                     G, lda, M, K, Xp, p.ldp, N, alpha, bias, U, ldu, p.tilesM, p.tilesN, p.ksplit, p.kchunk, part);
  e = hipGetLastError();
  if (e != hipSuccess || p.ksplit <= 1) return e;
  return launch_splitk_reduce(part, p.ksplit, M, N, alpha, 0.0, bias, U, 1, ldu, s);
}
