// The BF16x3 split product (step 3 with G and rho each written as two
// bfloat16 parts, hi + lo; the products hi*hi, hi*lo and lo*hi summed in FP32)
// on a one-wave-per-SIMD tile.
//
// The product is bound by the operand stream into LDS: two G parts and two
// rho parts per k step feed three products, so the wider the output tile the
// fewer bytes per product.  With only two FP32 accumulator sets (the leading
// product, and the two corrections together) a wave holds 64 x 128 outputs in
// the 256 accumulation registers, and a 4-wave workgroup (2 x 2) a tile of
// 128 rows of G x 256 right-hand sides: 64 bytes of operands per k for 256 x
// 128 x 3 products, a third fewer than the 128 x 128 tiles of the int8
// kernel's bfloat16 form.
//
// Operands move global -> LDS with global_load_lds_dwordx4 in 64-byte row
// pieces (32 bfloat16 of k), whose 16-byte chunks are XOR-swizzled (chunk c of
// row r at position c ^ ((r >> 2) & 3)) so that a fragment read -- 16
// consecutive rows, one chunk per lane group -- is free of bank conflicts.
// Three 48 KB stages, two in flight; one barrier per k step.  The step's 96
// products (v_mfma_f32_16x16x32_bf16, accumulators updated in place by
// inline-asm products) run while the next stage's 24 fragments are read into
// the second register set and the stage three ahead is loaded.
//
// v_mfma_f32_16x16x32_bf16 (lane l): A(i = l%16, k = 8(l/16) + t),
// B(k = 8(l/16) + t, j = l%16), t = 0..7; D(i = 4(l/16) + r, j = l%16).
//
// Layouts (those of the split path): G parts [2+][P][P] bf16 (part stride
// P*P, zero past column n), rho parts [2][Rpad][P] bf16 with Rpad a multiple
// of 256 (zero past row n and column nrhs); u column-major (stride ldu).  The
// sum hi*hi + (hi*lo + lo*hi) is formed in FP64 from the two FP32
// accumulators and scaled once; with a k split each split's sums go to
// part[z][r][m] (FP64) for launch_splitk_reduce.

#include "common.h"

#include <type_traits>

#define PINV_LDS(p) ((__attribute__((address_space(3))) void*)(p))

namespace {

constexpr int BTM = 128, BTN = 256, BKE = 32;    // tile rows, tile columns, k per stage (bf16)
constexpr int ROWB = 64;                          // bytes per LDS row (BKE bf16)
constexpr int A_PART = BTM * ROWB, B_PART = BTN * ROWB;
constexpr int A_BYTES = 2 * A_PART, B_BYTES = 2 * B_PART;
constexpr int BSTAGE = A_BYTES + B_BYTES;        // 48 KB
constexpr int BNST = 3;

template <int V>
__device__ inline void wait_vm() {
  static_assert(V >= 0 && V < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((V & 15) | (((V >> 4) & 3) << 14) | (7 << 4) | (15 << 8));
}
__device__ inline void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4)); }
__device__ inline void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }

__device__ inline int swz4(int row, int c) { return c ^ ((row >> 2) & 3); }

__device__ inline void mfma_bf16_acc(v4f& acc, const v4i& a, const v4i& b) {
  asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %2, %0" : "+a"(acc) : "v"(a), "v"(b));
}

__global__ __launch_bounds__(256, 1) void gemm_bf16x3_w4_kernel(
    const int8_t* __restrict__ Ga, int64_t P, const int8_t* __restrict__ Xa, int Rpad, int nrows, int nrhs,
    double alpha, const double* __restrict__ w, double* __restrict__ U, int64_t ldu, int tilesM, int tilesN,
    int ksplit, int kchunk, double* __restrict__ part) {
  __shared__ __attribute__((aligned(1024))) int8_t sm[BNST * BSTAGE];
  constexpr int IA = 4, IB = 8, ND = IA + IB;   // DMA instructions per wave per stage

  // XCD-aware tile order, row-major: the column tiles of one row block share
  // an XCD's L2
  const int T = tilesM * tilesN;
  const int per = (T + 7) / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= T) return;
  const int mt = tile / tilesN, nt = tile % tilesN;
  const int m0 = mt * BTM, n0 = nt * BTN;
  const int kz = blockIdx.y;
  const int64_t kb = ksplit > 1 ? (int64_t)kz * kchunk : 0;
  const int64_t ke = ksplit > 1 ? min(P, kb + kchunk) : P;
  const int nsteps = (int)((ke - kb) / BKE);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t rowb = P * 2;  // bytes per operand row

  // DMA: A instruction j (0..15) = part j / 8, rows 16 (j % 8) .. + 15 of the
  // tile; B instruction j (0..31) = part j / 16, rows 16 (j % 16) .. + 15.
  // Wave w issues A instructions 4w .. 4w + 3 and B instructions 8w .. 8w + 7,
  // so all of its instructions fall in part w / 2, row blocks 4 (w % 2) + d
  // of A and 8 (w % 2) + d of B.  Lane l lands at row l / 4, chunk position
  // l % 4 of its 16-row block and loads the logical chunk the swizzle puts
  // there.
  const int lrow = lane >> 2;
  const int lchunk = (lane & 3) ^ ((lane >> 4) & 3);
  const int wpart = wave >> 1, whalf = wave & 1;
  const int8_t* srcA = Ga + (int64_t)wpart * P * P * 2 + (int64_t)m0 * rowb;
  const int8_t* srcB = Xa + (int64_t)wpart * Rpad * rowb + (int64_t)n0 * rowb;
  const int dstA = wpart * A_PART + whalf * IA * 1024;
  const int dstB = A_BYTES + wpart * B_PART + whalf * IB * 1024;
  uint32_t oa[IA], ob[IB];
#pragma unroll
  for (int q = 0; q < IA; ++q) oa[q] = (uint32_t)(((whalf * IA + q) * 16 + lrow) * rowb + lchunk * 16);
#pragma unroll
  for (int q = 0; q < IB; ++q) ob[q] = (uint32_t)(((whalf * IB + q) * 16 + lrow) * rowb + lchunk * 16);
  auto dma = [&](int step, int buf, int d) {
    const int64_t k0 = (int64_t)__builtin_amdgcn_readfirstlane((int)((kb + (int64_t)step * BKE) * 2));
    int8_t* dst = sm + buf * BSTAGE;
    if (d < IA)
      __builtin_amdgcn_global_load_lds((const void*)(srcA + k0 + oa[d]), PINV_LDS(dst + dstA + d * 1024), 16, 0, 0);
    else
      __builtin_amdgcn_global_load_lds((const void*)(srcB + k0 + ob[d - IA]),
                                       PINV_LDS(dst + dstB + (d - IA) * 1024), 16, 0, 0);
  };

  // fragment reads: row lane % 16 of a 16-row block, logical chunk lane / 16
  // (block bases are multiples of 16 rows, where the swizzle's row term is 0)
  const int fr = lane & 15, g = lane >> 4;
  const int foff = fr * ROWB + swz4(fr, g) * 16;
  const int aoff = wm * 64 * ROWB, boff = A_BYTES + wn * 128 * ROWB;

  // two FP32 accumulator sets (hi*hi; hi*lo + lo*hi), 64 x 128 per wave,
  // homed in the accumulation registers by a zero product
  v4f hi[4][8], lo[4][8];
  const v4i zero = {0, 0, 0, 0};
  asm volatile("s_nop 4" ::: "memory");
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, 0" : "=a"(hi[i][j]) : "v"(zero));
      asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, 0" : "=a"(lo[i][j]) : "v"(zero));
    }

  // fragment sets: A part p block i, B part p block j
  v4i fa0[2][4], fb0[2][8], fa1[2][4], fb1[2][8];
  auto read = [&](const int8_t* base, int f, v4i (&fa)[2][4], v4i (&fb)[2][8]) {
    if (f < 8) {
      fa[f / 4][f % 4] = *(const v4i*)(base + aoff + (f / 4) * A_PART + (f % 4) * 16 * ROWB + foff);
    } else {
      const int q = f - 8;
      fb[q / 8][q % 8] = *(const v4i*)(base + boff + (q / 8) * B_PART + (q % 8) * 16 * ROWB + foff);
    }
  };
  // one k step: the 96 products of (fa, fb) with the 24 reads of the next
  // stage into (na, nb) and the stage's DMA spread between them
  auto compute = [&](const v4i (&fa)[2][4], const v4i (&fb)[2][8], const int8_t* nbase, v4i (&na)[2][4],
                     v4i (&nb)[2][8], int dstep, int dbuf) {
    constexpr int M_ = 96, RR = 24;
#pragma unroll
    for (int q = 0; q < M_; ++q) {
      const int pr = q / 32, i = (q / 8) % 4, j = q % 8;
      if (pr == 0) mfma_bf16_acc(hi[i][j], fa[0][i], fb[0][j]);
      else if (pr == 1) mfma_bf16_acc(lo[i][j], fa[0][i], fb[1][j]);
      else mfma_bf16_acc(lo[i][j], fa[1][i], fb[0][j]);
#pragma unroll
      for (int r = (q * RR + M_ - 1) / M_; r < ((q + 1) * RR + M_ - 1) / M_; ++r) read(nbase, r, na, nb);
#pragma unroll
      for (int d = (q * ND + M_ - 1) / M_; d < ((q + 1) * ND + M_ - 1) / M_; ++d) dma(dstep, dbuf, d);
    }
  };

  // prologue: stages 0-2 in flight (past the end: the last stage again), stage
  // 0 read once it has landed
#pragma unroll
  for (int p = 0; p < BNST; ++p)
#pragma unroll
    for (int d = 0; d < ND; ++d) dma(min(p, nsteps - 1), p, d);
  wait_vm<2 * ND>();
  lds_barrier();
#pragma unroll
  for (int f = 0; f < 24; ++f) read(sm, f, fa0, fb0);

  // step k: this wave's reads of stage k are complete and stage k + 1 has
  // landed (stage k + 2 may be in flight), barrier (every wave is done with
  // stage k's buffer); then the products of stage k (read during step k - 1)
  // with the reads of stage k + 1 and the DMA of stage k + 3 into stage k's
  // buffer.  Past the end the DMA loads the last stage again (in bounds; that
  // buffer is not read again), keeping the wait counts fixed; the last step's
  // reads of "stage k + 1" go unused.
  int buf = 0;
  auto step = [&](int k, const v4i (&fa)[2][4], const v4i (&fb)[2][8], v4i (&na)[2][4], v4i (&nb)[2][8]) {
    wait_lgkm0();
    wait_vm<ND>();
    lds_barrier();
    const int nbuf = buf == BNST - 1 ? 0 : buf + 1;
    compute(fa, fb, sm + nbuf * BSTAGE, na, nb, min(k + BNST, nsteps - 1), buf);
    buf = nbuf;
  };
  int k = 0;
  for (; k + 2 <= nsteps; k += 2) {
    step(k, fa0, fb0, fa1, fb1);
    step(k + 1, fa1, fb1, fa0, fb0);
  }
  if (k < nsteps) step(k, fa0, fb0, fa1, fb1);
  wait_vm<0>();
  wait_lgkm0();
  // the accumulators are read below by ordinary instructions: let the last
  // products retire first (the hazard checks do not see inside inline asm)
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");

#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n = n0 + wn * 128 + j * 16 + fr;
      if (n >= nrhs) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + 4 * g + r;
        if (m >= nrows) continue;
        const double sum = (double)hi[i][j][r] + (double)lo[i][j][r];
        if (ksplit > 1) {
          part[((int64_t)kz * nrhs + n) * nrows + m] = sum;
        } else {
          double v = alpha * sum;
          if (w) v += w[m];
          U[(int64_t)n * ldu + m] = v;
        }
      }
    }
  }
}

}  // namespace

BF16W4Plan bf16x3_w4_plan(int64_t P, int nrhs) {
  BF16W4Plan p;
  p.Rpad = (nrhs + BTN - 1) / BTN * BTN;
  p.tilesM = (int)(P / BTM);
  p.tilesN = p.Rpad / BTN;
  // one workgroup per compute unit: split k over up to 8 workgroups per tile
  // where the tiles leave units idle, at least 512 of k per split, whole steps
  const int T = p.tilesM * p.tilesN;
  int z = T > 0 ? 256 / T : 1;
  if (z > 8) z = 8;
  while (z > 1 && P / z < 512) --z;
  p.ksplit = 1;
  p.kchunk = (int)P;
  if (z >= 2) {
    int64_t chunk = (P + z - 1) / z;
    chunk = (chunk + BKE - 1) / BKE * BKE;
    p.ksplit = (int)((P + chunk - 1) / chunk);
    p.kchunk = (int)chunk;
  }
  return p;
}

hipError_t launch_gemm_bf16x3_w4(const BF16W4Plan& p, const __bf16* Gb, int64_t P, const __bf16* Xb, int nrows,
                                 int nrhs, double alpha, const double* w, double* U, int64_t ldu, double* part,
                                 hipStream_t s) {
  if (nrhs <= 0 || nrows <= 0) return hipSuccess;
  // operands cover whole tiles and whole k steps; 32-bit in-tile offsets
  if (P % 256 != 0 || p.Rpad % BTN != 0 || p.Rpad < nrhs || nrows > P || (uint64_t)BTN * P * 2 >= (1ull << 32) ||
      ((uintptr_t)Gb % 16) != 0 || ((uintptr_t)Xb % 16) != 0 || (p.ksplit > 1 && !part) ||
      p.tilesM != (int)(P / BTM) || p.tilesN != p.Rpad / BTN || p.kchunk % BKE != 0 ||
      (int64_t)p.kchunk * (p.ksplit - 1) >= P)
    return hipErrorInvalidValue;
  const int T = p.tilesM * p.tilesN;
  hipLaunchKernelGGL(gemm_bf16x3_w4_kernel, dim3((unsigned)(((T + 7) / 8) * 8), (unsigned)p.ksplit), dim3(256), 0, s,
                     (const int8_t*)Gb, P, (const int8_t*)Xb, p.Rpad, nrows, nrhs, alpha, w, U, ldu, p.tilesM,
                     p.tilesN, p.ksplit, p.kchunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.ksplit <= 1) return e;
  return launch_splitk_reduce(part, p.ksplit, nrows, nrhs, alpha, 0.0, w, U, 1, ldu, s);
}
