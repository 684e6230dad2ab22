// Int8 digit-slice matrix-core product: the quantised form of step 3, u = L^{-1} rho.
//
// G^ = diag(2^e) Q / M_S with Q = sum_s 256^(S-1-s) Q_s (S int8 digit planes)
// and rho^ = X diag(2^f) / M_SR with X = sum_t 256^(SR-1-t) X_t, so
//   Q X = sum_c 256^(S+SR-2-c) A_c,   A_c = sum_{s+t=c} Q_s X_t.
// Each class accumulator A_c is an exact int32 sum of int8 x int8 products
// (v_mfma_i32_16x16x64_i8); the host checks that no class can overflow.  The
// epilogue recombines the classes exactly in int64 (Horner in base 256),
// converts once to double, multiplies by c * 2^(e_i + f_r) (c = -h^2/(M_S M_SR))
// and adds the lift w_i: two roundings, no fused multiply-add (the library is
// compiled with contraction off).
//
// Tiling: 128 (rows of G) x 128 (right-hand sides) per 512-thread workgroup,
// 8 waves in 4x2 (two per SIMD, so one wave's waits are covered by the other's
// matrix-core work), each 32x64 = 2x4 blocks of v_mfma_i32_16x16x64_i8 per
// class (128 accumulator registers per wave at four classes); or 64 x 128 per
// 256-thread workgroup, two workgroups per compute unit.
// Operand tiles move global -> LDS with global_load_lds_dwordx4 (no staging
// registers): one instruction fills 1 KB of LDS (one block of rows) per wave.
// LDS rows (BK = 128 or 64 bytes of k) are unpadded; the 16-byte chunks of a
// row are XOR-swizzled so the 16 lanes of a 128-bit fragment read (16
// consecutive rows, same logical chunk) hit 16 distinct 4-bank groups, and a
// lane of the DMA loads the global chunk that belongs at its own LDS slot.
// NST LDS stages (as many as fit, at most 4) keep NST-1 k steps of loads in
// flight.  Each wave waits for its own DMA group (vmcnt), then a plain
// s_barrier (no fence: a fence would drain all in-flight stages) makes the
// stage visible to all waves and frees the stage read one step earlier.
// The digit planes and quantised right-hand sides are zero-padded to the tile
// grid, so the main loop has no bounds checks.
//
// The variants (tile shape, k depth, tile order, fragment-read schedule) are
// listed above launch_v; all compute the same class sums.  Optional split-K
// (partial class sums added by a second kernel) and grouped launches (several
// operators, each workgroup finding its group in a device table) reuse the
// same kernel.
//
// v_mfma_i32_16x16x64_i8 layout (lane l, result register r):
//   A(i = l%16, k = 16*(l/16) + b), B(k = 16*(l/16) + b, j = l%16),
//   D(i = 4*(l/16) + r, j = l%16).

#include "common.h"

#include <type_traits>

#define PINV_LDS(p) ((__attribute__((address_space(3))) void*)(p))

namespace {

constexpr int BN = 128;               // right-hand sides per tile
constexpr int LDS_BYTES = 163840;     // per compute unit

// Tile processed by workgroup bid out of T: MAP 0 hands XCD x (workgroups
// x, x+8, ...) a contiguous range of tiles, so tiles sharing a row block of G
// share that XCD's L2; MAP 1 is linear.
template <int MAP>
__device__ inline int tile_index(int bid, int T) {
  const int per = (T + 7) / 8;
  return MAP == 0 ? (bid % 8) * per + bid / 8 : bid;
}

// s_waitcnt with only the vector-memory counter constrained (<= V)
template <int V>
__device__ inline void wait_vm() {
  static_assert(V >= 0 && V < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((V & 15) | (((V >> 4) & 3) << 14) | (7 << 4) | (15 << 8));
}

__device__ inline void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }

// s_waitcnt lgkmcnt(0) only (vector-memory and export counters unconstrained)
__device__ inline void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4)); }

// Kernel variants (picked per operator by pinv_autotune_int8): BK = k bytes
// per stage, 128 (full 128-byte cache lines per row, two stages) or 64 (as many
// stages as fit, at most 4); MAP 0 = XCD-aware tile order, 1 = linear; PF =
// read all operand fragments of a k half before its matrix-core work.
template <int S, int SR, int BK_, int NW_>
struct Cfg {
  static constexpr int NW = NW_;                           // waves per workgroup
  static constexpr int NT = NW * 64;
  static constexpr int BM = NW * 16;                       // rows per tile: waves in (BM/32) x 2
  static constexpr int WGS = NW == 8 ? 1 : 2;              // workgroups per compute unit
  static constexpr int C = S + SR - 1;
  static constexpr int BK = BK_;
  static constexpr int CH = BK / 16;                       // 16-byte chunks per row
  static constexpr int PLANE_A = BM * BK;                  // bytes of one G plane per stage
  static constexpr int PLANE_B = BN * BK;                  // bytes of one rho plane per stage
  static constexpr int STAGE = S * PLANE_A + SR * PLANE_B;
  static constexpr int NST_ = LDS_BYTES / WGS / STAGE;
  static constexpr int NST = NST_ > 4 ? 4 : NST_;
  static constexpr int RPI = 1024 / BK;                    // rows filled by one DMA instruction
  static constexpr int IPA = BM / NW / RPI;                // DMA instructions per G plane per wave
  static constexpr int IPB = BN / NW / RPI;                // DMA instructions per rho plane per wave
  static constexpr int L = S * IPA + SR * IPB;             // DMA instructions per thread per stage
  static_assert(NST >= 2, "two LDS stages must fit");
  static_assert(IPA >= 1 && IPB >= 1, "a wave fills at least one DMA block per plane");
};

// rho digits whose half-step products are deferred past the barrier in the
// split-step pipeline: registers per lane ~ 32 C (accumulators) + 4 (2S + 4SR)
// (fragments being read) + 4 (2S + 4DT) (fragments held) + misc <= 256
// (misc = registers for addresses and loop state: 8 when the compiler
// schedules freely, 24 with the order pinned)
constexpr int dt_of(int S, int SR, int misc, int acc_sets) {
  int dt = SR;
  while (dt > 1 && 32 * acc_sets + 4 * (2 * S + 4 * SR) + 4 * (2 * S + 4 * dt) + misc > 256) --dt;
  return dt;
}

template <int KIND> struct AccOf { using T = v4i; };   // int8 digit classes
template <> struct AccOf<1> { using T = v4f; };        // bfloat16 parts

// Swizzle: the 16-byte chunk c of tile row r sits at chunk position
// c ^ ((r >> 1) & 7) (128-byte rows) or c ^ ((r >> 2) & 3) (64-byte rows), so
// each 16 lanes of a fragment read (16 consecutive rows, one chunk) hit 16
// distinct 4-bank groups.
template <int CH>
__device__ inline int swz(int row, int c) {
  return CH == 8 ? (c ^ ((row >> 1) & 7)) : (c ^ ((row >> 2) & 3));
}

// KIND 0: int8 digit planes, int32 class accumulators (the quantised apply).
// KIND 1: bfloat16 split parts (S = SR = number of parts), two FP32
// accumulators; the operand movement is byte for byte the same.
template <int S, int SR, int BKV, int MAP, int PF, int NWV, int KIND = 0>
__global__ __launch_bounds__(NWV * 64, NWV == 8 ? 1 : 2) void gemm_i8_kernel(GemmI8Args a_in, int tilesM, int tilesN,
                                                                         const GemmI8Group* __restrict__ groups,
                                                                         int ngroups, int total, double* partf) {
  using K = Cfg<S, SR, BKV, NWV>;
  constexpr int C = K::C, BK = K::BK, CH = K::CH, STAGE = K::STAGE, NST = K::NST;
  constexpr int CA = KIND == 0 ? C : 2;  // accumulator sets
  using AT = typename AccOf<KIND>::T;
  constexpr int BM = K::BM, NW = K::NW, PLANE_A = K::PLANE_A, PLANE_B = K::PLANE_B;
  constexpr int RPI = K::RPI, IPA = K::IPA, IPB = K::IPB, L = K::L;
  __shared__ __attribute__((aligned(1024))) int8_t sm[NST * STAGE];

  // tile of this workgroup; in a grouped launch, also its group (binary
  // search over the groups' first tiles, uniform per workgroup) and the
  // group's arguments
  GemmI8Args a = a_in;
  int tN = tilesN;
  const int T = groups ? total : tilesM * tilesN;
  int tile = tile_index<MAP>(blockIdx.x, T);
  if (tile >= T) return;
  if (groups) {
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (groups[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    a = groups[lo].a;
    tN = groups[lo].tilesN;
    tile -= groups[lo].tile0;
  }
  const int mt = tile / tN, nt = tile % tN;
  const int m0 = (a.mt0 + mt) * BM, n0 = nt * BN;
  const int64_t prow = (int64_t)tilesM * BM;  // rows of the split-K partial sums
  const int64_t P = a.P;
  const int64_t KBY = a.kbytes ? a.kbytes : P;  // bytes of k per row
  // k steps of this workgroup: all of k, or its split's share
  const int z = blockIdx.y;
  const int kfirst = a.ksplit > 1 ? z * (a.kchunk / BK) : 0;
  const int nsteps = a.ksplit > 1 ? (int)(min(KBY, (int64_t)(z + 1) * a.kchunk) / BK) - kfirst : (int)(KBY / BK);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;     // (BM/32) x 2 waves, each 32 rows x 64 right-hand sides

  // DMA: instruction j of wave w fills plane rows w*(rows/NW) + j*RPI .. + RPI-1;
  // lane l lands at LDS byte l*16 of that block = row l / CH, chunk position
  // l % CH, so it loads the logical chunk whose swizzled position is l % CH.
  // The address is a wave-uniform plane base plus a 32-bit per-lane offset.
  uint32_t offa[IPA], offb[IPB];
#pragma unroll
  for (int j = 0; j < IPA; ++j) {
    const int row = wave * (BM / NW) + j * RPI + lane / CH;
    offa[j] = (uint32_t)row * (uint32_t)KBY + (uint32_t)(swz<CH>(row, lane % CH) * 16);  // swizzle is an involution
  }
#pragma unroll
  for (int j = 0; j < IPB; ++j) {
    const int row = wave * (BN / NW) + j * RPI + lane / CH;
    offb[j] = (uint32_t)row * (uint32_t)KBY + (uint32_t)(swz<CH>(row, lane % CH) * 16);
  }
  const int8_t* tileA = a.Q + (int64_t)m0 * KBY;
  const int8_t* tileB = a.X + (int64_t)n0 * KBY;
  const int64_t planeA = P * KBY, planeB = (int64_t)a.Rpad * KBY;

  auto issue = [&](int step) {
    int8_t* dst = sm + (step % NST) * STAGE;
    // (through readfirstlane, so the compiler keeps one scalar base per plane
    // and a 32-bit lane offset instead of strength-reducing every DMA address
    // into a 64-bit vector register)
    const int64_t k0 = (int64_t)__builtin_amdgcn_readfirstlane((kfirst + step) * BK);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int8_t* b = tileA + s * planeA + k0;
      int8_t* d = dst + s * PLANE_A + wave * (BM / NW) * BK;
#pragma unroll
      for (int j = 0; j < IPA; ++j)
        __builtin_amdgcn_global_load_lds((const void*)(b + offa[j]), PINV_LDS(d + j * 1024), 16, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < SR; ++t) {
      const int8_t* b = tileB + t * planeB + k0;
      int8_t* d = dst + S * PLANE_A + t * PLANE_B + wave * (BN / NW) * BK;
#pragma unroll
      for (int j = 0; j < IPB; ++j)
        __builtin_amdgcn_global_load_lds((const void*)(b + offb[j]), PINV_LDS(d + j * 1024), 16, 0, 0);
    }
  };

  // fragment read offsets (bytes within a plane) for k half h: rows
  // (16-row block base) + lane%16, logical chunk 4h + lane/16
  const int frow = lane & 15;
  int foff[BK / 64];
#pragma unroll
  for (int h = 0; h < BK / 64; ++h) foff[h] = frow * BK + swz<CH>(frow, 4 * h + (lane >> 4)) * 16;

  AT acc[CA][2][4];
#pragma unroll
  for (int c = 0; c < CA; ++c)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[c][i][j] = AT{0, 0, 0, 0};

  // one product of digit s of G with digit t of rho (KIND 1: of part s of G
  // with part t of rho, kept only when s + t <= S - 1)
  auto mma = [&](int s, int t, int i, int j, const v4i& fa, const v4i& fb) {
    if constexpr (KIND == 0) {
      acc[s + t][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa, fb, acc[s + t][i][j], 0, 0, 0);
    } else {
      if (s + t > S - 1) return;
      const int q = s + t == 0 ? 0 : 1;
      acc[q][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, fa), __builtin_bit_cast(v8bf, fb),
                                                             acc[q][i][j], 0, 0, 0);
    }
  };

  // fragment reads of k half h of the stage at `base` and the products of one
  // k half (16-row blocks start at multiples of 16, where the swizzle of the
  // block base is zero, so one lane offset serves every block)
  auto read_a = [&](const int8_t* base, int h, int s, v4i (&fa)[2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) fa[i] = *(const v4i*)(base + s * PLANE_A + (wm * 32 + i * 16) * BK + foff[h]);
  };
  auto read_b_t = [&](const int8_t* base, int h, int t0, int t1, v4i (&fb)[SR][4]) {
#pragma unroll
    for (int t = t0; t < t1; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        fb[t][j] = *(const v4i*)(base + S * PLANE_A + t * PLANE_B + (wn * 64 + j * 16) * BK + foff[h]);
  };
  auto read_b = [&](const int8_t* base, int h, v4i (&fb)[SR][4]) {
#pragma unroll
    for (int t = 0; t < SR; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        fb[t][j] = *(const v4i*)(base + S * PLANE_A + t * PLANE_B + (wn * 64 + j * 16) * BK + foff[h]);
  };
  auto products_t = [&](int s, int t0, int t1, const v4i (&fa)[2], const v4i (&fb)[SR][4]) {
#pragma unroll
    for (int t = t0; t < t1; ++t)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) mma(s, t, i, j, fa[i], fb[t][j]);
  };
  auto products = [&](int s, const v4i (&fa)[2], const v4i (&fb)[SR][4]) {
#pragma unroll
    for (int t = 0; t < SR; ++t)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) mma(s, t, i, j, fa[i], fb[t][j]);
  };

  if constexpr (PF >= 2 && NST == 2 && BK == 128) {
    // Split-step pipeline: the barrier sits inside the second k half of a
    // step.  Before it a wave multiplies half 0 while reading half 1, then the
    // first SR - DT rho digits of half 1; after it the wave multiplies the last
    // DT rho digits of half 1 (fragments already in registers) while reading
    // half 0 of the next stage, so the matrix cores have work while the fresh
    // stage's first fragments are in flight.  DT is as large as the registers
    // allow (the fragments held across the barrier are 2S + 4DT registers of
    // 128 bits).
    constexpr int DT = dt_of(S, SR, PF == 3 ? 24 : 8, CA);
    v4i xa[S][2], xb[SR][4], ya[S][2], yb[SR][4];
    issue(0);
    wait_vm<0>();
    lds_barrier();
    if (nsteps > 1) issue(1);
    read_b(sm, 0, xb);
#pragma unroll
    for (int s = 0; s < S; ++s) read_a(sm, 0, s, xa[s]);
    for (int k = 0; k < nsteps; ++k) {
      const int8_t* base = sm + (k & 1) * STAGE;
      if constexpr (PF == 3) {
        // order pinned: half 1's rho fragments first, then after the products
        // of each G digit of half 0 the reads of that digit for half 1 (into
        // registers it has just freed), so every read has a digit's products
        // to hide behind and no more than one and a half fragment sets live
        read_b(base, 1, yb);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          __builtin_amdgcn_sched_barrier(0);
          products(s, xa[s], xb);
          __builtin_amdgcn_sched_barrier(0);
          read_a(base, 1, s, ya[s]);
        }
        __builtin_amdgcn_sched_barrier(0);
      } else {
        read_b(base, 1, yb);
#pragma unroll
        for (int s = 0; s < S; ++s) read_a(base, 1, s, ya[s]);
#pragma unroll
        for (int s = 0; s < S; ++s) products(s, xa[s], xb);
      }
#pragma unroll
      for (int s = 0; s < S; ++s) products_t(s, 0, SR - DT, ya[s], yb);
      // this wave's reads of stage k are complete before any wave may
      // overwrite it; its own DMA of stage k + 1 has landed
      wait_lgkm0();
      wait_vm<0>();
      lds_barrier();
      __builtin_amdgcn_sched_barrier(0);
      if (k + 2 < nsteps) issue(k + 2);
      // (the reads of the next stage are unconditional: after the last step
      // they re-read a stage that no DMA writes any more, and the values go
      // unused; a branch here would stretch the fragments' live ranges over
      // both paths)
      const int8_t* next = sm + ((k + 1) & 1) * STAGE;
      if constexpr (PF == 3) {
        // order pinned: the rho fragments whose registers are already free,
        // then after the deferred products of each G digit that digit's next
        // fragments (into the registers just freed), the rest of rho last
        read_b_t(next, 0, 0, SR - DT, xb);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          __builtin_amdgcn_sched_barrier(0);
          products_t(s, SR - DT, SR, ya[s], yb);
          __builtin_amdgcn_sched_barrier(0);
          read_a(next, 0, s, xa[s]);
        }
        read_b_t(next, 0, SR - DT, SR, xb);
        __builtin_amdgcn_sched_barrier(0);
      } else {
        read_b(next, 0, xb);
#pragma unroll
        for (int s = 0; s < S; ++s) read_a(next, 0, s, xa[s]);
#pragma unroll
        for (int s = 0; s < S; ++s) products_t(s, SR - DT, SR, ya[s], yb);
      }
    }
  } else {
    // Every step issues one DMA group; past the last k step the group re-loads
    // the last step into the stage freed one step earlier (never read again),
    // so the number of groups in flight after group k is always NST-2.
#pragma unroll
    for (int p = 0; p < NST - 1; ++p) issue(min(p, nsteps - 1));

    for (int k = 0; k < nsteps; ++k) {
      wait_vm<(NST - 2) * L>();
      lds_barrier();
      // (an explicit branch, not min(): it keeps the DMA issue in its own
      // scheduling region, away from the matrix-core block)
      if (k + NST - 1 < nsteps)
        issue(k + NST - 1);
      else
        issue(nsteps - 1);

      const int8_t* base = sm + (k % NST) * STAGE;
#pragma unroll
      for (int h = 0; h < BK / 64; ++h) {
        v4i fb[SR][4];
        read_b(base, h, fb);
        if constexpr (PF != 0) {
          // all fragments of this k half first: the reads complete in order,
          // so the matrix-core work of digit s waits only for its own reads
          v4i fa[S][2];
#pragma unroll
          for (int s = 0; s < S; ++s) read_a(base, h, s, fa[s]);
          // keep the scheduler from sinking the reads back between the products
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int s = 0; s < S; ++s) products(s, fa[s], fb);
        } else {
#pragma unroll
          for (int s = 0; s < S; ++s) {
            v4i fa[2];
            read_a(base, h, s, fa);
            products(s, fa, fb);
          }
        }
      }
    }
  }

  if constexpr (KIND == 1) {
    // bfloat16 parts: leading and correction sums combined in FP64
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + wn * 64 + j * 16 + (lane & 15);
        if (n >= a.nrhs) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
          if (m >= a.n) continue;
          const double sum = (double)acc[0][i][j][r] + (double)acc[1][i][j][r];
          if (a.ksplit > 1) {
            partf[((int64_t)z * a.nrhs + n) * a.n + m] = sum;
          } else {
            double v = a.c * sum;
            if (a.w) v += a.w[m];
            a.U[(int64_t)n * a.ldu + m] = v;
          }
        }
      }
    return;
  }

  if (a.ksplit > 1) {
    // raw class sums of this split, rows m fastest
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + wn * 64 + j * 16 + (lane & 15);
        if (n >= a.nrhs) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
          if (m >= a.n) continue;
#pragma unroll
          for (int c = 0; c < C; ++c)
            a.part[(((int64_t)z * C + c) * a.Rpad + n) * prow + (m - a.mt0 * BM)] = acc[c][i][j][r];
        }
      }
    return;
  }

  // exact recombination and the single scaling; the exponents, lift values
  // and output columns of this lane's 8 rows and 4 columns are loaded before
  // the first store (loads and stores share one in-order counter, so a load
  // after a store would wait for the store)
  int erow[2][4], ecol[4];
  double wrow[2][4];
  double* ucol[4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
      erow[i][r] = (m < a.n && a.row_exp) ? a.row_exp[m] : 0;
      wrow[i][r] = (m < a.n && a.w) ? a.w[m] : 0.0;
    }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn * 64 + j * 16 + (lane & 15);
    const bool in = n < a.nrhs;
    ecol[j] = in ? a.col_exp[n] : 0;
    ucol[j] = !in ? nullptr : a.ucols ? a.ucols[n] : a.U + (int64_t)n * a.ldu;
  }
  __builtin_amdgcn_s_waitcnt(0);
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + (lane & 15);
      if (n >= a.nrhs) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (m >= a.n) continue;
        int64_t v = acc[0][i][j][r];
#pragma unroll
        for (int c = 1; c < C; ++c) v = v * 256 + (int64_t)acc[c][i][j][r];
        const double scale = ldexp(a.c, erow[i][r] + ecol[j]);
        double u = (double)v * scale;
        if (a.w) u = u + wrow[i][r];
        ucol[j][m] = u;
      }
    }
  }
}

// Split-K epilogue: one thread per output (rows fastest); the splits' class
// sums are added exactly in int64, then recombined and scaled as in the GEMM
// epilogue (same operations, so the result is bit-identical).
// Rows m0 .. m0 + rows - 1 of the output, partial sums with row stride prow.
__global__ __launch_bounds__(256) void gemm_i8_splitk_epilogue(GemmI8Args a, int C, int m0, int rows, int64_t prow) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)rows * a.nrhs) return;
  const int mr = (int)(idx % rows), n = (int)(idx / rows);
  const int m = m0 + mr;
  int64_t cls[5] = {0, 0, 0, 0, 0};
  for (int z = 0; z < a.ksplit; ++z)
    for (int c = 0; c < C; ++c) cls[c] += a.part[(((int64_t)z * C + c) * a.Rpad + n) * prow + mr];
  int64_t v = cls[0];
  for (int c = 1; c < C; ++c) v = v * 256 + cls[c];
  const int em = a.row_exp ? a.row_exp[m] : 0;
  const double scale = ldexp(a.c, em + a.col_exp[n]);
  double u = (double)v * scale;
  if (a.w) u = u + a.w[m];
  double* ucol = a.ucols ? a.ucols[n] : a.U + (int64_t)n * a.ldu;
  ucol[m] = u;
}

// One wave per SIMD: 256-thread workgroups of 4 waves in 2 x 2, tile 128 rows x
// 128 right-hand sides, each wave 64 x 64 per class (4 x 4 blocks of 16 x 16).
// A wave then reads 4 S + 4 SR fragments per 64 bytes of k for 16 S SR
// products (against 2 S + 4 SR for 8 S SR at 32 x 64), so the LDS reads per
// product drop by a third.  The C = S + SR - 1 <= 4 class accumulators (64 C
// registers per lane, up to the whole accumulation register file) are
// operands of inline-asm products, which read and write each accumulator in
// place: compiled builtins at this register count copied accumulators between
// the two register files on every iteration.
//
// Schedule of 128-byte k step k (two LDS stages, k in one, k + 1 in the other):
// the fragments of the next k half are read into a second register set in the
// first RW products of each half.  In the first half, once this wave's reads
// of stage k are complete, a barrier frees stage k's buffer, and the DMA of
// stage k + 2 into it starts right away: N0 instructions over the rest of the
// first half, the others over the second half.  The middle of the step waits
// for stage k + 1 (issued one step earlier; the N0 newest instructions may
// still be in flight) and a barrier makes it visible.  The DMA is thus spread
// over about 160 of the step's 192 products (a DMA instruction holds up its
// wave's issue for tens of cycles while the operand stream is busy, so
// bunching the 20 instructions into one half leaves the matrix cores idle).
template <int S, int SR>
struct W4 {
  static constexpr int C = S + SR - 1;
  static constexpr int BK = 128;                   // k bytes per stage
  static constexpr int PLANE = 128 * BK;           // bytes of one operand plane per stage
  static constexpr int STAGE = (S + SR) * PLANE;
  static constexpr int IPP = 4;                    // DMA instructions per plane per wave (32 rows)
  static constexpr int NDMA = (S + SR) * IPP;      // DMA instructions per wave per stage
  static constexpr int M = S * SR * 16;            // products per wave per k half
  static constexpr int R = 4 * (S + SR);           // fragment reads per wave per k half
  static constexpr int RW = R < M / 2 ? R : M / 2; // the reads go into the first RW products
  static constexpr int PB = RW + 8 < M - 8 ? RW + 8 : M - 8;  // barrier after product PB of the first half
  static constexpr int N0 = NDMA * (M - 1 - PB) / (2 * M - 1 - PB);  // DMA instructions in the first half
  static constexpr bool ok = C <= 4 && 2 * STAGE <= LDS_BYTES;
};

// One 16-byte-per-lane DMA into LDS through a buffer resource made for the
// plane (nrec bytes from base): lane offset voff, scalar k offset soff, and the
// LDS row block of instruction j (0 .. 3) as the immediate offset 1024 j (it
// applies to both addresses, so voff has it taken off).
__device__ __forceinline__ void dma_plane(const int8_t* base, int nrec, int8_t* lds, uint32_t voff, int soff, int j) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, nrec, 0x00020000);
  switch (j) {  // (the immediate offset must be a constant)
    case 0: __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, PINV_LDS(lds), 16, voff, soff, 0, 0); break;
    case 1: __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, PINV_LDS(lds), 16, voff, soff, 1024, 0); break;
    case 2: __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, PINV_LDS(lds), 16, voff, soff, 2048, 0); break;
    default: __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, PINV_LDS(lds), 16, voff, soff, 3072, 0); break;
  }
}

// the product acc += fa * fb on the matrix cores, accumulator in place
__device__ inline void mfma_i8_acc(v4i& acc, const v4i& fa, const v4i& fb) {
  asm volatile("v_mfma_i32_16x16x64_i8 %0, %1, %2, %0" : "+a"(acc) : "v"(fa), "v"(fb));
}

template <int S, int SR, int MAP>
__global__ __launch_bounds__(256, 1) void gemm_i8_w4_kernel(GemmI8Args a_in, int tilesM, int tilesN,
                                                            const GemmI8Group* __restrict__ groups, int ngroups,
                                                            int total) {
  using K = W4<S, SR>;
  static_assert(K::ok, "one-wave-per-SIMD form: at most 4 classes and two stages in LDS");
  constexpr int C = K::C, BK = K::BK, PLANE = K::PLANE, STAGE = K::STAGE, IPP = K::IPP;
  constexpr int M = K::M, R = K::R, NDMA = K::NDMA;
  __shared__ __attribute__((aligned(1024))) int8_t sm[2 * STAGE];

  GemmI8Args a = a_in;
  int tN = tilesN;
  const int T = groups ? total : tilesM * tilesN;
  int tile = tile_index<MAP>(blockIdx.x, T);
  if (tile >= T) return;
  if (groups) {
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (groups[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    a = groups[lo].a;
    tN = groups[lo].tilesN;
    tile -= groups[lo].tile0;
  }
  const int mt = tile / tN, nt = tile % tN;
  const int m0 = (a.mt0 + mt) * 128, n0 = nt * 128;
  const int64_t prow = (int64_t)tilesM * 128;  // rows of the split-K partial sums
  const int64_t P = a.P;
  const int64_t KBY = a.kbytes ? a.kbytes : P;
  const int z = blockIdx.y;
  const int kfirst = a.ksplit > 1 ? z * (a.kchunk / BK) : 0;
  const int nsteps = a.ksplit > 1 ? (int)(min(KBY, (int64_t)(z + 1) * a.kchunk) / BK) - kfirst : (int)(KBY / BK);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;

  // DMA: instruction j of wave w fills rows w*32 + j*8 .. + 7 of every plane;
  // lane l lands at row l / 8, chunk position l % 8 of that block and loads
  // the logical chunk that the swizzle puts there (the swizzle is an involution)
  uint32_t off[IPP];
#pragma unroll
  for (int j = 0; j < IPP; ++j) {
    const int row = wave * 32 + j * 8 + lane / 8;
    off[j] = (uint32_t)row * (uint32_t)KBY + (uint32_t)(swz<8>(row, lane % 8) * 16);
  }
  const int8_t* tileA = a.Q + (int64_t)m0 * KBY;
  const int8_t* tileB = a.X + (int64_t)n0 * KBY;
  const int64_t planeA = P * KBY, planeB = (int64_t)a.Rpad * KBY;
  // The LDS row block of DMA instruction j is its immediate offset 1024 j
  // (applied to both addresses, so the row offsets drop it), and the 4
  // instructions of a plane share one LDS base; the global address is a
  // scalar base (plane, tile, k) plus the lane's 32-bit row offset.  DMA
  // instruction d (0 .. NDMA-1) of stage `step`: plane d / IPP, row block
  // d % IPP.
#pragma unroll
  for (int j = 0; j < IPP; ++j) off[j] -= (uint32_t)(j * 1024);
  auto dma = [&](int step, int d) {
    const int p = d / IPP, j = d % IPP;
    const int k0 = __builtin_amdgcn_readfirstlane((kfirst + step) * BK);
    const int8_t* base = p < S ? tileA + p * planeA : tileB + (p - S) * planeB;
    dma_plane(base, (int)(128 * KBY), sm + (step & 1) * STAGE + p * PLANE + wave * 32 * BK, off[j], k0, j);
  };

  // fragment read offsets within a plane for k half h: row lane % 16 of the
  // 16-row block (block bases are multiples of 16 rows, where the swizzle's
  // row term is zero), logical chunk 4h + lane / 16
  const int frow = lane & 15;
  const int foff0 = frow * BK + swz<8>(frow, lane >> 4) * 16;
  const int foff1 = frow * BK + swz<8>(frow, 4 + (lane >> 4)) * 16;
  const int aoff = (wm * 64) * BK, boff = S * PLANE + (wn * 64) * BK;

  v4i acc[C][4][4];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[c][i][j] = v4i{0, 0, 0, 0};

  v4i fa0[S][4], fb0[SR][4], fa1[S][4], fb1[SR][4];

  // read r (0 .. R-1) of a k half into (fa, fb): G digit r / 4 block r % 4
  // for r < 4S, else rho digit (r - 4S) / 4 block (r - 4S) % 4
  auto read = [&](const int8_t* base, int foff, int r, v4i (&fa)[S][4], v4i (&fb)[SR][4]) {
    if (r < 4 * S) {
      fa[r / 4][r % 4] = *(const v4i*)(base + (r / 4) * PLANE + aoff + (r % 4) * 16 * BK + foff);
    } else {
      const int q = r - 4 * S;
      fb[q / 4][q % 4] = *(const v4i*)(base + (q / 4) * PLANE + boff + (q % 4) * 16 * BK + foff);
    }
  };

  constexpr int RW = K::RW, PB = K::PB, N0 = K::N0;

  // one k half: the M products of (fa, fb), with the R reads of the next half
  // into (na, nb) in the first RW products; in the first half (FIRST) the wait
  // for those reads and the barrier that frees the stage after product PB; ND
  // DMA instructions D0 .. D0 + ND - 1 of stage dstep spread over the products
  // after the barrier (first half) or over all of them (second half)
  auto half = [&](const v4i (&fa)[S][4], const v4i (&fb)[SR][4], const int8_t* nbase, int nfoff, v4i (&na)[S][4],
                  v4i (&nb)[SR][4], int dstep, auto first, auto nd, auto d0) {
    constexpr bool FIRST = decltype(first)::value;
    constexpr int ND = decltype(nd)::value, D0 = decltype(d0)::value;
    constexpr int Q0 = FIRST ? PB + 1 : 0, W = M - Q0;
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const int s = q / (SR * 16), t = (q / 16) % SR, i = (q / 4) % 4, j = q % 4;
      mfma_i8_acc(acc[s + t][i][j], fa[s][i], fb[t][j]);
      if (q < RW) {
#pragma unroll
        for (int r = (q * R + RW - 1) / RW; r < ((q + 1) * R + RW - 1) / RW; ++r) read(nbase, nfoff, r, na, nb);
      }
      if constexpr (FIRST) {
        if (q == PB) {
          wait_lgkm0();
          lds_barrier();
        }
      }
      if constexpr (ND > 0) {
        if (q >= Q0) {
          const int qq = q - Q0;
#pragma unroll
          for (int d = (qq * ND + W - 1) / W; d < ((qq + 1) * ND + W - 1) / W; ++d) dma(dstep, D0 + d);
        }
      }
    }
  };

  using DmaOn = std::true_type;
  using DmaOff = std::false_type;

  // prologue: stages 0 and 1 in flight, wait for stage 0, read its first half
#pragma unroll
  for (int d = 0; d < NDMA; ++d) dma(0, d);
  if (nsteps > 1) {
#pragma unroll
    for (int d = 0; d < NDMA; ++d) dma(1, d);
    wait_vm<NDMA>();
  } else {
    wait_vm<0>();
  }
  lds_barrier();
#pragma unroll
  for (int r = 0; r < R; ++r) read(sm, foff0, r, fa0, fb0);

  // step k: half 0 (reads of stage k's half 1, barrier, DMA of stage k + 2
  // begins); this wave's DMA of stage k + 1 has landed, barrier; half 1 (rest
  // of the DMA of stage k + 2, reads of stage k + 1's half 0).  Without DMA
  // (the last two steps) the wait is for everything.
  auto step = [&](int k, auto on) {
    constexpr bool ON = decltype(on)::value;
    using I = std::integral_constant<int, 0>;
    using N0c = std::integral_constant<int, ON ? N0 : 0>;
    using N1c = std::integral_constant<int, ON ? NDMA - N0 : 0>;
    using D1c = std::integral_constant<int, N0>;
    const int8_t* cur = sm + (k & 1) * STAGE;
    const int8_t* nxt = sm + ((k + 1) & 1) * STAGE;
    half(fa0, fb0, cur, foff1, fa1, fb1, k + 2, std::true_type{}, N0c{}, I{});
    wait_lgkm0();
    if constexpr (ON) wait_vm<N0>(); else wait_vm<0>();
    lds_barrier();
    half(fa1, fb1, nxt, foff0, fa0, fb0, k + 2, std::false_type{}, N1c{}, D1c{});
  };
  int k = 0;
  for (; k + 2 < nsteps; ++k) step(k, DmaOn{});
  for (; k < nsteps; ++k) step(k, DmaOff{});
  // (the last step's reads of "stage k + 1" re-read a released buffer; the
  // values go unused)
  wait_lgkm0();
  // the accumulators are read below by ordinary instructions: let the last
  // products retire first (the hazard checks do not see inside inline asm)
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");

  if (a.ksplit > 1) {
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
#pragma unroll
          for (int c = 0; c < C; ++c)
            a.part[(((int64_t)z * C + c) * a.Rpad + n) * prow + (m - a.mt0 * 128)] = acc[c][i][j][r];
        }
      }
    return;
  }

  // the exponents of this lane's 16 rows and 4 columns are loaded before the
  // first store (loads and stores share one in-order counter, so a load
  // after a store would wait for the store)
  int erow[4][4], ecol[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
      erow[i][r] = (m < a.n && a.row_exp) ? a.row_exp[m] : 0;
    }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn * 64 + j * 16 + (lane & 15);
    ecol[j] = n < a.nrhs ? a.col_exp[n] : 0;
  }
  // (one wait for all of them here, so none is left for the compiler to place
  // among the stores)
  __builtin_amdgcn_s_waitcnt(0);
  asm volatile("" ::: "memory");
  if (!a.ucols && !a.w) {
    // output columns at a fixed stride, no lift: no loads among the stores
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + wn * 64 + j * 16 + (lane & 15);
        if (n >= a.nrhs) continue;
        double* ucol = a.U + (int64_t)n * a.ldu;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
          if (m >= a.n) continue;
          int64_t v = acc[0][i][j][r];
#pragma unroll
          for (int c = 1; c < C; ++c) v = v * 256 + (int64_t)acc[c][i][j][r];
          const double scale = ldexp(a.c, erow[i][r] + ecol[j]);
          ucol[m] = (double)v * scale;
        }
      }
    }
    return;
  }
  // with a lift or a table of output columns, those are loaded first too
  double wrow[4][4];
  double* ucol[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
      wrow[i][r] = (m < a.n && a.w) ? a.w[m] : 0.0;
    }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn * 64 + j * 16 + (lane & 15);
    ucol[j] = n >= a.nrhs ? nullptr : a.ucols ? a.ucols[n] : a.U + (int64_t)n * a.ldu;
  }
  __builtin_amdgcn_s_waitcnt(0);
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + (lane & 15);
      if (n >= a.nrhs) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        if (m >= a.n) continue;
        int64_t v = acc[0][i][j][r];
#pragma unroll
        for (int c = 1; c < C; ++c) v = v * 256 + (int64_t)acc[c][i][j][r];
        const double scale = ldexp(a.c, erow[i][r] + ecol[j]);
        double u = (double)v * scale;
        if (a.w) u = u + wrow[i][r];
        ucol[j][m] = u;
      }
    }
  }
}

// Variants 0-7 (8-wave workgroups, 128 x 128 tiles, one per compute unit):
// BK = 128 if v % 2 == 0 (falls back to 64 when two 128-byte stages do not
// fit), else 64; MAP = (v / 2) % 2; PF = v / 4 (fragment reads per digit, or all
// up front).  Variants 8-9: split-step pipeline (PF = 2, BK = 128 where two
// such stages fit, else as variant 4), MAP = v - 8.  Variants 10-11: 4-wave
// workgroups with 64 x 128 tiles, two per compute unit (their barriers are
// independent, so one workgroup's waits are covered by the other's products),
// all fragments up front, BK = 128 where two stages fit in half the LDS, else
// 64; MAP = v - 10.  Variant 12: the split-step pipeline with its instruction
// order pinned (PF = 3), XCD order.
template <int S, int SR>
constexpr int bk_of(int v) {
  if (v == 12) return 2 * (S + SR) * 128 * 128 <= LDS_BYTES ? 128 : 64;
  if (v >= 10) return 2 * ((S * 64 + SR * 128) * 128) <= LDS_BYTES / 2 ? 128 : 64;
  return ((v >= 8 || v % 2 == 0) && 2 * (S + SR) * 128 * 128 <= LDS_BYTES) ? 128 : 64;
}

template <int S, int SR, int V>
hipError_t launch_v(const GemmI8Args& a, const GemmI8Group* groups, int ngroups, int total, hipStream_t s);

// Variants 13-14: one wave per SIMD (gemm_i8_w4_kernel), MAP = v - 13; where
// it does not apply (more than 4 classes) they run variants 8-9 instead.
template <int S, int SR, int V>
hipError_t launch_w4(const GemmI8Args& a, const GemmI8Group* groups, int ngroups, int total, hipStream_t s) {
  if constexpr (!W4<S, SR>::ok) {
    return launch_v<S, SR, V - 5>(a, groups, ngroups, total, s);
  } else {
    constexpr int MAP = V - 13;
    const int tilesM = groups ? 0 : (a.mtiles ? a.mtiles : (int)(a.P / 128) - a.mt0), tilesN = groups ? 0 : a.Rpad / BN;
    const int T = groups ? total : tilesM * tilesN;
    const int grid = MAP == 0 ? ((T + 7) / 8) * 8 : T;
    const int zs = (!groups && a.ksplit > 1) ? a.ksplit : 1;
    hipLaunchKernelGGL((gemm_i8_w4_kernel<S, SR, MAP>), dim3(grid, zs), dim3(256), 0, s, a, tilesM, tilesN, groups,
                       ngroups, total);
    return hipGetLastError();
  }
}

template <int S, int SR, int V>
hipError_t launch_v(const GemmI8Args& a, const GemmI8Group* groups, int ngroups, int total, hipStream_t s) {
  constexpr int NWV = (V == 10 || V == 11) ? 4 : 8;
  constexpr int BKV = bk_of<S, SR>(V);
  constexpr int MAP = V == 12 ? 0 : V >= 10 ? V - 10 : V >= 8 ? V - 8 : (V / 2) % 2;
  constexpr int PF = V == 12 ? 3 : V >= 10 ? 1 : V >= 8 ? 2 : V / 4;
  using K = Cfg<S, SR, BKV, NWV>;
  const int tilesM = groups ? 0 : (a.mtiles ? a.mtiles : (int)(a.P / K::BM) - a.mt0), tilesN = groups ? 0 : a.Rpad / BN;
  const int T = groups ? total : tilesM * tilesN;
  const int grid = MAP == 0 ? ((T + 7) / 8) * 8 : T;
  const int zs = (!groups && a.ksplit > 1) ? a.ksplit : 1;
  hipLaunchKernelGGL((gemm_i8_kernel<S, SR, BKV, MAP, PF, NWV>), dim3(grid, zs), dim3(K::NT), 0, s, a, tilesM, tilesN,
                     groups, ngroups, total, (double*)nullptr);
  return hipGetLastError();
}

template <int S, int SR>
hipError_t launch_t(const GemmI8Args& a, int variant, const GemmI8Group* g, int ng, int tot, hipStream_t s) {
  switch (variant) {
    case 1: return launch_v<S, SR, 1>(a, g, ng, tot, s);
    case 2: return launch_v<S, SR, 2>(a, g, ng, tot, s);
    case 3: return launch_v<S, SR, 3>(a, g, ng, tot, s);
    case 4: return launch_v<S, SR, 4>(a, g, ng, tot, s);
    case 5: return launch_v<S, SR, 5>(a, g, ng, tot, s);
    case 6: return launch_v<S, SR, 6>(a, g, ng, tot, s);
    case 7: return launch_v<S, SR, 7>(a, g, ng, tot, s);
    case 8: return launch_v<S, SR, 8>(a, g, ng, tot, s);
    case 9: return launch_v<S, SR, 9>(a, g, ng, tot, s);
    case 10: return launch_v<S, SR, 10>(a, g, ng, tot, s);
    case 11: return launch_v<S, SR, 11>(a, g, ng, tot, s);
    case 12: return launch_v<S, SR, 12>(a, g, ng, tot, s);
    case 13: return launch_w4<S, SR, 13>(a, g, ng, tot, s);
    case 14: return launch_w4<S, SR, 14>(a, g, ng, tot, s);
    default: return launch_v<S, SR, 0>(a, g, ng, tot, s);
  }
}

hipError_t dispatch(int S, int SR, const GemmI8Args& a, int variant, const GemmI8Group* g, int ng, int tot,
                    hipStream_t s) {
  switch (S * 4 + SR) {
    case 1 * 4 + 1: return launch_t<1, 1>(a, variant, g, ng, tot, s);
    case 1 * 4 + 2: return launch_t<1, 2>(a, variant, g, ng, tot, s);
    case 1 * 4 + 3: return launch_t<1, 3>(a, variant, g, ng, tot, s);
    case 2 * 4 + 1: return launch_t<2, 1>(a, variant, g, ng, tot, s);
    case 2 * 4 + 2: return launch_t<2, 2>(a, variant, g, ng, tot, s);
    case 2 * 4 + 3: return launch_t<2, 3>(a, variant, g, ng, tot, s);
    case 3 * 4 + 1: return launch_t<3, 1>(a, variant, g, ng, tot, s);
    case 3 * 4 + 2: return launch_t<3, 2>(a, variant, g, ng, tot, s);
    case 3 * 4 + 3: return launch_t<3, 3>(a, variant, g, ng, tot, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int gemm_i8_variants() { return 15; }

int gemm_i8_tile_rows(int variant) { return (variant == 10 || variant == 11) ? 64 : 128; }

namespace {

// k split into z parts of whole 128-byte steps
void split_k(int64_t P, int z, int* ksplit, int* kchunk) {
  int64_t chunk = (P + z - 1) / z;
  chunk = (chunk + 127) / 128 * 128;
  *ksplit = (int)((P + chunk - 1) / chunk);
  *kchunk = (int)chunk;
}

}  // namespace

void gemm_i8_split_plan(int64_t P, int Rpad, int variant, int* ksplit, int* kchunk, int* tail_rows) {
  // W workgroups are resident at once.  With fewer tiles than that (T < W),
  // every tile splits k: z = min(W / T, 4).  With more, the tiles run in
  // rounds of W; when the last round is at most half full, only its row tiles
  // split (z = min(W / tail tiles, 4)), so that it takes about 1/z of a
  // round instead of a whole one.  At least 2048 of k per split.  (A last
  // round more than half full is not split: splitting it measured no gain, the
  // product being limited by the operand stream into LDS rather than by idle
  // units.)
  const int rows = gemm_i8_tile_rows(variant);
  const int tM = (int)(P / rows), tN = Rpad / BN;
  const int T = tM * tN;
  const int W = rows == 128 ? 256 : 512;
  *ksplit = 1;
  *kchunk = (int)P;
  *tail_rows = 0;
  if (T <= 0) return;
  int zz = 1, trows = 0;
  if (T < W) {
    zz = W / T;
  } else if (T % W != 0 && T % W <= W / 2) {
    const int main_rows = (T / W) * W / tN;  // row tiles of the whole rounds
    trows = tM - main_rows;
    zz = W / (trows * tN);
  }
  if (zz > 4) zz = 4;
  while (zz > 1 && P / zz < 2048) --zz;
  if (zz < 2) return;
  split_k(P, zz, ksplit, kchunk);
  *tail_rows = trows;
}

size_t gemm_i8_part_bytes(int64_t P, int Rpad, int variant, int C, int ksplit, int tail_rows) {
  if (ksplit <= 1) return 0;
  const int64_t rows = tail_rows > 0 ? (int64_t)tail_rows * gemm_i8_tile_rows(variant) : P;
  return (size_t)ksplit * C * Rpad * rows * sizeof(int32_t);
}

hipError_t launch_gemm_i8(const GemmI8Args& a_in, hipStream_t s) {
  if (a_in.nrhs <= 0) return hipSuccess;
  if (a_in.P % 256 != 0 || a_in.Rpad % BN != 0) return hipErrorInvalidValue;  // tiles cover P and Rpad exactly
  const bool split = a_in.ksplit > 1;
  if (split && (!a_in.part || a_in.kchunk <= 0 || a_in.kchunk % 128 != 0 ||
                (int64_t)a_in.kchunk * (a_in.ksplit - 1) >= a_in.P))
    return hipErrorInvalidValue;
  const int rows = gemm_i8_tile_rows(a_in.variant);
  const int tM = (int)(a_in.P / rows);
  if (a_in.tail_rows < 0 || a_in.tail_rows >= tM) return hipErrorInvalidValue;
  GemmI8Args a = a_in;
  a.mt0 = 0;
  a.mtiles = 0;
  hipError_t e;
  if (split && a_in.tail_rows > 0) {
    // the whole rounds unsplit, then the last row tiles split
    GemmI8Args m = a;
    m.ksplit = 1;
    m.kchunk = (int)a.P;
    m.part = nullptr;
    m.mtiles = tM - a_in.tail_rows;
    e = dispatch(m.S, m.SR, m, m.variant, nullptr, 0, 0, s);
    if (e != hipSuccess) return e;
    a.mt0 = tM - a_in.tail_rows;
    a.mtiles = a_in.tail_rows;
  }
  e = dispatch(a.S, a.SR, a, a.variant, nullptr, 0, 0, s);
  if (e != hipSuccess || !split) return e;
  const int m0 = a.mt0 * rows;
  const int64_t prow = (int64_t)(tM - a.mt0) * rows;
  const int out_rows = a.n - m0;
  if (out_rows <= 0) return hipSuccess;
  const int64_t outs = (int64_t)out_rows * a.nrhs;
  hipLaunchKernelGGL(gemm_i8_splitk_epilogue, dim3((unsigned)((outs + 255) / 256)), dim3(256), 0, s, a,
                     a.S + a.SR - 1, m0, out_rows, prow);
  return hipGetLastError();
}

hipError_t launch_gemm_i8_grouped(const GemmI8Group* d_groups, int ngroups, int total_tiles, int S, int SR,
                                  int variant, hipStream_t s) {
  if (ngroups <= 0 || total_tiles <= 0) return hipSuccess;
  if (!d_groups || variant < 0 || variant >= gemm_i8_variants()) return hipErrorInvalidValue;
  GemmI8Args none{};
  return dispatch(S, SR, none, variant, d_groups, ngroups, total_tiles, s);
}

hipError_t launch_gemm_bf16_parts(const GemmI8Args& a, double* partf, hipStream_t s) {
  if (a.nrhs <= 0) return hipSuccess;
  if (a.P % 256 != 0 || a.Rpad % BN != 0 || a.kbytes != 2 * a.P || a.S != a.SR) return hipErrorInvalidValue;
  const bool split = a.ksplit > 1;
  if (split && (!partf || a.kchunk <= 0 || a.kchunk % 128 != 0 || (int64_t)a.kchunk * (a.ksplit - 1) >= a.kbytes))
    return hipErrorInvalidValue;
  // 8-wave 128 x 128 tiles, all fragments of a k half read up front, XCD order;
  // 128-byte k steps where two stages fit, else 64
  const int tilesM = (int)(a.P / 128), tilesN = a.Rpad / BN;
  const int T = tilesM * tilesN;
  const dim3 grid(((T + 7) / 8) * 8, split ? a.ksplit : 1);
  switch (a.S) {
    case 2:
      hipLaunchKernelGGL((gemm_i8_kernel<2, 2, 128, 0, 1, 8, 1>), grid, dim3(512), 0, s, a, tilesM, tilesN,
                         (const GemmI8Group*)nullptr, 0, 0, partf);
      break;
    case 3:
      hipLaunchKernelGGL((gemm_i8_kernel<3, 3, 64, 0, 1, 8, 1>), grid, dim3(512), 0, s, a, tilesM, tilesN,
                         (const GemmI8Group*)nullptr, 0, 0, partf);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
