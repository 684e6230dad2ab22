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
// class (128 accumulator registers per wave).
// Operand tiles move global -> LDS with global_load_lds_dwordx4 (no staging
// registers): one instruction fills 1 KB of LDS (one block of rows) per wave.
// LDS rows are unpadded; the four 16-byte chunks of row r are stored at chunk
// position c ^ ((r >> 2) & 3), so the 16 lanes of a 128-bit fragment read
// (16 consecutive rows, same logical chunk) hit 16 distinct 4-bank groups.  A
// lane of the DMA loads the global chunk that belongs at its own LDS slot.
// NST LDS stages (4 when they fit in the 160 KB of a CU, else 3) keep NST-1 k
// steps of loads in flight.  Each wave waits for its own DMA group (vmcnt),
// then a plain s_barrier (no fence: a fence would drain all in-flight stages)
// makes the stage visible to all waves and frees the stage read one step
// earlier.
// The digit planes and quantised right-hand sides are zero-padded to the tile
// grid, so the main loop has no bounds checks.
//
// v_mfma_i32_16x16x64_i8 layout (lane l, result register r):
//   A(i = l%16, k = 16*(l/16) + b), B(k = 16*(l/16) + b, j = l%16),
//   D(i = 4*(l/16) + r, j = l%16).

#include "common.h"

#define PINV_LDS(p) ((__attribute__((address_space(3))) void*)(p))

namespace {

constexpr int BM = 128, BN = 128;
constexpr int NW = 8;                 // waves per workgroup (two per SIMD)
constexpr int NT = NW * 64;
constexpr int LDS_BYTES = 163840;

template <int MAP>
__device__ inline void tile_of(int bid, int tilesM, int tilesN, int& mt, int& nt, bool& valid) {
  const int T = tilesM * tilesN;
  const int per = (T + 7) / 8;
  const int tile = MAP == 0 ? (bid % 8) * per + bid / 8 : bid;
  valid = tile < T;
  mt = valid ? tile / tilesN : 0;
  nt = valid ? tile % tilesN : 0;
}

// s_waitcnt with only the vector-memory counter constrained (<= V)
template <int V>
__device__ inline void wait_vm() {
  static_assert(V >= 0 && V < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((V & 15) | (((V >> 4) & 3) << 14) | (7 << 4) | (15 << 8));
}

__device__ inline void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }

// Kernel variants (picked per operator by pinv_autotune_int8): BK = k bytes
// per stage, 128 (full 128-byte cache lines per row, two stages) or 64 (as many
// stages as fit, at most 4); MAP 0 = XCD-aware tile order, 1 = linear; PF =
// read all operand fragments of a k half before its matrix-core work.
template <int S, int SR, int BK_>
struct Cfg {
  static constexpr int C = S + SR - 1;
  static constexpr int BK = BK_;
  static constexpr int CH = BK / 16;                       // 16-byte chunks per row
  static constexpr int PLANE = 128 * BK;                   // bytes of one plane per stage
  static constexpr int STAGE = (S + SR) * PLANE;
  static constexpr int NST_ = LDS_BYTES / STAGE;
  static constexpr int NST = NST_ > 4 ? 4 : NST_;
  static constexpr int RPI = 1024 / BK;                    // rows filled by one DMA instruction
  static constexpr int RPW = 128 / NW;                     // rows of a plane filled by one wave
  static constexpr int IPP = RPW / RPI;                    // DMA instructions per plane per wave
  static constexpr int L = (S + SR) * IPP;                 // DMA instructions per thread per stage
  static_assert(NST >= 2, "two LDS stages must fit");
  static_assert(IPP >= 1, "a wave fills at least one DMA block per plane");
};

// Swizzle: the 16-byte chunk c of tile row r sits at chunk position
// c ^ ((r >> 1) & 7) (128-byte rows) or c ^ ((r >> 2) & 3) (64-byte rows), so
// each 16 lanes of a fragment read (16 consecutive rows, one chunk) hit 16
// distinct 4-bank groups.
template <int CH>
__device__ inline int swz(int row, int c) {
  return CH == 8 ? (c ^ ((row >> 1) & 7)) : (c ^ ((row >> 2) & 3));
}

template <int S, int SR, int BKV, int MAP, bool PF>
__global__ __launch_bounds__(NT, 1) void gemm_i8_kernel(GemmI8Args a, int tilesM, int tilesN) {
  using K = Cfg<S, SR, BKV>;
  constexpr int C = K::C, BK = K::BK, CH = K::CH, PLANE = K::PLANE, STAGE = K::STAGE, NST = K::NST;
  constexpr int RPI = K::RPI, RPW = K::RPW, IPP = K::IPP, L = K::L;
  __shared__ __attribute__((aligned(1024))) int8_t sm[NST * STAGE];

  int mt, nt;
  bool valid;
  tile_of<MAP>(blockIdx.x, tilesM, tilesN, mt, nt, valid);
  if (!valid) return;
  const int m0 = mt * BM, n0 = nt * BN;
  const int64_t P = a.P;
  const int nsteps = (int)(P / BK);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;     // 4 x 2 waves, each 32 rows x 64 right-hand sides

  // DMA: instruction j of wave w fills plane rows w*RPW + j*RPI .. + RPI-1; lane l
  // lands at LDS byte l*16 of that block = row l / CH, chunk position l % CH,
  // so it loads the logical chunk whose swizzled position is l % CH.  The
  // address is a wave-uniform plane base plus a 32-bit per-lane offset.
  uint32_t off[IPP];
#pragma unroll
  for (int j = 0; j < IPP; ++j) {
    const int row = wave * RPW + j * RPI + lane / CH;
    off[j] = (uint32_t)row * (uint32_t)P + (uint32_t)(swz<CH>(row, lane % CH) * 16);  // swizzle is an involution
  }
  const int8_t* tileA = a.Q + (int64_t)m0 * P;
  const int8_t* tileB = a.X + (int64_t)n0 * P;
  const int64_t planeA = P * P, planeB = (int64_t)a.Rpad * P;

  auto issue = [&](int step) {
    int8_t* dst = sm + (step % NST) * STAGE + wave * RPW * BK;
    const int64_t k0 = (int64_t)step * BK;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int8_t* b = tileA + s * planeA + k0;
#pragma unroll
      for (int j = 0; j < IPP; ++j)
        __builtin_amdgcn_global_load_lds((const void*)(b + off[j]), PINV_LDS(dst + s * PLANE + j * 1024), 16, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < SR; ++t) {
      const int8_t* b = tileB + t * planeB + k0;
#pragma unroll
      for (int j = 0; j < IPP; ++j)
        __builtin_amdgcn_global_load_lds((const void*)(b + off[j]), PINV_LDS(dst + (S + t) * PLANE + j * 1024), 16, 0, 0);
    }
  };

  // fragment read offsets (bytes within a plane) for k half h: rows
  // (16-row block base) + lane%16, logical chunk 4h + lane/16
  const int frow = lane & 15;
  int foff[BK / 64];
#pragma unroll
  for (int h = 0; h < BK / 64; ++h) foff[h] = frow * BK + swz<CH>(frow, 4 * h + (lane >> 4)) * 16;

  v4i acc[C][2][4];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[c][i][j] = v4i{0, 0, 0, 0};

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
      // 16-row blocks start at multiples of 16, where the swizzle of the block
      // base is zero, so one lane offset serves every block
      v4i fb[SR][4];
#pragma unroll
      for (int t = 0; t < SR; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          fb[t][j] = *(const v4i*)(base + (S + t) * PLANE + (wn * 64 + j * 16) * BK + foff[h]);
      if constexpr (PF) {
        // all fragments of this k half first: the reads complete in order, so
        // the matrix-core work of digit s waits only for its own reads
        v4i fa[S][2];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int i = 0; i < 2; ++i)
            fa[s][i] = *(const v4i*)(base + s * PLANE + (wm * 32 + i * 16) * BK + foff[h]);
        // keep the scheduler from sinking the reads back between the products
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int t = 0; t < SR; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                acc[s + t][i][j] =
                    __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[s][i], fb[t][j], acc[s + t][i][j], 0, 0, 0);
      } else {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          v4i fa[2];
#pragma unroll
          for (int i = 0; i < 2; ++i)
            fa[i] = *(const v4i*)(base + s * PLANE + (wm * 32 + i * 16) * BK + foff[h]);
#pragma unroll
          for (int t = 0; t < SR; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                acc[s + t][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[i], fb[t][j], acc[s + t][i][j], 0, 0, 0);
        }
      }
    }
  }

  // exact recombination and the single scaling
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + (lane & 15);
      if (n >= a.nrhs) continue;
      const int fn = a.col_exp[n];
      double* ucol = a.ucols ? a.ucols[n] : a.U + (int64_t)n * a.ldu;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (m >= a.n) continue;
        int64_t v = acc[0][i][j][r];
#pragma unroll
        for (int c = 1; c < C; ++c) v = v * 256 + (int64_t)acc[c][i][j][r];
        const int em = a.row_exp ? a.row_exp[m] : 0;
        const double scale = ldexp(a.c, em + fn);
        double u = (double)v * scale;
        if (a.w) u = u + a.w[m];
        ucol[m] = u;
      }
    }
  }
}

// variant v: BK = 128 if v % 2 == 0 (falls back to 64 when two 128-byte stages
// do not fit), else 64; MAP = (v / 2) % 2; PF = v >= 4
template <int S, int SR>
constexpr int bk_of(int v) {
  return (v % 2 == 0 && 2 * (S + SR) * 128 * 128 <= LDS_BYTES) ? 128 : 64;
}

template <int S, int SR, int V>
hipError_t launch_v(const GemmI8Args& a, hipStream_t s) {
  constexpr int BKV = bk_of<S, SR>(V);
  constexpr int MAP = (V / 2) % 2;
  constexpr bool PF = V >= 4;
  const int tilesM = (int)(a.P / BM), tilesN = a.Rpad / BN;
  const int T = tilesM * tilesN;
  const int grid = MAP == 0 ? ((T + 7) / 8) * 8 : T;
  hipLaunchKernelGGL((gemm_i8_kernel<S, SR, BKV, MAP, PF>), dim3(grid), dim3(NT), 0, s, a, tilesM, tilesN);
  return hipGetLastError();
}

template <int S, int SR>
hipError_t launch_t(const GemmI8Args& a, hipStream_t s) {
  switch (a.variant) {
    case 1: return launch_v<S, SR, 1>(a, s);
    case 2: return launch_v<S, SR, 2>(a, s);
    case 3: return launch_v<S, SR, 3>(a, s);
    case 4: return launch_v<S, SR, 4>(a, s);
    case 5: return launch_v<S, SR, 5>(a, s);
    case 6: return launch_v<S, SR, 6>(a, s);
    case 7: return launch_v<S, SR, 7>(a, s);
    default: return launch_v<S, SR, 0>(a, s);
  }
}

}  // namespace

int gemm_i8_variants() { return 8; }

hipError_t launch_gemm_i8(const GemmI8Args& a, hipStream_t s) {
  if (a.nrhs <= 0) return hipSuccess;
  if (a.P % 256 != 0 || a.Rpad % BN != 0) return hipErrorInvalidValue;
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
