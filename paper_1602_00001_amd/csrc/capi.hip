// C-ABI entry points of libpinv (declared in include/pinv.h): argument checks,
// ownership of device memory, and dispatch to the kernels.

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "common.h"

// ---------------------------------------------------------------------------
// helpers

int32_t pinv_hip_status(hipError_t e) {
  if (e == hipSuccess) return PINV_OK;
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return PINV_E_OOM;
  return PINV_E_HIP;
}

void pinv_log(const char* fmt, ...) {
  static const bool on = [] {
    const char* v = std::getenv("PINV_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  if (!on) return;
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "[pinv] ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
}

namespace {

struct TraceRec {
  const char* name;
  hipEvent_t a, b;
};
std::atomic<int> g_trace_on{0};
std::mutex g_trace_mu;
std::vector<TraceRec> g_trace;

}  // namespace

TraceScope::TraceScope(const char* name, hipStream_t s) : name_(name), s_(s) {
  if (!name || !g_trace_on.load(std::memory_order_relaxed)) return;
  if (hipEventCreate(&a_) != hipSuccess) return;
  if (hipEventCreate(&b_) != hipSuccess) {
    (void)hipEventDestroy(a_);
    return;
  }
  on_ = hipEventRecord(a_, s_) == hipSuccess;
  if (!on_) {
    (void)hipEventDestroy(a_);
    (void)hipEventDestroy(b_);
  }
}

TraceScope::~TraceScope() {
  if (!on_) return;
  if (hipEventRecord(b_, s_) != hipSuccess) {
    (void)hipEventDestroy(a_);
    (void)hipEventDestroy(b_);
    return;
  }
  std::lock_guard<std::mutex> lk(g_trace_mu);
  g_trace.push_back({name_, a_, b_});
}

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// The stream-ordered pool keeps freed scratch cached, so the per-call scratch
// of the apply (quantised right-hand sides) costs no device allocation after
// the first call of a given size.
void configure_pool_once() {
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  });
}

bool grid_ok(const pinv_grid* g) {
  if (!g) return false;
  if (g->nx < 3 || g->ny < 3) return false;
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return false;
  const int64_t n = (int64_t)(g->nx - 2) * (int64_t)(g->ny - 2);
  return n <= (int64_t)1 << 20;  // dense N x N inverse: 8 TB at this bound
}

pinv_op new_op(const pinv_grid* g) {
  pinv_op op = new (std::nothrow) pinv_op_s();
  if (!op) return nullptr;
  op->nx = g->nx;
  op->ny = g->ny;
  op->mx = g->nx - 2;
  op->my = g->ny - 2;
  op->n = op->mx * op->my;
  op->h = g->h;
  op->ldg = (op->n + 31) / 32 * 32;
  (void)hipGetDevice(&op->device);
  return op;
}

void purge_batch_plans(pinv_op op);

// Sets op->g_symmetric: whether G equals its transpose bit for bit (then the
// FP64 adjoint runs the forward product).  One pass over G; synchronises.
int32_t detect_symmetry(pinv_op op, hipStream_t s) {
  op->g_symmetric = 0;
  if (!op->G) return PINV_OK;
  int* flag = nullptr;
  PINV_HIP_TRY(hipMalloc(&flag, sizeof(int)));
  int hflag = 1;
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
  if (e == hipSuccess) e = launch_sym_check(op->G, op->ldg, op->n, 0.0, flag, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(flag);
  if (e != hipSuccess) return pinv_hip_status(e);
  op->g_symmetric = hflag == 0;
  return PINV_OK;
}

void free_quant(pinv_op op) {
  purge_batch_plans(op);  // batched plans hold the digit planes' addresses
  if (op->Q) (void)hipFree(op->Q);
  if (op->QT) (void)hipFree(op->QT);
  if (op->e) (void)hipFree(op->e);
  if (op->S) op->bytes -= 2 * (int64_t)op->S * op->P * op->P + op->P * (int64_t)sizeof(int32_t);
  op->Q = op->QT = nullptr;
  op->e = nullptr;
  op->S = 0;
}

void free_op(pinv_op op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  free_quant(op);
  if (op->G) (void)hipFree(op->G);
  if (op->w) (void)hipFree(op->w);
  if (op->ub) (void)hipFree(op->ub);
  if (op->G32) (void)hipFree(op->G32);
  if (op->Gb) (void)hipFree(op->Gb);
  if (op->Gsym) (void)hipFree(op->Gsym);
  if (op->Gt16) (void)hipFree(op->Gt16);
  if (op->Et16) (void)hipFree(op->Et16);
  if (op->Gt16T) (void)hipFree(op->Gt16T);
  if (op->Et16T) (void)hipFree(op->Et16T);
  if (op->xc) (void)hipFree(op->xc);
  if (op->yc) (void)hipFree(op->yc);
  delete op;
}

int32_t copy_nodal(const double* host, int nodes, double** dev, hipStream_t s) {
  *dev = nullptr;
  if (!host) return PINV_OK;
  PINV_HIP_TRY(hipMalloc(dev, (size_t)nodes * sizeof(double)));
  hipError_t e = hipMemcpyAsync(*dev, host, (size_t)nodes * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    (void)hipFree(*dev);
    *dev = nullptr;
    return pinv_hip_status(e);
  }
  return PINV_OK;
}

bool boundary_nonzero(const pinv_grid* g, const double* ub) {
  if (!ub) return false;
  for (int i = 0; i < g->ny; ++i)
    for (int j = 0; j < g->nx; ++j) {
      const bool b = (i == 0 || i == g->ny - 1 || j == 0 || j == g->nx - 1);
      if (b && ub[(int64_t)i * g->nx + j] != 0.0) return true;
    }
  return false;
}

int slices_of_bits(int bits) { return (bits == 8 || bits == 16 || bits == 24) ? bits / 8 : 0; }

// int32 class headroom: the largest class has min(S, SR) slice pairs, each
// contributing at most n * 128 * 128 in magnitude.  The int64 recombination
// needs n * M_S * M_SR < 2^63.
// The exact recombination in int64 holds while N M_S M_SR < 2^63.
bool int8_total_ok(int n, int S, int SR) {
  return (double)n * (double)pinv_max_mag(S) * (double)pinv_max_mag(SR) < 9.2e18;
}

// Largest k range one int32 class accumulator may cover: every term of a class
// is at most 128 * 128 per digit pair, and at most min(S, SR) pairs share a
// class, so k * 16384 * pairs must stay below 2^31.  A multiple of 256.
int64_t int8_k_limit(int S, int SR) {
  const int64_t pairs = S < SR ? S : SR;
  return (2147483647LL / (16384LL * pairs)) / 256 * 256;
}

// The whole of k in one accumulation (the grouped launches do not split k).
bool int8_headroom_ok(int n, int S, int SR) {
  const int pairs = S < SR ? S : SR;
  return (double)n * 16384.0 * pairs < 2147483648.0 && int8_total_ok(n, S, SR);
}

// The k split of one int8 apply of `variant`: where the tiles leave workgroup
// slots empty (gemm_i8_split_plan: all tiles, or the last round's row tiles),
// and wherever one int32 accumulation over k could overflow (then every tile
// splits; the parts are added exactly in int64).
void int8_split(pinv_op op, int SR, int Rpad, int variant, int* ksplit, int* kchunk, int* tail_rows) {
  gemm_i8_split_plan(op->P, Rpad, variant, ksplit, kchunk, tail_rows);
  const int64_t klim = int8_k_limit(op->S, SR);
  if (op->P > klim && (*tail_rows > 0 || *kchunk > klim)) {
    *tail_rows = 0;
    *kchunk = (int)klim;
    *ksplit = (int)((op->P + klim - 1) / klim);
  }
}

// The quantisation of the right-hand sides and the slice product of one int8
// apply, on caller-provided scratch: Xq [SR][Rpad][P] int8, f [Rpad] int32
// and, when ksplit > 1, the partial sums (gemm_i8_part_bytes).
// (trace = false: no timing events, for the allocation-free entry point)
hipError_t int8_launch(pinv_op op, const int8_t* Q, const int32_t* row_exp, const int32_t* pre_exp, int SR,
                       const double* X, int64_t ldx, int nrhs, const double* w, double* U, int64_t ldu,
                       int Rpad, int variant, int ksplit, int kchunk, int tail_rows, int8_t* Xq, int32_t* f,
                       int32_t* part, hipStream_t s, bool trace = true) {
  hipError_t e;
  {
    TraceScope ts(trace ? "quantize_cols" : nullptr, s);
    e = launch_quantize_cols(X, ldx, nullptr, op->n, nrhs, Rpad, SR, op->P, pre_exp, Xq, f, s);
  }
  if (e != hipSuccess) return e;
  // few right-hand sides: a pass over the digit planes (HBM-bound), else the
  // tiled matrix-core product
  const bool gemv = nrhs <= GEMV_I8_MAX_RHS;
  TraceScope ts(trace ? (gemv ? "gemv_i8" : "gemm_i8") : nullptr, s);
  GemmI8Args a{};
  a.Q = Q; a.S = op->S;
  a.X = Xq; a.SR = SR;
  a.P = op->P; a.Rpad = Rpad;
  a.n = op->n; a.nrhs = nrhs;
  a.row_exp = row_exp;
  a.col_exp = f;
  a.c = -(op->h * op->h) / ((double)pinv_max_mag(op->S) * (double)pinv_max_mag(SR));
  a.w = w;
  a.U = U; a.ldu = ldu;
  a.variant = variant;
  a.ksplit = ksplit;
  a.kchunk = kchunk;
  a.part = ksplit > 1 ? part : nullptr;
  a.tail_rows = ksplit > 1 ? tail_rows : 0;
  return gemv ? launch_gemv_i8(a, s) : launch_gemm_i8(a, s);
}

int32_t int8_apply(pinv_op op, const int8_t* Q, const int32_t* row_exp, const int32_t* pre_exp, int SR,
                   const double* X, int64_t ldx, int nrhs, const double* w, double* U, int64_t ldu,
                   hipStream_t s) {
  const int Rpad = (nrhs + 127) / 128 * 128;
  const int variant = op->i8_variant[SR];
  int ksplit = 1, kchunk = (int)op->P, tail_rows = 0;
  // (the few-right-hand-side pass adds its lanes' class sums in int64: no split)
  if (nrhs > GEMV_I8_MAX_RHS) int8_split(op, SR, Rpad, variant, &ksplit, &kchunk, &tail_rows);
  const size_t xq_bytes = (size_t)SR * Rpad * op->P;
  const size_t f_bytes = ((size_t)Rpad * sizeof(int32_t) + 255) / 256 * 256;
  const size_t part_bytes = gemm_i8_part_bytes(op->P, Rpad, variant, op->S + SR - 1, ksplit, tail_rows);
  void* scratch = nullptr;
  configure_pool_once();
  PINV_HIP_TRY(hipMallocAsync(&scratch, xq_bytes + f_bytes + part_bytes, s));
  const hipError_t e = int8_launch(op, Q, row_exp, pre_exp, SR, X, ldx, nrhs, w, U, ldu, Rpad, variant, ksplit, kchunk,
                                   tail_rows, (int8_t*)scratch, (int32_t*)((char*)scratch + xq_bytes),
                                   (int32_t*)((char*)scratch + xq_bytes + f_bytes), s);
  hipError_t e2 = hipFreeAsync(scratch, s);
  if (e != hipSuccess) return pinv_hip_status(e);
  return pinv_hip_status(e2);
}

int32_t fp64_apply(pinv_op op, bool transpose, const double* X, int64_t ldx, int nrhs, const double* bias,
                   double* U, int64_t ldu, hipStream_t s) {
  const double alpha = -(op->h * op->h);
  // G^T = G bit for bit: the adjoint is the forward product
  if (transpose && op->g_symmetric) transpose = false;
  if (!transpose && nrhs <= 4) {
    TraceScope ts("gemv_f64", s);
    PINV_HIP_TRY(launch_gemv_f64(op->G, op->ldg, op->n, X, ldx, nrhs, alpha, bias, U, ldu, s));
    return PINV_OK;
  }
  if (!transpose) {
    // the forward product: one wave per SIMD, 256 x 128 tiles; right-hand
    // sides in chunks whose padded copy holds fewer than 2^31 values
    const int64_t ldp = ((int64_t)op->n + 31) / 32 * 32;
    const int chunk = (int)std::max<int64_t>(128, (((int64_t)1 << 31) / ldp) / 128 * 128);
    configure_pool_once();
    TraceScope ts("gemm_f64", s);
    for (int c0 = 0; c0 < nrhs; c0 += chunk) {
      const int nc = std::min(chunk, nrhs - c0);
      const ApplyF64Plan p = apply_f64_plan(op->n, nc, op->n);
      void* scratch = nullptr;
      PINV_HIP_TRY(hipMallocAsync(&scratch, p.pack_bytes + p.part_bytes, s));
      const hipError_t e = launch_apply_f64(p, op->G, op->ldg, op->n, op->n, X + (int64_t)c0 * ldx, ldx, nc, alpha,
                                            bias, U + (int64_t)c0 * ldu, ldu, scratch, s);
      const hipError_t e2 = hipFreeAsync(scratch, s);
      if (e != hipSuccess) return pinv_hip_status(e);
      if (e2 != hipSuccess) return pinv_hip_status(e2);
    }
    return PINV_OK;
  }
  GemmF64Args a{};
  a.A = op->G; a.lda = op->ldg; a.a_kcontig = transpose ? 0 : 1;
  a.B = X; a.ldb = ldx; a.b_kcontig = 1;
  a.C = U; a.csm = 1; a.csn = ldu;
  a.M = op->n; a.N = nrhs; a.K = op->n;
  a.alpha = alpha; a.beta = 0.0; a.bias = bias;
  a.ksplit = 1;
  // the forward product (both operands k-contiguous) splits k when the tile
  // grid alone would leave compute units idle
  if (!transpose) gemm_f64_split_plan(a.M, a.N, a.K, &a.ksplit, &a.kchunk);
  void* part = nullptr;
  if (a.ksplit > 1) {
    configure_pool_once();
    PINV_HIP_TRY(hipMallocAsync(&part, (size_t)a.ksplit * a.M * a.N * sizeof(double), s));
    a.part = (double*)part;
  }
  hipError_t e;
  {
    TraceScope ts("gemm_f64", s);
    e = launch_gemm_f64(a, s);
  }
  const hipError_t e2 = part ? hipFreeAsync(part, s) : hipSuccess;
  if (e != hipSuccess) return pinv_hip_status(e);
  return pinv_hip_status(e2);
}

int32_t check_vectors(pinv_op op, const void* in, int64_t ld_in, int nrhs, const void* out, int64_t ld_out) {
  if (!op) return PINV_E_INVALID_ARG;
  if (nrhs < 0) return PINV_E_INVALID_ARG;
  if (nrhs == 0) return PINV_OK;
  if (!in || !out) return PINV_E_INVALID_ARG;
  if (ld_in < op->n || ld_out < op->n) return PINV_E_INVALID_ARG;
  // overlap check of the two column-major blocks
  const char* a0 = (const char*)in;
  const char* a1 = a0 + ((int64_t)(nrhs - 1) * ld_in + op->n) * 8;
  const char* b0 = (const char*)out;
  const char* b1 = b0 + ((int64_t)(nrhs - 1) * ld_out + op->n) * 8;
  if (a0 < b1 && b0 < a1) return PINV_E_INVALID_ARG;
  return PINV_OK;
}

// ---- batched int8 applies: cached plans ---------------------------------------
// A plan holds everything one request list needs on the device: the column
// pointer table, the grouped-launch tables and the scratch of the quantised
// right-hand sides, plus the host image the tables were uploaded from (pinned,
// alive as long as the plan, so the upload needs no wait).  Plans are keyed by
// the request list, the rho width, the ops' digit counts and kernel variants,
// and the stream; a call with a known key only launches kernels (so it can be
// captured into a HIP graph, which then stays valid while the plan is kept).
// At most kMaxPlans are kept (least recently used goes first); plans naming an
// op are dropped when the op is destroyed or re-quantised.
struct BatchLaunch {
  int S, variant;
  int q0, nq, qcols;       // ordinary-width quantisation groups
  int qw0, nqw, qcols_w;   // wide-column quantisation groups
  int g0, ng, tiles;       // product groups
};

struct BatchPlan {
  std::vector<char> key;
  std::vector<pinv_op> ops;
  char* dtable = nullptr;   // device: column pointers, QuantColsGroup[], GemmI8Group[]
  char* scratch = nullptr;  // device: quantised rho and exponents
  char* host = nullptr;     // pinned image of dtable
  size_t dbytes = 0;
  size_t q_off = 0, g_off = 0;  // offsets of the two group tables in dtable
  std::vector<BatchLaunch> launches;
  uint64_t last_use = 0;
};

constexpr size_t kMaxPlans = 4;
std::mutex g_plan_mu;
uint64_t g_plan_clock = 0;

// (never destroyed: freeing device memory from a static destructor could run
// after the runtime has shut down)
std::vector<BatchPlan*>& g_plans() {
  static std::vector<BatchPlan*>* v = new std::vector<BatchPlan*>();
  return *v;
}

void free_plan(BatchPlan* p) {
  if (p->dtable) (void)hipFree(p->dtable);
  if (p->scratch) (void)hipFree(p->scratch);
  if (p->host) (void)hipHostFree(p->host);
  delete p;
}

void purge_batch_plans(pinv_op op) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  std::vector<BatchPlan*>& v = g_plans();
  bool synced = false;
  for (size_t i = 0; i < v.size();) {
    BatchPlan* p = v[i];
    if (std::find(p->ops.begin(), p->ops.end(), op) == p->ops.end()) {
      ++i;
      continue;
    }
    if (!synced) {
      (void)hipDeviceSynchronize();  // no launch of the plan may still be running
      synced = true;
    }
    free_plan(p);
    v.erase(v.begin() + (long)i);
  }
}

template <class T>
void put(std::vector<char>& k, const T& x) {
  const char* b = (const char*)&x;
  k.insert(k.end(), b, b + sizeof(T));
}

std::vector<char> plan_key(const pinv_request* reqs, int nreq, int SR, hipStream_t s) {
  std::vector<char> k;
  k.reserve(48 + (size_t)nreq * 48);
  put(k, SR);
  put(k, s);
  put(k, nreq);
  for (int i = 0; i < nreq; ++i) {
    const pinv_request& r = reqs[i];
    put(k, r.op);
    put(k, r.rho);
    put(k, r.u);
    put(k, r.ld);
    put(k, r.nrhs);
    put(k, r.op->S);
  }
  return k;
}

hipError_t run_quantize(const BatchPlan& plan, const BatchLaunch& L, int SR, hipStream_t s) {
  const QuantColsGroup* dq = (const QuantColsGroup*)(plan.dtable + plan.q_off);
  TraceScope ts("quantize_cols", s);
  hipError_t e = launch_quantize_cols_grouped(dq + L.q0, L.nq, L.qcols, SR, false, s);
  if (e == hipSuccess) e = launch_quantize_cols_grouped(dq + L.qw0, L.nqw, L.qcols_w, SR, true, s);
  return e;
}

hipError_t run_product(const BatchPlan& plan, const BatchLaunch& L, int variant, int SR, hipStream_t s) {
  const GemmI8Group* dg = (const GemmI8Group*)(plan.dtable + plan.g_off);
  return launch_gemm_i8_grouped(dg + L.g0, L.ng, L.tiles, L.S, SR, variant, s);
}

// The kernel variant of each of a new plan's product launches: every variant
// with 128-row tiles is timed on the launch itself (the plan's own groups and
// right-hand sides, best of two runs after a warm-up); the results are
// bit-identical whichever runs, so the launches write the caller's u with the
// final values.  A one-time cost of the first call with a request list.
int32_t tune_plan(BatchPlan* plan, int SR, hipStream_t s) {
  hipEvent_t a = nullptr, b = nullptr;
  PINV_HIP_TRY(hipEventCreate(&a));
  hipError_t e = hipEventCreate(&b);
  for (BatchLaunch& L : plan->launches) {
    if (e == hipSuccess) e = run_quantize(*plan, L, SR, s);
    double best = 1e30;
    for (int v = 0; v < gemm_i8_variants() && e == hipSuccess; ++v) {
      if (gemm_i8_tile_rows(v) != 128) continue;
      e = run_product(*plan, L, v, SR, s);
      double t = 1e30;
      for (int r = 0; r < 2 && e == hipSuccess; ++r) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess) e = run_product(*plan, L, v, SR, s);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess) t = std::min(t, (double)ms);
      }
      if (e == hipSuccess && t < best) {
        best = t;
        L.variant = v;
      }
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return pinv_hip_status(e);
}

// Builds a plan: requests grouped by op (in order of first appearance); per
// digit count S one grouped product launch (kernel variant timed on it), with
// two grouped quantisation launches (ordinary and 16385-40960-entry columns).
int32_t make_plan(const pinv_request* reqs, int nreq, int SR, hipStream_t s, BatchPlan* plan) {
  std::vector<pinv_op>& ops = plan->ops;
  std::unordered_map<pinv_op, std::vector<int>> members;
  for (int i = 0; i < nreq; ++i) {
    if (reqs[i].nrhs == 0) continue;
    pinv_op op = reqs[i].op;
    auto it = members.find(op);
    if (it == members.end()) {
      ops.push_back(op);
      members[op] = {i};
    } else {
      it->second.push_back(i);
    }
  }
  const int ng = (int)ops.size();
  std::vector<int64_t> first(ng), count(ng), Rpad(ng), xq_off(ng), f_off(ng);
  std::vector<const void*> cols;
  size_t xq_bytes = 0, f_bytes = 0;
  for (int g = 0; g < ng; ++g) {
    first[g] = (int64_t)cols.size();
    for (int i : members[ops[g]])
      for (int j = 0; j < reqs[i].nrhs; ++j) cols.push_back(reqs[i].rho + (int64_t)j * reqs[i].ld);
    count[g] = (int64_t)cols.size() - first[g];
    for (int i : members[ops[g]])
      for (int j = 0; j < reqs[i].nrhs; ++j) cols.push_back(reqs[i].u + (int64_t)j * reqs[i].ld);
    Rpad[g] = (count[g] + 127) / 128 * 128;
    xq_off[g] = (int64_t)xq_bytes;
    xq_bytes += (size_t)SR * Rpad[g] * ops[g]->P;
    f_off[g] = (int64_t)f_bytes;
    f_bytes += (size_t)Rpad[g] * sizeof(int32_t);
  }
  auto align256 = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t cols_bytes = align256(cols.size() * sizeof(void*));
  const size_t qg_bytes = align256(ng * sizeof(QuantColsGroup));
  const size_t gg_bytes = align256(ng * sizeof(GemmI8Group));
  plan->dbytes = cols_bytes + qg_bytes + gg_bytes;
  plan->q_off = cols_bytes;
  plan->g_off = cols_bytes + qg_bytes;
  PINV_HIP_TRY(hipMalloc((void**)&plan->dtable, plan->dbytes));
  PINV_HIP_TRY(hipMalloc((void**)&plan->scratch, align256(xq_bytes) + f_bytes));
  PINV_HIP_TRY(hipHostMalloc((void**)&plan->host, plan->dbytes, hipHostMallocDefault));
  std::memset(plan->host, 0, plan->dbytes);
  const void* const* dcols = (const void* const*)plan->dtable;
  int8_t* Xq = (int8_t*)plan->scratch;
  int32_t* F = (int32_t*)(plan->scratch + align256(xq_bytes));
  std::memcpy(plan->host, cols.data(), cols.size() * sizeof(void*));
  QuantColsGroup* hq = (QuantColsGroup*)(plan->host + cols_bytes);
  GemmI8Group* hg = (GemmI8Group*)(plan->host + cols_bytes + qg_bytes);

  // launches: one per digit count S, in order of S; all variants considered
  // below have 128-row tiles, so the tables do not depend on the choice
  int slot = 0;
  for (int S = 1; S <= 3; ++S) {
    bool has = false;
    for (int g = 0; g < ng; ++g) has = has || ops[g]->S == S;
    if (!has) continue;
    BatchLaunch L{S, 0, slot, 0, 0, 0, 0, 0, slot, 0, 0};
    const int rows = 128;
    // ordinary-width columns first, then the wide ones (their quantisation
    // runs in a launch of its own); the product groups keep the same order
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) L.qw0 = slot;
      for (int g = 0; g < ng; ++g) {
        pinv_op op = ops[g];
        if (op->S != L.S || quantize_cols_wide(op->n) != (pass == 1)) continue;
        QuantColsGroup& q = hq[slot];
        q.xcols = (const double* const*)(dcols + first[g]);
        q.Xq = Xq + xq_off[g];
        q.f = (int32_t*)((char*)F + f_off[g]);
        q.P = op->P;
        q.n = op->n;
        q.nrhs = (int)count[g];
        q.Rpad = (int)Rpad[g];
        q.col0 = pass == 0 ? L.qcols : L.qcols_w;
        GemmI8Group& G = hg[slot];
        G.a.Q = op->Q; G.a.S = op->S;
        G.a.X = q.Xq; G.a.SR = SR;
        G.a.P = op->P; G.a.Rpad = (int)Rpad[g];
        G.a.n = op->n; G.a.nrhs = (int)count[g];
        G.a.row_exp = op->e;
        G.a.col_exp = q.f;
        G.a.c = -(op->h * op->h) / ((double)pinv_max_mag(op->S) * (double)pinv_max_mag(SR));
        G.a.w = op->w;
        G.a.U = nullptr; G.a.ldu = 0;
        G.a.ucols = (double* const*)(dcols + first[g] + count[g]);
        G.tilesM = (int)(op->P / rows);
        G.tilesN = (int)(Rpad[g] / 128);
        G.tile0 = L.tiles;
        if (pass == 0) {
          L.qcols += (int)Rpad[g];
          ++L.nq;
        } else {
          L.qcols_w += (int)Rpad[g];
          ++L.nqw;
        }
        L.tiles += G.tilesM * G.tilesN;
        ++L.ng;
        ++slot;
      }
    }
    plan->launches.push_back(L);
  }
  // the pinned image lives as long as the plan, so the upload is not waited for
  PINV_HIP_TRY(hipMemcpyAsync(plan->dtable, plan->host, plan->dbytes, hipMemcpyHostToDevice, s));
  return tune_plan(plan, SR, s);
}

int32_t find_or_make_plan(const pinv_request* reqs, int nreq, int SR, hipStream_t s, BatchPlan** out) {
  std::vector<char> key = plan_key(reqs, nreq, SR, s);
  std::vector<BatchPlan*>& v = g_plans();
  for (BatchPlan* p : v)
    if (p->key == key) {
      p->last_use = ++g_plan_clock;
      *out = p;
      return PINV_OK;
    }
  // a new plan allocates: not while the stream is being captured
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  PINV_HIP_TRY(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) {
    pinv_log("pinv_apply_batched: a request list seen for the first time cannot be planned under stream capture");
    return PINV_E_STATE;
  }
  if (v.size() >= kMaxPlans) {
    size_t lru = 0;
    for (size_t i = 1; i < v.size(); ++i)
      if (v[i]->last_use < v[lru]->last_use) lru = i;
    PINV_HIP_TRY(hipDeviceSynchronize());  // its launches may still be running
    free_plan(v[lru]);
    v.erase(v.begin() + (long)lru);
  }
  BatchPlan* p = new (std::nothrow) BatchPlan();
  if (!p) return PINV_E_OOM;
  p->key = std::move(key);
  const int32_t st = make_plan(reqs, nreq, SR, s, p);
  if (st != PINV_OK) {
    free_plan(p);
    return st;
  }
  p->last_use = ++g_plan_clock;
  v.push_back(p);
  *out = p;
  return PINV_OK;
}

hipError_t run_plan(const BatchPlan& plan, int SR, hipStream_t s) {
  for (const BatchLaunch& L : plan.launches) {
    hipError_t e = run_quantize(plan, L, SR, s);
    if (e != hipSuccess) return e;
    TraceScope ts("gemm_i8", s);
    e = run_product(plan, L, L.variant, SR, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---- allocation-free int8 apply ---------------------------------------------
// Scratch of pinv_apply_inverse_noalloc: the quantised right-hand sides
// (Xq [SR][Rpad][P] int8) and their exponents (f [Rpad] int32).  Every GPU the
// library runs on holds its own copy of this array until the process ends.
// In host code the array's name is only a stand-in for the symbol: its device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) int8_t scratch[PINV_NOALLOC_SCRATCH_BYTES];

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64] = {};

// The device address of `scratch` on the current device (looked up on the
// first call on that device, with that device current).
int32_t noalloc_scratch(void** out) {
  int dev = 0;
  PINV_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return PINV_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      pinv_log("pinv_apply_inverse_noalloc: hipGetSymbolAddress of the scratch array failed on device %d (%s)", dev,
               hipGetErrorString(e));
      return e != hipSuccess ? pinv_hip_status(e) : PINV_E_HIP;
    }
    g_noalloc_ptr[dev] = ptr;
  }
  *out = g_noalloc_ptr[dev];
  return PINV_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// entry points

extern "C" {

const char* pinv_version(void) { return "0.1.0"; }

const char* pinv_status_string(int32_t st) {
  switch (st) {
    case PINV_OK: return "ok";
    case PINV_E_INVALID_ARG: return "invalid argument";
    case PINV_E_NOT_SPD: return "operator is not symmetric positive definite (non-positive Cholesky pivot)";
    case PINV_E_OOM: return "out of device memory (or more scratch than pinv_apply_inverse_noalloc holds)";
    case PINV_E_HIP: return "HIP runtime error";
    case PINV_E_UNSUPPORTED: return "unsupported size or mode";
    case PINV_E_STATE: return "the op does not hold the representation this call needs";
    case PINV_E_IO: return "file could not be opened, read or written";
    default: return "unknown status";
  }
}

// Steps 1-2 for a new op (2-D or 3-D): device copies of the nodal data, the
// device build, the Dirichlet data kept for the eps-gradient.
int32_t build_op(pinv_op op, int nodes, bool has_ub, const double* eps_nodes, const double* u_boundary,
                 hipStream_t s, pinv_op* out, const GeneralGrid* gen = nullptr);

int32_t pinv_build_inverse(const pinv_grid* g, const double* eps_nodes, const double* u_boundary, void* stream,
                           pinv_op* out) {
  if (!out) return PINV_E_INVALID_ARG;
  *out = nullptr;
  if (!grid_ok(g)) return PINV_E_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  pinv_op op = new_op(g);
  if (!op) return PINV_E_OOM;
  return build_op(op, g->nx * g->ny, boundary_nonzero(g, u_boundary), eps_nodes, u_boundary, s, out);
}

int32_t pinv_build_inverse_3d(const pinv_grid3* g, const double* eps_nodes, const double* u_boundary, void* stream,
                              pinv_op* out) {
  if (!out) return PINV_E_INVALID_ARG;
  *out = nullptr;
  if (!g || g->nx < 3 || g->ny < 3 || g->nz < 3 || !(g->h > 0.0) || !std::isfinite(g->h)) return PINV_E_INVALID_ARG;
  const int64_t n = (int64_t)(g->nx - 2) * (g->ny - 2) * (g->nz - 2);
  if (n > (int64_t)1 << 20) return PINV_E_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  pinv_grid g2{g->nx, g->ny, g->h};
  pinv_op op = new_op(&g2);
  if (!op) return PINV_E_OOM;
  op->nz = g->nz;
  op->mz = g->nz - 2;
  op->n = (int)n;
  op->ldg = (op->n + 31) / 32 * 32;
  const int nodes = g->nx * g->ny * g->nz;
  bool has_ub = false;
  if (u_boundary)
    for (int k = 0; k < g->nz && !has_ub; ++k)
      for (int i = 0; i < g->ny && !has_ub; ++i)
        for (int j = 0; j < g->nx; ++j) {
          const bool b = k == 0 || k == g->nz - 1 || i == 0 || i == g->ny - 1 || j == 0 || j == g->nx - 1;
          if (b && u_boundary[((int64_t)k * g->ny + i) * g->nx + j] != 0.0) {
            has_ub = true;
            break;
          }
        }
  return build_op(op, nodes, has_ub, eps_nodes, u_boundary, s, out);
}

int32_t pinv_build_inverse_general(const pinv_grid_general* g, const double* eps_x, const double* eps_y,
                                   const double* u_boundary, void* stream, pinv_op* out) {
  if (!out) return PINV_E_INVALID_ARG;
  *out = nullptr;
  if (!g || g->nx < 3 || g->ny < 3 || !g->x || !g->y) return PINV_E_INVALID_ARG;
  for (int j = 0; j < g->nx; ++j)
    if (!std::isfinite(g->x[j]) || (j > 0 && !(g->x[j] > g->x[j - 1]))) return PINV_E_INVALID_ARG;
  for (int i = 0; i < g->ny; ++i)
    if (!std::isfinite(g->y[i]) || (i > 0 && !(g->y[i] > g->y[i - 1]))) return PINV_E_INVALID_ARG;
  const int64_t n64 = (int64_t)(g->nx - 2) * (g->ny - 2);
  if (n64 > (int64_t)1 << 20) return PINV_E_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  pinv_grid g2{g->nx, g->ny, 1.0};
  pinv_op op = new_op(&g2);
  if (!op) return PINV_E_OOM;
  op->general = 1;
  const int nodes = g->nx * g->ny;
  GeneralGrid gen{};
  double *x_d = nullptr, *y_d = nullptr, *ey_d = nullptr, *area_d = nullptr;
  int32_t st = copy_nodal(g->x, g->nx, &x_d, s);
  if (st == PINV_OK) st = copy_nodal(g->y, g->ny, &y_d, s);
  if (st == PINV_OK) st = copy_nodal(eps_y, nodes, &ey_d, s);
  if (st == PINV_OK) {
    const hipError_t e = hipMalloc(&area_d, (size_t)op->n * sizeof(double));
    if (e != hipSuccess) st = pinv_hip_status(e);
  }
  if (st != PINV_OK) {
    if (x_d) (void)hipFree(x_d);
    if (y_d) (void)hipFree(y_d);
    if (ey_d) (void)hipFree(ey_d);
    delete op;
    return st;
  }
  gen.x = x_d;
  gen.y = y_d;
  gen.eps_y = ey_d;
  gen.area = area_d;
  st = build_op(op, nodes, boundary_nonzero(&g2, u_boundary), eps_x, u_boundary, s, out, &gen);
  (void)hipStreamSynchronize(s);
  if (st == PINV_OK) {
    // the node coordinates stay with the op for the eps-gradient
    (*out)->xc = x_d;
    (*out)->yc = y_d;
    (*out)->bytes += (int64_t)(g->nx + g->ny) * sizeof(double);
  } else {
    (void)hipFree(x_d);
    (void)hipFree(y_d);
  }
  if (ey_d) (void)hipFree(ey_d);
  (void)hipFree(area_d);
  return st;
}

int32_t pinv_build_inverse_beta(const pinv_grid* g, const double* beta, const double* u_boundary, void* stream,
                                pinv_op* out) {
  if (!out) return PINV_E_INVALID_ARG;
  *out = nullptr;
  if (!g || !beta) return PINV_E_INVALID_ARG;
  pinv_grid g2{g->nx, g->ny, 1.0};
  if (!grid_ok(&g2)) return PINV_E_INVALID_ARG;
  const int nodes = g->nx * g->ny;
  for (int64_t k = 0; k < 4 * (int64_t)nodes; ++k)
    if (!std::isfinite(beta[k])) return PINV_E_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  pinv_op op = new_op(&g2);
  if (!op) return PINV_E_OOM;
  op->beta = 1;
  const size_t need = 2 * (size_t)op->n * op->ldg * sizeof(double);
  size_t freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) == hipSuccess && need > freeb) {
    delete op;
    return PINV_E_OOM;
  }
  double *beta_d = nullptr, *ub_d = nullptr;
  int32_t st = PINV_OK;
  {
    const hipError_t e = hipMalloc(&beta_d, 4 * (size_t)nodes * sizeof(double));
    if (e != hipSuccess) st = pinv_hip_status(e);
    else {
      const hipError_t e2 =
          hipMemcpyAsync(beta_d, beta, 4 * (size_t)nodes * sizeof(double), hipMemcpyHostToDevice, s);
      if (e2 != hipSuccess) st = pinv_hip_status(e2);
    }
  }
  if (st == PINV_OK && boundary_nonzero(&g2, u_boundary)) st = copy_nodal(u_boundary, nodes, &ub_d, s);
  if (st == PINV_OK) st = build_inverse_lu_device(op, beta_d, ub_d, s);
  (void)hipStreamSynchronize(s);
  if (beta_d) (void)hipFree(beta_d);
  if (st != PINV_OK) {
    if (ub_d) (void)hipFree(ub_d);
    free_op(op);
    return st;
  }
  op->ub = ub_d;
  if (ub_d) op->bytes += (int64_t)nodes * sizeof(double);
  *out = op;
  return PINV_OK;
}

int32_t build_op(pinv_op op, int nodes, bool has_ub, const double* eps_nodes, const double* u_boundary,
                 hipStream_t s, pinv_op* out, const GeneralGrid* gen) {
  const size_t need = 2 * (size_t)op->n * op->ldg * sizeof(double);
  size_t freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) == hipSuccess && need > freeb) {
    delete op;
    return PINV_E_OOM;
  }
  double *eps_d = nullptr, *ub_d = nullptr;
  int32_t st = copy_nodal(eps_nodes, nodes, &eps_d, s);
  if (st == PINV_OK && has_ub) st = copy_nodal(u_boundary, nodes, &ub_d, s);
  if (st == PINV_OK) st = build_inverse_device(op, eps_d, ub_d, gen, s);
  if (eps_d) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(eps_d);
  }
  if (st != PINV_OK) {
    if (ub_d) (void)hipFree(ub_d);
    free_op(op);
    return st;
  }
  op->ub = ub_d;
  if (ub_d) op->bytes += (int64_t)nodes * sizeof(double);
  st = detect_symmetry(op, s);
  if (st != PINV_OK) {
    free_op(op);
    return st;
  }
  pinv_log("build_inverse: n=%d ldg=%lld bytes=%lld symmetric=%d", op->n, (long long)op->ldg, (long long)op->bytes,
           op->g_symmetric);
  *out = op;
  return PINV_OK;
}

int32_t pinv_import_inverse(const pinv_grid* g, const double* G_host, int64_t ldg, const double* eps_nodes,
                            const double* u_boundary, const double* w_host, void* stream, pinv_op* out) {
  if (!out) return PINV_E_INVALID_ARG;
  *out = nullptr;
  if (!grid_ok(g) || !G_host) return PINV_E_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  pinv_op op = new_op(g);
  if (!op) return PINV_E_OOM;
  if (ldg < op->n) {
    delete op;
    return PINV_E_INVALID_ARG;
  }
  const int n = op->n, nodes = g->nx * g->ny;
  int32_t st = PINV_OK;
  hipError_t e = hipMalloc(&op->G, (size_t)n * op->ldg * sizeof(double));
  // rows are padded to 32 doubles with zeros (the FP64 apply reads whole
  // 16-double pieces of k)
  if (e == hipSuccess) e = hipMemsetAsync(op->G, 0, (size_t)n * op->ldg * sizeof(double), s);
  if (e != hipSuccess) {
    free_op(op);
    return pinv_hip_status(e);
  }
  op->bytes += (int64_t)n * op->ldg * sizeof(double);
  e = hipMemcpy2DAsync(op->G, op->ldg * sizeof(double), G_host, ldg * sizeof(double), n * sizeof(double), n,
                       hipMemcpyHostToDevice, s);
  if (e != hipSuccess) st = pinv_hip_status(e);
  const bool has_ub = boundary_nonzero(g, u_boundary);
  if (st == PINV_OK && has_ub) {
    st = copy_nodal(u_boundary, nodes, &op->ub, s);
    if (st == PINV_OK) op->bytes += (int64_t)nodes * sizeof(double);
  }
  if (st == PINV_OK && (w_host || has_ub)) {
    e = hipMalloc(&op->w, (size_t)n * sizeof(double));
    if (e == hipSuccess) {
      op->bytes += (int64_t)n * sizeof(double);
      if (w_host) {
        e = hipMemcpyAsync(op->w, w_host, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s);
      } else {
        double *eps_d = nullptr, *bB = nullptr;
        st = copy_nodal(eps_nodes, nodes, &eps_d, s);
        if (st == PINV_OK) {
          e = hipMalloc(&bB, (size_t)n * sizeof(double));
          if (e == hipSuccess) e = launch_assemble(g->nx, g->ny, 0, eps_d, op->ub, nullptr, 0, bB, s);
          if (e == hipSuccess) e = launch_gemv_f64(op->G, op->ldg, n, bB, n, 1, 1.0, nullptr, op->w, n, s);
          (void)hipStreamSynchronize(s);
          if (bB) (void)hipFree(bB);
        }
        if (eps_d) (void)hipFree(eps_d);
      }
    }
    if (e != hipSuccess && st == PINV_OK) st = pinv_hip_status(e);
  }
  if (st == PINV_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = pinv_hip_status(e);
  }
  if (st == PINV_OK) st = detect_symmetry(op, s);
  if (st != PINV_OK) {
    free_op(op);
    return st;
  }
  *out = op;
  return PINV_OK;
}

int32_t pinv_export_inverse(pinv_op op, double* G_host, int64_t ldg, double* w_host, void* stream) {
  if (!op) return PINV_E_INVALID_ARG;
  if (!op->G) return PINV_E_STATE;
  hipStream_t s = as_stream(stream);
  if (G_host) {
    if (ldg < op->n) return PINV_E_INVALID_ARG;
    PINV_HIP_TRY(hipMemcpy2DAsync(G_host, ldg * sizeof(double), op->G, op->ldg * sizeof(double),
                                  op->n * sizeof(double), op->n, hipMemcpyDeviceToHost, s));
  }
  if (w_host) {
    if (op->w)
      PINV_HIP_TRY(hipMemcpyAsync(w_host, op->w, (size_t)op->n * sizeof(double), hipMemcpyDeviceToHost, s));
    else
      std::memset(w_host, 0, (size_t)op->n * sizeof(double));
  }
  PINV_HIP_TRY(hipStreamSynchronize(s));
  return PINV_OK;
}

int32_t pinv_quantize_inverse(pinv_op op, int32_t bits, int32_t scale_mode, int32_t keep_fp64, void* stream) {
  if (!op) return PINV_E_INVALID_ARG;
  const int S = slices_of_bits(bits);
  if (!S || scale_mode != PINV_SCALE_ROW) return PINV_E_INVALID_ARG;
  if (!op->G) return PINV_E_STATE;
  hipStream_t s = as_stream(stream);
  PINV_HIP_TRY(hipStreamSynchronize(s));
  free_quant(op);
  const int64_t P = pinv_pad_dim(op->n);
  const size_t plane_bytes = (size_t)S * P * P;
  hipError_t e = hipMalloc(&op->Q, plane_bytes);
  if (e == hipSuccess) e = hipMalloc(&op->QT, plane_bytes);
  if (e == hipSuccess) e = hipMalloc(&op->e, (size_t)P * sizeof(int32_t));
  if (e != hipSuccess) {
    free_quant(op);
    return pinv_hip_status(e);
  }
  op->S = S;
  op->P = P;
  op->bytes += 2 * (int64_t)plane_bytes + P * (int64_t)sizeof(int32_t);
  e = launch_quantize_rows(op->G, op->ldg, op->n, S, P, op->Q, op->e, s);
  if (e == hipSuccess) e = launch_transpose_planes(op->Q, op->QT, S, P, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_quant(op);
    return pinv_hip_status(e);
  }
  if (!keep_fp64) {
    (void)hipFree(op->G);
    op->G = nullptr;
    op->bytes -= (int64_t)op->n * op->ldg * sizeof(double);
  }
  pinv_log("quantize_inverse: bits=%d P=%lld", bits, (long long)P);
  return PINV_OK;
}

int32_t pinv_prepare_split(pinv_op op, int32_t mode, void* stream) {
  if (!op) return PINV_E_INVALID_ARG;
  if (mode != PINV_FP32 && mode != PINV_BF16X3 && mode != PINV_BF16X6 && mode != PINV_FP64_SYM &&
      mode != PINV_FIX16_TILE)
    return PINV_E_INVALID_ARG;
  if (!op->G) return PINV_E_STATE;
  hipStream_t s = as_stream(stream);
  if (mode == PINV_FIX16_TILE) {
    // G's integers and exponents for the apply, G^T's for the adjoint
    if (!op->Gt16) {
      const size_t qb = (size_t)op->n * (size_t)tile16_ld(op->n) * sizeof(int16_t);
      const size_t eb = (size_t)tile16_tiles(op->n) * (size_t)tile16_tiles(op->n) * sizeof(int32_t);
      void* p[4] = {nullptr, nullptr, nullptr, nullptr};
      hipError_t e = hipSuccess;
      for (int k = 0; k < 4 && e == hipSuccess; ++k) e = hipMalloc(&p[k], (k & 1) ? eb : qb);
      if (e != hipSuccess) {
        for (void* q : p)
          if (q) (void)hipFree(q);
        return pinv_hip_status(e);
      }
      op->Gt16 = (int16_t*)p[0];
      op->Et16 = (int32_t*)p[1];
      op->Gt16T = (int16_t*)p[2];
      op->Et16T = (int32_t*)p[3];
      op->bytes += (int64_t)(2 * (qb + eb));
    }
    PINV_HIP_TRY(launch_quantize_tiles16(op->G, op->ldg, op->n, 0, op->Gt16, op->Et16, s));
    PINV_HIP_TRY(launch_quantize_tiles16(op->G, op->ldg, op->n, 1, op->Gt16T, op->Et16T, s));
    PINV_HIP_TRY(hipStreamSynchronize(s));
    return PINV_OK;
  }
  if (mode == PINV_FP64_SYM) {
    // only a G symmetric to 1e-12 (relative to its diagonal) may be stored as
    // its upper triangle
    int* flag = nullptr;
    PINV_HIP_TRY(hipMalloc(&flag, sizeof(int)));
    int hflag = 0;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
    if (e == hipSuccess) e = launch_sym_check(op->G, op->ldg, op->n, 1e-12, flag, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(flag);
    if (e != hipSuccess) return pinv_hip_status(e);
    if (hflag) return PINV_E_UNSUPPORTED;
    if (!op->Gsym) {
      const size_t bytes = sym_packed_elems(op->n) * sizeof(double);
      PINV_HIP_TRY(hipMalloc(&op->Gsym, bytes));
      op->bytes += (int64_t)bytes;
    }
    PINV_HIP_TRY(launch_pack_upper(op->G, op->ldg, op->n, op->Gsym, s));
    PINV_HIP_TRY(hipStreamSynchronize(s));
    return PINV_OK;
  }
  const int64_t P = pinv_pad_dim(op->n);
  const size_t elems = (size_t)P * P;  // zero-padded P x P planes
  if (mode == PINV_FP32) {
    if (!op->G32) {
      PINV_HIP_TRY(hipMalloc(&op->G32, elems * sizeof(float)));
      op->bytes += (int64_t)(elems * sizeof(float));
    }
    PINV_HIP_TRY(launch_make_fp32(op->G, op->ldg, op->n, op->G32, s));
  } else {
    const int parts = mode == PINV_BF16X3 ? 2 : 3;
    if (op->Gb && op->nbf < parts) {
      (void)hipFree(op->Gb);
      op->bytes -= (int64_t)(op->nbf * elems * sizeof(__bf16));
      op->Gb = nullptr;
      op->nbf = 0;
    }
    if (!op->Gb) {
      PINV_HIP_TRY(hipMalloc(&op->Gb, parts * elems * sizeof(__bf16)));
      op->bytes += (int64_t)(parts * elems * sizeof(__bf16));
      op->nbf = parts;
    }
    PINV_HIP_TRY(launch_make_bf16_parts(op->G, op->ldg, op->n, op->nbf, op->Gb, s));
  }
  PINV_HIP_TRY(hipStreamSynchronize(s));
  return PINV_OK;
}

int32_t pinv_export_tile16(pinv_op op, int16_t* q_host, int32_t* exponents_host, void* stream) {
  if (!op) return PINV_E_INVALID_ARG;
  if (!op->Gt16) return PINV_E_STATE;
  hipStream_t s = as_stream(stream);
  const int n = op->n, tk = tile16_tiles(n);
  if (q_host)
    PINV_HIP_TRY(hipMemcpy2DAsync(q_host, (size_t)n * sizeof(int16_t), op->Gt16,
                                  (size_t)tile16_ld(n) * sizeof(int16_t), (size_t)n * sizeof(int16_t), n,
                                  hipMemcpyDeviceToHost, s));
  if (exponents_host)
    PINV_HIP_TRY(hipMemcpyAsync(exponents_host, op->Et16, (size_t)tk * tk * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PINV_HIP_TRY(hipStreamSynchronize(s));
  return PINV_OK;
}

int32_t pinv_export_quantized(pinv_op op, int8_t* slices_host, int32_t* exponents_host, void* stream) {
  if (!op) return PINV_E_INVALID_ARG;
  if (!op->S) return PINV_E_STATE;
  hipStream_t s = as_stream(stream);
  const int n = op->n;
  if (slices_host)
    for (int p = 0; p < op->S; ++p)
      PINV_HIP_TRY(hipMemcpy2DAsync(slices_host + (int64_t)p * n * n, n, op->Q + (int64_t)p * op->P * op->P, op->P, n,
                                    n, hipMemcpyDeviceToHost, s));
  if (exponents_host)
    PINV_HIP_TRY(hipMemcpyAsync(exponents_host, op->e, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PINV_HIP_TRY(hipStreamSynchronize(s));
  return PINV_OK;
}

// ---- checkpoint: save / load an op ------------------------------------------
namespace {

// File layout (host byte order): the header, then, each present according to
// the flags, node coordinates x [nx] and y [ny] (non-uniform grids), the
// Dirichlet data [nodes], the lift w [n], G [n][n] row-major FP64, the row
// exponents [P] int32 and the digit planes [S][P][P] int8.
constexpr char kMagic[8] = {'P', 'I', 'N', 'V', 'O', 'P', '0', '1'};
enum : int32_t { kHasG = 1, kHasW = 2, kHasUb = 4, kHasQ = 8, kHasXY = 16 };

struct FileHeader {
  char magic[8];
  int32_t version;
  int32_t nx, ny, nz;
  int32_t general, beta;
  int32_t n;
  int32_t flags;
  int32_t S;
  int32_t i8_variant[4];
  int32_t _pad;
  int64_t P;
  double h;
};

int64_t op_nodes(int nx, int ny, int nz) { return (int64_t)nx * ny * (nz > 0 ? nz : 1); }

// bytes of the payload that the header announces
int64_t payload_bytes(const FileHeader& f) {
  int64_t b = 0;
  if (f.flags & kHasXY) b += (int64_t)(f.nx + f.ny) * 8;
  if (f.flags & kHasUb) b += op_nodes(f.nx, f.ny, f.nz) * 8;
  if (f.flags & kHasW) b += (int64_t)f.n * 8;
  if (f.flags & kHasG) b += (int64_t)f.n * f.n * 8;
  if (f.flags & kHasQ) b += f.P * 4 + (int64_t)f.S * f.P * f.P;
  return b;
}

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};

constexpr size_t kChunk = (size_t)64 << 20;

// device -> file in chunks of whole rows (rows of `width` bytes, `pitch` apart)
int32_t write_rows(FILE* f, const void* dev, size_t pitch, size_t width, int64_t rows, std::vector<char>& buf,
                   hipStream_t s) {
  const int64_t per = std::max<int64_t>(1, (int64_t)(kChunk / width));
  for (int64_t r0 = 0; r0 < rows; r0 += per) {
    const int64_t nr = std::min(per, rows - r0);
    buf.resize((size_t)nr * width);
    PINV_HIP_TRY(hipMemcpy2DAsync(buf.data(), width, (const char*)dev + r0 * pitch, pitch, width, (size_t)nr,
                                  hipMemcpyDeviceToHost, s));
    PINV_HIP_TRY(hipStreamSynchronize(s));
    if (std::fwrite(buf.data(), 1, buf.size(), f) != buf.size()) return PINV_E_IO;
  }
  return PINV_OK;
}

// file -> device in chunks of whole rows
int32_t read_rows(FILE* f, void* dev, size_t pitch, size_t width, int64_t rows, std::vector<char>& buf,
                  hipStream_t s) {
  const int64_t per = std::max<int64_t>(1, (int64_t)(kChunk / width));
  for (int64_t r0 = 0; r0 < rows; r0 += per) {
    const int64_t nr = std::min(per, rows - r0);
    buf.resize((size_t)nr * width);
    if (std::fread(buf.data(), 1, buf.size(), f) != buf.size()) return PINV_E_IO;
    PINV_HIP_TRY(hipMemcpy2DAsync((char*)dev + r0 * pitch, pitch, buf.data(), width, width, (size_t)nr,
                                  hipMemcpyHostToDevice, s));
    PINV_HIP_TRY(hipStreamSynchronize(s));
  }
  return PINV_OK;
}

int32_t alloc_read(FILE* f, size_t bytes, void** dev, std::vector<char>& buf, hipStream_t s) {
  PINV_HIP_TRY(hipMalloc(dev, bytes));
  return read_rows(f, *dev, bytes, bytes, 1, buf, s);
}

}  // namespace

int32_t pinv_save(pinv_op op, const char* path, void* stream) {
  if (!op || !path || !*path) return PINV_E_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  FileHeader h{};
  std::memcpy(h.magic, kMagic, 8);
  h.version = 1;
  h.nx = op->nx;
  h.ny = op->ny;
  h.nz = op->nz;
  h.general = op->general;
  h.beta = op->beta;
  h.n = op->n;
  h.h = op->h;
  h.S = op->S;
  h.P = op->S ? op->P : 0;
  for (int i = 0; i < 4; ++i) h.i8_variant[i] = op->i8_variant[i];
  h.flags = (op->G ? kHasG : 0) | (op->w ? kHasW : 0) | (op->ub ? kHasUb : 0) | (op->S ? kHasQ : 0) |
            (op->xc && op->yc ? kHasXY : 0);
  if (!(h.flags & (kHasG | kHasQ))) return PINV_E_STATE;
  PINV_HIP_TRY(hipStreamSynchronize(s));
  File file;
  file.f = std::fopen(path, "wb");
  if (!file.f) return PINV_E_IO;
  if (std::fwrite(&h, sizeof h, 1, file.f) != 1) return PINV_E_IO;
  std::vector<char> buf;
  int32_t st = PINV_OK;
  if (h.flags & kHasXY) {
    st = write_rows(file.f, op->xc, (size_t)h.nx * 8, (size_t)h.nx * 8, 1, buf, s);
    if (st == PINV_OK) st = write_rows(file.f, op->yc, (size_t)h.ny * 8, (size_t)h.ny * 8, 1, buf, s);
  }
  const size_t nodes_b = (size_t)op_nodes(h.nx, h.ny, h.nz) * 8;
  if (st == PINV_OK && (h.flags & kHasUb)) st = write_rows(file.f, op->ub, nodes_b, nodes_b, 1, buf, s);
  if (st == PINV_OK && (h.flags & kHasW)) st = write_rows(file.f, op->w, (size_t)h.n * 8, (size_t)h.n * 8, 1, buf, s);
  if (st == PINV_OK && (h.flags & kHasG))
    st = write_rows(file.f, op->G, (size_t)op->ldg * 8, (size_t)h.n * 8, h.n, buf, s);
  if (st == PINV_OK && (h.flags & kHasQ)) {
    st = write_rows(file.f, op->e, (size_t)h.P * 4, (size_t)h.P * 4, 1, buf, s);
    if (st == PINV_OK) st = write_rows(file.f, op->Q, (size_t)h.P, (size_t)h.P, (int64_t)h.S * h.P, buf, s);
  }
  if (st == PINV_OK && std::fflush(file.f) != 0) st = PINV_E_IO;
  return st;
}

int32_t pinv_load(const char* path, void* stream, pinv_op* out) {
  if (!out) return PINV_E_INVALID_ARG;
  *out = nullptr;
  if (!path || !*path) return PINV_E_INVALID_ARG;
  File file;
  file.f = std::fopen(path, "rb");
  if (!file.f) return PINV_E_IO;
  FileHeader h{};
  if (std::fread(&h, sizeof h, 1, file.f) != 1) return PINV_E_IO;
  // the header and the file's length must agree before anything is allocated
  // (sizes are bounded before they are multiplied)
  constexpr int32_t kMaxSide = (1 << 20) + 2;
  if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != 1 || h.nx < 3 || h.ny < 3 || h.nx > kMaxSide ||
      h.ny > kMaxSide || (h.nz != 0 && (h.nz < 3 || h.nz > kMaxSide)))
    return PINV_E_INVALID_ARG;
  const int64_t n3 = (int64_t)(h.nx - 2) * (h.ny - 2) * (h.nz > 0 ? h.nz - 2 : 1);  // < 2^63
  if (n3 != h.n || h.n > (1 << 20) || !(h.h > 0.0) || !std::isfinite(h.h) ||
      (h.flags & ~(kHasG | kHasW | kHasUb | kHasQ | kHasXY)) != 0 || !(h.flags & (kHasG | kHasQ)) ||
      ((h.flags & kHasQ) ? (h.S < 1 || h.S > 3 || h.P != pinv_pad_dim(h.n)) : (h.S != 0 || h.P != 0)) ||
      ((h.flags & kHasXY) != 0) != (h.general != 0) || (h.general && (h.beta || h.nz != 0)))
    return PINV_E_INVALID_ARG;
  for (int i = 0; i < 4; ++i)
    if (h.i8_variant[i] < 0 || h.i8_variant[i] >= gemm_i8_variants()) return PINV_E_INVALID_ARG;
  if (std::fseek(file.f, 0, SEEK_END) != 0) return PINV_E_IO;
  const long end = std::ftell(file.f);
  if (end < 0 || (int64_t)end != (int64_t)sizeof h + payload_bytes(h)) return PINV_E_INVALID_ARG;
  if (std::fseek(file.f, (long)sizeof h, SEEK_SET) != 0) return PINV_E_IO;

  hipStream_t s = as_stream(stream);
  pinv_grid g2{h.nx, h.ny, h.h};
  pinv_op op = new_op(&g2);
  if (!op) return PINV_E_OOM;
  op->nz = h.nz;
  op->mz = h.nz > 0 ? h.nz - 2 : 1;
  op->n = h.n;
  op->ldg = (op->n + 31) / 32 * 32;
  op->general = h.general;
  op->beta = h.beta;
  for (int i = 0; i < 4; ++i) op->i8_variant[i] = h.i8_variant[i];
  std::vector<char> buf;
  int32_t st = PINV_OK;
  if (h.flags & kHasXY) {
    st = alloc_read(file.f, (size_t)h.nx * 8, (void**)&op->xc, buf, s);
    if (st == PINV_OK) st = alloc_read(file.f, (size_t)h.ny * 8, (void**)&op->yc, buf, s);
    if (st == PINV_OK) op->bytes += (int64_t)(h.nx + h.ny) * 8;
  }
  const size_t nodes_b = (size_t)op_nodes(h.nx, h.ny, h.nz) * 8;
  if (st == PINV_OK && (h.flags & kHasUb)) {
    st = alloc_read(file.f, nodes_b, (void**)&op->ub, buf, s);
    if (st == PINV_OK) op->bytes += (int64_t)nodes_b;
  }
  if (st == PINV_OK && (h.flags & kHasW)) {
    st = alloc_read(file.f, (size_t)h.n * 8, (void**)&op->w, buf, s);
    if (st == PINV_OK) op->bytes += (int64_t)h.n * 8;
  }
  if (st == PINV_OK && (h.flags & kHasG)) {
    const size_t gb = (size_t)op->n * op->ldg * sizeof(double);
    hipError_t e = hipMalloc(&op->G, gb);
    // rows padded with zeros, as at build and import
    if (e == hipSuccess) e = hipMemsetAsync(op->G, 0, gb, s);
    st = pinv_hip_status(e);
    if (st == PINV_OK) {
      op->bytes += (int64_t)gb;
      st = read_rows(file.f, op->G, (size_t)op->ldg * 8, (size_t)h.n * 8, h.n, buf, s);
    }
  }
  if (st == PINV_OK && (h.flags & kHasQ)) {
    const size_t plane_bytes = (size_t)h.S * h.P * h.P;
    hipError_t e = hipMalloc(&op->Q, plane_bytes);
    if (e == hipSuccess) e = hipMalloc(&op->QT, plane_bytes);
    if (e == hipSuccess) e = hipMalloc(&op->e, (size_t)h.P * sizeof(int32_t));
    st = pinv_hip_status(e);
    if (st == PINV_OK) {
      op->S = h.S;
      op->P = h.P;
      op->bytes += 2 * (int64_t)plane_bytes + h.P * (int64_t)sizeof(int32_t);
      st = read_rows(file.f, op->e, (size_t)h.P * 4, (size_t)h.P * 4, 1, buf, s);
    }
    if (st == PINV_OK) st = read_rows(file.f, op->Q, (size_t)h.P, (size_t)h.P, (int64_t)h.S * h.P, buf, s);
    if (st == PINV_OK) st = pinv_hip_status(launch_transpose_planes(op->Q, op->QT, h.S, h.P, s));
  }
  if (st == PINV_OK) st = pinv_hip_status(hipStreamSynchronize(s));
  if (st == PINV_OK) st = detect_symmetry(op, s);
  if (st != PINV_OK) {
    free_op(op);
    return st;
  }
  pinv_log("load: %s n=%d flags=%d S=%d", path, op->n, h.flags, op->S);
  *out = op;
  return PINV_OK;
}

namespace {
// u = -h^2 G x + bias from the symmetric-packed copy (also the adjoint: G = G^T)
int32_t sym_apply(pinv_op op, const double* X, int64_t ldx, int nrhs, const double* bias, double* U, int64_t ldu,
                  hipStream_t s) {
  if (!op->Gsym) return PINV_E_STATE;
  configure_pool_once();
  void* Y = nullptr;
  PINV_HIP_TRY(hipMallocAsync(&Y, sym_scratch_bytes(op->n, nrhs), s));
  hipError_t e;
  {
    TraceScope ts("gemv_sym", s);
    e = launch_gemv_sym(op->Gsym, op->n, X, ldx, nrhs, -(op->h * op->h), bias, U, ldu, (double*)Y, s);
  }
  const hipError_t e2 = hipFreeAsync(Y, s);
  if (e != hipSuccess) return pinv_hip_status(e);
  return pinv_hip_status(e2);
}
}  // namespace

int32_t pinv_apply_inverse(pinv_op op, int32_t mode, int32_t rho_bits, const double* rho, int64_t ld_rho,
                           int32_t nrhs, double* u, int64_t ld_u, void* stream) {
  int32_t st = check_vectors(op, rho, ld_rho, nrhs, u, ld_u);
  if (st != PINV_OK || nrhs == 0) return st;
  hipStream_t s = as_stream(stream);
  switch (mode) {
    case PINV_FP64:
      if (!op->G) return PINV_E_STATE;
      return fp64_apply(op, false, rho, ld_rho, nrhs, op->w, u, ld_u, s);
    case PINV_FP64_SYM:
      return sym_apply(op, rho, ld_rho, nrhs, op->w, u, ld_u, s);
    case PINV_FIX16_TILE: {
      if (!op->Gt16) return PINV_E_STATE;
      TraceScope ts("gemv_tile16", s);
      return pinv_hip_status(
          launch_gemv_tile16(op->Gt16, op->Et16, op->n, rho, ld_rho, nrhs, op->h, op->w, u, ld_u, s));
    }
    case PINV_INT8: {
      const int SR = slices_of_bits(rho_bits);
      if (!SR) return PINV_E_INVALID_ARG;
      if (!op->S) return PINV_E_STATE;
      if (!int8_total_ok(op->n, op->S, SR)) return PINV_E_UNSUPPORTED;
      return int8_apply(op, op->Q, op->e, nullptr, SR, rho, ld_rho, nrhs, op->w, u, ld_u, s);
    }
    case PINV_FP32:
    case PINV_BF16X3:
    case PINV_BF16X6: {
      if (mode == PINV_FP32 ? !op->G32 : (!op->Gb || op->nbf < (mode == PINV_BF16X3 ? 2 : 3))) return PINV_E_STATE;
      configure_pool_once();
      const size_t sb = split_scratch_bytes(mode, op, nrhs);
      void* scratch = nullptr;
      PINV_HIP_TRY(hipMallocAsync(&scratch, sb ? sb : 256, s));
      hipError_t e;
      {
        TraceScope ts("gemm_split", s);
        e = launch_gemm_split(mode, op, rho, ld_rho, nrhs, -(op->h * op->h), u, ld_u, s, scratch, sb);
      }
      hipError_t e2 = hipFreeAsync(scratch, s);
      if (e != hipSuccess) return pinv_hip_status(e);
      return pinv_hip_status(e2);
    }
    default:
      return PINV_E_INVALID_ARG;
  }
}

int32_t pinv_apply_inverse_noalloc(pinv_op op, int32_t rho_bits, const double* rho, int64_t ld_rho, int32_t nrhs,
                                   double* u, int64_t ld_u, void* stream) {
  int32_t st = check_vectors(op, rho, ld_rho, nrhs, u, ld_u);
  if (st != PINV_OK || nrhs == 0) return st;
  const int SR = slices_of_bits(rho_bits);
  if (!SR) return PINV_E_INVALID_ARG;
  if (!op->S) return PINV_E_STATE;
  // one int32 accumulation over the whole of k must not overflow (a k split
  // would need a partial-sum buffer)
  if (!int8_headroom_ok(op->n, op->S, SR)) return PINV_E_UNSUPPORTED;
  int dev = 0;
  PINV_HIP_TRY(hipGetDevice(&dev));
  if (dev != op->device) return PINV_E_INVALID_ARG;
  const int Rpad = (nrhs + 127) / 128 * 128;
  const size_t xq_bytes = ((size_t)SR * Rpad * op->P + 255) / 256 * 256;
  const size_t f_bytes = (size_t)Rpad * sizeof(int32_t);
  if (xq_bytes + f_bytes > PINV_NOALLOC_SCRATCH_BYTES) {
    pinv_log("pinv_apply_inverse_noalloc: %zu bytes of scratch needed (%d right-hand sides, %d-bit, %lld padded "
             "unknowns), more than the %zu bytes held",
             xq_bytes + f_bytes, nrhs, rho_bits, (long long)op->P, (size_t)PINV_NOALLOC_SCRATCH_BYTES);
    return PINV_E_OOM;
  }
  void* ptr = nullptr;
  st = noalloc_scratch(&ptr);
  if (st != PINV_OK) return st;
  // the quantisation writes every byte of Xq and f the product reads, so
  // nothing has to start at zero; k is not split (the integer class sums are
  // exact in any order, so the result equals pinv_apply_inverse's)
  const hipError_t e = int8_launch(op, op->Q, op->e, nullptr, SR, rho, ld_rho, nrhs, op->w, u, ld_u, Rpad,
                                   op->i8_variant[SR], 1, (int)op->P, 0, (int8_t*)ptr,
                                   (int32_t*)((char*)ptr + xq_bytes), nullptr, as_stream(stream), false);
  return pinv_hip_status(e);
}

int32_t pinv_apply_inverse_adjoint(pinv_op op, int32_t mode, int32_t g_bits, const double* g, int64_t ld_g,
                                   int32_t nrhs, double* lambda, int64_t ld_lambda, void* stream) {
  int32_t st = check_vectors(op, g, ld_g, nrhs, lambda, ld_lambda);
  if (st != PINV_OK || nrhs == 0) return st;
  hipStream_t s = as_stream(stream);
  switch (mode) {
    case PINV_FP64:
      if (!op->G) return PINV_E_STATE;
      return fp64_apply(op, true, g, ld_g, nrhs, nullptr, lambda, ld_lambda, s);
    case PINV_FP64_SYM:
      return sym_apply(op, g, ld_g, nrhs, nullptr, lambda, ld_lambda, s);
    case PINV_FIX16_TILE: {
      if (!op->Gt16T) return PINV_E_STATE;
      TraceScope ts("gemv_tile16", s);
      return pinv_hip_status(
          launch_gemv_tile16(op->Gt16T, op->Et16T, op->n, g, ld_g, nrhs, op->h, nullptr, lambda, ld_lambda, s));
    }
    case PINV_INT8: {
      const int SR = slices_of_bits(g_bits);
      if (!SR) return PINV_E_INVALID_ARG;
      if (!op->S) return PINV_E_STATE;
      if (!int8_total_ok(op->n, op->S, SR)) return PINV_E_UNSUPPORTED;
      return int8_apply(op, op->QT, nullptr, op->e, SR, g, ld_g, nrhs, nullptr, lambda, ld_lambda, s);
    }
    default:
      return PINV_E_UNSUPPORTED;
  }
}

int32_t pinv_grad_eps(pinv_op op, const double* u, int64_t ld_u, const double* lambda, int64_t ld_lambda,
                      int32_t nrhs, double* grad_nodes, void* stream) {
  if (!op || !grad_nodes || nrhs < 0) return PINV_E_INVALID_ARG;
  if (nrhs > 0 && (!u || !lambda || ld_u < op->n || ld_lambda < op->n)) return PINV_E_INVALID_ARG;
  if (op->general || op->beta) return PINV_E_UNSUPPORTED;
  hipStream_t s = as_stream(stream);
  const int chunks = grad_eps_chunks(nrhs);
  const size_t nodes = (size_t)op->nx * op->ny * (op->nz ? op->nz : 1);
  void* part = nullptr;
  if (chunks > 1) {
    configure_pool_once();
    PINV_HIP_TRY(hipMallocAsync(&part, (size_t)chunks * nodes * sizeof(double), s));
  }
  hipError_t e;
  {
    TraceScope ts("grad_eps", s);
    e = launch_grad_eps(op->nx, op->ny, op->nz, op->h, u, ld_u, lambda, ld_lambda, nrhs, op->ub, (double*)part, grad_nodes,
                        s);
  }
  const hipError_t e2 = part ? hipFreeAsync(part, s) : hipSuccess;
  if (e != hipSuccess) return pinv_hip_status(e);
  return pinv_hip_status(e2);
}

int32_t pinv_grad_eps_general(pinv_op op, const double* u, int64_t ld_u, const double* lambda, int64_t ld_lambda,
                              int32_t nrhs, double* grad_x, double* grad_y, void* stream) {
  if (!op || !grad_x || nrhs < 0 || grad_x == grad_y) return PINV_E_INVALID_ARG;
  if (nrhs > 0 && (!u || !lambda || ld_u < op->n || ld_lambda < op->n)) return PINV_E_INVALID_ARG;
  if (!op->general || !op->xc || !op->yc) return PINV_E_UNSUPPORTED;
  hipStream_t s = as_stream(stream);
  const int chunks = grad_eps_chunks(nrhs);
  const size_t nodes = (size_t)op->nx * op->ny;
  void* part = nullptr;
  if (chunks > 1) {
    configure_pool_once();
    PINV_HIP_TRY(hipMallocAsync(&part, 2 * (size_t)chunks * nodes * sizeof(double), s));
  }
  hipError_t e;
  {
    TraceScope ts("grad_eps", s);
    e = launch_grad_eps_general(op->nx, op->ny, op->xc, op->yc, u, ld_u, lambda, ld_lambda, nrhs, op->ub,
                                (double*)part, grad_x, grad_y, s);
  }
  const hipError_t e2 = part ? hipFreeAsync(part, s) : hipSuccess;
  if (e != hipSuccess) return pinv_hip_status(e);
  return pinv_hip_status(e2);
}

int32_t pinv_grad_beta(pinv_op op, const double* u, int64_t ld_u, const double* lambda, int64_t ld_lambda,
                       int32_t nrhs, double* grad_beta, void* stream) {
  if (!op || !grad_beta || nrhs < 0) return PINV_E_INVALID_ARG;
  if (nrhs > 0 && (!u || !lambda || ld_u < op->n || ld_lambda < op->n)) return PINV_E_INVALID_ARG;
  if (!op->beta) return PINV_E_UNSUPPORTED;
  hipStream_t s = as_stream(stream);
  const int chunks = grad_eps_chunks(nrhs);
  const size_t nodes = (size_t)op->nx * op->ny;
  void* part = nullptr;
  if (chunks > 1) {
    configure_pool_once();
    PINV_HIP_TRY(hipMallocAsync(&part, 4 * (size_t)chunks * nodes * sizeof(double), s));
  }
  hipError_t e;
  {
    TraceScope ts("grad_eps", s);
    e = launch_grad_beta(op->nx, op->ny, u, ld_u, lambda, ld_lambda, nrhs, op->ub, (double*)part, grad_beta, s);
  }
  const hipError_t e2 = part ? hipFreeAsync(part, s) : hipSuccess;
  if (e != hipSuccess) return pinv_hip_status(e);
  return pinv_hip_status(e2);
}

int32_t pinv_apply_batched(const pinv_request* reqs, int32_t nreq, int32_t mode, int32_t rho_bits, void* stream) {
  if (nreq < 0 || (nreq > 0 && !reqs)) return PINV_E_INVALID_ARG;
  // every request is checked before anything is launched
  for (int i = 0; i < nreq; ++i) {
    const pinv_request& r = reqs[i];
    if (!r.op) return PINV_E_INVALID_ARG;
    const int32_t st = check_vectors(r.op, r.rho, r.ld, r.nrhs, r.u, r.ld);
    if (st != PINV_OK) return st;
  }
  if (mode != PINV_INT8) {
    for (int i = 0; i < nreq; ++i) {
      const int32_t st = pinv_apply_inverse(reqs[i].op, mode, rho_bits, reqs[i].rho, reqs[i].ld, reqs[i].nrhs,
                                            reqs[i].u, reqs[i].ld, stream);
      if (st != PINV_OK) return st;
    }
    return PINV_OK;
  }
  const int SR = slices_of_bits(rho_bits);
  if (!SR) return PINV_E_INVALID_ARG;
  bool any = false;
  for (int i = 0; i < nreq; ++i) {
    if (reqs[i].nrhs == 0) continue;
    if (!reqs[i].op->S) return PINV_E_STATE;
    if (!int8_headroom_ok(reqs[i].op->n, reqs[i].op->S, SR)) return PINV_E_UNSUPPORTED;
    any = true;
  }
  if (!any) return PINV_OK;
  hipStream_t s = as_stream(stream);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  BatchPlan* plan = nullptr;
  const int32_t st = find_or_make_plan(reqs, nreq, SR, s, &plan);
  if (st != PINV_OK) return st;
  return pinv_hip_status(run_plan(*plan, SR, s));
}

int32_t pinv_batched_release(void) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  if (g_plans().empty()) return PINV_OK;
  const hipError_t e = hipDeviceSynchronize();
  for (BatchPlan* p : g_plans()) free_plan(p);
  g_plans().clear();
  return pinv_hip_status(e);
}

int32_t pinv_get_info(pinv_op op, pinv_info* info) {
  if (!op || !info) return PINV_E_INVALID_ARG;
  info->nx = op->nx;
  info->ny = op->ny;
  info->n = op->n;
  info->h = op->h;
  info->has_fp64 = op->G != nullptr;
  info->int8_slices = op->S;
  info->has_fp32 = op->G32 != nullptr;
  info->has_bf16 = op->nbf;
  info->has_lift = op->w != nullptr;
  info->device_bytes = op->bytes;
  info->nz = op->nz;
  info->beta = op->beta;
  info->has_sym = op->Gsym != nullptr;
  info->has_tile16 = op->Gt16 != nullptr;
  info->general = op->general;
  info->fp64_symmetric = op->G != nullptr && op->g_symmetric;
  return PINV_OK;
}

int32_t pinv_int8_variants(void) { return gemm_i8_variants(); }

int32_t pinv_set_int8_variant(pinv_op op, int32_t rho_bits, int32_t variant) {
  const int SR = slices_of_bits(rho_bits);
  if (!op || !SR || variant < 0 || variant >= gemm_i8_variants()) return PINV_E_INVALID_ARG;
  op->i8_variant[SR] = variant;
  return PINV_OK;
}

int32_t pinv_autotune_int8(pinv_op op, int32_t rho_bits, const double* rho, int64_t ld_rho, int32_t nrhs,
                           int32_t reps, double* variant_ms, int32_t n_ms, int32_t* best, void* stream) {
  const int SR = slices_of_bits(rho_bits);
  if (!op || !SR || nrhs <= 0 || reps <= 0 || n_ms < 0 || (n_ms > 0 && !variant_ms)) return PINV_E_INVALID_ARG;
  if (rho && ld_rho < op->n) return PINV_E_INVALID_ARG;
  if (!op->S) return PINV_E_STATE;
  hipStream_t s = as_stream(stream);
  const int Rpad = (nrhs + 127) / 128 * 128;
  const int nv = gemm_i8_variants();
  // a stored choice for this device kind and problem, if a cache file is named
  const char* cache = std::getenv("PINV_AUTOTUNE_CACHE");
  std::string dkey;
  if (cache && *cache) {
    dkey = tune_device_key(op->device);
    int v = 0;
    double vms = 0.0;
    if (tune_cache_lookup(cache, dkey, op->n, op->S, SR, Rpad, nv, &v, &vms)) {
      for (int i = 0; i < n_ms; ++i) variant_ms[i] = i == v ? vms : -1.0;
      op->i8_variant[SR] = v;
      if (best) *best = v;
      pinv_log("autotune_int8: n=%d S=%d SR=%d Rpad=%d: variant %d from %s", op->n, op->S, SR, Rpad, v, cache);
      return PINV_OK;
    }
  }
  // every variant is timed with the k split its applies would use
  std::vector<int> ksplit(nv, 1), kchunk(nv, (int)op->P), tail(nv, 0);
  size_t part_bytes = 0;
  for (int v = 0; v < nv; ++v) {
    int8_split(op, SR, Rpad, v, &ksplit[v], &kchunk[v], &tail[v]);
    part_bytes = std::max(part_bytes, gemm_i8_part_bytes(op->P, Rpad, v, op->S + SR - 1, ksplit[v], tail[v]));
  }
  const size_t xq_bytes = (size_t)SR * Rpad * op->P;
  const size_t f_bytes = ((size_t)Rpad * sizeof(int32_t) + 255) / 256 * 256;
  const size_t u_bytes = ((size_t)nrhs * op->n * sizeof(double) + 255) / 256 * 256;
  char* buf = nullptr;
  PINV_HIP_TRY(hipMalloc(&buf, xq_bytes + f_bytes + u_bytes + part_bytes));
  int8_t* Xq = (int8_t*)buf;
  int32_t* f = (int32_t*)(buf + xq_bytes);
  double* U = (double*)(buf + xq_bytes + f_bytes);
  int32_t* part = (int32_t*)(buf + xq_bytes + f_bytes + u_bytes);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipError_t e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  if (rho) {
    if (e == hipSuccess) e = launch_quantize_cols(rho, ld_rho, nullptr, op->n, nrhs, Rpad, SR, op->P, nullptr, Xq, f, s);
  } else {
    if (e == hipSuccess) e = launch_fill_random_i8(Xq, xq_bytes, 12345u, s);
    if (e == hipSuccess) e = hipMemsetAsync(f, 0, f_bytes, s);
  }
  GemmI8Args a{};
  a.Q = op->Q; a.S = op->S;
  a.X = Xq; a.SR = SR;
  a.P = op->P; a.Rpad = Rpad;
  a.n = op->n; a.nrhs = nrhs;
  a.row_exp = op->e;
  a.col_exp = f;
  a.c = -(op->h * op->h) / ((double)pinv_max_mag(op->S) * (double)pinv_max_mag(SR));
  a.w = nullptr;
  a.U = U; a.ldu = op->n;
  // three rounds over all variants (so that clock drift during the call does
  // not favour one position); each variant keeps its best round
  std::vector<double> t(nv, 0.0);
  for (int round = 0; round < 3 && e == hipSuccess; ++round) {
    for (int v = 0; v < nv && e == hipSuccess; ++v) {
      a.variant = v;
      a.ksplit = ksplit[v];
      a.kchunk = kchunk[v];
      a.part = ksplit[v] > 1 ? part : nullptr;
      a.tail_rows = ksplit[v] > 1 ? tail[v] : 0;
      e = launch_gemm_i8(a, s);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(ev0, s);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_gemm_i8(a, s);
      if (e == hipSuccess) e = hipEventRecord(ev1, s);
      if (e == hipSuccess) e = hipEventSynchronize(ev1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
      if (e != hipSuccess) break;
      const double avg = (double)ms / reps;
      if (round == 0 || avg < t[v]) t[v] = avg;
    }
  }
  int pick = 0;
  for (int v = 0; v < nv; ++v) {
    if (v < n_ms) variant_ms[v] = t[v];
    if (t[v] < t[pick]) pick = v;
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  const hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return pinv_hip_status(e);
  op->i8_variant[SR] = pick;
  if (best) *best = pick;
  if (cache && *cache) tune_cache_store(cache, dkey, op->n, op->S, SR, Rpad, pick, t[pick]);
  return PINV_OK;
}

int32_t pinv_trace_enable(int32_t on) {
  g_trace_on.store(on ? 1 : 0);
  return PINV_OK;
}

int32_t pinv_trace_read(const char* kernel, double* total_ms, int64_t* launches) {
  return pinv_trace_read_each(kernel, nullptr, 0, total_ms, launches);
}

int32_t pinv_trace_read_each(const char* kernel, double* ms_each, int64_t cap, double* total_ms,
                             int64_t* launches) {
  if (!kernel || cap < 0 || (cap > 0 && !ms_each)) return PINV_E_INVALID_ARG;
  double tot = 0.0;
  int64_t cnt = 0;
  int32_t st = PINV_OK;
  std::lock_guard<std::mutex> lk(g_trace_mu);
  std::vector<TraceRec> keep;
  keep.reserve(g_trace.size());
  for (const TraceRec& r : g_trace) {
    if (std::strcmp(r.name, kernel) != 0) {
      keep.push_back(r);
      continue;
    }
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) st = pinv_hip_status(e);
    tot += ms;
    if (cnt < cap) ms_each[cnt] = ms;
    ++cnt;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_trace.swap(keep);
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return st;
}

int32_t pinv_destroy(pinv_op op) {
  if (!op) return PINV_E_INVALID_ARG;
  free_op(op);
  return PINV_OK;
}

}  // extern "C"
