// Permittivity gradient of a loss through the solve (not in the paper).
//
// For a face f = (p, q) of the operator, dLoss/deps_f = (1/h^2) sum_r
// (lambda_p - lambda_q)(u_p - u_q), with lambda the adjoint output
// (dLoss/drho) and u the forward solution; a boundary node carries
// lambda = 0 and its Dirichlet value.  eps_f is the mean of the two nodal
// values, so a node receives half of the gradient of each face it touches.
// Faces that join two boundary nodes are not part of the operator.
//
// The right-hand sides are split into chunks of RC; workgroup (b, c) takes 256
// nodes and chunk c, one thread per node: for each of its right-hand sides the
// thread reads its own (u, lambda) and those of its four neighbours (the
// threads of a wave read consecutive nodes, so the loads are coalesced and the
// neighbours' come from cache) and adds the four face products.  Each chunk's
// partial sums go to scratch; a second kernel adds the chunks in order and
// scales.  Every sum has a fixed order, so the result is deterministic.

#include "common.h"

namespace {

constexpr int RC = 16;

__global__ __launch_bounds__(256) void grad_eps_partial_kernel(int nx, int ny, double h, const double* __restrict__ u,
                                                              int64_t ldu, const double* __restrict__ lam,
                                                              int64_t ldl, int nrhs, const double* __restrict__ ub,
                                                              double* __restrict__ out, int final_scale) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  const int nodes = nx * ny;
  if (node >= nodes) return;
  const int r0 = blockIdx.y * RC;
  const int r1 = min(nrhs, r0 + RC);
  const int i = node / nx, j = node % nx;
  const int mx = nx - 2;
  const bool bp = (i == 0 || i == ny - 1 || j == 0 || j == nx - 1);
  const int ni[4] = {i - 1, i + 1, i, i};
  const int nj[4] = {j, j, j - 1, j + 1};
  const int64_t pp = bp ? 0 : (int64_t)(i - 1) * mx + (j - 1);
  const double ubp = (bp && ub) ? ub[node] : 0.0;
  bool use[4], bq[4];
  int64_t qq[4];
  double ubq[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = ni[t], l = nj[t];
    const bool inside = k >= 0 && k < ny && l >= 0 && l < nx;
    bq[t] = !inside || k == 0 || k == ny - 1 || l == 0 || l == nx - 1;
    use[t] = inside && !(bp && bq[t]);
    qq[t] = bq[t] ? 0 : (int64_t)(k - 1) * mx + (l - 1);
    ubq[t] = (use[t] && bq[t] && ub) ? ub[(int64_t)k * nx + l] : 0.0;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = r0; r < r1; ++r) {
    const double* ur = u + (int64_t)r * ldu;
    const double* lr = lam + (int64_t)r * ldl;
    const double up = bp ? ubp : ur[pp];
    const double lp = bp ? 0.0 : lr[pp];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (!use[t]) continue;
      const double uq = bq[t] ? ubq[t] : ur[qq[t]];
      const double lq = bq[t] ? 0.0 : lr[qq[t]];
      acc[t] += (lp - lq) * (up - uq);
    }
  }
  const double total = ((acc[0] + acc[1]) + acc[2]) + acc[3];
  if (final_scale)
    out[node] = 0.5 * total / (h * h);
  else
    out[(int64_t)blockIdx.y * nodes + node] = total;
}

__global__ __launch_bounds__(256) void grad_eps_reduce_kernel(int nodes, int chunks, double h,
                                                             const double* __restrict__ part,
                                                             double* __restrict__ grad) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nodes) return;
  double total = 0.0;
  for (int c = 0; c < chunks; ++c) total += part[(int64_t)c * nodes + node];
  grad[node] = 0.5 * total / (h * h);
}

}  // namespace

int grad_eps_chunks(int nrhs) { return (nrhs + RC - 1) / RC; }

hipError_t launch_grad_eps(int nx, int ny, double h, const double* u, int64_t ldu, const double* lam, int64_t ldl,
                           int nrhs, const double* ub, double* part, double* grad, hipStream_t s) {
  const int nodes = nx * ny;
  const int chunks = grad_eps_chunks(nrhs);
  const dim3 blocks((nodes + 255) / 256);
  if (chunks <= 1) {
    // zero or one chunk: the partial kernel writes the scaled result directly
    hipLaunchKernelGGL(grad_eps_partial_kernel, dim3(blocks.x, 1), dim3(256), 0, s, nx, ny, h, u, ldu, lam, ldl,
                       nrhs, ub, grad, 1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(grad_eps_partial_kernel, dim3(blocks.x, chunks), dim3(256), 0, s, nx, ny, h, u, ldu, lam, ldl,
                     nrhs, ub, part, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(grad_eps_reduce_kernel, blocks, dim3(256), 0, s, nodes, chunks, h, part, grad);
  return hipGetLastError();
}
