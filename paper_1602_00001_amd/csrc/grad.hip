// Permittivity gradient of a loss through the solve (not in the paper).
//
// For a face f = (p, q) of the operator, dLoss/deps_f = (1/h^2) sum_r
// (lambda_p - lambda_q)(u_p - u_q), with lambda the adjoint output
// (dLoss/drho) and u the forward solution; a boundary node carries
// lambda = 0 and its Dirichlet value.  eps_f is the mean of the two nodal
// values, so a node receives half of the gradient of each face it touches.
// Faces that join two boundary nodes are not part of the operator.
//
// One thread per node; for each right-hand side the threads of a wave read
// consecutive nodes, so the loads are coalesced.  Each node sums its own
// faces in a fixed order (deterministic).

#include "common.h"

namespace {

__global__ __launch_bounds__(256) void grad_eps_kernel(int nx, int ny, double h, const double* __restrict__ u,
                                                      int64_t ldu, const double* __restrict__ lam, int64_t ldl,
                                                      int nrhs, const double* __restrict__ ub,
                                                      double* __restrict__ grad) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nx * ny) return;
  const int i = node / nx, j = node % nx;
  const int mx = nx - 2;
  const bool bp = (i == 0 || i == ny - 1 || j == 0 || j == nx - 1);
  const int ni[4] = {i - 1, i + 1, i, i};
  const int nj[4] = {j, j, j - 1, j + 1};
  const int64_t pp = bp ? -1 : (int64_t)(i - 1) * mx + (j - 1);
  const double ubp = (bp && ub) ? ub[node] : 0.0;
  double total = 0.0;
  for (int t = 0; t < 4; ++t) {
    const int k = ni[t], l = nj[t];
    if (k < 0 || k >= ny || l < 0 || l >= nx) continue;
    const bool bq = (k == 0 || k == ny - 1 || l == 0 || l == nx - 1);
    if (bp && bq) continue;
    const int64_t qq = bq ? -1 : (int64_t)(k - 1) * mx + (l - 1);
    const double ubq = (bq && ub) ? ub[(int64_t)k * nx + l] : 0.0;
    double sf = 0.0;
    for (int r = 0; r < nrhs; ++r) {
      const double up = bp ? ubp : u[(int64_t)r * ldu + pp];
      const double uq = bq ? ubq : u[(int64_t)r * ldu + qq];
      const double lp = bp ? 0.0 : lam[(int64_t)r * ldl + pp];
      const double lq = bq ? 0.0 : lam[(int64_t)r * ldl + qq];
      sf += (lp - lq) * (up - uq);
    }
    total += sf;
  }
  grad[node] = 0.5 * total / (h * h);
}

}  // namespace

hipError_t launch_grad_eps(int nx, int ny, double h, const double* u, int64_t ldu, const double* lam, int64_t ldl,
                           int nrhs, const double* ub, double* grad, hipStream_t s) {
  const int nodes = nx * ny;
  hipLaunchKernelGGL(grad_eps_kernel, dim3((nodes + 255) / 256), dim3(256), 0, s, nx, ny, h, u, ldu, lam, ldl, nrhs,
                     ub, grad);
  return hipGetLastError();
}
