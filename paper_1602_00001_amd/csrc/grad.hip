// Permittivity gradient of a loss through the solve (not in the paper).
//
// For a face f = (p, q) of the operator, dLoss/deps_f = (1/h^2) sum_r
// (lambda_p - lambda_q)(u_p - u_q), with lambda the adjoint output
// (dLoss/drho) and u the forward solution; a boundary node carries
// lambda = 0 and its Dirichlet value.  eps_f is the mean of the two nodal
// values, so a node receives half of the gradient of each face it touches.
// Faces that join two boundary nodes are not part of the operator.
//
// The right-hand sides are split into chunks of RC; a workgroup takes 256
// nodes and one chunk, one thread per node, and for each right-hand side adds
// the products of the node's faces.  The 3-D form reads each node's own
// (u, lambda) and its 6 neighbours' from global memory (the threads of a wave
// read consecutive nodes, so the loads are coalesced and the neighbours' come
// from cache); the 2-D form stages a tile with its halo in LDS first.  Each
// chunk's partial sums go to scratch; a second kernel adds the chunks in order
// and scales.  Every sum has a fixed order, so the result is deterministic.

#include "common.h"

namespace {

constexpr int RC = 16;

// D = 2: nodes [n_y][n_x], 4 faces per node; D = 3: nodes [n_z][n_y][n_x]
// (slowest axis z), 6 faces per node.  Interior vectors follow the operator's
// row-major interior order.
template <int D>
__global__ __launch_bounds__(256) void grad_eps_partial_kernel(int nx, int ny, int nz, double h,
                                                              const double* __restrict__ u, int64_t ldu,
                                                              const double* __restrict__ lam, int64_t ldl, int nrhs,
                                                              const double* __restrict__ ub,
                                                              double* __restrict__ out, int final_scale) {
  constexpr int F = 2 * D;
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  const int nodes = nx * ny * (D == 3 ? nz : 1);
  if (node >= nodes) return;
  const int r0 = blockIdx.y * RC;
  const int r1 = min(nrhs, r0 + RC);
  const int j = node % nx;
  const int i = (node / nx) % ny;
  const int k = D == 3 ? node / (nx * ny) : 0;
  const int mx = nx - 2, my = ny - 2;
  const int zlo = D == 3 ? 0 : -1, zhi = D == 3 ? nz - 1 : -1;  // no z boundary in 2-D
  auto boundary = [&](int c, int a, int b) { return c == zlo || c == zhi || a == 0 || a == ny - 1 || b == 0 || b == nx - 1; };
  auto interior = [&](int c, int a, int b) {
    return ((int64_t)(D == 3 ? c - 1 : 0) * my + (a - 1)) * mx + (b - 1);
  };
  const bool bp = boundary(k, i, j);
  const int nk[6] = {k, k, k, k, k - 1, k + 1};
  const int ni[6] = {i - 1, i + 1, i, i, i, i};
  const int nj[6] = {j, j, j - 1, j + 1, j, j};
  const int64_t pp = bp ? 0 : interior(k, i, j);
  const double ubp = (bp && ub) ? ub[node] : 0.0;
  bool use[F], bq[F];
  int64_t qq[F];
  double ubq[F];
#pragma unroll
  for (int t = 0; t < F; ++t) {
    const int c = nk[t], a = ni[t], b = nj[t];
    const bool inside = a >= 0 && a < ny && b >= 0 && b < nx && (D == 2 || (c >= 0 && c < nz));
    bq[t] = !inside || boundary(c, a, b);
    use[t] = inside && !(bp && bq[t]);
    qq[t] = bq[t] ? 0 : interior(c, a, b);
    ubq[t] = (use[t] && bq[t] && ub) ? ub[((int64_t)c * ny + a) * nx + b] : 0.0;
  }
  double acc[F];
#pragma unroll
  for (int t = 0; t < F; ++t) acc[t] = 0.0;
  for (int r = r0; r < r1; ++r) {
    const double* ur = u + (int64_t)r * ldu;
    const double* lr = lam + (int64_t)r * ldl;
    const double up = bp ? ubp : ur[pp];
    const double lp = bp ? 0.0 : lr[pp];
#pragma unroll
    for (int t = 0; t < F; ++t) {
      if (!use[t]) continue;
      const double uq = bq[t] ? ubq[t] : ur[qq[t]];
      const double lq = bq[t] ? 0.0 : lr[qq[t]];
      acc[t] += (lp - lq) * (up - uq);
    }
  }
  double total = acc[0];
#pragma unroll
  for (int t = 1; t < F; ++t) total += acc[t];
  if (final_scale)
    out[node] = 0.5 * total / (h * h);
  else
    out[(int64_t)blockIdx.y * nodes + node] = total;
}

// 2-D form with the right-hand side's values staged in LDS: a workgroup takes
// a tile of TY rows x TX columns of nodes; for each right-hand side of its
// chunk the tile and a one-node halo of (u, lambda) are loaded once into LDS
// (u_B and 0 on boundary nodes; coalesced row segments), then each thread
// forms the face products of its node from LDS.  Two LDS buffers alternate,
// so one barrier per right-hand side suffices.  Same products, same order of
// summation as the node kernel above, so the results are identical.
constexpr int TX = 64, TY = 4;
constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;

__global__ __launch_bounds__(256) void grad_eps_tile_kernel(int nx, int ny, double h, const double* __restrict__ u,
                                                           int64_t ldu, const double* __restrict__ lam, int64_t ldl,
                                                           int nrhs, const double* __restrict__ ub,
                                                           double* __restrict__ out, int final_scale) {
  __shared__ double su[2][HN], sl[2][HN];
  const int tilesX = (nx + TX - 1) / TX;
  const int tx0 = (int)(blockIdx.x % tilesX) * TX, ty0 = (int)(blockIdx.x / tilesX) * TY;
  const int r0 = blockIdx.y * RC;
  const int r1 = min(nrhs, r0 + RC);
  const int tid = threadIdx.x;
  const int mx = nx - 2;
  auto boundary = [&](int a, int b) { return a == 0 || a == ny - 1 || b == 0 || b == nx - 1; };

  // staged nodes of this thread: e = tid and tid + 256 (of HN = 396)
  constexpr int SPT = (HN + 255) / 256;
  int64_t off[SPT];
  bool inter[SPT], live[SPT];
  double ubv[SPT];
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int e = tid + 256 * k;
    const int gi = ty0 - 1 + e / HX, gj = tx0 - 1 + e % HX;
    live[k] = e < HN;
    const bool valid = live[k] && gi >= 0 && gi < ny && gj >= 0 && gj < nx;
    inter[k] = valid && !boundary(gi, gj);
    off[k] = inter[k] ? (int64_t)(gi - 1) * mx + (gj - 1) : 0;
    ubv[k] = (valid && !inter[k] && ub) ? ub[(int64_t)gi * nx + gj] : 0.0;
  }

  // this thread's node and its faces (the node kernel's rule)
  const int li = tid / TX, lj = tid % TX;
  const int i = ty0 + li, j = tx0 + lj;
  const bool mine = i < ny && j < nx;
  const bool bp = mine && boundary(i, j);
  const int ni[4] = {i - 1, i + 1, i, i};
  const int nj[4] = {j, j, j - 1, j + 1};
  const int slot_p = (li + 1) * HX + (lj + 1);
  const int dslot[4] = {-HX, HX, -1, 1};
  bool use[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = ni[t], l = nj[t];
    const bool inside = k >= 0 && k < ny && l >= 0 && l < nx;
    const bool bq = !inside || boundary(k, l);
    use[t] = mine && inside && !(bp && bq);
  }

  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = r0; r < r1; ++r) {
    const int b = (r - r0) & 1;
    const double* ur = u + (int64_t)r * ldu;
    const double* lr = lam + (int64_t)r * ldl;
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      // (unconditional loads from a valid offset; the value is selected after)
      const double uv = ur[off[k]];
      const double lv = lr[off[k]];
      if (live[k]) {
        su[b][tid + 256 * k] = inter[k] ? uv : ubv[k];
        sl[b][tid + 256 * k] = inter[k] ? lv : 0.0;
      }
    }
    __syncthreads();
    const double up = su[b][slot_p], lp = sl[b][slot_p];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (!use[t]) continue;
      const double uq = su[b][slot_p + dslot[t]], lq = sl[b][slot_p + dslot[t]];
      acc[t] += (lp - lq) * (up - uq);
    }
  }
  if (!mine) return;
  const int node = i * nx + j;
  const double total = ((acc[0] + acc[1]) + acc[2]) + acc[3];
  if (final_scale)
    out[node] = 0.5 * total / (h * h);
  else
    out[(int64_t)blockIdx.y * nx * ny + node] = total;
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

// Non-uniform tensor grid with a permittivity per direction (the finite-volume
// operator K u = -A rho + b_B, stored inverse K^{-1} diag(A)): the face
// coefficient is eps_f times the geometric factor s_f (cell height / node
// distance for an x-face, cell width / node distance for a y-face), and
// mu = K^{-1} g = -lambda / A, so dLoss/dc_f = sum_r (lambda_p/A_p -
// lambda_q/A_q)(u_p - u_q); each end node receives s_f/2 of it, x-faces in the
// x gradient and y-faces in the y gradient.  Same chunking as above; the
// partial sums go to part[0 (x) or 1 (y)][chunk][node].
__global__ __launch_bounds__(256) void grad_eps_general_partial_kernel(
    int nx, int ny, const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ u,
    int64_t ldu, const double* __restrict__ lam, int64_t ldl, int nrhs, const double* __restrict__ ub,
    double* __restrict__ part, double* __restrict__ gx, double* __restrict__ gy) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  const int nodes = nx * ny;
  if (node >= nodes) return;
  const int r0 = blockIdx.y * RC;
  const int r1 = min(nrhs, r0 + RC);
  const int i = node / nx, j = node % nx;
  const int mx = nx - 2;
  auto boundary = [&](int a, int b) { return a == 0 || a == ny - 1 || b == 0 || b == nx - 1; };
  auto area = [&](int a, int b) { return (0.5 * (x[b + 1] - x[b - 1])) * (0.5 * (y[a + 1] - y[a - 1])); };
  const bool bp = boundary(i, j);
  const int ni[4] = {i - 1, i + 1, i, i};
  const int nj[4] = {j, j, j - 1, j + 1};
  const int64_t pp = bp ? 0 : (int64_t)(i - 1) * mx + (j - 1);
  const double inv_ap = bp ? 0.0 : 1.0 / area(i, j);
  const double ubp = (bp && ub) ? ub[node] : 0.0;
  bool use[4], bq[4];
  int64_t qq[4];
  double ubq[4], inv_aq[4], sf[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = ni[t], l = nj[t];
    const bool inside = k >= 0 && k < ny && l >= 0 && l < nx;
    bq[t] = !inside || boundary(k, l);
    use[t] = inside && !(bp && bq[t]);
    qq[t] = bq[t] ? 0 : (int64_t)(k - 1) * mx + (l - 1);
    ubq[t] = (use[t] && bq[t] && ub) ? ub[(int64_t)k * nx + l] : 0.0;
    inv_aq[t] = (use[t] && !bq[t]) ? 1.0 / area(k, l) : 0.0;
    // a used face has an interior end, so the row (x-face) or column (y-face)
    // it lies on is interior and its cell extent is defined
    sf[t] = !use[t] ? 0.0
            : t < 2 ? 0.5 * (x[j + 1] - x[j - 1]) / fabs(y[k] - y[i])
                    : 0.5 * (y[i + 1] - y[i - 1]) / fabs(x[l] - x[j]);
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = r0; r < r1; ++r) {
    const double* ur = u + (int64_t)r * ldu;
    const double* lr = lam + (int64_t)r * ldl;
    const double up = bp ? ubp : ur[pp];
    const double mp = bp ? 0.0 : lr[pp] * inv_ap;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (!use[t]) continue;
      const double uq = bq[t] ? ubq[t] : ur[qq[t]];
      const double mq = bq[t] ? 0.0 : lr[qq[t]] * inv_aq[t];
      acc[t] += (mp - mq) * (up - uq);
    }
  }
  const double sy = sf[0] * acc[0] + sf[1] * acc[1];
  const double sx = sf[2] * acc[2] + sf[3] * acc[3];
  if (part) {
    part[(int64_t)blockIdx.y * nodes + node] = sx;
    part[((int64_t)gridDim.y + blockIdx.y) * nodes + node] = sy;
  } else if (gy) {
    gx[node] = 0.5 * sx;
    gy[node] = 0.5 * sy;
  } else {
    gx[node] = 0.5 * (sx + sy);
  }
}

__global__ __launch_bounds__(256) void grad_eps_general_reduce_kernel(int nodes, int chunks,
                                                                     const double* __restrict__ part,
                                                                     double* __restrict__ gx,
                                                                     double* __restrict__ gy) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nodes) return;
  double sx = 0.0, sy = 0.0;
  for (int c = 0; c < chunks; ++c) {
    sx += part[(int64_t)c * nodes + node];
    sy += part[((int64_t)chunks + c) * nodes + node];
  }
  if (gy) {
    gx[node] = 0.5 * sx;
    gy[node] = 0.5 * sy;
  } else {
    gx[node] = 0.5 * (sx + sy);
  }
}

// Eq. 3's coefficients: dLoss/dbeta_d(p) = (1/4) sum_r lambda_p U_{q_d}
// (lambda = A^{-T} g is the adjoint output; U is u at interior nodes and u_B on
// the boundary).  One thread per node and a chunk of RC right-hand sides per
// workgroup as above; part[chunk][d][node], or the scaled result directly.
__global__ __launch_bounds__(256) void grad_beta_partial_kernel(int nx, int ny, const double* __restrict__ u,
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
  auto boundary = [&](int a, int b) { return a == 0 || a == ny - 1 || b == 0 || b == nx - 1; };
  const bool bp = boundary(i, j);
  const int ni[4] = {i - 1, i + 1, i, i};
  const int nj[4] = {j, j, j - 1, j + 1};
  bool bq[4];
  int64_t qq[4];
  double ubq[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = ni[t], l = nj[t];
    bq[t] = bp || boundary(k, l);  // (unused when p is a boundary node)
    qq[t] = bq[t] ? 0 : (int64_t)(k - 1) * mx + (l - 1);
    ubq[t] = (!bp && bq[t] && ub) ? ub[(int64_t)k * nx + l] : 0.0;
  }
  const int64_t pp = bp ? 0 : (int64_t)(i - 1) * mx + (j - 1);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (!bp) {
    for (int r = r0; r < r1; ++r) {
      const double* ur = u + (int64_t)r * ldu;
      const double lp = lam[(int64_t)r * ldl + pp];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double uq = bq[t] ? ubq[t] : ur[qq[t]];
        acc[t] += lp * uq;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (final_scale)
      out[(int64_t)t * nodes + node] = 0.25 * acc[t];
    else
      out[((int64_t)blockIdx.y * 4 + t) * nodes + node] = acc[t];
  }
}

__global__ __launch_bounds__(256) void grad_beta_reduce_kernel(int nodes, int chunks, const double* __restrict__ part,
                                                              double* __restrict__ grad) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nodes) return;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[((int64_t)c * 4 + t) * nodes + node];
    grad[(int64_t)t * nodes + node] = 0.25 * s;
  }
}

}  // namespace

int grad_eps_chunks(int nrhs) { return (nrhs + RC - 1) / RC; }

hipError_t launch_grad_eps(int nx, int ny, int nz, double h, const double* u, int64_t ldu, const double* lam,
                           int64_t ldl, int nrhs, const double* ub, double* part, double* grad, hipStream_t s) {
  const int nodes = nx * ny * (nz ? nz : 1);
  const int chunks = grad_eps_chunks(nrhs);
  const dim3 blocks((nodes + 255) / 256);
  auto partial = [&](dim3 grid, double* dst, int final_scale) {
    if (nz)
      hipLaunchKernelGGL(grad_eps_partial_kernel<3>, grid, dim3(256), 0, s, nx, ny, nz, h, u, ldu, lam, ldl, nrhs,
                         ub, dst, final_scale);
    else
      hipLaunchKernelGGL(grad_eps_tile_kernel, dim3(((nx + TX - 1) / TX) * ((ny + TY - 1) / TY), grid.y), dim3(256), 0,
                         s, nx, ny, h, u, ldu, lam, ldl, nrhs, ub, dst, final_scale);
    return hipGetLastError();
  };
  // zero or one chunk: the partial kernel writes the scaled result directly
  if (chunks <= 1) return partial(dim3(blocks.x, 1), grad, 1);
  hipError_t e = partial(dim3(blocks.x, chunks), part, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(grad_eps_reduce_kernel, blocks, dim3(256), 0, s, nodes, chunks, h, part, grad);
  return hipGetLastError();
}

hipError_t launch_grad_eps_general(int nx, int ny, const double* x, const double* y, const double* u, int64_t ldu,
                                   const double* lam, int64_t ldl, int nrhs, const double* ub, double* part,
                                   double* gx, double* gy, hipStream_t s) {
  const int nodes = nx * ny;
  const int chunks = grad_eps_chunks(nrhs);
  const dim3 blocks((nodes + 255) / 256);
  if (chunks <= 1) {
    hipLaunchKernelGGL(grad_eps_general_partial_kernel, dim3(blocks.x, 1), dim3(256), 0, s, nx, ny, x, y, u, ldu, lam,
                       ldl, nrhs, ub, (double*)nullptr, gx, gy);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(grad_eps_general_partial_kernel, dim3(blocks.x, chunks), dim3(256), 0, s, nx, ny, x, y, u, ldu,
                     lam, ldl, nrhs, ub, part, gx, gy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(grad_eps_general_reduce_kernel, blocks, dim3(256), 0, s, nodes, chunks, part, gx, gy);
  return hipGetLastError();
}

hipError_t launch_grad_beta(int nx, int ny, const double* u, int64_t ldu, const double* lam, int64_t ldl, int nrhs,
                            const double* ub, double* part, double* grad, hipStream_t s) {
  const int nodes = nx * ny;
  const int chunks = grad_eps_chunks(nrhs);
  const dim3 blocks((nodes + 255) / 256);
  if (chunks <= 1) {
    hipLaunchKernelGGL(grad_beta_partial_kernel, dim3(blocks.x, 1), dim3(256), 0, s, nx, ny, u, ldu, lam, ldl, nrhs,
                       ub, grad, 1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(grad_beta_partial_kernel, dim3(blocks.x, chunks), dim3(256), 0, s, nx, ny, u, ldu, lam, ldl,
                     nrhs, ub, part, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(grad_beta_reduce_kernel, blocks, dim3(256), 0, s, nodes, chunks, part, grad);
  return hipGetLastError();
}
