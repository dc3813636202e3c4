// k_adjoint.hip -- agent distances read from a built map, and their adjoint
// with respect to the source positions.
//
// An agent a in pixel p takes the pixel's parent g (Section 1: grid lookup of
// the parent) and the distance D(a) = |a - x_g(a)| + cost(g), where x_g(a) is
// g itself, or for a segment source the segment's closest point to a
// (Section 4).  With the parent chains held fixed, only the last leg of the
// path depends on where the sources are: from v -- the agent itself when g is
// a source, else the corner just before the chain's root -- to the root source.
//   point source s:       dD/ds = (s - v) / |s - v|
//   segment source A-B:   q* = A + t (B - A) closest to v, n = (q* - v)/|q* - v|,
//                         dD/dA = (1 - t) n,  dD/dB = t n
// (at fixed t this is the derivative of |v - q(t)|, and t itself does not
// move the distance to first order because q* is the closest point).
// Obstacle corners do not move.
#include <math.h>

#include "spm_internal.hpp"

namespace spm {

// root (source id) and preroot (last corner before the root, -1 for sources
// and unreachable generators) of every generator, walking the parent chain
__global__ void k_roots(int Gmax, int nsrc, const int* __restrict__ n_gen, const int* __restrict__ gen_parent,
                        int* __restrict__ root, int* __restrict__ preroot) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int G = n_gen[0];
  if (g >= G || g >= Gmax) return;
  if (g < nsrc) {
    root[g] = g;
    preroot[g] = -1;
    return;
  }
  int prev = g, cur = gen_parent[g];
  int steps = 0;
  while (cur >= nsrc && steps <= G) {
    prev = cur;
    cur = gen_parent[cur];
    ++steps;
  }
  if (cur < 0 || steps > G) {
    root[g] = -1;
    preroot[g] = -1;
  } else {
    root[g] = cur;
    preroot[g] = prev;
  }
}

// parent generator of the agent's pixel, or -1 (outside the grid / no parent)
__device__ __forceinline__ int agent_parent(float ax, float ay, int W, int H, const int* parent) {
  if (!(ax >= 0.0f && ay >= 0.0f && ax < (float)W && ay < (float)H)) return -1;
  const int i = min((int)floorf(ax), W - 1), j = min((int)floorf(ay), H - 1);
  return parent[(size_t)j * W + i];
}

// closest point parameter t in [0, 1] of segment A-B to (x, y), double
__device__ __forceinline__ double seg_t(double ax, double ay, double bx, double by, double x, double y) {
  const double ex = bx - ax, ey = by - ay;
  const double t = ((x - ax) * ex + (y - ay) * ey) / (ex * ex + ey * ey);
  return fmin(1.0, fmax(0.0, t));
}

__global__ void k_agent_dist(int W, int H, int n, const float* __restrict__ agents, const int* __restrict__ parent,
                             const int* __restrict__ gen_kind, const int* __restrict__ gen_xy,
                             const double* __restrict__ gen_cost, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float ax = agents[2 * i], ay = agents[2 * i + 1];
  const int g = agent_parent(ax, ay, W, H, parent);
  if (g < 0) {
    out[i] = INFINITY;
    return;
  }
  const double x = ax, y = ay;
  double qx = gen_xy[4 * g], qy = gen_xy[4 * g + 1];
  if (gen_kind[g] == SPM_GEN_SEGMENT) {
    const double bx = gen_xy[4 * g + 2], by = gen_xy[4 * g + 3];
    const double t = seg_t(qx, qy, bx, by, x, y);
    qx = qx + t * (bx - qx);
    qy = qy + t * (by - qy);
  }
  out[i] = (float)(sqrt((x - qx) * (x - qx) + (y - qy) * (y - qy)) + gen_cost[g]);
}

// Each agent's gradient contribution: the root source it reaches and up to
// four partial derivatives (2 for a point, 4 for a segment's endpoints),
// already weighted by dL/dD.
__global__ void k_agent_grad(int W, int H, int n, int nsrc, const float* __restrict__ agents,
                             const float* __restrict__ dLdD, const int* __restrict__ parent,
                             const int* __restrict__ gen_kind, const int* __restrict__ gen_xy,
                             const int* __restrict__ root, const int* __restrict__ preroot,
                             int* __restrict__ csrc, double* __restrict__ contrib) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  int r = -1;
  const float ax = agents[2 * i], ay = agents[2 * i + 1];
  const int g = agent_parent(ax, ay, W, H, parent);
  const float w = dLdD[i];
  if (g >= 0 && w != 0.0f) {
    double vx = ax, vy = ay;
    if (g < nsrc) r = g;
    else {
      r = root[g];
      const int pr = preroot[g];
      if (pr >= 0) {
        vx = gen_xy[4 * pr];
        vy = gen_xy[4 * pr + 1];
      } else {
        r = -1;
      }
    }
    if (r >= 0) {
      const double sx = gen_xy[4 * r], sy = gen_xy[4 * r + 1];
      if (gen_kind[r] == SPM_GEN_POINT) {
        const double dx = sx - vx, dy = sy - vy, L = sqrt(dx * dx + dy * dy);
        if (L > 0.0) { c[0] = w * dx / L; c[1] = w * dy / L; }
      } else {
        const double bx = gen_xy[4 * r + 2], by = gen_xy[4 * r + 3];
        const double t = seg_t(sx, sy, bx, by, vx, vy);
        const double qx = sx + t * (bx - sx), qy = sy + t * (by - sy);
        const double dx = qx - vx, dy = qy - vy, L = sqrt(dx * dx + dy * dy);
        if (L > 0.0) {
          const double nx = w * dx / L, ny = w * dy / L;
          c[0] = (1.0 - t) * nx; c[1] = (1.0 - t) * ny;
          c[2] = t * nx; c[3] = t * ny;
        }
      }
    }
  }
  csrc[i] = r;
  for (int k = 0; k < 4; ++k) contrib[4 * (size_t)i + k] = c[k];
}

// One workgroup per source: the sum of its agents' contributions in a fixed
// order (per-thread strided sums, then a fixed tree), so the result does not
// depend on scheduling.
__global__ __launch_bounds__(256) void k_grad_reduce(int n, int np, const int* __restrict__ csrc,
                                                     const double* __restrict__ contrib,
                                                     float* __restrict__ grad_pts, float* __restrict__ grad_segs) {
  const int src = blockIdx.x;
  __shared__ double part[256][4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (csrc[i] == src)
      for (int k = 0; k < 4; ++k) acc[k] += contrib[4 * (size_t)i + k];
  for (int k = 0; k < 4; ++k) part[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 4; ++k) part[threadIdx.x][k] += part[threadIdx.x + s][k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (src < np) {
      grad_pts[2 * src] = (float)part[0][0];
      grad_pts[2 * src + 1] = (float)part[0][1];
    } else {
      const int k = src - np;
      for (int q = 0; q < 4; ++q) grad_segs[4 * k + q] = (float)part[0][q];
    }
  }
}

size_t agent_ws_bytes(int Gmax, int n_agents) {
  size_t o = 0;
  o = align_up(o + (size_t)(Gmax > 0 ? Gmax : 1) * sizeof(int), 256);   // root
  o = align_up(o + (size_t)(Gmax > 0 ? Gmax : 1) * sizeof(int), 256);   // preroot
  o = align_up(o + (size_t)(n_agents > 0 ? n_agents : 1) * sizeof(int), 256);
  o = align_up(o + (size_t)(n_agents > 0 ? n_agents : 1) * 4 * sizeof(double), 256);
  return o;
}

hipError_t launch_agent_dist(int W, int H, int n, const float* agents, const spm_out* out, float* d_out,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_agent_dist, dim3((n + 255) / 256), dim3(256), 0, s, W, H, n, agents, out->parent,
                     out->gen_kind, out->gen_xy, out->gen_cost, d_out);
  return hipGetLastError();
}

hipError_t launch_backward(int W, int H, int Gmax, int np, int ns, int n, const float* agents, const float* dLdD,
                           const spm_out* out, float* grad_pts, float* grad_segs, char* ws, hipStream_t s) {
  size_t o = 0;
  int* root = (int*)(ws + o);
  o = align_up(o + (size_t)(Gmax > 0 ? Gmax : 1) * sizeof(int), 256);
  int* preroot = (int*)(ws + o);
  o = align_up(o + (size_t)(Gmax > 0 ? Gmax : 1) * sizeof(int), 256);
  int* csrc = (int*)(ws + o);
  o = align_up(o + (size_t)(n > 0 ? n : 1) * sizeof(int), 256);
  double* contrib = (double*)(ws + o);
  const int nsrc = np + ns;
  if (Gmax > 0)
    hipLaunchKernelGGL(k_roots, dim3((Gmax + 255) / 256), dim3(256), 0, s, Gmax, nsrc, out->n_gen, out->gen_parent,
                       root, preroot);
  if (n > 0)
    hipLaunchKernelGGL(k_agent_grad, dim3((n + 255) / 256), dim3(256), 0, s, W, H, n, nsrc, agents, dLdD,
                       out->parent, out->gen_kind, out->gen_xy, root, preroot, csrc, contrib);
  if (nsrc > 0)
    hipLaunchKernelGGL(k_grad_reduce, dim3(nsrc), dim3(256), 0, s, n, np, csrc, contrib, grad_pts, grad_segs);
  return hipGetLastError();
}

}  // namespace spm
