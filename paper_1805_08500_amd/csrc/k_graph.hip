// k_graph.hip -- generator costs for libspm.
//
// The paper expands generators one at a time in cost order (Procedure 1),
// shades their cones and relaxes every visible DataArray entry (Procedure 4),
// which is Dijkstra's algorithm on the visibility graph of the generators.
// Here the same costs come from three kernels:
//   k_genvis   every (corner, generator) arc of the visibility graph, as a
//              bit matrix (one wavefront per 64 arcs, exact predicates);
//   k_relax    a single-workgroup Bellman-Ford over that matrix in double
//              precision, iterated to its fixed point (which Dijkstra also
//              reaches), then each corner's parent: the smallest id among the
//              visible predecessors that attain its cost;
//   k_gsort    the reached generators ordered by (float cost, id), the order
//              the pixel stage walks them in.
#include <math.h>

#include "spm_internal.hpp"

namespace spm {

// Arc weight from generator u to the corner at doubled (vx, vy), double.
__device__ __forceinline__ double arc_len(const GenRec& u, int vx, int vy) {
  if (u.kind != SPM_GEN_SEGMENT) {
    const double dx = (double)(vx - u.x), dy = (double)(vy - u.y);
    return 0.5 * sqrt(dx * dx + dy * dy);
  }
  const long long ex = u.x2 - u.x, ey = u.y2 - u.y;
  const long long L = ex * ex + ey * ey;
  const long long num = (long long)(vx - u.x) * ex + (long long)(vy - u.y) * ey;
  if (num <= 0) {
    const double dx = (double)(vx - u.x), dy = (double)(vy - u.y);
    return 0.5 * sqrt(dx * dx + dy * dy);
  }
  if (num >= L) {
    const double dx = (double)(vx - u.x2), dy = (double)(vy - u.y2);
    return 0.5 * sqrt(dx * dx + dy * dy);
  }
  const long long cr = ex * (vy - u.y) - ey * (vx - u.x);
  return 0.5 * fabs((double)cr) / sqrt((double)L);
}

// One wavefront per (row corner v, block of 64 generators u): bit u of row v
// is set iff the arc u -> v exists (u a source or another corner that sees v;
// for a segment source, v sees the segment's closest point to v).
__global__ __launch_bounds__(256) void k_genvis(int Gmax, int RW, const int* __restrict__ misc,
                                                const GenRec* __restrict__ gens,
                                                const EdgeRec* __restrict__ edges,
                                                const EdgeExt* __restrict__ ext,
                                                const int4* __restrict__ chunks, int E, int NC,
                                                u64* __restrict__ vis) {
  const int wid = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int v = wid / RW, blk = wid - v * RW;
  const int G = uni(misc[MISC_G]);
  if (v >= G) return;
  const int lane = lane_id();
  const Geo geo{edges, ext, chunks, E, NC};
  const int vkind = uni(gens[v].kind);
  if (vkind != SPM_GEN_VERTEX) return;
  const int gx = uni(gens[v].x), gy = uni(gens[v].y);
  const int gux = uni(gens[v].ux), guy = uni(gens[v].uy), gnx = uni(gens[v].nx), gny = uni(gens[v].ny);
  const int u = blk * 64 + lane;
  const bool valid = u < G && u != v;
  GenRec gu = {};
  if (valid) gu = gens[u];
  const bool fast = valid && gu.kind != SPM_GEN_SEGMENT;
  const bool seg = valid && gu.kind == SPM_GEN_SEGMENT;
  bool ok = false;
  const u64 fm = ballot(fast);
  if (fm) {
    const int bx0 = wave_min_i(fast ? gu.x : (1 << 30)), bx1 = wave_max_i(fast ? gu.x : -(1 << 30));
    const int by0 = wave_min_i(fast ? gu.y : (1 << 30)), by1 = wave_max_i(fast ? gu.y : -(1 << 30));
    u64 dummy[8];
    const bool pv = gu.kind == SPM_GEN_VERTEX;
    const u64 bl = wave_blocked_uniform<false>(geo, gu.x, gu.y, fm, gx, gy, true, gux, guy, gnx, gny, pv, gu.ux,
                                               gu.uy, gu.nx, gu.ny, bx0, by0, bx1, by1, dummy);
    ok = fast && !((bl >> lane) & 1ull);
  }
  if (ballot(seg)) {
    int clamp;
    const RPt q = seg_closest(gu.x, gu.y, gu.x2, gu.y2, gx, gy, &clamp);
    const int sx0 = wave_min_i(seg ? min(gu.x, gu.x2) : (1 << 30));
    const int sx1 = wave_max_i(seg ? max(gu.x, gu.x2) : -(1 << 30));
    const int sy0 = wave_min_i(seg ? min(gu.y, gu.y2) : (1 << 30));
    const int sy1 = wave_max_i(seg ? max(gu.y, gu.y2) : -(1 << 30));
    const bool vs = lane_visible_rational(geo, gx, gy, true, gux, guy, gnx, gny, q, seg, min(sx0, gx),
                                          min(sy0, gy), max(sx1, gx), max(sy1, gy));
    if (seg) ok = vs;
  }
  const u64 bits = ballot(ok);
  if (lane == 0) vis[(size_t)v * RW + blk] = bits;
}

// Single workgroup Bellman-Ford over the arc matrix.  Sources start at 0;
// a round relaxes every corner from the generators whose cost changed in the
// previous round, updating in place; it stops at the first round without a
// change.  Positive arc weights make the double-precision fixed point unique,
// so the result does not depend on thread timing.
template <bool LDS>
__global__ __launch_bounds__(1024) void k_relax(int Gmax, int RW, const GenRec* __restrict__ gens,
                                                const u64* __restrict__ vis, double* __restrict__ cost_g, int* misc,
                                                double* __restrict__ gen_cost, int* __restrict__ gen_parent) {
  extern __shared__ u64 shm[];
  u64* chg_a = shm;
  u64* chg_b = shm + RW;
  double* cost = LDS ? (double*)(shm + 2 * RW) : cost_g;
  __shared__ int any;
  __shared__ int reached;
  const int tid = threadIdx.x;
  const int G = misc[MISC_G];
  for (int k = tid; k < RW; k += blockDim.x) { chg_a[k] = 0; chg_b[k] = 0; }
  if (tid == 0) reached = 0;
  __syncthreads();
  for (int g = tid; g < G; g += blockDim.x) {
    const bool src = gens[g].kind != SPM_GEN_VERTEX;
    cost[g] = src ? 0.0 : INFINITY;
    if (src) atomicOr(&chg_a[g >> 6], 1ull << (g & 63));
  }
  __syncthreads();
  u64* cur = chg_a;
  u64* nxt = chg_b;
  int rounds = 0;
  for (; rounds <= G; ++rounds) {
    if (tid == 0) any = 0;
    __syncthreads();
    for (int v = tid; v < G; v += blockDim.x) {
      const GenRec gv = gens[v];
      if (gv.kind != SPM_GEN_VERTEX) continue;
      const double old = cost[v];
      double best = old;
      const u64* row = vis + (size_t)v * RW;
      for (int k = 0; k < RW; ++k) {
        const u64 c = cur[k];
        if (!c) continue;
        u64 m = row[k] & c;
        while (m) {
          const int u = k * 64 + __builtin_ctzll(m);
          m &= m - 1;
          const double cu = cost[u];
          if (!(cu < INFINITY)) continue;
          const double cand = cu + arc_len(gens[u], gv.x, gv.y);
          if (cand < best) best = cand;
        }
      }
      if (best < old) {
        cost[v] = best;
        atomicOr(&nxt[v >> 6], 1ull << (v & 63));
        any = 1;
      }
    }
    __syncthreads();
    if (!any) break;
    u64* t = cur;
    cur = nxt;
    nxt = t;
    for (int k = tid; k < RW; k += blockDim.x) nxt[k] = 0;
    __syncthreads();
  }
  // parents and outputs
  int mine = 0;
  for (int v = tid; v < G; v += blockDim.x) {
    const GenRec gv = gens[v];
    const double c = cost[v];
    int par = -1;
    if (gv.kind != SPM_GEN_VERTEX) par = v;
    else if (c < INFINITY) {
      const u64* row = vis + (size_t)v * RW;
      for (int k = 0; k < RW && par < 0; ++k) {
        u64 m = row[k];
        while (m) {
          const int u = k * 64 + __builtin_ctzll(m);
          m &= m - 1;
          const double cu = cost[u];
          if (cu < INFINITY && cu + arc_len(gens[u], gv.x, gv.y) == c) { par = u; break; }
        }
      }
    }
    gen_cost[v] = c;
    gen_parent[v] = par;
    if (LDS) cost_g[v] = c;
    if (c < INFINITY) ++mine;
  }
  atomicAdd(&reached, mine);
  __syncthreads();
  if (tid == 0) {
    misc[MISC_REACHED] = reached;
    misc[MISC_ROUNDS] = rounds;
  }
}

// One wavefront per generator: rank by (float cost, id) among all generators;
// unreached ones (+inf) rank last and are not copied.
__global__ __launch_bounds__(256) void k_gsort(int* misc, const GenRec* __restrict__ gens,
                                               const double* __restrict__ cost64, GenRec* __restrict__ sgen,
                                               float* __restrict__ sgcost, int4* __restrict__ sgbb) {
  const int g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int G = uni(misc[MISC_G]);
  if (g == 0 && threadIdx.x == 0) misc[MISC_TILE_CTR] = 0;  // tile queue of the pixel stage
  if (g >= G) return;
  const int lane = lane_id();
  const float cf = (float)cost64[g];
  const u64 key = ((u64)__float_as_uint(cf) << 32) | (u64)(unsigned)g;
  int rank = 0;
  for (int h = lane; h - lane < G; h += 64) {
    bool lt = false;
    if (h < G) {
      const float ch = (float)cost64[h];
      lt = (((u64)__float_as_uint(ch) << 32) | (u64)(unsigned)h) < key;
    }
    rank += __popcll(ballot(lt));
  }
  if (lane == 0 && cf < INFINITY) {
    GenRec r = gens[g];
    r.costf = cf;
    sgen[rank] = r;
    sgcost[rank] = cf;
    sgbb[rank] = make_int4(min(r.x, r.x2), min(r.y, r.y2), max(r.x, r.x2), max(r.y, r.y2));
  }
}

hipError_t launch_genvis(const Dev& d, hipStream_t s) {
  if (d.Gmax == 0) return hipSuccess;
  const long long waves = (long long)d.Gmax * d.RW;
  hipLaunchKernelGGL(k_genvis, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, d.Gmax, d.RW, d.misc, d.gens,
                     d.edges, d.ext, d.chunks, d.E, d.NC, d.vis);
  return hipGetLastError();
}

hipError_t launch_relax(const Dev& d, hipStream_t s) {
  const size_t chg = 2 * (size_t)(d.RW > 0 ? d.RW : 1) * sizeof(u64);
  if (d.Gmax <= kRelaxLdsMaxGen) {
    const size_t shm = chg + (size_t)(d.Gmax > 0 ? d.Gmax : 1) * sizeof(double);
    hipLaunchKernelGGL(k_relax<true>, dim3(1), dim3(kRelaxThreads), shm, s, d.Gmax, d.RW, d.gens, d.vis,
                       d.cost64, d.misc, d.gen_cost, d.gen_parent);
  } else {
    hipLaunchKernelGGL(k_relax<false>, dim3(1), dim3(kRelaxThreads), chg, s, d.Gmax, d.RW, d.gens, d.vis,
                       d.cost64, d.misc, d.gen_cost, d.gen_parent);
  }
  return hipGetLastError();
}

hipError_t launch_gsort(const Dev& d, hipStream_t s) {
  if (d.Gmax == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gsort, dim3((d.Gmax + 3) / 4), dim3(256), 0, s, d.misc, d.gens, d.cost64, d.sgen, d.sgcost,
                     d.sgbb);
  return hipGetLastError();
}

}  // namespace spm
