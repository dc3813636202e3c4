// k_graph.hip -- generator costs for libspm.
//
// The paper expands generators one at a time in cost order (Procedure 1),
// shades their cones and relaxes every visible DataArray entry (Procedure 4),
// which is Dijkstra's algorithm on the visibility graph of the generators.
// Here the same costs come from three kernels (templates over the scene
// source, like the ingest kernels):
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
// for a segment source, v sees the segment's closest point to v).  Rows and
// bits are indexed by spatial position (gorder), so the 64 generators of a
// wavefront are neighbours in space and share few relevant edges.  LDSE: the
// edges and chunk boxes are staged in LDS first.  Workgroups never straddle
// scenes (each scene's wavefronts are padded to whole workgroups).
template <class S, bool LDSE>
__global__ __launch_bounds__(256) void k_genvis(S src) {
  int sc, blk4;
  if (!src.locate(STG_GVBLK, blockIdx.x, sc, blk4)) return;
  const Dev& d = src.scene(sc);
  extern __shared__ int4 smem[];
  const int E = d.E, NC = d.NC, RW = d.RW;
  Geo geo{d.edges, d.ext, d.chunks, E, NC};
  if (LDSE) {
    EdgeRec* s_edges = (EdgeRec*)smem;
    int4* s_chunks = (int4*)(s_edges + E);
    const int4* se = (const int4*)d.edges;
    for (int k = threadIdx.x; k < E * 2; k += blockDim.x) ((int4*)s_edges)[k] = se[k];
    for (int k = threadIdx.x; k < NC; k += blockDim.x) s_chunks[k] = d.chunks[k];
    __syncthreads();
    geo.edges = s_edges;
    geo.chunks = s_chunks;
  }
  const int wid = blk4 * 4 + (threadIdx.x >> 6);
  const int r = wid / RW, blk = wid - r * RW;
  const int G = uni(d.misc[MISC_G]);
  const int nsrc = d.np + d.ns;
  if (r >= G || r < nsrc) return;  // only corner rows are read
  const int lane = lane_id();
  const int v = uni(d.gorder[r]);
  const int gx = uni(d.gens[v].x), gy = uni(d.gens[v].y);
  const int gux = uni(d.gens[v].ux), guy = uni(d.gens[v].uy), gnx = uni(d.gens[v].nx), gny = uni(d.gens[v].ny);
  const int upos = blk * 64 + lane;
  const int u = upos < G ? d.gorder[upos] : -1;
  const bool valid = u >= 0 && u != v;
  GenRec gu = {};
  if (valid) gu = d.gens[u];
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
  if (lane == 0) d.vis[(size_t)r * RW + blk] = bits;
}

// Arc weight from a generator with doubled coordinates (x, y, x2, y2) --
// a segment iff (x, y) != (x2, y2) -- to the corner at (vx, vy).
__device__ __forceinline__ double arc_len4(int4 u, int vx, int vy) {
  GenRec r;
  r.kind = (u.x != u.z || u.y != u.w) ? SPM_GEN_SEGMENT : SPM_GEN_POINT;
  r.x = u.x; r.y = u.y; r.x2 = u.z; r.y2 = u.w;
  return arc_len(r, vx, vy);
}

constexpr int kRelaxFront = 2048;   // largest frontier kept as a list (push rounds)

// One workgroup per scene: Bellman-Ford over the arc matrix, iterated to its
// fixed point (the costs Dijkstra reaches).  Sources start at 0.  Each round
// relaxes the arcs leaving the generators whose cost changed in the previous
// round:
//   pull  (large frontier): every corner v scans row v restricted to the
//         frontier and keeps the best candidate;
//   push  (small frontier, corners only): for each frontier corner u, every
//         corner v of row u -- corner-to-corner visibility is symmetric -- takes
//         cost(u) + |u - v| through an atomic minimum on the IEEE bits of the
//         non-negative doubles, which order like the values.
// Positive arc weights make the double-precision fixed point unique, so the
// result does not depend on thread timing or on the pull/push schedule.
// LDS: costs, generator coordinates and change masks live in LDS when they
// fit, else in global memory.  Everything is indexed by spatial position;
// outputs go back to canonical ids.
template <class S, bool LDS>
__global__ __launch_bounds__(1024) void k_relax(S src, int Gcap, int RWcap) {
  int sc, one;
  if (!src.locate(STG_SCENE, blockIdx.x, sc, one)) return;
  const Dev& d = src.scene(sc);
  extern __shared__ u64 shm[];
  __shared__ int any, nfront, reached;
  __shared__ int front[kRelaxFront];
  const int RW = d.RW;
  const u64* __restrict__ vis = d.vis;
  const int* __restrict__ gorder = d.gorder;
  u64* chg_a = shm;
  u64* chg_b = shm + RWcap;
  u64* cost = LDS ? (shm + 2 * RWcap) : d.costpos;   // indexed by spatial position
  int4* gxy = LDS ? (int4*)(shm + 2 * RWcap + Gcap) : d.gxy;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int G = d.misc[MISC_G];
  const int nsrc = d.np + d.ns;
  for (int k = tid; k < RW; k += nt) { chg_a[k] = 0; chg_b[k] = 0; }
  if (tid == 0) { reached = 0; nfront = -1; }
  __syncthreads();
  for (int g = tid; g < G; g += nt) {
    const GenRec r = d.gens[gorder[g]];
    const bool srcg = g < nsrc;
    cost[g] = (u64)__double_as_longlong(srcg ? 0.0 : INFINITY);
    gxy[g] = make_int4(r.x, r.y, r.x2, r.y2);
    if (srcg) atomicOr(&chg_a[g >> 6], 1ull << (g & 63));
  }
  __syncthreads();
  u64* cur = chg_a;
  u64* nxt = chg_b;
  int rounds = 0;
  for (; rounds <= G; ++rounds) {
    if (tid == 0) any = 0;
    const int nf = nfront;  // frontier list size, or -1 when only the mask is valid
    __syncthreads();
    if (nf < 0) {
      for (int v = tid; v < G; v += nt) {
        if (v < nsrc) continue;  // sources keep cost 0
        const int4 pv = gxy[v];
        const double old = __longlong_as_double((long long)cost[v]);
        double best = old;
        const u64* row = vis + (size_t)v * RW;
        for (int k = 0; k < RW; ++k) {
          const u64 c = cur[k];
          if (!c) continue;
          u64 m = row[k] & c;
          while (m) {
            const int u = k * 64 + __builtin_ctzll(m);
            m &= m - 1;
            const double cu = __longlong_as_double((long long)cost[u]);
            if (!(cu < best)) continue;
            const double cand = cu + arc_len4(gxy[u], pv.x, pv.y);
            if (cand < best) best = cand;
          }
        }
        if (best < old) {
          cost[v] = (u64)__double_as_longlong(best);
          atomicOr(&nxt[v >> 6], 1ull << (v & 63));
          any = 1;
        }
      }
    } else {
      for (int it = tid; it < nf * RW; it += nt) {
        const int f = it / RW, k = it - f * RW;
        const int u = front[f];
        u64 m = vis[(size_t)u * RW + k];
        if (!m) continue;
        const double cu = __longlong_as_double((long long)cost[u]);
        const int4 pu = gxy[u];
        while (m) {
          const int v = k * 64 + __builtin_ctzll(m);
          m &= m - 1;
          const double cv = __longlong_as_double((long long)cost[v]);
          if (!(cu < cv)) continue;
          const int4 pv = gxy[v];
          const double cand = cu + arc_len4(pu, pv.x, pv.y);
          if (cand < cv) {
            const u64 ob = atomicMin(&cost[v], (u64)__double_as_longlong(cand));
            if (__longlong_as_double((long long)ob) > cand) {
              atomicOr(&nxt[v >> 6], 1ull << (v & 63));
              any = 1;
            }
          }
        }
      }
    }
    __syncthreads();
    if (!any) break;
    // next frontier: a list when small enough (all corners), else the mask alone
    if (tid == 0) nfront = 0;
    __syncthreads();
    for (int k = tid; k < RW; k += nt) {
      const u64 m = nxt[k];
      if (!m) continue;
      const int n = __popcll(m);
      const int at = atomicAdd(&nfront, n);
      u64 mm = m;
      for (int t = 0; t < n; ++t) {
        const int b = __builtin_ctzll(mm);
        mm &= mm - 1;
        if (at + t < kRelaxFront) front[at + t] = k * 64 + b;
      }
    }
    __syncthreads();
    if (tid == 0 && nfront > kRelaxFront / 4) nfront = -1;  // large frontier: pull round
    u64* t = cur;
    cur = nxt;
    nxt = t;
    for (int k = tid; k < RW; k += nt) nxt[k] = 0;
    __syncthreads();
  }
  // parents (smallest canonical id attaining the cost) and outputs, in canonical order
  int mine = 0;
  for (int p = tid; p < G; p += nt) {
    const double c = __longlong_as_double((long long)cost[p]);
    const int v = gorder[p];
    int par = -1;
    if (p < nsrc) par = v;
    else if (c < INFINITY) {
      const int4 pv = gxy[p];
      const u64* row = vis + (size_t)p * RW;
      for (int k = 0; k < RW; ++k) {
        u64 m = row[k];
        while (m) {
          const int up = k * 64 + __builtin_ctzll(m);
          m &= m - 1;
          const double cu = __longlong_as_double((long long)cost[up]);
          if (!(cu < c)) continue;
          if (cu + arc_len4(gxy[up], pv.x, pv.y) == c) {
            const int u = gorder[up];
            if (par < 0 || u < par) par = u;
          }
        }
      }
    }
    d.gen_cost[v] = c;
    d.gen_parent[v] = par;
    d.cost64[v] = c;
    if (c < INFINITY) ++mine;
  }
  atomicAdd(&reached, mine);
  __syncthreads();
  if (tid == 0) {
    d.misc[MISC_REACHED] = reached;
    d.misc[MISC_ROUNDS] = rounds;
  }
}

// One wavefront per generator: rank by (float cost, id) among all generators;
// unreached ones (+inf) rank last and are not copied.
template <class S>
__global__ __launch_bounds__(256) void k_gsort(S src) {
  int sc, g;
  if (!src.locate(STG_GEN, blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), sc, g)) return;
  const Dev& d = src.scene(sc);
  const int G = uni(d.misc[MISC_G]);
  if (g >= G) return;
  const int lane = lane_id();
  const float cf = (float)d.cost64[g];
  const u64 key = ((u64)__float_as_uint(cf) << 32) | (u64)(unsigned)g;
  int rank = 0;
  for (int h = lane; h - lane < G; h += 64) {
    bool lt = false;
    if (h < G) {
      const float ch = (float)d.cost64[h];
      lt = (((u64)__float_as_uint(ch) << 32) | (u64)(unsigned)h) < key;
    }
    rank += __popcll(ballot(lt));
  }
  if (lane == 0 && cf < INFINITY) {
    GenRec r = d.gens[g];
    r.costf = cf;
    d.sgen[rank] = r;
    d.sgcost[rank] = cf;
    d.sgbb[rank] = make_int4(min(r.x, r.x2), min(r.y, r.y2), max(r.x, r.x2), max(r.y, r.y2));
  }
}

static int max_lds_per_block() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  if (!cached[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    cached[dev] = v;
  }
  return cached[dev];
}

template <class S>
hipError_t launch_genvis(const S& src, const Plan& p, hipStream_t s) {
  if (p.total[STG_GVBLK] <= 0) return hipSuccess;
  const dim3 grid((unsigned)p.total[STG_GVBLK]);
  if (p.genvis_lds > 0 && p.genvis_lds <= 32768)
    hipLaunchKernelGGL((k_genvis<S, true>), grid, dim3(256), p.genvis_lds, s, src);
  else
    hipLaunchKernelGGL((k_genvis<S, false>), grid, dim3(256), 0, s, src);
  return hipGetLastError();
}

template <class S>
hipError_t launch_relax(const S& src, const Plan& p, hipStream_t s) {
  const int RWcap = p.maxRW > 0 ? p.maxRW : 1;
  const int Gcap = p.maxGmax > 0 ? p.maxGmax : 1;
  const size_t chg = 2 * (size_t)RWcap * sizeof(u64);
  const size_t shm = chg + (size_t)Gcap * (sizeof(u64) + sizeof(int4));
  const size_t static_lds = 4 * 3 + kRelaxFront * 4 + 64;
  const dim3 grid((unsigned)p.total[STG_SCENE]);
  if (shm + static_lds <= (size_t)max_lds_per_block()) {
    if (shm > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)k_relax<S, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_relax<S, true>), grid, dim3(kRelaxThreads), shm, s, src, Gcap, RWcap);
  } else {
    hipLaunchKernelGGL((k_relax<S, false>), grid, dim3(kRelaxThreads), chg, s, src, Gcap, RWcap);
  }
  return hipGetLastError();
}

template <class S>
hipError_t launch_gsort(const S& src, const Plan& p, hipStream_t s) {
  if (p.total[STG_GEN] <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gsort<S>, dim3((unsigned)((p.total[STG_GEN] + 3) / 4)), dim3(256), 0, s, src);
  return hipGetLastError();
}

template hipError_t launch_genvis<SingleSrc>(const SingleSrc&, const Plan&, hipStream_t);
template hipError_t launch_genvis<BatchSrc>(const BatchSrc&, const Plan&, hipStream_t);
template hipError_t launch_relax<SingleSrc>(const SingleSrc&, const Plan&, hipStream_t);
template hipError_t launch_relax<BatchSrc>(const BatchSrc&, const Plan&, hipStream_t);
template hipError_t launch_gsort<SingleSrc>(const SingleSrc&, const Plan&, hipStream_t);
template hipError_t launch_gsort<BatchSrc>(const BatchSrc&, const Plan&, hipStream_t);

}  // namespace spm
