// k_pixel.hip -- the pixel propagation stage of libspm (the hot path).
//
// The paper shades one clipped cone per generator over the whole framebuffer:
// every pixel that sees the generator (is not in its shadow, Procedure 2)
// takes cost(g) + |p - g| when that beats its current value (Procedure 3,
// the depth test keeps the minimum).  After all generators the framebuffer
// holds lambda* and the parent of every pixel.  Segment sources use the
// distance to the closest point of the segment (Section 4).
//
// This kernel computes the same minimum pixel-major: one wavefront owns a
// tile of 64 pixels (one per lane) and walks the generators in ascending
// (cost, id) order -- the order the paper expands them in -- so that
//   * a generator whose cost reaches the tile's largest current value ends
//     the walk (no later cone can win anywhere in the tile);
//   * a generator whose cone cannot reach below that value anywhere in the
//     tile is skipped for the whole wavefront (lane-parallel tile bound);
//   * per lane, a candidate that cannot beat the lane's value is dropped
//     before any visibility work (squared compare, no square root);
//   * visibility of the remaining (lane, generator) pairs uses the exact
//     integer predicates of wave_blocked_uniform (point and corner
//     generators) or lane_visible_rational (segment sources).
// Ties keep the earlier generator in that order (strict comparison, as the
// paper's depth test and Procedures 3-4 do).  Distances are float.
#include <math.h>

#include "spm_internal.hpp"

namespace spm {

enum { ST_TILES = 0, ST_BATCHES, ST_BOUND, ST_VISWAVE, ST_RELEV, ST_LANEEDGE, ST_OCCL, ST_ACCEPT };

// Box (doubled pixel-centre coordinates) of the lanes set in m.
template <int TW>
__device__ __forceinline__ void mask_box(u64 m, int i0, int j0, int& bx0, int& by0, int& bx1, int& by1) {
  constexpr int TH = 64 / TW;
  constexpr u64 rowm = (TW == 64) ? ~0ull : ((1ull << TW) - 1ull);
  unsigned cols = 0;
  int r0 = TH, r1 = -1;
#pragma unroll
  for (int r = 0; r < TH; ++r) {
    const unsigned bits = (unsigned)((m >> (r * TW)) & rowm);
    cols |= bits;
    if (bits) { r0 = min(r0, r); r1 = r; }
  }
  const int c0 = __builtin_ctz(cols), c1 = 31 - __builtin_clz(cols);
  bx0 = 2 * (i0 + c0) + 1;
  bx1 = 2 * (i0 + c1) + 1;
  by0 = 2 * (j0 + r0) + 1;
  by1 = 2 * (j0 + r1) + 1;
}

// Lane mask of quadrant q (0..3) of a TW x (64/TW) tile: the tile is halved in
// both directions so that the tile bound can use four boxes and four upper
// bounds instead of one.
template <int TW>
__host__ __device__ constexpr u64 quad_mask(int q) {
  u64 m = 0;
  for (int l = 0; l < 64; ++l) {
    const int c = l % TW, r = l / TW;
    const int lq = (c >= TW / 2 ? 1 : 0) + (r >= (64 / TW) / 2 ? 2 : 0);
    if (lq == q) m |= 1ull << l;
  }
  return m;
}

// Per-quadrant maximum of v over the lanes of each quadrant (4 exchange steps).
template <int TW>
__device__ __forceinline__ float quad_max(float v) {
  constexpr int TH = 64 / TW;
#pragma unroll
  for (int m = 1; m < TW / 2; m <<= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
#pragma unroll
  for (int m = TW; m < (TH / 2) * TW; m <<= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
  return v;
}

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// conservative test: can a generator with cost c and bounding box (x0..y1) come
// below ub anywhere in the box (bx0..by1)?
__device__ __forceinline__ bool box_may_win(float c, int x0, int y0, int x1, int y1, int bx0, int by0, int bx1,
                                            int by1, float ub) {
  const int dx = max(max(x0 - bx1, bx0 - x1), 0);
  const int dy = max(max(y0 - by1, by0 - y1), 0);
  const float room = ub - c;
  return room > 0.0f && (float)(dx * dx + dy * dy) < 4.0f * room * room * (1.0f + 2e-6f);
}

// One tile: the per-lane minimum over generators for 64 pixels.  The
// generator tables and the edges come through plain pointers that point
// either into LDS (staged by the kernel) or into global memory.
template <int TW, bool STATS>
__device__ __forceinline__ void tile_work(int tile, int W, int H, int W32, int G, const unsigned* __restrict__ inside,
                                          const GenRec* sgen, const float* sgcost, const int4* sgbb, const Geo& geo,
                                          float* __restrict__ dist, int* __restrict__ parent, u64* st) {
  constexpr int TH = 64 / TW;
  constexpr int QL[4] = {0, TW / 2, (TH / 2) * TW, (TH / 2) * TW + TW / 2};  // first lane of each quadrant
  const int lane = lane_id();
  const int ntx = (W + TW - 1) / TW;
  const int ty = tile / ntx, tx = tile - ty * ntx;
  const int i0 = tx * TW, j0 = ty * TH;
  const int i = i0 + (lane % TW), j = j0 + (lane / TW);
  const bool valid = i < W && j < H;
  const int px = 2 * i + 1, py = 2 * j + 1;
  bool ins = false;
  if (valid) ins = (inside[(size_t)j * W32 + (i >> 5)] >> (i & 31)) & 1u;
  const bool active = valid && !ins;
  if (STATS) st[ST_TILES] += 1;
  float best = INFINITY;
  int par = -1;
  const u64 act = ballot(active);
  if (act) {
    // quadrant upper bounds; quadrant q spans pixel columns i0 + (q & 1) * TW/2 .. + TW/2 - 1 and rows
    // j0 + (q >> 1) * TH/2 .. + TH/2 - 1 (doubled centres below)
    float ubq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ubq[q] = (act & quad_mask<TW>(q)) ? INFINITY : -INFINITY;
    const int qx0 = 2 * i0 + 1, qx1 = qx0 + TW, qy0 = 2 * j0 + 1, qy1 = qy0 + TH;  // lower-half / upper-half starts
    float UB = INFINITY;
    bool done = false;
    for (int base = 0; base < G && !done; base += 64) {
      if (sgcost[base] >= UB) break;
      if (STATS) st[ST_BATCHES] += 1;
      // lane-parallel tile bound against the four quadrants
      const int g = base + lane;
      bool cand = false;
      float c = INFINITY;
      int4 bb = make_int4(0, 0, 0, 0);
      if (g < G) {
        c = sgcost[g];
        bb = sgbb[g];
        cand = box_may_win(c, bb.x, bb.y, bb.z, bb.w, qx0, qy0, qx1 - 2, qy1 - 2, ubq[0]) ||
               box_may_win(c, bb.x, bb.y, bb.z, bb.w, qx1, qy0, qx1 + TW - 2, qy1 - 2, ubq[1]) ||
               box_may_win(c, bb.x, bb.y, bb.z, bb.w, qx0, qy1, qx1 - 2, qy1 + TH - 2, ubq[2]) ||
               box_may_win(c, bb.x, bb.y, bb.z, bb.w, qx1, qy1, qx1 + TW - 2, qy1 + TH - 2, ubq[3]);
      }
      u64 cm = ballot(cand);
      while (cm) {
        const int jl = first_bit(cm);
        cm &= cm - 1;
        const int k = base + jl;
        const float gc = readlane_f(c, jl);
        if (gc >= UB) { done = true; break; }
        const int x0 = readlane_i(bb.x, jl), y0 = readlane_i(bb.y, jl);
        const int x1 = readlane_i(bb.z, jl), y1 = readlane_i(bb.w, jl);
        bool upd = false;
        const bool is_seg = !(x0 == x1 && y0 == y1);
        float cc = 0.0f;  // segment: this lane's candidate value
        int clamp = 0;    // segment: closest point is A (0), B (1) or interior (2)
        int ax = x0, ay = y0, bx = x1, by = y1;
        const int ddx = px - x0, ddy = py - y0;
        const int d2 = mad24(ddx, ddx, mul24(ddy, ddy));   // point or corner: squared doubled distance
        bool need;
        if (!is_seg) {
          // cost + |p - g| < best  <=>  d2 < 4 (best - cost)^2; the factor keeps the filter conservative
          const float room = best - gc;
          need = active && room > 0.0f && (float)d2 < 4.0f * room * room * (1.0f + 1e-6f);
        } else {
          ax = sgen[k].x; ay = sgen[k].y; bx = sgen[k].x2; by = sgen[k].y2;
          const RPt q = seg_closest(ax, ay, bx, by, px, py, &clamp);
          (void)q;
          float dd;
          if (clamp == 0) {
            dd = 0.5f * sqrtf((float)(mad24(px - ax, px - ax, mul24(py - ay, py - ay))));
          } else if (clamp == 1) {
            dd = 0.5f * sqrtf((float)(mad24(px - bx, px - bx, mul24(py - by, py - by))));
          } else {
            const long long ex = bx - ax, ey = by - ay;
            const long long cr = ex * (py - ay) - ey * (px - ax);
            dd = 0.5f * fabsf((float)cr) / sqrtf((float)(ex * ex + ey * ey));
          }
          cc = gc + dd;
          need = active && cc < best;
        }
        const u64 nm = ballot(need);
        if (STATS) st[ST_BOUND] += __popcll(act);
        if (!nm) continue;
        // visibility groups: a point or corner is one group at (x0, y0); a segment has up to three
        // (lanes reaching endpoint A, endpoint B, or an interior point)
        const u64 mA = is_seg ? ballot(need && clamp == 0) : nm;
        const u64 mB = is_seg ? ballot(need && clamp == 1) : 0ull;
        const u64 mI = nm & ~mA & ~mB;
        const bool gv = !is_seg && sgen[k].kind == SPM_GEN_VERTEX;
        u64 bl = 0;
        for (int grp = 0; grp < 2; ++grp) {
          const u64 m = grp ? mB : mA;
          if (!m) continue;
          if (STATS) st[ST_VISWAVE] += 1;
          int bx0, by0, bx1, by1;
          mask_box<TW>(m, i0, j0, bx0, by0, bx1, by1);
          const int gx = grp ? bx : ax, gy = grp ? by : ay;
          bl |= wave_blocked_uniform<STATS>(geo, px, py, m, gx, gy, gv, gv ? sgen[k].ux : 0, gv ? sgen[k].uy : 0,
                                            gv ? sgen[k].nx : 0, gv ? sgen[k].ny : 0, false, 0, 0, 0, 0, bx0, by0,
                                            bx1, by1, st);
        }
        if (mI) {
          if (STATS) st[ST_VISWAVE] += 1;
          int bx0, by0, bx1, by1;
          mask_box<TW>(mI, i0, j0, bx0, by0, bx1, by1);
          bl |= wave_blocked_perp<STATS>(geo, px, py, mI, ax, ay, bx, by, bx0, by0, bx1, by1, st);
        }
        if (need && !((bl >> lane) & 1ull)) {
          if (!is_seg) cc = gc + 0.5f * sqrtf((float)d2);
          if (cc < best) { best = cc; par = sgen[k].id; upd = true; }
        }
        const u64 um = ballot(upd);
        if (um) {
          if (STATS) st[ST_ACCEPT] += __popcll(um);
          const float qm = quad_max<TW>(active ? best : -INFINITY);
#pragma unroll
          for (int q = 0; q < 4; ++q) ubq[q] = readlane_f(qm, QL[q]);
          UB = fmaxf(fmaxf(ubq[0], ubq[1]), fmaxf(ubq[2], ubq[3]));
        }
      }
    }
  }
  if (valid) {
    const size_t o = (size_t)j * W + i;
    dist[o] = best;
    parent[o] = par;
  }
}

constexpr int kPixelThreads = 512;
constexpr size_t kPixelLdsMax = 64 * 1024;

size_t pixel_lds_bytes(int Gmax, int E, int NC) {
  return (size_t)Gmax * (sizeof(GenRec) + 4 + 16) + 16 + (size_t)E * sizeof(EdgeRec) + (size_t)NC * 16;
}

// Persistent kernel: every wavefront takes tiles from a device queue
// (misc[MISC_TILE_CTR], reset by the generator sort) until none is left.
// LDSD: the cost-sorted generator table, the edges and the chunk boxes are
// first staged in LDS, so the wave-uniform reads of the hot loops are LDS
// broadcasts instead of L2 round trips.
template <int TW, bool STATS, bool LDSD>
__global__ __launch_bounds__(kPixelThreads, 6) void k_pixel(int W, int H, int W32, int Gmax, int* misc,
                                                         const unsigned* __restrict__ inside,
                                                         const GenRec* __restrict__ sgen_g,
                                                         const float* __restrict__ sgcost_g,
                                                         const int4* __restrict__ sgbb_g,
                                                         const EdgeRec* __restrict__ edges_g,
                                                         const EdgeExt* __restrict__ ext,
                                                         const int4* __restrict__ chunks_g, int E, int NC,
                                                         float* __restrict__ dist, int* __restrict__ parent,
                                                         u64* __restrict__ stats) {
  constexpr int TH = 64 / TW;
  extern __shared__ int4 smem[];
  const int G = misc[MISC_REACHED];
  const GenRec* sgen = sgen_g;
  const float* sgcost = sgcost_g;
  const int4* sgbb = sgbb_g;
  Geo geo{edges_g, ext, chunks_g, E, NC};
  if (LDSD) {
    GenRec* s_gen = (GenRec*)smem;
    int4* s_bb = (int4*)(s_gen + Gmax);
    EdgeRec* s_edges = (EdgeRec*)(s_bb + Gmax);
    int4* s_chunks = (int4*)(s_edges + E);
    float* s_cost = (float*)(s_chunks + NC);
    const int t = threadIdx.x, nt = blockDim.x;
    const int4* src = (const int4*)sgen_g;
    for (int k = t; k < G * 4; k += nt) ((int4*)s_gen)[k] = src[k];
    for (int k = t; k < G; k += nt) { s_bb[k] = sgbb_g[k]; s_cost[k] = sgcost_g[k]; }
    const int4* se = (const int4*)edges_g;
    for (int k = t; k < E * 2; k += nt) ((int4*)s_edges)[k] = se[k];
    for (int k = t; k < NC; k += nt) s_chunks[k] = chunks_g[k];
    __syncthreads();
    sgen = s_gen;
    sgcost = s_cost;
    sgbb = s_bb;
    geo.edges = s_edges;
    geo.chunks = s_chunks;
  }
  const int ntiles = ((W + TW - 1) / TW) * ((H + TH - 1) / TH);
  u64 st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (;;) {
    int tile = 0;
    if (lane_id() == 0) tile = atomicAdd(&misc[MISC_TILE_CTR], 1);
    tile = __shfl(tile, 0, 64);
    if (tile >= ntiles) break;
    tile_work<TW, STATS>(tile, W, H, W32, G, inside, sgen, sgcost, sgbb, geo, dist, parent, st);
  }
  if (STATS && lane_id() == 0) {
#pragma unroll
    for (int s = 0; s < 8; ++s) atomicAdd(&stats[s], st[s]);
  }
}

static int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

template <int TW, bool STATS, bool LDSD>
static hipError_t launch_variant(const Dev& d, hipStream_t s, size_t shm) {
  auto kern = k_pixel<TW, STATS, LDSD>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kPixelThreads, shm) != hipSuccess || per_cu < 1)
    per_cu = 1;
  constexpr int TH = 64 / TW;
  const long long tiles = (long long)((d.W + TW - 1) / TW) * ((d.H + TH - 1) / TH);
  const long long waves_needed = tiles;
  long long blocks = (long long)device_cus() * per_cu;
  const long long max_blocks = (waves_needed + (kPixelThreads / 64) - 1) / (kPixelThreads / 64);
  if (blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kPixelThreads), shm, s, d.W, d.H, d.W32, d.Gmax, d.misc,
                     d.inside, d.sgen, d.sgcost, d.sgbb, d.edges, d.ext, d.chunks, d.E, d.NC, d.dist, d.parent,
                     d.stats);
  return hipGetLastError();
}

template <int TW>
static hipError_t launch_tw(const Dev& d, hipStream_t s) {
  const size_t shm = pixel_lds_bytes(d.Gmax, d.E, d.NC);
  const bool lds = shm <= kPixelLdsMax;
  if (d.stats) return lds ? launch_variant<TW, true, true>(d, s, shm) : launch_variant<TW, true, false>(d, s, 0);
  return lds ? launch_variant<TW, false, true>(d, s, shm) : launch_variant<TW, false, false>(d, s, 0);
}

hipError_t launch_pixel(const Dev& d, hipStream_t s) {
  if (d.tile_w == 16) return launch_tw<16>(d, s);
  if (d.tile_w == 4) return launch_tw<4>(d, s);
  return launch_tw<8>(d, s);
}

// Batched pixel stage: one persistent launch for every scene of a batch.  A
// workgroup takes a work item -- kSlice tiles of one scene -- from the batch
// queue, stages that scene's generator table and edges in LDS when it differs
// from the scene already staged, and its wavefronts share the slice's tiles
// through an LDS counter.  Tile shapes may differ between scenes.
template <bool LDSD>
__global__ __launch_bounds__(kPixelThreads, 4) void k_pixel_batch(BatchSrc src, int* ctr) {
  extern __shared__ int4 smem[];
  __shared__ int item_scene, item_t0, item_t1, staged, next_tile;
  const int tid = threadIdx.x;
  if (tid == 0) staged = -1;
  u64 st[8];
  for (;;) {
    if (tid == 0) {
      const int it = atomicAdd(ctr, 1);
      int sc, local;
      if (src.locate(STG_SLICE, it, sc, local)) {
        const Dev& d0 = src.scene(sc);
        const int nt = tiles_of(d0.W, d0.H, d0.tile_w);
        item_scene = sc;
        item_t0 = local * kSlice;
        item_t1 = min(nt, item_t0 + kSlice);
      } else {
        item_scene = -1;
      }
      next_tile = 0;
    }
    __syncthreads();
    const int sc = item_scene;
    if (sc < 0) break;
    const Dev& d = src.scene(sc);
    const int G = d.misc[MISC_REACHED];
    const GenRec* sgen = d.sgen;
    const float* sgcost = d.sgcost;
    const int4* sgbb = d.sgbb;
    Geo geo{d.edges, d.ext, d.chunks, d.E, d.NC};
    if (LDSD) {
      GenRec* s_gen = (GenRec*)smem;
      int4* s_bb = (int4*)(s_gen + d.Gmax);
      EdgeRec* s_edges = (EdgeRec*)(s_bb + d.Gmax);
      int4* s_chunks = (int4*)(s_edges + d.E);
      float* s_cost = (float*)(s_chunks + d.NC);
      if (sc != staged) {
        const int4* gsrc = (const int4*)d.sgen;
        for (int k = tid; k < G * 4; k += blockDim.x) ((int4*)s_gen)[k] = gsrc[k];
        for (int k = tid; k < G; k += blockDim.x) { s_bb[k] = d.sgbb[k]; s_cost[k] = d.sgcost[k]; }
        const int4* se = (const int4*)d.edges;
        for (int k = tid; k < d.E * 2; k += blockDim.x) ((int4*)s_edges)[k] = se[k];
        for (int k = tid; k < d.NC; k += blockDim.x) s_chunks[k] = d.chunks[k];
        __syncthreads();
        if (tid == 0) staged = sc;
      }
      sgen = s_gen;
      sgcost = s_cost;
      sgbb = s_bb;
      geo.edges = s_edges;
      geo.chunks = s_chunks;
    }
    for (;;) {
      int t = 0;
      if (lane_id() == 0) t = atomicAdd(&next_tile, 1);
      t = __shfl(t, 0, 64);
      const int tile = item_t0 + t;
      if (tile >= item_t1) break;
      if (d.tile_w == 16)
        tile_work<16, false>(tile, d.W, d.H, d.W32, G, d.inside, sgen, sgcost, sgbb, geo, d.dist, d.parent, st);
      else if (d.tile_w == 4)
        tile_work<4, false>(tile, d.W, d.H, d.W32, G, d.inside, sgen, sgcost, sgbb, geo, d.dist, d.parent, st);
      else
        tile_work<8, false>(tile, d.W, d.H, d.W32, G, d.inside, sgen, sgcost, sgbb, geo, d.dist, d.parent, st);
    }
    __syncthreads();
  }
}

__global__ void k_reset_counter(int* ctr) { *ctr = 0; }

hipError_t launch_pixel_batch(const BatchSrc& b, const Plan& p, int* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, ctr);
  const size_t shm = p.pixel_lds;
  const bool lds = shm > 0 && shm <= kPixelLdsMax;
  auto kern = lds ? k_pixel_batch<true> : k_pixel_batch<false>;
  const size_t use = lds ? shm : 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kPixelThreads, use) != hipSuccess || per_cu < 1)
    per_cu = 1;
  long long blocks = (long long)device_cus() * per_cu;
  if (blocks > p.total[STG_SLICE]) blocks = p.total[STG_SLICE];
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kPixelThreads), use, s, b, ctr);
  return hipGetLastError();
}

}  // namespace spm
