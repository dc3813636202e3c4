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

template <int TW, bool STATS>
__global__ __launch_bounds__(256) void k_pixel(int W, int H, int W32, const int* __restrict__ misc,
                                               const unsigned* __restrict__ inside,
                                               const GenRec* __restrict__ sgen, const float* __restrict__ sgcost,
                                               const int4* __restrict__ sgbb, const EdgeRec* __restrict__ edges,
                                               const EdgeExt* __restrict__ ext, const int4* __restrict__ chunks,
                                               int E, int NC, float* __restrict__ dist, int* __restrict__ parent,
                                               u64* __restrict__ stats) {
  constexpr int TH = 64 / TW;
  const int lane = lane_id();
  const int wid = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int ntx = (W + TW - 1) / TW, nty = (H + TH - 1) / TH;
  if (wid >= ntx * nty) return;
  const Geo geo{edges, ext, chunks, E, NC};
  const int ty = wid / ntx, tx = wid - ty * ntx;
  const int i0 = tx * TW, j0 = ty * TH;
  const int i = i0 + (lane % TW), j = j0 + (lane / TW);
  const bool valid = i < W && j < H;
  const int px = 2 * i + 1, py = 2 * j + 1;
  bool ins = false;
  if (valid) ins = (inside[(size_t)j * W32 + (i >> 5)] >> (i & 31)) & 1u;
  const bool active = valid && !ins;
  u64 st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (STATS) st[ST_TILES] += 1;
  float best = INFINITY;
  int par = -1;
  const u64 act = ballot(active);
  if (act) {
    const int G = uni(misc[MISC_REACHED]);
    int tbx0, tby0, tbx1, tby1;
    mask_box<TW>(act, i0, j0, tbx0, tby0, tbx1, tby1);
    float UB = INFINITY;
    bool done = false;
    for (int base = 0; base < G && !done; base += 64) {
      if (sgcost[base] >= UB) break;
      if (STATS) st[ST_BATCHES] += 1;
      // lane-parallel tile bound: cost + distance from the generator to the tile
      const int g = base + lane;
      bool cand = false;
      if (g < G) {
        const float c = sgcost[g];
        const int4 bb = sgbb[g];
        const int dx = max(max(bb.x - tbx1, tbx0 - bb.z), 0);
        const int dy = max(max(bb.y - tby1, tby0 - bb.w), 0);
        const float lb = (c + 0.5f * sqrtf((float)(dx * dx + dy * dy))) * (1.0f - 1e-6f);
        cand = lb < UB;
      }
      u64 cm = ballot(cand);
      while (cm) {
        const int k = base + first_bit(cm);
        cm &= cm - 1;
        const float gc = sgcost[k];
        if (gc >= UB) { done = true; break; }
        const int kind = sgen[k].kind;
        const int gx = sgen[k].x, gy = sgen[k].y;
        bool upd = false;
        if (kind != SPM_GEN_SEGMENT) {
          const int dx = px - gx, dy = py - gy;
          const int d2 = mad24(dx, dx, mul24(dy, dy));
          const float room = best - gc;
          const bool need = active && room > 0.0f && (float)d2 < 4.0f * room * room * (1.0f + 1e-6f);
          const u64 nm = ballot(need);
          if (STATS) st[ST_BOUND] += __popcll(act);
          if (!nm) continue;
          if (STATS) st[ST_VISWAVE] += 1;
          int bx0, by0, bx1, by1;
          mask_box<TW>(nm, i0, j0, bx0, by0, bx1, by1);
          const bool gv = kind == SPM_GEN_VERTEX;
          const u64 bl = wave_blocked_uniform<STATS>(geo, px, py, nm, gx, gy, gv, sgen[k].ux, sgen[k].uy,
                                                     sgen[k].nx, sgen[k].ny, false, 0, 0, 0, 0, bx0, by0, bx1,
                                                     by1, st);
          if (need && !((bl >> lane) & 1ull)) {
            const float c = gc + 0.5f * sqrtf((float)d2);
            if (c < best) { best = c; par = sgen[k].id; upd = true; }
          }
        } else {
          const int ax = gx, ay = gy, bx = sgen[k].x2, by = sgen[k].y2;
          int clamp;
          const RPt q = seg_closest(ax, ay, bx, by, px, py, &clamp);
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
          const float c = gc + dd;
          const bool need = active && c < best;
          const u64 nm = ballot(need);
          if (STATS) st[ST_BOUND] += __popcll(act);
          if (!nm) continue;
          if (STATS) st[ST_VISWAVE] += 1;
          int bx0, by0, bx1, by1;
          mask_box<TW>(nm, i0, j0, bx0, by0, bx1, by1);
          const bool vs = lane_visible_rational(geo, px, py, false, 0, 0, 0, 0, q, need, min(bx0, min(ax, bx)),
                                                min(by0, min(ay, by)), max(bx1, max(ax, bx)),
                                                max(by1, max(ay, by)));
          if (need && vs) { best = c; par = sgen[k].id; upd = true; }
        }
        if (ballot(upd)) {
          if (STATS) st[ST_ACCEPT] += __popcll(ballot(upd));
          UB = wave_max(active ? best : -INFINITY);
        }
      }
    }
  }
  if (valid) {
    const size_t o = (size_t)j * W + i;
    dist[o] = best;
    parent[o] = par;
  }
  if (STATS && lane == 0) {
#pragma unroll
    for (int s = 0; s < 8; ++s) atomicAdd(&stats[s], st[s]);
  }
}

template <int TW>
static void launch_tw(const Dev& d, hipStream_t s) {
  constexpr int TH = 64 / TW;
  const long long tiles = (long long)((d.W + TW - 1) / TW) * ((d.H + TH - 1) / TH);
  const dim3 grid((unsigned)((tiles + 3) / 4));
  if (d.stats)
    hipLaunchKernelGGL((k_pixel<TW, true>), grid, dim3(256), 0, s, d.W, d.H, d.W32, d.misc, d.inside, d.sgen,
                       d.sgcost, d.sgbb, d.edges, d.ext, d.chunks, d.E, d.NC, d.dist, d.parent, d.stats);
  else
    hipLaunchKernelGGL((k_pixel<TW, false>), grid, dim3(256), 0, s, d.W, d.H, d.W32, d.misc, d.inside, d.sgen,
                       d.sgcost, d.sgbb, d.edges, d.ext, d.chunks, d.E, d.NC, d.dist, d.parent, d.stats);
}

hipError_t launch_pixel(const Dev& d, hipStream_t s) {
  if (d.tile_w == 16) launch_tw<16>(d, s);
  else if (d.tile_w == 4) launch_tw<4>(d, s);
  else launch_tw<8>(d, s);
  return hipGetLastError();
}

}  // namespace spm
