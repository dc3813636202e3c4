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

enum { ST_TILES = 0, ST_BATCHES, ST_BOUND, ST_VISWAVE, ST_RELEV, ST_LANEEDGE, ST_OCCL, ST_ACCEPT, ST_CACHE_TEST,
       ST_CACHE_HIT, ST_SEG_LANE, ST_CL_MEMBERS, ST_CL_TRIED, ST_CL_HIDDEN, ST_CL_UMBRA, ST_CL_UMBRA_TESTS, ST_COUNT };

// Occluder cache of one tile: one obstacle edge per lane.  The exact test of
// a candidate generator g against a tile first asks whether a single edge hides
// the whole tile box from g (every segment from the box to g properly crosses
// it, the box strictly on its obstacle side: Procedure 2's shadow of that edge
// covers the tile).  Every lane tries its own edge, so one pass tries 64
// occluders; an edge that the full test finds hiding the box takes the next
// slot (round robin).  Candidates that a tile cannot see are mostly hidden by
// the walls around the tile or around the generator, the same few edges over
// and over, so most tests end here.  A hit is exact (the same test the full
// scan applies to every edge); a miss only falls back to the full test.
struct OccCache {
  unsigned w, v;   // this lane's edge w -> v (obstacle on the left), x | y << 16 (doubled coordinates
                   // are below 2^15); w == v: an empty slot
  int slot;        // next slot to fill (wave-uniform)
  // The umbra of the tile box U (ux0..uy1, the active pixels' box) behind this
  // lane's edge: the points g that the edge hides from every point of U.  For
  // U strictly on the obstacle side (E > 0 on U) and g strictly on the free
  // side (E(g) < 0), seen from g the edge runs clockwise from w to v, and U lies
  // strictly inside that wedge iff every corner P of U satisfies
  // cross(P - w, g - w) < 0 and cross(P - v, g - v) > 0.  Over the corners
  // these are half-planes through w (through v); with E(g) < 0 the binding one
  // is the corner direction most counter-clockwise seen from w (most clockwise
  // seen from v).  So the umbra is the intersection of three open half-planes
  // h_i(g) = A_i gx + B_i gy + C_i < 0: the edge line (i = 0), the tangent
  // through w (1) and the tangent through v (2).  |A|, |B| < 2^15, |C| < 2^30,
  // so each h_i is an exact int32 value.  A lane whose edge does not have U
  // strictly on its obstacle side (or an empty slot) gets h_1 = 1: never.
  int ab0, c0, ab1, c1, ab2, c2;   // (A_i | B_i << 16, C_i)
  unsigned pp0, pp1, pp2;          // max(A_i, 0) | max(B_i, 0) << 16
  int ux0, uy0, ux1, uy1;          // U (wave-uniform)
  __device__ __forceinline__ void reset() {
    w = v = 0u;
    slot = 0;
    ux0 = uy0 = ux1 = uy1 = 0;
    ab0 = c0 = ab1 = ab2 = c2 = 0;
    pp0 = pp1 = pp2 = 0u;
    c1 = 1;
  }
  // Sets this lane's umbra from its edge (every lane; exact integer work).
  __device__ __forceinline__ void set_umbra() {
    const int wx = (int)(w & 0xffffu), wy = (int)(w >> 16), vx = (int)(v & 0xffffu), vy = (int)(v >> 16);
    const int a = wy - vy, b = vx - wx, c = -(a * wx + b * wy);
    const int loE = mad24(a, a > 0 ? ux0 : ux1, mad24(b, b > 0 ? uy0 : uy1, c));
    // corner directions from w: keep the most counter-clockwise (cross(d, e) > 0: e is counter-clockwise of d)
    int dx = ux0 - wx, dy = uy0 - wy;
    auto ccw = [&](int ex, int ey) {
      if (mul24(dx, ey) - mul24(dy, ex) > 0) { dx = ex; dy = ey; }
    };
    ccw(ux1 - wx, uy0 - wy);
    ccw(ux0 - wx, uy1 - wy);
    ccw(ux1 - wx, uy1 - wy);
    // from v: keep the most clockwise
    int ex = ux0 - vx, ey = uy0 - vy;
    auto cw = [&](int fx, int fy) {
      if (mul24(ex, fy) - mul24(ey, fx) < 0) { ex = fx; ey = fy; }
    };
    cw(ux1 - vx, uy0 - vy);
    cw(ux0 - vx, uy1 - vy);
    cw(ux1 - vx, uy1 - vy);
    const bool ok = loE > 0;
    ab0 = pack16(a, b);
    c0 = c;
    // cross(d, g - w) < 0:  -dy gx + dx gy + (dy wx - dx wy) < 0
    ab1 = ok ? pack16(-dy, dx) : 0;
    c1 = ok ? mul24(dy, wx) - mul24(dx, wy) : 1;
    // cross(e, g - v) > 0:  ey gx - ex gy + (ex vy - ey vx) < 0
    ab2 = pack16(ey, -ex);
    c2 = mul24(ex, vy) - mul24(ey, vx);
    pp0 = (unsigned)pack16(max(a, 0), max(b, 0));
    pp1 = ok ? (unsigned)pack16(max(-dy, 0), max(dx, 0)) : 0u;
    pp2 = (unsigned)pack16(max(ey, 0), max(-ex, 0));
  }
  // Does some cached edge hide the point g from the whole of U (all three
  // h_i(g) < 0)?  Tested for the points g = (px, py) of lanes 0..kCluster-1
  // whose bits are set in pts; the bits of the hidden ones are cleared from
  // keep.
  __device__ __forceinline__ void umbra_filter(u64 pts, int px, int py, u64& keep) const {
    const int pg = pack16(px, py);
#pragma unroll
    for (int j = 0; j < kCluster; ++j) {
      if (!((pts >> j) & 1ull)) continue;
      const int g = readlane(pg, j);   // (gx, gy), both below 2^15
      const int h = max(max(dot2(ab0, g, c0), dot2(ab1, g, c1)), dot2(ab2, g, c2));
      if (ballot(h < 0)) keep &= ~(1ull << j);
    }
  }
  // Does some cached edge hide the whole box K (kx0..ky1) from the whole of
  // U?  K lies in the (convex) umbra iff the largest value of each h_i over K
  // is negative.
  // The largest value is the value at the corner (kx0, ky0) plus the positive
  // parts of A_i and B_i times the box's extent (each partial sum is the value
  // at a point of K, so every step stays an exact int32).
  __device__ __forceinline__ bool umbra_hides_box(int kx0, int ky0, int kx1, int ky1) const {
    const int k0 = pack16(kx0, ky0), ext = pack16(kx1 - kx0, ky1 - ky0);   // wave-uniform
    auto hmax = [&](int ab, unsigned pp, int c) { return dot2((int)pp, ext, dot2(ab, k0, c)); };
    return ballot(max(max(hmax(ab0, pp0, c0), hmax(ab1, pp1, c1)), hmax(ab2, pp2, c2)) < 0) != 0ull;
  }
  // does some cached edge hide the box (bx0..by1) from g?
  __device__ __forceinline__ bool hides(int gx, int gy, int bx0, int by0, int bx1, int by1) const {
    const int wx = (int)(w & 0xffffu), wy = (int)(w >> 16), vx = (int)(v & 0xffffu), vy = (int)(v >> 16);
    EdgeRec r;
    r.wx = wx; r.wy = wy; r.vx = vx; r.vy = vy;
    r.a = wy - vy;
    r.b = vx - wx;
    r.c = -(r.a * wx + r.b * wy);
    r.nc = -r.c;
    bool rel, occ;
    edge_vs_cone(r, gx, gy, bx0, by0, bx1, by1, bx0 - gx, bx1 - gx, by0 - gy, by1 - gy, rel, occ);
    return ballot(occ) != 0ull;
  }
  __device__ __forceinline__ void insert(const EdgeRec& r) {   // r wave-uniform
    if (lane_id() == (slot & 63)) {
      w = (unsigned)r.wx | ((unsigned)r.wy << 16);
      v = (unsigned)r.vx | ((unsigned)r.vy << 16);
    }
    ++slot;
  }
  // the same, keeping the umbrae current
  __device__ __forceinline__ void insert_umbra(const EdgeRec& r) {
    insert(r);
    set_umbra();
  }
  // Fills the slots with edges near the box (bx0..by1) whose line has the
  // whole box strictly on its obstacle side (only such an edge can hide the
  // box from anything): the edges of the chunks within 32, then 128 units of
  // the box, until every slot is taken.  The walls around a tile hide most of
  // what it cannot see, so the cache starts warm.
  template <class GEO>
  __device__ void fill_near(const GEO& geo, int bx0, int by0, int bx1, int by1) {
    const int lane = lane_id();
    for (int cb = 0; cb < geo.NC && slot < 64; cb += kWave) {
      const int ci = cb + lane;
      int gap = 1 << 30;
      if (ci < geo.NC) {
        const int4 bb = geo.chunk(ci);
        gap = max(max(max(bb.x - bx1, bx0 - bb.z), max(bb.y - by1, by0 - bb.w)), 0);
      }
      const u64 near = ballot(gap <= 64), mid = ballot(gap > 64 && gap <= 256);
      for (int cl = 0; cl < 2 && slot < 64; ++cl) {
        u64 cm = cl ? mid : near;
        while (cm && slot < 64) {
          const int chunk = cb + first_bit(cm);
          cm &= cm - 1;
          const int e = chunk * kChunk + lane;
          bool ok = false;
          EdgeRec r = {0, 0, 0, 0, 0, 0, 0, 0};
          if (e < geo.E) {
            r = geo.edge(e);
            const int loE = mad24(r.a, r.a > 0 ? bx0 : bx1, mad24(r.b, r.b > 0 ? by0 : by1, r.c));
            ok = loE > 0;
          }
          u64 om = ballot(ok);
          while (om && slot < 64) {
            const int ql = first_bit(om);
            om &= om - 1;
            const unsigned pw = (unsigned)readlane(r.wx, ql) | ((unsigned)readlane(r.wy, ql) << 16);
            const unsigned pv = (unsigned)readlane(r.vx, ql) | ((unsigned)readlane(r.vy, ql) << 16);
            if (lane == slot) { w = pw; v = pv; }
            ++slot;
          }
        }
      }
    }
  }
};

// Least unsigned value over lanes 0..kCluster-1 (a cluster's members),
// returned through a readlane: two quad exchanges and the half-row mirror
// (lane i of each group of 8 takes lane 7 - i) give the least of each group of
// 8, the row mirror that of each row of 16, a broadcast of lane 15 into the
// next row that of lanes 0..31.
__device__ __forceinline__ unsigned min_members_u32(unsigned v) {
  static_assert(kCluster == 8 || kCluster == 16 || kCluster == 32, "cluster size");
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0xB1, 0xF, 0xF, false));    // quad_perm 1,0,3,2
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x4E, 0xF, 0xF, false));    // quad_perm 2,3,0,1
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x141, 0xF, 0xF, false));   // row_half_mirror
  if constexpr (kCluster > 8)
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x140, 0xF, 0xF, false));   // row_mirror
  if constexpr (kCluster > 16)
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xA, 0xF, false));   // row_bcast 15
  return (unsigned)readlane((int)v, kCluster > 16 ? 31 : 0);
}

// Box (doubled pixel-centre coordinates) of the lanes set in m (m != 0; a
// wave-uniform mask, so this is scalar work).  Lane l is column l % TW of row
// l / TW: the rows are the first and last set bit divided by TW, the columns
// the set bits of the OR of all rows (folded by halving shifts).
template <int TW>
__device__ __forceinline__ void mask_box(u64 m, int i0, int j0, int& bx0, int& by0, int& bx1, int& by1) {
  u64 f = m;
#pragma unroll
  for (int s = 32; s >= TW; s >>= 1) f |= f >> s;
  const unsigned cols = (unsigned)f & ((1u << TW) - 1u);
  const int r0 = __builtin_ctzll(m) / TW, r1 = (63 - __builtin_clzll(m)) / TW;
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

// Hardware square root, reciprocal square root and reciprocal (each within 1
// ulp, without the correction steps of the correctly rounded library calls).
// Every value the pixel stage compares or stores comes from these same
// instructions, so orders and ties are the same whichever path computes them.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// (value, walk position) order.  The walk keeps, per lane, the least pair over
// the visible candidates: the generator the cost-ordered walk would settle on
// (ties keep the earlier generator, as the paper's strict depth test does).
// Because the pair order is total, the result does not depend on the order in
// which candidates are tried, so a tile may try a few likely winners (seeds)
// before the walk without changing any output bit.
__device__ __forceinline__ bool lex_less(float v, int k, float best, int bpos) {
  return v < best || (v == best && k < bpos);
}

// Room below an upper bound ub for a generator of cost c, widened by 1e-6 ub so
// that every candidate whose float value can round to ub or below passes the
// square-root-free filters (they are conservative; the exact float compare
// decides).  ub = -inf (no active lane) gives -inf.
__device__ __forceinline__ float room_below(float ub, float c) { return (ub - c) + 1e-6f * ub; }

// conservative test: can a generator with cost c and bounding box (x0..y1) come
// to ub or below anywhere in the box (bx0..by1)?
__device__ __forceinline__ bool box_may_win(float c, int x0, int y0, int x1, int y1, int bx0, int by0, int bx1,
                                            int by1, float ub) {
  const int dx = max(max(x0 - bx1, bx0 - x1), 0);
  const int dy = max(max(y0 - by1, by0 - y1), 0);
  const float room = room_below(ub, c);
  return room > 0.0f && (float)(dx * dx + dy * dy) < 4.0f * room * room * (1.0f + 2e-6f);
}

constexpr int kMaxTried = 8;    // seeds remembered per tile (skipped by the walk)
constexpr int kSeedTries = 128; // candidates one seed search may reject
#ifndef SPM_SEED_TRIES_UNCACHED
#define SPM_SEED_TRIES_UNCACHED 4
#endif
constexpr int kSeedTriesUncached = SPM_SEED_TRIES_UNCACHED;   // the same when each try recomputes every estimate
constexpr int kEstCache = 8;    // seed-search estimates kept in registers per lane
#ifndef SPM_PRIO_TRIES
#define SPM_PRIO_TRIES 3
#endif
constexpr int kPrioTries = SPM_PRIO_TRIES;   // tests after which a tile raises its wave's priority
// the same for the cluster walk, whose tiles nearly all make a few tests (maze: 12 against 3 is 2-3 %
// faster; 8 to 16 are about equal; the other walks prefer 3)
constexpr int kPrioTriesCluster = 12;
#ifndef SPM_SEED_WIDE
#define SPM_SEED_WIDE 4
#endif
constexpr int kSeedWide = SPM_SEED_WIDE;   // candidates per round once a seed search has made kPrioTries tries
// How a tile walks the generators (a template parameter chosen on the host
// from the scene's largest possible generator count):
//   kWalkCached  up to kEstCache * 64 generators: lower-bound order, every
//                estimate in registers;
//   kWalkRefill  up to kEstWalkMax (8192): lower-bound order, the least
//                kEstCache per lane in registers, refilled when needed;
//   kWalkCost    beyond: seed searches, then (cost, id) order.
//   kWalkCluster up to kClusterWalkMax: spatial clusters of kCluster
//                generators in order of a lower bound over the tile, every
//                cluster estimate in registers; a cluster that one edge hides
//                from the whole tile is skipped at once, the members of the
//                others are tried one by one.
enum { kWalkCached = 0, kWalkRefill = 1, kWalkCost = 2, kWalkCluster = 3 };
// Cluster estimates per lane.  Sixteen, even where fewer would do: the walk
// reads slot np of its sorted keys with a wave-uniform np, which the compiler
// turns into one indexed register move for sixteen registers but into a chain
// of compares and selects for eight.
constexpr int kClSlots = 16;
constexpr int kClusterWalkMax = 8192;   // generators
static_assert(kClusterWalkMax <= kClSlots * 64 * kCluster, "cluster slots");
constexpr int kEstWalkMax = 128 * 64;   // a lane owns up to 128 generators (two 64-bit taken masks)
#ifndef SPM_REFILL_AUTO_MAX
#define SPM_REFILL_AUTO_MAX 4096
#endif
constexpr int kRefillAutoMax = SPM_REFILL_AUTO_MAX;   // largest generator count that picks it by default
inline int walk_mode(int gmax) {
  if (gmax <= kEstCache * 64) return kWalkCached;
  if (gmax <= kRefillAutoMax) return kWalkRefill;
  return gmax <= kClusterWalkMax ? kWalkCluster : kWalkCost;
}
#ifndef SPM_SEED_SHARE
#define SPM_SEED_SHARE 1   // later seed searches of a tile skip the candidates earlier ones tried
#endif

// The segment [P, q] for the cheap seed test: a proper crossing with edge r
// (endpoints strictly on opposite sides of line P-q and P, q strictly on
// opposite sides of the edge line).
__device__ __forceinline__ bool seed_crosses(const EdgeRec& r, int px, int py, float qx, float qy) {
  const float dqx = qx - px, dqy = qy - py;
  const float o1 = dqx * (float)(r.wy - py) - dqy * (float)(r.wx - px);
  const float o2 = dqx * (float)(r.vy - py) - dqy * (float)(r.vx - px);
  const float e1 = (float)(r.a * px + r.b * py + r.c);
  const float e2 = r.a * qx + r.b * qy + (float)r.c;
  return o1 * o2 < 0.0f && e1 * e2 < 0.0f;
}

// The point of generator h that P sees (the generator, or a segment's closest
// point); false when h is a corner and the direction toward P enters its own
// interior angle (P cannot see it).
__device__ __forceinline__ bool seed_target(const GenRec* sgen, int h, int px, int py, float& qx, float& qy) {
  const int kind = sgen[h].kind;
  const int gx = sgen[h].x, gy = sgen[h].y;
  qx = (float)gx;
  qy = (float)gy;
  if (kind == SPM_GEN_SEGMENT) {
    const float ex = (float)(sgen[h].x2 - gx), ey = (float)(sgen[h].y2 - gy);
    const float t = fminf(fmaxf(((px - gx) * ex + (py - gy) * ey) * frcp(ex * ex + ey * ey), 0.0f), 1.0f);
    qx = gx + t * ex;
    qy = gy + t * ey;
    return true;
  }
  return !(kind == SPM_GEN_VERTEX &&
           into_interior(sgen[h].ux, sgen[h].uy, gx, gy, sgen[h].nx, sgen[h].ny, px - gx, py - gy));
}

// Takes the least (estimate, generator) pair out of the register cache (lane l,
// slot s holds generator l + 64 s) and returns its generator, or -1 when the
// cache is empty; v = its estimate.
__device__ __forceinline__ int seed_pop(float (&ec)[kEstCache], unsigned& rej, float& v) {
  const int lane = lane_id();
  float bv = INFINITY;
  int bs = 0;
#pragma unroll
  for (int s = 0; s < kEstCache; ++s)
    if (ec[s] < bv) { bv = ec[s]; bs = s; }
  // estimates are >= 0, so their bits order as unsigned; ties go to the lower lane (the lower generator
  // among equal estimates of one slot)
  const unsigned key = __float_as_uint(bv);
  const unsigned mk = wave_min_u32(key);
  if (mk >= 0x7f800000u) return -1;
  const u64 wm = ballot(key == mk);
  if (!wm) return -1;
  const int wl = first_bit(wm);
  const int ws = readlane(bs, wl);
#pragma unroll
  for (int s = 0; s < kEstCache; ++s)
    if (lane == wl && s == ws) { ec[s] = INFINITY; rej |= 1u << s; }
  v = __uint_as_float(mk);
  return wl + 64 * ws;
}

// Puts generator k with estimate v back into the cache (undoes seed_pop).
__device__ __forceinline__ void seed_unpop(float (&ec)[kEstCache], unsigned& rej, int k, float v) {
  const int lane = lane_id();
#pragma unroll
  for (int s = 0; s < kEstCache; ++s)
    if (lane + 64 * s == k) { ec[s] = v; rej &= ~(1u << s); }
}

// One round of a long seed search: the next kSeedWide candidates at once, the
// wavefront split into groups of 64 / kSeedWide lanes, group g testing the
// g-th least remaining candidate against the edges of the chunks its segment's
// box meets (each lane kSeedWide edges of a chunk per step).  Returns the
// least candidate of the round that passes (the one a one-at-a-time search
// would return), -1 if none does, -2 if the cache is empty; n = candidates
// taken.  Candidates after the one returned go back into the cache.
template <bool STATS>
__device__ int seed_round_wide(const Geo& geo, const GenRec* sgen, int px, int py, float (&ec)[kEstCache],
                               unsigned& rej, int& sblk, int& n, u64* st) {
  constexpr int GL = 64 / kSeedWide;   // lanes per group
  const int lane = lane_id();
  const int grp = lane / GL, gl = lane % GL;
  int my = -1;
  int pk[kSeedWide];
  float pv[kSeedWide];
  n = 0;
#pragma unroll
  for (int r = 0; r < kSeedWide; ++r) {
    pk[r] = seed_pop(ec, rej, pv[r]);
    if (pk[r] < 0) break;
    if (grp == r) my = pk[r];
    ++n;
  }
  if (n == 0) return -2;
  // the candidate of group g passes: give back the later ones
  auto found = [&](int g) -> int {
#pragma unroll
    for (int r = 0; r < kSeedWide; ++r)
      if (r > g && r < n) seed_unpop(ec, rej, pk[r], pv[r]);
    n = g + 1;
    int k = pk[0];
#pragma unroll
    for (int r = 1; r < kSeedWide; ++r)
      if (r == g) k = pk[r];
    return k;
  };
  float qx = (float)px, qy = (float)py;
  bool live = my >= 0 && seed_target(sgen, my, px, py, qx, qy);
  if (live && sblk >= 0 && seed_crosses(geo.edges[sblk], px, py, qx, qy)) live = false;
  const int bx0 = min(px, (int)floorf(qx)), bx1 = max(px, (int)ceilf(qx));
  const int by0 = min(py, (int)floorf(qy)), by1 = max(py, (int)ceilf(qy));
  // groups still in the running (bit g), as seen by every lane
  unsigned alive = 0;
  {
    const u64 lb = ballot(live);
#pragma unroll
    for (int g = 0; g < kSeedWide; ++g)
      if ((lb >> (g * GL)) & 1ull) alive |= 1u << g;
  }
  for (int cb = 0; cb < geo.NC && alive; cb += kWave) {
    const bool last = cb + kWave >= geo.NC;
    const int ci = cb + lane;
    int4 cbx = make_int4(1, 1, 0, 0);
    if (ci < geo.NC) cbx = geo.chunks[ci];
    u64 hm[kSeedWide];
#pragma unroll
    for (int g = 0; g < kSeedWide; ++g) {
      const int gx0 = readlane(bx0, g * GL), gx1 = readlane(bx1, g * GL);
      const int gy0 = readlane(by0, g * GL), gy1 = readlane(by1, g * GL);
      hm[g] = ((alive >> g) & 1u) ? ballot(ci < geo.NC && cbx.x <= gx1 && cbx.z >= gx0 && cbx.y <= gy1 &&
                                           cbx.w >= gy0)
                                  : 0ull;
    }
    for (;;) {
      // the least live candidate has no chunk left: nothing can block it any more
      if (last && alive) {
        const int g0 = __builtin_ctz(alive);
        if (!hm[g0]) return found(g0);
      }
      int c = -1;
      bool any = false;
#pragma unroll
      for (int g = 0; g < kSeedWide; ++g) {
        if (hm[g]) {
          const int cg = cb + first_bit(hm[g]);
          hm[g] &= hm[g] - 1;
          if (grp == g) c = cg;
          any = true;
        }
      }
      if (!any) break;
      if (STATS) st[ST_RELEV] += 1;
      bool x = false;
      int xe = -1;
      if (c >= 0) {
#pragma unroll
        for (int m = 0; m < kSeedWide; ++m) {
          const int e = c * kChunk + gl + GL * m;
          if (!x && e < geo.E && seed_crosses(geo.edges[e], px, py, qx, qy)) { x = true; xe = e; }
        }
      }
      const u64 xb = ballot(x);
      if (xb) sblk = readlane(xe, first_bit(xb));
#pragma unroll
      for (int g = 0; g < kSeedWide; ++g)
        if ((xb >> (g * GL)) & ((GL == 64) ? ~0ull : ((1ull << GL) - 1ull))) { alive &= ~(1u << g); hm[g] = 0; }
    }
  }
  return alive ? found(__builtin_ctz(alive)) : -1;
}

// Seed search for one free pixel P (doubled coordinates, wave-uniform): try
// generators in order of cost + |P - x_g(P)| -- the exact value whenever g is
// visible -- until one that P appears to see; that one is P's own winner.
// "Appears": a cheap test, lane-parallel over edges, in which only a proper
// crossing of [P, x_g] with an edge, or a start into a corner's own interior
// angle, blocks.  It may accept a grazing path the exact rule rejects; such a
// seed costs time, never correctness, because the tile re-evaluates every
// seed exactly.  After kPrioTries single tries a search that is still going
// takes its candidates kSeedWide at a time.  Returns the sorted position, or
// -1 after about kSeedTries rejections.
//   rej:  per lane, the cache slots that earlier searches of the tile have
//         taken; they are not tried again.
//   sblk: an edge index (or -1) tried first against each candidate; set to
//         the last edge that blocked one (nearby candidates tend to hide
//         behind the same obstacle).
template <bool STATS>
__device__ int seed_search(const Geo& geo, const GenRec* sgen, const float* sgcost, const int4* sgbb, int G, int px,
                           int py, unsigned& rej, int& sblk, u64* st) {
  const int lane = lane_id();
  // cost + |P - x_g(P)| of sorted generator h
  auto est_of = [&](int h) -> float {
    const int4 hb = sgbb[h];
    if (hb.x == hb.z && hb.y == hb.w) {
      const float dx = (float)(px - hb.x), dy = (float)(py - hb.y);
      return sgcost[h] + 0.5f * fsqrt(dx * dx + dy * dy);
    }
    const float ax = (float)sgen[h].x, ay = (float)sgen[h].y;
    const float ex = (float)sgen[h].x2 - ax, ey = (float)sgen[h].y2 - ay;
    const float t = fminf(fmaxf(((px - ax) * ex + (py - ay) * ey) * frcp(ex * ex + ey * ey), 0.0f), 1.0f);
    const float dx = px - (ax + t * ex), dy = py - (ay + t * ey);
    return sgcost[h] + 0.5f * fsqrt(dx * dx + dy * dy);
  };
  // Up to kEstCache * 64 generators the estimates stay in registers (lane l
  // holds generators l, l + 64, ...) and a tried candidate is crossed out;
  // beyond that each try recomputes them and takes the least pair above the
  // previous candidate.
  const bool cached = G <= kEstCache * 64;
  float ec[kEstCache];
#pragma unroll
  for (int s = 0; s < kEstCache; ++s) {
    const int h = lane + 64 * s;
    ec[s] = (cached && h < G && !(SPM_SEED_SHARE && ((rej >> s) & 1u))) ? est_of(h) : INFINITY;
  }
  if (STATS && cached) st[ST_BATCHES] += (G + 63) / 64;
  float lastv = -INFINITY;
  int lastk = -1;
  for (int it = 0; it < kSeedTries;) {
    if (!cached && it >= kSeedTriesUncached) return -1;
    if (it >= kPrioTries) __builtin_amdgcn_s_setprio(2);
    if (cached && it >= kPrioTries) {
      int n = 0;
      const int k = seed_round_wide<STATS>(geo, sgen, px, py, ec, rej, sblk, n, st);
      if (k >= 0) return k;
      if (k == -2) return -1;
      it += n;
      continue;
    }
    ++it;
    int bk;
    if (cached) {
      float v;
      bk = seed_pop(ec, rej, v);
      if (bk < 0) return -1;
    } else {
      if (STATS) st[ST_BATCHES] += (G + 63) / 64;
      float bv = INFINITY;
      bk = 0x7fffffff;
      for (int h = lane; h < G; h += 64) {
        const float v = est_of(h);
        // the least (v, h) above the previous candidate
        if ((v > lastv || (v == lastv && h > lastk)) && (v < bv || (v == bv && h < bk))) { bv = v; bk = h; }
      }
      const unsigned key = __float_as_uint(bv);
      const unsigned mk = wave_min_u32(key);
      if (mk >= 0x7f800000u) return -1;   // none left
      // lanes holding the least estimate: the least generator among them
      bk = (int)wave_min_u32(key == mk ? (unsigned)bk : 0xffffffffu);
      if (bk < 0 || bk >= G) return -1;
      lastv = __uint_as_float(mk);
      lastk = bk;
    }
    float qx, qy;
    if (!seed_target(sgen, bk, px, py, qx, qy)) continue;
    if (sblk >= 0 && ballot(seed_crosses(geo.edges[sblk], px, py, qx, qy))) continue;
    const int bx0 = min(px, (int)floorf(qx)), bx1 = max(px, (int)ceilf(qx));
    const int by0 = min(py, (int)floorf(qy)), by1 = max(py, (int)ceilf(qy));
    bool blocked = false;
    for (int cb = 0; cb < geo.NC && !blocked; cb += kWave) {
      const int ci = cb + lane;
      bool hit = false;
      if (ci < geo.NC) {
        const int4 cbx = geo.chunks[ci];
        hit = cbx.x <= bx1 && cbx.z >= bx0 && cbx.y <= by1 && cbx.w >= by0;
      }
      u64 cm = ballot(hit);
      while (cm) {
        const int e = (cb + first_bit(cm)) * kChunk + lane;
        cm &= cm - 1;
        if (STATS) st[ST_RELEV] += 1;
        const bool x = e < geo.E && seed_crosses(geo.edges[e], px, py, qx, qy);
        const u64 xb = ballot(x);
        if (xb) {
          sblk = e - lane + first_bit(xb);
          blocked = true;
          break;
        }
      }
    }
    if (!blocked) return bk;
  }
  return -1;
}


// One tile: the per-lane minimum over generators for 64 pixels.  The
// generator tables and the edges come through plain pointers that point
// either into LDS (staged by the kernel) or into global memory.
//
//   prevpos: per lane, the walk position of the winner of the previous tile of
//            the same work item (-1: none).  Its distinct values are tried
//            first (neighbouring pixels mostly share their parent).
//   samples: how many seed searches (seed_search) to run, each from a pixel
//            still without a value after the seeds tried so far.
// Returns this tile's per-lane winner position (for the next tile).
// The cost-sorted generator table as the tile walk reads it: the 64-byte
// records with separate float costs and boxes (global memory, or an LDS copy
// for small scenes).
struct TabFull {
  const GenRec* sgen;
  const float* cost;
  const int4* bb;
  // spatial clusters (cluster walk): per member (sorted position, float cost bits) and box, kCluster
  // per cluster; per cluster the box and least cost
  const int2* clk;
  const int4* clmb;
  const int4* clbb;
  const float* clc;
  int ncl;
  __device__ __forceinline__ float c(int k) const { return cost[k]; }
  __device__ __forceinline__ int4 box(int k) const { return bb[k]; }
  __device__ __forceinline__ int4 seg(int k) const { return make_int4(sgen[k].x, sgen[k].y, sgen[k].x2, sgen[k].y2); }
  // a corner (then nb = its previous and next vertex)?
  __device__ __forceinline__ bool corner(int k, int4& nb) const {
    nb = make_int4(sgen[k].ux, sgen[k].uy, sgen[k].nx, sgen[k].ny);
    return sgen[k].kind == SPM_GEN_VERTEX;
  }
  __device__ __forceinline__ int id(int k) const { return sgen[k].id; }
};
// Edge records packed for LDS (the cluster walk of scenes whose full tables
// do not fit): w and v as x | y << 16 (doubled coordinates are below 2^15);
// the line terms are recomputed, the same integers the ingest stage stores.
// The edge reads of the occluder searches then stay in the CU.
struct GeoPacked {
  const uint2* pe;
  const EdgeExt* ext;
  const int4* chunks;
  int E, NC;
  __device__ __forceinline__ EdgeRec edge(int e) const {
    const uint2 p = pe[e];
    EdgeRec r;
    r.wx = (int)(p.x & 0xffffu);
    r.wy = (int)(p.x >> 16);
    r.vx = (int)(p.y & 0xffffu);
    r.vy = (int)(p.y >> 16);
    r.a = r.wy - r.vy;
    r.b = r.vx - r.wx;
    r.c = -(r.a * r.wx + r.b * r.wy);
    r.nc = -r.c;
    return r;
  }
  __device__ __forceinline__ int4 chunk(int c) const { return chunks[c]; }
};
__host__ __device__ inline size_t packed_edge_lds_bytes(int E, int NC) {
  return (size_t)NC * 16 + (size_t)((E + 1) / 2) * 16;   // chunk boxes, then the packed edges (16-byte units)
}
// The refilled walk also stages the generator boxes and float costs (20 bytes
// a generator, after the packed edges) when the whole staging keeps two
// 512-thread workgroups per CU; its refills then read them from LDS.
constexpr size_t kStageLdsMax = 80 * 1024;
__host__ __device__ inline bool refill_stages_tables(int Gmax, int E, int NC) {
  return packed_edge_lds_bytes(E, NC) + (size_t)Gmax * 20 <= kStageLdsMax;
}

template <int TW, bool STATS, int WALK, class TAB, class GEO>
__device__ __forceinline__ int tile_work(int tile, int W, int H, int W32, int G, const unsigned* __restrict__ inside,
                                         const TAB& tab, const GEO& geo, float* __restrict__ dist,
                                         int* __restrict__ parent, int prevpos, int samples, u64* st) {
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
  int bpos = 0x7fffffff;
  const u64 act = ballot(active);
  if (act) {
    // quadrant upper bounds; quadrant q spans pixel columns i0 + (q & 1) * TW/2 .. + TW/2 - 1 and rows
    // j0 + (q >> 1) * TH/2 .. + TH/2 - 1 (doubled centres below)
    float ubq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ubq[q] = (act & quad_mask<TW>(q)) ? INFINITY : -INFINITY;
    const int qx0 = 2 * i0 + 1, qx1 = qx0 + TW, qy0 = 2 * j0 + 1, qy1 = qy0 + TH;  // lower-half / upper-half starts
    float UB = INFINITY;
    int tried[kMaxTried] = {};
    int ntried = 0;
    int nvis = 0;
    int occ[kOccHints];   // the edges that last hid the whole tile from a generator (most recent first)
#pragma unroll
    for (int h = 0; h < kOccHints; ++h) occ[h] = -1;
    OccCache oc;
    oc.reset();
    int sblk = -1;   // the edge that last blocked a seed candidate

    // Evaluate sorted generator k (cost gc, bounding box x0..y1) for every
    // lane that it could still improve: per-lane filter, wave-level exact
    // visibility, (value, position) acceptance, then the quadrant bounds.
    auto try_gen = [&](int k, float gc, int x0, int y0, int x1, int y1) {
      const bool is_seg = !(x0 == x1 && y0 == y1);
      float cc = 0.0f;  // segment: this lane's candidate value
      int clamp = 0;    // segment: closest point is A (0), B (1) or interior (2)
      int ax = x0, ay = y0, bx = x1, by = y1;
      const int ddx = px - x0, ddy = py - y0;
      const int d2 = mad24(ddx, ddx, mul24(ddy, ddy));   // point or corner: squared doubled distance
      bool need;
      if (!is_seg) {
        // cost + |p - g| <= best  =>  d2 < 4 room^2 (conservative)
        const float room = room_below(best, gc);
        need = active && room > 0.0f && (float)d2 < 4.0f * room * room * (1.0f + 1e-6f);
      } else {
        const int4 sg = tab.seg(k);
        ax = sg.x; ay = sg.y; bx = sg.z; by = sg.w;
        const RPt q = seg_closest(ax, ay, bx, by, px, py, &clamp);
        (void)q;
        float dd;
        if (clamp == 0) {
          dd = 0.5f * fsqrt((float)(mad24(px - ax, px - ax, mul24(py - ay, py - ay))));
        } else if (clamp == 1) {
          dd = 0.5f * fsqrt((float)(mad24(px - bx, px - bx, mul24(py - by, py - by))));
        } else {
          const long long ex = bx - ax, ey = by - ay;
          const long long cr = ex * (py - ay) - ey * (px - ax);
          dd = 0.5f * fabsf((float)cr) * frsq((float)(ex * ex + ey * ey));
        }
        cc = gc + dd;
        need = active && lex_less(cc, k, best, bpos);
        if (STATS) st[ST_SEG_LANE] += __popcll(ballot(active));
      }
      const u64 nm = ballot(need);
      if (STATS) st[ST_BOUND] += __popcll(act);
      if (!nm) return;
      // a tile that keeps testing visibility is on the critical path of the launch: let its wave
      // issue ahead of the others on its SIMD
      if (++nvis == (WALK == kWalkCluster ? kPrioTriesCluster : kPrioTries)) __builtin_amdgcn_s_setprio(2);
      // visibility groups: a point or corner is one group at (x0, y0); a segment has up to three
      // (lanes reaching endpoint A, endpoint B, or an interior point)
      const u64 mA = is_seg ? ballot(need && clamp == 0) : nm;
      const u64 mB = is_seg ? ballot(need && clamp == 1) : 0ull;
      const u64 mI = nm & ~mA & ~mB;
      u64 bl = 0;
      for (int grp = 0; grp < 2; ++grp) {
        const u64 m = grp ? mB : mA;
        if (!m) continue;
        if (STATS) st[ST_VISWAVE] += 1;
        int bx0, by0, bx1, by1;
        mask_box<TW>(m, i0, j0, bx0, by0, bx1, by1);
        const int gx = grp ? bx : ax, gy = grp ? by : ay;
        if (STATS) st[ST_CACHE_TEST] += 1;
        if (oc.hides(gx, gy, bx0, by0, bx1, by1)) {
          if (STATS) st[ST_CACHE_HIT] += 1;
          bl |= m;
          continue;
        }
        int4 nb;
        const bool gv = !is_seg && tab.corner(k, nb);
        int found = -1;
        // no occluder hints: every edge the full test finds goes to the cache, which holds the last 64 and
        // was just tried on this very box and point
        bl |= wave_blocked_uniform<STATS>(geo, px, py, m, gx, gy, gv, gv ? nb.x : 0, gv ? nb.y : 0, gv ? nb.z : 0,
                                          gv ? nb.w : 0, false, 0, 0, 0, 0, bx0, by0, bx1, by1, nullptr, st, &found);
        if (found >= 0) {
          if constexpr (WALK == kWalkCluster || WALK == kWalkRefill) oc.insert_umbra(geo.edge(found));
          else oc.insert(geo.edge(found));
        }
      }
      if (mI) {
        if (STATS) st[ST_VISWAVE] += 1;
        int bx0, by0, bx1, by1;
        mask_box<TW>(mI, i0, j0, bx0, by0, bx1, by1);
        bl |= wave_blocked_perp<STATS>(geo, px, py, mI, ax, ay, bx, by, false, 0, 0, 0, 0, bx0, by0, bx1, by1, occ, st);
      }
      bool upd = false;
      if (need && !((bl >> lane) & 1ull)) {
        if (!is_seg) cc = gc + 0.5f * fsqrt((float)d2);
        if (lex_less(cc, k, best, bpos)) { best = cc; bpos = k; upd = true; }
      }
      const u64 um = ballot(upd);
      if (um) {
        if (STATS) st[ST_ACCEPT] += __popcll(um);
        const float qm = quad_max<TW>(active ? best : -INFINITY);
#pragma unroll
        for (int q = 0; q < 4; ++q) ubq[q] = readlane_f(qm, QL[q]);
        UB = fmaxf(fmaxf(ubq[0], ubq[1]), fmaxf(ubq[2], ubq[3]));
      }
    };
    if constexpr (WALK == kWalkCached) {
      // Up to kEstCache * 64 generators: every estimate fits in the registers
      // (lane l, slot q: generator l + 64 q), the same order as below without
      // refills.
      int bx0, by0, bx1, by1;
      mask_box<TW>(act, i0, j0, bx0, by0, bx1, by1);
      float ec[kEstCache];
#pragma unroll
      for (int q = 0; q < kEstCache; ++q) {
        const int h = lane + 64 * q;
        float v = INFINITY;
        if (h < G) {
          const int4 b = tab.box(h);
          const float dx = (float)max(max(b.x - bx1, bx0 - b.z), 0), dy = (float)max(max(b.y - by1, by0 - b.w), 0);
          v = (tab.c(h) + 0.5f * fsqrt(dx * dx + dy * dy)) * (1.0f - 4e-6f);
        }
        ec[q] = v;
      }
      unsigned rej = 0;
      for (;;) {
        float m;
        const int k = seed_pop(ec, rej, m);
        if (k < 0 || m > UB) break;
        if (STATS) st[ST_BATCHES] += 1;
        const int4 kb = tab.box(k);
        const float kc = unif(tab.c(k));
        const int kx0 = uni(kb.x), ky0 = uni(kb.y), kx1 = uni(kb.z), ky1 = uni(kb.w);
        if (!(box_may_win(kc, kx0, ky0, kx1, ky1, qx0, qy0, qx1 - 2, qy1 - 2, ubq[0]) ||
              box_may_win(kc, kx0, ky0, kx1, ky1, qx1, qy0, qx1 + TW - 2, qy1 - 2, ubq[1]) ||
              box_may_win(kc, kx0, ky0, kx1, ky1, qx0, qy1, qx1 - 2, qy1 + TH - 2, ubq[2]) ||
              box_may_win(kc, kx0, ky0, kx1, ky1, qx1, qy1, qx1 + TW - 2, qy1 + TH - 2, ubq[3])))
          continue;
        try_gen(k, kc, kx0, ky0, kx1, ky1);
      }
    } else if constexpr (WALK == kWalkCluster) {
      // Spatial clusters of kCluster generators in order of a lower bound
      // over the active pixels' box, cost + |box - cluster box| (shaded as in
      // the other walks); every member's own bound is at least its cluster's,
      // so the walk stops once the least cluster estimate exceeds the tile's
      // largest value.  A cluster that one cached edge hides from the whole
      // box is skipped; the members of the others are tried in turn.
      int bx0, by0, bx1, by1;
      mask_box<TW>(act, i0, j0, bx0, by0, bx1, by1);
      oc.fill_near(geo, bx0, by0, bx1, by1);
      oc.ux0 = bx0; oc.uy0 = by0; oc.ux1 = bx1; oc.uy1 = by1;
      oc.set_umbra();
      auto est_of = [&](const int4& b, float c) -> float {
        const float dx = (float)max(max(b.x - bx1, bx0 - b.z), 0), dy = (float)max(max(b.y - by1, by0 - b.w), 0);
        return (c + 0.5f * fsqrt(dx * dx + dy * dy)) * (1.0f - 4e-6f);
      };
      // Lane l holds clusters l + 64 q.  Their keys -- the estimate's bits (non-negative floats order as
      // unsigned) with the low four replaced by q, which only lowers a lower bound -- are sorted within
      // the lane once (a bitonic network on registers); the walk then takes the least of the lanes'
      // first untaken keys.
      unsigned key[kClSlots];
#pragma unroll
      for (int q = 0; q < kClSlots; ++q) {
        const int c = lane + 64 * q;
        const float e = c < tab.ncl ? est_of(tab.clbb[c], tab.clc[c]) : INFINITY;
        key[q] = (__float_as_uint(e) & ~15u) | (unsigned)q;
      }
#pragma unroll
      for (int kk = 2; kk <= kClSlots; kk <<= 1)
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1)
#pragma unroll
          for (int i = 0; i < kClSlots; ++i) {
            const int l = i ^ jj;
            if (l > i) {
              const unsigned lo = min(key[i], key[l]), hi = max(key[i], key[l]);
              key[i] = (i & kk) == 0 ? lo : hi;
              key[l] = (i & kk) == 0 ? hi : lo;
            }
          }
      unsigned hk = key[0];   // this lane's first untaken key
      int ptr = 0;
      for (;;) {
        const unsigned mk = wave_min_u32(hk);
        if (mk >= 0x7f800000u || __uint_as_float(mk & ~15u) > UB) break;
        const int wl = first_bit(ballot(hk == mk));
        const int c = wl + 64 * (int)(mk & 15u);
        const int np = readlane(ptr, wl) + 1;
        if (lane == wl) {
          // np is wave-uniform: one indexed register move
          hk = np < kClSlots ? key[np & (kClSlots - 1)] : 0xffffffffu;
          ptr = np;
        }
        if (STATS) st[ST_BATCHES] += 1;
        const int4 kb = tab.clbb[c];
        const int cx0 = uni(kb.x), cy0 = uni(kb.y), cx1 = uni(kb.z), cy1 = uni(kb.w);
        if (STATS) st[ST_CACHE_TEST] += 1;
        if (oc.umbra_hides_box(cx0, cy0, cx1, cy1)) {
          if (STATS) st[ST_CACHE_HIT] += 1;
          if (STATS) st[ST_CL_HIDDEN] += 1;
          continue;
        }
        int k = -1;
        float kc = INFINITY, ek = INFINITY;
        int4 b = make_int4(0, 0, 0, 0);
        if (lane < kCluster) {
          // the members' records are stored cluster by cluster: two coalesced loads
          const int2 kk = tab.clk[c * kCluster + lane];
          b = tab.clmb[c * kCluster + lane];
          k = kk.x;
          kc = __int_as_float(kk.y);   // +inf (and an empty box) past the end: then ek = +inf
          ek = est_of(b, kc);
        }
        u64 mm = ballot(k >= 0 && ek <= UB);
        if (STATS) st[ST_CL_MEMBERS] += __popcll(mm);
        if (mm) {
          // point members that a cached edge hides from the whole tile: all tested in one pass, the
          // umbra coefficients unpacked once (segment members go on to the full test)
          const u64 pts = mm & ballot(b.x == b.z && b.y == b.w);
          oc.umbra_filter(pts, b.x, b.y, mm);
          if (STATS) st[ST_CL_UMBRA] += __popcll(pts & ~mm);
          if (STATS) st[ST_CL_UMBRA_TESTS] += __popcll(pts);
        }
        while (mm) {
          // the least estimate first (the likely winner tightens the bounds for the rest)
          const float e_here = ((mm >> lane) & 1ull) ? ek : INFINITY;
          const unsigned mk = min_members_u32(__float_as_uint(e_here));
          const int jl = first_bit(ballot(__float_as_uint(e_here) == mk) & mm);
          mm &= ~(1ull << jl);
          if (__uint_as_float(mk) > UB) break;   // the bounds tightened since: the rest are larger still
          // (the quadrant bounds of the other walks reject about 1 % of these members here: not worth
          // their uniform float work; try_gen's per-lane bound decides)
          const int gx0 = readlane_i(b.x, jl), gy0 = readlane_i(b.y, jl), gx1 = readlane_i(b.z, jl),
                    gy1 = readlane_i(b.w, jl);
          if (STATS) st[ST_CL_TRIED] += 1;
          try_gen(readlane_i(k, jl), readlane_f(kc, jl), gx0, gy0, gx1, gy1);
        }
      }
    } else if constexpr (WALK == kWalkRefill) {
      // All generators in order of a lower bound of their value over the
      // active pixels' box, cost + |box - box(g)| (shaded down by 4e-6 so that
      // rounding keeps it below every pixel's float value).  Lane l owns the
      // generators l + 64 j; it keeps the kEstCache least of those not yet
      // taken in registers, and T is the least estimate left out of every
      // lane's cache: while the least cached estimate is at most T it is the
      // least of all, else the caches are refilled.  Once the least estimate
      // exceeds the tile's largest value no generator can improve any pixel.
      // The first candidates are the likely winners, so the bounds tighten at
      // once and no seed search is needed.
      int bx0, by0, bx1, by1;
      mask_box<TW>(act, i0, j0, bx0, by0, bx1, by1);
      // the occluder cache starts with the edges around the tile; their umbrae hide single candidates
      oc.fill_near(geo, bx0, by0, bx1, by1);
      oc.ux0 = bx0; oc.uy0 = by0; oc.ux1 = bx1; oc.uy1 = by1;
      oc.set_umbra();
      auto est_box = [&](int h) -> float {
        const int4 b = tab.box(h);
        const float dx = (float)max(max(b.x - bx1, bx0 - b.z), 0), dy = (float)max(max(b.y - by1, by0 - b.w), 0);
        return (tab.c(h) + 0.5f * fsqrt(dx * dx + dy * dy)) * (1.0f - 4e-6f);
      };
      const int nj = lane < G ? (G - lane + 63) / 64 : 0;   // generators this lane owns
      float ec[kEstCache];
      int ej[kEstCache];
      u64 taken0 = 0, taken1 = 0;   // per lane: the j already taken out (j < 64, j >= 64)
      auto is_taken = [&](int j) -> bool { return ((j < 64 ? taken0 : taken1) >> (j & 63)) & 1ull; };
      float T = INFINITY;   // least estimate left out of the caches (wave-uniform)
      auto refill = [&]() {
        float tl = INFINITY;
#pragma unroll
        for (int q = 0; q < kEstCache; ++q) {
          ec[q] = (q < nj && !((taken0 >> q) & 1ull)) ? est_box(lane + 64 * q) : INFINITY;
          ej[q] = q;
        }
        for (int j = kEstCache; j < nj; ++j) {
          if (is_taken(j)) continue;
          const float v = est_box(lane + 64 * j);
          float mx = ec[0];
          int ms = 0;
#pragma unroll
          for (int q = 1; q < kEstCache; ++q)
            if (ec[q] > mx) { mx = ec[q]; ms = q; }
          if (v < mx) {
            tl = fminf(tl, mx);
#pragma unroll
            for (int q = 0; q < kEstCache; ++q)
              if (q == ms) { ec[q] = v; ej[q] = j; }
          } else {
            tl = fminf(tl, v);
          }
        }
        T = __uint_as_float(wave_min_u32(__float_as_uint(tl)));
      };
      refill();
      // every pass takes a generator out or refills (after which the least cached estimate is at most T)
      for (int pass = 0; pass < 2 * G + 2; ++pass) {
        float bv = INFINITY;
        int bs = 0;
#pragma unroll
        for (int q = 0; q < kEstCache; ++q)
          if (ec[q] < bv) { bv = ec[q]; bs = q; }
        const unsigned key = __float_as_uint(bv);
        const unsigned mk = wave_min_u32(key);
        const float m = __uint_as_float(mk);
        if (m > T) {   // a generator left out of the caches may come first
          refill();
          continue;
        }
        if (mk >= 0x7f800000u || m > UB) break;
        const int wl = first_bit(ballot(key == mk));
        int jq = ej[0];
#pragma unroll
        for (int q = 1; q < kEstCache; ++q)
          if (q == bs) jq = ej[q];
        if (lane == wl) {
          if (jq < 64) taken0 |= 1ull << jq;
          else taken1 |= 1ull << (jq - 64);
#pragma unroll
          for (int q = 0; q < kEstCache; ++q)
            if (q == bs) ec[q] = INFINITY;
        }
        const int k = wl + 64 * readlane_i(jq, wl);
        if (STATS) st[ST_BATCHES] += 1;
        const int4 kb = tab.box(k);
        const float kc = unif(tab.c(k));
        const int kx0 = uni(kb.x), ky0 = uni(kb.y), kx1 = uni(kb.z), ky1 = uni(kb.w);
        if (!(box_may_win(kc, kx0, ky0, kx1, ky1, qx0, qy0, qx1 - 2, qy1 - 2, ubq[0]) ||
              box_may_win(kc, kx0, ky0, kx1, ky1, qx1, qy0, qx1 + TW - 2, qy1 - 2, ubq[1]) ||
              box_may_win(kc, kx0, ky0, kx1, ky1, qx0, qy1, qx1 - 2, qy1 + TH - 2, ubq[2]) ||
              box_may_win(kc, kx0, ky0, kx1, ky1, qx1, qy1, qx1 + TW - 2, qy1 + TH - 2, ubq[3])))
          continue;
        // a point that one cached edge hides from the whole tile
        if (kx0 == kx1 && ky0 == ky1 && oc.umbra_hides_box(kx0, ky0, kx1, ky1)) continue;
        try_gen(k, kc, kx0, ky0, kx1, ky1);
      }
    } else {
    // Seeds first: the previous tile's winners (distinct values), then seed
    // searches from pixels that still have no value.  Each is evaluated
    // exactly for every lane and remembered, so the walk skips it.
    {
      u64 pm = ballot(prevpos >= 0 && prevpos < G);
      int samples_left = samples;
      unsigned rej = 0;   // per lane: estimate-cache slots an earlier search of this tile has tried
      while (ntried < kMaxTried) {
        int k = -1;
        if (pm) {
          k = readlane_i(prevpos, first_bit(pm));
          pm &= ~ballot(prevpos == k);
        } else {
          const u64 un = ballot(active && best == INFINITY);
          if (samples_left <= 0 || !un) break;
          --samples_left;
          // sample the first pixel without a value, starting from the tile centre
          const u64 hi = un & ~((1ull << ((TH / 2) * TW + TW / 2)) - 1ull);
          const int l = first_bit(hi ? hi : un);
          k = seed_search<STATS>(geo, tab.sgen, tab.cost, tab.bb, G, readlane_i(px, l), readlane_i(py, l), rej, sblk,
                                 st);
          bool seen = k < 0;
#pragma unroll
          for (int t = 0; t < kMaxTried; ++t) seen |= t < ntried && tried[t] == k;
          if (seen) break;   // nothing new to try: the walk decides
        }
#pragma unroll
        for (int t = 0; t < kMaxTried; ++t)
          if (t == ntried) tried[t] = k;
        ntried = min(ntried + 1, kMaxTried);
        const int4 kb = tab.box(k);
        try_gen(k, unif(tab.c(k)), uni(kb.x), uni(kb.y), uni(kb.z), uni(kb.w));
      }
    }
    // the walk in (cost, id) order
    const int g = lane;   // this lane's generator within a walk batch is base + g
    for (int base = 0; base < G; base += 64) {
      if (tab.c(base) > UB) break;
      if (STATS) st[ST_BATCHES] += 1;
      // lane-parallel tile bound against the four quadrants
      float c = INFINITY;
      int4 bb = make_int4(0, 0, 0, 0);
      if (base + g < G) {
        c = tab.c(base + g);
        bb = tab.box(base + g);
      }
      auto bound = [&]() {
        return base + g < G && (box_may_win(c, bb.x, bb.y, bb.z, bb.w, qx0, qy0, qx1 - 2, qy1 - 2, ubq[0]) ||
                                box_may_win(c, bb.x, bb.y, bb.z, bb.w, qx1, qy0, qx1 + TW - 2, qy1 - 2, ubq[1]) ||
                                box_may_win(c, bb.x, bb.y, bb.z, bb.w, qx0, qy1, qx1 - 2, qy1 + TH - 2, ubq[2]) ||
                                box_may_win(c, bb.x, bb.y, bb.z, bb.w, qx1, qy1, qx1 + TW - 2, qy1 + TH - 2, ubq[3]));
      };
      u64 cm = ballot(bound());
#pragma unroll
      for (int t = 0; t < kMaxTried; ++t) {
        const int o = tried[t] - base;
        if (t < ntried && o >= 0 && o < 64) cm &= ~(1ull << o);
      }
      bool done = false;
      while (cm) {
        const int jl = first_bit(cm);
        cm &= cm - 1;
        const float gc = readlane_f(c, jl);
        if (gc > UB) { done = true; break; }
        const float ub0 = UB;
        try_gen(base + jl, gc, readlane_i(bb.x, jl), readlane_i(bb.y, jl), readlane_i(bb.z, jl),
                readlane_i(bb.w, jl));
        if (UB != ub0) cm &= ballot(bound());   // the bounds tightened: drop what they now exclude
      }
      if (done) break;
    }
    }
  }
  if (valid) {
    const size_t o = (size_t)j * W + i;
    dist[o] = best;
    parent[o] = best < INFINITY ? tab.id(bpos) : -1;
  }
  __builtin_amdgcn_s_setprio(0);
  return best < INFINITY ? bpos : -1;
}

#ifndef SPM_TILE_ORDER
#define SPM_TILE_ORDER 1   // hand out work items by k_tile_order's classes (0: row-major)
#endif
constexpr size_t kPixelLdsMax = 64 * 1024;
#ifndef SPM_PIXEL_MIN_WAVES
#define SPM_PIXEL_MIN_WAVES 4   // waves per SIMD the register budget of k_pixel is sized for
#endif
#ifndef SPM_PIXEL_MIN_WAVES_CACHED
#define SPM_PIXEL_MIN_WAVES_CACHED 6   // the same for the register-cached walk (80 VGPRs)
#endif

size_t pixel_lds_bytes(int Gmax, int E, int NC) {
  return (size_t)Gmax * (sizeof(GenRec) + 4 + 16) + 16 + (size_t)E * sizeof(EdgeRec) + (size_t)NC * 16;
}

// Work order of the pixel stage.  How long a tile takes grows with how many
// generators come near to winning in it: far (in geodesic terms) from the
// sources, behind obstacles, the cost-ordered walk and the seed searches meet
// many candidates that the tile cannot see.  The lower bound
//   lb = min_g cost(g) + |c - box(g)|
// at the centre c of a work item ranks items well by that time, so items are
// handed out class by class, largest lb first (kOrderBins classes of equal
// width over 0 .. (W + H) / 2 domain units, the last one open-ended): the long
// items start at the beginning of the launch instead of ending it.  No output
// depends on the order in which items run.  One wavefront per item, lanes
// over the cost-sorted generators (staged in LDS when LDS is set); each
// workgroup takes kOrderItems items and appends them to their classes with
// one atomic per class.
constexpr int kOrderThreads = 512;
#ifndef SPM_ORDER_ITEMS
#define SPM_ORDER_ITEMS 64
#endif
constexpr int kOrderItems = SPM_ORDER_ITEMS;   // work items per workgroup of k_tile_order
constexpr size_t kOrderLdsMax = 48 * 1024;

template <int TW, bool LDS>
__global__ __launch_bounds__(kOrderThreads) void k_tile_order(int W, int H, int strip, int Gcap,
                                                              const int* __restrict__ misc,
                                                              const float* __restrict__ sgcost_g,
                                                              const int4* __restrict__ sgbb_g, int* __restrict__ obins,
                                                              int* __restrict__ order, int ocap) {
  constexpr int TH = 64 / TW;
  constexpr int kPerWave = kOrderItems / (kOrderThreads / 64);
  extern __shared__ int4 osm[];
  __shared__ int lcount[kOrderBins], lbase[kOrderBins];
  __shared__ int icls[kOrderItems], islot[kOrderItems];
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / 64;
  if (tid < kOrderBins) lcount[tid] = 0;
  const int G = misc[MISC_REACHED];
  const float* sgcost = sgcost_g;
  const int4* sgbb = sgbb_g;
  if (LDS) {
    int4* s_bb = osm;
    float* s_cost = (float*)(osm + Gcap);
    for (int k = tid; k < G; k += kOrderThreads) { s_bb[k] = sgbb_g[k]; s_cost[k] = sgcost_g[k]; }
    sgbb = s_bb;
    sgcost = s_cost;
  }
  __syncthreads();
  const int ntx = (W + TW - 1) / TW, nty = (H + TH - 1) / TH;
  const int spr = (ntx + strip - 1) / strip;
  const int nitems = spr * nty;
  const float scale = (float)(2 * kOrderBins) / (float)(W + H);
  // the wavefront's kPerWave items in one pass over the generators: each generator's record is read
  // once for all of them
  int cx[kPerWave], cy[kPerWave];
  float lb[kPerWave];
#pragma unroll
  for (int k = 0; k < kPerWave; ++k) {
    const int item = min(blockIdx.x * kOrderItems + wv * kPerWave + k, nitems - 1);
    const int ty = item / spr, sx = item - ty * spr;
    const int t0 = sx * strip, t1 = min(t0 + strip, ntx);
    cx[k] = (t0 + t1) * TW;   // item centre, doubled coordinates
    cy[k] = (2 * ty + 1) * TH;
    lb[k] = INFINITY;
  }
  for (int h0 = 0; h0 < G; h0 += 64) {
    // the generators are in cost order: once the least cost of the next 64 reaches every item's bound
    // found so far, none of the rest can lower one (checked every eighth step)
    if (h0 > 0 && (h0 & 511) == 0) {
      float most = 0.0f;
#pragma unroll
      for (int k = 0; k < kPerWave; ++k) most = fmaxf(most, __uint_as_float(wave_min_u32(__float_as_uint(lb[k]))));
      if (unif(sgcost[h0]) >= most) break;
    }
    const int h = h0 + lane;
    if (h >= G) continue;
    const int4 b = sgbb[h];
    const float ch = sgcost[h];
#pragma unroll
    for (int k = 0; k < kPerWave; ++k) {
      const float dx = (float)max(max(b.x - cx[k], cx[k] - b.z), 0), dy = (float)max(max(b.y - cy[k], cy[k] - b.w), 0);
      lb[k] = fminf(lb[k], ch + 0.5f * fsqrt(dx * dx + dy * dy));
    }
  }
#pragma unroll
  for (int k = 0; k < kPerWave; ++k) {
    const int li = wv * kPerWave + k;
    if (blockIdx.x * kOrderItems + li >= nitems) break;
    // lb >= 0, so its bits order as unsigned
    const float f = __uint_as_float(wave_min_u32(__float_as_uint(lb[k]))) * scale;
    const int c = f < (float)(kOrderBins - 1) ? (int)f : kOrderBins - 1;
    if (lane == 0) {
      const int cls = kOrderBins - 1 - c;
      icls[li] = cls;
      islot[li] = atomicAdd(&lcount[cls], 1);
    }
  }
  __syncthreads();
  if (tid < kOrderBins) lbase[tid] = lcount[tid] ? atomicAdd(&obins[tid], lcount[tid]) : 0;
  __syncthreads();
  if (tid < kOrderItems) {
    const int item = blockIdx.x * kOrderItems + tid;
    if (item < nitems) order[(size_t)icls[tid] * ocap + lbase[icls[tid]] + islot[tid]] = item;
  }
}

// Persistent kernel.  A work item is a strip of `strip` consecutive tiles of
// one tile row, done left to right, so that each tile after the first is
// seeded with the winners of the tile to its left.  Every wavefront takes its
// global index as its first item; further items come from kQueues device
// queues (qctr), one per group of workgroups that the dispatcher places on
// the same XCD, each handing out every kQueues-th item.  That keeps the
// number of contended atomics small: a single queue for every wavefront of
// the chip serialises at one address.  Queue positions map to items through
// the work order of k_tile_order when one is given (order != nullptr).
//
// LDSD: the cost-sorted generator table, the edges and the chunk boxes are
// first staged in LDS (when they fit 64 KB), so the wave-uniform reads of the
// hot loops are LDS broadcasts instead of L2 round trips.  (Compact 20-byte
// generator and 8-byte edge records in 160 KB of LDS per 1024-thread
// workgroup were measured for the large scenes: slower than L2, since the
// large scenes are bound by VALU issue, not by load latency.)
constexpr int kPixelThreads = 512;

template <int TW, bool STATS, int WALK, class TAB, class GEO>
__device__ __forceinline__ void pixel_items(int W, int H, int W32, int G, const unsigned* __restrict__ inside,
                                            const TAB& tab, const GEO& geo, float* __restrict__ dist,
                                            int* __restrict__ parent, int strip, int samples,
                                            int* __restrict__ qctr, const int* __restrict__ order, int ocap,
                                            const int* opre, u64* st) {
  constexpr int TH = 64 / TW;
  const int ntx = (W + TW - 1) / TW, nty = (H + TH - 1) / TH;
  const int spr = (ntx + strip - 1) / strip;   // strips per tile row
  const int nitems = spr * nty;
  const int wpb = blockDim.x / kWave;
  const int nw = gridDim.x * wpb;                       // wavefronts in the grid
  const int nq = min(kQueues, (int)gridDim.x);          // queues in use (each has a workgroup)
  const int q = blockIdx.x % nq;
  // the item at queue position n: the (n - opre[c])-th of class c, the last class starting at or before n
  auto item_at = [&](int n) -> int {
    if (!order) return n;
    const int l = lane_id();
    const int c = __popcll(ballot(l < kOrderBins && opre[l] <= n)) - 1;
    const int it = order[(size_t)c * ocap + (n - opre[c])];
    return (unsigned)it < (unsigned)nitems ? it : n;
  };
  int pos = blockIdx.x * wpb + (threadIdx.x / kWave);  // first position: the wavefront's index
  while (pos < nitems) {
    const int item = uni(item_at(pos));
    const int ty = item / spr, sx = item - ty * spr;
    const int t0 = sx * strip, t1 = min(t0 + strip, ntx);
    int prev = -1;
    for (int t = t0; t < t1; ++t)
      prev = tile_work<TW, STATS, WALK>(ty * ntx + t, W, H, W32, G, inside, tab, geo, dist, parent, prev, samples,
                                        st);
    int n = 0;
    if (lane_id() == 0) n = atomicAdd(&qctr[q * kQueueStride], 1);
    n = __shfl(n, 0, 64);
    pos = nw + q + nq * n;
  }
}

template <int TW, bool STATS, bool LDSD, int WALK>
__global__ __launch_bounds__(kPixelThreads, WALK == kWalkCached ? SPM_PIXEL_MIN_WAVES_CACHED : SPM_PIXEL_MIN_WAVES)
void k_pixel(int W, int H, int W32, int Gmax, int* misc, const unsigned* __restrict__ inside,
             const GenRec* __restrict__ sgen_g, const float* __restrict__ sgcost_g, const int4* __restrict__ sgbb_g,
             const EdgeRec* __restrict__ edges_g, const EdgeExt* __restrict__ ext, const int4* __restrict__ chunks_g,
             int E, int NC, const int2* __restrict__ clk, const int4* __restrict__ clmb,
             const int4* __restrict__ clbb, const float* __restrict__ clc,
             float* __restrict__ dist, int* __restrict__ parent, int strip, int samples, int* __restrict__ qctr,
             const int* __restrict__ obins, const int* __restrict__ order, int ocap, u64* __restrict__ stats) {
  extern __shared__ int4 smem[];
  __shared__ int opre[kOrderBins];   // first queue position of each work class
  const int G = misc[MISC_REACHED];
  const int t = threadIdx.x, nt = blockDim.x;
  u64 st[ST_COUNT] = {};
  if (order && t < 64) {
    // exclusive prefix of the class sizes
    const int l = lane_id();
    int v = l < kOrderBins ? obins[l] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(v, o, 64);
      if (l >= o) v += u;
    }
    if (l < kOrderBins) opre[l] = v - obins[l];
  }
  TabFull tab{sgen_g, sgcost_g, sgbb_g, clk, clmb, clbb, clc, (misc[MISC_G] + kCluster - 1) / kCluster};
  Geo geo{edges_g, ext, chunks_g, E, NC};
  if (LDSD) {
    GenRec* s_gen = (GenRec*)smem;
    int4* s_bb = (int4*)(s_gen + Gmax);
    EdgeRec* s_edges = (EdgeRec*)(s_bb + Gmax);
    int4* s_chunks = (int4*)(s_edges + E);
    float* s_cost = (float*)(s_chunks + NC);
    const int4* src = (const int4*)sgen_g;
    for (int k = t; k < G * 4; k += nt) ((int4*)s_gen)[k] = src[k];
    for (int k = t; k < G; k += nt) { s_bb[k] = sgbb_g[k]; s_cost[k] = sgcost_g[k]; }
    const int4* se = (const int4*)edges_g;
    for (int k = t; k < E * 2; k += nt) ((int4*)s_edges)[k] = se[k];
    for (int k = t; k < NC; k += nt) s_chunks[k] = chunks_g[k];
    tab.sgen = s_gen;
    tab.cost = s_cost;
    tab.bb = s_bb;
    geo.edges = s_edges;
    geo.chunks = s_chunks;
  }
  if constexpr (!LDSD && (WALK == kWalkCluster || WALK == kWalkRefill)) {
    // chunk boxes, then the packed edges (then, for the refilled walk, boxes and costs)
    int4* s_chunks = smem;
    uint2* s_pe = (uint2*)(s_chunks + NC);
    for (int k = t; k < NC; k += nt) s_chunks[k] = chunks_g[k];
    for (int k = t; k < E; k += nt) {
      const EdgeRec r = edges_g[k];
      s_pe[k] = make_uint2((unsigned)r.wx | ((unsigned)r.wy << 16), (unsigned)r.vx | ((unsigned)r.vy << 16));
    }
    if constexpr (WALK == kWalkRefill) {
      if (refill_stages_tables(Gmax, E, NC)) {
        int4* s_bb = smem + packed_edge_lds_bytes(E, NC) / 16;
        float* s_cost = (float*)(s_bb + Gmax);
        for (int k = t; k < G; k += nt) { s_bb[k] = sgbb_g[k]; s_cost[k] = sgcost_g[k]; }
        tab.bb = s_bb;
        tab.cost = s_cost;
      }
    }
    __syncthreads();
    const GeoPacked gp{s_pe, ext, s_chunks, E, NC};
    pixel_items<TW, STATS, WALK>(W, H, W32, G, inside, tab, gp, dist, parent, strip, samples, qctr, order, ocap,
                                 opre, st);
  } else {
    __syncthreads();
    pixel_items<TW, STATS, WALK>(W, H, W32, G, inside, tab, geo, dist, parent, strip, samples, qctr, order, ocap,
                                 opre, st);
  }
  if (STATS && lane_id() == 0) {
#pragma unroll
    for (int s = 0; s < ST_COUNT; ++s) atomicAdd(&stats[s], st[s]);
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

// Spatial clusters for the cluster walk: kCluster consecutive positions of the
// spatial generator order (sources first, then corners in Morton order of
// their edges) form a cluster; its members are their cost-sorted positions
// (-1 for an unreached generator or past the end), stored with their float
// cost and box in cluster order, its box the union of their boxes and its
// cost their least float cost.  One thread per position; the
// kCluster threads of a cluster are neighbouring lanes of one wavefront.
__global__ __launch_bounds__(256) void k_clusters(const int* __restrict__ misc, const int* __restrict__ gorder,
                                                  const int* __restrict__ krank, const int4* __restrict__ sgbb,
                                                  const float* __restrict__ sgcost, int2* __restrict__ clk,
                                                  int4* __restrict__ clmb, int4* __restrict__ clbb,
                                                  float* __restrict__ clc, int Gmax) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int Gc = misc[MISC_G];
  const int ncl = (Gc + kCluster - 1) / kCluster;
  int k = -1;
  if (p < Gc) k = krank[gorder[p]];
  int4 b = make_int4(1 << 20, 1 << 20, -(1 << 20), -(1 << 20));
  float c = INFINITY;
  if (k >= 0) {
    b = sgbb[k];
    c = sgcost[k];
  }
  const int4 own_b = k >= 0 ? b : make_int4(0, 0, 0, 0);
  const float own_c = c;
#pragma unroll
  for (int o = 1; o < kCluster; o <<= 1) {
    b.x = min(b.x, __shfl_xor(b.x, o, 64));
    b.y = min(b.y, __shfl_xor(b.y, o, 64));
    b.z = max(b.z, __shfl_xor(b.z, o, 64));
    b.w = max(b.w, __shfl_xor(b.w, o, 64));
    c = fminf(c, __shfl_xor(c, o, 64));
  }
  if (p < ncl * kCluster && p < ((Gmax + kCluster - 1) / kCluster) * kCluster) {
    clk[p] = make_int2(k, __float_as_int(own_c));
    clmb[p] = own_b;
    if (p % kCluster == 0) {
      clbb[p / kCluster] = c < INFINITY ? b : make_int4(0, 0, 0, 0);
      clc[p / kCluster] = c;
    }
  }
}

// phase 0 queues what the pixel kernel reads besides the generator tables
// (the cluster tables of the cluster walk, the work order when it is not built
// in the sort's launch); phase 1 the pixel kernel itself.  Both phases take the
// same decisions.
template <int TW, bool STATS, bool LDSD, int WALK>
static hipError_t launch_variant(const Dev& d, hipStream_t s, size_t shm, int phase) {
  auto kern = k_pixel<TW, STATS, LDSD, WALK>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kPixelThreads, shm) != hipSuccess || per_cu < 1)
    per_cu = 1;
  constexpr int TH = 64 / TW;
  const long long ntx = (d.W + TW - 1) / TW;
  const long long waves_needed = (ntx + d.strip - 1) / d.strip * ((d.H + TH - 1) / TH);
  long long blocks = (long long)device_cus() * per_cu;
  const long long max_blocks = (waves_needed + (kPixelThreads / 64) - 1) / (kPixelThreads / 64);
  if (blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  if (phase == 0 && WALK == kWalkCluster && d.Gmax > 0) {
    const int npos = (d.Gmax + kCluster - 1) / kCluster * kCluster;
    hipLaunchKernelGGL(k_clusters, dim3((unsigned)((npos + 255) / 256)), dim3(256), 0, s, d.misc, d.gorder, d.krank,
                       d.sgbb, d.sgcost, d.clk, d.clmb, d.clbb, d.clc, d.Gmax);
  }
  // the work order matters only when some items wait for a free wavefront
  const int* order = nullptr;
  auto launch_main = [&]() {
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kPixelThreads), shm, s, d.W, d.H, d.W32, d.Gmax, d.misc,
                       d.inside, d.sgen, d.sgcost, d.sgbb, d.edges, d.ext, d.chunks, d.E, d.NC, d.clk, d.clmb,
                       d.clbb, d.clc, d.dist, d.parent, d.strip, d.samples, d.qctr, d.obins, order, d.ocap, d.stats);
    return hipGetLastError();
  };
  if (SPM_TILE_ORDER && waves_needed > blocks * (kPixelThreads / 64) && order_fused(d)) {
    order = d.order;   // built in the generator sort's launch
  } else if (SPM_TILE_ORDER && waves_needed > blocks * (kPixelThreads / 64)) {
    order = d.order;
    if (phase == 1) return launch_main();
    const dim3 og((unsigned)((waves_needed + kOrderItems - 1) / kOrderItems));
    const size_t osh = (size_t)d.Gmax * (sizeof(int4) + sizeof(float));
    if (osh <= kOrderLdsMax)
      hipLaunchKernelGGL((k_tile_order<TW, true>), og, dim3(kOrderThreads), osh, s, d.W, d.H, d.strip, d.Gmax, d.misc,
                         d.sgcost, d.sgbb, d.obins, d.order, d.ocap);
    else
      hipLaunchKernelGGL((k_tile_order<TW, false>), og, dim3(kOrderThreads), 0, s, d.W, d.H, d.strip, d.Gmax, d.misc,
                         d.sgcost, d.sgbb, d.obins, d.order, d.ocap);
    return hipGetLastError();
  }
  return phase == 1 ? launch_main() : hipGetLastError();
}

template <int TW, int WALK>
static hipError_t launch_tw_walk(const Dev& d, hipStream_t s, int phase) {
  const size_t shm = pixel_lds_bytes(d.Gmax, d.E, d.NC);
  const bool lds = shm <= kPixelLdsMax;
  if (!lds && (WALK == kWalkCluster || WALK == kWalkRefill)) {
    // the cluster and refilled walks keep the packed edges in LDS (at most 8192 edges: 66 KB), the
    // refilled walk also the boxes and costs when they fit
    size_t pk = packed_edge_lds_bytes(d.E, d.NC);
    if (WALK == kWalkRefill && refill_stages_tables(d.Gmax, d.E, d.NC)) pk += (size_t)d.Gmax * 20;
    if (phase == 1 && pk > kPixelLdsMax) {
      auto k0 = d.stats ? k_pixel<TW, true, false, WALK> : k_pixel<TW, false, false, WALK>;
      const hipError_t e = hipFuncSetAttribute((const void*)k0, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pk);
      if (e != hipSuccess) return e;
    }
    return d.stats ? launch_variant<TW, true, false, WALK>(d, s, pk, phase)
                   : launch_variant<TW, false, false, WALK>(d, s, pk, phase);
  }
  if (d.stats)
    return lds ? launch_variant<TW, true, true, WALK>(d, s, shm, phase)
               : launch_variant<TW, true, false, WALK>(d, s, 0, phase);
  return lds ? launch_variant<TW, false, true, WALK>(d, s, shm, phase)
             : launch_variant<TW, false, false, WALK>(d, s, 0, phase);
}

template <int TW>
static hipError_t launch_tw(const Dev& d, hipStream_t s, int phase) {
  switch (d.walk > 0 ? d.walk - 1 : walk_mode(d.Gmax)) {
    case kWalkCached: return launch_tw_walk<TW, kWalkCached>(d, s, phase);
    case kWalkRefill: return launch_tw_walk<TW, kWalkRefill>(d, s, phase);
    case kWalkCluster: return launch_tw_walk<TW, kWalkCluster>(d, s, phase);
    default: return launch_tw_walk<TW, kWalkCost>(d, s, phase);
  }
}

hipError_t launch_pixel(const Dev& d, hipStream_t s, int phase) {
  if (d.tile_w == 16) return launch_tw<16>(d, s, phase);
  if (d.tile_w == 4) return launch_tw<4>(d, s, phase);
  return launch_tw<8>(d, s, phase);
}

// Batched pixel stage: one persistent launch for every tile of every scene.
// A workgroup takes a work item -- kSlice tiles of one scene -- from the
// launch's queue, stages the scene's generator table and edges in LDS when
// it differs from the scene already staged, and its wavefronts share the
// slice's tiles through an LDS counter.  Each scene keeps its own tile shape
// (the walk is compiled for all three shapes and chosen per scene).
template <bool LDSD, int WALK>
__global__ __launch_bounds__(kPixelThreads, SPM_PIXEL_MIN_WAVES) void k_pixel_batch(BatchSrc src, int* ctr) {
  extern __shared__ int4 smem[];
  __shared__ int item_scene, item_t0, item_t1, staged, next_tile;
  const int tid = threadIdx.x;
  if (tid == 0) staged = -1;
  u64 st[ST_COUNT];
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
    if (sc == -1) break;
    const Dev& d = src.scene(sc);
    const int G = d.misc[MISC_REACHED];
    TabFull tab{d.sgen, d.sgcost, d.sgbb};
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
      tab = TabFull{s_gen, s_cost, s_bb};
      geo.edges = s_edges;
      geo.chunks = s_chunks;
    }
    // the slice's tiles in strips of d.strip consecutive tiles (seeded left to right)
    for (;;) {
      int t = 0;
      if (lane_id() == 0) t = atomicAdd(&next_tile, d.strip);
      t = __shfl(t, 0, 64);
      const int ta = item_t0 + t;
      if (ta >= item_t1) break;
      const int tb = min(ta + d.strip, item_t1);
      int prev = -1;
      for (int tile = ta; tile < tb; ++tile) {
        if (d.tile_w == 16)
          prev = tile_work<16, false, WALK>(tile, d.W, d.H, d.W32, G, d.inside, tab, geo, d.dist, d.parent, prev,
                                            d.samples, st);
        else if (d.tile_w == 4)
          prev = tile_work<4, false, WALK>(tile, d.W, d.H, d.W32, G, d.inside, tab, geo, d.dist, d.parent, prev,
                                           d.samples, st);
        else
          prev = tile_work<8, false, WALK>(tile, d.W, d.H, d.W32, G, d.inside, tab, geo, d.dist, d.parent, prev,
                                           d.samples, st);
      }
    }
    __syncthreads();
  }
}

__global__ void k_reset_counter(int* ctr) {
  if (threadIdx.x == 0) *ctr = 0;
}

template <int WALK>
static hipError_t launch_batch_walk(const BatchSrc& b, const Plan& p, int* ctr, hipStream_t s) {
  const size_t shm = p.pixel_lds;
  const bool lds = shm > 0 && shm <= kPixelLdsMax;
  auto kern = lds ? k_pixel_batch<true, WALK> : k_pixel_batch<false, WALK>;
  const size_t use = lds ? shm : 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kPixelThreads, use) != hipSuccess || per_cu < 1)
    per_cu = 1;
  // waves per SIMD asked for: a 512-thread workgroup holds two waves of each of the CU's four SIMDs
  if (p.pixel_waves > 0) per_cu = max(1, min(per_cu, p.pixel_waves / 2));
  long long blocks = (long long)device_cus() * per_cu;
  if (blocks > p.total[STG_SLICE]) blocks = p.total[STG_SLICE];
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kPixelThreads), use, s, b, ctr);
  return hipGetLastError();
}

// ctr: the queue counter of the launch (reset by a kernel, so the launch can sit in a graph)
hipError_t launch_pixel_batch(const BatchSrc& b, const Plan& p, int* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, ctr);
  const int w = p.walk > 0 ? p.walk - 1 : walk_mode(p.maxGmax);
  switch (w) {
    case kWalkCached: return launch_batch_walk<kWalkCached>(b, p, ctr, s);
    case kWalkRefill: return launch_batch_walk<kWalkRefill>(b, p, ctr, s);
    default: return launch_batch_walk<kWalkCost>(b, p, ctr, s);
  }
}

}  // namespace spm
