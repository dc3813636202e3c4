// k_graph.hip -- generator costs for libspm.
//
// The paper expands generators one at a time in cost order (Procedure 1),
// shades their cones and relaxes every visible DataArray entry (Procedure 4),
// which is Dijkstra's algorithm on the visibility graph of the generators.
// Here the same costs come from three kernels (templates over the scene
// source, like the ingest kernels):
//   k_genvis   every (corner, generator) arc of the visibility graph, as a
//              bit matrix (exact predicates; by pairs with lanes over edges,
//              or lanes over generators), and the columns of segment sources;
//   k_relax_chaos, k_relax_wide, k_relax, k_relax_queue
//              Bellman-Ford over that matrix in double precision, iterated to
//              its fixed point (which Dijkstra also reaches): the first rounds
//              chip-wide, the rest in one workgroup (rounds, or a work queue for
//              deep graphs; batches of small graphs on the queue alone);
//   k_gsort_parents
//              the reached generators ordered by (float cost, id), the order
//              the pixel stage walks them in; and each corner's parent: the
//              smallest id among the visible predecessors that attain its
//              cost.
#include <math.h>

#include <type_traits>

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

// Generator visibility, one launch, two kinds of wavefronts (the matrix was
// cleared by k_gen_table; every wavefront ORs its bits in):
//
// Point columns: one wavefront per (row corner v, gv_sub consecutive
// generators u): bit u of row v is set iff the arc u -> v exists (u a point
// source or another corner that sees v).  Rows and bits are indexed by
// spatial position (gorder), so the generators of a wavefront are
// neighbours in space and the box that culls the edges stays small.
//
// Segment columns: one wavefront per (segment source s, kSegCols corner positions).
// A corner v sees s when it sees the closest point q*(v) of s (Section 4).
// Lanes whose closest point is an endpoint share that endpoint (the
// wave-level point test); for the others [v, q*] is perpendicular to s (the
// wave-level perpendicular test).
//
// LDSE: the edges and chunk boxes are staged in LDS first.  Workgroups never
// straddle scenes for the first kind (each scene's wavefronts are padded to
// whole workgroups).
// The relaxation's starting state, by spatial position (entry wid * 64 + lane
// of it; the point-column wavefronts cover all of it): sources at cost 0 and
// marked changed, everything else at +inf; generator coordinates; the
// barrier-free rounds' progress mark at 0.
__device__ __forceinline__ void relax_init(const Dev& d, int wid, int G, int nsrc) {
  const int RW = d.RW;
  const int t = wid * 64 + lane_id();
  if (t < kChaosSlots) d.cmark[t * kQueueStride] = 0;
  if (t < G) {
    const GenRec gt = d.gens[d.gorder[t]];
    d.costpos[t] = (u64)__double_as_longlong(t < nsrc ? 0.0 : INFINITY);
    d.gxy[t] = make_int4(gt.x, gt.y, gt.x2, gt.y2);
  }
  if (t < 3 * RW) {
    u64 m = 0;
    if (t < RW) {
      const int lo = t * 64, hi = min(nsrc, lo + 64);
      if (hi > lo) m = (hi - lo == 64) ? ~0ull : ((1ull << (hi - lo)) - 1ull);
    }
    d.rmask[t] = m;
  }
}

template <class S>
__device__ __forceinline__ void genvis_points(const Dev& d, const Geo& geo, int wid) {
  const int RW = d.RW;
  const int sb = d.gv_sub, per_row = 64 / sb;
  const int r = wid / (RW * per_row), rest = wid - r * (RW * per_row);
  const int blk = rest / per_row, sub = rest - blk * per_row;
  const int G = uni(d.misc[MISC_G]);
  const int nsrc = d.np + d.ns;
  const int lane = lane_id();
  relax_init(d, wid, G, nsrc);
  if (r >= G || r < nsrc) return;  // only corner rows are read
  const int v = uni(d.gorder[r]);
  const int gx = uni(d.gens[v].x), gy = uni(d.gens[v].y);
  const int gux = uni(d.gens[v].ux), guy = uni(d.gens[v].uy), gnx = uni(d.gens[v].nx), gny = uni(d.gens[v].ny);
  const int bit = sub * sb + lane;
  const int upos = blk * 64 + bit;
  const int u = (lane < sb && upos < G) ? d.gorder[upos] : -1;
  const bool valid = u >= 0 && u != v;
  GenRec gu = {};
  if (valid) gu = d.gens[u];
  // segment sources are the columns of the other kind of wavefront
  const bool fast = valid && gu.kind != SPM_GEN_SEGMENT;
  bool ok = false;
  const u64 fm = ballot(fast);
  if (fm) {
    const int bx0 = wave_min_i(fast ? gu.x : (1 << 30)), bx1 = wave_max_i(fast ? gu.x : -(1 << 30));
    const int by0 = wave_min_i(fast ? gu.y : (1 << 30)), by1 = wave_max_i(fast ? gu.y : -(1 << 30));
    u64 dummy[8];
    const bool pv = gu.kind == SPM_GEN_VERTEX;
    const u64 bl = wave_blocked_uniform<false>(geo, gu.x, gu.y, fm, gx, gy, true, gux, guy, gnx, gny, pv, gu.ux,
                                               gu.uy, gu.nx, gu.ny, bx0, by0, bx1, by1, nullptr, dummy);
    ok = fast && !((bl >> lane) & 1ull);
  }
  const u64 bits = ballot(ok);
  if (lane == 0 && bits) atomicOr(&d.vis[(size_t)r * RW + blk], bits << (sub * sb));
}


// Closed-segment visibility of one pair, P (a point source or a corner) and
// the corner g, lanes over edges -- the exact rules of wave_blocked_uniform
// for a single P: the segment is blocked when it enters an obstacle through
// the interior of an edge front-facing to g (endpoints strictly on opposite
// sides of line P-g, P strictly on the obstacle side), or through a vertex
// strictly between P and g (the vertex rule), or leaves P or g into their own
// interior angle.  Only the chunks whose box meets the segment's box and
// straddles or touches its line can hold such an edge or vertex.
__device__ __forceinline__ bool pair_visible(const Geo& geo, int px, int py, bool pvert, int pux, int puy, int pnx,
                                             int pny, int gx, int gy, int gux, int guy, int gnx, int gny,
                                             int* found = nullptr) {
  const int lane = lane_id();
  if (into_interior(gux, guy, gx, gy, gnx, gny, px - gx, py - gy)) return false;
  if (pvert && into_interior(pux, puy, px, py, pnx, pny, gx - px, gy - py)) return false;
  // line through P and g: o(x) = A x + B y + C = cross(g - P, x - P)
  const int A = py - gy, B = gx - px;
  const int C = -(mul24(A, px) + mul24(B, py));
  const int len2 = mad24(B, B, mul24(A, A));
  const int sx0 = min(px, gx), sx1 = max(px, gx), sy0 = min(py, gy), sy1 = max(py, gy);
  for (int cb = 0; cb < geo.NC; cb += kWave) {
    const int ci = cb + lane;
    bool hit = false;
    if (ci < geo.NC) {
      const int4 bb = geo.chunks[ci];
      if (bb.x <= sx1 && bb.z >= sx0 && bb.y <= sy1 && bb.w >= sy0) {
        const int o00 = mad24(A, bb.x, mad24(B, bb.y, C)), o10 = mad24(A, bb.z, mad24(B, bb.y, C));
        const int o01 = mad24(A, bb.x, mad24(B, bb.w, C)), o11 = mad24(A, bb.z, mad24(B, bb.w, C));
        hit = !((o00 > 0 && o10 > 0 && o01 > 0 && o11 > 0) || (o00 < 0 && o10 < 0 && o01 < 0 && o11 < 0));
      }
    }
    u64 cm = ballot(hit);
    while (cm) {
      const int e = (cb + first_bit(cm)) * kChunk + lane;
      cm &= cm - 1;
      bool blk = false;
      if (e < geo.E) {
        const EdgeRec r = geo.edges[e];
        const int ow = mad24(A, r.wx, mad24(B, r.wy, C));
        const int ov = mad24(A, r.vx, mad24(B, r.vy, C));
        const int Eg = mad24(r.a, gx, mad24(r.b, gy, r.c));
        // sign of ow * ov: converting to float keeps every sign and every zero exact
        blk = Eg < 0 && (float)ow * (float)ov < 0.0f && mad24(r.a, px, mul24(r.b, py)) > r.nc;
        if (ow == 0) {
          const int dw = mad24(r.wx - px, B, mul24(r.wy - py, -A));
          if (dw > 0 && dw < len2) {
            const EdgeExt x = geo.ext[e];
            blk = blk || into_interior(x.ux, x.uy, r.wx, r.wy, r.vx, r.vy, px - r.wx, py - r.wy) ||
                  into_interior(x.ux, x.uy, r.wx, r.wy, r.vx, r.vy, gx - r.wx, gy - r.wy);
          }
        }
      }
      const u64 bm = ballot(blk);
      if (bm) {
        if (found) *found = readlane(e, first_bit(bm));
        return false;
      }
    }
  }
  return true;
}

// Occluder cache of one row of the pair visibility, one edge per lane: edges
// that the row's corner g lies strictly outside of (only those can block a
// segment from g), first the nearby ones, then every edge a full test found
// blocking.  The pair (P, g) is blocked by a cached edge when P lies strictly
// on its obstacle side and the line P-g separates its endpoints strictly (a
// proper crossing into the obstacle: the rule of pair_visible), i.e. when P
// lies in the edge's shadow from g; a hit is exact, a miss falls back to
// pair_visible.
struct PairCache {
  unsigned w, v;   // x | y << 16 of the edge's endpoints; w == v: empty
  int slot;
  __device__ __forceinline__ void fill_near(const Geo& geo, int gx, int gy) {
    const int lane = lane_id();
    w = v = 0u;
    slot = 0;
    for (int cb = 0; cb < geo.NC && slot < 64; cb += kWave) {
      const int ci = cb + lane;
      int gap = 1 << 30;
      if (ci < geo.NC) {
        const int4 bb = geo.chunks[ci];
        gap = max(max(max(bb.x - gx, gx - bb.z), max(bb.y - gy, gy - bb.w)), 0);
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
            r = geo.edges[e];
            ok = mad24(r.a, gx, mad24(r.b, gy, r.c)) < 0;
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
  __device__ __forceinline__ void insert(const EdgeRec& r) {   // r wave-uniform, g strictly outside its line
    if (lane_id() == (slot & 63)) {
      w = (unsigned)r.wx | ((unsigned)r.wy << 16);
      v = (unsigned)r.vx | ((unsigned)r.vy << 16);
    }
    ++slot;
  }
  // The shadow of this lane's edge w -> v cast by g (strictly outside its
  // line, E(g) < 0): the points P for which [P, g] properly crosses the edge
  // into the obstacle, E(P) > 0 and the line P-g separating w and v strictly.
  // Seen from g the edge runs clockwise from w to v (cross(w - g, v - g) =
  // E(g) < 0), so with E(P) > 0
  // that separation is P strictly inside the wedge of rays g->w, g->v:
  // cross(w - g, P - g) < 0 < cross(v - g, P - g).  Three open half-planes
  // h_i(P) = A_i Px + B_i Py + C_i < 0 (|A|, |B| <= 2^14, |C| < 2^30: exact in
  // int32); an empty slot gets h_0 = 1, never.
  // Every slot's coefficients go to this wavefront's LDS block, (A_i | B_i
  // << 16, C_i) in 2 int4 a slot, where a test of slot e reads them at one
  // address for all lanes.
  int4* sh;
  __device__ __forceinline__ void set_shadow(int gx, int gy) {
    int sa[3], sb[3], sc[3];
    const int wx = (int)(w & 0xffffu), wy = (int)(w >> 16), vx = (int)(v & 0xffffu), vy = (int)(v >> 16);
    const int a = wy - vy, b = vx - wx, c = -(a * wx + b * wy);
    const bool empty = w == v;
    sa[0] = empty ? 0 : -a;
    sb[0] = empty ? 0 : -b;
    sc[0] = empty ? 1 : -c;
    sa[1] = -(wy - gy);
    sb[1] = wx - gx;
    sc[1] = mul24(wy - gy, gx) - mul24(wx - gx, gy);
    sa[2] = vy - gy;
    sb[2] = -(vx - gx);
    sc[2] = mul24(vx - gx, gy) - mul24(vy - gy, gx);
    const int l = lane_id();
    sh[2 * l] = make_int4(pack16(sa[0], sb[0]), sc[0], pack16(sa[1], sb[1]), sc[1]);
    sh[2 * l + 1] = make_int4(pack16(sa[2], sb[2]), sc[2], 0, 0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // lanes hold the points P (pp = px | py << 16): is P in the shadow of the slot-e edge? (e wave-uniform)
  __device__ __forceinline__ bool in_shadow(int e, int pp) const {
    const int4 p0 = sh[2 * e], p1 = sh[2 * e + 1];   // one address for every lane
    return max(max(dot2(p0.x, pp, p0.y), dot2(p0.z, pp, p0.w)), dot2(p1.x, pp, p1.y)) < 0;
  }
};

// Point columns by pairs (few edges): one wavefront per row of a
// kGvPairRows x kGvPairRows block of the lower triangle of the matrix (blocks
// numbered row by row), testing its pairs (row corner v, column u < v) one at
// a time; spread: the same pairs dealt round-robin instead (smaller graphs).  Corner-corner visibility is symmetric, so a visible pair sets both
// v's bit u and u's bit v; point-source columns set v's bit only (source rows
// are never read) and segment columns are left to the segment wavefronts.
template <class S>
__device__ __forceinline__ void genvis_pairs(const Dev& d, const Geo& geo, int wid, bool spread) {
  const int RW = d.RW;
  const int G = uni(d.misc[MISC_G]);
  const int nsrc = d.np + d.ns;
  const int lane = lane_id();
  relax_init(d, wid, G, nsrc);
  if (spread) {
  // The pairs of the block enumeration (block b, row i, column c), dealt
  // round-robin: lane j < kGvPairRows holds pair q = wid + j * NW, so every
  // wavefront mixes pairs from all over the triangle (pairs far apart cross
  // more chunks, and whole blocks off the diagonal are far apart).
  const int Bn = (d.Gmax + kGvPairRows - 1) / kGvPairRows;
  const int NW = kGvPairRows * (Bn * (Bn + 1) / 2);
  if (wid >= NW) return;
  int r = G, u = G;
  if (lane < kGvPairRows) {
    const int q = wid + lane * NW;
    const int rowid = q / kGvPairRows, c = q - rowid * kGvPairRows;
    const int b = rowid / kGvPairRows, i = rowid - b * kGvPairRows;
    int R = (int)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
    while (R > 0 && R * (R + 1) / 2 > b) --R;
    while ((R + 1) * (R + 2) / 2 <= b) ++R;
    r = R * kGvPairRows + i;
    u = (b - R * (R + 1) / 2) * kGvPairRows + c;
  }
  const bool ok = r < G && r >= nsrc && u < r;
  GenRec gr = {}, gu = {};
  if (ok) {
    gr = d.gens[d.gorder[r]];
    gu = d.gens[d.gorder[u]];
  }
  u64 todo = ballot(ok && gu.kind != SPM_GEN_SEGMENT);
  bool seen = false;
  while (todo) {
    const int j = (int)__builtin_ctzll(todo);
    todo &= todo - 1;
    const bool pv = readlane(gu.kind, j) == SPM_GEN_VERTEX;
    const bool vj = pair_visible(geo, readlane(gu.x, j), readlane(gu.y, j), pv, readlane(gu.ux, j), readlane(gu.uy, j),
                                 readlane(gu.nx, j), readlane(gu.ny, j), readlane(gr.x, j), readlane(gr.y, j),
                                 readlane(gr.ux, j), readlane(gr.uy, j), readlane(gr.nx, j), readlane(gr.ny, j));
    if (lane == j) seen = vj;
  }
  if (seen) {
    atomicOr(&d.vis[(size_t)r * RW + (u >> 6)], 1ull << (u & 63));
    if (u >= nsrc) atomicOr(&d.vis[(size_t)u * RW + (r >> 6)], 1ull << (r & 63));
  }
  return;
  }
  const int b = wid / kGvPairRows, i = wid - b * kGvPairRows;
  // block row R of block b: R (R + 1) / 2 <= b < (R + 1) (R + 2) / 2
  int R = (int)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
  while (R > 0 && R * (R + 1) / 2 > b) --R;
  while ((R + 1) * (R + 2) / 2 <= b) ++R;
  const int Cb = b - R * (R + 1) / 2;
  const int r = R * kGvPairRows + i, u0 = Cb * kGvPairRows;
  if (r >= G || r < nsrc || u0 >= r) return;
  const int v = uni(d.gorder[r]);
  const int gx = uni(d.gens[v].x), gy = uni(d.gens[v].y);
  const int gux = uni(d.gens[v].ux), guy = uni(d.gens[v].uy), gnx = uni(d.gens[v].nx), gny = uni(d.gens[v].ny);
  // lane j < kGvPairRows holds column u0 + j
  const int nu = min(kGvPairRows, r - u0);
  GenRec gu = {};
  if (lane < nu) gu = d.gens[d.gorder[u0 + lane]];
  unsigned bits = 0;
  for (int j = 0; j < nu; ++j) {
    if (readlane(gu.kind, j) == SPM_GEN_SEGMENT) continue;
    const bool pv = readlane(gu.kind, j) == SPM_GEN_VERTEX;
    if (pair_visible(geo, readlane(gu.x, j), readlane(gu.y, j), pv, readlane(gu.ux, j), readlane(gu.uy, j),
                     readlane(gu.nx, j), readlane(gu.ny, j), gx, gy, gux, guy, gnx, gny))
      bits |= 1u << j;
  }
  if (!bits) return;
  if (lane == 0) atomicOr(&d.vis[(size_t)r * RW + (u0 >> 6)], (u64)bits << (u0 & 63));
  const int u = u0 + lane;
  if (lane < nu && ((bits >> lane) & 1u) && u >= nsrc) atomicOr(&d.vis[(size_t)u * RW + (r >> 6)], 1ull << (r & 63));
}

// Point columns by row segments (many generators): wavefront wid takes the
// kGvSeg pairs (row corner g, columns u in [s kGvSeg, min((s + 1) kGvSeg, r)))
// of row r, 64 columns at a time, lanes over the columns: the corner rules,
// then the shadows that the row's cached occluders cast from g, then
// pair_visible for each column left (its blocking edge joins the cache and is
// tried at once on the columns still to do).  On the maze almost every pair is
// blocked by a wall next to g, so the first few cached edges decide nearly all
// of them.  Bits as in genvis_pairs.
template <class S>
__device__ __forceinline__ void genvis_rows(const Dev& d, const Geo& geo, int wid) {
  const int RW = d.RW;
  const int G = uni(d.misc[MISC_G]);
  const int nsrc = d.np + d.ns;
  const int lane = lane_id();
  relax_init(d, wid, G, nsrc);
  const int seg = d.gv_seg;
  if ((long long)wid >= rowseg_prefix(d.Gmax, seg)) return;
  int lo = 0, hi = d.Gmax;   // the row: the largest r with rowseg_prefix(r, seg) <= wid
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rowseg_prefix(mid, seg) <= wid) lo = mid;
    else hi = mid;
  }
  const int r = lo, s = wid - (int)rowseg_prefix(r, seg);
  if (r >= G || r < nsrc) return;   // only corner rows are read
  const int gpos = uni(d.gorder[r]);
  const int gx = uni(d.gens[gpos].x), gy = uni(d.gens[gpos].y);
  const int gux = uni(d.gens[gpos].ux), guy = uni(d.gens[gpos].uy), gnx = uni(d.gens[gpos].nx),
            gny = uni(d.gens[gpos].ny);
  const int u0 = s * seg, u1 = min(u0 + seg, r);
  PairCache pc;
  __shared__ int4 s_shadow[4][64 * 2];   // 256-thread workgroups: four wavefronts
  pc.sh = s_shadow[threadIdx.x >> 6];
  pc.fill_near(geo, gx, gy);
  pc.set_shadow(gx, gy);
  for (int ub = u0; ub < u1; ub += kWave) {
    const int u = ub + lane;
    const bool valid = u < u1;
    GenRec gu = {};
    if (valid) gu = d.gens[d.gorder[u]];
    // lanes over the columns: the corner rules, then the shadows of the cached edges (nearest first,
    // stopping once every column is decided), then the full test for each column left
    const bool pv = gu.kind == SPM_GEN_VERTEX;
    bool out = !valid || gu.kind == SPM_GEN_SEGMENT;
    if (!out) {
      out = into_interior(gux, guy, gx, gy, gnx, gny, gu.x - gx, gu.y - gy) ||
            (pv && into_interior(gu.ux, gu.uy, gu.x, gu.y, gu.nx, gu.ny, gx - gu.x, gy - gu.y));
    }
    const int ncache = min(pc.slot, kWave);
    const int gp = pack16(gu.x, gu.y);
    for (int e = 0; e < ncache && ballot(!out); e += 4) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (e + t < ncache) out = out || pc.in_shadow(e + t, gp);
    }
    u64 todo = ballot(!out);
    bool seen = false;
    while (todo) {
      const int j = first_bit(todo);
      todo &= todo - 1;
      const int px = readlane(gu.x, j), py = readlane(gu.y, j);
      const int pux = readlane(gu.ux, j), puy = readlane(gu.uy, j), pnx = readlane(gu.nx, j),
                pny = readlane(gu.ny, j);
      int found = -1;
      const bool vj = pair_visible(geo, px, py, readlane((int)pv, j) != 0, pux, puy, pnx, pny, gx, gy, gux, guy, gnx,
                                   gny, &found);
      if (lane == j) seen = vj;
      // a blocker found by the vertex rule may face away from g: the shadow test holds only for edges g is outside
      // of.  A new one joins the cache and is tried at once on the columns still to do.
      if (found >= 0) {
        const EdgeRec fr = geo.edges[found];
        if (mad24(fr.a, gx, mad24(fr.b, gy, fr.c)) < 0) {
          const int at = pc.slot & 63;
          pc.insert(fr);
          pc.set_shadow(gx, gy);
          if (todo) todo &= ~ballot(pc.in_shadow(at, gp));
        }
      }
    }
    const u64 bits = ballot(seen);
    if (bits && lane == 0) atomicOr(&d.vis[(size_t)r * RW + (ub >> 6)], bits);
    if (seen && u >= nsrc) atomicOr(&d.vis[(size_t)u * RW + (r >> 6)], 1ull << (r & 63));
  }
}

__device__ __forceinline__ void genvis_segments(const Dev& d, const Geo& geo, int item) {
  const int nsrc = d.np + d.ns;
  const int nblk = (d.Gmax - nsrc + kSegCols - 1) / kSegCols;
  const int s = item / nblk, blk = item - s * nblk;
  const int G = uni(d.misc[MISC_G]);
  const int lane = lane_id();
  const int r = nsrc + blk * kSegCols + lane;   // this lane's corner position (lanes below kSegCols)
  const int spos = d.np + s;                    // the segment's position (= its id)
  const bool valid = lane < kSegCols && r < G;
  GenRec cv = {};
  if (valid) cv = d.gens[d.gorder[r]];
  const GenRec sg = d.gens[spos];
  const int ax = uni(sg.x), ay = uni(sg.y), bx = uni(sg.x2), by = uni(sg.y2);
  int clamp = 0;
  const RPt q = seg_closest(ax, ay, bx, by, cv.x, cv.y, &clamp);
  (void)q;
  if (!ballot(valid)) return;
  u64 dummy[8];
  u64 bl = 0;
  for (int grp = 0; grp < 3; ++grp) {
    const bool inm = valid && clamp == grp;
    const u64 m = ballot(inm);
    if (!m) continue;
    const int x0 = wave_min_i(inm ? cv.x : (1 << 30)), x1 = wave_max_i(inm ? cv.x : -(1 << 30));
    const int y0 = wave_min_i(inm ? cv.y : (1 << 30)), y1 = wave_max_i(inm ? cv.y : -(1 << 30));
    if (grp < 2)
      bl |= wave_blocked_uniform<false>(geo, cv.x, cv.y, m, grp ? bx : ax, grp ? by : ay, false, 0, 0, 0, 0, true,
                                        cv.ux, cv.uy, cv.nx, cv.ny, x0, y0, x1, y1, nullptr, dummy) & m;
    else
      bl |= wave_blocked_perp<false>(geo, cv.x, cv.y, m, ax, ay, bx, by, true, cv.ux, cv.uy, cv.nx, cv.ny, x0, y0,
                                     x1, y1, nullptr, dummy) & m;
  }
  if (valid && !((bl >> lane) & 1ull)) atomicOr(&d.vis[(size_t)r * d.RW + (spos >> 6)], 1ull << (spos & 63));
}

template <class S, bool LDSE>
__global__ __launch_bounds__(256) void k_genvis(S src, int nblk_points) {
  const bool pts = (int)blockIdx.x < nblk_points;
  const int wid = (pts ? blockIdx.x : blockIdx.x - nblk_points) * 4 + (threadIdx.x >> 6);
  int sc, item;
  // a whole workgroup of point columns belongs to one scene (padded); segment waves locate alone
  if (!src.locate(pts ? STG_GVBLK : STG_SEGVIS, pts ? (int)blockIdx.x : wid, sc, item)) return;
  const Dev& d = src.scene(sc);
  extern __shared__ int4 smem[];
  Geo geo{d.edges, d.ext, d.chunks, d.E, d.NC};
  if (LDSE && pts) {
    EdgeRec* s_edges = (EdgeRec*)smem;
    int4* s_chunks = (int4*)(s_edges + d.E);
    const int4* se = (const int4*)d.edges;
    for (int k = threadIdx.x; k < d.E * 2; k += blockDim.x) ((int4*)s_edges)[k] = se[k];
    for (int k = threadIdx.x; k < d.NC; k += blockDim.x) s_chunks[k] = d.chunks[k];
    __syncthreads();
    geo.edges = s_edges;
    geo.chunks = s_chunks;
  }
  if (pts) {
    if (d.gv_sub == -2) genvis_rows<S>(d, geo, item * 4 + (threadIdx.x >> 6));
    else if (d.gv_sub <= 0) genvis_pairs<S>(d, geo, item * 4 + (threadIdx.x >> 6), d.gv_sub < 0);
    else genvis_points<S>(d, geo, item * 4 + (threadIdx.x >> 6));
  } else {
    genvis_segments(d, geo, item);
  }
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
constexpr int kRelaxQueueSlack = 64;   // work-queue ring entries beyond one per generator
constexpr int kRelaxQueueSpin = 1 << 22;   // spin limit of the work queue's waits (about a second)
constexpr long long kRelaxListMaxWords = 16384;   // matrix words (corner rows) up to which the queue builds lists

// A lower bound, in double, of the arc weight from u (doubled coordinates
// x, y, x2, y2) to the corner (vx, vy): the hardware float square root with a
// relative margin of 1e-6 (far above its error) when u is a point or corner;
// 0 for a segment, whose weight is only ever computed exactly.  Lets the
// relaxation skip the exact double-precision weight of arcs that cannot win.
__device__ __forceinline__ double arc_lower(int4 u, int vx, int vy) {
  if (u.x != u.z || u.y != u.w) return 0.0;
  const float dx = (float)(vx - u.x), dy = (float)(vy - u.y);
  return (double)(0.5f * __builtin_amdgcn_sqrtf(dx * dx + dy * dy)) * (1.0 - 1e-6);
}

// One workgroup per scene: the remaining Bellman-Ford rounds, from the costs
// and change mask the wide rounds left, iterated to the fixed point (the
// costs Dijkstra reaches).  Each round relaxes the arcs leaving the
// generators whose cost changed in the previous round:
//   pull  (large frontier): one item per (corner row v, 64-bit word k): the
//         best candidate over the changed generators of that word, merged
//         into cost(v) by an atomic minimum;
//   push  (small frontier, corners only): one item per (frontier corner u,
//         word k of row u) -- corner-to-corner visibility is symmetric -- and
//         every corner v of it takes cost(u) + |u - v| by an atomic minimum.
// A float lower bound of each weight skips most exact ones.
// Atomic minima act on the IEEE bits of non-negative doubles, which order like
// the values.  Positive arc weights make the double-precision fixed point
// unique, so the result does not depend on thread timing or on the pull/push
// schedule.  LDS: costs, generator coordinates and change masks live in LDS
// when they fit, else in global memory; VLDS: the arc matrix too.  Everything is indexed by
// spatial position; outputs go back to canonical ids.
// One Bellman-Ford round over the whole chip (the first rounds, whose
// frontiers are the largest): one thread per (corner row v, byte of word k),
// pulling the changed generators there into cost(v) by an atomic minimum on
// the global cost array.  Round r reads change mask r % 3, marks mask
// (r + 1) % 3 and clears mask (r + 2) % 3 for the round after.
template <class S>
__global__ __launch_bounds__(256) void k_relax_wide(S src, int round) {
  int sc, it;
  if (!src.locate(STG_RELAXW, blockIdx.x * blockDim.x + threadIdx.x, sc, it)) return;
  const Dev& d = src.scene(sc);
  const int RW = d.RW, nsrc = d.np + d.ns;
  u64* Mc = d.rmask + (round % 3) * RW;
  u64* Mn = d.rmask + ((round + 1) % 3) * RW;
  if (it < RW) d.rmask[((round + 2) % 3) * RW + it] = 0;
  const int vk = it >> 3, sh = (it & 7) * 8;
  const int v = nsrc + vk / RW, k = vk - (vk / RW) * RW;
  if (v >= d.misc[MISC_G]) return;
  const u64 m = (Mc[k] >> sh) & (d.vis[(size_t)v * RW + k] >> sh) & 0xffull;
  if (!m) return;
  u64* cost = d.costpos;
  // the (up to eight) candidates' costs and coordinates, all requested before any is used
  const int u0 = k * 64 + sh;
  double cu[8];
  int4 pu[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    cu[j] = INFINITY;
    if ((m >> j) & 1ull) {
      cu[j] = __longlong_as_double((long long)cost[u0 + j]);
      pu[j] = d.gxy[u0 + j];
    }
  }
  const int4 pv = d.gxy[v];
  const double old = __longlong_as_double((long long)cost[v]);
  double best = old;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (!(cu[j] < best)) continue;
    if (!(cu[j] + arc_lower(pu[j], pv.x, pv.y) < best)) continue;
    const double cand = cu[j] + arc_len4(pu[j], pv.x, pv.y);
    if (cand < best) best = cand;
  }
  if (best < old) {
    const u64 ob = atomicMin(&cost[v], (u64)__double_as_longlong(best));
    if (__longlong_as_double((long long)ob) > best) atomicOr(&Mn[v >> 6], 1ull << (v & 63));
  }
}

// The first rounds without a barrier between them: one thread per (corner row
// v, byte of word k) relaxes its (up to eight) arcs up to iters times, reading
// the current costs each time (coherent loads) and merging by an atomic
// minimum; every vertex it lowers is marked in change mask 1.  Costs only fall
// and every arc is relaxed at least once from its source's value at the time,
// so afterwards an arc (u, v) can still lower v only if u was lowered during
// the launch, i.e. u is marked: a chip-wide round from mask 1 (round 1 of
// k_relax_wide) restores the exact change mask the one-workgroup kernel starts
// from.  That holds whenever a thread stops, so stopping is a matter of speed
// alone.  ADAPT (large graphs, whose shortest paths take many arcs): a
// wavefront that lowers a cost in its pass t raises its workgroup's progress
// mark (one of kChaosSlots, spread over cache lines) to t + 1, and every
// wavefront stops once the largest mark shows kChaosQuiet passes in a row
// without a lowering; otherwise all iters passes run, with no mark traffic.
// The arc weights are computed once.
template <class S, bool ADAPT>
__global__ __launch_bounds__(256) void k_relax_chaos(S src, int iters) {
  int sc, it;
  if (!src.locate(STG_RELAXW, blockIdx.x * blockDim.x + threadIdx.x, sc, it)) return;
  const Dev& d = src.scene(sc);
  const int RW = d.RW, nsrc = d.np + d.ns;
  const int vk = it >> 3, sh = (it & 7) * 8;
  const int v = nsrc + vk / RW, k = vk - (vk / RW) * RW;
  if (v >= d.misc[MISC_G]) return;
  const u64 m = (d.vis[(size_t)v * RW + k] >> sh) & 0xffull;
  if (!m) return;
  u64* cost = d.costpos;
  const int u0 = k * 64 + sh;
  const int4 pv = d.gxy[v];
  double w[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) w[j] = ((m >> j) & 1ull) ? arc_len4(d.gxy[u0 + j], pv.x, pv.y) : INFINITY;
  for (int t = 0; t < iters; ++t) {
    int seen = 0;
    if (ADAPT) {
#pragma unroll
      for (int q = 0; q < kChaosSlots; ++q)
        seen = max(seen, __hip_atomic_load(d.cmark + q * kQueueStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    double cu[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      cu[j] = ((m >> j) & 1ull) ? __longlong_as_double((long long)__hip_atomic_load(
                                      &cost[u0 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                                : INFINITY;
    const double old =
        __longlong_as_double((long long)__hip_atomic_load(&cost[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    // no lowering seen in the last kChaosQuiet passes (the mark is wave-uniform once read by lane 0)
    if (ADAPT && t >= kChaosQuiet && __builtin_amdgcn_readfirstlane(seen) <= t - kChaosQuiet) break;
    double best = old;
#pragma unroll
    for (int j = 0; j < 8; ++j) best = fmin(best, cu[j] + w[j]);
    bool lowered = false;
    if (best < old) {
      const u64 ob = atomicMin(&cost[v], (u64)__double_as_longlong(best));
      if (__longlong_as_double((long long)ob) > best) {
        atomicOr(&d.rmask[RW + (v >> 6)], 1ull << (v & 63));
        lowered = true;
      }
    }
    if (ADAPT) {
      const u64 any = ballot(lowered);
      if (any && lane_id() == (int)__builtin_ctzll(any) && __builtin_amdgcn_readfirstlane(seen) <= t)
        atomicMax(d.cmark + (blockIdx.x % kChaosSlots) * kQueueStride, t + 1);
    }
  }
}

// Parents, once the costs are final: one wavefront per spatial position p,
// lanes over the 64 generators of each bit word of row p (four words per
// step, all loads requested together): the smallest canonical id among the
// visible predecessors attaining cost(p).  Sources are their own parents,
// unreached generators have none (-1).
template <class S>
__device__ __forceinline__ void parent_wave(const S& src, int wid) {
  int sc, p;
  if (!src.locate(STG_GEN, wid, sc, p)) return;
  const Dev& d = src.scene(sc);
  const int G = uni(d.misc[MISC_G]);
  if (p >= G) return;
  const int lane = lane_id();
  const int RW = d.RW, nsrc = d.np + d.ns;
  const int g = uni(d.gorder[p]);
  const double c = __longlong_as_double((long long)d.costpos[p]);
  int best = 0x7fffffff;
  if (p >= nsrc && c < INFINITY) {
    const int4 pv = d.gxy[p];
    const int RWg = min(RW, (G + 63) >> 6);   // words of columns below G
    for (int k0 = 0; k0 < RWg; k0 += 4) {
      double cu[4];
      int4 pu[4];
      int gu[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + q, u = 64 * k + lane;
        cu[q] = INFINITY;
        if (k < RW && u < G && ((d.vis[(size_t)p * RW + k] >> lane) & 1ull)) {
          cu[q] = __longlong_as_double((long long)d.costpos[u]);
          pu[q] = d.gxy[u];
          gu[q] = d.gorder[u];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!(cu[q] < c)) continue;
        if (cu[q] + arc_lower(pu[q], pv.x, pv.y) > c) continue;
        if (cu[q] + arc_len4(pu[q], pv.x, pv.y) == c) best = min(best, gu[q]);
      }
    }
    best = wave_min_i(best);
  }
  if (lane == 0) d.gen_parent[g] = p < nsrc ? g : ((c < INFINITY && best != 0x7fffffff) ? best : -1);
}

template <class S, bool LDS, bool VLDS>
__global__ __launch_bounds__(1024) void k_relax(S src, int Gcap, int RWcap, int m0idx, int rounds0) {
  int sc, one;
  if (!src.locate(STG_SCENE, blockIdx.x, sc, one)) return;
  const Dev& d = src.scene(sc);
  extern __shared__ u64 shm[];
  __shared__ int any, nfront, reached;
  __shared__ int front[kRelaxFront];
  const int RW = d.RW;
  const u64* vis = d.vis;
  u64* chg_a = shm;
  u64* chg_b = shm + RWcap;
  u64* cost = LDS ? (shm + 2 * RWcap) : d.costpos;   // indexed by spatial position
  const int4* gxy = d.gxy;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int G = d.misc[MISC_G];
  const int nsrc = d.np + d.ns;
  const int ncr = G - nsrc;   // corner rows
  // nothing changed in the last chip-wide round: the costs are final, skip the staging
  const u64* m0 = d.rmask + m0idx * RW;
  if (tid == 0) any = 0;
  __syncthreads();
  for (int k = tid; k < RW; k += nt)
    if (m0[k]) any = 1;
  __syncthreads();
  const bool idle = !any;
  if (LDS && !idle) {
    int4* s_gxy = (int4*)(shm + 2 * RWcap + Gcap);
    for (int g = tid; g < G; g += nt) { cost[g] = d.costpos[g]; s_gxy[g] = d.gxy[g]; }
    gxy = s_gxy;
  }
  if (VLDS && !idle) {
    // the arc matrix itself in LDS (G rows of RW words)
    u64* s_vis = shm + 2 * RWcap + 3 * (size_t)Gcap;
    for (int k = tid; k < G * RW; k += nt) s_vis[k] = d.vis[k];
    vis = s_vis;
  }
  // the change mask left by the wide rounds
  for (int k = tid; k < RW; k += nt) { chg_a[k] = m0[k]; chg_b[k] = 0; }
  if (tid == 0) { reached = 0; nfront = -1; }
  __syncthreads();
  u64* cur = chg_a;
  u64* nxt = chg_b;
  int rounds = 0;
  for (; !idle && rounds <= G; ++rounds) {
    if (tid == 0) any = 0;
    const int nf = nfront;  // frontier list size, or -1 when only the mask is valid
    __syncthreads();
    if (nf < 0) {
      // one item per (corner row v, word k)
      for (int it = tid; it < ncr * RW; it += nt) {
        const int v = nsrc + it / RW, k = it - (it / RW) * RW;
        const int sh = 0;
        const u64 c = cur[k];
        if (!c) continue;
        u64 m = vis[(size_t)v * RW + k] & c;
        if (!m) continue;
        const int4 pv = gxy[v];
        const double old = __longlong_as_double((long long)cost[v]);
        double best = old;
        while (m) {
          const int u = k * 64 + sh + __builtin_ctzll(m);
          m &= m - 1;
          const double cu = __longlong_as_double((long long)cost[u]);
          if (!(cu < best)) continue;
          const int4 pu = gxy[u];
          if (!(cu + arc_lower(pu, pv.x, pv.y) < best)) continue;
          const double cand = cu + arc_len4(pu, pv.x, pv.y);
          if (cand < best) best = cand;
        }
        if (best < old) {
          const u64 ob = atomicMin(&cost[v], (u64)__double_as_longlong(best));
          if (__longlong_as_double((long long)ob) > best) {
            atomicOr(&nxt[v >> 6], 1ull << (v & 63));
            any = 1;
          }
        }
      }
    } else {
      // one item per (frontier corner u, word k of row u)
      for (int it = tid; it < nf * RW; it += nt) {
        const int f = it / RW, k = it - f * RW;
        const int sh = 0;
        const int u = front[f];
        u64 m = vis[(size_t)u * RW + k];
        if (!m) continue;
        const double cu = __longlong_as_double((long long)cost[u]);
        const int4 pu = gxy[u];
        while (m) {
          const int v = k * 64 + sh + __builtin_ctzll(m);
          m &= m - 1;
          const double cv = __longlong_as_double((long long)cost[v]);
          if (!(cu < cv)) continue;
          const int4 pv = gxy[v];
          if (!(cu + arc_lower(pu, pv.x, pv.y) < cv)) continue;
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
  // outputs by canonical id; parents follow in k_gsort_parents
  int mine = 0;
  const u64* fin = (LDS && !idle) ? cost : d.costpos;
  for (int p = tid; p < G; p += nt) {
    const double c = __longlong_as_double((long long)fin[p]);
    const int v = d.gorder[p];
    if (LDS && !idle) d.costpos[p] = cost[p];
    d.gen_cost[v] = c;
    d.cost64[v] = c;
    if (c < INFINITY) ++mine;
  }
  atomicAdd(&reached, mine);
  __syncthreads();
  if (tid == 0) {
    d.misc[MISC_REACHED] = reached;
    d.misc[MISC_ROUNDS] = rounds0 + rounds;
  }
}

// Deep graphs (the maze: shortest paths of hundreds of arcs) need as many
// synchronous rounds as their deepest path has arcs, each a few microseconds
// of barriers and L2 round trips in k_relax.  This kernel relaxes them without
// rounds: label-correcting with a FIFO work queue (Bellman-Ford-Moore) in one
// workgroup, costs in LDS.  Each wavefront takes a corner u off the queue,
// reads row u of the matrix (corner-corner visibility is symmetric, so its
// bits are the corners u sees) and lowers each such corner v by an LDS atomic
// minimum; a v it lowers goes on the queue unless it is already there.  A
// corner is taken off (its flag cleared) before its cost is read, so a later
// lowering puts it back.  `pending` counts corners queued and not yet fully
// relaxed; the workgroup is done when it is zero (no corner can still change,
// and nothing is in flight).  Every relaxation uses the same double-precision
// weight and sum as the other kernels, and the minimum over the same candidate
// values is reached whatever the order (the costs only fall to the one fixed
// point), so the costs are the same bits as k_relax's.
// Two starts: after the chip-wide rounds (m0idx >= 0: the corners that round
// lowered are queued), or from the sources alone (m0idx < 0, batches of small
// graphs: every corner takes its best arc from a source and the reached ones
// are queued; one workgroup per scene).
// LDS: cost (u64) and corner coordinates (int2) per position, the ring of
// positions (Gcap + 64 entries, -1 = empty), the queued flags, the adjacency
// list offsets (Gcap + 1) and, in the rest of lds_bytes, the lists (u16).
size_t relax_queue_lds_bytes(int Gcap) {
  return (size_t)Gcap * 16 + (size_t)(Gcap + kRelaxQueueSlack) * 4 + (size_t)((Gcap + 31) / 32) * 4 + 64 +
         (size_t)(Gcap + 1) * 4;
}

template <class S>
__global__ __launch_bounds__(1024) void k_relax_queue(S src, int Gcap, int m0idx, int rounds0, int lds_bytes) {
  int sc, one;
  if (!src.locate(STG_SCENE, blockIdx.x, sc, one)) return;
  const Dev& d = src.scene(sc);
  extern __shared__ u64 shm[];
  __shared__ int head, tail, pending, reached, narcs;
  u64* cost = shm;
  int2* xy = (int2*)(shm + Gcap);
  const int cap = Gcap + kRelaxQueueSlack;
  int* ring = (int*)(xy + Gcap);
  unsigned* inq = (unsigned*)(ring + cap);
  int* off = (int*)(inq + (Gcap + 31) / 32);   // adjacency list offsets (Gcap + 1), then the lists (u16)
  unsigned short* adj = (unsigned short*)(off + Gcap + 1);
  const long long adj_cap = ((long long)lds_bytes - (long long)((char*)adj - (char*)shm)) / 2;
  const int tid = threadIdx.x, nt = blockDim.x, lane = lane_id();
  const int G = d.misc[MISC_G];
  const int RW = d.RW, nsrc = d.np + d.ns;
  const int RWg = min(RW, (G + 63) >> 6);
  const u64* m0 = d.rmask + (m0idx >= 0 ? m0idx : 0) * RW;
  for (int g = tid; g < G; g += nt) {
    cost[g] = d.costpos[g];
    const int4 r = d.gxy[g];
    xy[g] = make_int2(r.x, r.y);
  }
  for (int k = tid; k < cap; k += nt) ring[k] = -1;
  for (int k = tid; k < (G + 31) / 32; k += nt) inq[k] = 0u;
  for (int g = tid; g <= G; g += nt) off[g] = 0;
  if (tid == 0) { head = 0; tail = 0; pending = 0; reached = 0; narcs = 0; }
  __syncthreads();
  // Corner-corner arcs as adjacency lists in LDS for small matrices whose lists fit (16-bit positions): one
  // pass counts the corners of each row, a scan gives the offsets, a second pass writes them.  Then relaxing
  // a corner reads no global memory.  Otherwise the rows are read from the matrix (for the maze's 1 MB
  // matrix the two passes by one workgroup cost more than they save: 0.82 -> 0.92 ms).
  const int ncr = G - nsrc;
  const long long nitems = (long long)ncr * RW;
  auto arc_word = [&](long long it, int& u, int& k) -> u64 {
    u = nsrc + (int)(it / RW);
    k = (int)(it - (long long)(u - nsrc) * RW);
    u64 w = d.vis[(size_t)u * RW + k];
    const int lo = nsrc - 64 * k, hi = G - 64 * k;   // keep the corners nsrc .. G - 1
    if (lo > 0) w = lo >= 64 ? 0ull : (w & (~0ull << lo));
    if (hi < 64) w = hi <= 0 ? 0ull : (w & ((1ull << hi) - 1ull));
    return w;
  };
  const bool short_ids = G <= 65535 && nitems <= kRelaxListMaxWords;
  if (short_ids) {
    for (long long it = tid; it < nitems; it += nt) {
      int u, k;
      const u64 w = arc_word(it, u, k);
      if (w) atomicAdd(&off[u + 1], __popcll(w));
    }
  }
  __syncthreads();
  if (short_ids && tid < 64) {
    // inclusive scan of off[1..G] by one wavefront, 64 at a time, carried serially
    int carry = 0;
    for (int b = 1; b <= G; b += 64) {
      const int g = b + lane;
      int x = g <= G ? off[g] : 0;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (g <= G) off[g] = carry + x;
      carry += __shfl(x, 63, 64);
    }
    if (lane == 0) narcs = carry;
  }
  __syncthreads();
  const bool lists = short_ids && (long long)narcs <= adj_cap;   // the same in every thread
  if (lists) {
    // each row's next free entry, kept in the ring (cleared after)
    for (int g = tid; g < G; g += nt) ring[g] = off[g];
    __syncthreads();
    for (long long it = tid; it < nitems; it += nt) {
      int u, k;
      u64 w = arc_word(it, u, k);
      if (!w) continue;
      const int at = atomicAdd(&ring[u], __popcll(w));
      for (int j = 0; w; ++j) {
        adj[at + j] = (unsigned short)(k * 64 + __builtin_ctzll(w));
        w &= w - 1;
      }
    }
    __syncthreads();
    for (int k = tid; k < cap; k += nt) ring[k] = -1;
    __syncthreads();
  }
  if (m0idx >= 0) {
    // the corners the last chip-wide round lowered: their arcs out are still to relax
    for (int v = nsrc + tid; v < G; v += nt) {
      if ((m0[v >> 6] >> (v & 63)) & 1ull) {
        atomicOr(&inq[v >> 5], 1u << (v & 31));
        const int t = atomicAdd(&tail, 1);
        ring[t] = v;
        atomicAdd(&pending, 1);
      }
    }
  } else {
    // from the sources (no chip-wide rounds before): every corner takes its best arc from a source
    // (sources cost 0; the same double sum as the other kernels), and the corners reached are queued
    for (int v = nsrc + tid; v < G; v += nt) {
      const int2 pv = xy[v];
      double best = INFINITY;
      for (int k = 0; 64 * k < nsrc; ++k) {
        u64 m = d.vis[(size_t)v * RW + k];
        if (nsrc - 64 * k < 64) m &= (1ull << (nsrc - 64 * k)) - 1ull;
        while (m) {
          const int u = 64 * k + __builtin_ctzll(m);
          m &= m - 1;
          best = fmin(best, 0.0 + arc_len4(d.gxy[u], pv.x, pv.y));
        }
      }
      if (best < INFINITY) {
        cost[v] = (u64)__double_as_longlong(best);
        atomicOr(&inq[v >> 5], 1u << (v & 31));
        const int t = atomicAdd(&tail, 1);
        ring[t] = v;
        atomicAdd(&pending, 1);
      }
    }
  }
  __syncthreads();
  // Both waits below end by construction (a queued corner is always being relaxed by a running wavefront,
  // and an entry is written right after its position is claimed); their spin limits only guard that
  // reasoning: a wavefront that reaches one stops and flags the build (MISC_ROUNDS = -1).
  bool stuck = false;
  for (;;) {
    // take a corner: lane 0 claims the next queue position, or sees that all work is done
    int h = -1;
    if (lane == 0) {
      for (int spin = 0; spin < kRelaxQueueSpin; ++spin) {
        const int hh = __hip_atomic_load(&head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int tt = __hip_atomic_load(&tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (hh < tt) {
          if (atomicCAS(&head, hh, hh + 1) == hh) { h = hh; break; }
          continue;
        }
        if (__hip_atomic_load(&pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) { h = -2; break; }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    h = __shfl(h, 0, 64);
    if (h == -1) stuck = true;
    if (h < 0) break;
    int u = -1;
    if (lane == 0) {
      // the producer writes the entry right after claiming its position
      int* slot = &ring[h % cap];
      for (int spin = 0; spin < kRelaxQueueSpin; ++spin) {
        u = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (u >= 0) break;
        __builtin_amdgcn_s_sleep(1);
      }
      if (u >= 0) {
        __hip_atomic_store(slot, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        // off the queue before its cost is read: a later lowering queues it again
        atomicAnd(&inq[u >> 5], ~(1u << (u & 31)));
      }
    }
    u = __shfl(u, 0, 64);
    if (u < 0) { stuck = true; break; }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const double cu = __longlong_as_double((long long)__hip_atomic_load(&cost[u], __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_WORKGROUP));
    const int2 pu2 = xy[u];
    const int4 pu = make_int4(pu2.x, pu2.y, pu2.x, pu2.y);
    // relax u -> v (a corner), queueing v when it is lowered and not queued yet
    auto relax = [&](int v) {
      const double cv = __longlong_as_double((long long)__hip_atomic_load(&cost[v], __ATOMIC_RELAXED,
                                                                           __HIP_MEMORY_SCOPE_WORKGROUP));
      if (!(cu < cv)) return;
      const int2 pv = xy[v];
      if (!(cu + arc_lower(pu, pv.x, pv.y) < cv)) return;
      const double cand = cu + arc_len4(pu, pv.x, pv.y);
      if (!(cand < cv)) return;
      const u64 ob = atomicMin(&cost[v], (u64)__double_as_longlong(cand));
      if (__longlong_as_double((long long)ob) > cand) {
        const unsigned bit = 1u << (v & 31);
        if (!(atomicOr(&inq[v >> 5], bit) & bit)) {
          atomicAdd(&pending, 1);
          const int t = atomicAdd(&tail, 1);
          __hip_atomic_store(&ring[t % cap], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    };
    if (lists) {
      const int a1 = off[u + 1];
      for (int i = off[u] + lane; i < a1; i += kWave) relax((int)adj[i]);
    } else {
      // the words of columns below G (the rest of a row is never set): one pass of loads up to 4096
      // corners, not a second dependent one
      for (int k0 = 0; k0 < RWg; k0 += kWave) {
        const int k = k0 + lane;
        u64 m = k < RWg ? d.vis[(size_t)u * RW + k] : 0ull;
        while (m) {
          const int v = k * 64 + __builtin_ctzll(m);
          m &= m - 1;
          if (v >= nsrc && v < G) relax(v);   // sources keep cost 0
        }
      }
    }
    // every corner this one lowered is counted before it stops counting
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (lane == 0) atomicSub(&pending, 1);
  }
  __syncthreads();
  // outputs by canonical id; parents follow in k_gsort_parents
  int mine = 0;
  for (int p = tid; p < G; p += nt) {
    const double c = __longlong_as_double((long long)cost[p]);
    const int v = d.gorder[p];
    d.costpos[p] = cost[p];
    d.gen_cost[v] = c;
    d.cost64[v] = c;
    if (c < INFINITY) ++mine;
  }
  atomicAdd(&reached, mine);
  __syncthreads();
  if (tid == 0) {
    d.misc[MISC_REACHED] = reached;
    d.misc[MISC_ROUNDS] = rounds0;
  }
  __syncthreads();
  if (stuck && lane == 0) d.misc[MISC_ROUNDS] = -1;
}

// One wavefront per generator: rank by (float cost, id) among all generators;
// unreached ones (+inf) rank last and are not copied.
template <class S>
__device__ __forceinline__ void gsort_wave(const S& src, int wid) {
  int sc, g;
  if (!src.locate(STG_GEN, wid, sc, g)) return;
  const Dev& d = src.scene(sc);
  const int G = uni(d.misc[MISC_G]);
  if (g >= G) return;
  const int lane = lane_id();
  // requested up front: this generator's record (written after the rank)
  GenRec r = d.gens[g];
  const float cf = (float)d.cost64[g];
  const u64 key = ((u64)__float_as_uint(cf) << 32) | (u64)(unsigned)g;
  int rank = 0;
  for (int base = 0; base < G; base += 256) {
    // four batches of 64 keys requested together
    float ch[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int h = base + 64 * q + lane;
      ch[q] = h < G ? (float)d.cost64[h] : INFINITY;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int h = base + 64 * q + lane;
      rank += __popcll(ballot(h < G && (((u64)__float_as_uint(ch[q]) << 32) | (u64)(unsigned)h) < key));
    }
  }
  if (lane == 0 && cf < INFINITY) {
    r.costf = cf;
    d.sgen[rank] = r;
    d.sgcost[rank] = cf;
    d.sgbb[rank] = make_int4(min(r.x, r.x2), min(r.y, r.y2), max(r.x, r.x2), max(r.y, r.y2));
  }
  if (lane == 0) d.krank[g] = cf < INFINITY ? rank : -1;
}

// The generator sort and the parents in one launch: the first nsort
// workgroups rank generators, the next nsort find parents (four wavefronts
// each); for a single scene, norder more build the pixel stage's work order
// (tile_order_group) from the canonical costs and coordinates, staged in LDS.
template <class S>
__global__ __launch_bounds__(256) void k_gsort_parents(S src, int nsort, int norder) {
  const int b = blockIdx.x;
  if (b < nsort) {
    gsort_wave(src, b * 4 + (threadIdx.x >> 6));
  } else if (b < 2 * nsort) {
    parent_wave(src, (b - nsort) * 4 + (threadIdx.x >> 6));
  } else if (b < 2 * nsort + norder) {
    extern __shared__ int4 gsm[];
    __shared__ int lcount[kOrderBins], lbase[kOrderBins], icls[kOrderGroup], islot[kOrderGroup];
    const Dev& d = src.scene(0);
    const int G = d.misc[MISC_G];
    int4* bb = gsm;
    float* cost = (float*)(gsm + d.Gmax);
    // the minimum runs over all generators, so the compact arrays by spatial position serve
    for (int g = threadIdx.x; g < G; g += blockDim.x) {
      const int4 r = d.gxy[g];
      bb[g] = make_int4(min(r.x, r.z), min(r.y, r.w), max(r.x, r.z), max(r.y, r.w));
      cost[g] = (float)__longlong_as_double((long long)d.costpos[g]);
    }
    if (threadIdx.x < kOrderBins) lcount[threadIdx.x] = 0;
    __syncthreads();
    tile_order_group(d, b - 2 * nsort, G, bb, cost, lcount, lbase, icls, islot);
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
  const long long nb = p.total[STG_GVBLK], ns = (p.total[STG_SEGVIS] + 3) / 4;
  if (nb + ns <= 0) return hipSuccess;
  const dim3 grid((unsigned)(nb + ns));
  if (p.genvis_lds > 0 && p.genvis_lds <= 32768)
    hipLaunchKernelGGL((k_genvis<S, true>), grid, dim3(256), p.genvis_lds, s, src, (int)nb);
  else
    hipLaunchKernelGGL((k_genvis<S, false>), grid, dim3(256), 0, s, src, (int)nb);
  return hipGetLastError();
}

template <class S>
hipError_t launch_relax(const S& src, const Plan& p, hipStream_t s) {
  const long long nw = p.total[STG_RELAXW];
  const unsigned wblocks = (unsigned)((nw + 255) / 256);
  const int RWcap = p.maxRW > 0 ? p.maxRW : 1;
  const int Gcap = p.maxGmax > 0 ? p.maxGmax : 1;
  const size_t chg = 2 * (size_t)RWcap * sizeof(u64);
  const size_t shm = chg + (size_t)Gcap * (sizeof(u64) + sizeof(int4));
  const size_t shm_v = shm + (size_t)Gcap * RWcap * sizeof(u64);
  const size_t static_lds = 4 * 3 + kRelaxFront * 4 + 64;
  const size_t lim = (size_t)max_lds_per_block();
  const dim3 grid((unsigned)p.total[STG_SCENE]);
  auto big = [&](const void* f, size_t bytes) {
    return bytes > 65536 ? hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)
                         : hipSuccess;
  };
  hipError_t e = hipSuccess;
  const size_t shm_q = relax_queue_lds_bytes(Gcap);
  // the queue kernel takes what LDS a workgroup may have beyond its tables for its adjacency lists
  const size_t shm_qr = lim > 256 + shm_q ? lim - 256 : shm_q;
  const bool adapt = p.maxGmax > kChaosAdaptMinGen;
  const bool batch = p.total[STG_SCENE] > 1;
  if (kRelaxQueueSrc > 0 && (batch || kRelaxQueueSrc > 1) && !adapt && shm_q + 64 <= lim) {
    // small graphs: the whole relaxation on the work queue, from the sources, one workgroup per scene
    if ((e = big((const void*)k_relax_queue<S>, shm_qr)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_relax_queue<S>), grid, dim3(kRelaxThreads), shm_qr, s, src, Gcap, -1, 0, (int)shm_qr);
    return hipGetLastError();
  }
  // the large early rounds chip-wide: without barriers then one exact round, or kRelaxWideRounds rounds
  int m0idx = kRelaxWideRounds % 3, rounds0 = kRelaxWideRounds;
  if (kRelaxChaos > 0) {
    m0idx = 2;
    rounds0 = (adapt ? kRelaxChaosMax : kRelaxChaos) + 1;
    if (nw > 0) {
      if (adapt)
        hipLaunchKernelGGL((k_relax_chaos<S, true>), dim3(wblocks), dim3(256), 0, s, src, kRelaxChaosMax);
      else
        hipLaunchKernelGGL((k_relax_chaos<S, false>), dim3(wblocks), dim3(256), 0, s, src, kRelaxChaos);
      hipLaunchKernelGGL(k_relax_wide<S>, dim3(wblocks), dim3(256), 0, s, src, 1);
    }
  } else if (nw > 0) {
    for (int r = 0; r < kRelaxWideRounds; ++r)
      hipLaunchKernelGGL(k_relax_wide<S>, dim3(wblocks), dim3(256), 0, s, src, r);
  }
  if (kRelaxQueue && kRelaxChaos > 0 && adapt && shm_q + 64 <= lim) {
    // deep graphs: the rest without rounds
    if ((e = big((const void*)k_relax_queue<S>, shm_qr)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_relax_queue<S>), grid, dim3(kRelaxThreads), shm_qr, s, src, Gcap, m0idx, rounds0,
                       (int)shm_qr);
  } else if (shm_v + static_lds <= lim) {
    if ((e = big((const void*)k_relax<S, true, true>, shm_v)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_relax<S, true, true>), grid, dim3(kRelaxThreads), shm_v, s, src, Gcap, RWcap, m0idx, rounds0);
  } else if (shm + static_lds <= lim) {
    if ((e = big((const void*)k_relax<S, true, false>, shm)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_relax<S, true, false>), grid, dim3(kRelaxThreads), shm, s, src, Gcap, RWcap, m0idx, rounds0);
  } else {
    hipLaunchKernelGGL((k_relax<S, false, false>), grid, dim3(kRelaxThreads), chg, s, src, Gcap, RWcap, m0idx, rounds0);
  }
  return hipGetLastError();
}

template <class S>
hipError_t launch_gsort(const S& src, const Plan& p, hipStream_t s) {
  if (p.total[STG_GEN] <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((p.total[STG_GEN] + 3) / 4);
  unsigned norder = 0;
  size_t shm = 0;
  if constexpr (std::is_same<S, SingleSrc>::value) {
    if (order_fused(src.d)) {
      norder = (unsigned)((order_items(src.d) + kOrderGroup - 1) / kOrderGroup);
      shm = (size_t)src.d.Gmax * (sizeof(int4) + sizeof(float));
    }
  }
  hipLaunchKernelGGL(k_gsort_parents<S>, dim3(2 * nb + norder), dim3(256), shm, s, src, (int)nb, (int)norder);
  return hipGetLastError();
}

template hipError_t launch_genvis<SingleSrc>(const SingleSrc&, const Plan&, hipStream_t);
template hipError_t launch_genvis<BatchSrc>(const BatchSrc&, const Plan&, hipStream_t);
template hipError_t launch_relax<SingleSrc>(const SingleSrc&, const Plan&, hipStream_t);
template hipError_t launch_relax<BatchSrc>(const BatchSrc&, const Plan&, hipStream_t);
template hipError_t launch_gsort<SingleSrc>(const SingleSrc&, const Plan&, hipStream_t);
template hipError_t launch_gsort<BatchSrc>(const BatchSrc&, const Plan&, hipStream_t);

}  // namespace spm
