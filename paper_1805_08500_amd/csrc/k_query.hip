// k_query.hip -- map queries at arbitrary points, refined by the neighbouring
// pixels' parents, and the whole path of each query.
//
// A query point q takes, from the built map, the parents of the 3 x 3 pixels
// around it and keeps the one of least cost(g) + |q - x_g(q)| among those that
// q actually sees.  A point near the border of two regions can belong to the
// region of a neighbouring pixel; comparing the neighbours' parents at q
// itself removes the first-turn error a pixel lookup would make (Section 5.1, Discussion).
// If q sees none of them, every generator is compared.  Then the path is the
// chain of parents down to a source (Section 1: one lookup, then a walk).
//
// Exactness: q is snapped to the lattice of kQueryQW-ths of a doubled unit
// (1/512 domain unit); visibility from the snapped point uses exact integer
// predicates (64-bit, 128-bit for the one product of a segment's closest
// point), under the closed-free-space rule the pixel stage uses.  The
// distance is evaluated in double precision.
#include <math.h>

#include "spm_internal.hpp"

namespace spm {

constexpr long long kQueryQW = 256;   // lattice: doubled coordinates times kQueryQW

struct QueryArgs {
  int W, H, n_polys, nv;
  const int* poly_start;
  const int* vx;
  const int* vy;
  const int* parent;     // [H * W]
  const int* gen_kind;   // [G]
  const int* gen_xy;     // [G * 4] domain units
  const double* gen_cost;
  const int* gen_parent;
  const int* n_gen;
  const float* pts;      // [n * 2] domain units
  int n, cap;
  float* dist;           // [n]
  int* par;              // [n]
  float* path_xy;        // [n * cap * 2] or null
  int* path_n;           // [n] or null
};

__device__ __forceinline__ int sgn64(long long v) { return (v > 0) - (v < 0); }

// vertex i of the scene: its loop neighbours (prev, next), by a binary search of poly_start
__device__ __forceinline__ void loop_nbrs(const QueryArgs& a, int i, int& prv, int& nxt) {
  int lo = 0, hi = a.n_polys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.poly_start[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  const int s = a.poly_start[lo], e = a.poly_start[lo + 1];
  prv = i == s ? e - 1 : i - 1;
  nxt = i == e - 1 ? s : i + 1;
}

// Lane-parallel over vertices (vertex i and its edge i -> next(i)): is the
// closed segment from q to the target free?  Target: the lattice point
// (tx, ty) (fine units), or -- perp -- the closest point of segment A-B,
// strictly inside it, whose segment [q, q*] is perpendicular to e = B - A.
// tv: the target is the scene vertex with that index (its own-angle rule).
__device__ bool query_visible(const QueryArgs& a, long long qx, long long qy, bool perp, long long tx, long long ty,
                              int tv, long long Ax, long long Ay, long long Bx, long long By) {
  const int lane = lane_id();
  const long long Q = kQueryQW * 2;   // fine units per domain unit
  // perpendicular family: D(x) = e . x, F(x) = cross(e, x - A) (fine units; e in doubled units)
  const long long ex = (Bx - Ax) / kQueryQW, ey = (By - Ay) / kQueryQW;
  const long long Dq = ex * qx + ey * qy;
  const long long Fq = ex * (qy - Ay) - ey * (qx - Ax);
  const long long L = ex * ex + ey * ey;
  const long long num = (qx - Ax) * ex + (qy - Ay) * ey;   // (q - A) . e, in (0, L * QW)
  bool blocked = false;
  if (tv >= 0 && lane == 0) {
    int pr, nx;
    loop_nbrs(a, tv, pr, nx);
    blocked = into_interior64(2 * a.vx[pr], 2 * a.vy[pr], 2 * a.vx[tv], 2 * a.vy[tv], 2 * a.vx[nx], 2 * a.vy[nx],
                              qx - tx, qy - ty);
  }
  for (int base = 0; base < a.nv && !ballot(blocked); base += kWave) {
    const int i = base + lane;
    if (i >= a.nv) continue;
    int pr, nx;
    loop_nbrs(a, i, pr, nx);
    const long long wx = Q * a.vx[i], wy = Q * a.vy[i], vx = Q * a.vx[nx], vy = Q * a.vy[nx];
    // the edge's line: E(x) = cross(v - w, x - w)
    const long long Eq = (vx - wx) * (qy - wy) - (vy - wy) * (qx - wx);
    bool cross = false, onl = false;
    if (!perp) {
      const long long ow = (tx - qx) * (wy - qy) - (ty - qy) * (wx - qx);
      const long long ov = (tx - qx) * (vy - qy) - (ty - qy) * (vx - qx);
      const long long Et = (vx - wx) * (ty - wy) - (vy - wy) * (tx - wx);
      cross = sgn64(ow) * sgn64(ov) < 0 && sgn64(Eq) * sgn64(Et) < 0;
      if (ow == 0) {
        // w on line q-t strictly between q and t
        const long long d1 = (wx - qx) * (tx - qx) + (wy - qy) * (ty - qy);
        const long long d2 = (tx - qx) * (tx - qx) + (ty - qy) * (ty - qy);
        onl = d1 > 0 && d1 < d2;
      }
    } else {
      const long long Dw = ex * wx + ey * wy, Dv = ex * vx + ey * vy;
      // E(q*) * L * QW = E(A) * L * QW + num * (E(B) - E(A)), in 128 bits
      const long long EA = (vx - wx) * (Ay - wy) - (vy - wy) * (Ax - wx);
      const long long EB = (vx - wx) * (By - wy) - (vy - wy) * (Bx - wx);
      const __int128 Es = (__int128)EA * L * kQueryQW + (__int128)num * (EB - EA);
      const int sEs = (Es > 0) - (Es < 0);
      cross = sgn64(Dw - Dq) * sgn64(Dv - Dq) < 0 && sgn64(Eq) * sEs < 0;
      if (Dw == Dq) {
        // w on line q-q* strictly between q and q* (F runs from F(q) to 0)
        const long long Fw = ex * (wy - Ay) - ey * (wx - Ax);
        onl = Fq > 0 ? (Fw > 0 && Fw < Fq) : (Fw < 0 && Fw > Fq);
      }
    }
    if (onl) {
      // the vertex rule at w: neither direction along the segment enters its interior angle
      long long d1x, d1y, d2x, d2y;
      if (!perp) {
        d1x = qx - wx; d1y = qy - wy; d2x = tx - wx; d2y = ty - wy;
      } else {
        // toward q: +-(-ey, ex) with the sign of F(q); toward q*: the opposite
        const long long s = Fq > 0 ? 1 : -1;
        d1x = -ey * s; d1y = ex * s; d2x = -d1x; d2y = -d1y;
      }
      const int ux = 2 * a.vx[pr], uy = 2 * a.vy[pr], cx = 2 * a.vx[i], cy = 2 * a.vy[i];
      const int nx2 = 2 * a.vx[nx], ny2 = 2 * a.vy[nx];
      if (into_interior64(ux, uy, cx, cy, nx2, ny2, d1x, d1y) || into_interior64(ux, uy, cx, cy, nx2, ny2, d2x, d2y))
        cross = true;
    }
    blocked = blocked || cross;
  }
  return !ballot(blocked);
}

// closed inside-obstacle test of q (lane-parallel crossing parity)
__device__ bool query_inside(const QueryArgs& a, long long qx, long long qy) {
  const int lane = lane_id();
  const long long Q = kQueryQW * 2;
  int parity = 0;
  bool on = false;
  for (int base = 0; base < a.nv; base += kWave) {
    const int i = base + lane;
    bool flip = false;
    if (i < a.nv) {
      int pr, nx;
      loop_nbrs(a, i, pr, nx);
      const long long wx = Q * a.vx[i], wy = Q * a.vy[i], vx = Q * a.vx[nx], vy = Q * a.vy[nx];
      const long long c = (vx - wx) * (qy - wy) - (vy - wy) * (qx - wx);
      if (c == 0 && qx >= min(wx, vx) && qx <= max(wx, vx) && qy >= min(wy, vy) && qy <= max(wy, vy)) on = true;
      // the ray from q toward +x crosses the edge (half-open in y)
      if ((wy > qy) != (vy > qy)) flip = (c > 0) == (vy > wy);
    }
    parity ^= __popcll(ballot(flip)) & 1;
  }
  return ballot(on) != 0 || parity;
}

// target of generator g seen from q (fine units): a lattice point, or the
// perpendicular foot on a segment (perp); value in domain units, double
__device__ double query_value(const QueryArgs& a, int g, long long qx, long long qy, bool& perp, long long& tx,
                              long long& ty, long long& Ax, long long& Ay, long long& Bx, long long& By) {
  const long long Q = kQueryQW * 2;
  const int* xy = a.gen_xy + 4 * g;
  perp = false;
  tx = Q * xy[0];
  ty = Q * xy[1];
  Ax = tx; Ay = ty; Bx = Q * xy[2]; By = Q * xy[3];
  if (a.gen_kind[g] == SPM_GEN_SEGMENT) {
    const long long ex = (Bx - Ax) / kQueryQW, ey = (By - Ay) / kQueryQW;   // doubled units
    const long long L = ex * ex + ey * ey;
    const long long num = (qx - Ax) * ex + (qy - Ay) * ey;
    if (num >= L * kQueryQW) { tx = Bx; ty = By; }
    else if (num > 0) {
      perp = true;
      const double cr = (double)(ex * (qy - Ay) - ey * (qx - Ax));
      return a.gen_cost[g] + fabs(cr) / ((double)Q * sqrt((double)L));
    }
  }
  const double dx = (double)(qx - tx) / (double)Q, dy = (double)(qy - ty) / (double)Q;
  return a.gen_cost[g] + sqrt(dx * dx + dy * dy);
}

// scene vertex index of a corner generator at (x, y) domain units (lane-parallel search)
__device__ int vertex_at(const QueryArgs& a, int x, int y) {
  for (int base = 0; base < a.nv; base += kWave) {
    const int i = base + lane_id();
    const u64 m = ballot(i < a.nv && a.vx[i] == x && a.vy[i] == y);
    if (m) return base + first_bit(m);
  }
  return -1;
}

// One wavefront per query point.
__global__ __launch_bounds__(256) void k_query_points(QueryArgs a) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= a.n) return;
  const int lane = lane_id();
  const int G = a.n_gen[0];
  const float fx = a.pts[2 * k], fy = a.pts[2 * k + 1];
  const long long Q = kQueryQW * 2;
  double best = INFINITY;
  int bestg = -1;
  long long qx = 0, qy = 0;
  const bool in_dom = fx >= 0.0f && fy >= 0.0f && fx <= (float)a.W && fy <= (float)a.H;
  if (in_dom) {
    qx = llrint((double)fx * (double)Q);
    qy = llrint((double)fy * (double)Q);
  }
  if (in_dom && !query_inside(a, qx, qy)) {
    const int i = min((int)floorf(fx), a.W - 1), j = min((int)floorf(fy), a.H - 1);
    // the 3 x 3 neighbourhood's parents (lanes 0..8)
    int cand = -1;
    if (lane < 9) {
      const int ii = i + lane % 3 - 1, jj = j + lane / 3 - 1;
      if (ii >= 0 && jj >= 0 && ii < a.W && jj < a.H) cand = a.parent[(size_t)jj * a.W + ii];
      if (cand >= G) cand = -1;
    }
    for (int pass = 0; pass < 2 && bestg < 0; ++pass) {
      // pass 0: the distinct neighbour parents; pass 1 (none of them visible): every generator
      u64 m = pass == 0 ? ballot(cand >= 0) : 0;
      const int count = pass == 0 ? 64 : G;
      for (int t = 0; t < count; ++t) {
        int g;
        if (pass == 0) {
          if (!m) break;
          g = readlane(cand, first_bit(m));
          m &= ~ballot(cand == g);
        } else {
          g = t;
        }
        if (!(a.gen_cost[g] < INFINITY)) continue;
        bool perp;
        long long tx, ty, Ax, Ay, Bx, By;
        const double v = query_value(a, g, qx, qy, perp, tx, ty, Ax, Ay, Bx, By);
        // (value, id) order, as the map's own ties
        if (!(v < best || (v == best && g < bestg))) continue;
        const int tv = a.gen_kind[g] == SPM_GEN_VERTEX ? vertex_at(a, a.gen_xy[4 * g], a.gen_xy[4 * g + 1]) : -1;
        if (query_visible(a, qx, qy, perp, tx, ty, tv, Ax, Ay, Bx, By)) {
          best = v;
          bestg = g;
        }
      }
    }
  }
  if (lane != 0) return;
  a.dist[k] = (float)best;
  a.par[k] = bestg;
  if (!a.path_n) return;
  // the path: q, the corners of the parent chain, then the source (a segment's closest point)
  int n = 0;
  float* o = a.path_xy ? a.path_xy + (size_t)k * a.cap * 2 : nullptr;
  auto put = [&](float x, float y) {
    if (o && n < a.cap) { o[2 * n] = x; o[2 * n + 1] = y; }
    ++n;
  };
  if (bestg >= 0) {
    put((float)((double)qx / (double)Q), (float)((double)qy / (double)Q));
    double lx = (double)qx / (double)Q, ly = (double)qy / (double)Q;
    int g = bestg;
    for (int steps = 0; steps <= G; ++steps) {
      const int* xy = a.gen_xy + 4 * g;
      if (a.gen_kind[g] == SPM_GEN_SEGMENT) {
        const double ax = xy[0], ay = xy[1], ex = xy[2] - ax, ey = xy[3] - ay;
        const double t = fmin(1.0, fmax(0.0, ((lx - ax) * ex + (ly - ay) * ey) / (ex * ex + ey * ey)));
        put((float)(ax + t * ex), (float)(ay + t * ey));
        break;
      }
      put((float)xy[0], (float)xy[1]);
      if (a.gen_kind[g] == SPM_GEN_POINT) break;
      lx = xy[0];
      ly = xy[1];
      const int pg = a.gen_parent[g];
      if (pg < 0 || pg == g) break;
      g = pg;
    }
  }
  a.path_n[k] = n;
}

hipError_t launch_query_points(const spm_scene* s, const spm_out* out, int n, const float* pts, int cap, float* dist,
                               int* par, float* path_xy, int* path_n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  QueryArgs a;
  a.W = s->width; a.H = s->height; a.n_polys = s->n_polys; a.nv = s->n_vertices;
  a.poly_start = s->poly_start; a.vx = s->vx; a.vy = s->vy;
  a.parent = out->parent; a.gen_kind = out->gen_kind; a.gen_xy = out->gen_xy; a.gen_cost = out->gen_cost;
  a.gen_parent = out->gen_parent; a.n_gen = out->n_gen;
  a.pts = pts; a.n = n; a.cap = cap; a.dist = dist; a.par = par; a.path_xy = path_xy; a.path_n = path_n;
  hipLaunchKernelGGL(k_query_points, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace spm
