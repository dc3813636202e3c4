/*
 * spm_oracle.c -- reference CPU implementation of a multi-source shortest path
 * map (SPM).  TEST INFRASTRUCTURE ONLY: nothing in the product library links,
 * loads or calls this file.  It shares no code with the GPU library.
 *
 * What it computes (the plain definition the paper's method reaches):
 *   For every pixel centre p of a W x H grid over the domain [0,W]x[0,H]
 *   (Section 3, the framebuffer covers the domain), D(p) is the length of the
 *   shortest obstacle-avoiding path from p to the nearest source -- a point
 *   source (Section 3) or any point of a segment source (Section 4) -- and
 *   parent(p) is the first point the path turns at: an obstacle vertex, or the
 *   source itself (Section 3, ParentId; Section 1, path maps share a parent).
 *
 * How: the textbook route the paper cites (Section 2: visibility graph plus
 * graph search).  Generators are the point sources, the segment sources and
 * the obstacle corners a shortest path can bend at (corners whose obstacle
 * interior angle is below 180 degrees).  Their costs come from Dijkstra on the
 * generator visibility graph (the generator order and costs of Procedures 1
 * and 4); then every pixel takes the minimum over visible generators of
 * cost(g) + |p - x_g(p)| (the cone of Procedure 3), where x_g(p) is g itself,
 * or for a segment source the closest point of the segment to p (Section 4:
 * distance to an endpoint or to the projection).
 *
 * Exactness: all geometry runs on "doubled" integer coordinates (every domain
 * coordinate times 2, so the pixel centre (i+1/2, j+1/2) becomes (2i+1, 2j+1)).
 * Orientation tests are exact determinants of homogeneous points in __int128;
 * distances and costs are IEEE double.
 *
 * Visibility rule (the paper draws shadows by rasterization and never defines
 * grazing contacts; the reading used here is the closed-free-space one):
 * the closed segment [a,b] is visible iff it does not meet the open interior
 * of any obstacle, i.e. (i) it properly crosses no edge, and (ii) at every
 * obstacle vertex w lying on [a,b], neither the direction toward a nor the
 * direction toward b points strictly into the obstacle's interior angle at w.
 *
 * Tie-break: among equal totals the candidate with the smaller cost and then
 * the smaller generator id wins (the paper expands generators in cost order
 * and keeps the first cone that reaches a value: strict comparison in
 * Procedures 3 and 4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

enum { ORC_OK = 0, ORC_ERR = -1 };
enum { ORC_POINT = 0, ORC_SEGMENT = 1, ORC_VERTEX = 2 };

typedef struct {
  int width, height;
  int n_polys;
  const int *poly_start; /* n_polys + 1 */
  const int *vx, *vy;    /* domain units */
  int n_points;
  const int *pts; /* n_points * 2 */
  int n_segs;
  const int *segs; /* n_segs * 4 */
} orc_scene;

/* homogeneous rational point (x/w, y/w), w > 0, doubled coordinates */
typedef struct {
  i128 x, y, w;
} hpt;

static hpt hp(i128 x, i128 y) {
  hpt r = {x, y, 1};
  return r;
}

/* sign of the orientation determinant of a, b, c (counter-clockwise > 0) */
static int orient(hpt a, hpt b, hpt c) {
  i128 d = a.x * (b.y * c.w - b.w * c.y) - a.y * (b.x * c.w - b.w * c.x) + a.w * (b.x * c.y - b.y * c.x);
  return (d > 0) - (d < 0);
}

static int same_point(hpt a, hpt b) { return a.x * b.w == b.x * a.w && a.y * b.w == b.y * a.w; }

/* scene in doubled coordinates with per-vertex neighbours */
typedef struct {
  int W, H;
  int nv;          /* number of obstacle vertices = number of edges */
  int64_t *x, *y;  /* doubled vertex coords */
  int *prev, *next;
  int np, ns;
  int64_t *px, *py;              /* doubled point sources */
  int64_t *sax, *say, *sbx, *sby; /* doubled segment sources */
  int G;
  int *gkind, *gref; /* gref: point index, segment index or vertex index */
} oscene;

static void free_oscene(oscene *s) {
  free(s->x); free(s->y); free(s->prev); free(s->next);
  free(s->px); free(s->py);
  free(s->sax); free(s->say); free(s->sbx); free(s->sby);
  free(s->gkind); free(s->gref);
}

static int load_oscene(const orc_scene *in, oscene *s) {
  memset(s, 0, sizeof(*s));
  s->W = in->width;
  s->H = in->height;
  int nv = in->n_polys > 0 ? in->poly_start[in->n_polys] : 0;
  s->nv = nv;
  s->x = (int64_t *)malloc(sizeof(int64_t) * (nv + 1));
  s->y = (int64_t *)malloc(sizeof(int64_t) * (nv + 1));
  s->prev = (int *)malloc(sizeof(int) * (nv + 1));
  s->next = (int *)malloc(sizeof(int) * (nv + 1));
  for (int p = 0; p < in->n_polys; ++p) {
    int a = in->poly_start[p], b = in->poly_start[p + 1];
    for (int i = a; i < b; ++i) {
      s->x[i] = 2 * (int64_t)in->vx[i];
      s->y[i] = 2 * (int64_t)in->vy[i];
      s->prev[i] = (i == a) ? b - 1 : i - 1;
      s->next[i] = (i == b - 1) ? a : i + 1;
    }
  }
  s->np = in->n_points;
  s->ns = in->n_segs;
  s->px = (int64_t *)malloc(sizeof(int64_t) * (s->np + 1));
  s->py = (int64_t *)malloc(sizeof(int64_t) * (s->np + 1));
  for (int i = 0; i < s->np; ++i) {
    s->px[i] = 2 * (int64_t)in->pts[2 * i];
    s->py[i] = 2 * (int64_t)in->pts[2 * i + 1];
  }
  s->sax = (int64_t *)malloc(sizeof(int64_t) * (s->ns + 1));
  s->say = (int64_t *)malloc(sizeof(int64_t) * (s->ns + 1));
  s->sbx = (int64_t *)malloc(sizeof(int64_t) * (s->ns + 1));
  s->sby = (int64_t *)malloc(sizeof(int64_t) * (s->ns + 1));
  for (int i = 0; i < s->ns; ++i) {
    s->sax[i] = 2 * (int64_t)in->segs[4 * i];
    s->say[i] = 2 * (int64_t)in->segs[4 * i + 1];
    s->sbx[i] = 2 * (int64_t)in->segs[4 * i + 2];
    s->sby[i] = 2 * (int64_t)in->segs[4 * i + 3];
  }
  /* generators in canonical order: points, segments, then every obstacle
   * corner with a left turn (interior angle < 180 deg for CCW loops) */
  int G = s->np + s->ns;
  for (int i = 0; i < nv; ++i) {
    hpt u = hp(s->x[s->prev[i]], s->y[s->prev[i]]), w = hp(s->x[i], s->y[i]), v = hp(s->x[s->next[i]], s->y[s->next[i]]);
    if (orient(u, w, v) > 0) ++G;
  }
  s->G = G;
  s->gkind = (int *)malloc(sizeof(int) * (G + 1));
  s->gref = (int *)malloc(sizeof(int) * (G + 1));
  int k = 0;
  for (int i = 0; i < s->np; ++i) { s->gkind[k] = ORC_POINT; s->gref[k++] = i; }
  for (int i = 0; i < s->ns; ++i) { s->gkind[k] = ORC_SEGMENT; s->gref[k++] = i; }
  for (int i = 0; i < nv; ++i) {
    hpt u = hp(s->x[s->prev[i]], s->y[s->prev[i]]), w = hp(s->x[i], s->y[i]), v = hp(s->x[s->next[i]], s->y[s->next[i]]);
    if (orient(u, w, v) > 0) { s->gkind[k] = ORC_VERTEX; s->gref[k++] = i; }
  }
  return ORC_OK;
}

/* is the direction d (from vertex i) strictly inside the obstacle's interior angle at i? */
static int dir_into_interior(const oscene *s, int i, i128 dx, i128 dy) {
  i128 ux = s->x[s->prev[i]], uy = s->y[s->prev[i]];
  i128 wx = s->x[i], wy = s->y[i];
  i128 vx = s->x[s->next[i]], vy = s->y[s->next[i]];
  i128 turn = (wx - ux) * (vy - wy) - (wy - uy) * (vx - wx);
  i128 c1 = (wx - ux) * dy - (wy - uy) * dx; /* d left of the incoming edge */
  i128 c2 = (vx - wx) * dy - (vy - wy) * dx; /* d left of the outgoing edge */
  if (turn > 0) return c1 > 0 && c2 > 0; /* convex corner: both */
  return c1 > 0 || c2 > 0;               /* reflex corner: either */
}

static i128 floor_div(i128 x, i128 w) { return x >= 0 ? x / w : -((-x + w - 1) / w); }
static i128 ceil_div(i128 x, i128 w) { return -floor_div(-x, w); }

/* closed segment [a,b] avoids every open obstacle interior */
static int visible(const oscene *s, hpt a, hpt b) {
  if (same_point(a, b)) return 1;
  /* integer box around [a,b] (rounded outward): an edge or vertex outside it
   * cannot meet the segment, so both loops skip it.  Speed only. */
  i128 ax0 = floor_div(a.x, a.w), ax1 = ceil_div(a.x, a.w), ay0 = floor_div(a.y, a.w), ay1 = ceil_div(a.y, a.w);
  i128 bx0 = floor_div(b.x, b.w), bx1 = ceil_div(b.x, b.w), by0 = floor_div(b.y, b.w), by1 = ceil_div(b.y, b.w);
  int64_t lox = (int64_t)(ax0 < bx0 ? ax0 : bx0), hix = (int64_t)(ax1 > bx1 ? ax1 : bx1);
  int64_t loy = (int64_t)(ay0 < by0 ? ay0 : by0), hiy = (int64_t)(ay1 > by1 ? ay1 : by1);
  /* (i) proper crossings */
  for (int i = 0; i < s->nv; ++i) {
    int64_t ex0 = s->x[i], ey0 = s->y[i], ex1 = s->x[s->next[i]], ey1 = s->y[s->next[i]];
    if ((ex0 < lox && ex1 < lox) || (ex0 > hix && ex1 > hix) || (ey0 < loy && ey1 < loy) ||
        (ey0 > hiy && ey1 > hiy))
      continue;
    hpt p1 = hp(s->x[i], s->y[i]);
    hpt p2 = hp(s->x[s->next[i]], s->y[s->next[i]]);
    int o1 = orient(a, b, p1), o2 = orient(a, b, p2);
    if (o1 * o2 >= 0) continue;
    int o3 = orient(p1, p2, a), o4 = orient(p1, p2, b);
    if (o3 * o4 < 0) return 0;
  }
  /* (ii) vertices lying on the closed segment */
  for (int i = 0; i < s->nv; ++i) {
    if (s->x[i] < lox || s->x[i] > hix || s->y[i] < loy || s->y[i] > hiy) continue;
    hpt w = hp(s->x[i], s->y[i]);
    if (orient(a, b, w) != 0) continue;
    /* collinear: is w between a and b?  compare scaled coordinates */
    i128 ax = a.x, ay = a.y, bx = b.x * 1, by = b.y;
    i128 wxa = w.x * a.w, wya = w.y * a.w; /* w scaled to a's denominator */
    i128 wxb = w.x * b.w, wyb = w.y * b.w;
    /* (w - a) . (b - a) >= 0 and (w - b) . (a - b) >= 0, in homogeneous form */
    i128 dax = wxa - ax, day = wya - ay;                /* (w - a) * a.w */
    i128 bax = bx * a.w - ax * b.w, bay = by * a.w - ay * b.w; /* (b - a) * a.w * b.w */
    i128 dbx = wxb - bx, dby = wyb - by;                /* (w - b) * b.w */
    if (dax * bax + day * bay < 0) continue;
    if (-(dbx * bax + dby * bay) < 0) continue;
    /* direction toward a (if w != a) and toward b (if w != b) */
    if (!same_point(w, a) && dir_into_interior(s, i, ax - wxa, ay - wya)) return 0;
    if (!same_point(w, b) && dir_into_interior(s, i, bx - wxb, by - wyb)) return 0;
  }
  return 1;
}

/* closest point of segment source k to the integer point (x, y): homogeneous, and
 * the Euclidean distance in domain units (Section 4: endpoint or projection) */
static hpt seg_closest(const oscene *s, int k, int64_t x, int64_t y, double *dist) {
  int64_t ax = s->sax[k], ay = s->say[k], bx = s->sbx[k], by = s->sby[k];
  int64_t ex = bx - ax, ey = by - ay;
  int64_t L = ex * ex + ey * ey;
  int64_t num = (x - ax) * ex + (y - ay) * ey;
  if (num <= 0) {
    double dx = (double)(x - ax), dy = (double)(y - ay);
    *dist = 0.5 * sqrt(dx * dx + dy * dy);
    return hp(ax, ay);
  }
  if (num >= L) {
    double dx = (double)(x - bx), dy = (double)(y - by);
    *dist = 0.5 * sqrt(dx * dx + dy * dy);
    return hp(bx, by);
  }
  int64_t cr = ex * (y - ay) - ey * (x - ax);
  *dist = 0.5 * fabs((double)cr) / sqrt((double)L);
  hpt q;
  q.x = (i128)ax * L + (i128)num * ex;
  q.y = (i128)ay * L + (i128)num * ey;
  q.w = L;
  return q;
}

static double pt_dist(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  double dx = (double)(ax - bx), dy = (double)(ay - by);
  return 0.5 * sqrt(dx * dx + dy * dy);
}

/* point inside or on the boundary of some obstacle (closed test) */
static int in_closed_obstacle(const oscene *s, int64_t px, int64_t py) {
  int parity = 0;
  for (int i = 0; i < s->nv; ++i) {
    int64_t ax = s->x[i], ay = s->y[i], bx = s->x[s->next[i]], by = s->y[s->next[i]];
    i128 c = (i128)(bx - ax) * (py - ay) - (i128)(by - ay) * (px - ax);
    if (c == 0 && px >= (ax < bx ? ax : bx) && px <= (ax > bx ? ax : bx) && py >= (ay < by ? ay : by) &&
        py <= (ay > by ? ay : by))
      return 1;
    if ((ay > py) != (by > py)) {
      if ((c > 0) == (by > ay)) parity ^= 1;
    }
  }
  return parity;
}

/* ------------------------------------------------------------------------ */
/* exported API                                                               */
/* ------------------------------------------------------------------------ */

int orc_num_generators(const orc_scene *in) {
  oscene s;
  load_oscene(in, &s);
  int G = s.G;
  free_oscene(&s);
  return G;
}

/* generator table: kind, ref (point / segment / vertex index), and the domain
 * coordinates x, y (and x2, y2 for segments) */
int orc_generators(const orc_scene *in, int *kind, int *ref, int *xy4) {
  oscene s;
  load_oscene(in, &s);
  for (int g = 0; g < s.G; ++g) {
    kind[g] = s.gkind[g];
    ref[g] = s.gref[g];
    int r = s.gref[g];
    int *o = xy4 + 4 * g;
    if (s.gkind[g] == ORC_POINT) { o[0] = (int)(s.px[r] / 2); o[1] = (int)(s.py[r] / 2); o[2] = o[0]; o[3] = o[1]; }
    else if (s.gkind[g] == ORC_SEGMENT) { o[0] = (int)(s.sax[r] / 2); o[1] = (int)(s.say[r] / 2); o[2] = (int)(s.sbx[r] / 2); o[3] = (int)(s.sby[r] / 2); }
    else { o[0] = (int)(s.x[r] / 2); o[1] = (int)(s.y[r] / 2); o[2] = o[0]; o[3] = o[1]; }
  }
  int G = s.G;
  free_oscene(&s);
  return G;
}

/* visibility of two rational points given in doubled coordinates (x/w, y/w) */
int orc_visible(const orc_scene *in, int64_t ax, int64_t ay, int64_t aw, int64_t bx, int64_t by, int64_t bw) {
  oscene s;
  load_oscene(in, &s);
  hpt a = {ax, ay, aw}, b = {bx, by, bw};
  int r = visible(&s, a, b);
  free_oscene(&s);
  return r;
}

/* the arc weight from generator u to the corner generator v, or -1 when the
 * arc does not exist (not visible, or u is not a source / corner) */
static double arc_weight(const oscene *s, int u, int v) {
  int iv = s->gref[v];
  hpt pv = hp(s->x[iv], s->y[iv]);
  if (s->gkind[u] == ORC_POINT) {
    int k = s->gref[u];
    if (!visible(s, hp(s->px[k], s->py[k]), pv)) return -1.0;
    return pt_dist(s->px[k], s->py[k], s->x[iv], s->y[iv]);
  }
  if (s->gkind[u] == ORC_SEGMENT) {
    double d;
    hpt q = seg_closest(s, s->gref[u], s->x[iv], s->y[iv], &d);
    if (!visible(s, pv, q)) return -1.0;
    return d;
  }
  int iu = s->gref[u];
  if (iu == iv) return -1.0;
  if (!visible(s, hp(s->x[iu], s->y[iu]), pv)) return -1.0;
  return pt_dist(s->x[iu], s->y[iu], s->x[iv], s->y[iv]);
}

/* Generator costs: multi-source Dijkstra on the generator visibility graph
 * (sources at cost 0; Procedure 1 picks the unexpanded entry of least cost,
 * Procedure 4 relaxes every visible entry).  cost[g] = +inf and gparent = -1
 * when unreachable; a source's parent is itself.  weights (optional, G*G)
 * receives the arc matrix with -1 for missing arcs.  Returns G. */
int orc_costs(const orc_scene *in, double *cost, int *gparent, double *weights, int nthreads) {
  oscene s;
  load_oscene(in, &s);
  int G = s.G;
  double *w = weights ? weights : (double *)malloc(sizeof(double) * (size_t)G * G);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int v = 0; v < G; ++v) {
    for (int u = 0; u < G; ++u) {
      double x = -1.0;
      if (s.gkind[v] == ORC_VERTEX && u != v) {
        if (s.gkind[u] == ORC_VERTEX && u > v) x = -2.0; /* filled from the mirror below */
        else x = arc_weight(&s, u, v);
      }
      w[(size_t)v * G + u] = x;
    }
  }
  for (int v = 0; v < G; ++v)
    for (int u = v + 1; u < G; ++u)
      if (w[(size_t)v * G + u] == -2.0) w[(size_t)v * G + u] = w[(size_t)u * G + v];
  char *done = (char *)calloc(G + 1, 1);
  for (int g = 0; g < G; ++g) {
    cost[g] = (s.gkind[g] == ORC_VERTEX) ? INFINITY : 0.0;
    gparent[g] = (s.gkind[g] == ORC_VERTEX) ? -1 : g;
  }
  for (;;) {
    int best = -1;
    for (int g = 0; g < G; ++g)
      if (!done[g] && isfinite(cost[g]) && (best < 0 || cost[g] < cost[best])) best = g;
    if (best < 0) break;
    done[best] = 1;
    for (int v = 0; v < G; ++v) {
      double x = w[(size_t)v * G + best];
      if (x < 0.0 || done[v]) continue;
      double c = cost[best] + x;
      if (c < cost[v]) cost[v] = c;
    }
  }
  /* parent: the visible predecessor attaining the cost, smallest id on ties */
  for (int v = 0; v < G; ++v) {
    if (s.gkind[v] != ORC_VERTEX || !isfinite(cost[v])) continue;
    int par = -1;
    for (int u = 0; u < G; ++u) {
      double x = w[(size_t)v * G + u];
      if (x < 0.0 || !isfinite(cost[u])) continue;
      if (cost[u] + x == cost[v]) { par = u; break; }
    }
    gparent[v] = par;
  }
  free(done);
  if (!weights) free(w);
  free_oscene(&s);
  return G;
}

typedef struct {
  double c, cost;
  int id;
} cand_t;

static int cand_cmp(const void *a, const void *b) {
  const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
  if (x->c != y->c) return x->c < y->c ? -1 : 1;
  if (x->cost != y->cost) return x->cost < y->cost ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

/* the point x_g(p) a pixel connects to, and its distance */
static hpt gen_point(const oscene *s, int g, int64_t px, int64_t py, double *d) {
  int r = s->gref[g];
  if (s->gkind[g] == ORC_POINT) { *d = pt_dist(px, py, s->px[r], s->py[r]); return hp(s->px[r], s->py[r]); }
  if (s->gkind[g] == ORC_SEGMENT) return seg_closest(s, r, px, py, d);
  *d = pt_dist(px, py, s->x[r], s->y[r]);
  return hp(s->x[r], s->y[r]);
}

/* Per-pixel map (Procedure 3 over all generators at once).  pix[k] is the
 * row-major pixel index j*W+i.  Outputs: dist32 (the double minimum rounded to
 * float), parent, dist64, and second (the least total over the OTHER visible
 * generators, +inf if none).  Pixels whose centre is inside or on an obstacle
 * get +inf / -1. */
int orc_pixels(const orc_scene *in, const double *cost, int n, const int64_t *pix, float *dist32, int *parent,
               double *dist64, double *second, int nthreads) {
  oscene s;
  load_oscene(in, &s);
  int G = s.G;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (G + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
    for (int k = 0; k < n; ++k) {
      int64_t i = pix[k] % s.W, j = pix[k] / s.W;
      int64_t px = 2 * i + 1, py = 2 * j + 1;
      double b1 = INFINITY, b2 = INFINITY;
      int par = -1;
      if (!in_closed_obstacle(&s, px, py)) {
        int nc = 0;
        for (int g = 0; g < G; ++g) {
          if (!isfinite(cost[g])) continue;
          double d;
          gen_point(&s, g, px, py, &d);
          cand[nc].c = cost[g] + d;
          cand[nc].cost = cost[g];
          cand[nc].id = g;
          ++nc;
        }
        qsort(cand, nc, sizeof(cand_t), cand_cmp);
        int found = 0;
        for (int t = 0; t < nc && found < 2; ++t) {
          double d;
          hpt q = gen_point(&s, cand[t].id, px, py, &d);
          if (!visible(&s, hp(px, py), q)) continue;
          if (found == 0) { b1 = cand[t].c; par = cand[t].id; }
          else b2 = cand[t].c;
          ++found;
        }
      }
      dist64[k] = b1;
      dist32[k] = (float)b1;
      parent[k] = par;
      second[k] = b2;
    }
    free(cand);
  }
  free_oscene(&s);
  return ORC_OK;
}

/* The value one generator offers one pixel (Procedure 3's cone, Section 4's
 * segment distance): cost(g) + |p - x_g(p)| when g has a finite cost and the
 * pixel centre sees x_g(p), +inf otherwise (also for a centre in or on an
 * obstacle).  Pair k is (pix[k], gen[k]).  Used to check that a map's parent
 * at a near-tie pixel is one of the valid choices. */
int orc_candidates(const orc_scene *in, const double *cost, int n, const int64_t *pix, const int *gen,
                   double *value, int nthreads) {
  oscene s;
  load_oscene(in, &s);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int k = 0; k < n; ++k) {
    int64_t i = pix[k] % s.W, j = pix[k] / s.W;
    int64_t px = 2 * i + 1, py = 2 * j + 1;
    int g = gen[k];
    double v = INFINITY;
    if (g >= 0 && g < s.G && isfinite(cost[g]) && !in_closed_obstacle(&s, px, py)) {
      double d;
      hpt q = gen_point(&s, g, px, py, &d);
      if (visible(&s, hp(px, py), q)) v = cost[g] + d;
    }
    value[k] = v;
  }
  free_oscene(&s);
  return ORC_OK;
}

/* closed inside-obstacle mask for the listed pixels */
int orc_inside(const orc_scene *in, int n, const int64_t *pix, unsigned char *inside) {
  oscene s;
  load_oscene(in, &s);
  for (int k = 0; k < n; ++k) {
    int64_t i = pix[k] % s.W, j = pix[k] / s.W;
    inside[k] = (unsigned char)in_closed_obstacle(&s, 2 * i + 1, 2 * j + 1);
  }
  free_oscene(&s);
  return ORC_OK;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Map value at rational points (Section 5.1, Discussion: the exact first turn of a query
 * point, not its pixel's).  Query k is (qxy[2k] / qw, qxy[2k+1] / qw) in
 * doubled coordinates.  Same rule as orc_pixels, over every generator:
 * dist64 / parent / second; a point in or on an obstacle, or outside the
 * domain, gets +inf / -1. */
static int in_closed_rational(const oscene *s, i128 X, i128 Y, i128 w) {
  int parity = 0;
  for (int i = 0; i < s->nv; ++i) {
    i128 ax = s->x[i] * w, ay = s->y[i] * w, bx = s->x[s->next[i]] * w, by = s->y[s->next[i]] * w;
    i128 c = (bx - ax) * (Y - ay) - (by - ay) * (X - ax);
    if (c == 0 && X >= (ax < bx ? ax : bx) && X <= (ax > bx ? ax : bx) && Y >= (ay < by ? ay : by) &&
        Y <= (ay > by ? ay : by))
      return 1;
    if ((ay > Y) != (by > Y)) {
      if ((c > 0) == (by > ay)) parity ^= 1;
    }
  }
  return parity;
}

/* x_g(q) for a rational q and its distance in domain units */
static hpt gen_point_rational(const oscene *s, int g, int64_t X, int64_t Y, int64_t w, double *d) {
  int r = s->gref[g];
  int64_t gx, gy;
  if (s->gkind[g] == ORC_SEGMENT) {
    int64_t ax = s->sax[r], ay = s->say[r], ex = s->sbx[r] - ax, ey = s->sby[r] - ay;
    int64_t L = ex * ex + ey * ey;
    i128 num = (i128)(X - ax * w) * ex + (i128)(Y - ay * w) * ey; /* (q - A).e * w */
    if (num > 0 && num < (i128)L * w) {
      i128 cr = (i128)ex * (Y - ay * w) - (i128)ey * (X - ax * w);
      *d = 0.5 * fabs((double)cr) / ((double)w * sqrt((double)L));
      hpt q = {(i128)ax * w * L + num * ex, (i128)ay * w * L + num * ey, (i128)w * L};
      return q;
    }
    gx = num <= 0 ? ax : s->sbx[r];
    gy = num <= 0 ? ay : s->sby[r];
  } else if (s->gkind[g] == ORC_POINT) {
    gx = s->px[r];
    gy = s->py[r];
  } else {
    gx = s->x[r];
    gy = s->y[r];
  }
  double dx = (double)(X - gx * w) / (double)w, dy = (double)(Y - gy * w) / (double)w;
  *d = 0.5 * sqrt(dx * dx + dy * dy);
  return hp(gx, gy);
}

int orc_points(const orc_scene *in, const double *cost, int n, const int64_t *qxy, int64_t qw, double *dist64,
               int *parent, double *second, int nthreads) {
  oscene s;
  load_oscene(in, &s);
  int G = s.G;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (G + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
    for (int k = 0; k < n; ++k) {
      int64_t X = qxy[2 * k], Y = qxy[2 * k + 1];
      double b1 = INFINITY, b2 = INFINITY;
      int par = -1;
      int outside = X < 0 || Y < 0 || X > 2 * (int64_t)s.W * qw || Y > 2 * (int64_t)s.H * qw;
      if (!outside && !in_closed_rational(&s, X, Y, qw)) {
        int nc = 0;
        for (int g = 0; g < G; ++g) {
          if (!isfinite(cost[g])) continue;
          double d;
          gen_point_rational(&s, g, X, Y, qw, &d);
          cand[nc].c = cost[g] + d;
          cand[nc].cost = cost[g];
          cand[nc].id = g;
          ++nc;
        }
        qsort(cand, nc, sizeof(cand_t), cand_cmp);
        int found = 0;
        hpt q = {X, Y, qw};
        for (int t = 0; t < nc && found < 2; ++t) {
          double d;
          hpt tg = gen_point_rational(&s, cand[t].id, X, Y, qw, &d);
          if (!visible(&s, q, tg)) continue;
          if (found == 0) { b1 = cand[t].c; par = cand[t].id; }
          else b2 = cand[t].c;
          ++found;
        }
      }
      dist64[k] = b1;
      parent[k] = par;
      second[k] = b2;
    }
    free(cand);
  }
  free_oscene(&s);
  return ORC_OK;
}
