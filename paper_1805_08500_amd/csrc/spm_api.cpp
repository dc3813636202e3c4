// spm_api.cpp -- the C ABI of libspm (declared in include/spm.h).
//
// Host responsibilities only: argument checks, exact scene validation,
// workspace layout, stage timing and kernel queueing.  Every step of the map
// computation runs in the HIP kernels of k_ingest.hip, k_graph.hip and
// k_pixel.hip; spm_query_path walks a host copy of a built map.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "spm_internal.hpp"

using namespace spm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return SPM_OK;
}

int check_counts(const spm_scene* s) {
  if (!s) return fail(SPM_ERR_INVALID_ARG, "scene is NULL");
  if (s->width < 1 || s->height < 1 || s->width > SPM_MAX_SIDE || s->height > SPM_MAX_SIDE)
    return fail(SPM_ERR_RANGE, "width/height %d x %d outside [1, %d]", s->width, s->height, SPM_MAX_SIDE);
  if (s->n_polys < 0 || s->n_vertices < 0 || s->n_points < 0 || s->n_segs < 0)
    return fail(SPM_ERR_INVALID_ARG, "negative count");
  if (s->n_polys == 0 && s->n_vertices != 0) return fail(SPM_ERR_INVALID_ARG, "vertices without polygons");
  if (s->n_polys > 0 && s->n_vertices < 3 * s->n_polys)
    return fail(SPM_ERR_INVALID_ARG, "fewer than 3 vertices per polygon");
  if ((long long)s->n_points + s->n_segs + s->n_vertices > (1ll << 30))
    return fail(SPM_ERR_INVALID_ARG, "too many generators");
  if (s->n_points + s->n_segs == 0) return fail(SPM_ERR_INVALID_ARG, "no source");
  return SPM_OK;
}

int check_ptrs(const spm_scene* s) {
  if (s->n_polys > 0 && (!s->poly_start || !s->vx || !s->vy))
    return fail(SPM_ERR_INVALID_ARG, "polygon arrays are NULL");
  if (s->n_points > 0 && !s->pts) return fail(SPM_ERR_INVALID_ARG, "pts is NULL");
  if (s->n_segs > 0 && !s->segs) return fail(SPM_ERR_INVALID_ARG, "segs is NULL");
  return SPM_OK;
}

// ---------------------------------------------------------------- validation
typedef long long ll;

struct P2 {
  ll x, y;
};

inline ll cross(P2 o, P2 a, P2 b) { return (a.x - o.x) * (b.y - o.y) - (a.y - o.y) * (b.x - o.x); }
inline int sgn(ll v) { return (v > 0) - (v < 0); }

inline bool on_seg(P2 a, P2 b, P2 p) {  // p on closed segment [a,b], given collinear
  return std::min(a.x, b.x) <= p.x && p.x <= std::max(a.x, b.x) && std::min(a.y, b.y) <= p.y &&
         p.y <= std::max(a.y, b.y);
}

bool seg_meet(P2 a, P2 b, P2 c, P2 d) {  // closed segments share a point
  int d1 = sgn(cross(c, d, a)), d2 = sgn(cross(c, d, b)), d3 = sgn(cross(a, b, c)), d4 = sgn(cross(a, b, d));
  if (d1 * d2 < 0 && d3 * d4 < 0) return true;
  if (d1 == 0 && on_seg(c, d, a)) return true;
  if (d2 == 0 && on_seg(c, d, b)) return true;
  if (d3 == 0 && on_seg(a, b, c)) return true;
  if (d4 == 0 && on_seg(a, b, d)) return true;
  return false;
}

// p inside or on the boundary of polygon [a, b) of the vertex arrays
bool in_closed_poly(const int* vx, const int* vy, int a, int b, P2 p) {
  bool in = false;
  for (int i = a; i < b; ++i) {
    int k = (i + 1 < b) ? i + 1 : a;
    P2 u{vx[i], vy[i]}, v{vx[k], vy[k]};
    ll c = cross(u, v, p);
    if (c == 0 && on_seg(u, v, p)) return true;
    if ((u.y > p.y) != (v.y > p.y)) {
      if ((c > 0) == (v.y > u.y)) in = !in;
    }
  }
  return in;
}

struct Seg {
  P2 a, b;
  int poly, idx;  // idx: position within the polygon, -1 for a source segment
  ll x0, x1;
};

}  // namespace

extern "C" {

const char* spm_last_error(void) { return g_err.c_str(); }

int spm_validate(const spm_scene* s) {
  int rc = check_counts(s);
  if (rc) return rc;
  if ((rc = check_ptrs(s))) return rc;
  const int W = s->width, H = s->height;
  if (s->n_polys > 0) {
    if (s->poly_start[0] != 0) return fail(SPM_ERR_INVALID_ARG, "poly_start[0] != 0");
    for (int p = 0; p < s->n_polys; ++p)
      if (s->poly_start[p + 1] - s->poly_start[p] < 3)
        return fail(SPM_ERR_GEOMETRY, "polygon %d has fewer than 3 vertices", p);
    if (s->poly_start[s->n_polys] != s->n_vertices)
      return fail(SPM_ERR_INVALID_ARG, "poly_start[n_polys] != n_vertices");
  }
  for (int i = 0; i < s->n_vertices; ++i)
    if (s->vx[i] < 0 || s->vx[i] > W || s->vy[i] < 0 || s->vy[i] > H)
      return fail(SPM_ERR_RANGE, "vertex %d (%d,%d) outside the domain", i, s->vx[i], s->vy[i]);
  for (int i = 0; i < s->n_points; ++i)
    if (s->pts[2 * i] < 0 || s->pts[2 * i] > W || s->pts[2 * i + 1] < 0 || s->pts[2 * i + 1] > H)
      return fail(SPM_ERR_RANGE, "point source %d outside the domain", i);
  for (int i = 0; i < s->n_segs; ++i)
    for (int k = 0; k < 2; ++k)
      if (s->segs[4 * i + 2 * k] < 0 || s->segs[4 * i + 2 * k] > W || s->segs[4 * i + 2 * k + 1] < 0 ||
          s->segs[4 * i + 2 * k + 1] > H)
        return fail(SPM_ERR_RANGE, "segment source %d outside the domain", i);
  // per polygon: distinct consecutive vertices, no collinear triple, counter-clockwise
  for (int p = 0; p < s->n_polys; ++p) {
    const int a = s->poly_start[p], b = s->poly_start[p + 1];
    ll area2 = 0;
    for (int i = a; i < b; ++i) {
      const int ip = (i == a) ? b - 1 : i - 1, in = (i + 1 < b) ? i + 1 : a;
      P2 u{s->vx[ip], s->vy[ip]}, w{s->vx[i], s->vy[i]}, v{s->vx[in], s->vy[in]};
      if (w.x == v.x && w.y == v.y) return fail(SPM_ERR_GEOMETRY, "polygon %d repeats vertex %d", p, i - a);
      if (cross(u, w, v) == 0) return fail(SPM_ERR_GEOMETRY, "polygon %d: collinear corner at vertex %d", p, i - a);
      area2 += w.x * v.y - v.x * w.y;
    }
    if (area2 <= 0) return fail(SPM_ERR_GEOMETRY, "polygon %d is not counter-clockwise", p);
  }
  // all edges (obstacles and source segments), swept by min x
  std::vector<Seg> segs;
  segs.reserve((size_t)s->n_vertices + s->n_segs);
  for (int p = 0; p < s->n_polys; ++p) {
    const int a = s->poly_start[p], b = s->poly_start[p + 1];
    for (int i = a; i < b; ++i) {
      const int in = (i + 1 < b) ? i + 1 : a;
      Seg e{{s->vx[i], s->vy[i]}, {s->vx[in], s->vy[in]}, p, i - a, 0, 0};
      e.x0 = std::min(e.a.x, e.b.x);
      e.x1 = std::max(e.a.x, e.b.x);
      segs.push_back(e);
    }
  }
  for (int k = 0; k < s->n_segs; ++k) {
    Seg e{{s->segs[4 * k], s->segs[4 * k + 1]}, {s->segs[4 * k + 2], s->segs[4 * k + 3]}, -1 - k, -1, 0, 0};
    if (e.a.x == e.b.x && e.a.y == e.b.y) return fail(SPM_ERR_GEOMETRY, "segment source %d has zero length", k);
    e.x0 = std::min(e.a.x, e.b.x);
    e.x1 = std::max(e.a.x, e.b.x);
    segs.push_back(e);
  }
  std::vector<int> order(segs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return segs[x].x0 < segs[y].x0; });
  for (size_t oi = 0; oi < order.size(); ++oi) {
    const Seg& e = segs[order[oi]];
    for (size_t oj = oi + 1; oj < order.size(); ++oj) {
      const Seg& f = segs[order[oj]];
      if (f.x0 > e.x1) break;
      if (e.poly < 0 && f.poly < 0) continue;  // two sources may cross
      if (std::max(std::min(e.a.y, e.b.y), std::min(f.a.y, f.b.y)) >
          std::min(std::max(e.a.y, e.b.y), std::max(f.a.y, f.b.y)))
        continue;
      if (e.poly == f.poly && e.poly >= 0) {
        const int n = s->poly_start[e.poly + 1] - s->poly_start[e.poly];
        const int d = std::abs(e.idx - f.idx);
        if (d == 1 || d == n - 1) continue;  // neighbours share exactly one vertex (no collinear corner)
      }
      if (seg_meet(e.a, e.b, f.a, f.b)) {
        if (e.poly >= 0 && f.poly >= 0) {
          if (e.poly == f.poly) return fail(SPM_ERR_GEOMETRY, "polygon %d is not simple", e.poly);
          return fail(SPM_ERR_GEOMETRY, "obstacles %d and %d meet", e.poly, f.poly);
        }
        return fail(SPM_ERR_GEOMETRY, "segment source %d meets an obstacle", e.poly < 0 ? -1 - e.poly : -1 - f.poly);
      }
    }
  }
  // nesting between polygons (edges are disjoint, so test one vertex)
  for (int p = 0; p < s->n_polys; ++p) {
    const int a = s->poly_start[p], b = s->poly_start[p + 1];
    for (int q = 0; q < s->n_polys; ++q) {
      if (q == p) continue;
      const int c = s->poly_start[q], d = s->poly_start[q + 1];
      if (in_closed_poly(s->vx, s->vy, c, d, P2{s->vx[a], s->vy[a]}))
        return fail(SPM_ERR_GEOMETRY, "obstacle %d lies inside obstacle %d", p, q);
      (void)b;
    }
  }
  for (int k = 0; k < s->n_points; ++k) {
    P2 p{s->pts[2 * k], s->pts[2 * k + 1]};
    for (int q = 0; q < s->n_polys; ++q)
      if (in_closed_poly(s->vx, s->vy, s->poly_start[q], s->poly_start[q + 1], p))
        return fail(SPM_ERR_GEOMETRY, "point source %d is inside or on obstacle %d", k, q);
  }
  for (int k = 0; k < s->n_segs; ++k) {
    P2 p{s->segs[4 * k], s->segs[4 * k + 1]};
    for (int q = 0; q < s->n_polys; ++q)
      if (in_closed_poly(s->vx, s->vy, s->poly_start[q], s->poly_start[q + 1], p))
        return fail(SPM_ERR_GEOMETRY, "segment source %d is inside obstacle %d", k, q);
  }
  return ok();
}

int spm_query_sizes(const spm_scene* s, int32_t* max_gen, size_t* workspace_bytes) {
  int rc = check_counts(s);
  if (rc) return rc;
  Layout L = make_layout(s->width, s->height, s->n_polys, s->n_vertices, s->n_points, s->n_segs);
  if (max_gen) *max_gen = L.Gmax;
  if (workspace_bytes) *workspace_bytes = L.total;
  return ok();
}

// ---------------------------------------------------------------- timer
struct spm_timer {
  int cap = 0;
  int n = 0;
  std::vector<hipEvent_t> ev;  // cap * (SPM_N_STAGES) events: boundaries of the 7 stages + 1
};

int spm_timer_create(spm_timer** t) {
  if (!t) return fail(SPM_ERR_INVALID_ARG, "timer out pointer is NULL");
  spm_timer* x = new (std::nothrow) spm_timer();
  if (!x) return fail(SPM_ERR_INVALID_ARG, "out of host memory");
  x->cap = 256;
  x->ev.resize((size_t)x->cap * SPM_N_STAGES);
  for (auto& e : x->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      delete x;
      return fail(SPM_ERR_HIP, "hipEventCreate failed");
    }
  }
  *t = x;
  return ok();
}

int spm_timer_destroy(spm_timer* t) {
  if (!t) return ok();
  for (auto& e : t->ev) (void)hipEventDestroy(e);
  delete t;
  return ok();
}

int spm_timer_reset(spm_timer* t) {
  if (!t) return fail(SPM_ERR_INVALID_ARG, "timer is NULL");
  t->n = 0;
  return ok();
}

int spm_timer_elapsed(spm_timer* t, float* ms, int32_t* n_builds) {
  if (!t || !ms) return fail(SPM_ERR_INVALID_ARG, "timer or output is NULL");
  for (int k = 0; k < SPM_N_STAGES; ++k) ms[k] = 0.0f;
  const int n = std::min(t->n, t->cap);
  if (n_builds) *n_builds = n;
  if (n == 0) return ok();
  if (hipEventSynchronize(t->ev[(size_t)(n - 1) * SPM_N_STAGES + SPM_N_STAGES - 1]) != hipSuccess)
    return fail(SPM_ERR_HIP, "hipEventSynchronize failed");
  for (int b = 0; b < n; ++b) {
    hipEvent_t* e = &t->ev[(size_t)b * SPM_N_STAGES];
    for (int k = 0; k + 1 < SPM_N_STAGES; ++k) {
      float x = 0.0f;
      if (hipEventElapsedTime(&x, e[k], e[k + 1]) != hipSuccess) return fail(SPM_ERR_HIP, "hipEventElapsedTime failed");
      ms[k] += x;
    }
    float tot = 0.0f;
    if (hipEventElapsedTime(&tot, e[0], e[SPM_N_STAGES - 1]) != hipSuccess)
      return fail(SPM_ERR_HIP, "hipEventElapsedTime failed");
    ms[SPM_N_STAGES - 1] += tot;
  }
  return ok();
}

// ---------------------------------------------------------------- build
}  // extern "C"

namespace {

// Device view of one scene's build: inputs, its sub-workspace and outputs.
void fill_dev(Dev& d, const spm_scene* s, const spm_out* out, char* ws, const Layout& L, int tw, u64* stats) {
  d = Dev{};
  d.W = L.W; d.H = L.H; d.nv = L.nv; d.np = L.np; d.ns = L.ns; d.n_polys = s->n_polys;
  d.E = L.E; d.NC = L.NC; d.Gmax = L.Gmax; d.RW = L.RW; d.W32 = L.W32;
  d.poly_start = s->poly_start; d.vx = s->vx; d.vy = s->vy; d.pts = s->pts; d.segs = s->segs;
  d.edges_raw = (EdgeRec*)(ws + L.off_edges_raw);
  d.ext_raw = (EdgeExt*)(ws + L.off_ext_raw);
  d.keys = (u64*)(ws + L.off_keys);
  d.edges = (EdgeRec*)(ws + L.off_edges);
  d.ext = (EdgeExt*)(ws + L.off_ext);
  d.chunks = (int4*)(ws + L.off_chunks);
  d.convex = (int*)(ws + L.off_convex);
  d.gens = (GenRec*)(ws + L.off_gens);
  d.vis = (u64*)(ws + L.off_vis);
  d.sgen = (GenRec*)(ws + L.off_sgen);
  d.sgcost = (float*)(ws + L.off_sgcost);
  d.sgbb = (int4*)(ws + L.off_sgbb);
  d.inside = (unsigned*)(ws + L.off_inside);
  d.cost64 = (double*)(ws + L.off_cost64);
  d.gxy = (int4*)(ws + L.off_gxy);
  d.misc = (int*)(ws + L.off_misc);
  d.vsorted = (int*)(ws + L.off_vsorted);
  d.vtx2gid = (int*)(ws + L.off_vtx2gid);
  d.gorder = (int*)(ws + L.off_gorder);
  d.costpos = (u64*)(ws + L.off_costpos);
  d.rmask = (u64*)(ws + L.off_rmask);
  d.qctr = (int*)(ws + L.off_qctr);
  d.cmark = (int*)(ws + L.off_cmark);
  d.obins = (int*)(ws + L.off_obins);
  d.order = (int*)(ws + L.off_order);
  d.krank = (int*)(ws + L.off_krank);
  d.clk = (int2*)(ws + L.off_clk);
  d.clmb = (int4*)(ws + L.off_clmb);
  d.clbb = (int4*)(ws + L.off_clbb);
  d.clc = (float*)(ws + L.off_clc);
  d.ocap = L.ocap;
  d.dist = out->dist; d.parent = out->parent; d.gen_kind = out->gen_kind; d.gen_xy = out->gen_xy;
  d.gen_cost = out->gen_cost; d.gen_parent = out->gen_parent; d.n_gen = out->n_gen;
  d.tile_w = tw; d.tile_h = 64 / tw;
  d.strip = kDefaultStrip;
  d.samples = kDefaultSamples;
  d.walk = 0;
  // generator visibility: the narrowest wavefronts (smallest culling boxes) that keep the launch
  // within about two rounds of resident wavefronts
  d.gv_sub = 64;
  while (d.gv_sub > 16 && (long long)L.Gmax * L.RW * (64 / (d.gv_sub / 2)) <= 16384) d.gv_sub /= 2;
  // beyond a few wavefronts' worth of generators: every arc by itself, 64 edges per step
  if (L.Gmax >= SPM_GV_PAIR_MIN_GEN) d.gv_sub = 0;
  // up to kGvSpreadMaxGen generators each wavefront takes pairs from all over the triangle
  if (d.gv_sub == 0 && L.Gmax <= kGvSpreadMaxGen) d.gv_sub = -1;
  // beyond, row segments with an occluder cache: longer segments (fewer caches to fill) when the
  // graph gives wavefronts enough anyway (maze, 5632 generators: 512 columns 0.49 against 0.52 ms
  // with 256; the 20 x 20 grid, 1601: 128 columns 0.29 against 0.36 ms)
  if (d.gv_sub == 0 && SPM_GV_ROWS) d.gv_sub = -2;
  d.gv_seg = L.Gmax >= 4096 ? 512 : (L.Gmax >= 2048 ? 256 : 128);
  d.stats = stats;
}

void plan_add(Plan& p, const Dev& d) {
  for (int k = 0; k < STG_COUNT; ++k) p.total[k] += stage_count(d, k);
  p.maxGmax = std::max(p.maxGmax, d.Gmax);
  p.maxRW = std::max(p.maxRW, d.RW);
  p.maxW = std::max(p.maxW, d.W);
  p.maxE = std::max(p.maxE, d.E);
  p.maxNC = std::max(p.maxNC, d.NC);
  p.pixel_lds = std::max(p.pixel_lds, pixel_lds_bytes(d.Gmax, d.E, d.NC));
  p.genvis_lds = std::max(p.genvis_lds, (size_t)d.E * sizeof(EdgeRec) + (size_t)d.NC * 16);
}

int check_out(const spm_out* out) {
  if (!out || !out->dist || !out->parent || !out->gen_kind || !out->gen_xy || !out->gen_cost || !out->gen_parent ||
      !out->n_gen)
    return fail(SPM_ERR_INVALID_ARG, "an output pointer is NULL");
  return SPM_OK;
}

int check_tile(int tw, int th) {
  if (!((tw == 8 && th == 8) || (tw == 16 && th == 4) || (tw == 4 && th == 16)))
    return fail(SPM_ERR_INVALID_ARG, "unsupported tile %d x %d", tw, th);
  return SPM_OK;
}

const char* kStageNames[7] = {"ingest", "edge sort and inside mask", "generator order and chunk boxes",
                              "generator visibility", "relaxation", "generator sort and pixel tables", "pixel propagation"};

// queue the seven stages of a build for a scene source; marks timer events.
// prep() queues the pixel kernel's own tables after the generator sort (timed
// with it), pixel() the pixel kernel alone.
template <class S, class PrepFn, class PixelFn>
int run_stages(const S& src, const Plan& p, hipStream_t st, spm_timer* tm, PrepFn prep, PixelFn pixel) {
  hipEvent_t* ev = nullptr;
  if (tm && tm->n < tm->cap) ev = &tm->ev[(size_t)tm->n * SPM_N_STAGES];
  auto mark = [&](int k) -> int {
    if (ev && hipEventRecord(ev[k], st) != hipSuccess) return fail(SPM_ERR_HIP, "hipEventRecord failed");
    return SPM_OK;
  };
  int rc;
  if ((rc = mark(0))) return rc;
  for (int k = 0; k < 7; ++k) {
    hipError_t e = hipSuccess;
    switch (k) {
      case 0: e = launch_ingest(src, p, st); break;
      case 1: e = launch_edge_sort(src, p, st); break;
      case 2: e = launch_gorder(src, p, st); break;
      case 3: e = launch_genvis(src, p, st); break;
      case 4: e = launch_relax(src, p, st); break;
      case 5:
        e = launch_gsort(src, p, st);
        if (e == hipSuccess) e = prep();
        break;
      default: e = pixel(); break;
    }
    if (e != hipSuccess) return fail(SPM_ERR_HIP, "%s launch failed: %s", kStageNames[k], hipGetErrorString(e));
    if ((rc = mark(k + 1))) return rc;
  }
  if (ev) tm->n++;
  return SPM_OK;
}

// batch workspace: [counter][descriptor table][stage offsets][scene workspaces]
struct BatchLayout {
  size_t off_ctr, off_tab, off_offs, total;
  std::vector<size_t> off_scene;
  std::vector<Layout> L;
};

int batch_layout(const spm_batch* b, BatchLayout& B) {
  if (!b || b->n < 1 || !b->scenes || !b->outs) return fail(SPM_ERR_INVALID_ARG, "empty or NULL batch");
  if (b->pixel_waves < 0 || b->pixel_waves > 8)
    return fail(SPM_ERR_INVALID_ARG, "pixel_waves %d outside 0..8", b->pixel_waves);
  if (b->walk < 0 || b->walk > 3) return fail(SPM_ERR_INVALID_ARG, "batch walk %d outside 0..3", b->walk);
  const int n = b->n;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + (bytes ? bytes : 1), 256); return r; };
  B.off_ctr = take(256);
  B.off_tab = take((size_t)n * sizeof(Dev));
  B.off_offs = take((size_t)STG_COUNT * (n + 1) * sizeof(int));
  B.off_scene.resize(n);
  B.L.resize(n);
  for (int i = 0; i < n; ++i) {
    int rc = check_counts(&b->scenes[i]);
    if (rc) return fail(rc, "scene %d: %s", i, g_err.c_str());
    if ((rc = check_ptrs(&b->scenes[i]))) return fail(rc, "scene %d: %s", i, g_err.c_str());
    if ((rc = check_out(&b->outs[i]))) return fail(rc, "scene %d: %s", i, g_err.c_str());
    const int tw = b->tile_w ? b->tile_w[i] : 8;
    if ((rc = check_tile(tw, tw ? 64 / tw : 0))) return fail(rc, "scene %d: %s", i, g_err.c_str());
    const spm_scene* s = &b->scenes[i];
    B.L[i] = make_layout(s->width, s->height, s->n_polys, s->n_vertices, s->n_points, s->n_segs);
    B.off_scene[i] = take(B.L[i].total);
  }
  B.total = o;
  return SPM_OK;
}

int batch_devs(const spm_batch* b, const BatchLayout& B, char* ws, std::vector<Dev>& devs, Plan& p) {
  const int n = b->n;
  devs.resize(n);
  p = Plan{};
  for (int i = 0; i < n; ++i) {
    const int tw = b->tile_w ? b->tile_w[i] : 8;
    fill_dev(devs[i], &b->scenes[i], &b->outs[i], ws + B.off_scene[i], B.L[i], tw, nullptr);
  }
  // Pair visibility by rows with the occluders' shadows does the least work per pair, but one scene of a
  // few hundred generators gives it too few wavefronts; a batch whose scenes together give enough takes it
  // for every scene that would test pairs.
  long long row_waves = 0;
  for (int i = 0; i < n; ++i) {
    devs[i].gv_seg = kGvSeg;
    row_waves += rowseg_prefix(devs[i].Gmax, kGvSeg);
  }
  for (int i = 0; i < n; ++i) {
    if (SPM_GV_ROWS && row_waves >= kGvRowsBatchWaves && devs[i].gv_sub <= 0) devs[i].gv_sub = -2;
    plan_add(p, devs[i]);
  }
  p.pixel_waves = b->pixel_waves;
  p.walk = b->walk;
  if ((p.walk == 1 && p.maxGmax > 512) || (p.walk == 2 && p.maxGmax > 8192))
    return fail(SPM_ERR_INVALID_ARG, "batch walk %d needs at most %d generators per scene (a scene has up to %d)",
                p.walk, p.walk == 1 ? 512 : 8192, p.maxGmax);
  return SPM_OK;
}

}  // namespace

struct spm_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

int spm_build_ex(const spm_scene* s, const spm_out* out, void* d_ws, size_t ws_bytes, void* stream,
                 const spm_build_opts* opts) {
  int rc = check_counts(s);
  if (rc) return rc;
  if ((rc = check_ptrs(s))) return rc;
  if ((rc = check_out(out))) return rc;
  Layout L = make_layout(s->width, s->height, s->n_polys, s->n_vertices, s->n_points, s->n_segs);
  if (!d_ws) return fail(SPM_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < L.total) return fail(SPM_ERR_CAPACITY, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  int tw = 8;
  if (opts && opts->tile_w) {
    tw = opts->tile_w;
    if ((rc = check_tile(opts->tile_w, opts->tile_h))) return rc;
  }
  if (opts && (opts->strip < 0 || opts->strip > kMaxStrip))
    return fail(SPM_ERR_INVALID_ARG, "strip %d outside 0..%d", opts->strip, kMaxStrip);
  if (opts && opts->samples < -1)
    return fail(SPM_ERR_INVALID_ARG, "samples %d below -1", opts->samples);
  if (opts && (opts->walk < 0 || opts->walk > 4))
    return fail(SPM_ERR_INVALID_ARG, "walk %d outside 0..4", opts->walk);
  if (opts && ((opts->walk == 1 && L.Gmax > 512) || ((opts->walk == 2 || opts->walk == 4) && L.Gmax > 8192)))
    return fail(SPM_ERR_INVALID_ARG, "walk %d needs at most %d generators (scene has up to %d)", opts->walk,
                opts->walk == 1 ? 512 : 8192, L.Gmax);
  SingleSrc src;
  fill_dev(src.d, s, out, (char*)d_ws, L, tw, opts ? (u64*)opts->d_stats : nullptr);
  if (opts && opts->strip) src.d.strip = opts->strip;
  if (opts && opts->samples) src.d.samples = opts->samples < 0 ? 0 : opts->samples;
  if (opts) src.d.walk = opts->walk;
  Plan p{};
  plan_add(p, src.d);
  hipStream_t st = (hipStream_t)stream;
  const Dev& d = src.d;
  rc = run_stages(src, p, st, opts ? opts->timer : nullptr, [&]() { return launch_pixel(d, st, 0); },
                  [&]() { return launch_pixel(d, st, 1); });
  if (rc) return rc;
  return ok();
}

}  // extern "C"

namespace {

// Pinned host staging for spm_build: a ring of slots, each holding one scene until the
// copy queued from it has completed (its event), so a caller may free its host scene as
// soon as spm_build returns and consecutive builds need not wait for each other.
constexpr int kStageSlots = 4;
struct StageSlot {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  int dev = -1;
  bool pending = false;
};
std::mutex g_stage_mu;
StageSlot g_stage[kStageSlots];
unsigned g_stage_next = 0;

// pack the host scene into `dst` in the workspace's scene-block layout
void pack_scene(const spm_scene* s, const Layout& L, int* dst) {
  std::memset(dst, 0, L.scene_ints * sizeof(int));
  if (s->n_polys > 0) std::memcpy(dst + L.sc_poly, s->poly_start, ((size_t)s->n_polys + 1) * sizeof(int));
  if (s->n_vertices > 0) {
    std::memcpy(dst + L.sc_vx, s->vx, (size_t)s->n_vertices * sizeof(int));
    std::memcpy(dst + L.sc_vy, s->vy, (size_t)s->n_vertices * sizeof(int));
  }
  if (s->n_points > 0) std::memcpy(dst + L.sc_pts, s->pts, 2 * (size_t)s->n_points * sizeof(int));
  if (s->n_segs > 0) std::memcpy(dst + L.sc_segs, s->segs, 4 * (size_t)s->n_segs * sizeof(int));
}

// copy the packed scene through a pinned slot into the workspace, on `st`
int stage_scene(const spm_scene* s, const Layout& L, char* ws, hipStream_t st) {
  const size_t bytes = L.scene_ints * sizeof(int);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SPM_ERR_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(g_stage_mu);
  StageSlot& sl = g_stage[g_stage_next++ % kStageSlots];
  if (sl.pending) {
    if (hipEventSynchronize(sl.ev) != hipSuccess) return fail(SPM_ERR_HIP, "staging event wait failed");
    sl.pending = false;
  }
  if (sl.cap < bytes) {  // grows to the largest scene seen, then stays
    if (sl.host) (void)hipHostFree(sl.host);
    sl.host = nullptr;
    sl.cap = 0;
    const size_t cap = std::max(bytes, (size_t)1 << 16);
    if (hipHostMalloc(&sl.host, cap, hipHostMallocDefault) != hipSuccess || !sl.host)
      return fail(SPM_ERR_HIP, "pinned staging allocation of %zu bytes failed", cap);
    sl.cap = cap;
  }
  if (!sl.ev || sl.dev != dev) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    sl.ev = nullptr;
    if (hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess)
      return fail(SPM_ERR_HIP, "staging event creation failed");
    sl.dev = dev;
  }
  pack_scene(s, L, (int*)sl.host);
  if (hipMemcpyAsync(ws + L.off_scene, sl.host, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(SPM_ERR_HIP, "scene upload failed");
  if (hipEventRecord(sl.ev, st) != hipSuccess) return fail(SPM_ERR_HIP, "staging event record failed");
  sl.pending = true;
  return SPM_OK;
}

}  // namespace

extern "C" {

int spm_build(const spm_scene* s, const spm_out* out, void* d_ws, size_t ws_bytes, void* stream) {
  // every check that can fail runs before any device work is queued
  int rc = check_counts(s);
  if (rc) return rc;
  if ((rc = check_ptrs(s))) return rc;
  if ((rc = check_out(out))) return rc;
  Layout L = make_layout(s->width, s->height, s->n_polys, s->n_vertices, s->n_points, s->n_segs);
  if (!d_ws) return fail(SPM_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < L.total) return fail(SPM_ERR_CAPACITY, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  if ((rc = spm_validate(s))) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return fail(SPM_ERR_HIP, "hipStreamIsCapturing failed");
  if (cs != hipStreamCaptureStatusNone)
    return fail(SPM_ERR_INVALID_ARG, "spm_build stages a host scene and cannot be captured; capture spm_build_ex "
                                     "with a device scene instead");
  char* ws = (char*)d_ws;
  if ((rc = stage_scene(s, L, ws, st))) return rc;
  const int* sc = (const int*)(ws + L.off_scene);
  spm_scene dev = *s;
  dev.poly_start = sc + L.sc_poly;
  dev.vx = sc + L.sc_vx;
  dev.vy = sc + L.sc_vy;
  dev.pts = sc + L.sc_pts;
  dev.segs = sc + L.sc_segs;
  return spm_build_ex(&dev, out, d_ws, ws_bytes, stream, nullptr);
}

}  // extern "C"

namespace {

// Device scratch of spm_build_noalloc: one array per GPU, allocated with the
// code object and kept until the process ends.  Host code never uses the
// array's name as an address: each device's address comes from
// hipGetSymbolAddress with that device current, once, and is kept per device.
constexpr size_t kScratchBytes = (size_t)SPM_NOALLOC_MAX_WS;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SPM_ERR_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(SPM_ERR_HIP, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(SPM_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SPM_OK;
}

}  // namespace

extern "C" {

int spm_build_noalloc(const spm_scene* s, const spm_out* out, void* stream) {
  int rc = check_counts(s);
  if (rc) return rc;
  if ((rc = check_ptrs(s))) return rc;
  if ((rc = check_out(out))) return rc;
  const Layout L = make_layout(s->width, s->height, s->n_polys, s->n_vertices, s->n_points, s->n_segs);
  if (L.total > kScratchBytes)
    return fail(SPM_ERR_CAPACITY, "scene needs %zu bytes of workspace; spm_build_noalloc holds at most %zu",
                L.total, kScratchBytes);
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return spm_build_ex(s, out, ws, kScratchBytes, stream, nullptr);
}

int spm_batch_query_sizes(const spm_batch* b, size_t* workspace_bytes) {
  BatchLayout B;
  int rc = batch_layout(b, B);
  if (rc) return rc;
  if (workspace_bytes) *workspace_bytes = B.total;
  return ok();
}

int spm_batch_prepare(const spm_batch* b, void* d_ws, size_t ws_bytes) {
  BatchLayout B;
  int rc = batch_layout(b, B);
  if (rc) return rc;
  if (!d_ws) return fail(SPM_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < B.total) return fail(SPM_ERR_CAPACITY, "workspace has %zu bytes, needs %zu", ws_bytes, B.total);
  char* ws = (char*)d_ws;
  std::vector<Dev> devs;
  Plan p;
  if ((rc = batch_devs(b, B, ws, devs, p))) return rc;
  const int n = b->n;
  std::vector<int> offs((size_t)STG_COUNT * (n + 1), 0);
  for (int k = 0; k < STG_COUNT; ++k) {
    long long acc = 0;
    for (int i = 0; i < n; ++i) {
      offs[(size_t)k * (n + 1) + i] = (int)acc;
      acc += stage_count(devs[i], k);
    }
    if (acc > 0x7fffffffLL) return fail(SPM_ERR_CAPACITY, "batch too large for 32-bit work offsets");
    offs[(size_t)k * (n + 1) + n] = (int)acc;
  }
  if (hipMemcpy(ws + B.off_tab, devs.data(), (size_t)n * sizeof(Dev), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ws + B.off_offs, offs.data(), offs.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return fail(SPM_ERR_HIP, "descriptor upload failed");
  return ok();
}

int spm_build_batch(const spm_batch* b, void* d_ws, size_t ws_bytes, void* stream, spm_timer* timer) {
  BatchLayout B;
  int rc = batch_layout(b, B);
  if (rc) return rc;
  if (!d_ws) return fail(SPM_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < B.total) return fail(SPM_ERR_CAPACITY, "workspace has %zu bytes, needs %zu", ws_bytes, B.total);
  char* ws = (char*)d_ws;
  std::vector<Dev> devs;
  Plan p;
  if ((rc = batch_devs(b, B, ws, devs, p))) return rc;
  BatchSrc src{(const Dev*)(ws + B.off_tab), (const int*)(ws + B.off_offs), b->n};
  hipStream_t st = (hipStream_t)stream;
  int* ctr = (int*)(ws + B.off_ctr);
  rc = run_stages(src, p, st, timer, [&]() { return hipSuccess; },
                  [&]() { return launch_pixel_batch(src, p, ctr, st); });
  if (rc) return rc;
  return ok();
}

int spm_agent_query_ws(const spm_scene* s, int32_t n_agents, size_t* workspace_bytes) {
  int rc = check_counts(s);
  if (rc) return rc;
  if (n_agents < 0) return fail(SPM_ERR_INVALID_ARG, "negative agent count");
  if (workspace_bytes) *workspace_bytes = agent_ws_bytes(s->n_points + s->n_segs + s->n_vertices, n_agents);
  return ok();
}

int spm_agent_distance(const spm_scene* s, const spm_out* out, int32_t n_agents, const float* d_agents_xy,
                       float* d_dist, void* stream) {
  int rc = check_counts(s);
  if (rc) return rc;
  if ((rc = check_out(out))) return rc;
  if (n_agents < 0) return fail(SPM_ERR_INVALID_ARG, "negative agent count");
  if (n_agents > 0 && (!d_agents_xy || !d_dist)) return fail(SPM_ERR_INVALID_ARG, "agent arrays are NULL");
  hipError_t e = launch_agent_dist(s->width, s->height, n_agents, d_agents_xy, out, d_dist, (hipStream_t)stream);
  if (e != hipSuccess) return fail(SPM_ERR_HIP, "agent distance launch failed: %s", hipGetErrorString(e));
  return ok();
}

int spm_query_points(const spm_scene* s, const spm_out* out, int32_t n, const float* d_pts, float* d_dist,
                     int32_t* d_parent, int32_t cap, float* d_path_xy, int32_t* d_path_n, void* stream) {
  int rc = check_counts(s);
  if (rc) return rc;
  if ((rc = check_ptrs(s))) return rc;
  if ((rc = check_out(out))) return rc;
  if (n < 0) return fail(SPM_ERR_INVALID_ARG, "negative query count");
  if (n > 0 && (!d_pts || !d_dist || !d_parent)) return fail(SPM_ERR_INVALID_ARG, "query arrays are NULL");
  if (d_path_xy && (!d_path_n || cap < 1)) return fail(SPM_ERR_INVALID_ARG, "path output needs d_path_n and cap >= 1");
  hipError_t e = launch_query_points(s, out, n, d_pts, cap, d_dist, d_parent, d_path_xy, d_path_n,
                                     (hipStream_t)stream);
  if (e != hipSuccess) return fail(SPM_ERR_HIP, "query launch failed: %s", hipGetErrorString(e));
  return ok();
}

int spm_backward(const spm_scene* s, const spm_out* out, int32_t n_agents, const float* d_agents_xy,
                 const float* d_dL_dD, float* d_grad_pts, float* d_grad_segs, void* d_ws, size_t ws_bytes,
                 void* stream) {
  int rc = check_counts(s);
  if (rc) return rc;
  if ((rc = check_out(out))) return rc;
  if (n_agents < 0) return fail(SPM_ERR_INVALID_ARG, "negative agent count");
  if (n_agents > 0 && (!d_agents_xy || !d_dL_dD)) return fail(SPM_ERR_INVALID_ARG, "agent arrays are NULL");
  if ((s->n_points > 0 && !d_grad_pts) || (s->n_segs > 0 && !d_grad_segs))
    return fail(SPM_ERR_INVALID_ARG, "gradient arrays are NULL");
  const int Gmax = s->n_points + s->n_segs + s->n_vertices;
  const size_t need = agent_ws_bytes(Gmax, n_agents);
  if (!d_ws) return fail(SPM_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < need) return fail(SPM_ERR_CAPACITY, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  hipError_t e = launch_backward(s->width, s->height, Gmax, s->n_points, s->n_segs, n_agents, d_agents_xy, d_dL_dD,
                                 out, d_grad_pts, d_grad_segs, (char*)d_ws, (hipStream_t)stream);
  if (e != hipSuccess) return fail(SPM_ERR_HIP, "backward launch failed: %s", hipGetErrorString(e));
  return ok();
}

int spm_graph_capture_batch(const spm_batch* b, void* d_ws, size_t ws_bytes, void* stream, spm_graph** out) {
  if (!out) return fail(SPM_ERR_INVALID_ARG, "graph out pointer is NULL");
  if (!stream) return fail(SPM_ERR_INVALID_ARG, "capture needs a non-null stream");
  hipStream_t st = (hipStream_t)stream;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess)
    return fail(SPM_ERR_HIP, "hipStreamBeginCapture failed");
  const int rc = spm_build_batch(b, d_ws, ws_bytes, stream, nullptr);
  const std::string msg = g_err;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(rc, "%s", msg.c_str());
  }
  if (e != hipSuccess || !graph) return fail(SPM_ERR_HIP, "hipStreamEndCapture failed");
  spm_graph* g = new (std::nothrow) spm_graph();
  if (!g) {
    (void)hipGraphDestroy(graph);
    return fail(SPM_ERR_INVALID_ARG, "out of host memory");
  }
  g->graph = graph;
  if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete g;
    return fail(SPM_ERR_HIP, "hipGraphInstantiate failed");
  }
  *out = g;
  return ok();
}

int spm_graph_launch(spm_graph* g, void* stream) {
  if (!g || !g->exec) return fail(SPM_ERR_INVALID_ARG, "graph is NULL");
  if (hipGraphLaunch(g->exec, (hipStream_t)stream) != hipSuccess) return fail(SPM_ERR_HIP, "hipGraphLaunch failed");
  return ok();
}

int spm_graph_destroy(spm_graph* g) {
  if (!g) return ok();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return ok();
}

// ---------------------------------------------------------------- path query
int spm_query_path(const spm_map_host* m, float qx, float qy, float* out_xy, int32_t cap, int32_t* n_out,
                   float* out_len) {
  if (!m || !m->parent || !m->gen_kind || !m->gen_xy || !m->gen_parent || !out_xy || !n_out || !out_len)
    return fail(SPM_ERR_INVALID_ARG, "NULL argument");
  if (m->width < 1 || m->height < 1 || m->n_gen < 0) return fail(SPM_ERR_INVALID_ARG, "bad map sizes");
  if (!(qx >= 0.0f && qy >= 0.0f && qx <= (float)m->width && qy <= (float)m->height))
    return fail(SPM_ERR_RANGE, "query point outside the domain");
  if (cap < 2) return fail(SPM_ERR_CAPACITY, "capacity below 2");
  int i = std::min((int)std::floor(qx), m->width - 1), j = std::min((int)std::floor(qy), m->height - 1);
  int g = m->parent[(size_t)j * m->width + i];
  if (g < 0 || g >= m->n_gen) return fail(SPM_ERR_UNREACHABLE, "pixel (%d,%d) has no path", i, j);
  int n = 0;
  double len = 0.0, cx = qx, cy = qy;
  out_xy[2 * n] = qx;
  out_xy[2 * n + 1] = qy;
  ++n;
  int steps = 0;
  while (m->gen_kind[g] == SPM_GEN_VERTEX) {
    if (n >= cap) return fail(SPM_ERR_CAPACITY, "path longer than capacity %d", cap);
    const double x = m->gen_xy[4 * g], y = m->gen_xy[4 * g + 1];
    len += std::hypot(x - cx, y - cy);
    cx = x;
    cy = y;
    out_xy[2 * n] = (float)x;
    out_xy[2 * n + 1] = (float)y;
    ++n;
    const int nxt = m->gen_parent[g];
    if (nxt < 0 || nxt >= m->n_gen || ++steps > m->n_gen) return fail(SPM_ERR_UNREACHABLE, "broken parent chain");
    g = nxt;
  }
  if (n >= cap) return fail(SPM_ERR_CAPACITY, "path longer than capacity %d", cap);
  double ex, ey;
  if (m->gen_kind[g] == SPM_GEN_POINT) {
    ex = m->gen_xy[4 * g];
    ey = m->gen_xy[4 * g + 1];
  } else {
    // closest point of the segment source (Section 4: endpoint or projection)
    const double ax = m->gen_xy[4 * g], ay = m->gen_xy[4 * g + 1], bx = m->gen_xy[4 * g + 2],
                 by = m->gen_xy[4 * g + 3];
    const double dx = bx - ax, dy = by - ay;
    double t = ((cx - ax) * dx + (cy - ay) * dy) / (dx * dx + dy * dy);
    t = std::min(1.0, std::max(0.0, t));
    ex = ax + t * dx;
    ey = ay + t * dy;
  }
  len += std::hypot(ex - cx, ey - cy);
  out_xy[2 * n] = (float)ex;
  out_xy[2 * n + 1] = (float)ey;
  ++n;
  *n_out = n;
  *out_len = (float)len;
  return ok();
}

}  // extern "C"
