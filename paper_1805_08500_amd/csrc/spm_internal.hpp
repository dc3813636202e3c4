// spm_internal.hpp -- records, workspace layout and device helpers shared by
// the libspm kernels (HIP, gfx950).  Not part of the public ABI.
//
// Geometry is carried in "doubled" integer coordinates: every domain
// coordinate times 2, so the pixel centre (i + 1/2, j + 1/2) is the integer
// point (2i + 1, 2j + 1).  With W, H <= 8192 every doubled coordinate is at
// most 2^14, every coordinate difference fits in 15 signed bits, every
// orientation determinant of three lattice points fits in 30 bits, and the
// 24-bit integer multiply-add of the VALU is exact for all of them.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/spm.h"

namespace spm {

typedef unsigned long long u64;

constexpr int kWave = 64;
constexpr int kChunk = 64;        // edges per spatial chunk
constexpr int kRelaxThreads = 1024;
#ifndef SPM_RELAX_WIDE
#define SPM_RELAX_WIDE 6
#endif
constexpr int kRelaxWideRounds = SPM_RELAX_WIDE;   // Bellman-Ford rounds run chip-wide before the one-workgroup rounds
#ifndef SPM_RELAX_CHAOS
#define SPM_RELAX_CHAOS 16
#endif
constexpr int kRelaxChaos = SPM_RELAX_CHAOS;   // > 0: instead, that many rounds in one launch without barriers (small graphs)
#ifndef SPM_CHAOS_QUIET
#define SPM_CHAOS_QUIET 3
#endif
constexpr int kChaosQuiet = SPM_CHAOS_QUIET;   // the barrier-free rounds stop after that many passes without a lowering
#ifndef SPM_RELAX_CHAOS_MAX
#define SPM_RELAX_CHAOS_MAX 64
#endif
constexpr int kRelaxChaosMax = SPM_RELAX_CHAOS_MAX;   // their cap when they stop by themselves
#ifndef SPM_CHAOS_ADAPT_MIN_GEN
#define SPM_CHAOS_ADAPT_MIN_GEN 1024
#endif
constexpr int kChaosAdaptMinGen = SPM_CHAOS_ADAPT_MIN_GEN;   // above that many generators they do
constexpr int kChaosSlots = 8;     // progress marks, spread over cache lines to keep atomics apart
#ifndef SPM_RELAX_QUEUE
#define SPM_RELAX_QUEUE 1
#endif
constexpr int kRelaxQueue = SPM_RELAX_QUEUE;   // large graphs finish their relaxation on a work queue
#ifndef SPM_RELAX_QUEUE_SRC
#define SPM_RELAX_QUEUE_SRC 1
#endif
constexpr int kRelaxQueueSrc = SPM_RELAX_QUEUE_SRC;   // small graphs relax on the queue alone: 1 batches, 2 all
constexpr int kIngestFuseMax = 1024;   // scenes up to that many vertices ingest in the generator-table launch
constexpr int kDefaultStrip = 1;      // tiles per pixel-stage work item
constexpr int kDefaultSamples = 3;    // seed searches per pixel tile
constexpr int kMaxStrip = 64;
constexpr int kQueues = 8;         // pixel-stage work queues (one per XCD)
constexpr int kQueueStride = 32;   // ints between queue counters (one 128-byte line each)
constexpr int kOrderBins = 32;     // pixel-stage work classes (tiles ranked by a distance lower bound)
#ifndef SPM_CLUSTER
#define SPM_CLUSTER 16
#endif
constexpr int kCluster = SPM_CLUSTER;   // generators per spatial cluster of the pixel stage's cluster walk (8, 16 or 32)
#ifndef SPM_SEG_COLS
#define SPM_SEG_COLS 16
#endif
constexpr int kSegCols = SPM_SEG_COLS;   // corners per segment-column wavefront of generator visibility
#ifndef SPM_GV_PAIR_ROWS
#define SPM_GV_PAIR_ROWS 16
#endif
constexpr int kGvPairRows = SPM_GV_PAIR_ROWS;   // generator visibility by pairs: rows (and columns) per triangle block
#ifndef SPM_GV_PAIR_MIN_GEN
#define SPM_GV_PAIR_MIN_GEN 128    // generator visibility by pairs from this many generators on
#endif
#ifndef SPM_GV_SPREAD_MAX_GEN
#define SPM_GV_SPREAD_MAX_GEN 1024
#endif
constexpr int kGvSpreadMaxGen = SPM_GV_SPREAD_MAX_GEN;   // pairs dealt round-robin over the triangle up to this many generators
#ifndef SPM_GV_ROWS
#define SPM_GV_ROWS 1
#endif
constexpr long long kGvRowsBatchWaves = 4096;   // a batch uses the row mode when it would give the batch this many wavefronts
constexpr int kGvSeg = 512;   // beyond: one wavefront per (row, gv_seg columns) with an occluder cache; the
                              // batches' segment length (config 4: 1.25-1.27 ms against 1.29 with 256, 1.37
                              // with 128)

// Generator visibility by row segments of L columns: row r holds the pairs
// (r, u < r) in ceil(r / L) items; the items of rows 0 .. N-1 number
// sum_{r < N} ceil(r / L) = L q (q + 1) / 2 + (q + 1) (N - 1 - q L), q = (N - 1) / L.
__host__ __device__ inline long long rowseg_prefix(long long N, long long L) {
  if (N <= 1) return 0;
  const long long q = (N - 1) / L;
  return L * q * (q + 1) / 2 + (q + 1) * (N - 1 - q * L);
}

// One obstacle edge w -> v (obstacle on the left), with its line function
// E(x, y) = a x + b y + c, positive on the obstacle side.
struct EdgeRec {
  int wx, wy, vx, vy;
  int a, b, c, nc;  // nc = -c
};
// Neighbours needed by the vertex rule: prev(w) and next(v).
struct EdgeExt {
  int ux, uy, nx, ny;
};

// Generator record (canonical order and cost-sorted order share the layout).
struct GenRec {
  int kind, id;       // SPM_GEN_*; canonical id
  int x, y;           // point / segment A / vertex (doubled)
  int x2, y2;         // segment B (doubled); else = x, y
  int ux, uy;         // VERTEX: previous vertex (doubled)
  int nx, ny;         // VERTEX: next vertex (doubled)
  float costf;        // cost rounded to float (sorted table only)
  int vtx;            // VERTEX: input vertex index; else -1
  int pad0, pad1, pad2, pad3;
};
static_assert(sizeof(GenRec) == 64, "GenRec must be 64 bytes");

// misc ints in the workspace
enum { MISC_G = 0, MISC_REACHED = 1, MISC_ROUNDS = 2, MISC_TILE_CTR = 3, MISC_N = 16 };

__host__ __device__ inline int tiles_of(int W, int H, int tw) {
  const int th = 64 / tw;
  return ((W + tw - 1) / tw) * ((H + th - 1) / th);
}

struct Layout {
  int W, H, nv, np, ns, np_polys;
  int E, NC, Gmax, RW, W32;
  size_t off_edges_raw, off_ext_raw, off_keys, off_edges, off_ext, off_chunks, off_convex;
  size_t off_gens, off_vis, off_sgen, off_sgcost, off_sgbb, off_inside, off_cost64, off_gxy, off_misc;
  size_t off_vsorted, off_vtx2gid, off_gorder, off_costpos, off_qctr, off_rmask, off_cmark;
  size_t off_obins, off_order;
  size_t off_krank, off_clk, off_clmb, off_clbb, off_clc;   // generator clusters of the pixel stage
  // a host scene staged into the workspace (spm_build): poly_start, vx, vy, pts, segs, each at
  // a 16-int boundary from off_scene
  size_t off_scene, scene_ints, sc_poly, sc_vx, sc_vy, sc_pts, sc_segs;
  int ocap;   // capacity of each work class (the most tiles any tile shape gives)
  size_t total;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline Layout make_layout(int W, int H, int n_polys, int nv, int np, int ns) {
  Layout L{};
  L.W = W; L.H = H; L.nv = nv; L.np = np; L.ns = ns; L.np_polys = n_polys;
  L.E = nv;
  L.NC = (nv + kChunk - 1) / kChunk;
  L.Gmax = np + ns + nv;
  L.RW = (L.Gmax + 63) / 64;
  L.W32 = (W + 31) / 32;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + (bytes ? bytes : 1), 256); return r; };
  size_t E1 = (size_t)(L.E > 0 ? L.E : 1);
  size_t G1 = (size_t)(L.Gmax > 0 ? L.Gmax : 1);
  L.off_edges_raw = take(E1 * sizeof(EdgeRec));
  L.off_ext_raw = take(E1 * sizeof(EdgeExt));
  L.off_keys = take(E1 * sizeof(u64));
  L.off_edges = take(E1 * sizeof(EdgeRec));
  L.off_ext = take(E1 * sizeof(EdgeExt));
  L.off_chunks = take((size_t)(L.NC > 0 ? L.NC : 1) * 16);
  L.off_convex = take(E1 * sizeof(int));
  L.off_gens = take(G1 * sizeof(GenRec));
  L.off_vis = take(G1 * (size_t)(L.RW > 0 ? L.RW : 1) * sizeof(u64));
  L.off_sgen = take(G1 * sizeof(GenRec));
  L.off_sgcost = take(G1 * sizeof(float));
  L.off_sgbb = take(G1 * 16);
  L.off_inside = take((size_t)H * L.W32 * sizeof(unsigned));
  L.off_cost64 = take(G1 * sizeof(double));
  L.off_gxy = take(G1 * 16);
  L.off_misc = take(MISC_N * sizeof(int));
  L.off_vsorted = take(E1 * sizeof(int));
  L.off_vtx2gid = take(E1 * sizeof(int));
  L.off_gorder = take(G1 * sizeof(int));
  L.off_costpos = take(G1 * sizeof(u64));
  L.off_qctr = take(kQueues * kQueueStride * sizeof(int));
  L.off_cmark = take(kChaosSlots * kQueueStride * sizeof(int));
  L.off_rmask = take(3 * (size_t)(L.RW > 0 ? L.RW : 1) * sizeof(u64));
  L.ocap = tiles_of(W, H, 4);
  if (tiles_of(W, H, 8) > L.ocap) L.ocap = tiles_of(W, H, 8);
  if (tiles_of(W, H, 16) > L.ocap) L.ocap = tiles_of(W, H, 16);
  L.off_obins = take(kOrderBins * sizeof(int));
  L.off_order = take((size_t)kOrderBins * (size_t)(L.ocap > 0 ? L.ocap : 1) * sizeof(int));
  const size_t ncl = (G1 + kCluster - 1) / kCluster;
  L.off_krank = take(G1 * sizeof(int));
  L.off_clk = take(ncl * kCluster * 2 * sizeof(int));
  L.off_clmb = take(ncl * kCluster * 16);
  L.off_clbb = take(ncl * 16);
  L.off_clc = take(ncl * sizeof(float));
  size_t si = 0;
  auto part = [&](size_t ints) { size_t r = si; si = align_up(si + ints, 16); return r; };
  L.sc_poly = part((size_t)n_polys + 1);
  L.sc_vx = part((size_t)nv);
  L.sc_vy = part((size_t)nv);
  L.sc_pts = part(2 * (size_t)np);
  L.sc_segs = part(4 * (size_t)ns);
  L.scene_ints = si;
  L.off_scene = take(si * sizeof(int));
  L.total = o;
  return L;
}

// Device view of one build's workspace and outputs.
struct Dev {
  int W, H, nv, np, ns, n_polys;
  int E, NC, Gmax, RW, W32;
  // inputs (device)
  const int* poly_start;
  const int* vx;
  const int* vy;
  const int* pts;
  const int* segs;
  // workspace
  EdgeRec* edges_raw;
  EdgeExt* ext_raw;
  u64* keys;
  EdgeRec* edges;
  EdgeExt* ext;
  int4* chunks;
  int* convex;
  GenRec* gens;
  u64* vis;
  GenRec* sgen;
  float* sgcost;
  int4* sgbb;
  unsigned* inside;
  double* cost64;
  int4* gxy;
  int* misc;
  int* vsorted;   // vertex index at each Morton-sorted edge position
  int* vtx2gid;   // generator id of each convex vertex
  int* gorder;    // generator id at each spatial position (sources first)
  u64* costpos;   // relaxation costs by spatial position (IEEE bits) when they do not fit in LDS
  u64* rmask;     // wide relaxation rounds: three rotating change masks of RW words
  int* qctr;      // pixel-stage queue counters, kQueues of them kQueueStride ints apart
  int* cmark;     // the barrier-free rounds' progress marks, kChaosSlots of them kQueueStride ints apart
  int* obins;     // pixel-stage work classes: item count of each (kOrderBins)
  int* order;     // work items of class c at order[c * ocap ...], in no particular order within it
  int* krank;     // canonical generator g: its position in the cost-sorted table, -1 when unreached
  int2* clk;      // cluster c: (sorted position, float cost bits) of its kCluster members (position -1:
                  // none), in spatial order
  int4* clmb;     // cluster c: its members' boxes (same order)
  int4* clbb;     // cluster c: bounding box of its members
  float* clc;     // cluster c: least float cost of its members (+inf: none)
  int ocap;
  // outputs
  float* dist;
  int* parent;
  int* gen_kind;
  int* gen_xy;
  double* gen_cost;
  int* gen_parent;
  int* n_gen;
  // options
  int tile_w, tile_h;
  int strip;       // pixel stage: tiles per wavefront work item (>= 1)
  int samples;     // pixel stage: seed searches per tile (>= 0)
  int walk;        // pixel stage: 0 by generator count, else 1 + the walk (cached, refilled, cost order)
  int gv_sub;      // generator visibility: columns per wavefront (64, 32 or 16); 0: one pair at a time,
                   // lanes over edges (kGvPairRows x kGvPairRows blocks of the lower triangle);
                   // -1: the same pairs dealt round-robin over the triangle; -2: row segments of
                   // gv_seg pairs with an occluder cache
  int gv_seg;      // row segment length (128, 256 or 512)
  u64* stats;
};

// Read-only geometry view handed to the device helpers.  Kernels build it from
// __restrict__ arguments so the compiler may serve uniform reads from the
// scalar cache.
struct Geo {
  const EdgeRec* edges;
  const EdgeExt* ext;
  const int4* chunks;
  int E, NC;
#ifdef __HIPCC__
  __device__ __forceinline__ EdgeRec edge(int e) const { return edges[e]; }
  __device__ __forceinline__ int4 chunk(int c) const { return chunks[c]; }
#endif
};

// ------------------------------------------------------------------------
// Work decomposition.  Every stage kernel runs over "items" of one kind; a
// build of one scene and a batch of scenes use the same kernels, with the
// scene of an item found from per-stage prefix offsets in the batch case.
// ------------------------------------------------------------------------
enum StageKind {
  STG_VTX = 0,   // one thread per obstacle vertex
  STG_SCENE,     // one workgroup per scene
  STG_EDGE,      // one wavefront per edge
  STG_CHUNK,     // one thread per edge chunk
  STG_ROW,       // one wavefront per pixel row
  STG_GVBLK,     // one 4-wavefront workgroup per 4 (row, gv_sub columns) generator-visibility items
  STG_GEN,       // one wavefront per generator slot
  STG_SLICE,     // one pixel-tile slice (batched pixel stage)
  STG_SEGVIS,    // one wavefront per (segment source, kSegCols corner positions)
  STG_RELAXW,    // one thread per (corner row, byte of a 64-bit word) of the visibility matrix
  STG_COUNT
};
constexpr int kSlice = 64;   // tiles per work item of the batched pixel stage

__host__ __device__ inline int stage_count(const Dev& d, int stage) {
  switch (stage) {
    case STG_VTX: return d.nv;
    case STG_SCENE: return 1;
    case STG_EDGE: return d.E;
    case STG_CHUNK: return d.NC;
    case STG_ROW: return d.H;
    case STG_GVBLK: {
      if (d.gv_sub == -2) return (int)((rowseg_prefix(d.Gmax, d.gv_seg) + 3) / 4);
      if (d.gv_sub <= 0) {
        const long long B = (d.Gmax + kGvPairRows - 1) / kGvPairRows;
        return (int)((kGvPairRows * (B * (B + 1) / 2) + 3) / 4);
      }
      return (int)(((long long)d.Gmax * d.RW * (64 / d.gv_sub) + 3) / 4);
    }
    case STG_GEN: return d.Gmax;
    case STG_SLICE: return (tiles_of(d.W, d.H, d.tile_w) + kSlice - 1) / kSlice;
    case STG_SEGVIS: return d.ns * ((d.Gmax - d.np - d.ns + kSegCols - 1) / kSegCols);
    case STG_RELAXW: return (d.Gmax - d.np - d.ns) * d.RW * 8;
    default: return 0;
  }
}

// One scene, carried by value in the kernel arguments.
struct SingleSrc {
  Dev d;
  __device__ __forceinline__ bool locate(int stage, int idx, int& s, int& local) const {
    s = 0;
    local = idx;
    return idx < stage_count(d, stage);
  }
  __device__ __forceinline__ const Dev& scene(int) const { return d; }
};

// A batch: per-scene descriptors and per-stage prefix offsets in device memory
// (offs[stage * (n + 1) + s] = first item of scene s).
struct BatchSrc {
  const Dev* tab;
  const int* offs;
  int n;
  __device__ __forceinline__ bool locate(int stage, int idx, int& s, int& local) const {
    const int* o = offs + stage * (n + 1);
    if (idx < 0 || idx >= o[n]) return false;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (o[mid] <= idx) lo = mid;
      else hi = mid - 1;
    }
    s = lo;
    local = idx - o[lo];
    return true;
  }
  __device__ __forceinline__ const Dev& scene(int s) const { return tab[s]; }
};

// Host-side totals of a build (single scene or batch): items per stage and
// the largest per-scene sizes that set LDS allocations.
struct Plan {
  long long total[STG_COUNT];
  int maxGmax, maxRW, maxW, maxE, maxNC;
  size_t pixel_lds, genvis_lds;
  int pixel_waves;   // batched pixel stage: waves per SIMD asked for (0 = as many as fit)
  int walk;          // batched pixel stage: forced walk (0 = by the largest generator count)
};

// host launchers (each queues kernels on the stream and returns hipError_t)
template <class S> hipError_t launch_ingest(const S& src, const Plan& p, hipStream_t s);
template <class S> hipError_t launch_edge_sort(const S& src, const Plan& p, hipStream_t s);

template <class S> hipError_t launch_gorder(const S& src, const Plan& p, hipStream_t s);
template <class S> hipError_t launch_genvis(const S& src, const Plan& p, hipStream_t s);
template <class S> hipError_t launch_relax(const S& src, const Plan& p, hipStream_t s);
template <class S> hipError_t launch_gsort(const S& src, const Plan& p, hipStream_t s);
// phase 0: the pixel kernel's own tables (clusters, a separate work order); phase 1: the pixel kernel
hipError_t launch_pixel(const Dev& d, hipStream_t s, int phase);
hipError_t launch_pixel_batch(const BatchSrc& b, const Plan& p, int* batch_ctr, hipStream_t s);
size_t pixel_lds_bytes(int Gmax, int E, int NC);
size_t agent_ws_bytes(int Gmax, int n_agents);
hipError_t launch_agent_dist(int W, int H, int n, const float* agents, const spm_out* out, float* d_out,
                             hipStream_t s);
hipError_t launch_query_points(const spm_scene* s, const spm_out* out, int n, const float* pts, int cap, float* dist,
                               int* par, float* path_xy, int* path_n, hipStream_t st);
hipError_t launch_backward(int W, int H, int Gmax, int np, int ns, int n, const float* agents, const float* dLdD,
                           const spm_out* out, float* grad_pts, float* grad_segs, char* ws, hipStream_t s);

#ifdef __HIPCC__
// ------------------------------------------------------------------------
// device helpers
// ------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ u64 ballot(bool p) { return (u64)__ballot(p); }
__device__ __forceinline__ int first_bit(u64 m) { return __builtin_ctzll(m); }
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Minimum of an unsigned value over the wavefront, in every lane: DPP steps
// within each row of 16 lanes (quad exchanges, then rotations by 4 and 8),
// then the four row minima on the scalar unit.
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x124, 0xF, 0xF, false));  // row_ror 4
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x128, 0xF, 0xF, false));  // row_ror 8
  // every lane of a row now holds the row's least: fold rows 0 -> 1, 2 -> 3, then 1 -> 3
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast 15
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast 31
  return (unsigned)readlane((int)v, 63);
}
__device__ __forceinline__ float unif(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ int mul24(int a, int b) { return __mul24(a, b); }
__device__ __forceinline__ int mad24(int a, int b, int c) { return __mul24(a, b) + c; }
__device__ __forceinline__ int sgn3(int x) { return min(max(x, -1), 1); }
// 16-bit halves packed in one register (doubled coordinates and coefficients below 2^15)
__device__ __forceinline__ int pack16(int lo, int hi) { return (int)(((unsigned)lo & 0xffffu) | ((unsigned)hi << 16)); }
__device__ __forceinline__ int lo16(int x) { return (int)(short)(x & 0xffff); }
__device__ __forceinline__ int hi16(int x) { return x >> 16; }
// lo16(a) lo16(b) + hi16(a) hi16(b) + c in one instruction (v_dot2_i32_i16).
// The products are exact and the sum wraps modulo 2^32, so the result is the
// exact value whenever that fits an int32.
typedef short spm_short2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int dot2(int a, int b, int c) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(spm_short2, a), __builtin_bit_cast(spm_short2, b), c, false);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// Direction (dx, dy) leaving corner w strictly into the obstacle's interior
// angle; u = previous and n = next vertex of w (counter-clockwise loop).
__device__ __forceinline__ bool into_interior(int ux, int uy, int wx, int wy, int nx, int ny, int dx, int dy) {
  int turn = (wx - ux) * (ny - wy) - (wy - uy) * (nx - wx);
  int c1 = (wx - ux) * dy - (wy - uy) * dx;
  int c2 = (nx - wx) * dy - (ny - wy) * dx;
  return turn > 0 ? (c1 > 0 && c2 > 0) : (c1 > 0 || c2 > 0);
}
__device__ __forceinline__ bool into_interior64(int ux, int uy, int wx, int wy, int nx, int ny, long long dx,
                                                long long dy) {
  long long turn = (long long)(wx - ux) * (ny - wy) - (long long)(wy - uy) * (nx - wx);
  long long c1 = (long long)(wx - ux) * dy - (long long)(wy - uy) * dx;
  long long c2 = (long long)(nx - wx) * dy - (long long)(ny - wy) * dx;
  return turn > 0 ? (c1 > 0 && c2 > 0) : (c1 > 0 || c2 > 0);
}

// Closest point of segment A-B to the integer point P (Section 4: endpoint or
// projection), as a homogeneous point (qx/qw, qy/qw), qw > 0.
struct RPt {
  long long x, y, w;
};
__device__ __forceinline__ RPt seg_closest(int ax, int ay, int bx, int by, int px, int py, int* clamp) {
  long long ex = bx - ax, ey = by - ay;
  long long L = ex * ex + ey * ey;
  long long num = (long long)(px - ax) * ex + (long long)(py - ay) * ey;
  RPt q;
  if (num <= 0) { q.x = ax; q.y = ay; q.w = 1; *clamp = 0; }
  else if (num >= L) { q.x = bx; q.y = by; q.w = 1; *clamp = 1; }
  else { q.x = (long long)ax * L + num * ex; q.y = (long long)ay * L + num * ey; q.w = L; *clamp = 2; }
  return q;
}

// Per-lane visibility of the closed segment [P, Q] for an integer point P and
// a rational point Q (used for segment sources, whose closest point varies per
// lane).  Exact 64-bit predicates over every edge of the chunks whose bounding
// box meets the box (cx0..cy1), which must contain P and Q.  P may be an
// obstacle corner (pv = 1 with its neighbours), Q is free.
template <class GEO>
__device__ __forceinline__ bool lane_visible_rational(const GEO& d, int px, int py, bool pv, int pux, int puy,
                                                      int pnx, int pny, RPt q, bool need, int cx0, int cy0,
                                                      int cx1, int cy1) {
  bool blocked = false;
  long long dqx = q.x - (long long)px * q.w, dqy = q.y - (long long)py * q.w;
  if (dqx == 0 && dqy == 0) return true;
  if (need && pv && into_interior64(pux, puy, px, py, pnx, pny, dqx, dqy)) blocked = true;
  for (int cb = 0; cb < d.NC; cb += kWave) {
    int ci = cb + lane_id();
    bool hit = false;
    if (ci < d.NC) {
      int4 bb = d.chunk(ci);
      hit = bb.x <= cx1 && bb.z >= cx0 && bb.y <= cy1 && bb.w >= cy0;
    }
    u64 cm = ballot(hit);
    while (cm) {
      int k = first_bit(cm);
      cm &= cm - 1;
      int e0 = (cb + k) * kChunk;
      int e1 = min(e0 + kChunk, d.E);
      if (ballot(need && !blocked) == 0) return false;
      for (int e = e0; e < e1; ++e) {
        EdgeRec r = d.edge(e);
        if (need && !blocked) {
          long long o1 = dqx * (r.wy - py) - dqy * (r.wx - px);
          long long o2 = dqx * (r.vy - py) - dqy * (r.vx - px);
          if ((o1 > 0 && o2 < 0) || (o1 < 0 && o2 > 0)) {
            long long o3 = (long long)r.a * px + (long long)r.b * py + r.c;
            long long o4 = (long long)r.a * q.x + (long long)r.b * q.y + (long long)r.c * q.w;
            if ((o3 > 0 && o4 < 0) || (o3 < 0 && o4 > 0)) blocked = true;
          }
          if (o1 == 0 && !blocked) {
            // w on the line PQ: strictly between P and Q?
            long long tw, tl;
            if (dqx != 0) { tw = (long long)(r.wx - px) * q.w; tl = dqx; }
            else { tw = (long long)(r.wy - py) * q.w; tl = dqy; }
            if (tl < 0) { tw = -tw; tl = -tl; }
            if (tw > 0 && tw < tl) {
              EdgeExt x = d.ext[e];
              if (into_interior64(x.ux, x.uy, r.wx, r.wy, r.vx, r.vy, px - r.wx, py - r.wy) ||
                  into_interior64(x.ux, x.uy, r.wx, r.wy, r.vx, r.vy, q.x - (long long)r.wx * q.w,
                                  q.y - (long long)r.wy * q.w))
                blocked = true;
            }
          }
        }
      }
    }
  }
  return !blocked;
}

// Culled chunks of one 64-chunk batch, split into three classes by the gap
// between the chunk box and the lanes' box (doubled units): touching or within
// 64, within 256, farther.  Walking the near classes first finds the nearby
// occluders -- which usually decide visibility -- before the far ones.
template <class GEO>
__device__ __forceinline__ void chunk_classes(const GEO& d, int NC, int cb, int cx0, int cy0, int cx1, int cy1,
                                              int bx0, int by0, int bx1, int by1, u64 cls[3]) {
  const int ci = cb + lane_id();
  bool hit = false;
  int gap = 0;
  if (ci < NC) {
    const int4 bb = d.chunk(ci);
    hit = bb.x <= cx1 && bb.z >= cx0 && bb.y <= cy1 && bb.w >= cy0;
    gap = max(max(max(bb.x - bx1, bx0 - bb.z), max(bb.y - by1, by0 - bb.w)), 0);
  }
  cls[0] = ballot(hit && gap <= 64);
  cls[1] = ballot(hit && gap <= 256) & ~cls[0];
  cls[2] = ballot(hit) & ~cls[0] & ~cls[1];
}

// Wave-level visibility between per-lane integer points P (lanes in `need`)
// and one wave-uniform integer point g.  (bx0..by1) is a box containing every
// needed P.  Returns the mask of needed lanes whose closed segment [P, g]
// meets an obstacle's open interior.
//
//   * Only edges front-facing to g (g strictly outside the edge line) can be
//     entered on the way from g to P; an entry at an edge interior is a proper
//     crossing of such an edge with P strictly on its obstacle side, and an
//     entry at a vertex happens at an endpoint of such an edge.
//   * Lane-parallel culling: chunk boxes against the box of the cone (box + g),
//     then edge relevance against the box: an edge whose endpoints stay
//     strictly on one side of every line P-g, or whose obstacle side contains
//     no point of the box, cannot block any lane.  An edge that properly
//     crosses every such segment hides the whole box at once.
//   * Per-lane test for relevant edges: endpoints strictly on opposite sides
//     of line P-g and P strictly on the obstacle side (a proper crossing).  An
//     endpoint exactly on line P-g flags the lane for the exact vertex rule.
//   * g being a corner: the direction toward P must not enter g's own
//     interior angle; P being a corner (pv): likewise toward g.
#ifndef SPM_OCC_HINTS
#define SPM_OCC_HINTS 3
#endif
constexpr int kOccHints = SPM_OCC_HINTS;   // occluding edges a tile remembers (most recent first)

// Occluder list updates: move entry h to the front; put a new edge in front.
__device__ __forceinline__ void occ_hint_front(int* hint, int h) {
  const int e = hint[h];
#pragma unroll
  for (int k = kOccHints - 1; k > 0; --k)
    if (k <= h) hint[k] = hint[k - 1];
  hint[0] = e;
}
__device__ __forceinline__ void occ_hint_push(int* hint, int e) {
#pragma unroll
  for (int k = kOccHints - 1; k > 0; --k) hint[k] = hint[k - 1];
  hint[0] = e;
}

// Edge r against the cone from g to the box (bx0..by1; rx0..ry1 = the box
// relative to g): rel = it can block some segment [P, g] with P in the box;
// occ = it properly crosses every such segment with the box on its obstacle
// side (it hides the whole box from g).
__device__ __forceinline__ void edge_vs_cone(const EdgeRec& r, int gx, int gy, int bx0, int by0, int bx1, int by1,
                                             int rx0, int rx1, int ry0, int ry1, bool& rel, bool& occ) {
  rel = occ = false;
  const int Eg = mad24(r.a, gx, mad24(r.b, gy, r.c));
  if (Eg < 0) {
    const int hiE = mad24(r.a, r.a > 0 ? bx1 : bx0, mad24(r.b, r.b > 0 ? by1 : by0, r.c));
    const int loE = mad24(r.a, r.a > 0 ? bx0 : bx1, mad24(r.b, r.b > 0 ? by0 : by1, r.c));
    // f_w(P) = cross(w - g, P - g), affine in P; range over the box
    const int aw = gy - r.wy, bw = r.wx - gx;
    const int hiw = mul24(aw, aw > 0 ? rx1 : rx0) + mul24(bw, bw > 0 ? ry1 : ry0);
    const int low = mul24(aw, aw > 0 ? rx0 : rx1) + mul24(bw, bw > 0 ? ry0 : ry1);
    const int av = gy - r.vy, bv = r.vx - gx;
    const int hiv = mul24(av, av > 0 ? rx1 : rx0) + mul24(bv, bv > 0 ? ry1 : ry0);
    const int lov = mul24(av, av > 0 ? rx0 : rx1) + mul24(bv, bv > 0 ? ry0 : ry1);
    const bool same = (low > 0 && lov > 0) || (hiw < 0 && hiv < 0);
    rel = hiE > 0 && !same;
    occ = loE > 0 && ((low > 0 && hiv < 0) || (hiw < 0 && lov > 0));
  }
}

//   occ_hint: when not null, kOccHints edge indices (or -1), the most recent
//             first, tried before the scan as occluders of the whole box;
//             the occluder found goes to the front.  Neighbouring generators
//             are often hidden by the same few edges.
//   found:    when not null, receives the index of the edge that hid the
//             whole box (hint or scan), or keeps its value when none did.
template <bool STATS, class GEO>
__device__ __forceinline__ u64 wave_blocked_uniform(const GEO& d, int px, int py, u64 need, int gx, int gy, bool gvert,
                                                    int gux, int guy, int gnx, int gny, bool pv, int pux, int puy,
                                                    int pnx, int pny, int bx0, int by0, int bx1, int by1,
                                                    int* occ_hint, u64* st, int* found = nullptr) {
  const int lane = lane_id();
  const bool me = (need >> lane) & 1ull;
  bool blk = false;
  if (me && gvert && into_interior(gux, guy, gx, gy, gnx, gny, px - gx, py - gy)) blk = true;
  if (me && pv && into_interior(pux, puy, px, py, pnx, pny, gx - px, gy - py)) blk = true;
  u64 blocked = ballot(blk) & need;
  if (blocked == need) return need;
  // line through P and g: o(x) = A x + B y + C = cross(g - P, x - P)
  const int A = py - gy, B = gx - px;
  const int C = -(mul24(A, px) + mul24(B, py));
  bool dg = false;
  const int cx0 = min(bx0, gx), cy0 = min(by0, gy), cx1 = max(bx1, gx), cy1 = max(by1, gy);
  const int rx0 = bx0 - gx, rx1 = bx1 - gx, ry0 = by0 - gy, ry1 = by1 - gy;
  if (occ_hint) {
#pragma unroll
    for (int h = 0; h < kOccHints; ++h) {
      if (occ_hint[h] < 0) break;
      bool rel, occ;
      edge_vs_cone(d.edge(occ_hint[h]), gx, gy, bx0, by0, bx1, by1, rx0, rx1, ry0, ry1, rel, occ);
      if (ballot(occ)) {
        if (STATS) st[6] += 1;
        if (found) *found = occ_hint[h];
        occ_hint_front(occ_hint, h);
        return need;
      }
    }
  }
  for (int cb = 0; cb < d.NC; cb += kWave) {
    u64 cls[3];
    chunk_classes(d, d.NC, cb, cx0, cy0, cx1, cy1, bx0, by0, bx1, by1, cls);
    for (int cl = 0; cl < 3; ++cl) {
    u64 cm = cls[cl];
    while (cm) {
      const int chunk = cb + first_bit(cm);
      cm &= cm - 1;
      const int e = chunk * kChunk + lane;
      bool rel = false, occ = false;
      EdgeRec r = {0, 0, 0, 0, 0, 0, 0, 0};
      if (e < d.E) {
        r = d.edge(e);
        edge_vs_cone(r, gx, gy, bx0, by0, bx1, by1, rx0, rx1, ry0, ry1, rel, occ);
      }
      if (STATS) st[4] += 1;
      const u64 om = ballot(occ);
      if (om) {
        if (STATS) st[6] += 1;
        if (occ_hint) occ_hint_push(occ_hint, chunk * kChunk + first_bit(om));
        if (found) *found = chunk * kChunk + first_bit(om);
        return need;
      }
      u64 rm = ballot(rel);
      while (rm) {
        // the edge's fields from the lane that holds it
        const int ql = first_bit(rm);
        rm &= rm - 1;
        const int wx = readlane(r.wx, ql), wy = readlane(r.wy, ql), vx = readlane(r.vx, ql), vy = readlane(r.vy, ql);
        const int ea = readlane(r.a, ql), eb = readlane(r.b, ql), enc = readlane(r.nc, ql);
        if (STATS) st[5] += (u64)__popcll(need & ~blocked);
        const int ow = mad24(A, wx, mad24(B, wy, C));
        const int ov = mad24(A, vx, mad24(B, vy, C));
        // sign of ow * ov: converting to float keeps every sign and every zero exact
        const float prod = (float)ow * (float)ov;
        const int ep = mad24(ea, px, mul24(eb, py));
        blk = blk || (prod < 0.0f && ep > enc);
        if (prod == 0.0f) {
          // an endpoint exactly on line P-g matters only strictly between P and g (the vertex rule
          // below); P itself is the corner rule checked above, g is not on a front-facing edge
          const int gpx = gx - px, gpy = gy - py, len2 = mad24(gpx, gpx, mul24(gpy, gpy));
          const int dw = mad24(wx - px, gpx, mul24(wy - py, gpy));
          const int dv = mad24(vx - px, gpx, mul24(vy - py, gpy));
          dg = dg || (ow == 0 && dw > 0 && dw < len2) || (ov == 0 && dv > 0 && dv < len2);
        }
      }
      blocked = ballot(blk) & need;
      if (blocked == need) return need;
    }
    }
  }
  // exact vertex rule for lanes with an endpoint exactly on their line P-g: every vertex w (the start of
  // one edge) of the chunks meeting the cone hull, lanes over the chunk's edges, one such lane P at a
  // time (few lanes need it; on lattice-aligned scenes many tiles have some)
  u64 slow = ballot(dg) & need & ~blocked;
  if (slow) {
    for (int cb = 0; cb < d.NC && slow; cb += kWave) {
      int ci = cb + lane;
      bool hit = false;
      if (ci < d.NC) {
        int4 bb = d.chunk(ci);
        hit = bb.x <= cx1 && bb.z >= cx0 && bb.y <= cy1 && bb.w >= cy0;
      }
      u64 cm = ballot(hit);
      while (cm && slow) {
        const int chunk = cb + first_bit(cm);
        cm &= cm - 1;
        const int e = chunk * kChunk + lane;
        const bool have = e < d.E;
        EdgeRec r = {0, 0, 0, 0, 0, 0, 0, 0};
        if (have) r = d.edge(e);
        u64 sm = slow;
        while (sm) {
          const int j = first_bit(sm);
          sm &= sm - 1;
          const int qx = readlane(px, j), qy = readlane(py, j);   // lane j's P
          const int Aj = qy - gy, Bj = gx - qx;
          const int Cj = -(mul24(Aj, qx) + mul24(Bj, qy));
          const int len2 = mul24(gx - qx, gx - qx) + mul24(gy - qy, gy - qy);
          bool on = false;
          if (have && mad24(Aj, r.wx, mad24(Bj, r.wy, Cj)) == 0) {
            const int dot = mul24(r.wx - qx, gx - qx) + mul24(r.wy - qy, gy - qy);
            if (dot > 0 && dot < len2) {
              const EdgeExt x = d.ext[e];
              on = into_interior(x.ux, x.uy, r.wx, r.wy, r.vx, r.vy, qx - r.wx, qy - r.wy) ||
                   into_interior(x.ux, x.uy, r.wx, r.wy, r.vx, r.vy, gx - r.wx, gy - r.wy);
            }
          }
          if (ballot(on)) {
            slow &= ~(1ull << j);
            if (lane == j) blk = true;
          }
        }
      }
    }
    blocked = ballot(blk) & need;
  }
  return blocked;
}
// Wave-level visibility between per-lane pixel points P and their closest
// points q*(P) on one segment source A-B, for lanes whose closest point lies
// strictly inside the segment.  Then [P, q*] is perpendicular to e = B - A, so
// with D(x) = e . x the endpoints w, v of an edge lie strictly on opposite
// sides of line P-q* iff D(P) is strictly between D(w) and D(v); and the
// obstacle-side sign of q* is the common sign of E(A) and E(B) unless the edge
// line cuts the segment (then it is computed per lane, exactly, in 64 bits).
// Lanes with a vertex exactly on their line strictly between P and q* fall
// back to the generic test.  P may be an obstacle corner (pv, with its
// neighbours): then the direction toward q* must not enter its own angle.
// (bx0..by1) is a box containing every needed P.
// Edge r against the band between the pixel box (bx0..by1) and the segment
// source A-B (direction e = B - A; Pmin..Pmax = the box's range of e . P):
// rel = it can block some perpendicular [P, q*(P)]; occ = it crosses every
// such segment with the box on its obstacle side.
__device__ __forceinline__ void edge_vs_band(const EdgeRec& r, int ax, int ay, int bx, int by, int ex, int ey,
                                             int Pmin, int Pmax, int bx0, int by0, int bx1, int by1, bool& rel,
                                             bool& occ) {
  const int EA = r.a * ax + r.b * ay + r.c, EB = r.a * bx + r.b * by + r.c;
  const int hiE = r.a * (r.a > 0 ? bx1 : bx0) + r.b * (r.b > 0 ? by1 : by0) + r.c;
  const int loE = r.a * (r.a > 0 ? bx0 : bx1) + r.b * (r.b > 0 ? by0 : by1) + r.c;
  const int Dw = ex * r.wx + ey * r.wy, Dv = ex * r.vx + ey * r.vy;
  const int lo = min(Dw, Dv), hi = max(Dw, Dv);
  const bool strad = Pmax >= lo && Pmin <= hi;
  bool side, full;
  if (EA > 0 && EB > 0) { side = loE < 0; full = hiE < 0; }
  else if (EA < 0 && EB < 0) { side = hiE > 0; full = loE > 0; }
  else if (EA == 0 && EB == 0) { side = false; full = false; }
  else { side = loE < 0 || hiE > 0; full = false; }
  rel = strad && side;
  occ = full && lo < Pmin && Pmax < hi;
}

//   occ_hint: as for wave_blocked_uniform (an edge tried first as an occluder
//             of the whole band, updated with the occluder found).
template <bool STATS, class GEO>
__device__ __forceinline__ u64 wave_blocked_perp(const GEO& d, int px, int py, u64 need, int ax, int ay, int bx,
                                                 int by, bool pv, int pux, int puy, int pnx, int pny, int bx0,
                                                 int by0, int bx1, int by1, int* occ_hint, u64* st) {
  const int lane = lane_id();
  const int ex = bx - ax, ey = by - ay;
  const int L = ex * ex + ey * ey;
  const int DA = ex * ax + ey * ay;
  const int Pp = ex * px + ey * py;  // D(P)
  const long long num = (long long)Pp - DA;  // (P - A) . e, in (0, L) for needed lanes
  // F(x) = cross(e, x - A): zero on the segment's line, so a vertex w on line P-q* lies strictly
  // between P and q* iff F(w) lies strictly between 0 and F(P)
  const int FP = ex * (py - ay) - ey * (px - ax);
  const int Pmin = ex * (ex > 0 ? bx0 : bx1) + ey * (ey > 0 ? by0 : by1);
  const int Pmax = ex * (ex > 0 ? bx1 : bx0) + ey * (ey > 0 ? by1 : by0);
  // culling box: the pixel box and the part of the segment it projects onto
  const float t0 = fminf(fmaxf((float)(Pmin - DA) / (float)L, 0.0f), 1.0f);
  const float t1 = fminf(fmaxf((float)(Pmax - DA) / (float)L, 0.0f), 1.0f);
  const float qx0 = ax + t0 * ex, qx1 = ax + t1 * ex, qy0 = ay + t0 * ey, qy1 = ay + t1 * ey;
  const int cx0 = min(bx0, (int)floorf(fminf(qx0, qx1)) - 1), cx1 = max(bx1, (int)ceilf(fmaxf(qx0, qx1)) + 1);
  const int cy0 = min(by0, (int)floorf(fminf(qy0, qy1)) - 1), cy1 = max(by1, (int)ceilf(fmaxf(qy0, qy1)) + 1);
  bool blk = false, dg = false;
  if (pv && ((need >> lane) & 1ull)) {
    // P a corner: the direction toward q* must not enter P's own interior angle
    const long long qx = (long long)ax * L + num * ex, qy = (long long)ay * L + num * ey;
    blk = into_interior64(pux, puy, px, py, pnx, pny, qx - (long long)px * L, qy - (long long)py * L);
  }
  u64 blocked = ballot(blk) & need;
  if (blocked == need) return need;
  if (occ_hint) {
#pragma unroll
    for (int h = 0; h < kOccHints; ++h) {
      if (occ_hint[h] < 0) break;
      bool rel, occ;
      edge_vs_band(d.edge(occ_hint[h]), ax, ay, bx, by, ex, ey, Pmin, Pmax, bx0, by0, bx1, by1, rel, occ);
      if (ballot(occ)) {
        if (STATS) st[6] += 1;
        occ_hint_front(occ_hint, h);
        return need;
      }
    }
  }
  for (int cb = 0; cb < d.NC; cb += kWave) {
    u64 cls[3];
    chunk_classes(d, d.NC, cb, cx0, cy0, cx1, cy1, bx0, by0, bx1, by1, cls);
    for (int cl = 0; cl < 3; ++cl) {
    u64 cm = cls[cl];
    while (cm) {
      const int chunk = cb + first_bit(cm);
      cm &= cm - 1;
      const int e = chunk * kChunk + lane;
      bool rel = false, occ = false;
      EdgeRec r = {0, 0, 0, 0, 0, 0, 0, 0};
      if (e < d.E) {
        r = d.edge(e);
        edge_vs_band(r, ax, ay, bx, by, ex, ey, Pmin, Pmax, bx0, by0, bx1, by1, rel, occ);
      }
      if (STATS) st[4] += 1;
      const u64 om = ballot(occ);
      if (om) {
        if (STATS) st[6] += 1;
        if (occ_hint) occ_hint_push(occ_hint, chunk * kChunk + first_bit(om));
        return need;
      }
      u64 rm = ballot(rel);
      while (rm) {
        const int ql = first_bit(rm);
        rm &= rm - 1;
        const int wx = readlane(r.wx, ql), wy = readlane(r.wy, ql), vx = readlane(r.vx, ql), vy = readlane(r.vy, ql);
        const int ea = readlane(r.a, ql), eb = readlane(r.b, ql), ec = readlane(r.c, ql);
        if (STATS) st[5] += (u64)__popcll(need & ~blocked);
        const int Dw = ex * wx + ey * wy, Dv = ex * vx + ey * vy;
        const int lo = min(Dw, Dv), hi = max(Dw, Dv);
        const int EA = ea * ax + eb * ay + ec, EB = ea * bx + eb * by + ec;
        const bool str = Pp > lo && Pp < hi;
        if (Pp == lo || Pp == hi) {
          const int Fw = ex * (wy - ay) - ey * (wx - ax), Fv = ex * (vy - ay) - ey * (vx - ax);
          const bool bw = Pp == Dw && (FP > 0 ? (Fw > 0 && Fw < FP) : (Fw < 0 && Fw > FP));
          const bool bv = Pp == Dv && (FP > 0 ? (Fv > 0 && Fv < FP) : (Fv < 0 && Fv > FP));
          dg = dg || bw || bv;
        }
        const int ep = mad24(ea, px, mad24(eb, py, ec));
        bool opp;
        if (EA > 0 && EB > 0) opp = ep < 0;
        else if (EA < 0 && EB < 0) opp = ep > 0;
        else if (EA == 0 && EB == 0) opp = false;
        else {
          // E(q*) * L = E(A) * L + num * (E(B) - E(A)), exact in 64 bits
          const long long eq = (long long)EA * L + num * (long long)(EB - EA);
          opp = (ep > 0 && eq < 0) || (ep < 0 && eq > 0);
        }
        blk = blk || (str && opp);
      }
      blocked = ballot(blk) & need;
      if (blocked == need) return need;
    }
    }
  }
  u64 slow = ballot(dg) & need & ~blocked;
  if (slow) {
    int clamp;
    const RPt q = seg_closest(ax, ay, bx, by, px, py, &clamp);
    const bool mine = (slow >> lane) & 1ull;
    const bool vs = lane_visible_rational(d, px, py, pv, pux, puy, pnx, pny, q, mine, min(cx0, bx0), min(cy0, by0),
                                          max(cx1, bx1), max(cy1, by1));
    blk = blk || (mine && !vs);
    blocked = ballot(blk) & need;
  }
  return blocked;
}
#endif  // __HIPCC__

// Work order of the pixel stage (the order itself is described with k_pixel):
// item classes by lb = min_g cost(g) + |c - box(g)| at the item centre c.
// One call handles kOrderGroup items with a 256-thread workgroup (eight per
// wavefront): bb and cost hold the G generators' boxes and float costs (any
// order; +inf for unreached ones).  Each class count is raised with one
// atomic per workgroup and the items go to order[class * ocap + slot].
constexpr int kOrderGroup = 32;
constexpr size_t kOrderFuseLds = 48 * 1024;
inline int order_items(const Dev& d) {
  const int tw = d.tile_w, th = 64 / tw;
  const int ntx = (d.W + tw - 1) / tw, nty = (d.H + th - 1) / th;
  return (ntx + d.strip - 1) / d.strip * nty;
}
// The order comes from the generator sort's launch when its tables fit in LDS
// there and the scene has more items than a launch of the pixel stage keeps
// resident at 4 waves per SIMD (below that every item starts at once); the
// pixel launch asks the same question, so the two always agree.
constexpr int kOrderMinItems = 256 * 16;
inline bool order_fused(const Dev& d) {
  return (size_t)d.Gmax * (sizeof(int4) + sizeof(float)) <= kOrderFuseLds && order_items(d) > kOrderMinItems;
}
__device__ __forceinline__ void tile_order_group(const Dev& d, int grp, int G, const int4* bb, const float* cost,
                                                 int* lcount, int* lbase, int* icls, int* islot) {
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / 64;
  const int TW = d.tile_w, TH = 64 / TW;
  const int ntx = (d.W + TW - 1) / TW, nty = (d.H + TH - 1) / TH;
  const int spr = (ntx + d.strip - 1) / d.strip;
  const int nitems = spr * nty;
  const float scale = (float)(2 * kOrderBins) / (float)(d.W + d.H);
  constexpr int kPer = kOrderGroup / 4;
  for (int k = 0; k < kPer; ++k) {
    const int li = wv * kPer + k;
    const int item = grp * kOrderGroup + li;
    if (item >= nitems) break;
    const int ty = item / spr, sx = item - ty * spr;
    const int t0 = sx * d.strip, t1 = min(t0 + d.strip, ntx);
    const int cx = (t0 + t1) * TW, cy = (2 * ty + 1) * TH;   // item centre, doubled coordinates
    float lb = INFINITY;
    for (int h = lane; h < G; h += 64) {
      const int4 b = bb[h];
      const float dx = (float)max(max(b.x - cx, cx - b.z), 0), dy = (float)max(max(b.y - cy, cy - b.w), 0);
      lb = fminf(lb, cost[h] + 0.5f * __builtin_amdgcn_sqrtf(dx * dx + dy * dy));
    }
    // lb >= 0, so its bits order as unsigned
    const float f = __uint_as_float(wave_min_u32(__float_as_uint(lb))) * scale;
    const int c = f < (float)(kOrderBins - 1) ? (int)f : kOrderBins - 1;
    if (lane == 0) {
      const int cls = kOrderBins - 1 - c;
      icls[li] = cls;
      islot[li] = atomicAdd(&lcount[cls], 1);
    }
  }
  __syncthreads();
  if (tid < kOrderBins) lbase[tid] = lcount[tid] ? atomicAdd(&d.obins[tid], lcount[tid]) : 0;
  __syncthreads();
  if (tid < kOrderGroup) {
    const int item = grp * kOrderGroup + tid;
    if (item < nitems) d.order[(size_t)icls[tid] * d.ocap + lbase[icls[tid]] + islot[tid]] = item;
  }
}


}  // namespace spm
