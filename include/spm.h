/*
 * spm.h -- C ABI of libspm, a GPU builder of multi-source shortest path maps
 * (SPMs) for polygonal scenes, after Farias & Kallmann, "Improved Shortest
 * Path Maps with GPU Shaders".
 *
 * Problem (Section 3 and Section 4 of the paper): a rectangular domain
 * [0,W] x [0,H] covered by a W x H pixel grid, polygonal obstacles with n
 * vertices in total, point sources and segment sources.  For every pixel
 * centre p the map stores lambda*(p), the length of the shortest
 * obstacle-avoiding path from p to the closest source (a source point or any
 * point of a segment source), and the parent: the first point that path turns
 * at (an obstacle vertex) or the source itself.  Following parents gives the
 * whole path (Section 1: grid lookup, then a walk linear in the path length).
 *
 * Units and conventions used by every entry point:
 *   - coordinates are int32 domain units (1 unit = 1 pixel), 0 <= x <= W,
 *     0 <= y <= H, with 1 <= W, H <= SPM_MAX_SIDE;
 *   - pixel (i, j) has its centre at (i + 1/2, j + 1/2) and is stored at
 *     row-major index j * W + i;
 *   - obstacles are simple polygons given as counter-clockwise loops (the
 *     obstacle lies to the left of every directed edge), without repeated or
 *     collinear consecutive vertices, pairwise disjoint as closed sets;
 *   - point sources lie strictly outside every closed obstacle; a segment
 *     source has distinct endpoints and the closed segment meets no closed
 *     obstacle;
 *   - generators (the paper's DataArray entries, Section 3) are numbered in a
 *     canonical order: point sources, then segment sources, then every
 *     obstacle corner whose interior angle is below 180 degrees (the only
 *     corners a shortest path can bend at), by polygon and vertex order.
 *     Parent ids index this order.
 *
 * Errors: every entry point returns SPM_OK or a negative spm_status; no
 * exception or abort crosses the ABI.  spm_last_error() gives a message for
 * the calling thread's last failure.  Validation that can fail runs on the
 * host before any device work is queued.
 */
#ifndef SPM_H
#define SPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPM_MAX_SIDE 8192      /* largest W or H (keeps exact predicates in 32/64-bit integers) */
#define SPM_N_STAGES 8         /* stages reported by spm_timer_elapsed */

typedef enum {
  SPM_OK = 0,
  SPM_ERR_INVALID_ARG = -1,  /* null pointer, negative count, bad size */
  SPM_ERR_GEOMETRY = -2,     /* polygon not simple/CCW, obstacles meet, source not free */
  SPM_ERR_RANGE = -3,        /* a coordinate outside [0,W]x[0,H] or a side above SPM_MAX_SIDE */
  SPM_ERR_CAPACITY = -4,     /* workspace or output buffer too small */
  SPM_ERR_HIP = -5,          /* the HIP runtime reported an error */
  SPM_ERR_UNREACHABLE = -6   /* spm_query_path: the query point has no path */
} spm_status;

enum { SPM_GEN_POINT = 0, SPM_GEN_SEGMENT = 1, SPM_GEN_VERTEX = 2 };

/* A scene.  For spm_validate and spm_build the arrays are host memory, read
 * before the call returns; for spm_build_ex, the batched builds and
 * spm_query_points they are device memory, read by the queued work (keep
 * them until it completes).  The counts are always host values. */
typedef struct {
  int32_t width, height;     /* W, H */
  int32_t n_polys;           /* number of obstacle polygons */
  int32_t n_vertices;        /* total obstacle vertices = poly_start[n_polys] */
  int32_t n_points;          /* point sources */
  int32_t n_segs;            /* segment sources */
  const int32_t* poly_start; /* [n_polys + 1] offsets into vx/vy, poly_start[0] = 0 */
  const int32_t* vx;         /* [n_vertices] */
  const int32_t* vy;         /* [n_vertices] */
  const int32_t* pts;        /* [n_points * 2] (x, y) */
  const int32_t* segs;       /* [n_segs * 4] (ax, ay, bx, by) */
} spm_scene;

/* Outputs of a build: device memory owned by the caller.  max_gen comes from
 * spm_query_sizes; the generator arrays hold *n_gen entries, and their entries
 * from *n_gen up to max_gen are left as they were (unspecified). */
typedef struct {
  float* dist;          /* [H * W] lambda* in domain units; +inf inside or on an obstacle, or unreachable */
  int32_t* parent;      /* [H * W] generator id of the winning cone; -1 where dist is +inf */
  int32_t* gen_kind;    /* [max_gen] SPM_GEN_* */
  int32_t* gen_xy;      /* [max_gen * 4] x, y (and x2, y2 for segments; else repeated) */
  double* gen_cost;     /* [max_gen] lambda* of the generator (0 for sources, +inf unreachable) */
  int32_t* gen_parent;  /* [max_gen] next generator toward the source; a source stores its own id; -1 unreachable */
  int32_t* n_gen;       /* [1] number of generators G */
} spm_out;

const char* spm_last_error(void);

/* Exact host-side check of a host-memory scene against the conventions above
 * (O(n^2) in the vertex count).  Returns SPM_OK, SPM_ERR_INVALID_ARG,
 * SPM_ERR_RANGE or SPM_ERR_GEOMETRY.  spm_build runs it on every call;
 * spm_build_ex and the batched builds take its result as a prerequisite. */
int spm_validate(const spm_scene* host_scene);

/* Capacities for a scene's counts (only the scalar fields are read):
 * max_gen = n_points + n_segs + n_vertices, and the device workspace bytes a
 * build needs.  Returns SPM_ERR_INVALID_ARG / SPM_ERR_RANGE for bad counts. */
int spm_query_sizes(const spm_scene* scene, int32_t* max_gen, size_t* workspace_bytes);

/* Build the map of a host-memory scene: the problem statement of Sections 3
 * and 4 (obstacles, point and segment sources) in, the grid of distance and
 * parent (Section 3: the map's per-pixel distance and ParentId) plus the
 * generator table out.
 *   1. On the host, before any device work: argument checks, then spm_validate
 *      (any failure returns its code: SPM_ERR_INVALID_ARG, SPM_ERR_RANGE,
 *      SPM_ERR_GEOMETRY; SPM_ERR_CAPACITY when ws_bytes is below
 *      spm_query_sizes' figure).
 *   2. The scene is copied into the library's pinned staging (a ring of four
 *      slots, each grown once to the largest scene it has held and kept until
 *      the process ends), so the caller may free or change it as soon as the
 *      call returns, and from there into d_ws by an asynchronous copy on
 *      `stream` (a hipStream_t; NULL = the null stream).  Reusing a slot waits
 *      for the copy queued from it four calls earlier.
 *   3. Every step of the build is queued on `stream`; the call returns without
 *      waiting for it.
 * d_ws (device memory, workspace_bytes from spm_query_sizes) stays owned by
 * the caller and must not be shared by builds that can run concurrently.
 * Because of the host staging the call cannot be captured in a HIP graph
 * (SPM_ERR_INVALID_ARG while `stream` is capturing): capture spm_build_ex.
 * SPM_ERR_HIP if a HIP call fails. */
int spm_build(const spm_scene* host_scene, const spm_out* out, void* d_ws, size_t ws_bytes, void* stream);

/* Optional per-stage timing: a timer records HIP events around each build
 * stage on the build's stream.  spm_timer_elapsed synchronises on the last
 * recorded event and returns the per-stage milliseconds summed over every
 * build recorded since the last reset (stage order: ingest, edge sort and
 * inside mask, generator order and chunk boxes, generator visibility,
 * relaxation, generator sort (with the pixel kernel's work order and cluster
 * tables when they need launches of their own), pixel propagation (the pixel
 * kernel alone), total) and the number of builds. */
typedef struct spm_timer spm_timer;
int spm_timer_create(spm_timer** t);
int spm_timer_destroy(spm_timer* t);
int spm_timer_reset(spm_timer* t);
int spm_timer_elapsed(spm_timer* t, float* ms /* [SPM_N_STAGES] */, int32_t* n_builds);

/* Build options.  tile_w x tile_h is the pixel tile one wavefront owns
 * (8x8, 16x4 or 4x16; 0 = 8x8).  strip is the number of consecutive tiles of
 * one tile row a wavefront takes at a time (1..64; 0 = the default): each
 * tile after the first first tries the winners of the tile to its left.
 * samples is the number of seed searches a tile runs, each from one of its
 * pixels that still has no value: candidates in order of cost + distance,
 * checked with a cheap visibility test, until one is seen (0 = the default,
 * -1 = none).  walk selects how a tile goes through the generators: 0 = by
 * the scene's largest possible generator count G (np + ns + nv); 1 = in order
 * of a lower bound over the tile, every estimate in registers (G <= 512);
 * 2 = the same with the least estimates cached and refilled (G <= 8192);
 * 3 = seed searches, then (cost, id) order; 4 = spatial clusters of 8
 * generators in order of a lower bound over the tile, a cluster that one edge
 * hides from the whole tile skipped at once (G <= 8192).  A forced walk that does not fit
 * G fails with SPM_ERR_INVALID_ARG.  strip, samples and walk change speed
 * only, never an output bit.
 * d_stats, when not NULL, selects the instrumented pixel kernel, which adds
 * its work counters to SPM_N_STATS unsigned 64-bit device counters: [0]
 * tiles, [1] generators taken by the lower-bound walk or batches of 64
 * lane-parallel bound / seed-search tests, [2] lane bound tests, [3] wave
 * visibility tests, [4] edge relevance or seed-search edge tests (x64 lanes),
 * [5] lane edge tests, [6] tests ended by one edge hiding the whole tile, [7]
 * accepted candidates, [8] occluder-cache tests, [9] occluder-cache hits,
 * [10] lane closest-point computations for segment sources, [11] cluster
 * members within the bound, [12] cluster members tried, [13] clusters hidden
 * whole, [14] cluster members that a cached edge hides from the whole tile
 * (not tried), [15] cluster members tested against the cached edges' umbrae. */
#define SPM_N_STATS 16
typedef struct {
  int32_t tile_w, tile_h;
  spm_timer* timer;
  uint64_t* d_stats;
  int32_t strip;
  int32_t samples;
  int32_t walk;
} spm_build_opts;
/* The same build from a scene already in device memory (dev_scene's arrays;
 * its counts are host values), with options (opts may be NULL: defaults).
 * Nothing is copied or allocated and the host never waits, so the call can be
 * captured in a HIP graph and replayed.  Prerequisite: the scene passed
 * spm_validate (as host arrays with the same contents); it is not checked
 * again here, and a scene that breaks the conventions gives unspecified
 * outputs.  Argument errors (SPM_ERR_INVALID_ARG, SPM_ERR_CAPACITY) are found
 * before any launch; SPM_ERR_HIP if a launch fails. */
int spm_build_ex(const spm_scene* dev_scene, const spm_out* out, void* d_ws, size_t ws_bytes, void* stream,
                 const spm_build_opts* opts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the build
 * of spm_build_ex with default options, using a workspace inside the library
 * instead of d_ws -- a static device array of SPM_NOALLOC_MAX_WS bytes per
 * GPU, held from the library's load until the process ends.  dev_scene and
 * out are as for spm_build_ex (device memory, the scene validated
 * beforehand); nothing is allocated and the host never waits.  Scenes whose
 * workspace (spm_query_sizes) exceeds SPM_NOALLOC_MAX_WS fail with
 * SPM_ERR_CAPACITY before any launch.  Every call on one GPU shares that
 * array: calls that can overlap on one GPU (different streams without
 * ordering, or different host threads) race and give unspecified outputs;
 * calls ordered on one stream are safe.  Each build clears the counters it
 * uses, so leftovers of an earlier call do not matter. */
#define SPM_NOALLOC_MAX_WS (16u << 20)
int spm_build_noalloc(const spm_scene* dev_scene, const spm_out* out, void* stream);

/* ---------------------------------------------------------------------
 * Batched builds.  Many independent scenes are built by one launch per
 * stage over all of them; the pixel stage is a single persistent launch whose
 * workgroups take (scene, slice of 64 tiles) items from one device queue,
 * each scene with its own tile shape.  The paper motivates cheap rebuilds of
 * many maps for dynamic scenes (Section 1); this batches them.  Each scene
 * follows the conventions above (validated beforehand) and gets its own
 * outputs.  Zero-initialised option fields select the defaults.
 * ------------------------------------------------------------------- */
typedef struct {
  int32_t n;                /* number of scenes, >= 1 */
  const spm_scene* scenes;  /* [n] device-memory scenes (counts are host values) */
  const spm_out* outs;      /* [n] outputs, sized by spm_query_sizes per scene */
  const int32_t* tile_w;    /* [n] tile width per scene: 8 (8x8), 16 (16x4) or 4 (4x16); NULL = all 8 */
  int32_t pixel_waves;      /* waves per SIMD of the persistent pixel launch, 1..8 (fewer if they do not
                               fit); 0 = as many as fit */
  int32_t walk;             /* 0 = by the batch's largest possible generator count; 1..3 as in
                               spm_build_opts.walk (the cluster walk, 4, is not offered for batches) */
} spm_batch;

/* Device workspace bytes for a batch (host arithmetic only). */
int spm_batch_query_sizes(const spm_batch* b, size_t* workspace_bytes);

/* Writes the batch's per-scene descriptors into d_ws with a synchronous
 * host-to-device copy.  Must be called (outside any stream capture) before
 * spm_build_batch, and again whenever any pointer, count or tile width of
 * the batch changes; the scene contents may change freely in between. */
int spm_batch_prepare(const spm_batch* b, void* d_ws, size_t ws_bytes);

/* Queues the batched build on `stream` (kernels only: no allocation, no host
 * synchronisation, no copies), so it can be captured in a HIP graph.  b must
 * describe the same batch as the last spm_batch_prepare on d_ws.  timer may
 * be NULL (see spm_timer_elapsed for the stage order). */
int spm_build_batch(const spm_batch* b, void* d_ws, size_t ws_bytes, void* stream, spm_timer* timer);

/* A batched build captured in a HIP graph on a non-null `stream`; replay with
 * spm_graph_launch on any stream.  The graph keeps the batch's pointers: the
 * buffers must outlive it. */
typedef struct spm_graph spm_graph;
int spm_graph_capture_batch(const spm_batch* b, void* d_ws, size_t ws_bytes, void* stream, spm_graph** g);
int spm_graph_launch(spm_graph* g, void* stream);
int spm_graph_destroy(spm_graph* g);

/* ---------------------------------------------------------------------
 * Agents and the adjoint.  An agent at a (domain units) reads its pixel's
 * parent g from a built map (Section 1: grid lookup) and its distance
 * D(a) = |a - x_g(a)| + cost(g), x_g(a) being g, or the closest point of a
 * segment source (Section 4).  With the parent chains held fixed, D depends
 * on the sources only through the last leg of each path, which gives the
 * gradient of any loss L(D) with respect to the point sources and the
 * segment endpoints (obstacle corners are fixed).  Device memory, queued on
 * `stream`; the scene argument is only read for its counts and sizes.
 * ------------------------------------------------------------------- */

/* Workspace bytes of spm_backward for n_agents agents. */
int spm_agent_query_ws(const spm_scene* scene, int32_t n_agents, size_t* workspace_bytes);

/* d_dist[i] = D(agent i) (float), +inf for agents outside the grid or in a
 * pixel without parent.  d_agents_xy is [n_agents][2]. */
int spm_agent_distance(const spm_scene* scene, const spm_out* map, int32_t n_agents, const float* d_agents_xy,
                       float* d_dist, void* stream);

/* Refined map values and paths at arbitrary points (Section 5.1, Discussion: a point near
 * the border of two regions may take the wrong first turn from its own
 * pixel; comparing the parents of the neighbouring pixels at the point itself
 * removes that error).  For query point i (domain units, d_pts[2i], d_pts[2i+1]),
 * snapped to 1/512 domain unit: among the parents of the 3 x 3 pixels around
 * it, the least cost + distance that the point sees (exact integer
 * visibility under the closed-free-space rule; every generator when it sees
 * none of them).  d_dist[i] (float) and d_parent[i] (generator id) receive
 * it; +inf / -1 for points outside the domain, in or on an obstacle, or
 * unreachable.  When d_path_n is not NULL, the path is walked too: the
 * snapped point, the corners of the parent chain and the source point (a
 * segment source's closest point to the last corner); d_path_n[i] receives
 * its number of points (0 when unreachable) and d_path_xy, when not NULL,
 * its first min(count, cap) points ([n][cap][2] floats).  The scene must be
 * the one the map was built from (device arrays; read here for the obstacle
 * edges).  All pointers are device memory, queued on `stream`. */
int spm_query_points(const spm_scene* dev_scene, const spm_out* map, int32_t n, const float* d_pts, float* d_dist,
                     int32_t* d_parent, int32_t cap, float* d_path_xy, int32_t* d_path_n, void* stream);

/* Gradient of L with respect to the sources, given dL/dD per agent:
 * d_grad_pts[n_points][2] and d_grad_segs[n_segs][4] (dA then dB) are
 * overwritten.  Contributions are accumulated in double in a fixed order, so
 * the result is bitwise reproducible.  Agents without a parent contribute 0. */
int spm_backward(const spm_scene* scene, const spm_out* map, int32_t n_agents, const float* d_agents_xy,
                 const float* d_dL_dD, float* d_grad_pts, float* d_grad_segs, void* d_ws, size_t ws_bytes,
                 void* stream);

/* Host copy of a built map for path queries. */
typedef struct {
  int32_t width, height;
  const int32_t* parent;     /* [H * W] */
  int32_t n_gen;
  const int32_t* gen_kind;   /* [n_gen] */
  const int32_t* gen_xy;     /* [n_gen * 4] */
  const int32_t* gen_parent; /* [n_gen] */
  const double* gen_cost;    /* [n_gen] */
} spm_map_host;

/* Shortest path from the query point q (domain units, inside the domain) to
 * its closest source, read from the map (Section 1: constant-time grid
 * lookup of the parent, then the chain of parents, linear in the path
 * length).  Writes the polyline q, parent, ..., source point (the last point
 * is the closest point of a segment source when the path ends on one) as
 * float pairs to out_xy[2 * cap], its vertex count to *n_out and its length
 * to *out_len.  Host memory only; no device work.  SPM_ERR_UNREACHABLE when
 * q's pixel has no parent, SPM_ERR_CAPACITY when cap is too small. */
int spm_query_path(const spm_map_host* map, float qx, float qy, float* out_xy, int32_t cap, int32_t* n_out,
                   float* out_len);

#ifdef __cplusplus
}
#endif
#endif /* SPM_H */
