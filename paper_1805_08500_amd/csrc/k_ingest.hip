// k_ingest.hip -- device-side scene ingest for libspm.
//
// Builds, from the caller's device arrays, everything the later stages read:
// doubled-coordinate edge records with their line functions, the generator
// table (the paper's DataArray, Section 3: sources first, then the obstacle
// corners a path can bend at), a spatially sorted copy of the edges cut into
// chunks with bounding boxes, a spatial order of the generators, and the
// closed inside-obstacle mask of the pixel grid (pixel centres on or inside an
// obstacle get no distance).
//
// Every kernel is a template over its scene source: one scene carried in the
// kernel arguments, or a batch of scenes found from prefix offsets.
#include "spm_internal.hpp"

namespace spm {

// Obstacle vertex i: the edge i -> next(i), its neighbours, the corner's
// convexity and a Morton key of the edge midpoint.
__device__ __forceinline__ void ingest_vertex(const Dev& d, int i) {
  int lo = 0, hi = d.n_polys - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (d.poly_start[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  const int a = d.poly_start[lo], b = d.poly_start[lo + 1];
  const int ip = (i == a) ? b - 1 : i - 1;
  const int in = (i == b - 1) ? a : i + 1;
  const int inn = (in == b - 1) ? a : in + 1;
  const int wx = 2 * d.vx[i], wy = 2 * d.vy[i];
  const int nx = 2 * d.vx[in], ny = 2 * d.vy[in];
  const int ux = 2 * d.vx[ip], uy = 2 * d.vy[ip];
  EdgeRec r;
  r.wx = wx; r.wy = wy; r.vx = nx; r.vy = ny;
  r.a = wy - ny;
  r.b = nx - wx;
  r.c = -(r.a * wx + r.b * wy);
  r.nc = -r.c;
  d.edges_raw[i] = r;
  EdgeExt x;
  x.ux = ux; x.uy = uy; x.nx = 2 * d.vx[inn]; x.ny = 2 * d.vy[inn];
  d.ext_raw[i] = x;
  d.convex[i] = ((wx - ux) * (ny - wy) - (wy - uy) * (nx - wx)) > 0 ? 1 : 0;
  // Morton code of the midpoint (15 bits per axis)
  unsigned mx = (unsigned)((wx + nx) >> 1) & 0x7fffu, my = (unsigned)((wy + ny) >> 1) & 0x7fffu;
  unsigned code = 0;
  for (int k = 0; k < 15; ++k) code |= (((mx >> k) & 1u) << (2 * k)) | (((my >> k) & 1u) << (2 * k + 1));
  d.keys[i] = ((u64)code << 32) | (u64)(unsigned)i;
}

// One thread per obstacle vertex, chip-wide (scenes with many vertices).
template <class S>
__global__ __launch_bounds__(256) void k_ingest_edges(S src) {
  int sc, i;
  if (!src.locate(STG_VTX, blockIdx.x * blockDim.x + threadIdx.x, sc, i)) return;
  ingest_vertex(src.scene(sc), i);
}

// One workgroup per scene: the canonical generator table.  Points, then
// segments, then every convex corner (left turn) in vertex order; ids by a
// block scan.  Also resets the scene's pixel tile queue.  EDGES: the
// workgroup first ingests the scene's vertices itself (scenes of at most
// kIngestFuseMax vertices), saving the chip-wide launch.
template <class S, bool EDGES>
__global__ __launch_bounds__(1024) void k_gen_table(S src) {
  int sc, one;
  if (!src.locate(STG_SCENE, blockIdx.x, sc, one)) return;
  const Dev& d = src.scene(sc);
  if (EDGES) {
    for (int i = threadIdx.x; i < d.nv; i += blockDim.x) ingest_vertex(d, i);
    __syncthreads();
  }
  __shared__ int wave_tot[16];
  __shared__ int running;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int np = d.np, ns = d.ns, nv = d.nv;
  // the generator visibility matrix is filled by atomic ORs: clear it
  for (size_t k = tid; k < (size_t)d.Gmax * d.RW; k += blockDim.x) d.vis[k] = 0;
  for (int g = tid; g < np + ns; g += blockDim.x) {
    GenRec r = {};
    r.id = g;
    r.vtx = -1;
    if (g < np) {
      r.kind = SPM_GEN_POINT;
      r.x = r.x2 = 2 * d.pts[2 * g];
      r.y = r.y2 = 2 * d.pts[2 * g + 1];
    } else {
      const int k = g - np;
      r.kind = SPM_GEN_SEGMENT;
      r.x = 2 * d.segs[4 * k];
      r.y = 2 * d.segs[4 * k + 1];
      r.x2 = 2 * d.segs[4 * k + 2];
      r.y2 = 2 * d.segs[4 * k + 3];
    }
    r.ux = r.nx = r.x;
    r.uy = r.ny = r.y;
    d.gens[g] = r;
    d.gen_kind[g] = r.kind;
    d.gen_xy[4 * g] = r.x / 2;
    d.gen_xy[4 * g + 1] = r.y / 2;
    d.gen_xy[4 * g + 2] = r.x2 / 2;
    d.gen_xy[4 * g + 3] = r.y2 / 2;
  }
  if (tid == 0) running = np + ns;
  __syncthreads();
  for (int base = 0; base < nv; base += blockDim.x) {
    const int i = base + tid;
    const bool f = i < nv && d.convex[i];
    const u64 m = ballot(f);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wv] = __popcll(m);
    __syncthreads();
    int off = running;
    for (int k = 0; k < wv; ++k) off += wave_tot[k];
    if (f) {
      const int g = off + before;
      const EdgeRec e = d.edges_raw[i];
      const EdgeExt x = d.ext_raw[i];
      GenRec r = {};
      r.kind = SPM_GEN_VERTEX;
      r.id = g;
      r.x = r.x2 = e.wx;
      r.y = r.y2 = e.wy;
      r.ux = x.ux; r.uy = x.uy;
      r.nx = e.vx; r.ny = e.vy;
      r.vtx = i;
      d.gens[g] = r;
      d.vtx2gid[i] = g;
      d.gen_kind[g] = SPM_GEN_VERTEX;
      d.gen_xy[4 * g] = d.gen_xy[4 * g + 2] = e.wx / 2;
      d.gen_xy[4 * g + 1] = d.gen_xy[4 * g + 3] = e.wy / 2;
    }
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += wave_tot[k];
      running += t;
    }
    __syncthreads();
  }
  if (tid == 0) {
    d.misc[MISC_G] = running;
    d.misc[MISC_TILE_CTR] = 0;
    d.n_gen[0] = running;
  }
  if (tid < kQueues) d.qctr[tid * kQueueStride] = 0;
  if (tid < kOrderBins) d.obins[tid] = 0;
}

// One wavefront per edge: its rank among the Morton keys, then a scatter into
// sorted order.  Any edge order gives the same result; the sort only makes
// each chunk of consecutive edges spatially compact for culling.
template <class S>
__device__ __forceinline__ void edge_rank_wave(const S& src, int wid) {
  int sc, w;
  if (!src.locate(STG_EDGE, wid, sc, w)) return;
  const Dev& d = src.scene(sc);
  const int lane = lane_id();
  const int E = d.E;
  const u64 k = d.keys[w];
  int cnt = 0;
  for (int j = lane; j - lane < E; j += 64) {
    bool lt = j < E && d.keys[j] < k;
    cnt += __popcll(ballot(lt));
  }
  if (lane == 0) {
    d.edges[cnt] = d.edges_raw[w];
    d.ext[cnt] = d.ext_raw[w];
    d.vsorted[cnt] = w;
  }
}

// One workgroup per scene: the spatial generator order used by the
// generator-graph kernels.  Sources keep their ids as positions; then come the
// convex corners in the Morton order of their outgoing edges.
template <class S>
__device__ __forceinline__ void gorder_block(const S& src, int item, int* wave_tot, int& running) {
  int sc, one;
  if (!src.locate(STG_SCENE, item, sc, one)) return;
  const Dev& d = src.scene(sc);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nsrc = d.np + d.ns, E = d.E;
  for (int g = tid; g < nsrc; g += blockDim.x) d.gorder[g] = g;
  if (tid == 0) running = nsrc;
  __syncthreads();
  for (int base = 0; base < E; base += blockDim.x) {
    const int s = base + tid;
    int vi = -1;
    if (s < E) vi = d.vsorted[s];
    const bool f = vi >= 0 && d.convex[vi];
    const u64 m = ballot(f);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wv] = __popcll(m);
    __syncthreads();
    int off = running;
    for (int k = 0; k < wv; ++k) off += wave_tot[k];
    if (f) d.gorder[off + before] = d.vtx2gid[vi];
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += wave_tot[k];
      running += t;
    }
    __syncthreads();
  }
}

// One wavefront per chunk of kChunk sorted edges (one edge per lane): the
// bounding box of their endpoints.
template <class S>
__device__ __forceinline__ void chunk_box_wave(const S& src, int wid) {
  int sc, c;
  if (!src.locate(STG_CHUNK, wid, sc, c)) return;
  const Dev& d = src.scene(sc);
  const int e = c * kChunk + lane_id();
  int x0 = 1 << 30, y0 = 1 << 30, x1 = -(1 << 30), y1 = -(1 << 30);
  if (e < d.E) {
    const EdgeRec r = d.edges[e];
    x0 = min(r.wx, r.vx);
    x1 = max(r.wx, r.vx);
    y0 = min(r.wy, r.vy);
    y1 = max(r.wy, r.vy);
  }
  x0 = wave_min_i(x0);
  y0 = wave_min_i(y0);
  x1 = wave_max_i(x1);
  y1 = wave_max_i(y1);
  if (lane_id() == 0) d.chunks[c] = make_int4(x0, y0, x1, y1);
}

__device__ __forceinline__ int floor_div(int a, int b) {  // b > 0
  int q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
}

// One wavefront per pixel row: the closed inside-obstacle mask.  The row's
// centre line y = 2j + 1 is odd and every vertex y is even, so the line never
// passes through a vertex; each edge crossing it toggles the parity of the
// pixels to its left, and a centre exactly on an edge counts as inside.
// Toggles and on-edge centres are bits in the wavefront's own LDS words
// (lds: 2 * TW of them, TW = (W + 32) / 32), merged by LDS atomics; pixel i is
// inside iff the toggles at positions above i have odd parity, found per word
// by a shift-xor suffix scan plus the parity of the later words (a ballot over
// the lanes, each owning a run of words).
__device__ __forceinline__ void lds_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <class S>
__device__ __forceinline__ void inside_row_wave(const S& src, int wid, unsigned* lds) {
  int sc, j;
  if (!src.locate(STG_ROW, wid, sc, j)) return;
  const Dev& d = src.scene(sc);
  const int W = d.W, E = d.E, W32 = d.W32;
  const int TW = (W + 32) >> 5;   // words of toggle positions 0..W
  unsigned* tog = lds;
  unsigned* on = lds + TW;
  const int lane = lane_id();
  for (int k = lane; k < TW; k += 64) { tog[k] = 0u; on[k] = 0u; }
  lds_wave_sync();
  const int y = 2 * j + 1;
  for (int e = lane; e < E; e += 64) {
    const EdgeRec r = d.edges_raw[e];
    if ((r.wy > y) == (r.vy > y)) continue;
    // crossing x = N / Dn; |N| < 2^30 in doubled coordinates
    int Dn = r.vy - r.wy;
    int N = r.wx * Dn + (y - r.wy) * (r.vx - r.wx);
    if (Dn < 0) { Dn = -Dn; N = -N; }
    const int f = floor_div(N - 1, Dn);       // largest integer strictly left of the crossing
    int cnt = floor_div(f + 1, 2);            // pixels i with 2i + 1 < crossing
    cnt = cnt < 0 ? 0 : (cnt > W ? W : cnt);
    atomicXor(&tog[cnt >> 5], 1u << (cnt & 31));
    if (N >= 0 && N % Dn == 0) {
      const int xc = N / Dn;
      if (xc & 1) {
        const int i = (xc - 1) / 2;
        if (i >= 0 && i < W) atomicOr(&on[i >> 5], 1u << (i & 31));
      }
    }
  }
  lds_wave_sync();
  const int per = (TW + 63) >> 6;
  const int k0 = min(lane * per, TW), k1 = min(k0 + per, TW);
  unsigned par = 0u;
  for (int k = k0; k < k1; ++k) par ^= (unsigned)__popc(tog[k]) & 1u;
  const u64 pm = ballot(par != 0u);
  unsigned c = lane < 63 ? ((unsigned)__popcll(pm >> (lane + 1)) & 1u) : 0u;   // parity of later lanes' words
  for (int k = k1 - 1; k >= k0; --k) {
    const unsigned t = tog[k];
    unsigned x = t >> 1;   // bit b: xor of toggles b + 1 .. 31 of this word, after the scan
    x ^= x >> 1; x ^= x >> 2; x ^= x >> 4; x ^= x >> 8; x ^= x >> 16;
    if (c) x = ~x;
    if (k < W32) {
      unsigned bits = x | on[k];
      const int rem = W - k * 32;
      if (rem < 32) bits &= (1u << rem) - 1u;
      d.inside[(size_t)j * W32 + k] = bits;
    }
    c ^= (unsigned)__popc(t) & 1u;
  }
}

static inline unsigned blocks_for(long long items, int per_block) {
  return (unsigned)((items + per_block - 1) / per_block);
}

// Two independent steps in one launch: the first nrank workgroups rank the
// edges (one wavefront per edge), the others build the inside mask (one
// wavefront per pixel row, from the raw edges; lds_words LDS words each).
template <class S>
__global__ __launch_bounds__(256) void k_rank_inside(S src, int nrank, int lds_words) {
  extern __shared__ unsigned shw[];
  const int wv = threadIdx.x >> 6;
  if ((int)blockIdx.x < nrank) edge_rank_wave(src, blockIdx.x * 4 + wv);
  else inside_row_wave(src, ((int)blockIdx.x - nrank) * 4 + wv, shw + wv * lds_words);
}

// Two independent steps on the sorted edges in one launch: the first
// ngorder workgroups order the generators (one per scene), the others box the
// edge chunks (one wavefront per chunk).
template <class S>
__global__ __launch_bounds__(1024) void k_gorder_boxes(S src, int ngorder) {
  __shared__ int wave_tot[16];
  __shared__ int running;
  if ((int)blockIdx.x < ngorder) gorder_block(src, blockIdx.x, wave_tot, running);
  else chunk_box_wave(src, (blockIdx.x - ngorder) * 16 + (threadIdx.x >> 6));
}

template <class S>
hipError_t launch_ingest(const S& src, const Plan& p, hipStream_t s) {
  if (p.maxE <= kIngestFuseMax) {
    hipLaunchKernelGGL((k_gen_table<S, true>), dim3((unsigned)p.total[STG_SCENE]), dim3(1024), 0, s, src);
    return hipGetLastError();
  }
  if (p.total[STG_VTX] > 0)
    hipLaunchKernelGGL(k_ingest_edges<S>, dim3(blocks_for(p.total[STG_VTX], 256)), dim3(256), 0, s, src);
  hipLaunchKernelGGL((k_gen_table<S, false>), dim3((unsigned)p.total[STG_SCENE]), dim3(1024), 0, s, src);
  return hipGetLastError();
}

// Stage "edge sort": edge ranks and the inside mask.
template <class S>
hipError_t launch_edge_sort(const S& src, const Plan& p, hipStream_t s) {
  const unsigned nrank = p.total[STG_EDGE] > 0 ? blocks_for(p.total[STG_EDGE], 4) : 0u;
  const int lds_words = 2 * ((p.maxW + 32) >> 5);
  const size_t shm = 4 * (size_t)lds_words * sizeof(unsigned);
  hipLaunchKernelGGL(k_rank_inside<S>, dim3(nrank + blocks_for(p.total[STG_ROW], 4)), dim3(256), shm, s, src,
                     (int)nrank, lds_words);
  return hipGetLastError();
}

// Stage "generator order": the spatial generator order and the chunk boxes.
template <class S>
hipError_t launch_gorder(const S& src, const Plan& p, hipStream_t s) {
  const unsigned ng = (unsigned)p.total[STG_SCENE];
  const unsigned nb = p.total[STG_CHUNK] > 0 ? blocks_for(p.total[STG_CHUNK], 16) : 0u;
  hipLaunchKernelGGL(k_gorder_boxes<S>, dim3(ng + nb), dim3(1024), 0, s, src, (int)ng);
  return hipGetLastError();
}

template hipError_t launch_ingest<SingleSrc>(const SingleSrc&, const Plan&, hipStream_t);
template hipError_t launch_ingest<BatchSrc>(const BatchSrc&, const Plan&, hipStream_t);
template hipError_t launch_edge_sort<SingleSrc>(const SingleSrc&, const Plan&, hipStream_t);
template hipError_t launch_edge_sort<BatchSrc>(const BatchSrc&, const Plan&, hipStream_t);
template hipError_t launch_gorder<SingleSrc>(const SingleSrc&, const Plan&, hipStream_t);
template hipError_t launch_gorder<BatchSrc>(const BatchSrc&, const Plan&, hipStream_t);

}  // namespace spm
