// k_ingest.hip -- device-side scene ingest for libspm.
//
// Builds, from the caller's device arrays, everything the later stages read:
// doubled-coordinate edge records with their line functions, the generator
// table (the paper's DataArray, Section 3: sources first, then the obstacle
// corners a path can bend at), a spatially sorted copy of the edges cut into
// chunks with bounding boxes, and the closed inside-obstacle mask of the
// pixel grid (pixel centres on or inside an obstacle get no distance).
#include "spm_internal.hpp"

namespace spm {

// One thread per obstacle vertex i: the edge i -> next(i), its neighbours,
// the corner's convexity and a Morton key of the edge midpoint.
__global__ void k_ingest_edges(int nv, int n_polys, const int* __restrict__ poly_start,
                               const int* __restrict__ vx, const int* __restrict__ vy,
                               EdgeRec* __restrict__ edges_raw, EdgeExt* __restrict__ ext_raw,
                               int* __restrict__ convex, u64* __restrict__ keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  int lo = 0, hi = n_polys - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (poly_start[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  const int a = poly_start[lo], b = poly_start[lo + 1];
  const int ip = (i == a) ? b - 1 : i - 1;
  const int in = (i == b - 1) ? a : i + 1;
  const int inn = (in == b - 1) ? a : in + 1;
  const int wx = 2 * vx[i], wy = 2 * vy[i];
  const int nx = 2 * vx[in], ny = 2 * vy[in];
  const int ux = 2 * vx[ip], uy = 2 * vy[ip];
  EdgeRec r;
  r.wx = wx; r.wy = wy; r.vx = nx; r.vy = ny;
  r.a = wy - ny;
  r.b = nx - wx;
  r.c = -(r.a * wx + r.b * wy);
  r.nc = -r.c;
  edges_raw[i] = r;
  EdgeExt x;
  x.ux = ux; x.uy = uy; x.nx = 2 * vx[inn]; x.ny = 2 * vy[inn];
  ext_raw[i] = x;
  convex[i] = ((wx - ux) * (ny - wy) - (wy - uy) * (nx - wx)) > 0 ? 1 : 0;
  // Morton code of the midpoint (15 bits per axis)
  unsigned mx = (unsigned)((wx + nx) >> 1) & 0x7fffu, my = (unsigned)((wy + ny) >> 1) & 0x7fffu;
  unsigned code = 0;
  for (int k = 0; k < 15; ++k) code |= (((mx >> k) & 1u) << (2 * k)) | (((my >> k) & 1u) << (2 * k + 1));
  keys[i] = ((u64)code << 32) | (u64)(unsigned)i;
}

// Single workgroup: the canonical generator table.  Points, then segments,
// then every convex corner (left turn) in vertex order; ids by a block scan.
__global__ __launch_bounds__(1024) void k_gen_table(int np, int ns, int nv, int n_polys,
                                                    const int* __restrict__ pts, const int* __restrict__ segs,
                                                    const EdgeRec* __restrict__ edges_raw,
                                                    const EdgeExt* __restrict__ ext_raw,
                                                    const int* __restrict__ convex, GenRec* __restrict__ gens,
                                                    int* __restrict__ misc, int* __restrict__ n_gen,
                                                    int* __restrict__ gen_kind, int* __restrict__ gen_xy,
                                                    int* __restrict__ vtx2gid) {
  __shared__ int wave_tot[16];
  __shared__ int running;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  for (int g = tid; g < np + ns; g += blockDim.x) {
    GenRec r = {};
    r.id = g;
    r.vtx = -1;
    if (g < np) {
      r.kind = SPM_GEN_POINT;
      r.x = r.x2 = 2 * pts[2 * g];
      r.y = r.y2 = 2 * pts[2 * g + 1];
    } else {
      const int k = g - np;
      r.kind = SPM_GEN_SEGMENT;
      r.x = 2 * segs[4 * k];
      r.y = 2 * segs[4 * k + 1];
      r.x2 = 2 * segs[4 * k + 2];
      r.y2 = 2 * segs[4 * k + 3];
    }
    r.ux = r.nx = r.x;
    r.uy = r.ny = r.y;
    gens[g] = r;
    gen_kind[g] = r.kind;
    gen_xy[4 * g] = r.x / 2;
    gen_xy[4 * g + 1] = r.y / 2;
    gen_xy[4 * g + 2] = r.x2 / 2;
    gen_xy[4 * g + 3] = r.y2 / 2;
  }
  if (tid == 0) running = np + ns;
  __syncthreads();
  for (int base = 0; base < nv; base += blockDim.x) {
    const int i = base + tid;
    const bool f = i < nv && convex[i];
    const u64 m = ballot(f);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wv] = __popcll(m);
    __syncthreads();
    int off = running;
    for (int k = 0; k < wv; ++k) off += wave_tot[k];
    if (f) {
      const int g = off + before;
      const EdgeRec e = edges_raw[i];
      const EdgeExt x = ext_raw[i];
      GenRec r = {};
      r.kind = SPM_GEN_VERTEX;
      r.id = g;
      r.x = r.x2 = e.wx;
      r.y = r.y2 = e.wy;
      r.ux = x.ux; r.uy = x.uy;
      r.nx = e.vx; r.ny = e.vy;
      r.vtx = i;
      gens[g] = r;
      vtx2gid[i] = g;
      gen_kind[g] = SPM_GEN_VERTEX;
      gen_xy[4 * g] = gen_xy[4 * g + 2] = e.wx / 2;
      gen_xy[4 * g + 1] = gen_xy[4 * g + 3] = e.wy / 2;
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
    misc[MISC_G] = running;
    n_gen[0] = running;
  }
}

// One wavefront per edge: its rank among the Morton keys, then a scatter into
// sorted order.  Any edge order gives the same result; the sort only makes
// each chunk of consecutive edges spatially compact for culling.
__global__ __launch_bounds__(256) void k_edge_rank(int E, const u64* __restrict__ keys,
                                                   const EdgeRec* __restrict__ edges_raw,
                                                   const EdgeExt* __restrict__ ext_raw, EdgeRec* __restrict__ edges,
                                                   EdgeExt* __restrict__ ext, int* __restrict__ vsorted) {
  const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= E) return;
  const int lane = lane_id();
  const u64 k = keys[w];
  int cnt = 0;
  for (int j = lane; j - lane < E; j += 64) {
    bool lt = j < E && keys[j] < k;
    cnt += __popcll(ballot(lt));
  }
  if (lane == 0) {
    edges[cnt] = edges_raw[w];
    ext[cnt] = ext_raw[w];
    vsorted[cnt] = w;
  }
}

// Single workgroup: the spatial generator order used by the generator graph
// kernels.  Sources keep their ids as positions; then come the convex corners
// in the Morton order of their outgoing edges.
__global__ __launch_bounds__(1024) void k_gorder(int nsrc, int E, const int* __restrict__ vsorted,
                                                 const int* __restrict__ convex, const int* __restrict__ vtx2gid,
                                                 int* __restrict__ gorder) {
  __shared__ int wave_tot[16];
  __shared__ int running;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int g = tid; g < nsrc; g += blockDim.x) gorder[g] = g;
  if (tid == 0) running = nsrc;
  __syncthreads();
  for (int base = 0; base < E; base += blockDim.x) {
    const int s = base + tid;
    int vi = -1;
    if (s < E) vi = vsorted[s];
    const bool f = vi >= 0 && convex[vi];
    const u64 m = ballot(f);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wv] = __popcll(m);
    __syncthreads();
    int off = running;
    for (int k = 0; k < wv; ++k) off += wave_tot[k];
    if (f) gorder[off + before] = vtx2gid[vi];
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += wave_tot[k];
      running += t;
    }
    __syncthreads();
  }
}

// One thread per chunk of kChunk sorted edges: bounding box of its endpoints.
__global__ void k_chunk_boxes(int E, int NC, const EdgeRec* __restrict__ edges, int4* __restrict__ chunks) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= NC) return;
  int x0 = 1 << 30, y0 = 1 << 30, x1 = -(1 << 30), y1 = -(1 << 30);
  const int e1 = min((c + 1) * kChunk, E);
  for (int e = c * kChunk; e < e1; ++e) {
    const EdgeRec r = edges[e];
    x0 = min(x0, min(r.wx, r.vx));
    x1 = max(x1, max(r.wx, r.vx));
    y0 = min(y0, min(r.wy, r.vy));
    y1 = max(y1, max(r.wy, r.vy));
  }
  chunks[c] = make_int4(x0, y0, x1, y1);
}

__device__ __forceinline__ long long floor_div(long long a, long long b) {  // b > 0
  long long q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
}

// One workgroup per pixel row: the closed inside-obstacle mask.  The row's
// centre line y = 2j + 1 is odd and every vertex y is even, so the line never
// passes through a vertex; each edge crossing it toggles the parity of the
// pixels to its left, and a centre exactly on an edge counts as inside.
__global__ __launch_bounds__(256) void k_inside(int W, int H, int E, int W32, const EdgeRec* __restrict__ edges,
                                                unsigned* __restrict__ inside) {
  extern __shared__ int sh[];
  int* tog = sh;                    // [W + 1]
  unsigned char* on = (unsigned char*)(sh + W + 1);   // [W]
  __shared__ int part[256];
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const long long y = 2 * j + 1;
  for (int k = tid; k <= W; k += blockDim.x) tog[k] = 0;
  for (int k = tid; k < W; k += blockDim.x) on[k] = 0;
  __syncthreads();
  for (int e = tid; e < E; e += blockDim.x) {
    const EdgeRec r = edges[e];
    if ((r.wy > y) == (r.vy > y)) continue;
    long long Dn = r.vy - r.wy;
    long long N = (long long)r.wx * Dn + (y - r.wy) * (long long)(r.vx - r.wx);
    if (Dn < 0) { Dn = -Dn; N = -N; }
    const long long f = floor_div(N - 1, Dn);       // largest integer strictly left of the crossing
    long long cnt = floor_div(f + 1, 2);            // pixels i with 2i + 1 < crossing
    cnt = cnt < 0 ? 0 : (cnt > W ? W : cnt);
    atomicXor(&tog[cnt], 1);
    if (N >= 0 && N % Dn == 0) {
      const long long xc = N / Dn;
      if (xc & 1) {
        const long long i = (xc - 1) / 2;
        if (i >= 0 && i < W) on[i] = 1;
      }
    }
  }
  __syncthreads();
  // suffix xor: inside(i) = xor of tog[k] for k > i
  const int per = (W + 1 + blockDim.x - 1) / blockDim.x;
  const int k0 = tid * per, k1 = min(k0 + per, W + 1);
  int x = 0;
  for (int k = k0; k < k1; ++k) x ^= tog[k];
  part[tid] = x;
  __syncthreads();
  int acc = 0;
  for (int t = tid + 1; t < (int)blockDim.x; ++t) acc ^= part[t];
  for (int k = k1 - 1; k >= k0; --k) {
    const int nxt = acc;     // xor of tog[m] for m > k
    acc ^= tog[k];
    tog[k] = nxt;            // now tog[k] = xor over m > k
  }
  __syncthreads();
  for (int wd = tid; wd < W32; wd += blockDim.x) {
    unsigned bits = 0;
    for (int b = 0; b < 32; ++b) {
      const int i = wd * 32 + b;
      if (i < W && ((tog[i] & 1) || on[i])) bits |= 1u << b;
    }
    inside[(size_t)j * W32 + wd] = bits;
  }
}

hipError_t launch_ingest(const Dev& d, hipStream_t s) {
  if (d.nv > 0) {
    hipLaunchKernelGGL(k_ingest_edges, dim3((d.nv + 255) / 256), dim3(256), 0, s, d.nv, d.n_polys, d.poly_start,
                       d.vx, d.vy, d.edges_raw, d.ext_raw, d.convex, d.keys);
  }
  hipLaunchKernelGGL(k_gen_table, dim3(1), dim3(1024), 0, s, d.np, d.ns, d.nv, d.n_polys, d.pts, d.segs,
                     d.edges_raw, d.ext_raw, d.convex, d.gens, d.misc, d.n_gen, d.gen_kind, d.gen_xy, d.vtx2gid);
  return hipGetLastError();
}

hipError_t launch_edge_sort(const Dev& d, hipStream_t s) {
  if (d.E == 0) {
    hipLaunchKernelGGL(k_gorder, dim3(1), dim3(1024), 0, s, d.np + d.ns, 0, d.vsorted, d.convex, d.vtx2gid,
                       d.gorder);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_edge_rank, dim3((d.E + 3) / 4), dim3(256), 0, s, d.E, d.keys, d.edges_raw, d.ext_raw,
                     d.edges, d.ext, d.vsorted);
  hipLaunchKernelGGL(k_gorder, dim3(1), dim3(1024), 0, s, d.np + d.ns, d.E, d.vsorted, d.convex, d.vtx2gid,
                     d.gorder);
  hipLaunchKernelGGL(k_chunk_boxes, dim3((d.NC + 127) / 128), dim3(128), 0, s, d.E, d.NC, d.edges, d.chunks);
  return hipGetLastError();
}

hipError_t launch_inside(const Dev& d, hipStream_t s) {
  const size_t shm = (size_t)(d.W + 1) * sizeof(int) + (size_t)d.W + 16;
  hipLaunchKernelGGL(k_inside, dim3(d.H), dim3(256), shm, s, d.W, d.H, d.E, d.W32, d.edges_raw, d.inside);
  return hipGetLastError();
}

}  // namespace spm
