"""Python face of libspm: device scenes, builds, timers and path queries.

PyTorch supplies device memory and streams; every step of a build runs in the
library's HIP kernels (see include/spm.h for the contract of each call).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as C


def _host_scene_struct(flat: dict, keep: list) -> C.SpmScene:
    arrs = {k: np.ascontiguousarray(flat[k], np.int32) for k in ("poly_start", "vx", "vy", "pts", "segs")}
    keep.append(arrs)

    def p(a):
        return a.ctypes.data if a.size else None

    n_polys = len(arrs["poly_start"]) - 1
    return C.SpmScene(int(flat["width"]), int(flat["height"]), n_polys, int(arrs["vx"].size),
                      int(arrs["pts"].size // 2), int(arrs["segs"].size // 4), p(arrs["poly_start"]),
                      p(arrs["vx"]), p(arrs["vy"]), p(arrs["pts"]), p(arrs["segs"]))


def validate(scene) -> None:
    """Exact host-side check of a scene (raises SpmError with the reason)."""
    keep = []
    s = _host_scene_struct(scene.flat(), keep)
    C.check(C.lib().spm_validate(ctypes.byref(s)))


def query_sizes(width, height, n_polys, n_vertices, n_points, n_segs):
    s = C.SpmScene(width, height, n_polys, n_vertices, n_points, n_segs, None, None, None, None, None)
    mg = C.c_i32(0)
    ws = ctypes.c_size_t(0)
    C.check(C.lib().spm_query_sizes(ctypes.byref(s), ctypes.byref(mg), ctypes.byref(ws)))
    return int(mg.value), int(ws.value)


class DeviceScene:
    """A scene uploaded to device memory (int32 tensors) plus its C descriptor."""

    def __init__(self, scene, device="cuda", check: bool = True):
        if check:
            validate(scene)
        f = scene.flat()
        self.width, self.height = int(f["width"]), int(f["height"])
        self.scene = scene

        def up(a):
            a = np.ascontiguousarray(a, np.int32)
            return torch.from_numpy(a if a.size else np.zeros(1, np.int32)).to(device)

        self.t = {k: up(f[k]) for k in ("poly_start", "vx", "vy", "pts", "segs")}
        self.n_polys = len(f["poly_start"]) - 1
        self.n_vertices = int(f["vx"].size)
        self.n_points = int(f["pts"].size // 2)
        self.n_segs = int(f["segs"].size // 4)
        self.c = C.SpmScene(self.width, self.height, self.n_polys, self.n_vertices, self.n_points, self.n_segs,
                            self.t["poly_start"].data_ptr(), self.t["vx"].data_ptr(), self.t["vy"].data_ptr(),
                            self.t["pts"].data_ptr(), self.t["segs"].data_ptr())

    @property
    def sizes(self):
        return query_sizes(self.width, self.height, self.n_polys, self.n_vertices, self.n_points, self.n_segs)


@dataclass
class Map:
    dist: torch.Tensor        # (H, W) float32
    parent: torch.Tensor      # (H, W) int32
    gen_kind: torch.Tensor    # (max_gen,) int32
    gen_xy: torch.Tensor      # (max_gen, 4) int32
    gen_cost: torch.Tensor    # (max_gen,) float64
    gen_parent: torch.Tensor  # (max_gen,) int32
    n_gen: torch.Tensor       # (1,) int32

    def host(self) -> dict:
        G = int(self.n_gen.item())
        return {
            "dist": self.dist.cpu().numpy(), "parent": self.parent.cpu().numpy(), "n_gen": G,
            "gen_kind": self.gen_kind[:G].cpu().numpy(), "gen_xy": self.gen_xy[:G].cpu().numpy(),
            "gen_cost": self.gen_cost[:G].cpu().numpy(), "gen_parent": self.gen_parent[:G].cpu().numpy(),
        }


class Timer:
    """Per-stage HIP-event timing of builds (stage names in _lib.STAGES)."""

    def __init__(self):
        h = ctypes.c_void_p()
        C.check(C.lib().spm_timer_create(ctypes.byref(h)))
        self.h = h

    def reset(self):
        C.check(C.lib().spm_timer_reset(self.h))

    def elapsed(self):
        ms = (ctypes.c_float * C.SPM_N_STAGES)()
        n = C.c_i32(0)
        C.check(C.lib().spm_timer_elapsed(self.h, ms, ctypes.byref(n)))
        return {name: float(ms[k]) for k, name in enumerate(C.STAGES)}, int(n.value)

    def __del__(self):
        try:
            C.lib().spm_timer_destroy(self.h)
        except Exception:
            pass


class Builder:
    """Owns the outputs and workspace of one scene's builds.

    tile: pixel tile of one wavefront; strip: tiles per work item (0 = library
    default); samples: seed searches per tile (0 = default, -1 = none); walk:
    how tiles go through the generators (0 = by generator count, 1 = register
    cache, 2 = refilled cache, 3 = seed searches and cost order, 4 = spatial clusters).  strip,
    samples and walk change speed only."""

    def __init__(self, dscene: DeviceScene, tile=(8, 8), strip: int = 0, samples: int = 0, walk: int = 0):
        self.ds = dscene
        dev = dscene.t["vx"].device
        self.max_gen, self.ws_bytes = dscene.sizes
        H, W = dscene.height, dscene.width
        G = max(self.max_gen, 1)
        self.map = Map(
            dist=torch.empty((H, W), dtype=torch.float32, device=dev),
            parent=torch.empty((H, W), dtype=torch.int32, device=dev),
            gen_kind=torch.empty((G,), dtype=torch.int32, device=dev),
            gen_xy=torch.empty((G, 4), dtype=torch.int32, device=dev),
            gen_cost=torch.empty((G,), dtype=torch.float64, device=dev),
            gen_parent=torch.empty((G,), dtype=torch.int32, device=dev),
            n_gen=torch.empty((1,), dtype=torch.int32, device=dev),
        )
        self.ws = torch.empty((self.ws_bytes,), dtype=torch.uint8, device=dev)
        m = self.map
        self.out = C.SpmOut(m.dist.data_ptr(), m.parent.data_ptr(), m.gen_kind.data_ptr(), m.gen_xy.data_ptr(),
                            m.gen_cost.data_ptr(), m.gen_parent.data_ptr(), m.n_gen.data_ptr())
        self.tile = tuple(tile)
        self.strip = int(strip)
        self.samples = int(samples)
        self.walk = int(walk)

    def build_host(self, scene=None, stream=None) -> Map:
        """Queue one build through spm_build from a host scene (default: the scene this builder's device
        scene was made from): the library validates it, stages it through pinned memory into the
        workspace and builds from there.  The scene must have the same counts as the device scene."""
        keep = []
        hs = _host_scene_struct((scene if scene is not None else self.ds.scene).flat(), keep)
        for f in ("width", "height", "n_polys", "n_vertices", "n_points", "n_segs"):
            if getattr(hs, f) != getattr(self.ds.c, f):
                raise ValueError(f"scene {f} {getattr(hs, f)} differs from the builder's {getattr(self.ds.c, f)}")
        if stream is not None:
            handle = stream.cuda_stream
        elif self.ws.device.type == "cuda":
            handle = torch.cuda.current_stream(self.ws.device).cuda_stream
        else:
            handle = 0   # not a device buffer: the library's host checks run, and no build can follow
        C.check(C.lib().spm_build(ctypes.byref(hs), ctypes.byref(self.out), self.ws.data_ptr(), self.ws_bytes,
                                  ctypes.c_void_p(handle)))
        return self.map

    def build_noalloc(self, stream=None) -> Map:
        """Queue one build of the device scene through spm_build_noalloc: the library's static device
        workspace instead of this builder's (nothing is allocated; calls on one GPU share it)."""
        if stream is None:
            stream = torch.cuda.current_stream(self.ws.device)
        C.check(C.lib().spm_build_noalloc(ctypes.byref(self.ds.c), ctypes.byref(self.out),
                                          ctypes.c_void_p(stream.cuda_stream)))
        return self.map

    def build(self, stream=None, timer: Timer = None, stats: torch.Tensor = None) -> Map:
        """Queue one build of the device scene through spm_build_ex on `stream` (default: torch's
        current stream)."""
        if stream is None:
            stream = torch.cuda.current_stream(self.ws.device)
        opts = C.SpmBuildOpts(self.tile[0], self.tile[1], timer.h if timer is not None else None,
                              stats.data_ptr() if stats is not None else None, self.strip, self.samples,
                              self.walk)
        C.check(C.lib().spm_build_ex(ctypes.byref(self.ds.c), ctypes.byref(self.out), self.ws.data_ptr(),
                                     self.ws_bytes, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(opts)))
        return self.map


def agent_distance(builder: Builder, agents: torch.Tensor, stream=None) -> torch.Tensor:
    """D(a) for agents (n, 2) float32 on the device, read from the builder's last map."""
    agents = agents.contiguous().to(torch.float32)
    n = agents.shape[0]
    out = torch.empty((n,), dtype=torch.float32, device=agents.device)
    if stream is None:
        stream = torch.cuda.current_stream(agents.device)
    C.check(C.lib().spm_agent_distance(ctypes.byref(builder.ds.c), ctypes.byref(builder.out), n,
                                       agents.data_ptr() if n else None, out.data_ptr() if n else None,
                                       ctypes.c_void_p(stream.cuda_stream)))
    return out


def query_points(builder: Builder, pts: torch.Tensor, cap: int = 0, stream=None):
    """Refined map values at arbitrary points (n, 2) float32 on the device: the least cost + distance
    among the 3 x 3 neighbouring pixels' parents that each point sees.  Returns (dist, parent) and,
    with cap > 0, also (path_xy (n, cap, 2), path_n (n,)): each point's whole path."""
    pts = pts.contiguous().to(torch.float32)
    n = pts.shape[0]
    dev = pts.device
    dist = torch.empty((n,), dtype=torch.float32, device=dev)
    par = torch.empty((n,), dtype=torch.int32, device=dev)
    pxy = torch.empty((n, max(cap, 1), 2), dtype=torch.float32, device=dev) if cap > 0 else None
    pn = torch.empty((n,), dtype=torch.int32, device=dev) if cap > 0 else None
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    C.check(C.lib().spm_query_points(ctypes.byref(builder.ds.c), ctypes.byref(builder.out), n,
                                     pts.data_ptr() if n else None, dist.data_ptr() if n else None,
                                     par.data_ptr() if n else None, int(cap),
                                     pxy.data_ptr() if (pxy is not None and n) else None,
                                     pn.data_ptr() if (pn is not None and n) else None,
                                     ctypes.c_void_p(stream.cuda_stream)))
    if cap > 0:
        return dist, par, pxy, pn
    return dist, par


def source_gradients(builder: Builder, agents: torch.Tensor, dL_dD: torch.Tensor, stream=None):
    """Gradients of a loss w.r.t. the point sources (n_points, 2) and the segment endpoints
    (n_segs, 4), given dL/dD per agent, through the builder's last map."""
    agents = agents.contiguous().to(torch.float32)
    dL_dD = dL_dD.contiguous().to(torch.float32)
    n = agents.shape[0]
    ds = builder.ds
    dev = agents.device
    gp = torch.zeros((max(ds.n_points, 1), 2), dtype=torch.float32, device=dev)
    gs = torch.zeros((max(ds.n_segs, 1), 4), dtype=torch.float32, device=dev)
    wsb = ctypes.c_size_t(0)
    C.check(C.lib().spm_agent_query_ws(ctypes.byref(ds.c), n, ctypes.byref(wsb)))
    ws = torch.empty((int(wsb.value),), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    C.check(C.lib().spm_backward(ctypes.byref(ds.c), ctypes.byref(builder.out), n,
                                 agents.data_ptr() if n else None, dL_dD.data_ptr() if n else None,
                                 gp.data_ptr(), gs.data_ptr(), ws.data_ptr(), int(wsb.value),
                                 ctypes.c_void_p(stream.cuda_stream)))
    return gp[:ds.n_points], gs[:ds.n_segs]


class SPMDistance(torch.autograd.Function):
    """D(agents) as a differentiable function of the source positions.

    forward(pts (n_points, 2), segs (n_segs, 4), agents (n, 2), builder): rounds the
    source coordinates to the integer lattice the exact predicates need (so a move of
    less than half a unit leaves the map unchanged), rebuilds the map from the updated
    host scene through spm_build, which validates it first (a source moved onto or into
    an obstacle, out of the domain, or a segment made to touch an obstacle or shrink to
    a point raises SpmError and leaves the builder's scene as it was), and returns D per
    agent.  backward: gradients for pts and segs through the fixed parent chains
    (spm_backward); agents and builder get none.
    """

    @staticmethod
    def forward(ctx, pts, segs, agents, builder):
        ds = builder.ds
        sc = ds.scene
        new_pts = torch.round(pts.detach()).to(torch.int64).cpu().numpy().reshape(-1, 2) if ds.n_points else None
        new_segs = torch.round(segs.detach()).to(torch.int64).cpu().numpy().reshape(-1, 4) if ds.n_segs else None
        moved = type(sc)(sc.width, sc.height, sc.polys, new_pts, new_segs)
        builder.build_host(moved)
        ds.scene = moved
        if ds.n_points:
            ds.t["pts"].copy_(torch.from_numpy(np.ascontiguousarray(new_pts.reshape(-1), np.int32)))
        if ds.n_segs:
            ds.t["segs"].copy_(torch.from_numpy(np.ascontiguousarray(new_segs.reshape(-1), np.int32)))
        D = agent_distance(builder, agents)
        ctx.save_for_backward(agents)
        ctx.builder = builder
        return D

    @staticmethod
    def backward(ctx, gD):
        (agents,) = ctx.saved_tensors
        gp, gs = source_gradients(ctx.builder, agents, gD)
        return gp, gs, None, None


def _alloc_map(H, W, max_gen, dev) -> Map:
    G = max(max_gen, 1)
    return Map(
        dist=torch.empty((H, W), dtype=torch.float32, device=dev),
        parent=torch.empty((H, W), dtype=torch.int32, device=dev),
        gen_kind=torch.empty((G,), dtype=torch.int32, device=dev),
        gen_xy=torch.empty((G, 4), dtype=torch.int32, device=dev),
        gen_cost=torch.empty((G,), dtype=torch.float64, device=dev),
        gen_parent=torch.empty((G,), dtype=torch.int32, device=dev),
        n_gen=torch.empty((1,), dtype=torch.int32, device=dev),
    )


def _out_struct(m: Map) -> C.SpmOut:
    return C.SpmOut(m.dist.data_ptr(), m.parent.data_ptr(), m.gen_kind.data_ptr(), m.gen_xy.data_ptr(),
                    m.gen_cost.data_ptr(), m.gen_parent.data_ptr(), m.n_gen.data_ptr())


class Graph:
    """A batched build captured in a HIP graph (replay with launch())."""

    def __init__(self, handle, owner):
        self.h = handle
        self._owner = owner   # keeps the buffers the graph points at alive

    def launch(self, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        C.check(C.lib().spm_graph_launch(self.h, ctypes.c_void_p(stream.cuda_stream)))

    def __del__(self):
        try:
            C.lib().spm_graph_destroy(self.h)
        except Exception:
            pass


class BatchBuilder:
    """Outputs and workspace for batched builds of many independent scenes.

    tile_w: None (8x8 everywhere), a list of per-scene tile widths (8, 16, 4),
    or a dict {side: tile_w}; pixel_waves: waves per SIMD of the persistent
    pixel launch (0 = as many as fit); walk: 0 = by the largest generator
    count, 1-3 forced.  autotune.tune() returns all three as a dict that can be
    passed as `tuned`.
    """

    def __init__(self, scenes, device="cuda", tile_w=None, check: bool = True, pixel_waves: int = 0, walk: int = 0,
                 tuned: dict = None):
        if tuned is not None:
            tile_w = tuned.get("tile_w", tile_w)
            pixel_waves = int(tuned.get("pixel_waves", pixel_waves))
            walk = int(tuned.get("walk", walk))
        self.ds = [DeviceScene(s, device, check=check) for s in scenes]
        n = len(self.ds)
        if n < 1:
            raise ValueError("empty batch")
        self.maps = []
        for d in self.ds:
            mg, _ = d.sizes
            self.maps.append(_alloc_map(d.height, d.width, mg, d.t["vx"].device))
        if isinstance(tile_w, dict):
            tiles = [int(tile_w.get(max(d.width, d.height), tile_w.get(str(max(d.width, d.height)), 8)))
                     for d in self.ds]
        elif tile_w is None:
            tiles = [8] * n
        else:
            tiles = [int(t) for t in tile_w]
        self.tile_w = tiles
        self._scenes = (C.SpmScene * n)(*[d.c for d in self.ds])
        self._outs = (C.SpmOut * n)(*[_out_struct(m) for m in self.maps])
        self._tiles = (C.c_i32 * n)(*tiles)
        self.pixel_waves = int(pixel_waves)
        self.walk = int(walk)
        self.c = C.SpmBatch(n, self._scenes, self._outs, self._tiles, self.pixel_waves, self.walk)
        ws = ctypes.c_size_t(0)
        C.check(C.lib().spm_batch_query_sizes(ctypes.byref(self.c), ctypes.byref(ws)))
        self.ws_bytes = int(ws.value)
        self.ws = torch.empty((self.ws_bytes,), dtype=torch.uint8, device=self.ds[0].t["vx"].device)
        C.check(C.lib().spm_batch_prepare(ctypes.byref(self.c), self.ws.data_ptr(), self.ws_bytes))

    def set_options(self, pixel_waves: int = None, walk: int = None):
        """Change the pixel launch's waves per SIMD or walk (no new spm_batch_prepare needed)."""
        if pixel_waves is not None:
            self.pixel_waves = self.c.pixel_waves = int(pixel_waves)
        if walk is not None:
            self.walk = self.c.walk = int(walk)

    def build(self, stream=None, timer: Timer = None):
        if stream is None:
            stream = torch.cuda.current_stream(self.ws.device)
        C.check(C.lib().spm_build_batch(ctypes.byref(self.c), self.ws.data_ptr(), self.ws_bytes,
                                        ctypes.c_void_p(stream.cuda_stream), timer.h if timer is not None else None))
        return self.maps

    def capture(self, stream) -> Graph:
        """Capture one batched build on the (non-default) torch stream `stream`."""
        h = ctypes.c_void_p()
        C.check(C.lib().spm_graph_capture_batch(ctypes.byref(self.c), self.ws.data_ptr(), self.ws_bytes,
                                                ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        return Graph(h, self)

    @property
    def pairs(self) -> int:
        """Sum over scenes of W * H * G (needs the generator counts, so it synchronises)."""
        return int(sum(d.width * d.height * int(m.n_gen.item()) for d, m in zip(self.ds, self.maps)))


def build(scene, device="cuda", tile=(8, 8)) -> Map:
    """Upload, build and return the map (device tensors; the build is queued on the current stream)."""
    b = Builder(DeviceScene(scene, device), tile=tile)
    return b.build()


def query_path(host_map: dict, qx: float, qy: float, cap: int = 4096):
    """Path from (qx, qy) to its closest source from a host copy of a map (Map.host()).
    Returns (points (n, 2) float32, length)."""
    keep = {k: np.ascontiguousarray(host_map[k]) for k in ("parent", "gen_kind", "gen_xy", "gen_parent",
                                                           "gen_cost")}
    keep["parent"] = keep["parent"].astype(np.int32, copy=False)
    keep["gen_kind"] = keep["gen_kind"].astype(np.int32, copy=False)
    keep["gen_xy"] = keep["gen_xy"].astype(np.int32, copy=False)
    keep["gen_parent"] = keep["gen_parent"].astype(np.int32, copy=False)
    keep["gen_cost"] = keep["gen_cost"].astype(np.float64, copy=False)
    H, W = keep["parent"].shape
    m = C.SpmMapHost(W, H, keep["parent"].ctypes.data, int(host_map["n_gen"]), keep["gen_kind"].ctypes.data,
                     keep["gen_xy"].ctypes.data, keep["gen_parent"].ctypes.data, keep["gen_cost"].ctypes.data)
    out = np.zeros(2 * cap, np.float32)
    n = C.c_i32(0)
    L = ctypes.c_float(0)
    C.check(C.lib().spm_query_path(ctypes.byref(m), float(qx), float(qy),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), cap, ctypes.byref(n),
                                   ctypes.byref(L)))
    return out[:2 * n.value].reshape(-1, 2), float(L.value)
