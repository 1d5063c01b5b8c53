"""ctypes binding of libradray (include/radray.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Device memory comes from torch tensors on the context's device;
work is enqueued on the torch stream that was current when the context was
created.  There is no CPU fallback: if the library is missing or the device
is not available, the constructor raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libradray.so")

RR_OK, RR_EINVAL, RR_ENOMEM, RR_EHIP, RR_ESTATE, RR_EOVERFLOW, RR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
NOALLOC_MAX_PATHS, NOALLOC_MAX_TX = 65536, 4096
TX_PER_ELEMENT, TX_SHARED = 0, 1
UNIFORM, PROPOSAL, PER_TRIANGLE = 0, 1, 2
EXACT, SEPARABLE = 0, 1
ENGINE_AUTO, DIRECT_FP32, GEMM_BF16X3, GEMM_EXACT = 0, 1, 2, 3
KMAX = 4
ALPHA_PER_OBJECT, ALPHA_PER_TRIANGLE = 0, 1

EXPORTED = [
    "rr_create", "rr_destroy", "rr_last_error", "rr_version", "rr_scene_upload", "rr_set_array",
    "rr_set_chirp", "rr_trace", "rr_trace_rays", "rr_get_path_count", "rr_get_hits",
    "rr_get_paths", "rr_set_paths", "rr_synthesize", "rr_last_kernel_ms", "rr_backproject",
    "rr_max_projection", "rr_scene_set_alpha", "rr_scene_update_vertices", "rr_get_bvh_nodes",
    "rr_set_casting", "rr_casting_pieces", "rr_trace_work", "rr_synthesize_noalloc",
]


class RadrayError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"radray error {code}: {msg}")
        self.code = code


class Chirp(C.Structure):
    _fields_ = [("f0", C.c_double), ("bandwidth", C.c_double), ("t_chirp", C.c_double),
                ("t_rep", C.c_double), ("n_samples", C.c_int32), ("n_chirps", C.c_int32)]


class TraceParams(C.Structure):
    _fields_ = [("n_rays", C.c_int64), ("max_bounces", C.c_int32), ("seed", C.c_uint64),
                ("az_min", C.c_double), ("az_max", C.c_double), ("el_min", C.c_double),
                ("el_max", C.c_double), ("sampler", C.c_int32), ("record_hits", C.c_int32),
                ("path_cap", C.c_int64)]


class Volume(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double), ("step", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class Paths(C.Structure):
    _fields_ = [("src", C.c_void_p), ("K", C.c_void_p), ("ray", C.c_void_p), ("tri", C.c_void_p),
                ("vid", C.c_void_p), ("p", C.c_void_p), ("L", C.c_void_p), ("amp", C.c_void_p),
                ("stride", C.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libradray.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libradray.so not built at {path}: run paper_2307_15412_amd/build.py")
    L = C.CDLL(path)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.rr_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    L.rr_destroy.argtypes = [vp]
    L.rr_destroy.restype = None
    L.rr_last_error.restype = C.c_char_p
    L.rr_version.restype = C.c_char_p
    L.rr_scene_upload.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, i32, vp, vp, vp, i32]
    L.rr_scene_set_alpha.argtypes = [vp, vp, i64, i32]
    L.rr_scene_update_vertices.argtypes = [vp, vp, i64]
    L.rr_get_bvh_nodes.argtypes = [vp, vp, i64, C.POINTER(i64)]
    L.rr_set_array.argtypes = [vp, vp, i32, vp, i32, f64, i32]
    L.rr_set_casting.argtypes = [vp, f64, i32]
    L.rr_casting_pieces.argtypes = [vp, C.POINTER(TraceParams), C.POINTER(i64)]
    L.rr_set_chirp.argtypes = [vp, C.POINTER(Chirp)]
    L.rr_trace.argtypes = [vp, C.POINTER(TraceParams), C.POINTER(i64)]
    L.rr_trace_work.argtypes = [vp, C.POINTER(TraceParams), C.POINTER(i64), vp]
    L.rr_trace_rays.argtypes = [vp, vp, vp, vp, vp, i64, C.c_int32, C.c_uint64, C.c_int32,
                                C.POINTER(i64)]
    L.rr_get_path_count.argtypes = [vp, C.POINTER(i64)]
    L.rr_backproject.argtypes = [vp, vp, i64, C.POINTER(Volume), vp, i64, i32]
    L.rr_max_projection.argtypes = [vp, vp, C.POINTER(Volume), vp, C.c_float]
    L.rr_get_hits.argtypes = [vp, vp, i64]
    L.rr_get_paths.argtypes = [vp, C.POINTER(Paths), C.POINTER(i64)]
    L.rr_set_paths.argtypes = [vp, C.POINTER(Paths), i64]
    L.rr_synthesize.argtypes = [vp, i32, i32, vp, i64, vp, i64]
    L.rr_synthesize_noalloc.argtypes = [vp, i32, vp, i64]
    L.rr_last_kernel_ms.argtypes = [vp, i32, C.POINTER(f64)]
    _lib = L
    return L


def _np(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, (a.ctypes.data if a.size else None)


class Context:
    """One library context on a GPU, bound to the current torch stream."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("radray needs a ROCm GPU; torch.cuda.is_available() is False")
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self._check(self.lib.rr_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.n_paths = None
        self.n_traced = 0
        self.max_bounces = 0
        self.n_ch = self.M = self.K = 0

    def _check(self, rc: int):
        if rc != RR_OK:
            raise RadrayError(rc, self.lib.rr_last_error().decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.rr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- inputs
    def scene_upload(self, verts, tris, tri_obj, obj_alpha, obj_vel, pt_pos=None, pt_vel=None,
                     pt_aperture=None):
        v, pv = _np(verts, np.float32)
        t, pt = _np(tris, np.int32)
        o, po = _np(tri_obj, np.int32)
        a, pa = _np(obj_alpha, np.float32)
        ov, pov = _np(obj_vel, np.float64)
        pp, ppp = _np(np.zeros((0, 3)) if pt_pos is None else pt_pos, np.float64)
        pvv, ppv = _np(np.zeros((0, 3)) if pt_vel is None else pt_vel, np.float64)
        pa2, ppa = _np(np.zeros((0,)) if pt_aperture is None else pt_aperture, np.float64)
        self._check(self.lib.rr_scene_upload(self.h, pv, v.size // 3, pt, po, t.size // 3, pa, pov,
                                             a.size, ppp, ppv, ppa, pp.size // 3))
        self.n_tris = t.size // 3

    def upload(self, scene):
        """Upload an object with verts/tris/tri_obj/obj_alpha/obj_vel/pt_* fields
        (and per-face alpha when its tri_alpha is not None)."""
        self.scene_upload(scene.verts, scene.tris, scene.tri_obj, scene.obj_alpha, scene.obj_vel,
                          scene.pt_pos, scene.pt_vel, scene.pt_aperture)
        ta = getattr(scene, "tri_alpha", None)
        if ta is not None:
            self.set_alpha(ta, per=ALPHA_PER_TRIANGLE)

    def update_vertices(self, verts):
        """Move the scene's vertices (same topology); the BVH is refit on the GPU."""
        v, pv = _np(verts, np.float32)
        self._check(self.lib.rr_scene_update_vertices(self.h, pv, v.size // 3))

    def bvh_nodes(self):
        """The BVH node array, float32 [n_nodes][16] (host copy)."""
        n = C.c_int64()
        self._check(self.lib.rr_get_bvh_nodes(self.h, None, 0, C.byref(n)))
        out = np.zeros(n.value, dtype=np.float32)
        self._check(self.lib.rr_get_bvh_nodes(self.h, out.ctypes.data if n.value else None,
                                              n.value, C.byref(n)))
        return out.reshape(-1, 16)

    def set_alpha(self, alpha, per=ALPHA_PER_OBJECT):
        """Replace the scene's material mix (Eq. 3) per object or per face."""
        a, pa = _np(alpha, np.float32)
        self._check(self.lib.rr_scene_set_alpha(self.h, pa, a.size, int(per)))

    def set_array(self, tx, rx, rx_radius=0.25, mode=TX_PER_ELEMENT):
        tx, ptx = _np(tx, np.float64)
        rx, prx = _np(rx, np.float64)
        self._check(self.lib.rr_set_array(self.h, ptx, tx.size // 3, prx, rx.size // 3,
                                          float(rx_radius), int(mode)))
        self.n_tx, self.n_rx, self.mode = tx.size // 3, rx.size // 3, int(mode)
        self.n_ch = self.n_tx * self.n_rx

    def set_casting(self, max_solid_angle=0.0, max_depth=8):
        """Subdivision of the per-triangle launch's triangles into pieces."""
        self._check(self.lib.rr_set_casting(self.h, float(max_solid_angle), int(max_depth)))

    def casting_pieces(self, az_min=-math.pi / 2, az_max=math.pi / 2, el_min=-math.pi / 2,
                       el_max=math.pi / 2) -> int:
        """Number of pieces a per-triangle trace with this field of view casts at."""
        tp = TraceParams(0, 1, 0, az_min, az_max, el_min, el_max, PER_TRIANGLE, 0, 0)
        n = C.c_int64()
        self._check(self.lib.rr_casting_pieces(self.h, C.byref(tp), C.byref(n)))
        return n.value

    def set_chirp(self, f0, bandwidth, t_chirp, t_rep, n_samples, n_chirps):
        ch = Chirp(f0, bandwidth, t_chirp, t_rep, n_samples, n_chirps)
        self._check(self.lib.rr_set_chirp(self.h, C.byref(ch)))
        self.M, self.K = int(n_chirps), int(n_samples)

    # -------------------------------------------------------------- trace
    def trace(self, n_rays, max_bounces=2, seed=0, az_min=-math.pi / 2, az_max=math.pi / 2,
              el_min=-math.pi / 2, el_max=math.pi / 2, sampler=UNIFORM, record_hits=True,
              path_cap=0, sync=True):
        """Returns the number of stored paths; with sync=False the call does
        not wait for the GPU and returns None (the count stays on the device
        until path_count() or a synthesis needs it)."""
        tp = TraceParams(int(n_rays), int(max_bounces), int(seed) & (2**64 - 1), az_min, az_max,
                         el_min, el_max, int(sampler), int(bool(record_hits)), int(path_cap))
        n = C.c_int64()
        self._check(self.lib.rr_trace(self.h, C.byref(tp), C.byref(n) if sync else None))
        self.n_paths = n.value if sync else None
        n_src = 1 if self.mode == TX_SHARED else self.n_tx
        if sampler == PER_TRIANGLE:
            per = self.casting_pieces(az_min, az_max, el_min, el_max) * int(n_rays)
        else:
            per = int(n_rays) if self.mode == TX_SHARED else int(n_rays) // self.n_tx
        self.n_traced = n_src * per
        self.max_bounces = int(max_bounces)
        self.record_hits = bool(record_hits)
        return self.n_paths

    def trace_rays(self, orig, dirs, amp, src, max_bounces=2, seed=0, record_hits=True) -> int:
        """Trace caller-supplied rays: orig, dirs [n][3] and amp [n] as float64,
        src [n] int32 (host or device tensors or arrays)."""
        torch = self.torch
        dev = lambda x, dt: torch.as_tensor(x).to(device=self.device, dtype=dt).contiguous()
        o = dev(orig, torch.float64).reshape(-1, 3)
        d = dev(dirs, torch.float64).reshape(-1, 3)
        a = dev(amp, torch.float64).reshape(-1)
        s = dev(src, torch.int32).reshape(-1)
        n = o.shape[0]
        if d.shape[0] != n or a.shape[0] != n or s.shape[0] != n:
            raise ValueError("orig, dirs, amp and src must have the same number of rays")
        cnt = C.c_int64()
        ptr = lambda t: C.c_void_p(t.data_ptr()) if n else None
        self._check(self.lib.rr_trace_rays(self.h, ptr(o), ptr(d), ptr(a), ptr(s), n,
                                           int(max_bounces), int(seed) & (2**64 - 1),
                                           int(bool(record_hits)), C.byref(cnt)))
        self.n_paths = cnt.value
        self.n_traced = n
        self.max_bounces = int(max_bounces)
        self.record_hits = bool(record_hits)
        return self.n_paths

    def hits(self):
        torch = self.torch
        out = torch.empty((self.n_traced, self.max_bounces + 1), dtype=torch.int32,
                          device=self.device)
        if out.numel() == 0:
            return out
        self._check(self.lib.rr_get_hits(self.h, C.c_void_p(out.data_ptr()), out.numel()))
        self.stream.synchronize()
        return out

    def trace_work(self, n_rays, max_bounces=2, seed=0, az_min=-math.pi / 2, az_max=math.pi / 2,
                   el_min=-math.pi / 2, el_max=math.pi / 2, sampler=UNIFORM, record_hits=False,
                   path_cap=0):
        """trace() through the counting kernel: returns (paths, work) with work
        = dict(rays, queries, nodes, tris) summed over the launch."""
        tp = TraceParams(int(n_rays), int(max_bounces), int(seed) & (2**64 - 1), az_min, az_max,
                         el_min, el_max, int(sampler), int(bool(record_hits)), int(path_cap))
        n = C.c_int64()
        w = (C.c_int64 * 4)()
        self._check(self.lib.rr_trace_work(self.h, C.byref(tp), C.byref(n), w))
        self.n_paths = n.value
        n_src = 1 if self.mode == TX_SHARED else self.n_tx
        self.n_traced = n_src * (int(n_rays) if self.mode == TX_SHARED else int(n_rays) // self.n_tx)
        self.max_bounces = int(max_bounces)
        self.record_hits = bool(record_hits)
        return n.value, dict(rays=w[0], queries=w[1], nodes=w[2], tris=w[3])

    def path_count(self) -> int:
        """Stored paths of the last trace (waits for a trace run with sync=False)."""
        n = C.c_int64()
        self._check(self.lib.rr_get_path_count(self.h, C.byref(n)))
        self.n_paths = n.value
        return n.value

    def paths(self):
        """Context paths as device tensors: src, K, ray [n]; tri, vid [KMAX][n];
        p [3*KMAX][n]; L, amp [n]."""
        torch = self.torch
        n = C.c_int64()
        self._check(self.lib.rr_get_path_count(self.h, C.byref(n)))
        n = max(n.value, 1)
        d = self.device
        out = dict(src=torch.empty(n, dtype=torch.int32, device=d),
                   K=torch.empty(n, dtype=torch.int32, device=d),
                   ray=torch.empty(n, dtype=torch.int64, device=d),
                   tri=torch.empty((KMAX, n), dtype=torch.int32, device=d),
                   vid=torch.empty((KMAX, n), dtype=torch.int32, device=d),
                   p=torch.empty((3 * KMAX, n), dtype=torch.float64, device=d),
                   L=torch.empty(n, dtype=torch.float64, device=d),
                   amp=torch.empty(n, dtype=torch.float64, device=d))
        ps = Paths(*(C.c_void_p(out[k].data_ptr()) for k in ("src", "K", "ray", "tri", "vid", "p", "L", "amp")), n)
        cnt = C.c_int64()
        self._check(self.lib.rr_get_paths(self.h, C.byref(ps), C.byref(cnt)))
        m = cnt.value
        return {k: (v[..., :m] if v.dim() == 2 else v[:m]) for k, v in out.items()}

    def set_paths(self, paths: dict):
        torch = self.torch
        n = int(paths["K"].numel())
        keep = {}
        for k, dt, shape in (("src", torch.int32, (n,)), ("K", torch.int32, (n,)),
                             ("ray", torch.int64, (n,)), ("tri", torch.int32, (KMAX, n)),
                             ("vid", torch.int32, (KMAX, n)), ("p", torch.float64, (3 * KMAX, n)),
                             ("L", torch.float64, (n,)), ("amp", torch.float64, (n,))):
            if k in paths:
                keep[k] = paths[k].to(device=self.device, dtype=dt).contiguous().reshape(shape)
        ptr = lambda k: C.c_void_p(keep[k].data_ptr()) if k in keep and n else None
        ps = Paths(ptr("src"), ptr("K"), ptr("ray"), ptr("tri"), ptr("vid"), ptr("p"), ptr("L"),
                   ptr("amp"), n)
        self._check(self.lib.rr_set_paths(self.h, C.byref(ps), n))
        self.n_paths = n

    # ---------------------------------------------------------- synthesis
    def synthesize(self, model=EXACT, engine=ENGINE_AUTO, sample_idx=None, out=None):
        """Full cube [C][M][K] complex64, or the flat entries sample_idx."""
        torch = self.torch
        if sample_idx is None:
            if out is None:
                out = torch.empty((self.n_ch, self.M, self.K), dtype=torch.complex64,
                                  device=self.device)
            check_out(out, self.device, torch.complex64, self.n_ch * self.M * self.K, "cube")
            self._check(self.lib.rr_synthesize(self.h, int(model), int(engine),
                                               C.c_void_p(out.data_ptr()), out.numel(), None, 0))
            return out
        idx = torch.as_tensor(sample_idx, dtype=torch.int64).to(self.device).contiguous()
        if out is None:
            out = torch.empty(idx.numel(), dtype=torch.complex64, device=self.device)
        check_out(out, self.device, torch.complex64, idx.numel(), "sampled entries")
        self._check(self.lib.rr_synthesize(self.h, int(model), int(engine),
                                           C.c_void_p(out.data_ptr()), out.numel(),
                                           C.c_void_p(idx.data_ptr()), idx.numel()))
        self._keep_idx = idx
        return out

    def synthesize_noalloc(self, model=EXACT, out=None):
        """Full cube through rr_synthesize_noalloc (direct engine, no device
        allocation in the library; `out` must be given to avoid one here)."""
        torch = self.torch
        if out is None:
            out = torch.empty((self.n_ch, self.M, self.K), dtype=torch.complex64,
                              device=self.device)
        check_out(out, self.device, torch.complex64, self.n_ch * self.M * self.K, "cube")
        self._check(self.lib.rr_synthesize_noalloc(self.h, int(model), C.c_void_p(out.data_ptr()),
                                                   out.numel()))
        return out

    # ------------------------------------------------------------ imaging
    def backproject(self, cube, grid, out=None, engine=ENGINE_AUTO):
        """Delay-and-sum image (complex64 [nx][ny][nz]) of `cube` (this
        context's array and chirp) on grid = (origin (x0, y0, z0), step,
        (nx, ny, nz)) as scenegen.imaging_grid returns it; engine
        DIRECT_FP32 (Horner, vector units), GEMM_EXACT (matrix cores) or AUTO."""
        torch = self.torch
        (x0, y0, z0), step, (nx, ny, nz) = grid
        vol = Volume(float(x0), float(y0), float(z0), float(step), int(nx), int(ny), int(nz))
        check_out(cube, self.device, torch.complex64, self.n_ch * self.M * self.K, "cube")
        if out is None:
            out = torch.empty((nx, ny, nz), dtype=torch.complex64, device=self.device)
        check_out(out, self.device, torch.complex64, nx * ny * nz, "image")
        self._check(self.lib.rr_backproject(self.h, C.c_void_p(cube.data_ptr()), cube.numel(),
                                            C.byref(vol), C.c_void_p(out.data_ptr()), out.numel(),
                                            int(engine)))
        return out

    def max_projection(self, image, grid, floor_db=-15.0, out=None):
        """Maximum over range of |image| per (y, z) in dB, float32 [ny][nz]."""
        torch = self.torch
        (x0, y0, z0), step, (nx, ny, nz) = grid
        vol = Volume(float(x0), float(y0), float(z0), float(step), int(nx), int(ny), int(nz))
        check_out(image, self.device, torch.complex64, nx * ny * nz, "image")
        if out is None:
            out = torch.empty((ny, nz), dtype=torch.float32, device=self.device)
        check_out(out, self.device, torch.float32, ny * nz, "projection")
        self._check(self.lib.rr_max_projection(self.h, C.c_void_p(image.data_ptr()), C.byref(vol),
                                               C.c_void_p(out.data_ptr()), float(floor_db)))
        return out

    def kernel_ms(self, which: int) -> float:
        ms = C.c_double()
        self._check(self.lib.rr_last_kernel_ms(self.h, int(which), C.byref(ms)))
        return ms.value

    # ------------------------------------------------------ conveniences
    def setup(self, workload):
        """Upload a workload-like object (scene, array, chirp)."""
        self.upload(workload.scene)
        a = workload.array
        self.set_array(a.tx, a.rx, a.rx_radius, a.mode)
        ch = workload.chirp
        self.set_chirp(ch.f0, ch.bandwidth, ch.t_chirp, ch.t_rep, ch.n_samples, ch.n_chirps)

    def trace_workload(self, workload, record_hits=True, **kw):
        tp = workload.trace
        args = dict(n_rays=tp.n_rays, max_bounces=tp.max_bounces, seed=tp.seed, az_min=tp.az_min,
                    az_max=tp.az_max, el_min=tp.el_min, el_max=tp.el_max,
                    record_hits=record_hits, path_cap=getattr(workload, "path_cap", None) or 0)
        rpt = int(getattr(tp, "rays_per_tri", 0) or 0)
        if rpt > 0:
            args.update(n_rays=rpt, sampler=PER_TRIANGLE)
            self.set_casting(getattr(tp, "tri_omega_max", 0.0), getattr(tp, "tri_depth_max", 8))
        args.update(kw)
        return self.trace(**args)


# --------------------------------------------------------------------------
# learned proposal
# --------------------------------------------------------------------------
PROP_NAZ, PROP_NEL, MLP_PARAMS = 128, 64, 9601
_PROP_DECLARED = False


def _declare_proposal(L):
    global _PROP_DECLARED
    if _PROP_DECLARED:
        return
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.rr_proposal_set_cdf.argtypes = [vp, vp, i32, i32]
    L.rr_proposal_get_cdf.argtypes = [vp, vp, i64]
    L.rr_proposal_probe.argtypes = [vp, C.c_double, C.c_double, vp]
    L.rr_proposal_histogram.argtypes = [vp, vp]
    L.rr_mlp_init.argtypes = [vp, C.c_uint64]
    L.rr_mlp_set_params.argtypes = [vp, vp, i64]
    L.rr_mlp_get_params.argtypes = [vp, vp, i64]
    L.rr_mlp_forward.argtypes = [vp, vp, i32, vp]
    L.rr_mlp_train_step.argtypes = [vp, vp, vp, i32, C.c_float, C.POINTER(C.c_float), vp]
    L.rr_proposal_train.argtypes = [vp, vp, vp, i32, i32, i32, C.c_float, C.c_uint64, vp]
    L.rr_proposal_build.argtypes = [vp, vp, C.c_float, C.c_float]
    L.rr_proposal_build_cost.argtypes = [vp, vp, C.c_float, C.c_float]
    _PROP_DECLARED = True


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def check_out(t, device, dtype, numel, what="output"):
    """An output tensor handed to the library must be a contiguous tensor of
    `dtype` on the context's device with at least `numel` elements: the
    library receives only its address."""
    if (not hasattr(t, "data_ptr") or t.device != device or t.dtype != dtype
            or not t.is_contiguous() or t.numel() < numel):
        raise ValueError(f"{what} must be a contiguous {dtype} tensor on {device} with at least "
                         f"{numel} elements")


class _ProposalMixin:
    def _pl(self):
        _declare_proposal(self.lib)
        return self.lib

    def proposal_set_cdf(self, cdf, n_az=PROP_NAZ, n_el=PROP_NEL):
        c = np.ascontiguousarray(cdf, dtype=np.float64)
        self._check(self._pl().rr_proposal_set_cdf(self.h, c.ctypes.data, int(n_az), int(n_el)))

    def proposal_get_cdf(self):
        out = np.zeros(PROP_NAZ * PROP_NEL + 1)
        self._check(self._pl().rr_proposal_get_cdf(self.h, out.ctypes.data, out.size))
        return out

    def proposal_probe(self, az_min=-math.pi / 2, az_max=math.pi / 2):
        out = self.torch.empty(16, dtype=self.torch.float32, device=self.device)
        self._check(self._pl().rr_proposal_probe(self.h, az_min, az_max, _ptr(out)))
        return out

    def proposal_histogram(self):
        out = self.torch.empty(PROP_NAZ * PROP_NEL, dtype=self.torch.float32, device=self.device)
        self._check(self._pl().rr_proposal_histogram(self.h, _ptr(out)))
        return out

    def mlp_init(self, seed=0):
        self._check(self._pl().rr_mlp_init(self.h, int(seed) & (2**64 - 1)))

    def mlp_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self._pl().rr_mlp_set_params(self.h, p.ctypes.data, p.size))

    def mlp_get_params(self):
        p = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._check(self._pl().rr_mlp_get_params(self.h, p.ctypes.data, p.size))
        return p

    def mlp_forward(self, codes):
        codes = codes.to(self.device, self.torch.float32).contiguous().reshape(-1, 16)
        out = self.torch.empty((codes.shape[0], PROP_NAZ * PROP_NEL), dtype=self.torch.float32,
                               device=self.device)
        self._check(self._pl().rr_mlp_forward(self.h, _ptr(codes), codes.shape[0], _ptr(out)))
        return out

    def mlp_train_step(self, codes, hists, lr, want_grad=False):
        codes = codes.to(self.device, self.torch.float32).contiguous().reshape(-1, 16)
        hists = hists.to(self.device, self.torch.float32).contiguous().reshape(-1, PROP_NAZ * PROP_NEL)
        grad = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device=self.device) if want_grad else None
        loss = C.c_float()
        self._check(self._pl().rr_mlp_train_step(self.h, _ptr(codes), _ptr(hists), codes.shape[0],
                                                 float(lr), C.byref(loss),
                                                 _ptr(grad) if grad is not None else None))
        return (loss.value, grad) if want_grad else loss.value

    def proposal_train(self, codes, hists, steps, batch=16, lr=1e-3, seed=0):
        """`steps` Adam steps on minibatches drawn in the library; returns the
        per-step losses (numpy float32 [steps])."""
        codes = codes.to(self.device, self.torch.float32).contiguous().reshape(-1, 16)
        hists = hists.to(self.device, self.torch.float32).contiguous().reshape(-1, PROP_NAZ * PROP_NEL)
        if codes.shape[0] != hists.shape[0]:
            raise ValueError("codes and histograms must have the same number of scenes")
        loss = np.zeros(max(int(steps), 1), dtype=np.float32)
        self._check(self._pl().rr_proposal_train(self.h, _ptr(codes), _ptr(hists), codes.shape[0],
                                                  int(steps), int(batch), float(lr),
                                                  int(seed) & (2**64 - 1), loss.ctypes.data))
        return loss[: int(steps)]

    def proposal_build_cost(self, code, beta=0.1, kappa=1.0):
        """Cost-aware sampling table: q ~ sqrt(x / (kappa + x)), x = n_bins softmax(z)."""
        code = code.to(self.device, self.torch.float32).contiguous().reshape(16)
        self._check(self._pl().rr_proposal_build_cost(self.h, _ptr(code), float(beta), float(kappa)))
        self._keep_code = code

    def proposal_build(self, code, beta=0.1, power=0.5):
        code = code.to(self.device, self.torch.float32).contiguous().reshape(16)
        self._check(self._pl().rr_proposal_build(self.h, _ptr(code), float(beta), float(power)))
        self._keep_code = code


for _name, _fn in list(vars(_ProposalMixin).items()):
    if callable(_fn) and not _name.startswith("__"):
        setattr(Context, _name, _fn)
EXPORTED += ["rr_proposal_set_cdf", "rr_proposal_get_cdf", "rr_proposal_probe",
             "rr_proposal_histogram", "rr_mlp_init", "rr_mlp_set_params", "rr_mlp_get_params",
             "rr_mlp_forward", "rr_mlp_train_step", "rr_proposal_train", "rr_proposal_build",
             "rr_proposal_build_cost"]


# --------------------------------------------------------------------------
# batched launch
# --------------------------------------------------------------------------
def _declare_batch(L):
    if getattr(L, "_batch_declared", False):
        return
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.rr_batch_create.argtypes = [vp, i32, C.POINTER(vp)]
    L.rr_batch_destroy.argtypes = [vp]
    L.rr_batch_destroy.restype = None
    L.rr_batch_set_scene.argtypes = [vp, i32, vp, i64, vp, vp, i64, vp, vp, i32, vp, vp, vp, i32,
                                     vp, i32, vp, i32, f64, i32, C.POINTER(Chirp),
                                     C.POINTER(TraceParams)]
    L.rr_batch_set_alpha.argtypes = [vp, i32, vp, i64, i32]
    L.rr_batch_launch.argtypes = [vp, vp, vp]
    L.rr_batch_tune.argtypes = [vp, vp]
    L.rr_batch_get_tiles.argtypes = [vp, vp]
    L.rr_batch_get_plan.argtypes = [vp, vp, vp]
    L.rr_batch_set_engine.argtypes = [vp, i32, i32, i32]
    L.rr_batch_stats.argtypes = [vp, C.POINTER(f64), C.POINTER(f64), C.POINTER(i64)]
    L._batch_declared = True


class Batch:
    """A batch of scenes traced and synthesised by one captured launch."""

    def __init__(self, ctx: "Context", n_scenes: int):
        self.ctx = ctx
        self.lib = ctx.lib
        _declare_batch(self.lib)
        h = C.c_void_p()
        ctx._check(self.lib.rr_batch_create(ctx.h, int(n_scenes), C.byref(h)))
        self.h = h
        self.n = int(n_scenes)
        self.shapes = [None] * self.n

    def close(self):
        if getattr(self, "h", None):
            self.lib.rr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_workload(self, slot, w):
        sc, a, ch, tp = w.scene, w.array, w.chirp, w.trace
        if int(getattr(tp, "rays_per_tri", 0) or 0) > 0:
            raise ValueError("batched launches use the uniform sampler (no per-triangle casting)")
        keep = []

        def P(x, dt):
            x = np.ascontiguousarray(x, dtype=dt)
            keep.append(x)
            return x.ctypes.data if x.size else None

        chirp = Chirp(ch.f0, ch.bandwidth, ch.t_chirp, ch.t_rep, ch.n_samples, ch.n_chirps)
        t = TraceParams(int(tp.n_rays), int(tp.max_bounces), int(tp.seed) & (2**64 - 1), tp.az_min,
                        tp.az_max, tp.el_min, tp.el_max, UNIFORM, 0, 0)
        self.ctx._check(self.lib.rr_batch_set_scene(
            self.h, int(slot), P(sc.verts, np.float32), sc.verts.shape[0], P(sc.tris, np.int32),
            P(sc.tri_obj, np.int32), sc.tris.shape[0], P(sc.obj_alpha, np.float32),
            P(sc.obj_vel, np.float64), sc.obj_alpha.shape[0], P(sc.pt_pos, np.float64),
            P(sc.pt_vel, np.float64), P(sc.pt_aperture, np.float64), sc.pt_pos.shape[0],
            P(a.tx, np.float64), a.tx.shape[0], P(a.rx, np.float64), a.rx.shape[0],
            float(a.rx_radius), int(a.mode), C.byref(chirp), C.byref(t)))
        self.shapes[slot] = (a.tx.shape[0] * a.rx.shape[0], ch.n_chirps, ch.n_samples)
        ta = getattr(sc, "tri_alpha", None)
        if ta is not None:
            self.set_alpha(slot, ta, per=ALPHA_PER_TRIANGLE)

    def set_alpha(self, slot, alpha, per=ALPHA_PER_OBJECT):
        """Replace slot's material mix (Eq. 3) per object or per face."""
        a, pa = _np(alpha, np.float32)
        self.ctx._check(self.lib.rr_batch_set_alpha(self.h, int(slot), pa, a.size, int(per)))

    def alloc_cubes(self):
        torch = self.ctx.torch
        return [torch.empty(s, dtype=torch.complex64, device=self.ctx.device) for s in self.shapes]

    def _ptrs(self, cubes):
        if len(cubes) != self.n:
            raise ValueError(f"{self.n} cubes expected")
        torch = self.ctx.torch
        for s, (c, shape) in enumerate(zip(cubes, self.shapes)):
            if shape is None:
                raise ValueError(f"batch slot {s} has no scene")
            check_out(c, self.ctx.device, torch.complex64, int(np.prod(shape)), f"cube {s}")
        arr = (C.c_void_p * self.n)(*[c.data_ptr() for c in cubes])
        self._keep = arr
        return arr

    def launch(self, cubes, want_counts=True):
        counts = np.zeros(self.n, dtype=np.int64) if want_counts else None
        self.ctx._check(self.lib.rr_batch_launch(self.h, self._ptrs(cubes),
                                                 counts.ctypes.data if want_counts else None))
        return counts

    def tune(self, cubes):
        self.ctx._check(self.lib.rr_batch_tune(self.h, self._ptrs(cubes)))
        tiles = np.zeros(self.n, dtype=np.int32)
        self.ctx._check(self.lib.rr_batch_get_tiles(self.h, tiles.ctypes.data))
        return tiles

    def set_engine(self, slot, engine=ENGINE_AUTO, tile=0):
        """Pin slot's synthesis engine (ENGINE_AUTO, DIRECT_FP32, or
        GEMM_EXACT with product layout tile: 16, 32, 48, 64 or 96 square
        Tx x Rx tiles, 1 = per-channel sample split, 0 = least modelled
        time)."""
        self.ctx._check(self.lib.rr_batch_set_engine(self.h, int(slot), int(engine), int(tile)))

    def plan(self):
        """(engine, tile) per scene: DIRECT_FP32 with its samples per lane, or
        GEMM_EXACT with its product tile."""
        e = np.zeros(self.n, dtype=np.int32)
        t = np.zeros(self.n, dtype=np.int32)
        self.ctx._check(self.lib.rr_batch_get_plan(self.h, e.ctypes.data, t.ctypes.data))
        return e, t

    def stats(self):
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        self.ctx._check(self.lib.rr_batch_stats(self.h, C.byref(a), C.byref(b), C.byref(n)))
        return dict(ms_total=a.value, ms_synth_tuned=b.value, paths=n.value)


EXPORTED += ["rr_batch_create", "rr_batch_destroy", "rr_batch_set_scene", "rr_batch_set_alpha",
             "rr_batch_launch",
             "rr_batch_tune", "rr_batch_get_tiles", "rr_batch_get_plan", "rr_batch_set_engine",
             "rr_batch_stats"]
