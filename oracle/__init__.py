"""CPU oracle for the radar ray-tracing hot path (TEST INFRASTRUCTURE).

A plain single-threaded FP64 implementation in C (`oracle.c`) wrapped with
ctypes, plus an FP64 numpy implementation of the proposal network
(`oracle.mlp`).  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package.  It shares no code with the GPU
library and never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KMAX = 8

PATH_DTYPE = np.dtype([
    ("src", np.int32), ("K", np.int32), ("ray", np.int64),
    ("tri", np.int32, (KMAX,)), ("vid", np.int32, (KMAX,)),
    ("p", np.float64, (KMAX, 3)), ("L", np.float64), ("amp", np.float64),
], align=True)


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("verts", C.c_void_p), ("nv", C.c_int64), ("tris", C.c_void_p),
                ("tri_obj", C.c_void_p), ("nt", C.c_int64), ("obj_alpha", C.c_void_p),
                ("obj_vel", C.c_void_p), ("nobj", C.c_int32), ("pt_pos", C.c_void_p),
                ("pt_vel", C.c_void_p), ("pt_ap", C.c_void_p), ("npts", C.c_int32),
                ("tri_alpha", C.c_void_p)]


class _Array(C.Structure):
    _fields_ = [("tx", C.c_void_p), ("ntx", C.c_int32), ("rx", C.c_void_p), ("nrx", C.c_int32),
                ("rx_radius", C.c_double), ("shared", C.c_int32)]


class _Chirp(C.Structure):
    _fields_ = [("f0", C.c_double), ("bandwidth", C.c_double), ("t_chirp", C.c_double),
                ("t_rep", C.c_double), ("n_samples", C.c_int32), ("n_chirps", C.c_int32)]


class _Trace(C.Structure):
    _fields_ = [("n_rays", C.c_int64), ("max_bounces", C.c_int32), ("seed", C.c_uint64),
                ("az_min", C.c_double), ("az_max", C.c_double), ("el_min", C.c_double),
                ("el_max", C.c_double), ("cdf", C.c_void_p), ("n_az", C.c_int32),
                ("n_el", C.c_int32), ("tri_g", C.c_int32), ("tri_omega_max", C.c_double),
                ("tri_depth_max", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_philox4x64.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_sincos_turn.argtypes = [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_closest.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                                  C.POINTER(C.c_double)]
        L.orc_closest.restype = C.c_int64
        L.orc_bounce.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                                 C.c_void_p]
        L.orc_launch_dir.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                     C.c_void_p]
        L.orc_trace.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                C.POINTER(C.c_int64)]
        L.orc_trace_rays.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int64, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_uint64,
                                     C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
        L.orc_synth.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_int, C.c_void_p, C.c_int64, C.c_void_p]
        L.orc_backproject.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_void_p,
                                      C.c_void_p, C.c_int64, C.c_void_p]
        L.orc_pieces.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_int64]
        L.orc_pieces.restype = C.c_int64
        L.orc_release.argtypes = []
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None and a.size else None


class _Keep:
    """Holds the numpy buffers a ctypes struct points into."""

    def __init__(self):
        self.bufs = []

    def add(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.bufs.append(a)
        return a


def _scene(s, keep):
    v = keep.add(s.verts, np.float32)
    t = keep.add(s.tris, np.int32)
    o = keep.add(s.tri_obj, np.int32)
    a = keep.add(s.obj_alpha, np.float32)
    ov = keep.add(s.obj_vel, np.float64)
    pp = keep.add(s.pt_pos, np.float64)
    pv = keep.add(s.pt_vel, np.float64)
    pa = keep.add(s.pt_aperture, np.float64)
    ta = getattr(s, "tri_alpha", None)
    ta = None if ta is None else keep.add(ta, np.float32)
    st = _Scene(_p(v), v.shape[0], _p(t), _p(o), t.shape[0], _p(a), _p(ov), a.shape[0],
                _p(pp), _p(pv), _p(pa), pp.shape[0], None if ta is None else _p(ta))
    keep.bufs.append(st)
    return st


def _array(a, keep):
    tx = keep.add(a.tx, np.float64)
    rx = keep.add(a.rx, np.float64)
    st = _Array(_p(tx), tx.shape[0], _p(rx), rx.shape[0], float(a.rx_radius), int(a.mode))
    keep.bufs.append(st)
    return st


def _trace(tp, keep, cdf=None, n_az=0, n_el=0):
    c = None if cdf is None else keep.add(cdf, np.float64)
    st = _Trace(int(tp.n_rays), int(tp.max_bounces), int(tp.seed) & (2**64 - 1), tp.az_min,
                tp.az_max, tp.el_min, tp.el_max, _p(c), n_az, n_el, tri_grid(tp),
                float(getattr(tp, "tri_omega_max", 0.0) or 0.0),
                int(getattr(tp, "tri_depth_max", 8)))
    keep.bufs.append(st)
    return st


def _chirp(ch):
    return _Chirp(ch.f0, ch.bandwidth, ch.t_chirp, ch.t_rep, ch.n_samples, ch.n_chirps)


# ----------------------------------------------------------------------------
# primitives
# ----------------------------------------------------------------------------

def philox4x64(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def sincos_turn(u: float) -> tuple[float, float]:
    s, c = C.c_double(), C.c_double()
    lib().orc_sincos_turn(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def closest(scene, o, d, skip=-1, use_bvh=False):
    keep = _Keep()
    sc = _scene(scene, keep)
    o = keep.add(o, np.float64)
    d = keep.add(d, np.float64)
    t = C.c_double()
    h = lib().orc_closest(C.addressof(sc), o.ctypes.data, d.ctypes.data, int(skip), int(use_bvh),
                          C.byref(t))
    lib().orc_release()
    return int(h), t.value


def bounce(d, n, alpha, u0, u1) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_bounce(d.ctypes.data, n.ctypes.data, float(alpha), float(u0), float(u1),
                     out.ctypes.data)
    return out


def launch_dir(scene, array, tp, i, t, cdf=None, n_az=0, n_el=0) -> np.ndarray:
    keep = _Keep()
    out = np.zeros(4)
    lib().orc_launch_dir(C.addressof(_scene(scene, keep)), C.addressof(_array(array, keep)),
                         C.addressof(_trace(tp, keep, cdf, n_az, n_el)), int(i), int(t),
                         out.ctypes.data)
    return out


# ----------------------------------------------------------------------------
# trace and synthesis
# ----------------------------------------------------------------------------

def tri_grid(tp) -> int:
    """g of per-triangle casting (g^2 rays per triangle and source), 0 if off."""
    n = int(getattr(tp, "rays_per_tri", 0) or 0)
    if n <= 0:
        return 0
    g = int(round(n ** 0.5))
    if g * g != n:
        raise ValueError("rays_per_tri must be a perfect square")
    return g


def pieces(scene, array, omega_max=0.0, depth_max=8, fov=None):
    """The per-triangle launch's pieces: (vertices float64 [n][3][3], parent
    triangle int64 [n]).  fov = (az_min, az_max, el_min, el_max) drops the
    pieces no ray of which can enter that field of view (None: keep all)."""
    keep = _Keep()
    sc = _scene(scene, keep)
    ar = _array(array, keep)
    fv = None
    if fov is not None:
        fv = np.ascontiguousarray(fov, dtype=np.float64)
        keep.bufs.append(fv)
    fp = fv.ctypes.data if fv is not None else None
    n = lib().orc_pieces(C.addressof(sc), C.addressof(ar), float(omega_max), int(depth_max), fp,
                         None, None, 0)
    if n < 0:
        raise RuntimeError("orc_pieces failed")
    v = np.zeros((max(n, 1), 3, 3))
    par = np.zeros(max(n, 1), dtype=np.int64)
    lib().orc_pieces(C.addressof(sc), C.addressof(ar), float(omega_max), int(depth_max), fp,
                     v.ctypes.data, par.ctypes.data, n)
    return v[:n], par[:n]


def fov_of(tp):
    """(az_min, az_max, el_min, el_max) of trace parameters."""
    return (tp.az_min, tp.az_max, tp.el_min, tp.el_max)


def n_per_src(scene, array, tp) -> int:
    g = tri_grid(tp)
    if g:
        om = float(getattr(tp, "tri_omega_max", 0.0) or 0.0)
        n = len(pieces(scene, array, om, int(getattr(tp, "tri_depth_max", 8)), fov_of(tp))[1])
        return n * g * g
    return int(tp.n_rays) if array.mode == 1 else int(tp.n_rays) // array.n_tx


def n_src(array) -> int:
    return 1 if array.mode == 1 else array.n_tx


def n_virtual(scene, array, tp) -> int:
    return n_src(array) * (n_per_src(scene, array, tp) + scene.n_pts)


def trace(scene, array, tp, vids=None, use_bvh=None, cdf=None, n_az=0, n_el=0,
          want_hits=True, cap=None):
    """Trace virtual rays `vids` (all when None).  Returns (hits, paths):
    hits int32 [n][max_bounces+1] (or None), paths: structured PATH_DTYPE array
    in (virtual ray, bounce) order."""
    if use_bvh is None:
        use_bvh = scene.n_tris > 1000
    keep = _Keep()
    sc = _scene(scene, keep)
    ar = _array(array, keep)
    tr = _trace(tp, keep, cdf, n_az, n_el)
    v = None if vids is None else keep.add(vids, np.int64)
    n = n_virtual(scene, array, tp) if vids is None else v.shape[0]
    hits = np.full((n, tp.max_bounces + 1), -1, dtype=np.int32) if want_hits else None
    if cap is None:
        cap = max(1024, n // 16)
    while True:
        paths = np.zeros(cap, dtype=PATH_DTYPE)
        npaths = C.c_int64()
        rc = lib().orc_trace(C.addressof(sc), C.addressof(ar), C.addressof(tr), int(use_bvh),
                             _p(v), n, _p(hits), paths.ctypes.data, cap, C.byref(npaths))
        if rc != 0:
            raise RuntimeError(f"orc_trace failed: {rc}")
        if npaths.value <= cap:
            break
        cap = npaths.value
    lib().orc_release()
    return hits, paths[: npaths.value].copy()


def trace_rays(scene, array, orig, dirs, amp, src, max_bounces, seed, use_bvh=None,
               want_hits=True):
    """Trace caller-supplied rays: orig, dirs float64 [n][3] (directions are
    normalised), amp float64 [n], src int32 [n] (-1 for a shared launch, else
    ascending Tx indices).  Returns (hits, paths) as trace() does, with
    ray = the index of the ray."""
    if use_bvh is None:
        use_bvh = scene.n_tris > 1000
    keep = _Keep()
    sc = _scene(scene, keep)
    ar = _array(array, keep)
    o = keep.add(orig, np.float64).reshape(-1, 3)
    d = keep.add(dirs, np.float64).reshape(-1, 3)
    a = keep.add(amp, np.float64).reshape(-1)
    s = keep.add(src, np.int32).reshape(-1)
    n = o.shape[0]
    assert d.shape[0] == n and a.shape[0] == n and s.shape[0] == n
    hits = np.full((n, max_bounces + 1), -1, dtype=np.int32) if want_hits else None
    cap = max(1024, n // 8)
    while True:
        paths = np.zeros(cap, dtype=PATH_DTYPE)
        npaths = C.c_int64()
        rc = lib().orc_trace_rays(C.addressof(sc), C.addressof(ar), int(use_bvh), n, _p(o), _p(d),
                                  _p(a), _p(s), int(max_bounces), int(seed) & (2**64 - 1),
                                  _p(hits), paths.ctypes.data, cap, C.byref(npaths))
        if rc != 0:
            raise ValueError(f"orc_trace_rays rejected its input ({rc})")
        if npaths.value <= cap:
            break
        cap = npaths.value
    lib().orc_release()
    return hits, paths[: npaths.value].copy()


def backproject(array, f0, df, cube, voxels) -> np.ndarray:
    """Delay-and-sum image (complex128 [nv]) of a single-sweep cube
    (complex [n_tx n_rx][nf], frequencies f0 + n df) at voxels [nv][3]."""
    keep = _Keep()
    ar = _array(array, keep)
    cb = np.ascontiguousarray(np.asarray(cube).reshape(array.n_ch, -1).astype(np.complex128))
    nf = cb.shape[1]
    cr = keep.add(np.stack([cb.real, cb.imag], -1), np.float64)
    vx = keep.add(voxels, np.float64).reshape(-1, 3)
    out = np.zeros((vx.shape[0], 2))
    rc = lib().orc_backproject(C.addressof(ar), float(f0), float(df), nf, cr.ctypes.data,
                               _p(vx), vx.shape[0], out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_backproject failed: {rc}")
    return out[:, 0] + 1j * out[:, 1]


def synth(paths, scene, array, chirp, model=0, idx=None) -> np.ndarray:
    """Cube entries (complex128) for model 0 (exact) or 1 (separable).  With
    idx None: the full cube [C][M][K]; else the flat entries idx."""
    keep = _Keep()
    paths = np.ascontiguousarray(paths, dtype=PATH_DTYPE)
    sc = _scene(scene, keep)
    ar = _array(array, keep)
    ch = _chirp(chirp)
    ix = None if idx is None else keep.add(idx, np.int64)
    n = array.n_ch * chirp.n_chirps * chirp.n_samples if ix is None else ix.shape[0]
    out = np.zeros((n, 2))
    rc = lib().orc_synth(paths.ctypes.data if paths.size else None, paths.shape[0],
                         C.addressof(sc), C.addressof(ar), C.byref(ch), int(model), _p(ix), n,
                         out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_synth failed: {rc}")
    z = out[:, 0] + 1j * out[:, 1]
    if ix is None:
        z = z.reshape(array.n_ch, chirp.n_chirps, chirp.n_samples)
    return z


def to_soa(p, kmax: int = 4) -> dict:
    """Oracle path records -> the library's structure-of-arrays layout
    (src, K, ray [n]; tri, vid [kmax][n]; p [3*kmax][n]; L, amp [n])."""
    n = len(p)
    return dict(src=p["src"].astype(np.int32), K=p["K"].astype(np.int32),
                ray=p["ray"].astype(np.int64),
                tri=np.ascontiguousarray(p["tri"][:, :kmax].T.astype(np.int32)),
                vid=np.ascontiguousarray(p["vid"][:, :kmax].T.astype(np.int32)),
                p=np.ascontiguousarray(p["p"][:, :kmax, :].reshape(n, 3 * kmax).T),
                L=p["L"].astype(np.float64), amp=p["amp"].astype(np.float64))


def probe_code(scene, array, tp, use_bvh=None) -> np.ndarray:
    """16-value scene code of the learned proposal (see orc_probe)."""
    if use_bvh is None:
        use_bvh = scene.n_tris > 1000
    keep = _Keep()
    L = lib()
    L.orc_probe.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    out = np.zeros(16)
    rc = L.orc_probe(C.addressof(_scene(scene, keep)), C.addressof(_array(array, keep)),
                     C.addressof(_trace(tp, keep)), int(use_bvh), out.ctypes.data)
    L.orc_release()
    if rc != 0:
        raise RuntimeError(f"orc_probe failed: {rc}")
    return out


def uniform_bins(scene, array, tp, n_az=128, n_el=64) -> np.ndarray:
    L = lib()
    L.orc_uniform_bins.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                   C.c_void_p]
    per, ns = n_per_src(scene, array, tp), n_src(array)
    bins = np.zeros(per * ns, dtype=np.int32)
    L.orc_uniform_bins(int(tp.seed) & (2**64 - 1), per, ns, n_az, n_el, bins.ctypes.data)
    return bins


def histogram(scene, array, tp, hits, paths, n_az=128, n_el=64) -> np.ndarray:
    """Training target of the proposal from a uniform trace: per direction bin,
    the sum over its rays of (returned power P_i = sum of w^2 over the ray's
    paths) + 0.1 * (first segment hit an object other than 0)."""
    per, ns = n_per_src(scene, array, tp), n_src(array)
    vps = per + scene.n_pts
    bins = uniform_bins(scene, array, tp, n_az, n_el)
    H = np.zeros(n_az * n_el)
    traced = paths[paths["tri"][:, 0] >= 0]
    v = traced["ray"]
    g = (v // vps) * per + (v % vps)
    w = traced["amp"] * per
    np.add.at(H, bins[g], w * w)
    first = hits[:, 0]
    hit = (first >= 0) & (scene.tri_obj[np.maximum(first, 0)] != 0)
    np.add.at(H, bins, 0.1 * hit)
    return H
