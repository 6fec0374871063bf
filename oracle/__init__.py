"""FP64 CPU oracle for Differentiable Radiative Rasterization (DRR).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU product path.  It shares no
code with the GPU path; the arithmetic lives in ``oracle.c`` (plain C,
float64, plus the fixed float32 "key path" for depth and bounding
rectangles) and this module only marshals numpy arrays through ctypes.

Each function cites the part of the paper it follows:
  camera()         Eq. 12 (extrinsic/intrinsic from scanner parameters)
  project()        Eq. 7-9 and the 2-D covariance of Sec. 3.2
  pairs()          Sec. 3.2: tile assignment, depth-sorted per-tile lists
  render_brute()   Eq. 10 by brute force over all Gaussians
  render_binned()  Eq. 10 over the per-tile lists of Sec. 3.2
  backward()       exact derivative of Eq. 10 (and Eq. 7-9) with all
                   discrete decisions held fixed
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
ABI = 4

FLAG_ALPHA_MIN = 1
FLAG_T_MIN = 2
FLAG_CLAMP = 4


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (IEEE float32, no contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Cam(C.Structure):
    _fields_ = [("rot", C.c_float * 9), ("trans", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class Set(C.Structure):
    _fields_ = [("lowpass", C.c_float), ("alpha_min", C.c_float), ("alpha_max", C.c_float),
                ("t_min", C.c_float), ("near_z", C.c_float), ("tile", C.c_int32)]


class Proj(C.Structure):
    _fields_ = [("kept", C.c_int32), ("depth_bits", C.c_uint32), ("rect", C.c_int32 * 4),
                ("key_u", C.c_float * 2), ("key_s", C.c_float * 3), ("t", C.c_double * 3),
                ("u", C.c_double * 2), ("sig", C.c_double * 3), ("conic", C.c_double * 3)]


_PROJ_DTYPE = np.dtype({
    "names": [f[0] for f in Proj._fields_],
    "formats": ["<i4", "<u4", ("<i4", (4,)), ("<f4", (2,)), ("<f4", (3,)), ("<f8", (3,)),
                ("<f8", (2,)), ("<f8", (3,)), ("<f8", (3,))],
    "offsets": [getattr(Proj, f[0]).offset for f in Proj._fields_],
    "itemsize": C.sizeof(Proj)})


@dataclass
class Settings:
    """Renderer constants (readings of the paper; see module docs of oracle.c)."""

    lowpass: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    near_z: float = 0.2
    tile: int = 16

    def c(self) -> Set:
        return Set(self.lowpass, self.alpha_min, self.alpha_max, self.t_min, self.near_z, self.tile)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.orc_abi_version.restype = C.c_int
        assert L.orc_abi_version() == ABI, "stale liboracle.so"
        L.orc_threads.restype = C.c_int
        L.orc_kappa.restype = C.c_float
        L.orc_kappa.argtypes = [C.c_float]
        L.orc_camera.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                 C.c_double, C.c_double, C.POINTER(Cam)]
        L.orc_total_tiles.restype = C.c_int64
        L.orc_total_tiles.argtypes = [C.c_int32, C.POINTER(Cam), C.c_int32]
        P = C.c_void_p
        L.orc_project.argtypes = [C.c_int32, P, P, P, P, C.POINTER(Cam), C.POINTER(Set), P]
        L.orc_emit_pairs.restype = C.c_int64
        L.orc_emit_pairs.argtypes = [C.c_int32, P, P, P, P, C.c_int32, C.POINTER(Cam),
                                     C.POINTER(Set), P, P]
        L.orc_sort_pairs.argtypes = [C.c_int64, P, P]
        L.orc_ranges.argtypes = [C.c_int64, P, C.c_int64, P]
        L.orc_render_brute.argtypes = [C.c_int32, P, P, P, P, P, C.POINTER(Cam), C.POINTER(Set),
                                       C.c_int64, P, P, P, P, P, P, P]
        L.orc_render_binned.argtypes = [C.c_int32, P, P, P, P, P, C.c_int32, C.POINTER(Cam),
                                        C.POINTER(Set), P, P, P, P, P, P, P, P, P]
        L.orc_backward.argtypes = [C.c_int32, P, P, P, P, P, C.c_int32, C.POINTER(Cam),
                                   C.POINTER(Set), P, C.c_int32, P, P, P, P, P, P, P, P, P, P]
        L.orc_block_contributors.argtypes = [C.c_int32, P, P, P, P, P, C.c_int32, C.POINTER(Cam),
                                             C.POINTER(Set), P, P, P]
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().orc_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _g64(g: dict) -> dict:
    """Gaussian arrays as contiguous float64 (exact for float32 inputs)."""
    return {k: np.ascontiguousarray(g[k], dtype=np.float64) for k in
            ("means", "scales", "quats", "opacity", "intensity")}


def kappa(alpha_min: float) -> float:
    return float(lib().orc_kappa(alpha_min))


def camera(phi: float, l_so: float, l_sd: float, w: int, h: int, det_w: float, det_h: float) -> Cam:
    """Eq. 12: camera of the source at azimuth ``phi``."""
    c = Cam()
    lib().orc_camera(phi, l_so, l_sd, w, h, det_w, det_h, C.byref(c))
    return c


def cam_array(cams) -> C.Array:
    arr = (Cam * len(cams))()
    for k, c in enumerate(cams):
        arr[k] = c
    return arr


def total_tiles(cams, tile: int) -> int:
    return int(lib().orc_total_tiles(len(cams), cam_array(cams), tile))


def project(g: dict, cam: Cam, st: Settings) -> dict:
    """Eq. 7-9 per Gaussian: key-path (float32) depth/rect and float64 u, Sigma'', conic."""
    g = _g64(g)
    n = g["means"].shape[0]
    out = (Proj * max(n, 1))()
    s = st.c()
    lib().orc_project(n, _p(g["means"]), _p(g["scales"]), _p(g["quats"]), _p(g["opacity"]),
                      C.byref(cam), C.byref(s), C.cast(out, C.c_void_p))
    raw = np.frombuffer(out, dtype=_PROJ_DTYPE, count=max(n, 1))[:n]
    return {
        "kept": raw["kept"].astype(bool), "depth_bits": raw["depth_bits"].astype(np.uint32),
        "rect": raw["rect"].astype(np.int32), "key_u": raw["key_u"].copy(),
        "key_s": raw["key_s"].copy(), "t": raw["t"].copy(), "u": raw["u"].copy(),
        "sig": raw["sig"].copy(), "conic": raw["conic"].copy(),
    }


def pairs(g: dict, cams, st: Settings, sort: bool = True) -> dict:
    """Sec. 3.2 tile lists: (key, value) pairs, sorted, and per-tile ranges."""
    g = _g64(g)
    n = g["means"].shape[0]
    ca = cam_array(cams)
    s = st.c()
    L = lib()
    args = (n, _p(g["means"]), _p(g["scales"]), _p(g["quats"]), _p(g["opacity"]), len(cams),
            ca, C.byref(s))
    p = int(L.orc_emit_pairs(*args, None, None))
    keys = np.zeros(max(p, 1), dtype=np.uint64)
    vals = np.zeros(max(p, 1), dtype=np.uint32)
    L.orc_emit_pairs(*args, _p(keys), _p(vals))
    keys, vals = keys[:p], vals[:p]
    if sort:
        L.orc_sort_pairs(p, _p(keys), _p(vals))
    nt = total_tiles(cams, st.tile)
    ranges = np.zeros(2 * nt, dtype=np.uint32)
    if sort:
        L.orc_ranges(p, _p(keys), nt, _p(ranges))
    return {"keys": keys, "values": vals, "ranges": ranges.reshape(nt, 2), "n_pairs": p,
            "n_tiles": nt}


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def render_brute(g: dict, cam: Cam, st: Settings, pix=None, flip=None) -> dict:
    """Eq. 10 by brute force for pixels ``pix`` (flat y*W+x) of one view.
    ``flip`` (per selected pixel): render the other branch of the pixel's
    first flagged decision."""
    g = _g64(g)
    n = g["means"].shape[0]
    if pix is None:
        pix = np.arange(cam.width * cam.height, dtype=np.int32)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    m = pix.shape[0]
    img = np.zeros(m)
    tf = np.zeros(m)
    last = np.zeros(m, dtype=np.int32)
    ev = np.zeros(m, dtype=np.int32)
    fl = np.zeros(m, dtype=np.int32)
    s = st.c()
    lib().orc_render_brute(n, _p(g["means"]), _p(g["scales"]), _p(g["quats"]), _p(g["opacity"]),
                           _p(g["intensity"]), C.byref(cam), C.byref(s), m, _p(pix),
                           _p(_u8(flip)), _p(img), _p(tf), _p(last), _p(ev), _p(fl))
    return {"image": img, "final_t": tf, "last": last, "evals": ev, "flags": fl}


def render_binned(g: dict, cams, st: Settings, values, ranges, flip=None, only=None) -> dict:
    """Eq. 10 over the per-tile sorted lists, all pixels of all views (concatenated).

    ``flip`` (per pixel, nullable): take the other branch of the pixel's
    first flagged decision.  ``only`` (per pixel, nullable): render just
    these pixels (the others read as zero)."""
    g = _g64(g)
    n = g["means"].shape[0]
    npx = int(sum(c.width * c.height for c in cams))
    img = np.zeros(npx)
    tf = np.zeros(npx)
    nc = np.zeros(npx, dtype=np.int32)
    ev = np.zeros(npx, dtype=np.int32)
    fl = np.zeros(npx, dtype=np.int32)
    values = np.ascontiguousarray(values, dtype=np.uint32)
    ranges = np.ascontiguousarray(ranges, dtype=np.uint32)
    s = st.c()
    lib().orc_render_binned(n, _p(g["means"]), _p(g["scales"]), _p(g["quats"]),
                            _p(g["opacity"]), _p(g["intensity"]), len(cams), cam_array(cams),
                            C.byref(s), _p(values), _p(ranges), _p(_u8(flip)), _p(_u8(only)),
                            _p(img), _p(tf), _p(nc), _p(ev), _p(fl))
    return {"image": img, "final_t": tf, "n_contrib": nc, "evals": ev, "flags": fl}


def block_contributors(g: dict, cams, st: Settings, values, ranges) -> np.ndarray:
    """Per 8 x 8 pixel block (8-aligned in each view): the number of distinct
    Gaussians contributing to at least one of its pixels, stored at the
    block's first pixel of the concatenated image layout (0 elsewhere)."""
    g = _g64(g)
    n = g["means"].shape[0]
    npx = int(sum(c.width * c.height for c in cams))
    out = np.zeros(npx, dtype=np.int32)
    values = np.ascontiguousarray(values, dtype=np.uint32)
    ranges = np.ascontiguousarray(ranges, dtype=np.uint32)
    s = st.c()
    lib().orc_block_contributors(n, _p(g["means"]), _p(g["scales"]), _p(g["quats"]),
                                 _p(g["opacity"]), _p(g["intensity"]), len(cams), cam_array(cams),
                                 C.byref(s), _p(values), _p(ranges), _p(out))
    return out


def n_flags(flags) -> np.ndarray:
    """Number of flagged decisions per pixel (decisions within a relative
    margin of a threshold)."""
    return np.asarray(flags) >> 8


def backward(g: dict, cams, st: Settings, dl_di, binned=None, sel=None, want_2d=False,
             flip=None) -> dict:
    """Adjoint of Eq. 10 and Eq. 7-9 for upstream gradient ``dl_di`` (concatenated views).

    ``binned`` = (values, ranges) to traverse tile lists, else brute force.
    ``sel`` = boolean mask of Gaussians whose gradients must be exact (only
    pixels inside their rectangles are processed).  ``flip`` (per pixel):
    differentiate the other branch of the pixel's first flagged decision.
    """
    g = _g64(g)
    n = g["means"].shape[0]
    dl = np.ascontiguousarray(dl_di, dtype=np.float32)
    out = {"means": np.zeros((n, 3)), "scales": np.zeros((n, 3)), "quats": np.zeros((n, 4)),
           "opacity": np.zeros(n), "intensity": np.zeros(n)}
    g2d = np.zeros((len(cams), n, 7)) if want_2d else None
    vals = rng = None
    if binned is not None:
        vals = np.ascontiguousarray(binned[0], dtype=np.uint32)
        rng = np.ascontiguousarray(binned[1], dtype=np.uint32)
    sl = None if sel is None else np.ascontiguousarray(sel, dtype=np.uint8)
    s = st.c()
    lib().orc_backward(n, _p(g["means"]), _p(g["scales"]), _p(g["quats"]), _p(g["opacity"]),
                       _p(g["intensity"]), len(cams), cam_array(cams), C.byref(s), _p(dl),
                       1 if binned is not None else 0, _p(vals), _p(rng), _p(sl),
                       _p(_u8(flip)), _p(out["means"]), _p(out["scales"]), _p(out["quats"]),
                       _p(out["opacity"]), _p(out["intensity"]), _p(g2d))
    if want_2d:
        out["g2d"] = g2d
    return out


def render_views(g: dict, cams, st: Settings) -> dict:
    """Brute-force images of several views, concatenated (small scenes)."""
    parts = [render_brute(g, c, st) for c in cams]
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
