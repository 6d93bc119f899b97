"""CPU FP64 oracle for MOREA objective evaluation -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the product path never imports it.  It shares no code with the HIP
library: the C source ``morea_oracle.c`` is built here with gcc (no fast-math)
and driven through ctypes.

Functions follow the paper's definitions (see the header of
``morea_oracle.c`` for the sections each one follows and the readings taken
where the paper is silent).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "morea_oracle.c")
LIB = os.path.join(HERE, "libmorea_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 -fopenmp (no fast-math, no contraction
    of a * b + c into one rounding: the Sobol sample points are formed with
    explicit fmaf only)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("MOREA_ORACLE_LIB")   # a mutant build, used by the mutation test
        if path is None:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build(force=True)
            path = LIB
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.oracle_eval.argtypes = [P, P, ctypes.c_int, P, P, P, P, P]
        L.oracle_eval.restype = ctypes.c_int
        L.oracle_distance_map.argtypes = [ctypes.c_int] * 4 + [P, P]
        L.oracle_tet_voxels.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
        L.oracle_tet_voxels.restype = ctypes.c_int
        L.oracle_map.argtypes = [P, P, P, P, P]
        L.oracle_map.restype = ctypes.c_int
        L.oracle_trilinear.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
        L.oracle_trilinear.restype = ctypes.c_double
        L.oracle_orient.argtypes = [P]
        L.oracle_orient.restype = ctypes.c_double
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_eval_sobol.argtypes = [P, P, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, P, P, P, P, P]
        L.oracle_eval_sobol.restype = ctypes.c_int
        L.oracle_sobol_coord.argtypes = [ctypes.c_int, ctypes.c_uint32]
        L.oracle_sobol_coord.restype = ctypes.c_uint32
        L.oracle_neg_ln_f32.argtypes = [ctypes.c_float]
        L.oracle_neg_ln_f32.restype = ctypes.c_float
        L.oracle_sobol_points.argtypes = [P, P, ctypes.c_int, ctypes.c_uint64, ctypes.c_double, P, P,
                                          ctypes.c_int64]
        L.oracle_sobol_points.restype = ctypes.c_int64
        L.oracle_dvf.argtypes = [P, P, P, P, P]
        L.oracle_dvf.restype = ctypes.c_int
        L.oracle_point_guidance.argtypes = [P, P, P, P, ctypes.c_int, P, P]
        L.oracle_point_guidance.restype = ctypes.c_int
        _lib = L
    return _lib


class _CProblem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("img_s", ctypes.c_void_p), ("img_t", ctypes.c_void_p),
                ("n_points", ctypes.c_int), ("n_tets", ctypes.c_int),
                ("tets", ctypes.c_void_p), ("ref_points", ctypes.c_void_p),
                ("elasticity", ctypes.c_void_p), ("n_sets", ctypes.c_int),
                ("set_off_s", ctypes.c_void_p), ("set_off_t", ctypes.c_void_p),
                ("dmap_s", ctypes.c_void_p), ("dmap_t", ctypes.c_void_p),
                ("radius", ctypes.c_float)]


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


def distance_map(dims, points) -> np.ndarray:
    """d(p, C) at all voxel centres of a grid of ``dims`` = (nx, ny, nz), FP32."""
    nx, ny, nz = dims
    pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
    out = np.empty((nz, ny, nx), dtype=np.float32)
    lib().oracle_distance_map(nx, ny, nz, pts.shape[0], _ptr(pts), _ptr(out))
    return out


class Problem:
    """Problem data as the oracle sees it (all arrays host, contiguous)."""

    def __init__(self, dims, image_src, image_tgt, tets, ref_points, elasticity, sets_src, sets_tgt,
                 radius):
        self.dims = tuple(int(d) for d in dims)
        nx, ny, nz = self.dims
        self.image_src = np.ascontiguousarray(image_src, dtype=np.float32).reshape(nz, ny, nx)
        self.image_tgt = np.ascontiguousarray(image_tgt, dtype=np.float32).reshape(nz, ny, nx)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.ref_points = np.ascontiguousarray(ref_points, dtype=np.float32)
        self.elasticity = np.ascontiguousarray(elasticity, dtype=np.float32)
        self.sets_src = [np.ascontiguousarray(s, dtype=np.float32).reshape(-1, 3) for s in sets_src]
        self.sets_tgt = [np.ascontiguousarray(s, dtype=np.float32).reshape(-1, 3) for s in sets_tgt]
        self.radius = float(np.float32(radius))
        self.set_off_s = np.cumsum([0] + [len(s) for s in self.sets_src]).astype(np.int32)
        self.set_off_t = np.cumsum([0] + [len(s) for s in self.sets_tgt]).astype(np.int32)
        n = len(self.sets_src)
        self.dmap_s = np.stack([distance_map(self.dims, s) for s in self.sets_src]) if n else \
            np.zeros((0, nz, ny, nx), np.float32)
        self.dmap_t = np.stack([distance_map(self.dims, s) for s in self.sets_tgt]) if n else \
            np.zeros((0, nz, ny, nx), np.float32)
        self._c = _CProblem(nx, ny, nz, self.image_src.ctypes.data, self.image_tgt.ctypes.data,
                            self.ref_points.shape[0], self.tets.shape[0], self.tets.ctypes.data,
                            self.ref_points.ctypes.data, self.elasticity.ctypes.data, n,
                            self.set_off_s.ctypes.data, self.set_off_t.ctypes.data,
                            self.dmap_s.ctypes.data, self.dmap_t.ctypes.data, self.radius)

    @classmethod
    def from_synth(cls, p, image_src=None, image_tgt=None):
        return cls(p.dims, p.image_src if image_src is None else image_src,
                   p.image_tgt if image_tgt is None else image_tgt, p.tets, p.ref_points,
                   p.elasticity, p.sets_src, p.sets_tgt, p.radius)

    @property
    def n_points(self):
        return self.ref_points.shape[0]

    @property
    def n_tets(self):
        return self.tets.shape[0]

    def evaluate(self, pts, records=False):
        """Full evaluation of candidates ``pts`` float32 [pop][2][3][n_points].

        Returns a dict with obj [pop][3] (intensity, magnitude, guidance),
        flags [pop] (bit0 source fold, bit1 target fold, bit2 invalid),
        severity [pop], counts [pop][2] (|P_s|, |P_t|) and, with
        ``records``, per-(candidate, tet, direction) records
        [pop][n_tets][2][6] = (h sum, guidance sum, samples, magnitude,
        violating volume, violation 1/0)."""
        pts = np.ascontiguousarray(pts, dtype=np.float32)
        pop = pts.shape[0]
        assert pts.shape[1:] == (2, 3, self.n_points), pts.shape
        obj = np.empty((pop, 3), np.float64)
        flags = np.empty(pop, np.uint8)
        sev = np.empty(pop, np.float64)
        counts = np.empty((pop, 2), np.int64)
        rec = np.empty((pop, self.n_tets, 2, 6), np.float64) if records else None
        lib().oracle_eval(ctypes.byref(self._c), _ptr(pts), pop, _ptr(obj), _ptr(flags), _ptr(sev),
                          _ptr(counts), _ptr(rec))
        out = dict(obj=obj, flags=flags, severity=sev, counts=counts)
        if records:
            out["records"] = rec
        return out

    def point_guidance(self, pts):
        """Point-based guidance error of candidates pts [pop][2][3][n_points]
        (the prior work's form that Sec. 4.1.3 replaces): mean over all points c
        of C_s of the squared distance from T(c) to the closest point of the
        set's C_t.  Returns (f [pop] FP64, unmapped [pop] points in no tet)."""
        pts = np.ascontiguousarray(pts, dtype=np.float32)
        pop = pts.shape[0]
        assert pts.shape[1:] == (2, 3, self.n_points), pts.shape
        cs = np.ascontiguousarray(np.concatenate(self.sets_src) if self.sets_src else np.zeros((1, 3)),
                                  dtype=np.float32)
        ct = np.ascontiguousarray(np.concatenate(self.sets_tgt) if self.sets_tgt else np.zeros((1, 3)),
                                  dtype=np.float32)
        f = np.empty(pop, np.float64)
        unmapped = np.empty(pop, np.int32)
        lib().oracle_point_guidance(ctypes.byref(self._c), _ptr(cs), _ptr(ct), _ptr(pts), pop, _ptr(f),
                                    _ptr(unmapped))
        return f, unmapped

    def dvf(self, cand):
        """Forward and inverse deformation vector fields of one candidate
        cand float32 [2][3][n_points] (Sec. 5.4): fwd, inv [nz][ny][nx][3]
        (FP64 displacements q - p in voxels), cover [2][nz][ny][nx] (tets
        containing each voxel centre)."""
        c = np.ascontiguousarray(cand, dtype=np.float32)
        assert c.shape == (2, 3, self.n_points), c.shape
        nx, ny, nz = self.dims
        fwd = np.empty((nz, ny, nx, 3), np.float64)
        inv = np.empty((nz, ny, nx, 3), np.float64)
        cover = np.empty((2, nz, ny, nx), np.int32)
        lib().oracle_dvf(ctypes.byref(self._c), _ptr(c), _ptr(fwd), _ptr(inv), _ptr(cover))
        return fwd, inv, cover

    def evaluate_sobol(self, pts, rate=1.0, seed=0, records=False):
        """The same outputs from the Sobol-sampled estimator (App. A.2):
        round(rate * volume) random barycentric points per tet and direction,
        the sequence seeded from ``seed`` and the tet's coordinates; counts
        are the numbers of points."""
        pts = np.ascontiguousarray(pts, dtype=np.float32)
        pop = pts.shape[0]
        assert pts.shape[1:] == (2, 3, self.n_points), pts.shape
        obj = np.empty((pop, 3), np.float64)
        flags = np.empty(pop, np.uint8)
        sev = np.empty(pop, np.float64)
        counts = np.empty((pop, 2), np.int64)
        rec = np.empty((pop, self.n_tets, 2, 6), np.float64) if records else None
        if lib().oracle_eval_sobol(ctypes.byref(self._c), _ptr(pts), pop, float(rate), int(seed), _ptr(obj),
                                   _ptr(flags), _ptr(sev), _ptr(counts), _ptr(rec)) != 0:
            raise ValueError("rate must be > 0")
        out = dict(obj=obj, flags=flags, severity=sev, counts=counts)
        if records:
            out["records"] = rec
        return out


def tet_voxels(verts, dims) -> np.ndarray:
    """Flat indices of the voxel centres inside one tet (tie rule applied)."""
    v = np.ascontiguousarray(verts, dtype=np.float32).reshape(12)
    nx, ny, nz = dims
    cap = nx * ny * nz
    out = np.empty(cap, np.int32)
    n = lib().oracle_tet_voxels(_ptr(v), nx, ny, nz, _ptr(out), cap)
    return out[:n].copy()


def map_point(own, oth, p):
    """Barycentric map of integer voxel ``p`` from tet ``own`` to tet ``oth``."""
    a = np.ascontiguousarray(own, dtype=np.float32).reshape(12)
    b = np.ascontiguousarray(oth, dtype=np.float32).reshape(12)
    pi = np.ascontiguousarray(p, dtype=np.int32).reshape(3)
    q = np.empty(3, np.float64)
    ex = np.empty(3, np.int32)
    if lib().oracle_map(_ptr(a), _ptr(b), _ptr(pi), _ptr(q), _ptr(ex)) != 0:
        raise ValueError("degenerate tet")
    return q, ex.astype(bool)


def trilinear(img, q, clamp=False) -> float:
    img = np.ascontiguousarray(img, dtype=np.float32)
    nz, ny, nx = img.shape
    qq = np.ascontiguousarray(q, dtype=np.float64).reshape(3)
    return lib().oracle_trilinear(_ptr(img), nx, ny, nz, _ptr(qq), int(clamp))


def orient(verts) -> float:
    """6 x signed volume of a tet in units of 2^-30 voxel^3 (exact integer)."""
    v = np.ascontiguousarray(verts, dtype=np.float32).reshape(12)
    return lib().oracle_orient(_ptr(v))


def quantize(img, storage: str) -> np.ndarray:
    """Round FP32 values to the reduced storage type (nearest, ties to even)
    and return them exactly upcast to FP32."""
    a = np.ascontiguousarray(img, dtype=np.float32)
    if storage == "f32":
        return a.copy()
    if storage == "f16":
        return a.astype(np.float16).astype(np.float32)
    if storage == "bf16":
        u = a.view(np.uint32).astype(np.uint64)
        rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
        return (rounded.astype(np.uint32) << 16).view(np.float32)
    raise ValueError(storage)


def sobol_coord(j: int, n: int) -> int:
    """Coordinate j (0..3) of point n of the unshifted 4-D Sobol sequence, as
    a 32-bit integer (natural order)."""
    return int(lib().oracle_sobol_coord(int(j), int(n)))


def neg_ln_f32(r: float) -> float:
    """-ln(r) as the Sobol estimator computes it in FP32."""
    return float(lib().oracle_neg_ln_f32(float(r)))


def sobol_points(own, oth, direction=0, seed=0, rate=1.0, cap=1 << 20):
    """Sample points of one tet: p [N][3] in ``own``, q [N][3] in ``oth``
    (vertices float32 [4][3])."""
    a = np.ascontiguousarray(own, dtype=np.float32).reshape(12)
    b = np.ascontiguousarray(oth, dtype=np.float32).reshape(12)
    p = np.empty((cap, 3), np.float32)
    q = np.empty((cap, 3), np.float32)
    n = lib().oracle_sobol_points(_ptr(a), _ptr(b), int(direction), int(seed), float(rate), _ptr(p), _ptr(q),
                                  int(cap))
    if n < 0:
        raise ValueError("rate must be > 0")
    m = min(n, cap)
    return p[:m].copy(), q[:m].copy(), int(n)


def threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    """Set the threads of the oracle's OpenMP loops."""
    lib().oracle_set_threads(int(n))


def timed_evaluate(problem: Problem, pts):
    t = time.perf_counter()
    out = problem.evaluate(pts)
    return out, time.perf_counter() - t
