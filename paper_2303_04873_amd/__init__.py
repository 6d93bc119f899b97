"""Python binding of libmorea (MOREA objective evaluation on MI355X).

Argument marshalling only: every step of an evaluation runs in the HIP
kernels of ``libmorea.so``.  The functions carry the names of the C-ABI
(``include/morea.h``); :class:`Problem` bundles them for device tensors.
PyTorch provides device memory and streams.  The library must be built
(``python paper_2303_04873_amd/build.py``); importing the binding without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MOREA_LIB names another build of the same library (e.g. one whose host code
# carries sanitizers); by default the in-tree build is loaded
LIB_PATH = os.environ.get("MOREA_LIB") or os.path.join(HERE, "libmorea.so")

MOREA_OK, MOREA_EINVAL, MOREA_ENOMEM, MOREA_EDEVICE, MOREA_ERANGE, MOREA_ESTATE = 0, -1, -2, -3, -4, -5
STORE = {"f32": 0, "bf16": 1, "f16": 2}

EXPORTS = ["morea_problem_create", "morea_problem_destroy", "morea_cache_bytes", "morea_eval_full",
           "morea_eval_sobol", "morea_repair_folds", "morea_rasterize_dvf", "morea_rasterize_dvf_static",
           "morea_point_guidance",
           "morea_build_fos",
           "morea_set_groups", "morea_reserve_partial", "morea_eval_partial", "morea_accept_partial", "morea_select_clusters",
           "morea_archive_clear", "morea_archive_update", "morea_mark_improvements", "morea_adapt_multipliers",
           "morea_mixing_bytes", "morea_estimate_distributions", "morea_sample_partial",
           "morea_debug_distance_map", "morea_tune_partial", "morea_partial_shape", "morea_set_partial_shape",
           "morea_partial_graphs",
           "morea_surrogate_num_params", "morea_surrogate_num_features", "morea_surrogate_create",
           "morea_surrogate_destroy", "morea_surrogate_features", "morea_surrogate_targets",
           "morea_surrogate_train_step",
           "morea_surrogate_gradients", "morea_surrogate_predict_rows", "morea_surrogate_prescreen",
           "morea_surrogate_scale", "morea_surrogate_select", "morea_surrogate_get_params", "morea_surrogate_set_params",
           "morea_surrogate_stats", "morea_last_error"]


class MoreaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libmorea status {status}: {msg}")
        self.status = status


class morea_problem_desc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3),
                ("image_src", ctypes.c_void_p), ("image_tgt", ctypes.c_void_p),
                ("storage", ctypes.c_int32),
                ("n_points", ctypes.c_int32), ("n_tets", ctypes.c_int32),
                ("tets", ctypes.c_void_p), ("ref_points", ctypes.c_void_p),
                ("elasticity", ctypes.c_void_p),
                ("n_sets", ctypes.c_int32),
                ("set_off_src", ctypes.c_void_p), ("set_off_tgt", ctypes.c_void_p),
                ("set_pts_src", ctypes.c_void_p), ("set_pts_tgt", ctypes.c_void_p),
                ("radius", ctypes.c_float), ("max_population", ctypes.c_int32)]


_lib = None


def load_library():
    """Load libmorea.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2303_04873_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, I32 = ctypes.c_void_p, ctypes.c_int32
    L.morea_problem_create.argtypes = [ctypes.POINTER(morea_problem_desc), ctypes.POINTER(P)]
    L.morea_problem_create.restype = I32
    L.morea_problem_destroy.argtypes = [P]
    L.morea_problem_destroy.restype = None
    L.morea_cache_bytes.argtypes = [P, I32]
    L.morea_cache_bytes.restype = ctypes.c_size_t
    L.morea_eval_full.argtypes = [P, P, I32, P, P, P, P, P, P]
    L.morea_eval_full.restype = I32
    L.morea_eval_sobol.argtypes = [P, P, I32, ctypes.c_float, ctypes.c_uint64, P, P, P, P, P]
    L.morea_eval_sobol.restype = I32
    L.morea_repair_folds.argtypes = [P, P, I32, P, I32, P, P, P]
    L.morea_repair_folds.restype = I32
    L.morea_rasterize_dvf.argtypes = [P, P, P, P, P, P, P]
    L.morea_rasterize_dvf.restype = I32
    L.morea_rasterize_dvf_static.argtypes = [P, P, P, P, P, P]
    L.morea_rasterize_dvf_static.restype = I32
    L.morea_point_guidance.argtypes = [P, P, I32, P, P, P]
    L.morea_point_guidance.restype = I32
    L.morea_build_fos.argtypes = [I32, I32, P, I32, P, P, P, P]
    L.morea_build_fos.restype = I32
    L.morea_set_groups.argtypes = [P, I32, P, P]
    L.morea_set_groups.restype = I32
    L.morea_reserve_partial.argtypes = [P, I32]
    L.morea_reserve_partial.restype = I32
    L.morea_eval_partial.argtypes = [P, P, I32, P, I32, P, P, P, P, P, P, P, P]
    L.morea_eval_partial.restype = I32
    L.morea_accept_partial.argtypes = [P, P, I32, P, I32, P, P, P, P, P, P, P, P, P, P, P, I32, ctypes.c_float, P,
                                       P]
    L.morea_accept_partial.restype = I32
    L.morea_select_clusters.argtypes = [P, P, P, I32, I32, I32, ctypes.c_float, P, P, P, P, I32, P, P]
    L.morea_select_clusters.restype = I32
    L.morea_archive_clear.argtypes = [I32, P, P, P, P, P]
    L.morea_archive_clear.restype = I32
    L.morea_archive_update.argtypes = [I32, P, P, P, P, I32, ctypes.c_float, I32, P, P, P, P, P, P, P, P]
    L.morea_archive_update.restype = I32
    L.morea_mark_improvements.argtypes = [I32, P, P, P, P, I32, P, I32, I32, P, P]
    L.morea_mark_improvements.restype = I32
    L.morea_adapt_multipliers.argtypes = [I32, I32, P, P, P, P]
    L.morea_adapt_multipliers.restype = I32
    L.morea_mixing_bytes.argtypes = [P, I32]
    L.morea_mixing_bytes.restype = ctypes.c_size_t
    L.morea_estimate_distributions.argtypes = [P, P, I32, I32, P, P, I32, P, P, ctypes.c_size_t, P]
    L.morea_estimate_distributions.restype = I32
    L.morea_sample_partial.argtypes = [P, P, I32, P, ctypes.c_size_t, I32, P, I32, P, P, P, P, P, P, P]
    L.morea_sample_partial.restype = I32
    L.morea_tune_partial.argtypes = [P, P, I32, P, I32, P, P, P, P, P, P, P, P, P]
    L.morea_tune_partial.restype = I32
    L.morea_partial_shape.argtypes = [P, P, P]
    L.morea_partial_shape.restype = I32
    L.morea_set_partial_shape.argtypes = [P, I32, I32]
    L.morea_set_partial_shape.restype = I32
    L.morea_partial_graphs.argtypes = [P, P, P]
    L.morea_partial_graphs.restype = I32
    L.morea_debug_distance_map.argtypes = [P, I32, I32, P, P]
    L.morea_debug_distance_map.restype = I32
    L.morea_surrogate_num_params.argtypes = []
    L.morea_surrogate_num_params.restype = I32
    L.morea_surrogate_num_features.argtypes = []
    L.morea_surrogate_num_features.restype = I32
    L.morea_surrogate_create.argtypes = [P, I32, ctypes.c_uint64, ctypes.POINTER(P)]
    L.morea_surrogate_create.restype = I32
    L.morea_surrogate_destroy.argtypes = [P]
    L.morea_surrogate_destroy.restype = None
    L.morea_surrogate_predict_rows.argtypes = [P, P, I32, P, P]
    L.morea_surrogate_predict_rows.restype = I32
    L.morea_surrogate_targets.argtypes = [P, P, I32, P, I32, P, P, P]
    L.morea_surrogate_targets.restype = I32
    L.morea_surrogate_scale.argtypes = [P, P]
    L.morea_surrogate_scale.restype = I32
    for name in ["features", "prescreen"]:
        f = getattr(L, "morea_surrogate_" + name)
        f.argtypes = [P, P, I32, P, I32, P, P, P, P]
        f.restype = I32
    L.morea_surrogate_train_step.argtypes = [P, P, P, I32, ctypes.c_float, P, P]
    L.morea_surrogate_train_step.restype = I32
    L.morea_surrogate_gradients.argtypes = [P, P, P, I32, P, P, P]
    L.morea_surrogate_gradients.restype = I32
    L.morea_surrogate_select.argtypes = [P, I32, I32, P, I32, P, P, P]
    L.morea_surrogate_select.restype = I32
    for name in ["get_params", "set_params"]:
        f = getattr(L, "morea_surrogate_" + name)
        f.argtypes = [P, P]
        f.restype = I32
    L.morea_surrogate_stats.argtypes = [P, P, P]
    L.morea_surrogate_stats.restype = I32
    L.morea_last_error.argtypes = []
    L.morea_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def morea_last_error() -> str:
    return load_library().morea_last_error().decode()


def _check(status):
    if status != MOREA_OK:
        raise MoreaError(status, morea_last_error())


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def morea_problem_create(desc: morea_problem_desc) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load_library().morea_problem_create(ctypes.byref(desc), ctypes.byref(h)))
    return h


def morea_problem_destroy(handle):
    load_library().morea_problem_destroy(handle)


def morea_cache_bytes(handle, pop: int) -> int:
    return load_library().morea_cache_bytes(handle, pop)


def morea_eval_full(handle, pts, pop, obj, flags, severity, counts, cache, stream):
    _check(load_library().morea_eval_full(handle, _dev_ptr(pts), pop, _dev_ptr(obj), _dev_ptr(flags),
                                          _dev_ptr(severity), _dev_ptr(counts), _dev_ptr(cache),
                                          _stream_ptr(stream)))


def morea_eval_sobol(handle, pts, pop, rate, seed, obj, flags, severity, counts, stream):
    _check(load_library().morea_eval_sobol(handle, _dev_ptr(pts), pop, float(rate), int(seed), _dev_ptr(obj),
                                           _dev_ptr(flags), _dev_ptr(severity), _dev_ptr(counts),
                                           _stream_ptr(stream)))


def build_fos(n_points, tets):
    """Linkage model (Sec. 4.2.1) of a mesh: (elements int32 [n][2], colours
    int32 [n], number of colours) -- host arrays, computed by the library."""
    t = np.ascontiguousarray(tets, dtype=np.int32)
    ep = np.empty((n_points, 2), np.int32)
    col = np.empty(n_points, np.int32)
    ne, nc = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().morea_build_fos(n_points, len(t), t.ctypes.data_as(ctypes.c_void_p), n_points,
                                          ep.ctypes.data_as(ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.byref(ne), ctypes.byref(nc)))
    return ep[:ne.value].copy(), col[:ne.value].copy(), nc.value


def morea_set_groups(handle, grp_off, grp_pts):
    off = _host(grp_off, np.int32)
    pts = _host(grp_pts, np.int32)
    _check(load_library().morea_set_groups(handle, len(off) - 1, off.ctypes.data_as(ctypes.c_void_p),
                                           pts.ctypes.data_as(ctypes.c_void_p)))


def morea_reserve_partial(handle, max_evals: int):
    _check(load_library().morea_reserve_partial(handle, max_evals))


def morea_eval_partial(handle, parent_pts, n_parents, parent_cache, n_evals, eval_parent, eval_group,
                       new_coords, obj, flags, severity, counts, stream):
    _check(load_library().morea_eval_partial(
        handle, _dev_ptr(parent_pts), n_parents, _dev_ptr(parent_cache), n_evals,
        _dev_ptr(eval_parent), _dev_ptr(eval_group), _dev_ptr(new_coords), _dev_ptr(obj),
        _dev_ptr(flags), _dev_ptr(severity), _dev_ptr(counts), _stream_ptr(stream)))


def morea_accept_partial(handle, parent_pts, n_parents, parent_cache, n_evals, eval_parent, eval_group,
                         new_coords, child_obj, child_flags, child_sev, parent_obj, parent_flags, parent_sev,
                         parent_counts, archive_obj, n_archive, guidance_max, accepted, stream):
    _check(load_library().morea_accept_partial(
        handle, _dev_ptr(parent_pts), n_parents, _dev_ptr(parent_cache), n_evals,
        _dev_ptr(eval_parent), _dev_ptr(eval_group), _dev_ptr(new_coords), _dev_ptr(child_obj),
        _dev_ptr(child_flags), _dev_ptr(child_sev), _dev_ptr(parent_obj), _dev_ptr(parent_flags),
        _dev_ptr(parent_sev), _dev_ptr(parent_counts), _dev_ptr(archive_obj), n_archive, guidance_max,
        _dev_ptr(accepted), _stream_ptr(stream)))


def select_clusters(out, size, k, guidance_max=None, stream=None):
    """Selection and clustering (Sec. 3) of a population from its evaluation
    outputs `out` (obj, flags, severity CUDA tensors).  Returns a dict of CUDA
    int32 tensors: selection, n_selected [1], clu_off [k + 1], clu_members,
    cluster_of; clu_members is sized k * ceil(2 min(size, n) / k)."""
    import torch
    n = out["flags"].shape[0]
    s = min(size, n)
    cap = max(1, k * ((2 * s + k - 1) // k))
    dev = out["flags"].device
    res = dict(selection=torch.empty(n, dtype=torch.int32, device=dev),
               n_selected=torch.empty(1, dtype=torch.int32, device=dev),
               clu_off=torch.empty(k + 1, dtype=torch.int32, device=dev),
               clu_members=torch.empty(cap, dtype=torch.int32, device=dev),
               cluster_of=torch.empty(n, dtype=torch.int32, device=dev))
    _check(load_library().morea_select_clusters(
        _dev_ptr(out["obj"]), _dev_ptr(out["flags"]), _dev_ptr(out["severity"]), n, int(size), int(k),
        float("inf") if guidance_max is None else float(guidance_max), _dev_ptr(res["selection"]),
        _dev_ptr(res["n_selected"]), _dev_ptr(res["clu_off"]), _dev_ptr(res["clu_members"]), cap,
        _dev_ptr(res["cluster_of"]), _stream_ptr(stream)))
    return res


class Archive:
    """Elitist archive in device memory (morea_archive_clear / _update):
    obj [capacity][3], stamp [capacity], pts [capacity][2][3][n_points] (or
    None), state [4], best [1] -- torch CUDA tensors owned by this object."""

    def __init__(self, capacity, n_points=0, stream=None):
        import torch
        self.capacity = int(capacity)
        self.n_points = int(n_points)
        dev = "cuda"
        self.obj = torch.empty((self.capacity, 3), dtype=torch.float32, device=dev)
        self.stamp = torch.empty(self.capacity, dtype=torch.int32, device=dev)
        self.pts = (torch.empty((self.capacity, 2, 3, self.n_points), dtype=torch.float32, device=dev)
                    if self.n_points else None)
        self.state = torch.empty(4, dtype=torch.int32, device=dev)
        self.best = torch.empty(1, dtype=torch.float32, device=dev)
        self.clear(stream)

    def clear(self, stream=None):
        _check(load_library().morea_archive_clear(self.capacity, _dev_ptr(self.obj), _dev_ptr(self.stamp),
                                                  _dev_ptr(self.state), _dev_ptr(self.best),
                                                  _stream_ptr(stream)))

    def update(self, out, pts=None, guidance_max=None, inserted=None, slot_of=None, stream=None):
        """Offer the solutions whose evaluation outputs are `out` (obj, flags,
        severity) and, when the archive keeps points, their points `pts`.
        Returns (inserted uint8 [n], slot_of int32 [n])."""
        import torch
        n = out["flags"].shape[0]
        if inserted is None:
            inserted = torch.empty(n, dtype=torch.uint8, device="cuda")
        if slot_of is None:
            slot_of = torch.empty(n, dtype=torch.int32, device="cuda")
        if (pts is None) != (self.pts is None):
            raise ValueError("points are offered exactly when the archive keeps them")
        _check(load_library().morea_archive_update(
            n, _dev_ptr(out["obj"]), _dev_ptr(out["flags"]), _dev_ptr(out["severity"]), _dev_ptr(pts),
            self.n_points, float("inf") if guidance_max is None else float(guidance_max), self.capacity,
            _dev_ptr(self.obj), _dev_ptr(self.stamp), _dev_ptr(self.pts), _dev_ptr(self.state),
            _dev_ptr(self.best), _dev_ptr(inserted), _dev_ptr(slot_of), _stream_ptr(stream)))
        return inserted, slot_of


def morea_mark_improvements(eval_parent, eval_group, eval_cluster, accepted, parent_inserted, improved,
                            stream=None):
    """improved: uint8 CUDA [n_clusters][n_groups] (marks set in place)."""
    _check(load_library().morea_mark_improvements(
        eval_parent.shape[0], _dev_ptr(eval_parent), _dev_ptr(eval_group), _dev_ptr(eval_cluster),
        _dev_ptr(accepted), parent_inserted.shape[0], _dev_ptr(parent_inserted), improved.shape[0],
        improved.shape[1], _dev_ptr(improved), _stream_ptr(stream)))


def morea_adapt_multipliers(improved, mult, no_improvement, stream=None):
    """improved uint8, mult float32, no_improvement int32: CUDA [k][n_groups]."""
    _check(load_library().morea_adapt_multipliers(improved.shape[0], improved.shape[1], _dev_ptr(improved),
                                                  _dev_ptr(mult), _dev_ptr(no_improvement),
                                                  _stream_ptr(stream)))


def morea_tune_partial(handle, parent_pts, n_parents, parent_cache, n_evals, eval_parent, eval_group,
                       new_coords, obj, flags, severity, counts, stream) -> float:
    best = ctypes.c_float()
    _check(load_library().morea_tune_partial(
        handle, _dev_ptr(parent_pts), n_parents, _dev_ptr(parent_cache), n_evals,
        _dev_ptr(eval_parent), _dev_ptr(eval_group), _dev_ptr(new_coords), _dev_ptr(obj),
        _dev_ptr(flags), _dev_ptr(severity), _dev_ptr(counts), _stream_ptr(stream),
        ctypes.byref(best)))
    return best.value


def morea_partial_shape(handle):
    b, c = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().morea_partial_shape(handle, ctypes.byref(b), ctypes.byref(c)))
    return b.value, c.value


def morea_set_partial_shape(handle, blocks, chunk):
    _check(load_library().morea_set_partial_shape(handle, int(blocks), int(chunk)))


def morea_partial_graphs(handle):
    """(graphs held by the partial-evaluation cache, graphs captured so far)."""
    n, c = ctypes.c_int32(), ctypes.c_int64()
    _check(load_library().morea_partial_graphs(handle, ctypes.byref(n), ctypes.byref(c)))
    return n.value, c.value


def morea_debug_distance_map(handle, image: int, set_index: int, shape):
    out = np.empty(shape, np.float32)
    band = np.empty(shape, np.uint8)
    _check(load_library().morea_debug_distance_map(handle, image, set_index,
                                                   out.ctypes.data_as(ctypes.c_void_p),
                                                   band.ctypes.data_as(ctypes.c_void_p)))
    return out, band


class Problem:
    """A problem on the current GPU; candidates and outputs are torch tensors."""

    def __init__(self, dims, image_src, image_tgt, tets, ref_points, elasticity, sets_src=(),
                 sets_tgt=(), radius=0.0, storage="f32", max_population=1):
        nx, ny, nz = (int(d) for d in dims)
        self.dims = (nx, ny, nz)
        self._keep = []

        def host(a, dt):
            h = _host(a, dt)
            self._keep.append(h)
            return h.ctypes.data

        sets_src = [np.asarray(s, np.float32).reshape(-1, 3) for s in sets_src]
        sets_tgt = [np.asarray(s, np.float32).reshape(-1, 3) for s in sets_tgt]
        n_sets = len(sets_src)
        off_s = np.cumsum([0] + [len(s) for s in sets_src]).astype(np.int32)
        off_t = np.cumsum([0] + [len(s) for s in sets_tgt]).astype(np.int32)
        pts_s = np.concatenate(sets_src) if n_sets else np.zeros((1, 3), np.float32)
        pts_t = np.concatenate(sets_tgt) if n_sets else np.zeros((1, 3), np.float32)
        tets = _host(tets, np.int32)
        ref_points = _host(ref_points, np.float32)
        d = morea_problem_desc()
        d.dims[:] = [nx, ny, nz]
        d.image_src = host(image_src, np.float32)
        d.image_tgt = host(image_tgt, np.float32)
        d.storage = STORE[storage]
        d.n_points = ref_points.shape[0]
        d.n_tets = tets.shape[0]
        d.tets = host(tets, np.int32)
        d.ref_points = host(ref_points, np.float32)
        d.elasticity = host(elasticity, np.float32)
        d.n_sets = n_sets
        d.set_off_src = host(off_s, np.int32)
        d.set_off_tgt = host(off_t, np.int32)
        d.set_pts_src = host(pts_s, np.float32)
        d.set_pts_tgt = host(pts_t, np.float32)
        d.radius = float(radius)
        d.max_population = int(max_population)
        self.n_points = d.n_points
        self.n_tets = d.n_tets
        self.tets_host = tets
        self.n_sets = n_sets
        self.max_population = int(max_population)
        self.handle = morea_problem_create(d)
        self._keep = []

    @classmethod
    def from_synth(cls, p, storage="f32", max_population=1, image_src=None, image_tgt=None):
        return cls(p.dims, p.image_src if image_src is None else image_src,
                   p.image_tgt if image_tgt is None else image_tgt, p.tets, p.ref_points,
                   p.elasticity, p.sets_src, p.sets_tgt, p.radius, storage, max_population)

    def close(self):
        if getattr(self, "handle", None):
            morea_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cache_bytes(self, pop):
        return morea_cache_bytes(self.handle, pop)

    def new_cache(self, pop):
        import torch
        return torch.empty(self.cache_bytes(pop), dtype=torch.uint8, device="cuda")

    def cache_records(self, cache, pop):
        """The per-(candidate, tet, direction) records of a cache as a NumPy
        structured array [pop][n_tets][2] (fields h, g, n, mag, vol, bits)."""
        dt = np.dtype([("h", "<f4"), ("g", "<f4"), ("n", "<u4"), ("mag", "<f4"), ("vol", "<f4"),
                       ("bits", "<u4")])
        assert dt.itemsize == 24
        nbytes = pop * self.n_tets * 2 * dt.itemsize
        raw = cache[:nbytes].cpu().numpy()
        return raw.view(dt).reshape(pop, self.n_tets, 2)

    def outputs(self, n):
        import torch
        dev = "cuda"
        return dict(obj=torch.empty((n, 3), dtype=torch.float32, device=dev),
                    flags=torch.empty(n, dtype=torch.uint8, device=dev),
                    severity=torch.empty(n, dtype=torch.float32, device=dev),
                    counts=torch.empty((n, 2), dtype=torch.int32, device=dev))

    def eval_full(self, pts, cache=None, out=None, stream=None):
        """pts: float32 CUDA tensor [pop][2][3][n_points]."""
        assert pts.is_cuda and pts.dtype.is_floating_point and pts.is_contiguous()
        pop = pts.shape[0]
        assert tuple(pts.shape[1:]) == (2, 3, self.n_points)
        out = self.outputs(pop) if out is None else out
        morea_eval_full(self.handle, pts, pop, out["obj"], out["flags"], out["severity"],
                        out["counts"], cache, stream)
        return out

    def eval_sobol(self, pts, rate=1.0, seed=0, out=None, stream=None):
        """The random-sampling estimator (App. A.2): round(rate * volume)
        Sobol points per tet and direction; outputs as eval_full."""
        assert pts.is_cuda and pts.dtype.is_floating_point and pts.is_contiguous()
        pop = pts.shape[0]
        assert tuple(pts.shape[1:]) == (2, 3, self.n_points)
        out = self.outputs(pop) if out is None else out
        morea_eval_sobol(self.handle, pts, pop, rate, seed, out["obj"], out["flags"], out["severity"],
                         out["counts"], stream)
        return out

    def repair_folds(self, pts, draws, pinned=None, info=None, stream=None):
        """Fold repair in place (Sec. 4.3.1): pts float32 CUDA [pop][2][3][n_points],
        draws float32 CUDA [pop][K][64][3] standard normal, pinned uint8 CUDA
        [n_points] (bit a: axis a fixed) or None.  Returns info int32 [pop][2]
        (moves, outcome)."""
        import torch
        assert pts.is_cuda and pts.dtype == torch.float32 and pts.is_contiguous()
        pop = pts.shape[0]
        assert tuple(pts.shape[1:]) == (2, 3, self.n_points)
        assert draws.is_cuda and draws.dtype == torch.float32 and draws.is_contiguous()
        assert draws.shape[0] == pop and tuple(draws.shape[2:]) == (64, 3)
        if pinned is not None:
            assert pinned.is_cuda and pinned.dtype == torch.uint8 and pinned.numel() == self.n_points
        info = torch.empty((pop, 2), dtype=torch.int32, device="cuda") if info is None else info
        _check(load_library().morea_repair_folds(self.handle, _dev_ptr(pts), pop, _dev_ptr(draws), draws.shape[1],
                                                 _dev_ptr(pinned), _dev_ptr(info), _stream_ptr(stream)))
        return info

    def rasterize_dvf(self, cand, out=None, stream=None):
        """Forward and inverse DVF of one candidate cand float32 CUDA
        [2][3][n_points] (Sec. 5.4): dict fwd, inv [nz][ny][nx][3], cover
        [2][nz][ny][nx] (int32 tensor of the uint32 counts), work (owners)."""
        import torch
        assert cand.is_cuda and cand.dtype == torch.float32 and cand.is_contiguous()
        assert tuple(cand.shape) == (2, 3, self.n_points)
        nx, ny, nz = self.dims
        if out is None:
            out = dict(fwd=torch.empty((nz, ny, nx, 3), dtype=torch.float32, device="cuda"),
                       inv=torch.empty((nz, ny, nx, 3), dtype=torch.float32, device="cuda"),
                       cover=torch.empty((2, nz, ny, nx), dtype=torch.int32, device="cuda"),
                       work=torch.empty((2, nz, ny, nx), dtype=torch.int32, device="cuda"))
        _check(load_library().morea_rasterize_dvf(self.handle, _dev_ptr(cand), _dev_ptr(out["fwd"]),
                                                  _dev_ptr(out["inv"]), _dev_ptr(out["cover"]),
                                                  _dev_ptr(out["work"]), _stream_ptr(stream)))
        return out

    def rasterize_dvf_static(self, cand, out, stream=None):
        """The allocation-free variant (morea_rasterize_dvf_static): `out`
        holds preallocated fwd, inv, cover tensors as for rasterize_dvf; no
        workspace is passed and the call allocates nothing."""
        import torch
        assert cand.is_cuda and cand.dtype == torch.float32 and cand.is_contiguous()
        assert tuple(cand.shape) == (2, 3, self.n_points)
        _check(load_library().morea_rasterize_dvf_static(self.handle, _dev_ptr(cand), _dev_ptr(out["fwd"]),
                                                         _dev_ptr(out["inv"]), _dev_ptr(out["cover"]),
                                                         _stream_ptr(stream)))
        return out

    def point_guidance(self, pts, stream=None):
        """Point-based guidance error of candidates pts float32 CUDA
        [pop][2][3][n_points]: (f [pop] float32, unmapped [pop] int32)."""
        import torch
        assert pts.is_cuda and pts.dtype == torch.float32 and pts.is_contiguous()
        pop = pts.shape[0]
        assert tuple(pts.shape[1:]) == (2, 3, self.n_points)
        f = torch.empty(pop, dtype=torch.float32, device="cuda")
        un = torch.empty(pop, dtype=torch.int32, device="cuda")
        _check(load_library().morea_point_guidance(self.handle, _dev_ptr(pts), pop, _dev_ptr(f), _dev_ptr(un),
                                                   _stream_ptr(stream)))
        return f, un

    def set_groups(self, grp_off, grp_pts):
        morea_set_groups(self.handle, grp_off, grp_pts)
        self._group_sizes = np.diff(np.asarray(grp_off, dtype=np.int64))

    def mixing_workspace(self, n_clusters):
        """Device workspace of the optimal-mixing distributions (uint8 tensor)."""
        import torch
        n = load_library().morea_mixing_bytes(self.handle, int(n_clusters))
        if n == 0:
            raise MoreaError(MOREA_ESTATE, "call set_groups and reserve_partial first")
        return torch.empty(n, dtype=torch.uint8, device="cuda")

    def estimate_distributions(self, pts, clu_off, clu_members, work, pinned=None, stream=None):
        """Distributions of every (cluster, group) from the clusters' members
        (Sec. 3); clu_off int32 CUDA [k + 1], clu_members int32 CUDA."""
        n_clusters = clu_off.shape[0] - 1
        _check(load_library().morea_estimate_distributions(
            self.handle, _dev_ptr(pts), pts.shape[0], n_clusters, _dev_ptr(clu_off), _dev_ptr(clu_members),
            clu_members.shape[0], _dev_ptr(pinned), _dev_ptr(work), work.numel(), _stream_ptr(stream)))

    def sample_partial(self, pts, work, n_clusters, eval_parent, eval_group, eval_cluster, z, pinned=None,
                       mult=None, out=None, stream=None):
        """New coordinates [rows][2][3] of every evaluation sampled from its
        cluster's distribution of its group (Sec. 3)."""
        import torch
        if out is None:
            eg = eval_group.cpu().numpy()
            ok = (eg >= 0) & (eg < len(self._group_sizes))
            rows = int(self._group_sizes[eg[ok]].sum())
            out = torch.empty((rows, 2, 3), dtype=torch.float32, device="cuda")
        _check(load_library().morea_sample_partial(
            self.handle, _dev_ptr(pts), pts.shape[0], _dev_ptr(work), work.numel(), int(n_clusters), _dev_ptr(mult),
            eval_parent.shape[0], _dev_ptr(eval_parent), _dev_ptr(eval_group), _dev_ptr(eval_cluster), _dev_ptr(z),
            _dev_ptr(pinned), _dev_ptr(out), _stream_ptr(stream)))
        return out

    def reserve_partial(self, max_evals):
        morea_reserve_partial(self.handle, max_evals)

    def eval_partial(self, parent_pts, parent_cache, eval_parent, eval_group, new_coords, out=None,
                     stream=None):
        n = eval_parent.shape[0]
        out = self.outputs(n) if out is None else out
        morea_eval_partial(self.handle, parent_pts, parent_pts.shape[0], parent_cache, n,
                           eval_parent, eval_group, new_coords, out["obj"], out["flags"],
                           out["severity"], out["counts"], stream)
        return out

    def accept_partial(self, parent_pts, parent_cache, eval_parent, eval_group, new_coords, child, parent,
                       archive=None, guidance_max=None, accepted=None, stream=None):
        """Acceptance after eval_partial with the same first five arguments
        (Sec. 3): `child` the decision inputs (the outputs of eval_partial),
        `parent` the parents' outputs dict (rewritten with the evaluation of
        the updated parents), `archive` FP32 CUDA [m][3] or None,
        `guidance_max` the steering bound (None: off).  Updates
        parent_pts and parent_cache in place; returns `accepted` (uint8)."""
        import torch
        n = eval_parent.shape[0]
        if accepted is None:
            accepted = torch.empty(n, dtype=torch.uint8, device="cuda")
        m = 0 if archive is None else archive.shape[0]
        if archive is not None:
            assert archive.is_cuda and archive.dtype == torch.float32 and archive.is_contiguous()
        morea_accept_partial(self.handle, parent_pts, parent_pts.shape[0], parent_cache, n, eval_parent, eval_group,
                             new_coords, child["obj"], child["flags"], child["severity"], parent["obj"],
                             parent["flags"], parent["severity"], parent["counts"], archive if m else None, m,
                             float("inf") if guidance_max is None else float(guidance_max), accepted, stream)
        return accepted

    def tune_partial(self, parent_pts, parent_cache, eval_parent, eval_group, new_coords, out=None,
                     stream=None):
        n = eval_parent.shape[0]
        out = self.outputs(n) if out is None else out
        ms = morea_tune_partial(self.handle, parent_pts, parent_pts.shape[0], parent_cache, n,
                                eval_parent, eval_group, new_coords, out["obj"], out["flags"],
                                out["severity"], out["counts"], stream)
        return ms, morea_partial_shape(self.handle)

    def set_partial_shape(self, blocks, chunk):
        """Launch shape of partial evaluation: persistent (blocks, chunk) or
        (0, 0) for the grid form."""
        morea_set_partial_shape(self.handle, blocks, chunk)

    def partial_shape(self):
        return morea_partial_shape(self.handle)

    def distance_map(self, image, set_index):
        return morea_debug_distance_map(self.handle, image, set_index, self.dims[::-1])


class Surrogate:
    """The learned pre-screen (see include/morea.h); tensors are CUDA tensors."""

    def __init__(self, problem: "Problem", max_rows: int = 1 << 16, seed: int = 0):
        self.problem = problem
        self.n_params = load_library().morea_surrogate_num_params()
        self.n_features = load_library().morea_surrogate_num_features()
        h = ctypes.c_void_p()
        _check(load_library().morea_surrogate_create(problem.handle, int(max_rows), int(seed),
                                                     ctypes.byref(h)))
        self.handle = h
        self.max_rows = int(max_rows)

    def close(self):
        if getattr(self, "handle", None):
            load_library().morea_surrogate_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def features(self, pts, parent_pts, parent_cache, parent_of, stream=None):
        """Input rows [pop][n_tets][23] of offspring `pts` whose parents are
        `parent_pts` (evaluated into `parent_cache`); parent_of int32 CUDA
        [pop]."""
        import torch
        out = torch.empty((pts.shape[0], self.problem.n_tets, self.n_features), dtype=torch.float32,
                          device="cuda")
        _check(load_library().morea_surrogate_features(self.handle, _dev_ptr(pts), pts.shape[0],
                                                       _dev_ptr(parent_pts), parent_pts.shape[0],
                                                       _dev_ptr(parent_cache), _dev_ptr(parent_of),
                                                       _dev_ptr(out), _stream_ptr(stream)))
        return out

    @property
    def h_scale(self):
        """The mean of (I_s - I_t)^2 over the grid (1 when 0): the unit of
        the h-valued features, the targets and the predictions."""
        v = ctypes.c_float()
        _check(load_library().morea_surrogate_scale(self.handle, ctypes.byref(v)))
        return v.value

    def targets(self, cache, pop, parent_cache, n_parents, parent_of, stream=None):
        """Targets [pop][n_tets]: each offspring's per-tet mean term (from
        `cache`) minus its parent's (from `parent_cache`), over h_scale."""
        import torch
        out = torch.empty((pop, self.problem.n_tets), dtype=torch.float32, device="cuda")
        _check(load_library().morea_surrogate_targets(self.handle, _dev_ptr(cache), pop, _dev_ptr(parent_cache),
                                                      n_parents, _dev_ptr(parent_of), _dev_ptr(out),
                                                      _stream_ptr(stream)))
        return out

    def train_step(self, feats, targets, lr, loss_out=None, stream=None):
        n = targets.numel()
        _check(load_library().morea_surrogate_train_step(self.handle, _dev_ptr(feats), _dev_ptr(targets),
                                                         n, float(lr), _dev_ptr(loss_out),
                                                         _stream_ptr(stream)))

    def gradients(self, feats, targets, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(load_library().morea_surrogate_gradients(self.handle, _dev_ptr(feats), _dev_ptr(targets),
                                                        targets.numel(), _dev_ptr(g), _dev_ptr(loss),
                                                        _stream_ptr(stream)))
        return g, loss

    def predict_rows(self, feats, stream=None):
        import torch
        n = feats.numel() // self.n_features
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(load_library().morea_surrogate_predict_rows(self.handle, _dev_ptr(feats), n, _dev_ptr(y),
                                                           _stream_ptr(stream)))
        return y

    def prescreen(self, pts, parent_pts, parent_cache, parent_of, score=None, stream=None):
        """Scores [pop] of offspring `pts` (parents as for `features`)."""
        import torch
        score = torch.empty(pts.shape[0], dtype=torch.float32, device="cuda") if score is None else score
        _check(load_library().morea_surrogate_prescreen(self.handle, _dev_ptr(pts), pts.shape[0],
                                                        _dev_ptr(parent_pts), parent_pts.shape[0],
                                                        _dev_ptr(parent_cache), _dev_ptr(parent_of),
                                                        _dev_ptr(score), _stream_ptr(stream)))
        return score

    def get_params(self):
        out = np.empty(self.n_params, np.float32)
        _check(load_library().morea_surrogate_get_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, params):
        a = _host(params, np.float32)
        assert a.size == self.n_params
        _check(load_library().morea_surrogate_set_params(self.handle, a.ctypes.data_as(ctypes.c_void_p)))

    def stats(self):
        st = np.empty((self.problem.n_tets, 8), np.float32)
        cnt = np.empty(self.problem.n_tets, np.int32)
        _check(load_library().morea_surrogate_stats(self.handle, st.ctypes.data_as(ctypes.c_void_p),
                                                    cnt.ctypes.data_as(ctypes.c_void_p)))
        return st, cnt


def morea_surrogate_select(score, k, pts=None, n_points=0, stream=None):
    """Indices of the k lowest scores and (optionally) the selected candidates."""
    import torch
    idx = torch.empty(k, dtype=torch.int32, device="cuda")
    sel = None
    if pts is not None:
        sel = torch.empty((k,) + tuple(pts.shape[1:]), dtype=torch.float32, device="cuda")
        n_points = pts.shape[-1]
    _check(load_library().morea_surrogate_select(_dev_ptr(score), score.numel(), k, _dev_ptr(pts),
                                                 n_points, _dev_ptr(idx), _dev_ptr(sel),
                                                 _stream_ptr(stream)))
    return idx, sel
