"""Seeded synthetic inputs for MOREA objective evaluation.

This module only *draws* inputs: phantom image pairs, the Kuhn grid mesh,
guidance point sets, per-tetrahedron elasticity factors, candidate
populations, FOS point groups and partial-evaluation children.  It contains
none of the arithmetic of the objectives themselves (no rasterization, no
barycentric mapping, no interpolation of the sampled image, no sums of the
objectives), so that both the CPU oracle and the GPU path can take their
inputs from here without sharing any of the method.

The paper's clinical CT pairs, contours and masks (Sec. 5.1) are private; these
phantoms stand in for them at the shapes of the evaluated workloads:

* organs are axis-aligned ellipsoids with a smooth one-voxel edge profile and
  background exactly 0 (zero intensity is background, Sec. 4.1.2);
* the target is the source warped by a smooth, invertible sum of four Gaussian
  radial basis displacements, optionally with one organ removed (content
  mismatch, Sec. 1);
* both images get independent Gaussian noise on foreground voxels only;
* the mesh is a regular grid split into 6 Kuhn tetrahedra per cell (the
  paper uses a Delaunay mesh of contour points, Sec. 4.2.1; the evaluator
  accepts any tetrahedral mesh);
* guidance sets are points on the organ surfaces in the source and their
  forward-warped positions in the target (Sec. 4.1.3);
* elasticity per tetrahedron mixes three tissue factors by the estimated
  fraction of each class inside the initial source tetrahedron (App. A.1).

Coordinates are in voxel index units: voxel (i, j, k) has its centre at the
point (i, j, k); images are ``float32[nz][ny][nx]`` (x fastest).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# sub-stream ids of the per-configuration seed sequence
ORGANS, DISPLACEMENT, NOISE_S, NOISE_T, GUIDANCE, POPULATION, GROUPS, OFFSPRING = range(8)

SOFT, ELASTIC, RIGID = 1.0, 0.5, 10.0   # tissue factors: other, bladder-like, bone-like

CONFIGS = {
    1: dict(dims=(32, 32, 32), n_organs=3, intensities=(0.2, 0.5, 0.8), removed=None,
            amplitude=3.0, mesh=(5, 5, 5), n_guidance=20, guidance_organs=(0,),
            radius=0.8, population=16, perturb_source=False, fold_fraction=0.0),
    2: dict(dims=(128, 128, 96), n_organs=6, intensities=None, removed=5,
            amplitude=12.0, mesh=(10, 10, 8), n_guidance=200, guidance_organs=None,
            radius=3.2, population=512, perturb_source=True, fold_fraction=1.0 / 16),
    4: dict(dims=(192, 192, 128), n_organs=6, intensities=None, removed=5,
            amplitude=18.0, mesh=(14, 14, 10), n_guidance=200, guidance_organs=None,
            radius=4.8, population=256, perturb_source=True, fold_fraction=1.0 / 16),
}
CONFIGS[3] = dict(CONFIGS[2])
CONFIGS[5] = dict(CONFIGS[2], perturb_source=False, fold_fraction=0.0)

N_GROUPS = 64
GROUP_SIZES = (4, 48)
NOISE_SIGMA = 0.02
POINT_SIGMA = 0.5


def rng(seed: int, stream: int) -> np.random.Generator:
    """PCG64 generator for sub-stream ``stream`` of master seed ``seed``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(8)[stream]))


@dataclasses.dataclass
class Problem:
    config: int
    dims: tuple            # (nx, ny, nz)
    image_src: np.ndarray  # float32 [nz][ny][nx]
    image_tgt: np.ndarray
    grid_shape: tuple      # mesh points per axis (px, py, pz)
    ref_points: np.ndarray  # float32 [n_points][3], the initial (grid) mesh
    target_base: np.ndarray  # float32 [n_points][3], grid pushed by the true displacement
    tets: np.ndarray        # int32 [n_tets][4]
    elasticity: np.ndarray  # float32 [n_tets]
    sets_src: list          # list of float32 [n_i][3]
    sets_tgt: list
    radius: float
    fixed_axes: np.ndarray  # bool [n_points][3]: coordinate pinned to the box face
    organs: list            # organ parameters (for tests)
    displacement: "Displacement"

    @property
    def n_points(self):
        return self.ref_points.shape[0]

    @property
    def n_tets(self):
        return self.tets.shape[0]


# --------------------------------------------------------------------------- organs
@dataclasses.dataclass
class Organ:
    center: np.ndarray
    semi: np.ndarray
    value: float
    tissue: float


def make_organs(cfg: dict, seed: int) -> list:
    g = rng(seed, ORGANS)
    n = np.array(cfg["dims"], dtype=np.float64)
    organs = []
    for k in range(cfg["n_organs"]):
        c = g.uniform(0.3 * n, 0.7 * n)
        s = g.uniform(0.12 * n, 0.25 * n)
        v = cfg["intensities"][k] if cfg["intensities"] else float(g.uniform(0.2, 0.9))
        tissue = ELASTIC if k == 0 else (RIGID if k == 1 else SOFT)
        organs.append(Organ(c, s, float(v), tissue))
    return organs


def organ_field(organs, x, y, z):
    """Clean phantom intensity at arbitrary points (max over smooth ellipsoids)."""
    out = np.zeros(np.broadcast(x, y, z).shape, dtype=np.float64)
    for o in organs:
        rho = np.sqrt(((x - o.center[0]) / o.semi[0]) ** 2 + ((y - o.center[1]) / o.semi[1]) ** 2
                      + ((z - o.center[2]) / o.semi[2]) ** 2)
        sd = (1.0 - rho) * float(np.cbrt(np.prod(o.semi)))   # ~ signed distance, voxels
        t = np.clip((sd + 1.0) * 0.5, 0.0, 1.0)
        out = np.maximum(out, o.value * t * t * (3.0 - 2.0 * t))
    return out


def organ_label(organs, x, y, z):
    """Index of the organ whose ellipsoid contains the point (last wins), else -1."""
    lab = np.full(np.broadcast(x, y, z).shape, -1, dtype=np.int32)
    for k, o in enumerate(organs):
        rho2 = (((x - o.center[0]) / o.semi[0]) ** 2 + ((y - o.center[1]) / o.semi[1]) ** 2
                + ((z - o.center[2]) / o.semi[2]) ** 2)
        lab[rho2 < 1.0] = k
    return lab


# ---------------------------------------------------------------------- displacement
@dataclasses.dataclass
class Displacement:
    centers: np.ndarray   # [4][3]
    weights: np.ndarray   # [4][3]
    sigma: float

    def __call__(self, p):
        p = np.asarray(p, dtype=np.float64)
        u = np.zeros_like(p)
        for c, w in zip(self.centers, self.weights):
            r2 = np.sum((p - c) ** 2, axis=-1, keepdims=True)
            u += w * np.exp(-r2 / (2 * self.sigma ** 2))
        return u

    def inverse(self, y, iters=20):
        x = np.array(y, dtype=np.float64)
        for _ in range(iters):
            x = y - self(x)
        return x


def make_displacement(cfg: dict, seed: int) -> Displacement:
    g = rng(seed, DISPLACEMENT)
    n = np.array(cfg["dims"], dtype=np.float64)
    sigma = float(np.mean(n)) / 4.0
    centers = g.uniform(0.2 * n, 0.8 * n, size=(4, 3))
    weights = g.normal(size=(4, 3))
    d = Displacement(centers, weights, sigma)
    grid = _voxel_centers(cfg["dims"], step=4)
    scale = cfg["amplitude"] / np.max(np.linalg.norm(d(grid), axis=-1))
    d.weights = weights * scale
    return d


def _voxel_centers(dims, step=1):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(0, nz, step), np.arange(0, ny, step), np.arange(0, nx, step),
                          indexing="ij")
    return np.stack([x, y, z], axis=-1).astype(np.float64)


# ------------------------------------------------------------------------------ mesh
def kuhn_grid(dims, shape):
    """Grid points over the box [-0.5, n-0.5] per axis and 6 Kuhn tets per cell."""
    px, py, pz = shape
    axes = [-0.5 + np.arange(p) * (n / (p - 1)) for p, n in zip(shape, dims)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    points = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=-1)

    def idx(i, j, k):
        return i + px * (j + py * k)

    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for k in range(pz - 1):
        for j in range(py - 1):
            for i in range(px - 1):
                for perm in perms:
                    c = [0, 0, 0]
                    verts = [idx(i, j, k)]
                    for a in perm:
                        c[a] += 1
                        verts.append(idx(i + c[0], j + c[1], k + c[2]))
                    tets.append(verts)
    fixed = np.zeros((points.shape[0], 3), dtype=bool)
    gi = np.stack(np.meshgrid(np.arange(pz), np.arange(py), np.arange(px), indexing="ij"), -1)
    gi = gi.reshape(-1, 3)[:, ::-1]   # (i, j, k) per point
    for a, p in enumerate(shape):
        fixed[:, a] = (gi[:, a] == 0) | (gi[:, a] == p - 1)
    return points, np.asarray(tets, dtype=np.int32), fixed


def mesh_edges(tets, n_points):
    """Sorted adjacency lists of the mesh graph (tet edges)."""
    nb = [set() for _ in range(n_points)]
    for t in tets:
        for a in range(4):
            for b in range(a + 1, 4):
                nb[t[a]].add(int(t[b]))
                nb[t[b]].add(int(t[a]))
    return [sorted(s) for s in nb]


# ------------------------------------------------------------------------- problem
def make_problem(config: int, seed: int | None = None) -> Problem:
    cfg = CONFIGS[config]
    seed = config if seed is None else seed
    nx, ny, nz = cfg["dims"]
    organs = make_organs(cfg, seed)
    disp = make_displacement(cfg, seed)
    vox = _voxel_centers(cfg["dims"])
    X, Y, Z = vox[..., 0], vox[..., 1], vox[..., 2]

    clean_s = organ_field(organs, X, Y, Z)
    tgt_organs = [o for k, o in enumerate(organs) if k != cfg["removed"]]
    pre = disp.inverse(vox)
    clean_t = organ_field(tgt_organs, pre[..., 0], pre[..., 1], pre[..., 2])

    def noisy(clean, stream):
        g = rng(seed, stream)
        noise = g.normal(0.0, NOISE_SIGMA, size=clean.shape)
        out = np.where(clean > 0, np.clip(clean + noise, 0.0, 1.0), 0.0)
        return out.astype(np.float32)

    image_src = noisy(clean_s, NOISE_S)
    image_tgt = noisy(clean_t, NOISE_T)

    points, tets, fixed = kuhn_grid(cfg["dims"], cfg["mesh"])
    u = disp(points)
    u[fixed] = 0.0
    target_base = points + u

    # guidance: points on organ surfaces present in both images, counts by area
    g = rng(seed, GUIDANCE)
    present = [k for k in range(len(organs)) if k != cfg["removed"]]
    if cfg["guidance_organs"] is not None:
        present = list(cfg["guidance_organs"])
    areas = np.array([_ellipsoid_area(organs[k].semi) for k in present])
    counts = _apportion(cfg["n_guidance"], areas)
    sets_src, sets_tgt = [], []
    for k, cnt in zip(present, counts):
        if cnt == 0:
            continue
        d = g.normal(size=(cnt, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        ps = organs[k].center + d * organs[k].semi
        pt = ps + disp(ps)
        sets_src.append(ps.astype(np.float32))
        sets_tgt.append(pt.astype(np.float32))

    elasticity = _elasticity(organs, points, tets,
                             np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 8]))))
    return Problem(config, (nx, ny, nz), image_src, image_tgt, tuple(cfg["mesh"]),
                   points.astype(np.float32), target_base.astype(np.float32), tets,
                   elasticity, sets_src, sets_tgt, float(cfg["radius"]), fixed, organs, disp)


def _ellipsoid_area(s):
    p = 1.6075
    a, b, c = s
    return 4 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3) ** (1 / p)


def _apportion(total, weights):
    w = np.asarray(weights, dtype=np.float64) / np.sum(weights)
    raw = w * total
    cnt = np.floor(raw).astype(int)
    for i in np.argsort(-(raw - cnt))[: total - cnt.sum()]:
        cnt[i] += 1
    return cnt


def _elasticity(organs, points, tets, g):
    """Tissue factor mix per tet from a Monte-Carlo estimate of class fractions.

    The fractions are estimated from 64 uniform random points per tetrahedron
    with the label of their nearest voxel centre; the factor is the
    fraction-weighted mean of the tissue factors (App. A.1)."""
    n = 64
    bary = g.dirichlet(np.ones(4), size=(tets.shape[0], n))            # [T][n][4]
    v = points[tets]                                                   # [T][4][3]
    pos = np.einsum("tnk,tkd->tnd", bary, v)
    pos = np.rint(pos)
    lab = organ_label(organs, pos[..., 0], pos[..., 1], pos[..., 2])
    factor = np.array([o.tissue for o in organs] + [SOFT])            # label -1 -> SOFT
    return factor[lab].mean(axis=1).astype(np.float32)


# ----------------------------------------------------------------------- population
def perturb(g, base, fixed, sigma):
    """Gaussian move of every coordinate that is not pinned to a box face."""
    noise = g.normal(0.0, sigma, size=base.shape)
    noise[..., fixed] = 0.0
    return base + noise


def make_population(prob: Problem, pop: int | None = None, seed: int | None = None,
                    perturb_source: bool | None = None, fold_fraction: float | None = None):
    """Candidates as float32 [pop][2][3][n_points] (mesh 0 = source S, 1 = target T)."""
    cfg = CONFIGS[prob.config]
    pop = cfg["population"] if pop is None else pop
    seed = prob.config if seed is None else seed
    perturb_source = cfg["perturb_source"] if perturb_source is None else perturb_source
    fold_fraction = cfg["fold_fraction"] if fold_fraction is None else fold_fraction
    g = rng(seed, POPULATION)
    out = np.empty((pop, 2, 3, prob.n_points), dtype=np.float32)
    interior = np.flatnonzero(~prob.fixed_axes.any(axis=1))
    for c in range(pop):
        s = perturb(g, prob.ref_points.astype(np.float64), prob.fixed_axes, POINT_SIGMA) \
            if perturb_source else prob.ref_points.astype(np.float64)
        t = perturb(g, prob.target_base.astype(np.float64), prob.fixed_axes, POINT_SIGMA)
        meshes = [s, t]
        if fold_fraction > 0 and c % int(round(1 / fold_fraction)) == 0:
            m = int(g.integers(2))
            v = int(g.choice(interior))
            tet = prob.tets[int(g.choice(np.flatnonzero((prob.tets == v).any(axis=1))))]
            face = [int(w) for w in tet if w != v]
            cf = meshes[m][face].mean(axis=0)
            meshes[m][v] = cf + 0.3 * (cf - meshes[m][v])
        out[c, 0] = meshes[0].T
        out[c, 1] = meshes[1].T
    return out


def make_groups(prob: Problem, n_groups: int = N_GROUPS, sizes=GROUP_SIZES, seed: int | None = None):
    """FOS point groups (CSR) grown by breadth-first search on the mesh graph."""
    seed = prob.config if seed is None else seed
    g = rng(seed, GROUPS)
    nb = mesh_edges(prob.tets, prob.n_points)
    off, pts = [0], []
    for _ in range(n_groups):
        size = int(g.integers(sizes[0], sizes[1] + 1))
        start = int(g.integers(prob.n_points))
        seen, queue = {start}, [start]
        order = []
        while queue and len(order) < size:
            v = queue.pop(0)
            order.append(v)
            for w in nb[v]:
                if w not in seen:
                    seen.add(w)
                    queue.append(w)
        pts.extend(order)
        off.append(len(pts))
    return np.asarray(off, dtype=np.int32), np.asarray(pts, dtype=np.int32)


def make_children(prob: Problem, parents: np.ndarray, grp_off, grp_pts, seed: int | None = None,
                  n_parents: int | None = None):
    """Every (parent, group) pair: eval e = parent * n_groups + group.

    Returns eval_parent, eval_group (int32) and new_coords float32
    [sum of group sizes][2][3]: the group's points moved by N(0, 0.5) in both
    meshes (pinned coordinates stay)."""
    seed = prob.config if seed is None else seed
    g = rng(seed, OFFSPRING)
    n_par = parents.shape[0] if n_parents is None else n_parents
    n_grp = len(grp_off) - 1
    ep = np.repeat(np.arange(n_par, dtype=np.int32), n_grp)
    eg = np.tile(np.arange(n_grp, dtype=np.int32), n_par)
    chunks = []
    for p, gr in zip(ep, eg):
        idx = grp_pts[grp_off[gr]:grp_off[gr + 1]]
        base = parents[p][:, :, idx].transpose(2, 0, 1).astype(np.float64)   # [k][2][3]
        fx = prob.fixed_axes[idx][:, None, :].repeat(2, axis=1)
        chunks.append(perturb(g, base, fx, POINT_SIGMA))
    return ep, eg, np.concatenate(chunks).astype(np.float32)


def apply_child(parents, grp_off, grp_pts, ep, eg, new_coords, e):
    """The full child candidate [2][3][n_points] of evaluation ``e``."""
    off = 0
    for k in range(e):
        off += grp_off[eg[k] + 1] - grp_off[eg[k]]
    idx = grp_pts[grp_off[eg[e]]:grp_off[eg[e] + 1]]
    child = parents[ep[e]].copy()
    child[:, :, idx] = new_coords[off:off + len(idx)].transpose(1, 2, 0)
    return child


def make_offspring(prob: Problem, n_parents=512, per_parent=8, seed=None, stream=OFFSPRING):
    """Surrogate workload: source fixed at the grid, target = parent + N(0, 0.5).

    Returns (parents [n_par][2][3][P], offspring [n_par*per_parent][2][3][P])."""
    seed = prob.config if seed is None else seed
    parents = make_population(prob, pop=n_parents, seed=seed, perturb_source=False, fold_fraction=0.0)
    g = rng(seed + 1000 * stream, stream)
    out = np.repeat(parents, per_parent, axis=0)
    fx = prob.fixed_axes.T
    for c in range(out.shape[0]):
        noise = g.normal(0.0, POINT_SIGMA, size=(3, prob.n_points))
        noise[fx] = 0.0
        out[c, 1] += noise.astype(np.float32)
    return parents, out
