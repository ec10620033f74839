"""The five seeded workloads: plain forward, non-watertight forward, differentiable,
batched, served.  Sizes follow the voxel resolutions and face counts of the
paper's Experiments section (resolutions 32 to 256; meshes of about 1k to 270k faces).

Seeds: C1 = 1, C2 = 2, C3 mesh = 3 / target = 4 / open variant = 3 + 1,
C4 = 5, C5 meshes = 6 / arrivals = 7.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .meshgen import (
    Grid,
    Ellipsoid,
    delete_faces,
    ellipsoid_target_on_grid,
    ellipsoid_union,
    icosphere,
    jitter,
    random_ellipsoid,
    uv_resolution_for_faces,
)

SEEDS = {"c1": 1, "c2": 2, "c3_mesh": 3, "c3_target": 4, "c4": 5, "c5_mesh": 6, "c5_arrivals": 7,
         "eval_reconstruction": 8, "eval_reference": 9}


@dataclass
class Workload:
    name: str
    V: np.ndarray            # float64 [nV, 3]
    F: np.ndarray            # int64 [nF, 3]
    grid: Grid
    occ_mode: str = "threshold"
    tau: float = 0.5
    k: float = 50.0
    target: np.ndarray | None = None   # float32 [P] loss target, differentiable workloads only
    extra: dict = field(default_factory=dict)

    @property
    def pairs(self) -> int:
        return self.grid.size * len(self.F)


def config1_icosphere(res: int = 32) -> Workload:
    """Icosphere s=3 (1280 faces, 642 vertices) of radius 0.4, jitter sigma 0.01, 32^3 grid."""
    rng = np.random.default_rng(SEEDS["c1"])
    V, F = icosphere(3)
    V = jitter(V * 0.4, 0.01, rng)
    return Workload("icosphere-s3-1280f-32cube", V, F, Grid.cube(res), "threshold")


def config2_ellipsoid_union(res: int = 128) -> Workload:
    """8 ellipsoids of 2500 faces (20 000), 1000 faces (5 %) deleted, 128^3 grid."""
    rng = np.random.default_rng(SEEDS["c2"])
    V, F, ells = ellipsoid_union(rng, 8, 2500, axes=(0.05, 0.3), centres=(-0.3, 0.3))
    F = delete_faces(F, round(0.05 * len(F)), rng)
    return Workload("ellipsoid-union-19000f-128cube", V, F, Grid.cube(res), "threshold",
                    extra={"ellipsoids": ells})


def config3_target_ellipsoid() -> Ellipsoid:
    rng = np.random.default_rng(SEEDS["c3_target"])
    return random_ellipsoid(rng, 0.25, 0.4, -0.05, 0.05)


def config3_differentiable(res: int = 64, open_variant: bool = False) -> Workload:
    """Icosphere s=4 (5120 faces, 2562 vertices), radius 0.4, jitter 0.01, 64^3 grid,
    sigmoid k=50 around 0.5, MSE (mean over voxels) against a solid ellipsoid target.

    ``open_variant`` deletes 5 % of the faces (seed 3 + 1) so that the hole rims
    carry a non-zero vertex gradient."""
    rng = np.random.default_rng(SEEDS["c3_mesh"])
    V, F = icosphere(4)
    V = jitter(V * 0.4, 0.01, rng)
    name = "icosphere-s4-5120f-64cube-sigmoid-mse"
    if open_variant:
        F = delete_faces(F, round(0.05 * len(F)), np.random.default_rng(SEEDS["c3_mesh"] + 1))
        name = "open-" + name
    grid = Grid.cube(res)
    e = config3_target_ellipsoid()
    return Workload(name, V, F, grid, "sigmoid", 0.5, 50.0, ellipsoid_target_on_grid(grid, e),
                    extra={"target_ellipsoid": e})


def random_union_mesh(rng, faces: int, n_ell: int, del_frac: float):
    per = max(8, faces // n_ell)
    V, F, ells = ellipsoid_union(rng, n_ell, per, axes=(0.05, 0.3), centres=(-0.3, 0.3))
    F = delete_faces(F, int(round(del_frac * len(F))), rng)
    return V, F, ells


def config4_batch(n_meshes: int = 64, face_lo: int = 500, face_hi: int = 50_000,
                  resolutions=(32, 64, 128), seed: int | None = None) -> list[Workload]:
    """64 meshes: F ~ LogUniform(500, 50k), unions of U{1..8} ellipsoids, 0-10 % of faces
    deleted, each with its own grid drawn from {32^3, 64^3, 128^3}."""
    rng = np.random.default_rng(SEEDS["c4"] if seed is None else seed)
    out = []
    for i in range(n_meshes):
        faces = int(round(math.exp(rng.uniform(math.log(face_lo), math.log(face_hi)))))
        n_ell = int(rng.integers(1, 9))
        del_frac = float(rng.uniform(0.0, 0.10))
        res = int(rng.choice(resolutions))
        V, F, _ = random_union_mesh(rng, faces, n_ell, del_frac)
        out.append(Workload(f"batch{i}-{len(F)}f-{res}cube", V, F, Grid.cube(res), "threshold"))
    return out


@dataclass
class Request:
    rid: int
    arrival: float            # seconds from trace start
    faces: int
    res: int
    wants_grad: bool
    mesh_seed: int

    def build(self) -> Workload:
        """Materialise the request's mesh (and target, for gradient requests)."""
        rng = np.random.default_rng(self.mesh_seed)
        n_ell = int(rng.integers(1, 9))
        V, F, _ = random_union_mesh(rng, self.faces, n_ell, float(rng.uniform(0.0, 0.10)))
        grid = Grid.cube(self.res)
        if self.wants_grad:
            e = random_ellipsoid(rng, 0.1, 0.4, -0.1, 0.1)
            return Workload(f"req{self.rid}", V, F, grid, "sigmoid", 0.5, 50.0,
                            ellipsoid_target_on_grid(grid, e))
        return Workload(f"req{self.rid}", V, F, grid, "threshold")


def config5_trace(n_requests: int, rate: float, face_lo: int = 1000, face_hi: int = 100_000,
                  resolutions=(64, 128, 256), grad_frac: float = 0.3) -> list[Request]:
    """Poisson arrivals at ``rate`` requests/s (exponential gaps, seed 7); per-request
    F ~ LogUniform(1k, 100k), resolution from {64, 128, 256}, 30 % also want dL/dV."""
    ra = np.random.default_rng(SEEDS["c5_arrivals"])
    rm = np.random.default_rng(SEEDS["c5_mesh"])
    t = 0.0
    reqs = []
    for i in range(n_requests):
        t += float(ra.exponential(1.0 / rate))
        faces = int(round(math.exp(rm.uniform(math.log(face_lo), math.log(face_hi)))))
        res = int(rm.choice(resolutions))
        wants = bool(rm.uniform() < grad_frac)
        reqs.append(Request(i, t, faces, res, wants, int(rm.integers(0, 2**31 - 1))))
    return reqs


def uniform_samples(n: int, seed: int) -> np.ndarray:
    """n rows of three uniform numbers in [0, 1) (float64): the random input of surface
    sampling, drawn here so that both sides of a comparison use the same numbers."""
    return np.random.default_rng(seed).random((n, 3))


def evaluation_samples(n: int = 20000, repeat: int = 0):
    """The two uniform streams of the evaluation chain (reconstruction, reference mesh);
    20 000 samples per surface as in the paper's experiments.  ``repeat`` selects one of
    the independent repeats over which the paper reports a mean and standard deviation
    (repeat 0 uses seeds 8 and 9, repeat r seeds 8 + 100 r and 9 + 100 r)."""
    return (uniform_samples(n, SEEDS["eval_reconstruction"] + 100 * repeat),
            uniform_samples(n, SEEDS["eval_reference"] + 100 * repeat))
