"""The six synthetic workloads and their seeded inputs.

Sizes follow the paper's workload shape (Sec. V.C: 3-level surface point
clouds, k = 6, a halo as deep as the 15 message-passing layers; Sec. V.D:
15 layers) scaled to synthetic stand-ins, since the car dataset is absent.

Seeds for workload i: geometry 1000 i + 1, bump modes 1000 i + 2, weights
1000 i + 3, targets 1000 i + 4, partition sizes 1000 i + 5.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import geometry


@dataclass(frozen=True)
class Config:
    idx: int
    name: str
    geometry: str                 # "sphere" | "ellipsoid" | "car"
    levels: tuple                 # nested level sizes, coarse to fine
    k_intra: int
    k_cross: int
    hidden: int
    layers: int
    n_parts: int = 1
    part_jitter: float = 0.0      # relative spread of partition sizes
    halo: int = 0
    precision: str = "fp32"
    activation: str = "relu"
    fourier: tuple = ()           # frequencies f of the sin / cos(2 pi f x) input features

    @property
    def n_nodes(self) -> int:
        return self.levels[-1]

    @property
    def node_in(self) -> int:
        return NODE_IN + 6 * len(self.fourier)

    def seed(self, what: str) -> int:
        off = {"geom": 1, "modes": 2, "weights": 3, "targets": 4, "parts": 5}[what]
        return 1000 * self.idx + off


CONFIGS = {
    1: Config(1, "sphere-2k", "sphere", (2000,), 6, 0, 128, 2),
    2: Config(2, "ellipsoid-200k", "ellipsoid", (200_000,), 6, 0, 128, 15),
    3: Config(3, "ellipsoid-ms-400k", "ellipsoid", (25_000, 100_000, 400_000), 6, 3, 128, 15,
              precision="bf16"),
    4: Config(4, "ellipsoid-ms-1m-24p", "ellipsoid", (62_500, 250_000, 1_000_000), 6, 3, 128, 15,
              n_parts=24, part_jitter=0.4, halo=15, precision="bf16"),
    5: Config(5, "car-ms-4m-16p", "car", (250_000, 1_000_000, 4_000_000), 6, 3, 256, 15,
              n_parts=16, part_jitter=0.0, halo=15, precision="bf16"),
    # the paper's own training shape (Sec. V.C-D): 3 levels of 0.5M/1M/2M
    # points, 21 partitions with 15-hop halos, H = 512, SiLU, 24 inputs
    # (position, normal and their Fourier features at 2 pi, 4 pi, 8 pi)
    6: Config(6, "car-ms-2m-21p-h512", "car", (500_000, 1_000_000, 2_000_000), 6, 3, 512, 15,
              n_parts=21, part_jitter=0.0, halo=15, precision="bf16", activation="silu", fourier=(1, 2, 4)),
}

NODE_IN = 6     # position + normal
EDGE_IN = 4     # relative displacement + its norm
OUT_DIM = 4     # pressure + 3 wall-shear components stand-in


def points(cfg: Config, n: int | None = None):
    """(pos, normal) float32 [n][3] for the config's geometry (n defaults to
    the finest level)."""
    n = cfg.n_nodes if n is None else n
    if cfg.geometry == "sphere":
        return geometry.sphere(n, cfg.seed("geom"))
    if cfg.geometry == "ellipsoid":
        return geometry.bumpy_ellipsoid(n, cfg.seed("geom"), cfg.seed("modes"))
    if cfg.geometry == "car":
        return geometry.car_body(n, cfg.seed("geom"))
    raise ValueError(cfg.geometry)


def zscore(x: np.ndarray) -> np.ndarray:
    """Per-channel z-score with statistics taken in float64 (Sec. V.C
    normalises inputs with per-variable global mean and std)."""
    x64 = x.astype(np.float64)
    mu = x64.mean(axis=0)
    sd = x64.std(axis=0)
    sd[sd == 0] = 1.0
    return ((x64 - mu) / sd).astype(np.float32)


def fourier_features(pos: np.ndarray, freqs) -> np.ndarray:
    """[sin(2 pi f x_c), cos(2 pi f x_c)] for every frequency f and coordinate
    c, in float64 from the float32 positions: float32 [n][6 len(freqs)]."""
    x = pos.astype(np.float64)
    cols = []
    for f in freqs:
        cols += [np.sin(2.0 * np.pi * f * x), np.cos(2.0 * np.pi * f * x)]
    return np.concatenate(cols, axis=1).astype(np.float32) if cols else np.zeros((len(pos), 0), np.float32)


def edge_norm_for(pos: np.ndarray) -> np.ndarray:
    """Affine normalisation (mean, std) for the 4 edge-input channels.

    The scale s is the mean point spacing of a surface sample, estimated from
    the bounding box alone: s = sqrt(A / n) with A the box's surface area.
    Returns float32 [2][4]: row 0 = mean, row 1 = std.
    """
    ext = pos.max(axis=0).astype(np.float64) - pos.min(axis=0).astype(np.float64)
    area = 2.0 * (ext[0] * ext[1] + ext[1] * ext[2] + ext[0] * ext[2])
    s = float(np.sqrt(area / max(len(pos), 1)))
    return np.array([[0.0, 0.0, 0.0, s], [s, s, s, 0.5 * s]], dtype=np.float32)


def partition_sizes(cfg: Config, n: int | None = None, n_parts: int | None = None) -> np.ndarray:
    """Integer partition sizes summing to n.  With jitter j the raw weights
    are 1 + j u_p, u_p ~ U(-1, 1); they are scaled to sum to n, rounded, and
    the rounding remainder goes to the last part."""
    n = cfg.n_nodes if n is None else n
    p = cfg.n_parts if n_parts is None else n_parts
    g = np.random.Generator(np.random.PCG64(cfg.seed("parts")))
    w = 1.0 + cfg.part_jitter * g.uniform(-1.0, 1.0, p)
    sizes = np.rint(w / w.sum() * n).astype(np.int64)
    sizes[-1] = n - sizes[:-1].sum()
    if (sizes <= 0).any():
        raise ValueError("partition sizes must be positive")
    return sizes.astype(np.int32)


def init_params(entries, seed: int) -> np.ndarray:
    """Flat float32 parameter blob from a list of (kind, shape) entries.

    kind "weight": Xavier-normal, N(0, 2 / (fan_in + fan_out)) with
    shape = (fan_out, fan_in); "bias" and "beta": N(0, 0.05^2); "gamma":
    1 + N(0, 0.05^2).  Drawn in float64 in entry order, then rounded once.
    """
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for kind, shape in entries:
        cnt = int(np.prod(shape))
        if kind == "weight":
            fo, fi = shape
            v = g.standard_normal(cnt) * np.sqrt(2.0 / (fi + fo))
        elif kind in ("bias", "beta"):
            v = 0.05 * g.standard_normal(cnt)
        elif kind == "gamma":
            v = 1.0 + 0.05 * g.standard_normal(cnt)
        else:
            raise ValueError(kind)
        parts.append(v)
    return np.concatenate(parts).astype(np.float32)


@dataclass
class Inputs:
    cfg: Config
    pos: np.ndarray          # float32 [N][3]
    normal: np.ndarray       # float32 [N][3]
    level_end: np.ndarray    # int32 [levels]
    node_in: np.ndarray      # float32 [N][node_in] z-scored [pos, normal, Fourier features]
    edge_norm: np.ndarray    # float32 [2][4]
    targets: np.ndarray      # float32 [N][4]
    part_sizes: np.ndarray   # int32 [n_parts]
    extra: dict = field(default_factory=dict)


def make_inputs(cfg: Config, n: int | None = None, levels=None, n_parts=None) -> Inputs:
    """All seeded inputs of a config.  ``levels`` may override the level
    sizes (for reduced-size parity cases of the same recipe)."""
    levels = tuple(cfg.levels if levels is None else levels)
    n = levels[-1] if n is None else n
    pos, nrm = points(cfg, n)
    node_in = zscore(np.concatenate([pos, nrm, fourier_features(pos, cfg.fourier)], axis=1))
    g = np.random.Generator(np.random.PCG64(cfg.seed("targets")))
    targets = g.standard_normal((n, OUT_DIM)).astype(np.float32)
    return Inputs(cfg, pos, nrm, np.array(levels, dtype=np.int32), node_in,
                  edge_norm_for(pos), targets,
                  partition_sizes(cfg, n, n_parts))
