"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds no arithmetic of the method: it only draws numbers and
arranges them in the canonical parameter order.  Both the FP64 oracle and the
GPU path take what it returns as plain inputs.

Random numbers come from numpy's Philox-4x64 counter-based generator, keyed
by (seed, stream); a stream id names what is drawn (processor, block,
tensor), so every tensor is reproducible on its own.  Values are drawn in
float64 and rounded once to float32; the float32 arrays are the master
values both sides start from.

Shapes of the latent grid follow the paper's 2-degree latent over
720 x 1440 (0.25 degree, south-pole row dropped, App. A.1) with pressure level
as the third axis (Sec. 2.1): (Z=level, Y=lat, X=lon), channels last.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Grid", "CFG1", "CFG2", "block_param_layout", "block_param_count",
    "latent_state", "processor_params", "split_block_params",
    "serving_trace",
]


@dataclasses.dataclass(frozen=True)
class Grid:
    """Latent grid and block shape.  Axis order is (Z=level, Y=lat, X=lon)."""
    Z: int
    Y: int
    X: int
    C: int
    heads: int
    Kz: int
    Ky: int
    Kx: int
    periodic_mask: int = 0x4   # bit0 = Z, bit1 = Y, bit2 = X (lon wraps)
    mlp_ratio: int = 4

    @property
    def T(self) -> int:
        return self.Z * self.Y * self.X

    @property
    def d(self) -> int:
        return self.C // self.heads

    @property
    def rpb_shape(self):
        return (self.heads, 2 * self.Kz - 1, 2 * self.Ky - 1, 2 * self.Kx - 1)


# Small single-block case: 5 x 45 x 90, C=128, 4 heads, window 3x5x5.
CFG1 = Grid(Z=5, Y=45, X=90, C=128, heads=4, Kz=3, Ky=5, Kx=5)
# Full-size processor: 8 x 90 x 180, C=512, 16 heads, window 5x7x7.
CFG2 = Grid(Z=8, Y=90, X=180, C=512, heads=16, Kz=5, Ky=7, Kx=7)

# Stream ids of the generator.
_STREAM_STATE = 1
_STREAM_PARAM = 2
_STREAM_ARRIVAL = 3
_STREAM_SMOOTH = 4


def block_param_layout(g: Grid):
    """Canonical order of one block's parameters: list of (name, shape).

    Linear maps are stored [in, out] (y = x @ W + b).  QKV columns are
    [Q | K | V], each with channel c = head * d + e.
    """
    C, F = g.C, g.C * g.mlp_ratio
    return [
        ("ln1_g", (C,)), ("ln1_b", (C,)),
        ("w_qkv", (C, 3 * C)), ("b_qkv", (3 * C,)),
        ("rpb", g.rpb_shape),
        ("w_o", (C, C)), ("b_o", (C,)),
        ("ln2_g", (C,)), ("ln2_b", (C,)),
        ("w_1", (C, F)), ("b_1", (F,)),
        ("w_2", (F, C)), ("b_2", (C,)),
    ]


def block_param_count(g: Grid) -> int:
    return int(sum(np.prod(s) for _, s in block_param_layout(g)))


def _rng(seed: int, stream: int, a: int = 0, b: int = 0, c: int = 0):
    key = [int(seed) & 0xFFFFFFFFFFFFFFFF,
           ((stream & 0xFF) << 56) | ((a & 0xFFFF) << 40) | ((b & 0xFFFF) << 24) | (c & 0xFFFFFF)]
    return np.random.Generator(np.random.Philox(key=key))


def latent_state(g: Grid, B: int = 1, seed: int = 0, index0: int = 0) -> np.ndarray:
    """Latent states [B, Z, Y, X, C] float32, i.i.d. N(0, 1).

    State b is drawn from its own stream (index0 + b), so a state is the same
    whether drawn alone or inside a batch.
    """
    out = np.empty((B, g.Z, g.Y, g.X, g.C), dtype=np.float32)
    for b in range(B):
        r = _rng(seed, _STREAM_STATE, index0 + b)
        out[b] = r.standard_normal((g.Z, g.Y, g.X, g.C)).astype(np.float32)
    return out


def smooth_state(g: Grid, B: int = 1, seed: int = 0, noise: float = 0.1) -> np.ndarray:
    """Latent states [B, Z, Y, X, C] float32 with large-scale structure: per
    channel, a sum of low-order modes, cos(m lon + phase) cos(n colat + phase)
    with m = 1..3 around the periodic longitude and n = 1..2 in colatitude,
    times a level profile cos(l pi (z + 1/2) / Z), l = 0..1, with random
    amplitudes; scaled to unit variance per channel, plus noise * N(0, 1).
    A stand-in for smooth analysis fields (FP8 scales see a realistic
    dynamic range).
    """
    lon = 2.0 * np.pi * np.arange(g.X) / g.X
    colat = np.pi * (np.arange(g.Y) + 0.5) / g.Y
    lev = np.pi * (np.arange(g.Z) + 0.5) / g.Z
    out = np.empty((B, g.Z, g.Y, g.X, g.C), dtype=np.float32)
    for b in range(B):
        r = _rng(seed, _STREAM_SMOOTH, b)
        f = np.zeros((g.Z, g.Y, g.X, g.C), dtype=np.float32)
        for m in (1, 2, 3):
            for n in (1, 2):
                for l in (0, 1):
                    amp = r.standard_normal(g.C)
                    pl, pc = r.uniform(0, 2 * np.pi, g.C), r.uniform(0, 2 * np.pi, g.C)
                    fz = (np.cos(l * lev)[:, None] * amp).astype(np.float32)          # [Z, C]
                    fy = np.cos(n * colat[:, None] + pc).astype(np.float32)            # [Y, C]
                    fx = np.cos(m * lon[:, None] + pl).astype(np.float32)              # [X, C]
                    f += (fz[:, None, :] * fy[None, :, :])[:, :, None, :] * fx[None, None, :, :]
        f /= f.reshape(-1, g.C).std(axis=0) + 1e-12
        out[b] = (f + noise * r.standard_normal(f.shape)).astype(np.float32)
    return out


def processor_params(g: Grid, n_blocks: int, seed: int = 1, proc: int = 0,
                     std: float = 0.02) -> np.ndarray:
    """All parameters of an n_blocks processor, flat float32, canonical order.

    Matrices, biases and the relative-position bias ~ N(0, std); LayerNorm
    gains 1 + N(0, std) and shifts N(0, std), so the affine path is used.
    """
    chunks = []
    for blk in range(n_blocks):
        for t, (name, shape) in enumerate(block_param_layout(g)):
            r = _rng(seed, _STREAM_PARAM, proc, blk, t)
            v = r.standard_normal(shape) * std
            if name in ("ln1_g", "ln2_g"):
                v = v + 1.0
            chunks.append(v.astype(np.float32).ravel())
    return np.concatenate(chunks)


def split_block_params(g: Grid, flat: np.ndarray, block: int = 0) -> dict:
    """View the parameters of one block as a dict of named arrays."""
    n = block_param_count(g)
    base = flat[block * n:(block + 1) * n]
    out, off = {}, 0
    for name, shape in block_param_layout(g):
        size = int(np.prod(shape))
        out[name] = base[off:off + size].reshape(shape)
        off += size
    return out


def serving_trace(n: int, rate_per_s: float, seed: int = 3, lead_max: int = 336):
    """Poisson arrival times (s) and lead times uniform in 1..lead_max hours."""
    r = _rng(seed, _STREAM_ARRIVAL)
    gaps = r.exponential(1.0 / rate_per_s, size=n)
    leads = r.integers(1, lead_max + 1, size=n)
    return np.cumsum(gaps), leads.astype(np.int64)
