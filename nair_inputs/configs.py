"""Named synthetic workloads (upwind DG transport on quads).

Each entry restates one benchmark configuration: mesh, element order, flow
field, reaction coefficient, Neumann degree and precision.  Seeds: cell
permutation 101, nodal source 102, vertex jitter 103, target solution 104,
per-cell sigma 105, angle j source 200+j.
"""
from __future__ import annotations

import math

import numpy as np

from .dg_quad import dg_quad


def _curved(x, y):
    # b(x,y) = (y + 1/4, -(x + 1/4)): b_x in [1/4, 5/4] > 0, b_y < 0 on [0,1]^2,
    # so b.n has one sign on every axis-aligned face and the cell graph is acyclic.
    return (y + 0.25, -(x + 0.25))


CONFIGS = {
    # 32x32 Q1, 4,096 DOFs, 4x4 blocks, b = (cos pi/8, sin pi/8), sigma = 1, degree 1
    "dg_q1_32": dict(N=32, p=1, b=(math.cos(math.pi / 8), math.sin(math.pi / 8)),
                     sigma=1.0, jitter=0.0, degree=1),
    # 256x256 Q2, 589,824 DOFs, 9x9 blocks, curved b, sigma = 0.5, degree 2
    "dg_q2_256_curved": dict(N=256, p=2, b=_curved, sigma=0.5, jitter=0.0, degree=2),
    # 512x512 jittered Q4, 6,553,600 DOFs, 25x25 blocks, b = (cos .3, sin .3), sigma = 1
    "dg_q4_512_jitter": dict(N=512, p=4, b=(math.cos(0.3), math.sin(0.3)), sigma=1.0,
                             jitter=0.2, degree=2),
    # 256x256 Q3, 1,048,576 DOFs, 16x16 blocks, curved b, per-cell sigma ~ U[0.5, 2]
    "dg_q3_256_curved_sigma": dict(N=256, p=3, b=_curved, sigma="random", jitter=0.0, degree=2),
}


def config_names():
    return list(CONFIGS)


def make_config(name: str, N: int | None = None, seed_perm: int | None = 101, **overrides):
    """Build the system for a named configuration (optionally at another mesh size N).

    Returns (DGSystem, degree).
    """
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    if N is not None:
        cfg["N"] = N
    degree = cfg.pop("degree")
    sigma = cfg.pop("sigma")
    if isinstance(sigma, str):
        rng = np.random.Generator(np.random.PCG64(105))
        sigma = rng.uniform(0.5, 2.0, size=cfg["N"] * cfg["N"])
    sysm = dg_quad(cfg.pop("N"), cfg.pop("p"), cfg.pop("b"), sigma=sigma,
                   jitter=cfg.pop("jitter"), seed_perm=seed_perm, **cfg)
    return sysm, degree


def angle_flow(j: int, nang: int = 64):
    """Discrete-ordinate direction theta_j = 2 pi (j + 1/2) / nang (never axis-aligned)."""
    th = 2.0 * math.pi * (j + 0.5) / nang
    return (math.cos(th), math.sin(th))
