"""Shared helpers of the GPU parity tests (inputs from scenegen, expected
values from the oracle, results through the C ABI binding)."""
from __future__ import annotations

import numpy as np
import scipy.ndimage as ndi
import torch

import scenegen as sg

DEV = torch.device("cuda:0")


def to_dev(a, dtype=None) -> torch.Tensor:
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def f32(a) -> np.ndarray:
    """Round to float32 (the interface precision) and widen back exactly."""
    return np.asarray(a, np.float32).astype(np.float64)


def upload_scene(hdof, ctx, scene: sg.Scene):
    return hdof.hdof_build_bvh(ctx, to_dev(scene.verts), to_dev(scene.albedo))


def chebyshev_dilate(mask: np.ndarray, r: int) -> np.ndarray:
    if r <= 0 or not mask.any():
        return mask.copy()
    return ndi.binary_dilation(mask, structure=np.ones((2 * r + 1, 2 * r + 1), bool))


def tile_footprint(mask: np.ndarray, tile: int, dil: int) -> np.ndarray:
    """Pixels whose tile lies within `dil` tiles of a tile containing a marked pixel."""
    H, W = mask.shape
    TH, TW = -(-H // tile), -(-W // tile)
    t = np.zeros((TH, TW), bool)
    ys, xs = np.nonzero(mask)
    t[ys // tile, xs // tile] = True
    t = chebyshev_dilate(t, dil)
    return np.repeat(np.repeat(t, tile, 0), tile, 1)[:H, :W]


def excl_cumsum(s: np.ndarray) -> np.ndarray:
    flat = s.reshape(-1).astype(np.int64)
    return np.concatenate([[0], np.cumsum(flat)[:-1]]).reshape(s.shape)


def print_case(name: str) -> None:
    print(f"[case] {name}", flush=True)
