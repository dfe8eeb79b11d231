"""Rendering and image quality on held-out views (Sec. IV, rendering).

The converged parameters are rendered with a step of one voxel and the opacity threshold
rule (a ray whose volume opacity 1 - T is below 0.7 shows the volume as empty).  PSNR
against held-out images comes from the library's own objective on those images:
F = 1/2 sum r^2 over 3 colour residuals per ray, so MSE = 2F / (3 rays).
"""
from __future__ import annotations

import dataclasses
import math

import torch

from .scene import Scene


def render_scene(spec, cams, targets=None, threshold: float = 0.7, step_vox: float = 1.0,
                 device: str = "cuda:0") -> Scene:
    """A scene for rendering: same grid and layers, the given cameras, the render step."""
    sp = dataclasses.replace(spec, step_vox=step_vox)
    return Scene(sp, cams, targets, device=device, render_threshold=threshold)


def psnr(x: torch.Tensor, spec, cams, images: torch.Tensor, threshold: float = 0.7, step_vox: float = 1.0) -> float:
    """PSNR in dB of the rendering of x against images ([rays * 3] float32, colours in [0, 1])."""
    sc = render_scene(spec, cams, images, threshold, step_vox, device=str(images.device))
    _, F = sc.render_residuals(x, want_r=False)
    mse = 2.0 * float(F.item()) / (3.0 * sc.n_rays)
    return 10.0 * math.log10(1.0 / mse) if mse > 0 else float("inf")
