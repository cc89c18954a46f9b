"""Seeded synthetic surveillance video and workload descriptors.

This module is the single source of inputs shared by the FP64 oracle and the
HIP path.  It holds none of the coding method's arithmetic: it only draws
frames (uint8 luma) and picks per-stream parameters.

The paper measures on two QCIF surveillance sequences (Section 4) that are not
available here; the generator stands in for them with the same structure: a
static, smooth, lightly textured background, a few constant-velocity objects,
and sensor noise, so that frame-to-frame residuals are sparse (Section 2.1).
"""
from .video import surveillance_video, VideoSpec
from .workloads import (StreamSpec, qcif_tiny, cif_sweep, vga_precision,
                        mixed_streams, serving_cameras, phi_key)

__all__ = ["surveillance_video", "VideoSpec", "StreamSpec", "qcif_tiny",
           "cif_sweep", "vga_precision", "mixed_streams", "serving_cameras",
           "phi_key"]
