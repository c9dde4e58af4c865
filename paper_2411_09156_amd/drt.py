"""Dynamic resolution training schedule (Sec. 3.4, Eq. 15).

The resolution scale follows a cosine from `start` to `end` over the first
`fraction` of training (Sec. 4.2: 0.26 to 1 over 75% of the iterations) and
stays at `end` afterwards:
    value = end + 0.5 (start - end) (1 + cos(pi * it / total)),  total = fraction * iterations.
"""
from __future__ import annotations

import math


def drt_scale(iteration: int, iterations: int, start: float = 0.26, end: float = 1.0,
              fraction: float = 0.75) -> float:
    total = fraction * iterations
    if total <= 0 or iteration >= total:
        return end
    return end + 0.5 * (start - end) * (1.0 + math.cos(math.pi * iteration / total))


def drt_resolution(width: int, height: int, scale: float):
    """Per-view image size at a schedule value (rounded to the nearest pixel, at least 1)."""
    return max(1, int(round(width * scale))), max(1, int(round(height * scale)))
