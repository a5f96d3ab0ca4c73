"""Oracle evaluation on crops of very large images (sampled parity checks).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The transform is local: a coefficient depends only on image samples within a
bounded footprint (radius 4 samples per scale for CDF 9/7, so roughly
8 * 2^l pixels after l scales).  The oracle run on a crop therefore equals the
oracle run on the whole image at every coefficient whose footprint stays away
from the crop's artificial edges; at a real image edge the crop keeps the real
edge and its symmetric extension.  Crops start at multiples of 2^levels so the
subbands of the crop are exact slices of the subbands of the whole image.
"""
from __future__ import annotations

import numpy as np

from .lifting import level_shapes


def band_boxes(h: int, w: int, levels: int):
    """[(level, band, r0, r1, c0, c1)] of every subband of a Mallat pyramid.

    Bands are 'HL', 'LH', 'HH' per level (1 = finest) and 'LL' of the last."""
    out = []
    shapes = level_shapes(h, w, levels)
    for lvl, (hl, wl) in enumerate(shapes, start=1):
        he, we = (hl + 1) // 2, (wl + 1) // 2
        out += [(lvl, "HL", 0, he, we, wl), (lvl, "LH", he, hl, 0, we), (lvl, "HH", he, hl, we, wl)]
        if lvl == levels:
            out.append((lvl, "LL", 0, he, 0, we))
    return out


def crop_pyramid(Y: np.ndarray, levels: int, r0: int, r1: int, c0: int, c1: int) -> np.ndarray:
    """The Mallat pyramid of the crop X[r0:r1, c0:c1], cut out of the pyramid Y
    of the whole image (subband by subband)."""
    H, W = Y.shape
    s = 1 << levels
    assert r0 % s == 0 and c0 % s == 0
    assert (r1 % s == 0 or r1 == H) and (c1 % s == 0 or c1 == W)
    ch, cw = r1 - r0, c1 - c0
    full = band_boxes(H, W, levels)
    crop = band_boxes(ch, cw, levels)
    out = np.empty((ch, cw), dtype=Y.dtype)
    for (lv, b, fr0, fr1, fc0, fc1), (lv2, b2, cr0, cr1, cc0, cc1) in zip(full, crop):
        assert (lv, b) == (lv2, b2)
        ro, co = r0 >> lv, c0 >> lv
        out[cr0:cr1, cc0:cc1] = Y[fr0 + ro: fr0 + ro + (cr1 - cr0), fc0 + co: fc0 + co + (cc1 - cc0)]
    return out


def crop_valid_mask(H: int, W: int, levels: int, r0: int, r1: int, c0: int, c1: int,
                    margin: int) -> np.ndarray:
    """Mask over the crop pyramid: True where a coefficient's image position
    lies at least `margin` pixels from every artificial (non-image) crop edge."""
    ch, cw = r1 - r0, c1 - c0
    mask = np.zeros((ch, cw), dtype=bool)
    for lv, b, cr0, cr1, cc0, cc1 in band_boxes(ch, cw, levels):
        rows = (np.arange(cr1 - cr0) << lv) + r0
        cols = (np.arange(cc1 - cc0) << lv) + c0
        okr = np.ones(len(rows), bool)
        okc = np.ones(len(cols), bool)
        if r0 > 0:
            okr &= rows - r0 >= margin
        if r1 < H:
            okr &= r1 - rows >= margin
        if c0 > 0:
            okc &= cols - c0 >= margin
        if c1 < W:
            okc &= c1 - cols >= margin
        mask[cr0:cr1, cc0:cc1] = np.outer(okr, okc)
    return mask


def default_margin(levels: int) -> int:
    """Crop margin (pixels) that covers the footprint growth over `levels`."""
    return 16 * (1 << levels) + 16


def probe_crops(H: int, W: int, levels: int, size: int = 256):
    """Crop boxes at the four corners, the four edge midpoints and the centre,
    each extended by the default margin and aligned to 2^levels."""
    s = 1 << levels
    m = default_margin(levels)
    boxes = []
    size = max(size, s)
    for fr in (0.0, 0.5, 1.0):
        for fc in (0.0, 0.5, 1.0):
            rc = int(fr * (H - size)) // s * s
            cc = int(fc * (W - size)) // s * s
            r0 = max(0, (rc - m) // s * s)
            c0 = max(0, (cc - m) // s * s)
            r1 = rc + size + m
            c1 = cc + size + m
            r1 = H if r1 >= H else -(-r1 // s) * s
            c1 = W if c1 >= W else -(-c1 // s) * s
            r1, c1 = min(r1, H), min(c1, W)
            boxes.append((r0, r1, c0, c1))
    return boxes
