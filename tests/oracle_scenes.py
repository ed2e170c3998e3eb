"""Hand-built tiny scenes for the oracle pins (no renderer arithmetic)."""
import math

import numpy as np

from paper_2501_08174_amd.scenes import Camera, Scene, make_camera

Y00 = 0.5 / math.sqrt(math.pi)


def front_camera(size=64, dist=4.0):
    """R = I at (0, 0, -dist), 60 degree horizontal field of view."""
    return make_camera(np.eye(3), np.array([0.0, 0.0, -dist]), size, size)


def scene_from(means, scales, quats, opac, rgb, cams, sh_extra=None):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    sh = ((np.asarray(rgb, np.float64).reshape(n, 3) - 0.5) / Y00)[:, None, :]
    deg = 0
    if sh_extra is not None:
        sh = np.concatenate([sh, sh_extra], axis=1)
        deg = int(round(math.sqrt(sh.shape[1]))) - 1
    return Scene(means=means,
                 scales=np.asarray(scales, np.float32).reshape(n, 2),
                 quats=np.asarray(quats, np.float32).reshape(n, 4),
                 opac=np.asarray(opac, np.float32).reshape(n),
                 sh=np.asarray(sh, np.float32), sh_degree=deg, cams=list(cams),
                 masks=[np.ones((c.height, c.width), np.uint8) for c in cams])


def centre_on_pixel(cam: Camera, i: int, j: int, depth: float):
    """World point whose projection in the front camera (R = I, centre at
    z = -4) is pixel (i, j)'s centre, up to float32 rounding."""
    x = (i + 0.5 - cam.cx) * depth / cam.fx
    y = (j + 0.5 - cam.cy) * depth / cam.fy
    return np.array([x, y, depth - 4.0])
