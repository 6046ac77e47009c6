"""Class solution of Table 1 for a 15 Gy prostate boost: eq. 1 parameters
(w_min, D_min [Gy], D_max [Gy], w_max) per structure, volume and surface
points.  Row order: target, urethra, bladder, rectum."""
import numpy as np

STRUCTURES = ("target", "urethra", "bladder", "rectum")

VOLUME = np.array([
    [200.0, 15.0, 22.5, 1.0],    # target
    [30.0, 14.0, 16.0, 160.0],   # urethra
    [0.0, 0.0, 7.5, 60.0],       # bladder
    [0.0, 0.0, 7.5, 15.0],       # rectum
])

SURFACE = np.array([
    [200.0, 15.0, 22.5, 80.0],
    [30.0, 14.0, 16.0, 160.0],
    [0.0, 0.0, 7.5, 60.0],
    [0.0, 0.0, 7.5, 15.0],
])

# Both rows per structure, surface first: the 8 parameter groups of a case
# with surface and volume points (group 2 j + 0 surface, 2 j + 1 volume of
# structure j).
SURFACE_VOLUME = np.stack([SURFACE, VOLUME], axis=1).reshape(8, 4)

PRESCRIPTION_GY = 15.0
