"""Seeded synthetic inputs for the gMCO dwell-time optimisation.

This module only draws geometry, weights and random start values.  It holds
none of the method's arithmetic (no dose law, no objective, no optimiser): the
FP64 oracle and the HIP library both receive the arrays it produces and
compute everything else on their own.

The clinical cohort of the paper (Sec. 2.1.1: 562 prostate cases, 16-18
catheters, 102-385 active dwells, 2,753-15,998 optimisation points) is not
available, so seeded synthetic cases of the same structure stand in for it:

* target: points uniform inside an ellipsoid centred at the origin,
  semi-axes (a_x, a_y, a_z) = (2.0, 1.75, 1.75) cm (full lengths 4 x 3.5 x 3.5);
* urethra: points on a 0.3 cm radius cylinder about the z axis, |z| <= a_z;
* rectum: points uniform in the slab y in [-a_y-1.0, -a_y-0.5] whose
  footprint is the ellipse (x/a_x)^2 + (z/a_z)^2 <= 1;
* bladder: the mirror slab y in [a_y+0.5, a_y+1.0], same footprint;
* catheters parallel to z at half-integer nodes of a 1 cm grid, ordered by
  (radius, polar angle in [0, 2 pi)) and the first n_cath kept; each carries
  n_dwell dwells at z_k = (k - (n_dwell-1)/2) * (5 cm / n_dwell).

Structure order follows Table 1: 0 target, 1 urethra, 2 bladder, 3 rectum.
Points are emitted grouped by structure in that order.

Hidden weights (Sec. 2.1.2, eq. (obj)) are drawn log-uniform in [0.1, 10] per
structure and normalised so that each plan's weights sum to one.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TARGET, URETHRA, BLADDER, RECTUM = 0, 1, 2, 3
STRUCTURE_NAMES = ("target", "urethra", "bladder", "rectum")
PRESCRIPTION_GY = 15.0

URETHRA_RADIUS_CM = 0.3
SLAB_NEAR_CM = 0.5
SLAB_FAR_CM = 1.0
DWELL_SPAN_CM = 5.0


@dataclass
class Case:
    """One synthetic patient: geometry, structure labels and volumes."""

    dwell_xyz: np.ndarray          # (K, 3) float64, cm
    pt_xyz: np.ndarray             # (M, 3) float64, cm
    group: np.ndarray              # (M,) int32 structure id
    volume_cc: np.ndarray          # (4,) float64 analytic structure volumes
    semi_axes: tuple = (2.0, 1.75, 1.75)
    prescription_gy: float = PRESCRIPTION_GY
    meta: dict = field(default_factory=dict)
    # surface / volume variant: group -> organ map and a separate DVH point set
    group_organ: np.ndarray = None  # (G,) int32, None: every group is an organ
    dvh_xyz: np.ndarray = None      # (M_dvh, 3) float64, cm
    dvh_organ: np.ndarray = None    # (M_dvh,) int32

    @property
    def K(self) -> int:
        return int(self.dwell_xyz.shape[0])

    @property
    def M(self) -> int:
        return int(self.pt_xyz.shape[0])

    def counts(self) -> np.ndarray:
        return np.bincount(self.group, minlength=4).astype(np.int64)


def catheter_nodes(n_cath: int) -> np.ndarray:
    """(n_cath, 2) catheter (x, y) positions in cm.

    Half-integer nodes of a 1 cm grid sorted by squared radius (exact for
    half-integers) and then by polar angle in [0, 2 pi)."""
    span = int(math.ceil(math.sqrt(n_cath))) + 2
    nodes = []
    for ix in range(-span, span):
        for iy in range(-span, span):
            x, y = ix + 0.5, iy + 0.5
            ang = math.atan2(y, x)
            if ang < 0.0:
                ang += 2.0 * math.pi
            nodes.append((x * x + y * y, ang, x, y))
    nodes.sort(key=lambda n: (n[0], n[1]))
    return np.array([[n[2], n[3]] for n in nodes[:n_cath]], dtype=np.float64)


def dwell_positions(n_cath: int, n_dwell: int, z_scale: float = 1.0) -> np.ndarray:
    """(n_cath * n_dwell, 3) dwell coordinates, catheter-major."""
    xy = catheter_nodes(n_cath)
    step = DWELL_SPAN_CM / n_dwell * z_scale
    z = (np.arange(n_dwell, dtype=np.float64) - (n_dwell - 1) / 2.0) * step
    out = np.empty((n_cath * n_dwell, 3), dtype=np.float64)
    for c in range(n_cath):
        out[c * n_dwell:(c + 1) * n_dwell, 0] = xy[c, 0]
        out[c * n_dwell:(c + 1) * n_dwell, 1] = xy[c, 1]
        out[c * n_dwell:(c + 1) * n_dwell, 2] = z
    return out


def _uniform_ellipsoid(rng, n, a):
    out = np.empty((0, 3))
    while out.shape[0] < n:
        u = rng.uniform(-1.0, 1.0, size=(2 * n + 16, 3))
        u = u[(u * u).sum(1) <= 1.0]
        out = np.concatenate([out, u * np.asarray(a)])
    return out[:n]


def _urethra(rng, n, a):
    ang = rng.uniform(0.0, 2.0 * math.pi, size=n)
    z = rng.uniform(-a[2], a[2], size=n)
    return np.stack([URETHRA_RADIUS_CM * np.cos(ang),
                     URETHRA_RADIUS_CM * np.sin(ang), z], axis=1)


def _slab(rng, n, a, y_lo, y_hi):
    out = np.empty((0, 3))
    while out.shape[0] < n:
        u = rng.uniform(-1.0, 1.0, size=(2 * n + 16, 2))
        u = u[(u * u).sum(1) <= 1.0]
        y = rng.uniform(y_lo, y_hi, size=u.shape[0])
        pts = np.stack([u[:, 0] * a[0], y, u[:, 1] * a[2]], axis=1)
        out = np.concatenate([out, pts])
    return out[:n]


def structure_volumes(a) -> np.ndarray:
    ax, ay, az = a
    slab = (SLAB_FAR_CM - SLAB_NEAR_CM) * math.pi * ax * az
    return np.array([4.0 / 3.0 * math.pi * ax * ay * az,
                     math.pi * URETHRA_RADIUS_CM ** 2 * 2.0 * az,
                     slab, slab], dtype=np.float64)


def make_case(n_cath: int, n_dwell: int, n_points, seed: int,
              semi_axes=(2.0, 1.75, 1.75), jitter: float = 0.0) -> Case:
    """Seeded synthetic case.

    n_points = (n_target, n_urethra, n_bladder, n_rectum).  jitter > 0 scales
    each semi-axis by U(1 - jitter, 1 + jitter) and the dwell z spacing with
    the z semi-axis."""
    rng = np.random.default_rng(seed)
    a = np.asarray(semi_axes, dtype=np.float64)
    z_scale = 1.0
    if jitter > 0.0:
        f = rng.uniform(1.0 - jitter, 1.0 + jitter, size=3)
        a = a * f
        z_scale = f[2]
    nt, nu, nb, nr = (int(v) for v in n_points)
    pts = [
        _uniform_ellipsoid(rng, nt, a),
        _urethra(rng, nu, a),
        _slab(rng, nb, a, a[1] + SLAB_NEAR_CM, a[1] + SLAB_FAR_CM),
        _slab(rng, nr, a, -a[1] - SLAB_FAR_CM, -a[1] - SLAB_NEAR_CM),
    ]
    group = np.concatenate([np.full(n, g, dtype=np.int32)
                            for g, n in enumerate((nt, nu, nb, nr))])
    return Case(dwell_xyz=dwell_positions(n_cath, n_dwell, z_scale),
                pt_xyz=np.ascontiguousarray(np.concatenate(pts, axis=0)),
                group=group,
                volume_cc=structure_volumes(a),
                semi_axes=tuple(float(v) for v in a),
                meta=dict(n_cath=n_cath, n_dwell=n_dwell, seed=seed,
                          jitter=jitter))


# ---------------------------------------------------------------------------
# Surface and volume points (Table 1 lists both for every organ): 8 groups,
# group 2 j + 0 the surface and 2 j + 1 the volume points of organ j, and a
# separate, denser DVH point set labelled by organ (Sec. 2.1.1 counts about
# five DVH points per optimisation point).
#   target surface: points on the ellipsoid (scaled unit directions);
#   urethra surface: the 0.3 cm cylinder; urethra volume: inside it;
#   bladder / rectum surface: the two faces of the slab over its footprint.
# ---------------------------------------------------------------------------
SV_GROUP_ORGAN = np.array([0, 0, 1, 1, 2, 2, 3, 3], dtype=np.int32)


def _ellipsoid_surface(rng, n, a):
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return u * np.asarray(a)


def _urethra_volume(rng, n, a):
    ang = rng.uniform(0.0, 2.0 * math.pi, size=n)
    r = URETHRA_RADIUS_CM * np.sqrt(rng.uniform(0.0, 1.0, size=n))
    z = rng.uniform(-a[2], a[2], size=n)
    return np.stack([r * np.cos(ang), r * np.sin(ang), z], axis=1)


def _slab_faces(rng, n, a, y_lo, y_hi):
    pts = _slab(rng, n, a, y_lo, y_hi)
    pts[:, 1] = np.where(rng.uniform(size=n) < 0.5, y_lo, y_hi)
    return pts


def _organ_samplers(a):
    yb = (a[1] + SLAB_NEAR_CM, a[1] + SLAB_FAR_CM)
    yr = (-a[1] - SLAB_FAR_CM, -a[1] - SLAB_NEAR_CM)
    surface = [lambda r, n: _ellipsoid_surface(r, n, a), lambda r, n: _urethra(r, n, a),
               lambda r, n: _slab_faces(r, n, a, *yb), lambda r, n: _slab_faces(r, n, a, *yr)]
    volume = [lambda r, n: _uniform_ellipsoid(r, n, a), lambda r, n: _urethra_volume(r, n, a),
              lambda r, n: _slab(r, n, a, *yb), lambda r, n: _slab(r, n, a, *yr)]
    return surface, volume


def make_case_sv(n_cath: int, n_dwell: int, n_points, seed: int, dvh_points=None,
                 semi_axes=(2.0, 1.75, 1.75), jitter: float = 0.0) -> Case:
    """Seeded case with surface and volume points.  n_points = 8 counts in
    group order (target surface, target volume, urethra surface, ...);
    dvh_points = 4 per-organ counts of the DVH set (None: no DVH set)."""
    rng = np.random.default_rng(seed)
    a = np.asarray(semi_axes, dtype=np.float64)
    z_scale = 1.0
    if jitter > 0.0:
        f = rng.uniform(1.0 - jitter, 1.0 + jitter, size=3)
        a = a * f
        z_scale = f[2]
    surface, volume = _organ_samplers(a)
    counts = [int(v) for v in n_points]
    pts, group = [], []
    for g, n in enumerate(counts):
        j, kind = divmod(g, 2)
        pts.append((surface if kind == 0 else volume)[j](rng, n))
        group.append(np.full(n, g, dtype=np.int32))
    c = Case(dwell_xyz=dwell_positions(n_cath, n_dwell, z_scale),
             pt_xyz=np.ascontiguousarray(np.concatenate(pts, axis=0)),
             group=np.concatenate(group), volume_cc=structure_volumes(a),
             semi_axes=tuple(float(v) for v in a),
             meta=dict(n_cath=n_cath, n_dwell=n_dwell, seed=seed, jitter=jitter, surface_volume=True),
             group_organ=SV_GROUP_ORGAN.copy())
    if dvh_points is not None:
        drng = np.random.default_rng(seed + 100_000)
        dp, dl = [], []
        for j, n in enumerate(int(v) for v in dvh_points):
            dp.append(volume[j](drng, n))
            dl.append(np.full(n, j, dtype=np.int32))
        c.dvh_xyz = np.ascontiguousarray(np.concatenate(dp, axis=0))
        c.dvh_organ = np.concatenate(dl)
    return c


def case_sv_small() -> Case:
    """8-group case for parity tests: 12 x 8 dwells, 1,300 optimisation points,
    a DVH set of 3,250."""
    return make_case_sv(12, 8, (150, 500, 100, 100, 75, 150, 75, 150), seed=31,
                        dvh_points=(1300, 500, 725, 725))


def case_sv_c2() -> Case:
    """The 360-dwell paper-scale layout with surface and volume points
    (20,000: target 2,000 + 8,000, urethra 1,000 + 1,000, bladder and rectum
    1,000 + 3,000 each) and a 5x denser DVH set (100,000 points)."""
    return make_case_sv(18, 20, (2000, 8000, 1000, 1000, 1000, 3000, 1000, 3000), seed=2,
                        dvh_points=(50000, 10000, 20000, 20000))


def hidden_weights(n_plans: int, seed: int, n_struct: int = 4,
                   lo: float = 0.1, hi: float = 10.0) -> np.ndarray:
    """(n_plans, n_struct) log-uniform weights normalised to sum one per plan."""
    rng = np.random.default_rng(seed)
    w = np.exp(rng.uniform(math.log(lo), math.log(hi), size=(n_plans, n_struct)))
    return w / w.sum(axis=1, keepdims=True)


def uniform_draws(shape, seed: int) -> np.ndarray:
    """U(0, 1) draws, e.g. for degenerate random starts; the caller maps them."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=shape)


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the configurations the method is measured on.
# ---------------------------------------------------------------------------

def case_c1() -> Case:
    """160 dwells (16 catheters x 10), 2,400 points (1200/300/450/450)."""
    return make_case(16, 10, (1200, 300, 450, 450), seed=1)


def weights_c1() -> np.ndarray:
    return hidden_weights(8, seed=11)


def case_c2() -> Case:
    """360 dwells (18 catheters x 20), 20,000 points (10000/2000/4000/4000)."""
    return make_case(18, 20, (10000, 2000, 4000, 4000), seed=2)


def weights_c2(n_plans: int = 1000) -> np.ndarray:
    return hidden_weights(n_plans, seed=12)


def case_batch(index: int) -> Case:
    """One case of the uneven 64-case batch: K in [120, 400], M in [8k, 30k]
    split 50/10/20/20, semi-axes jittered by +-20 %."""
    rng = np.random.default_rng(1000 + index)
    K = int(rng.integers(120, 401))
    M = int(rng.integers(8000, 30001))
    n_dwell = 20
    n_cath = max(1, int(round(K / n_dwell)))
    n_dwell = int(math.ceil(K / n_cath))
    nt = M // 2
    nu = M // 10
    nb = M // 5
    nr = M - nt - nu - nb
    c = make_case(n_cath, n_dwell, (nt, nu, nb, nr), seed=1000 + index, jitter=0.2)
    c.dwell_xyz = c.dwell_xyz[:K]
    c.meta["K_target"] = K
    return c


def small_case(K_cath=4, n_dwell=4, n_points=(60, 20, 25, 25), seed=3) -> Case:
    """A tiny case for brute-force and unit checks."""
    return make_case(K_cath, n_dwell, n_points, seed=seed)


def case_learned(index: int) -> Case:
    """Cases for the learned warm start: the paper-scale layout (18 x 20 = 360
    dwells, 20,000 points 50/10/20/20) with semi-axes jittered by +-20 %."""
    return make_case(18, 20, (10000, 2000, 4000, 4000), seed=5000 + index, jitter=0.2)


def weights_learned(index: int, n_plans: int = 1000) -> np.ndarray:
    return hidden_weights(n_plans, seed=6000 + index)


def mlp_init(sizes, seed: int) -> np.ndarray:
    """Seeded He-uniform initial parameters of a fully connected network,
    flat: for each layer W (n_out x n_in, row-major) then b (zeros)."""
    rng = np.random.default_rng(seed)
    parts = []
    for k in range(len(sizes) - 1):
        n_in, n_out = sizes[k], sizes[k + 1]
        lim = math.sqrt(6.0 / n_in)
        parts.append(rng.uniform(-lim, lim, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts)


def batch_order(n_samples: int, n_steps: int, batch: int, seed: int) -> np.ndarray:
    """(n_steps * batch,) int32 sample indices: consecutive seeded shuffles."""
    rng = np.random.default_rng(seed)
    out = []
    need = n_steps * batch
    while sum(len(o) for o in out) < need:
        out.append(rng.permutation(n_samples))
    return np.concatenate(out)[:need].astype(np.int32)
