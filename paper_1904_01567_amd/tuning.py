"""Cache of autotuned launch shapes, keyed by shape bucket and kernel family.

`gmco_autotune` times launch shapes (split count, tile-to-XCD mapping,
workgroup shape) on one loaded case.  Cases of one padded dwell count, a
similar point count and the same plan capacity choose alike, so a tuned
shape can be reused instead of timed again: this module keys the tuning by
(kernel family, padded dwells, point-count bucket, padded plans) and keeps
it in a JSON file.  Only the lookup and the marshalling are here; the timing
and the shapes themselves live in the library (gmco_autotune,
gmco_get_tuning / gmco_set_tuning).
"""
from __future__ import annotations

import json
import os
from typing import Optional

K_ALIGN = 32   # padded dwell count granularity of the library
P_ALIGN = 64   # plans per tile


def _round_up(v: int, a: int) -> int:
    return (v + a - 1) // a * a


def family(dtype: str) -> str:
    """Kernel family a dtype's tuning belongs to (the FP32-operand modes share
    split and mapping; the FP64-accumulated kernel has its own shapes)."""
    return {"bf16": "lp", "fp8": "lp", "f32": "f32", "f32chunk64": "f32", "f32acc64": "f32acc64"}[dtype]


class TuningCache:
    def __init__(self, path: Optional[str] = None, point_bucket: int = 4000):
        self.path = path
        self.point_bucket = int(point_bucket)
        self.entries: dict = {}
        self.hits = self.misses = 0
        if path and os.path.exists(path):
            with open(path) as fh:
                data = json.load(fh)
            if data.get("point_bucket") == self.point_bucket:
                self.entries = dict(data.get("entries", {}))

    def key(self, planner, dtype: str) -> str:
        kp = _round_up(planner.K, K_ALIGN)
        mb = (planner.M + self.point_bucket // 2) // self.point_bucket
        pp = _round_up(planner.max_plans, P_ALIGN)
        return f"{family(dtype)}:Kp{kp}:M{mb * self.point_bucket}:Pp{pp}"

    def tune(self, planner, dtype: str, reps: int = 3) -> dict:
        """Apply the cached tuning of the planner's bucket, else autotune it
        (timing on the planner's loaded case and weight batch) and remember
        the result.  Returns the tuning in effect."""
        k = self.key(planner, dtype)
        t = self.entries.get(k)
        if t is not None:
            planner.set_tuning(t["split"], lp_shape=t["lp_shape"], xcd_map=t["xcd_map"], dtype=dtype)
            self.hits += 1
        else:
            planner.autotune(dtype=dtype, reps=reps)
            t = planner.tuning(dtype)
            self.entries[k] = {"split": int(t["split"]), "lp_shape": int(t["lp_shape"]),
                               "xcd_map": int(t["xcd_map"])}
            self.misses += 1
        return planner.tuning(dtype)

    def save(self, path: Optional[str] = None) -> None:
        path = path or self.path
        if not path:
            return
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump({"point_bucket": self.point_bucket, "entries": self.entries}, fh, indent=1,
                      sort_keys=True)
        os.replace(tmp, path)
