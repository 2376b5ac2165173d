"""Launch-shape tuning of the BF16/FP16 face kernels with a JSON cache.

`tuned(prob, mlp, q, ws)` returns the launch shapes for a problem: it runs
neno6_autotune (which times the library's candidate shapes on the GPU) once
per (device, equation, precision, face-count bucket) and keeps the winner in
a JSON file, so later runs of similar problems start tuned.  The cache file
is $NENO6_TUNING_CACHE, else $XDG_CACHE_HOME/neno6_tuning.json (default
~/.cache).  Host logic only; the timing itself is done by the library.
"""
from __future__ import annotations

import json
import math
import os
import tempfile

import torch

from . import native


def default_path() -> str:
    p = os.environ.get("NENO6_TUNING_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "neno6_tuning.json")


def cache_key(prob: native.Problem, device=None, mlp: native.Mlp | None = None) -> str:
    """Device name, equation, precision (and the two-part FP16 re-check when
    mlp selects it) and the face count rounded to a half-octave bucket
    (shapes tuned at one size serve nearby sizes)."""
    name = torch.cuda.get_device_name(device)
    bucket = round(2.0 * math.log2(max(prob.n_faces, 1))) / 2.0
    rc = ("|rc%d" % mlp.recheck_mode if mlp is not None and mlp.recheck_mode
          and prob.precision == native.FP16 else "")
    return "%s|eq%d|prec%d%s|faces~2^%.1f" % (name, prob.equation, prob.precision, rc, bucket)


def _read(path: str) -> dict:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _write(path: str, d: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(prefix=".neno6_tuning.", dir=os.path.dirname(os.path.abspath(path)))
    with os.fdopen(fd, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(prob: native.Problem, mlp: native.Mlp, q: torch.Tensor, ws: torch.Tensor,
          path: str | None = None, reps: int = 3, refresh: bool = False):
    """Sets prob's launch shapes from the cache, tuning first if the key is
    missing (or refresh).  Returns (shapes dict, ms per face pass or None if
    the shapes came from the cache)."""
    path = path or default_path()
    key = cache_key(prob, q.device, mlp)
    cache = _read(path)
    ent = cache.get(key)
    fields = [k for k, _ in native.TuningStruct._fields_]
    if ent is not None and not refresh and all(k in ent for k in fields):
        shapes = {k: int(ent[k]) for k in fields}
        prob.set_tuning(shapes)
        return shapes, None
    best, ms = native.neno6_autotune(prob, mlp, q, ws, reps)
    shapes = best.as_dict()
    cache = _read(path)  # re-read: another process may have written meanwhile
    cache[key] = dict(shapes, ms=ms)
    try:
        _write(path, cache)
    except OSError:  # read-only location: the shapes still apply to this run
        pass
    prob.set_tuning(shapes)
    return shapes, ms
