"""Cache of the autotuner's launch shapes (spmesl_autotune), as JSON.

A context's launch shapes (the dense tier's block size b, the zero fill's
grid, the row-tiled KKT pass's rows per tile, the screen factor) are picked
by timing solves of the caller's problem on the device
(`Context.autotune`, the library's `spmesl_autotune`).  This module keeps
the results across processes, keyed by device name, precision and shape
(n, p), in a JSON file (``$SPMESL_TUNING_CACHE`` or
``~/.cache/spmesl/tuning.json``).  Host logic only: every timing runs in the
library.
"""
from __future__ import annotations

import json
import os

FIELDS = ("dense_block", "fill_blocks", "kkt_rows", "screen_permille", "fill_split")


def cache_path() -> str:
    return os.environ.get("SPMESL_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "spmesl", "tuning.json"))


def key(device: str, precision: str, n: int, p: int) -> str:
    return f"{device}|{precision}|n={int(n)}|p={int(p)}"


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(entry_key: str, tuning: dict, ms: float, path: str | None = None) -> None:
    path = path or cache_path()
    data = load(path)
    data[entry_key] = {"tuning": {f: int(tuning[f]) for f in FIELDS}, "ms_per_solve": float(ms)}
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(ctx, X, lambda0, tol=1e-8, precision="fp64", reps=5, path=None, device_name=None, retune=False):
    """The launch shapes for this problem's device, precision and shape: from
    the cache, or found by ctx.autotune (and cached).  They are set on ctx.
    Returns (tuning dict, ms per solve when tuned here else the cached one,
    whether it came from the cache)."""
    if device_name is None:
        import torch
        device_name = torch.cuda.get_device_name(X.device)
    n, p = X.shape
    k = key(device_name, precision, n, p)
    hit = None if retune else load(path).get(k)
    if hit is not None and all(f in hit.get("tuning", {}) for f in FIELDS):
        ctx.set_tuning(hit["tuning"])
        return dict(hit["tuning"]), float(hit.get("ms_per_solve", 0.0)), True
    t, ms = ctx.autotune(X, lambda0, tol, precision, reps=reps)
    store(k, t, ms, path)
    return t, ms, False
