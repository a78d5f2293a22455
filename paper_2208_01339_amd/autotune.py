"""Autotuner cache for the batched block product.

pp_batch_autotune (C ABI) times every supported lanes-per-row layout on one
polynomial step of the handle's own operator and keeps the fastest.  This
module remembers the choice per problem shape in a JSON file so that later
handles of the same shape skip the timing: the path comes from the
environment variable PP_AUTOTUNE_CACHE (default ~/.cache/ppcg/autotune.json).
"""
from __future__ import annotations

import json
import os

from . import binding as B


def cache_path() -> str:
    return os.environ.get("PP_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ppcg", "autotune.json"))


def _key(stats: dict, mixed: bool) -> str:
    return "n%d_nnz%d_nb%d_nsys%d_%s" % (stats["n"], stats["nnz_stored"], stats["nb"], stats["nsys"],
                                        "f32" if mixed else "f64")


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(handle, mixed: bool, use_cache: bool = True) -> dict:
    """Pick the layout for `handle` (after pp_batch_setup); returns {"w", "us", "cached"}."""
    st = B.pp_batch_get_stats(handle)
    key = _key(st, mixed)
    path = cache_path()
    db = _load(path) if use_cache else {}
    if key in db:
        B.pp_batch_set_layout(handle, db[key]["w"])
        return dict(db[key], cached=True)
    w, us = B.pp_batch_autotune(handle)
    rec = {"w": int(w), "us": float(us)}
    if use_cache:
        db[key] = rec
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(db, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass
    return dict(rec, cached=False)
