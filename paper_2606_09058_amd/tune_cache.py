"""Persistent cache of autotuned plan knobs (a JSON file).

A plan created with KS_PLAN_AUTOTUNE times its knobs on its own buffers (the
symmetric product's tiles per workgroup, by column segment; the back-transform
block; the large-GEMM threshold; the divide-and-conquer leaf).  The cache keeps
the chosen knobs per (architecture, operation, dtype, order, batch, spin,
precision, route), so that a later plan of the same key takes them with
ks_plan_set_tuning and times nothing.  Host-side only: reading and writing the
file, no device work.
"""
from __future__ import annotations

import json
import os
import tempfile

VERSION = 1
KNOBS = ("tiles_per_workgroup", "nseg", "seg_first", "seg_tiles", "backtr_block", "gemm_big_min_k", "dc_leaf")


def cache_key(arch: str, op: str, dtype: str, order: int, batch: int, spin: str, precision: str,
              route: str) -> str:
    """The key of one plan shape, e.g. 'gfx950/gevd/real64/6656/1/collinear/fp64/onestage'."""
    for part in (arch, op, dtype, spin, precision, route):
        if not part or "/" in part:
            raise ValueError("cache key parts must be non-empty and contain no '/': %r" % (part,))
    if int(order) < 1 or int(batch) < 1:
        raise ValueError("order and batch must be positive")
    return "/".join([arch, op, dtype, str(int(order)), str(int(batch)), spin, precision, route])


def load(path: str) -> dict:
    """All entries of the cache file ({} if it does not exist)."""
    if not os.path.exists(path):
        return {}
    with open(path, "r", encoding="utf-8") as f:
        doc = json.load(f)
    if not isinstance(doc, dict) or doc.get("version") != VERSION or not isinstance(doc.get("entries"), dict):
        raise ValueError("%s is not a tuning cache of version %d" % (path, VERSION))
    return doc["entries"]


def lookup(path: str, key: str):
    """The knobs stored under key, or None."""
    e = load(path).get(key)
    if e is None:
        return None
    missing = [k for k in KNOBS if k not in e]
    if missing:
        raise ValueError("cache entry %s lacks %s" % (key, ", ".join(missing)))
    return e


def store(path: str, key: str, entry: dict) -> None:
    """Add or replace one entry; the file is replaced atomically (write to a
    temporary file in the same directory, then rename)."""
    missing = [k for k in KNOBS if k not in entry]
    if missing:
        raise ValueError("entry lacks %s" % ", ".join(missing))
    entries = load(path)
    entries[key] = entry
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(prefix=".tune_cache.", dir=d)
    try:
        with os.fdopen(fd, "w", encoding="utf-8") as f:
            json.dump({"version": VERSION, "entries": entries}, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.unlink(tmp)
        raise
