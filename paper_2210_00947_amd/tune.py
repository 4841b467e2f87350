"""Launch-shape tuning with an on-disk JSON cache.

The library's own timing loop (``mgar_autotune``) picks, for every stencil mode
on every grid level and precision class, the fastest of its candidate launch
shapes. Tuning one grid takes well under a second; the cache stores the
winning shapes under a key made of the GPU architecture and the grid shape, so
later handles on the same kind of GPU and grid install them without timing.

Cache file: ``$MGAR_TUNE_CACHE`` if set, else ``~/.cache/mgar/tune.json``.
"""
import json
import os
import tempfile

NMODES = 7


def cache_path():
    return os.environ.get("MGAR_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "mgar", "tune.json")


def cache_key(params, arch):
    """Architecture + grid shape + precision: everything a shape choice depends on."""
    dims = (params.nelx, params.nely, params.nelz if params.dim == 3 else 0)
    return f"{arch}|d{params.dim}|{dims[0]}x{dims[1]}x{dims[2]}|L{params.levels}|prec{params.precision}"


def _load(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path, data):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tune-", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def read_shapes(handle, levels):
    """Every installed shape as {"cls/level/mode": [kind, kz, zd, ntx]}."""
    return {f"{c}/{l}/{m}": handle.mgar_tune_get(c, l, m)
            for c in range(2) for l in range(levels) for m in range(NMODES)}


def apply_shapes(handle, shapes):
    for k, v in shapes.items():
        c, l, m = (int(s) for s in k.split("/"))
        handle.mgar_tune_set(c, l, m, v)


def autotune(handle, params, arch, path=None, reps=20, refresh=False):
    """Install tuned launch shapes on ``handle``: from the cache when it holds
    this (arch, grid) key, else by timing, then store. Returns (shapes, source)
    with source "cache" or "timed"."""
    path = path or cache_path()
    key = cache_key(params, arch)
    data = _load(path)
    entry = data.get(key)
    if entry and not refresh:
        try:
            apply_shapes(handle, entry["shapes"])
            return entry["shapes"], "cache"
        except Exception:   # stale or foreign entry: time again
            pass
    best = handle.mgar_autotune(reps)
    shapes = read_shapes(handle, params.levels)
    data[key] = {"shapes": shapes, "best_us": best}
    try:
        _store(path, data)
    except OSError:
        pass                # read-only home: the shapes are installed anyway
    return shapes, "timed"


def device_arch(device=0):
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
