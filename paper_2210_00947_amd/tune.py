"""Launch-shape tuning with an on-disk JSON cache.

The library's own timing loop (``mgar_autotune``) picks, for every stencil mode
on every grid level and precision class, the fastest of its candidate launch
shapes. Tuning one grid takes well under a second; the cache stores the
winning shapes under a key made of the GPU architecture and the grid shape, so
later handles on the same kind of GPU and grid install them without timing.

Cache file: ``$MGAR_TUNE_CACHE`` if set, else ``~/.cache/mgar/tune.json``.
Keys missing from it are looked up in ``tune_shipped.json`` beside this
module (shapes tuned on a reference GPU of the same architecture, written by
``python -m paper_2210_00947_amd.tune --ship WORKLOAD...``), and timed only
when neither holds them.
"""
import json
import os
import tempfile

NMODES = 7
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_shipped.json")


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


def autotune(handle, params, arch, path=None, reps=20, refresh=False, shipped=SHIPPED):
    """Install tuned launch shapes on ``handle``: from the cache when it holds
    this (arch, grid) key, else from the shipped table, else by timing, then
    store. Returns (shapes, source) with source "cache", "shipped" or "timed"."""
    path = path or cache_path()
    key = cache_key(params, arch)
    data = _load(path)
    if not refresh:
        for src, table in (("cache", data), ("shipped", _load(shipped) if shipped else {})):
            entry = table.get(key)
            if not entry:
                continue
            try:
                apply_shapes(handle, entry["shapes"])
                return entry["shapes"], src
            except Exception:   # stale or foreign entry: try the next source
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


def ship(names, reps=50, out=SHIPPED):
    """Time every candidate shape of the named workloads (both precisions) on
    this GPU and write them as the shipped table."""
    import workloads as W
    from . import mgar as M
    arch = device_arch()
    table = _load(out)
    for name in names:
        prob = W.CONFIGS.get(name) or next(p for p in W.CONFIGS.values() if p.name == name)
        for prec in (M.PREC_FP64, M.PREC_MIXED):
            params = M.params_for(prob, precision=prec)
            h = M.Handle(params)
            best = h.mgar_autotune(reps)
            table[cache_key(params, arch)] = {"shapes": read_shapes(h, params.levels), "best_us": best}
            h.close()
            print(f"[tune] {prob.name} precision {prec}: finest apply+dot {best[0][0][1]:.2f} us",
                  flush=True)
    _store(out, table)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="Write the shipped launch-shape table.")
    ap.add_argument("--ship", nargs="+", required=True, help="workload keys or names, e.g. c3 3d-64^3")
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--out", default=SHIPPED)
    a = ap.parse_args()
    ship(a.ship, a.reps, a.out)
