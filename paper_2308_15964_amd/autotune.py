"""Persisted tile tables for the batched launch (spx_autotune_batched / spx_set_tile_table).

The library's autotuner times every candidate tile size on synthetic SPD matrices of each
probe size and keeps the fastest; this module stores the resulting table as JSON, keyed
by device name, update precision and right-hand-side count, so a later process restores
it instead of tuning again.
"""
import json
import os

DEFAULT_SIZES = [32, 48, 64, 96, 128, 192, 256, 320, 384, 448, 512]


def _device_name(ctx):
    return ctx.torch.cuda.get_device_name(ctx.device)


def _key(ctx, prec, nrhs):
    return f"{_device_name(ctx)}|prec={prec}|nrhs={nrhs}"


def load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(path, tables):
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(tables, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def ensure(ctx, prec, path, sizes=DEFAULT_SIZES, nrhs=4, copies=256, reps=2, retune=False):
    """Sets the context's tile table for `prec` from `path`, tuning (and saving) first if
    the file holds no table for this device, precision and right-hand-side count.
    Returns the entry: {"table": [[n_max, tile], ...], "ms": {...}}."""
    tables = load(path)
    key = _key(ctx, prec, nrhs)
    entry = tables.get(key)
    if retune or entry is None or [int(s) for s, _ in entry["table"]] != [int(s) for s in sizes]:
        r = ctx.autotune_batched(sizes, prec=prec, nrhs=nrhs, copies=copies, reps=reps)
        entry = {"table": [[int(a), int(b)] for a, b in r["table"]], "ms": {str(k): {str(b): t for b, t in v.items()} for k, v in r["ms"].items()},
                 "copies": copies, "reps": reps}
        tables[key] = entry
        save(path, tables)
    else:
        ctx.set_tile_table(prec, [(int(a), int(b)) for a, b in entry["table"]])
    return entry
