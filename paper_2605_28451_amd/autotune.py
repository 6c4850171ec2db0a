"""Autotuner front end with a JSON cache.

The timing loop runs in the library (fft_autotune: every candidate of the
plan's tuning space -- engine, persistent-grid size, rows per thread and
radix plan --
timed with HIP events on the caller's buffers); this module keys the winners by device
architecture, size, precision, operation and batch bucket and stores them in
``$BFP_AUTOTUNE_CACHE`` (default ``~/.cache/bfpfft/autotune.json``), so later
plans of the same shape start from the tuned configuration.
"""
import json
import os

import torch

OPS = {"forward": 0, "inverse": 1, "compress": 2}


def cache_path() -> str:
    return os.environ.get("BFP_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "bfpfft", "autotune.json"))


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _key(plan, op: str) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    if hasattr(plan, "batch"):
        bucket = 1 << max(0, int(plan.batch - 1).bit_length())
        return f"{arch}|n={plan.n}|prec={plan.prec}|op={op}|rows<={bucket}"
    return f"{arch}|uneven|prec={plan.prec}|count={plan.count}|total={plan.total}"


def apply_cached(plan, op: str = "forward") -> bool:
    """Apply a cached configuration if one exists; returns whether it did."""
    entry = _load().get(_key(plan, op))
    if entry is None:
        return False
    _apply(plan, entry)
    return True


def _apply(plan, entry):
    if hasattr(plan, "set_tuning_ex"):
        plan.set_tuning_ex(entry["engine"], entry["blocks_per_cu"], entry.get("rows_per_thread", 1),
                           entry.get("radix_plan", 0))
    else:
        plan.set_tuning(entry["engine"], entry["blocks_per_cu"])


def tune(plan, op: str, x, out, filt=None, reps: int = 20, force: bool = False) -> dict:
    """Tune `plan` for `op` on (x, out) unless cached; returns the entry."""
    d = _load()
    k = _key(plan, op)
    if not force and k in d:
        _apply(plan, d[k])
        return d[k]
    ms = plan.autotune_on(OPS.get(op, 0), x, out, filt, reps)
    if hasattr(plan, "get_tuning_ex"):
        e, b, rr, pl = plan.get_tuning_ex()
    else:
        (e, b), rr, pl = plan.get_tuning(), 1, 0
    d[k] = {"engine": e, "blocks_per_cu": b, "rows_per_thread": rr, "radix_plan": pl, "ms": ms}
    _save(d)
    return d[k]
