"""Tile-configuration autotuner.

The library offers BF_TILE_CONFIGS tile configurations (output rows per lane
in the column pass, output columns per lane in the row pass + combine). This
module times each one on the caller's own workload with HIP events, keeps the
fastest per key, and persists the choice as JSON so later processes reuse it.

Key: (GPU architecture, forward or batched, stack type, radius bucket, plane
bucket, size bucket). Buckets are powers of two, so one measurement serves
nearby shapes. Cache file: $BFGC_AUTOTUNE_CACHE, else
~/.cache/bfgc/autotune.json. A missing or unreadable cache is rebuilt.
"""
from __future__ import annotations

import json
import math
import os
import threading

__all__ = ["cache_path", "forward_key", "batched_key", "lookup", "tune_forward", "tune_batched", "clear_memory"]

_lock = threading.Lock()
_mem: dict | None = None


def cache_path() -> str:
    p = os.environ.get("BFGC_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "bfgc", "autotune.json")


def _bucket(x: float) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1.0, float(x))))))


def _arch() -> str:
    import torch
    try:
        return str(torch.cuda.get_device_properties(0).gcnArchName).split(":")[0]
    except Exception:
        return "unknown"


def forward_key(height, width, sigma_s, degree, stack_dtype, arch=None) -> str:
    from . import radius
    return "|".join([arch or _arch(), "fwd", str(stack_dtype), f"W{_bucket(radius(sigma_s))}",
                     f"P{_bucket(degree + 2)}", f"px{_bucket(height * width)}"])


def batched_key(shapes, sigmas_s, degrees, stack_dtype, arch=None) -> str:
    from . import radius
    px = sum(h * w for h, w in shapes)
    wmean = sum(radius(s) * h * w for s, (h, w) in zip(sigmas_s, shapes)) / max(1, px)
    pmean = sum((d + 2) * h * w for d, (h, w) in zip(degrees, shapes)) / max(1, px)
    return "|".join([arch or _arch(), "batched", str(stack_dtype), f"W{_bucket(wmean)}", f"P{_bucket(pmean)}",
                     f"px{_bucket(px)}", f"n{_bucket(len(shapes))}"])


def _load() -> dict:
    global _mem
    if _mem is None:
        try:
            with open(cache_path()) as fh:
                data = json.load(fh)
            _mem = data if isinstance(data, dict) else {}
        except (OSError, ValueError):
            _mem = {}
    return _mem


def _store(key: str, cfg: int, times_ms: list) -> None:
    with _lock:
        data = _load()
        data[key] = {"config": int(cfg), "times_ms": [None if t is None else round(t, 5) for t in times_ms]}
        path = cache_path()
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + f".tmp{os.getpid()}"
            with open(tmp, "w") as fh:
                json.dump(data, fh, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass          # the in-memory choice still holds for this process


def lookup(key: str):
    """Cached configuration index for `key`, or None."""
    with _lock:
        ent = _load().get(key)
    if isinstance(ent, dict) and isinstance(ent.get("config"), int):
        return ent["config"]
    return None


def clear_memory() -> None:
    """Forget the in-memory copy (the next lookup rereads the file)."""
    global _mem
    with _lock:
        _mem = None


def _time(fn, repeats: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(repeats):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / repeats


def tune_forward(f, sigma_s, sigma_r, degree, stack_dtype="f32", repeats=3, out=None, workspace=None):
    """Times every tile configuration bf_gc_forward accepts for (f, sigma_s,
    sigma_r, degree, stack_dtype), caches the fastest and returns (config,
    times_ms), times_ms[c] being None for a configuration that does not
    apply."""
    import torch
    from . import TILE_CONFIGS, gc_filter, tile_configs_for, workspace_bytes
    out = torch.empty_like(f) if out is None else out
    if workspace is None:
        workspace = torch.empty(max(256, workspace_bytes(f.shape[0], f.shape[1], sigma_s, degree, stack_dtype)),
                                dtype=torch.uint8, device=f.device)
    times = [None] * len(TILE_CONFIGS)
    for c in tile_configs_for(stack_dtype, sigma_s):
        times[c] = _time(lambda: gc_filter(f, sigma_s, sigma_r, degree, stack_dtype=stack_dtype, out=out,
                                           workspace=workspace, tile_config=c), repeats)
    best = min((c for c in range(len(times)) if times[c] is not None), key=times.__getitem__)
    _store(forward_key(f.shape[0], f.shape[1], sigma_s, degree, stack_dtype), best, times)
    return best, times


def tune_batched(images, sigmas_s, sigmas_r, degrees, stack_dtype="f32", repeats=2, graph=True,
                 allow_ill_conditioned=False, workspace=None):
    """Times every tile configuration of bf_gc_batched on this batch, caches
    the fastest and returns (config, times_ms)."""
    from . import TILE_CONFIGS, TILE_FUSED, FUSED_MAX_RADIUS, _dtype_code, gc_filter_batched, radius
    outs = None
    times = [None] * len(TILE_CONFIGS)
    cfgs = list(range(TILE_FUSED))
    if _dtype_code(stack_dtype) != 0 and all(radius(s) <= FUSED_MAX_RADIUS for s in sigmas_s):
        cfgs.append(TILE_FUSED)
    for c in cfgs:
        def run():
            nonlocal outs
            outs, _ = gc_filter_batched(images, sigmas_s, sigmas_r, degrees, stack_dtype=stack_dtype, graph=graph,
                                        tile_config=c, allow_ill_conditioned=allow_ill_conditioned, outs=outs,
                                        workspace=workspace)
        times[c] = _time(run, repeats)
    best = min(cfgs, key=times.__getitem__)
    _store(batched_key([tuple(x.shape) for x in images], sigmas_s, degrees, stack_dtype), best, times)
    return best, times
