"""Autotuner for the launch shape of batched (and single-table) builds.

The timing runs on the device inside the library (``alias_tune_build``: one
untimed build per candidate, then timed builds between two HIP events); this
module picks the candidates and keeps a JSON cache of the winners, keyed by
the device architecture and the shape of the batch (number of tables, total
items and the size spread, in powers of two), so that a workload is tuned
once and later builds reuse its options.

Cache file: ``$ALIAS_TUNE_CACHE`` or ``~/.cache/alias_mi355x/tune.json``.
"""
import ctypes as C
import json
import math
import os

from . import AliasError, ALIAS_EINVAL, BuildOpts, _check_dev, _opts, _ptr, _stream, lib

CHUNKS = (256, 512, 1024, 2048)
WAVES = (1, 2, 4)

_registered = False


def _register():
    global _registered
    if _registered:
        return
    L = lib()
    vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
    L.alias_tune_workspace_bytes.argtypes = [u32, u64, C.POINTER(BuildOpts), vp, u32]
    L.alias_tune_workspace_bytes.restype = C.c_size_t
    L.alias_tune_build.argtypes = [vp, vp, u32, u64, vp, vp, C.c_size_t, vp,
                                   C.POINTER(BuildOpts), vp, u32, vp, u32, u32, vp,
                                   C.POINTER(BuildOpts), vp]
    L.alias_tune_build.restype = C.c_int
    _registered = True


def cache_path():
    return os.environ.get("ALIAS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "alias_mi355x",
                                       "tune.json"))


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def workload_key(arch, T, total, sizes_min, sizes_max, split="binary"):
    """Cache key: architecture, split method and the batch shape in powers of two."""
    def lg(x):
        return int(math.floor(math.log2(max(int(x), 1))))
    return f"{arch}|{split}|T2^{lg(T)}|N2^{lg(total)}|n2^{lg(sizes_min)}-2^{lg(sizes_max)}"


def tune(w, offsets, sizes_min, sizes_max, split="binary", model=None, model_stride=0,
         chunks=CHUNKS, waves=WAVES, reps=3, cache=True, stream=None):
    """Time every valid (chunk, pack_waves) pair on this batch and return
    dict(chunk=, pack_waves=, ms=, times={...}, key=, cached=).  w: float64
    device tensor; offsets: int64 device tensor of T+1 entries; sizes_min /
    sizes_max: the smallest and largest table (host ints, for the cache key)."""
    import torch

    _register()
    _check_dev(w, torch.float64, "w")
    _check_dev(offsets, torch.int64, "offsets")
    T, total = offsets.numel() - 1, w.numel()
    arch = torch.cuda.get_device_properties(w.device).gcnArchName.split(":")[0]
    key = workload_key(arch, T, total, sizes_min, sizes_max, split)
    path = cache_path()
    if cache:
        hit = _load_cache(path).get(key)
        if hit:
            return dict(hit, key=key, cached=True)
    base = _opts(None, split, model, model_stride)
    if model is not None and model_stride:
        base.split_model_bytes = int(model_stride)
    ch = (C.c_uint32 * len(chunks))(*chunks)
    wv = (C.c_uint32 * len(waves))(*waves)
    L = lib()
    wsb = L.alias_tune_workspace_bytes(T, total, C.byref(base), ch, len(chunks))
    if wsb == 0:
        raise AliasError(ALIAS_EINVAL, "alias_tune_workspace_bytes")
    ws = torch.empty(wsb, dtype=torch.uint8, device=w.device)
    rows = torch.empty((total, 4), dtype=torch.int32, device=w.device)
    status = torch.zeros(T, dtype=torch.int32, device=w.device)
    times = (C.c_float * (len(chunks) * len(waves)))()
    best = BuildOpts()
    st = L.alias_tune_build(_ptr(w), _ptr(offsets), T, total, _ptr(rows), _ptr(ws), wsb,
                            _ptr(status), C.byref(base), ch, len(chunks), wv, len(waves),
                            int(reps), times, C.byref(best), _stream(stream))
    if st:
        raise AliasError(st, "alias_tune_build")
    table = {f"{c}x{v}": round(float(times[i * len(waves) + j]), 4)
             for i, c in enumerate(chunks) for j, v in enumerate(waves)
             if times[i * len(waves) + j] >= 0}
    res = dict(chunk=int(best.chunk_items), pack_waves=int(best.pack_waves),
               ms=min(table.values()), times=table)
    if cache:
        data = _load_cache(path)
        data[key] = res
        _save_cache(path, data)
    return dict(res, key=key, cached=False)
