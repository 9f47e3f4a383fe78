"""Persistent cache of launch shapes found by rpa_autotune.

The key is the device architecture and CU count, the grid, the number of
occupied orbitals, the precision, whether projectors are present, N_l, the
HBM budget and a hash of the kernel library, so a rebuilt library or another
GPU tunes again.  The cache is a JSON file (default
$XDG_CACHE_HOME/paper_2609_16408_amd/tune.json).
"""
from __future__ import annotations

import hashlib
import json
import os

from . import LIB_PATH, Handle

_lib_hash = None


def _library_hash() -> str:
    global _lib_hash
    if _lib_hash is None:
        with open(LIB_PATH, "rb") as f:
            _lib_hash = hashlib.sha256(f.read()).hexdigest()[:16]
    return _lib_hash


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_2609_16408_amd", "tune.json")


def cache_key(n, n_occ, precision, with_proj, n_lanczos, hbm_budget) -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", p.name)
    return "|".join(str(v) for v in (arch, p.multi_processor_count, tuple(int(x) for x in n),
                                     int(n_occ), precision, bool(with_proj), int(n_lanczos),
                                     int(hbm_budget), _library_hash()))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned_handle(n, L, v_loc, psi, eps, n_lanczos=8, cache_path=None, retune=False, **kw):
    """A Handle whose tile rows, workgroups per CU and batch come from the
    cache, or from rpa_autotune on a miss (then stored).  Returns
    (handle, shape dict, cache hit flag)."""
    path = cache_path or default_cache_path()
    key = cache_key(n, len(eps), kw.get("precision", "fp64"), kw.get("proj") is not None,
                    n_lanczos, kw.get("hbm_budget", 0))
    cache = _load(path)
    if not retune and key in cache:
        shape = cache[key]
        kw.update(tile_y=shape["tile_y"], slots_per_cu=shape["slots_per_cu"], batch=shape["batch"])
        return Handle(n, L, v_loc, psi, eps, **kw), shape, True
    h = Handle(n, L, v_loc, psi, eps, **kw)
    shape = h.autotune(n_lanczos=n_lanczos)
    cache = _load(path)            # merge with entries written meanwhile
    cache[key] = shape
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return h, shape, False


def tuned_handle_for_cell(cell, **kw):
    kw.setdefault("proj", cell.proj)
    return tuned_handle(cell.n, cell.L, cell.v_loc, cell.psi, cell.eps, **kw)
