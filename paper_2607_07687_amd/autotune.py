"""Cache of sweep tile choices found by gmg_autotune, keyed by device
architecture, level shape and precision, stored as JSON.

    tiles = autotune.tune(h, x, sigma, dtype="f32", storage="f32",
                          cache="tiles.json")

Levels whose key is already cached get the stored choice (gmg_set_tiles,
gmg_set_pair_sweeps);
otherwise the library times the candidates (gmg_autotune) and the cache is
updated.  The solver's results do not depend on the tile choice.
"""
from __future__ import annotations

import json
import os

from . import gmg as G


def _arch():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _key(arch, n, dtype, storage):
    return f"{arch}|{n[0]}x{n[1]}x{n[2]}|{dtype}|{storage}"


def tune(h, x, sigma, dtype="f32", storage="f32", cache=None, reps=5):
    arch = _arch()
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    nl = G.gmg_num_levels(h)
    keys = [_key(arch, G.gmg_level_shape(h, l)[0], dtype, storage) for l in range(nl)]
    if all(k in table and "pair_ty" in table[k] for k in keys):
        for l, k in enumerate(keys):
            G.gmg_set_tiles(h, l, table[k]["ty"], table[k]["kchunk"])
            try:
                G.gmg_set_pair_sweeps(h, l, table[k]["pair_kchunk"], table[k]["pair_ty"])
            except G.GMGError:  # this handle's parameters do not allow passes
                G.gmg_set_pair_sweeps(h, l, 0)
        return [dict(level=l, **table[k], cached=True) for l, k in enumerate(keys)]
    res = G.gmg_autotune(h, x, sigma, reps)
    for r, k in zip(res, keys):
        table[k] = dict(ty=r["ty"], kchunk=r["kchunk"], us=r["us"],
                        pair_kchunk=r["pair_kchunk"], pair_ty=r["pair_ty"], us_pair=r["us_pair"])
    if cache:
        d = os.path.dirname(cache)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return res
