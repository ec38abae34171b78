"""Cache of the tile shapes isdc_autotune picks, as JSON.

The choice depends on the device and on the plan's shape only (dimension,
grid, V-cycle precision, smoother and smoothing steps), so it is stored under
a key of those and reused by later plans instead of timing again.  The file
is $ISDC_TUNE_CACHE, else ~/.cache/isdc/tile_shapes.json.
"""
from __future__ import annotations

import json
import os

VERSION = 3  # 2: the shape of a z-marched 3D level selects its column depth; 3: shape 1 there fits one round


def path() -> str:
    return os.environ.get("ISDC_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "isdc",
                                                              "tile_shapes.json")


def key(plan) -> str:
    import torch
    props = torch.cuda.get_device_properties(plan.device)
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    p = plan.params
    # VERSION changes whenever what a shape number selects changes
    return (f"v{VERSION}:{arch}:d{plan.dim}:n{plan.n}:stencil{plan.stencil}:prec{p.precision}"
            f":smoother{p.smoother}:nu{p.nu_pre}{p.nu_post}")


def _load() -> dict:
    try:
        with open(path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(k: str):
    v = _load().get(k)
    return list(v) if isinstance(v, list) else None


def store(k: str, shapes: list) -> None:
    data = _load()
    data[k] = list(shapes)
    os.makedirs(os.path.dirname(path()), exist_ok=True)
    tmp = path() + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path())
