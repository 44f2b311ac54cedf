"""Cached launch shapes from the native autotuner (ranc_autotune).

The tuned shape of a network depends on its shape (cores, axons, neurons,
axon types, weight precision, max delay), the number of samples and the path,
and on the GPU. ``tuned`` looks the key up in a JSON cache file and applies
the stored shape; on a miss it runs the autotuner on the caller's inputs and
stores the result.
"""
from __future__ import annotations

import json
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ranc_mi355x", "launch_shapes.json")


def shape_key(net, num_samples: int, path: str, device_name: str) -> str:
    return (f"{device_name}|{path}|C{net.num_cores}A{net.num_axons}N{net.num_neurons}G{net.num_types}"
            f"b{net.weight_bits}D{net.max_delay}S{num_samples}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned(g, inputs, num_ticks: int, cache_path: str | None = DEFAULT_CACHE) -> dict:
    """Give RancNet ``g`` its tuned launch shape (from the cache, or by running
    the autotuner on ``inputs``, which leaves ``g`` at tick 0). Returns the
    shape and whether it came from the cache."""
    import torch

    key = shape_key(g.net, g.S, g.path, torch.cuda.get_device_name(g.stream.device))
    cache = _load(cache_path) if cache_path else {}
    if key in cache:
        shape = g.launch_shape(cache[key])
        return dict(shape, cached=True)
    shape = g.autotune(inputs, num_ticks)
    if cache_path:
        cache = _load(cache_path)
        cache[key] = {k: shape[k] for k in ("samples_per_wg", "route_samples_per_block", "route_split",
                                            "route_stage", "route_lanes_per_word")}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return dict(shape, cached=False)
