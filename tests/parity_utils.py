"""Helpers for GPU-vs-oracle parity tests (bit-exact comparison)."""
from __future__ import annotations

import sys

import numpy as np

from oracle import ranc_oracle as O


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(net, inputs, T, path, S=None, chunks=None, device_inputs=False):
    """Run the HIP library; returns the RancNet (results read per sample)."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet

    S = S if S is not None else (inputs.shape[0] if inputs is not None else 1)
    chunks = chunks or [T]
    g = RancNet(net, S, max(chunks), path=path)
    t0 = 0
    for tc in chunks:
        x = None
        if inputs is not None:
            x = np.ascontiguousarray(inputs[:, t0:t0 + tc])
            if device_inputs:
                x = torch.from_numpy(x.view(np.int32)).cuda()
        g.run(x, tc)
        t0 += tc
    torch.cuda.synchronize()
    return g


def oracle_results(net, inputs, T, samples):
    return {r["sample"]: r for r in O.simulate(net, inputs, T, samples=samples)}


def assert_sample_equal(g, ref, s, T, what=""):
    ev = g.spikes(s, max(0, T - g.RT), T)
    want = ref["events"]
    want = want[want[:, 0] >= max(0, T - g.RT)]
    assert ev.shape == want.shape and np.array_equal(ev, want), \
        f"{what} sample {s}: output spikes differ ({len(ev)} vs {len(want)}); first rows gpu={ev[:3].tolist()} ref={want[:3].tolist()}"
    v = g.potentials(s)
    if not np.array_equal(v, ref["v"]):
        bad = np.argwhere(v != ref["v"])
        c, n = bad[0]
        raise AssertionError(f"{what} sample {s}: {len(bad)} potentials differ, first (core {c}, neuron {n}): "
                             f"gpu {v[c, n]} ref {ref['v'][c, n]}")
    cnt = g.counters(s)
    for k in ("emitted", "routed", "delivered", "out", "events"):
        assert cnt[k] == ref["counters"][k], f"{what} sample {s}: counter {k} gpu {cnt[k]} ref {ref['counters'][k]}"


def assert_parity(net, inputs, T, path, samples=None, S=None, chunks=None, device_inputs=False, what=""):
    S = S if S is not None else inputs.shape[0]
    samples = list(range(S)) if samples is None else list(samples)
    log(f"[parity] {what or net.name} path={path} S={S} T={T} checking {len(samples)} samples")
    g = gpu_run(net, inputs, T, path, S=S, chunks=chunks, device_inputs=device_inputs)
    assert g.tick == T
    ref = oracle_results(net, inputs, T, samples)
    for s in samples:
        assert_sample_equal(g, ref[s], s, T, what=f"{what or net.name}/{g.path}")
    return g
