#!/usr/bin/env python3
"""Throughput of the RANC tick engine on one MI355X.

Workload: the 512-core layered feed-forward net shaped like the paper's
MNIST-512c application (4 layers x 128 cores of 256 axons x 256 neurons,
crossbar density 0.2, 4 axon types, signed 9-bit weights, delays 1-4,
rate-coded 784-pixel input), 1024 independent samples. One step advances all
1024 samples by 32 ticks (every tick: scheduler slot + input, integration,
leak/threshold/reset, routing into the delayed-delivery scheduler), on the
batched int8-MFMA path, as one replay of the captured 32-tick HIP graph.
Inputs are synthetic and resident in HBM before timing starts. The same steps
are also timed on the plain path.

Output: one JSON line. ``value`` is synaptic events per second (events =
(spiking axon, connected neuron) pairs, counted by the GPU itself over the
timed steps); core-ticks per second is reported beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "synaptic events/sec & core-ticks/sec at 512 cores; batched-MFMA vs plain, bit-exact"
HBM_PEAK_GBS = 8000.0
INT8_MFMA_PEAK_TOPS = 5000.0   # MI355X dense int8 MFMA
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_integrate_mfma_mnist512_s1024.txt")
TRAFFIC_FILE_MESH = os.path.join(ROOT, "profiles", "traffic_integrate_mesh16384_s64.txt")
# Sources whose text decides each measured kernel's device code: a traffic
# summary under profiles/ is used only while these hash to the value it
# records.
_CSRC = "paper_2404_16208_amd/csrc/"
KERNEL_SOURCES_MFMA = [_CSRC + f for f in ("kern_mfma.hip", "kern_mfma_unit.h", "kern_mfma_cb.hip", "kern_common.h",
                                              "kern_bits.h", "ranc_internal.h")]
KERNEL_SOURCES_MESH = KERNEL_SOURCES_MFMA + [_CSRC + "kern_sparse.hip"]


def kernel_source_hash(files=KERNEL_SOURCES_MFMA) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def integrate_algorithmic_bytes(net, S: int, path: str) -> dict:
    """Bytes one integration launch must move at minimum (one tick, all samples).

    Per (sample, core): potentials read + written (8 N), the tick's axon spike
    bits read (A/8) and the spike bits written (N/8). Per (sample, input core):
    external input bits (A/8). Per (sample, output word): 4 bytes of raster.
    Per core, once per launch: the network's parameters in their compact form
    (crossbar bits A*N/8, per-type weights 4GN, axon types as type masks
    GA/8, leak, threshold and reset 12 N), whatever form the path keeps them
    in. The MFMA path's kernel reads them as crossbar column words (A*N/8),
    per-type plane bytes (8 per neuron and weight plane) and axon-type bytes
    (A) per core, and builds its int8 B tiles from those in registers; that
    form's size is reported as ``b_source``.
    """
    C, A, N, G = net.num_cores, net.num_axons, net.num_neurons, net.num_types
    Cin = len(net.input_cores)
    out_words = int(((net.dest_kind == 2).reshape(C, N // 32, 32).any(axis=2)).sum())
    per_unit = 8 * N + A // 8 + N // 8
    state = S * C * per_unit + S * Cin * (A // 8) + S * out_words * 4
    params = C * (A * N // 8 + 4 * G * N + G * A // 8 + 12 * N)
    pl = 2 if net.weight_bits > 8 else 1
    b_source = C * (A * N // 8 + 8 * pl * N + A) if path == "mfma" else 0
    return dict(per_unit=per_unit, units=S * C, total=state + params, state=state, params=params,
                b_source=b_source)


def resident_algorithmic_bytes(net, S: int, T: int) -> dict:
    """Bytes one state-resident launch (T ticks, all samples) must move at
    minimum: the potentials read and written once per call (8 N per (sample,
    core)); per tick the axon spike bits read and the spike bits written
    (A/8 + N/8 per (sample, core)), the external input bits and the raster
    words; the network's compact parameters once (as for the per-tick
    launch)."""
    C, A, N = net.num_cores, net.num_axons, net.num_neurons
    tick = integrate_algorithmic_bytes(net, S, "mfma")
    per_tick_state = tick["state"] - S * C * 8 * N
    total = S * C * 8 * N + T * per_tick_state + tick["params"]
    return dict(total=total, potentials=S * C * 8 * N, per_tick=per_tick_state, params=tick["params"])


def mfma_ops_per_launch(net, S: int) -> int:
    """int8 multiply-adds the MFMA path executes per launch, counted as 2 ops
    each: every 64-sample tile of every core multiplies [64 x A] by [A x N]
    once per weight plane (samples padded to a multiple of 64)."""
    planes = 2 if net.weight_bits > 8 else 1
    S64 = (S + 63) // 64 * 64
    return 2 * planes * S64 * net.num_cores * net.num_axons * net.num_neurons


def read_traffic(src_hash: str, path: str = TRAFFIC_FILE, key: str = "hbm_bytes_per_launch"):
    """HBM traffic per integration launch from a committed rocprofv3 PMC
    summary, or None if it is absent or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != src_hash:
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def time_steps(g, xd, T, warmup, steps, torch, graph=False, resident=False):
    """Time `steps` calls of T ticks; the library's HIP events on the launch
    stream time every kernel launch (or every graph or state-resident launch)
    inside the same timed region."""
    for _ in range(warmup):
        g.run(xd, T, graph=graph, resident=resident)
    torch.cuda.synchronize()
    before = g.total_counters()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g.profile(True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        g.run(xd, T, graph=graph, resident=resident)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = g.profile_read()
    g.profile(False)
    after = g.total_counters()
    delta = {k: after[k] - before[k] for k in after}
    return ms, delta, prof


def kernel_profile(g, xd, T, steps, torch):
    g.profile(True)
    for _ in range(steps):
        g.run(xd, T)
    torch.cuda.synchronize()
    p = g.profile_read()
    g.profile(False)
    return p


def cpu_baseline(net, x, T, n_samples, gpu_net, torch):
    """The serial oracle on a bounded sample (test-infrastructure code), timed
    on the host; the same samples are compared bit for bit with a fresh GPU run."""
    from oracle import ranc_oracle as O

    threads = max(1, min(16, os.cpu_count() or 1, n_samples))
    O.build(force=False)
    t0 = time.perf_counter()
    res = O.simulate(net, x, T, samples=range(n_samples), threads=threads)
    dt = time.perf_counter() - t0
    events = sum(r["counters"]["events"] for r in res)
    # the same oracle on one thread (the paper's serial baseline), two samples
    n1 = min(2, n_samples)
    t0 = time.perf_counter()
    res1 = O.simulate(net, x, T, samples=range(n1), threads=1)
    dt1 = time.perf_counter() - t0
    events1 = sum(r["counters"]["events"] for r in res1)
    gpu_net.reset()
    gpu_net.run(torch.from_numpy(x.view("int32")).cuda(), T)
    torch.cuda.synchronize()
    import numpy as np
    exact = True
    for r in res:
        s = r["sample"]
        exact &= bool(np.array_equal(gpu_net.spikes(s), r["events"]))
        exact &= bool(np.array_equal(gpu_net.potentials(s), r["v"]))
        c = gpu_net.counters(s)
        exact &= all(c[k] == r["counters"][k] for k in c)
    return {"value": events / dt, "unit": "synaptic events/s", "cores": threads, "kind": "oracle",
            "sample": f"samples 0..{n_samples - 1} of the 1024-sample batch x {T} ticks "
                      f"(serial C oracle, one sample per thread), {dt:.2f} s wall",
            "core_ticks_per_s": n_samples * net.num_cores * T / dt,
            "single_thread": {"value": events1 / dt1, "unit": "synaptic events/s", "cores": 1,
                              "sample": f"samples 0..{n1 - 1} x {T} ticks, {dt1:.2f} s"},
            "gpu_bit_exact_on_sample": exact}


def sparse_mesh_algorithmic_bytes(net, S: int, delivered: float, ext_bits: float) -> dict:
    """Bytes one tick of the sample-tiled paths must move on the large sparse
    mesh: potentials read + written (8 N per (sample, core)), the tick's spike
    bits out (N/8) and the history bits gathered (A/8 per (sample, core)), the
    external input bits, plus per core the network's parameters in compact
    form (crossbar A*N/8, G weights per neuron, type masks, neuron parameters)
    for both paths."""
    C, A, N, G = net.num_cores, net.num_axons, net.num_neurons, net.num_types
    state = S * C * (8 * N + N // 8 + A // 8) + ext_bits / 8
    compact = state + C * (A * N // 8 + 4 * G * N + G * A // 8 + 12 * N)
    return {"mfma": compact, "sparse": compact}


def bench_sparse_mesh(args, torch, np):
    """Large sparse mesh (16384 cores of 256x256 on a 128x128 mesh, 64
    samples): the event-driven path against dense MFMA integration, each as
    graph replays of a 10-tick chunk with the inputs resident in HBM. Both are
    held to the same algorithmic bytes (the network's compact parameters,
    which both paths read in a compact form of their own)."""
    from paper_2404_16208_amd import workloads as W
    from paper_2404_16208_amd.ranc import RancNet

    S, T = 64, 10
    # recurrent activity builds up over the first ~100 ticks (delays up to 15);
    # the timed steps start after SETTLE_TICKS untimed ticks
    SETTLE_TICKS = 150
    warm = max(args.warmup, SETTLE_TICKS // T)
    print("[bench] generating the 16384-core sparse mesh and 64x10 inputs", file=sys.stderr, flush=True)
    net = W.sparse_mesh_net(0)
    x = W.sparse_mesh_inputs(0, net, S, T)
    ext_bits = float(np.unpackbits(x.view(np.uint8)).sum())
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    C, A = net.num_cores, net.num_axons
    out = {"metric": "synaptic events/s and ms per tick, large sparse mesh: event-driven vs dense MFMA",
           "unit": "synaptic events/s", "n_gpus": 1, "data": "synthetic", "dtype": "int32 (sparse), int8 (mfma)",
           "config": {"workload": "16384-core sparse mesh (128x128 cores of 256 axons x 256 neurons, crossbar "
                                  "density 0.05, delays 1-15, input rate 1-5% per sample), 64 samples x 10 ticks "
                                  "per step, timed after the activity has settled", "cores": C, "samples": S,
                      "ticks_per_step": T, "untimed_ticks_before_timing": warm * T},
           "steps": args.steps, "warmup": warm}
    for path in ("sparse", "mfma"):
        print(f"[bench] {path} path", file=sys.stderr, flush=True)
        g = RancNet(net, S, T, path=path)
        ms, delta, prof = time_steps(g, xd, T, warm, args.steps, torch, graph=True)
        ticks = args.steps * T
        per_tick = prof["graph_ms"] / max(1, prof["graph_launches"] * T)
        byts = sparse_mesh_algorithmic_bytes(net, S, delta["delivered"] / ticks, ext_bits)[path]
        traffic = read_traffic(kernel_source_hash(KERNEL_SOURCES_MESH), TRAFFIC_FILE_MESH,
                               f"{path}_hbm_bytes_per_launch")
        out[path] = {"value": delta["events"] / (ms / 1e3), "ms_per_tick": ms / ticks,
                     "core_ticks_per_s": S * C * ticks / (ms / 1e3),
                     "integrate_avg_ms": per_tick,
                     "roofline": {"bound": "hbm", "achieved": byts / (per_tick / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": byts / (per_tick / 1e3) / 1e9 / HBM_PEAK_GBS,
                                  "traffic": (traffic / (per_tick / 1e3) / 1e9) if traffic else None,
                                  "algorithmic_bytes_per_launch": byts},
                     "delivered_axon_rate": delta["delivered"] / (S * C * A * ticks),
                     "input_axon_rate": ext_bits / (S * C * A * T),
                     "spike_rate": delta["emitted"] / (S * C * net.num_neurons * ticks)}
        g.close()
        del g
        torch.cuda.empty_cache()
    out["value"] = out["sparse"]["value"]
    out["ms_per_step"] = out["sparse"]["ms_per_tick"] * T
    out["sparse_speedup_vs_mfma"] = out["mfma"]["ms_per_tick"] / out["sparse"]["ms_per_tick"]
    print(json.dumps(out), flush=True)


def bench_table1(args, torch, np):
    """The shapes of the paper's Table I applications as seeded synthetic
    networks, one instance each, simulated for the table's number of ticks
    (graph replays of 128-tick calls, inputs resident in HBM). The networks
    are stand-ins of the same core counts and core sizes (random crossbars of
    density 0.2, 4 axon types, 9-bit weights, random routing with delays
    1..4, Bernoulli(0.1) input on a quarter of the cores); the TrueNorth
    reference runs without any input or leak, so no neuron ever spikes (the
    engine's fixed cost per tick). Path: --path (default: auto, the plain path
    for one instance)."""
    from paper_2404_16208_amd import workloads as W
    from paper_2404_16208_amd.ranc import RancNet

    RT = 128
    rows = []
    apps = [a.strip() for a in args.apps.split(",")] if args.apps else None
    for name, T, C, A, N in W.TABLE1:
        if apps is not None and name not in apps:
            continue
        print(f"[bench] {name}: {C} cores of {A}x{N}, {T} ticks", file=sys.stderr, flush=True)
        net = W.table1_net(name)
        xi = W.table1_inputs(name, net, 1, RT)
        x = None if xi is None else torch.from_numpy(xi.view(np.int32)).cuda()
        g = RancNet(net, 1, RT, path=args.path)
        full, rem = divmod(T, RT)
        xr = None if x is None or rem == 0 else x[:, :rem].contiguous()

        def run_all():
            for _ in range(full):
                g.run(x, RT, graph=True)
            if rem:
                g.run(xr, rem, graph=True)

        run_all()   # captures both graphs
        g.reset()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run_all()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        c = g.counters(0)
        rows.append({"application": name, "ticks": T, "cores": C, "axons": A, "neurons": N, "path": g.path,
                     "ms": ms, "us_per_tick": 1e3 * ms / T, "core_ticks_per_s": C * T / (ms / 1e3),
                     "spikes_emitted": c["emitted"], "synaptic_events": c["events"]})
        g.close()
        del g
        torch.cuda.empty_cache()
    out = {"metric": "simulated time per run of the paper's Table I application shapes (one instance each)",
           "unit": "ms", "n_gpus": 1, "data": "synthetic", "higher_is_better": False,
           "config": {"workload": "Table I shapes as seeded random networks, 1 sample, the table's tick counts, "
                                  f"graph replays of {RT}-tick calls", "calls_ticks": RT},
           "value": sum(r["ms"] for r in rows), "applications": rows}
    print(json.dumps(out), flush=True)


def class_masks(net, out_neurons, np):
    """Per class, u32 masks over the output-neuron words of a by-sample raster
    (class of an output neuron = its global neuron index mod 10)."""
    from paper_2404_16208_amd import workloads as W
    cls = W.mnist_class_of_output(net)[out_neurons[:, 0], out_neurons[:, 1]]
    nw = (len(out_neurons) + 31) // 32
    m = np.zeros((10, nw * 32), dtype=bool)
    m[cls, np.arange(len(out_neurons))] = True
    return np.packbits(m, axis=1, bitorder="little").view(np.uint32)


def class_votes(words, masks, np):
    """Spikes per class of every sample from a by-sample raster [T][S][NW]."""
    w = words.reshape(-1, words.shape[1], words.shape[2])
    return np.stack([np.bitwise_count(w & masks[c]).sum(axis=(0, 2), dtype=np.int64)
                     for c in range(len(masks))], axis=1)


def bench_stream(args, torch, np):
    """Streaming, as the paper runs its applications: one instance of the
    512-core MNIST-shaped net for 10010 ticks with the inputs in pinned host
    memory, through paper_2404_16208_amd.stream: 128-tick chunks, the next
    chunk's inputs uploaded on a second stream while the current chunk runs
    (graph replay), each chunk's output spikes packed by ranc_copy_raster and
    drained to pinned host memory on a third stream, and the host counting
    spikes per class of the previous chunk meanwhile. Host clock over the
    whole run (upload, simulation, drain, read-out), against the same ticks
    simulated with the inputs already on the GPU and no output drained."""
    from paper_2404_16208_amd import workloads as W
    from paper_2404_16208_amd.ranc import RancNet
    from paper_2404_16208_amd.stream import Streamer

    T, RT = 10010, 128
    print(f"[bench] generating the 512-core net and 1 x {T} inputs", file=sys.stderr, flush=True)
    net = W.mnist_net(0)
    x = W.mnist_inputs(0, 1, T)
    host = torch.from_numpy(x.view(np.int32)).pin_memory()
    g = RancNet(net, 1, RT, path=args.path)
    masks = class_masks(net, g.output_neurons(), np)
    st = Streamer(g, RT)
    votes = np.zeros((1, 10), np.int64)

    def consume(t0, words):
        votes[:] += class_votes(words, masks, np)

    st.run(host, T, consume)   # captures the tick loops (both input buffers and the last chunk)
    g.reset()
    votes[:] = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.run(host, T, consume)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same ticks with the inputs resident on the GPU, no output drained
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    chunks = [(t, min(RT, T - t)) for t in range(0, T, RT)]
    bufs = {}
    for t, k in chunks:
        bufs.setdefault(k, torch.empty((1, k) + tuple(xd.shape[2:]), dtype=torch.int32, device="cuda"))
    sim_runs = []
    for rep in range(2):   # the first pass captures the loops
        g.reset()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for t, k in chunks:
            b = bufs[k]
            b.copy_(xd[:, t:t + k])
            g.run(b, k, graph=True)
        e1.record()
        torch.cuda.synchronize()
        sim_runs.append(e0.elapsed_time(e1) / 1e3)
    sim = sim_runs[-1]
    out = {"metric": "end-to-end time of a streamed 10010-tick single-instance run (512-core MNIST-shaped net)",
           "unit": "s", "value": dt, "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"512-core MNIST-shaped net, 1 instance, {T} ticks in {RT}-tick chunks, inputs "
                                  "in pinned host memory uploaded on a second stream, output rasters drained to "
                                  "pinned host memory on a third stream while the next chunk runs, spikes counted "
                                  "per class on the host", "path": g.path},
           "ticks_per_s": T / dt, "us_per_tick": 1e6 * dt / T,
           "simulation_s": sim, "end_to_end_over_simulation": dt / sim,
           "output_spikes": int(votes.sum()), "class_votes": votes[0].tolist()}
    g.close()
    print(json.dumps(out), flush=True)


def bench_sweep(args, torch, np):
    """Uneven design-space sweep: 64 seeded network variants (cores 16..4096,
    axons and neurons 64..512, 2-8 axon types, 4-9 bit weights) with 64
    samples each, advanced together (graph replay; per tick one launch per
    MFMA shape class and one integration and one routing launch for the
    plain-path networks). Each network is loaded on both the MFMA and the
    plain path, each handle's launch shape is autotuned, and the faster of
    the two (one 64-tick call each, timed) is the per-network choice; the
    batch of those choices and the all-MFMA batch are timed and the faster is
    kept. Compared with: the same networks advanced one after another, and
    the batch with one persistent MFMA launch per tick."""
    from paper_2404_16208_amd import workloads as W
    from paper_2404_16208_amd.ranc import RancNet, run_batch

    from paper_2404_16208_amd import autotune

    S, T = 64, 64
    nets, xs = [], []
    print("[bench] generating 64 sweep variants and their inputs", file=sys.stderr, flush=True)
    for v in range(64):
        net, _ = W.sweep_variant(0, v)
        nets.append(net)
        xs.append(torch.from_numpy(W.bernoulli_inputs(v, net, S, T, 0.1, config_id=4).view(np.int32)).cuda())
    core_ticks = sum(n.num_cores for n in nets) * S * T

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    print("[bench] loading every network on both paths, autotuning each handle, picking the faster path",
          file=sys.stderr, flush=True)
    gm, gp, gs, shapes, picks = [], [], [], [], []
    for net, x in zip(nets, xs):
        m, p = RancNet(net, S, T, path="mfma"), RancNet(net, S, T, path="plain")
        shapes.append((autotune.tuned(m, x, 8, cache_path=None), autotune.tuned(p, x, 8, cache_path=None)))
        tm = timed(lambda: m.run(x, T, graph=True), 2)
        tp = timed(lambda: p.run(x, T, graph=True), 2)
        gm.append(m)
        gp.append(p)
        gs.append(p if tp < tm else m)
        picks.append({"network": net.name, "mfma_ms": tm, "plain_ms": tp})

    def counters():
        tot = 0
        for g in gs:
            tot += sum(g.counters(s)["events"] for s in range(S))
        return tot

    # the per-network choice is made on each network alone; in the batch the
    # plain-path networks add launches of their own, so the all-MFMA batch is
    # timed too and the faster of the two batches is kept
    ms_mixed = timed(lambda: run_batch(gs, xs, T, graph=True), max(2, args.steps // 2))
    ms_all_mfma = timed(lambda: run_batch(gm, xs, T, graph=True), max(2, args.steps // 2))
    if ms_all_mfma <= ms_mixed:
        gs = gm
    ev0 = counters()
    ms_batch = timed(lambda: run_batch(gs, xs, T, graph=True), args.steps)
    ev1 = counters()
    ms_pers = timed(lambda: run_batch(gs, xs, T, graph=True, persistent=True), max(2, args.steps // 2))
    ms_each = timed(lambda: [g.run(x, T, graph=True) for g, x in zip(gs, xs)], max(2, args.steps // 2))
    paths = [g.path for g in gs]
    out = {"metric": "core-ticks/s and synaptic events/s, 64-variant uneven design-space sweep in one batch",
           "unit": "core-ticks/s", "value": core_ticks / (ms_batch / 1e3), "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "64 seeded sweep variants (cores 16..4096, axons/neurons 64..512, 2-8 types, "
                                  "4-9 bit weights, density 0.05-0.3, potential widths 12-32, floors and linear "
                                  "reset on some), 64 samples each, 64 ticks per step, launch shapes autotuned "
                                  "per network and path, the faster of the per-network path choice and all-MFMA",
                      "networks": 64, "mfma_networks": paths.count("mfma"), "plain_networks": paths.count("plain"),
                      "cores_total": sum(n.num_cores for n in nets), "samples": S, "ticks_per_step": T},
           "steps": args.steps, "ms_per_step": ms_batch, "ms_per_tick": ms_batch / T,
           "synaptic_events_per_s": (ev1 - ev0) / ((args.steps + 1) * ms_batch / 1e3),
           "one_by_one_ms_per_step": ms_each, "batch_speedup_vs_one_by_one": ms_each / ms_batch,
           "persistent_queue_ms_per_step": ms_pers,
           "all_mfma_batch_ms_per_step": ms_all_mfma, "per_network_choice_batch_ms_per_step": ms_mixed,
           "one_call_ms_by_network": picks,
           "autotuned_samples_per_wg": sorted({sh[0]["samples_per_wg"] for sh in shapes if sh[0]["samples_per_wg"]})}
    for g in gm + gp:
        g.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--samples", type=int, default=1024)
    ap.add_argument("--ticks", type=int, default=32)
    ap.add_argument("--cpu-samples", type=int, default=16)
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time per-launch calls instead of graph replays")
    ap.add_argument("--skip-resident", action="store_true", help="skip the state-resident tick loop leg")
    ap.add_argument("--skip-links", action="store_true", help="skip the leg with mesh link counting on")
    ap.add_argument("--workload", default="mnist512",
                    choices=["mnist512", "sparse-mesh", "sweep", "table1", "stream"],
                    help="mnist512: the headline line (default); sparse-mesh: the event-driven vs dense "
                         "comparison on the 16384-core mesh; sweep: 64 uneven variants in one batch; table1: "
                         "the paper's Table I application shapes, one instance each; stream: one instance "
                         "streamed for 10010 ticks from host memory, end to end")
    ap.add_argument("--path", default="auto", choices=["auto", "plain", "mfma", "sparse"],
                    help="integration path of the table1 and stream runs (default auto: the plain path for "
                         "one instance, with the lane-split router the fastest on every Table I shape)")
    ap.add_argument("--apps", default="",
                    help="table1 only: comma-separated application names to run (default: all)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this engine runs on one GPU; runs on several GPUs are not supported "
                                   "(samples would shard across GPUs with no communication between them)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    if args.apps:
        from paper_2404_16208_amd.workloads import TABLE1
        unknown = sorted({a.strip() for a in args.apps.split(",")} - {r[0] for r in TABLE1})
        if args.workload != "table1" or unknown:
            ap.error(f"--apps applies to --workload table1 and takes names from {[r[0] for r in TABLE1]}")

    import numpy as np
    import torch

    from paper_2404_16208_amd import workloads as W
    from paper_2404_16208_amd.ranc import RancNet

    torch.cuda.set_device(0)
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20)
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {n} bytes done", file=sys.stderr, flush=True)
        del a, b
    if args.workload == "sparse-mesh":
        bench_sparse_mesh(args, torch, np)
        return
    if args.workload == "sweep":
        bench_sweep(args, torch, np)
        return
    if args.workload == "table1":
        bench_table1(args, torch, np)
        return
    if args.workload == "stream":
        bench_stream(args, torch, np)
        return
    S, T = args.samples, args.ticks
    print(f"[bench] generating 512-core net and {S}x{T} inputs", file=sys.stderr, flush=True)
    net = W.mnist_net(0)
    x = W.mnist_inputs(0, S, T)
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    C = net.num_cores

    print("[bench] mfma path: load + warmup + timed steps", file=sys.stderr, flush=True)
    g = RancNet(net, S, T, path="mfma")
    graph = not args.no_graph
    ms, delta, prof = time_steps(g, xd, T, args.warmup, args.steps, torch, graph=graph)
    secs = ms / 1e3
    events_per_s = delta["events"] / secs
    core_ticks = S * C * T * args.steps
    ib = integrate_algorithmic_bytes(net, S, "mfma")
    if graph:
        # graph launches hold T integration launches and one tick-advance
        # launch each: the per-tick share bounds the kernel's duration from above
        avg_int_ms = prof["graph_ms"] / max(1, prof["graph_launches"] * T)
        launches = prof["graph_launches"] * T
    else:
        avg_int_ms = prof["integrate_ms"] / max(1, prof["integrate_launches"])
        launches = prof["integrate_launches"]
    avg_route_ms = prof["route_ms"] / max(1, prof["route_launches"])
    achieved = ib["total"] / (avg_int_ms / 1e3) / 1e9
    eprof = kernel_profile(g, xd, T, max(2, min(args.steps, 10)), torch)
    eager_int_ms = eprof["integrate_ms"] / max(1, eprof["integrate_launches"])
    src_hash = kernel_source_hash()
    traffic = read_traffic(src_hash)
    out = {
        "metric": METRIC,
        "value": events_per_s,
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": f"512-core layered feed-forward net (4 layers x 128 cores of 256 axons x 256 "
                               f"neurons, MNIST-shaped), {S} samples x {T} ticks per step, batched int8-MFMA",
                   "cores": C, "axons": 256, "neurons": 256, "samples": S, "ticks_per_step": T, "path": "mfma",
                   "parallelism": "single GPU"},
        "core_ticks_per_s": core_ticks / secs,
        "dense_synapse_evals_per_s": core_ticks * net.num_axons * net.num_neurons / secs,
        "synaptic_events_per_step": delta["events"] / args.steps,
        "spikes_emitted_per_step": delta["emitted"] / args.steps,
        "tick_loop": "hip graph replay" if graph else "per-tick launches",
        "kernels": {"integrate_mfma_avg_ms": avg_int_ms, "route_avg_ms": avg_route_ms,
                    "launches_timed": launches,
                    "timing": ("graph launch time / ticks, HIP events on the launch stream over the timed steps"
                               if graph else "HIP events around each launch over the timed steps"),
                    "integrate_mfma_eager_avg_ms": eager_int_ms,
                    "eager_launches_profiled": eprof["integrate_launches"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (traffic / (avg_int_ms / 1e3) / 1e9) if traffic else None,
                     "kernel": "k_integrate_mfma<256,256,two planes>",
                     "algorithmic_bytes_per_launch": ib["total"],
                     "bytes_per_unit": ib["per_unit"], "units_per_launch": ib["units"],
                     "params_bytes_per_launch": ib["params"],
                     "b_source_bytes_per_launch": ib["b_source"],
                     "kernel_source_sha256_16": src_hash},
        "mfma": {"bound": "mfma", "executed_int8_ops_per_launch": mfma_ops_per_launch(net, S),
                 "achieved": mfma_ops_per_launch(net, S) / (avg_int_ms / 1e3) / 1e12,
                 "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOPS",
                 "util": mfma_ops_per_launch(net, S) / (avg_int_ms / 1e3) / 1e12 / INT8_MFMA_PEAK_TOPS,
                 "useful_ops_per_launch": 2 * delta["events"] / max(1, args.steps * T),
                 "note": "executed int8 ops (both weight planes, padded tiles) per average launch duration; "
                         "useful ops = 2 x synaptic events"},
    }
    g.close()
    del g
    torch.cuda.empty_cache()

    if not args.skip_resident:
        # the same steps as state-resident launches (one per call)
        print("[bench] mfma path, state-resident tick loop", file=sys.stderr, flush=True)
        gr = RancNet(net, S, T, path="mfma")
        rms, rdelta, rprof = time_steps(gr, xd, T, args.warmup, args.steps, torch, resident=True)
        r_launch_ms = rprof["resident_ms"] / max(1, rprof["resident_launches"])
        rb = resident_algorithmic_bytes(net, S, T)
        r_ops = T * mfma_ops_per_launch(net, S)
        out["resident"] = {
            "value": rdelta["events"] / (rms / 1e3), "unit": "synaptic events/s", "ms_per_step": rms / args.steps,
            "steps": args.steps, "launch_avg_ms": r_launch_ms, "launches_timed": rprof["resident_launches"],
            "same_events_as_graph": rdelta["events"] == delta["events"],
            "roofline": {"bound": "hbm", "achieved": rb["total"] / (r_launch_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": rb["total"] / (r_launch_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_launch": rb["total"], "kernel": "k_mfma_resident<256,two planes>"},
            "mfma": {"bound": "mfma", "executed_int8_ops_per_launch": r_ops,
                     "achieved": r_ops / (r_launch_ms / 1e3) / 1e12, "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOPS",
                     "util": r_ops / (r_launch_ms / 1e3) / 1e12 / INT8_MFMA_PEAK_TOPS},
            "note": "all ticks of a call in one cooperative launch; potentials of each 64-sample group kept "
                    "in LDS across the call's ticks; one grid barrier per tick"}
        out["resident_speedup_vs_graph"] = out["ms_per_step"] / out["resident"]["ms_per_step"]
        gr.close()
        del gr
        torch.cuda.empty_cache()

    if not args.skip_links:
        # the same steps with packets per mesh link counted on every tick
        print("[bench] mfma path with mesh link counts", file=sys.stderr, flush=True)
        gl = RancNet(net, S, T, path="mfma")
        gl.count_links(True)
        lms, _, lprof = time_steps(gl, xd, T, args.warmup, max(2, args.steps // 4), torch, graph=graph)
        out["link_counts"] = {"ms_per_step": lms / max(2, args.steps // 4),
                              "overhead_vs_headline": (lms / max(2, args.steps // 4)) / out["ms_per_step"] - 1.0,
                              "note": "packets per mesh link (XY route) counted per sample on every tick"}
        gl.close()
        del gl
        torch.cuda.empty_cache()

    # End to end, as a user sees one step from a cold handle: load (parameter
    # upload), one step with the inputs in host memory (staged over PCIe), and
    # every sample's output spikes back in host memory (ranc_copy_raster, by
    # sample, then one copy to pinned host memory); host clock, first call
    # included (no graph capture). The class read-out from those bits on the
    # host is timed beside it.
    n_out_neurons = int((net.dest_kind == 2).sum())
    rbytes = T * S * ((n_out_neurons + 31) // 32) * 4
    rdev = torch.empty(rbytes, dtype=torch.uint8, device="cuda")
    rhost = torch.empty(rbytes, dtype=torch.uint8, pin_memory=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ge = RancNet(net, S, T, path="mfma")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert ge.raster_bytes(T, "sample") == rbytes
    ge.run(x, T)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ge.copy_raster(0, T, rdev, "sample")
    rhost.copy_(rdev)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    words = rhost.numpy().view(np.uint32).reshape(T, S, -1)
    votes = class_votes(words, class_masks(net, ge.output_neurons(), np), np)
    t4 = time.perf_counter()
    n_out = int(votes.sum())
    out["end_to_end"] = {"ms": (t3 - t0) * 1e3, "load_ms": (t1 - t0) * 1e3, "run_ms": (t2 - t1) * 1e3,
                         "read_ms": (t3 - t2) * 1e3, "readout_ms": (t4 - t3) * 1e3, "output_spikes": n_out,
                         "raster_bytes": rbytes,
                         "includes": f"load + host-input staging + {T} ticks + every sample's output-bus spikes "
                                     "in pinned host memory as a by-sample bit raster (host clock; buffer "
                                     "allocation excluded); readout_ms: spikes per class of all samples on the "
                                     "host, not included"}
    ge.close()
    del ge
    torch.cuda.empty_cache()

    if not args.skip_plain:
        print("[bench] plain path", file=sys.stderr, flush=True)
        gp = RancNet(net, S, T, path="plain")
        psteps = max(2, args.steps // 4)
        pms, pdelta, pprof = time_steps(gp, xd, T, 1, psteps, torch)
        pint = pprof["integrate_ms"] / max(1, pprof["integrate_launches"])
        pib = integrate_algorithmic_bytes(net, S, "plain")
        out["plain"] = {"value": pdelta["events"] / (pms / 1e3), "unit": "synaptic events/s",
                        "core_ticks_per_s": S * C * T * psteps / (pms / 1e3), "ms_per_step": pms / psteps,
                        "steps": psteps, "integrate_plain_avg_ms": pint,
                        "route_avg_ms": pprof["route_ms"] / max(1, pprof["route_launches"]),
                        "integrate_hbm_frac": pib["total"] / (pint / 1e3) / 1e9 / HBM_PEAK_GBS}
        out["mfma_speedup_vs_plain"] = out["plain"]["ms_per_step"] and (out["plain"]["ms_per_step"] / out["ms_per_step"])
        gp.close()
        del gp
        torch.cuda.empty_cache()

    if not args.skip_plain:
        # the 100-sample configuration of the same net: plain and MFMA paths
        # (graph replay), and the class read-out of every sample (spikes per
        # class from the by-sample raster, argmax with the lowest class on ties)
        S2 = 100
        print(f"[bench] {S2}-sample configuration, plain and MFMA paths", file=sys.stderr, flush=True)
        x2 = np.ascontiguousarray(x[:S2])
        xd2 = torch.from_numpy(x2.view(np.int32)).cuda()
        c2 = {"samples": S2, "ticks_per_step": T}
        for path in ("plain", "mfma"):
            g2 = RancNet(net, S2, T, path=path)
            ms2, d2, _ = time_steps(g2, xd2, T, 2, max(4, args.steps // 2), torch, graph=True)
            n2 = max(4, args.steps // 2)
            c2[path] = {"ms_per_step": ms2 / n2, "synaptic_events_per_s": d2["events"] / (ms2 / 1e3),
                        "core_ticks_per_s": S2 * C * T * n2 / (ms2 / 1e3)}
            if path == "plain":
                g2.reset()
                g2.run(xd2, T, graph=True)
                rb = torch.empty(g2.raster_bytes(T, "sample"), dtype=torch.uint8, device="cuda")
                g2.copy_raster(0, T, rb, "sample")
                torch.cuda.synchronize()
                words = rb.cpu().numpy().view(np.uint32).reshape(T, S2, -1)
                votes = class_votes(words, class_masks(net, g2.output_neurons(), np), np)
                c2["class_counts"] = np.bincount(np.argmax(votes, axis=1), minlength=10).tolist()
            g2.close()
            del g2
        c2["mfma_speedup_vs_plain"] = c2["plain"]["ms_per_step"] / c2["mfma"]["ms_per_step"]
        out["c2_100_samples"] = c2
        torch.cuda.empty_cache()

    if not args.skip_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        gc = RancNet(net, S, T, path="mfma")
        out["cpu_baseline"] = cpu_baseline(net, x, T, min(args.cpu_samples, S), gc, torch)
        gc.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
