"""Seeded synthetic RANC networks and input spike bitmaps.

This module only *draws* networks and inputs. It holds none of the
simulation's arithmetic (no integration, no leak/threshold/reset, no routing),
so both the serial oracle and the HIP path can take their inputs from it.

Every random draw comes from ``numpy.random.default_rng`` seeded by
``SeedSequence([seed, config_id, purpose, ...])`` so any sub-stream (one
sample's inputs, one network's crossbar) can be regenerated on its own.
Per-sample input streams are keyed by the sample index, so the first samples
of a large batch equal a smaller batch drawn with the same seed.

Network description (the problem statement of RANC, GPU-RANC Sec. II):
cores on a ``grid_w x grid_h`` mesh (core index ``y * grid_w + x``), each with
``A`` axons and ``N`` neurons, a binary crossbar of synaptic connections, an
axon type per axon, ``G`` signed weights per neuron (one per axon type), and
per-neuron leak, threshold, reset potential and destination
(NONE / a (core, axon) at a relative mesh offset with a tick delay / the
output bus).

Bit layouts (little-endian bit order inside 32-bit words):
  crossbar   uint32 [C, A, ceil(N/32)]  bit n%32 of word n//32 = axon a
                                         connects to neuron n
  inputs     uint32 [S, T, C_in, ceil(A/32)]  bit a%32 of word a//32 = an
                                         external spike on axon a of input
                                         core ``input_cores[k]`` at tick t
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Tuple

import numpy as np

DEST_NONE = 0
DEST_CORE = 1
DEST_OUT = 2

# purposes of random streams
_P_XBAR, _P_TYPE, _P_W, _P_PARAM, _P_DEST, _P_PIXMAP, _P_INTENS, _P_TICKU, _P_EXT, _P_MODEL = range(10)


def rng_for(seed: int, *key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed)] + [int(k) for k in key]))


def pack_bits(b: np.ndarray) -> np.ndarray:
    """Pack a boolean array along its last axis into little-endian uint32 words."""
    b = np.asarray(b, dtype=bool)
    n = b.shape[-1]
    nw = (n + 31) // 32
    pad = nw * 32 - n
    if pad:
        b = np.concatenate([b, np.zeros(b.shape[:-1] + (pad,), dtype=bool)], axis=-1)
    by = np.packbits(b, axis=-1, bitorder="little")
    return np.ascontiguousarray(by).view("<u4").reshape(b.shape[:-1] + (nw,))


def unpack_bits(w: np.ndarray, n: int) -> np.ndarray:
    """Inverse of :func:`pack_bits`: uint32 words -> bool array with ``n`` entries."""
    w = np.ascontiguousarray(w, dtype="<u4")
    by = w.view(np.uint8).reshape(w.shape[:-1] + (w.shape[-1] * 4,))
    return np.unpackbits(by, axis=-1, bitorder="little")[..., :n].astype(bool)


@dataclasses.dataclass
class Net:
    num_cores: int
    num_axons: int
    num_neurons: int
    num_types: int
    weight_bits: int
    potential_bits: int
    max_delay: int
    grid_w: int
    grid_h: int
    crossbar: np.ndarray      # uint32 [C, A, ceil(N/32)]
    axon_type: np.ndarray     # uint8  [C, A]
    weight: np.ndarray        # int16  [C, N, G]
    leak: np.ndarray          # int32  [C, N]
    threshold: np.ndarray     # int32  [C, N]
    reset: np.ndarray         # int32  [C, N]
    v_init: np.ndarray        # int32  [C, N]
    dest_kind: np.ndarray     # uint8  [C, N]
    dest_dx: np.ndarray       # int16  [C, N]
    dest_dy: np.ndarray       # int16  [C, N]
    dest_axon: np.ndarray     # uint16 [C, N]
    dest_delay: np.ndarray    # uint8  [C, N]
    input_cores: np.ndarray   # int32  [C_in]
    name: str = ""
    leak_bits: int = 32       # leaks are signed values of this many bits
    reset_bits: int = 32      # reset potentials are signed values of this many bits
    floor: np.ndarray | None = None       # int32 [C, N]: lowest potential kept without firing (None: none)
    reset_mode: np.ndarray | None = None  # uint8 [C, N]: 0 absolute reset, 1 linear reset (None: all absolute)

    @property
    def shape(self) -> Tuple[int, int, int, int]:
        return self.num_cores, self.num_axons, self.num_neurons, self.num_types

    def contiguous(self) -> "Net":
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            if isinstance(v, np.ndarray):
                setattr(self, f.name, np.ascontiguousarray(v))
        return self


def relative_offsets(src_core: np.ndarray, dst_core: np.ndarray, grid_w: int):
    """(dx, dy) on the mesh from absolute source/destination core indices.

    The description stores destinations as relative mesh offsets, the way a
    RANC spike packet carries them (GPU-RANC Sec. III-D); this only converts
    the generator's absolute choice into that form.
    """
    sx, sy = src_core % grid_w, src_core // grid_w
    tx, ty = dst_core % grid_w, dst_core // grid_w
    return (tx - sx).astype(np.int16), (ty - sy).astype(np.int16)


def random_net(seed: int, C: int, A: int, N: int, G: int, weight_bits: int = 9,
               potential_bits: int = 32, max_delay: int = 4, grid_w: int | None = None,
               density: float = 0.2, p_core: float = 0.8, p_out: float = 0.1,
               leak_range=(-8, 8), thr_range=(64, 512), reset_range=(0, 0),
               vinit_range=(0, 0), input_cores=None, config_id: int = 99,
               weight_range=None, floor_range=None, linear_frac: float = 0.0,
               leak_bits: int = 32, reset_bits: int = 32) -> Net:
    """A generic seeded random network (any C, A, N, G), used by tests.

    Each neuron independently gets a CORE destination with probability
    ``p_core`` (uniform random core and axon, delay uniform in
    1..max_delay), OUT with probability ``p_out``, else NONE. Neuron-model
    options (drawn from a stream of their own, so they leave every other
    draw unchanged): ``floor_range`` draws a floor per neuron (clipped to the
    potential range), ``linear_frac`` puts that fraction of the neurons in
    linear-reset mode.
    """
    if grid_w is None:
        grid_w = C
    grid_h = (C + grid_w - 1) // grid_w
    assert grid_w * grid_h == C, "cores must fill the grid"
    NW = (N + 31) // 32
    r = rng_for(seed, config_id, _P_XBAR)
    xbar = np.empty((C, A, NW), dtype=np.uint32)
    for c0 in range(0, C, 512):            # chunked draw: same stream as one call
        c1 = min(C, c0 + 512)
        xbar[c0:c1] = pack_bits(r.random((c1 - c0, A, N)) < density)
    r = rng_for(seed, config_id, _P_TYPE)
    atype = r.integers(0, G, size=(C, A), dtype=np.int64).astype(np.uint8)
    r = rng_for(seed, config_id, _P_W)
    if weight_range is None:
        wmax = (1 << (weight_bits - 1)) - 1
        weight_range = (-wmax, wmax)
    w = r.integers(weight_range[0], weight_range[1] + 1, size=(C, N, G)).astype(np.int16)
    r = rng_for(seed, config_id, _P_PARAM)
    leak = r.integers(leak_range[0], leak_range[1] + 1, size=(C, N)).astype(np.int32)
    thr = r.integers(thr_range[0], thr_range[1] + 1, size=(C, N)).astype(np.int32)
    rst = r.integers(reset_range[0], reset_range[1] + 1, size=(C, N)).astype(np.int32)
    v0 = r.integers(vinit_range[0], vinit_range[1] + 1, size=(C, N)).astype(np.int32)
    r = rng_for(seed, config_id, _P_DEST)
    u = r.random((C, N))
    kind = np.where(u < p_core, DEST_CORE, np.where(u < p_core + p_out, DEST_OUT, DEST_NONE)).astype(np.uint8)
    dcore = r.integers(0, C, size=(C, N))
    daxon = r.integers(0, A, size=(C, N)).astype(np.uint16)
    ddel = r.integers(1, max_delay + 1, size=(C, N)).astype(np.uint8)
    src = np.repeat(np.arange(C)[:, None], N, axis=1)
    dx, dy = relative_offsets(src, dcore, grid_w)
    core_mask = kind == DEST_CORE
    dx = np.where(core_mask, dx, 0).astype(np.int16)
    dy = np.where(core_mask, dy, 0).astype(np.int16)
    daxon = np.where(core_mask, daxon, 0).astype(np.uint16)
    ddel = np.where(core_mask, ddel, 0).astype(np.uint8)
    if input_cores is None:
        input_cores = np.arange(max(1, C // 2))
    floor = mode = None
    if floor_range is not None or linear_frac > 0:
        r = rng_for(seed, config_id, _P_MODEL)
        lo, hi = -(1 << (potential_bits - 1)), (1 << (potential_bits - 1)) - 1
        if floor_range is not None:
            floor = np.clip(r.integers(floor_range[0], floor_range[1] + 1, size=(C, N)), lo, hi).astype(np.int32)
        if linear_frac > 0:
            mode = (r.random((C, N)) < linear_frac).astype(np.uint8)
    return Net(C, A, N, G, weight_bits, potential_bits, max_delay, grid_w, grid_h,
               xbar, atype, w, leak, thr, rst, v0, kind, dx, dy, daxon, ddel,
               np.asarray(input_cores, dtype=np.int32), name=f"random{C}x{A}x{N}g{G}",
               leak_bits=leak_bits, reset_bits=reset_bits, floor=floor, reset_mode=mode).contiguous()


def bernoulli_inputs(seed: int, net: Net, S: int, T: int, rate, config_id: int = 99,
                     first_sample: int = 0) -> np.ndarray:
    """External input bitmaps [S, T, C_in, ceil(A/32)], Bernoulli(rate) per axon per tick.

    ``rate`` is a scalar or a per-sample array. Sample ``s`` is drawn from its
    own stream so batches of different sizes agree on common samples.
    """
    Cin, A = len(net.input_cores), net.num_axons
    rates = np.broadcast_to(np.asarray(rate, dtype=np.float64), (S,))
    out = np.empty((S, T, Cin, (A + 31) // 32), dtype=np.uint32)
    for i in range(S):
        r = rng_for(seed, config_id, _P_EXT, first_sample + i)
        out[i] = pack_bits(r.random((T, Cin, A)) < rates[i])
    return out


# --------------------------------------------------------------------------
# The five workload shapes (tiny plain net, 512-core MNIST-shaped net and its
# 1024-sample batch, the uneven design-space sweep, the large sparse mesh).
# --------------------------------------------------------------------------

def tiny_net(seed: int = 0) -> Net:
    """5 cores of 256x256: cores 0-3 receive external input and all feed core 4.

    Neuron n of input core k targets (core 4, axon n) with delay 1, so every
    axon of core 4 has fan-in 4 (simultaneous arrivals merge). Core 4's
    neurons drive the output bus.
    """
    C, A, N, G = 5, 256, 256, 4
    net = random_net(seed, C, A, N, G, weight_bits=9, potential_bits=32, max_delay=1,
                     grid_w=5, density=0.1, p_core=1.0, p_out=0.0, config_id=1,
                     input_cores=np.arange(4))
    n = np.arange(N)
    for k in range(4):
        net.dest_kind[k] = DEST_CORE
        dx, dy = relative_offsets(np.full(N, k), np.full(N, 4), 5)
        net.dest_dx[k], net.dest_dy[k] = dx, dy
        net.dest_axon[k] = n.astype(np.uint16)
        net.dest_delay[k] = 1
    net.dest_kind[4] = DEST_OUT
    net.dest_dx[4] = 0
    net.dest_dy[4] = 0
    net.dest_axon[4] = 0
    net.dest_delay[4] = 0
    net.name = "tiny5"
    return net


def tiny_inputs(seed: int, S: int = 10, T: int = 16) -> np.ndarray:
    return bernoulli_inputs(seed, tiny_net(seed), S, T, 0.1, config_id=1)


MNIST_LAYERS = 4
MNIST_CORES_PER_LAYER = 128
MNIST_PIXELS = 784


def mnist_net(seed: int = 0) -> Net:
    """512-core layered feed-forward net shaped like the paper's MNIST-512c.

    4 layers x 128 cores of 256x256 on a 32x16 mesh, crossbar density 0.2,
    4 axon types, signed 9-bit weights. Every neuron of layers 0-2 targets a
    distinct axon of the next layer (a seeded permutation of its 32768 axons)
    with delay uniform in 1..4; layer-3 neurons drive the output bus.
    Layer-0 cores take the rate-coded pixel input.
    """
    L, CPL, A, N, G = MNIST_LAYERS, MNIST_CORES_PER_LAYER, 256, 256, 4
    C = L * CPL
    net = random_net(seed, C, A, N, G, weight_bits=9, potential_bits=32, max_delay=4,
                     grid_w=32, density=0.2, p_core=1.0, p_out=0.0, config_id=2,
                     input_cores=np.arange(CPL))
    r = rng_for(seed, 2, _P_DEST, 1000)
    per_layer = CPL * N
    for l in range(L - 1):
        perm = r.permutation(CPL * A)            # destination axon slot of each source neuron
        src = np.arange(l * CPL, (l + 1) * CPL)
        dcore = (l + 1) * CPL + perm // A
        daxon = perm % A
        dcore = dcore.reshape(CPL, N)
        dx, dy = relative_offsets(np.repeat(src[:, None], N, axis=1), dcore, 32)
        net.dest_kind[src] = DEST_CORE
        net.dest_dx[src] = dx
        net.dest_dy[src] = dy
        net.dest_axon[src] = daxon.reshape(CPL, N).astype(np.uint16)
        net.dest_delay[src] = r.integers(1, 5, size=(CPL, N)).astype(np.uint8)
    last = np.arange((L - 1) * CPL, L * CPL)
    net.dest_kind[last] = DEST_OUT
    net.dest_dx[last] = 0
    net.dest_dy[last] = 0
    net.dest_axon[last] = 0
    net.dest_delay[last] = 0
    assert per_layer == CPL * A
    net.name = "mnist512"
    return net


def mnist_pixel_map(seed: int = 0) -> np.ndarray:
    """Pixel index read by each layer-0 axon, int64 [128, 256], uniform over 784 pixels."""
    r = rng_for(seed, 2, _P_PIXMAP)
    return r.integers(0, MNIST_PIXELS, size=(MNIST_CORES_PER_LAYER, 256))


def mnist_inputs(seed: int, S: int, T: int, first_sample: int = 0) -> np.ndarray:
    """Rate-coded pixel input [S, T, 128, 8] for :func:`mnist_net`.

    Sample s has 784 pixel intensities ~ U[0,1]; at tick t pixel p spikes iff
    a fresh U[0,1) draw is below its intensity; layer-0 axon (c, a) carries
    pixel ``pixel_map[c, a]``.
    """
    pm = mnist_pixel_map(seed).reshape(-1)
    out = np.empty((S, T, MNIST_CORES_PER_LAYER, 8), dtype=np.uint32)
    for i in range(S):
        s = first_sample + i
        inten = rng_for(seed, 2, _P_INTENS, s).random(MNIST_PIXELS)
        u = rng_for(seed, 2, _P_TICKU, s).random((T, MNIST_PIXELS))
        spk = u[:, pm] < inten[pm][None, :]
        out[i] = pack_bits(spk.reshape(T, MNIST_CORES_PER_LAYER, 256))
    return out


def mnist_class_of_output(net: Net) -> np.ndarray:
    """Class label of each output neuron: global neuron index mod 10 ([C, N], -1 if not OUT)."""
    C, N = net.num_cores, net.num_neurons
    cls = (np.arange(C * N).reshape(C, N) % 10).astype(np.int64)
    return np.where(net.dest_kind == DEST_OUT, cls, -1)


def sparse_mesh_net(seed: int = 0, side: int = 128) -> Net:
    """Large sparse net: side x side cores of 256x256 on a 2-D mesh.

    Crossbar density 0.05; 99% of neurons target a uniformly random
    (core, axon) with delay uniform in 1..15, 1% drive the output bus;
    leak ~ U[-8,0]; every core takes external input. Thresholds are drawn
    U[64,512] and then multiplied by SPARSE_MESH_THRESHOLD_SCALE = 4: with the
    unscaled draw the recurrent activity settles near 17% spikes per neuron
    per tick and a total axon rate (delivered + external) near 16% on the
    128 x 128 mesh, outside the intended 1-5%; factor 3 gave 3.1% spikes and
    a 5.8% axon rate (2.6% delivered + 3.2% external), factor 4 brings the
    axon rate inside the range (about 1% delivered).
    """
    C = side * side
    net = random_net(seed, C, 256, 256, 4, weight_bits=9, potential_bits=32, max_delay=15,
                     grid_w=side, density=0.05, p_core=0.99, p_out=0.01,
                     leak_range=(-8, 0), thr_range=(64, 512), config_id=5,
                     input_cores=np.arange(C))
    net.threshold = (net.threshold * SPARSE_MESH_THRESHOLD_SCALE).astype(np.int32)
    net.name = f"sparse{C}"
    return net


SPARSE_MESH_THRESHOLD_SCALE = 4


SPARSE_MESH_INPUT_BLOCK = 10   # ticks drawn from one random stream


def bernoulli_bits(r: np.random.Generator, n: int, p: float) -> np.ndarray:
    """n independent Bernoulli(p) draws as a bool array, from the gaps between
    successes (geometric with parameter p), so the cost follows n * p."""
    out = np.zeros(n, dtype=bool)
    if p <= 0.0:
        return out
    pos = -1
    while True:
        k = max(1024, int(1.2 * (n - pos) * p) + 64)
        hits = pos + np.cumsum(r.geometric(p, size=k))
        inside = hits[hits < n]
        out[inside] = True
        if len(inside) < k:
            return out
        pos = int(hits[-1])


def sparse_mesh_inputs(seed: int, net: Net, S: int, T: int, t0: int = 0, samples=None) -> np.ndarray:
    """Bernoulli(r_s) input on every axon for ticks [t0, t0 + T), with
    r_s ~ U[0.01, 0.05] per sample; [len(samples), T, C_in, A/32] (samples:
    default 0..S-1). Ticks come in blocks of SPARSE_MESH_INPUT_BLOCK, each
    from its own (sample, block) stream, so any tick range of any sample can be
    drawn alone and agrees with a longer draw."""
    samples = list(range(S)) if samples is None else [int(s) for s in samples]
    rates = rng_for(seed, 5, _P_INTENS).uniform(0.01, 0.05, size=max(64, max(samples) + 1))
    Cin, A = len(net.input_cores), net.num_axons
    B = SPARSE_MESH_INPUT_BLOCK
    out = np.empty((len(samples), T, Cin, A // 32), dtype=np.uint32)
    for i, s in enumerate(samples):
        for b in range(t0 // B, (t0 + T + B - 1) // B):
            bits = bernoulli_bits(rng_for(seed, 5, _P_EXT, s, b), B * Cin * A, float(rates[s]))
            words = pack_bits(bits.reshape(B, Cin, A))
            lo, hi = max(t0, b * B), min(t0 + T, (b + 1) * B)
            out[i, lo - t0:hi - t0] = words[lo - b * B:hi - b * B]
    return out


def sweep_variant(seed: int, v: int) -> Tuple[Net, Dict]:
    """One variant of the 64-variant uneven design-space sweep.

    C log-uniform in 16..4096 (powers of two), A and N from {64,128,256,512},
    G from {2,4,8}, weight bits 4..9, density U[0.05,0.3];
    W ~ U[-wmax, wmax], threshold ~ U[wmax/4, 2 wmax], leak ~ U[-wmax/32, wmax/32];
    90% of neurons target a random (core, axon) with delay 1..4, the rest OUT;
    external input on the first ceil(C/4) cores.
    Neuron-model axes (Sec. I and Sec. V: the widths of leak, potential and
    reset are configurable), from a stream of their own: potential width 32
    for half the variants, else uniform in [max(b + 4, 12), 31]; leak width
    just wide enough for the leak range plus 0..3 bits; reset width 2..P; a
    floor U[-4 wmax, 0] per neuron for a quarter of the variants and linear
    reset for half the neurons of another quarter.
    """
    r = rng_for(seed, 4, 7000 + v)
    C = int(2 ** r.integers(4, 13))
    A = int(r.choice([64, 128, 256, 512]))
    N = int(r.choice([64, 128, 256, 512]))
    G = int(r.choice([2, 4, 8]))
    b = int(r.integers(4, 10))
    dens = float(r.uniform(0.05, 0.3))
    wmax = (1 << (b - 1)) - 1
    gw = 1 << ((int(math.log2(C)) + 1) // 2)
    lk = wmax // 32
    m = rng_for(seed, 4, 8000 + v)
    P = 32 if m.random() < 0.5 else int(m.integers(max(b + 4, 12), 32))
    leak_bits = max(2, int(lk).bit_length() + 1) + int(m.integers(0, 4))
    reset_bits = int(m.integers(2, P + 1))
    u = m.random()
    floor_range = (-4 * wmax, 0) if u < 0.25 else None
    linear_frac = 0.5 if 0.25 <= u < 0.5 else 0.0
    net = random_net(seed * 1000 + v, C, A, N, G, weight_bits=b, potential_bits=P, max_delay=4,
                     grid_w=gw, density=dens, p_core=0.9, p_out=0.1,
                     leak_range=(-lk, lk), thr_range=(max(1, wmax // 4), 2 * wmax),
                     config_id=4, input_cores=np.arange((C + 3) // 4),
                     floor_range=floor_range, linear_frac=linear_frac,
                     leak_bits=leak_bits, reset_bits=reset_bits)
    model = f"_P{P}" + ("_floor" if floor_range else "") + ("_linear" if linear_frac else "")
    net.name = f"sweep{v}_C{C}_A{A}_N{N}_G{G}_b{b}{model}"
    return net, dict(C=C, A=A, N=N, G=G, b=b, density=dens, P=P, leak_bits=leak_bits, reset_bits=reset_bits,
                     floor=floor_range is not None, linear=linear_frac > 0)


# --------------------------------------------------------------------------
# The applications of the paper's Table I: name, ticks, cores, axons and
# neurons per core. Their trained networks and data are not available; the
# networks below are seeded random stand-ins of the same core counts and core
# sizes (crossbar density 0.2, 4 axon types, 9-bit weights, random routing
# with delays 1..4, Bernoulli(0.1) input on every fourth core). The TrueNorth
# reference runs without input or leak, so no neuron ever spikes.
# --------------------------------------------------------------------------

TABLE1 = [("MNIST-12c", 10010, 12, 256, 256), ("MNIST-128c", 10010, 128, 256, 256),
          ("MNIST-512c", 10010, 512, 256, 256), ("VMM 32x32", 788, 21, 256, 256),
          ("VMM 50x50", 889, 45, 512, 256), ("VMM 60x60", 1095, 51, 512, 256),
          ("CIFAR10", 10010, 36, 256, 256), ("TrueNorth Ref.", 500, 4096, 256, 256)]
TABLE1_GRID_W = {12: 4, 128: 16, 512: 32, 21: 7, 45: 9, 51: 17, 36: 6, 4096: 64}


def table1_net(name: str) -> Net:
    i = [r[0] for r in TABLE1].index(name)
    _, _, C, A, N = TABLE1[i]
    idle = name.startswith("TrueNorth")
    net = random_net(900 + i, C, A, N, 4, weight_bits=9, max_delay=4, grid_w=TABLE1_GRID_W[C], density=0.2,
                     p_core=0.8, p_out=0.1, leak_range=(0, 0) if idle else (-8, 8),
                     input_cores=[] if idle else list(range(0, C, 4)), config_id=716)
    net.name = name
    return net


def table1_inputs(name: str, net: Net, S: int, T: int):
    """Input bitmaps of a Table I stand-in, or None for the TrueNorth reference."""
    i = [r[0] for r in TABLE1].index(name)
    if name.startswith("TrueNorth"):
        return None
    return bernoulli_inputs(i, net, S, T, 0.1, config_id=716)
