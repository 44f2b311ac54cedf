"""GPU parity: the HIP library against the serial oracle, bit for bit.

Every test compares output-bus spikes (tick, core, neuron), final potentials
and the five counters per sample. Sizes are chosen so the oracle finishes in
seconds while the GPU launch still spans several tiles and a ragged tail
(e.g. 70 or 100 samples = one full 64-sample MFMA tile plus a partial one).
"""
import numpy as np
import pytest

from paper_2404_16208_amd import workloads as W
from tests.parity_utils import assert_parity, gpu_run, log, oracle_results, assert_sample_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_16208_amd import ranc  # noqa: F401  (fails loudly if the library is missing)


# ----------------------------------------------------------- tiny 5-core net

@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
def test_tiny_net_all_samples(path):
    net = W.tiny_net(0)
    x = W.tiny_inputs(0, S=10, T=16)
    assert_parity(net, x, 16, path, what="tiny5")


# ----------------------------------------------------------- random shapes

SHAPES = [
    # C, A, N, G, weight_bits, potential_bits, max_delay, grid_w, S, T
    (6, 256, 256, 4, 9, 32, 4, 3, 70, 12),
    (4, 64, 64, 2, 4, 8, 2, 2, 70, 10),
    (8, 128, 64, 8, 8, 16, 7, 4, 100, 9),
    (4, 64, 128, 1, 9, 12, 15, 2, 65, 20),
    (4, 128, 256, 4, 6, 32, 3, 4, 64, 8),
    (3, 512, 128, 4, 8, 32, 5, 3, 66, 6),
    (2, 512, 512, 2, 9, 32, 3, 2, 5, 6),
    (4, 256, 64, 4, 9, 10, 1, 2, 129, 7),
    (4, 64, 128, 2, 4, 8, 2, 2, 70, 10),
    (4, 256, 128, 4, 9, 10, 1, 2, 129, 7),
    (4, 128, 128, 2, 9, 16, 4, 2, 130, 8),
    (2, 512, 256, 4, 8, 32, 3, 2, 100, 6),
    # 512 neurons: two 256-neuron slices per core on the MFMA path
    (3, 256, 512, 4, 9, 32, 4, 3, 130, 8),
    (2, 512, 512, 2, 8, 16, 3, 2, 100, 6),
    (4, 128, 512, 4, 6, 32, 2, 2, 70, 8),
    # 512 axons with 9-bit weights: one weight plane per wavefront (plane split)
    (2, 512, 512, 2, 9, 32, 3, 2, 100, 6),
    (3, 512, 128, 4, 9, 16, 4, 3, 70, 8),
    (4, 512, 64, 2, 9, 32, 2, 2, 66, 6),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "C{}A{}N{}G{}b{}P{}D{}".format(*s[:7]))
@pytest.mark.parametrize("path", ["plain", "auto", "sparse"])
def test_random_shapes(shape, path):
    C, A, N, G, b, P, D, gw, S, T = shape
    wmax = (1 << (b - 1)) - 1
    lim = (1 << (P - 1)) - 1
    net = W.random_net(1000 + C * A + N + G + b + P + D, C, A, N, G, weight_bits=b, potential_bits=P,
                       max_delay=D, grid_w=gw, density=0.25, p_core=0.7, p_out=0.25,
                       leak_range=(-4, 4), thr_range=(max(1, wmax // 2), min(lim, 4 * wmax)),
                       reset_range=(-3, 2), vinit_range=(-5, 5),
                       input_cores=list(range(0, C, 2)), config_id=700,
                       weight_range=(-wmax - 1, wmax))
    x = W.bernoulli_inputs(11, net, S, T, 0.3, config_id=700)
    assert_parity(net, x, T, path, what=f"rand{shape[:7]}")


def _random_shape_net(shape):
    C, A, N, G, b, P, D, gw, S, T = shape
    wmax = (1 << (b - 1)) - 1
    lim = (1 << (P - 1)) - 1
    return W.random_net(1000 + C * A + N + G + b + P + D, C, A, N, G, weight_bits=b, potential_bits=P,
                        max_delay=D, grid_w=gw, density=0.25, p_core=0.7, p_out=0.25,
                        leak_range=(-4, 4), thr_range=(max(1, wmax // 2), min(lim, 4 * wmax)),
                        reset_range=(-3, 2), vinit_range=(-5, 5),
                        input_cores=list(range(0, C, 2)), config_id=700,
                        weight_range=(-wmax - 1, wmax))


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "C{}A{}N{}G{}b{}P{}D{}".format(*s[:7]))
def test_random_shapes_compact_b(shape, monkeypatch):
    """The MFMA kernel with its B tiles built from the compact crossbar
    (column words, per-type plane bytes, axon types) instead of read from the
    int8 weight planes, forced for networks this small (by default it is
    chosen for large networks of wide cores only)."""
    monkeypatch.setenv("RANC_MFMA_BSRC", "compact")
    net = _random_shape_net(shape)
    S, T = shape[8], shape[9]
    x = W.bernoulli_inputs(11, net, S, T, 0.3, config_id=700)
    assert_parity(net, x, T, "mfma", what=f"compact{shape[:7]}")


@pytest.mark.parametrize("shape,S", [(s, 3) for s in SHAPES] + [(SHAPES[i], S) for i in (0, 5, 12, 15)
                                                                  for S in (1, 8)],
                         ids=lambda v: "S{}".format(v) if isinstance(v, int) else
                         "C{}A{}N{}G{}b{}P{}D{}".format(*v[:7]))
def test_sparse_small_batch(shape, S):
    """The event-driven path with at most 8 samples, whose integration takes
    the samples in turn with the wavefront's lanes over a row's entries
    (rows staged in LDS or read from memory, every neuron-model option):
    every sample against the oracle."""
    net = _random_shape_net(shape)
    T = shape[9]
    x = W.bernoulli_inputs(11, net, S, T, 0.3, config_id=700)
    assert_parity(net, x, T, "sparse", what=f"sparse S{S}{shape[:7]}")


@pytest.mark.parametrize("bsrc", ["planes", "compact"])
@pytest.mark.parametrize("shape", [s for s in SHAPES if s[8] > 64],
                         ids=lambda s: "C{}A{}N{}G{}b{}P{}D{}".format(*s[:7]))
def test_random_shapes_weight_planes(shape, bsrc, monkeypatch):
    """Both B sources with more than one 64-sample chunk per core (64 samples
    per workgroup): several workgroups of a core read (or build) the same B
    tiles."""
    monkeypatch.setenv("RANC_MFMA_SPW", "64")
    monkeypatch.setenv("RANC_MFMA_BSRC", bsrc)
    net = _random_shape_net(shape)
    S, T = shape[8], shape[9]
    x = W.bernoulli_inputs(11, net, S, T, 0.3, config_id=700)
    assert_parity(net, x, T, "mfma", what=f"{bsrc}{shape[:7]}")


@pytest.mark.parametrize("lanes", [1, 8], ids=["one_lane", "lane_split"])
def test_large_core_count_unstaged_route(lanes):
    # 1280 cores x 512 neurons: the per-sample spike bitmap (80 KiB) exceeds the
    # LDS staging size, so the one-lane router reads spikes from global memory
    # (forced here: with 3 samples the automatic choice is the lane-split form)
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(77, 1280, 64, 512, 2, weight_bits=9, max_delay=6, grid_w=40, density=0.3,
                       p_core=0.8, p_out=0.1, input_cores=list(range(0, 1280, 3)), config_id=701)
    x = W.bernoulli_inputs(12, net, 3, 5, 0.3, config_id=701)
    g = RancNet(net, 3, 5, path="plain")
    auto = g.launch_shape()
    assert auto["route_lanes_per_word"] == 8 and auto["route_stage"] == 0
    shape = g.launch_shape(dict(auto, route_lanes_per_word=lanes))
    assert shape["route_lanes_per_word"] == lanes and shape["route_stage"] == 0
    g.run(x, 5)
    ref = oracle_results(net, x, 5, [0, 1, 2])
    for s2 in (0, 1, 2):
        assert_sample_equal(g, ref[s2], s2, 5, what=f"C1280N512/lanes{lanes}")


@pytest.mark.parametrize("D", [3, 7, 12], ids=["dmax4", "dmax8", "dmax16"])
@pytest.mark.parametrize("form", ["one_lane_staged", "one_lane_unstaged", "lane_split"])
def test_router_forms(D, form):
    """Every router form with every delay-register width (4, 8, 16), forced
    through the launch shape and reported back by it: per-tick launches for
    the first call, a graph replay for the second, the scheduler ring wrapping
    more than once; every sample against the oracle."""
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(300 + D, 24, 128, 128, 4, max_delay=D, grid_w=6, density=0.25, p_core=0.85, p_out=0.1,
                       thr_range=(32, 200), input_cores=list(range(0, 24, 3)), config_id=703)
    S, T1, T2 = 37, D + 2, 2 * D + 3
    x = W.bernoulli_inputs(20 + D, net, S, T1 + T2, 0.25, config_id=703)
    g = RancNet(net, S, max(T1, T2), path="plain")
    lanes = 8 if form == "lane_split" else 1
    stage = 1 if form == "one_lane_staged" else 0
    shape = g.launch_shape({"route_samples_per_block": 2, "route_split": 2, "route_stage": stage,
                            "route_lanes_per_word": lanes})
    assert shape["route_lanes_per_word"] == lanes and shape["route_stage"] == stage
    g.run(np.ascontiguousarray(x[:, :T1]), T1)
    g.run(np.ascontiguousarray(x[:, T1:]), T2, graph=True)
    ref = oracle_results(net, x, T1 + T2, range(S))
    for s2 in range(S):
        assert_sample_equal(g, ref[s2], s2, T1 + T2, what=f"router/{form}/D{D}")


def test_router_automatic_form():
    """The automatic choice: the lane-split router while the one-lane launch
    would have fewer blocks than the GPU has compute units, else one lane."""
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(310, 24, 128, 128, 4, max_delay=4, grid_w=6, input_cores=[0], config_id=703)
    small = RancNet(net, 8, 4, path="plain").launch_shape()
    big = RancNet(net, 4096, 4, path="plain").launch_shape()
    assert small["route_lanes_per_word"] == 8
    assert big["route_lanes_per_word"] == 1
    blocks = big["route_split"] * -(-4096 // big["route_samples_per_block"])
    assert blocks >= 256


def test_no_input_no_output_cores():
    net = W.random_net(78, 4, 64, 128, 2, max_delay=2, grid_w=2, p_core=1.0, p_out=0.0,
                       leak_range=(5, 20), thr_range=(10, 40), input_cores=[], config_id=702)
    assert len(net.input_cores) == 0 and not (net.dest_kind == W.DEST_OUT).any()
    for path in ("plain", "mfma", "sparse"):
        g = gpu_run(net, None, 9, path, S=64)
        ref = oracle_results(net, None, 9, [0])[0]
        for s in (0, 31, 63):
            assert_sample_equal(g, ref, s, 9, what=f"noio/{path}")


@pytest.mark.parametrize("spw", [128, 512])
def test_mfma_many_tiles_per_workgroup(spw, monkeypatch):
    # several 64-sample tiles per workgroup (the software pipeline), with a
    # ragged last tile inside the last chunk; fan-in up to 6 per axon
    monkeypatch.setenv("RANC_MFMA_SPW", str(spw))
    net = W.random_net(81, 6, 256, 256, 4, weight_bits=9, max_delay=3, grid_w=3, density=0.2, p_core=0.9,
                       p_out=0.1, input_cores=[0, 2, 4], config_id=705)
    x = W.bernoulli_inputs(15, net, 300, 9, 0.3, config_id=705)
    assert_parity(net, x, 9, "mfma", samples=[0, 1, 63, 64, 127, 128, 200, 255, 256, 298, 299],
                  what=f"spw{spw}")


def test_mfma_neuron_slices_many_tiles(monkeypatch):
    # 512-neuron cores as two slices, several tiles per workgroup, ragged
    # last tile; fan-in up to 6 per axon, outputs from both slices
    monkeypatch.setenv("RANC_MFMA_SPW", "128")
    net = W.random_net(82, 4, 256, 512, 4, weight_bits=9, max_delay=4, grid_w=2, density=0.2, p_core=0.8,
                       p_out=0.15, input_cores=[0, 3], config_id=706)
    x = W.bernoulli_inputs(16, net, 200, 9, 0.3, config_id=706)
    assert_parity(net, x, 9, "mfma", samples=[0, 1, 63, 64, 127, 128, 150, 198, 199], what="slices")


@pytest.mark.parametrize("C,N,spw,path", [(8, 512, 64, "mfma"), (16, 256, 128, "mfma"), (32, 128, 64, "mfma"),
                                          (32, 256, 128, "sparse")])
def test_xcd_grouped_units(C, N, spw, path, monkeypatch):
    # a multiple of 8 cores: a core's slices and sample chunks are numbered
    # 8 apart inside runs of 8 cores; several chunks, ragged last tile
    monkeypatch.setenv("RANC_MFMA_SPW", str(spw))
    net = W.random_net(86 + C, C, 128, N, 4, weight_bits=8, max_delay=3, grid_w=4, density=0.2, p_core=0.85,
                       p_out=0.1, input_cores=[0, 3, 5, C - 1], config_id=714)
    x = W.bernoulli_inputs(20, net, 300, 7, 0.3, config_id=714)
    assert_parity(net, x, 7, path, samples=[0, 63, 64, 130, 255, 256, 299], what=f"xcd C{C}N{N}/{path}")


def test_mfma_64_neuron_cores_many_tiles(monkeypatch):
    # 64-neuron cores as a 128-neuron workgroup with two dead blocks, several
    # tiles per workgroup, ragged last tile, 8-bit potentials (clamped)
    monkeypatch.setenv("RANC_MFMA_SPW", "128")
    net = W.random_net(85, 6, 512, 64, 4, weight_bits=8, potential_bits=8, max_delay=3, grid_w=3,
                       density=0.25, p_core=0.8, p_out=0.15, thr_range=(20, 120),
                       input_cores=[0, 2, 5], config_id=710)
    x = W.bernoulli_inputs(18, net, 200, 9, 0.3, config_id=710)
    assert_parity(net, x, 9, "mfma", samples=[0, 1, 63, 64, 127, 128, 170, 199], what="n64")


def test_batch_splits_large_shape_class():
    """Fourteen networks of one MFMA shape class (more than one grouped launch
    holds) and two of another, with their own core and sample counts, in one
    batch under graph replay: each equals the same network run alone."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet, run_batch
    nets, S = [], []
    for i in range(14):
        nets.append(W.random_net(90 + i, 2 + i % 5, 128, 128, 4, weight_bits=8, max_delay=3, grid_w=1,
                                 input_cores=[0], config_id=711))
        S.append(64 + 32 * (i % 3))
    for i in range(2):
        nets.append(W.random_net(110 + i, 3, 256, 256, 2, weight_bits=9, max_delay=2, grid_w=3,
                                 input_cores=[1], config_id=712))
        S.append(70)
    T = 6
    xs = [W.bernoulli_inputs(19, n, s, T, 0.2, config_id=713) for n, s in zip(nets, S)]
    log(f"[batch-split] {len(nets)} networks")
    gs = [RancNet(n, s, T) for n, s in zip(nets, S)]
    assert all(g.path == "mfma" for g in gs)
    bufs = [torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).cuda() for x in xs]
    run_batch(gs, bufs, T, graph=True)
    torch.cuda.synchronize()
    for i, (n, s, x) in enumerate(zip(nets, S, xs)):
        a = RancNet(n, s, T)
        a.run(np.ascontiguousarray(x), T)
        for smp in (0, s // 2, s - 1):
            assert np.array_equal(gs[i].potentials(smp), a.potentials(smp)), (i, smp)
            assert np.array_equal(gs[i].spikes(smp), a.spikes(smp)), (i, smp)
            assert gs[i].counters(smp) == a.counters(smp), (i, smp)
        a.close()
    ref = oracle_results(nets[13], xs[13], T, [0])
    assert_sample_equal(gs[13], ref[0], 0, T, what="batch-split/oracle")


@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
def test_fully_connected_core_all_axons_spiking(path):
    # 512 x 512 crossbar fully connected and every axon spiking every tick:
    # 2^18 synaptic events per sample and tick, the largest count a tick's
    # packed counter word must hold
    net = W.random_net(87, 1, 512, 512, 4, weight_bits=9, max_delay=2, density=1.0, p_core=0.5, p_out=0.5,
                       input_cores=[0], config_id=715)
    x = W.bernoulli_inputs(21, net, 64, 3, 1.0, config_id=715)
    g = assert_parity(net, x, 3, path, samples=[0, 31, 63], what=f"full512/{path}")
    assert g.counters(0)["events"] >= 3 * 512 * 512


# ----------------------------------------------------------- resume / state

@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
def test_chunked_run_equals_single_run(path):
    net = W.random_net(79, 6, 128, 128, 4, max_delay=5, grid_w=3, density=0.3, p_core=0.7, p_out=0.3,
                       input_cores=[0, 1, 2], config_id=703)
    x = W.bernoulli_inputs(13, net, 70, 17, 0.35, config_id=703)
    # chunks of 5 + 5 + 7 ticks: deliveries scheduled past a chunk end must survive
    assert_parity(net, x, 17, path, chunks=[5, 5, 7], what="chunked")


@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
def test_device_inputs_and_reset(path):
    net = W.tiny_net(0)
    x = W.tiny_inputs(0, S=64, T=16)
    g = assert_parity(net, x, 16, path, samples=[0, 7, 63], device_inputs=True, what="devinputs")
    v_before = [g.potentials(s) for s in (0, 63)]
    e_before = [g.spikes(s) for s in (0, 63)]
    g.reset()
    assert g.tick == 0
    g.run(np.ascontiguousarray(x), 16)
    for i, s in enumerate((0, 63)):
        assert np.array_equal(g.potentials(s), v_before[i])
        assert np.array_equal(g.spikes(s), e_before[i])


@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
def test_graph_replay_matches_eager(path):
    """The tick loop captured as one HIP graph (first call) and replayed
    (later calls, with eager copies, reads and synchronizations between
    them): every replay equals the per-launch run, the end state equals the
    oracle, and a replay after reset starts again from tick 0."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(82, 6, 256, 256, 4, weight_bits=9, max_delay=4, grid_w=3, density=0.2, p_core=0.85,
                       p_out=0.15, input_cores=[0, 1, 2], config_id=706)
    S, TC, NC = 70, 6, 4          # 4 calls of 6 ticks; Q = 5, so the slot phase moves between calls
    x = W.bernoulli_inputs(16, net, S, TC * NC, 0.3, config_id=706)
    ge = RancNet(net, S, TC, path=path)
    gg = RancNet(net, S, TC, path=path)
    xbuf = torch.empty((S, TC) + x.shape[2:], dtype=torch.int32, device="cuda")
    samples = [0, 5, 63, 64, 69]
    first = {}
    for call in range(NC):
        log(f"[graph/{path}] call {call}")
        chunk = np.ascontiguousarray(x[:, call * TC:(call + 1) * TC])
        ge.run(chunk, TC)
        xbuf.copy_(torch.from_numpy(chunk.view(np.int32)))
        if call == NC - 1:
            gg.profile(True)
        gg.run(xbuf, TC, graph=True)
        torch.cuda.synchronize()
        for s in samples:
            assert np.array_equal(ge.potentials(s), gg.potentials(s)), (call, s)
            assert np.array_equal(ge.spikes(s), gg.spikes(s)), (call, s)
            assert ge.counters(s) == gg.counters(s), (call, s)
            if call == 0:
                first[s] = (gg.potentials(s), gg.spikes(s), gg.counters(s))
    prof = gg.profile_read()
    assert prof["graph_launches"] == 1 and prof["integrate_launches"] == 0 and prof["graph_ms"] > 0
    ref = oracle_results(net, x, TC * NC, samples)
    for s in samples:
        assert_sample_equal(gg, ref[s], s, TC * NC, what=f"graph/{path}")
    gg.reset()
    xbuf.copy_(torch.from_numpy(np.ascontiguousarray(x[:, :TC]).view(np.int32)))
    gg.run(xbuf, TC, graph=True)
    torch.cuda.synchronize()
    assert gg.tick == TC
    for s in samples:
        v, e, c = first[s]
        assert np.array_equal(gg.potentials(s), v) and np.array_equal(gg.spikes(s), e) and gg.counters(s) == c


def _small_sweep_variants(limit_neuron_axons=1 << 22):
    out = []
    for v in range(64):
        r = W.rng_for(0, 4, 7000 + v)
        C = int(2 ** r.integers(4, 13))
        A = int(r.choice([64, 128, 256, 512]))
        N = int(r.choice([64, 128, 256, 512]))
        if C * A * N <= limit_neuron_axons:
            out.append(v)
    return out


@pytest.mark.parametrize("graph,persistent,phase_mb,bsrc", [(False, False, None, None), (True, False, None, None),
                                                           (False, True, None, None), (True, True, None, None),
                                                           (False, False, "1", None), (True, False, "1", None),
                                                           (False, False, None, "compact"),
                                                           (True, False, None, "compact")])
def test_batch_of_uneven_variants(graph, persistent, phase_mb, bsrc, monkeypatch):
    """Design-space sweep variants of different core counts, core sizes, axon
    types and weight precisions (both paths) advanced together (per tick one
    launch per MFMA shape class, or one persistent launch, and one per plain
    step; with a 1 MB phase budget every network runs all its ticks in a phase
    of its own), in two calls; plus a 6-core net on each path with its own
    sample count. Every network equals the oracle on sampled instances and
    equals the same network run alone on every instance. bsrc "compact": the
    MFMA-path launches build their B tiles from the compact crossbar."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet, run_batch
    vs = _small_sweep_variants()
    assert len(vs) >= 8
    nets = [W.sweep_variant(0, v)[0] for v in vs]
    nets.append(W.random_net(83, 6, 256, 256, 4, weight_bits=9, max_delay=4, grid_w=3, input_cores=[0, 1],
                             config_id=707))
    nets.append(W.random_net(84, 4, 128, 512, 2, weight_bits=6, potential_bits=12, max_delay=3, grid_w=2,
                             input_cores=[1, 3], config_id=708))
    S = [64] * len(vs) + [70, 5]
    T, TC = 12, 6
    xs = [W.bernoulli_inputs(17, n, s, T, 0.1, config_id=709) for n, s in zip(nets, S)]
    if phase_mb is not None:
        monkeypatch.setenv("RANC_BATCH_PHASE_MB", phase_mb)
    if bsrc is not None:
        monkeypatch.setenv("RANC_MFMA_BSRC", bsrc)
    log(f"[batch] {len(nets)} networks, graph={graph}, persistent={persistent}, phase_mb={phase_mb}, bsrc={bsrc}")
    gs = [RancNet(n, s, TC) for n, s in zip(nets, S)]
    paths = [g.path for g in gs]
    assert "mfma" in paths and "plain" in paths
    bufs = [torch.empty((s, TC) + x.shape[2:], dtype=torch.int32, device="cuda") for s, x in zip(S, xs)]
    for call in range(T // TC):
        for b, x in zip(bufs, xs):
            b.copy_(torch.from_numpy(np.ascontiguousarray(x[:, call * TC:(call + 1) * TC]).view(np.int32)))
        run_batch(gs, bufs, TC, graph=graph, persistent=persistent)
        torch.cuda.synchronize()
    alone = []
    for n, s, x in zip(nets, S, xs):
        g = RancNet(n, s, TC)
        for call in range(T // TC):
            g.run(np.ascontiguousarray(x[:, call * TC:(call + 1) * TC]), TC)
        alone.append(g)
    torch.cuda.synchronize()
    for i, (g, a) in enumerate(zip(gs, alone)):
        assert g.tick == T
        for s in range(S[i]):
            assert np.array_equal(g.potentials(s), a.potentials(s)), (nets[i].name, s)
            assert g.counters(s) == a.counters(s), (nets[i].name, s)
            assert np.array_equal(g.spikes(s), a.spikes(s)), (nets[i].name, s)
        samples = [0, S[i] - 1]
        ref = oracle_results(nets[i], xs[i], T, samples)
        for s in samples:
            assert_sample_equal(g, ref[s], s, T, what=f"batch/{nets[i].name}/{g.path}")


@pytest.mark.parametrize("path", ["plain", "mfma"])
def test_autotune_keeps_results_exact(path, tmp_path):
    """The autotuner times every launch shape, keeps the fastest and returns
    the state to tick 0; results with the tuned shape equal the oracle; the
    JSON cache gives a second handle the same shape without tuning."""
    from paper_2404_16208_amd import autotune
    from paper_2404_16208_amd.ranc import RancNet
    N = 512 if path == "plain" else 256
    net = W.random_net(85, 6, 256, N, 4, weight_bits=9, max_delay=4, grid_w=3, input_cores=[0, 1, 2],
                       config_id=710)
    S, T = 200, 8
    x = W.bernoulli_inputs(18, net, S, T, 0.2, config_id=710)
    g = RancNet(net, S, T, path=path)
    cache = str(tmp_path / "shapes.json")
    shape = autotune.tuned(g, x, 4, cache_path=cache)
    assert not shape["cached"] and shape["candidates"] >= 2 and shape["ms_per_tick"] > 0
    assert g.tick == 0
    if path == "mfma":
        assert shape["samples_per_wg"] in (64, 128, 256)
    else:
        assert shape["route_samples_per_block"] in (1, 2, 4, 8) and shape["route_split"] >= 1
    g.run(x, T)
    ref = oracle_results(net, x, T, [0, 99, 199])
    for s, r in ref.items():
        assert_sample_equal(g, r, s, T, what=f"autotuned/{path}")
    g2 = RancNet(net, S, T, path=path)
    shape2 = autotune.tuned(g2, x, 4, cache_path=cache)
    assert shape2["cached"]
    for k in ("samples_per_wg", "route_samples_per_block", "route_split", "route_stage"):
        assert shape2[k] == shape[k], k


@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
def test_single_instance_long_run(path):
    """One instance for 300 ticks as graph replays of 128-tick calls plus a
    44-tick call: scheduler slots and raster rows wrap many times and the
    packed per-tick counts are folded once per call; the end state and the
    output spikes the raster still holds (the last 128 ticks, across calls)
    equal the oracle's."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(88, 12, 256, 256, 4, weight_bits=9, max_delay=4, grid_w=4, density=0.2, p_core=0.8,
                       p_out=0.1, input_cores=[0, 4, 8], config_id=717)
    T, RT = 300, 128
    x = W.bernoulli_inputs(22, net, 1, T, 0.1, config_id=717)
    g = RancNet(net, 1, RT, path=path)
    assert g.path == path
    t0 = 0
    while t0 < T:
        k = min(RT, T - t0)
        xd = torch.from_numpy(np.ascontiguousarray(x[:, t0:t0 + k]).view(np.int32)).cuda()
        g.run(xd, k, graph=True)
        t0 += k
    torch.cuda.synchronize()
    ref = oracle_results(net, x, T, [0])[0]
    assert np.array_equal(g.potentials(0), ref["v"]), "potentials"
    cnt = g.counters(0)
    assert all(cnt[k] == ref["counters"][k] for k in cnt), (cnt, ref["counters"])
    ev = ref["events"]
    assert np.array_equal(g.spikes(0), ev[ev[:, 0] >= T - RT]), "output spikes of the last 128 ticks"
    assert np.array_equal(g.spikes(0, T - 44, T), ev[ev[:, 0] >= T - 44]), "output spikes of the last call"


def test_read_window_errors():
    from paper_2404_16208_amd import ranc as R
    net = W.tiny_net(0)
    x = W.tiny_inputs(0, S=2, T=16)
    g = gpu_run(net, x, 16, "plain", chunks=[8, 8])
    with pytest.raises(R.RancError) as ei:
        R.ranc_read_spikes(g.handle, 0, 0, 16)       # ticks 0..7 were overwritten
    assert ei.value.status == R.RANC_ESTATE
    with pytest.raises(R.RancError) as ei:
        R.ranc_read_spikes(g.handle, 2, 8, 16)       # sample out of range
    assert ei.value.status == R.RANC_EINVAL


def test_call_errors_leave_state_untouched():
    """Too many ticks for the handle, an unknown flag, the same handle twice
    in one batch and a spike buffer that is too small are refused with their
    status; the refused calls queue nothing, so the run continues exactly."""
    import ctypes
    import torch
    from paper_2404_16208_amd import ranc as R
    net = W.tiny_net(0)
    x = W.tiny_inputs(0, S=64, T=16)
    g = R.RancNet(net, 64, 8, path="mfma")
    g.run(np.ascontiguousarray(x[:, :8]), 8)
    stream = torch.cuda.current_stream().cuda_stream
    for flags, ticks, handles, status in ((0, 9, [g.handle], R.RANC_EINVAL), (0, 0, [g.handle], R.RANC_EINVAL),
                                          (16, 4, [g.handle], R.RANC_EINVAL),
                                          (0, 4, [g.handle, g.handle], R.RANC_EINVAL)):
        with pytest.raises(R.RancError) as ei:
            R.ranc_run_ticks(handles, None, flags, ticks, stream)
        assert ei.value.status in (status, R.RANC_ERANGE), (flags, ticks, ei.value.status)
    assert g.tick == 8
    g.run(np.ascontiguousarray(x[:, 8:]), 8)
    ref = oracle_results(net, x, 16, [0, 63])
    for s in (0, 63):
        assert_sample_equal(g, ref[s], s, 16, what="after refused calls")
    # a buffer of one spike for a sample with more: ETRUNC and the needed count
    count = ctypes.c_int64(0)
    buf = np.zeros(1, dtype=R.SPIKE_DTYPE)
    st = R._lib.ranc_read_spikes(g.handle, 0, 8, 16, buf.ctypes.data, 1, ctypes.byref(count))
    n_out = len(g.spikes(0, 8, 16))
    if n_out > 1:
        assert st == R.RANC_ETRUNC and count.value == n_out
    else:
        assert st == R.RANC_OK


# ----------------------------------------------------------- 512-core MNIST-shaped net

@pytest.fixture(scope="module")
def mnist():
    log("[gen] mnist net + 100x32 inputs")
    return W.mnist_net(0), W.mnist_inputs(0, 100, 32)


@pytest.mark.parametrize("path", ["plain", "mfma"])
def test_mnist512_100x32(mnist, path):
    net, x = mnist
    samples = [0, 1, 2, 3, 13, 37, 63, 64, 65, 77, 98, 99]
    assert_parity(net, x, 32, path, samples=samples, what="mnist512")


def test_mnist512_paths_agree_all_samples(mnist):
    net, x = mnist
    gp = gpu_run(net, x, 32, "plain")
    gm = gpu_run(net, x, 32, "mfma")
    for s in range(100):
        assert np.array_equal(gp.potentials(s), gm.potentials(s)), s
        assert np.array_equal(gp.spikes(s), gm.spikes(s)), s
        assert gp.counters(s) == gm.counters(s), s


@pytest.mark.parametrize("S,chunks", [(1, [5, 27]), (60, None), (61, None)])
def test_mnist512_router_split_boundary(mnist, S, chunks):
    """The 512-core net on the plain path at one instance and on both sides of
    the router's switch to eight lanes per destination word (its default
    one-lane launch has 16 blocks per group of 4 samples, so eight lanes per
    word run while that is under 256 blocks, up to 60 samples, and one lane
    per word from 61 on), every sample against the oracle. At one sample the
    5-tick call folds its counts with a thread per counter row and the
    27-tick call with a wavefront per row."""
    net, x = mnist
    xs = np.ascontiguousarray(x[:S])
    assert_parity(net, xs, 32, "plain", chunks=chunks, what=f"mnist512 router boundary S={S}")


def test_mnist512_batched_1024_samples():
    """The 1024-sample batch on the MFMA path: sampled samples against the
    oracle, every sample against the plain GPU path, and the first 100 samples
    equal to the 100-sample batch (samples are independent instances)."""
    import torch
    net = W.mnist_net(0)
    log("[gen] mnist 1024x32 inputs")
    x = W.mnist_inputs(0, 1024, 32)
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    from paper_2404_16208_amd.ranc import RancNet
    gm = RancNet(net, 1024, 32, path="mfma").run(xd, 32)
    ref = oracle_results(net, x, 32, [0, 511, 640, 1000, 1023])
    for s, r in ref.items():
        assert_sample_equal(gm, r, s, 32, what="mnist1024/mfma")
    gp = RancNet(net, 1024, 32, path="plain").run(xd, 32)
    torch.cuda.synchronize()
    for s in range(0, 1024, 7):
        assert np.array_equal(gp.potentials(s), gm.potentials(s)), s
        assert np.array_equal(gp.spikes(s), gm.spikes(s)), s
        assert gp.counters(s) == gm.counters(s), s


# ----------------------------------------------------------- saturation edges

@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
@pytest.mark.parametrize("pbits", [32, 2, 7])
def test_saturation_extremes(path, pbits):
    """Potentials at the ends of the P-bit range, leaks at +-2^30, thresholds
    at the int32 limits: the exact int64 oracle against the saturating 32-bit
    update of the kernels."""
    net = W.random_net(80 + pbits, 4, 64, 128, 2, weight_bits=9, potential_bits=pbits, max_delay=2, grid_w=2,
                       density=0.5, p_core=0.5, p_out=0.5, input_cores=[0, 1, 2, 3], config_id=704)
    r = np.random.default_rng(pbits)
    lo, hi = -(1 << (pbits - 1)), (1 << (pbits - 1)) - 1
    shape = net.v_init.shape
    net.v_init[:] = r.choice(np.array([lo, hi, lo + 1, hi - 1, 0], np.int64), size=shape)
    net.reset[:] = r.choice(np.array([lo, hi, 0], np.int64), size=shape)
    net.leak[:] = r.choice(np.array([-(1 << 30), 1 << 30, -1, 1, 0, hi, lo], np.int64)
                           .clip(-(1 << 30), 1 << 30), size=shape)
    net.threshold[:] = r.choice(np.array([2**31 - 1, -2**31, hi, lo, 0, 100], np.int64), size=shape)
    x = W.bernoulli_inputs(14, net, 70, 12, 0.4, config_id=704)
    assert_parity(net, x, 12, path, what=f"saturation_P{pbits}")


# ----------------------------------------------------------- large sparse mesh (reduced)

def test_sparse_mesh_paths_agree():
    """The large sparse mesh shape (random destinations over the mesh, delays
    up to 15, 1-5% input rates) at 16 x 16 cores: the event-driven path
    against the oracle on sampled instances and against the MFMA path on
    every instance, over 2 calls of 10 ticks."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet
    net = W.sparse_mesh_net(0, side=16)
    S, T, TC = 64, 20, 10
    x = W.sparse_mesh_inputs(0, net, S, T)
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    gs = RancNet(net, S, TC, path="sparse")
    gm = RancNet(net, S, TC, path="mfma")
    for call in range(T // TC):
        chunk = xd[:, call * TC:(call + 1) * TC].contiguous()
        gs.run(chunk, TC)
        gm.run(chunk, TC)
    torch.cuda.synchronize()
    for s in range(S):
        assert np.array_equal(gs.potentials(s), gm.potentials(s)), s
        assert np.array_equal(gs.spikes(s), gm.spikes(s)), s
        assert gs.counters(s) == gm.counters(s), s
    ref = oracle_results(net, x, T, [0, 37, 63])
    for s, r in ref.items():
        assert_sample_equal(gs, r, s, T, what="sparse16x16/sparse")
    tot = gs.total_counters()
    assert tot["delivered"] > 0 and tot["events"] > 0


def test_captured_loop_cache_is_bounded():
    """20 input buffers at 20 addresses, each run as a graph replay: the handle
    keeps at most 16 captured loops (the least recently replayed ones are
    dropped), a dropped loop is captured again on its next use, and results
    stay exact throughout."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(320, 8, 128, 128, 4, max_delay=3, grid_w=4, input_cores=[0, 2, 5], config_id=711)
    S, TC, calls = 70, 2, 24
    x = W.bernoulli_inputs(21, net, S, TC * calls, 0.2, config_id=711)
    bufs = [torch.empty((S, TC) + x.shape[2:], dtype=torch.int32, device="cuda") for _ in range(20)]
    g = RancNet(net, S, TC, path="mfma")
    g.profile(True)
    for i in range(calls):
        b = bufs[i % 20]   # buffers 0..3 come back after 16 others were captured
        b.copy_(torch.from_numpy(np.ascontiguousarray(x[:, i * TC:(i + 1) * TC]).view(np.int32)))
        g.run(b, TC, graph=True)
    prof = g.profile_read()
    assert prof["graphs_held"] == 16 and prof["graphs_dropped"] == 8, prof
    T = TC * calls
    ref = oracle_results(net, x, T, [0, 35, 69])
    for s2, r in ref.items():
        assert_sample_equal(g, r, s2, T, what="graph cache")
    g.close()


@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
def test_workspace_poisoned_before_load(path):
    """A workspace filled with 0xA5 bytes before load gives the same results as
    the oracle: the library reads no workspace byte it has not written (state,
    scheduler, history, counters, raster, link counts), across two calls, one
    of them a graph replay."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet, decode_raster
    net = W.random_net(321, 12, 128, 256, 4, max_delay=5, grid_w=4, density=0.25, p_core=0.7, p_out=0.25,
                       thr_range=(32, 200), input_cores=[0, 3, 7, 11], config_id=712)
    S, T1, T2 = 70, 5, 6
    x = W.bernoulli_inputs(22, net, S, T1 + T2, 0.2, config_id=712)
    g = RancNet(net, S, 6, path=path, workspace_fill=0xA5)
    g.count_links(True)
    g.run(np.ascontiguousarray(x[:, :T1]), T1)
    g.run(torch.from_numpy(np.ascontiguousarray(x[:, T1:]).view(np.int32)).cuda(), T2, graph=True)
    raster = torch.empty(g.raster_bytes(T2, "neuron"), dtype=torch.uint8, device="cuda")
    g.copy_raster(T1, T1 + T2, raster, "neuron")
    torch.cuda.synchronize()
    T = T1 + T2
    ref = oracle_results(net, x, T, [0, 33, 69])
    words = raster.cpu().numpy().view(np.uint64).reshape(T2, -1, 2)
    for s2, r in ref.items():
        assert_sample_equal(g, r, s2, T, what=f"poisoned/{path}")
        assert np.array_equal(g.links(s2), r["links"]), f"poisoned/{path}: links of sample {s2}"
        ev = r["events"]
        assert np.array_equal(decode_raster(words, g.output_neurons(), T1, s2, "neuron"), ev[ev[:, 0] >= T1])
    g.close()
