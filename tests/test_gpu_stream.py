"""GPU tests of the bulk output raster (ranc_copy_raster) and of streaming
execution (paper_2404_16208_amd.stream): results are compared with the
oracle element by element (every output-bus spike of every tick, final
potentials, counters), and the bulk raster with the per-sample readout.
"""
import numpy as np
import pytest

from oracle import ranc_oracle as O
from paper_2404_16208_amd import workloads as W
from tests.parity_utils import log

pytestmark = pytest.mark.gpu

PATHS = ["plain", "mfma", "sparse"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_16208_amd import ranc  # noqa: F401


@pytest.mark.parametrize("layout", ["sample", "neuron"])
@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("S", [1, 70])
def test_bulk_raster_equals_per_sample_readout(path, layout, S):
    """A 12-tick run in calls of 5 and 7 ticks (7 retained): ticks 3..4 copied
    after the first call into device memory, ticks 5..11 after the second into
    pinned host memory; every sample's decode equals RancNet.spikes, and the
    oracle on three samples."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet, decode_raster
    net = W.random_net(61, 12, 128, 128, 4, grid_w=4, max_delay=5, density=0.3, p_core=0.6, p_out=0.35,
                       thr_range=(32, 160), config_id=830)
    T = 12
    x = W.bernoulli_inputs(3, net, S, T, 0.2, config_id=830)
    g = RancNet(net, S, 7, path=path)
    g.run(torch.from_numpy(np.ascontiguousarray(x[:, :5]).view(np.int32)).cuda(), 5)
    d1 = torch.empty(g.raster_bytes(2, layout), dtype=torch.uint8, device="cuda")
    g.copy_raster(3, 5, d1, layout)
    g.run(torch.from_numpy(np.ascontiguousarray(x[:, 5:]).view(np.int32)).cuda(), 7)
    h2 = torch.empty(g.raster_bytes(7, layout), dtype=torch.uint8, pin_memory=True)
    g.copy_raster(5, 12, h2, layout)
    torch.cuda.synchronize()
    on = g.output_neurons()
    assert len(on) == int((net.dest_kind == 2).sum())
    nw = (len(on) + 31) // 32 if layout == "sample" else (S + 63) // 64

    def words(buf, k):
        a = buf.cpu().numpy() if buf.is_cuda else buf.numpy()
        return a.view(np.uint32).reshape(k, S, nw) if layout == "sample" else a.view(np.uint64).reshape(k, -1, nw)

    w1, w2 = words(d1, 2), words(h2, 7)
    ref = {r["sample"]: r for r in O.simulate(net, x, T, samples=sorted({0, S // 2, S - 1}))}
    for s in range(S):
        got = np.concatenate([decode_raster(w1, on, 3, s, layout), decode_raster(w2, on, 5, s, layout)])
        assert np.array_equal(got[got[:, 0] >= 5], g.spikes(s, 5, 12)), f"{path}/{layout} sample {s}"
        if s in ref:
            ev = ref[s]["events"]
            assert np.array_equal(got, ev[ev[:, 0] >= 3]), f"{path}/{layout} sample {s} vs oracle"
    if layout == "sample":   # padding bits past Nout are zero
        tail = len(on) % 32
        if tail:
            assert not (w2[:, :, -1] >> np.uint32(tail)).any()
    else:                    # padding bits past S are zero
        if S % 64:
            assert not (w2[:, :, -1] >> np.uint64(S % 64)).any()
    g.close()


def test_copy_raster_rejects_ticks_outside_the_window():
    import torch
    from paper_2404_16208_amd import ranc as R
    net = W.random_net(62, 4, 64, 64, 2, grid_w=2, max_delay=2, p_out=0.5, config_id=831)
    g = R.RancNet(net, 2, 4, path="plain")
    g.run(None, 4)
    g.run(None, 3)
    buf = torch.empty(g.raster_bytes(4), dtype=torch.uint8, device="cuda")
    for t0, t1 in [(2, 5), (3, 8), (5, 5), (6, 5)]:
        with pytest.raises(R.RancError) as e:
            g.copy_raster(t0, t1, buf)
        assert e.value.status == R.RANC_ESTATE
    small = torch.empty(g.raster_bytes(4) - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RancError) as e:
        g.copy_raster(3, 7, small)
    assert e.value.status == R.RANC_ENOMEM
    g.copy_raster(3, 7, buf)
    torch.cuda.synchronize()
    g.close()


def _mnist12():
    """A 12-core network of the MNIST-12c application's shape (Table I): 12
    cores of 256 x 256 on a 4 x 3 mesh, seeded random weights and routing."""
    return W.random_net(900, 12, 256, 256, 4, weight_bits=9, max_delay=4, grid_w=4, density=0.2, p_core=0.8,
                        p_out=0.1, input_cores=list(range(0, 12, 4)), config_id=716)


@pytest.fixture(scope="module")
def stream12():
    net = _mnist12()
    T = 10010
    x = W.bernoulli_inputs(0, net, 1, T, 0.1, config_id=716)
    log(f"[stream] oracle: one instance of the 12-core net, {T} ticks")
    ref = O.simulate(net, x, T)[0]
    return net, x, T, ref


@pytest.mark.timeout(600)
@pytest.mark.parametrize("path", PATHS)
def test_streamed_10010_ticks_single_instance(stream12, path):
    """10010 ticks of one instance streamed in 128-tick chunks: inputs from
    pinned host memory, output rasters drained while the next chunk runs;
    every output spike, the final potentials and the counters against the
    oracle."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet, decode_raster
    from paper_2404_16208_amd.stream import Streamer
    net, x, T, ref = stream12
    g = RancNet(net, 1, 128, path=path)
    host = torch.from_numpy(x.view(np.int32)).pin_memory()
    on = g.output_neurons()
    got = []
    Streamer(g, 128).run(host, T, consume=lambda t0, w: got.append(decode_raster(w, on, t0, 0)))
    torch.cuda.synchronize()
    ev = np.concatenate(got)
    log(f"[stream] {path}: {len(ev)} output spikes over {T} ticks")
    assert len(ref["events"]) > 1000
    assert np.array_equal(ev, ref["events"]), f"{path}: {len(ev)} vs {len(ref['events'])} output spikes"
    assert np.array_equal(g.potentials(0), ref["v"])
    c = g.counters(0)
    assert all(c[k] == ref["counters"][k] for k in c), (c, ref["counters"])
    g.close()


@pytest.mark.timeout(600)
def test_streamed_512_core_instance():
    """The 512-core MNIST-shaped net, one instance streamed for 10010 ticks
    (plain path) against a run of the same ticks in 128-tick calls read back
    per call with ranc_read_spikes (every spike), and the first 256 ticks
    against the oracle."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet, decode_raster
    from paper_2404_16208_amd.stream import Streamer
    net = W.mnist_net(0)
    T = 10010
    x = W.mnist_inputs(0, 1, T)
    host = torch.from_numpy(x.view(np.int32)).pin_memory()
    g = RancNet(net, 1, 128, path="plain")
    on = g.output_neurons()
    got = []
    Streamer(g, 128).run(host, T, consume=lambda t0, w: got.append(decode_raster(w, on, t0, 0)))
    ev = np.concatenate(got)
    h = RancNet(net, 1, 128, path="plain")
    want = []
    for t0 in range(0, T, 128):
        k = min(128, T - t0)
        h.run(np.ascontiguousarray(x[:, t0:t0 + k]), k)
        want.append(h.spikes(0, t0, t0 + k))
    want = np.concatenate(want)
    assert np.array_equal(ev, want)
    assert np.array_equal(g.potentials(0), h.potentials(0))
    log("[stream] 512-core: oracle on the first 256 ticks")
    ref = O.simulate(net, x[:, :256], 256)[0]["events"]
    assert np.array_equal(ev[ev[:, 0] < 256], ref)
    g.close()
    h.close()
