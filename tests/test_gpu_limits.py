"""GPU parity at the library's size limits: the largest network it accepts
(num_cores * num_neurons = 2^23 neurons: 16384 cores of 64 axons x 512
neurons on a 128 x 128 mesh, delays up to 15) and the largest batch
(65535 samples), on all three paths, against the oracle (every output-bus
spike, final potentials and counters of the checked samples) and, for the
large batch, every sample's output raster and the potentials of every 97th
sample across paths."""
import numpy as np
import pytest

from paper_2404_16208_amd import workloads as W
from tests.parity_utils import assert_sample_equal, gpu_run, log, oracle_results

pytestmark = pytest.mark.gpu

PATHS = ["plain", "mfma", "sparse"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_16208_amd import ranc  # noqa: F401  (fails loudly if the library is missing)


@pytest.fixture(scope="module")
def max_neurons():
    log("[limits] generating 16384 cores x 512 neurons (2^23 neurons)")
    net = W.random_net(901, 16384, 64, 512, 2, weight_bits=9, max_delay=15, grid_w=128, density=0.1,
                       p_core=0.9, p_out=0.05, thr_range=(16, 128), config_id=880)
    assert net.num_cores * net.num_neurons == 1 << 23
    T = 5
    x = W.bernoulli_inputs(11, net, 2, T, 0.1, config_id=880)
    log("[limits] oracle: 2 samples x 5 ticks")
    ref = oracle_results(net, x, T, [0, 1])
    assert ref[0]["counters"]["emitted"] > 0 and ref[0]["counters"]["delivered"] > 0
    return net, x, T, ref


@pytest.mark.timeout(600)
@pytest.mark.parametrize("path", PATHS)
def test_largest_network(max_neurons, path):
    net, x, T, ref = max_neurons
    log(f"[limits] 2^23 neurons, {path} path, calls of 3 and 2 ticks")
    g = gpu_run(net, x, T, path, S=2, chunks=[3, 2], device_inputs=True)
    for s in (0, 1):
        assert_sample_equal(g, ref[s], s, T, what=f"2^23 neurons/{path}")
    g.close()


@pytest.fixture(scope="module")
def max_samples():
    net = W.random_net(902, 4, 64, 64, 2, weight_bits=8, max_delay=3, grid_w=2, density=0.3, p_core=0.7,
                       p_out=0.3, thr_range=(16, 96), config_id=881)
    S, T = 65535, 4
    log("[limits] generating 65535 x 4 inputs")
    x = W.bernoulli_inputs(12, net, S, T, 0.2, config_id=881)
    return net, x, S, T


@pytest.mark.timeout(600)
def test_largest_batch(max_samples):
    """65535 samples: a few samples against the oracle on every path, every
    sample's output raster and every 97th sample's potentials equal across
    the three paths."""
    import torch
    net, x, S, T = max_samples
    picks = [0, 1, 63, 64, 32767, 65472, 65534]
    ref = oracle_results(net, x, T, picks)
    rasters, pots = {}, {}
    for path in PATHS:
        log(f"[limits] 65535 samples, {path} path")
        g = gpu_run(net, x, T, path, S=S, chunks=[T], device_inputs=True)
        for s in picks:
            assert_sample_equal(g, ref[s], s, T, what=f"S=65535/{path}")
        buf = torch.empty(g.raster_bytes(T, "sample"), dtype=torch.uint8, device="cuda")
        g.copy_raster(0, T, buf, "sample")
        torch.cuda.synchronize()
        rasters[path] = buf.cpu().numpy()
        pots[path] = np.stack([g.potentials(s) for s in range(0, S, 97)])
        g.close()
    assert rasters["plain"].any()
    for path in ("mfma", "sparse"):
        assert np.array_equal(rasters[path], rasters["plain"]), path
        assert np.array_equal(pots[path], pots["plain"]), path
